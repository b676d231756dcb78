"""Host-side checks of the checkpointed-gradient plan: a symbolic run of its operation lists
(buffer contents tracked as node ids) must feed every operation the partials of the right
nodes, give every branch exactly one gradient, and hold fewer post-order buffers than
store mode."""
import numpy as np
import pytest

import synth
from paper_2606_27607_amd.checkpoint import CheckpointPlan


def simulate(plan, children):
    ch = np.asarray(children)
    N = plan.n_tips
    root = 2 * N - 2
    post = {}                                      # buffer id -> node whose partial it holds

    def ref(x, node):
        if node < N:
            assert x == node, "a tip child must be referenced by its own index"
        else:
            assert post.get(x) == node, f"buffer {x} holds {post.get(x)}, not node {node}"

    for dest, c1, m1, c2, m2, _ in plan.forward_ops:
        v = int(np.where((ch[:, 0] == m1) & (ch[:, 1] == m2))[0][0])
        ref(c1, m1)
        ref(c2, m2)
        post[dest] = v
    assert post[plan.root_buf] == root
    for v in plan.checkpoints:
        assert v in post.values()
    pre = {}
    grads = []
    for kind, ops in plan.steps:
        if kind == "post":
            for dest, c1, m1, c2, m2, _ in ops:
                v = int(np.where((ch[:, 0] == m1) & (ch[:, 1] == m2))[0][0])
                ref(c1, m1)
                ref(c2, m2)
                post[dest] = v
        else:
            for pp, c1, m1, q1, g1, c2, m2, q2, g2 in ops:
                n = int(np.where((ch[:, 0] == m1) & (ch[:, 1] == m2))[0][0])
                if n == root:
                    assert pp == -1
                else:
                    assert pre.get(pp) == n
                ref(c1, m1)
                ref(c2, m2)
                if m1 >= N:
                    pre[q1] = m1
                if m2 >= N:
                    pre[q2] = m2
                grads += [g1, g2]
    assert sorted(grads) == list(range(2 * N - 2))
    # the single-launch form of the backward pass is the same operations in the same order
    flat = [([0] + list(r) + [0, 0, 0]) if kind == "post" else ([1] + list(r))
            for kind, ops in plan.steps for r in ops]
    assert np.array_equal(plan.mixed_ops, np.array(flat, dtype=np.int32).reshape(-1, 10))
    assert max(post) - N + 1 <= plan.n_post_buffers
    assert (max(pre) + 1 if pre else 1) <= plan.n_pre_buffers


@pytest.mark.parametrize("n,seed", [(2, 0), (3, 1), (9, 2), (64, 3), (256, 4)])
@pytest.mark.parametrize("period", [1, 2, 3, 4, 1000])
def test_plan_feeds_every_operation_its_partials(n, seed, period):
    tree = synth.trees.yule_tree(n, np.random.default_rng(seed)) if n > 2 else None
    children = tree.children if tree is not None else np.array([[-1, -1], [-1, -1], [0, 1]])
    plan = CheckpointPlan(children, period)
    simulate(plan, children)


def test_caterpillar_and_buffer_savings():
    n = 64
    ch = -np.ones((2 * n - 1, 2), dtype=np.int64)
    prev = 0
    for i, v in enumerate(range(n, 2 * n - 1)):     # a caterpillar: height grows by one each node
        ch[v] = (prev, i + 1)
        prev = v
    plan = CheckpointPlan(ch, 4)
    simulate(plan, ch)
    assert plan.n_post_buffers < n - 1
    yule = synth.trees.yule_tree(256, np.random.default_rng(7)).children
    store = CheckpointPlan(yule, 1)                  # every internal node is a checkpoint
    ck = CheckpointPlan(yule, 4)
    simulate(ck, yule)
    assert store.n_post_buffers >= 255 and ck.n_post_buffers < store.n_post_buffers // 2
    assert ck.n_segments > 0 and store.n_segments == 0


def test_period_beyond_height_keeps_only_the_root():
    """With m above the tree height only the root is a checkpoint: the backward pass then
    recomputes every other internal node, in segments below the root's children."""
    yule = synth.trees.yule_tree(40, np.random.default_rng(3)).children
    plan = CheckpointPlan(yule, 10_000)
    simulate(plan, yule)
    assert list(plan.checkpoints) == [2 * 40 - 2]
    recomputed = sum(len(ops) for kind, ops in plan.steps if kind == "post")
    assert recomputed == 40 - 2          # every internal node but the root, exactly once



class _SymbolicInstance:
    """Stands in for a library instance on the CPU: each post buffer holds (node, version of
    the branch lengths it was computed from), the matrices hold a version, and every call
    that is not read-only bumps ``generation`` as the binding does.  A pre-order batch
    records, per gradient slot, the version of every partial it read."""

    def __init__(self, n_tips, n_partials):
        import torch
        self.torch, self.device = torch, "cpu"
        self.n_tips, self.generation = n_tips, 0
        self.mats = None
        self.post = {}
        self.read_versions = {}

    def update_matrices(self, idx, t):
        self.generation += 1
        self.mats = float(np.asarray(t)[0])       # the first branch length names the version

    def update_post(self, ops):
        self.generation += 1
        for dest, c1, m1, c2, m2, _ in ops:
            vs = {self.post[c][1] for c in (c1, c2) if c >= self.n_tips} | {self.mats}
            assert len(vs) == 1, "a partial combined children of different evaluations"
            self.post[int(dest)] = (int(m1), self.mats)

    def root_lnl(self, root_buf):
        self.generation += 1
        return self.post[root_buf][1]

    def pre_gradients_device(self, ops, acc):
        self.generation += 1
        self._pre(ops, acc)
        return acc

    def _pre(self, ops, acc):
        for pp, c1, m1, q1, g1, c2, m2, q2, g2 in ops:
            for c, g in ((c1, g1), (c2, g2)):
                v = self.post[c][1] if c >= self.n_tips else self.mats
                self.read_versions.setdefault(int(g), set()).add(v)
                acc[int(g)] += v

    def traverse_gradients_device(self, ops, acc):
        """The mixed list, in order: kind 0 a recomputation, kind 1 a pre-order operation."""
        self.generation += 1
        for row in ops:
            if row[0] == 0:
                dest, c1, m1, c2, m2, _ = row[1:7]
                vs = {self.post[c][1] for c in (c1, c2) if c >= self.n_tips} | {self.mats}
                assert len(vs) == 1, "a partial combined children of different evaluations"
                self.post[int(dest)] = (int(m1), self.mats)
            else:
                self._pre([row[1:]], acc)
        return acc


def _symbolic_checkpointed(n=40, period=3, n_states=4):
    """n_states 4 takes the backward pass as one mixed list, more states as step-wise calls."""
    from paper_2606_27607_amd.checkpoint import Checkpointed
    yule = synth.trees.yule_tree(n, np.random.default_rng(11)).children
    plan = CheckpointPlan(yule, period)
    inst = _SymbolicInstance(n, plan.n_post_buffers)
    inst.desc = type("D", (), {"n_partials": plan.n_post_buffers, "n_pre_partials": plan.n_pre_buffers,
                               "n_states": n_states})
    return Checkpointed(inst, plan), inst, 2 * n - 2


@pytest.mark.parametrize("n_states", [4, 61])
def test_backward_after_a_second_forward_reads_its_own_evaluation(n_states):
    """Two forward passes, then the backward pass of the first: it must not read the second
    evaluation's partials or matrices (it runs the first forward pass again)."""
    ck, inst, nb = _symbolic_checkpointed(n_states=n_states)
    t1, t2 = np.full(nb, 0.1), np.full(nb, 0.2)
    ck.lnl(t1)
    tok1, saved1 = ck.forward_token, ck.last_t
    ck.lnl(t2)
    g = ck.gradients(saved1, tok1)
    assert all(v == {0.1} for v in inst.read_versions.values())
    assert np.allclose(g, 0.1)                          # each slot read once, at version 0.1


@pytest.mark.parametrize("n_states", [4, 61])
def test_repeated_backward_reruns_the_forward_pass(n_states):
    """A backward pass consumes the forward state: a second backward pass of the same
    forward call (retain_graph) runs the forward pass again, and gives the same values."""
    ck, inst, nb = _symbolic_checkpointed(period=2, n_states=n_states)
    ck.lnl(np.full(nb, 0.3))
    tok, saved = ck.forward_token, ck.last_t
    g1 = ck.gradients(saved, tok)
    assert ck.forward_token is None
    gen = inst.generation
    g2 = ck.gradients(saved, tok)
    assert inst.generation > gen + 3                    # forward (3 calls) + backward ran
    assert np.array_equal(g1, g2)
    # with the state live, no forward pass runs again
    ck.lnl(np.full(nb, 0.4))
    gen = inst.generation
    ck.gradients()
    n_backward = 1                                      # one mixed-list launch
    assert inst.generation == gen + n_backward


@pytest.mark.parametrize("n_states", [4, 61])
def test_intervening_call_invalidates_the_forward_state(n_states):
    ck, inst, nb = _symbolic_checkpointed(n_states=n_states)
    ck.lnl(np.full(nb, 0.5))
    tok, saved = ck.forward_token, ck.last_t
    inst.update_matrices(np.arange(nb), np.full(nb, 0.9))   # any other use of the instance
    ck.gradients(saved, tok)
    assert all(v == {0.5} for v in inst.read_versions.values())
