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

