"""Branch-length gradients with post-order partials kept only at every m-th level.

Whole-tree evaluation in store mode keeps the post-order partials of all N-1 internal nodes
from the post-order pass to the pre-order pass.  Here only checkpoint nodes keep theirs:
internal nodes whose height (edges on the longest path down to a tip) is a multiple of the
period m, and the root.  The pre-order walk recomputes the partials between checkpoints,
one segment at a time, just before it needs them: the segment of a non-checkpoint node c is
c and every internal node below it reached without passing a checkpoint, recomputed from
the checkpoints and tips under it.  Post-order buffers in use are then the checkpoints
plus the segments on the current root-to-tip path, instead of N-1, at the cost of about
one more post-order pass.

Everything runs through the operation-level calls (hp_update_post, hp_root_lnl, and for the
backward pass one hp_traverse_gradients_device launch over the recomputations and pre-order
operations as one list; the step-wise form, one hp_update_post or hp_pre_gradients_device
launch per segment, gives the same bits) of an instance created with the buffer counts the
plan reports; the rescale flags are the library's own plan for the instance's scaling
policy, so a recomputed partial is bitwise the one the forward pass produced.
"""
from __future__ import annotations

import numpy as np

from . import _lib


class _Pool:
    """Buffer ids handed out lowest-first and returned when their contents are consumed."""

    def __init__(self, base: int):
        self.base, self.free, self.n = base, [], 0

    def take(self) -> int:
        if self.free:
            self.free.sort()
            return self.free.pop(0)
        self.n += 1
        return self.base + self.n - 1

    def give(self, b: int) -> None:
        self.free.append(b)


class CheckpointPlan:
    """Operation lists of the checkpointed evaluation of one tree (host only).

    ``forward_ops``: the post-order list (hp_post_op rows) that leaves every checkpoint's
    partial in its buffer; ``root_buf``: the root's post buffer; ``steps``: the backward pass
    as ("post", ops) recomputations and ("pre", ops) pre-order/gradient batches, in order.
    ``n_post_buffers`` / ``n_pre_buffers`` are the buffer counts the instance needs.
    """

    def __init__(self, children, period: int, scaling: str = "every_k", scale_period: int = 4):
        if period < 1:
            raise ValueError("period must be >= 1")
        ch = np.asarray(children, dtype=np.int64)
        N = (ch.shape[0] + 1) // 2
        self.n_tips, self.period = N, period
        root = 2 * N - 2
        post, pre = _lib.plan_tree(ch, scaling, scale_period)
        self._resc = {int(r[0]): int(r[5]) for r in post}
        height = np.zeros(2 * N - 1, dtype=np.int64)
        for r in post:
            height[r[0]] = 1 + max(height[r[1]], height[r[3]])
        self.checkpoints = {v for v in range(N, 2 * N - 1) if height[v] % period == 0} | {root}
        kids = {int(r[0]): (int(r[1]), int(r[3])) for r in post}
        parent_of = {c: v for v, kv in kids.items() for c in kv}

        # ---- forward: every internal node once; non-checkpoint buffers are recycled as
        # soon as the parent has combined them
        pool = _Pool(N)
        buf = {}
        fwd = []
        for r in post:
            v, a, b = int(r[0]), int(r[1]), int(r[3])
            buf[v] = pool.take()
            fwd.append((buf[v], a if a < N else buf[a], a, b if b < N else buf[b], b, self._resc[v]))
            for c in (a, b):
                if c >= N and c not in self.checkpoints:
                    pool.give(buf.pop(c))
        self.forward_ops = np.array(fwd, dtype=np.int32).reshape(-1, 6)
        self.root_buf = buf[root]
        pool.give(buf.pop(root))                       # the backward pass needs only the children

        # ---- backward: the library's pre-order list (parents first); a child whose partial
        # is not held is recomputed, with its segment, right before the operation using it
        pre_pool = _Pool(0)
        pre_buf = {}
        steps, batch = [], []

        def flush():
            if batch:
                steps.append(("pre", np.array(batch, dtype=np.int32).reshape(-1, 9)))
                batch.clear()

        def recompute(c):
            seg = []
            stack = [(c, False)]
            while stack:                               # post-order over the segment
                v, done = stack.pop()
                if done:
                    seg.append(v)
                    continue
                stack.append((v, True))
                for x in kids[v][::-1]:
                    if x >= N and x not in buf:
                        stack.append((x, False))
            # every recomputed partial stays held until its parent's pre-order operation
            ops = []
            for v in seg:
                a, b = kids[v]
                buf[v] = pool.take()
                ops.append((buf[v], a if a < N else buf[a], a, b if b < N else buf[b], b, self._resc[v]))
            flush()                   # pending pre-order operations still read recycled buffers
            steps.append(("post", np.array(ops, dtype=np.int32).reshape(-1, 6)))

        for r in pre:
            a, b = int(r[1]), int(r[5])
            n = parent_of[a]
            for c in (a, b):
                if c >= N and c not in buf:
                    recompute(c)
            ca = a if a < N else buf[a]
            cb = b if b < N else buf[b]
            qa = -1
            qb = -1
            if a >= N:
                pre_buf[a] = qa = pre_pool.take()
            if b >= N:
                pre_buf[b] = qb = pre_pool.take()
            batch.append((-1 if n == root else pre_buf[n], ca, a, qa, a, cb, b, qb, b))
            if n != root:
                pre_pool.give(pre_buf.pop(n))
            for c in (a, b):                           # a child's partial is read only here
                if c >= N:
                    pool.give(buf.pop(c))
        flush()
        self.steps = steps
        self.n_post_buffers = pool.n
        self.n_pre_buffers = max(1, pre_pool.n)
        # the same backward pass as one list for a single launch (hp_traverse_gradients_device):
        # rows of (kind, fields), kind 0 for a recomputation, 1 for a pre-order operation
        rows = []
        for kind, ops in steps:
            for r in ops:
                rows.append(([0] + list(r) + [0] * 3) if kind == "post" else ([1] + list(r)))
        self.mixed_ops = np.array(rows, dtype=np.int32).reshape(-1, 10)

    @property
    def n_segments(self) -> int:
        return sum(1 for kind, _ in self.steps if kind == "post")


class Checkpointed:
    """An instance evaluated through a CheckpointPlan: ``lnl(t)`` (forward, host lnL) then
    ``gradients()`` (backward, host array of the 2N-2 branch gradients).  ``create`` sizes a
    new instance for the plan (post-order buffers: the plan's count, not N-1).

    The backward pass reuses the segment buffers, so it consumes the state the forward pass
    left.  Each forward pass returns with a token (``forward_token``: the instance's call
    generation right after it); ``gradients(t, token)`` uses the buffers as they are only if
    no other call has touched the instance since that forward pass and no backward pass has
    consumed it.  Otherwise it first runs the forward pass again at ``t``, the branch
    lengths whose gradient is wanted, so a second forward call or a repeated backward pass
    never reads another evaluation's partials."""

    @classmethod
    def create(cls, n_tips, n_patterns, n_states, n_categories, children, period, *,
               precision="f32", scaling="every_k", scale_period=4, device=0):
        from .instance import Instance
        plan = CheckpointPlan(children, period, scaling, scale_period)
        inst = Instance(n_tips, n_patterns, n_states, n_categories, precision=precision, scaling=scaling,
                        scale_period=scale_period, n_partials=plan.n_post_buffers,
                        n_matrices=2 * n_tips - 2, n_pre_partials=plan.n_pre_buffers, device=device)
        return cls(inst, plan)

    def load(self, tips, weights, V, Vinv, lam, pi, rates, cat_weights):
        self.inst.load(tips, weights, V, Vinv, lam, pi, rates, cat_weights)
        self._live = None
        return self

    def __init__(self, inst, plan: CheckpointPlan):
        if inst.n_tips != plan.n_tips:
            raise ValueError("the instance and the plan differ in taxa")
        if inst.desc.n_partials < plan.n_post_buffers or \
                (inst.desc.n_pre_partials or inst.desc.n_partials) < plan.n_pre_buffers:
            raise ValueError(f"the instance needs n_partials >= {plan.n_post_buffers} and "
                             f"n_pre_partials >= {plan.n_pre_buffers}")
        self.inst, self.plan = inst, plan
        self._last_t = None     # branch lengths of the last forward pass
        self._live = None       # its token while its buffers are intact, else None

    @property
    def forward_token(self):
        """Token of the last forward pass (None once a backward pass has consumed it)."""
        return self._live

    @property
    def last_t(self):
        return None if self._last_t is None else self._last_t.copy()

    def lnl(self, t) -> float:
        nb = 2 * self.plan.n_tips - 2
        tt = np.array(np.asarray(t, dtype=np.float64)[:nb])
        self.inst.update_matrices(np.arange(nb), tt)
        self.inst.update_post(self.plan.forward_ops)
        out = self.inst.root_lnl(self.plan.root_buf)
        self._last_t = tt
        self._live = self.inst.generation
        return out

    def gradients(self, t=None, token=None) -> np.ndarray:
        """The 2N-2 branch gradients as a host array, at branch lengths ``t`` (default: those
        of the last forward pass).  The forward pass is run again first unless ``token`` (by
        default the last forward pass's) is still live.  The pre-order batches add their
        gradients into one device vector (stream-ordered), so the host waits once."""
        if t is None:
            if self._last_t is None:
                raise RuntimeError("gradients() before any forward pass and without t")
            t, token = self._last_t, self._live if token is None else token
        if token is None or token != self._live or self.inst.generation != token:
            self.lnl(t)
        self._live = None       # the backward pass overwrites the segment buffers
        torch = self.inst.torch
        nb = 2 * self.plan.n_tips - 2
        acc = torch.zeros(nb, dtype=torch.float64, device=self.inst.device)
        if self.inst.desc.n_states <= 64:
            # the whole backward pass as one mixed list, one launch (the 4-state walk or the
            # operation-level matrix-core walk)
            self.inst.traverse_gradients_device(self.plan.mixed_ops, acc)
            return acc.cpu().numpy()
        for kind, ops in self.plan.steps:
            if kind == "post":
                self.inst.update_post(ops)
            else:
                self.inst.pre_gradients_device(ops, acc)
        return acc.cpu().numpy()
