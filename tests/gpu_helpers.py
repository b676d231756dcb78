"""Helpers shared by the GPU parity tests: instances built from synthetic workloads,
oracle evaluations of the same inputs, and operation lists written independently of the
library's own scheduler."""
from __future__ import annotations

import json
import os
import sys

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def announce(msg: str) -> None:
    """Name the case before a GPU step (flushed, so a fault still leaves it in the log)."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def make_instance(wl, precision="f64", scaling="every_node", scale_period=4, tree=True, **kw):
    from paper_2606_27607_amd import Instance
    announce(f"instance {wl.name} N={wl.n_tips} P={wl.n_patterns} S={wl.n_states} "
             f"K={wl.n_categories} {precision} {scaling}/{scale_period}")
    inst = Instance(wl.n_tips, wl.n_patterns, wl.n_states, wl.n_categories, precision=precision,
                    scaling=scaling, scale_period=scale_period, **kw)
    inst.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights,
              children=wl.tree.children if tree else None)
    return inst


def oracle_eval(wl, t=None, want_grad=True):
    return oracle.lnl_and_grad(wl.tree.children, wl.n_tips, wl.t if t is None else t, wl.Q, wl.pi,
                               wl.rates, wl.cat_weights, wl.tips, wl.weights, want_grad=want_grad)


def golden(name):
    path = os.path.join(GOLDEN, f"oracle_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def postorder(children, n_tips):
    root = 2 * n_tips - 2
    out, stack = [], [(root, False)]
    while stack:
        v, done = stack.pop()
        if v < n_tips:
            continue
        if done:
            out.append(v)
        else:
            stack += [(v, True), (int(children[v][1]), False), (int(children[v][0]), False)]
    return out


def post_ops(children, n_tips, rescale=1):
    """[dest, child1, mat1, child2, mat2, rescale]: node v uses post buffer v, branch c matrix c."""
    return np.array([[v, children[v][0], children[v][0], children[v][1], children[v][1], rescale]
                     for v in postorder(children, n_tips)], dtype=np.int32)


def pre_ops(children, n_tips):
    """[parent_pre, c1_post, mat1, c1_pre, grad1, c2_post, mat2, c2_pre, grad2] parents first."""
    N, root = n_tips, 2 * n_tips - 2
    rows = []
    for v in reversed(postorder(children, n_tips)):
        a, b = int(children[v][0]), int(children[v][1])
        rows.append([-1 if v == root else v - N, a, a, a - N if a >= N else -1, a,
                     b, b, b - N if b >= N else -1, b])
    return np.array(rows, dtype=np.int32)


def rel(a, b):
    return abs(a - b) / abs(b)


def grad_err(g, g_ref):
    """max |g - g_ref| relative to max |g_ref| (gradients can cross zero, so per-branch
    relative errors are not meaningful for every branch)."""
    return float(np.max(np.abs(np.asarray(g) - g_ref)) / np.max(np.abs(g_ref)))


def branch_err(g, g_ref, floor=0.1):
    """Largest per-branch relative error over the branches whose gradient is at least
    `floor` of max |g_ref| (away from zero crossings a per-branch bound is meaningful)."""
    g, g_ref = np.asarray(g, dtype=np.float64), np.asarray(g_ref, dtype=np.float64)
    big = np.abs(g_ref) >= floor * np.max(np.abs(g_ref))
    return float(np.max(np.abs(g[big] - g_ref[big]) / np.abs(g_ref[big])))


# Parity bounds against the FP64 oracle, per precision form:
#   (relative error of lnL, gradient error as a fraction of max |g|, per-branch relative
#    gradient error on branches with |g_c| >= 0.1 max |g|).
# lnL: 1e-12 where both sides are FP64, the required 1e-5 for FP32 and 1e-4 for the
# 16-bit partial forms.  Gradients: tens of times the largest error observed over the GPU
# suite (FP64 up to ~2e-11 of max |g|: FP64 pattern sums of 10^5 ratios of both signs;
# FP32 up to ~1.4e-6; BF16 partials round to 2^-9 and FP16 to
# 2^-12 at every stored node, observed up to ~4e-3 and ~2e-3), so that a wrong term on any
# branch that matters fails.  "f64mc": FP64 on the matrix-core path (64-term MFMA
# contractions in another order than the oracle's; observed ~1e-11).  "bf16x3": FP32 partials
# with split-BF16 products (~2^-17 relative per product, against FP32's 2^-24).
TOL = {
    "f64": (1e-12, 2e-10, 5e-10),
    "f64mc": (1e-12, 1e-9, 1e-8),
    "f32": (1e-5, 1e-5, 1e-4),
    "bf16x3": (1e-5, 1e-4, 1e-3),
    "bf16": (1e-4, 1e-2, 5e-2),
    "f16": (1e-4, 5e-3, 2e-2),
}


def tol_key(precision, n_states=4):
    return "f64mc" if precision == "f64" and n_states > 4 else precision


def record(**fields):
    """Append observed errors to the JSON-lines file named by HIPPHYLO_ERRLOG (if set)."""
    path = os.environ.get("HIPPHYLO_ERRLOG")
    if not path:
        return
    fields["test"] = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0]
    with open(path, "a") as f:
        f.write(json.dumps(fields) + "\n")


def check(lnl, lnl_ref, g, g_ref, precision, n_states=4, scale=1.0, what=""):
    """Assert parity of lnL (and gradients, if g is not None) within TOL[precision] x scale."""
    key = tol_key(precision, n_states)
    tl, tg, tb = (x * scale for x in TOL[key])
    e_l = rel(lnl, lnl_ref)
    fields = dict(what=what, key=key, lnl_rel=e_l)
    if g is not None:
        fields.update(grad=grad_err(g, g_ref), branch=branch_err(g, g_ref))
    record(**fields)
    assert e_l < tl, (what, key, "lnL", e_l, tl)
    if g is not None:
        assert fields["grad"] < tg, (what, key, "grad", fields["grad"], tg)
        assert fields["branch"] < tb, (what, key, "branch", fields["branch"], tb)
