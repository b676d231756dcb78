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
    relative errors are not meaningful)."""
    return float(np.max(np.abs(np.asarray(g) - g_ref)) / np.max(np.abs(g_ref)))
