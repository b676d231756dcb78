"""Plain FP64 pruning, pre-order partials and branch gradients (test infrastructure only).

Notation.  Tree nodes: tips 0..N-1, internal N..2N-2, root 2N-2; branch c is
the edge above node c with length t[c].  K rate categories with rates r_k and
weights w_k; S states; stationary frequencies pi; pattern weights c_p.
Partials are arrays [K, P, S] (category, pattern, state).

    P_k(t)        = expm(r_k t Q)
    post_tip[x]   = 1 if x is the observed state (all ones if unknown)
    post_n        = (P_k(t_a) post_a) * (P_k(t_b) post_b)            (pruning)
    L_p           = sum_k w_k sum_x pi_x post_root[k,p,x]
    pre_root      = pi
    pre_c         = P_k(t_c)^T (pre_n * (P_k(t_s) post_s))           (s = sibling of c)
    L_p           = sum_k w_k <pre_v, post_v>  for every node v      (inner product)
    dlnL/dt_c     = sum_p c_p [sum_k w_k r_k pre_c^T Q post_c] / [sum_k w_k pre_c^T post_c]

The derivative follows from dP_k/dt = r_k Q P_k = r_k P_k Q: differentiating
the inner product at the parent moves one Q between pre_c and post_c.

Scaling (oracle only): every internal post partial is divided by its
per-pattern maximum over (category, state), with the log of the divisor
accumulated per pattern; every pre partial is divided by its per-pattern
maximum and the divisor discarded (it cancels in the gradient ratio because
numerator and denominator carry the same factor).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def postorder_nodes(children: np.ndarray, n_tips: int, root: int) -> list[int]:
    """Internal nodes with every child before its parent (iterative depth-first)."""
    order, stack = [], [(root, False)]
    while stack:
        v, done = stack.pop()
        if v < n_tips:
            continue
        if done:
            order.append(v)
        else:
            stack.append((v, True))
            stack.append((int(children[v][1]), False))
            stack.append((int(children[v][0]), False))
    return order


def transition_matrices(Q: np.ndarray, rates: np.ndarray, t: np.ndarray) -> np.ndarray:
    """P[c, k] = expm(r_k t_c Q) by scaling-and-squaring Pade (scipy), float64 [C, K, S, S]."""
    Q = np.asarray(Q, dtype=np.float64)
    return np.array([[expm((r * tc) * Q) for r in rates] for tc in np.asarray(t, dtype=np.float64)])


def tip_partials(states: np.ndarray, S: int, K: int) -> np.ndarray:
    """One-hot tip partials [K, P, S]; state S (unknown) gives the all-ones vector."""
    states = np.asarray(states)
    p = np.zeros((states.shape[0], S))
    known = states < S
    p[np.nonzero(known)[0], states[known]] = 1.0
    p[~known] = 1.0
    return np.broadcast_to(p, (K,) + p.shape).copy()


def _propagate(Pc: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(P_k x_k) for every category and pattern: out[k,p,i] = sum_j P[k,i,j] x[k,p,j]."""
    return np.matmul(x, np.transpose(Pc, (0, 2, 1)))


def _propagate_transpose(Pc: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(P_k^T x_k): out[k,p,j] = sum_i P[k,i,j] x[k,p,i]."""
    return np.matmul(x, Pc)


def post_order(children, n_tips, P, tips, S, scale=True):
    """Post-order partials for every node and per-pattern log scale factors.

    Returns (post, logscale): post[v] is [K, P, S]; logscale[v] is the
    accumulated log of the divisors applied in the subtree below v ([P]).
    """
    K = P.shape[1]
    n_pat = tips.shape[1]
    root = 2 * n_tips - 2
    post = [None] * (2 * n_tips - 1)
    logscale = [np.zeros(n_pat) for _ in range(2 * n_tips - 1)]
    for v in range(n_tips):
        post[v] = tip_partials(tips[v], S, K)
    for n in postorder_nodes(children, n_tips, root):
        a, b = int(children[n][0]), int(children[n][1])
        x = _propagate(P[a], post[a]) * _propagate(P[b], post[b])
        ls = logscale[a] + logscale[b]
        if scale:
            m = x.max(axis=(0, 2))
            x = x / m[None, :, None]
            ls = ls + np.log(m)
        post[n], logscale[n] = x, ls
    return post, logscale


def root_site_loglik(post_root, logscale_root, pi, cat_weights) -> np.ndarray:
    """l_p = log(sum_k w_k sum_x pi_x post_root[k,p,x]) + accumulated log scale."""
    L = np.einsum("k,kpx,x->p", np.asarray(cat_weights), post_root, np.asarray(pi))
    with np.errstate(divide="ignore"):
        return np.log(L) + logscale_root


def pre_order(children, n_tips, P, post, pi, scale=True):
    """Pre-order partials pre[v] ([K, P, S]) for every node (root: pi)."""
    K, n_pat, S = post[0].shape
    root = 2 * n_tips - 2
    pre = [None] * (2 * n_tips - 1)
    pre[root] = np.broadcast_to(np.asarray(pi, dtype=np.float64), (K, n_pat, S)).copy()
    for n in reversed(postorder_nodes(children, n_tips, root)):
        a, b = int(children[n][0]), int(children[n][1])
        for c, s in ((a, b), (b, a)):
            x = _propagate_transpose(P[c], pre[n] * _propagate(P[s], post[s]))
            if scale:
                x = x / x.max(axis=(0, 2))[None, :, None]
            pre[c] = x
    return pre


def branch_gradients(n_tips, post, pre, Q, rates, cat_weights, weights) -> np.ndarray:
    """dlnL/dt_c for every branch c = 0..2N-3 (the edge above node c)."""
    w = np.asarray(cat_weights, dtype=np.float64)
    wr = w * np.asarray(rates, dtype=np.float64)
    g = np.zeros(2 * n_tips - 2)
    for c in range(2 * n_tips - 2):
        Qpost = np.matmul(post[c], np.asarray(Q).T)          # (Q post_c)[k,p,x]
        num = np.einsum("k,kpx,kpx->p", wr, pre[c], Qpost)
        den = np.einsum("k,kpx,kpx->p", w, pre[c], post[c])
        g[c] = np.dot(weights, num / den)
    return g


def _chunk_eval(tree_children, n_tips, P, tips, weights, Q, pi, rates, cat_weights, S, want_grad,
                scale):
    root = 2 * n_tips - 2
    post, logscale = post_order(tree_children, n_tips, P, tips, S, scale=scale)
    site = root_site_loglik(post[root], logscale[root], pi, cat_weights)
    g = None
    if want_grad:
        pre = pre_order(tree_children, n_tips, P, post, pi, scale=scale)
        g = branch_gradients(n_tips, post, pre, Q, rates, cat_weights, weights)
    return site, g


def lnl_and_grad(children, n_tips, t, Q, pi, rates, cat_weights, tips, weights, *,
                 want_grad=True, chunk=20000, scale=True, P=None):
    """Log-likelihood, site log-likelihoods and branch gradients, FP64.

    Patterns are processed in chunks of ``chunk`` (they are conditionally
    independent given the tree and model) and the chunk results are summed in
    FP64 in order.  Returns (lnL, site_lnL [P], grad [2N-2] or None).
    """
    tips = np.asarray(tips)
    weights = np.asarray(weights, dtype=np.float64)
    S = np.asarray(Q).shape[0]
    if P is None:
        P = transition_matrices(Q, rates, np.asarray(t)[: 2 * n_tips - 1])
    n_pat = tips.shape[1]
    sites = np.empty(n_pat)
    grad = np.zeros(2 * n_tips - 2) if want_grad else None
    for lo in range(0, n_pat, max(1, chunk)):
        hi = min(n_pat, lo + chunk)
        site, g = _chunk_eval(children, n_tips, P, tips[:, lo:hi], weights[lo:hi], Q, pi, rates,
                              cat_weights, S, want_grad, scale)
        sites[lo:hi] = site
        if want_grad:
            grad += g
    lnl = float(np.dot(weights, sites))
    return lnl, sites, grad


def log_likelihood(children, n_tips, t, Q, pi, rates, cat_weights, tips, weights, **kw) -> float:
    return lnl_and_grad(children, n_tips, t, Q, pi, rates, cat_weights, tips, weights,
                        want_grad=False, **kw)[0]
