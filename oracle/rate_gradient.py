"""Approximate gradient of lnL with respect to the rate-matrix entries (test infrastructure only).

Random-effects substitution models put a free multiplier on every off-diagonal entry of
the rate matrix Q, so a sampler needs d lnL / d Q_ij for all (i, j).  The paper obtains it
as the gradient with respect to the entries of Q (chained by the client to the model
parameters), with the derivative of each matrix exponential taken to first order (Key
Improvements, Algorithmic advances; Magee et al. 2024).

Exactly, d P_k(t) / d Q_ij = int_0^1 exp(s r_k t Q) r_k t E_ij exp((1-s) r_k t Q) ds, with E_ij
the matrix unit at (i, j).  To first order (the s = 0 end of the integral):

    d P_k(t) / d Q_ij  ~=  r_k t E_ij P_k(t)

Each branch c contributes through its own matrix.  Write the likelihood at branch c as

    L_p = sum_k w_k top_c^T P_k(t_c) post_c,   top_c = pre_n o (P_k(t_s) post_s)

where n is the parent of c and s its sibling.  top_c is the partial at the top of branch c:
everything outside c's subtree, carried to n.  Then (E_ij P) post_c = e_i (u_c)_j with
u_c = P_k(t_c) post_c, and

    G_ij = sum_c t_c sum_p c_p [sum_k w_k r_k (top_c)_i (u_c)_j] / [sum_k w_k top_c . u_c]

The denominator is L_p times the per-pattern scale factors of top_c and post_c.  Those
factors are shared by all categories and by the numerator, so they cancel; this is the
same argument as for the branch gradient.

In the direction of Q itself the approximation is exact: d/de exp(r t (1+e) Q) = r t Q P at
e = 0, on either side.  Hence sum_ij Q_ij G_ij = sum_c t_c dlnL/dt_c, which is one of the
pins.
"""
from __future__ import annotations

import numpy as np

from .pruning import (_propagate, post_order, postorder_nodes, pre_order, root_site_loglik,
                      transition_matrices)


def _chunk_rate_gradient(children, n_tips, t, P, tips, weights, pi, rates, cat_weights, S, scale):
    root = 2 * n_tips - 2
    post, logscale = post_order(children, n_tips, P, tips, S, scale=scale)
    site = root_site_loglik(post[root], logscale[root], pi, cat_weights)
    pre = pre_order(children, n_tips, P, post, pi, scale=scale)
    w = np.asarray(cat_weights, dtype=np.float64)
    wr = w * np.asarray(rates, dtype=np.float64)
    G = np.zeros((S, S))
    for n in postorder_nodes(children, n_tips, root):
        a, b = int(children[n][0]), int(children[n][1])
        for c, s in ((a, b), (b, a)):
            top = pre[n] * _propagate(P[s], post[s])            # [K, P, S]
            u = _propagate(P[c], post[c])                         # [K, P, S]
            den = np.einsum("k,kpx,kpx->p", w, top, u)
            num = np.einsum("k,kpi,kpj->pij", wr, top, u)
            G += t[c] * np.einsum("p,pij->ij", weights / den, num)
    return site, G


def rate_matrix_gradient(children, n_tips, t, Q, pi, rates, cat_weights, tips, weights, *,
                         chunk=20000, scale=True):
    """(lnL, G): G[i, j] is the first-order approximation of d lnL / d Q_ij (every entry,
    diagonal included, each taken as free), FP64.  Patterns are processed in chunks and
    summed in order."""
    tips = np.asarray(tips)
    weights = np.asarray(weights, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    S = np.asarray(Q).shape[0]
    P = transition_matrices(Q, rates, t[: 2 * n_tips - 1])
    n_pat = tips.shape[1]
    lnl = 0.0
    G = np.zeros((S, S))
    for lo in range(0, n_pat, max(1, chunk)):
        hi = min(n_pat, lo + chunk)
        site, g = _chunk_rate_gradient(children, n_tips, t, P, tips[:, lo:hi], weights[lo:hi], pi,
                                       rates, cat_weights, S, scale)
        lnl += float(np.dot(weights[lo:hi], site))
        G += g
    return lnl, G
