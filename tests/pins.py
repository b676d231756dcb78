"""Independent references used to pin the oracle (no code shared with ``oracle/``).

* ``uniformized_P``      - transition matrices by uniformisation, a third route to exp(Qt)
                           (the oracle uses scipy's Pade expm, the library an eigensystem);
* ``brute_force_site_lik`` - the likelihood of each pattern as the explicit sum over every
                           assignment of states to internal nodes (the definition that
                           Felsenstein's pruning algorithm factorises);
* ``brute_force_rate_gradient`` - the first-order rate-matrix gradient by the same
                           enumeration, with each edge's matrix moved along r t E_ij P;
* ``jc69_two_taxon``     - closed forms for two taxa under Jukes-Cantor;
* ``reroot``             - re-rooting of a tree on another edge (reversible models leave
                           the likelihood unchanged).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def uniformized_P(Q: np.ndarray, t: float, tol: float = 1e-17) -> np.ndarray:
    """P(t) = sum_n e^{-mu t} (mu t)^n / n! R^n with R = I + Q/mu (all terms non-negative)."""
    Q = np.asarray(Q, dtype=np.float64)
    S = Q.shape[0]
    mu = float(np.max(-np.diag(Q))) * 1.01 + 1e-300
    R = np.eye(S) + Q / mu
    x = mu * t
    out = np.zeros((S, S))
    term_mat = np.eye(S)
    log_coef = -x
    n = 0
    while True:
        coef = math.exp(log_coef)
        out += coef * term_mat
        n += 1
        if n > x and coef < tol:
            break
        if n > 100000:
            raise RuntimeError("uniformisation did not converge")
        term_mat = term_mat @ R
        log_coef += math.log(x) - math.log(n) if x > 0 else -math.inf
        if x == 0:
            break
    return out


def brute_force_site_lik(children, n_tips, t, Q, pi, rates, cat_weights, tips) -> np.ndarray:
    """L_p = sum_k w_k sum_{internal states} pi[s_root] prod_{edges v->c} P_k(t_c)[s_v, s_c]."""
    S = Q.shape[0]
    root = 2 * n_tips - 2
    internal = list(range(n_tips, 2 * n_tips - 1))
    edges = [(v, int(c)) for v in internal for c in children[v]]
    tips = np.asarray(tips)
    n_pat = tips.shape[1]
    total = np.zeros(n_pat)
    for k, (r, w) in enumerate(zip(rates, cat_weights)):
        Pk = {c: uniformized_P(Q, r * t[c]) for _, c in edges}
        lik_k = np.zeros(n_pat)
        for assign in itertools.product(range(S), repeat=len(internal)):
            st = dict(zip(internal, assign))
            term = np.full(n_pat, pi[st[root]])
            for v, c in edges:
                if c >= n_tips:
                    term = term * Pk[c][st[v], st[c]]
                else:
                    obs = tips[c]
                    row = Pk[c][st[v]]
                    # unknown tip state: the sum over its states, i.e. the row sum
                    f = np.where(obs < S, row[np.minimum(obs, S - 1)], row.sum())
                    term = term * f
            lik_k += term
        total += w * lik_k
    return total


def brute_force_rate_gradient(children, n_tips, t, Q, pi, rates, cat_weights, tips, weights):
    """sum_p c_p (dL_p / L_p) with every P_k(t_c) moved along r_k t_c E_ij P_k(t_c), by
    explicit enumeration of internal states.

    The likelihood is linear in each edge's matrix, so the derivative along that direction is
    the sum over edges of the enumeration with that edge's factor P[x, y] replaced by
    r t (E_ij P)[x, y] = r t [x == i] P[j, y].  Returns (G [S, S], L [P])."""
    S = Q.shape[0]
    root = 2 * n_tips - 2
    internal = list(range(n_tips, 2 * n_tips - 1))
    edges = [(v, int(c)) for v in internal for c in children[v]]
    tips = np.asarray(tips)
    n_pat = tips.shape[1]
    L = np.zeros(n_pat)
    dL = np.zeros((S, S, n_pat))

    def factor(M, st_v, c):
        """M[st_v, state of c] per pattern (a tip's unknown state sums the row)."""
        if c >= n_tips:
            return None
        obs = tips[c]
        row = M[st_v]
        return np.where(obs < S, row[np.minimum(obs, S - 1)], row.sum())

    for k, (r, w) in enumerate(zip(rates, cat_weights)):
        Pk = {c: uniformized_P(Q, r * t[c]) for _, c in edges}
        for assign in itertools.product(range(S), repeat=len(internal)):
            st = dict(zip(internal, assign))
            fac = {}
            for v, c in edges:
                f = factor(Pk[c], st[v], c)
                fac[c] = np.full(n_pat, Pk[c][st[v], st[c]]) if f is None else f
            term = np.full(n_pat, pi[st[root]])
            for v, c in edges:
                term = term * fac[c]
            L += w * term
            for v, c in edges:
                rest = np.full(n_pat, pi[st[root]])
                for v2, c2 in edges:
                    if c2 != c:
                        rest = rest * fac[c2]
                # (E_ij P)[x, y] is nonzero only for x = i (the parent's state): row j of P
                i = st[v]
                for j in range(S):
                    f = factor(Pk[c], j, c)
                    fj = np.full(n_pat, Pk[c][j, st[c]]) if f is None else f
                    dL[i, j] += w * r * t[c] * rest * fj
    G = np.einsum("p,ijp->ij", np.asarray(weights, dtype=np.float64) / L, dL)
    return G, L


def jc69_two_taxon(d: float, rates, cat_weights):
    """Per-site likelihood and its derivative in d = t1 + t2 for identical / different states.

    Under JC69 (with rate-one normalisation) P_ii(t) = 1/4 + 3/4 e^{-4t/3} and
    P_ij(t) = 1/4 - 1/4 e^{-4t/3}; with root frequencies 1/4 the two-taxon
    likelihood depends only on d.
    """
    r = np.asarray(rates, dtype=np.float64)
    w = np.asarray(cat_weights, dtype=np.float64)
    e = np.exp(-4.0 * r * d / 3.0)
    L_same = 0.25 * np.sum(w * (0.25 + 0.75 * e))
    L_diff = 0.25 * np.sum(w * (0.25 - 0.25 * e))
    dL_same = -0.25 * np.sum(w * r * e)
    dL_diff = (1.0 / 12.0) * np.sum(w * r * e)
    return L_same, L_diff, dL_same / L_same, dL_diff / L_diff


def reroot(children, n_tips, t, edge_node: int, frac: float):
    """Re-root a rooted binary tree on the edge above ``edge_node`` at fraction ``frac`` of its
    length from ``edge_node``.  Returns (children, t, old_to_new) with the standard numbering
    (tips keep their labels; internal nodes renumbered, root last)."""
    N = n_tips
    root = 2 * N - 2
    # unrooted adjacency (the old root of degree two is suppressed)
    adj = {v: {} for v in range(2 * N - 1)}
    for v in range(N, 2 * N - 1):
        for c in children[v]:
            adj[v][int(c)] = t[c]
            adj[int(c)][v] = t[c]
    a, b = (int(c) for c in children[root])
    del adj[a][root], adj[b][root], adj[root]
    adj[a][b] = t[a] + t[b]
    adj[b][a] = t[a] + t[b]
    # find the neighbour of edge_node on the original edge (its old parent, or the sibling
    # if the old parent was the suppressed root)
    old_parent = next(v for v in range(N, 2 * N - 1) if edge_node in [int(c) for c in children[v]])
    other = old_parent if old_parent != root else (b if edge_node == a else a)
    L = adj[edge_node][other]
    kids = {}
    blen = {}
    counter = [0]

    def new_key():
        counter[0] += 1
        return ("n", counter[0])

    def build(v, came_from):
        nbrs = [u for u in adj[v] if u != came_from]
        if not nbrs:
            return ("tip", v)
        assert len(nbrs) == 2
        key = new_key()
        kk = []
        for u in nbrs:
            ck = build(u, v)
            blen[ck] = adj[v][u]
            kk.append(ck)
        kids[key] = tuple(kk)
        return key

    rk = ("root", 0)
    left = build(edge_node, other)
    right = build(other, edge_node)
    blen[left] = frac * L
    blen[right] = (1 - frac) * L
    kids[rk] = (left, right)
    # renumber: tips keep labels, internal nodes in post-order
    new_children = np.full((2 * N - 1, 2), -1, dtype=np.int64)
    new_t = np.zeros(2 * N - 1)
    label = {}
    nxt = [N]

    def number(key):
        if key[0] == "tip":
            label[key] = key[1]
            return key[1]
        ch = [number(c) for c in kids[key]]
        label[key] = nxt[0]
        nxt[0] += 1
        new_children[label[key]] = ch
        for c_key, c_lab in zip(kids[key], ch):
            new_t[c_lab] = blen[c_key]
        return label[key]

    number(rk)
    assert label[rk] == 2 * N - 2
    return new_children, new_t
