"""Simulation of site patterns down a tree with the CTMC jump chain.

Each site draws a rate category uniformly, a root state from the stationary
frequencies, and evolves every branch with exact continuous-time Markov chain
simulation: exponential holding times with rate -Q_ii * r_k and jumps to
j != i with probability Q_ij / -Q_ii.  No transition-probability matrix is
formed, so the simulator shares no arithmetic with the likelihood code.
Each simulated site is one pattern (no de-duplication).
"""
from __future__ import annotations

import numpy as np

from .trees import Tree


def _preorder(tree: Tree):
    order = [tree.root]
    i = 0
    while i < len(order):
        v = order[i]
        i += 1
        if v >= tree.n_tips:
            order.extend(int(c) for c in tree.children[v])
    return order


def simulate_patterns(tree: Tree, t: np.ndarray, Q: np.ndarray, pi: np.ndarray,
                      rates: np.ndarray, n_sites: int, rng: np.random.Generator) -> np.ndarray:
    """Return uint8 tip states [N, n_sites]."""
    S = Q.shape[0]
    K = len(rates)
    exit_rate = -np.diag(Q)
    jump = Q / exit_rate[:, None]
    np.fill_diagonal(jump, 0.0)
    cum = np.cumsum(jump, axis=1)
    cum[:, -1] = 1.0
    cat = rng.integers(K, size=n_sites)
    site_rate = np.asarray(rates)[cat]
    states = np.empty((tree.n_nodes, n_sites), dtype=np.int64)
    states[tree.root] = rng.choice(S, size=n_sites, p=pi / pi.sum())
    for v in _preorder(tree):
        if v < tree.n_tips:
            continue
        for c in tree.children[v]:
            s = states[v].copy()
            remaining = site_rate * t[c]
            active = np.nonzero(remaining > 0)[0]
            while active.size:
                wait = rng.exponential(1.0, size=active.size) / exit_rate[s[active]]
                jumps = wait < remaining[active]
                active = active[jumps]
                if not active.size:
                    break
                remaining[active] -= wait[jumps]
                u = rng.random(active.size)
                s[active] = np.minimum((cum[s[active]] < u[:, None]).sum(axis=1), S - 1)
            states[c] = s
    return states[: tree.n_tips].astype(np.uint8)


def pattern_weights(n_patterns: int, rng: np.random.Generator, low: int = 1, high: int = 5) -> np.ndarray:
    """Integer pattern weights, iid uniform on {low..high}, as float64."""
    return rng.integers(low, high + 1, size=n_patterns).astype(np.float64)
