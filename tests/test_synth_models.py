"""Pins for the synthetic-input generators: rate matrices, eigensystems, discrete gamma,
trees and the jump-chain simulator."""
import numpy as np
import pytest
from scipy import integrate, stats

import synth
from synth import models


def _check_reversible(Q, pi):
    assert np.allclose(Q.sum(axis=1), 0.0, atol=1e-13)
    assert np.allclose(pi @ Q, 0.0, atol=1e-13)                       # stationarity
    F = pi[:, None] * Q
    assert np.allclose(F, F.T, atol=1e-14)                            # detailed balance
    assert abs(-np.dot(pi, np.diag(Q)) - 1.0) < 1e-13                 # one substitution / unit
    off = Q - np.diag(np.diag(Q))
    assert (off >= 0).all()


@pytest.mark.parametrize("kind", ["hky", "gtr", "aa", "gy94", "jc69"])
def test_rate_matrix_invariants(kind):
    wl = synth.make_workload(kind, 4, 10, seed=3)
    _check_reversible(wl.Q, wl.pi)
    V, Vinv, lam = wl.V, wl.Vinv, wl.lam
    assert np.allclose(V @ Vinv, np.eye(len(lam)), atol=1e-12)
    assert np.allclose(V @ np.diag(lam) @ Vinv, wl.Q, atol=1e-12)
    assert np.max(lam) == pytest.approx(0.0, abs=1e-12)               # one zero eigenvalue
    assert (lam <= 1e-12).all()


def test_hky_structure():
    pi = np.array([0.1, 0.2, 0.3, 0.4])
    Q = models.hky85(2.0, pi)
    # transitions A<->G and C<->T at kappa times the transversion rate, times pi_j
    ratio = (Q[0, 2] / pi[2]) / (Q[0, 1] / pi[1])
    assert ratio == pytest.approx(2.0)
    assert (Q[1, 3] / pi[3]) / (Q[1, 2] / pi[2]) == pytest.approx(2.0)


def test_genetic_code_and_gy94_structure():
    assert len(synth.CODONS) == 61
    assert all(synth.GENETIC_CODE[c] != "*" for c in synth.CODONS)
    assert {c for c, a in synth.GENETIC_CODE.items() if a == "*"} == {"TAA", "TAG", "TGA"}
    assert synth.GENETIC_CODE["ATG"] == "M" and synth.GENETIC_CODE["TGG"] == "W"
    pi = np.full(61, 1 / 61)
    Q = models.gy94(2.0, 0.3, pi)
    C = synth.CODONS
    for i in range(61):
        for j in range(61):
            nd = sum(a != b for a, b in zip(C[i], C[j]))
            if i != j and nd != 1:
                assert Q[i, j] == 0.0
    # AAA (Lys) -> AAG (Lys): synonymous transition; AAA -> AAC (Asn): nonsynonymous transversion
    i, j, k = C.index("AAA"), C.index("AAG"), C.index("AAC")
    assert Q[i, j] / Q[i, k] == pytest.approx(2.0 / 0.3)


def test_discrete_gamma_by_quadrature():
    alpha, K = 0.5, 4
    r, w = models.discrete_gamma(alpha, K)
    assert np.sum(w * r) == pytest.approx(1.0, abs=1e-13)
    dist = stats.gamma(a=alpha, scale=1.0 / alpha)
    edges = [0.0] + [dist.ppf(k / K) for k in range(1, K)] + [np.inf]
    for k in range(K):
        prob = integrate.quad(dist.pdf, edges[k], edges[k + 1], limit=200)[0]
        assert prob == pytest.approx(1.0 / K, rel=1e-8)
        mean = integrate.quad(lambda x: x * dist.pdf(x), edges[k], edges[k + 1], limit=200)[0] / prob
        assert r[k] == pytest.approx(mean, rel=1e-7)


def test_discrete_gamma_golden():
    # tests/golden/discrete_gamma_a0.5_k4.txt: Yang (1994) mean-of-category rates
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "discrete_gamma_a0.5_k4.txt")
    vals = [float(x) for x in open(path).read().split("\n") if x and not x.startswith("#")]
    r, _ = models.discrete_gamma(0.5, 4)
    assert np.allclose(r, vals, atol=6e-5)


@pytest.mark.parametrize("n", [2, 3, 8, 33])
def test_trees_well_formed(n):
    rng = np.random.default_rng(n)
    for tree in (synth.yule_tree(n, rng), synth.balanced_tree(n), synth.caterpillar_tree(n)):
        tree.validate()
        assert tree.root == 2 * n - 2
        # children precede parents in the numbering of internal nodes
        for v in range(n, 2 * n - 1):
            assert (tree.children[v] < v).all()


def test_simulator_branch_transition_frequencies():
    """Jump-chain simulation of one branch: the empirical transition frequencies must match
    uniformisation's P(t) (an independent route to exp(Qt))."""
    from pins import uniformized_P
    rng = np.random.default_rng(11)
    pi = rng.dirichlet(np.full(4, 10.0))
    Q = models.gtr(rng.gamma(2.0, 1.0, 6), pi)
    tree = synth.two_taxon_tree()
    t = np.array([0.0, 0.7, 0.0])  # all change on branch 1; tip 0 keeps the root state
    tips = synth.simulate_patterns(tree, t, Q, pi, np.ones(1), 200_000, rng)
    P = uniformized_P(Q, 0.7)
    counts = np.zeros((4, 4))
    np.add.at(counts, (tips[0], tips[1]), 1)
    expected = pi[:, None] * P * tips.shape[1]
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert stats.chi2.sf(chi2, 15) > 1e-4
