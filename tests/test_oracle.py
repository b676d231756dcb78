"""Pins for the FP64 oracle against closed forms, brute force, invariants and finite differences.

None of these checks re-types the oracle's formulas: brute force enumerates every internal
state assignment with transition matrices from uniformisation, the Jukes-Cantor cases use
closed forms, and the gradient is checked by central finite differences and by the
complex-step derivative of the likelihood.
"""
import itertools

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from pins import brute_force_site_lik, jc69_two_taxon, reroot, uniformized_P


def run(wl, t=None, tips=None, weights=None, children=None, **kw):
    return oracle.lnl_and_grad(wl.tree.children if children is None else children, wl.n_tips,
                               wl.t if t is None else t, wl.Q, wl.pi, wl.rates, wl.cat_weights,
                               wl.tips if tips is None else tips,
                               wl.weights if weights is None else weights, **kw)


# ---------------------------------------------------------------------------------- P(t)

@pytest.mark.parametrize("kind", ["hky", "gtr", "aa", "gy94"])
def test_transition_matrices(kind):
    wl = synth.make_workload(kind, 3, 4, seed=5)
    Q, pi = wl.Q, wl.pi
    ts = np.array([0.0, 1e-4, 0.05, 0.3, 1.7])
    P = oracle.transition_matrices(Q, np.array([1.0, 2.5]), ts)
    assert P.shape == (5, 2) + Q.shape
    assert np.allclose(P[0, 0], np.eye(len(pi)), atol=0)
    assert np.allclose(P.sum(axis=-1), 1.0, atol=1e-13)
    assert (P >= -1e-15).all()
    for c in range(5):
        for k in range(2):
            assert np.allclose(pi @ P[c, k], pi, atol=1e-13)
            F = pi[:, None] * P[c, k]
            assert np.allclose(F, F.T, atol=1e-13)
    # Chapman-Kolmogorov: P(0.05) P(0.3) = P(0.35)
    P35 = oracle.transition_matrices(Q, np.ones(1), np.array([0.35]))[0, 0]
    assert np.allclose(P[2, 0] @ P[3, 0], P35, atol=1e-13)
    # rate r scales time: P_k(t) with r = 2.5 equals P(2.5 t)
    assert np.allclose(P[3, 1], oracle.transition_matrices(Q, np.ones(1), np.array([0.75]))[0, 0],
                       atol=1e-13)
    # an independent route (uniformisation)
    assert np.allclose(P[3, 0], uniformized_P(Q, 0.3), atol=1e-12)
    # long branches forget the start state
    Pinf = oracle.transition_matrices(Q, np.ones(1), np.array([500.0]))[0, 0]
    assert np.allclose(Pinf, np.broadcast_to(pi, Pinf.shape), atol=1e-10)


def test_jc69_transition_closed_form():
    Q, _ = synth.jc69()
    for t in (0.0, 0.01, 0.2, 1.3):
        P = oracle.transition_matrices(Q, np.ones(1), np.array([t]))[0, 0]
        e = np.exp(-4.0 * t / 3.0)
        assert np.allclose(np.diag(P), 0.25 + 0.75 * e, atol=1e-15)
        off = P[~np.eye(4, dtype=bool)]
        assert np.allclose(off, 0.25 - 0.25 * e, atol=1e-15)


def test_tip_partials():
    x = oracle.tip_partials(np.array([0, 3, 4, 1], dtype=np.uint8), 4, 2)
    assert x.shape == (2, 4, 4)
    assert (x[0, 0] == [1, 0, 0, 0]).all() and (x[1, 1] == [0, 0, 0, 1]).all()
    assert (x[0, 2] == 1).all()                                        # unknown -> all ones


# ------------------------------------------------------------------- likelihood pins

def _jc_workload(K, t1, t2):
    wl = synth.make_workload("jc69", 2, 16, seed=1, n_categories=K, tree=synth.two_taxon_tree())
    wl.t[:] = [t1, t2, 0.0]
    wl.tips = np.array([[a for a in range(4) for b in range(4)],
                        [b for a in range(4) for b in range(4)]], dtype=np.uint8)
    wl.weights = np.arange(1, 17, dtype=np.float64)
    return wl


@pytest.mark.parametrize("K", [1, 4])
def test_two_taxon_jc69_closed_form(K):
    wl = _jc_workload(K, 0.13, 0.31)
    lnl, site, grad = run(wl)
    Ls, Ld, gs, gd = jc69_two_taxon(0.44, wl.rates, wl.cat_weights)
    same = wl.tips[0] == wl.tips[1]
    assert np.allclose(site[same], np.log(Ls), rtol=0, atol=1e-14)
    assert np.allclose(site[~same], np.log(Ld), rtol=0, atol=1e-14)
    expect_g = np.sum(wl.weights * np.where(same, gs, gd))
    assert grad == pytest.approx([expect_g, expect_g], rel=1e-13)
    assert lnl == pytest.approx(np.sum(wl.weights * np.where(same, np.log(Ls), np.log(Ld))),
                                rel=1e-14)


def test_jc69_gradient_vanishes_at_distance_mle():
    n_same, n_diff = 70.0, 30.0
    p = n_diff / (n_same + n_diff)
    d_hat = -0.75 * np.log(1.0 - 4.0 * p / 3.0)
    wl = _jc_workload(1, 0.5 * d_hat, 0.5 * d_hat)
    wl.tips = np.array([[0, 0], [0, 1]], dtype=np.uint8)
    _, _, grad = run(wl, weights=np.array([n_same, n_diff]))
    assert np.abs(grad).max() < 1e-10
    _, _, grad2 = run(wl, weights=np.array([n_same, n_diff]), t=np.array([0.4 * d_hat, 0.5 * d_hat, 0]))
    assert (grad2 > 1.0).all()                                         # short of the MLE: uphill


def _small_cases():
    rng = np.random.default_rng(7)
    cases = []
    for n in (2, 3, 4, 5):
        for topo in ("yule", "cat"):
            tree = synth.yule_tree(n, rng) if topo == "yule" else synth.caterpillar_tree(n)
            cases.append(("gtr", n, tree, 40))
    cases.append(("hky", 5, synth.balanced_tree(5), 40))
    cases.append(("aa", 3, None, 25))
    cases.append(("aa", 4, synth.caterpillar_tree(4), 10))
    cases.append(("gy94", 3, None, 12))
    return cases


@pytest.mark.parametrize("kind,n,tree,npat", _small_cases())
def test_brute_force(kind, n, tree, npat):
    wl = synth.make_workload(kind, n, npat, seed=n * 31 + npat, tree=tree, unknown_frac=0.1)
    lnl, site, _ = run(wl, want_grad=False)
    L = brute_force_site_lik(wl.tree.children, n, wl.t, wl.Q, wl.pi, wl.rates, wl.cat_weights,
                             wl.tips)
    assert np.allclose(site, np.log(L), rtol=0, atol=1e-12)
    assert lnl == pytest.approx(np.dot(wl.weights, np.log(L)), rel=1e-13)


# ------------------------------------------------------------------- pre-order pins

@pytest.mark.parametrize("kind,n", [("gtr", 6), ("hky", 9), ("aa", 5), ("gy94", 4)])
def test_inner_product_identity_every_node(kind, n):
    """Sum_k w_k <pre_v, post_v> equals the site likelihood at every node (unscaled FP64)."""
    wl = synth.make_workload(kind, n, 30, seed=17 + n, unknown_frac=0.05)
    P = oracle.transition_matrices(wl.Q, wl.rates, wl.t)
    post, ls = oracle.post_order(wl.tree.children, n, P, wl.tips, wl.n_states, scale=False)
    assert np.all(ls[wl.tree.root] == 0)
    pre = oracle.pre_order(wl.tree.children, n, P, post, wl.pi, scale=False)
    L = brute_force_site_lik(wl.tree.children, n, wl.t, wl.Q, wl.pi, wl.rates, wl.cat_weights,
                             wl.tips) if wl.n_states ** (n - 1) <= 20000 else None
    Lroot = np.einsum("k,kpx,x->p", wl.cat_weights, post[wl.tree.root], wl.pi)
    if L is not None:
        assert np.allclose(Lroot, L, rtol=1e-12, atol=0)
    for v in range(2 * n - 1):
        Lv = np.einsum("k,kpx,kpx->p", wl.cat_weights, pre[v], post[v])
        assert np.allclose(Lv, Lroot, rtol=1e-12, atol=0), v


# ------------------------------------------------------------------- gradient pins

def _fd_check(wl, h=1e-6, **kw):
    lnl, _, g = run(wl, **kw)
    fd = np.empty_like(g)
    for c in range(len(g)):
        tp, tm = wl.t.copy(), wl.t.copy()
        tp[c] += h
        tm[c] -= h
        fd[c] = (run(wl, t=tp, want_grad=False, **kw)[0] - run(wl, t=tm, want_grad=False, **kw)[0]) / (2 * h)
    eps = np.finfo(float).eps
    tol = 1e-5 * np.maximum(np.abs(g), 1e-3 * np.abs(g).max()) + 64 * eps * abs(lnl) / h
    return g, fd, tol


@pytest.mark.parametrize("kind,n,npat,seed", [("hky", 8, 1000, 0), ("gtr", 12, 300, 1),
                                              ("aa", 5, 60, 2), ("gy94", 4, 40, 3)])
def test_gradient_central_differences(kind, n, npat, seed):
    if kind == "hky" and n == 8:
        wl = synth.config_workload("nuc8")                             # the 8-taxon FP64 case
    else:
        wl = synth.make_workload(kind, n, npat, seed=seed, unknown_frac=0.05)
    g, fd, tol = _fd_check(wl)
    assert (np.abs(g - fd) <= tol).all(), np.abs(g - fd) / tol


@pytest.mark.parametrize("kind,n,npat,seed", [("hky", 6, 200, 4), ("gtr", 9, 150, 5),
                                              ("aa", 5, 60, 6), ("gy94", 4, 30, 7)])
def test_gradient_complex_step(kind, n, npat, seed):
    """Complex-step derivative of the oracle's own likelihood (no subtraction, so exact to
    rounding): with t_c -> t_c + i h, Im lnL / h = dlnL/dt_c to about 1e-15.  The pruning
    and root functions run unchanged in complex arithmetic (unscaled: these trees are too
    small to underflow), so this pins the pre-order sandwich gradient far below the
    finite-difference tolerance."""
    from scipy.linalg import expm
    wl = synth.make_workload(kind, n, npat, seed=seed, unknown_frac=0.05)
    _, _, g = run(wl)
    N, S, root = wl.n_tips, wl.n_states, wl.tree.root
    h = 1e-20
    cs = np.zeros_like(g)
    for c in range(2 * N - 2):
        t = wl.t[: 2 * N - 1].astype(complex)
        t[c] += 1j * h
        P = np.array([[expm((r * tc) * wl.Q) for r in wl.rates] for tc in t])
        post, ls = oracle.post_order(wl.tree.children, N, P, wl.tips, S, scale=False)
        site = oracle.root_site_loglik(post[root], ls[root], wl.pi, wl.cat_weights)
        cs[c] = np.dot(wl.weights, site).imag / h
    assert np.abs(g - cs).max() <= 1e-10 * np.abs(cs).max(), np.abs(g - cs).max() / np.abs(cs).max()


def test_directional_derivative_scaling_all_branches():
    """d/ds lnL(s t) at s = 1 equals sum_c t_c g_c."""
    wl = synth.make_workload("gtr", 10, 200, seed=9)
    _, _, g = run(wl)
    h = 1e-6
    up = run(wl, t=wl.t * (1 + h), want_grad=False)[0]
    dn = run(wl, t=wl.t * (1 - h), want_grad=False)[0]
    assert (up - dn) / (2 * h) == pytest.approx(np.dot(wl.t[:-1], g), rel=1e-6)


# ------------------------------------------------------------------- invariances

@pytest.mark.parametrize("kind", ["gtr", "aa"])
def test_root_position_invariance(kind):
    wl = synth.make_workload(kind, 7, 80, seed=21)
    lnl, _, g = run(wl)
    root = wl.tree.root
    a, b = (int(c) for c in wl.tree.children[root])
    # the two root branches only enter through their sum
    assert g[a] == pytest.approx(g[b], rel=1e-10)
    t = wl.t.copy()
    delta = 0.4 * min(t[a], t[b])
    t[a] += delta
    t[b] -= delta
    assert run(wl, t=t, want_grad=False)[0] == pytest.approx(lnl, rel=1e-12)
    # re-root on every edge not adjacent to the root
    for e in range(2 * wl.n_tips - 2):
        if e in (a, b):
            continue
        ch, tt = reroot(wl.tree.children, wl.n_tips, wl.t, e, 0.3)
        assert run(wl, t=tt, children=ch, want_grad=False)[0] == pytest.approx(lnl, rel=1e-12), e


def test_weights_permutation_and_scaling_policy():
    wl = synth.make_workload("gtr", 9, 120, seed=4)
    lnl, site, g = run(wl)
    lnl2, _, g2 = run(wl, weights=2 * wl.weights)
    assert lnl2 == pytest.approx(2 * lnl, rel=1e-14) and np.allclose(g2, 2 * g, rtol=1e-13)
    perm = np.random.default_rng(0).permutation(wl.n_patterns)
    lnl3, site3, g3 = run(wl, tips=wl.tips[:, perm], weights=wl.weights[perm])
    assert lnl3 == pytest.approx(lnl, rel=1e-13) and np.allclose(site3, site[perm], rtol=1e-14)
    assert np.allclose(g3, g, rtol=1e-11)
    # splitting a pattern of weight w into two copies of weight w/2 changes nothing
    tips4 = np.concatenate([wl.tips, wl.tips[:, :1]], axis=1)
    w4 = np.concatenate([wl.weights, [wl.weights[0] / 2]])
    w4[0] /= 2
    lnl4, _, g4 = run(wl, tips=tips4, weights=w4)
    assert lnl4 == pytest.approx(lnl, rel=1e-13) and np.allclose(g4, g, rtol=1e-11)
    # scaling only changes rounding; chunking only changes summation order
    lnl5, site5, g5 = run(wl, scale=False)
    assert np.allclose(site5, site, rtol=1e-13) and np.allclose(g5, g, rtol=1e-10)
    lnl6, _, g6 = run(wl, chunk=7)
    assert lnl6 == pytest.approx(lnl, rel=1e-13) and np.allclose(g6, g, rtol=1e-11)


def test_no_rate_variation_single_category():
    wl = synth.make_workload("hky", 6, 50, seed=8, n_categories=1)
    assert wl.rates[0] == 1.0 and wl.cat_weights[0] == 1.0
    lnl, site, _ = run(wl, want_grad=False)
    L = brute_force_site_lik(wl.tree.children, 6, wl.t, wl.Q, wl.pi, wl.rates, wl.cat_weights, wl.tips)
    assert np.allclose(site, np.log(L), atol=1e-12)


def test_simulated_pattern_frequencies_match_oracle():
    """Chi-square goodness of fit of jump-chain simulated patterns against exp(site lnL)
    computed by the oracle for all 64 patterns of a 3-taxon nucleotide tree."""
    wl = synth.make_workload("gtr", 3, 200_000, seed=12, branch_mean=0.4)
    all_pats = np.array(list(itertools.product(range(4), repeat=3)), dtype=np.uint8).T
    _, site, _ = run(wl, tips=all_pats, weights=np.ones(64), want_grad=False)
    prob = np.exp(site)
    assert prob.sum() == pytest.approx(1.0, abs=1e-13)                # probabilities sum to one
    idx = wl.tips[0].astype(int) * 16 + wl.tips[1].astype(int) * 4 + wl.tips[2].astype(int)
    counts = np.bincount(idx, minlength=64)
    expected = prob * wl.n_patterns
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-4
