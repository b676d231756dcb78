"""Pins of the oracle's rate-matrix gradient (first-order derivative of each transition
matrix): brute-force enumeration, the exact identity in the direction of Q, agreement with
the exact derivative as branches shorten, and planted mistakes that the pins catch."""
import numpy as np
import pytest

import oracle
import oracle.rate_gradient as rg
import synth
from pins import brute_force_rate_gradient


def _wl(kind, n, npat, seed, **kw):
    return synth.make_workload(kind, n, npat, seed=seed, unknown_frac=0.1, **kw)


def _oracle_G(wl, t=None, Q=None, **kw):
    t = wl.t if t is None else t
    return oracle.rate_matrix_gradient(wl.tree.children, wl.n_tips, t, wl.Q if Q is None else Q,
                                       wl.pi, wl.rates, wl.cat_weights, wl.tips, wl.weights, **kw)


@pytest.mark.parametrize("kind,n,npat,seed", [("gtr", 2, 30, 1), ("gtr", 3, 40, 2), ("hky", 4, 25, 3),
                                              ("bin", 5, 20, 4), ("aa", 3, 12, 5)])
def test_matches_brute_force(kind, n, npat, seed):
    wl = _wl(kind, n, npat, seed)
    lnl, G = _oracle_G(wl)
    Gb, L = brute_force_rate_gradient(wl.tree.children, n, wl.t, wl.Q, wl.pi, wl.rates,
                                      wl.cat_weights, wl.tips, wl.weights)
    assert np.isclose(lnl, np.dot(wl.weights, np.log(L)), rtol=1e-11)
    assert np.allclose(G, Gb, rtol=1e-9, atol=1e-9 * np.abs(Gb).max())


@pytest.mark.parametrize("kind,n,seed", [("gtr", 12, 6), ("gy94", 5, 7), ("aa", 7, 8)])
def test_direction_of_Q_is_exact(kind, n, seed):
    """sum_ij Q_ij G_ij = sum_c t_c dlnL/dt_c: in the direction of Q the first-order
    derivative is exact, and scaling Q is scaling every branch."""
    wl = _wl(kind, n, 60, seed)
    _, G = _oracle_G(wl)
    _, _, g = oracle.lnl_and_grad(wl.tree.children, n, wl.t, wl.Q, wl.pi, wl.rates, wl.cat_weights,
                                  wl.tips, wl.weights)
    lhs = float(np.sum(wl.Q * G))
    rhs = float(np.dot(wl.t[: 2 * n - 2], g))
    assert np.isclose(lhs, rhs, rtol=1e-10)


def _fd_dQ(wl, i, j, t, h=1e-6):
    def lnl(e):
        Q = wl.Q.copy()
        Q[i, j] += e
        P = oracle.transition_matrices(Q, wl.rates, t[: 2 * wl.n_tips - 1])
        return oracle.lnl_and_grad(wl.tree.children, wl.n_tips, t, Q, wl.pi, wl.rates, wl.cat_weights,
                                   wl.tips, wl.weights, want_grad=False, P=P)[0]
    return (lnl(h) - lnl(-h)) / (2 * h)


def test_converges_to_exact_derivative_as_branches_shorten():
    """The first-order error of each matrix derivative is O(r t |Q|): with branches scaled
    by s the relative error against central differences of the exact lnL shrinks ~ s."""
    wl = _wl("hky", 6, 200, 9)
    errs = []
    for s in (1.0, 0.1, 0.01):
        t = wl.t * s
        _, G = _oracle_G(wl, t=t)
        pairs = [(0, 1), (2, 3), (1, 0), (3, 3), (0, 2)]
        fd = np.array([_fd_dQ(wl, i, j, t) for i, j in pairs])
        ap = np.array([G[i, j] for i, j in pairs])
        errs.append(np.max(np.abs(ap - fd)) / np.max(np.abs(fd)))
    assert errs[2] < 5e-3
    assert errs[2] < errs[1] < errs[0]
    assert errs[1] / errs[2] > 4 and errs[0] / errs[1] > 3


def test_scaling_and_chunking_do_not_change_G():
    wl = _wl("gtr", 15, 333, 10)
    _, G1 = _oracle_G(wl)
    _, G2 = _oracle_G(wl, scale=False)
    _, G3 = _oracle_G(wl, chunk=50)
    assert np.allclose(G1, G2, rtol=1e-11, atol=1e-11 * np.abs(G1).max())
    assert np.allclose(G1, G3, rtol=1e-11, atol=1e-11 * np.abs(G1).max())


# ----------------------------------------------------------------- planted mistakes

def _brute(wl):
    return brute_force_rate_gradient(wl.tree.children, wl.n_tips, wl.t, wl.Q, wl.pi, wl.rates,
                                      wl.cat_weights, wl.tips, wl.weights)[0]


@pytest.fixture(scope="module")
def small():
    return _wl("gtr", 4, 30, 11)


def _caught(G, Gb):
    return not np.allclose(G, Gb, rtol=1e-6, atol=1e-6 * np.abs(Gb).max())


def test_unmutated_passes(small):
    assert not _caught(_oracle_G(small)[1], _brute(small))


def test_right_sided_derivative_is_caught(small, monkeypatch):
    """P E_ij instead of E_ij P: (pre_c)_i (post_c)_j in place of (top_c)_i (u_c)_j."""
    def wrong(children, n_tips, t, P, tips, weights, pi, rates, cat_weights, S, scale):
        root = 2 * n_tips - 2
        post, logscale = rg.post_order(children, n_tips, P, tips, S, scale=scale)
        site = rg.root_site_loglik(post[root], logscale[root], pi, cat_weights)
        pre = rg.pre_order(children, n_tips, P, post, pi, scale=scale)
        w = np.asarray(cat_weights)
        wr = w * np.asarray(rates)
        G = np.zeros((S, S))
        for c in range(2 * n_tips - 2):
            den = np.einsum("k,kpx,kpx->p", w, pre[c], post[c])
            num = np.einsum("k,kpi,kpj->pij", wr, pre[c], post[c])
            G += t[c] * np.einsum("p,pij->ij", weights / den, num)
        return site, G
    monkeypatch.setattr(rg, "_chunk_rate_gradient", wrong)
    assert _caught(_oracle_G(small)[1], _brute(small))


def test_dropped_branch_length_is_caught(small):
    G = _oracle_G(small)[1]
    _, G1 = _oracle_G(small, t=np.ones_like(small.t))
    assert _caught(G1, _brute(small)) and not _caught(G, _brute(small))


def test_dropped_category_rate_is_caught(small, monkeypatch):
    orig = rg._chunk_rate_gradient

    def wrong(children, n_tips, t, P, tips, weights, pi, rates, cat_weights, S, scale):
        return orig(children, n_tips, t, P, tips, weights, pi, np.ones_like(rates), cat_weights, S, scale)
    monkeypatch.setattr(rg, "_chunk_rate_gradient", wrong)
    assert _caught(_oracle_G(small)[1], _brute(small))


def test_transposed_outer_product_is_caught(small, monkeypatch):
    orig = rg._chunk_rate_gradient

    def wrong(*a):
        site, G = orig(*a)
        return site, G.T
    monkeypatch.setattr(rg, "_chunk_rate_gradient", wrong)
    assert _caught(_oracle_G(small)[1], _brute(small))
