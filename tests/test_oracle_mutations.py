"""Planted mistakes in the oracle (on the CPU) must be caught by the pins.

Each case patches one step of the oracle with a plausible bug: a transposed
operand, a dropped factor, a wrong sign or index, and asserts that at least
one of the independent checks (brute force, finite differences, the
inner-product identity) rejects the result.
"""
import numpy as np
import pytest

import oracle
import oracle.pruning as op
import synth
from pins import brute_force_site_lik


@pytest.fixture(scope="module")
def wl():
    return synth.make_workload("gtr", 5, 30, seed=77, unknown_frac=0.05)


def _lnl_ok(wl, **kw):
    lnl, site, _ = oracle.lnl_and_grad(wl.tree.children, wl.n_tips, wl.t, wl.Q, wl.pi, wl.rates,
                                       wl.cat_weights, wl.tips, wl.weights, want_grad=False, **kw)
    L = brute_force_site_lik(wl.tree.children, wl.n_tips, wl.t, wl.Q, wl.pi, wl.rates,
                             wl.cat_weights, wl.tips)
    return np.allclose(site, np.log(L), atol=1e-10)


def _grad_ok(wl, rates=None, Q=None):
    rates = wl.rates if rates is None else rates
    Qg = wl.Q if Q is None else Q
    P = oracle.transition_matrices(wl.Q, wl.rates, wl.t)
    post, _ = oracle.post_order(wl.tree.children, wl.n_tips, P, wl.tips, 4)
    pre = oracle.pre_order(wl.tree.children, wl.n_tips, P, post, wl.pi)
    g = oracle.branch_gradients(wl.n_tips, post, pre, Qg, rates, wl.cat_weights, wl.weights)
    h = 1e-6
    for c in range(len(g)):
        tp, tm = wl.t.copy(), wl.t.copy()
        tp[c] += h
        tm[c] -= h
        f = lambda t: oracle.log_likelihood(wl.tree.children, wl.n_tips, t, wl.Q, wl.pi, wl.rates,
                                            wl.cat_weights, wl.tips, wl.weights)
        fd = (f(tp) - f(tm)) / (2 * h)
        if abs(fd - g[c]) > 1e-5 * max(abs(g[c]), 1e-3) + 1e-6:
            return False
    return True


def test_unmutated_oracle_passes(wl):
    assert _lnl_ok(wl) and _grad_ok(wl)


def test_transposed_P_in_post_order_is_caught(wl, monkeypatch):
    monkeypatch.setattr(op, "_propagate", lambda Pc, x: np.matmul(x, Pc))
    assert not _lnl_ok(wl)


def test_P_instead_of_P_transpose_in_pre_order_is_caught(wl, monkeypatch):
    monkeypatch.setattr(op, "_propagate_transpose",
                        lambda Pc, x: np.matmul(x, np.transpose(Pc, (0, 2, 1))))
    assert not _grad_ok(wl)


def test_dropped_category_rate_in_gradient_is_caught(wl):
    assert not _grad_ok(wl, rates=np.ones_like(wl.rates))


def test_wrong_sign_of_Q_in_gradient_is_caught(wl):
    assert not _grad_ok(wl, Q=-wl.Q)


def test_transposed_Q_in_gradient_is_caught(wl):
    assert not _grad_ok(wl, Q=wl.Q.T.copy())


def test_uniform_root_frequencies_are_caught(wl, monkeypatch):
    orig = op.root_site_loglik
    monkeypatch.setattr(op, "root_site_loglik",
                        lambda post, ls, pi, w: orig(post, ls, np.full_like(pi, 0.25), w))
    assert not _lnl_ok(wl)


def test_dropped_log_scale_is_caught(wl, monkeypatch):
    orig = op.root_site_loglik
    monkeypatch.setattr(op, "root_site_loglik", lambda post, ls, pi, w: orig(post, 0 * ls, pi, w))
    assert not _lnl_ok(wl)


def test_unweighted_categories_are_caught(wl, monkeypatch):
    orig = op.root_site_loglik
    monkeypatch.setattr(op, "root_site_loglik", lambda post, ls, pi, w: orig(post, ls, pi, np.ones_like(w)))
    assert not _lnl_ok(wl)


def test_swapped_children_branch_lengths_are_caught(wl):
    # using the sibling's branch length for a child: swap t of the two children of one node
    n = wl.n_tips
    v = n  # first internal node in post-order numbering
    a, b = wl.tree.children[v]
    t = wl.t.copy()
    t[a], t[b] = t[b], t[a]
    lnl_good = oracle.log_likelihood(wl.tree.children, n, wl.t, wl.Q, wl.pi, wl.rates,
                                     wl.cat_weights, wl.tips, wl.weights)
    lnl_bad = oracle.log_likelihood(wl.tree.children, n, t, wl.Q, wl.pi, wl.rates,
                                    wl.cat_weights, wl.tips, wl.weights)
    assert abs(lnl_good - lnl_bad) > 1e-6
