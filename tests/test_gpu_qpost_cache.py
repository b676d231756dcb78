"""The Q . post cache (HP_FLAG_QPOST_CACHE) of the operation-level matrix-core calls: the
post-order pass keeps w_v = Q post_v beside every post-order buffer, the matrix kernel the
tip columns (Q P)[:, s], and the gradient numerators are read from them instead of forming
Q P post.  Gradients against the oracle (the cache changes no partial, so lnL is bitwise the
uncached one) in every precision form, with unknown tips, 1 to 6 categories, a gradient list
whose internal children keep no pre-order partial, and the full codon configuration."""
import numpy as np
import pytest

import synth
from gpu_helpers import (TOL, announce, check, golden, make_instance, oracle_eval, post_ops, pre_ops,
                         record, rel, tol_key)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _op_eval(inst, wl, post, pre):
    N = wl.n_tips
    nb = 2 * N - 2
    inst.update_matrices(np.arange(nb), wl.t[:nb])
    inst.update_post(post)
    lnl = inst.root_lnl(2 * N - 2)
    return lnl, inst.pre_gradients(pre, nb)


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("kind,n,npat,K,seed", [("gy94", 11, 400, 4, 41), ("aa", 17, 700, 1, 42),
                                                ("gy94", 6, 90, 6, 43)])
def test_cached_gradients_match_oracle(precision, kind, n, npat, K, seed):
    wl = synth.make_workload(kind, n, npat, seed=seed, n_categories=K, unknown_frac=0.05)
    announce(f"qpost cache {kind} N={n} P={npat} K={K} {precision}")
    N = wl.n_tips
    post, pre = post_ops(wl.tree.children, N, rescale=1), pre_ops(wl.tree.children, N)
    cached = make_instance(wl, precision, "every_node", tree=False, qpost_cache=True)
    plain = make_instance(wl, precision, "every_node", tree=False)
    lnl, g = _op_eval(cached, wl, post, pre)
    lnl_p, g_p = _op_eval(plain, wl, post, pre)
    lnl_o, _, g_o = oracle_eval(wl)
    assert lnl == lnl_p                       # the cache leaves every partial as it was
    check(lnl, lnl_o, g, g_o, precision, wl.n_states, what=f"qpost cache {kind}")


@pytest.mark.parametrize("precision", ["f64", "bf16"])
def test_root_children_without_stored_pre_partials(precision):
    """One pre-order operation at the root with both children's pre-order destinations
    omitted (-1): an internal child's numerator still needs P_c^T v, which the kernel then
    forms for the gradient alone.  Both root-branch gradients against the oracle, as a fraction
    of the largest gradient of the tree (the error measure of every gradient check), and
    against the same list without the cache."""
    wl = synth.make_workload("gy94", 12, 300, seed=44, unknown_frac=0.05)
    N = wl.n_tips
    root = 2 * N - 2
    a, b = (int(c) for c in wl.tree.children[root])
    assert a >= N or b >= N
    inst = make_instance(wl, precision, "every_node", tree=False, qpost_cache=True)
    nb = 2 * N - 2
    inst.update_matrices(np.arange(nb), wl.t[:nb])
    inst.update_post(post_ops(wl.tree.children, N, rescale=1))
    lnl = inst.root_lnl(root)
    op = np.array([[-1, a, a, -1, a, b, b, -1, b]], dtype=np.int32)
    g = inst.pre_gradients(op, nb)
    lnl_o, _, g_o = oracle_eval(wl)
    sel = [a, b]
    assert np.all(np.delete(g, sel) == 0.0)
    tl, tg, tb = TOL[tol_key(precision, wl.n_states)]
    e_l, e_g = rel(lnl, lnl_o), float(np.max(np.abs(g[sel] - g_o[sel])) / np.max(np.abs(g_o)))
    record(what="root branches, cached", key=tol_key(precision, wl.n_states), lnl_rel=e_l, grad=e_g)
    assert e_l < tl and e_g < tg, (e_l, e_g)
    plain = make_instance(wl, precision, "every_node", tree=False)
    plain.update_matrices(np.arange(nb), wl.t[:nb])
    plain.update_post(post_ops(wl.tree.children, N, rescale=1))
    g_p = plain.pre_gradients(op, nb)
    assert np.max(np.abs(g[sel] - g_p[sel])) / np.max(np.abs(g_o)) < tg


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_codon64_full_size_cached(precision):
    """The 64-taxon codon configuration through the operation-level calls with the cache, at
    the rescaling policy the benchmark uses, against the stored oracle values."""
    from paper_2606_27607_amd import _lib, default_scaling
    gold = golden("codon64")
    if gold is None:
        pytest.skip("tests/golden/oracle_codon64.json not generated")
    wl = synth.config_workload("codon64")
    sc = default_scaling(wl.n_states, precision)
    post, pre = _lib.plan_tree(wl.tree.children, *sc)
    announce(f"qpost cache codon64 {precision} {sc}")
    inst = make_instance(wl, precision, *sc, tree=False, qpost_cache=True,
                         n_pre_partials=_lib.plan_pre_buffers(wl.tree.children))
    lnl, g = _op_eval(inst, wl, post, pre)
    check(lnl, gold["lnl"], g, np.array(gold["grad"]), precision, wl.n_states, what="codon64 cached")
