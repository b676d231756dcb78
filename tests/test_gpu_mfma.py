"""GPU parity of the matrix-core path (4 < S <= 64: amino-acid and codon models) against the
FP64 oracle, in FP64, FP32, BF16 and FP16.

Tolerances (gpu_helpers.TOL): FP64 1e-12 relative on lnL and 1e-9 of max|g| (61-term
contractions at every node and pattern sums of both signs: observed ~2e-11); FP32 1e-5
relative on lnL and 1e-5 of max|g|; BF16/FP16 1e-4 relative on lnL (the mixed-precision
bound) and a stated gradient error, bounded at 1e-2 of max|g| for BF16 and 5e-3 for FP16
(16-bit partials carry 2^-9 / 2^-12 relative rounding per stored value).
"""
import numpy as np
import pytest

import synth
from gpu_helpers import TOL as _TOL, announce, check, golden, grad_err, make_instance, oracle_eval, post_ops, pre_ops, rel

pytestmark = pytest.mark.gpu

TOL = {p: _TOL["f64mc" if p == "f64" else p][:2] for p in ("f64", "f32", "bf16", "f16", "bf16x3")}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("kind,n,npat,seed", [("gy94", 12, 300, 1), ("aa", 17, 200, 2),
                                              ("gy94", 3, 37, 3), ("aa", 40, 130, 4)])
def test_evaluate_matches_oracle(precision, kind, n, npat, seed):
    wl = synth.make_workload(kind, n, npat, seed=seed, unknown_frac=0.05)
    inst = make_instance(wl, precision, "every_node")
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, precision, wl.n_states)
    assert inst.evaluate(wl.t, want_grad=False) == lnl


@pytest.mark.parametrize("S", [5, 13, 33, 64])
def test_odd_state_counts_fp64(S):
    rng = np.random.default_rng(S)
    pi = rng.dirichlet(np.ones(S) * 5)
    R = np.zeros((S, S))
    R[np.triu_indices(S, 1)] = rng.gamma(1.0, 1.0, S * (S - 1) // 2)
    Q = synth.models.reversible(R + R.T, pi)
    wl = synth.make_workload("gtr", 9, 90, seed=S)
    V, Vinv, lam = synth.eigensystem(Q, pi)
    wl.Q, wl.pi, wl.V, wl.Vinv, wl.lam = Q, pi, V, Vinv, lam
    wl.tips = rng.integers(0, S + 1, size=(9, 90)).astype(np.uint8)
    inst = make_instance(wl, "f64", "every_node")
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, "f64", S)


@pytest.mark.parametrize("precision", ["f32", "bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("K", [1, 6, 8])
def test_category_counts_mfma(K, precision):
    # K = 6 runs the 8-wave workgroups (one tile per wave), whose pending pre-order
    # partials also wait in LDS
    wl = synth.make_workload("gy94", 8, 100, seed=K, n_categories=K)
    inst = make_instance(wl, precision, "every_node")
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, precision, wl.n_states)


@pytest.mark.parametrize("precision", ["f64", "bf16"])
def test_op_level_api_mfma(precision):
    wl = synth.make_workload("gy94", 10, 150, seed=9, unknown_frac=0.05)
    inst = make_instance(wl, precision, "every_node", tree=False)
    N = wl.n_tips
    nb = 2 * N - 2
    inst.update_matrices(np.arange(nb), wl.t[:nb])
    inst.update_post(post_ops(wl.tree.children, N, rescale=1))
    lnl, site = inst.root_lnl(2 * N - 2, site=True)
    lnl_o, site_o, g_o = oracle_eval(wl)
    tl, tg = TOL[precision]
    assert rel(lnl, lnl_o) < tl
    # per-site log-likelihoods: absolute error in nats (BF16 partials round to 2^-9 at
    # every node, so a site carries ~sqrt(nodes) * 2^-9 of noise that averages out in lnL)
    site_tol = {"f64": 1e-9, "bf16": 0.05}[precision]
    err = np.abs(site - site_o).max()
    print(f"{precision}: max |site lnL error| {err:.3e} nats")
    assert err < site_tol
    g = inst.pre_gradients(pre_ops(wl.tree.children, N), nb)
    check(lnl, lnl_o, g, g_o, precision, wl.n_states, what="op-level")


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_op_level_more_tiles_than_resident_workgroups(precision):
    """Operation-level launches hold at most one workgroup per tile that the device keeps
    resident (768 for 64 padded states): 14,000 patterns (876 tiles) make workgroups walk a
    second tile in their grid-stride loop, and the reduction columns follow the launch."""
    from paper_2606_27607_amd import _lib
    wl = synth.make_workload("gy94", 5, 14000, seed=31, unknown_frac=0.05)
    inst = make_instance(wl, precision, "every_node", tree=False)
    announce(f"op-level gy94 N=5 P=14000 {precision}")
    N = wl.n_tips
    nb = 2 * N - 2
    inst.update_matrices(np.arange(nb), wl.t[:nb])
    inst.update_post(post_ops(wl.tree.children, N, rescale=1))
    lnl = inst.root_lnl(2 * N - 2)
    g = inst.pre_gradients(pre_ops(wl.tree.children, N), nb)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, precision, wl.n_states)
    assert inst.query(_lib.HP_Q_PATTERN_PAD) // 16 == 876


@pytest.mark.parametrize("kind,precision", [("aa", "f32"), ("gy94", "f16"), ("gy94", "bf16"), ("aa", "bf16x3")])
def test_many_tiles_per_workgroup_and_determinism(kind, precision):
    """More tile groups than the device holds workgroups at once: the launch is sized to the
    resident capacity and each workgroup loops over several groups."""
    from paper_2606_27607_amd import _lib
    npat = 40_000 if kind == "aa" else 24_000
    wl = synth.make_workload(kind, 6, npat, seed=10)
    inst = make_instance(wl, precision, "every_node")
    blocks = inst.query(_lib.HP_Q_BLOCKS)
    tiles = inst.query(_lib.HP_Q_PATTERN_PAD) // 16
    assert blocks < tiles // 2                      # several groups per workgroup
    a = inst.evaluate(wl.t)
    b = inst.evaluate(wl.t)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
    lnl_o, _, g_o = oracle_eval(wl)
    check(a[0], lnl_o, a[1], g_o, precision, wl.n_states)


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("policy", ["every_node", "benched"])
def test_codon64_full_size(precision, policy):
    """The codon workload at full size (64 taxa, 10,000 patterns) against the stored oracle
    result, with rescaling at every node and with the policy the benchmark runs
    (default_scaling: every 4 levels, every node for FP16 partials)."""
    from paper_2606_27607_amd import _lib
    gold = golden("codon64")
    if gold is None:
        pytest.skip("tests/golden/oracle_codon64.json not generated")
    wl = synth.config_workload("codon64")
    scaling = ("every_node", 1) if policy == "every_node" else _lib.default_scaling(wl.n_states, precision)
    announce(f"codon64 full size {precision} {scaling}")
    inst = make_instance(wl, precision, *scaling)
    lnl, g = inst.evaluate(wl.t)
    print(f"codon64 {precision} {scaling}: lnL rel err {rel(lnl, gold['lnl']):.3e}, "
          f"grad err {grad_err(g, np.array(gold['grad'])):.3e}")
    check(lnl, gold["lnl"], g, np.array(gold["grad"]), precision, wl.n_states, what=f"codon64 {scaling}")


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("kind,n,npat,seed", [("gy94", 360, 40, 21), ("aa", 530, 40, 22)])
def test_large_trees_and_periodic_rescaling(precision, kind, n, npat, seed):
    """Trees whose tip states exceed the workgroup's LDS staging (N x tile-group bytes over
    its staging bytes, so each operation copies its tip children's states from global memory
    into rows of the wave's own; FP64's one-tile groups still stage them all), each evaluated
    with rescaling every third level (post-order operations with no exchange between the
    category waves, exponents forwarded from the previous operation) and at every node
    (FP16 partials, with their 5-bit exponent, at every node only)."""
    wl = synth.make_workload(kind, n, npat, seed=seed, unknown_frac=0.05)
    lnl_o, _, g_o = oracle_eval(wl)
    policies = (("every_k", 3), ("every_node", 1)) if precision != "f16" else (("every_node", 1),)
    for scaling, period in policies:
        inst = make_instance(wl, precision, scaling, period)
        lnl, g = inst.evaluate(wl.t)
        check(lnl, lnl_o, g, g_o, precision, wl.n_states, what=scaling)
        inst.close()
