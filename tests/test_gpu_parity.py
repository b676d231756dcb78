"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Tolerances (gpu_helpers.TOL): FP64 on the GPU agrees with the oracle to rounding (1e-12
relative on lnL, 1e-11 of the largest gradient); FP32 meets the 1e-5 relative lnL bound and
its gradient error is bounded at 1e-5 of the largest gradient and 1e-4 relative on every
branch whose gradient is at least a tenth of the largest (per-pattern FP32 ratios carry
~1e-7 relative error; the observed gradient error is ~2e-7 of max |g|).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import (announce, check, golden, grad_err, make_instance, oracle_eval, post_ops, pre_ops,
                         rel)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# --------------------------------------------------------------- whole-tree evaluation

def test_nuc8_fp64_full_config():
    wl = synth.config_workload("nuc8")
    inst = make_instance(wl, "f64", "none")
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, "f64", what="nuc8")
    gold = golden("nuc8")
    if gold:
        check(lnl, gold["lnl"], g, np.array(gold["grad"]), "f64", what="nuc8 golden")


@pytest.mark.parametrize("precision,scaling,period", [("f64", "every_node", 1), ("f64", "every_k", 3),
                                                      ("f32", "every_k", 4), ("f32", "every_node", 1)])
@pytest.mark.parametrize("kind,n,npat,seed", [("gtr", 24, 1000, 1), ("hky", 9, 300, 2),
                                              ("gtr", 2, 77, 3), ("gtr", 60, 65, 4)])
def test_evaluate_matches_oracle(precision, scaling, period, kind, n, npat, seed):
    wl = synth.make_workload(kind, n, npat, seed=seed, unknown_frac=0.05)
    inst = make_instance(wl, precision, scaling, period)
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, precision)
    lnl_only = inst.evaluate(wl.t, want_grad=False)
    assert lnl_only == lnl


@pytest.mark.parametrize("K", [1, 3, 8])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_category_counts(K, precision):
    wl = synth.make_workload("gtr", 13, 200, seed=K, n_categories=K)
    inst = make_instance(wl, precision, "every_node")
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, precision)


@pytest.mark.parametrize("kind", ["bin", "three"])
def test_fewer_than_four_states(kind):
    wl = synth.make_workload(kind, 11, 130, seed=5, unknown_frac=0.1)
    inst = make_instance(wl, "f64", "every_node")
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, "f64")


def test_two_taxon_jc69_closed_form_on_gpu():
    from pins import jc69_two_taxon
    wl = synth.make_workload("jc69", 2, 16, seed=1, tree=synth.two_taxon_tree())
    wl.t[:] = [0.13, 0.31, 0.0]
    wl.tips = np.array([[a for a in range(4) for b in range(4)],
                        [b for a in range(4) for b in range(4)]], dtype=np.uint8)
    wl.weights = np.arange(1, 17, dtype=np.float64)
    inst = make_instance(wl, "f64", "none")
    lnl, g = inst.evaluate(wl.t)
    Ls, Ld, gs, gd = jc69_two_taxon(0.44, wl.rates, wl.cat_weights)
    same = wl.tips[0] == wl.tips[1]
    assert rel(lnl, np.sum(wl.weights * np.where(same, np.log(Ls), np.log(Ld)))) < 1e-13
    expect = np.sum(wl.weights * np.where(same, gs, gd))
    assert np.allclose(g, [expect, expect], rtol=1e-12)


def test_deep_caterpillar_needs_rescaling():
    """A 300-taxon ladder: without rescaling FP32 partials underflow; with it lnL stays within
    the FP32 tolerance."""
    wl = synth.make_workload("gtr", 300, 200, seed=6, tree=synth.caterpillar_tree(300),
                             branch_mean=0.1)
    lnl_o, _, g_o = oracle_eval(wl)
    inst = make_instance(wl, "f32", "every_k", 4)
    lnl, g = inst.evaluate(wl.t)
    check(lnl, lnl_o, g, g_o, "f32")
    inst64 = make_instance(wl, "f64", "every_k", 8)
    lnl64, g64 = inst64.evaluate(wl.t)
    check(lnl64, lnl_o, g64, g_o, "f64", scale=10)


def test_single_pattern_and_zero_branch():
    wl = synth.make_workload("hky", 7, 1, seed=7)
    wl.t[3] = 0.0
    inst = make_instance(wl, "f64", "every_node")
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, "f64")


# --------------------------------------------------------------- operation-level API

@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_op_level_api(precision):
    wl = synth.make_workload("gtr", 17, 333, seed=8, unknown_frac=0.05)
    inst = make_instance(wl, precision, "every_node", tree=False)
    N = wl.n_tips
    nb = 2 * N - 2
    inst.update_matrices(np.arange(nb), wl.t[:nb])
    inst.update_post(post_ops(wl.tree.children, N, rescale=1))
    lnl, site = inst.root_lnl(2 * N - 2, site=True)
    lnl_o, site_o, g_o = oracle_eval(wl)
    tol = 1e-12 if precision == "f64" else 1e-5
    assert rel(lnl, lnl_o) < tol
    assert np.allclose(site, site_o, rtol=tol, atol=0)
    g = inst.pre_gradients(pre_ops(wl.tree.children, N), nb)
    check(lnl, lnl_o, g, g_o, precision, what="op-level")
    # pre partials alone, then the same list again with gradients: same answer
    inst.update_pre(pre_ops(wl.tree.children, N))
    g2 = inst.pre_gradients(pre_ops(wl.tree.children, N), nb)
    assert np.array_equal(g, g2)


def test_partial_update_after_branch_change():
    """Change one branch, recompute only the path to the root: lnL equals a full evaluation."""
    wl = synth.make_workload("gtr", 20, 250, seed=9)
    inst = make_instance(wl, "f64", "every_node", tree=False)
    N = wl.n_tips
    nb = 2 * N - 2
    inst.update_matrices(np.arange(nb), wl.t[:nb])
    ops = post_ops(wl.tree.children, N)
    inst.update_post(ops)
    c = 5
    t2 = wl.t.copy()
    t2[c] *= 1.7
    inst.update_matrices([c], [t2[c]])
    path, v = [], c
    while v != 2 * N - 2:
        v = int(wl.tree.parent[v])
        path.append(v)
    sub = np.array([o for o in ops if o[0] in path], dtype=np.int32)
    inst.update_post(sub)
    lnl = inst.root_lnl(2 * N - 2)
    assert rel(lnl, oracle_eval(wl, t=t2, want_grad=False)[0]) < 1e-12


# --------------------------------------------------------------- determinism

def test_bitwise_repeatable_and_device_path():
    import torch
    wl = synth.make_workload("gtr", 40, 5000, seed=10)
    inst = make_instance(wl, "f32", "every_k", 4)
    a = inst.evaluate(wl.t)
    b = inst.evaluate(wl.t)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
    t_dev = torch.tensor(wl.t[: 2 * wl.n_tips - 2], dtype=torch.float64, device="cuda")
    out = inst.evaluate_device(t_dev)
    inst.status()
    o = out.cpu().numpy()
    assert o[0] == a[0] and np.array_equal(o[1:], a[1])
    # a second instance on another stream, interleaved: identical bits
    inst2 = make_instance(wl, "f32", "every_k", 4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out2 = inst2.evaluate_device(t_dev)
    out1 = inst.evaluate_device(t_dev)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)


# --------------------------------------------------------------- tile shapes (4-state path)

@pytest.fixture
def force_small_ppl(monkeypatch):
    """Force the 4-state traversal tile (64 or 128 patterns per workgroup) for instances
    created inside the test; the library reads the override at hp_create."""
    def force(ppl):
        monkeypatch.setenv("HIPPHYLO_SMALL_PPL", str(ppl))
    return force


@pytest.mark.parametrize("ppl", [1, 2])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("kind,n,npat,K,seed", [("gtr", 31, 333, 4, 1), ("hky", 5, 129, 3, 2),
                                                ("gtr", 70, 1, 4, 3), ("gtr", 17, 4100, 8, 4)])
def test_tile_shapes_match_oracle(force_small_ppl, ppl, precision, kind, n, npat, K, seed):
    """Both tiles, with ragged last tiles (333 = 2*128 + 77, 129 = 128 + 1, one pattern) and
    K = 3 and 8 categories, against the oracle; whole-tree and operation-level paths."""
    from paper_2606_27607_amd import _lib
    force_small_ppl(ppl)
    wl = synth.make_workload(kind, n, npat, seed=seed, n_categories=K, unknown_frac=0.05)
    inst = make_instance(wl, precision, "every_k", 2)
    assert inst.query(_lib.HP_Q_TILE) == 64 * ppl
    assert inst.query(_lib.HP_Q_BLOCKS) == -(-npat // (64 * ppl))
    assert inst.query(_lib.HP_Q_PATTERN_PAD) % 128 == 0
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, precision)
    tol = (1e-12, 1e-11) if precision == "f64" else (1e-5, 1e-5)
    nb = 2 * n - 2
    inst.update_matrices(np.arange(nb), wl.t[:nb])
    inst.update_post(post_ops(wl.tree.children, n, rescale=1))
    lnl2, site = inst.root_lnl(nb, site=True)
    _, site_o, _ = oracle_eval(wl, want_grad=False)
    assert rel(lnl2, lnl_o) < tol[0]
    assert np.allclose(site[:npat], site_o, rtol=tol[0] * 10, atol=0)


@pytest.mark.parametrize("K", [4, 8])
def test_small_walk_prefetch_forms_bitwise_equal(monkeypatch, K):
    """The FP32 4-state walk's two prefetch forms (the next operation's inputs loaded on every
    path, which instances on a half-filled device take, and the plain one) give bitwise the
    same lnL and gradients, in the fused, store and operation-level modes, and match the
    oracle."""
    import torch
    wl = synth.make_workload("gtr", 40, 3000, seed=[20260075, K], n_categories=K, unknown_frac=0.03)
    nb = 2 * wl.n_tips - 2
    out = []
    monkeypatch.setenv("HIPPHYLO_SMALL_PPL", "1")
    for pf in ("0", "1"):
        monkeypatch.setenv("HIPPHYLO_SMALL_PF", pf)
        announce(f"4-state prefetch form {pf}, K={K}")
        inst = make_instance(wl, "f32", "every_k", 4)
        lnl, g = inst.evaluate(wl.t)
        td = torch.tensor(wl.t[:nb], dtype=torch.float64, device=inst.device)
        fwd = inst.evaluate_device(td, want_grad=False).cpu().numpy()
        st = inst.gradients_device().cpu().numpy()
        inst.update_matrices(np.arange(nb), wl.t[:nb])
        inst.update_post(post_ops(wl.tree.children, wl.n_tips, rescale=1))
        lop = inst.root_lnl(nb)
        out.append((lnl, g, fwd, st, lop))
        inst.close()
    a, b = out
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3]) and a[4] == b[4]
    lnl_o, _, g_o = oracle_eval(wl)
    check(b[0], lnl_o, b[1], g_o, "f32", wl.n_states, what="every-path prefetch")


def test_tile_choice_and_batch_tile_check(force_small_ppl):
    """The automatic tile fills whole rounds: 131,072 patterns (2,048 one-pattern
    workgroups, more than the device holds at once in FP32) take the two-pattern tile, and
    instances of different tiles are not batched together."""
    import ctypes

    import torch
    from paper_2606_27607_amd import Instance, _lib
    big = Instance(8, 131072, 4, 4, precision="f32", scaling="every_k", scale_period=4)
    small = Instance(8, 1000, 4, 4, precision="f32", scaling="every_k", scale_period=4)
    assert big.query(_lib.HP_Q_TILE) == 128 and small.query(_lib.HP_Q_TILE) == 64
    wl = synth.make_workload("gtr", 8, 1000, seed=3)
    force_small_ppl(2)
    a = make_instance(wl, "f32", "every_k", 4)
    force_small_ppl(1)
    b = make_instance(wl, "f32", "every_k", 4)
    t = torch.tensor(np.r_[wl.t[:14], 0.0], dtype=torch.float64, device="cuda")
    out = torch.zeros(64, dtype=torch.float64, device="cuda")
    lib = _lib.load()
    rc = lib.hp_batch_evaluate_device((ctypes.c_void_p * 2)(a._inst.value, b._inst.value),
                                      (ctypes.c_void_p * 2)(t.data_ptr(), t.data_ptr()),
                                      (ctypes.c_void_p * 2)(out.data_ptr(), out.data_ptr()), 2, 1, None)
    assert rc == _lib.HP_ERR_UNSUPPORTED
    la, ga = a.evaluate(wl.t)
    lb, gb = b.evaluate(wl.t)
    assert rel(la, lb) < 1e-6 and grad_err(ga, gb) < 1e-4
    for inst in (big, small, a, b):
        inst.close()


# --------------------------------------------------------------- full-size configurations

@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_nuc128_full_size(precision):
    """The benchmark workload at full size (128 taxa, 100,000 patterns, rescaling every 4
    levels) against the stored full-size oracle result."""
    gold = golden("nuc128")
    if gold is None:
        pytest.skip("tests/golden/oracle_nuc128.json not generated")
    wl = synth.config_workload("nuc128")
    announce(f"nuc128 full size {precision}")
    inst = make_instance(wl, precision, "every_k", 4)
    lnl, g = inst.evaluate(wl.t)
    check(lnl, gold["lnl"], g, np.array(gold["grad"]), precision, what="nuc128 full size")
    tol_l = 1e-12 if precision == "f64" else 1e-5
    # sampled site log-likelihoods from the operation-level root call
    inst.update_matrices(np.arange(254), wl.t[:254])
    inst.update_post(post_ops(wl.tree.children, 128, rescale=1))
    lnl2, site = inst.root_lnl(254, site=True)
    idx = np.array(gold["site_idx"])
    assert np.allclose(site[idx], gold["site_lnl"], rtol=tol_l, atol=0)
    assert rel(lnl2, gold["lnl"]) < tol_l


# --------------------------------------------------------------- errors

def test_error_codes():
    from paper_2606_27607_amd import HPError
    from paper_2606_27607_amd import _lib
    wl = synth.make_workload("gtr", 6, 50, seed=11)
    inst = make_instance(wl, "f64", "every_node")
    t = wl.t.copy()
    t[2] = np.nan
    with pytest.raises(HPError) as e:
        inst.evaluate(t)
    assert e.value.code == _lib.HP_ERR_VALUE
    t[2] = -0.1
    with pytest.raises(HPError) as e:
        inst.update_matrices([2], [t[2]])
    assert e.value.code == _lib.HP_ERR_VALUE
    bad = wl.tips[0].copy()
    bad[3] = 9
    with pytest.raises(HPError) as e:
        inst.set_tip_states(0, bad)
    assert e.value.code == _lib.HP_ERR_VALUE
    with pytest.raises(HPError) as e:
        inst.update_post([[3, 0, 1, 1, 1, 1]])                 # dest is a tip
    assert e.value.code == _lib.HP_ERR_INDEX
    with pytest.raises(HPError) as e:
        inst.update_post([[6, 0, 99, 1, 1, 1]])                # matrix out of range
    assert e.value.code == _lib.HP_ERR_INDEX
    with pytest.raises(HPError) as e:
        inst.pre_gradients([[-1, 0, 0, -1, 0, 1, 1, -1, 0]], 10)  # slot used twice
    assert e.value.code == _lib.HP_ERR_ARG
    with pytest.raises(HPError) as e:
        inst.set_frequencies(np.full(4, 0.3))
    assert e.value.code == _lib.HP_ERR_VALUE
    from paper_2606_27607_amd import Instance
    blank = Instance(6, 50, 4, 4, precision="f64")
    with pytest.raises(HPError) as e:
        blank.evaluate(wl.t)
    assert e.value.code == _lib.HP_ERR_STATE
    # the instance still works after all the rejected calls
    lnl, g = inst.evaluate(wl.t)
    assert rel(lnl, oracle_eval(wl, want_grad=False)[0]) < 1e-12
    # device-side validation of branch lengths in the stream-ordered path
    import torch
    td = torch.tensor(np.r_[wl.t[:9], -1.0], dtype=torch.float64, device="cuda")
    inst.evaluate_device(td)
    with pytest.raises(HPError) as e:
        inst.status()
    assert e.value.code == _lib.HP_ERR_VALUE
    inst.status()                                               # cleared


@pytest.mark.parametrize("kind,n,npat,precision", [("gtr", 300, 700, "f32"), ("gtr", 64, 2000, "f64"),
                                                   ("gy94", 40, 300, "bf16"), ("aa", 90, 500, "f32")])
def test_minimal_pre_buffers_bitwise_equal(kind, n, npat, precision):
    """Whole-tree instances sized with hp_plan_pre_buffers (buffers reused along the pre-order
    walk) give exactly the results of instances with one pre-order buffer per node."""
    from paper_2606_27607_amd import _lib
    wl = synth.make_workload(kind, n, npat, seed=n, unknown_frac=0.05)
    need = _lib.plan_pre_buffers(wl.tree.children)
    assert need < n // 3
    sc = ("every_k", 4) if wl.n_states <= 4 else ("every_node", 1)
    full = make_instance(wl, precision, *sc)
    small = make_instance(wl, precision, *sc, n_pre_partials=need)
    assert small.workspace_bytes < full.workspace_bytes
    a, b = full.evaluate(wl.t), small.evaluate(wl.t)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
    with pytest.raises(Exception):
        make_instance(wl, precision, *sc, n_pre_partials=need - 1)


def test_op_level_calls_across_stream_switches():
    """Operation-level calls whose uploads are staged without waiting for the device give
    the same results when the caller's stream changes between them (the library completes
    the previous stream's work first) as on one stream."""
    import torch
    wl = synth.make_workload("gtr", 30, 700, seed=13)
    N = wl.n_tips
    nb = 2 * N - 2
    post, pre = post_ops(wl.tree.children, N), pre_ops(wl.tree.children, N)

    def run(inst, streams):
        out = []
        for rep, s in enumerate(streams):
            with torch.cuda.stream(s):
                t = wl.t[:nb] * (1.0 + 0.01 * rep)
                inst.update_matrices(np.arange(nb), t)
                inst.update_post(post)
                lnl = inst.root_lnl(2 * N - 2)
                out.append((lnl, inst.pre_gradients(pre, nb)))
        return out

    announce("op-level calls across stream switches gtr30x700 f32")
    one = run(make_instance(wl, "f32", "every_k", 4, tree=False), [torch.cuda.current_stream()] * 6)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    many = run(make_instance(wl, "f32", "every_k", 4, tree=False), [streams[i % 2] for i in range(6)])
    for (l1, g1), (l2, g2) in zip(one, many):
        assert l1 == l2 and np.array_equal(g1, g2)

    # switches between the stream-ordered calls themselves: the matrices are updated on stream
    # A behind a kernel that keeps A busy for about a millisecond, and everything after it is
    # issued on stream B without a host wait; the switch must order B after A's pending work
    def run_split(inst):
        out = []
        a, b = streams
        for rep in range(4):
            t = wl.t[:nb] * (1.0 + 0.01 * rep)
            lnl = torch.zeros(1, dtype=torch.float64, device="cuda")
            acc = torch.zeros(nb, dtype=torch.float64, device="cuda")
            with torch.cuda.stream(a):
                torch.cuda._sleep(2_000_000)
                inst.update_matrices(np.arange(nb), t)
            with torch.cuda.stream(b):
                inst.update_post(post)
                inst.root_lnl_device(2 * N - 2, lnl)
                inst.pre_gradients_device(pre, acc)
            torch.cuda.synchronize()
            out.append((lnl.item(), acc.cpu().numpy()))
        return out

    split = run_split(make_instance(wl, "f32", "every_k", 4, tree=False))
    for (l1, g1), (l2, g2) in zip(one[:4], split):
        assert l1 == l2 and np.array_equal(g1, g2)


@pytest.mark.parametrize("kind,precision", [("gtr", "f64"), ("gtr", "f32"), ("gy94", "bf16"), ("aa", "bf16x3")])
def test_op_level_device_calls_without_host_sync(kind, precision):
    """One full evaluation through the operation-level calls with every result left in
    device memory (hp_update_matrices, hp_update_post, hp_root_lnl_device with the site
    values, hp_pre_gradients_device), synchronised once at the end, against the oracle; then
    the same with a second category-weight slot holding other weights."""
    import torch
    wl = synth.make_workload(kind, 21, 700, seed=14, unknown_frac=0.05)
    inst = make_instance(wl, precision, "every_node", tree=False, n_eigen=2)
    N = wl.n_tips
    nb = 2 * N - 2
    post, pre = post_ops(wl.tree.children, N, rescale=1), pre_ops(wl.tree.children, N)
    w2 = np.array([0.4, 0.3, 0.2, 0.1])
    inst.set_category_weights(w2, idx=1)
    for slot, cw in ((0, wl.cat_weights), (1, w2)):
        announce(f"op-level device calls {kind} {precision} category-weight slot {slot}")
        lnl = torch.zeros(1, dtype=torch.float64, device="cuda")
        site = torch.zeros(wl.n_patterns, dtype=torch.float64, device="cuda")
        acc = torch.zeros(nb, dtype=torch.float64, device="cuda")
        inst.update_matrices(np.arange(nb), wl.t[:nb])
        inst.update_post(post)
        inst.root_lnl_device(2 * N - 2, lnl, site, catw_idx=slot)
        inst.pre_gradients_device(pre, acc, catw_idx=slot)
        torch.cuda.synchronize()
        inst.status()
        lnl_o, site_o, g_o = oracle.lnl_and_grad(wl.tree.children, N, wl.t, wl.Q, wl.pi, wl.rates, cw,
                                                 wl.tips, wl.weights)
        check(lnl.item(), lnl_o, acc.cpu().numpy(), g_o, precision, wl.n_states, what=f"device calls slot {slot}")
        s = site.cpu().numpy()
        assert np.max(np.abs(s - site_o)) < (1e-9 if precision == "f64" else 1e-3 if precision == "f32" else 0.05)
        # the blocking calls give the same numbers
        assert inst.root_lnl(2 * N - 2, catw_idx=slot) == lnl.item()
