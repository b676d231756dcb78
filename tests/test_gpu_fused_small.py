"""The one-launch evaluation of small 4-state problems: every workgroup forms the transition
matrices in LDS, walks its 64 patterns with partials in LDS, and the last workgroup sums the
reduction rows in the fixed order of the reduction kernel.  It must give bitwise the results
of the three-launch evaluation (hp_evaluate_device_noalloc always takes that path) and of the
oracle within the usual bounds, launch exactly one kernel, keep its workgroup counter right
across calls, and report invalid branch lengths and zero site likelihoods as before."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, check, make_instance, oracle_eval

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _three_launch(inst, t):
    import torch
    td = torch.tensor(np.asarray(t, dtype=np.float64), device=inst.device)
    return inst.evaluate_device_noalloc(td, want_grad=True).cpu().numpy()


CASES = [("nuc8", "hky", 8, 1000, 4, "f64", "every_k"), ("hky16", "hky", 16, 3000, 4, "f32", "every_k"),
         ("gtr24", "gtr", 24, 2500, 8, "f64", "every_node"), ("bin12", "bin", 12, 700, 1, "f32", "none"),
         ("three9", "three", 9, 64, 3, "f64", "none"), ("gtr40", "gtr", 40, 4000, 4, "f32", "every_k"),
         # the smallest trees: 2 taxa (one operation each way, no pre-order buffer) and 3
         ("gtr2", "gtr", 2, 200, 4, "f64", "every_k"), ("gtr3", "gtr", 3, 130, 4, "f32", "every_node")]


@pytest.mark.parametrize("name,kind,n,npat,K,precision,scaling", CASES)
def test_one_launch_equals_three_launches_and_oracle(name, kind, n, npat, K, precision, scaling, monkeypatch):
    # the one launch walks 64 patterns per workgroup: keep the instance's tile there (hp_create
    # may otherwise choose 128 for a single workgroup of patterns)
    monkeypatch.setenv("HIPPHYLO_SMALL_PPL", "1")
    if name == "nuc8":
        wl = synth.config_workload("nuc8")
    else:
        wl = synth.make_workload(kind, n, npat, seed=[20260074, n], n_categories=K, unknown_frac=0.03)
    announce(f"one-launch {name} {precision} {scaling}")
    inst = make_instance(wl, precision, scaling, 1 if scaling == "every_k" else 4)
    nb = 2 * wl.n_tips - 2
    rng = np.random.default_rng(n)
    for rep in range(3):                          # the workgroup counter must reset each time
        t = wl.t[:nb] * np.exp(0.05 * rng.standard_normal(nb))
        inst.profile(True)
        inst.profile_read()
        lnl, g = inst.evaluate(t)
        prof = inst.profile_read()
        inst.profile(False)
        assert prof["traversal"][1] == 1 and prof["pmat"][1] == 0 and prof["reduce"][1] == 0, prof
        ref = _three_launch(inst, t)
        assert lnl == ref[0] and np.array_equal(g, ref[1:]), (rep, lnl - ref[0], np.max(np.abs(g - ref[1:])))
        import torch
        out = inst.evaluate_device(torch.tensor(t, device=inst.device), want_grad=True).cpu().numpy()
        inst.status()
        assert np.array_equal(out, ref)
    lnl_o, _, g_o = oracle_eval(wl, t)
    check(lnl, lnl_o, g, g_o, precision, wl.n_states, what=f"one-launch {name}")


def test_without_gradients_and_large_problems_take_three_launches():
    """lnL only (the store-mode backward reads the partials it leaves) and 128 workgroups of
    patterns are evaluated by the three launches."""
    wl = synth.make_workload("hky", 10, 8192 + 64, seed=[20260074, 99])
    inst = make_instance(wl, "f32", "every_k", 4)
    nb = 2 * wl.n_tips - 2
    for want_grad in (False, True):
        inst.profile(True)
        inst.profile_read()
        inst.evaluate(wl.t[:nb], want_grad=want_grad)
        prof = inst.profile_read()
        inst.profile(False)
        assert prof["pmat"][1] == 1 and prof["reduce"][1] == 1, (want_grad, prof)


def test_errors_in_one_launch():
    """A negative branch length given on the device raises the status word (HP_ERR_VALUE) and
    gives NaN; zero category weights give HP_ERR_NUMERIC on the blocking call (the status
    word written by the kernel into host memory), which clears the status."""
    import torch
    from paper_2606_27607_amd import HPError, _lib
    wl = synth.config_workload("nuc8")
    inst = make_instance(wl, "f64", "every_k", 1)
    nb = 2 * wl.n_tips - 2
    bad = wl.t[:nb].copy()
    bad[3] = -0.1
    out = inst.evaluate_device(torch.tensor(bad, device=inst.device), want_grad=True)
    with pytest.raises(HPError) as e:
        inst.status()
    assert e.value.code == _lib.HP_ERR_VALUE
    assert np.isnan(out.cpu().numpy()).any()
    inst.status()
    inst.set_category_weights(np.zeros(wl.n_categories))
    with pytest.raises(HPError) as e:
        inst.evaluate(wl.t[:nb])
    assert e.value.code == _lib.HP_ERR_NUMERIC
    inst.status()                                     # nothing left pending
    inst.set_category_weights(wl.cat_weights)
    lnl, g = inst.evaluate(wl.t[:nb])
    lnl_o, _, g_o = oracle_eval(wl)
    check(lnl, lnl_o, g, g_o, "f64", what="one-launch nuc8 after errors")
