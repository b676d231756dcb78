"""GPU parity of the eigensystem path (64 < S <= 254, few patterns: phylogeography) against
the FP64 oracle: state counts, category counts, one or several patterns, unknown tips,
deep trees that need rescaling on both passes, lnL-only evaluations, and the calls the path
does not offer."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, grad_err, make_instance, oracle_eval, record, rel

pytestmark = pytest.mark.gpu

TOL = {"f64": (1e-11, 1e-8), "f32": (1e-5, 1e-3)}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("S,n,npat,K,seed", [(65, 17, 3, 4, 1), (100, 40, 1, 4, 2), (200, 20, 2, 2, 3),
                                             (254, 8, 1, 1, 4), (120, 2, 1, 3, 5), (100, 300, 1, 1, 6),
                                             (80, 12, 2, 8, 7)])
def test_matches_oracle(precision, S, n, npat, K, seed):
    wl = synth.make_workload("geo", n, npat, seed=seed, n_categories=K, n_states=S, unknown_frac=0.1)
    inst = make_instance(wl, precision, "every_node")
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    tl, tg = TOL[precision]
    print(f"S={S} N={n} P={npat} K={K} {precision}: lnL rel {rel(lnl, lnl_o):.2e} grad {grad_err(g, g_o):.2e}")
    record(what="eig", lnl_rel=rel(lnl, lnl_o), grad=grad_err(g, g_o))
    assert rel(lnl, lnl_o) < tl and grad_err(g, g_o) < tg
    assert inst.evaluate(wl.t, want_grad=False) == lnl


def test_deep_caterpillar_rescales_both_passes():
    """A 150-taxon caterpillar (height 149): partials would leave FP64's range without the
    per-level power-of-two rescaling of post- and pre-order vectors."""
    wl = synth.make_workload("geo", 150, 1, seed=7, n_states=80, tree=synth.caterpillar_tree(150),
                             branch_mean=0.5)
    inst = make_instance(wl, "f64", "every_node")
    lnl, g = inst.evaluate(wl.t)
    lnl_o, _, g_o = oracle_eval(wl)
    assert np.isfinite(lnl) and rel(lnl, lnl_o) < 1e-10 and grad_err(g, g_o) < 1e-8


def test_device_form_and_unsupported_calls():
    import torch
    from paper_2606_27607_amd import HPError, _lib
    wl = synth.make_workload("geo", 12, 2, seed=8, n_states=90)
    inst = make_instance(wl, "f64", "every_node")
    lnl, g = inst.evaluate(wl.t)
    nb = 2 * wl.n_tips - 2
    t = torch.tensor(wl.t[:nb], dtype=torch.float64, device="cuda")
    out = inst.evaluate_device(t)
    torch.cuda.synchronize()
    inst.status()
    assert out[0].item() == lnl and np.array_equal(out[1:].cpu().numpy(), g)
    for call in (lambda: inst.update_matrices([0], [0.1]), lambda: inst.evaluate_rate_gradient(wl.t),
                 lambda: inst.update_post([[12, 0, 0, 1, 1, 1]])):
        with pytest.raises(HPError) as e:
            call()
        assert e.value.code == _lib.HP_ERR_UNSUPPORTED
    bad = wl.t.copy()
    bad[3] = -1.0
    with pytest.raises(HPError) as e:
        inst.evaluate(bad)
    assert e.value.code == _lib.HP_ERR_VALUE
