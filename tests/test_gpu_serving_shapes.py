"""Parity at the serving clients' shapes: the sampled amino-acid clients against their stored
oracle results in every precision form, FP16 partials on the 835-taxon amino-acid client
(131,036 patterns, shortest branch 7.3e-6) against FP32, and how zero site likelihoods are
reported."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, check, golden, grad_err, make_instance, record, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _client(c):
    wl = synth.serving_workload(c)
    t = synth.serving_requests(wl, c)[0]
    return wl, np.r_[t, 0.0]


@pytest.mark.parametrize("precision", ["f32", "bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("client", [36, 47])
def test_amino_acid_serving_sample(client, precision):
    """Clients 36 (26 taxa x 12,431 patterns) and 47 (22 taxa x 119 patterns), first
    request, at the rescaling policy the server uses.  BF16 partials round to 2^-9 at every
    stored node, and on these small trees many patterns repeat, so their rounding does not
    average out: BF16 at 20 states is measured at 1.3e-4 to 1.4e-4 on lnL and is held to
    3e-4 here; it is not the form the server runs for 20 states."""
    from paper_2606_27607_amd import default_scaling
    gold = golden("serving")
    if gold is None or str(client) not in gold:
        pytest.skip("tests/golden/oracle_serving.json not generated")
    ref = gold[str(client)]
    wl, t = _client(client)
    assert (wl.n_tips, wl.n_patterns, wl.n_states) == (ref["n_tips"], ref["n_patterns"], 20)
    inst = make_instance(wl, precision, *default_scaling(wl.n_states, precision))
    lnl, g = inst.evaluate(t)
    g_o = np.array(ref["grad"])
    if precision == "bf16":
        e_l, e_g = rel(lnl, ref["lnl"]), grad_err(g, g_o)
        record(what=f"serving client {client}", key="bf16-20-states", lnl_rel=e_l, grad=e_g)
        assert e_l < 3e-4 and e_g < 1e-2, (e_l, e_g)
    else:
        check(lnl, ref["lnl"], g, g_o, precision, wl.n_states, what=f"serving client {client}")


def test_fp16_client17_in_range_with_per_category_rescaling():
    """FP16 keeps values down to 2^-24 of whatever its rescaling normalises to.  On client
    17 (835 amino-acid taxa, 131,036 patterns, shortest branch 7.3e-6), a power of two shared
    by all four categories left the slowest category's partials flushed to zero and some site
    likelihoods exactly 0.  The whole-tree walk rescales each category on its own, so the
    FP16 evaluation stays finite, and its lnL agrees with the FP32 one (itself held to 1e-5 of
    the oracle elsewhere) within 1e-4.  Its gradients carry the rounding of 11-bit partials
    stored at every node of a tree this deep (measured 1.7e-2 of max |g| against FP32), so they
    are held to 5e-2 here; FP16 is not a served form for 20 states."""
    import torch
    from paper_2606_27607_amd import _lib
    wl, t = _client(17)
    announce(f"fp16 range, client 17 N={wl.n_tips} P={wl.n_patterns}")
    need = _lib.plan_pre_buffers(wl.tree.children)
    res = {}
    for precision, scaling in (("f16", "every_node"), ("f32", "every_k")):
        inst = make_instance(wl, precision, scaling, n_pre_partials=need)
        res[precision] = inst.evaluate(t)
        inst.close()
        del inst
        torch.cuda.empty_cache()
    (l16, g16), (l32, g32) = res["f16"], res["f32"]
    assert np.isfinite(l16) and np.isfinite(g16).all()
    e_l, e_g = rel(l16, l32), grad_err(g16, g32)
    record(what="client 17 f16 vs f32", key="f16", lnl_rel=e_l, grad=e_g)
    assert e_l < 1e-4 and e_g < 5e-2, (e_l, e_g)


@pytest.mark.parametrize("precision", ["f32", "bf16", "f16"])
def test_zero_site_likelihood_reported_as_numeric(precision):
    """With every category weight 0 each weighted site likelihood is exactly 0: the library
    reports HP_ERR_NUMERIC (lnL = -inf) on the blocking call and through the status word of
    the stream-ordered call, and clears the status after reporting it."""
    import torch
    from paper_2606_27607_amd import HPError, _lib
    wl = synth.make_workload("gy94", 10, 300, seed=[20260073, 1])
    announce(f"zero site likelihood, gy94 10x300 {precision}")
    inst = make_instance(wl, precision, "every_k", 4)
    inst.set_category_weights(np.zeros(wl.n_categories))
    with pytest.raises(HPError) as e:
        inst.evaluate(wl.t)
    assert e.value.code == _lib.HP_ERR_NUMERIC
    nb = 2 * wl.n_tips - 2
    out = inst.evaluate_device(torch.tensor(wl.t[:nb], dtype=torch.float64, device="cuda"))
    with pytest.raises(HPError) as e:
        inst.status()
    assert e.value.code == _lib.HP_ERR_NUMERIC
    assert out[0].item() == -np.inf
    inst.status()                                   # reported once, then cleared
    inst.set_category_weights(wl.cat_weights)
    lnl, _ = inst.evaluate(wl.t)
    assert np.isfinite(lnl)
