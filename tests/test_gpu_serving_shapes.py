"""Parity at the serving clients' shapes: the sampled amino-acid clients against their stored
oracle results in every precision form, and the range limit of FP16 partials on the
835-taxon amino-acid client (131,036 patterns, shortest branch 7.3e-6)."""
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


def test_fp16_range_limit_reported_as_numeric():
    """FP16 keeps values down to 2^-24 of a pattern's maximum.  On client 17's tree two
    children are left with disjoint supports after that flush, so a site likelihood is
    exactly 0: the library reports HP_ERR_NUMERIC (lnL = -inf) on the blocking call and
    through the status word of the stream-ordered call, and clears the status after
    reporting it."""
    import torch
    from paper_2606_27607_amd import HPError, _lib
    wl, t = _client(17)
    announce(f"fp16 range limit, client 17 N={wl.n_tips} P={wl.n_patterns}")
    need = _lib.plan_pre_buffers(wl.tree.children)
    inst = make_instance(wl, "f16", "every_node", n_pre_partials=need)
    with pytest.raises(HPError) as e:
        inst.evaluate(t)
    assert e.value.code == _lib.HP_ERR_NUMERIC
    nb = 2 * wl.n_tips - 2
    out = inst.evaluate_device(torch.tensor(t[:nb], dtype=torch.float64, device="cuda"))
    with pytest.raises(HPError) as e:
        inst.status()
    assert e.value.code == _lib.HP_ERR_NUMERIC
    assert out[0].item() == -np.inf
    inst.status()                                   # reported once, then cleared
    inst.close()
