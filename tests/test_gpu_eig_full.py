"""The phylogeography-shaped workload (1000 taxa, 200 locations, one pattern, 4 categories)
on the eigensystem path against its stored full-size oracle result."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, golden, grad_err, make_instance, record, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tl,tg", [("f64", 1e-11, 1e-8), ("f32", 1e-5, 1e-3)])
def test_geo200_full_size(precision, tl, tg):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gold = golden("geo200")
    if gold is None:
        pytest.skip("tests/golden/oracle_geo200.json not generated")
    wl = synth.geo_workload()
    announce(f"geo200 full size {precision}")
    inst = make_instance(wl, precision, "every_node")
    lnl, g = inst.evaluate(wl.t)
    print(f"geo200 {precision}: lnL rel {rel(lnl, gold['lnl']):.2e} grad {grad_err(g, np.array(gold['grad'])):.2e}")
    record(what="geo200", lnl_rel=rel(lnl, gold["lnl"]), grad=grad_err(g, np.array(gold["grad"])))
    assert rel(lnl, gold["lnl"]) < tl
    assert grad_err(g, np.array(gold["grad"])) < tg
