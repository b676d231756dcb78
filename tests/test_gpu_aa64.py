"""The 64-taxon amino-acid workload (20 states, 10,000 patterns) at full size: FP32 and the
20-state mixed form (FP32 partials with split-BF16 products, bf16x3) against the stored
FP64 oracle values, at the rescaling policy the benchmark uses, and FP16 partials (every
node rescaled) at the 16-bit bounds."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, check, golden, make_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision", ["f32", "bf16x3", "f16"])
def test_aa64_full_size(precision):
    from paper_2606_27607_amd import default_scaling
    gold = golden("aa64")
    if gold is None:
        pytest.skip("tests/golden/oracle_aa64.json not generated")
    wl = synth.config_workload("aa64")
    assert wl.n_states == 20 and gold["n_patterns"] == wl.n_patterns
    sc = default_scaling(wl.n_states, precision)
    announce(f"aa64 full size {precision} {sc}")
    inst = make_instance(wl, precision, *sc)
    lnl, g = inst.evaluate(wl.t[:2 * wl.n_tips - 2])
    check(lnl, gold["lnl"], g, np.array(gold["grad"]), precision, wl.n_states, what=f"aa64 {precision}")
