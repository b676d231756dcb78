"""The likelihood as a torch.autograd.Function over branch lengths: gradcheck (central finite
differences, h = 1e-6, FP64) on the GPU path, the three backward modes against each other
and against the oracle gradient, including both differentiation workloads at full size."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, check, golden, grad_err, make_instance, oracle_eval, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("mode", ["store", "recompute", "fused"])
@pytest.mark.parametrize("kind,n,npat", [("gtr", 7, 40), ("gy94", 4, 20)])
def test_gradcheck_fp64(mode, kind, n, npat):
    import torch
    from paper_2606_27607_amd.autograd import BranchLengthLnL
    wl = synth.make_workload(kind, n, npat, seed=3, unknown_frac=0.05)
    inst = make_instance(wl, "f64", "every_node")
    t = torch.tensor(wl.t[: 2 * n - 2], dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: BranchLengthLnL.apply(x, inst, mode), (t,), eps=1e-6,
                                    atol=1e-6, rtol=1e-5, nondet_tol=0.0)
    # and against the oracle gradient
    out = BranchLengthLnL.apply(t, inst, mode)
    (g,) = torch.autograd.grad(2.0 * out, t)
    lnl_o, _, g_o = oracle_eval(wl)
    assert rel(out.item(), lnl_o) < 1e-12
    assert grad_err(g.cpu().numpy() / 2.0, g_o) < 1e-9


def test_modes_agree_bitwise_and_store_detects_reuse():
    import torch
    from paper_2606_27607_amd.autograd import BranchLengthLnL
    wl = synth.make_workload("gtr", 40, 3000, seed=5)
    inst = make_instance(wl, "f32", "every_k", 4)
    t = torch.tensor(wl.t[:78], dtype=torch.float64, device="cuda", requires_grad=True)
    grads = {}
    for mode in ("store", "recompute", "fused"):
        out = BranchLengthLnL.apply(t, inst, mode)
        (grads[mode],) = torch.autograd.grad(out, t)
    assert torch.equal(grads["store"], grads["recompute"])
    assert torch.equal(grads["store"], grads["fused"])
    # forward at t, then another forward at t2 on the same instance, then backward of the
    # first: store mode must notice and recompute at t
    out1 = BranchLengthLnL.apply(t, inst, "store")
    t2 = (t.detach() * 1.3).requires_grad_(True)
    out2 = BranchLengthLnL.apply(t2, inst, "store")
    (g1,) = torch.autograd.grad(out1, t)
    assert torch.equal(g1, grads["store"])
    (g2,) = torch.autograd.grad(out2, t2)
    assert not torch.equal(g2, g1)


@pytest.mark.parametrize("name,precision,policy", [("nuc256", "f32", "benched"), ("codon32", "bf16", "benched"),
                                                  ("codon32", "bf16", "every_node")])
@pytest.mark.parametrize("mode", ["store", "recompute", "checkpoint"])
def test_differentiation_workloads_full_size(name, precision, policy, mode):
    """The differentiation workloads at full size against the stored oracle results, with
    the rescaling policy the benchmark runs (default_scaling: every 4 levels) and, for the
    codon tree, at every node."""
    import torch
    from paper_2606_27607_amd.autograd import BranchLengthLnL
    gold = golden(name)
    if gold is None:
        pytest.skip(f"tests/golden/oracle_{name}.json not generated")
    wl = synth.config_workload(name)
    announce(f"{name} full size {precision} {mode} {policy}")
    from paper_2606_27607_amd import _lib
    scaling = _lib.default_scaling(wl.n_states, precision) if policy == "benched" else ("every_node", 1)
    if mode == "checkpoint":
        # post-order partials kept every 4 levels, the rest recomputed in the backward pass
        from paper_2606_27607_amd.checkpoint import Checkpointed
        inst = Checkpointed.create(wl.n_tips, wl.n_patterns, wl.n_states, wl.n_categories, wl.tree.children,
                                   4, precision=precision, scaling=scaling[0], scale_period=scaling[1])
        inst.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights)
    else:
        inst = make_instance(wl, precision, *scaling)
    nb = 2 * wl.n_tips - 2
    t = torch.tensor(wl.t[:nb], dtype=torch.float64, device="cuda", requires_grad=True)
    out = BranchLengthLnL.apply(t, inst, mode)
    (g,) = torch.autograd.grad(out, t)
    g = g.cpu().numpy()
    print(f"{name} {precision} {mode}: lnL rel {rel(out.item(), gold['lnl']):.3e} "
          f"grad err {grad_err(g, np.array(gold['grad'])):.3e}")
    check(out.item(), gold["lnl"], g, np.array(gold["grad"]), precision, wl.n_states, what=f"{mode} {scaling}")
