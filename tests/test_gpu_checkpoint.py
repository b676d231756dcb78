"""GPU parity of checkpointed gradients (post-order partials kept at every m-th level only,
the rest recomputed in the backward pass) against the FP64 oracle and the store-mode
whole-tree evaluation, through the operation-level calls."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import TOL as _TOL, announce, check, grad_err, make_instance, oracle_eval, rel

pytestmark = pytest.mark.gpu

TOL = {p: _TOL["f64mc" if p == "f64" else p][:2] for p in ("f64", "f32", "bf16")}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def checkpointed(wl, period, precision, scaling, scale_period):
    from paper_2606_27607_amd.checkpoint import Checkpointed
    announce(f"checkpointed {wl.name} N={wl.n_tips} P={wl.n_patterns} S={wl.n_states} m={period} {precision}")
    ck = Checkpointed.create(wl.n_tips, wl.n_patterns, wl.n_states, wl.n_categories, wl.tree.children, period,
                             precision=precision, scaling=scaling, scale_period=scale_period)
    return ck.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights)


@pytest.mark.parametrize("kind,n,npat,precision,period", [
    ("gtr", 40, 300, "f64", 2), ("gtr", 40, 300, "f64", 3), ("hky", 64, 500, "f32", 4),
    ("aa", 30, 120, "f32", 2), ("gy94", 24, 80, "bf16", 3)])
def test_checkpointed_matches_oracle_and_store(kind, n, npat, precision, period):
    wl = synth.make_workload(kind, n, npat, seed=n + period, unknown_frac=0.05)
    scaling, sp = ("every_k", 2) if wl.n_states == 4 else ("every_node", 1)
    ck = checkpointed(wl, period, precision, scaling, sp)
    assert ck.plan.n_post_buffers < n - 1
    lnl = ck.lnl(wl.t)
    g = ck.gradients()
    lnl_o, _, g_o = oracle_eval(wl)
    tl, tg = TOL[precision]
    check(lnl, lnl_o, g, g_o, precision, wl.n_states)
    # store mode runs the whole-tree kernel, which rounds differently (16-bit paths store
    # u = P post instead of post): both are within the oracle tolerance, so within twice it
    # of each other
    store = make_instance(wl, precision, scaling, sp)
    lnl_s, g_s = store.evaluate(wl.t)
    assert rel(lnl, lnl_s) < 2 * tl and grad_err(g, g_s) < 2 * tg
    # a second evaluation at other branch lengths reuses the plan and the buffers
    t2 = wl.t * 1.3
    lnl2 = ck.lnl(t2)
    g2 = ck.gradients()
    lnl2_o, _, g2_o = oracle_eval(wl, t=t2)
    check(lnl2, lnl2_o, g2, g2_o, precision, wl.n_states, what="second evaluation")


def test_device_accumulation_equals_host_batches():
    """The stream-ordered pre-order gradient batches summed on the device give bitwise the
    host-returned batches summed on the host (each slot gains exactly one nonzero term)."""
    wl = synth.make_workload("gtr", 48, 400, seed=4)
    ck = checkpointed(wl, 3, "f32", "every_k", 2)
    ck.lnl(wl.t)
    g_dev = ck.gradients()
    nb = 2 * wl.n_tips - 2
    ck.lnl(wl.t)                 # the backward pass consumes the forward pass's buffers
    g_host = np.zeros(nb)
    for kind, ops in ck.plan.steps:
        if kind == "post":
            ck.inst.update_post(ops)
        else:
            g_host += ck.inst.pre_gradients(ops, nb)
    assert np.array_equal(g_dev, g_host)
    # a list that names no slot adds zero everywhere
    acc = torch.arange(nb, dtype=torch.float64, device="cuda")
    ck.inst.pre_gradients_device(np.zeros((0, 9), dtype=np.int32), acc)
    assert torch.equal(acc.cpu(), torch.arange(nb, dtype=torch.float64))


def test_checkpoint_autograd_mode():
    from paper_2606_27607_amd import autograd
    wl = synth.make_workload("gtr", 20, 150, seed=5)
    ck = checkpointed(wl, 2, "f64", "every_k", 2)
    t = torch.tensor(wl.t[: 2 * wl.n_tips - 2], dtype=torch.float64, device="cuda", requires_grad=True)
    out = autograd.lnl(t, ck, mode="checkpoint")
    (3.0 * out).backward()
    lnl_o, _, g_o = oracle_eval(wl)
    assert rel(out.item(), lnl_o) < 1e-12
    assert grad_err(t.grad.cpu().numpy() / 3.0, g_o) < 1e-9


@pytest.mark.parametrize("kind,n,npat,precision,period", [
    ("gtr", 70, 3000, "f64", 3), ("gtr", 70, 3000, "f32", 4), ("gtr", 70, 3000, "f32", 1000),
    ("gy94", 26, 500, "bf16", 3), ("gy94", 26, 500, "f32", 2), ("gy94", 18, 200, "f64", 2),
    ("aa", 30, 700, "bf16x3", 3), ("aa", 30, 700, "f16", 2)])
def test_one_launch_backward_equals_stepwise_calls(kind, n, npat, precision, period):
    """The backward pass runs as one mixed list (hp_traverse_gradients_device: the 4-state
    walk, or the operation-level matrix-core walk for 20 and 61 states); the same operations
    as step-wise hp_update_post / hp_pre_gradients_device calls give bitwise the same
    gradients, and one launch is all the backward pass issues."""
    wl = synth.make_workload(kind, n, npat, seed=[20260075, period, n], unknown_frac=0.02)
    from paper_2606_27607_amd import default_scaling
    ck = checkpointed(wl, period, precision, *default_scaling(wl.n_states, precision))
    nb = 2 * wl.n_tips - 2
    ck.lnl(wl.t)
    inst = ck.inst
    inst.profile(True)
    inst.profile_read()
    g_one = ck.gradients()
    prof = inst.profile_read()
    inst.profile(False)
    assert prof["traversal"][1] == 1 and prof["reduce"][1] == 1, prof
    ck.lnl(wl.t)
    acc = torch.zeros(nb, dtype=torch.float64, device=inst.device)
    for kind, ops in ck.plan.steps:
        if kind == "post":
            inst.update_post(ops)
        else:
            inst.pre_gradients_device(ops, acc)
    g_steps = acc.cpu().numpy()
    assert np.array_equal(g_one, g_steps), np.max(np.abs(g_one - g_steps))
    lnl_o, _, g_o = oracle_eval(wl)
    check(ck.lnl(wl.t), lnl_o, g_one, g_o, precision, wl.n_states, what="one-launch backward")


def test_mixed_list_validation():
    """Entries are validated as the operations they hold: a bad kind, a bad buffer and a
    repeated gradient slot are refused before anything runs."""
    from paper_2606_27607_amd import HPError, _lib
    wl = synth.make_workload("hky", 10, 200, seed=5)
    ck = checkpointed(wl, 2, "f64", "every_k", 2)
    ck.lnl(wl.t)
    acc = torch.zeros(2 * wl.n_tips - 2, dtype=torch.float64, device=ck.inst.device)
    good = ck.plan.mixed_ops
    for mutate, code in ((lambda o: o.__setitem__((0, 0), 2), _lib.HP_ERR_ARG),
                         (lambda o: o.__setitem__((0, 1), 10 ** 6), _lib.HP_ERR_INDEX)):
        bad = good.copy()
        mutate(bad)
        with pytest.raises(HPError) as e:
            ck.inst.traverse_gradients_device(bad, acc)
        assert e.value.code == code
    pre_rows = np.nonzero(good[:, 0] == 1)[0]
    bad = good.copy()
    bad[pre_rows[1], 5] = bad[pre_rows[0], 5]        # the same gradient slot twice
    with pytest.raises(HPError) as e:
        ck.inst.traverse_gradients_device(bad, acc)
    assert e.value.code == _lib.HP_ERR_ARG
