"""hp_evaluate_device_noalloc: the stream-ordered whole-tree evaluation with its reduction
scratch in the library's static device array, against hp_evaluate_device (the same kernels
with the rows in the instance's workspace).  Results must be bitwise equal, call after call,
including a second call with a smaller input on another instance, and an evaluation whose
rows would not fit the array must be refused before anything is enqueued."""
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


def _both(inst, t_host, want_grad=True):
    """(hp_evaluate_device, hp_evaluate_device_noalloc) outputs on the same inputs."""
    import torch
    t = torch.tensor(np.asarray(t_host, dtype=np.float64), device=inst.device)
    ref = inst.evaluate_device(t, want_grad=want_grad).cpu().numpy()
    n_out = ref.size
    out = torch.full((n_out,), float("nan"), dtype=torch.float64, device=inst.device)
    got = inst.evaluate_device_noalloc(t, want_grad=want_grad, out=out).cpu().numpy()
    inst.status()  # raises on a device-side error
    return ref, got


def _perturbed(wl, seed):
    rng = np.random.default_rng(seed)
    return wl.t * np.exp(0.05 * rng.standard_normal(wl.t.size))


def test_noalloc_matches_evaluate_device_two_calls_then_smaller():
    """A 96-taxon FP32 evaluation (20,000 patterns, rescaled every 4 levels) twice with
    different branch lengths, then a smaller 16-taxon FP64 one on another instance: every
    output bitwise equal to hp_evaluate_device's, and the FP64 one within the FP64 bound of
    the oracle."""
    big = synth.make_workload("gtr", 96, 20_000, branch_mean=0.05, seed=[20260071, 1])
    small = synth.make_workload("hky", 16, 3_000, branch_mean=0.1, seed=[20260071, 2])
    announce("noalloc gtr96x20000 f32 twice, then hky16x3000 f64")
    inst_b = make_instance(big, "f32", "every_k", 4)
    for s in (1, 2):
        ref, got = _both(inst_b, _perturbed(big, s))
        assert np.isfinite(ref).all()
        assert np.array_equal(ref, got), ("gtr96 f32", s, np.max(np.abs(ref - got)))
    inst_s = make_instance(small, "f64", "every_node")
    t = _perturbed(small, 3)
    ref, got = _both(inst_s, t)
    assert np.array_equal(ref, got), np.max(np.abs(ref - got))
    lnl_o, _, g_o = oracle_eval(small, t)
    check(got[0], lnl_o, got[1:], g_o, "f64", what="noalloc hky16 f64")
    # lnL only (one reduction row)
    ref, got = _both(inst_s, t, want_grad=False)
    assert ref.size == 1 and np.array_equal(ref, got)


def test_noalloc_matrix_core_path():
    """The matrix-core whole-tree kernel (61 codon states, BF16 partials) with its rows in
    the static array: bitwise equal to hp_evaluate_device, after a larger evaluation."""
    wl = synth.make_workload("gy94", 12, 1_000, branch_mean=0.1, seed=[20260071, 3])
    announce("noalloc gy94 12x1000 bf16")
    inst = make_instance(wl, "bf16", "every_k", 4)
    ref, got = _both(inst, _perturbed(wl, 4))
    assert np.isfinite(ref).all()
    assert np.array_equal(ref, got), np.max(np.abs(ref - got))


def test_noalloc_refuses_rows_beyond_the_array():
    """4,096 taxa x 40,000 patterns (one category, FP32): (2N-1) rows of one FP64 value per
    workgroup exceed the 16 MiB array.  The call returns HP_ERR_WORKSPACE without enqueueing
    anything; the lnL-only call (one row) still runs and equals hp_evaluate_device."""
    import torch
    from paper_2606_27607_amd import HPError, Instance, _lib
    N, P = 4096, 40_000
    rng = np.random.default_rng(20260072)
    tree = synth.trees.yule_tree(N, rng)
    t = synth.trees.exponential_branches(tree, 0.05, rng)
    Q, pi = synth.models.jc69()
    V, Vinv, lam = synth.models.eigensystem(Q, pi)
    tips = rng.integers(0, 4, size=(N, P), dtype=np.uint8)
    n_pre = _lib.plan_pre_buffers(tree.children)
    announce(f"noalloc refusal N={N} P={P} K=1 f32 (n_pre_partials={n_pre})")
    inst = Instance(N, P, 4, 1, precision="f32", scaling="every_k", scale_period=4, n_pre_partials=n_pre)
    inst.load(tips, np.ones(P), V, Vinv, lam, pi, np.ones(1), np.ones(1), children=tree.children)
    need = (2 * N - 1) * inst.query(_lib.HP_Q_BLOCKS) * 8
    assert need > 16 << 20, need
    td = torch.tensor(t, device=inst.device)
    out = torch.full((2 * N - 1,), -7.0, dtype=torch.float64, device=inst.device)
    with pytest.raises(HPError) as e:
        inst.evaluate_device_noalloc(td, want_grad=True, out=out)
    assert e.value.code == _lib.HP_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == -7.0).all()
    ref = inst.evaluate_device(td, want_grad=False).cpu().numpy()
    got = inst.evaluate_device_noalloc(td, want_grad=False, out=out[:1]).cpu().numpy()
    inst.status()  # raises on a device-side error
    assert np.isfinite(ref).all() and np.array_equal(ref, got)
