"""Benchmark: lnL + all-branch-gradient evaluations per second on one MI355X.

A step is one full evaluation of the hot path on the 128-taxon GTR workload (100,000
patterns, 4 gamma categories, FP32, rescaling every 4 levels): transition matrices for
all 254 branches, post-order partials, root integration, pre-order partials and all 254
branch gradients, with the inputs resident in HBM.  Each step uses a different set of
branch lengths (multiplicative N(0, 0.05) perturbations, as an MCMC proposal would).

Prints one JSON line (rank 0, N = 1) with the throughput, the roofline of the dominant
kernel (the traversal kernel, timed live with HIP events on the library's stream), the
error against the FP64 oracle, synchronous-call latency percentiles, the oracle timed on a
bounded sample of the same workload on the host cores, and the same measurements for the
FP64 form, for the 64-taxon codon workload in FP32 / BF16 / FP16 / FP64 and for a 64-taxon
amino-acid workload in FP32 / BF16x3 / BF16 / FP16 ("variants"),
the rate-matrix gradient, the operation-level calls against one whole-tree call, the autograd
modes, and the serving loop on 64 clients with Poisson arrivals ("serving").
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lnL+gradient evals/s vs plain FP32 at stated error; %roofline; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks of MI355X per operand type, TFLOP/s
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f16": 2500.0, "bf16x3": 2500.0, "f32": 157.3, "f64": 78.6}
# bytes per stored partial element (bf16x3: FP32 partials, split-BF16 products)
ELEM = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2, "bf16x3": 4}
KERNEL_SOURCES = {True: "paper_2606_27607_amd/csrc/kernels_small.hip",
                  False: "paper_2606_27607_amd/csrc/walk_mfma.inc"}


def algorithmic_bytes(n_tips: int, n_patterns: int, n_states: int, n_cat: int, elem: int) -> float:
    """Bytes one full evaluation must move with per-operation accounting: each of the N-2
    non-root internal nodes' partials is written and read once in the post-order pass and
    read (pre_n), read (post) and written (pre_c) in the pre-order pass - 5 (N-2) E b - plus
    the tip states read once in each pass (2 N P bytes).  E = P K S (algorithmic S)."""
    E = n_patterns * n_cat * n_states
    return 5.0 * (n_tips - 2) * E * elem + 2.0 * n_tips * n_patterns


def floor_bytes(n_tips: int, n_patterns: int, n_states: int, n_cat: int, elem: int) -> float:
    """The tile-resident floor: the bytes a full evaluation must move when every non-root
    internal node's post-order partial is written once and read once (pre-order partials
    never leave the chip) - 2 (N-2) E b - plus the tip states read once in each pass."""
    E = n_patterns * n_cat * n_states
    return 2.0 * (n_tips - 2) * E * elem + 2.0 * n_tips * n_patterns


def algorithmic_flops(n_tips: int, n_patterns: int, n_states: int, n_cat: int) -> float:
    """Flops of one full evaluation: one matrix-vector product (2 S^2) per pattern and
    category for every internal child edge in the post-order pass, and three (recomputed
    P post, P^T (pre o u), Q u) in the pre-order pass; tip edges are lookups."""
    return 4.0 * (n_tips - 2) * n_patterns * n_cat * 2.0 * n_states ** 2


# headers every traversal kernel includes; a change to them changes the kernels too
KERNEL_HEADERS = ("paper_2606_27607_amd/csrc/hp_internal.h", "paper_2606_27607_amd/csrc/lanes.h")


def kernel_sha(kernel_source: str):
    """sha256 over a kernel source file followed by the shared headers it includes, or None
    if the source is missing."""
    import hashlib
    h = hashlib.sha256()
    for rel in (kernel_source,) + KERNEL_HEADERS:
        path = os.path.join(ROOT, rel)
        if not os.path.exists(path):
            return None
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel_source: str, workload: str, precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source and headers (kernel_sha must match); None otherwise."""
    import glob
    sha = kernel_sha(kernel_source)
    if sha is None:
        return None
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.traffic.json")):
        with open(path) as f:
            rec = json.load(f)
        if (rec.get("source") == kernel_source and rec.get("source_sha256") == sha
                and rec.get("workload") == workload and rec.get("precision") == precision):
            return rec["bytes_per_launch"]
    return None


def _oracle_chunk(args) -> float:
    """One worker of the all-cores oracle timing: the oracle on one pattern chunk with one
    BLAS thread; returns its lnL."""
    from threadpoolctl import threadpool_limits

    import oracle
    children, n_tips, t, Q, pi, rates, cat_w, tips, w = args
    with threadpool_limits(1):
        return float(oracle.lnl_and_grad(children, n_tips, t, Q, pi, rates, cat_w, tips, w)[0])


# patterns of each configuration the oracle is timed on (about 1-5 s of one host core each)
CPU_SAMPLE = {"nuc8": 1000, "nuc128": 60000, "codon64": 2000, "nuc256": 10000, "codon32": 5000}


def cpu_baseline(wl, sample_patterns: int, max_procs: int = 16, all_cores: bool = True, repeats: int = 1):
    """The FP64 oracle on the first `sample_patterns` patterns, scaled to evals/s of the
    full workload: on one thread (the reported value; the median of `repeats` runs), and on
    all host cores as a pool of processes over pattern chunks (patterns are independent),
    one BLAS thread each."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    tips = wl.tips[:, :sample_patterns]
    w = wl.weights[:sample_patterns]
    runs = []
    with threadpool_limits(1):
        for _ in range(repeats):
            t0 = time.perf_counter()
            oracle.lnl_and_grad(wl.tree.children, wl.n_tips, wl.t, wl.Q, wl.pi, wl.rates,
                                wl.cat_weights, tips, w)
            runs.append(time.perf_counter() - t0)
    dt = sorted(runs)[len(runs) // 2]
    full = dt * wl.n_patterns / sample_patterns
    affinity = len(os.sched_getaffinity(0))
    res = {"value": 1.0 / full, "unit": "evals/s", "cores": 1, "kind": "oracle",
           "sample": f"first {sample_patterns} of {wl.n_patterns} patterns of {wl.name}, "
                     f"lnL + all {2 * wl.n_tips - 2} gradients, FP64 NumPy/SciPy, 1 thread; "
                     f"{dt:.3f} s measured" + (f" (median of {repeats})" if repeats > 1 else "")
                     + ", scaled by patterns",
           "seconds_per_eval": full, "host_cpus": affinity, "os_cpu_count": os.cpu_count()}
    if not all_cores:
        return res
    # all cores: the same sample in one chunk per process (spawned: this process has used
    # the GPU), median of three timed passes after a warm-up pass
    procs = max(1, min(affinity, max_procs))
    bounds = np.linspace(0, sample_patterns, procs + 1).astype(int)
    tasks = [(wl.tree.children, wl.n_tips, wl.t, wl.Q, wl.pi, wl.rates, wl.cat_weights,
              np.ascontiguousarray(tips[:, a:b]), w[a:b]) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    with mp.get_context("spawn").Pool(len(tasks)) as pool:
        pool.map(_oracle_chunk, tasks, chunksize=1)
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            pool.map(_oracle_chunk, tasks, chunksize=1)
            runs.append(time.perf_counter() - t0)
    dt_all = sorted(runs)[1]
    full_all = dt_all * wl.n_patterns / sample_patterns
    res["all_cores"] = {"value": 1.0 / full_all, "unit": "evals/s", "cores": len(tasks), "kind": "oracle",
                        "sample": f"the same {sample_patterns} patterns in {len(tasks)} chunks, one process "
                                  f"and one BLAS thread each; median of 3 passes ({dt_all:.2f} s) after a "
                                  f"warm-up, scaled by patterns",
                        "seconds_per_eval": full_all}
    return res


def measure(wl, precision: str, steps: int, warmup: int, latency_samples: int) -> dict:
    import numpy as np
    import torch

    from paper_2606_27607_amd import Instance, default_scaling

    N, P, S, K = wl.n_tips, wl.n_patterns, wl.n_states, wl.n_categories
    nb = 2 * N - 2
    small = S <= 4
    policy, period = default_scaling(S, precision)
    if small:
        period = max(1, wl.meta.get("scale_every", period))
    inst = Instance(N, P, S, K, precision=precision, scaling=policy, scale_period=period)
    scaling = f"rescaling every {period} levels" if policy == "every_k" else "rescaling every node"
    inst.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights,
              children=wl.tree.children)
    dev = inst.device
    rng = np.random.default_rng(1)
    n_sets = steps + warmup
    t_all = wl.t[:nb][None, :] * np.exp(0.05 * rng.standard_normal((n_sets, nb)))
    t_dev = torch.tensor(t_all, dtype=torch.float64, device=dev)
    out = torch.empty((n_sets, 1 + nb), dtype=torch.float64, device=dev)

    # accuracy at the workload's own branch lengths, against the full-size FP64 oracle
    lnl, g = inst.evaluate(wl.t)
    err = {}
    gold_path = os.path.join(ROOT, "tests", "golden", f"oracle_{wl.name}.json")
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
        gg = np.array(gold["grad"])
        err = {"lnl_rel": abs(lnl - gold["lnl"]) / abs(gold["lnl"]),
               "lnl_abs": abs(lnl - gold["lnl"]),
               "grad_maxabs_over_maxabs": float(np.max(np.abs(g - gg)) / np.max(np.abs(gg))),
               "grad_l2_rel": float(np.linalg.norm(g - gg) / np.linalg.norm(gg)),
               "reference": "FP64 oracle, full workload"}

    for i in range(warmup):
        inst.evaluate_device(t_dev[i], out=out[i])
    torch.cuda.synchronize()
    inst.status()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, n_sets):
        inst.evaluate_device(t_dev[i], out=out[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    inst.status()
    ms_per_step = 1000.0 * elapsed / steps

    # the same steps again with every kernel bracketed by HIP events on the library's stream
    inst.profile(True)
    inst.profile_read()
    for i in range(warmup, n_sets):
        inst.evaluate_device(t_dev[i], out=out[i])
    prof = inst.profile_read()
    inst.profile(False)
    trav_ms = prof["traversal"][0] / max(1, prof["traversal"][1])
    alg = algorithmic_bytes(N, P, S, K, ELEM[precision])
    gbs = alg / (trav_ms * 1e-3) / 1e9
    floor = floor_bytes(N, P, S, K, ELEM[precision])
    traffic = measured_traffic(KERNEL_SOURCES[small], wl.name, precision)
    # the same time against the tile-resident floor, and against the HBM bytes the counters saw
    fracs = {"floor_bytes": floor, "floor_frac": floor / (trav_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "counter_frac": (traffic / (trav_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None}
    if small:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, **fracs,
                "kernel": "walk_small (fused post-order + root + pre-order + gradients)",
                "kernel_ms": trav_ms, "algorithmic_bytes": alg}
    else:
        fl = algorithmic_flops(N, P, S, K)
        tf = fl / (trav_ms * 1e-3) / 1e12
        peak = MFMA_PEAK_TFLOPS[precision]
        roof = {"bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s",
                "frac": tf / peak, "traffic": traffic,
                "kernel": f"walk_mfma<{precision}> (fused post-order + root + pre-order + gradients)",
                "kernel_ms": trav_ms, "algorithmic_flops": fl, "algorithmic_bytes": alg,
                "hbm_GBs_algorithmic": gbs, "hbm_frac_algorithmic": gbs / HBM_PEAK_GBS, **fracs}

    lat = []
    for i in range(latency_samples):
        s = time.perf_counter()
        inst.evaluate(t_all[i % n_sets])
        lat.append(1000.0 * (time.perf_counter() - s))
    inst.close()
    return {
        "value": 1000.0 / ms_per_step, "unit": "evals/s", "ms_per_step": ms_per_step,
        "dtype": precision,
        "config": {"workload": f"{wl.name}: {N}-taxon Yule tree, {wl.meta['kind'].upper()}+G{K} "
                               f"(alpha 0.5), {P} simulated patterns, S={S}, {scaling}, "
                               f"lnL + all {nb} branch gradients per eval",
                   "taxa": N, "patterns": P, "states": S, "categories": K, "precision": precision},
        "roofline": roof,
        "kernels_ms_per_step": {k: v[0] / max(1, v[1]) for k, v in prof.items()},
        "error_vs_oracle": err,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mode": "synchronous hp_evaluate, host in/out"} if lat else None,
    }


def measure_rate_gradient(wl, precision: str, steps: int, warmup: int) -> dict:
    """lnL + branch gradients + the first-order rate-matrix gradient per evaluation:
    throughput, traversal time against the plain evaluation's, error vs the oracle."""
    import numpy as np
    import torch

    from paper_2606_27607_amd import Instance, default_scaling

    N, P, S, K = wl.n_tips, wl.n_patterns, wl.n_states, wl.n_categories
    nb = 2 * N - 2
    policy, period = default_scaling(S, precision)
    if S <= 4:
        period = max(1, wl.meta.get("scale_every", period))
    inst = Instance(N, P, S, K, precision=precision, scaling=policy, scale_period=period)
    inst.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights,
              children=wl.tree.children)
    rng = np.random.default_rng(2)
    n_sets = steps + warmup
    t_all = wl.t[:nb][None, :] * np.exp(0.05 * rng.standard_normal((n_sets, nb)))
    t_dev = torch.tensor(t_all, dtype=torch.float64, device=inst.device)
    out = torch.empty((n_sets, 1 + nb + S * S), dtype=torch.float64, device=inst.device)
    lnl, g, G = inst.evaluate_rate_gradient(wl.t)
    err = {}
    gold_path = os.path.join(ROOT, "tests", "golden", f"oracle_{wl.name}_rate.json")
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
        Go = np.array(gold["rate_grad"])
        err = {"lnl_rel": abs(lnl - gold["lnl"]) / abs(gold["lnl"]),
               "rate_grad_maxabs_over_maxabs": float(np.max(np.abs(G - Go)) / np.max(np.abs(Go))),
               "reference": "FP64 oracle, full workload"}
    res = {}
    for form in ("plain", "rate_gradient"):
        for i in range(warmup):
            if form == "plain":
                inst.evaluate_device(t_dev[i], out=out[i, : 1 + nb])
            else:
                inst.evaluate_rate_gradient_device(t_dev[i], out=out[i])
        torch.cuda.synchronize()
        inst.profile(True)
        inst.profile_read()
        t0 = time.perf_counter()
        for i in range(warmup, n_sets):
            if form == "plain":
                inst.evaluate_device(t_dev[i], out=out[i, : 1 + nb])
            else:
                inst.evaluate_rate_gradient_device(t_dev[i], out=out[i])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = inst.profile_read()
        inst.profile(False)
        inst.status()
        res[form] = {"evals_per_s": steps / el,
                     "traversal_ms": prof["traversal"][0] / max(1, prof["traversal"][1])}
    inst.close()
    return {"workload": f"{wl.name}: {N} taxa, {P} patterns, S={S}", "precision": precision,
            "evals_per_s": res["rate_gradient"]["evals_per_s"],
            "traversal_ms": res["rate_gradient"]["traversal_ms"],
            "plain_evals_per_s": res["plain"]["evals_per_s"],
            "plain_traversal_ms": res["plain"]["traversal_ms"],
            "overhead_vs_plain": res["plain"]["evals_per_s"] / res["rate_gradient"]["evals_per_s"] - 1.0,
            "error_vs_oracle": err}


def eig_flops(n_tips: int, n_patterns: int, n_states: int, n_cat: int) -> float:
    """Flops of one evaluation on the eigensystem path: every product is an S x S matrix
    (V, V^-1, V^T or V^-T) times one vector per (node, category, pattern): u of every branch
    (N tips + N-2 internal: V), y of every internal non-root node (V^-1), z of every branch
    (V^T) and q of every internal non-root node (V^-T); S counted, not S_pad."""
    vectors = (n_tips + (n_tips - 2) + (n_tips - 2) + (2 * n_tips - 2) + (n_tips - 2)) * n_cat * n_patterns
    return vectors * 2.0 * n_states ** 2


def measure_eig(wl, precision: str, steps: int, warmup: int) -> dict:
    """The phylogeography-shaped workload on the eigensystem path (transition matrices applied
    through V, V^-1 on the fly, never formed): throughput, traversal time, matrix-core rate,
    error vs the stored oracle result, and what forming every P(t) alone would cost."""
    import numpy as np
    import torch

    from paper_2606_27607_amd import Instance, default_scaling

    N, P, S, K = wl.n_tips, wl.n_patterns, wl.n_states, wl.n_categories
    nb = 2 * N - 2
    inst = Instance(N, P, S, K, precision=precision, scaling="every_node")
    inst.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights,
              children=wl.tree.children)
    lnl, g = inst.evaluate(wl.t)
    err = {}
    gold_path = os.path.join(ROOT, "tests", "golden", f"oracle_{wl.name}.json")
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
        gg = np.array(gold["grad"])
        err = {"lnl_rel": abs(lnl - gold["lnl"]) / abs(gold["lnl"]),
               "grad_maxabs_over_maxabs": float(np.max(np.abs(g - gg)) / np.max(np.abs(gg))),
               "reference": "FP64 oracle (scipy expm), full workload"}
    rng = np.random.default_rng(3)
    n_sets = steps + warmup
    t_dev = torch.tensor(wl.t[:nb][None, :] * np.exp(0.05 * rng.standard_normal((n_sets, nb))),
                         dtype=torch.float64, device=inst.device)
    out = torch.empty((n_sets, 1 + nb), dtype=torch.float64, device=inst.device)
    for i in range(warmup):
        inst.evaluate_device(t_dev[i], out=out[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, n_sets):
        inst.evaluate_device(t_dev[i], out=out[i])
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    inst.profile(True)
    inst.profile_read()
    for i in range(warmup, n_sets):
        inst.evaluate_device(t_dev[i], out=out[i])
    prof = inst.profile_read()
    inst.profile(False)
    inst.status()
    inst.close()
    trav = prof["traversal"][0] / max(1, prof["traversal"][1])
    fl = eig_flops(N, P, S, K)
    form_p = nb * K * 2.0 * S ** 3
    peak = MFMA_PEAK_TFLOPS[precision]
    return {"workload": f"{wl.name}: {N}-taxon Yule tree, {S} locations (random reversible rates), "
                        f"{P} pattern, {K} gamma categories, lnL + all {nb} branch gradients",
            "precision": precision, "evals_per_s": 1000.0 / ms, "ms_per_eval": ms,
            "traversal_ms": trav, "algorithmic_flops": fl,
            "mfma_TFLOPs": fl / (trav * 1e-3) / 1e12, "mfma_frac": fl / (trav * 1e-3) / 1e12 / peak,
            "forming_every_P_flops": form_p,
            "forming_every_P_ms_at_peak": form_p / (peak * 1e12) * 1e3,
            "error_vs_oracle": err}


def measure_operation_level(wl, precision: str, steps: int) -> dict:
    """One full evaluation through the operation-level calls (hp_update_matrices,
    hp_update_post, hp_root_lnl, hp_pre_gradients with the library's own operation lists),
    synchronous host in / host out, against the same evaluation as one hp_evaluate call on a
    whole-tree instance: median ms per evaluation, and the error against the oracle."""
    import numpy as np

    from paper_2606_27607_amd import Instance, _lib, default_scaling

    N, P, S, K = wl.n_tips, wl.n_patterns, wl.n_states, wl.n_categories
    nb = 2 * N - 2
    sc = default_scaling(S, precision)
    post, pre = _lib.plan_tree(wl.tree.children, *sc)
    op = Instance(N, P, S, K, precision=precision, scaling=sc[0], scale_period=sc[1],
                  n_pre_partials=_lib.plan_pre_buffers(wl.tree.children))
    op.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights)
    whole = Instance(N, P, S, K, precision=precision, scaling=sc[0], scale_period=sc[1])
    whole.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights,
               children=wl.tree.children)
    # the same calls with the Q . post cache (HP_FLAG_QPOST_CACHE, matrix-core path only)
    cached = None
    if 4 < S <= 64:
        cached = Instance(N, P, S, K, precision=precision, scaling=sc[0], scale_period=sc[1],
                          n_pre_partials=_lib.plan_pre_buffers(wl.tree.children), qpost_cache=True)
        cached.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights)
    t = wl.t[:nb]
    idx = np.arange(nb)

    def op_eval(inst):
        inst.update_matrices(idx, t)
        inst.update_post(post)
        lnl = inst.root_lnl(2 * N - 2)
        return lnl, inst.pre_gradients(pre, nb)

    for _ in range(3):
        lnl, g = op_eval(op)
        whole.evaluate(t)
        if cached is not None:
            lnl_c, g_c = op_eval(cached)
    t_op, t_whole, t_cached = [], [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        op_eval(op)
        t_op.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        whole.evaluate(t)
        t_whole.append(time.perf_counter() - t0)
        if cached is not None:
            t0 = time.perf_counter()
            op_eval(cached)
            t_cached.append(time.perf_counter() - t0)
    res = {"workload": wl.name, "precision": precision,
           "ms_per_eval_operation_level": 1000 * float(np.median(t_op)),
           "ms_per_eval_whole_tree": 1000 * float(np.median(t_whole))}
    if cached is not None:
        res["ms_per_eval_operation_level_qpost_cache"] = 1000 * float(np.median(t_cached))
    gold_path = os.path.join(ROOT, "tests", "golden", f"oracle_{wl.name}.json")
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
        gg = np.array(gold["grad"])
        err = lambda l, gr: {"lnl_rel": abs(l - gold["lnl"]) / abs(gold["lnl"]),
                             "grad_maxabs_over_maxabs": float(np.max(np.abs(gr - gg)) / np.max(np.abs(gg)))}
        res["error_vs_oracle"] = err(lnl, g)
        if cached is not None:
            res["error_vs_oracle_qpost_cache"] = err(lnl_c, g_c)
    op.close()
    whole.close()
    if cached is not None:
        cached.close()
    return res


def measure_autograd(wl, precision: str, steps: int, period: int = 4) -> dict:
    """Forward + backward of BranchLengthLnL per mode (store / recompute / fused, and the
    checkpoint variant keeping every period-th level's partials), ms per step and post-order
    buffers held."""
    import torch

    from paper_2606_27607_amd import Instance, default_scaling
    from paper_2606_27607_amd.autograd import BranchLengthLnL

    N, P, S, K = wl.n_tips, wl.n_patterns, wl.n_states, wl.n_categories
    scaling = default_scaling(S, precision)
    inst = Instance(N, P, S, K, precision=precision, scaling=scaling[0], scale_period=scaling[1])
    inst.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights,
              children=wl.tree.children)
    t = torch.tensor(wl.t[: 2 * N - 2], dtype=torch.float64, device=inst.device, requires_grad=True)
    res = {}
    for mode in ("store", "recompute", "fused"):
        for i in range(3 + steps):
            if i == 3:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            out = BranchLengthLnL.apply(t, inst, mode)
            (g,) = torch.autograd.grad(out, t)
        torch.cuda.synchronize()
        res[mode] = {"ms_per_forward_backward": 1000.0 * (time.perf_counter() - t0) / steps,
                     "post_buffers": N - 1}
    inst.close()
    from paper_2606_27607_amd.checkpoint import Checkpointed
    ck = Checkpointed.create(N, P, S, K, wl.tree.children, period, precision=precision, scaling=scaling[0],
                             scale_period=scaling[1])
    ck.load(wl.tips, wl.weights, wl.V, wl.Vinv, wl.lam, wl.pi, wl.rates, wl.cat_weights)
    for i in range(3 + steps):
        if i == 3:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        out = BranchLengthLnL.apply(t, ck, "checkpoint")
        (g,) = torch.autograd.grad(out, t)
    torch.cuda.synchronize()
    res[f"checkpoint every {period} levels"] = {
        "ms_per_forward_backward": 1000.0 * (time.perf_counter() - t0) / steps,
        "post_buffers": ck.plan.n_post_buffers, "recomputed_segments": ck.plan.n_segments}
    ck.inst.close()
    return {"workload": f"{wl.name}: {N} taxa, {P} patterns, S={S}", "precision": precision,
            "modes": res}


# Serving precisions, the fastest that keep lnL within 1e-4 relative on every client: FP32 for
# 4 states, FP32 partials with split-BF16 products (bf16x3) for 20, BF16 (FP32 exponent range)
# for 61.  FP16 runs faster but flushes values below 2^-24 of a pattern's maximum; on large
# trees with very short branches that can zero a site likelihood (HP_ERR_NUMERIC).  BF16
# partials for 20 states measured up to 1.3e-4 on small data sets.
SERVING_PRECISION = {4: "f32", 20: "bf16x3", 61: "bf16"}


def _serving_client(c):
    import synth
    wl = synth.serving_workload(c)
    return c, wl, synth.serving_requests(wl, c)


def serving_inputs(n_clients: int, jobs: int):
    """Every client's data set and requests, simulated in worker processes (forked before
    this process touches the GPU), largest first so that the pool finishes together."""
    import multiprocessing as mp

    import synth
    sizes = []
    for c in range(n_clients):
        d = synth.serving_dataset(c)
        sizes.append((-d["n_tips"] * d["n_patterns"], c))
    order = [c for _, c in sorted(sizes)]
    with mp.get_context("fork").Pool(max(1, jobs)) as pool:
        got = {c: (wl, reqs) for c, wl, reqs in pool.imap_unordered(_serving_client, order)}
    return [got[c] for c in range(n_clients)]


def serving_bench(inputs, loads=(0.5, 0.8, 1.0, 1.5), seed: int = 20260055) -> dict:
    """Many clients, continuous batching: isolated capacity, then Poisson arrivals at
    fractions of it; latency from submission to result, alone-vs-mix equality, and the
    oracle error on a stratified sample of clients."""
    import numpy as np

    from paper_2606_27607_amd.serve import Dataset, HipExecutor, Server

    n_clients = len(inputs)
    reqs = [(c, r) for c in range(n_clients) for r in range(len(inputs[c][1]))]
    work_b, work_f = {}, {}
    for c, (wl, _) in enumerate(inputs):
        prec = SERVING_PRECISION[wl.n_states]
        sp = 4 if wl.n_states <= 4 else (32 if wl.n_states <= 32 else 64)
        work_b[c] = algorithmic_bytes(wl.n_tips, wl.n_patterns, sp if sp == 4 else wl.n_states,
                                      wl.n_categories, ELEM[prec])
        work_f[c] = algorithmic_flops(wl.n_tips, wl.n_patterns, wl.n_states, wl.n_categories)
    import torch
    torch.cuda.empty_cache()          # sessions allocate straight from the device
    ex = HipExecutor(0)
    srv = Server(executor=ex, precision=SERVING_PRECISION).start()
    chunks = {c: srv.register(c, Dataset.from_workload(wl)) for c, (wl, _) in enumerate(inputs)}
    # isolated: one request at a time, each client's session loaded by an untimed first call
    t_start = time.perf_counter()
    alone, service, service_small = {}, [], []
    small = {c: all(s.tier == 0 for s in srv.sessions[c]) for c in range(n_clients)}
    for c, (wl, ts) in enumerate(inputs):
        srv.evaluate(c, ts[0])
        for r in range(len(ts)):
            s0 = time.perf_counter()
            alone[(c, r)] = srv.evaluate(c, ts[r])
            service.append(time.perf_counter() - s0)
            if small[c]:
                service_small.append(service[-1])
        if c % 16 == 15:
            print(f"[bench] serving: isolated pass, {c + 1} clients done", file=sys.stderr, flush=True)
    capacity = len(service) / sum(service)
    isolated = {"requests_per_s": capacity, "p50_ms": 1000 * float(np.percentile(service, 50)),
                "p99_ms": 1000 * float(np.percentile(service, 99)),
                "small_requests": len(service_small),
                "small_p50_ms": 1000 * float(np.percentile(service_small or [0.0], 50)),
                "small_p99_ms": 1000 * float(np.percentile(service_small or [0.0], 99)),
                "seconds": time.perf_counter() - t_start, "evictions": srv.stats()["evictions"]}
    rng = np.random.default_rng(seed)
    mixes = []
    mismatch = 0
    for load in loads:
        srv.reset_stats()
        order = rng.permutation(len(reqs))
        arrivals = np.cumsum(rng.exponential(1.0 / (load * capacity), len(reqs)))
        futs = []
        t0 = time.perf_counter()
        for i, idx in enumerate(order):
            while True:
                d = t0 + arrivals[i] - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(min(d, 5e-4))
            c, r = reqs[idx]
            futs.append(((c, r), srv.submit(c, inputs[c][1][r])))
        for key, f in futs:
            lnl, g = f.result(timeout=300)
            a_lnl, a_g = alone[key]
            mismatch += int(not (lnl == a_lnl and np.array_equal(g, a_g)))
        st = srv.stats()
        span = st["requests_per_s"] and st["completed"] / st["requests_per_s"]
        mixes.append({"load": load, "offered_requests_per_s": load * capacity,
                      "requests_per_s": st["requests_per_s"], "p50_ms": st["p50_ms"],
                      "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"], "mean_batch": st["mean_batch"],
                      "small_p50_ms": st["small_p50_ms"], "small_p99_ms": st["small_p99_ms"],
                      "batches": st["batches"], "max_concurrent_batches": st["max_concurrent_batches"],
                      "evictions": st["evictions"],
                      "algorithmic_GBs": sum(work_b[c] for c, _ in reqs) / span / 1e9,
                      "algorithmic_TFLOPs": sum(work_f[c] for c, _ in reqs) / span / 1e12})
        print(f"[bench] serving: load {load} done, p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms",
              file=sys.stderr, flush=True)
    srv.close()
    # lnL / gradient error of the served result against the stored oracle values
    err = {}
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_serving.json")
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
        for key, rec in gold.items():
            c = int(key)
            if c >= n_clients:
                continue
            lnl, g = alone[(c, rec["request"])]
            gg = np.array(rec["grad"])
            err[key] = {"states": rec["n_states"], "taxa": rec["n_tips"], "patterns": rec["n_patterns"],
                        "precision": SERVING_PRECISION[rec["n_states"]],
                        "lnl_rel": abs(lnl - rec["lnl"]) / abs(rec["lnl"]),
                        "grad_maxabs_over_maxabs": float(np.max(np.abs(g - gg)) / np.max(np.abs(gg)))}
    kinds = collections.Counter(inputs[c][0].n_states for c in range(n_clients))
    return {"clients": n_clients, "requests": len(reqs),
            "state_spaces": {str(k): v for k, v in sorted(kinds.items())},
            "precision": {str(k): v for k, v in SERVING_PRECISION.items()},
            "pattern_chunked_clients": sum(1 for v in chunks.values() if v > 1),
            "memory_budget_bytes": srv.memory_budget,
            "isolated": isolated, "mix": mixes, "mix_vs_alone_mismatches": mismatch,
            "error_vs_oracle_sample": err,
            "small_session_seconds": srv.small_seconds,
            "arrivals": "Poisson, rate = load x isolated capacity, requests in random order; "
                        "small = requests whose sessions are all estimated under small_session_seconds"}


def serving_cpu_baseline() -> dict:
    """The FP64 oracle on the serving sample (per state space the smallest client and the one
    of median size, first request), one host thread, on a prefix of each client's patterns
    (at most 4,000 / 1,000 / 100 for 4 / 20 / 61 states) scaled to the whole request."""
    from threadpoolctl import threadpool_limits

    import oracle
    import synth
    per = {}
    for c in synth.serving_oracle_sample():
        wl = synth.serving_workload(c)
        t = synth.serving_requests(wl, c)[0]
        import numpy as np
        n = min(wl.n_patterns, {4: 4000, 20: 1000, 61: 100}[wl.n_states])
        with threadpool_limits(1):
            t0 = time.perf_counter()
            oracle.lnl_and_grad(wl.tree.children, wl.n_tips, np.r_[t, 0.0], wl.Q, wl.pi, wl.rates, wl.cat_weights,
                                wl.tips[:, :n], wl.weights[:n])
            dt = time.perf_counter() - t0
        per[str(c)] = {"states": wl.n_states, "taxa": wl.n_tips, "patterns": wl.n_patterns,
                       "sample_patterns": n, "seconds_per_request": dt * wl.n_patterns / n}
    total = sum(v["seconds_per_request"] for v in per.values())
    return {"value": len(per) / total, "unit": "requests/s", "cores": 1, "kind": "oracle",
            "sample": "first request of the smallest and the median client per state space "
                      "(lnL + all branch gradients), pattern prefixes scaled to the whole request",
            "clients": per}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="nuc128")
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--cpu-sample", type=int, default=60000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--latency-samples", type=int, default=50)
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving benchmark (64 clients x 8 requests, mixed state "
                         "spaces, Poisson arrivals), which runs by default")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving benchmark")
    ap.add_argument("--serving-clients", type=int, default=64)
    ap.add_argument("--autograd-only", action="store_true",
                    help="run only the differentiation legs (nuc256 FP32, codon32 BF16: store, "
                         "recompute, fused and checkpoint modes)")
    ap.add_argument("--eig-only", metavar="PRECISIONS",
                    help="run only the eigensystem-path leg (geo200), e.g. f64 or f64,f32")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (10 times), the "
                         "reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 10}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the pattern "
              "partition across GPUs is described in the design notes and not implemented)", file=sys.stderr)
        sys.exit(2)

    import synth

    if args.autograd_only:
        print(json.dumps({"autograd": [measure_autograd(synth.config_workload("nuc256"), "f32", args.steps),
                                       measure_autograd(synth.config_workload("codon32"), "bf16", args.steps)]}),
              flush=True)
        return
    if args.eig_only:
        geo = synth.geo_workload()
        print(json.dumps({"eigensystem_path": [measure_eig(geo, p, max(10, args.steps // 4), 3)
                                               for p in args.eig_only.split(",")]}), flush=True)
        return

    serving_data = None
    if not args.no_serving or args.serving_only:
        # simulated before anything touches the GPU: the worker processes are forks of this one
        print(f"[bench] serving: simulating {args.serving_clients} client data sets", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        serving_data = serving_inputs(args.serving_clients, min(16, len(os.sched_getaffinity(0))))
        print(f"[bench] serving: data ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(serving_data)}), flush=True)
        return

    print(f"[bench] workload {args.workload} {args.precision}", file=sys.stderr, flush=True)
    wl = synth.config_workload(args.workload)
    head = measure(wl, args.precision, args.steps, args.warmup, args.latency_samples)
    line = {"metric": METRIC, "value": head["value"], "unit": "evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": args.precision, "data": "synthetic",
            "config": dict(head["config"], parallelism="single GPU"),
            "roofline": head["roofline"], "kernels_ms_per_step": head["kernels_ms_per_step"],
            "error_vs_oracle": head["error_vs_oracle"], "latency_ms": head["latency_ms"]}
    if not args.no_variants:
        variants = []
        baselined = {args.workload}
        # the 8-taxon FP64 case is latency-bound: its line is read for the per-call latency
        plan = [("nuc8", "f64")]
        plan += [("nuc128", "f64")] if args.workload == "nuc128" else []
        plan += [("codon64", p) for p in ("f32", "bf16x3", "bf16", "f16", "f64")]
        # 20 states: FP32 against the mixed forms (bf16x3 is the one held to 1e-5 on lnL)
        plan += [("aa64", p) for p in ("f32", "bf16x3", "bf16", "f16")]
        wls = {args.workload: wl}
        for name, prec in plan:
            if (name, prec) == (args.workload, args.precision):
                continue
            print(f"[bench] variant {name} {prec}", file=sys.stderr, flush=True)
            if name not in wls:
                wls[name] = synth.config_workload(name)
            variants.append(measure(wls[name], prec, max(10, args.steps // 2), 3, 200 if name == "nuc8" else 10))
            if not args.no_cpu_baseline and name not in baselined and name in CPU_SAMPLE:
                # the oracle on this configuration (once per workload), beside its GPU line
                baselined.add(name)
                print(f"[bench] cpu baseline (oracle) {name}", file=sys.stderr, flush=True)
                variants[-1]["cpu_baseline"] = cpu_baseline(
                    wls[name], min(CPU_SAMPLE[name], wls[name].n_patterns), all_cores=name != "nuc8",
                    repeats=21 if name == "nuc8" else 1)
        line["variants"] = variants
        by = {(v["config"]["states"], v["dtype"]): v for v in variants}
        for key, states, forms in (("codon_mixed_vs_fp32", 61, ("bf16x3", "bf16", "f16")),
                                   ("aa_mixed_vs_fp32", 20, ("bf16x3", "bf16", "f16"))):
            ref = by.get((states, "f32"))
            if ref:
                line[key] = {
                    p: {"speedup_vs_f32": by[(states, p)]["value"] / ref["value"],
                        "lnl_rel_err": by[(states, p)]["error_vs_oracle"].get("lnl_rel"),
                        "grad_err": by[(states, p)]["error_vs_oracle"].get("grad_maxabs_over_maxabs")}
                    for p in forms if (states, p) in by}
        print("[bench] rate-matrix gradient", file=sys.stderr, flush=True)
        line["rate_matrix_gradient"] = (
            [measure_rate_gradient(synth.config_workload("nuc128"), p, max(10, args.steps // 2), 3)
             for p in ("f32", "f64")]
            + [measure_rate_gradient(wls.get("codon64") or synth.config_workload("codon64"), p,
                                     max(10, args.steps // 4), 3) for p in ("f32", "bf16")])
        print("[bench] eigensystem path (phylogeography)", file=sys.stderr, flush=True)
        geo = synth.geo_workload()
        line["eigensystem_path"] = [measure_eig(geo, p, max(10, args.steps // 4), 3) for p in ("f64", "f32")]
        print("[bench] operation-level calls", file=sys.stderr, flush=True)
        line["operation_level"] = [
            measure_operation_level(synth.config_workload("nuc128"), "f32", 20),
            measure_operation_level(wls.get("codon64") or synth.config_workload("codon64"), "bf16", 20),
            measure_operation_level(wls.get("codon64") or synth.config_workload("codon64"), "f32", 20)]
        print("[bench] autograd modes", file=sys.stderr, flush=True)
        line["autograd"] = [measure_autograd(synth.config_workload("nuc256"), "f32", 20),
                            measure_autograd(synth.config_workload("codon32"), "bf16", 20)]
        if not args.no_cpu_baseline:
            for rec, name in zip(line["autograd"], ("nuc256", "codon32")):
                print(f"[bench] cpu baseline (oracle) {name}", file=sys.stderr, flush=True)
                rec["cpu_baseline"] = cpu_baseline(synth.config_workload(name), CPU_SAMPLE[name])
    if serving_data is not None:
        print("[bench] serving", file=sys.stderr, flush=True)
        try:
            line["serving"] = serving_bench(serving_data)
        except Exception as e:  # noqa: BLE001 - report it; the rest of the line stands
            line["serving"] = {"error": f"{type(e).__name__}: {e}"}
        serving_data = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, min(args.cpu_sample, wl.n_patterns))
        if "serving" in line and "error" not in line["serving"]:
            print("[bench] cpu baseline (oracle) serving sample", file=sys.stderr, flush=True)
            line["serving"]["cpu_baseline"] = serving_cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
