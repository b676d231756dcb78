"""Write full-size FP64 oracle results for the named workloads (calls only oracle/ and synth/).

    python tests/golden/make_oracle_golden.py nuc8 nuc128 ...
    python tests/golden/make_oracle_golden.py serving     # the serving clients' oracle sample
    python tests/golden/make_oracle_golden.py nuc8_rate nuc128_rate   # rate-matrix gradients
    python tests/golden/make_oracle_golden.py geo         # the phylogeography workload

For the serving sample, oracle_serving.json holds, per sampled client, lnL and every branch
gradient at that client's first request.

Each tests/golden/oracle_<name>.json holds the log-likelihood, every branch gradient and
the site log-likelihoods of a fixed sample of patterns (every (P // 509)-th pattern plus
the last one, so the ragged tail of the pattern padding is covered).  The GPU parity tests
compare the library's full-size results with these values; nothing here comes from the
GPU path.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def sample_indices(n_patterns: int) -> np.ndarray:
    step = max(1, n_patterns // 509)
    idx = np.arange(0, n_patterns, step)
    return np.unique(np.concatenate([idx, [n_patterns - 1]]))


def serving():
    out = {}
    for c in synth.serving_oracle_sample():
        t0 = time.time()
        wl = synth.serving_workload(c)
        t = synth.serving_requests(wl, c)[0]
        lnl, _, grad = oracle.lnl_and_grad(wl.tree.children, wl.n_tips, np.r_[t, 0.0], wl.Q, wl.pi,
                                           wl.rates, wl.cat_weights, wl.tips, wl.weights,
                                           chunk=2000 if wl.n_states > 4 else 20000)
        out[str(c)] = {"n_tips": wl.n_tips, "n_patterns": wl.n_patterns, "n_states": wl.n_states,
                       "request": 0, "lnl": lnl, "grad": grad.tolist(),
                       "oracle_seconds": time.time() - t0}
        print(f"serving client {c}: N={wl.n_tips} P={wl.n_patterns} S={wl.n_states} "
              f"lnL {lnl:.6f} in {time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "oracle_serving.json"), "w") as f:
        json.dump(out, f)


def rate_gradient(names):
    """oracle_<name>_rate.json: the first-order rate-matrix gradient at the workload's own
    branch lengths (4-state workloads)."""
    for name in names:
        t0 = time.time()
        wl = synth.config_workload(name)
        lnl, G = oracle.rate_matrix_gradient(wl.tree.children, wl.n_tips, wl.t, wl.Q, wl.pi, wl.rates,
                                             wl.cat_weights, wl.tips, wl.weights, chunk=10000)
        out = {"workload": name, "n_tips": wl.n_tips, "n_patterns": wl.n_patterns,
               "n_states": wl.n_states, "lnl": lnl, "rate_grad": G.tolist(), "Q": wl.Q.tolist(),
               "oracle_seconds": time.time() - t0}
        with open(os.path.join(HERE, f"oracle_{name}_rate.json"), "w") as f:
            json.dump(out, f)
        print(f"{name} rate gradient in {time.time() - t0:.1f} s", flush=True)


def geo():
    """oracle_geo200.json: lnL and every branch gradient of the phylogeography workload."""
    t0 = time.time()
    wl = synth.geo_workload()
    lnl, _, grad = oracle.lnl_and_grad(wl.tree.children, wl.n_tips, wl.t, wl.Q, wl.pi, wl.rates,
                                       wl.cat_weights, wl.tips, wl.weights)
    out = {"workload": wl.name, "n_tips": wl.n_tips, "n_patterns": wl.n_patterns,
           "n_states": wl.n_states, "lnl": lnl, "grad": grad.tolist(),
           "oracle_seconds": time.time() - t0}
    with open(os.path.join(HERE, f"oracle_{wl.name}.json"), "w") as f:
        json.dump(out, f)
    print(f"{wl.name}: lnL {lnl:.6f} in {time.time() - t0:.1f} s", flush=True)


def main(names):
    if "geo" in names:
        geo()
        names = [n for n in names if n != "geo"]
    if "serving" in names:
        serving()
        names = [n for n in names if n != "serving"]
    rate = [n[: -len("_rate")] for n in names if n.endswith("_rate")]
    if rate:
        rate_gradient(rate)
        names = [n for n in names if not n.endswith("_rate")]
    for name in names:
        t0 = time.time()
        wl = synth.config_workload(name)
        lnl, site, grad = oracle.lnl_and_grad(wl.tree.children, wl.n_tips, wl.t, wl.Q, wl.pi,
                                              wl.rates, wl.cat_weights, wl.tips, wl.weights,
                                              chunk=10000 if wl.n_states > 4 else 20000)
        idx = sample_indices(wl.n_patterns)
        out = {"workload": name, "n_tips": wl.n_tips, "n_patterns": wl.n_patterns,
               "n_states": wl.n_states, "seed": wl.meta["seed"], "lnl": lnl,
               "grad": grad.tolist(), "site_idx": idx.tolist(), "site_lnl": site[idx].tolist(),
               "oracle_seconds": time.time() - t0}
        with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
            json.dump(out, f)
        print(f"{name}: lnL {lnl:.6f} in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["nuc8", "nuc128", "codon64", "nuc256", "codon32"])
