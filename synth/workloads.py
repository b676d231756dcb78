"""Seeded synthetic workloads shaped like the paper's benchmarks.

The paper benchmarks HMC over branch-specific rates on a fixed tree with HKY
and GY94 models (1,024 taxa, patterns swept) and a GTR dengue data set; none
of those data sets ship here, so every workload is simulated from a seed.
The five named configurations are:

1. ``nuc8``     - 8 taxa, HKY85 (kappa 2), freqs ~ Dir(10,10,10,10), branches ~ Exp(mean 0.1),
                  4 gamma categories (alpha 0.5), 1,000 patterns, weights U{1..5}; FP64.
2. ``nuc128``   - 128 taxa, GTR (exchangeabilities ~ Gamma(2,1), freqs ~ Dir(10^4)),
                  branches ~ Exp(0.05), 4 categories, 100,000 patterns, rescaling every 4 levels.
3. ``codon64``  - 64 taxa, GY94 (omega 0.3, kappa 2, F3x4 with each position ~ Dir(10^4)),
                  branches ~ Exp(0.1), 4 categories, 10,000 patterns.
4. ``nuc256`` / ``codon32`` - the differentiation workloads: 256-taxon GTR with 50,000 patterns
                  and 32-taxon GY94 with 5,000 patterns.
5. serving     - per-client data sets drawn by :func:`serving_dataset`.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import models
from .simulate import pattern_weights, simulate_patterns
from .trees import Tree, exponential_branches, yule_tree

SEED_BASE = 20260000


@dataclass
class Workload:
    name: str
    tree: Tree
    t: np.ndarray            # float64 [2N-1] branch lengths (t[root] = 0)
    Q: np.ndarray            # float64 [S, S] normalised rate matrix
    pi: np.ndarray           # float64 [S]
    rates: np.ndarray        # float64 [K] category rates
    cat_weights: np.ndarray  # float64 [K]
    V: np.ndarray            # eigensystem handed to the library: Q = V diag(lam) Vinv
    Vinv: np.ndarray
    lam: np.ndarray
    tips: np.ndarray         # uint8 [N, P]; value S means "unknown"
    weights: np.ndarray      # float64 [P] pattern weights
    meta: dict = field(default_factory=dict)

    @property
    def n_tips(self) -> int:
        return self.tree.n_tips

    @property
    def n_states(self) -> int:
        return self.Q.shape[0]

    @property
    def n_categories(self) -> int:
        return len(self.rates)

    @property
    def n_patterns(self) -> int:
        return self.tips.shape[1]


def _model(kind: str, rng: np.random.Generator, **kw):
    if kind == "jc69":
        return models.jc69()
    if kind == "bin":
        pi = rng.dirichlet(np.full(2, 10.0))
        return models.binary(pi), pi
    if kind == "three":
        pi = rng.dirichlet(np.full(3, 10.0))
        R = np.zeros((3, 3))
        R[np.triu_indices(3, 1)] = rng.gamma(2.0, 1.0, size=3)
        return models.reversible(R + R.T, pi), pi
    if kind == "hky":
        pi = rng.dirichlet(np.full(4, 10.0))
        return models.hky85(kw.get("kappa", 2.0), pi), pi
    if kind == "gtr":
        pi = rng.dirichlet(np.full(4, 10.0))
        return models.gtr(rng.gamma(2.0, 1.0, size=6), pi), pi
    if kind == "aa":
        pi = rng.dirichlet(np.ones(20))
        return models.random_aa(rng.gamma(1.0, 1.0, size=190), pi), pi
    if kind == "gy94":
        f = [rng.dirichlet(np.full(4, 10.0)) for _ in range(3)]
        pi = models.f3x4(*f)
        return models.gy94(kw.get("kappa", 2.0), kw.get("omega", 0.3), pi), pi
    if kind == "geo":
        # discrete-location (phylogeography) model: S locations, exchangeability between
        # every pair ~ Gamma(1, 1), location frequencies ~ Dir(1^S)
        S = int(kw.get("n_states", 100))
        pi = rng.dirichlet(np.ones(S))
        R = np.zeros((S, S))
        R[np.triu_indices(S, 1)] = rng.gamma(1.0, 1.0, size=S * (S - 1) // 2)
        return models.reversible(R + R.T, pi), pi
    raise ValueError(f"unknown model kind {kind!r}")


def make_workload(kind: str, n_tips: int, n_patterns: int, *, branch_mean: float = 0.1,
                  n_categories: int = 4, alpha: float = 0.5, seed=0, name: str | None = None,
                  tree: Tree | None = None, unknown_frac: float = 0.0, **model_kw) -> Workload:
    """Build one workload from a seed.  ``unknown_frac`` marks that fraction of tip
    states as unknown (state S) to exercise the all-ones tip vector."""
    ss = np.random.SeedSequence(seed)
    s_tree, s_model, s_sim, s_w = ss.spawn(4)
    r_tree = np.random.default_rng(s_tree)
    if tree is None:
        tree = yule_tree(n_tips, r_tree)
    t = exponential_branches(tree, branch_mean, r_tree)
    Q, pi = _model(kind, np.random.default_rng(s_model), **model_kw)
    rates, cw = models.discrete_gamma(alpha, n_categories)
    V, Vinv, lam = models.eigensystem(Q, pi)
    r_sim = np.random.default_rng(s_sim)
    tips = simulate_patterns(tree, t, Q, pi, rates, n_patterns, r_sim)
    if unknown_frac > 0:
        mask = r_sim.random(tips.shape) < unknown_frac
        tips[mask] = Q.shape[0]
    w = pattern_weights(n_patterns, np.random.default_rng(s_w))
    return Workload(name or f"{kind}{n_tips}x{n_patterns}", tree, t, Q, pi, rates, cw, V, Vinv, lam,
                    tips, w, meta={"kind": kind, "seed": seed, "branch_mean": branch_mean,
                                   "alpha": alpha})


# name -> (model kind, taxa, patterns, branch mean, scaling period in levels)
CONFIG_SPECS = {
    "nuc8": ("hky", 8, 1000, 0.1, 0),
    "nuc128": ("gtr", 128, 100_000, 0.05, 4),
    "codon64": ("gy94", 64, 10_000, 0.1, 1),
    "nuc256": ("gtr", 256, 50_000, 0.05, 4),
    "codon32": ("gy94", 32, 5_000, 0.1, 1),
    # an amino-acid stand-in beside the five configurations (20 states, random exchangeabilities
    # and Dirichlet(1) frequencies, as the serving mix draws them), for the 20-state precision
    # forms; seeded at SEED_BASE + 6
    "aa64": ("aa", 64, 10_000, 0.1, 1),
}
CONFIG_INDEX = {"nuc8": 1, "nuc128": 2, "codon64": 3, "nuc256": 4, "codon32": 4, "aa64": 6}


def config_workload(name: str, n_patterns: int | None = None) -> Workload:
    """One of the named configurations, seeded by SeedSequence(20260000 + config number).
    ``n_patterns`` overrides the pattern count (a prefix-independent re-simulation)."""
    kind, n, p, mean, _ = CONFIG_SPECS[name]
    seed = SEED_BASE + CONFIG_INDEX[name]
    if name == "codon32":
        seed = [seed, 1]
    wl = make_workload(kind, n, p if n_patterns is None else n_patterns, branch_mean=mean,
                       seed=seed, name=name)
    wl.meta["scale_every"] = CONFIG_SPECS[name][4]
    return wl


def serving_dataset(client: int, rng_seed: int = SEED_BASE + 50, max_tips: int = 1024,
                    max_patterns: int = 200_000) -> dict:
    """Shape of one serving client's data set: taxa and patterns log-uniform over
    [16, 1024] and [100, 200,000]; state space uniform over {4 (GTR), 20 (random AA), 61 (GY94)}."""
    rng = np.random.default_rng(np.random.SeedSequence([rng_seed, client]))
    n = int(round(np.exp(rng.uniform(np.log(16), np.log(max_tips)))))
    p = int(round(np.exp(rng.uniform(np.log(100), np.log(max_patterns)))))
    kind = ["gtr", "aa", "gy94"][int(rng.integers(3))]
    return {"kind": kind, "n_tips": n, "n_patterns": p, "seed": int(rng.integers(2**31))}


def serving_workload(client: int) -> Workload:
    """The data set of one serving client (shape from :func:`serving_dataset`), branches
    ~ Exp(mean 0.1), 4 gamma categories (alpha 0.5)."""
    spec = serving_dataset(client)
    return make_workload(spec["kind"], spec["n_tips"], spec["n_patterns"], branch_mean=0.1,
                         seed=spec["seed"], name=f"serve{client}")


def serving_requests(wl: Workload, client: int, n_requests: int = 8,
                     rng_seed: int = SEED_BASE + 51) -> np.ndarray:
    """Branch-length vectors [n_requests, 2N-2] of one client, as an MCMC proposal makes
    them: the data set's branch lengths times exp(0.05 Z), Z ~ N(0, 1) per branch."""
    rng = np.random.default_rng(np.random.SeedSequence([rng_seed, client]))
    nb = 2 * wl.n_tips - 2
    return wl.t[:nb][None, :] * np.exp(0.05 * rng.standard_normal((n_requests, nb)))


def serving_oracle_sample(n_clients: int = 64) -> list:
    """Clients whose first request is checked against the oracle: for each state space the
    smallest data set and the one of median size (by taxa x patterns x states^2)."""
    by_kind = {}
    for c in range(n_clients):
        spec = serving_dataset(c)
        s = {"gtr": 4, "aa": 20, "gy94": 61}[spec["kind"]]
        by_kind.setdefault(spec["kind"], []).append((spec["n_tips"] * spec["n_patterns"] * s * s, c))
    out = []
    for kind in ("gtr", "aa", "gy94"):
        rows = sorted(by_kind.get(kind, []))
        if rows:
            out += sorted({rows[0][1], rows[(len(rows) - 1) // 2][1]})
    return out


def geo_workload(n_tips: int = 1000, n_states: int = 200, n_categories: int = 4) -> Workload:
    """Phylogeography-shaped workload for the eigensystem path: one site (each tip's sampled
    location among n_states), a Yule tree with branches ~ Exp(0.1), random reversible rates
    between locations, 4 gamma categories.  Seeded by SeedSequence(20260060)."""
    return make_workload("geo", n_tips, 1, branch_mean=0.1, n_categories=n_categories,
                         seed=SEED_BASE + 60, name=f"geo{n_states}", n_states=n_states)

