"""Seeded synthetic inputs shared by the oracle tests, the HIP parity tests and the benchmark.

This package only *generates inputs*: trees, substitution models (rate matrix,
stationary frequencies, the eigensystem a client hands to the library),
discrete-gamma rate categories, simulated site patterns and pattern weights.
It contains none of the likelihood or gradient arithmetic (no pruning, no
pre-order, no transition-probability matrices): sequences are simulated with
the jump chain of the continuous-time Markov chain (Gillespie), so nothing here
computes exp(Qt).
"""
from .models import (
    NUCLEOTIDES, CODONS, GENETIC_CODE, hky85, gtr, jc69, gy94, random_aa, f3x4,
    normalise_rate, eigensystem, discrete_gamma,
)
from .trees import Tree, yule_tree, two_taxon_tree, balanced_tree, caterpillar_tree
from .simulate import simulate_patterns, pattern_weights
from .workloads import (Workload, make_workload, config_workload, CONFIG_SPECS, serving_dataset,
                        serving_workload, serving_requests, serving_oracle_sample, geo_workload)

__all__ = [
    "NUCLEOTIDES", "CODONS", "GENETIC_CODE", "hky85", "gtr", "jc69", "gy94", "random_aa", "f3x4",
    "normalise_rate", "eigensystem", "discrete_gamma",
    "Tree", "yule_tree", "two_taxon_tree", "balanced_tree", "caterpillar_tree",
    "simulate_patterns", "pattern_weights",
    "Workload", "make_workload", "config_workload", "CONFIG_SPECS", "serving_dataset",
    "serving_workload", "serving_requests", "serving_oracle_sample", "geo_workload",
]
