"""Substitution models and rate heterogeneity used to build synthetic workloads.

The paper benchmarks the HKY nucleotide model, the GTR nucleotide model and the
Goldman-Yang (GY94) codon model (Performance evaluation, scaling by taxa and
patterns; ARM NEON benchmark); the workloads also use a random amino-acid
model.  The paper gives no formulas for any of them, so the textbook
definitions are written out here:

* reversible models are parameterised as Q_ij = R_ij * pi_j (i != j) with a
  symmetric exchangeability matrix R and stationary frequencies pi, and
  Q_ii = -sum_{j != i} Q_ij;
* every Q is normalised to one expected substitution per unit time under pi;
* gamma rate variation uses the mean-of-category discretisation of Yang (1994)
  with equal category weights.

The eigensystem returned by :func:`eigensystem` is what a client passes to the
library (the paper notes that transition matrices come from a numerical
eigendecomposition of the rate matrix and are cached across patterns).
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy import special

NUCLEOTIDES = "ACGT"
_TRANSITIONS = {frozenset("AG"), frozenset("CT")}

# NCBI translation table 1 (the standard genetic code), codons in TCAG order.
_TCAG = "TCAG"
_TABLE1_TCAG = "FFLLSSSSYY**CC*WLLLLPPPPHHQQRRRRIIIMTTTTNNKKSSRRVVVVAAAADDEEGGGG"
GENETIC_CODE = {
    a + b + c: _TABLE1_TCAG[16 * _TCAG.index(a) + 4 * _TCAG.index(b) + _TCAG.index(c)]
    for a, b, c in itertools.product(_TCAG, repeat=3)
}
# The 61 sense codons in lexicographic ACGT order (state index = position here).
CODONS = tuple(
    "".join(c) for c in itertools.product(NUCLEOTIDES, repeat=3) if GENETIC_CODE["".join(c)] != "*"
)


def _is_transition(x: str, y: str) -> bool:
    return frozenset((x, y)) in _TRANSITIONS


def _reversible(R: np.ndarray, pi: np.ndarray) -> np.ndarray:
    """Q_ij = R_ij pi_j off the diagonal, rows summing to zero."""
    R = np.asarray(R, dtype=np.float64)
    pi = np.asarray(pi, dtype=np.float64)
    Q = R * pi[None, :]
    np.fill_diagonal(Q, 0.0)
    np.fill_diagonal(Q, -Q.sum(axis=1))
    return Q


def normalise_rate(Q: np.ndarray, pi: np.ndarray) -> np.ndarray:
    """Scale Q so that the expected number of substitutions per unit time is one."""
    mu = -float(np.dot(pi, np.diag(Q)))
    return Q / mu


def reversible(R, pi) -> np.ndarray:
    """Normalised reversible rate matrix from a symmetric exchangeability matrix R."""
    pi = np.asarray(pi, dtype=np.float64)
    return normalise_rate(_reversible(R, pi), pi)


def binary(pi) -> np.ndarray:
    """Two-state reversible model (used for state counts below four)."""
    return reversible(np.array([[0.0, 1.0], [1.0, 0.0]]), pi)


def jc69() -> tuple[np.ndarray, np.ndarray]:
    pi = np.full(4, 0.25)
    R = np.ones((4, 4))
    return normalise_rate(_reversible(R, pi), pi), pi


def hky85(kappa: float, pi) -> np.ndarray:
    """Hasegawa-Kishino-Yano 1985: transitions (A<->G, C<->T) at kappa times transversions."""
    pi = np.asarray(pi, dtype=np.float64)
    R = np.ones((4, 4))
    for i, x in enumerate(NUCLEOTIDES):
        for j, y in enumerate(NUCLEOTIDES):
            if i != j and _is_transition(x, y):
                R[i, j] = kappa
    return normalise_rate(_reversible(R, pi), pi)


def gtr(exchangeabilities, pi) -> np.ndarray:
    """General time-reversible model; exchangeabilities in the order AC, AG, AT, CG, CT, GT."""
    e = np.asarray(exchangeabilities, dtype=np.float64)
    if e.shape != (6,):
        raise ValueError("GTR needs 6 exchangeabilities")
    pi = np.asarray(pi, dtype=np.float64)
    R = np.zeros((4, 4))
    iu = np.triu_indices(4, 1)
    R[iu] = e
    R = R + R.T
    return normalise_rate(_reversible(R, pi), pi)


def random_aa(exchangeabilities, pi) -> np.ndarray:
    """A 20-state reversible model with 190 given exchangeabilities (upper triangle, row major)."""
    e = np.asarray(exchangeabilities, dtype=np.float64)
    if e.shape != (190,):
        raise ValueError("a 20-state model needs 190 exchangeabilities")
    R = np.zeros((20, 20))
    R[np.triu_indices(20, 1)] = e
    R = R + R.T
    return normalise_rate(_reversible(R, np.asarray(pi, dtype=np.float64)), pi)


def f3x4(f1, f2, f3) -> np.ndarray:
    """Codon frequencies proportional to the product of position-specific nucleotide frequencies,
    renormalised over the 61 sense codons."""
    f = [np.asarray(v, dtype=np.float64) for v in (f1, f2, f3)]
    pi = np.array([f[0][NUCLEOTIDES.index(c[0])] * f[1][NUCLEOTIDES.index(c[1])]
                   * f[2][NUCLEOTIDES.index(c[2])] for c in CODONS])
    return pi / pi.sum()


def gy94(kappa: float, omega: float, pi) -> np.ndarray:
    """Goldman-Yang 1994 codon model over the 61 sense codons.

    Codons that differ at more than one position do not exchange; a single
    change is weighted by kappa if it is a transition and by omega if it changes
    the amino acid.
    """
    pi = np.asarray(pi, dtype=np.float64)
    n = len(CODONS)
    R = np.zeros((n, n))
    for i, a in enumerate(CODONS):
        for j, b in enumerate(CODONS):
            diff = [p for p in range(3) if a[p] != b[p]]
            if len(diff) != 1:
                continue
            p = diff[0]
            r = 1.0
            if _is_transition(a[p], b[p]):
                r *= kappa
            if GENETIC_CODE[a] != GENETIC_CODE[b]:
                r *= omega
            R[i, j] = r
    return normalise_rate(_reversible(R, pi), pi)


def eigensystem(Q: np.ndarray, pi: np.ndarray):
    """Eigendecomposition Q = V diag(lam) Vinv of a reversible rate matrix.

    Reversibility makes A = D^{1/2} Q D^{-1/2} (D = diag(pi)) symmetric, so the
    decomposition is real: A = U diag(lam) U^T gives V = D^{-1/2} U and
    Vinv = U^T D^{1/2}.  Returned arrays are row-major float64.
    """
    pi = np.asarray(pi, dtype=np.float64)
    d = np.sqrt(pi)
    A = (d[:, None] * Q) / d[None, :]
    A = 0.5 * (A + A.T)
    lam, U = np.linalg.eigh(A)
    V = U / d[:, None]
    Vinv = U.T * d[None, :]
    return np.ascontiguousarray(V), np.ascontiguousarray(Vinv), np.ascontiguousarray(lam)


def discrete_gamma(alpha: float, n_categories: int):
    """Mean-of-category discrete gamma (Yang 1994) for a Gamma(alpha, rate alpha) rate distribution.

    Category boundaries are the k/K quantiles; each category's rate is the mean
    of the distribution inside it, which uses the identity x f(x; a, a) =
    f(x; a+1, a) so that the partial mean is a difference of regularised lower
    incomplete gamma functions.  Weights are equal (1/K).
    """
    K = int(n_categories)
    if K == 1:
        return np.ones(1), np.ones(1)
    q = np.arange(1, K) / K
    b = special.gammaincinv(alpha, q) / alpha  # quantiles of Gamma(alpha, rate alpha)
    cdf1 = np.concatenate(([0.0], special.gammainc(alpha + 1.0, alpha * b), [1.0]))
    rates = K * np.diff(cdf1)
    return rates, np.full(K, 1.0 / K)
