"""Seeded smooth fields and dense operands.

The paper times its operations on square matrices of unstated values and
measures accuracy on analytic functions; smooth periodic fields with a little
noise stand in for both.  A field is a sum of T 2-D sinusoids

    M[i, j] += a * sin(2 pi (u j + v i) / n + theta)

with amplitude a ~ U[0.5, 2], frequencies u, v ~ U[-F, F] cycles per side,
phase theta ~ U[0, 2 pi), drawn in that order per term from
numpy.random.default_rng(seed) (PCG64), plus sigma * N(0, 1) noise drawn
afterwards for the whole matrix.  The sinusoids are evaluated separably,
sin(x + y) = sin x cos y + cos x sin y, as one product of an n x 2T matrix of
row factors by a 2T x n matrix of column factors; its last bits may depend on
the BLAS build, which does not matter because every test and benchmark feeds
the one generated array to both sides.
"""
from __future__ import annotations

import numpy as np


def smooth_field(n: int, terms: int, max_freq: float, sigma: float, seed: int,
                 cols: int | None = None) -> np.ndarray:
    """rows=n, cols=cols or n; frequencies are in cycles per n samples."""
    rows = n
    cols = n if cols is None else cols
    rng = np.random.default_rng(seed)
    ii = np.arange(rows, dtype=np.float64)
    jj = np.arange(cols, dtype=np.float64)
    L = np.zeros((rows, 2 * terms))
    R = np.zeros((2 * terms, cols))
    for t in range(terms):
        a = rng.uniform(0.5, 2.0)
        u = rng.uniform(-max_freq, max_freq)
        v = rng.uniform(-max_freq, max_freq)
        theta = rng.uniform(0.0, 2.0 * np.pi)
        xj = 2.0 * np.pi * u * jj / n + theta          # depends on the column
        yi = 2.0 * np.pi * v * ii / n                  # depends on the row
        L[:, 2 * t], L[:, 2 * t + 1] = a * np.cos(yi), a * np.sin(yi)
        R[2 * t], R[2 * t + 1] = np.sin(xj), np.cos(xj)
    M = L @ R if terms > 0 else np.zeros((rows, cols))
    if sigma > 0.0:
        M += sigma * rng.standard_normal((rows, cols))
    return M


def uniform_matrix(rows: int, cols: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=(rows, cols))


# The workloads: name -> recipe.  Sizes, term counts, frequencies, noise and
# seeds as stated for each configuration.
WORKLOADS = {
    # two 64x64 fields, 4 sinusoids of <= 2 cycles/side, N(0, 1e-3) noise
    "plain-64": dict(n=64, terms=4, freq=2.0, sigma=1e-3, seeds=(101, 102)),
    # two 8192x8192 fields, 16 sinusoids of <= 8 cycles/side, N(0, 1e-3) noise
    "plain-8192": dict(n=8192, terms=16, freq=8.0, sigma=1e-3, seeds=(201, 202)),
    # compressed 4096x4096 field times dense U[-1, 1]; 4096 dot vectors U[-1, 1]
    "linalg-4096": dict(n=4096, terms=16, freq=8.0, sigma=1e-3, seeds=(301, 302, 303)),
    # one 16384x16384 field, 32 sinusoids of <= 32 cycles/side, N(0, 1e-4) noise
    "mixed-16384": dict(n=16384, terms=32, freq=32.0, sigma=1e-4, seeds=(401,)),
}


def workload_inputs(name: str, n: int | None = None):
    """The field(s) of a workload; ``n`` overrides the side (smaller test copies)."""
    w = WORKLOADS[name]
    side = w["n"] if n is None else n
    if name == "linalg-4096":
        A = smooth_field(side, w["terms"], w["freq"], w["sigma"], w["seeds"][0])
        B = uniform_matrix(side, side, w["seeds"][1])
        V = uniform_matrix(side, side, w["seeds"][2])
        return A, B, V
    return tuple(smooth_field(side, w["terms"], w["freq"], w["sigma"], s) for s in w["seeds"])
