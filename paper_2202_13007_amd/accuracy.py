"""Accuracy of the method on the paper's analytic test matrices (Table 1).

Section "Accuracy Measurements": M_k[i, j] = f_k(x_j, y_i) for the six
functions of Figure "figcurves", with the points on a uniform grid of
[-2, 2] x [-2, 2].  The paper states neither n nor the grid convention; here
the grid is numpy.linspace(-2, 2, n) on both axes (both end points
included) and n is swept.  The error of a result M' against the exact M is
the mean relative error of Eq. "eqmean", (1/n^2) sum |M'_ij - M_ij| / |M_ij|;
the paper does not say what happens where M_ij = 0, so such entries are
left out of the mean (and counted), and the normwise error
||M' - M||_F / ||M||_F is reported beside it.

Rows of the table, all computed with the library's kernels:
* compression / decompression: M' = decompress(compress(M_k));
* additions: M' = decompress(add(compress(M_i), compress(M_j))), i < j;
* multiplication by 2: M' = decompress(scale(compress(M_k), 2));
* products: M' = matmul(compress(M_i), compress(M_j)) (both partly
  decompressed, binary64 output) against the exact binary64 product M_i M_j.

Usage: python -m paper_2202_13007_amd.accuracy [--n 80 496 1000 2000] [--json PATH]
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np
import torch

from . import api

# The six functions of Figure "figcurves".
FUNCTIONS = {
    1: lambda x, y: x * y,
    2: lambda x, y: x * y / (1.0 + x * x + y * y),
    3: lambda x, y: x * x - y,
    4: lambda x, y: x * x * y * y,
    5: lambda x, y: np.cos(np.sqrt(x * x + y * y)),
    6: lambda x, y: np.cos(x * x + y * y) * np.exp(-0.1 * (x * x + y * y)),
}

# The blaz rows of Table 1 as printed (percent for the first three parts,
# plain relative error for the products; additions are the upper triangle).
PAPER_TABLE1 = {
    "compress": [0.43, 0.39, 0.53, 0.44, 1.95, 1.17],
    "add": {(1, 2): 0.98, (1, 3): 0.67, (1, 4): 0.91, (1, 5): 0.72, (1, 6): 0.78,
            (2, 3): 0.62, (2, 4): 1.07, (2, 5): 1.76, (2, 6): 1.61,
            (3, 4): 2.27, (3, 5): 0.71, (3, 6): 0.65,
            (4, 5): 1.68, (4, 6): 1.70,
            (5, 6): 0.94},
    "scale2": [0.43, 0.44, 0.53, 0.44, 1.95, 1.17],
    "matmul": [[2.0e-4, 2.0e-4, 1.0e-4, 5.1e-2, 3.6e-2, 9.2e-2],
               [2.0e-4, 2.0e-4, 1.0e-4, 5.3e-2, 3.6e-2, 1.0e-1],
               [3.4e-2, 3.5e-2, 7.9e-3, 9.0e-4, 5.0e-4, 5.0e-4],
               [3.7e-2, 3.4e-2, 2.1e-3, 8.0e-4, 6.0e-4, 5.0e-4],
               [4.4e-2, 4.5e-2, 1.7e-3, 8.0e-4, 1.1e-3, 1.7e-3],
               [1.8e-1, 3.7e-1, 2.0e-2, 8.0e-4, 7.0e-4, 2.9e-3]],
}


def analytic_matrix(k: int, n: int) -> np.ndarray:
    """M_k[i, j] = f_k(x_j, y_i), x and y = linspace(-2, 2, n)."""
    v = np.linspace(-2.0, 2.0, n)
    X, Y = np.meshgrid(v, v)  # X[i, j] = v[j], Y[i, j] = v[i]
    return np.ascontiguousarray(FUNCTIONS[k](X, Y), dtype=np.float64)


def errors(Mp: torch.Tensor, M: torch.Tensor) -> dict:
    """Mean relative error (Eq. eqmean, zeros of M left out) and normwise error."""
    nz = M != 0
    rel = torch.abs(Mp - M)[nz] / torch.abs(M[nz])
    return {"mean_rel": float(rel.mean().item()) if rel.numel() else math.nan,
            "zeros_excluded": int((~nz).sum().item()),
            "norm_rel": float((torch.linalg.norm(Mp - M) / torch.linalg.norm(M)).item())}


def table(n: int, device: str = "cuda") -> dict:
    """Every blaz row of Table 1 at size n (n a multiple of 8)."""
    M = {k: torch.from_numpy(analytic_matrix(k, n)).to(device) for k in FUNCTIONS}
    C = {k: api.compress(M[k]) for k in M}
    out = {"n": n, "grid": "linspace(-2, 2, n) on both axes", "compress": {}, "add": {}, "scale2": {},
           "matmul": {}}
    for k in M:
        out["compress"][k] = errors(api.decompress(C[k]), M[k])
        out["scale2"][k] = errors(api.decompress(api.scale(C[k], 2.0)), 2.0 * M[k])
    for i in M:
        for j in M:
            if i < j:
                out["add"][(i, j)] = errors(api.decompress(api.add(C[i], C[j])), M[i] + M[j])
            out["matmul"][(i, j)] = errors(api.matmul(C[i], C[j]), M[i] @ M[j])
    return out


def with_paper(t: dict) -> dict:
    """The table as JSON-ready rows, each measured value beside the printed one."""
    rows = {}
    for k in range(1, 7):
        rows[f"compress M{k}"] = dict(t["compress"][k], paper_mean_rel=PAPER_TABLE1["compress"][k - 1] / 100)
        rows[f"scale2 M{k}"] = dict(t["scale2"][k], paper_mean_rel=PAPER_TABLE1["scale2"][k - 1] / 100)
    for (i, j), e in t["add"].items():
        rows[f"add M{i}+M{j}"] = dict(e, paper_mean_rel=PAPER_TABLE1["add"][(i, j)] / 100)
    for (i, j), e in t["matmul"].items():
        rows[f"matmul M{i}xM{j}"] = dict(e, paper_mean_rel=PAPER_TABLE1["matmul"][i - 1][j - 1])
    return {"n": t["n"], "grid": t["grid"], "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, nargs="+", default=[80, 496, 1000, 2000])
    ap.add_argument("--json", default=None, help="write the tables here")
    args = ap.parse_args()
    res = []
    for n in args.n:
        t = with_paper(table(n))
        res.append(t)
        print(f"n = {n}")
        for name, r in t["rows"].items():
            print(f"  {name:<16} mean_rel {r['mean_rel']:.3e}  paper {r['paper_mean_rel']:.3e}  "
                  f"norm_rel {r['norm_rel']:.3e}  zeros {r['zeros_excluded']}")
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
