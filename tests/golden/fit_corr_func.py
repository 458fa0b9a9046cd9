"""Fit the leaf-draw skew of each Table corr-func-shaped generator
(synth/corr_func.py) so that the merged DAG has about the row's number of
vertices.  Builds the DAGs with the oracle only; prints the skews to paste into
synth.corr_func.PARAMS.

    python tests/golden/fit_corr_func.py [row ...]
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dag as OD          # noqa: E402
from synth import corr_func as CF     # noqa: E402


def vertices(row, skew):
    wl = CF.corr_func_like(row, skew=skew)
    return OD.build(wl.leaves, wl.graphs).n_nodes


def fit(row, iters=14):
    target = CF.TABLE[row]["V"]
    lo, hi = 0.0, 4.0
    if vertices(row, lo) <= target:
        return lo, vertices(row, lo)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if vertices(row, mid) > target:
            lo = mid
        else:
            hi = mid
    s = round(0.5 * (lo + hi), 4)
    return s, vertices(row, s)


if __name__ == "__main__":
    rows = sys.argv[1:] or list(CF.TABLE)
    for row in rows:
        s, v = fit(row)
        print(f"{row}: skew={s}  vertices={v} (table {CF.TABLE[row]['V']})", flush=True)
