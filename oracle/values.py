"""Correlator values in complex128 (the plain definition the method must reach).

Every graph is evaluated on its own from its op list, without the DAG's
sharing: the scheduling and eviction machinery changes only the order of work
and where tensors live, never the values, so the result is simply the full
contraction of each graph's tree at every time slice t.

Kinds, per time slice t (no index conventions are printed in the paper; these
are the engine's, with contracted axes trailing on the left operand and
leading on the right; the contraction costs O(N^3), O(N^4), O(N^4)/O(N^5) as
the paper states for meson and baryon systems):
  K22: O[i,j]   = sum_k  X[i,k]   Y[k,j]
  K32: O[i,j,l] = sum_k  X[i,j,k] Y[k,l]
  K33: O[i,m]   = sum_jl X[i,j,l] Y[j,l,m]
  HCA: C        = sum_ij P[i,j]   Q[j,i]       (the root's "contract all")
  C1, C2, C3: the last c = 1, 2, 3 axes of X against the first c axes of Y,
       e.g. C1 on two rank-3 tensors: O[i,j,l,m] = sum_k X[i,j,k] Y[k,l,m]
       (rank 4, O(N^5) per time slice); K22, K32 and K33 are C1, C1 and C2
       on ranks (2,2), (3,2) and (3,3).
  General pairs (kind SPEC_BASE + i, the workload's spec i): the axes
       pairs[k] = (a_k of X, b_k of Y) are summed; the output holds X's free
       axes in X's order, then Y's free axes in Y's order, rearranged so that
       output axis j is axis perm[j] of that list.
The cross-diagram sum of a correlator c is S_c(t) = sum_{g in c} w_g C_g(t),
taken as a correctly rounded sum (math.fsum) of the FP64 terms.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

K22, K32, K33, HCA = 0, 1, 2, 3
C1, C2, C3 = 4, 5, 6
SPEC_BASE = 16
_AXES = {K22: 1, K32: 1, K33: 2, C1: 1, C2: 2, C3: 3}


def contract_pairs(X: np.ndarray, Y: np.ndarray, pairs, perm) -> np.ndarray:
    """The general contraction written as one einsum, batched over the leading t
    axis: summed labels are shared by the paired axes; the output labels are X's
    free ones, then Y's, taken in the order perm gives."""
    rl, rr = X.ndim - 1, Y.ndim - 1
    letters = iter("abcdefghijklmnopqrsuvwxyz")      # t is the time slice
    lx = [next(letters) for _ in range(rl)]
    ly = [None] * rr
    for a, b in pairs:
        ly[b] = lx[a]
    for j in range(rr):
        if ly[j] is None:
            ly[j] = next(letters)
    paired_x = {a for a, _ in pairs}
    paired_y = {b for _, b in pairs}
    natural = [lx[i] for i in range(rl) if i not in paired_x] + [ly[j] for j in range(rr) if j not in paired_y]
    out = "".join(natural[p] for p in perm)
    return np.einsum(f"t{''.join(lx)},t{''.join(ly)}->t{out}", X, Y)


def contract(kind: int, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """One binary contraction batched over the leading t axis, in complex128.

    A batched matrix product (numpy.matmul) is the library primitive; the
    reshapes only group the free and contracted axes of the definitions above
    (free axes of X, then the c contracted ones; contracted axes of Y, then its
    free ones)."""
    if kind == HCA:
        return np.einsum("tij,tji->t", X, Y)
    nt, n = X.shape[0], X.shape[1]
    c = _AXES[kind]
    rl, rr = X.ndim - 1, Y.ndim - 1
    out = np.matmul(X.reshape(nt, n ** (rl - c), n ** c), Y.reshape(nt, n ** c, n ** (rr - c)))
    return out.reshape((nt,) + (n,) * (rl + rr - 2 * c))


def contract_einsum(kind: int, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """The same definitions written as plain einsum index strings (small inputs)."""
    if kind == HCA:
        return np.einsum("tij,tji->t", X, Y)
    c = _AXES[kind]
    rl, rr = X.ndim - 1, Y.ndim - 1
    free_l, summed, free_r = "abcd"[:rl - c], "efg"[:c], "hijk"[:rr - c]
    return np.einsum(f"t{free_l}{summed},t{summed}{free_r}->t{free_l}{free_r}", X, Y)


def evaluate_graph(leaves: Sequence[np.ndarray], ops, specs=()) -> np.ndarray:
    """C_g(t) for one graph: its ops in order; operand >= 0 is a leaf, < 0 an earlier op;
    a kind SPEC_BASE + i uses specs[i] (objects with .pairs and .perm)."""
    vals: List[np.ndarray] = []
    for kind, l, r in ops:
        X = np.asarray(leaves[l], dtype=np.complex128) if l >= 0 else vals[-l - 1]
        Y = np.asarray(leaves[r], dtype=np.complex128) if r >= 0 else vals[-r - 1]
        if kind >= SPEC_BASE:
            sp = specs[kind - SPEC_BASE]
            vals.append(contract_pairs(X, Y, sp.pairs, sp.perm))
        else:
            vals.append(contract(kind, X, Y))
    return vals[-1]


def correlators(workload, graphs: Sequence[int] = None) -> Dict[int, np.ndarray]:
    """{graph index: complex128 [nt]} for the chosen graphs (all by default)."""
    data = [lf.data for lf in workload.leaves]
    specs = getattr(workload, "specs", ())
    idx = range(len(workload.graphs)) if graphs is None else graphs
    return {g: evaluate_graph(data, workload.graphs[g].ops, specs) for g in idx}


def trace4_loops(A, B, C, D) -> np.ndarray:
    """tr(A B C D) per t by explicit index loops (tiny inputs only)."""
    nt, n = A.shape[0], A.shape[1]
    out = np.zeros(nt, dtype=np.complex128)
    for t in range(nt):
        a, b, c, d = (M[t].tolist() for M in (A, B, C, D))
        s = 0j
        for i in range(n):
            for j in range(n):
                aij = a[i][j]
                for k in range(n):
                    abk = aij * b[j][k]
                    ck = c[k]
                    for l in range(n):
                        s += abk * ck[l] * d[l][i]
        out[t] = s
    return out


def cross_sums(workload, corr_values: Dict[int, np.ndarray]) -> Dict[int, np.ndarray]:
    """S_c(t) = sum_g w_g C_g(t), correctly rounded per component (math.fsum)."""
    by_corr: Dict[int, List[int]] = {}
    for g, spec in enumerate(workload.graphs):
        by_corr.setdefault(spec.corr, []).append(g)
    out = {}
    for c, gs in by_corr.items():
        nt = len(corr_values[gs[0]])
        s = np.zeros(nt, dtype=np.complex128)
        for t in range(nt):
            terms = [complex(workload.graphs[g].w) * complex(corr_values[g][t]) for g in gs]
            s[t] = complex(math.fsum(z.real for z in terms), math.fsum(z.imag for z in terms))
        out[c] = s
    return out


def cross_sum_scale(workload, corr_values: Dict[int, np.ndarray]) -> Dict[int, np.ndarray]:
    """sum_g |w_g C_g(t)| per correlator: the condition-aware error scale for S_c(t)."""
    out: Dict[int, np.ndarray] = {}
    for g, spec in enumerate(workload.graphs):
        v = np.abs(complex(spec.w) * corr_values[g])
        out[spec.corr] = out.get(spec.corr, 0) + v
    return out
