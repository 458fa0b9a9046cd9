"""Pins of the oracle's correlator values (CPU only).

  * Brute force: tr(A_a A_b A_c A_d) by explicit index loops on the tiny workload.
  * Cyclic invariance of the trace and invariance under re-parenthesisation.
  * Identity leaves give tr(I^L) = N exactly; X.I = X exactly.
  * Permutation and selector tensors pick out entries exactly, which fixes every
    index convention (a transposed operand or wrong contracted axis fails).
  * Linearity in each leaf; the cross-diagram sum is correctly rounded.
  * General contractions (C1, C2, C3 over operand ranks 2..4) against explicit
    index loops.
"""
import itertools
import math

import numpy as np
import pytest

from synth import workloads as W
from oracle import values as V


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def tiny():
    return W.config("tiny")


def test_tiny_brute_force(tiny):
    vals = V.correlators(tiny)
    L = [lf.data for lf in tiny.leaves]
    for g, spec in enumerate(tiny.graphs):
        a, b = spec.ops[0][1:]
        c, d = spec.ops[1][1:]
        ref = V.trace4_loops(L[a], L[b], L[c], L[d])
        assert rel(vals[g], ref) < 1e-13


def test_cyclic_and_parenthesisation(tiny):
    L = [lf.data for lf in tiny.leaves]
    K22, HCA = W.K22, W.HCA
    base = V.evaluate_graph(L, [(K22, 0, 1), (K22, 2, 3), (HCA, -1, -2)])
    cyc = V.evaluate_graph(L, [(K22, 1, 2), (K22, 3, 0), (HCA, -1, -2)])
    cyc2 = V.evaluate_graph(L, [(K22, 3, 0), (K22, 1, 2), (HCA, -1, -2)])
    left = V.evaluate_graph(L, [(K22, 0, 1), (K22, -1, 2), (HCA, -2, 3)])
    right = V.evaluate_graph(L, [(K22, 2, 3), (K22, 1, -1), (HCA, 0, -2)])
    for v in (cyc, cyc2, left, right):
        assert rel(v, base) < 1e-13


def _ident(nt, n):
    return np.broadcast_to(np.eye(n, dtype=np.complex128), (nt, n, n)).copy()


def test_identity_leaves_exact():
    nt, n = 3, 7
    L = [_ident(nt, n) for _ in range(4)]
    ops = [(W.K22, 0, 1), (W.K22, -1, 2), (W.HCA, -2, 3)]
    assert np.array_equal(V.evaluate_graph(L, ops), np.full(nt, n, dtype=np.complex128))
    X = W._draw(np.random.default_rng(1), (nt, n, n), 1.0)
    assert np.array_equal(V.contract(W.K22, X, L[0]), X)
    assert np.array_equal(V.contract(W.K22, L[0], X), X)


def test_permutation_and_selector_tensors():
    rng = np.random.default_rng(2)
    nt, n = 2, 5
    pi = rng.permutation(n)
    perm = np.zeros((nt, n, n), dtype=np.complex128)
    for a in range(n):
        perm[:, a, pi[a]] = 1.0          # perm[k, j] = 1 iff j = pi(k)
    X2 = W._draw(rng, (nt, n, n), 1.0)
    X3 = W._draw(rng, (nt, n, n, n), 1.0)
    inv = np.argsort(pi)
    # K22: (X.perm)[i,j] = X[i, pi^-1(j)];  (perm.X)[i,j] = X[pi(i), j]
    assert np.array_equal(V.contract(W.K22, X2, perm), X2[:, :, inv])
    assert np.array_equal(V.contract(W.K22, perm, X2), X2[:, pi, :])
    # K32: O[i,j,l] = X[i,j,pi^-1(l)]
    assert np.array_equal(V.contract(W.K32, X3, perm), X3[:, :, :, inv])
    # K33 with E[j,l,m] = delta(j,m) delta(l,0): O[i,m] = X[i,m,0]
    E = np.zeros((nt, n, n, n), dtype=np.complex128)
    for m in range(n):
        E[:, m, 0, m] = 1.0
    assert np.array_equal(V.contract(W.K33, X3, E), X3[:, :, :, 0])
    # K33 with E[j,l,m] = delta(l,m) delta(j,0): O[i,m] = X[i,0,m]
    E2 = np.zeros((nt, n, n, n), dtype=np.complex128)
    for m in range(n):
        E2[:, 0, m, m] = 1.0
    assert np.array_equal(V.contract(W.K33, X3, E2), X3[:, :, 0, :])
    # HCA(P, perm) = sum_i P[i, ...]: sum_ij P[i,j] perm[j,i] = sum_j P[pi(j), j]
    want = sum(X2[:, pi[j], j] for j in range(n))
    assert np.allclose(V.contract(W.HCA, X2, perm), want, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("kind", [W.K22, W.K32, W.K33, W.HCA])
def test_matmul_form_equals_einsum_form(kind):
    rng = np.random.default_rng(kind + 10)
    nt, n = 3, 6
    shp = {W.K22: ((2, 2)), W.K32: ((3, 2)), W.K33: ((3, 3)), W.HCA: ((2, 2))}[kind]
    X = W._draw(rng, (nt,) + (n,) * shp[0], 1.0)
    Y = W._draw(rng, (nt,) + (n,) * shp[1], 1.0)
    assert rel(V.contract(kind, X, Y), V.contract_einsum(kind, X, Y)) < 1e-14


GENERAL = [(W.C1, 3, 3), (W.C1, 4, 2), (W.C1, 2, 4), (W.C2, 4, 3), (W.C2, 3, 4), (W.C2, 4, 4),
           (W.C2, 4, 2), (W.C3, 4, 4), (W.C1, 3, 2), (W.C2, 3, 3)]


@pytest.mark.parametrize("kind,rl,rr", GENERAL)
def test_general_contraction_by_index_loops(kind, rl, rr):
    """O[a.., h..] = sum_e.. X[a.., e..] Y[e.., h..] with c = kind - 3 summed axes,
    written as loops over every index tuple (N = 3, two time slices)."""
    rng = np.random.default_rng(100 + 10 * kind + rl + rr)
    nt, n, c = 2, 3, kind - 3
    X = W._draw(rng, (nt,) + (n,) * rl, 1.0)
    Y = W._draw(rng, (nt,) + (n,) * rr, 1.0)
    ro = rl + rr - 2 * c
    want = np.zeros((nt,) + (n,) * ro, dtype=np.complex128)
    for t in range(nt):
        for fl in itertools.product(range(n), repeat=rl - c):
            for fr in itertools.product(range(n), repeat=rr - c):
                acc = 0j
                for sm in itertools.product(range(n), repeat=c):
                    acc += X[(t,) + fl + sm] * Y[(t,) + sm + fr]
                want[(t,) + fl + fr] = acc
    got = V.contract(kind, X, Y)
    assert got.shape == want.shape
    assert rel(got, want) < 1e-14
    assert rel(V.contract_einsum(kind, X, Y), want) < 1e-14


def test_named_kinds_are_general_contractions():
    rng = np.random.default_rng(7)
    for named, general, rl, rr in ((W.K22, W.C1, 2, 2), (W.K32, W.C1, 3, 2), (W.K33, W.C2, 3, 3)):
        X = W._draw(rng, (2,) + (4,) * rl, 1.0)
        Y = W._draw(rng, (2,) + (4,) * rr, 1.0)
        assert np.array_equal(V.contract(named, X, Y), V.contract(general, X, Y))


def test_linearity():
    wl = W.baryon_mix(n_bar=3, n_mes=3, nvec=5, nt=2, n_graphs=4, seed=5)
    L = [lf.data for lf in wl.leaves]
    alpha = 0.75 - 0.5j
    for spec in wl.graphs:
        base = V.evaluate_graph(L, spec.ops)
        for leaf in {x for _, l, r in spec.ops for x in (l, r) if x >= 0}:
            L2 = list(L)
            L2[leaf] = alpha * L[leaf]
            assert rel(V.evaluate_graph(L2, spec.ops), alpha * base) < 1e-13


def test_cross_sum_correctly_rounded():
    class G:
        def __init__(self, corr, w):
            self.corr, self.w, self.ops = corr, w, []

    class Wl:
        graphs = [G(0, 1.0), G(0, 1.0), G(0, -1.0), G(1, 1.0)]

    vals = {0: np.array([1e16 + 0j]), 1: np.array([1.0 + 1e16j]),
            2: np.array([1e16 + 0j]), 3: np.array([3.0 - 2.0j])}
    s = V.cross_sums(Wl, vals)
    assert s[0][0] == complex(1.0, 1e16) and s[1][0] == 3.0 - 2.0j
    # exact for small integers regardless of order
    rng = np.random.default_rng(0)
    ints = rng.integers(-1000, 1000, size=100)
    assert math.fsum(float(i) for i in ints) == float(ints.sum())


def test_cross_sum_scale_by_hand():
    """sum_g |w_g C_g(t)|, the denominator of every cross-sum error bound, on
    values worked by hand: |3+4i| = 5, |2i (1+i)| = 2 sqrt 2, and a weight of
    -1 must count positively (a dropped abs or weight changes every entry)."""
    class G:
        def __init__(self, corr, w):
            self.corr, self.w, self.ops = corr, w, []

    class Wl:
        graphs = [G(0, 3 + 4j), G(0, -1.0), G(1, 2j), G(1, 0.5)]

    vals = {0: np.array([1 + 0j, 2j]), 1: np.array([3 - 4j, 0j]),
            2: np.array([1 + 1j, -1 + 0j]), 3: np.array([0j, -6 + 8j])}
    sc = V.cross_sum_scale(Wl, vals)
    assert set(sc) == {0, 1}
    assert np.allclose(sc[0], [5 + 5, 10 + 0], rtol=0, atol=1e-15)
    assert np.allclose(sc[1], [2 * math.sqrt(2) + 0, 2 + 5], rtol=0, atol=1e-15)
    # the scale bounds the sum it normalises: |S_c(t)| <= scale_c(t)
    s = V.cross_sums(Wl, vals)
    for c in sc:
        assert np.all(np.abs(s[c]) <= sc[c] * (1 + 1e-15))


def _loops_pairs(X, Y, pairs, perm):
    """The contraction over index pairs by explicit loops: every combination of
    free and summed indices, products accumulated into the output element the
    permutation names."""
    nt, n = X.shape[0], X.shape[1]
    rl, rr = X.ndim - 1, Y.ndim - 1
    px = [a for a, _ in pairs]
    py = [b for _, b in pairs]
    fx = [a for a in range(rl) if a not in px]
    fy = [b for b in range(rr) if b not in py]
    ro = len(fx) + len(fy)
    out = np.zeros((nt,) + (n,) * ro, dtype=np.complex128)
    for t in range(nt):
        for free in itertools.product(range(n), repeat=ro):
            natural = list(free)                       # indices of fx then fy
            s = 0j
            for summed in itertools.product(range(n), repeat=len(pairs)):
                ix = [0] * rl
                iy = [0] * rr
                for q, a in enumerate(fx):
                    ix[a] = natural[q]
                for q, b in enumerate(fy):
                    iy[b] = natural[len(fx) + q]
                for k in range(len(pairs)):
                    ix[px[k]] = summed[k]
                    iy[py[k]] = summed[k]
                s += X[(t, *ix)] * Y[(t, *iy)]
            # output axis j holds natural axis perm[j]
            out[(t, *[natural[perm[j]] for j in range(ro)])] = s
    return out


@pytest.mark.parametrize("i", range(len(W.PAIR_SPECS)))
def test_index_pair_contractions_by_loops(i):
    sp = W.PAIR_SPECS[i]
    rng = np.random.default_rng(40 + i)
    n, nt = 3, 2
    X = W._draw(rng, (nt,) + (n,) * sp.rank_l, 1.0)
    Y = W._draw(rng, (nt,) + (n,) * sp.rank_r, 1.0)
    got = V.contract_pairs(X, Y, sp.pairs, sp.perm)
    want = _loops_pairs(X, Y, sp.pairs, sp.perm)
    assert got.shape == want.shape
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


def test_index_pairs_hand_case():
    """X[i,j] = i + 2j, Y[i,k] = 1 + i k (n = 2): sum over i of X[i,j] Y[i,k],
    output (k, j): O[k,j] = (2j)(1) + (1 + 2j)(1 + k)."""
    X = np.array([[[0, 2], [1, 3]]], dtype=np.complex128)       # X[0][i][j] = i + 2j
    Y = np.array([[[1, 1], [1, 2]]], dtype=np.complex128)       # Y[0][i][k] = 1 + i k
    got = V.contract_pairs(X, Y, ((0, 0),), (1, 0))
    want = np.array([[[2 * j + (1 + 2 * j) * (1 + k) for j in range(2)] for k in range(2)]], dtype=np.complex128)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("c,rl,rr", [(1, 2, 2), (1, 3, 2), (2, 3, 3), (1, 3, 3), (2, 4, 3), (3, 4, 4)])
def test_trailing_leading_pairs_are_the_general_kinds(c, rl, rr):
    """Pairs (last c axes of X, first c axes of Y) in order with the natural
    output order are C_c (and so K22, K32, K33): the batched-matmul route."""
    rng = np.random.default_rng(7 * c + rl + rr)
    n, nt = 3, 2
    X = W._draw(rng, (nt,) + (n,) * rl, 1.0)
    Y = W._draw(rng, (nt,) + (n,) * rr, 1.0)
    pairs = tuple((rl - c + k, k) for k in range(c))
    ro = rl + rr - 2 * c
    got = V.contract_pairs(X, Y, pairs, tuple(range(ro)))
    assert np.allclose(got, V.contract((V.C1, V.C2, V.C3)[c - 1], X, Y), rtol=1e-13, atol=1e-13)
