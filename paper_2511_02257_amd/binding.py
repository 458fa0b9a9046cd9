"""ctypes binding of libcdagx.so (include/cdag.h): argument marshalling only.

Module-level functions carry the C ABI's names; `Context` wraps one cdag_ctx.
Every call raises CdagError on a non-zero status.  The library must have been
built (paper_2511_02257_amd/build.py); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcdagx.so")

OK, E_INVALID, E_STATE, E_BUDGET, E_HIP, E_NOMEM, E_RANGE = 0, -1, -2, -3, -4, -5, -6
K22, K32, K33, HCA = 0, 1, 2, 3
POLICY = {"input": 0, "sibling": 1, "tree": 2, "node": 3}
SCHED_CHECK = 0x100
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
OP_NAMES = {0: "D2H", 1: "DROP", 2: "H2D", 3: "ALLOC", 4: "EXEC", 5: "FREE"}
UNLIMITED = (1 << 64) - 1


class CdagError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cdag error {code}: {msg}")
        self.code = code


class cdag_leaf(C.Structure):
    _fields_ = [("rank", C.c_int32), ("nvec", C.c_int32), ("nt", C.c_int32),
                ("dtype", C.c_int32), ("host", C.c_void_p)]


class cdag_op(C.Structure):
    _fields_ = [("kind", C.c_int32), ("left", C.c_int32), ("right", C.c_int32)]


class cdag_spec(C.Structure):
    _fields_ = [("rank_l", C.c_int32), ("rank_r", C.c_int32), ("n_pairs", C.c_int32),
                ("pair_l", C.c_int32 * 3), ("pair_r", C.c_int32 * 3), ("perm", C.c_int32 * 4)]


SPEC_BASE = 16


class cdag_graph(C.Structure):
    _fields_ = [("n_ops", C.c_int32), ("corr_id", C.c_int32), ("ops", C.POINTER(cdag_op)),
                ("w_re", C.c_double), ("w_im", C.c_double)]


_PLAN_INT = ["n_nodes", "n_leaves", "n_contr", "n_roots", "n_steps", "peak_post", "peak_live",
             "peak_resident", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes", "budget",
             "arena_bytes", "tensor_highwater", "host_spill_bytes", "hec_items"]
_PLAN_DBL = ["flops", "t_sched_s", "t_plan_s"]


class cdag_plan_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in _PLAN_INT] + [(n, C.c_double) for n in _PLAN_DBL]


class cdag_exec_stats(C.Structure):
    _fields_ = [("plan", cdag_plan_stats), ("t_total_s", C.c_double), ("t_device_s", C.c_double),
                ("t_hec_s", C.c_double), ("hec_flops", C.c_double), ("hec_bytes", C.c_double),
                ("n_launches", C.c_int64), ("n_hec_launches", C.c_int64),
                ("n_graph_segments", C.c_int64), ("t_kernels_s", C.c_double), ("t_copy_s", C.c_double),
                ("arena_highwater", C.c_int64)]


class cdag_launch_record(C.Structure):
    _fields_ = [("type", C.c_int32), ("variant", C.c_int32), ("kinds", C.c_int32),
                ("interior", C.c_int32), ("step", C.c_int64), ("n_items", C.c_int64),
                ("flops", C.c_double), ("bytes", C.c_double), ("ms", C.c_double),
                ("trace_items", C.c_int64), ("trace_flops", C.c_double), ("trace_bytes", C.c_double)]


LAUNCH_TYPES = {0: "hec", 1: "reduce", 2: "hca", 3: "xsum", 4: "h2d", 5: "d2h"}


class cdag_trace_rec(C.Structure):
    _fields_ = [("op", C.c_int32), ("stream", C.c_int32), ("seq", C.c_int64), ("step", C.c_int64),
                ("node", C.c_int64), ("event", C.c_int64), ("space", C.c_int32), ("reserved", C.c_int32),
                ("off", C.c_int64), ("bytes", C.c_int64)]


TRACE_OPS = {0: "record", 1: "wait", 2: "read", 3: "write"}
TRACE_SPACES = {0: "arena", 1: "spill", 2: "stage"}

_lib = None


def lib():
    """Load the built library (raises if it has not been built).

    PyTorch ships its own HIP runtime under the same soname as the system one.
    torch is imported first so that the library binds to that same runtime:
    the arena pointer and stream handles it borrows from torch are only valid
    inside the runtime that created them, and two runtimes in one process do
    not share the device."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2511_02257_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, I64, I32 = C.c_void_p, C.c_int64, C.c_int32
        sig = {
            "cdag_create": [C.POINTER(C.c_void_p)],
            "cdag_destroy": [P],
            "build_cdag": [P, C.POINTER(cdag_leaf), I64, C.POINTER(cdag_graph), I64],
            "cdag_build_general": [P, I64, I64, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)],
            "cdag_set_specs": [P, C.POINTER(cdag_spec), I64],
            "schedule": [P, C.c_int, C.POINTER(I64), I64, C.POINTER(I64)],
            "set_mem_budget": [P, C.c_uint64],
            "cdag_set_order": [P, C.POINTER(I64), I64],
            "cdag_set_options": [P, C.c_int, C.c_int, I64, C.c_int],
            "cdag_set_timing": [P, C.c_int],
            "cdag_set_time_chunks": [P, I64],
            "cdag_set_trace_fusion": [P, C.c_int],
            "cdag_dag_stats": [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)],
            "cdag_launch_records": [P, C.POINTER(cdag_launch_record), I64, C.POINTER(I64)],
            "cdag_trace_execute": [P, C.c_int, C.c_int, C.POINTER(cdag_trace_rec), I64, C.POINTER(I64), I64],
            "cdag_set_tile": [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int],
            "cdag_get_tile": [P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                              C.POINTER(C.c_int), C.POINTER(C.c_int)],
            "cdag_memsim": [P, C.POINTER(I64), I64, C.c_int, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)],
            "cdag_plan": [P, C.c_int, C.c_int, C.POINTER(cdag_plan_stats)],
            "cdag_plan_ops": [P, C.POINTER(I32), C.POINTER(I64), C.POINTER(I64), I64, C.POINTER(I64)],
            "cdag_get_nodes": [P, C.POINTER(I32), C.POINTER(I64), C.POINTER(I64), I64, C.POINTER(I64)],
            "cdag_graph_roots": [P, C.POINTER(I64), I64],
            "cdag_bind_device": [P, C.c_int, P, P],
            "cdag_bind_arena": [P, P, C.c_uint64],
            "execute": [P, C.c_int, C.c_int, C.POINTER(cdag_exec_stats)],
            "cdag_execute_static": [P, C.c_int, C.c_int, C.POINTER(cdag_exec_stats)],
            "cdag_autotune": [P, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(I64)],
            "fetch_correlators": [P, C.POINTER(C.c_double), I64],
            "cdag_fetch_sums": [P, C.POINTER(C.c_double), I64],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.cdag_last_error.argtypes = []
        L.cdag_last_error.restype = C.c_char_p
        _lib = L
    return _lib


EXPORTED = ("cdag_create", "cdag_destroy", "cdag_last_error", "build_cdag", "cdag_build_general",
            "cdag_set_specs", "schedule",
            "set_mem_budget", "cdag_set_order", "cdag_set_options", "cdag_set_timing", "cdag_set_time_chunks",
            "cdag_set_trace_fusion",
            "cdag_launch_records",
            "cdag_trace_execute", "cdag_dag_stats", "cdag_set_tile", "cdag_get_tile", "cdag_memsim",
            "cdag_plan", "cdag_plan_ops",
            "cdag_get_nodes", "cdag_graph_roots", "cdag_bind_device", "cdag_bind_arena",
            "execute", "cdag_execute_static", "cdag_autotune", "fetch_correlators", "cdag_fetch_sums")


def _check(rc: int):
    if rc != OK:
        raise CdagError(rc, lib().cdag_last_error().decode(errors="replace"))


def _i64p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _struct_dict(s) -> dict:
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        out[name] = _struct_dict(v) if isinstance(v, C.Structure) else v
    return out


# ------------------------------------------------------------------ functions with the C names
def cdag_create() -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().cdag_create(C.byref(h)))
    return h


def cdag_destroy(h) -> None:
    _check(lib().cdag_destroy(h))


def build_cdag(h, leaves: Sequence, graphs: Sequence) -> None:
    """leaves: objects with rank, nvec, nt and data (complex128 [nt]+[nvec]*rank, or None);
    graphs: objects with ops [(kind, left, right)], corr and w."""
    n = len(leaves)
    L = (cdag_leaf * max(1, n))()
    keep = []
    for i, lf in enumerate(leaves):
        L[i].rank, L[i].nvec, L[i].nt = lf.rank, lf.nvec, lf.nt
        if getattr(lf, "data", None) is not None:
            dt = np.complex64 if lf.data.dtype == np.complex64 else np.complex128
            a = np.ascontiguousarray(lf.data, dtype=dt)
            if a.size != lf.nt * lf.nvec ** lf.rank:
                raise ValueError(f"leaf {i}: data has {a.size} elements")
            keep.append(a)
            L[i].dtype = 1 if dt == np.complex64 else 0
            L[i].host = a.ctypes.data
        else:
            L[i].dtype = 0
            L[i].host = None
    G = (cdag_graph * max(1, len(graphs)))()
    for g, spec in enumerate(graphs):
        ops = (cdag_op * len(spec.ops))(*[cdag_op(k, l, r) for k, l, r in spec.ops])
        keep.append(ops)
        w = complex(getattr(spec, "w", 1.0))
        G[g].n_ops, G[g].corr_id, G[g].ops = len(spec.ops), int(getattr(spec, "corr", 0)), ops
        G[g].w_re, G[g].w_im = w.real, w.imag
    _check(lib().build_cdag(h, L, n, G, len(graphs)))
    del keep


def cdag_set_specs(h, specs: Sequence) -> None:
    """specs: objects with rank_l, rank_r, pairs [(left axis, right axis), ...] and perm."""
    arr = (cdag_spec * max(1, len(specs)))()
    for i, sp in enumerate(specs):
        arr[i].rank_l, arr[i].rank_r, arr[i].n_pairs = sp.rank_l, sp.rank_r, len(sp.pairs)
        for k, (a, b) in enumerate(sp.pairs):
            arr[i].pair_l[k], arr[i].pair_r[k] = a, b
        for j, q in enumerate(sp.perm):
            arr[i].perm[j] = q
    _check(lib().cdag_set_specs(h, arr, len(specs)))


def cdag_build_general(h, n_leaves: int, sizes: Sequence[int], children: Sequence[Sequence[int]]) -> None:
    """A general DAG: sizes[u] in bytes for every node, children[u] (empty for the
    n_leaves leaves) in operand order."""
    n = len(sizes)
    if len(children) != n:
        raise ValueError("sizes and children differ in length")
    size = np.ascontiguousarray(sizes, dtype=np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(c) for c in children])
    flat = np.ascontiguousarray([x for c in children for x in c] or [0], dtype=np.int64)
    _check(lib().cdag_build_general(h, n, int(n_leaves), _i64p(size) if n else None, _i64p(off),
                                    _i64p(flat)))


def schedule(h, policy: str, check: bool = False) -> np.ndarray:
    """One schedule call: the order has at most one entry per DAG node."""
    p = POLICY[policy] | (SCHED_CHECK if check else 0)
    cap = max(1, cdag_dag_stats(h)["n_vertices"])
    out = np.empty(cap, dtype=np.int64)
    n = C.c_int64()
    _check(lib().schedule(h, p, _i64p(out), cap, C.byref(n)))
    return out[:n.value].copy()


def cdag_set_order(h, order: Sequence[int]) -> None:
    a = np.ascontiguousarray(order, dtype=np.int64)
    _check(lib().cdag_set_order(h, _i64p(a), len(a)))


def set_mem_budget(h, nbytes: Optional[int]) -> None:
    _check(lib().set_mem_budget(h, UNLIMITED if nbytes is None else int(nbytes)))


LOOKAHEAD_ALL = (1 << 63) - 1


GRAPH_MODES = {0: "eager", 1: "one-stream segments", 2: "three-stream graph"}


def cdag_set_options(h, leaves_resident=False, wave_max=4096, wave_lookahead=0,
                     use_graphs=1) -> None:
    """use_graphs: 0 (or False) eager, 1 (or True) one-stream captured segments,
    2 one three-stream captured graph."""
    _check(lib().cdag_set_options(h, int(leaves_resident), int(wave_max), int(wave_lookahead),
                                  int(use_graphs)))


def cdag_set_time_chunks(h, t_chunks: int) -> None:
    _check(lib().cdag_set_time_chunks(h, int(t_chunks)))


def cdag_set_trace_fusion(h, on: bool) -> None:
    _check(lib().cdag_set_trace_fusion(h, int(bool(on))))


def cdag_set_timing(h, on: bool) -> None:
    _check(lib().cdag_set_timing(h, int(bool(on))))


def cdag_dag_stats(h):
    """{n_vertices, n_edges, n_trees, f_v, f_e} of the merged DAG."""
    v, e, k = C.c_int64(), C.c_int64(), C.c_int64()
    fv, fe = C.c_double(), C.c_double()
    _check(lib().cdag_dag_stats(h, C.byref(v), C.byref(e), C.byref(k), C.byref(fv), C.byref(fe)))
    return {"n_vertices": v.value, "n_edges": e.value, "n_trees": k.value, "f_v": fv.value,
            "f_e": fe.value}


def cdag_launch_records(h):
    """Per-launch and per-transfer records of the last timed execute, as a list of dicts."""
    n = C.c_int64()
    _check(lib().cdag_launch_records(h, None, 0, C.byref(n)))
    buf = (cdag_launch_record * max(1, n.value))()
    _check(lib().cdag_launch_records(h, buf, n.value, C.byref(n)))
    out = []
    for r in buf[:n.value]:
        out.append({"type": LAUNCH_TYPES[r.type], "variant": r.variant, "interior": bool(r.interior),
                    "kinds": [k for k in range(8) if r.kinds >> k & 1], "step": r.step,
                    "n_items": r.n_items, "flops": r.flops, "bytes": r.bytes, "ms": r.ms,
                    "trace_items": r.trace_items, "trace_flops": r.trace_flops, "trace_bytes": r.trace_bytes})
    return out


TILES = {0: (64, 64), 1: (32, 32), 2: (48, 48), 3: (128, 64), 4: (64, 32), 5: (64, 64)}
TILE_THREADS = {0: 256, 1: 256, 2: 64, 3: 256, 4: 256, 5: 512}


GRIDS = {0: "persistent", 1: "one workgroup per item"}


def variant_index(tile: int, grid: int, lds_stages: int) -> int:
    """The library's single-integer encoding of a kernel variant."""
    return tile + len(TILES) * (grid + 2 * (2 - lds_stages))


def cdag_trace_execute(h, prec: str = "fp64", batched: bool = False, fail_at: int = -1) -> List[dict]:
    """The eager two-stream issue order of an execute, recorded without HIP."""
    n = C.c_int64()
    _check(lib().cdag_trace_execute(h, PREC[prec], int(batched), None, 0, C.byref(n), int(fail_at)))
    buf = (cdag_trace_rec * max(1, n.value))()
    _check(lib().cdag_trace_execute(h, PREC[prec], int(batched), buf, n.value, C.byref(n), int(fail_at)))
    return [{"op": TRACE_OPS[r.op], "stream": r.stream, "seq": r.seq, "step": r.step, "node": r.node,
             "event": r.event, "space": TRACE_SPACES.get(r.space), "off": r.off, "bytes": r.bytes}
            for r in buf[:n.value]]


def cdag_set_tile(h, prec: str, kind: int, nvec: int, tile: int, grid: int = 1,
                  lds_stages: int = 2, split_k: int = 1) -> None:
    _check(lib().cdag_set_tile(h, PREC[prec], int(kind), int(nvec), int(tile), int(grid),
                               int(lds_stages), int(split_k)))


def cdag_get_tile(h, prec: str, kind: int, nvec: int):
    """(tile, grid, lds_stages, split_k) in force for that shape."""
    t, g, st, sk = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    _check(lib().cdag_get_tile(h, PREC[prec], int(kind), int(nvec), C.byref(t), C.byref(g), C.byref(st),
                               C.byref(sk)))
    return t.value, g.value, st.value, sk.value


def cdag_memsim(h, order: Sequence[int], elem_bytes: int = 16):
    o = np.ascontiguousarray(order, dtype=np.int64)
    M = np.empty(max(1, o.size), dtype=np.int64)
    pp, pl = C.c_int64(), C.c_int64()
    _check(lib().cdag_memsim(h, _i64p(o), o.size, elem_bytes, _i64p(M), C.byref(pp), C.byref(pl)))
    return M[:o.size], pp.value, pl.value


def cdag_plan(h, prec: str = "fp64", batched: bool = False) -> dict:
    st = cdag_plan_stats()
    _check(lib().cdag_plan(h, PREC[prec], int(batched), C.byref(st)))
    return _struct_dict(st)


def cdag_plan_ops(h) -> List[tuple]:
    n = C.c_int64()
    _check(lib().cdag_plan_ops(h, None, None, None, 0, C.byref(n)))
    op = np.empty(n.value, dtype=np.int32)
    node = np.empty(n.value, dtype=np.int64)
    step = np.empty(n.value, dtype=np.int64)
    _check(lib().cdag_plan_ops(h, op.ctypes.data_as(C.POINTER(C.c_int32)), _i64p(node), _i64p(step),
                               n.value, None))
    return [(OP_NAMES[int(a)], int(b), int(c)) for a, b, c in zip(op, node, step)]


def cdag_get_nodes(h):
    n = C.c_int64()
    _check(lib().cdag_get_nodes(h, None, None, None, 0, C.byref(n)))
    kind = np.empty(n.value, dtype=np.int32)
    left = np.empty(n.value, dtype=np.int64)
    right = np.empty(n.value, dtype=np.int64)
    _check(lib().cdag_get_nodes(h, kind.ctypes.data_as(C.POINTER(C.c_int32)), _i64p(left), _i64p(right),
                                n.value, None))
    return kind, left, right


def cdag_graph_roots(h, n_graphs: int) -> np.ndarray:
    out = np.empty(max(1, n_graphs), dtype=np.int64)
    _check(lib().cdag_graph_roots(h, _i64p(out), n_graphs))
    return out[:n_graphs]


def cdag_bind_device(h, device: int, compute_stream: int, copy_stream: int) -> None:
    _check(lib().cdag_bind_device(h, device, C.c_void_p(compute_stream), C.c_void_p(copy_stream)))


def cdag_bind_arena(h, ptr: int, nbytes: int) -> None:
    _check(lib().cdag_bind_arena(h, C.c_void_p(ptr), nbytes))


def execute(h, prec: str = "fp64", batched: bool = False) -> dict:
    st = cdag_exec_stats()
    _check(lib().execute(h, PREC[prec], int(batched), C.byref(st)))
    return _struct_dict(st)


def cdag_execute_static(h, prec: str = "fp64", batched: bool = False) -> dict:
    st = cdag_exec_stats()
    _check(lib().cdag_execute_static(h, PREC[prec], int(batched), C.byref(st)))
    return _struct_dict(st)


STATIC_SCRATCH_BYTES = 64 << 20


def cdag_autotune(h, prec: str = "fp64", batched: bool = True, reps: int = 3,
                  in_situ: bool = False, uniform: bool = False) -> int:
    """Mode 0 synthetic per shape, 1 in situ per shape, 2 synthetic with one
    choice for every shape (one grouped launch per wave)."""
    n = C.c_int64()
    mode = 1 if in_situ else (2 if uniform else 0)
    _check(lib().cdag_autotune(h, PREC[prec], int(batched), int(reps), mode, C.byref(n)))
    return n.value


def fetch_correlators(h, nts: Sequence[int]) -> List[np.ndarray]:
    """Per input graph, complex128 [nt(g)]; nts: Nt of each graph in input order."""
    total = 2 * int(sum(nts))
    buf = np.empty(max(1, total), dtype=np.float64)
    _check(lib().fetch_correlators(h, buf.ctypes.data_as(C.POINTER(C.c_double)), total))
    out, o = [], 0
    for nt in nts:
        v = buf[o:o + 2 * nt]
        out.append(v[0::2] + 1j * v[1::2])
        o += 2 * nt
    return out


def cdag_fetch_sums(h, nts: Sequence[int]) -> List[np.ndarray]:
    total = 2 * int(sum(nts))
    buf = np.empty(max(1, total), dtype=np.float64)
    _check(lib().cdag_fetch_sums(h, buf.ctypes.data_as(C.POINTER(C.c_double)), total))
    out, o = [], 0
    for nt in nts:
        v = buf[o:o + 2 * nt]
        out.append(v[0::2] + 1j * v[1::2])
        o += 2 * nt
    return out


# ------------------------------------------------------------------ object wrapper
class Context:
    """One engine context; methods keep the C ABI's names."""

    def __init__(self):
        self.h = cdag_create()
        self.graph_nt: List[int] = []
        self.corr_nt: List[int] = []
        self.n_graphs = 0

    def close(self):
        if self.h is not None:
            cdag_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_cdag(self, leaves, graphs, specs=()):
        """specs: the contraction specs that op kinds SPEC_BASE + i name."""
        cdag_set_specs(self.h, specs)
        build_cdag(self.h, leaves, graphs)
        nt_of = []
        for spec in graphs:
            first = next(x for _, l, r in spec.ops for x in (l, r) if x >= 0)
            nt_of.append(leaves[first].nt)
        self.graph_nt = nt_of
        n_corr = 1 + max((int(getattr(s, "corr", 0)) for s in graphs), default=-1)
        self.corr_nt = [0] * n_corr
        for spec, nt in zip(graphs, nt_of):
            self.corr_nt[int(getattr(spec, "corr", 0))] = nt
        self.n_graphs = len(graphs)

    def build_general(self, n_leaves, sizes, children):
        cdag_build_general(self.h, n_leaves, sizes, children)
        self.graph_nt, self.corr_nt, self.n_graphs = [], [], 0

    def schedule(self, policy, check=False):
        return schedule(self.h, policy, check)

    def set_order(self, order):
        cdag_set_order(self.h, order)

    def set_mem_budget(self, nbytes):
        set_mem_budget(self.h, nbytes)

    def set_options(self, leaves_resident=False, wave_max=4096, wave_lookahead=0, use_graphs=1):
        cdag_set_options(self.h, leaves_resident, wave_max, wave_lookahead, use_graphs)

    def set_time_chunks(self, t_chunks=1):
        cdag_set_time_chunks(self.h, t_chunks)

    def set_trace_fusion(self, on=True):
        cdag_set_trace_fusion(self.h, on)

    def set_timing(self, on=True):
        cdag_set_timing(self.h, on)

    def launch_records(self):
        return cdag_launch_records(self.h)

    def dag_stats(self):
        return cdag_dag_stats(self.h)

    def set_tile(self, prec, kind, nvec, tile, grid=1, lds_stages=2, split_k=1):
        cdag_set_tile(self.h, prec, kind, nvec, tile, grid, lds_stages, split_k)

    def get_tile(self, prec, kind, nvec):
        return cdag_get_tile(self.h, prec, kind, nvec)

    def memsim(self, order, elem_bytes=16):
        return cdag_memsim(self.h, order, elem_bytes)

    def plan(self, prec="fp64", batched=False) -> Dict:
        return cdag_plan(self.h, prec, batched)

    def plan_ops(self):
        return cdag_plan_ops(self.h)

    def nodes(self):
        return cdag_get_nodes(self.h)

    def graph_roots(self):
        return cdag_graph_roots(self.h, self.n_graphs)

    def bind_device(self, device, compute_stream, copy_stream):
        cdag_bind_device(self.h, device, compute_stream, copy_stream)

    def bind_arena(self, ptr, nbytes):
        cdag_bind_arena(self.h, ptr, nbytes)

    def execute(self, prec="fp64", batched=False):
        return execute(self.h, prec, batched)

    def execute_static(self, prec="fp64", batched=False):
        return cdag_execute_static(self.h, prec, batched)

    def trace_execute(self, prec="fp64", batched=False, fail_at=-1):
        return cdag_trace_execute(self.h, prec, batched, fail_at)

    def autotune(self, prec="fp64", batched=True, reps=3, in_situ=False, uniform=False):
        return cdag_autotune(self.h, prec, batched, reps, in_situ, uniform)

    def fetch_correlators(self):
        return fetch_correlators(self.h, self.graph_nt)

    def fetch_sums(self):
        return cdag_fetch_sums(self.h, self.corr_nt)
