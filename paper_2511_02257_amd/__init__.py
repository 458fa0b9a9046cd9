"""Contraction-DAG engine for one MI355X: C++ host scheduler/planner and HIP
kernels in libcdagx.so, bound through ctypes."""
from .binding import (  # noqa: F401
    CdagError, Context, PREC, POLICY, UNLIMITED, EXPORTED,
    build_cdag, schedule, set_mem_budget, execute, fetch_correlators,
    cdag_create, cdag_destroy, cdag_plan, cdag_plan_ops, cdag_memsim, cdag_set_options, cdag_set_timing, cdag_launch_records, cdag_dag_stats, cdag_set_tile, cdag_get_tile, TILES,
    cdag_get_nodes, cdag_graph_roots, cdag_bind_device, cdag_bind_arena, cdag_fetch_sums, cdag_autotune,
    lib, LIB_PATH,
)
