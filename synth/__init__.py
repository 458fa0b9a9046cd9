"""Seeded synthetic workloads for contraction-DAG runs.

This package only draws random numbers and lays out graph structure
(which leaves meet in which binary contraction).  It performs none of the
method's arithmetic: no contraction, no scheduling, no memory accounting.
Both the CPU oracle and the GPU path take their inputs from here.
"""
from .workloads import (  # noqa: F401
    K22, K32, K33, HCA, KIND_NAMES,
    Leaf, GraphSpec, Workload,
    meson_ring, baryon_mix, tiny_meson_perm, fig1_dag, batched_mix,
    config, CONFIG_NAMES,
)
