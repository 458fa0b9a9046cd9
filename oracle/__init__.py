"""CPU oracle for contraction-DAG execution: TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct Python/numpy implementations of what the GPU
path computes, written from the paper's definitions:

  dag.py        CDAG formation from contraction trees (Sec. II-B), and general
                DAGs whose nodes have any number of children.
  schedules.py  input-order, Sibling (Algs. 1-3) and Tree (Sec. III-B, from the
                gain definition M - M' rather than the incremental Algs. 5-8),
                the node-based gain scheduler the conclusions propose (the same
                gain per ready node), the memory model of Sec. II-C, and a
                brute-force optimum.
  planner.py    the budgeted next-use eviction plan and wave cut.
  values.py     correlator values in complex128 and the cross-diagram sum.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library and never imports it.

Parity status: every function here is pinned by CPU tests (see tests/
test_oracle_*.py) against values printed in the paper (Table sch-mem),
closed forms, invariants or brute force, except where a docstring says
"parity unpinned".
"""
