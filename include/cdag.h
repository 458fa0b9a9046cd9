/*
 * cdag.h -- C ABI of the contraction-DAG engine (one MI355X GPU).
 *
 * The engine evaluates many-body correlation functions given as binary
 * contraction trees over hadron-node tensors (problem statement: Sec. II-B
 * "Notation" and Sec. II-C "Problem definition").  The trees are merged into
 * one contraction DAG, ordered by a scheduler (Sec. III: Sibling, Algs. 1-3;
 * Tree, Algs. 4-8; a node-based gain scheduler; or plain input order),
 * planned under a device-memory
 * budget with next-use eviction and host re-upload, and executed with
 * hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *   - Returns CDAG_OK (0) or a negative cdag_status; never throws.  A failed
 *     call leaves the context usable; cdag_last_error() describes the failure
 *     (thread-local string, valid until the next call on that thread).
 *   - Pointers are host pointers unless named dev_*.  Output arrays are owned
 *     by the caller; the caller passes their capacity.
 *   - Call order: cdag_create -> build_cdag -> schedule -> [set_mem_budget]
 *     -> [cdag_plan] -> cdag_bind_device + cdag_bind_arena -> execute ->
 *     fetch_correlators / cdag_fetch_sums.  Out-of-order calls return
 *     CDAG_E_STATE.  schedule, set_mem_budget, cdag_plan and execute may be
 *     repeated; build_cdag resets everything after it.
 *   - No entry point is thread-safe for one context; distinct contexts are
 *     independent.
 */
#ifndef CDAG_H
#define CDAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cdag_ctx cdag_ctx;

enum cdag_status {
  CDAG_OK = 0,
  CDAG_E_INVALID = -1, /* malformed argument or graph                          */
  CDAG_E_STATE = -2,   /* call out of order (e.g. execute before schedule)     */
  CDAG_E_BUDGET = -3,  /* one step's operands + outputs exceed the budget      */
  CDAG_E_HIP = -4,     /* a HIP runtime call failed                            */
  CDAG_E_NOMEM = -5,   /* host allocation failed, or the bound arena is small  */
  CDAG_E_RANGE = -6    /* an output capacity is too small                      */
};

/* Contraction kinds, per time slice t (row-major, contracted axes trailing on
 * the left operand and leading on the right):
 *   K22: O[i,j]   = sum_k  X[i,k]   Y[k,j]       meson x meson,   O(N^3)
 *   K32: O[i,j,l] = sum_k  X[i,j,k] Y[k,l]       baryon x meson,  O(N^4)
 *   K33: O[i,m]   = sum_jl X[i,j,l] Y[j,l,m]     baryon x baryon, O(N^4)
 *   HCA: C        = sum_ij P[i,j]   Q[j,i]       root "contract all" (trace)
 *   C1, C2, C3: the last c = 1, 2, 3 axes of X against the first c axes of
 *        Y, for operand and output ranks 2..4, e.g. C1 on two rank-3 tensors
 *        O[i,j,l,m] = sum_k X[i,j,k] Y[k,l,m] (rank 4, O(N^5)).  A C1 on ranks
 *        (2,2) or (3,2) and a C2 on (3,3) is stored as K22, K32 or K33.
 * (the hadron exterior contraction and contract-all operations of Sec. IV-B;
 * the general kinds give the rank-4 intermediates of larger systems). */
enum cdag_kind { CDAG_K22 = 0, CDAG_K32 = 1, CDAG_K33 = 2, CDAG_HCA = 3,
                 CDAG_C1 = 4, CDAG_C2 = 5, CDAG_C3 = 6 };
/* Op kind CDAG_SPEC_BASE + i: a contraction over any index pairs, described by
 * spec i of cdag_set_specs. */
#define CDAG_SPEC_BASE 16

/* A contraction over any index pairs (Sec. II-B's nodes contract hadron
 * tensors over whichever indices the quark lines join), per time slice: the
 * operands have ranks rank_l and rank_r (2..4); axis pair_l[k] of the left
 * operand is summed against axis pair_r[k] of the right one, k < n_pairs
 * (1..3, each axis at most once); the output lists the left operand's free
 * axes in order, then the right one's, and output axis j is axis perm[j] of
 * that list (perm: a permutation of 0..rank_l + rank_r - 2 n_pairs - 1, an
 * output rank of 2..4).  Axes count from 0 after the time axis.  A spec that
 * sums the last n_pairs axes of the left operand against the first ones of
 * the right one, in order, with perm the identity, is CDAG_C<n_pairs> and is
 * stored as that kind. */
typedef struct {
  int32_t rank_l, rank_r, n_pairs;
  int32_t pair_l[3], pair_r[3], perm[4];
} cdag_spec;

/* Schedulers: input order (each graph's tree in post-order, left first),
 * Sibling (Sec. III-A, Algs. 1-3), Tree (Sec. III-B, Algs. 4-8), and Node:
 * the node-based gain scheduler the conclusions propose as future work.  Node
 * runs next the ready contraction (non-leaf children already run) whose
 * execution lowers the Sec. II-C memory the most, i.e. the largest gain
 * M - M' of Sec. III-B for a single node: released children - leaves brought
 * in - its output (0 for a contraction without parents); ties to the lowest
 * node id. */
enum cdag_policy { CDAG_SCHED_INPUT = 0, CDAG_SCHED_SIBLING = 1, CDAG_SCHED_TREE = 2,
                   CDAG_SCHED_NODE = 3 };
/* OR into policy for Tree: at every selection recompute every live tree's
 * gain M - M' from scratch and fail with CDAG_E_STATE if an incrementally
 * maintained tgain differs (slow; a self-check).  For Node: at every pick
 * recompute the gain of every ready contraction and fail with CDAG_E_STATE if
 * a cached gain differs or the pick is not the largest. */
#define CDAG_SCHED_CHECK 0x100

/* Arithmetic of the exterior contractions.  FP64: complex128 storage and
 * arithmetic.  FP32, BF16X3 and BF16X6: complex64 storage, products on the
 * matrix cores with FP32 accumulation.  BF16X3 splits each FP32 operand into
 * a bf16 hi + lo pair and keeps three of the four piece products (about
 * 2^-16 relative error per product); BF16X6 splits it into three bf16 pieces
 * and keeps the six piece products whose order is at most 2^-16 (about the
 * FP32 rounding of the operands).  Traces and the cross-diagram sums are FP64
 * in every mode. */
enum cdag_prec { CDAG_FP64 = 0, CDAG_FP32 = 1, CDAG_BF16X3 = 2, CDAG_BF16X6 = 3 };

/* Plan op records (cdag_plan_ops). */
enum cdag_plan_op { CDAG_OP_D2H = 0, CDAG_OP_DROP = 1, CDAG_OP_H2D = 2,
                    CDAG_OP_ALLOC = 3, CDAG_OP_EXEC = 4, CDAG_OP_FREE = 5 };

/* A leaf tensor (hadron node): complex, shape [nt][nvec]^rank, rank 2 (meson),
 * 3 (baryon) or 4.  host: interleaved (re, im) in row-major order, complex128
 * (dtype CDAG_C128, doubles) or complex64 (dtype CDAG_C64, floats), read only
 * during build_cdag (the library keeps its own copy in that dtype); may be
 * NULL for a structure-only context (scheduling and planning work; execute
 * then fails with CDAG_E_STATE).  Complex64 leaves are promoted exactly in
 * FP64 mode. */
enum cdag_dtype { CDAG_C128 = 0, CDAG_C64 = 1 };
typedef struct {
  int32_t rank, nvec, nt, dtype;
  const void* host;
} cdag_leaf;

/* One binary contraction inside a graph.  Operand >= 0: a leaf id; operand
 * < 0: -(1 + index of an earlier op of the same graph). */
typedef struct {
  int32_t kind, left, right;
} cdag_op;

/* One graph (contraction tree, Sec. II-B): its last op is the root and must be
 * CDAG_HCA; every other op is used exactly once by a later op.  Its correlator
 * contributes w * C_g(t) to the cross-diagram sum of correlator corr_id. */
typedef struct {
  int32_t n_ops, corr_id;
  const cdag_op* ops;
  double w_re, w_im;
} cdag_graph;

typedef struct {
  int64_t n_nodes, n_leaves, n_contr, n_roots, n_steps;
  int64_t peak_post;     /* max_i M_i of Sec. II-C for the current schedule      */
  int64_t peak_live;     /* max resident bytes while one contraction runs        */
  int64_t peak_resident; /* max resident bytes of the budgeted plan              */
  int64_t n_evict, n_h2d, h2d_bytes, n_d2h, d2h_bytes;
  int64_t budget;        /* bytes the plan was made for (INT64_MAX: unlimited)   */
  int64_t arena_bytes;   /* device bytes cdag_bind_arena must provide            */
  int64_t tensor_highwater; /* physical high-water of the tensor pool           */
  int64_t host_spill_bytes; /* host bytes for spilled intermediates (pinned)     */
  int64_t hec_items;     /* exterior-contraction work items (output tiles x K splits) */
  double flops;          /* algorithmic flops, 8 per complex multiply-add        */
  double t_sched_s, t_plan_s;
} cdag_plan_stats;

typedef struct {
  cdag_plan_stats plan;
  double t_total_s;   /* execute(): first enqueue to results on the host      */
  double t_device_s;  /* compute stream, first kernel to last (HIP events)    */
  double t_hec_s;     /* summed exterior-contraction kernel time (timing on)  */
  double hec_flops;   /* algorithmic flops of the exterior contractions       */
  double hec_bytes;   /* algorithmic bytes: per launch, each distinct operand read once,
                         each output written once                                   */
  int64_t n_launches;
  int64_t n_hec_launches;
  int64_t n_graph_segments;
  double t_kernels_s;     /* summed duration of every kernel launch (timing on; else 0) */
  double t_copy_s;        /* summed duration of the host transfers on the upload and
                             spill streams (timing on; else 0)                      */
  int64_t arena_highwater; /* arena bytes the plan uses: leaf region, tensor pool
                              high-water, split-K workspace, descriptors, results   */
} cdag_exec_stats;

/* One kernel launch, or one host transfer, of a timed execute
 * (cdag_set_timing(c, 1)).  Transfers are the uploads and spills of a
 * budgeted plan (Sec. II-A's movement between host and device memory). */
enum cdag_launch_type { CDAG_LAUNCH_HEC = 0, CDAG_LAUNCH_REDUCE = 1, CDAG_LAUNCH_HCA = 2,
                        CDAG_LAUNCH_XSUM = 3, CDAG_LAUNCH_H2D = 4, CDAG_LAUNCH_D2H = 5 };
typedef struct {
  int32_t type;       /* cdag_launch_type                                                */
  int32_t variant;    /* HEC: kernel variant index; else 0                              */
  int32_t kinds;      /* bit k set when a contraction of cdag_kind k is in the launch (bit 7:
                         a contraction over any index pairs);
                         H2D, D2H: the moved tensor's cdag_kind bit (leaves: 0)         */
  int32_t interior;   /* HEC: 1 when every contraction of the launch is a whole number of
                         tiles and k-steps with aligned rows, so the kernel ran its
                         form without bounds tests; else 0                              */
  int64_t step;       /* plan step (wave); -1 for the cross-diagram sum                */
  int64_t n_items;    /* workgroup work items; H2D, D2H: 1                               */
  double flops;       /* algorithmic flops (8 per complex multiply-add); transfers: 0   */
  double bytes;       /* HEC, HCA: algorithmic bytes (each distinct operand of the launch
                         read once, each output written once); REDUCE: split-K
                         workspace read + output write; XSUM: 0;
                         H2D, D2H: the tensor's bytes                                   */
  double ms;          /* duration between HIP events around the launch or the copy, on
                         the stream that runs it (transfers: the upload or the spill
                         stream, after any wait for another stream)                     */
  int64_t trace_items;  /* HEC carrying its step's root traces (cdag_set_trace_fusion):
                           the (root, t) traces it ran besides n_items; else 0          */
  double trace_flops;   /* their algorithmic flops and bytes (not in flops and bytes);  */
  double trace_bytes;   /* else 0                                                       */
} cdag_launch_record;

/* One record of a traced execute (cdag_trace_execute). */
enum cdag_trace_op { CDAG_TR_RECORD = 0, CDAG_TR_WAIT = 1, CDAG_TR_READ = 2, CDAG_TR_WRITE = 3 };
enum cdag_trace_space { CDAG_SPACE_ARENA = 0, CDAG_SPACE_SPILL = 1, CDAG_SPACE_STAGE = 2 };
typedef struct {
  int32_t op;       /* cdag_trace_op                                                     */
  int32_t stream;   /* 0: the compute stream, 1: the upload stream, 2: the spill stream  */
  int64_t seq;      /* READ, WRITE: number of the operation (one host transfer, or all
                       kernels of one step) they belong to; -1 for events               */
  int64_t step;     /* plan step that issues the record                                  */
  int64_t node;     /* READ, WRITE: the tensor; -1 for events                            */
  int64_t event;    /* RECORD, WAIT: 3 * step + stream of the event's step and stream
                       (step counted over all passes); pass-end events:
                       3 * (passes * steps per pass + pass) + stream              */
  int32_t space;    /* READ, WRITE: cdag_trace_space of the range                        */
  int32_t reserved;
  int64_t off;      /* READ, WRITE: byte offset in the space (STAGE: within the leaf's
                       own staging buffer, 0 unless time-slice passes are in use)       */
  int64_t bytes;    /* READ, WRITE: bytes                                                */
} cdag_trace_rec;

/* Context lifetime: cdag_create stores a new, empty context in *out (owned by
 * the caller until cdag_destroy, which also releases the library's pinned
 * staging, spill pool, events and captured graphs; destroying NULL is a no-op).
 * CDAG_E_INVALID for a NULL out. */
int cdag_create(cdag_ctx** out);
int cdag_destroy(cdag_ctx* c);
/* Text of the last failure on the calling thread (empty after a success);
 * owned by the library, valid until the thread's next call. */
const char* cdag_last_error(void);

/* build_cdag -- Sec. II-B ("Notation"): the correlation function's graphs,
 * each a binary contraction tree over hadron-node tensors, are merged into one
 * contraction DAG whose vertices are tensors and whose edges join a
 * contraction's output to its operands; structurally identical sub-trees
 * become one vertex, so common intermediates are computed once.
 * Merge graphs into the DAG (hash-consing identical (kind, left, right)
 * contractions; identical graphs share their root).  Node ids: leaves
 * 0..n_leaves-1, then contractions in order of first appearance.
 * leaves[0..n_leaves) and graphs[0..n_graphs) are caller-owned and read during
 * the call only (each leaf's host data is copied).
 * CDAG_E_INVALID: bad shape, rank (operands and outputs 2..4; HCA on two
 * rank-2 operands), N or Nt mismatch, a GEMM dimension (N^(free or
 * contracted axes)) above 2^31, operand out of range or forward, identical
 * operands, root not HCA or HCA not last, unused op. */
int build_cdag(cdag_ctx* c, const cdag_leaf* leaves, int64_t n_leaves,
               const cdag_graph* graphs, int64_t n_graphs);

/* The contraction specs that op kinds CDAG_SPEC_BASE + i name in the graphs
 * of the next build_cdag (copied; at most 1024).  Such contractions run in
 * FP64 and FP32 on a general kernel with index-mapped loads and stores (no
 * split-K); planning in a split-BF16 mode fails with CDAG_E_INVALID.
 * build_cdag validates each use against its operands (CDAG_E_INVALID: ranks
 * that differ from the spec's, axes out of range or repeated, a perm that is
 * not a permutation, an output rank outside 2..4).  CDAG_E_INVALID for n
 * outside 0..1024 or a NULL specs with n > 0. */
int cdag_set_specs(cdag_ctx* c, const cdag_spec* specs, int64_t n);

/* Host-only: a general DAG for scheduling and the memory model, whose nodes
 * may have any number of children (Sec. II-B notes that the schedulers extend
 * to that case; Sec. III-B that the Tree scheduler needs neither two children
 * per node nor trees that are trees).  Nodes 0..n_leaves-1 are leaves; node
 * u >= n_leaves has the children child[child_off[u] .. child_off[u+1]-1]
 * (operand order; ids below u; no repeats; at least one); size_bytes[u] is
 * the size of u's tensor in bytes.  Trees are rooted at the non-leaf nodes
 * without parents, in ascending id.  All three arrays are read during the
 * call only (child_off has n_nodes + 1 entries, child_off[0] = 0).  Replaces
 * the DAG like build_cdag.  Afterwards schedule (input order, Tree and
 * Node; Sibling only when every non-leaf has two children), cdag_memsim
 * (elem_bytes is then ignored: the given sizes apply), cdag_get_nodes (kind 7
 * for non-leaves, left/right for two-child nodes, else -1) and cdag_dag_stats
 * apply;
 * cdag_plan, execute and cdag_autotune return CDAG_E_STATE.
 * CDAG_E_INVALID: counts out of range (n_nodes < 2^31), a NULL array, a
 * decreasing child_off, a leaf with children, a non-leaf without, a child id
 * outside [0, u), a repeated child, a negative size. */
int cdag_build_general(cdag_ctx* c, int64_t n_nodes, int64_t n_leaves, const int64_t* size_bytes,
                       const int64_t* child_off, const int64_t* child);

/* schedule -- Sec. III ("Scheduling heuristics"): a total order of the
 * contractions that respects the DAG (children before parents) and keeps the
 * Sec. II-C peak memory low.  policy: CDAG_SCHED_INPUT (each graph in turn,
 * post-order), CDAG_SCHED_SIBLING (Sec. III-A, Algs. 1-3 with the rank of
 * Eq. (1)), CDAG_SCHED_TREE (Sec. III-B, Algs. 4-8: the tree with the largest
 * gain M - M' next), CDAG_SCHED_NODE (the node-based gain scheduler named in
 * Sec. VI); OR CDAG_SCHED_CHECK for the self-check.  order_out (nullable,
 * caller-owned, capacity cap) receives node ids; *n_out (nullable) the number
 * of contractions.  CDAG_E_RANGE if cap is too small for a non-NULL
 * order_out; CDAG_E_INVALID for an unknown policy or Sibling on a node
 * without two children; CDAG_E_STATE before a DAG is built.  The order stays
 * in force for cdag_plan and execute. */
int schedule(cdag_ctx* c, int policy, int64_t* order_out, int64_t cap, int64_t* n_out);

/* Install a contraction order found earlier (a saved schedule) instead of
 * scheduling: order lists every contraction once, children before parents.
 * The paper notes that a schedule, once found, serves any N; the order
 * depends only on the DAG's structure, so an order saved from a DAG built
 * with other N or Nt applies when the node ids match.  The order is copied.
 * CDAG_E_INVALID: n differs from the number of contractions, an id out of
 * range, a leaf, a repeat, or a contraction before one of its children.
 * CDAG_E_STATE: no DAG built. */
int cdag_set_order(cdag_ctx* c, const int64_t* order, int64_t n);

/* set_mem_budget -- Sec. II-C ("Problem definition"): the device memory the
 * execution may hold at once.  Memory is charged as in Sec. II-C (a leaf from
 * its first use, an intermediate from its production until its last parent
 * has run; a root's scalar output costs nothing); when the schedule's live
 * bytes exceed the budget, the plan evicts (next use furthest away; an
 * intermediate is copied to host memory once) and uploads again, the data
 * movement Sec. IV-C counts.  bytes: the budget (UINT64_MAX: unlimited, the
 * default).  CDAG_E_STATE before a DAG is built.  A budget that one step cannot
 * fit in is reported by cdag_plan / execute with CDAG_E_BUDGET. */
int set_mem_budget(cdag_ctx* c, uint64_t bytes);

/* leaves_resident: 1 keeps every leaf in a device region of its own, outside
 * the budget, uploaded once per precision (never evicted); 0 (default) makes
 * leaves start on the host as in Sec. II-C.  wave_max: most contractions per
 * wave in batched mode (default 4096).  wave_lookahead: in batched mode a wave
 * takes the ready contractions (operands are leaves or earlier waves' outputs)
 * in schedule order and may pass over this many not-ready ones (default 0:
 * the schedule order is kept exactly; INT64_MAX: every ready contraction).
 * use_graphs: 0 issues every step eagerly on three streams (kernels, uploads,
 * spills) with event waits from the plan; 1 (default) replays captured HIP
 * graphs with every step on one stream (one graph, or segments of 64 steps
 * when the plan moves data); 2 replays one captured graph over the three
 * streams with the plan's waits as graph edges (uploads and spills overlap
 * kernels).  CDAG_E_INVALID for wave_max < 1, a negative lookahead or another
 * use_graphs. */
int cdag_set_options(cdag_ctx* c, int leaves_resident, int wave_max, int64_t wave_lookahead,
                     int use_graphs);

/* Time-slice passes.  Every exterior contraction and trace acts on each time
 * slice t on its own (Sec. II-B: hadron-node tensors batched over t), so the
 * DAG may run as t_chunks passes, pass k over slices [k nt / t_chunks,
 * (k + 1) nt / t_chunks) of every tensor.  Passes alternate between two halves
 * of the budget (each pass is planned with tensors of size / t_chunks bytes
 * under budget / 2), so the uploads of one pass overlap the kernels of the
 * pass before.  Plan statistics are those of the whole execution (counters
 * summed over passes, peak_resident over both halves); cdag_plan_ops lists
 * the ops of one pass.  Results are bit-identical to t_chunks = 1 (split-K
 * counts follow the whole nt).  t_chunks = 1 (default) keeps tensors whole,
 * the memory model of Sec. II-C.  CDAG_E_INVALID for t_chunks < 1; planning
 * fails with CDAG_E_INVALID when t_chunks does not divide every tensor's nt. */
int cdag_set_time_chunks(cdag_ctx* c, int64_t t_chunks);

/* Trace fusion (engine design, Sec. IV-B's execution queue): with on != 0 the
 * root traces of a plan step (Sec. IV-B, "contract all") ride in one of the
 * step's exterior-contraction launches, in workgroups after its contractions'
 * work items, instead of a launch of their own, so that a step whose
 * contractions and traces are both ready is one kernel.  The carrier is the
 * step's last contraction launch of one workgroup per item (not the general
 * kernel); a step without one keeps a trace launch.  Correlators are
 * bit-identical either way (the traces' summation order does not depend on
 * how they are launched).  Launch records then show the traces inside the
 * carrier (CDAG_KIND bit CDAG_HCA_TRACE in kinds; trace_items, trace_flops,
 * trace_bytes).  Default 1. */
int cdag_set_trace_fusion(cdag_ctx* c, int on);

/* timing: 1 records a HIP event pair around every kernel launch on the
 * compute stream and around every host transfer on its stream, reports
 * the summed exterior-contraction durations in t_hec_s and keeps per-launch
 * and per-transfer records (execution then runs without graph replay);
 * 0 (default) turns it off. */
int cdag_set_timing(cdag_ctx* c, int timing);
/* Host-only: the eager three-stream issue order that execute would follow for
 * (prec, batched), recorded without any HIP call: per step, the spill
 * stream's waits and spills (the ranges each reads and writes) and its event
 * record, the upload stream's waits, uploads and event record, the compute
 * stream's waits, the ranges the step's kernels read and write, and the
 * compute event record; per time-slice pass, the pass-end records and the
 * waits of the pass two later on them.  It lets a
 * CPU check that every pair of conflicting accesses is ordered by a stream or
 * an event (the plan's data movement, Sec. II-A and Sec. IV-C).  *n_out
 * (nullable) receives the count; at most cap records are written.
 * fail_at >= 0 makes the walk fail with CDAG_E_HIP at that record, as a failed
 * HIP call would (an error-path check).  Needs schedule; no device. */
int cdag_trace_execute(cdag_ctx* c, int prec, int batched, cdag_trace_rec* out, int64_t cap, int64_t* n_out,
                       int64_t fail_at);

/* Records of the last execute made with timing on, in issue order: one per
 * kernel launch and one per host transfer (a transfer comes before the
 * kernels of its step).  *n_out (nullable) receives the count; at most cap
 * records are written. */
int cdag_launch_records(cdag_ctx* c, cdag_launch_record* out, int64_t cap, int64_t* n_out);

/* Kernel variant of the exterior contractions of `kind` (K22, K32, K33, C1,
 * C2 or C3; a general kind shares one entry over all its operand ranks)
 * with N = nvec in precision `prec`.  tile: 0 = 64x64, 1 = 32x32, 2 = 48x48,
 * 3 = 128x64, 4 = 64x32, 5 = 64x64 with 512 threads (output rows x columns
 * per workgroup), -1 removes an explicit choice.  In FP64 and FP32, tiles 1,
 * 4 and 5 form each complex product from three real ones (Gauss), the others
 * from four.  grid: 0 = persistent (compute units x occupancy
 * workgroups striding over the work list), 1 = one workgroup per work item.
 * lds_stages: 2 = double-buffered operand tiles in LDS, 1 = a single buffer
 * refilled from registers (half the LDS, more workgroups per compute unit).
 * split_k: 1 = a contraction with fewer than 512 output tiles and K >= 512 is
 * cut into K splits summed by a fixed-order reduction; 0 = never split (one
 * work item per output tile, the whole K in one accumulator).
 * Without an explicit choice a default by N applies (split_k 1;
 * cdag_get_tile reports the choice in force).  Every choice gives results
 * within the precision's bound; bits may differ between choices, never with
 * the grouping of contractions into launches. */
int cdag_set_tile(cdag_ctx* c, int prec, int kind, int nvec, int tile, int grid, int lds_stages,
                  int split_k);
int cdag_get_tile(cdag_ctx* c, int prec, int kind, int nvec, int* tile, int* grid, int* lds_stages,
                  int* split_k);

/* Host-only: simulate Sec. II-C for `order` (n node ids, each contraction
 * once, topological) with element size elem_bytes (16 or 8; a general DAG
 * uses its given sizes).  M_out (nullable, capacity n) receives M_1..M_n. */
int cdag_memsim(cdag_ctx* c, const int64_t* order, int64_t n, int elem_bytes,
                int64_t* M_out, int64_t* peak_post, int64_t* peak_live);

/* Host-only: build the budgeted plan for (prec, batched) on the current
 * schedule and budget.  CDAG_E_BUDGET if one step cannot fit. */
int cdag_plan(cdag_ctx* c, int prec, int batched, cdag_plan_stats* out);

/* The last plan's op list: op[i] in cdag_plan_op, node[i], step[i]. */
int cdag_plan_ops(cdag_ctx* c, int32_t* op, int64_t* node, int64_t* step, int64_t cap,
                  int64_t* n_out);

/* Introspection of the merged DAG: per node kind (-1 leaf), left, right
 * (-1 for leaves); per input graph its root node id. */
int cdag_get_nodes(cdag_ctx* c, int32_t* kind, int64_t* left, int64_t* right, int64_t cap,
                   int64_t* n_out);
int cdag_graph_roots(cdag_ctx* c, int64_t* root_of_graph, int64_t cap);

/* Size of the merged DAG and the Sec. III-B runtime factors: F_v = average
 * over vertices of the number of trees containing the vertex; F_e = average
 * over edges (child, parent) of the number of trees containing both ends
 * (every tree that holds the parent holds its children).  Trees are counted
 * per unique root.  Any output pointer may be NULL. */
int cdag_dag_stats(cdag_ctx* c, int64_t* n_vertices, int64_t* n_edges, int64_t* n_trees, double* f_v,
                   double* f_e);

/* Device binding.  device: HIP ordinal.  compute_stream, copy_stream:
 * hipStream_t handles borrowed for the context's lifetime (copies run on the
 * second; both must be non-NULL and distinct).  The arena is device memory of
 * at least plan.arena_bytes bytes, 256-byte aligned, borrowed until rebound
 * or the context is destroyed. */
int cdag_bind_device(cdag_ctx* c, int device, void* compute_stream, void* copy_stream);
int cdag_bind_arena(cdag_ctx* c, void* dev_arena, uint64_t bytes);

/* execute -- Sec. II-C and Sec. IV-B/IV-C: evaluate every graph of the DAG
 * in the scheduled order under the memory budget, as the paper's runtime does
 * with its queue of exterior contractions, contract-all operations on roots,
 * deletions, and evictions with host re-uploads (Sec. II-A, GPU memory
 * management).
 * Plan (as cdag_plan) and run the whole DAG: uploads, evictions, exterior
 * contractions, traces, the cross-diagram sums and the copy of the results
 * to the host.  Blocks until the results are on the host.  prec: cdag_prec;
 * batched: 0 one contraction per step, 1 waves of ready contractions
 * (cdag_set_options).  out (nullable, caller-owned) receives the statistics.
 * CDAG_E_STATE without schedule, bound device and arena, or leaf data;
 * CDAG_E_NOMEM if the arena is smaller than plan.arena_bytes; CDAG_E_BUDGET as
 * cdag_plan; CDAG_E_HIP if a HIP call fails (the context stays usable).  Spilled
 * intermediates go to a pinned host pool of plan.host_spill_bytes; when a
 * pinned allocation of that size fails the pool is pageable memory and the
 * steps run eagerly (no captured segments).  CDAG_E_NOMEM if neither can be
 * allocated. */
int execute(cdag_ctx* c, int prec, int batched, cdag_exec_stats* out);

/* Size of the static device array behind cdag_execute_static. */
#define CDAG_STATIC_SCRATCH_BYTES (64LL << 20)

/* For callers that cannot allocate device or pinned host memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * execute with every device byte in a static array of
 * CDAG_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on until
 * the process ends, instead of the bound arena.  Results and statistics are
 * those of execute (bit-identical correlators for the same plan);
 * fetch_correlators and cdag_fetch_sums read them afterwards.  Everything runs
 * on the compute stream in plan order (no events, no graphs); leaves are
 * copied from the library's own host copy and converted to the device layout
 * on the device.  Needs a plan made beforehand with cdag_plan for the same
 * (prec, batched) (CDAG_E_STATE otherwise: planning allocates host memory),
 * one pass over the time slices and no spill to host memory (CDAG_E_BUDGET);
 * CDAG_E_NOMEM when the plan's arena plus a staging range for the largest leaf
 * exceed CDAG_STATIC_SCRATCH_BYTES.  The array is shared by every context on
 * that GPU and keeps the last call's contents: calls that overlap on one GPU
 * race (serialise them; none may overlap an execute of another context that
 * uses it). */
int cdag_execute_static(cdag_ctx* c, int prec, int batched, cdag_exec_stats* out);

/* Autotuner over the kernel variants of cdag_set_tile, for every distinct
 * (kind, N) among the exterior contractions of the DAG.  mode 0 (synthetic):
 * time each variant and split_k setting `reps` times on a batch of time
 * slices of that shape (at least 4096 work items, as in a wave of such
 * contractions, at most 64 contractions' worth; split counts as for one
 * contraction) placed in the bound arena's tensor pool (as planned for
 * (prec, batched); its contents are scratch between executes) and keep the
 * fastest per time slice.  mode 1 (in situ): execute the planned DAG `reps` times per
 * variant and split_k setting, shape by shape, with launch timing on, and keep
 * the least time of exterior contractions and split-K reductions in the
 * fastest of the reps
 * (needs leaf data; costs up to 40 * reps executes per shape).  mode 2
 * (synthetic, uniform): the timings of mode 0, then one choice for every
 * shape, the one whose summed time over the DAG (time per slice times the
 * slices of each shape) is least, so that each wave's exterior contractions
 * run in one grouped launch.  *n_tuned
 * (nullable) receives the number of shapes tuned.  Needs cdag_bind_device and
 * an arena of at least the plan's arena_bytes; invalidates the current plan
 * and results. */
int cdag_autotune(cdag_ctx* c, int prec, int batched, int reps, int mode, int64_t* n_tuned);

/* fetch_correlators -- Sec. I and Sec. II-B: the value of each graph, the
 * full contraction of its tree per time slice (the terms whose sum is the
 * correlation function).
 * Per input graph g, C_g(t) for t < nt(g), as (re, im) doubles, graphs in
 * input order, concatenated: 2 * sum_g nt(g) doubles into the caller-owned
 * out of capacity cap_doubles.  Graphs merged into one root get equal rows.
 * CDAG_E_STATE before a successful execute; CDAG_E_RANGE if cap_doubles is
 * too small. */
int fetch_correlators(cdag_ctx* c, double* out, int64_t cap_doubles);

/* Per correlator c = 0..max(corr_id), S_c(t) = sum_{g: corr_id = c} w_g C_g(t)
 * summed in FP64 in a fixed order (identical from run to run); 2 * sum_c nt(c)
 * doubles (nt of a correlator with no graph is 0). */
int cdag_fetch_sums(cdag_ctx* c, double* out, int64_t cap_doubles);

#ifdef __cplusplus
}
#endif

#endif /* CDAG_H */
