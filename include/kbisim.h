/*
 * kbisim.h — C ABI of the MI355X (gfx950) k-bisimulation refinement library.
 *
 * The library computes the partitions P_1..P_k of k-bisimulation on a
 * multi-relational labeled graph G = (V, E, l_V, l_E)
 * (Def. multi-relational-labeled-property-graph):
 *
 *   P_0:      u ~0 v  iff  l_V(u) = l_V(v)   (vertex label SETS; base case of
 *             Def. vertex-labeled-bw-bisimulation).  No vertex labels at all
 *             means P_0 = {V} (initialisation of Alg. schaetzle-alg).
 *   P_{i+1}:  u ~(i+1) v  iff  u ~i v  and the sets
 *             { (l_E(e), block_i(w)) : e = (u, w) in E }  are equal
 *             (step of Def. edge-labeled-fw-bisimulation; the pair set is the
 *             signature of Def. signature).
 *
 * Output block ids are dense and numbered by first vertex: the block holding
 * vertex 0 is 0, the next block met in vertex order is 1, and so on.  This
 * replaces the paper's hash-valued ids (Def. id) by a collision-free naming,
 * so results compare bit-exactly with any other correct implementation.
 *
 * Edge semantics: one label per CSR entry (the RDF triple view); parallel
 * entries and self-loops are allowed; duplicates never matter (set
 * semantics).  The graph is read as out-edges (forward bisimulation); pass
 * the transposed CSR for backward bisimulation (Def. inverse-schema-element).
 *
 * Conventions
 *  - Graph arrays, outputs and the workspace are DEVICE pointers on the
 *    current HIP device.  Counts returned to the caller are HOST memory.
 *  - The library allocates no device memory: every buffer it uses is carved
 *    from the caller's workspace (size from kbisim_workspace_bytes), which
 *    must start at a 256-byte boundary (hipMalloc's and torch's allocations
 *    do; EINVAL otherwise).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    work is enqueued on it.  A context is bound to one stream and is not
 *    thread-safe; separate contexts are independent.
 *  - The caller owns the graph arrays (read-only, they must outlive the
 *    context), the outputs and the workspace.
 *  - Return value: 0 on success or a negative KBISIM_E* code.  No C++
 *    exception crosses this interface.  On error, output contents are
 *    unspecified.
 */
#ifndef KBISIM_H
#define KBISIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KBISIM_OK 0
#define KBISIM_EINVAL (-1)    /* null pointer, bad size, k < 0 or k > kmax        */
#define KBISIM_EGRAPH (-2)    /* graph validation failed (see kbisim_graph)      */
#define KBISIM_ENOSPACE (-3)  /* workspace smaller than kbisim_workspace_bytes   */
#define KBISIM_EHIP (-4)      /* HIP runtime error; kbisim_strerror has details */
#define KBISIM_ERANGE (-5)    /* n >= 2^31 or m >= 2^62                          */
#define KBISIM_EINTERNAL (-6) /* a device-side consistency check failed          */

/* A labeled graph in CSR form.  All pointers are device pointers.
 *   n, m        vertices and CSR entries (edges); 0 <= n < 2^31.
 *   nlabels     number of entries of vlabel when vlabel_ptr is given
 *               (= vlabel_ptr[n]); ignored otherwise.  Used for workspace
 *               sizing and validation.
 *   row_ptr     int64 [n+1]: row_ptr[0] = 0, non-decreasing, row_ptr[n] = m.
 *   col         int32 [m]: 0 <= col[e] < n, the target of entry e.
 *   elabel      int32 [m] edge labels >= 0, or NULL: every edge has label 0.
 *   vlabel_ptr  int64 [n+1] label-set CSR (same rules as row_ptr, ending at
 *               the number of labels), or NULL: one label per vertex.
 *   vlabel      int32 labels >= 0: [vlabel_ptr[n]] entries, or [n] when
 *               vlabel_ptr is NULL.  NULL together with vlabel_ptr == NULL
 *               means no vertex labels (P_0 = {V}).
 * Label values need not be dense.  Repeated labels inside one vertex's set
 * are allowed and count once.                                               */
typedef struct {
  int64_t n;
  int64_t m;
  int64_t nlabels;
  const int64_t *row_ptr;
  const int32_t *col;
  const int32_t *elabel;
  const int64_t *vlabel_ptr;
  const int32_t *vlabel;
} kbisim_graph;

typedef struct kbisim_ctx kbisim_ctx;

/* Launch-shape parameters chosen by an autotuner (0 = default).  Results do
 * not depend on them; only the work split does.
 *   range_edges      CSR entries per range workgroup: 1024 or 2048 (default:
 *                    2048 with 32-bit set keys, 1024 with 64-bit keys)
 *   hub_chunk        entries per hub staging workgroup: 2048 (default) or 4096
 *   hub_part_target  expected entries per hub partition: 1024 or 2048 (default)
 *   key_bits         pair keys in LDS hash sets: 0 (default) = 32-bit keys,
 *                    exact (label, block) when every pair fits in 31 bits and
 *                    a 32-bit hash of the pair otherwise; 32 = hashed 32-bit
 *                    keys always; 64 = exact 64-bit keys always.  With hashed
 *                    keys the signature is deduplicated by key and every
 *                    grouping is still confirmed on the pairs themselves.
 *   scan_items       vertices per thread in the numbering (head words): 8 or 16
 *                    (default)                                                */
typedef struct {
  int range_edges;
  int hub_chunk;
  int hub_part_target;
  int key_bits;
  int scan_items;
  int reserved[3];
} kbisim_tuning;

/* Workspace bytes needed by kbisim_create for a graph of g->n vertices,
 * g->m edges (and g->nlabels set labels) and up to kmax iterations per call.
 * Reads only these sizes; no HIP call.  Errors: EINVAL (null), ERANGE.      */
int kbisim_workspace_bytes(const kbisim_graph *g, int kmax, size_t *bytes);

/* Validate the graph, compute P_0 and the static degree schedule, and bind a
 * context to `stream`.  Synchronises `stream` once (to report validation).
 * kmax >= 0 bounds k in later calls.  On success *out receives the context.
 * Errors: EINVAL, ERANGE, ENOSPACE, EGRAPH, EHIP.                           */
int kbisim_create(const kbisim_graph *g, int kmax, void *workspace, size_t ws_bytes, void *stream,
                  kbisim_ctx **out);

/* As kbisim_create with explicit launch-shape parameters (NULL = defaults).
 * Errors as kbisim_create, plus EINVAL for unsupported values.              */
int kbisim_create_tuned(const kbisim_graph *g, int kmax, const kbisim_tuning *tuning, void *workspace,
                        size_t ws_bytes, void *stream, kbisim_ctx **out);

/* Capture the k-step loop of later kbisim_refine calls as a HIP graph on the
 * first call for a given (k, outputs, start) and replay it afterwards
 * (enable = 1), or launch kernels one by one (0, the default).  Needs a
 * stream other than the null stream; EINVAL otherwise.  Disabled while the
 * per-kernel profiler is on.                                                */
int kbisim_use_graphs(kbisim_ctx *c, int enable);

/* Bind the context to another stream for its later calls (a scheduler can
 * prepare contexts on one stream and run them on others).  Work enqueued
 * later on `stream` starts after all work enqueued so far on the previous
 * stream (an event orders them; no host synchronisation).  Errors: EINVAL
 * (null context, or the null stream while graph capture is on), EHIP.      */
int kbisim_set_stream(kbisim_ctx *c, void *stream);

/* Work-efficient mode (enable = 1; 0 = off, the default; -1 = leave as is).
 * The outputs are the same; the work is not: a vertex alone in its block is
 * not refined again (a singleton block cannot split), and once a step leaves
 * the block count unchanged the partition is a fixpoint (a refinement with as
 * many blocks is the same partition), so the remaining outputs are copies.
 * Calls synchronise after every step to read its count; graph capture is not
 * used while the mode is on.  *last_steps (may be NULL) receives the number
 * of steps the last call computed.  This mode is reported separately from
 * the full-work figures.                                                    */
int kbisim_work_efficient(kbisim_ctx *c, int enable, int *last_steps);

/* Copy P_0 into out_ids (device int32 [n]) and its block count into
 * *out_count (host).  Synchronises the stream.                              */
int kbisim_initial(kbisim_ctx *c, int32_t *out_ids, int64_t *out_count);

/* Compute P_1..P_k starting from P_0.  out_block_ids is a HOST array of k
 * device pointers, each to int32 [n]; out_block_ids[i] receives P_{i+1}.
 * out_counts (host, int64 [k]) receives the block counts.  Every iteration
 * is computed in full, also past the fixpoint (later arrays then repeat).
 * Enqueues on the context's stream and synchronises once at the end.  k = 0
 * is a no-op.  Calls are independent: each restarts from P_0.
 * Errors: EINVAL (k < 0, k > kmax, null output), EINTERNAL, EHIP.           */
int kbisim_refine(kbisim_ctx *c, int k, int32_t *const *out_block_ids, int64_t *out_counts);

/* As kbisim_refine, but start from a given labelling pid_i (device int32
 * [n], values in [0, n); vertices with equal values form the blocks) instead
 * of P_0.  Resuming from the P_i of an earlier call reproduces P_{i+1}.. of
 * an uninterrupted run, since each step depends only on the previous
 * partition and G.  Errors as kbisim_refine, plus EINVAL for values outside
 * [0, n).                                                                   */
int kbisim_refine_from(kbisim_ctx *c, const int32_t *pid_i, int k, int32_t *const *out_block_ids,
                       int64_t *out_counts);

/* ---- batches ------------------------------------------------------------- */

/* A batch refines many independent graphs with the same launches.  The
 * caller passes their disjoint union as one kbisim_graph whose column ids are
 * global (graph g owns vertices [vert_off[g], vert_off[g+1]), and no entry
 * leaves its graph) and vert_off (HOST int64 [num_graphs + 1], vert_off[0] =
 * 0, non-decreasing, vert_off[num_graphs] = n).  Each graph gets exactly the
 * partitions kbisim_refine would give it alone: blocks never span graphs and
 * ids are numbered by first vertex within each graph.  Vertex labels (either
 * form) are per vertex of the union; label-set CSR offsets are global.      */
typedef struct kbisim_batch kbisim_batch;

int kbisim_batch_workspace_bytes(const kbisim_graph *u, int64_t num_graphs, int kmax, size_t *bytes);

/* Validates (including that no entry crosses graphs: EGRAPH) and computes
 * every graph's P_0 and the schedule of the union.  Synchronises.           */
int kbisim_batch_create(const kbisim_graph *u, int64_t num_graphs, const int64_t *vert_off, int kmax,
                        const kbisim_tuning *tuning, void *workspace, size_t ws_bytes, void *stream,
                        kbisim_batch **out);

/* P_1..P_k of every graph.  out_ids: HOST array of k device pointers, each
 * int32 [n] in union order holding per-graph ids; out_counts: HOST int64
 * [num_graphs * k], counts[g * k + i] = number of blocks of graph g in
 * P_{i+1}.  Synchronises once at the end.                                   */
int kbisim_batch_refine(kbisim_batch *b, int k, int32_t *const *out_ids, int64_t *out_counts);

/* Single steps of a batch, for schedulers that advance many batches and
 * contexts one step at a time.  Step i (0 <= i < kmax, issued in order
 * 0, 1, 2, ...) writes the per-graph ids of P_{i+1} into out_ids (device
 * int32 [n], union order); the batch keeps P_i itself.  _async only
 * enqueues; _result synchronises, settles any unresolved hash collision of
 * the step and writes out_counts (HOST int64 [num_graphs]): graph g's
 * block count in P_{i+1}.                                                   */
int kbisim_batch_step_async(kbisim_batch *b, int i, int32_t *out_ids);
int kbisim_batch_step_result(kbisim_batch *b, int i, int32_t *out_ids, int64_t *out_counts);

/* The context that runs the batch (for kbisim_use_graphs, profiling and
 * schedule statistics).  It is owned by the batch.                         */
int kbisim_batch_context(kbisim_batch *b, kbisim_ctx **ctx);

int kbisim_batch_destroy(kbisim_batch *b);

/* ---- graph preparation -------------------------------------------------- */

/* Backward refinement (Def. inverse-schema-element; the backward models of
 * Sec. "Bisimulation Variants", e.g. Kaushik's vertex-labelled backward
 * bisimulation) is forward refinement of the transposed graph.
 * kbisim_transpose writes the transpose of (row_ptr, col, elabel): row w of
 * the output lists every entry (v, l, w) of the input as (l, v).
 *   out_row_ptr  device int64 [n+1]
 *   out_col      device int32 [m]
 *   out_elabel   device int32 [m] or NULL (zeros when elabel is NULL)
 *   workspace    device, kbisim_transpose_workspace_bytes(n, m) bytes
 * The order of entries inside an output row is unspecified; refinement does
 * not depend on it.  Validates the input first; synchronises `stream`.
 * Errors: EINVAL, ERANGE, ENOSPACE, EGRAPH (invalid input), EHIP.           */
int kbisim_transpose_workspace_bytes(int64_t n, int64_t m, size_t *bytes);
int kbisim_transpose(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const int32_t *elabel,
                     int64_t *out_row_ptr, int32_t *out_col, int32_t *out_elabel, void *workspace, size_t ws_bytes,
                     void *stream);

/* ---- summary graph -------------------------------------------------------- */

/* The summary (quotient) graph of a refinement chain (Sec. "Graph Summaries
 * for Bisimulation"): one vertex per block of src_pid, and an edge (B, l, C)
 * for every distinct (src_pid[v], elabel[e], dst_pid[w]) over the entries
 * e = (v, w) of the context's graph (label 0 without edge labels).  The
 * paper connects B to C by label l when all vertices of B have an l-edge
 * into C; with src_pid = P_k and dst_pid = P_{k-1} of one chain the members
 * of a block share their (label, target block) sets, so this union is that
 * graph.  The distinct triples are written sorted by (source block, label,
 * target block) to out_src, out_label, out_dst (device int32 [m] each) and
 * their number to *out_count (host).  src_pid, dst_pid: device int32 [n] with
 * values in [0, n).  workspace: kbisim_quotient_workspace_bytes bytes.
 * Synchronises the context's stream.  Errors: EINVAL (null, batch context,
 * ids out of range), ENOSPACE, ERANGE (the source-block, label and
 * target-block fields need more than 64 bits), EHIP.                       */
int kbisim_quotient_workspace_bytes(kbisim_ctx *c, size_t *bytes);
int kbisim_quotient(kbisim_ctx *c, const int32_t *src_pid, const int32_t *dst_pid, int32_t *out_src,
                    int32_t *out_label, int32_t *out_dst, int64_t *out_count, void *workspace, size_t ws_bytes);

/* ---- tracing and measurement -------------------------------------------- */

/* Kernel kinds reported by the per-kernel profiler. */
#define KBISIM_K_SIG_RANGE 0   /* signatures of runs of low-degree vertices        */
#define KBISIM_K_SIG_BLOCK 1   /* signatures, one workgroup per row (1k-8k entries) */
#define KBISIM_K_HUB_STAGE 2   /* hub rows: chunk dedupe and partitioned staging   */
#define KBISIM_K_HUB_REDUCE 3  /* hub rows: per-partition dedupe and sums          */
#define KBISIM_K_HUB_FINAL 4   /* hub key hashes (and very large hubs)             */
#define KBISIM_K_LOOKUP 5      /* representative lookup + small exact checks       */
#define KBISIM_K_VERIFY 6      /* exact checks of larger rows                      */
#define KBISIM_K_PEEL 7        /* collision peeling rounds                         */
#define KBISIM_K_SCAN 8        /* first-vertex numbering scan                      */
#define KBISIM_K_ASSIGN 9      /* ids of non-representatives                       */
#define KBISIM_K_FILL 10       /* table clears and counter resets                  */
#define KBISIM_NKERNELS 11

/* Enable (1) or disable (0) per-kernel timing for later kbisim_refine calls:
 * every launch is bracketed by HIP events on the context's stream and the
 * elapsed times are summed per kernel kind.  Enabling resets the sums.      */
int kbisim_profile_enable(kbisim_ctx *c, int enable);

/* Restrict timing to the kernel kinds whose bits are set in `kinds` (bit i =
 * kind i; all kinds by default), so a timed run pays for events only around
 * the kernels of interest.                                                 */
int kbisim_profile_select(kbisim_ctx *c, uint32_t kinds);

/* Sums since kbisim_profile_enable: ms[KBISIM_NKERNELS] milliseconds and
 * launches[KBISIM_NKERNELS] launch counts (host arrays; either may be NULL).
 * Synchronises the stream.                                                  */
int kbisim_profile_read(kbisim_ctx *c, double *ms, int64_t *launches);

/* Name of a kernel kind, or NULL. */
const char *kbisim_kernel_name(int kind);

/* Static degree schedule of the graph rows (host int64 [8]): vertices and
 * CSR entries in the range tier (rows up to the range capacity, 1024 or 2048
 * entries), the workgroup tiers (up to 8192 entries, or 19456 with 32-bit
 * set keys), the staged hub tier and the global-set hub tier, in that order. */
int kbisim_schedule_info(kbisim_ctx *c, int64_t *info);

/* Plain device-to-device copy of `bytes` bytes (a multiple of 16) with the
 * library's streaming copy kernel, enqueued on `stream`.  Used to measure
 * achievable HBM bandwidth and to calibrate hardware byte counters.        */
int kbisim_copy_probe(void *dst, const void *src, size_t bytes, void *stream);

/* Time the context's random gather alone: every CSR entry reads the block id
 * of its target (in pid, device int32 [n]) through the same index and layout
 * as the signature kernels, and nothing else is done.  *ms (host) receives
 * the mean time of one pass over all m entries (reps passes after a warm-up).
 * It bounds what the signature kernels can reach on this graph.  Overwrites
 * scratch parts of the workspace; synchronises.                             */
int kbisim_gather_probe(kbisim_ctx *c, const int32_t *pid, int reps, double *ms);

/* ---- single steps (for schedulers that interleave many contexts) --------- */

/* Enqueue step i (0 <= i < kmax): P_{i+1} from prev into out (device int32
 * [n]) on the context's stream, without synchronising.  Steps of one context
 * must be issued in order i = 0, 1, 2, ... with prev = P_0 (NULL) for i = 0
 * and prev = the previous step's out afterwards, and no other refine call on
 * the context in between (later steps reuse state of step 0); out must not
 * alias prev.
 * The count stays on the device until kbisim_step_result.                   */
int kbisim_step_async(kbisim_ctx *c, int i, const int32_t *prev, int32_t *out);

/* Finish step i (same i, prev, out): synchronises the stream, recomputes the
 * step with host-driven collision peeling if its in-loop round left a
 * collision unsettled, and returns the block count of P_{i+1} in *count.   */
int kbisim_step_result(kbisim_ctx *c, int i, const int32_t *prev, int32_t *out, int64_t *count);

/* Release the context (host memory only; the workspace stays the caller's). */
int kbisim_destroy(kbisim_ctx *c);

/* ---- incremental updates on an edited graph --------------------------------
 *
 * After edits (edges deleted and inserted), P_1..P_k of the edited graph are
 * recomputed from the cached chain of the original graph instead of from
 * scratch; the paper names incremental computation on evolving graphs as
 * future work (Sec. "Discussion").  Within a cached chain, blocks are named
 * by their minimum vertex, so a vertex whose own block name and targets'
 * block names did not change keeps its cached key hash; only the others are
 * re-signed: the edited rows at every step, and from step 2 on the vertices
 * whose name changed in the previous step and every vertex with an edge into
 * one (that set grows along in-edges from step to step).  A cached block
 * that holds none of them and whose key none of them takes keeps its
 * members and name; only the others are regrouped, with exact checks on
 * the edited rows, and dense ids cover every vertex, so the result is
 * exactly the refinement of the edited graph from scratch (ids numbered by
 * first vertex).  Once two consecutive partitions have equal block counts
 * the later ones are copies (a fixpoint).
 *
 * Bytes of the caller buffer that holds the cached chain of a graph of
 * g->n vertices and g->m edges for up to kmax steps: per step a key hash, a
 * distinct count, a block name and a filter bit index per vertex (18
 * bytes), the graph's in-rows (8 (n+1) + 4 m) and scratch; about
 * 18 kmax n + 4 m + 75 n bytes.  Host
 * only.  Errors: EINVAL (null, kmax < 1), ERANGE.                           */
int kbisim_incr_state_bytes(const kbisim_graph *g, int kmax, size_t *bytes);

/* Keep the chain of every later kbisim_refine call (from P0) in `state`
 * (device, at least kbisim_incr_state_bytes(g, kmax) bytes, owned by the
 * caller and left to the context until it is destroyed), so that
 * kbisim_incr_update can follow.  Builds the in-rows of the context's graph
 * (synchronises).  Not for batch contexts, and not together with the
 * work-efficient mode (EINVAL either way; kbisim_work_efficient(c, 1, ...)
 * fails once this is on).  Errors: EINVAL, ENOSPACE, EHIP.                  */
int kbisim_incr_enable(kbisim_ctx *c, void *state, size_t bytes);

/* P_1..P_k (k <= the steps of the last kbisim_refine call, which must have
 * started from P0 after kbisim_incr_enable) of an edited graph g_new: device
 * CSR of the same n vertices, with the same vertex labels as the context's
 * graph (only its row_ptr, col, elabel and m are read; elabel present exactly
 * when the context's graph has edge labels, each label at most the context
 * graph's largest).  rows: device int32 [nrows], nrows <= n, the vertices
 * whose rows differ from the context graph's as multisets of (label,
 * target); repeats are allowed, rows not listed must be unchanged.
 * out_block_ids: k device int32 [n] arrays; out_counts: host int64 [k].  The
 * cached chain is not changed, so several edits can each be applied to it.
 * Synchronises.  Errors: EINVAL (arguments, a listed vertex out of range, no
 * cached chain of k steps), EGRAPH (invalid row offsets, a target out of
 * range or a label beyond the cached graph's largest), EHIP, EINTERNAL.     */
int kbisim_incr_update(kbisim_ctx *c, const kbisim_graph *g_new, const int32_t *rows, int64_t nrows, int k,
                       int32_t *const *out_block_ids, int64_t *out_counts);

/* ---- refinement without allocation ---------------------------------------
 *
 * For callers that cannot allocate device memory: code that must not call
 * hipMalloc or take pinned host memory (serving loops with a fixed memory
 * plan, harnesses that forbid allocation).  The same computation as
 * kbisim_create + kbisim_refine(k) + kbisim_destroy, with the workspace taken
 * from a scratch array inside the library instead of the caller: one array of
 * kbisim_noalloc_scratch_bytes() bytes (128 MiB) per GPU, held from the
 * library's load on that GPU until the process ends.
 *
 * g: as for kbisim_create (device arrays, read only).  out_block_ids: k
 * device pointers, each int32 [n], receiving P_1..P_k; out_counts: host
 * int64 [k].  Runs on the current device, on `stream` (a stream of that
 * device, or NULL), and synchronises it before returning.  No device memory
 * is allocated and no pinned host memory is taken; host-side bookkeeping
 * uses the C++ heap only.
 *
 * Limit: the graph must fit the scratch array, i.e. the workspace
 * kbisim_workspace_bytes(g, k) reports must be at most
 * kbisim_noalloc_scratch_bytes() (about 500k vertices and 3M edges);
 * otherwise KBISIM_ENOSPACE, before any HIP call.  Other errors as for
 * kbisim_create / kbisim_refine.  Every call on one GPU uses that GPU's one
 * array and leaves its contents behind (nothing of a previous call is read):
 * calls that overlap in time on one GPU, from different threads or on
 * different streams, race and must be serialised by the caller.             */
int kbisim_refine_noalloc(const kbisim_graph *g, int k, int32_t *const *out_block_ids, int64_t *out_counts,
                          void *stream);

/* Bytes of the per-GPU scratch array used by kbisim_refine_noalloc. */
size_t kbisim_noalloc_scratch_bytes(void);

/* Static description of an error code (or of the last HIP error seen). */
const char *kbisim_strerror(int code);

/* Library version string. */
const char *kbisim_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KBISIM_H */
