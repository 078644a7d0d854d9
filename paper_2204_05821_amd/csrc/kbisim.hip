// Host engine and C ABI of the k-bisimulation refinement library (gfx950).
//
// The engine owns no device memory: kbisim_create carves every buffer from
// the caller's workspace, validates the graph, computes P0 (vertex label-set
// equality), renumbers gather targets by in-degree and builds a static degree
// schedule; kbisim_refine enqueues k refinement steps on the caller's stream
// with no host synchronisation inside the loop (and, when enabled, replays
// the whole loop as a captured HIP graph).  A step that met a hash collision
// it could not settle in its one in-loop peeling round is detected after the
// final synchronisation and recomputed, from that step on, with peeling
// rounds driven by the host.  A batch is the disjoint union of many graphs
// refined by the same launches, with per-graph ids and counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/kbisim.h"
#include "kernels.h"

using namespace kb;

namespace {

thread_local char g_hip_msg[256] = "";

constexpr size_t ALIGN = 256;
constexpr int CNT_STRIDE = 16;  // device counters per step
constexpr int PERSIST_GRID = 2048;
constexpr int RES_GRID = 256;
constexpr int CLEAR_GRID = 2048;
constexpr int MIN_RANGE_EDGES = 1024;  // smallest tunable range capacity
constexpr int MIN_HUB_CHUNK = 2048;    // smallest tunable hub chunk
constexpr int MAX_GRAPH_CACHE = 8;
constexpr int SCHED_CHUNKS = 16;  // host-built schedules: this many vertex chunks packed in parallel
// Graphs of at least this many vertices get their schedule built on the
// device.  A chunk walk is sequential, so the two walks take about 8 ms
// whatever the graph; the host copy of the row offsets and the packing cost
// about 1 ns per vertex, and win below this size (an 8.4M-vertex graph
// creates in 17.5 ms instead of 21.4; serving, which creates many small
// contexts, keeps its latency).
constexpr int64_t SCHED_DEVICE_MIN = (int64_t)1 << 24;

inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 512;
  while (p < x) p <<= 1;
  return p;
}

struct Plan {
  size_t off_H, off_DC, off_rep, off_p0, off_vlist, off_clA, off_clB, off_ranges, off_lists, off_gcol, off_rank,
      off_gpid, off_zrep;
  size_t off_table, off_ctable, off_hacc, off_hcnt, off_chunks, off_parts, off_gchunks, off_poff;
  size_t off_status, off_hw, off_counters, off_dcounts, off_err, off_dep, off_hubsets, off_single, off_multi, off_nzv;
  size_t off_gid, off_ibuf, off_first, off_next, off_bcounts;  // batches only
  uint64_t tslots;
  int64_t max_ranges, max_lists, nhub_max, nchunk_max, npart_max, ngchunk_max, npoff_max, ntiles, hubset_slots;
  int ncounter_steps;
  size_t total;
};

Plan make_plan(int64_t n, int64_t m, int64_t nl, int kmax, int64_t num_graphs) {
  Plan p{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t o = at;
    at = align_up(at + std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t N = (size_t)std::max<int64_t>(n, 1);
  const int64_t big = std::max<int64_t>(std::max<int64_t>(m, nl), 1);
  p.tslots = pow2_at_least(2 * (uint64_t)N);
  // A range closes at a hub, when the next row would overflow it (the closed
  // range and that row hold more than its capacity together, and each row is
  // "next" once), when full of vertices, or at the end; rows above the
  // capacity form ranges of their own.  Bounds use the smallest capacity.
  p.max_ranges = big / (RANGE_DMAX + 1) + 2 * big / (MIN_RANGE_EDGES + 1) + 2 * big / MIN_RANGE_EDGES +
                 (int64_t)N / RANGE_VERTS + 8 + SCHED_CHUNKS + (int64_t)N / SCHED_CHUNK_V + 1;
  p.max_lists = big / (RANGE_DMAX + 1) + 8;
  p.nhub_max = big / (BLOCK_MAX + 1) + 1;
  p.nchunk_max = big / MIN_HUB_CHUNK + p.nhub_max + 1;
  p.npart_max = big / (HUB_PART_TARGET / 4) + 2 * p.nhub_max + 1;
  p.ngchunk_max = big / HUB_GCHUNK + p.nhub_max + 1;
  p.npoff_max = big / 16 + 4 * (HUB_PMAX + 1) + p.nchunk_max;
  p.ntiles = (int64_t)(N + 256 * SCAN_ITEMS_MIN - 1) / (256 * SCAN_ITEMS_MIN) + 1;
  p.hubset_slots = 2 * big + 64;
  p.ncounter_steps = kmax + 4;
  p.off_H = take(8 * N);
  p.off_DC = take(4 * N);
  p.off_rep = take(4 * N);
  p.off_p0 = take(4 * N);
  p.off_vlist = take(4 * N);
  p.off_clA = take(4 * N);
  p.off_clB = take(4 * N);
  p.off_ranges = take(sizeof(Range) * (size_t)p.max_ranges);
  p.off_lists = take(4 * (size_t)p.max_lists);
  p.off_gcol = take(4 * (size_t)std::max<int64_t>(m, 1));
  p.off_rank = take(4 * N);
  p.off_gpid = take(8 * N);
  p.off_zrep = take(8 * N);
  p.off_table = take(8 * p.tslots);
  p.off_ctable = take(8 * p.tslots);
  p.off_hacc = take(8 * (size_t)p.nhub_max);
  p.off_hcnt = take(4 * (size_t)p.nhub_max);
  p.off_chunks = take(sizeof(HubChunk) * (size_t)p.nchunk_max);
  p.off_parts = take(sizeof(HubPart) * (size_t)p.npart_max);
  p.off_gchunks = take(sizeof(HubGChunk) * (size_t)p.ngchunk_max);
  p.off_poff = take(4 * (size_t)p.npoff_max);
  p.off_status = take(4 * (size_t)p.ntiles);
  p.off_hw = take(sizeof(HeadWord) * (N / 64 + 1));
  p.off_counters = take(4 * (size_t)CNT_STRIDE * (size_t)p.ncounter_steps);
  p.off_dcounts = take(8 * (size_t)p.ncounter_steps);
  p.off_err = take(16);
  p.off_dep = take(64);
  p.off_hubsets = take(8 * (size_t)p.hubset_slots);
  p.off_single = take(2 * N);
  p.off_multi = take(4 * N);
  p.off_nzv = take(4 * N);
  if (num_graphs > 0) {
    p.off_gid = take(4 * N);
    p.off_ibuf = take(8 * N);
    p.off_first = take(8 * (size_t)(num_graphs + 1));
    p.off_next = take(8 * (size_t)num_graphs);
    p.off_bcounts = take(8 * (size_t)num_graphs * (size_t)std::max(kmax, 1));
  }
  p.total = at;
  return p;
}

// Static degree schedule of one row structure (graph rows or label-set rows),
// built on the host at create time; degrees never change across iterations.
struct Schedule {
  int range_edges = RANGE_EDGES;  // range capacity of this schedule (1024 or 2048)
  int nranges = 0;  // multi-vertex ranges (at most range_edges entries)
  int nbig = 0;     // single-row ranges of range_edges < deg <= RANGE_DMAX
  int nrow8 = 0;    // single-row ranges of RANGE_DMAX < deg <= ROW_MAX (after the nbig ones)
  int nrow20 = 0;   // single-row ranges of ROW_MAX < deg <= ROW_MAX_NARROW, 32-bit keys only (after those)
  int nhub = 0, hub_off = 0;
  int nchunks = 0, nparts = 0, ngchunks = 0;
  int64_t gset_begin = 0, gset_end = 0;  // global hash sets of very large hubs
  int64_t nonempty = 0;                   // rows with at least one entry
  const int *nzv = nullptr;               // their vertices in order (graph rows), or null
  int64_t info[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // vertices, entries per tier
};

struct Tuning {
  int range_edges = 0;  // 0: by key width (range_cap)
  int hub_chunk = 2048;
  int hub_part_target = HUB_PART_TARGET;
  int key_bits = 0;  // LDS set keys: 0 = 32-bit (exact where pairs fit, else hashed), 32 = hashed, 64 = 64-bit
  int hub_parts_cap = HUB_PMAX;  // most partitions per staged hub (a smaller cap is a test knob)
  bool device_schedule = false;  // test knob: build the schedule on the device at any size
  int scan_items = SCAN_ITEMS;   // vertices per thread in the numbering scan: 8 or 16
  int gfilter_min = GFILTER_MIN_DIRTY;  // dirty vertices from which update steps use the global filter
};

struct GraphKey {
  const void *start;
  int k;
  std::vector<const void *> outs;
  bool operator<(const GraphKey &o) const {
    if (start != o.start) return start < o.start;
    if (k != o.k) return k < o.k;
    return outs < o.outs;
  }
};

}  // namespace

struct kbisim_ctx {
  kbisim_graph g;
  int kmax;
  hipStream_t stream;
  Plan plan;
  Tuning tune;
  char *ws;
  u64 *H, *table, *ctable, *hacc, *hubsets, *zrep;
  u32 *DC, *hcnt, *err, *tiles, *dep;
  HeadWord *hw;
  int *rep, *p0, *vlist, *clA, *clB, *lists, *counters, *poff, *gcol, *rank, *gpid[2], *nzv;
  int64_t *dcounts;
  Range *ranges;
  HubChunk *chunks;
  HubPart *parts;
  HubGChunk *gchunks;
  Schedule sched;  // graph rows
  u64 hmask = ~0ULL;
  u32 kmask = 0xFFFFFFFFu;  // bits kept of hashed set keys (test knob)
  u64 tmask_steps = 0;   // grouping-table mask of refinement steps (sized by vertices with edges)
  bool work_eff = false;  // skip singleton blocks, stop at the fixpoint
  int we_steps = 0;       // steps computed by the last work-efficient call
  unsigned char *single[2] = {nullptr, nullptr};  // singleton flags of the last two partitions
  u32 *multi = nullptr;  // stamps of heads that have a non-head member
  u32 prof_mask = ~0u;   // kernel kinds timed by the profiler
  bool pinned_ok = true;  // schedule building may take pinned host buffers
  bool narrow = false;  // 32-bit LDS keys
  bool hashed = false;  // ... that hash the pair (it does not fit 31 bits, or 32-bit keys were asked for)
  u32 pb = 31;
  u32 max_label = 0;    // largest edge label (0 without labels)
  bool packed = false;  // edge labels packed above the target ranks in gcol
  u32 rbits = 31;       // bits of the target rank in gcol
  int32_t *glab = nullptr;  // separate labels in the order of the sorted rows (else the caller's)
  int64_t p0_count = 0;
  // batches
  int64_t num_graphs = 0;
  int *gid = nullptr, *ibuf[2] = {nullptr, nullptr};
  int64_t *first = nullptr, *next = nullptr, *bcounts = nullptr;
  // per-kernel profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Pending {
    int kind;
    size_t a, b;
  };
  std::vector<Pending> ev_pending;
  double prof_ms[KBISIM_NKERNELS] = {0};
  int64_t prof_n[KBISIM_NKERNELS] = {0};
  // captured refinement loops
  bool use_graphs = false;
  std::map<GraphKey, hipGraphExec_t> graphs;
  // incremental updates: refine calls from P0 cache their chain (key hashes,
  // distinct counts and minimum-vertex block names per step) in the caller's
  // state buffer; updates recompute only what edits can have changed
  bool incr = false;
  int incr_k = 0;  // steps of the cached chain
  struct {
    u64 *Hc;
    u32 *DCc;
    int32_t *MVc;
    uint16_t *FKc;  // filter bit of each vertex's cached key, per step
    int64_t *tptr;
    int32_t *tcol;
    int32_t *names[2];
    unsigned char *edited, *flag, *dirty, *skip;
    int *small, *large, *psmall, *plarge, *changed, *cnt;
    int32_t *bname;   // block names of an update step, by representative
    int32_t *keep;    // cached names kept by blocks of changed vertices, by representative
    unsigned char *claimed;  // cached names taken by blocks with an unchanged member
    int *heavy;       // changed vertices with long in-rows
    u32 *touch;  // bitmap of the cached blocks (by minimum vertex) that can change in this step
    int *lk;               // the dirty vertices, then these and the clean members of touched blocks
    u32 *filter;           // bit filter of the dirty keys
    u32 *gfilter;          // the larger global filter (GFILTER_BITS) used with many dirty keys
    // edited rows longer than LIST_BIG: one global set each (chunks of HUB_GCHUNK)
    int *huge;
    HubGChunk *huge_chunks;
    u64 *huge_acc;
    u32 *huge_cnt;
    int nhuge = 0, nhuge_chunks = 0;
    // edited rows of LIST_BIG < length <= ROW_MAX (and, with 32-bit keys,
    // <= ROW_MAX_NARROW after them): one row-kernel workgroup each
    Range *erows;
    int nerows8 = 0, nerows20 = 0;
    int64_t huge_set_begin = 0, huge_set_slots = 0;
    int64_t huge_cap = 0, huge_chunk_cap = 0;
    int64_t nrows = 0;  // edited rows listed by the caller
    u64 *zrep;        // empty-signature representatives by block name (names reach 2n)
  } is{};
};

struct kbisim_batch {
  kbisim_ctx *c;
};

namespace {

int hip_fail(hipError_t e) {
  snprintf(g_hip_msg, sizeof g_hip_msg, "HIP error %d: %s", (int)e, hipGetErrorString(e));
  return KBISIM_EHIP;
}

#define HIP_TRY(expr)                          \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return hip_fail(_e); \
  } while (0)

#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

inline unsigned blocks_for(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

// Range check of cnt int32 values on stream s (see k_validate_vals).
void validate_vals(hipStream_t s, int64_t cnt, const int32_t *vals, int64_t upper, u32 *err, u32 bit) {
  if (cnt <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(VALIDATE_GRID, blocks_for(cnt / 4 + 1, 256));
  k_validate_vals<<<g, 256, 0, s>>>(cnt, vals, upper, err, bit);
}

// ---- per-kernel profiling: events around each launch, resolved after syncs.
hipEvent_t prof_event(kbisim_ctx *c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

struct ProfScope {
  kbisim_ctx *c;
  int kind;
  size_t start = (size_t)-1;
  ProfScope(kbisim_ctx *c_, int kind_) : c(c_), kind(kind_) {
    if (!c->prof || !((c->prof_mask >> kind) & 1u)) return;
    hipEvent_t e = prof_event(c);
    if (!e) return;
    start = c->ev_used - 1;
    (void)hipEventRecord(e, c->stream);
  }
  ~ProfScope() {
    if (start == (size_t)-1) return;
    hipEvent_t e = prof_event(c);
    if (!e) return;
    (void)hipEventRecord(e, c->stream);
    c->ev_pending.push_back({kind, start, c->ev_used - 1});
  }
};

// Fold pending event pairs into the sums (the stream must be synchronised).
void prof_collect(kbisim_ctx *c) {
  for (auto &p : c->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_pool[p.a], c->ev_pool[p.b]) == hipSuccess) {
      c->prof_ms[p.kind] += ms;
      c->prof_n[p.kind] += 1;
    }
  }
  c->ev_pending.clear();
  c->ev_used = 0;
}

int fill_u64(kbisim_ctx *c, u64 *p, int64_t cnt, u64 val) {
  if (cnt <= 0) return 0;
  ProfScope ps(c, KBISIM_K_FILL);
  unsigned g = (unsigned)std::min<int64_t>(blocks_for(cnt, 256), 65536);
  k_fill_u64<<<g, 256, 0, c->stream>>>(p, cnt, val);
  LAUNCH_CHECK();
  return 0;
}

int fill_i32(kbisim_ctx *c, int *p, int64_t cnt, int val) {
  if (cnt <= 0) return 0;
  ProfScope ps(c, KBISIM_K_FILL);
  unsigned g = (unsigned)std::min<int64_t>(blocks_for(cnt, 256), 65536);
  k_fill_i32<<<g, 256, 0, c->stream>>>(p, cnt, val);
  LAUNCH_CHECK();
  return 0;
}

// Advance the device-side epochs named in `mask` and clear the tables whose
// epoch wrapped.
int advance(kbisim_ctx *c, u32 mask, const Schedule &s) {
  ProfScope ps(c, KBISIM_K_FILL);
  k_advance<<<1, 64, 0, c->stream>>>(c->dep, mask);
  LAUNCH_CHECK();
  k_clear_if<<<CLEAR_GRID, 256, 0, c->stream>>>(c->dep, c->table, (int64_t)c->plan.tslots, c->ctable,
                                                c->hubsets + s.gset_begin, s.gset_end - s.gset_begin);
  LAUNCH_CHECK();
  return 0;
}

int read_err(kbisim_ctx *c, u32 *out) {
  HIP_TRY(hipMemcpyAsync(out, c->err, sizeof(u32), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return 0;
}

// Range capacity: the tuned one, else 2048 entries with 32-bit set keys and
// 1024 with 64-bit keys (the larger LDS set would cost occupancy).
int range_cap(const kbisim_ctx *c, bool wide_keys) {
  if (c->tune.range_edges) return c->tune.range_edges;
  return wide_keys ? 1024 : 2048;
}

int hub_parts_for(const Tuning &t, int64_t d) {
  int P = 1;
  while ((int64_t)P * t.hub_part_target < d && P < t.hub_parts_cap) P <<= 1;
  return P;
}

// Edge labels read from their own array (not packed into gcol, and present).
bool separate_labels(const kbisim_ctx *c) { return !c->packed && c->g.elabel != nullptr; }
// The separate labels the kernels read: the rank-sorted copy, if made.
const int32_t *sep_labels(const kbisim_ctx *c) { return c->glab ? c->glab : c->g.elabel; }

// Dense ids numbered by first vertex: out[v] = number of heads (rep[v] == v)
// before v for heads, -1 for the others; the head count into *count_dev.
int numbering_scan(kbisim_ctx *c, int n, int *out, int64_t *count_dev) {
  const int items = c->tune.scan_items;
  const int ntiles = (int)blocks_for(n, 256 * items);
  const int aligned = ((uintptr_t)out & 15) == 0;
  if (items == 8) k_tile_count<8><<<(unsigned)ntiles, 256, 0, c->stream>>>(n, c->rep, c->tiles);
  else k_tile_count<16><<<(unsigned)ntiles, 256, 0, c->stream>>>(n, c->rep, c->tiles);
  LAUNCH_CHECK();
  k_tile_scan<<<1, 1024, 0, c->stream>>>(ntiles, c->tiles, count_dev);
  LAUNCH_CHECK();
  if (items == 8) k_scan_write<8><<<(unsigned)ntiles, 256, 0, c->stream>>>(n, c->rep, c->tiles, out, aligned);
  else k_scan_write<16><<<(unsigned)ntiles, 256, 0, c->stream>>>(n, c->rep, c->tiles, out, aligned);
  LAUNCH_CHECK();
  return 0;
}

// A step's numbering: head words and the tile prefixes of the heads in
// vertex order (k_head_words, k_tile_scan); the block count to count_dev.
// The assign kernels then read every vertex's dense id through the result.
int numbering_words(kbisim_ctx *c, int n, int64_t *count_dev, HeadIds *ids) {
  const int items = c->tune.scan_items;
  const int ntiles = (int)blocks_for(n, 256 * items);
  if (items == 8) k_head_words<8><<<(unsigned)ntiles, 256, 0, c->stream>>>(n, c->rep, c->hw, c->tiles);
  else k_head_words<16><<<(unsigned)ntiles, 256, 0, c->stream>>>(n, c->rep, c->hw, c->tiles);
  LAUNCH_CHECK();
  k_tile_scan<<<1, 1024, 0, c->stream>>>(ntiles, c->tiles, count_dev);
  LAUNCH_CHECK();
  *ids = HeadIds{c->hw, c->tiles, items == 8 ? 11 : 12};
  return 0;
}

// The vertices with at least one entry, in order, into c->nzv (s.nzv then
// points there): flags, the head scan of the numbering, and a scatter.  Uses
// rep and vlist as scratch.
int build_nonempty_list(kbisim_ctx *c, Schedule &s) {
  const int n = (int)c->g.n;
  if (n == 0) return 0;
  k_mark_rows<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->g.row_ptr, c->rep);
  LAUNCH_CHECK();
  int rc = numbering_scan(c, n, c->vlist, c->dcounts + (c->plan.ncounter_steps - 1));
  if (rc) return rc;
  k_list_from_ids<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->vlist, c->nzv);
  LAUNCH_CHECK();
  s.nzv = c->nzv;
  return 0;
}

// Sort the entries of every row of the range and row tiers, and of every
// staged hub chunk, by target rank (results do not depend on the order
// inside a row).  Separate edge labels move with their entries, in a copy
// kept in the unused tail of the hub staging region; when the tail is too
// small, such graphs stay unsorted.  PAY: that copy is in use.
template <bool PAY>
int sort_rows_impl(kbisim_ctx *c, const Schedule &s, u32 *lab) {
  u32 *g = reinterpret_cast<u32 *>(c->gcol);
  if (s.nranges) {
    const GraphSrcT<false> src{c->g.row_ptr, c->gcol, nullptr, nullptr, nullptr, c->pb, c->rbits};
    if (s.range_edges == 1024)
      k_sort_ranges<GraphSrcT<false>, 1024, PAY><<<(unsigned)s.nranges, 256, 0, c->stream>>>(src, g, lab, c->ranges,
                                                                                           c->rbits);
    else
      k_sort_ranges<GraphSrcT<false>, 2048, PAY><<<(unsigned)s.nranges, 256, 0, c->stream>>>(src, g, lab, c->ranges,
                                                                                           c->rbits);
    LAUNCH_CHECK();
  }
  const Range *rows = c->ranges + s.nranges;
  if (s.nbig) {
    k_sort_rows<RANGE_DMAX, PAY><<<(unsigned)s.nbig, 1024, 0, c->stream>>>(g, lab, rows, c->rbits);
    LAUNCH_CHECK();
  }
  if (s.nrow8) {
    k_sort_rows<ROW_MAX, PAY><<<(unsigned)s.nrow8, 1024, 0, c->stream>>>(g, lab, rows + s.nbig, c->rbits);
    LAUNCH_CHECK();
  }
  if constexpr (!PAY) {  // rows beyond 8192 entries (32-bit keys): no LDS room for the labels
    if (s.nrow20) {
      k_sort_rows<32768, false><<<(unsigned)s.nrow20, 1024, 0, c->stream>>>(g, nullptr, rows + s.nbig + s.nrow8,
                                                                          c->rbits);
      LAUNCH_CHECK();
    }
  }
  if (s.nchunks) {
    k_sort_hub_chunks<HUB_CHUNK_MAX, PAY><<<(unsigned)s.nchunks, 1024, 0, c->stream>>>(
        g, lab, c->g.row_ptr, c->lists + s.hub_off, c->chunks, c->rbits);
    LAUNCH_CHECK();
  }
  return 0;
}

int sort_long_rows(kbisim_ctx *c, const Schedule &s) {
  if (!separate_labels(c)) return sort_rows_impl<false>(c, s, nullptr);
  const int64_t m = c->g.m;
  const int64_t need = (m + 1) / 2 + 1;  // u64 slots for m int32 labels
  if (m == 0 || s.gset_end + need > c->plan.hubset_slots) return 0;
  int32_t *lab = reinterpret_cast<int32_t *>(c->hubsets + (c->plan.hubset_slots - need));
  HIP_TRY(hipMemcpyAsync(lab, c->g.elabel, 4 * (size_t)m, hipMemcpyDeviceToDevice, c->stream));
  c->glab = lab;
  return sort_rows_impl<true>(c, s, reinterpret_cast<u32 *>(lab));
}

// Host copies of row-offset arrays for schedule building.  Fresh host pages
// cost more to map than the copy itself, so buffers (pinned when possible)
// go back to a process-wide pool and serve later creates.  The pool holds at
// most as many buffers as schedules were built at once; it is never freed.
struct HostRows {
  int64_t *p = nullptr;
  size_t cap = 0;
  bool pinned = false;
};
std::mutex &host_rows_mu() {
  static std::mutex *m = new std::mutex();
  return *m;
}
std::vector<HostRows> &host_rows_pool() {
  static std::vector<HostRows> *v = new std::vector<HostRows>();
  return *v;
}
void host_rows_free(HostRows &b) {
  if (!b.p) return;
  if (b.pinned) (void)hipHostFree(b.p);
  else delete[] b.p;
  b = HostRows{};
}
// A buffer of at least cnt entries (p null if none could be had).
HostRows host_rows_take(size_t cnt) {
  HostRows old{};
  {
    std::lock_guard<std::mutex> lk(host_rows_mu());
    auto &pool = host_rows_pool();
    size_t best = pool.size();
    for (size_t i = 0; i < pool.size(); ++i)
      if (pool[i].cap >= cnt && (best == pool.size() || pool[i].cap < pool[best].cap)) best = i;
    if (best < pool.size()) {
      HostRows b = pool[best];
      pool.erase(pool.begin() + (std::ptrdiff_t)best);
      return b;
    }
    if (!pool.empty()) {  // replace the largest (too small) buffer
      size_t big = 0;
      for (size_t i = 1; i < pool.size(); ++i)
        if (pool[i].cap > pool[big].cap) big = i;
      old = pool[big];
      pool.erase(pool.begin() + (std::ptrdiff_t)big);
    }
  }
  host_rows_free(old);
  HostRows b;
  void *q = nullptr;
  if (hipHostMalloc(&q, 8 * cnt, hipHostMallocDefault) == hipSuccess) {
    b.p = static_cast<int64_t *>(q);
    b.pinned = true;
  } else {
    (void)hipGetLastError();
    b.p = new (std::nothrow) int64_t[cnt];
  }
  b.cap = b.p ? cnt : 0;
  return b;
}
struct HostRowsLease {
  HostRows b;
  ~HostRowsLease() {
    if (!b.p) return;
    std::lock_guard<std::mutex> lk(host_rows_mu());
    host_rows_pool().push_back(b);
  }
};

// Build the static schedule of the rows of `ptr` (NULL: every row has one
// item) on the host: runs of consecutive low-degree vertices, single-row
// ranges, and hub chunks, partitions and staging areas.  Synchronises.
// row_max: longest row with a workgroup of its own (longer rows are hubs);
// staged_max: longest hub staged in partitions (longer hubs use a global set).
// Hub plan (staged chunks and partitions, global-set chunks) of a schedule
// whose range lists are already counted in s, and the uploads: the range
// lists and the hub list when they were built on the host (host_ranges),
// then the hub plan.  Synchronises.
int plan_hubs(kbisim_ctx *c, Schedule &s, const std::vector<int> &hubs, const std::vector<int64_t> &hub_deg,
              int64_t staged_max, const std::vector<Range> *host_ranges) {
  const Tuning &t = c->tune;
  const int64_t nranges_total = (int64_t)s.nranges + s.nbig + s.nrow8 + s.nrow20;
  // hubs: staged (partitioned) unless very large or out of offset space
  std::vector<HubChunk> chunks;
  std::vector<HubPart> parts;
  std::vector<HubGChunk> gchunks;
  std::vector<char> is_staged(hubs.size(), 0);
  int64_t stage_at = 0, poff_at = 0;
  for (size_t i = 0; i < hubs.size(); ++i) {
    const int64_t d = hub_deg[i];
    const int64_t C = (d + t.hub_chunk - 1) / t.hub_chunk;
    const int P = hub_parts_for(t, d);
    const bool staged = d <= staged_max && C <= HUB_PMAX && poff_at + C * (P + 1) <= c->plan.npoff_max;
    if (!staged) continue;
    HubPart hp;
    hp.hub = (int)i;
    hp.chunk0 = (int)chunks.size();
    hp.nchunks = (int)C;
    for (int64_t k = 0; k < C; ++k) {
      HubChunk hc;
      hc.hub = (int)i;
      hc.parts = P;
      hc.b = k * t.hub_chunk;
      hc.e = std::min<int64_t>(d, (k + 1) * t.hub_chunk);
      hc.stage = stage_at;
      hc.poff = poff_at;
      stage_at += t.hub_chunk;
      poff_at += P + 1;
      chunks.push_back(hc);
    }
    for (int q = 0; q < P; ++q) {
      hp.part = q;
      parts.push_back(hp);
    }
    is_staged[i] = 1;
    s.info[4] += 1;
    s.info[5] += d;
  }
  // global sets of the remaining hubs follow the staging areas
  s.gset_begin = stage_at;
  int64_t gset_at = stage_at;
  for (size_t i = 0; i < hubs.size(); ++i) {
    if (is_staged[i]) continue;
    const int64_t d = hub_deg[i];
    const int64_t size = 2 * d;
    for (int64_t b = 0; b < d; b += HUB_GCHUNK) {
      HubGChunk g;
      g.hub = (int)i;
      g.pad = 0;
      g.b = b;
      g.e = std::min<int64_t>(d, b + HUB_GCHUNK);
      g.set_off = gset_at;
      g.set_size = size;
      gchunks.push_back(g);
    }
    gset_at += size;
    s.info[6] += 1;
    s.info[7] += d;
  }
  s.gset_end = gset_at;
  if (nranges_total > c->plan.max_ranges || gset_at > c->plan.hubset_slots ||
      (int64_t)chunks.size() > c->plan.nchunk_max || (int64_t)parts.size() > c->plan.npart_max ||
      (int64_t)gchunks.size() > c->plan.ngchunk_max || (int64_t)hubs.size() > c->plan.nhub_max ||
      (int64_t)hubs.size() > c->plan.max_lists)
    return KBISIM_EINTERNAL;
  s.hub_off = 0;
  s.nhub = (int)hubs.size();
  s.nchunks = (int)chunks.size();
  s.nparts = (int)parts.size();
  s.ngchunks = (int)gchunks.size();
  if (host_ranges && !host_ranges->empty())
    HIP_TRY(hipMemcpyAsync(c->ranges, host_ranges->data(), sizeof(Range) * host_ranges->size(), hipMemcpyHostToDevice,
                           c->stream));
  if (host_ranges && !hubs.empty())
    HIP_TRY(hipMemcpyAsync(c->lists, hubs.data(), 4 * hubs.size(), hipMemcpyHostToDevice, c->stream));
  if (!chunks.empty())
    HIP_TRY(hipMemcpyAsync(c->chunks, chunks.data(), sizeof(HubChunk) * chunks.size(), hipMemcpyHostToDevice,
                           c->stream));
  if (!parts.empty())
    HIP_TRY(hipMemcpyAsync(c->parts, parts.data(), sizeof(HubPart) * parts.size(), hipMemcpyHostToDevice, c->stream));
  if (!gchunks.empty())
    HIP_TRY(hipMemcpyAsync(c->gchunks, gchunks.data(), sizeof(HubGChunk) * gchunks.size(), hipMemcpyHostToDevice,
                           c->stream));
  int rc = 0;
  if (s.nhub) {
    if ((rc = fill_u64(c, c->hacc, s.nhub, 0))) return rc;
    if ((rc = fill_i32(c, (int *)c->hcnt, s.nhub, 0))) return rc;
    if ((rc = fill_u64(c, c->hubsets + s.gset_begin, s.gset_end - s.gset_begin, 0))) return rc;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return 0;
}

// The schedule of graph rows built on the device (k_sched_walk): two walks
// over fixed vertex chunks, a host scan of the per-chunk counts in between;
// only the counts, the hub list and the hubs' degrees come back to the host.
// Scratch: c->vlist (4n bytes; n >= 64).
int build_schedule_device(kbisim_ctx *c, const int64_t *ptr, Schedule &s, int range_edges, int64_t row_max,
                          int64_t staged_max) {
  const int64_t n = c->g.n;
  const int nch = (int)((n + SCHED_CHUNK_V - 1) / SCHED_CHUNK_V);
  int *cnt = c->vlist, *off = cnt + 5 * (size_t)nch, *base = off + 5 * (size_t)nch;
  int64_t *sums = reinterpret_cast<int64_t *>(c->vlist) + (10 * (size_t)nch + 4 + 1) / 2 + 1;
  if ((size_t)((char *)(sums + 5 * (size_t)nch) - (char *)c->vlist) > 4 * (size_t)n) return KBISIM_EINTERNAL;
  const unsigned grid = blocks_for(nch, 64);
  k_sched_walk<false><<<grid, 64, 0, c->stream>>>(ptr, n, nch, range_edges, row_max, cnt, sums, nullptr, nullptr,
                                                  nullptr, nullptr);
  LAUNCH_CHECK();
  std::vector<int> hc(5 * (size_t)nch);
  std::vector<int64_t> hs(5 * (size_t)nch);
  HIP_TRY(hipMemcpyAsync(hc.data(), cnt, 4 * hc.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(hs.data(), sums, 8 * hs.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  int64_t tot[5] = {0, 0, 0, 0, 0};
  std::vector<int> ho(5 * (size_t)nch);
  for (int l = 0; l < 5; ++l)
    for (int ci = 0; ci < nch; ++ci) {
      ho[(size_t)l * nch + ci] = (int)tot[l];
      tot[l] += hc[(size_t)l * nch + ci];
    }
  for (int ci = 0; ci < nch; ++ci) {
    for (int i = 0; i < 4; ++i) s.info[i] += hs[5 * (size_t)ci + i];
    s.nonempty += hs[5 * (size_t)ci + 4];
  }
  if (tot[0] + tot[1] + tot[2] + tot[3] > c->plan.max_ranges || tot[4] > c->plan.nhub_max ||
      tot[4] > c->plan.max_lists)
    return KBISIM_EINTERNAL;
  s.nranges = (int)tot[0];
  s.nbig = (int)tot[1];
  s.nrow8 = (int)tot[2];
  s.nrow20 = (int)tot[3];
  const int hb[4] = {0, (int)tot[0], (int)(tot[0] + tot[1]), (int)(tot[0] + tot[1] + tot[2])};
  HIP_TRY(hipMemcpyAsync(off, ho.data(), 4 * ho.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(base, hb, sizeof hb, hipMemcpyHostToDevice, c->stream));
  k_sched_walk<true><<<grid, 64, 0, c->stream>>>(ptr, n, nch, range_edges, row_max, nullptr, nullptr, off, base,
                                                 c->ranges, c->lists);
  LAUNCH_CHECK();
  const int nh = (int)tot[4];
  std::vector<int> hubs((size_t)nh);
  std::vector<int64_t> hub_deg((size_t)nh);
  if (nh > 0) {
    // the hubs' degrees, in the key-hash array (8n bytes, unused at create time; nh <= n)
    int64_t *deg = reinterpret_cast<int64_t *>(c->H);
    k_row_degrees<<<blocks_for(nh, 256), 256, 0, c->stream>>>(nh, c->lists, ptr, deg);
    LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(hubs.data(), c->lists, 4 * (size_t)nh, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hub_deg.data(), deg, 8 * (size_t)nh, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return plan_hubs(c, s, hubs, hub_deg, staged_max, nullptr);
}

int build_schedule(kbisim_ctx *c, const int64_t *ptr, Schedule &s, int range_edges, int64_t row_max,
                   int64_t staged_max) {
  const int64_t n = c->g.n;
  const Tuning &t = c->tune;
  s = Schedule{};
  s.range_edges = range_edges;
  // (the device walk needs 80 bytes of scratch per chunk in the 4n bytes of vlist)
  if (ptr && (n >= SCHED_DEVICE_MIN || (c->tune.device_schedule && n >= 64)))
    return build_schedule_device(c, ptr, s, range_edges, row_max, staged_max);
  HostRowsLease lease;
  std::vector<int64_t> pageable;  // when no pinned host memory may be taken
  const int64_t *rp = nullptr;
  if (ptr && n > 0) {
    int64_t *dst = nullptr;
    if (c->pinned_ok) {
      lease.b = host_rows_take((size_t)n + 1);
      dst = lease.b.p;
    } else {
      try {
        pageable.resize((size_t)n + 1);
      } catch (...) {
        return KBISIM_EINTERNAL;
      }
      dst = pageable.data();
    }
    if (!dst) return KBISIM_EINTERNAL;
    HIP_TRY(hipMemcpyAsync(dst, ptr, 8 * (size_t)(n + 1), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    rp = dst;
  }
  // Degree tiers.  Rows are packed greedily into ranges of consecutive
  // vertices; the vertex sequence is cut into SCHED_CHUNKS fixed chunks that
  // are packed in parallel (a range never crosses a chunk boundary), so the
  // schedule is the same on every machine.
  struct Part {
    std::vector<Range> ranges, big, row8, row20;
    std::vector<int> hubs;
    int64_t info[4] = {0, 0, 0, 0};
    int64_t nonempty = 0;
  };
  std::vector<Part> parts_((size_t)SCHED_CHUNKS);
  auto pack = [&](int ci) {
    Part &P = parts_[(size_t)ci];
    const int64_t v_begin = n * ci / SCHED_CHUNKS, v_end = n * (ci + 1) / SCHED_CHUNKS;
    if (!ptr) {
      // one label per vertex: every row has one item, ranges of RANGE_VERTS vertices
      for (int64_t v0 = v_begin; v0 < v_end; v0 += RANGE_VERTS)
      {
        const int64_t v1 = std::min<int64_t>(v_end, v0 + RANGE_VERTS);
        P.ranges.push_back(Range{(int)v0, (int)v1, (int)(v1 - v0), 0, v0});
      }
      P.info[0] = P.info[1] = P.nonempty = v_end - v_begin;
      return;
    }
    int64_t cur0 = -1, cur_e = 0;
    auto close = [&](int64_t vend) {
      if (cur0 >= 0) P.ranges.push_back(Range{(int)cur0, (int)vend, (int)cur_e, 0, rp[(size_t)cur0]});
      cur0 = -1;
      cur_e = 0;
    };
    for (int64_t v = v_begin; v < v_end; ++v) {
      const int64_t d = rp[(size_t)v + 1] - rp[(size_t)v];
      P.nonempty += d > 0;
      if (d > row_max) {
        close(v);
        P.hubs.push_back((int)v);
        continue;
      }
      if (d > ROW_MAX) {
        close(v);
        P.row20.push_back(Range{(int)v, (int)v + 1, (int)d, 0, rp[(size_t)v]});
        P.info[2] += 1;
        P.info[3] += d;
        continue;
      }
      if (d > RANGE_DMAX) {
        close(v);
        P.row8.push_back(Range{(int)v, (int)v + 1, (int)d, 0, rp[(size_t)v]});
        P.info[2] += 1;
        P.info[3] += d;
        continue;
      }
      if (d > range_edges) {
        close(v);
        P.big.push_back(Range{(int)v, (int)v + 1, (int)d, 0, rp[(size_t)v]});
        P.info[2] += 1;
        P.info[3] += d;
        continue;
      }
      if (cur0 >= 0 && (cur_e + d > range_edges || v - cur0 == RANGE_VERTS)) close(v);
      if (cur0 < 0) cur0 = v;
      cur_e += d;
      P.info[0] += 1;
      P.info[1] += d;
    }
    close(v_end);
  };
  // Chunks run on threads when there is enough work; a chunk whose thread
  // cannot be started is packed here (no exception leaves the library).
  std::vector<std::thread> th;
  std::vector<char> started((size_t)SCHED_CHUNKS, 0);
  if (n >= (int64_t)1 << 16) {
    for (int ci = 0; ci < SCHED_CHUNKS; ++ci) {
      try {
        th.emplace_back(pack, ci);
        started[(size_t)ci] = 1;
      } catch (...) {
        break;
      }
    }
  }
  for (int ci = 0; ci < SCHED_CHUNKS; ++ci)
    if (!started[(size_t)ci]) pack(ci);
  for (auto &x : th) x.join();
  std::vector<Range> ranges, big_ranges, row8_ranges, row20_ranges;
  std::vector<int> hubs;
  for (const Part &P : parts_) {
    row20_ranges.insert(row20_ranges.end(), P.row20.begin(), P.row20.end());
    ranges.insert(ranges.end(), P.ranges.begin(), P.ranges.end());
    big_ranges.insert(big_ranges.end(), P.big.begin(), P.big.end());
    row8_ranges.insert(row8_ranges.end(), P.row8.begin(), P.row8.end());
    hubs.insert(hubs.end(), P.hubs.begin(), P.hubs.end());
    for (int i = 0; i < 4; ++i) s.info[i] += P.info[i];
    s.nonempty += P.nonempty;
  }
  auto deg = [&](int64_t v) -> int64_t { return ptr ? rp[(size_t)v + 1] - rp[(size_t)v] : 1; };
  s.nranges = (int)ranges.size();
  s.nbig = (int)big_ranges.size();
  s.nrow8 = (int)row8_ranges.size();
  s.nrow20 = (int)row20_ranges.size();
  ranges.insert(ranges.end(), big_ranges.begin(), big_ranges.end());
  ranges.insert(ranges.end(), row8_ranges.begin(), row8_ranges.end());
  ranges.insert(ranges.end(), row20_ranges.begin(), row20_ranges.end());
  std::vector<int64_t> hub_deg(hubs.size());
  for (size_t i = 0; i < hubs.size(); ++i) hub_deg[i] = deg(hubs[i]);
  return plan_hubs(c, s, hubs, hub_deg, staged_max, &ranges);
}

// Bits needed for x (0 for 0).
int bit_width(uint64_t x) {
  int b = 0;
  while (b < 64 && (x >> b) != 0) ++b;
  return b;
}

// Rank vertices by decreasing in-degree (ties by vertex id) and renumber the
// targets of every CSR entry: gcol[e] = rank[col[e]].  Vertices no entry
// names get rank -1: they are never gathered.  A stable LSD radix sort of
// (in-degree key, vertex) on the device; the grouping tables serve as
// scratch, so this runs before they are cleared.  Synchronises.
int build_rank(kbisim_ctx *c) {
  const int64_t n = c->g.n, m = c->g.m;
  if (n == 0) return 0;
  int *indeg = c->vlist;  // scratch
  int rc = fill_i32(c, indeg, n, 0);
  if (rc) return rc;
  if (m > 0) {
    k_indegree<<<(unsigned)std::min<int64_t>(blocks_for(m, INDEG_CHUNK), 1 << 16), 256, 0, c->stream>>>(m, c->g.col,
                                                                                                       indeg);
    LAUNCH_CHECK();
  }
  u64 *ka = c->table, *kb = c->table + n;  // 8 * tslots >= 16 n bytes
  const int64_t rtiles = (n + RADIX_TILE - 1) / RADIX_TILE, hist_n = 256 * rtiles;
  int *hist = (int *)c->ctable;
  int64_t *offs = (int64_t *)(c->ctable) + (hist_n + 1) / 2 + 1;
  int64_t *tiles = offs + hist_n + 2;
  if ((size_t)((char *)(tiles + (hist_n + SCAN_TILE - 1) / SCAN_TILE + 1) - (char *)c->ctable) > 8 * c->plan.tslots)
    return KBISIM_EINTERNAL;
  k_rank_keys<<<(unsigned)std::min<int64_t>(blocks_for(n, 256), 1 << 16), 256, 0, c->stream>>>(n, indeg, ka);
  LAUNCH_CHECK();
  // stable LSD passes of 8 bits over key bits [32, 32 + bits)
  auto radix_passes = [&](int bits) -> int {
    for (int shift = 32; shift < 32 + bits; shift += 8) {
      k_radix_hist<<<(unsigned)rtiles, 256, 0, c->stream>>>(n, ka, shift, rtiles, hist);
      LAUNCH_CHECK();
      const int64_t nt = (hist_n + SCAN_TILE - 1) / SCAN_TILE;
      k_sum_tiles64<<<(unsigned)nt, 256, 0, c->stream>>>(hist_n, hist, tiles);
      k_scan_tiles64<<<1, 256, 0, c->stream>>>(nt, tiles);
      k_write_ptr64<<<(unsigned)nt, 256, 0, c->stream>>>(hist_n, hist, tiles, offs, nullptr);
      LAUNCH_CHECK();
      k_radix_scatter<<<(unsigned)rtiles, 256, 0, c->stream>>>(n, ka, shift, rtiles, offs, hist, kb);
      LAUNCH_CHECK();
      std::swap(ka, kb);
    }
    return 0;
  };
  if ((rc = radix_passes(RANK_KEYBITS))) return rc;
  if (c->num_graphs > 1) {
    // In a batch, ranks stay inside each graph's vertex range (ordered by
    // in-degree within the graph): a graph's gathers then touch its own
    // part of the partition only, instead of the whole union's.
    k_rank_gid_keys<<<(unsigned)std::min<int64_t>(blocks_for(n, 256), 1 << 16), 256, 0, c->stream>>>(n, ka, c->gid,
                                                                                                    kb);
    LAUNCH_CHECK();
    std::swap(ka, kb);
    if ((rc = radix_passes(bit_width((uint64_t)(c->num_graphs - 1))))) return rc;
  }
  k_rank_from_sorted<<<(unsigned)std::min<int64_t>(blocks_for(n, 256), 1 << 16), 256, 0, c->stream>>>(n, ka, indeg,
                                                                                                 c->rank);
  LAUNCH_CHECK();
  if (m > 0) {
    k_remap<<<(unsigned)std::min<int64_t>(blocks_for(m, 256), 1 << 16), 256, 0, c->stream>>>(
        m, c->g.col, c->rank, c->gcol, c->packed ? c->g.elabel : nullptr, c->rbits);
    LAUNCH_CHECK();
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return 0;
}

// One peeling round over `in_list` (count at in_cnt) into out_list/out_cnt.
template <class Src>
int peel_round(kbisim_ctx *c, const Src &src, int *in_cnt, int *in_list, int *out_cnt, int *out_list) {
  ProfScope ps(c, KBISIM_K_PEEL);
  k_res_insert<<<RES_GRID, 256, 0, c->stream>>>(in_cnt, in_list, c->H, c->ctable, c->plan.tslots - 1, c->dep);
  LAUNCH_CHECK();
  k_res_verify<Src><<<RES_GRID, 256, 0, c->stream>>>(src, in_cnt, in_list, c->H, c->DC, c->ctable,
                                                     c->plan.tslots - 1, c->dep, c->rep, out_cnt, out_list, c->err);
  LAUNCH_CHECK();
  return 0;
}

// Refinement steps group only vertices with edges (the rest go by previous
// block alone), so their table span is sized by that count; P0 uses it all.
template <class Src>
u64 table_mask(const kbisim_ctx *c) {
  if constexpr (Src::GRAPH) return c->tmask_steps;
  return c->plan.tslots - 1;
}

template <class Src, class K, bool SKIP>
int launch_range_kernel(kbisim_ctx *c, const Src &src, const Schedule &s, u64 tmask, int zfresh,
                        const unsigned char *skip) {
  ProfScope ps(c, KBISIM_K_SIG_RANGE);
  if (s.range_edges == 1024)
    k_sig_range<Src, 1024, K, SKIP><<<(unsigned)s.nranges, 256, 0, c->stream>>>(
        src, c->ranges, c->H, c->DC, c->table, tmask, c->dep, c->hmask, c->zrep, zfresh, skip);
  else
    k_sig_range<Src, 2048, K, SKIP><<<(unsigned)s.nranges, 256, 0, c->stream>>>(
        src, c->ranges, c->H, c->DC, c->table, tmask, c->dep, c->hmask, c->zrep, zfresh, skip);
  LAUNCH_CHECK();
  return 0;
}

// skip: singleton flags of the previous partition (work-efficient mode), or NULL.
template <class Src, class K>
int launch_ranges_k(kbisim_ctx *c, const Src &src, const Schedule &s, int zfresh, const unsigned char *skip,
                    bool range_tier = true) {
  const u64 tmask = table_mask<Src>(c);
  if (s.nranges && range_tier) {
    int rc = 0;
    if constexpr (Src::GRAPH) {
      rc = skip ? launch_range_kernel<Src, K, true>(c, src, s, tmask, zfresh, skip)
                : launch_range_kernel<Src, K, false>(c, src, s, tmask, zfresh, nullptr);
    } else {
      rc = launch_range_kernel<Src, K, false>(c, src, s, tmask, zfresh, nullptr);
    }
    if (rc) return rc;
  }
  if (s.nbig || s.nrow8 || s.nrow20) {
    ProfScope ps(c, KBISIM_K_SIG_BLOCK);
    if (s.nbig) {
      k_sig_row<Src, RANGE_DMAX, 512, K><<<(unsigned)s.nbig, 512, 0, c->stream>>>(
          src, c->ranges + s.nranges, c->H, c->DC, c->table, tmask, c->dep, c->hmask, c->zrep, skip);
      LAUNCH_CHECK();
    }
    if (s.nrow8) {
      k_sig_row<Src, ROW_MAX, 1024, K><<<(unsigned)s.nrow8, 1024, 0, c->stream>>>(
          src, c->ranges + s.nranges + s.nbig, c->H, c->DC, c->table, tmask, c->dep, c->hmask, c->zrep, skip);
      LAUNCH_CHECK();
    }
    if constexpr (std::is_same<K, u32>::value) {
      if (s.nrow20) {
        k_sig_row<Src, ROW_MAX_NARROW, 1024, u32><<<(unsigned)s.nrow20, 1024, 0, c->stream>>>(
            src, c->ranges + s.nranges + s.nbig + s.nrow8, c->H, c->DC, c->table, tmask, c->dep, c->hmask, c->zrep,
            skip);
        LAUNCH_CHECK();
      }
    }
  }
  return 0;
}

template <class Src>
int launch_ranges(kbisim_ctx *c, const Src &src, const Schedule &s, int zfresh, const unsigned char *skip,
                  bool range_tier = true) {
  if constexpr (Src::HASHED) {
    return launch_ranges_k<Src, u32>(c, src, s, zfresh, skip, range_tier);
  } else {
    if constexpr (Src::GRAPH) {
      if (c->narrow) return launch_ranges_k<Src, u32>(c, src, s, zfresh, skip, range_tier);
    }
    return launch_ranges_k<Src, u64>(c, src, s, zfresh, skip, range_tier);
  }
}

// Staged hub rows: chunk dedupe and partitioned staging, then per-partition
// dedupe and sums.  K: width of the staged keys.
template <class Src, class K>
int launch_hub_staged(kbisim_ctx *c, const Src &src, const Schedule &s, const int *hubs,
                      const unsigned char *skip) {
  K *stage = reinterpret_cast<K *>(c->hubsets);
  {
    ProfScope ps(c, KBISIM_K_HUB_STAGE);
    if (c->tune.hub_chunk == 2048)
      k_hub_stage<Src, 2048, K><<<(unsigned)s.nchunks, 256, 0, c->stream>>>(src, c->chunks, hubs, stage, c->poff,
                                                                            c->err, skip);
    else
      k_hub_stage<Src, 4096, K><<<(unsigned)s.nchunks, 256, 0, c->stream>>>(src, c->chunks, hubs, stage, c->poff,
                                                                            c->err, skip);
    LAUNCH_CHECK();
  }
  ProfScope ps(c, KBISIM_K_HUB_REDUCE);
  k_hub_reduce<Src, K><<<(unsigned)s.nparts, 256, 0, c->stream>>>(src, c->parts, c->chunks, stage, c->poff, c->hacc,
                                                                  c->hcnt, c->err, hubs, skip);
  LAUNCH_CHECK();
  return 0;
}

// One refinement step: src (previous partition inside) -> out, block count
// into *count_dev.  cnt: CNT_STRIDE zeroed device counters for this step.
// careful: settle every collision with host-driven peeling rounds.
// gpid_next: where to write the new partition in rank order (NULL: not needed).
// zfresh: group vertices with an empty signature afresh (the first step of a
// call); otherwise their representatives from that step are kept, since two
// such vertices share a block after a step exactly when they did before it.
// skip_in / single_out (work-efficient mode, else NULL): singleton flags of
// the previous partition (those vertices are not refined: a singleton block
// cannot split) and of the new one.
// Signatures of every vertex not flagged in skip_in (all tiers): key hash,
// distinct count and the insertion into the grouping table.
template <class Src>
int launch_signatures(kbisim_ctx *c, const Src &src, const Schedule &s, bool zfresh, const unsigned char *skip_in,
                      bool range_tier = true) {
  const u64 tmask = table_mask<Src>(c);
  int rc = 0;
  if ((rc = launch_ranges(c, src, s, zfresh ? 1 : 0, skip_in, range_tier))) return rc;
  if (s.nhub) {
    const int *hubs = c->lists + s.hub_off;
    if (s.nchunks) {
      if constexpr (Src::HASHED) {
        rc = launch_hub_staged<Src, u32>(c, src, s, hubs, skip_in);
      } else if constexpr (Src::GRAPH) {
        rc = c->narrow ? launch_hub_staged<Src, u32>(c, src, s, hubs, skip_in)
                       : launch_hub_staged<Src, u64>(c, src, s, hubs, skip_in);
      } else {
        rc = launch_hub_staged<Src, u64>(c, src, s, hubs, skip_in);
      }
      if (rc) return rc;
    }
    if (s.ngchunks) {
      ProfScope ps(c, KBISIM_K_HUB_STAGE);
      k_sig_hub_global<Src><<<(unsigned)s.ngchunks, 256, 0, c->stream>>>(src, c->gchunks, hubs, c->hubsets, c->hacc,
                                                                         c->hcnt, c->dep, skip_in);
      LAUNCH_CHECK();
    }
    ProfScope ps(c, KBISIM_K_HUB_FINAL);
    k_hub_final<Src><<<blocks_for(s.nhub, 256), 256, 0, c->stream>>>(src, hubs, s.nhub, c->hacc, c->hcnt, c->H, c->DC,
                                                                     c->table, tmask, c->dep, c->hmask, c->zrep,
                                                                     skip_in);
    LAUNCH_CHECK();
  }
  return 0;
}

// After the lookup: exact checks of longer rows, one peeling round and, when
// careful, host-driven peeling rounds until no collision is left.
template <class Src>
int settle_collisions(kbisim_ctx *c, const Src &src, const Schedule &s, int *cnt, bool careful) {
  const int n = (int)c->g.n;
  int rc = 0;
  {
    ProfScope ps(c, KBISIM_K_VERIFY);
    k_verify<Src><<<PERSIST_GRID, 256, 0, c->stream>>>(src, &cnt[0], c->vlist, c->DC, c->rep, &cnt[1], c->clA,
                                                       c->err);
    LAUNCH_CHECK();
  }
  rc = peel_round(c, src, &cnt[1], c->clA, &cnt[2], c->clB);
  if (rc) return rc;
  if (careful) {
    int *in_cnt = &cnt[2], *out_cnt = &cnt[3];
    int *in_list = c->clB, *out_list = c->clA;
    for (int round = 0;; ++round) {
      int left = 0;
      HIP_TRY(hipMemcpyAsync(&left, in_cnt, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      prof_collect(c);
      if (left == 0) break;
      if (round > n + 1) return KBISIM_EINTERNAL;
      if ((rc = fill_i32(c, out_cnt, 1, 0))) return rc;
      if ((rc = advance(c, ADV_CTABLE, s))) return rc;
      if ((rc = peel_round(c, src, in_cnt, in_list, out_cnt, out_list))) return rc;
      std::swap(in_cnt, out_cnt);
      std::swap(in_list, out_list);
    }
  }
  return 0;
}

template <class Src>
int run_step(kbisim_ctx *c, const Src &src, const Schedule &s, int *out, int64_t *count_dev, int *cnt,
             bool careful, int *gpid_next, bool zfresh, const unsigned char *skip_in = nullptr,
             unsigned char *single_out = nullptr, int32_t *names_out = nullptr) {
  const int n = (int)c->g.n;
  if (n == 0) return 0;
  const u64 tmask = table_mask<Src>(c);
  int rc = advance(c, ADV_TABLE | ADV_CTABLE | ADV_ZERO | (s.ngchunks ? ADV_HUB : 0u), s);
  if (rc) return rc;
  if ((rc = launch_signatures(c, src, s, zfresh, skip_in))) return rc;
  {
    ProfScope ps(c, KBISIM_K_LOOKUP);
    // after a call's first step only vertices with edges can change their
    // representative (the others keep the one of that step)
    const bool listed = !zfresh && s.nzv != nullptr;
    const int count = listed ? (int)s.nonempty : n;
    k_lookup<Src><<<blocks_for(std::max(count, 1), 256), 256, 0, c->stream>>>(
        src, count, listed ? s.nzv : nullptr, c->H, c->DC, c->table, tmask, c->dep, c->rep,
                                                             &cnt[0], c->vlist, &cnt[1], c->clA, c->err, c->zrep,
                                                             zfresh ? 1 : 0, skip_in, nullptr, nullptr);
    LAUNCH_CHECK();
  }
  if ((rc = settle_collisions(c, src, s, cnt, careful))) return rc;
  HeadIds ids{};
  {
    ProfScope ps(c, KBISIM_K_SCAN);
    if ((rc = numbering_words(c, n, count_dev, &ids))) return rc;
  }
  {
    ProfScope ps(c, KBISIM_K_ASSIGN);
    if (names_out) {
      k_assign_names<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->rep, ids, out, names_out,
                                                                gpid_next ? c->rank : nullptr, gpid_next, nullptr,
                                                                nullptr, nullptr, nullptr, nullptr);
    } else {
      k_assign<<<blocks_for((n + ASSIGN_V - 1) / ASSIGN_V, 256), 256, 0, c->stream>>>(
          n, c->rep, ids, out, gpid_next ? c->rank : nullptr, gpid_next, single_out ? c->multi : nullptr, c->dep);
    }
    LAUNCH_CHECK();
    if (single_out) {
      k_singletons<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->rep, c->multi, c->dep, single_out);
      LAUNCH_CHECK();
    }
  }
  return 0;
}

// Enqueue steps [i0, k) starting from partition `prev` (no host
// synchronisation unless careful).  In a batch, step i refines into an
// internal buffer of global ids and writes the caller's per-graph ids and
// counts (graph g's count of step i at bcounts[g * cstride + i]).  scatter:
// copy prev into the rank-ordered buffer first (false only when the previous
// step of this context already left it there).
int enqueue_steps(kbisim_ctx *c, const int32_t *prev, int i0, int k, int32_t *const *out, bool careful,
                  int cstride, bool scatter = true) {
  const int n = (int)c->g.n;
  const bool batch = c->num_graphs > 0;
  int rc = 0;
  if (scatter) {
    k_scatter_rank<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, prev, c->rank, c->gpid[i0 & 1]);
    LAUNCH_CHECK();
  }
  for (int i = i0; i < k; ++i) {
    if (careful && (rc = fill_i32(c, c->counters + CNT_STRIDE * i, CNT_STRIDE, 0))) return rc;
    int *dst = batch ? c->ibuf[i & 1] : out[i];
    // work-efficient mode: singletons of P_i (flags of step i-1) are not refined
    const unsigned char *skip_in = (c->work_eff && i > 0) ? c->single[(i - 1) & 1] : nullptr;
    unsigned char *single_out = c->work_eff ? c->single[i & 1] : nullptr;
    // with a cached chain (incremental updates) the next step names blocks by
    // their minimum vertex, written into the cache
    const bool cache = c->incr && !batch;
    int32_t *names_out = cache ? c->is.MVc + (size_t)i * (size_t)n : nullptr;
    auto step = [&](auto src) {
      return run_step(c, src, c->sched, dst, &c->dcounts[i], c->counters + CNT_STRIDE * i, careful,
                      c->gpid[(i + 1) & 1], i == 0, skip_in, single_out, names_out);
    };
    const int32_t *lab = separate_labels(c) ? sep_labels(c) : nullptr;
    if (c->hashed) {
      if (lab)
        rc = step(GraphSrcT<true, true>{c->g.row_ptr, c->gcol, lab, c->gpid[i & 1], prev, c->pb, c->rbits, c->kmask});
      else
        rc = step(
            GraphSrcT<false, true>{c->g.row_ptr, c->gcol, nullptr, c->gpid[i & 1], prev, c->pb, c->rbits, c->kmask});
    } else {
      if (lab) rc = step(GraphSrcT<true>{c->g.row_ptr, c->gcol, lab, c->gpid[i & 1], prev, c->pb, c->rbits});
      else rc = step(GraphSrcT<false>{c->g.row_ptr, c->gcol, nullptr, c->gpid[i & 1], prev, c->pb, c->rbits});
    }
    if (rc) return rc;
    if (batch) {
      k_rebase<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->gid, c->first, dst, out[i]);
      LAUNCH_CHECK();
      k_batch_counts<<<blocks_for(c->num_graphs, 256), 256, 0, c->stream>>>((int)c->num_graphs, c->first, c->next,
                                                                            dst, &c->dcounts[i], cstride, i, c->bcounts);
      LAUNCH_CHECK();
    }
    if (names_out) {
      const unsigned g = std::min<unsigned>(blocks_for(2 * (int64_t)n, 256), 65536);
      k_copy_i32<<<g, 256, 0, c->stream>>>(reinterpret_cast<int *>(c->is.Hc + (size_t)i * (size_t)n),
                                           reinterpret_cast<const int *>(c->H), 2 * (int64_t)n);
      k_copy_i32<<<g, 256, 0, c->stream>>>(reinterpret_cast<int *>(c->is.DCc + (size_t)i * (size_t)n),
                                           reinterpret_cast<const int *>(c->DC), (int64_t)n);
      k_filter_keys<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->H, c->DC, prev,
                                                                c->is.FKc + (size_t)i * (size_t)n);
      LAUNCH_CHECK();
      prev = names_out;
    } else {
      prev = dst;
    }
  }
  return 0;
}

// Work-efficient refinement: singleton blocks are not refined (skip flags
// from the previous step), and once a step leaves the block count unchanged
// the partition is a fixpoint (a refinement with as many blocks is the same
// partition), so the remaining outputs are copies.  Synchronises after every
// step to read its count.
int refine_we(kbisim_ctx *c, const int32_t *start, int k, int32_t *const *out, int64_t *counts) {
  const int n = (int)c->g.n;
  const bool batch = c->num_graphs > 0;
  const int32_t *p0 = start ? start : c->p0;
  int64_t prev_count = start ? -1 : c->p0_count;
  int rc = 0;
  if ((rc = fill_i32(c, c->counters, (int64_t)CNT_STRIDE * k, 0))) return rc;
  if ((rc = fill_i32(c, (int *)c->err, 1, 0))) return rc;
  int done = k;
  for (int i = 0; i < k; ++i) {
    const int32_t *prev = i == 0 ? p0 : (batch ? c->ibuf[(i - 1) & 1] : out[i - 1]);
    if ((rc = enqueue_steps(c, prev, i, i + 1, out, false, k, i == 0))) return rc;
    int left = 0;
    u32 err = 0;
    int64_t cnt = 0;
    HIP_TRY(hipMemcpyAsync(&left, c->counters + CNT_STRIDE * i + 2, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(&err, c->err, sizeof err, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(&cnt, &c->dcounts[i], 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    prof_collect(c);
    if (err) return KBISIM_EINTERNAL;
    if (left) {
      if ((rc = enqueue_steps(c, prev, i, i + 1, out, true, k, true))) return rc;
      HIP_TRY(hipMemcpyAsync(&err, c->err, sizeof err, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipMemcpyAsync(&cnt, &c->dcounts[i], 8, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      prof_collect(c);
      if (err) return KBISIM_EINTERNAL;
    }
    if (cnt == prev_count) {
      done = i + 1;
      break;
    }
    prev_count = cnt;
  }
  for (int j = done; j < k; ++j)
    HIP_TRY(hipMemcpyAsync(out[j], out[done - 1], 4 * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
  if (batch) {
    const int64_t G = c->num_graphs;
    HIP_TRY(hipMemcpyAsync(counts, c->bcounts, 8 * (size_t)(G * k), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int64_t g = 0; g < G; ++g)
      for (int j = done; j < k; ++j) counts[g * k + j] = counts[g * k + done - 1];
  } else {
    HIP_TRY(hipMemcpyAsync(counts, c->dcounts, 8 * (size_t)done, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int j = done; j < k; ++j) counts[j] = counts[done - 1];
  }
  c->we_steps = done;
  return KBISIM_OK;
}

int refine_impl(kbisim_ctx *c, const int32_t *start, int k, int32_t *const *out, int64_t *counts) {
  if (!c) return KBISIM_EINVAL;
  if (k < 0 || k > c->kmax) return KBISIM_EINVAL;
  if (k == 0) return KBISIM_OK;
  if (!out || !counts) return KBISIM_EINVAL;
  for (int i = 0; i < k; ++i)
    if (!out[i] && c->g.n > 0) return KBISIM_EINVAL;
  const int n = (int)c->g.n;
  const bool batch = c->num_graphs > 0;
  const int64_t ncounts = batch ? c->num_graphs * (int64_t)k : (int64_t)k;
  if (n == 0) {
    for (int64_t i = 0; i < ncounts; ++i) counts[i] = 0;
    return KBISIM_OK;
  }
  if (c->work_eff) return refine_we(c, start, k, out, counts);
  if (c->incr) c->incr_k = 0;  // until this call completes
  const int32_t *p0 = start ? start : c->p0;
  int rc = 0;
  const bool graphed = c->use_graphs && !c->prof;
  if (graphed) {
    GraphKey key{start, k, std::vector<const void *>(out, out + k)};
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
      if ((int)c->graphs.size() >= MAX_GRAPH_CACHE) {
        (void)hipGraphExecDestroy(c->graphs.begin()->second);
        c->graphs.erase(c->graphs.begin());
      }
      HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      int rc1 = fill_i32(c, c->counters, (int64_t)CNT_STRIDE * k, 0);
      if (!rc1) rc1 = fill_i32(c, (int *)c->err, 1, 0);
      if (!rc1) rc1 = enqueue_steps(c, p0, 0, k, out, false, k);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(c->stream, &graph);
      if (rc1) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc1;
      }
      if (e != hipSuccess) return hip_fail(e);
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_fail(e);
      it = c->graphs.emplace(key, exec).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, c->stream));
  } else {
    if ((rc = fill_i32(c, c->counters, (int64_t)CNT_STRIDE * k, 0))) return rc;
    if ((rc = fill_i32(c, (int *)c->err, 1, 0))) return rc;
    if ((rc = enqueue_steps(c, p0, 0, k, out, false, k))) return rc;
  }
  std::vector<int> hc((size_t)CNT_STRIDE * k);
  u32 err = 0;
  HIP_TRY(hipMemcpyAsync(hc.data(), c->counters, 4 * hc.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&err, c->err, sizeof err, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  prof_collect(c);
  if (err) return KBISIM_EINTERNAL;
  int first_bad = -1;
  for (int i = 0; i < k; ++i)
    if (hc[(size_t)CNT_STRIDE * i + 2] != 0) {
      first_bad = i;
      break;
    }
  if (first_bad >= 0) {
    const int32_t *prev = first_bad == 0 ? p0 : (batch ? c->ibuf[(first_bad - 1) & 1] : out[first_bad - 1]);
    if (c->incr && !batch && first_bad > 0) prev = c->is.MVc + (size_t)(first_bad - 1) * (size_t)n;
    if ((rc = enqueue_steps(c, prev, first_bad, k, out, true, k))) return rc;
    HIP_TRY(hipMemcpyAsync(&err, c->err, sizeof err, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    prof_collect(c);
    if (err) return KBISIM_EINTERNAL;
  }
  if (batch) {
    HIP_TRY(hipMemcpyAsync(counts, c->bcounts, 8 * (size_t)ncounts, hipMemcpyDeviceToHost, c->stream));
  } else {
    HIP_TRY(hipMemcpyAsync(counts, c->dcounts, 8 * (size_t)k, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->incr && !batch) c->incr_k = start ? 0 : k;  // the cache holds a chain from P0
  return KBISIM_OK;
}

// ---------------------------------------------------------------- incremental updates
// The cached chain lives in a caller buffer: per step the key hash, distinct
// count and minimum-vertex block name of every vertex, plus the in-rows of
// the cached graph (to find the vertices whose targets' names changed) and
// per-update scratch.
struct IncrPlan {
  size_t off_hc, off_dcc, off_mvc, off_fk, off_tptr, off_tcol, off_names, off_edited, off_flag, off_dirty, off_skip,
      off_small, off_large, off_psmall, off_plarge, off_changed, off_bname, off_keep, off_claimed, off_heavy, off_touch,
      off_lk, off_filter, off_gfilter, off_zrep, off_huge, off_hchunks, off_hacc, off_hcnt, off_erows, off_cnt, total;
  int64_t huge_cap, huge_chunk_cap;
};
IncrPlan incr_plan(int64_t n, int64_t m, int kmax) {
  IncrPlan p{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t o = at;
    at = align_up(at + std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t N = (size_t)std::max<int64_t>(n, 1), K = (size_t)std::max(kmax, 1);
  p.off_hc = take(8 * N * K);
  p.off_dcc = take(4 * N * K);
  p.off_mvc = take(4 * N * K);
  p.off_fk = take(2 * N * K);
  p.off_tptr = take(8 * (N + 1));
  p.off_tcol = take(4 * (size_t)std::max<int64_t>(m, 1));
  p.off_names = take(8 * N);
  p.off_edited = take(N);
  p.off_flag = take(N);
  p.off_dirty = take(N);
  p.off_skip = take(N);
  p.off_small = take(4 * N);
  p.off_large = take(4 * N);
  p.off_psmall = take(4 * N);
  p.off_plarge = take(4 * N);
  p.off_changed = take(4 * N);
  p.off_bname = take(4 * N);
  p.off_keep = take(4 * N);
  p.off_claimed = take(N);
  p.off_heavy = take(4 * N);
  p.off_touch = take(4 * (N / 32 + 1));
  p.off_lk = take(4 * N);
  p.off_filter = take(4 * FILTER_WORDS);
  p.off_gfilter = take(4 * (size_t)GFILTER_WORDS);
  p.off_zrep = take(16 * N);
  p.huge_cap = std::max<int64_t>(m, 0) / LIST_BIG + 1;
  p.huge_chunk_cap = std::max<int64_t>(m, 0) / HUB_GCHUNK + p.huge_cap + 1;
  p.off_huge = take(4 * (size_t)p.huge_cap);
  p.off_hchunks = take(sizeof(HubGChunk) * (size_t)p.huge_chunk_cap);
  p.off_hacc = take(8 * (size_t)p.huge_cap);
  p.off_hcnt = take(4 * (size_t)p.huge_cap);
  p.off_erows = take(sizeof(Range) * (size_t)p.huge_cap);
  p.off_cnt = take(64);
  p.total = at;
  return p;
}

constexpr int LIST_GRID_SMALL = 2048, LIST_GRID_LARGE = 1024, MARK_GRID = 2048;

// Grouping-table mask for about `keys` keys at a load of at most 1/4 (a
// small table stays in the caches), within the allocated table.
u64 mask_for_keys(const kbisim_ctx *c, int64_t keys) {
  return std::min<u64>(pow2_at_least((uint64_t)std::max<int64_t>(4 * keys, 4096)), c->plan.tslots) - 1;
}

// One update step: P'_{i+1} from names_prev (P0 for i = 0, else the block
// names of P'_i).  Vertices flagged dirty had their key inputs changed: the
// edited rows are read from the edited graph (list kernels); the others whose
// targets' names changed are signed by the list kernels too when they are few
// (prop_lists), else by the cached graph's tiers with every other vertex
// skipped.  With few dirty vertices (prop_lists; at most ndirty of them) only
// the touched cached blocks are regrouped (k_classify), in a
// table sized for them, and every other vertex keeps its cached block and
// name; otherwise all vertices take their cached key hashes and go through
// the table.  Exact checks read the edited graph; numbering covers every
// vertex; block names follow k_block_names_*.  Returns in *gpid_written
// whether the names were also written in rank order for the next step.
template <class K, class TierSrc, class ListSrc>
int update_step(kbisim_ctx *c, const TierSrc &tsrc, const ListSrc &lsrc, int i, const int32_t *names_prev,
                int32_t *out, int64_t *count_dev, int *cnt, bool prop_lists, int nbig, int64_t ndirty,
                bool *gpid_written) {
  const int n = (int)c->g.n;
  const size_t at = (size_t)i * (size_t)n;
  auto &S = c->is;
  c->tmask_steps = prop_lists ? mask_for_keys(c, ndirty) : c->plan.tslots - 1;
  u64 tmask = c->tmask_steps;
  const Schedule &s = c->sched;
  // the hub epoch starts at 0 and must be in 1..3 before any global set is used
  int rc = advance(c, ADV_TABLE | ADV_CTABLE | ADV_ZERO | (s.ngchunks || S.nhuge ? ADV_HUB : 0u), s);
  if (rc) return rc;
  auto lists = [&](int *count, int *small, int *large) -> int {
    k_sig_list_small<ListSrc, K><<<LIST_GRID_SMALL, 256, 0, c->stream>>>(lsrc, count, small, c->H, c->DC, c->table,
                                                                         tmask, c->dep, c->hmask, c->zrep);
    LAUNCH_CHECK();
    k_sig_list_large<ListSrc, K><<<LIST_GRID_LARGE, 256, 0, c->stream>>>(lsrc, count + 1, large, c->H, c->DC,
                                                                         c->table, tmask, c->dep, c->hmask, c->zrep,
                                                                         c->err);
    LAUNCH_CHECK();
    return 0;
  };
  if (prop_lists) {
    // short and medium rows from lists, long ones by the row and hub tiers
    if ((rc = lists(&cnt[8], S.psmall, S.plarge))) return rc;
    if (nbig && (rc = launch_signatures(c, tsrc, s, true, S.skip, false))) return rc;
  } else {
    k_skip_all_flagged<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, S.edited, S.dirty, S.skip);
    LAUNCH_CHECK();
    if ((rc = launch_signatures(c, tsrc, s, true, S.skip))) return rc;
  }
  if ((rc = lists(&S.cnt[0], S.small, S.large))) return rc;
  if (S.nerows8) {
    k_sig_row<ListSrc, ROW_MAX, 1024, K><<<(unsigned)S.nerows8, 1024, 0, c->stream>>>(
        lsrc, S.erows, c->H, c->DC, c->table, tmask, c->dep, c->hmask, c->zrep, nullptr);
    LAUNCH_CHECK();
  }
  if constexpr (std::is_same<K, u32>::value) {
    if (S.nerows20) {
      k_sig_row<ListSrc, ROW_MAX_NARROW, 1024, u32><<<(unsigned)S.nerows20, 1024, 0, c->stream>>>(
          lsrc, S.erows + S.nerows8, c->H, c->DC, c->table, tmask, c->dep, c->hmask, c->zrep, nullptr);
      LAUNCH_CHECK();
    }
  }
  if (S.nhuge) {
    // edited rows too long for one workgroup: global hash sets in the spare hub-set space
    if ((rc = fill_u64(c, c->hubsets + S.huge_set_begin, S.huge_set_slots, 0))) return rc;
    k_sig_hub_global<ListSrc><<<(unsigned)S.nhuge_chunks, 256, 0, c->stream>>>(
        lsrc, S.huge_chunks, S.huge, c->hubsets + S.huge_set_begin, S.huge_acc, S.huge_cnt, c->dep, nullptr);
    LAUNCH_CHECK();
    k_hub_final<ListSrc><<<blocks_for(S.nhuge, 256), 256, 0, c->stream>>>(lsrc, S.huge, S.nhuge, S.huge_acc,
                                                                          S.huge_cnt, c->H, c->DC, c->table, tmask,
                                                                          c->dep, c->hmask, c->zrep, nullptr);
    LAUNCH_CHECK();
  }
  int nlk = 0;
  if (prop_lists) {
    // touched blocks: the cached blocks of dirty vertices (k_update_flags) and
    // those whose key a dirty vertex now has (k_classify)
    if ((rc = fill_i32(c, (int *)S.filter, FILTER_WORDS, 0))) return rc;
    u32 *gfilter = ndirty >= c->tune.gfilter_min ? S.gfilter : nullptr;
    if (gfilter && (rc = fill_i32(c, (int *)gfilter, GFILTER_WORDS, 0))) return rc;
    if (ndirty > 0) {
      // the dirty vertices were listed by k_update_flags (count at cnt[12])
      k_build_filter<<<blocks_for(ndirty, 256), 256, 0, c->stream>>>(&cnt[12], S.lk, c->H, c->DC, names_prev,
                                                                      S.MVc + at, S.filter, gfilter);
      LAUNCH_CHECK();
    }
    k_classify<<<(unsigned)std::min<int64_t>(CLASSIFY_GRID, blocks_for(n, 256)), 256, 0, c->stream>>>(
        n, S.MVc + at, S.dirty, S.touch, S.FKc + at, S.Hc + at, S.DCc + at, names_prev, S.filter, gfilter, c->table,
        tmask, c->dep, c->zrep, c->H, c->DC, c->rep, S.names[i & 1], &cnt[11], S.lk);
    LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(&nlk, &cnt[11], sizeof nlk, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (2 * (int64_t)nlk > (int64_t)tmask + 1) {
      // more keys than the dirty-sized table holds: a larger one, all listed keys again
      if ((rc = advance(c, ADV_TABLE, s))) return rc;
      c->tmask_steps = tmask = mask_for_keys(c, nlk);
    }
    if (nlk) {
      k_insert_list<<<blocks_for(nlk, 256), 256, 0, c->stream>>>(nlk, S.lk, c->H, c->DC, names_prev, c->table, tmask,
                                                                  c->dep, c->zrep);
      k_lookup<ListSrc><<<blocks_for(nlk, 256), 256, 0, c->stream>>>(
          lsrc, nlk, S.lk, c->H, c->DC, c->table, tmask, c->dep, c->rep, &cnt[0], c->vlist, &cnt[1], c->clA, c->err,
          c->zrep, 1, nullptr, S.dirty, S.MVc + at);
      LAUNCH_CHECK();
    }
  } else {
    k_insert_cached<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, S.dirty, S.Hc + at, S.DCc + at, S.MVc + at,
                                                                names_prev, c->H, c->DC, c->table, tmask, c->dep,
                                                                c->zrep);
    LAUNCH_CHECK();
    k_lookup<ListSrc><<<blocks_for(n, 256), 256, 0, c->stream>>>(lsrc, n, nullptr, c->H, c->DC, c->table, tmask,
                                                                 c->dep, c->rep, &cnt[0], c->vlist, &cnt[1], c->clA,
                                                                 c->err, c->zrep, 1, nullptr, S.dirty, S.MVc + at);
    LAUNCH_CHECK();
  }
  if ((rc = settle_collisions(c, lsrc, s, cnt, true))) return rc;
  HeadIds ids{};
  if ((rc = numbering_words(c, n, count_dev, &ids))) return rc;
  if ((rc = fill_i32(c, reinterpret_cast<int *>(S.claimed), (n + 3) / 4, 0))) return rc;
  if (prop_lists) {
    k_assign_out<<<blocks_for((n + ASSIGN_V - 1) / ASSIGN_V, 256), 256, 0, c->stream>>>(n, c->rep, ids, out);
    LAUNCH_CHECK();
    if (nlk) {
      const unsigned g = blocks_for(nlk, 256);
      k_block_names_fresh<<<g, 256, 0, c->stream>>>(n, c->rep, S.bname, S.keep, nlk, S.lk);
      k_block_names_clean<<<g, 256, 0, c->stream>>>(n, c->rep, S.dirty, S.MVc + at, S.bname, S.claimed, nlk, S.lk);
      k_block_names_keep<<<g, 256, 0, c->stream>>>(n, c->rep, S.dirty, S.MVc + at, S.bname, S.claimed, S.keep, nlk,
                                                   S.lk);
      k_assign_names<<<g, 256, 0, c->stream>>>(n, c->rep, ids, nullptr, S.names[i & 1], nullptr, nullptr, S.bname,
                                               S.keep, S.MVc + at, &cnt[6], S.changed, nlk, S.lk);
      LAUNCH_CHECK();
    }
    *gpid_written = false;
  } else {
    k_block_names_fresh<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->rep, S.bname, S.keep);
    k_block_names_clean<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->rep, S.dirty, S.MVc + at, S.bname,
                                                                    S.claimed);
    k_block_names_keep<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->rep, S.dirty, S.MVc + at, S.bname,
                                                                   S.claimed, S.keep);
    k_assign_names<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->rep, ids, out, S.names[i & 1], c->rank,
                                                              c->gpid[(i + 1) & 1], S.bname, S.keep, S.MVc + at,
                                                              &cnt[6], S.changed);
    LAUNCH_CHECK();
    *gpid_written = true;
  }
  k_mark_in_neighbours<<<MARK_GRID, 256, 0, c->stream>>>(&cnt[6], S.changed, S.tptr, S.tcol, S.flag, &cnt[7],
                                                         S.heavy);
  k_mark_heavy<<<MARK_GRID, 256, 0, c->stream>>>(&cnt[7], S.heavy, S.tptr, S.tcol, S.flag);
  LAUNCH_CHECK();
  return 0;
}

template <bool HK, class K>
int update_steps_t(kbisim_ctx *c, const kbisim_graph *gn, int k, int32_t *const *out) {
  const int n = (int)c->g.n;
  auto &S = c->is;
  const int32_t *lab = separate_labels(c) ? sep_labels(c) : nullptr;
  int rc = 0;
  bool gpid_ok = false;  // gpid[i & 1] holds names_prev in rank order (written when a step needs it)
  for (int i = 0; i < k; ++i) {
    if (i >= 2) {
      // P'_{i-1} refines P'_{i-2}: with as many blocks it is the same
      // partition, and so is every later one (a step depends on the previous
      // partition alone): copies, no more steps
      int64_t pc[2] = {0, 0};
      HIP_TRY(hipMemcpyAsync(pc, &c->dcounts[i - 2], sizeof pc, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      if (pc[0] == pc[1]) {
        for (int j0 = i; j0 < k; j0 += CopyDsts::MAX) {
          CopyDsts d{};
          d.nd = std::min(k - j0, (int)CopyDsts::MAX);
          for (int q = 0; q < d.nd; ++q) d.d[q] = out[j0 + q];
          k_copy_multi<<<std::min<unsigned>(blocks_for(n, 256), 65536), 256, 0, c->stream>>>(d, out[i - 1], n);
          LAUNCH_CHECK();
        }
        for (int j = i; j < k; ++j)
          HIP_TRY(hipMemcpyAsync(&c->dcounts[j], &c->dcounts[i - 1], sizeof(int64_t), hipMemcpyDeviceToDevice,
                                 c->stream));
        return 0;
      }
    }
    const int32_t *names_prev = i == 0 ? c->p0 : S.names[(i - 1) & 1];
    int *cnt = c->counters + CNT_STRIDE * i;
    if ((rc = fill_i32(c, cnt, CNT_STRIDE, 0))) return rc;
    if ((rc = fill_i32(c, reinterpret_cast<int *>(S.touch), (n + 31) / 32, 0))) return rc;
    k_update_flags<<<blocks_for((n + FLAGS_GROUP - 1) / FLAGS_GROUP, 256), 256, 0, c->stream>>>(
        n, S.edited, S.flag, S.dirty, S.skip, gn->row_ptr, cnt + 8, S.psmall, S.plarge, S.MVc + (size_t)i * n, S.touch,
        S.lk);
    LAUNCH_CHECK();
    if ((rc = fill_i32(c, reinterpret_cast<int *>(S.flag), (n + 3) / 4, 0))) return rc;
    // few vertices flagged by the previous step: sign them from lists
    int np[3] = {0, 0, 0};
    HIP_TRY(hipMemcpyAsync(np, cnt + 8, sizeof np, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int64_t nprop = (int64_t)np[0] + np[1] + np[2];
    const bool prop_lists = nprop <= std::max<int64_t>(n / 8, 1);
    if ((!prop_lists || np[2] > 0) && !gpid_ok) {
      // the tier kernels read the previous names in rank order
      k_scatter_rank<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, names_prev, c->rank, c->gpid[i & 1]);
      LAUNCH_CHECK();
    }
    const PlainSrcT<HK> lsrc{gn->row_ptr, gn->col, gn->elabel, names_prev, c->pb, c->kmask};
    const int64_t ndirty = nprop + S.nrows;
    if (lab)
      rc = update_step<K>(c, GraphSrcT<true, HK>{c->g.row_ptr, c->gcol, lab, c->gpid[i & 1], names_prev, c->pb,
                                                 c->rbits, c->kmask},
                          lsrc, i, names_prev, out[i], &c->dcounts[i], cnt, prop_lists, np[2], ndirty, &gpid_ok);
    else
      rc = update_step<K>(c, GraphSrcT<false, HK>{c->g.row_ptr, c->gcol, nullptr, c->gpid[i & 1], names_prev, c->pb,
                                                  c->rbits, c->kmask},
                          lsrc, i, names_prev, out[i], &c->dcounts[i], cnt, prop_lists, np[2], ndirty, &gpid_ok);
    if (rc) return rc;
  }
  return 0;
}

int update_impl(kbisim_ctx *c, const kbisim_graph *gn, const int32_t *rows, int64_t nrows, int k,
                int32_t *const *out, int64_t *counts) {
  if (!c || !gn || !c->incr || c->num_graphs > 0) return KBISIM_EINVAL;
  if (k < 0 || k > c->incr_k) return KBISIM_EINVAL;
  if (k == 0) return KBISIM_OK;
  if (!out || !counts) return KBISIM_EINVAL;
  const int64_t n = c->g.n;
  if (gn->n != n || gn->m < 0 || (gn->elabel == nullptr) != (c->g.elabel == nullptr)) return KBISIM_EINVAL;
  if (gn->m >= (int64_t(1) << 62)) return KBISIM_ERANGE;
  if (nrows < 0 || nrows > n || (nrows > 0 && !rows)) return KBISIM_EINVAL;
  if (n == 0) {
    for (int i = 0; i < k; ++i) counts[i] = 0;
    return KBISIM_OK;
  }
  for (int i = 0; i < k; ++i)
    if (!out[i]) return KBISIM_EINVAL;
  if (!gn->row_ptr || (gn->m > 0 && !gn->col)) return KBISIM_EINVAL;
  auto &S = c->is;
  int rc = 0;
  // the edited graph: row offsets, every target and label (any row is read by
  // the exact checks), the listed vertices
  if ((rc = fill_i32(c, (int *)c->err, 1, 0))) return rc;
  k_validate_rows<<<blocks_for(n + 1, 256), 256, 0, c->stream>>>(n, gn->m, gn->row_ptr, c->err, ERR_GRAPH_ROWPTR);
  if (gn->m > 0) {
    validate_vals(c->stream, gn->m, gn->col, n, c->err, ERR_GRAPH_COL);
    if (gn->elabel)
      validate_vals(c->stream, gn->m, gn->elabel, (int64_t)c->max_label + 1, c->err, ERR_GRAPH_ELABEL);
  }
  if (nrows) validate_vals(c->stream, nrows, rows, n, c->err, ERR_BAD_PID);
  LAUNCH_CHECK();
  u32 err = 0;
  if ((rc = read_err(c, &err))) return rc;
  if (err & ERR_BAD_PID) return KBISIM_EINVAL;
  if (err) return KBISIM_EGRAPH;
  // flags and the edited rows, split by length
  if ((rc = fill_i32(c, reinterpret_cast<int *>(S.edited), (n + 3) / 4, 0))) return rc;
  if ((rc = fill_i32(c, reinterpret_cast<int *>(S.flag), (n + 3) / 4, 0))) return rc;
  if ((rc = fill_i32(c, S.cnt, 16, 0))) return rc;
  if ((rc = fill_i32(c, S.cnt + 2, 1, (int)nrows))) return rc;
  S.nhuge = 0;
  S.nhuge_chunks = 0;
  S.nerows8 = S.nerows20 = 0;
  S.nrows = nrows;
  if (nrows) {
    k_set_flags<<<std::min<unsigned>(blocks_for(nrows, 256), 65536), 256, 0, c->stream>>>(S.cnt + 2, rows, S.edited);
    // edited rows longer than LIST_BIG: a row-kernel workgroup each up to
    // what one workgroup's LDS holds, longer ones global sets when the spare
    // hub-set space holds them (else they stay with the multi-pass list kernel)
    const int64_t free_begin = c->sched.gset_end;
    const int64_t free_end = c->glab ? (int64_t)(reinterpret_cast<const u64 *>(c->glab) - c->hubsets)
                                     : c->plan.hubset_slots;
    const int64_t row_cap = c->narrow ? ROW_MAX_NARROW : ROW_MAX;
    k_split_list<<<blocks_for(nrows, 256), 256, 0, c->stream>>>((int)nrows, rows, gn->row_ptr, &S.cnt[0], S.small,
                                                                  &S.cnt[1], S.large, (int64_t)LIST_BIG, &S.cnt[3],
                                                                  S.huge);
    LAUNCH_CHECK();
    {
      int nh = 0;
      HIP_TRY(hipMemcpyAsync(&nh, &S.cnt[3], sizeof nh, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      if (nh > 0) {
        std::vector<int> hv((size_t)nh);
        std::vector<int64_t> be(2 * (size_t)nh);
        // extents staged in the chunk buffer (rewritten below)
        int64_t *be_dev = reinterpret_cast<int64_t *>(S.huge_chunks);
        k_row_extents<<<blocks_for(nh, 256), 256, 0, c->stream>>>(nh, S.huge, gn->row_ptr, be_dev);
        LAUNCH_CHECK();
        HIP_TRY(hipMemcpyAsync(hv.data(), S.huge, 4 * (size_t)nh, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipMemcpyAsync(be.data(), be_dev, 16 * (size_t)nh, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        std::vector<HubGChunk> ch;
        std::vector<int> keep_list;
        std::vector<Range> r8, r20;
        int64_t at = free_begin;
        int nglob = 0;
        for (int i = 0; i < nh; ++i) {
          const int v = hv[(size_t)i];
          const int64_t b = be[2 * (size_t)i], d = be[2 * (size_t)i + 1] - b;
          if (d <= row_cap) {
            (d <= ROW_MAX ? r8 : r20).push_back(Range{v, v + 1, (int)d, 0, b});
            continue;
          }
          if (at + 2 * d > free_end || (int64_t)ch.size() + d / HUB_GCHUNK + 1 > S.huge_chunk_cap) {
            keep_list.push_back(v);  // no room: back to the list kernel
            continue;
          }
          for (int64_t x = 0; x < d; x += HUB_GCHUNK)
            ch.push_back(HubGChunk{nglob, 0, x, std::min<int64_t>(d, x + HUB_GCHUNK), at - free_begin, 2 * d});
          hv[(size_t)nglob++] = v;
          at += 2 * d;
        }
        S.nerows8 = (int)r8.size();
        S.nerows20 = (int)r20.size();
        r8.insert(r8.end(), r20.begin(), r20.end());
        if (!r8.empty())
          HIP_TRY(hipMemcpyAsync(S.erows, r8.data(), sizeof(Range) * r8.size(), hipMemcpyHostToDevice, c->stream));
        S.nhuge = nglob;
        S.nhuge_chunks = (int)ch.size();
        S.huge_set_begin = free_begin;
        S.huge_set_slots = at - free_begin;
        if (S.nhuge) {
          HIP_TRY(hipMemcpyAsync(S.huge, hv.data(), 4 * (size_t)S.nhuge, hipMemcpyHostToDevice, c->stream));
          HIP_TRY(hipMemcpyAsync(S.huge_chunks, ch.data(), sizeof(HubGChunk) * ch.size(), hipMemcpyHostToDevice,
                                 c->stream));
        }
        if (!keep_list.empty()) {  // append to the large list (its count is on the device)
          int nl = 0;
          HIP_TRY(hipMemcpyAsync(&nl, &S.cnt[1], sizeof nl, hipMemcpyDeviceToHost, c->stream));
          HIP_TRY(hipStreamSynchronize(c->stream));
          HIP_TRY(hipMemcpyAsync(S.large + nl, keep_list.data(), 4 * keep_list.size(), hipMemcpyHostToDevice,
                                 c->stream));
          if ((rc = fill_i32(c, &S.cnt[1], 1, nl + (int)keep_list.size()))) return rc;
        }
        HIP_TRY(hipStreamSynchronize(c->stream));
      }
    }
  }
  // every vertex may carry a key in an update (edited rows can gain entries),
  // and empty signatures are grouped by block names below 2n
  const u64 tmask_saved = c->tmask_steps;
  u64 *zrep_saved = c->zrep;
  c->tmask_steps = c->plan.tslots - 1;
  c->zrep = S.zrep;
  if (c->hashed) rc = update_steps_t<true, u32>(c, gn, k, out);
  else if (c->narrow) rc = update_steps_t<false, u32>(c, gn, k, out);
  else rc = update_steps_t<false, u64>(c, gn, k, out);
  c->tmask_steps = tmask_saved;
  c->zrep = zrep_saved;
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(&err, c->err, sizeof err, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(counts, c->dcounts, 8 * (size_t)k, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  prof_collect(c);
  if (err) return KBISIM_EINTERNAL;
  return KBISIM_OK;
}

int incr_enable_impl(kbisim_ctx *c, void *state, size_t bytes) {
  if (!c || c->num_graphs > 0 || c->work_eff || c->kmax < 1 || !state) return KBISIM_EINVAL;
  const int64_t n = c->g.n, m = c->g.m;
  if (n >= (int64_t(1) << 30)) return KBISIM_ERANGE;  // update block names reach 2n
  const IncrPlan p = incr_plan(n, m, c->kmax);
  if (bytes < p.total) return KBISIM_ENOSPACE;
  char *w = (char *)state;
  auto &S = c->is;
  S.Hc = (u64 *)(w + p.off_hc);
  S.DCc = (u32 *)(w + p.off_dcc);
  S.MVc = (int32_t *)(w + p.off_mvc);
  S.FKc = (uint16_t *)(w + p.off_fk);
  S.tptr = (int64_t *)(w + p.off_tptr);
  S.tcol = (int32_t *)(w + p.off_tcol);
  S.names[0] = (int32_t *)(w + p.off_names);
  S.names[1] = S.names[0] + std::max<int64_t>(n, 1);
  S.edited = (unsigned char *)(w + p.off_edited);
  S.flag = (unsigned char *)(w + p.off_flag);
  S.dirty = (unsigned char *)(w + p.off_dirty);
  S.skip = (unsigned char *)(w + p.off_skip);
  S.small = (int *)(w + p.off_small);
  S.large = (int *)(w + p.off_large);
  S.psmall = (int *)(w + p.off_psmall);
  S.plarge = (int *)(w + p.off_plarge);
  S.changed = (int *)(w + p.off_changed);
  S.bname = (int32_t *)(w + p.off_bname);
  S.keep = (int32_t *)(w + p.off_keep);
  S.claimed = (unsigned char *)(w + p.off_claimed);
  S.heavy = (int *)(w + p.off_heavy);
  S.touch = (u32 *)(w + p.off_touch);
  S.lk = (int *)(w + p.off_lk);
  S.filter = (u32 *)(w + p.off_filter);
  S.gfilter = (u32 *)(w + p.off_gfilter);
  S.huge = (int *)(w + p.off_huge);
  S.huge_chunks = (HubGChunk *)(w + p.off_hchunks);
  S.huge_acc = (u64 *)(w + p.off_hacc);
  S.huge_cnt = (u32 *)(w + p.off_hcnt);
  S.erows = (Range *)(w + p.off_erows);
  S.huge_cap = p.huge_cap;
  S.huge_chunk_cap = p.huge_chunk_cap;
  S.zrep = (u64 *)(w + p.off_zrep);
  S.cnt = (int *)(w + p.off_cnt);
  int rc0 = 0;
  if (n > 0) {
    // in-rows of the cached graph: count per target, offsets, scatter
    int *cnt = S.names[0];
    auto *cursor = reinterpret_cast<unsigned long long *>(S.Hc);
    auto *tiles = reinterpret_cast<int64_t *>(S.small);
    const int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    int rc = fill_i32(c, cnt, n, 0);
    if (rc) return rc;
    if (m > 0)
      k_indegree<<<(unsigned)std::min<int64_t>(blocks_for(m, INDEG_CHUNK), 65536), 256, 0, c->stream>>>(m, c->g.col,
                                                                                                       cnt);
    k_sum_tiles64<<<(unsigned)nt, 256, 0, c->stream>>>(n, cnt, tiles);
    k_scan_tiles64<<<1, 256, 0, c->stream>>>(nt, tiles);
    k_write_ptr64<<<(unsigned)nt, 256, 0, c->stream>>>(n, cnt, tiles, S.tptr, cursor);
    if (m > 0)
      k_transpose_scatter<<<(unsigned)std::min<int64_t>(blocks_for(n * WAVE, 256), 65536), 256, 0, c->stream>>>(
          n, c->g.row_ptr, c->g.col, nullptr, cursor, S.tcol, nullptr);
    LAUNCH_CHECK();
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  if ((rc0 = fill_u64(c, S.zrep, 2 * std::max<int64_t>(n, 1), ~0ULL))) return rc0;
  if ((rc0 = fill_u64(c, S.huge_acc, S.huge_cap, 0))) return rc0;
  if ((rc0 = fill_i32(c, (int *)S.huge_cnt, S.huge_cap, 0))) return rc0;
  // Update steps name blocks below 2n, so pairs keep one more bit of block
  // name; a pair's value (label << 31 | name) does not depend on that width,
  // only whether exact 32-bit keys still fit does.
  {
    u32 pb = 1, lb = 0;
    while (pb < 31 && (int64_t(1) << pb) < 2 * n) ++pb;
    while (lb < 32 && (c->max_label >> lb) != 0) ++lb;
    c->pb = pb;
    c->hashed = c->narrow && (c->tune.key_bits == 32 || pb + lb > 31);
  }
  // loops captured before did not cache their steps
  for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->incr = true;
  c->incr_k = 0;
  return KBISIM_OK;
}

int check_sizes(const kbisim_graph *g) {
  if (!g) return KBISIM_EINVAL;
  if (g->n < 0 || g->m < 0 || g->nlabels < 0) return KBISIM_EINVAL;
  if (g->n >= (int64_t(1) << 31) || g->m >= (int64_t(1) << 62) || g->nlabels >= (int64_t(1) << 62))
    return KBISIM_ERANGE;
  return 0;
}

int read_tuning(const kbisim_tuning *t, Tuning &out) {
  out = Tuning{};
  if (!t) return 0;
  if (t->range_edges) {
    if (t->range_edges != 1024 && t->range_edges != 2048) return KBISIM_EINVAL;
    out.range_edges = t->range_edges;
  }
  if (t->hub_chunk) {
    if (t->hub_chunk != 2048 && t->hub_chunk != 4096) return KBISIM_EINVAL;
    out.hub_chunk = t->hub_chunk;
  }
  if (t->hub_part_target) {
    if (t->hub_part_target != 1024 && t->hub_part_target != 2048) return KBISIM_EINVAL;
    out.hub_part_target = t->hub_part_target;
  }
  if (t->key_bits) {
    if (t->key_bits != 32 && t->key_bits != 64) return KBISIM_EINVAL;
    out.key_bits = t->key_bits;
  }
  if (t->scan_items) {
    if (t->scan_items != 8 && t->scan_items != 16) return KBISIM_EINVAL;
    out.scan_items = t->scan_items;
  }
  return 0;
}

// Shared by kbisim_create and kbisim_batch_create.  With vert_off (host,
// num_graphs + 1) the graph is a batch of disjoint graphs.
int create_impl(const kbisim_graph *g, int kmax, const kbisim_tuning *tuning, void *workspace, size_t ws_bytes,
                void *stream, int64_t num_graphs, const int64_t *vert_off, kbisim_ctx **out,
                bool pinned_ok = true) {
  int rc = check_sizes(g);
  if (rc) return rc;
  if (!out || kmax < 0 || kmax > (1 << 20)) return KBISIM_EINVAL;
  *out = nullptr;
  Tuning tune;
  if ((rc = read_tuning(tuning, tune))) return rc;
  const int64_t n = g->n, m = g->m;
  if (n > 0 && !g->row_ptr) return KBISIM_EINVAL;
  if (m > 0 && !g->col) return KBISIM_EINVAL;
  if (g->vlabel_ptr && !g->vlabel && g->nlabels > 0) return KBISIM_EINVAL;
  if (!g->vlabel_ptr && !g->vlabel && g->nlabels > 0) return KBISIM_EINVAL;
  if (num_graphs > 0) {
    if (!vert_off || vert_off[0] != 0 || vert_off[num_graphs] != n) return KBISIM_EINVAL;
    for (int64_t i = 0; i < num_graphs; ++i)
      if (vert_off[i + 1] < vert_off[i]) return KBISIM_EINVAL;
  }
  const int64_t nl = g->vlabel_ptr ? g->nlabels : 0;
  Plan plan = make_plan(n, m, nl, kmax, num_graphs);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (ALIGN - 1))) return KBISIM_EINVAL;
  if (ws_bytes < plan.total) return KBISIM_ENOSPACE;

  kbisim_ctx *c = new (std::nothrow) kbisim_ctx();
  if (!c) return KBISIM_EINTERNAL;
  c->g = *g;
  c->kmax = kmax;
  c->pinned_ok = pinned_ok;
  c->stream = (hipStream_t)stream;
  c->plan = plan;
  c->tune = tune;
  c->ws = (char *)workspace;
  char *w = c->ws;
  c->H = (u64 *)(w + plan.off_H);
  c->DC = (u32 *)(w + plan.off_DC);
  c->rep = (int *)(w + plan.off_rep);
  c->p0 = (int *)(w + plan.off_p0);
  c->vlist = (int *)(w + plan.off_vlist);
  c->clA = (int *)(w + plan.off_clA);
  c->clB = (int *)(w + plan.off_clB);
  c->ranges = (Range *)(w + plan.off_ranges);
  c->lists = (int *)(w + plan.off_lists);
  c->table = (u64 *)(w + plan.off_table);
  c->ctable = (u64 *)(w + plan.off_ctable);
  c->hacc = (u64 *)(w + plan.off_hacc);
  c->hcnt = (u32 *)(w + plan.off_hcnt);
  c->chunks = (HubChunk *)(w + plan.off_chunks);
  c->parts = (HubPart *)(w + plan.off_parts);
  c->gchunks = (HubGChunk *)(w + plan.off_gchunks);
  c->poff = (int *)(w + plan.off_poff);
  c->tiles = (u32 *)(w + plan.off_status);
  c->hw = (HeadWord *)(w + plan.off_hw);
  c->gcol = (int *)(w + plan.off_gcol);
  c->rank = (int *)(w + plan.off_rank);
  c->gpid[0] = (int *)(w + plan.off_gpid);
  c->gpid[1] = c->gpid[0] + std::max<int64_t>(n, 1);
  c->zrep = (u64 *)(w + plan.off_zrep);
  c->counters = (int *)(w + plan.off_counters);
  c->dcounts = (int64_t *)(w + plan.off_dcounts);
  c->err = (u32 *)(w + plan.off_err);
  c->dep = (u32 *)(w + plan.off_dep);
  c->hubsets = (u64 *)(w + plan.off_hubsets);
  c->single[0] = (unsigned char *)(w + plan.off_single);
  c->single[1] = c->single[0] + std::max<int64_t>(n, 1);
  c->multi = (u32 *)(w + plan.off_multi);
  c->nzv = (int *)(w + plan.off_nzv);
  if (num_graphs > 0) {
    c->num_graphs = num_graphs;
    c->gid = (int *)(w + plan.off_gid);
    c->ibuf[0] = (int *)(w + plan.off_ibuf);
    c->ibuf[1] = c->ibuf[0] + std::max<int64_t>(n, 1);
    c->first = (int64_t *)(w + plan.off_first);
    c->next = (int64_t *)(w + plan.off_next);
    c->bcounts = (int64_t *)(w + plan.off_bcounts);
  }
  const char *dbg = getenv("KBISIM_DEBUG_HASH_BITS");
  if (dbg && *dbg) {
    int b = atoi(dbg);
    if (b >= 0 && b < 64) c->hmask = b == 0 ? 0ULL : ((1ULL << b) - 1ULL);
  }
  // Test knob: at most this many partitions per staged hub, so that hub
  // partitions overflow their sets and take the sub-pass path.
  const char *pdbg = getenv("KBISIM_DEBUG_HUB_PARTS");
  if (pdbg && *pdbg) {
    int q = atoi(pdbg);
    if (q >= 1 && q <= HUB_PMAX && (q & (q - 1)) == 0) c->tune.hub_parts_cap = q;
  }
  // Test knob: build the degree schedule on the device for small graphs too.
  const char *sdbg = getenv("KBISIM_DEBUG_DEVICE_SCHEDULE");
  if (sdbg && *sdbg == '1') c->tune.device_schedule = true;
  // Test knob: keep only this many bits of hashed set keys, so that keys
  // collide inside rows (the exact check must still separate the pair sets).
  const char *kdbg = getenv("KBISIM_DEBUG_KEY_BITS");
  if (kdbg && *kdbg) {
    int b = atoi(kdbg);
    if (b >= 1 && b < 32) c->kmask = (1u << b) - 1u;
  }
  // Test knob: update steps use the global dirty-key filter from this many
  // dirty vertices on (at least 1), so that small graphs take that path.
  const char *gdbg = getenv("KBISIM_DEBUG_GFILTER_MIN");
  if (gdbg && *gdbg) {
    int q = atoi(gdbg);
    if (q >= 1) c->tune.gfilter_min = q;
  }

  auto fail = [&](int code) {
    delete c;
    return code;
  };
  // Validation (Def. multi-relational-labeled-property-graph as a CSR contract).
  if ((rc = fill_i32(c, (int *)c->err, 4, 0))) return fail(rc);
  if ((rc = fill_i32(c, (int *)c->dep, 16, 0))) return fail(rc);
  if (n == 0 && m > 0) return fail(KBISIM_EGRAPH);
  if (n > 0) {
    k_validate_rows<<<blocks_for(n + 1, 256), 256, 0, c->stream>>>(n, m, g->row_ptr, c->err, ERR_GRAPH_ROWPTR);
    if (hipGetLastError() != hipSuccess) return fail(KBISIM_EHIP);
  }
  if (m > 0) {
    validate_vals(c->stream, m, g->col, n, c->err, ERR_GRAPH_COL);
    if (g->elabel) validate_vals(c->stream, m, g->elabel, -1, c->err, ERR_GRAPH_ELABEL);
  }
  if (g->vlabel_ptr) {
    k_validate_rows<<<blocks_for(n + 1, 256), 256, 0, c->stream>>>(n, nl, g->vlabel_ptr, c->err, ERR_GRAPH_VPTR);
    if (nl > 0) validate_vals(c->stream, nl, g->vlabel, -1, c->err, ERR_GRAPH_VLABEL);
  } else if (g->vlabel && n > 0) {
    validate_vals(c->stream, n, g->vlabel, -1, c->err, ERR_GRAPH_VLABEL);
  }
  if (hipGetLastError() != hipSuccess) return fail(KBISIM_EHIP);
  u32 err = 0;
  if ((rc = read_err(c, &err))) return fail(rc);
  if (err) return fail(KBISIM_EGRAPH);

  // Pairs keep block ids modulo 2^pb, pb = bit width of the largest graph's
  // vertex count (the block ids of one graph form an interval no longer than
  // that).  Keys inside LDS sets are (edge label << pb) | reduced block, in
  // 31 bits, when the labels allow.
  {
    int64_t gmax = n;
    if (num_graphs > 0) {
      gmax = 0;
      for (int64_t i = 0; i < num_graphs; ++i) gmax = std::max<int64_t>(gmax, vert_off[i + 1] - vert_off[i]);
    }
    u32 max_label = 0;
    if (g->elabel && m > 0) {
      k_max_i32<<<(unsigned)std::min<int64_t>(blocks_for(m, 256), 4096), 256, 0, c->stream>>>(m, g->elabel, c->err + 2);
      if (hipGetLastError() != hipSuccess) return fail(KBISIM_EHIP);
      if (hipMemcpyAsync(&max_label, c->err + 2, sizeof(u32), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
          hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(KBISIM_EHIP);
    }
    u32 pb = 1, lb = 0;
    while (pb < 31 && (int64_t(1) << pb) < gmax) ++pb;
    while (lb < 32 && (max_label >> lb) != 0) ++lb;
    c->pb = pb;
    c->max_label = max_label;
    // pack (label, rank) into one 32-bit gather index when both fit
    u32 rb = 1;
    while (rb < 31 && (int64_t(1) << rb) < n) ++rb;
    if (g->elabel && rb + lb <= 32) {
      c->packed = true;
      c->rbits = rb;
    }
    // 32-bit set keys unless 64-bit ones are asked for: exact when the label
    // and reduced block fit 31 bits together, else a hash of the pair
    // (key_bits = 32 asks for hashed keys in any case)
    c->narrow = c->tune.key_bits != 64;
    c->hashed = c->narrow && (c->tune.key_bits == 32 || pb + lb > 31);
  }

  if (num_graphs > 0) {
    // graph of every vertex; first vertex of the next non-empty graph
    std::vector<int64_t> nxt((size_t)num_graphs, -1);
    int64_t after = -1;
    for (int64_t i = num_graphs - 1; i >= 0; --i) {
      nxt[(size_t)i] = after;
      if (vert_off[i + 1] > vert_off[i]) after = vert_off[i];
    }
    if (hipMemcpyAsync(c->first, vert_off, 8 * (size_t)(num_graphs + 1), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(c->next, nxt.data(), 8 * (size_t)num_graphs, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return fail(KBISIM_EHIP);
    k_graph_ids<<<(unsigned)num_graphs, 256, 0, c->stream>>>((int)num_graphs, c->first, c->gid);
    if (hipGetLastError() != hipSuccess) return fail(KBISIM_EHIP);
    if (n > 0) {
      k_validate_batch<<<blocks_for(n, 256), 256, 0, c->stream>>>((int)n, g->row_ptr, g->col, c->gid, c->err);
      if (hipGetLastError() != hipSuccess) return fail(KBISIM_EHIP);
    }
    if ((rc = read_err(c, &err))) return fail(rc);
    if (err) return fail(KBISIM_EGRAPH);
  }

  // Gather renumbering: rank vertices by decreasing in-degree (ties by id).
  // Uses the grouping tables as scratch, before they are cleared below.
  if ((rc = build_rank(c))) return fail(rc);
  // Fresh state: tables start empty; empty-signature slots start above any entry.
  if ((rc = fill_u64(c, c->table, (int64_t)plan.tslots, 0))) return fail(rc);
  if ((rc = fill_u64(c, c->ctable, (int64_t)plan.tslots, 0))) return fail(rc);
  if ((rc = fill_u64(c, c->zrep, std::max<int64_t>(n, 1), ~0ULL))) return fail(rc);
  if ((rc = fill_i32(c, (int *)c->multi, std::max<int64_t>(n, 1), 0))) return fail(rc);

  // P0: blocks of equal vertex label sets, numbered by first vertex; in a
  // batch the graph id joins the key, so no block spans two graphs.
  if (!g->vlabel && num_graphs == 0) {
    if ((rc = fill_i32(c, c->p0, n, 0))) return fail(rc);
    c->p0_count = n > 0 ? 1 : 0;
  } else if (n > 0) {
    Schedule ls;
    LabelSrc src{g->vlabel_ptr, g->vlabel, c->gid};
    if (!g->vlabel) src = LabelSrc{nullptr, c->gid, nullptr};  // batch without labels: one block per graph
    if ((rc = build_schedule(c, src.ptr, ls, range_cap(c, true), ROW_MAX, HUB_STAGED_MAX_WIDE))) return fail(rc);
    int *cnt = c->counters + CNT_STRIDE * (plan.ncounter_steps - 2);
    if ((rc = fill_i32(c, cnt, CNT_STRIDE, 0))) return fail(rc);
    int64_t *dcount = c->dcounts + (plan.ncounter_steps - 2);
    if ((rc = run_step(c, src, ls, c->p0, dcount, cnt, true, nullptr, true))) return fail(rc);
    if (hipMemcpyAsync(&c->p0_count, dcount, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return fail(KBISIM_EHIP);
    if ((rc = read_err(c, &err))) return fail(rc);
    if (err) return fail(KBISIM_EINTERNAL);
  }
  // Static schedule of the graph rows.
  if ((rc = build_schedule(c, g->row_ptr, c->sched, range_cap(c, !c->narrow),
                           c->narrow ? ROW_MAX_NARROW : ROW_MAX, c->narrow ? HUB_STAGED_MAX : HUB_STAGED_MAX_WIDE)))
    return fail(rc);
  if ((rc = build_nonempty_list(c, c->sched))) return fail(rc);
  if ((rc = sort_long_rows(c, c->sched))) return fail(rc);
  // a load of at most 1/4 (within the planned table): shorter probe runs measured
  // faster than a smaller, more cache-resident span
  c->tmask_steps = std::min<u64>(pow2_at_least(4 * (uint64_t)std::max<int64_t>(c->sched.nonempty, 1)), plan.tslots) - 1;
  *out = c;
  return KBISIM_OK;
}

}  // namespace

extern "C" {

int kbisim_workspace_bytes(const kbisim_graph *g, int kmax, size_t *bytes) {
  int rc = check_sizes(g);
  if (rc) return rc;
  if (!bytes || kmax < 0 || kmax > (1 << 20)) return KBISIM_EINVAL;
  *bytes = make_plan(g->n, g->m, g->vlabel_ptr ? g->nlabels : 0, kmax, 0).total;
  return KBISIM_OK;
}

int kbisim_create(const kbisim_graph *g, int kmax, void *workspace, size_t ws_bytes, void *stream, kbisim_ctx **out) {
  return create_impl(g, kmax, nullptr, workspace, ws_bytes, stream, 0, nullptr, out);
}

int kbisim_create_tuned(const kbisim_graph *g, int kmax, const kbisim_tuning *tuning, void *workspace,
                        size_t ws_bytes, void *stream, kbisim_ctx **out) {
  return create_impl(g, kmax, tuning, workspace, ws_bytes, stream, 0, nullptr, out);
}

int kbisim_initial(kbisim_ctx *c, int32_t *out_ids, int64_t *out_count) {
  if (!c || !out_count || (c->g.n > 0 && !out_ids)) return KBISIM_EINVAL;
  if (c->g.n > 0) {
    k_copy_i32<<<std::min<unsigned>(blocks_for(c->g.n, 256), 65536), 256, 0, c->stream>>>(out_ids, c->p0, c->g.n);
    LAUNCH_CHECK();
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  *out_count = c->p0_count;
  return KBISIM_OK;
}

int kbisim_refine(kbisim_ctx *c, int k, int32_t *const *out_block_ids, int64_t *out_counts) {
  if (c && c->num_graphs > 0) return KBISIM_EINVAL;
  return refine_impl(c, nullptr, k, out_block_ids, out_counts);
}

int kbisim_refine_from(kbisim_ctx *c, const int32_t *pid_i, int k, int32_t *const *out_block_ids,
                       int64_t *out_counts) {
  if (!c || c->num_graphs > 0 || (c->g.n > 0 && !pid_i)) return KBISIM_EINVAL;
  if (c->g.n > 0) {
    int rc0 = fill_i32(c, (int *)c->err, 1, 0);
    if (rc0) return rc0;
    validate_vals(c->stream, c->g.n, pid_i, c->g.n, c->err, ERR_BAD_PID);
    LAUNCH_CHECK();
    u32 err = 0;
    int rc = read_err(c, &err);
    if (rc) return rc;
    if (err) return KBISIM_EINVAL;
  }
  return refine_impl(c, pid_i, k, out_block_ids, out_counts);
}

// Single steps.  Step i reads P_i (prev, P0 for i = 0; a batch keeps its own
// global-id copy) and writes P_{i+1} into out; the rank-ordered copy of the
// partition left by step i-1 is reused, so steps of one context go in order.
int step_async_impl(kbisim_ctx *c, int i, const int32_t *prev, int32_t *out) {
  if (!c || i < 0 || i >= c->kmax) return KBISIM_EINVAL;
  const bool batch = c->num_graphs > 0;
  if (c->g.n == 0) return KBISIM_OK;
  if (!out || (!batch && i > 0 && !prev) || (const int32_t *)out == prev) return KBISIM_EINVAL;
  const int32_t *p = i == 0 ? c->p0 : (batch ? c->ibuf[(i - 1) & 1] : prev);
  int rc = 0;
  if (c->incr) c->incr_k = 0;  // single steps do not keep a chain for updates
  if (i == 0 && (rc = fill_i32(c, (int *)c->err, 1, 0))) return rc;
  if ((rc = fill_i32(c, c->counters + CNT_STRIDE * i, CNT_STRIDE, 0))) return rc;
  std::vector<int32_t *> o((size_t)i + 1, out);  // indexed by step number
  return enqueue_steps(c, p, i, i + 1, o.data(), false, c->kmax, i == 0);
}

int step_result_impl(kbisim_ctx *c, int i, const int32_t *prev, int32_t *out) {
  if (!c || i < 0 || i >= c->kmax) return KBISIM_EINVAL;
  const bool batch = c->num_graphs > 0;
  if (c->g.n == 0) return KBISIM_OK;
  if (!out || (!batch && i > 0 && !prev)) return KBISIM_EINVAL;
  const int32_t *p = i == 0 ? c->p0 : (batch ? c->ibuf[(i - 1) & 1] : prev);
  int left = 0;
  u32 err = 0;
  HIP_TRY(hipMemcpyAsync(&left, c->counters + CNT_STRIDE * i + 2, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&err, c->err, sizeof err, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  prof_collect(c);
  if (err) return KBISIM_EINTERNAL;
  if (left) {
    std::vector<int32_t *> o((size_t)i + 1, out);
    int rc = enqueue_steps(c, p, i, i + 1, o.data(), true, c->kmax, true);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(&err, c->err, sizeof err, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    prof_collect(c);
    if (err) return KBISIM_EINTERNAL;
  }
  return KBISIM_OK;
}

int kbisim_step_async(kbisim_ctx *c, int i, const int32_t *prev, int32_t *out) {
  if (!c || c->num_graphs > 0) return KBISIM_EINVAL;
  return step_async_impl(c, i, prev, out);
}

int kbisim_step_result(kbisim_ctx *c, int i, const int32_t *prev, int32_t *out, int64_t *count) {
  if (!c || c->num_graphs > 0 || !count) return KBISIM_EINVAL;
  int rc = step_result_impl(c, i, prev, out);
  if (rc) return rc;
  if (c->g.n == 0) {
    *count = 0;
    return KBISIM_OK;
  }
  HIP_TRY(hipMemcpyAsync(count, &c->dcounts[i], 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return KBISIM_OK;
}

int kbisim_work_efficient(kbisim_ctx *c, int enable, int *last_steps) {
  if (!c) return KBISIM_EINVAL;
  if (enable > 0 && c->incr) return KBISIM_EINVAL;  // updates need every step of the chain cached
  if (last_steps) *last_steps = c->we_steps;
  if (enable >= 0) c->work_eff = enable != 0;
  return KBISIM_OK;
}

int kbisim_use_graphs(kbisim_ctx *c, int enable) {
  if (!c) return KBISIM_EINVAL;
  if (enable && c->stream == nullptr) return KBISIM_EINVAL;  // the null stream cannot be captured
  c->use_graphs = enable != 0;
  return KBISIM_OK;
}

int kbisim_set_stream(kbisim_ctx *c, void *stream) {
  if (!c) return KBISIM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (c->use_graphs && s == nullptr) return KBISIM_EINVAL;
  if (s == c->stream) return KBISIM_OK;
  hipEvent_t e = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipError_t r = hipEventRecord(e, c->stream);
  if (r == hipSuccess) r = hipStreamWaitEvent(s, e, 0);
  (void)hipEventDestroy(e);
  if (r != hipSuccess) return hip_fail(r);
  c->stream = s;
  return KBISIM_OK;
}

int kbisim_incr_state_bytes(const kbisim_graph *g, int kmax, size_t *bytes) {
  int rc = check_sizes(g);
  if (rc) return rc;
  if (!bytes || kmax < 1 || kmax > (1 << 20)) return KBISIM_EINVAL;
  *bytes = incr_plan(g->n, g->m, kmax).total;
  return KBISIM_OK;
}

int kbisim_incr_enable(kbisim_ctx *c, void *state, size_t bytes) { return incr_enable_impl(c, state, bytes); }

int kbisim_incr_update(kbisim_ctx *c, const kbisim_graph *g_new, const int32_t *rows, int64_t nrows, int k,
                       int32_t *const *out_block_ids, int64_t *out_counts) {
  return update_impl(c, g_new, rows, nrows, k, out_block_ids, out_counts);
}

int kbisim_destroy(kbisim_ctx *c) {
  if (c) {
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  }
  delete c;
  return KBISIM_OK;
}

int kbisim_profile_enable(kbisim_ctx *c, int enable) {
  if (!c) return KBISIM_EINVAL;
  HIP_TRY(hipStreamSynchronize(c->stream));
  prof_collect(c);
  c->prof = enable != 0;
  for (int i = 0; i < KBISIM_NKERNELS; ++i) {
    c->prof_ms[i] = 0.0;
    c->prof_n[i] = 0;
  }
  return KBISIM_OK;
}

int kbisim_profile_select(kbisim_ctx *c, uint32_t kinds) {
  if (!c) return KBISIM_EINVAL;
  c->prof_mask = kinds;
  return KBISIM_OK;
}

int kbisim_profile_read(kbisim_ctx *c, double *ms, int64_t *launches) {
  if (!c) return KBISIM_EINVAL;
  HIP_TRY(hipStreamSynchronize(c->stream));
  prof_collect(c);
  for (int i = 0; i < KBISIM_NKERNELS; ++i) {
    if (ms) ms[i] = c->prof_ms[i];
    if (launches) launches[i] = c->prof_n[i];
  }
  return KBISIM_OK;
}

const char *kbisim_kernel_name(int kind) {
  static const char *names[KBISIM_NKERNELS] = {"k_sig_range", "k_sig_row", "k_hub_stage", "k_hub_reduce",
                                               "k_hub_final", "k_lookup",    "k_verify",    "k_res_*",
                                               "k_scan",      "k_assign",    "k_fill_*"};
  return (kind >= 0 && kind < KBISIM_NKERNELS) ? names[kind] : nullptr;
}

int kbisim_schedule_info(kbisim_ctx *c, int64_t *info) {
  if (!c || !info) return KBISIM_EINVAL;
  for (int i = 0; i < 8; ++i) info[i] = c->sched.info[i];
  return KBISIM_OK;
}

int kbisim_copy_probe(void *dst, const void *src, size_t bytes, void *stream) {
  if (!dst || !src || bytes % 16) return KBISIM_EINVAL;
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return KBISIM_OK;
  const unsigned g = (unsigned)std::min<int64_t>((n16 + 255) / 256, 1 << 20);
  k_copy16<<<g, 256, 0, (hipStream_t)stream>>>((uint4 *)dst, (const uint4 *)src, n16);
  HIP_TRY(hipGetLastError());
  return KBISIM_OK;
}

int kbisim_gather_probe(kbisim_ctx *c, const int32_t *pid, int reps, double *ms) {
  if (!c || !pid || reps < 1 || !ms) return KBISIM_EINVAL;
  *ms = 0.0;
  const int64_t n = c->g.n, m = c->g.m;
  if (m == 0) return KBISIM_OK;
  k_scatter_rank<<<blocks_for(n, 256), 256, 0, c->stream>>>((int)n, pid, c->rank, c->gpid[0]);
  HIP_TRY(hipGetLastError());
  u32 slots = 1;  // output words: a power of two, at most 1024 and at most n
  while (slots < 1024 && (int64_t)slots * 2 <= n) slots *= 2;
  int rc = fill_i32(c, c->vlist, slots, 0);
  if (rc) return rc;
  // the probe reads the same gather index and pairs as the signature kernels
  const unsigned grid = (unsigned)std::min<int64_t>((m + 1023) / 1024, 1 << 20);
  const GraphSrcT<true> sep{c->g.row_ptr, c->gcol, sep_labels(c), c->gpid[0], pid, c->pb, c->rbits};
  const GraphSrcT<false> pk{c->g.row_ptr, c->gcol, nullptr, c->gpid[0], pid, c->pb, c->rbits};
  const bool s2 = separate_labels(c);
  auto probe = [&]() {
    if (s2) k_gather_probe<<<grid, 256, 0, c->stream>>>(sep, m, (u32 *)c->vlist, slots - 1);
    else k_gather_probe<<<grid, 256, 0, c->stream>>>(pk, m, (u32 *)c->vlist, slots - 1);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return KBISIM_EHIP;
  }
  probe();  // warm-up
  (void)hipEventRecord(e0, c->stream);
  for (int r = 0; r < reps; ++r) probe();
  (void)hipEventRecord(e1, c->stream);
  hipError_t e = hipStreamSynchronize(c->stream);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e);
  *ms = (double)t / reps;
  return KBISIM_OK;
}

int kbisim_batch_workspace_bytes(const kbisim_graph *u, int64_t num_graphs, int kmax, size_t *bytes) {
  int rc = check_sizes(u);
  if (rc) return rc;
  if (!bytes || num_graphs < 1 || num_graphs >= (int64_t(1) << 31) || kmax < 0 || kmax > (1 << 20))
    return KBISIM_EINVAL;
  *bytes = make_plan(u->n, u->m, u->vlabel_ptr ? u->nlabels : 0, kmax, num_graphs).total;
  return KBISIM_OK;
}

int kbisim_batch_create(const kbisim_graph *u, int64_t num_graphs, const int64_t *vert_off, int kmax,
                        const kbisim_tuning *tuning, void *workspace, size_t ws_bytes, void *stream,
                        kbisim_batch **out) {
  if (!out || num_graphs < 1 || num_graphs >= (int64_t(1) << 31) || !vert_off) return KBISIM_EINVAL;
  *out = nullptr;
  kbisim_ctx *c = nullptr;
  int rc = create_impl(u, kmax, tuning, workspace, ws_bytes, stream, num_graphs, vert_off, &c);
  if (rc) return rc;
  kbisim_batch *b = new (std::nothrow) kbisim_batch();
  if (!b) {
    kbisim_destroy(c);
    return KBISIM_EINTERNAL;
  }
  b->c = c;
  *out = b;
  return KBISIM_OK;
}

int kbisim_batch_refine(kbisim_batch *b, int k, int32_t *const *out_ids, int64_t *out_counts) {
  if (!b) return KBISIM_EINVAL;
  return refine_impl(b->c, nullptr, k, out_ids, out_counts);
}

int kbisim_batch_step_async(kbisim_batch *b, int i, int32_t *out_ids) {
  if (!b) return KBISIM_EINVAL;
  return step_async_impl(b->c, i, nullptr, out_ids);
}

int kbisim_batch_step_result(kbisim_batch *b, int i, int32_t *out_ids, int64_t *out_counts) {
  if (!b || !out_counts) return KBISIM_EINVAL;
  kbisim_ctx *c = b->c;
  int rc = step_result_impl(c, i, nullptr, out_ids);
  if (rc) return rc;
  const int64_t G = c->num_graphs;
  if (c->g.n == 0) {
    for (int64_t g = 0; g < G; ++g) out_counts[g] = 0;
    return KBISIM_OK;
  }
  // column i of the [graph][kmax] count table
  HIP_TRY(hipMemcpy2DAsync(out_counts, sizeof(int64_t), c->bcounts + i, sizeof(int64_t) * (size_t)c->kmax,
                           sizeof(int64_t), (size_t)G, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return KBISIM_OK;
}

int kbisim_batch_context(kbisim_batch *b, kbisim_ctx **ctx) {
  if (!b || !ctx) return KBISIM_EINVAL;
  *ctx = b->c;
  return KBISIM_OK;
}

int kbisim_batch_destroy(kbisim_batch *b) {
  if (b) kbisim_destroy(b->c);
  delete b;
  return KBISIM_OK;
}

namespace {
struct TransposePlan {
  size_t off_cnt, off_tiles, off_cursor, total;
  int64_t ntiles;
};
TransposePlan transpose_plan(int64_t n) {
  TransposePlan p{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t o = at;
    at = align_up(at + std::max<size_t>(bytes, 1));
    return o;
  };
  p.ntiles = (std::max<int64_t>(n, 1) + SCAN_TILE - 1) / SCAN_TILE;
  p.off_cnt = take(4 * (size_t)std::max<int64_t>(n, 1));
  p.off_tiles = take(8 * (size_t)p.ntiles);
  p.off_cursor = take(8 * (size_t)std::max<int64_t>(n, 1));
  p.total = at;
  return p;
}
}  // namespace

int kbisim_transpose_workspace_bytes(int64_t n, int64_t m, size_t *bytes) {
  if (!bytes || n < 0 || m < 0) return KBISIM_EINVAL;
  if (n >= (int64_t(1) << 31)) return KBISIM_ERANGE;
  *bytes = transpose_plan(n).total;
  return KBISIM_OK;
}

int kbisim_transpose(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const int32_t *elabel,
                     int64_t *out_row_ptr, int32_t *out_col, int32_t *out_elabel, void *workspace, size_t ws_bytes,
                     void *stream) {
  if (n < 0 || m < 0 || !row_ptr || !out_row_ptr || (m > 0 && (!col || !out_col))) return KBISIM_EINVAL;
  if (n >= (int64_t(1) << 31)) return KBISIM_ERANGE;
  const TransposePlan p = transpose_plan(n);
  if (!workspace || ws_bytes < p.total) return KBISIM_ENOSPACE;
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)workspace;
  int *cnt = (int *)(w + p.off_cnt);
  int64_t *tiles = (int64_t *)(w + p.off_tiles);
  unsigned long long *cursor = (unsigned long long *)(w + p.off_cursor);
  u32 *err = (u32 *)(w + p.off_tiles);  // scratch word, reused by the scan afterwards
  if (n == 0) {
    if (m > 0) return KBISIM_EGRAPH;
    k_fill_u64<<<1, 64, 0, s>>>((u64 *)out_row_ptr, 1, 0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return KBISIM_OK;
  }
  // validate the input (row offsets monotone from 0 to m, targets in range)
  k_fill_i32<<<1, 64, 0, s>>>((int *)err, 1, 0);
  k_validate_rows<<<blocks_for(n + 1, 256), 256, 0, s>>>(n, m, row_ptr, err, ERR_GRAPH_ROWPTR);
  if (m > 0) {
    validate_vals(s, m, col, n, err, ERR_GRAPH_COL);
    if (elabel) validate_vals(s, m, elabel, -1, err, ERR_GRAPH_ELABEL);
  }
  HIP_TRY(hipGetLastError());
  u32 bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, err, sizeof bad, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bad) return KBISIM_EGRAPH;
  k_fill_i32<<<blocks_for(n, 256), 256, 0, s>>>(cnt, n, 0);
  if (m > 0) k_indegree<<<(unsigned)std::min<int64_t>(blocks_for(m, INDEG_CHUNK), 65536), 256, 0, s>>>(m, col, cnt);
  k_sum_tiles64<<<(unsigned)p.ntiles, 256, 0, s>>>(n, cnt, tiles);
  k_scan_tiles64<<<1, 256, 0, s>>>(p.ntiles, tiles);
  k_write_ptr64<<<(unsigned)p.ntiles, 256, 0, s>>>(n, cnt, tiles, out_row_ptr, cursor);
  if (m > 0)
    k_transpose_scatter<<<(unsigned)std::min<int64_t>(blocks_for(n * WAVE, 256), 65536), 256, 0, s>>>(
        n, row_ptr, col, elabel, cursor, out_col, out_elabel);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return KBISIM_OK;
}

namespace {
struct QuotientPlan {
  size_t off_a, off_b, off_hist, off_offs, off_tiles, off_flag, off_pos, off_word, off_tgt, total;
  int64_t rtiles, hist_n, htiles, mtiles;
};
QuotientPlan quotient_plan(int64_t n, int64_t m) {
  QuotientPlan p{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t o = at;
    at = align_up(at + std::max<size_t>(bytes, 1));
    return o;
  };
  const int64_t M = std::max<int64_t>(m, 1);
  p.rtiles = (M + RADIX_TILE - 1) / RADIX_TILE;
  p.hist_n = 256 * p.rtiles;
  p.htiles = (p.hist_n + SCAN_TILE - 1) / SCAN_TILE;
  p.mtiles = (M + SCAN_TILE - 1) / SCAN_TILE;
  p.off_a = take(8 * (size_t)M);
  p.off_b = take(8 * (size_t)M);
  p.off_hist = take(4 * (size_t)p.hist_n);
  p.off_offs = take(8 * (size_t)(p.hist_n + 1));
  p.off_tiles = take(8 * (size_t)std::max(p.htiles, p.mtiles));
  p.off_flag = take(4 * (size_t)M);
  p.off_pos = take(8 * (size_t)(M + 1));
  p.off_word = take(16);
  p.off_tgt = take(4 * (size_t)std::max<int64_t>(n, 1));
  p.total = at;
  return p;
}

// One summary key per CSR entry, over the degree schedule of the context.
extern "C++" template <class Src>
int quotient_keys(kbisim_ctx *c, const Src &src, const int32_t *src_pid, const int32_t *tgt, QKey q, u64 *keys) {
  const Schedule &S = c->sched;
  hipStream_t st = c->stream;
  if (S.nranges) {
    if (S.range_edges == 1024)
      k_quotient_range<Src, 1024><<<(unsigned)S.nranges, 256, 0, st>>>(src, c->ranges, src_pid, tgt, q, keys);
    else
      k_quotient_range<Src, 2048><<<(unsigned)S.nranges, 256, 0, st>>>(src, c->ranges, src_pid, tgt, q, keys);
  }
  const int nrows = S.nbig + S.nrow8 + S.nrow20;
  if (nrows) k_quotient_rows<Src><<<(unsigned)nrows, 256, 0, st>>>(src, c->ranges + S.nranges, src_pid, tgt, q, keys);
  const int *hubs = c->lists + S.hub_off;
  if (S.nchunks)
    k_quotient_hubs<Src, HubChunk><<<(unsigned)S.nchunks, 256, 0, st>>>(src, c->chunks, hubs, src_pid, tgt, q, keys);
  if (S.ngchunks)
    k_quotient_hubs<Src, HubGChunk><<<(unsigned)S.ngchunks, 256, 0, st>>>(src, c->gchunks, hubs, src_pid, tgt, q,
                                                                          keys);
  HIP_TRY(hipGetLastError());
  return 0;
}

// Exclusive scan of cnt[0..len) into out[0..len] (64-bit), on `s`.
int scan64(hipStream_t s, int64_t len, const int *cnt, int64_t *tiles, int64_t *out) {
  const int64_t nt = (len + SCAN_TILE - 1) / SCAN_TILE;
  k_sum_tiles64<<<(unsigned)nt, 256, 0, s>>>(len, cnt, tiles);
  k_scan_tiles64<<<1, 256, 0, s>>>(nt, tiles);
  k_write_ptr64<<<(unsigned)nt, 256, 0, s>>>(len, cnt, tiles, out, nullptr);
  HIP_TRY(hipGetLastError());
  return 0;
}
}  // namespace

int kbisim_quotient_workspace_bytes(kbisim_ctx *c, size_t *bytes) {
  if (!c || !bytes || c->num_graphs > 0) return KBISIM_EINVAL;
  *bytes = quotient_plan(c->g.n, c->g.m).total;
  return KBISIM_OK;
}

int kbisim_quotient(kbisim_ctx *c, const int32_t *src_pid, const int32_t *dst_pid, int32_t *out_src,
                    int32_t *out_label, int32_t *out_dst, int64_t *out_count, void *workspace, size_t ws_bytes) {
  if (!c || c->num_graphs > 0 || !src_pid || !dst_pid || !out_count) return KBISIM_EINVAL;
  const int64_t n = c->g.n, m = c->g.m;
  *out_count = 0;
  if (m == 0) return KBISIM_OK;
  if (!out_src || !out_label || !out_dst) return KBISIM_EINVAL;
  const QuotientPlan p = quotient_plan(n, m);
  if (!workspace || ws_bytes < p.total) return KBISIM_ENOSPACE;
  hipStream_t s = c->stream;
  char *w = (char *)workspace;
  u64 *ka = (u64 *)(w + p.off_a), *kb = (u64 *)(w + p.off_b);
  int *hist = (int *)(w + p.off_hist);
  int64_t *offs = (int64_t *)(w + p.off_offs), *tiles = (int64_t *)(w + p.off_tiles);
  int *flag = (int *)(w + p.off_flag);
  int64_t *pos = (int64_t *)(w + p.off_pos);
  u32 *word = (u32 *)(w + p.off_word);  // [0] error bits, [1] max source id, [2] max target id
  int rc = 0;
  // both partitions must hold ids in [0, n)
  k_fill_i32<<<1, 64, 0, s>>>((int *)word, 4, 0);
  validate_vals(s, n, src_pid, n, word, ERR_BAD_PID);
  validate_vals(s, n, dst_pid, n, word, ERR_BAD_PID);
  k_max_i32<<<(unsigned)std::min<int64_t>(blocks_for(n, 256), 4096), 256, 0, s>>>(n, src_pid, word + 1);
  k_max_i32<<<(unsigned)std::min<int64_t>(blocks_for(n, 256), 4096), 256, 0, s>>>(n, dst_pid, word + 2);
  HIP_TRY(hipGetLastError());
  u32 hw[3] = {0, 0, 0};
  HIP_TRY(hipMemcpyAsync(hw, word, sizeof hw, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hw[0]) return KBISIM_EINVAL;
  QKey q;
  q.db = (u32)std::max(1, bit_width(hw[2]));
  q.lb = c->g.elabel ? (u32)bit_width(c->max_label) : 0u;
  const int sbits = std::max(1, bit_width(hw[1]));
  const int total_bits = sbits + (int)q.lb + (int)q.db;
  if (total_bits > 64) return KBISIM_ERANGE;
  // target blocks in rank order, then one key per entry over the schedule
  int32_t *tgt = (int32_t *)(w + p.off_tgt);
  k_scatter_rank<<<blocks_for(n, 256), 256, 0, s>>>((int)n, dst_pid, c->rank, tgt);
  HIP_TRY(hipGetLastError());
  const int32_t *lab = separate_labels(c) ? sep_labels(c) : nullptr;
  if (lab) rc = quotient_keys(c, GraphSrcT<true>{c->g.row_ptr, c->gcol, lab, tgt, src_pid, c->pb, c->rbits}, src_pid,
                             tgt, q, ka);
  else rc = quotient_keys(c, GraphSrcT<false>{c->g.row_ptr, c->gcol, nullptr, tgt, src_pid, c->pb, c->rbits}, src_pid,
                         tgt, q, ka);
  if (rc) return rc;
  for (int shift = 0; shift < total_bits; shift += 8) {
    k_radix_hist<<<(unsigned)p.rtiles, 256, 0, s>>>(m, ka, shift, p.rtiles, hist);
    HIP_TRY(hipGetLastError());
    if ((rc = scan64(s, p.hist_n, hist, tiles, offs))) return rc;
    k_radix_scatter<<<(unsigned)p.rtiles, 256, 0, s>>>(m, ka, shift, p.rtiles, offs, hist, kb);
    HIP_TRY(hipGetLastError());
    std::swap(ka, kb);
  }
  k_run_starts<<<(unsigned)std::min<int64_t>(blocks_for(m, 256), 65536), 256, 0, s>>>(m, ka, flag);
  HIP_TRY(hipGetLastError());
  if ((rc = scan64(s, m, flag, tiles, pos))) return rc;
  k_quotient_write<<<(unsigned)std::min<int64_t>(blocks_for(m, 256), 65536), 256, 0, s>>>(m, ka, flag, pos, q, out_src,
                                                                                          out_label, out_dst);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out_count, pos + m, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return KBISIM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- no-allocation entry point
// Scratch for kbisim_refine_noalloc: one array per GPU, held from the
// library's load on that GPU until the process ends.  In host code its name
// stands for the symbol only; its device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
std::mutex &scratch_mu() {
  static std::mutex *m = new std::mutex();
  return *m;
}

// Device address of the current device's scratch array (looked up on the
// first call on that device).
int scratch_address(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return KBISIM_EINTERNAL;
  std::lock_guard<std::mutex> lk(scratch_mu());
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!p) return KBISIM_EINTERNAL;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}
}  // namespace

extern "C" {

size_t kbisim_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

int kbisim_refine_noalloc(const kbisim_graph *g, int k, int32_t *const *out_block_ids, int64_t *out_counts,
                          void *stream) {
  int rc = check_sizes(g);
  if (rc) return rc;
  if (k < 0 || k > (1 << 20)) return KBISIM_EINVAL;
  if (k > 0 && (!out_block_ids || !out_counts)) return KBISIM_EINVAL;
  const size_t need = make_plan(g->n, g->m, g->vlabel_ptr ? g->nlabels : 0, k, 0).total;
  if (need > NOALLOC_SCRATCH_BYTES) return KBISIM_ENOSPACE;
  void *ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  kbisim_ctx *c = nullptr;
  if ((rc = create_impl(g, k, nullptr, ws, NOALLOC_SCRATCH_BYTES, stream, 0, nullptr, &c, false))) return rc;
  rc = refine_impl(c, nullptr, k, out_block_ids, out_counts);
  kbisim_destroy(c);
  return rc;
}

const char *kbisim_strerror(int code) {
  switch (code) {
    case KBISIM_OK: return "ok";
    case KBISIM_EINVAL: return "invalid argument";
    case KBISIM_EGRAPH: return "graph validation failed";
    case KBISIM_ENOSPACE: return "workspace too small";
    case KBISIM_EHIP: return g_hip_msg[0] ? g_hip_msg : "HIP runtime error";
    case KBISIM_ERANGE: return "size out of range";
    case KBISIM_EINTERNAL: return "internal consistency check failed";
    default: return "unknown error";
  }
}

const char *kbisim_version(void) { return "kbisim 0.3 gfx950"; }

}  // extern "C"
