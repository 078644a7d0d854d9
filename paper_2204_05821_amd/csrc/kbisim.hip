// Host engine and C ABI of the k-bisimulation refinement library (gfx950).
//
// The engine owns no device memory: kbisim_create carves every buffer from
// the caller's workspace, validates the graph, computes P0 (vertex label-set
// equality) and a static degree schedule, and kbisim_refine enqueues k
// refinement steps on the caller's stream with no host synchronisation
// inside the loop.  A step that met a hash collision it could not settle in
// its one in-loop peeling round is detected after the final synchronisation
// and recomputed, from that step on, with peeling rounds driven by the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
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

inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 64;
  while (p < x) p <<= 1;
  return p;
}

struct Plan {
  size_t off_H, off_DC, off_rep, off_p0, off_vlist, off_clA, off_clB, off_lw, off_lb, off_lh;
  size_t off_table, off_ctable, off_hubv, off_hacc, off_hcnt, off_hoff, off_hsize, off_hdeg, off_chunks;
  size_t off_status, off_counters, off_dcounts, off_err, off_hubsets;
  uint64_t tslots;
  int64_t nhub_max, nchunk_max, ntiles, hubset_slots;
  int ncounter_steps;
  size_t total;
};

Plan make_plan(int64_t n, int64_t m, int64_t nl, int kmax) {
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
  p.nhub_max = big / BLOCK_MAX + 1;
  p.nchunk_max = big / HUB_CHUNK + p.nhub_max + 1;
  p.ntiles = (int64_t)(N + SCAN_TILE - 1) / SCAN_TILE + 1;
  p.hubset_slots = 2 * big + 64;
  p.ncounter_steps = kmax + 4;
  p.off_H = take(8 * N);
  p.off_DC = take(4 * N);
  p.off_rep = take(4 * N);
  p.off_p0 = take(4 * N);
  p.off_vlist = take(4 * N);
  p.off_clA = take(4 * N);
  p.off_clB = take(4 * N);
  p.off_lw = take(4 * N);
  p.off_lb = take(4 * N);
  p.off_lh = take(4 * N);
  p.off_table = take(8 * p.tslots);
  p.off_ctable = take(8 * p.tslots);
  p.off_hubv = take(4 * (size_t)p.nhub_max);
  p.off_hacc = take(8 * (size_t)p.nhub_max);
  p.off_hcnt = take(4 * (size_t)p.nhub_max);
  p.off_hoff = take(8 * (size_t)p.nhub_max);
  p.off_hsize = take(8 * (size_t)p.nhub_max);
  p.off_hdeg = take(8 * (size_t)p.nhub_max);
  p.off_chunks = take(sizeof(HubChunk) * (size_t)p.nchunk_max);
  p.off_status = take(8 * (size_t)p.ntiles);
  p.off_counters = take(4 * (size_t)CNT_STRIDE * (size_t)p.ncounter_steps);
  p.off_dcounts = take(8 * (size_t)p.ncounter_steps);
  p.off_err = take(16);
  p.off_hubsets = take(8 * (size_t)p.hubset_slots);
  p.total = at;
  return p;
}

// Degree schedule of one row structure (graph rows or label-set rows).
struct Schedule {
  int nW = 0, nB = 0, nH = 0, nchunks = 0;
  int64_t hubset_used = 0;
};

}  // namespace

struct kbisim_ctx {
  kbisim_graph g;
  int kmax;
  hipStream_t stream;
  Plan plan;
  char *ws;
  u64 *H, *table, *ctable, *hacc, *hubsets, *status;
  u32 *DC, *hcnt, *err;
  int *rep, *p0, *vlist, *clA, *clB, *lw, *lb, *lh, *hubv, *counters;
  int64_t *hoff, *hsize, *hdeg, *dcounts;
  HubChunk *chunks;
  Schedule sched;      // graph rows
  u32 epoch = 0, cepoch = 0, hepoch = 0, stamp = 0;
  u64 hmask = ~0ULL;
  int64_t p0_count = 0;
};

namespace {

int hip_fail(hipError_t e) {
  snprintf(g_hip_msg, sizeof g_hip_msg, "HIP error %d: %s", (int)e, hipGetErrorString(e));
  return KBISIM_EHIP;
}

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return hip_fail(_e); \
  } while (0)

#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

inline unsigned blocks_for(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

int fill_u64(kbisim_ctx *c, u64 *p, int64_t cnt, u64 val) {
  if (cnt <= 0) return 0;
  unsigned g = (unsigned)std::min<int64_t>(blocks_for(cnt, 256), 65536);
  k_fill_u64<<<g, 256, 0, c->stream>>>(p, cnt, val);
  LAUNCH_CHECK();
  return 0;
}

int fill_i32(kbisim_ctx *c, int *p, int64_t cnt, int val) {
  if (cnt <= 0) return 0;
  unsigned g = (unsigned)std::min<int64_t>(blocks_for(cnt, 256), 65536);
  k_fill_i32<<<g, 256, 0, c->stream>>>(p, cnt, val);
  LAUNCH_CHECK();
  return 0;
}

// Next table epoch in 1..15; the table is cleared before an epoch repeats.
int next_epoch(kbisim_ctx *c, u32 &e, u64 *table) {
  if (e >= 15) {
    int rc = fill_u64(c, table, (int64_t)c->plan.tslots, 0);
    if (rc) return rc;
    e = 0;
  }
  ++e;
  return 0;
}

int next_hub_epoch(kbisim_ctx *c, const Schedule &s) {
  if (c->hepoch >= 3) {
    int rc = fill_u64(c, c->hubsets, s.hubset_used, 0);
    if (rc) return rc;
    c->hepoch = 0;
  }
  ++c->hepoch;
  return 0;
}

int read_err(kbisim_ctx *c, u32 *out) {
  HIP_TRY(hipMemcpyAsync(out, c->err, sizeof(u32), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return 0;
}

// Classify rows of `ptr` (NULL: every row has one item) into the wave, block
// and hub tiers and lay out hub hash sets and chunks.  Synchronises.
int build_schedule(kbisim_ctx *c, const int64_t *ptr, Schedule &s) {
  const int n = (int)c->g.n;
  s = Schedule{};
  int *cnt = c->counters + CNT_STRIDE * (c->plan.ncounter_steps - 1);
  int rc = fill_i32(c, cnt, CNT_STRIDE, 0);
  if (rc) return rc;
  if (n > 0) {
    k_classify<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, ptr, cnt, c->lw, c->lb, c->lh);
    LAUNCH_CHECK();
  }
  int h_cnt[3] = {0, 0, 0};
  HIP_TRY(hipMemcpyAsync(h_cnt, cnt, sizeof h_cnt, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  s.nW = h_cnt[0];
  s.nB = h_cnt[1];
  s.nH = h_cnt[2];
  if (s.nH > c->plan.nhub_max) return KBISIM_EINTERNAL;
  if (s.nH > 0) {
    k_hub_degrees<<<blocks_for(s.nH, 256), 256, 0, c->stream>>>(c->lh, s.nH, ptr, c->hdeg);
    LAUNCH_CHECK();
    std::vector<int64_t> deg((size_t)s.nH), off((size_t)s.nH), size((size_t)s.nH);
    HIP_TRY(hipMemcpyAsync(deg.data(), c->hdeg, 8 * (size_t)s.nH, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<HubChunk> chunks;
    int64_t at = 0;
    for (int i = 0; i < s.nH; ++i) {
      off[(size_t)i] = at;
      size[(size_t)i] = 2 * deg[(size_t)i];
      at += size[(size_t)i];
      for (int64_t b = 0; b < deg[(size_t)i]; b += HUB_CHUNK) {
        HubChunk hc;
        hc.hub = i;
        hc.pad = 0;
        hc.b = b;
        hc.e = std::min<int64_t>(b + HUB_CHUNK, deg[(size_t)i]);
        chunks.push_back(hc);
      }
    }
    if (at > c->plan.hubset_slots || (int64_t)chunks.size() > c->plan.nchunk_max) return KBISIM_EINTERNAL;
    s.nchunks = (int)chunks.size();
    s.hubset_used = at;
    HIP_TRY(hipMemcpyAsync(c->hoff, off.data(), 8 * (size_t)s.nH, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->hsize, size.data(), 8 * (size_t)s.nH, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->chunks, chunks.data(), sizeof(HubChunk) * chunks.size(), hipMemcpyHostToDevice,
                           c->stream));
    rc = fill_u64(c, c->hubsets, at, 0);
    if (rc) return rc;
    rc = fill_u64(c, c->hacc, s.nH, 0);
    if (rc) return rc;
    rc = fill_i32(c, (int *)c->hcnt, s.nH, 0);
    if (rc) return rc;
    c->hepoch = 0;
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return 0;
}

// One peeling round over `in_list` (count at in_cnt) into out_list/out_cnt.
template <class Src>
int peel_round(kbisim_ctx *c, const Src &src, int *in_cnt, int *in_list, int *out_cnt, int *out_list) {
  int rc = next_epoch(c, c->cepoch, c->ctable);
  if (rc) return rc;
  k_res_insert<<<RES_GRID, 256, 0, c->stream>>>(in_cnt, in_list, c->H, c->ctable, c->plan.tslots - 1, c->cepoch);
  LAUNCH_CHECK();
  k_res_verify<Src><<<RES_GRID, 256, 0, c->stream>>>(src, in_cnt, in_list, c->H, c->DC, c->ctable,
                                                     c->plan.tslots - 1, c->cepoch, c->rep, out_cnt, out_list,
                                                     c->err);
  LAUNCH_CHECK();
  return 0;
}

// One refinement step: src (previous partition inside) -> out, block count
// into *count_dev.  cnt: CNT_STRIDE zeroed device counters for this step.
// careful: settle every collision with host-driven peeling rounds.
template <class Src>
int run_step(kbisim_ctx *c, const Src &src, const Schedule &s, int *out, int64_t *count_dev, int *cnt,
             bool careful) {
  const int n = (int)c->g.n;
  if (n == 0) return 0;
  const u64 tmask = c->plan.tslots - 1;
  int rc = next_epoch(c, c->epoch, c->table);
  if (rc) return rc;
  const u32 ep = c->epoch;
  k_sig_small<Src><<<blocks_for(n, 256), 256, 0, c->stream>>>(src, n, c->H, c->DC, c->table, tmask, ep, c->hmask);
  LAUNCH_CHECK();
  if (s.nW) {
    k_sig_wave<Src><<<blocks_for(s.nW, 4), 256, 0, c->stream>>>(src, c->lw, s.nW, c->H, c->DC, c->table, tmask, ep,
                                                                c->hmask);
    LAUNCH_CHECK();
  }
  if (s.nB) {
    k_sig_block<Src><<<(unsigned)s.nB, 256, 0, c->stream>>>(src, c->lb, c->H, c->DC, c->table, tmask, ep, c->hmask);
    LAUNCH_CHECK();
  }
  if (s.nH) {
    rc = next_hub_epoch(c, s);
    if (rc) return rc;
    k_sig_hub<Src><<<(unsigned)s.nchunks, 256, 0, c->stream>>>(src, c->chunks, c->lh, c->hoff, c->hsize, c->hubsets,
                                                               c->hacc, c->hcnt, c->hepoch);
    LAUNCH_CHECK();
    k_hub_final<Src><<<blocks_for(s.nH, 256), 256, 0, c->stream>>>(src, c->lh, s.nH, c->hacc, c->hcnt, c->H, c->DC,
                                                                   c->table, tmask, ep, c->hmask);
    LAUNCH_CHECK();
  }
  k_lookup<Src><<<blocks_for(n, 256), 256, 0, c->stream>>>(src, n, c->H, c->DC, c->table, tmask, ep, c->rep, &cnt[0],
                                                           c->vlist, &cnt[1], c->clA, c->err);
  LAUNCH_CHECK();
  k_verify<Src><<<PERSIST_GRID, 256, 0, c->stream>>>(src, &cnt[0], c->vlist, c->DC, c->rep, &cnt[1], c->clA, c->err);
  LAUNCH_CHECK();
  rc = peel_round(c, src, &cnt[1], c->clA, &cnt[2], c->clB);
  if (rc) return rc;
  if (careful) {
    int *in_cnt = &cnt[2], *out_cnt = &cnt[3];
    int *in_list = c->clB, *out_list = c->clA;
    for (int round = 0;; ++round) {
      int left = 0;
      HIP_TRY(hipMemcpyAsync(&left, in_cnt, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
      if (left == 0) break;
      if (round > n + 1) return KBISIM_EINTERNAL;
      rc = fill_i32(c, out_cnt, 1, 0);
      if (rc) return rc;
      rc = peel_round(c, src, in_cnt, in_list, out_cnt, out_list);
      if (rc) return rc;
      std::swap(in_cnt, out_cnt);
      std::swap(in_list, out_list);
    }
  }
  k_scan<<<blocks_for(n, SCAN_TILE), 256, 0, c->stream>>>(n, c->rep, out, c->status, &cnt[4], count_dev, ++c->stamp,
                                                           c->err);
  LAUNCH_CHECK();
  k_assign<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, c->rep, out);
  LAUNCH_CHECK();
  return 0;
}

int refine_impl(kbisim_ctx *c, const int32_t *start, int k, int32_t *const *out, int64_t *counts) {
  if (!c) return KBISIM_EINVAL;
  if (k < 0 || k > c->kmax) return KBISIM_EINVAL;
  if (k == 0) return KBISIM_OK;
  if (!out || !counts) return KBISIM_EINVAL;
  for (int i = 0; i < k; ++i)
    if (!out[i] && c->g.n > 0) return KBISIM_EINVAL;
  const int n = (int)c->g.n;
  if (n == 0) {
    for (int i = 0; i < k; ++i) counts[i] = 0;
    return KBISIM_OK;
  }
  int rc = fill_i32(c, c->counters, (int64_t)CNT_STRIDE * k, 0);
  if (rc) return rc;
  rc = fill_i32(c, (int *)c->err, 1, 0);
  if (rc) return rc;
  const int32_t *prev = start ? start : c->p0;
  for (int i = 0; i < k; ++i) {
    GraphSrc src{c->g.row_ptr, c->g.col, c->g.elabel, prev};
    rc = run_step(c, src, c->sched, out[i], &c->dcounts[i], c->counters + CNT_STRIDE * i, false);
    if (rc) return rc;
    prev = out[i];
  }
  std::vector<int> hc((size_t)CNT_STRIDE * k);
  u32 err = 0;
  HIP_TRY(hipMemcpyAsync(hc.data(), c->counters, 4 * hc.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(counts, c->dcounts, 8 * (size_t)k, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&err, c->err, sizeof err, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (err) return KBISIM_EINTERNAL;
  int first_bad = -1;
  for (int i = 0; i < k; ++i)
    if (hc[(size_t)CNT_STRIDE * i + 2] != 0) { first_bad = i; break; }
  if (first_bad >= 0) {
    prev = first_bad == 0 ? (start ? start : c->p0) : out[first_bad - 1];
    for (int i = first_bad; i < k; ++i) {
      rc = fill_i32(c, c->counters + CNT_STRIDE * i, CNT_STRIDE, 0);
      if (rc) return rc;
      GraphSrc src{c->g.row_ptr, c->g.col, c->g.elabel, prev};
      rc = run_step(c, src, c->sched, out[i], &c->dcounts[i], c->counters + CNT_STRIDE * i, true);
      if (rc) return rc;
      prev = out[i];
    }
    HIP_TRY(hipMemcpyAsync(counts, c->dcounts, 8 * (size_t)k, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(&err, c->err, sizeof err, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (err) return KBISIM_EINTERNAL;
  }
  return KBISIM_OK;
}

int check_sizes(const kbisim_graph *g) {
  if (!g) return KBISIM_EINVAL;
  if (g->n < 0 || g->m < 0 || g->nlabels < 0) return KBISIM_EINVAL;
  if (g->n >= (int64_t(1) << 31) || g->m >= (int64_t(1) << 62) || g->nlabels >= (int64_t(1) << 62))
    return KBISIM_ERANGE;
  return 0;
}

}  // namespace

extern "C" {

int kbisim_workspace_bytes(const kbisim_graph *g, int kmax, size_t *bytes) {
  int rc = check_sizes(g);
  if (rc) return rc;
  if (!bytes || kmax < 0 || kmax > (1 << 20)) return KBISIM_EINVAL;
  *bytes = make_plan(g->n, g->m, g->vlabel_ptr ? g->nlabels : 0, kmax).total;
  return KBISIM_OK;
}

int kbisim_create(const kbisim_graph *g, int kmax, void *workspace, size_t ws_bytes, void *stream, kbisim_ctx **out) {
  int rc = check_sizes(g);
  if (rc) return rc;
  if (!out || kmax < 0 || kmax > (1 << 20)) return KBISIM_EINVAL;
  *out = nullptr;
  const int64_t n = g->n, m = g->m;
  if (n > 0 && !g->row_ptr) return KBISIM_EINVAL;
  if (m > 0 && !g->col) return KBISIM_EINVAL;
  if (g->vlabel_ptr && !g->vlabel && g->nlabels > 0) return KBISIM_EINVAL;
  if (!g->vlabel_ptr && !g->vlabel && g->nlabels > 0) return KBISIM_EINVAL;
  const int64_t nl = g->vlabel_ptr ? g->nlabels : 0;
  Plan plan = make_plan(n, m, nl, kmax);
  if (!workspace) return KBISIM_EINVAL;
  if (ws_bytes < plan.total) return KBISIM_ENOSPACE;

  kbisim_ctx *c = new (std::nothrow) kbisim_ctx();
  if (!c) return KBISIM_EINTERNAL;
  c->g = *g;
  c->kmax = kmax;
  c->stream = (hipStream_t)stream;
  c->plan = plan;
  c->ws = (char *)workspace;
  char *w = c->ws;
  c->H = (u64 *)(w + plan.off_H);
  c->DC = (u32 *)(w + plan.off_DC);
  c->rep = (int *)(w + plan.off_rep);
  c->p0 = (int *)(w + plan.off_p0);
  c->vlist = (int *)(w + plan.off_vlist);
  c->clA = (int *)(w + plan.off_clA);
  c->clB = (int *)(w + plan.off_clB);
  c->lw = (int *)(w + plan.off_lw);
  c->lb = (int *)(w + plan.off_lb);
  c->lh = (int *)(w + plan.off_lh);
  c->table = (u64 *)(w + plan.off_table);
  c->ctable = (u64 *)(w + plan.off_ctable);
  c->hubv = (int *)(w + plan.off_hubv);
  c->hacc = (u64 *)(w + plan.off_hacc);
  c->hcnt = (u32 *)(w + plan.off_hcnt);
  c->hoff = (int64_t *)(w + plan.off_hoff);
  c->hsize = (int64_t *)(w + plan.off_hsize);
  c->hdeg = (int64_t *)(w + plan.off_hdeg);
  c->chunks = (HubChunk *)(w + plan.off_chunks);
  c->status = (u64 *)(w + plan.off_status);
  c->counters = (int *)(w + plan.off_counters);
  c->dcounts = (int64_t *)(w + plan.off_dcounts);
  c->err = (u32 *)(w + plan.off_err);
  c->hubsets = (u64 *)(w + plan.off_hubsets);
  const char *dbg = getenv("KBISIM_DEBUG_HASH_BITS");
  if (dbg && *dbg) {
    int b = atoi(dbg);
    if (b >= 0 && b < 64) c->hmask = b == 0 ? 0ULL : ((1ULL << b) - 1ULL);
  }

  auto fail = [&](int code) {
    delete c;
    return code;
  };
  // Validation (Def. multi-relational-labeled-property-graph as a CSR contract).
  if ((rc = fill_i32(c, (int *)c->err, 4, 0))) return fail(rc);
  if (n == 0 && m > 0) return fail(KBISIM_EGRAPH);
  if (n > 0) {
    k_validate_rows<<<blocks_for(n + 1, 256), 256, 0, c->stream>>>(n, m, g->row_ptr, c->err, ERR_GRAPH_ROWPTR);
    if (hipGetLastError() != hipSuccess) return fail(KBISIM_EHIP);
  }
  if (m > 0) {
    k_validate_vals<<<blocks_for(m, 256), 256, 0, c->stream>>>(m, g->col, n, c->err, ERR_GRAPH_COL);
    if (g->elabel) k_validate_vals<<<blocks_for(m, 256), 256, 0, c->stream>>>(m, g->elabel, -1, c->err, ERR_GRAPH_ELABEL);
  }
  if (g->vlabel_ptr) {
    k_validate_rows<<<blocks_for(n + 1, 256), 256, 0, c->stream>>>(n, nl, g->vlabel_ptr, c->err, ERR_GRAPH_VPTR);
    if (nl > 0) k_validate_vals<<<blocks_for(nl, 256), 256, 0, c->stream>>>(nl, g->vlabel, -1, c->err, ERR_GRAPH_VLABEL);
  } else if (g->vlabel && n > 0) {
    k_validate_vals<<<blocks_for(n, 256), 256, 0, c->stream>>>(n, g->vlabel, -1, c->err, ERR_GRAPH_VLABEL);
  }
  if (hipGetLastError() != hipSuccess) return fail(KBISIM_EHIP);
  u32 err = 0;
  if ((rc = read_err(c, &err))) return fail(rc);
  if (err) return fail(KBISIM_EGRAPH);

  // Fresh state: tables and scan status start empty.
  if ((rc = fill_u64(c, c->table, (int64_t)plan.tslots, 0))) return fail(rc);
  if ((rc = fill_u64(c, c->ctable, (int64_t)plan.tslots, 0))) return fail(rc);
  if ((rc = fill_u64(c, c->status, plan.ntiles, 0))) return fail(rc);

  // P0: blocks of equal vertex label sets, numbered by first vertex.
  if (!g->vlabel) {
    if ((rc = fill_i32(c, c->p0, n, 0))) return fail(rc);
    c->p0_count = n > 0 ? 1 : 0;
  } else if (n > 0) {
    Schedule ls;
    if ((rc = build_schedule(c, g->vlabel_ptr, ls))) return fail(rc);
    int *cnt = c->counters + CNT_STRIDE * (plan.ncounter_steps - 2);
    if ((rc = fill_i32(c, cnt, CNT_STRIDE, 0))) return fail(rc);
    LabelSrc src{g->vlabel_ptr, g->vlabel};
    int64_t *dcount = c->dcounts + (plan.ncounter_steps - 2);
    if ((rc = run_step(c, src, ls, c->p0, dcount, cnt, true))) return fail(rc);
    if (hipMemcpyAsync(&c->p0_count, dcount, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return fail(KBISIM_EHIP);
    if ((rc = read_err(c, &err))) return fail(rc);
    if (err) return fail(KBISIM_EINTERNAL);
  }
  // Static schedule of the graph rows.
  if ((rc = build_schedule(c, g->row_ptr, c->sched))) return fail(rc);
  *out = c;
  return KBISIM_OK;
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
  return refine_impl(c, nullptr, k, out_block_ids, out_counts);
}

int kbisim_refine_from(kbisim_ctx *c, const int32_t *pid_i, int k, int32_t *const *out_block_ids,
                       int64_t *out_counts) {
  if (!c || (c->g.n > 0 && !pid_i)) return KBISIM_EINVAL;
  if (c->g.n > 0) {
    int rc0 = fill_i32(c, (int *)c->err, 1, 0);
    if (rc0) return rc0;
    k_validate_vals<<<blocks_for(c->g.n, 256), 256, 0, c->stream>>>(c->g.n, pid_i, -1, c->err, ERR_BAD_PID);
    LAUNCH_CHECK();
    u32 err = 0;
    int rc = read_err(c, &err);
    if (rc) return rc;
    if (err) return KBISIM_EINVAL;
  }
  return refine_impl(c, pid_i, k, out_block_ids, out_counts);
}

int kbisim_destroy(kbisim_ctx *c) {
  delete c;
  return KBISIM_OK;
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

const char *kbisim_version(void) { return "kbisim 0.1 gfx950"; }

}  // extern "C"
