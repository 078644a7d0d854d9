// Device kernels of the k-bisimulation refinement step for gfx950 (CDNA4,
// 64-wide wavefronts).  One refinement step (Def. edge-labeled-fw-bisimulation)
// runs as:
//
//   signature   per vertex v: gather the pairs (edge label, previous block of
//               target) over v's CSR row, remove duplicates (the signature is a
//               SET, Def. signature), and fold the distinct pairs and v's own
//               previous block into a 64-bit key hash.  Degree tiers: a thread
//               per vertex (deg <= 16, in vertex order), a wave per vertex with
//               an LDS hash set (deg <= 512), a workgroup per vertex with a
//               64 KB LDS hash set (deg <= 4096), and hub vertices split over
//               many workgroups sharing a global hash set.
//   group       every vertex inserts (key hash, v) into an open-addressing
//               table that keeps the minimum vertex per key; a lookup gives
//               each vertex its candidate representative.
//   exact check every vertex whose representative is another vertex is
//               compared with it exactly: same previous block, same number of
//               distinct pairs, and every pair of v present in the
//               representative's set.  Hash collisions found here are
//               regrouped by a peeling round (min vertex per hash among the
//               collided vertices, exact check again) until none remain.
//   numbering   representatives are exactly the first vertex of each block;
//               an exclusive scan over "v is its own representative" in
//               vertex order gives dense ids numbered by first vertex, and
//               every other vertex copies its representative's id.
//
// The paper's own block ids are hash values and are only correct without
// collisions; here hashing only accelerates the grouping and every group is
// verified, so the ids are exact.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kb {

typedef unsigned long long u64;
typedef uint32_t u32;

constexpr u64 EMPTY64 = ~0ULL;
constexpr int WAVE = 64;
constexpr int SMALL_MAX = 16;      // thread-per-vertex tier
constexpr int WAVE_MAX = 512;      // wave-per-vertex tier
constexpr int WAVE_SLOTS = 1024;   // LDS set slots per wave (8 KB)
constexpr int BLOCK_MAX = 4096;    // workgroup-per-vertex tier
constexpr int BLOCK_SLOTS = 8192;  // LDS set slots per workgroup (64 KB)
constexpr int HUB_CHUNK = 8192;    // edges per hub workgroup
constexpr int SCAN_ITEMS = 16;     // items per thread in the scan
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;

// Error bits reported through the workspace error word.
constexpr u32 ERR_LOOKUP_MISS = 1u;
constexpr u32 ERR_SPIN = 2u;
constexpr u32 ERR_VERIFY_OVERFLOW = 4u;
constexpr u32 ERR_GRAPH_ROWPTR = 16u;
constexpr u32 ERR_GRAPH_COL = 32u;
constexpr u32 ERR_GRAPH_ELABEL = 64u;
constexpr u32 ERR_GRAPH_VPTR = 128u;
constexpr u32 ERR_GRAPH_VLABEL = 256u;
constexpr u32 ERR_BAD_PID = 512u;

// ---------------------------------------------------------------- hashing
// Murmur3's 64-bit finalizer (Appleby, MurmurHash3, public domain) as the
// mixing function.  The key hash of a vertex is
//   H = fmix64( sum_{p distinct} fmix64(p ^ C1)  +  fmix64((own << 32 | dc) ^ C2) )
// with own = the vertex's previous block and dc = the number of distinct
// pairs.  The sum over distinct pairs makes the hash independent of the order
// in which a row's pairs are met, so no sort is needed to canonicalise.
__host__ __device__ inline u64 fmix64(u64 k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}
__device__ inline u64 mix_pair(u64 p) { return fmix64(p ^ 0x9ae16a3b2f90404fULL); }
__device__ inline u32 set_hash(u64 p) { return (u32)(fmix64(p + 0x2545f4914f6cdd1dULL) >> 32); }
__device__ inline u32 part_hash(u64 p) { return (u32)fmix64(p ^ 0x6a09e667f3bcc909ULL); }
__device__ inline u64 finalize_key(u64 acc, u32 dc, u32 own) {
  return fmix64(acc + fmix64((((u64)own) << 32 | (u64)dc) ^ 0xc2b2ae3d27d4eb4fULL));
}

// ---------------------------------------------------------------- sources
// A source describes, for each vertex, a row of items and how an item maps
// to a 64-bit pair.  GraphSrc is one refinement step: item = CSR entry,
// pair = (edge label << 31) | previous block of the target.  LabelSrc builds
// P0: item = one vertex label, pair = the label.
struct GraphSrc {
  const int64_t *row_ptr;
  const int32_t *col;
  const int32_t *elabel;  // may be null
  const int32_t *pid;     // previous partition
  __device__ inline int64_t begin(int v) const { return row_ptr[v]; }
  __device__ inline int64_t end(int v) const { return row_ptr[v + 1]; }
  __device__ inline u64 pair(int64_t e) const {
    u32 l = elabel ? (u32)elabel[e] : 0u;
    return ((u64)l << 31) | (u64)(u32)pid[col[e]];
  }
  __device__ inline u32 own(int v) const { return (u32)pid[v]; }
};

struct LabelSrc {
  const int64_t *ptr;  // may be null: one label per vertex
  const int32_t *lab;
  __device__ inline int64_t begin(int v) const { return ptr ? ptr[v] : (int64_t)v; }
  __device__ inline int64_t end(int v) const { return ptr ? ptr[v + 1] : (int64_t)v + 1; }
  __device__ inline u64 pair(int64_t e) const { return (u64)(u32)lab[e]; }
  __device__ inline u32 own(int) const { return 0u; }
};

// ---------------------------------------------------------------- wave helpers
__device__ inline u64 wave_sum_u64(u64 x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
  return x;
}
__device__ inline u32 wave_sum_u32(u32 x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
  return x;
}

// Append `item` to list[*counter] for every lane with pred set, one atomic
// per wave.  Works with any subset of active lanes.
__device__ inline void wave_append(int *counter, int *list, bool pred, int item) {
  u64 mask = __ballot(pred);
  if (mask == 0) return;
  int leader = __ffsll((long long)mask) - 1;
  int lane = threadIdx.x & (WAVE - 1);
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader, WAVE);
  if (pred) {
    u64 below = mask & ((1ULL << lane) - 1ULL);
    list[base + __popcll(below)] = item;
  }
}

// ---------------------------------------------------------------- grouping table
// Open addressing with linear probing.  Slot = (tag << 32) | vertex, tag =
// 28 hash bits above bit 36 plus a 4-bit epoch (1..15).  A slot whose epoch is
// not the current one is free, so the table is reused across iterations
// without clearing (it is cleared once every 15 epochs).  Home slot = low
// hash bits.  Every vertex with the same (tag, home) ends in the same slot,
// which holds the minimum such vertex.  Two different keys can share a slot;
// the exact check separates them.
__device__ inline u32 slot_tag(u64 h, u32 epoch) { return ((u32)(h >> 36) << 4) | epoch; }

__device__ inline void table_insert(u64 *table, u64 tmask, u64 h, u32 v, u32 epoch) {
  const u32 tag = slot_tag(h, epoch);
  const u64 want = ((u64)tag << 32) | (u64)v;
  u64 s = h & tmask;
  while (true) {
    u64 cur = __hip_atomic_load(&table[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while ((((u32)(cur >> 32)) & 15u) != epoch) {
      u64 old = atomicCAS(&table[s], cur, want);
      if (old == cur) return;
      cur = old;
    }
    if ((u32)(cur >> 32) == tag) {
      if ((u32)cur > v) atomicMin(&table[s], want);
      return;
    }
    s = (s + 1) & tmask;
  }
}

__device__ inline int table_lookup(const u64 *table, u64 tmask, u64 h, u32 epoch) {
  const u32 tag = slot_tag(h, epoch);
  u64 s = h & tmask;
  while (true) {
    u64 cur = table[s];
    u32 t = (u32)(cur >> 32);
    if (t == tag) return (int)(u32)cur;
    if ((t & 15u) != epoch) return -1;
    s = (s + 1) & tmask;
  }
}

// ---------------------------------------------------------------- validation
__global__ void k_validate_rows(int64_t n, int64_t m, const int64_t *__restrict__ ptr, u32 *err, u32 bit) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  int64_t a = ptr[i];
  bool bad = false;
  if (i == 0 && a != 0) bad = true;
  if (i == n && a != m) bad = true;
  if (i < n && ptr[i + 1] < a) bad = true;
  if (a < 0 || a > m) bad = true;
  if (bad) atomicOr(err, bit);
}

__global__ void k_validate_vals(int64_t cnt, const int32_t *__restrict__ vals, int64_t upper, u32 *err, u32 bit) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  int64_t x = vals[i];
  if (x < 0 || (upper >= 0 && x >= upper)) atomicOr(err, bit);
}

// ---------------------------------------------------------------- classification
// Static degree tiers (degrees never change across iterations).
__global__ void k_classify(int n, const int64_t *__restrict__ ptr, int *cnt, int *list_w, int *list_b,
                           int *list_h) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  bool in = v < n;
  int64_t d = in ? (ptr ? ptr[v + 1] - ptr[v] : 1) : 0;
  wave_append(&cnt[0], list_w, in && d > SMALL_MAX && d <= WAVE_MAX, v);
  wave_append(&cnt[1], list_b, in && d > WAVE_MAX && d <= BLOCK_MAX, v);
  wave_append(&cnt[2], list_h, in && d > BLOCK_MAX, v);
}

// ---------------------------------------------------------------- signature tiers
template <class Src>
__global__ void __launch_bounds__(256) k_sig_small(Src src, int n, u64 *__restrict__ H, u32 *__restrict__ DC,
                                                   u64 *table, u64 tmask, u32 epoch, u64 hmask) {
  __shared__ u64 buf[SMALL_MAX * 256];
  const int t = threadIdx.x;
  const int v = blockIdx.x * 256 + t;
  if (v >= n) return;
  const int64_t b = src.begin(v), e = src.end(v);
  if (e - b > SMALL_MAX) return;
  u64 acc = 0;
  u32 cnt = 0;
  for (int64_t i = b; i < e; ++i) {
    const u64 p = src.pair(i);
    bool dup = false;
    for (u32 j = 0; j < cnt; ++j)
      if (buf[j * 256 + t] == p) { dup = true; break; }
    if (!dup) {
      buf[cnt * 256 + t] = p;
      ++cnt;
      acc += mix_pair(p);
    }
  }
  const u64 h = finalize_key(acc, cnt, src.own(v)) & hmask;
  H[v] = h;
  DC[v] = cnt;
  table_insert(table, tmask, h, (u32)v, epoch);
}

template <class Src>
__global__ void __launch_bounds__(256) k_sig_wave(Src src, const int *__restrict__ list, int count,
                                                  u64 *__restrict__ H, u32 *__restrict__ DC, u64 *table, u64 tmask,
                                                  u32 epoch, u64 hmask) {
  __shared__ u64 sets[4][WAVE_SLOTS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int idx = blockIdx.x * 4 + w;
  u64 *set = sets[w];
  for (int i = threadIdx.x; i < 4 * WAVE_SLOTS; i += 256) (&sets[0][0])[i] = EMPTY64;
  __syncthreads();
  u64 acc = 0;
  u32 cnt = 0;
  int v = -1;
  if (idx < count) {
    v = list[idx];
    const int64_t b = src.begin(v), e = src.end(v);
    for (int64_t i = b + lane; i < e; i += WAVE) {
      const u64 p = src.pair(i);
      u32 s = set_hash(p) & (WAVE_SLOTS - 1);
      while (true) {
        u64 old = atomicCAS(&set[s], EMPTY64, p);
        if (old == EMPTY64) { acc += mix_pair(p); ++cnt; break; }
        if (old == p) break;
        s = (s + 1) & (WAVE_SLOTS - 1);
      }
    }
  }
  acc = wave_sum_u64(acc);
  cnt = wave_sum_u32(cnt);
  if (v >= 0 && lane == 0) {
    const u64 h = finalize_key(acc, cnt, src.own(v)) & hmask;
    H[v] = h;
    DC[v] = cnt;
    table_insert(table, tmask, h, (u32)v, epoch);
  }
}

__device__ inline void block_reduce_2(u64 &acc, u32 &cnt, u64 *sh_acc, u32 *sh_cnt) {
  acc = wave_sum_u64(acc);
  cnt = wave_sum_u32(cnt);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) { sh_acc[w] = acc; sh_cnt[w] = cnt; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 1; i < nw; ++i) { acc += sh_acc[i]; cnt += sh_cnt[i]; }
  }
}

template <class Src>
__global__ void __launch_bounds__(256) k_sig_block(Src src, const int *__restrict__ list, u64 *__restrict__ H,
                                                   u32 *__restrict__ DC, u64 *table, u64 tmask, u32 epoch,
                                                   u64 hmask) {
  __shared__ u64 set[BLOCK_SLOTS];
  __shared__ u64 sh_acc[4];
  __shared__ u32 sh_cnt[4];
  for (int i = threadIdx.x; i < BLOCK_SLOTS; i += 256) set[i] = EMPTY64;
  __syncthreads();
  const int v = list[blockIdx.x];
  const int64_t b = src.begin(v), e = src.end(v);
  u64 acc = 0;
  u32 cnt = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    const u64 p = src.pair(i);
    u32 s = set_hash(p) & (BLOCK_SLOTS - 1);
    while (true) {
      u64 old = atomicCAS(&set[s], EMPTY64, p);
      if (old == EMPTY64) { acc += mix_pair(p); ++cnt; break; }
      if (old == p) break;
      s = (s + 1) & (BLOCK_SLOTS - 1);
    }
  }
  block_reduce_2(acc, cnt, sh_acc, sh_cnt);
  if (threadIdx.x == 0) {
    const u64 h = finalize_key(acc, cnt, src.own(v)) & hmask;
    H[v] = h;
    DC[v] = cnt;
    table_insert(table, tmask, h, (u32)v, epoch);
  }
}

// Hub vertices: the row is split into chunks of HUB_CHUNK entries, one
// workgroup each.  Workgroups of one hub share a global hash set of 2*deg
// slots; slot = pair | (epoch << 62), 0 = never used, epochs 1..3.
struct HubChunk {
  int hub;     // index into the hub arrays
  int pad;
  int64_t b, e;  // entry range relative to the start of the hub's row
};

// floor(a * n / 2^32) for a 32-bit a and any 64-bit n: a slot index in [0, n).
__device__ inline u64 scale_to(u32 a, u64 n) { return __umul64hi(((u64)a) << 32, n); }

template <class Src>
__global__ void __launch_bounds__(256) k_sig_hub(Src src, const HubChunk *__restrict__ chunks,
                                                 const int *__restrict__ hubs, const int64_t *__restrict__ set_off,
                                                 const int64_t *__restrict__ set_size, u64 *sets,
                                                 u64 *hub_acc, u32 *hub_cnt, u32 hepoch) {
  __shared__ u64 sh_acc[4];
  __shared__ u32 sh_cnt[4];
  const HubChunk c = chunks[blockIdx.x];
  u64 *set = sets + set_off[c.hub];
  const u64 size = (u64)set_size[c.hub];
  const int64_t row = src.begin(hubs[c.hub]);
  u64 acc = 0;
  u32 cnt = 0;
  for (int64_t i = row + c.b + threadIdx.x; i < row + c.e; i += 256) {
    const u64 p = src.pair(i);
    const u64 want = p | ((u64)hepoch << 62);
    u64 s = scale_to(set_hash(p), size);
    while (true) {
      u64 cur = __hip_atomic_load(&set[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      bool done = false;
      while ((cur >> 62) != (u64)hepoch) {
        u64 old = atomicCAS(&set[s], cur, want);
        if (old == cur) { acc += mix_pair(p); ++cnt; done = true; break; }
        cur = old;
      }
      if (done || cur == want) break;
      s = (s + 1 == size) ? 0 : s + 1;
    }
  }
  block_reduce_2(acc, cnt, sh_acc, sh_cnt);
  if (threadIdx.x == 0) {
    if (acc) atomicAdd(&hub_acc[c.hub], acc);
    if (cnt) atomicAdd(&hub_cnt[c.hub], cnt);
  }
}

template <class Src>
__global__ void k_hub_final(Src src, const int *__restrict__ hubs, int nhub, u64 *hub_acc, u32 *hub_cnt,
                            u64 *__restrict__ H, u32 *__restrict__ DC, u64 *table, u64 tmask, u32 epoch,
                            u64 hmask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nhub) return;
  const int v = hubs[i];
  const u64 acc = hub_acc[i];
  const u32 cnt = hub_cnt[i];
  hub_acc[i] = 0;
  hub_cnt[i] = 0;
  const u64 h = finalize_key(acc, cnt, src.own(v)) & hmask;
  H[v] = h;
  DC[v] = cnt;
  table_insert(table, tmask, h, (u32)v, epoch);
}

// ---------------------------------------------------------------- lookup + exact check
// For each vertex: representative r = minimum vertex stored under its key.
// r == v: v heads its block.  Otherwise the key of v is compared exactly
// with r's: the previous block, the number of distinct pairs, and (for small
// rows, inline) every pair of v must occur in r's row.  Larger rows go to a
// verification list; mismatches (hash collisions) to the collision list
// with rep = -1.
template <class Src>
__global__ void __launch_bounds__(256) k_lookup(Src src, int n, const u64 *__restrict__ H,
                                                const u32 *__restrict__ DC, const u64 *table, u64 tmask,
                                                u32 epoch, int *__restrict__ rep, int *vcount, int *vlist,
                                                int *ccount, int *clist, u32 *err) {
  __shared__ u64 buf[SMALL_MAX * 256];
  const int t = threadIdx.x;
  const int v = blockIdx.x * 256 + t;
  bool to_verify = false, collided = false;
  if (v < n) {
    const int r = table_lookup(table, tmask, H[v], epoch);
    if (r < 0) {
      atomicOr(err, ERR_LOOKUP_MISS);
      rep[v] = v;
    } else if (r == v) {
      rep[v] = v;
    } else {
      const u32 dcv = DC[v];
      bool ok;
      if (src.own(v) != src.own(r) || dcv != DC[r]) {
        ok = false;
      } else if (dcv == 0) {
        ok = true;
      } else {
        const int64_t bv = src.begin(v), ev = src.end(v);
        const int64_t br = src.begin(r), er = src.end(r);
        if (ev - bv <= SMALL_MAX && er - br <= SMALL_MAX) {
          int nr = 0;
          for (int64_t i = br; i < er; ++i) buf[(nr++) * 256 + t] = src.pair(i);
          ok = true;
          for (int64_t i = bv; i < ev && ok; ++i) {
            const u64 p = src.pair(i);
            bool found = false;
            for (int j = 0; j < nr; ++j)
              if (buf[j * 256 + t] == p) { found = true; break; }
            ok = found;
          }
        } else {
          to_verify = true;
          ok = true;
        }
      }
      if (ok) {
        rep[v] = r;
      } else {
        rep[v] = -1;
        collided = true;
      }
    }
  }
  wave_append(vcount, vlist, to_verify, v);
  wave_append(ccount, clist, collided, v);
}

// Exact set check of v against r with one workgroup: the distinct pairs of r
// go into an LDS hash set (in several passes, split by a partition hash, when
// they do not fit), and every pair of v is looked up.  Result: 1 if every pair
// of v occurs in r's row, 0 if not, -1 if a pass overflowed the LDS set (the
// caller retries with more passes).  Must be called by the whole workgroup.
template <class Src>
__device__ int wg_subset_pass(const Src &src, int v, int r, u32 parts, u64 *set, int *sh_flag) {
  const int64_t bv = src.begin(v), ev = src.end(v);
  const int64_t br = src.begin(r), er = src.end(r);
  for (u32 q = 0; q < parts; ++q) {
    for (int i = threadIdx.x; i < BLOCK_SLOTS; i += blockDim.x) set[i] = EMPTY64;
    if (threadIdx.x == 0) { sh_flag[0] = 1; sh_flag[1] = 0; }
    __syncthreads();
    for (int64_t i = br + threadIdx.x; i < er; i += blockDim.x) {
      const u64 p = src.pair(i);
      if (parts > 1 && (part_hash(p) & (parts - 1)) != q) continue;
      u32 s = set_hash(p) & (BLOCK_SLOTS - 1);
      for (int probes = 0;; ++probes) {
        if (probes >= BLOCK_SLOTS) { sh_flag[1] = 1; break; }
        const u64 old = atomicCAS(&set[s], EMPTY64, p);
        if (old == EMPTY64 || old == p) break;
        s = (s + 1) & (BLOCK_SLOTS - 1);
      }
    }
    __syncthreads();
    const bool overflow = sh_flag[1] != 0;
    if (!overflow) {
      for (int64_t i = bv + threadIdx.x; i < ev; i += blockDim.x) {
        const u64 p = src.pair(i);
        if (parts > 1 && (part_hash(p) & (parts - 1)) != q) continue;
        u32 s = set_hash(p) & (BLOCK_SLOTS - 1);
        bool found = false;
        for (int probes = 0; probes < BLOCK_SLOTS; ++probes) {
          const u64 x = set[s];
          if (x == p) { found = true; break; }
          if (x == EMPTY64) break;
          s = (s + 1) & (BLOCK_SLOTS - 1);
        }
        if (!found) sh_flag[0] = 0;
      }
    }
    __syncthreads();
    const int res = overflow ? -1 : (sh_flag[0] != 0 ? 1 : 0);
    __syncthreads();
    if (res != 1) return res;
  }
  return 1;
}

template <class Src>
__device__ bool wg_subset(const Src &src, int v, int r, u32 dcr, u64 *set, int *sh_flag, u32 *err) {
  u32 parts = 1;
  while ((u64)parts * (BLOCK_SLOTS / 2) < (u64)dcr) parts <<= 1;
  while (true) {
    const int res = wg_subset_pass(src, v, r, parts, set, sh_flag);
    if (res >= 0) return res == 1;
    if (parts >= (1u << 24)) {
      if (threadIdx.x == 0) atomicOr(err, ERR_VERIFY_OVERFLOW);
      return false;
    }
    parts <<= 1;
  }
}

// Persistent: grid-strides over the verification list (count read on device).
template <class Src>
__global__ void __launch_bounds__(256) k_verify(Src src, const int *__restrict__ vcount, const int *__restrict__ vlist,
                                                const u32 *__restrict__ DC, int *__restrict__ rep, int *ccount,
                                                int *clist, u32 *err) {
  __shared__ u64 set[BLOCK_SLOTS];
  __shared__ int sh_flag[2];
  const int total = *vcount;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int v = vlist[item];
    const int r = rep[v];
    const bool ok = wg_subset(src, v, r, DC[r], set, sh_flag, err);
    if (threadIdx.x == 0 && !ok) {
      rep[v] = -1;
      const int at = atomicAdd(ccount, 1);
      clist[at] = v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- collision peeling
// One peeling round over a list of collided vertices: insert (hash, v) into a
// second table (minimum vertex per hash), then check every vertex exactly
// against that minimum.  The minimum itself heads its block; matches join it;
// the rest go to the next round's list.  Every round settles at least one
// block per hash value, so rounds end.
__global__ void k_res_insert(const int *__restrict__ count, const int *__restrict__ list, const u64 *__restrict__ H,
                             u64 *ctable, u64 tmask, u32 epoch) {
  const int total = *count;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int v = list[i];
    table_insert(ctable, tmask, H[v], (u32)v, epoch);
  }
}

template <class Src>
__global__ void __launch_bounds__(256) k_res_verify(Src src, const int *__restrict__ count, const int *__restrict__ list,
                                                    const u64 *__restrict__ H, const u32 *__restrict__ DC,
                                                    const u64 *ctable, u64 tmask, u32 epoch, int *__restrict__ rep,
                                                    int *next_count, int *next_list, u32 *err) {
  __shared__ u64 set[BLOCK_SLOTS];
  __shared__ int sh_flag[2];
  const int total = *count;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int v = list[item];
    const int r = table_lookup(ctable, tmask, H[v], epoch);
    bool ok;
    if (r < 0) {
      if (threadIdx.x == 0) atomicOr(err, ERR_LOOKUP_MISS);
      ok = true;  // leave v as its own block; the error is reported
    } else if (r == v) {
      ok = true;
    } else if (src.own(v) != src.own(r) || DC[v] != DC[r]) {
      ok = false;
    } else if (DC[v] == 0) {
      ok = true;
    } else {
      ok = wg_subset(src, v, r, DC[r], set, sh_flag, err);
    }
    if (threadIdx.x == 0) {
      if (ok) {
        rep[v] = r < 0 ? v : r;
      } else {
        const int at = atomicAdd(next_count, 1);
        next_list[at] = v;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- numbering
// Single-pass exclusive scan with decoupled look-back (Merrill and Garland,
// "Single-pass parallel prefix scan with decoupled look-back", 2016) over the
// flags "rep[v] == v" in vertex order.  A head's prefix is its dense id; the
// last tile writes the block count.  Tile status word: value (32 bits) |
// flag (2 bits: 1 aggregate, 2 inclusive) | stamp (30 bits, unique per scan
// launch, so the status array needs no clearing).
__device__ inline u64 pack_status(u32 value, u32 flag, u32 stamp) {
  return (u64)value | ((u64)flag << 32) | ((u64)stamp << 34);
}

__global__ void __launch_bounds__(256) k_scan(int n, const int *__restrict__ rep, int *__restrict__ out, u64 *status,
                                              int *tile_counter, int64_t *count_out, u32 stamp, u32 *err) {
  __shared__ int sh_tile;
  __shared__ u32 sh_wsum[4];
  __shared__ u32 sh_prefix;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) sh_tile = atomicAdd(tile_counter, 1);
  __syncthreads();
  const int tile = sh_tile;
  const int64_t base = (int64_t)tile * SCAN_TILE + (int64_t)t * SCAN_ITEMS;
  u32 bits = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    const int64_t v = base + j;
    if (v < n && rep[v] == (int)v) bits |= 1u << j;
  }
  const u32 mine = __popc(bits);
  // inclusive wave scan
  u32 x = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    u32 y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh_wsum[w] = x;
  __syncthreads();
  u32 wbase = 0;
  for (int i = 0; i < w; ++i) wbase += sh_wsum[i];
  const u32 tile_total = sh_wsum[0] + sh_wsum[1] + sh_wsum[2] + sh_wsum[3];
  const u32 excl_in_tile = wbase + x - mine;
  if (t == 0) {
    u32 prefix = 0;
    if (tile == 0) {
      __hip_atomic_store(&status[0], pack_status(tile_total, 2u, stamp), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&status[tile], pack_status(tile_total, 1u, stamp), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
      int j = tile - 1;
      long spins = 0;
      while (j >= 0) {
        const u64 s = __hip_atomic_load(&status[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const u32 f = (u32)(s >> 32) & 3u;
        if ((u32)(s >> 34) != stamp || f == 0) {
          if (++spins > (1L << 28)) { atomicOr(err, ERR_SPIN); break; }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        prefix += (u32)s;
        if (f == 2u) break;
        --j;
      }
      __hip_atomic_store(&status[tile], pack_status(prefix + tile_total, 2u, stamp), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    sh_prefix = prefix;
    const int64_t ntiles = ((int64_t)n + SCAN_TILE - 1) / SCAN_TILE;
    if (tile == ntiles - 1) *count_out = (int64_t)prefix + tile_total;
  }
  __syncthreads();
  u32 id = sh_prefix + excl_in_tile;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    if (bits & (1u << j)) out[base + j] = (int)id++;
  }
}

// Every non-head copies its representative's id (written by k_scan).
__global__ void k_assign(int n, const int *__restrict__ rep, int *out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int r = rep[v];
  if (r != v) out[v] = r >= 0 ? out[r] : -1;
}

// ---------------------------------------------------------------- utilities
__global__ void k_fill_u64(u64 *p, int64_t cnt, u64 val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}
__global__ void k_fill_i32(int *p, int64_t cnt, int val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}
__global__ void k_copy_i32(int *dst, const int *src, int64_t cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
// Degrees of the hub list (for host-side chunking at create time).
__global__ void k_hub_degrees(const int *hubs, int nhub, const int64_t *ptr, int64_t *deg_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nhub) {
    const int v = hubs[i];
    deg_out[i] = ptr ? ptr[v + 1] - ptr[v] : 1;
  }
}

}  // namespace kb
