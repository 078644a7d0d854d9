// Device kernels of the k-bisimulation refinement step for gfx950 (CDNA4,
// 64-wide wavefronts).  One refinement step (Def. edge-labeled-fw-bisimulation)
// runs as:
//
//   signature   per vertex v: gather the pairs (edge label, previous block of
//               target) over v's CSR row, remove duplicates (the signature is a
//               SET, Def. signature), and fold the distinct pairs and v's own
//               previous block into a 64-bit key hash.  Degree tiers, fixed at
//               create time: runs of consecutive low-degree vertices share a
//               workgroup and an LDS hash set (range tier, at most 1024 or
//               2048 entries per run), a row of up to 4096 entries gets a
//               workgroup of its own, and hub rows are split into chunks that
//               are deduplicated in two passes (chunk, then partition), or,
//               beyond 4M entries, through a global hash set.
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
constexpr int SMALL_MAX = 16;        // inline exact check limit (thread per vertex)
constexpr int RANGE_EDGES = 1024;    // CSR entries per multi-vertex range workgroup (or 2048)
constexpr int RANGE_VERTS = 256;     // vertices per range workgroup
constexpr int RANGE_DMAX = 4096;     // rows above RANGE_EDGES get a workgroup of 512 threads
constexpr int ROW_MAX = 8192;        // rows above RANGE_DMAX get one of 1024 threads; above this, hubs
constexpr int ROW_MAX_NARROW = 19456;  // with 32-bit keys rows up to this fit one workgroup's LDS (152 KB)
constexpr int BLOCK_MAX = ROW_MAX;
constexpr int BLOCK_SLOTS = 8192;    // LDS set slots for exact checks (64 KB)
constexpr int HUB_CHUNK_MAX = 4096;  // entries per hub staging workgroup: 2048 (default) or 4096
constexpr int HUB_PMAX = 1024;       // partitions per hub at most
constexpr int HUB_PART_TARGET = 2048;  // expected entries per hub partition
// LDS set slots per hub partition workgroup, and the largest staged hub (a
// larger one uses a global hash set): a partition then expects at most half
// as many distinct keys as its set has slots.  64-bit keys take half the
// slots (and half the staged hub size), so three workgroups fit a CU
// instead of two.
constexpr int HUB_PSLOTS = 8192;
constexpr int HUB_PSLOTS_WIDE = 4096;
constexpr int64_t HUB_STAGED_MAX = (int64_t)HUB_PMAX * HUB_PSLOTS / 2;
constexpr int64_t HUB_STAGED_MAX_WIDE = (int64_t)HUB_PMAX * HUB_PSLOTS_WIDE / 2;
constexpr int HUB_GCHUNK = 8192;     // entries per workgroup in the global-set path
constexpr int SCAN_ITEMS = 16;       // items per thread in the 64-bit offset scans (and the numbering, by default)
constexpr int SCAN_TILE = 256 * SCAN_ITEMS;
constexpr int SCAN_ITEMS_MIN = 8;    // smallest tunable items per thread of the numbering scan

// Device-resident epoch state (read by kernels at launch, advanced by
// k_advance), so a captured sequence of steps can be replayed.
constexpr int EP_TABLE = 0;    // grouping table epoch, 1..15
constexpr int EP_CTABLE = 1;   // peeling table epoch, 1..15
constexpr int EP_ZERO = 2;     // empty-signature epoch, increasing
constexpr int EP_HUB = 3;      // global hub set epoch, 1..3
constexpr int EP_CLR_TABLE = 4, EP_CLR_CTABLE = 5, EP_CLR_HUB = 6;
constexpr u32 ADV_TABLE = 1, ADV_CTABLE = 2, ADV_ZERO = 4, ADV_HUB = 8;

// Error bits reported through the workspace error word.
constexpr u32 ERR_LOOKUP_MISS = 1u;
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
// Slot position inside LDS hash sets: two 32-bit multiplies and a shift
// (the sets need spread, not collision resistance; equality is exact).
__device__ inline u32 set_hash(u64 p) {
  const u32 h = (u32)p * 0x9E3779B1u ^ ((u32)(p >> 32) + 0x7F4A7C15u) * 0x85EBCA77u;
  return h ^ (h >> 15);
}
__device__ inline u32 part_hash(u64 p) { return (u32)fmix64(p ^ 0x6a09e667f3bcc909ULL); }
__device__ inline u32 sub_hash(u64 p) { return (u32)(fmix64(p ^ 0xa0761d6478bd642fULL) >> 32); }
// Hashed 32-bit set key of a 64-bit pair (bits 16..47 of a Murmur3 fmix64);
// never the empty marker 0xFFFFFFFF.
__device__ inline u32 pair_key32(u64 p) {
  const u32 k = (u32)(fmix64(p ^ 0x3c6ef372fe94f82bULL) >> 16);
  return k == 0xFFFFFFFFu ? 0xFFFFFFFEu : k;
}
__device__ inline u64 finalize_key(u64 acc, u32 dc, u32 own) {
  return fmix64(acc + fmix64((((u64)own) << 32 | (u64)dc) ^ 0xc2b2ae3d27d4eb4fULL));
}

// ---------------------------------------------------------------- sources
// A source describes, for each vertex, a row of items and how an item maps
// to a 64-bit pair.  GraphSrc is one refinement step: item = CSR entry,
// pair = (edge label << 31) | previous block of the target.  LabelSrc builds
// P0: item = one vertex label, pair = the label.
// Gathers read the previous partition through a renumbered copy: gcol[e] =
// rank(col[e]) and gpid[rank(w)] = pid[w], where ranks order vertices by
// decreasing in-degree.  The targets most edges point to then share cache
// lines, which roughly halves the cost of the per-entry random gather.
// SEP: edge labels come from their own array (elabel); otherwise they sit
// above the rank in gcol (or there are none), and elabel is unused.
// HK: 32-bit set keys are a hash of the pair (used when the label and the
// reduced block do not fit 31 bits together); see key32_of.
template <bool SEP, bool HK = false>
struct GraphSrcT {
  static constexpr bool GRAPH = true;
  static constexpr bool HASHED = HK;
  const int64_t *row_ptr;
  const int32_t *gcol;    // targets renumbered by in-degree rank (and, packed, their labels)
  const int32_t *elabel;  // the labels when SEP
  const int32_t *gpid;    // previous partition in rank order
  const int32_t *pid;     // previous partition in vertex order
  __device__ inline int64_t begin(int v) const { return row_ptr[v]; }
  __device__ inline int64_t end(int v) const { return row_ptr[v + 1]; }
  // low word of begin(v): enough for offsets within a range (little endian)
  __device__ inline u32 begin_lo(int v) const { return reinterpret_cast<const u32 *>(row_ptr)[2 * (int64_t)v]; }
  // A pair keeps the target's block id modulo 2^pb.  The targets of one row
  // lie in one graph, whose block ids form an interval of at most 2^pb ids
  // (pb covers the largest graph; a single graph: all ids), so the reduction
  // is one-to-one within a row, and every kernel reduces the same way.
  u32 pb;
  // gcol[e] = (label << rbits) | rank when labels are packed (rbits < 31);
  // otherwise rbits = 31 and the label comes from elabel (SEP) or is 0.
  // Packing halves the streamed bytes per entry.
  u32 rbits;
  // bits kept of hashed keys (all but for tests that make key collisions routine)
  u32 kmask = 0xFFFFFFFFu;
  __device__ inline u32 hkey(u64 p) const { return pair_key32(p) & kmask; }
  __device__ inline u32 pmask() const { return pb >= 31 ? 0x7FFFFFFFu : (1u << pb) - 1u; }
  // (label, rank of the target) of entry e; streamed arrays are read
  // non-temporally so they do not evict the gather targets from the L2
  __device__ inline void entry(int64_t e, u32 &l, u32 &r) const {
    const u32 g = (u32)__builtin_nontemporal_load(&gcol[e]);
    if constexpr (SEP) l = (u32)__builtin_nontemporal_load(&elabel[e]);
    else l = g >> rbits;
    r = g & ((1u << rbits) - 1u);
  }
  // entry() for first + min(t + u*STRIDE, count - 1), u < U: all the
  // streamed words are requested together, with no branch among them
  template <int U, int STRIDE>
  __device__ inline void entries(int64_t first, int t, int count, u32 (&l)[U], u32 (&r)[U]) const {
    const u32 rm = (1u << rbits) - 1u;
    if constexpr (SEP) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = first + min(t + u * STRIDE, count - 1);
        r[u] = (u32)__builtin_nontemporal_load(&gcol[e]);
        l[u] = (u32)__builtin_nontemporal_load(&elabel[e]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] &= rm;
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = (u32)__builtin_nontemporal_load(&gcol[first + min(t + u * STRIDE, count - 1)]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        l[u] = r[u] >> rbits;
        r[u] &= rm;
      }
    }
  }
  // the pair of an entry whose (label, rank) entry() has read: one gather
  __device__ inline u64 pair_of(u32 l, u32 r) const { return ((u64)l << 31) | (u64)((u32)gpid[r] & pmask()); }
  __device__ inline u64 pair(int64_t e) const {
    u32 l, r;
    entry(e, l, r);
    return pair_of(l, r);
  }
  __device__ inline u32 own(int v) const { return (u32)pid[v]; }
  // Narrow form of a pair, used inside LDS sets.  When every edge label and
  // reduced block id fit together in 31 bits it is exact: (label << pb) |
  // block.  Otherwise (HK) it is a 32-bit hash of the pair.  Deduplicating
  // and summing hashed keys gives a function of the signature (equal pair
  // sets give equal key sets), so equal signatures still get equal key
  // hashes; the distinct count is then the number of distinct keys, and the
  // exact check compares pair sets in both directions (a key collision
  // inside a row could otherwise make a proper subset look equal).
  __device__ inline u32 key32_of(u32 l, u32 r) const {
    if constexpr (HK) return hkey(pair_of(l, r));
    else return (l << pb) | ((u32)gpid[r] & pmask());
  }
  __device__ inline u32 key32(int64_t e) const {
    u32 l, r;
    entry(e, l, r);
    return key32_of(l, r);
  }
  // The value a distinct narrow key contributes to the key-hash sum: the
  // pair itself for exact keys (so every tier mixes the same values), the
  // key for hashed ones.
  __device__ inline u64 mixin(u32 q) const {
    if constexpr (HK) return (u64)q;
    else return ((u64)(q >> pb) << 31) | (u64)(q & pmask());
  }
};

struct LabelSrc {
  static constexpr bool GRAPH = false;
  static constexpr bool HASHED = false;
  const int64_t *ptr;  // may be null: one label per vertex
  const int32_t *lab;
  const int32_t *gid;  // may be null; in a batch, the graph of each vertex (P0 never joins graphs)
  __device__ inline int64_t begin(int v) const { return ptr ? ptr[v] : (int64_t)v; }
  __device__ inline int64_t end(int v) const { return ptr ? ptr[v + 1] : (int64_t)v + 1; }
  __device__ inline u32 begin_lo(int v) const {
    return ptr ? reinterpret_cast<const u32 *>(ptr)[2 * (int64_t)v] : (u32)v;
  }
  __device__ inline u64 pair(int64_t e) const { return (u64)(u32)lab[e]; }
  __device__ inline void entry(int64_t e, u32 &l, u32 &r) const {
    l = (u32)lab[e];
    r = 0;
  }
  template <int U, int STRIDE>
  __device__ inline void entries(int64_t first, int t, int count, u32 (&l)[U], u32 (&r)[U]) const {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      l[u] = (u32)lab[first + min(t + u * STRIDE, count - 1)];
      r[u] = 0;
    }
  }
  __device__ inline u64 pair_of(u32 l, u32) const { return (u64)l; }
  __device__ inline u32 own(int v) const { return gid ? (u32)gid[v] : 0u; }
};

// LDS set keys: the 64-bit pair itself, or the narrow 32-bit form.
template <class K>
struct Keys;
template <>
struct Keys<u64> {
  static constexpr u64 EMPTY = EMPTY64;
  template <class Src>
  __device__ static inline u64 load(const Src &s, int64_t e) { return s.pair(e); }
  template <class Src>
  __device__ static inline u64 from(const Src &s, u32 l, u32 r) { return s.pair_of(l, r); }
  template <class Src>
  __device__ static inline u64 mixin(const Src &, u64 p) { return p; }
  __device__ static inline u32 hash(u64 p) { return set_hash(p); }
};
template <>
struct Keys<u32> {
  static constexpr u32 EMPTY = 0xFFFFFFFFu;
  template <class Src>
  __device__ static inline u32 load(const Src &s, int64_t e) { return s.key32(e); }
  template <class Src>
  __device__ static inline u32 from(const Src &s, u32 l, u32 r) { return s.key32_of(l, r); }
  template <class Src>
  __device__ static inline u64 mixin(const Src &s, u32 q) { return s.mixin(q); }
  __device__ static inline u32 hash(u32 q) {
    const u32 h = q * 0x9E3779B1u;
    return h ^ (h >> 15);
  }
};

// Load the keys of entries first + j*STRIDE (j = 0..U-1, only those below
// count are valid; the others become EMPTY).  All streamed words are
// requested before any gather, and no load sits under a branch, so a wave
// waits twice in all instead of twice per entry.  Invalid slots re-read the
// last valid entry (count >= 1 is required).
template <class K, int U, int STRIDE, class Src>
__device__ inline void load_keys(const Src &src, int64_t first, int t, int count, K (&out)[U]) {
  typedef Keys<K> KO;
  u32 l[U], r[U];
  src.template entries<U, STRIDE>(first, t, count, l, r);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const K p = KO::from(src, l[u], r[u]);
    out[u] = t + u * STRIDE < count ? p : KO::EMPTY;
  }
}

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

// Append v0 + j for every bit j of each lane's mask to list[*counter], one
// atomic per wave.  Must be called by the whole wave.
__device__ inline void wave_append_mask(int *counter, int *list, u32 mask, int64_t v0) {
  const int lane = threadIdx.x & (WAVE - 1);
  const u32 c = (u32)__popc(mask);
  u32 x = c;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const u32 y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  const u32 total = __shfl(x, WAVE - 1, WAVE);
  if (total == 0) return;
  int base = 0;
  if (lane == WAVE - 1) base = atomicAdd(counter, (int)total);
  base = __shfl(base, WAVE - 1, WAVE);
  int at = base + (int)(x - c);
  while (mask) {
    const int j = __ffs(mask) - 1;
    list[at++] = (int)(v0 + j);
    mask &= mask - 1u;
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
    // A plain load may return an older value of the slot (empty, or a larger
    // minimum); every decision taken on it is re-validated by the atomics, so
    // hot keys are served from the L1 instead of serialising on one L2 line.
    u64 cur = table[s];
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

// Vertices with an empty signature (no out-edges, or no labels in P0) are
// grouped exactly by their previous block alone: zrep[block] keeps
// (~epoch << 32 | min vertex), so entries of older epochs compare larger and
// are replaced, and no clearing is needed.  No hash and no check involved.
__device__ inline void zero_insert(u64 *zrep, u32 own, u32 v, u32 zep) {
  const u64 want = ((u64)(~zep) << 32) | (u64)v;
  const u64 cur = zrep[own];  // may be stale; atomicMin decides
  if (cur > want) atomicMin(&zrep[own], want);
}

__device__ inline void key_insert(u64 *table, u64 tmask, u64 *zrep, u64 h, u32 dc, u32 own, u32 v, u32 epoch,
                                  u32 zep) {
  if (dc == 0) zero_insert(zrep, own, v, zep);
  else table_insert(table, tmask, h, v, epoch);
}

// zero_insert for the lanes with pred set, one atomic per distinct block in
// the wave (device-wide atomics on one address serialise, and empty
// signatures share few blocks).  Must be reached by the whole wave.
__device__ inline void zero_insert_wave(u64 *zrep, bool pred, u32 own, u32 v, u32 zep) {
  const int lane = threadIdx.x & (WAVE - 1);
  u64 pending = __ballot(pred);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const u32 lo = __shfl(own, leader, WAVE);
    const bool mine = pred && own == lo;
    u32 mv = mine ? v : 0xFFFFFFFFu;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mv = min(mv, (u32)__shfl_xor(mv, o, WAVE));
    if (lane == leader) zero_insert(zrep, lo, mv, zep);
    pending &= ~__ballot(mine);
    pred = pred && !mine;
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

// Largest value of a non-negative array (atomicMax into *out, which starts at 0).
__global__ void k_max_i32(int64_t cnt, const int32_t *__restrict__ vals, u32 *out) {
  u32 mx = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    mx = max(mx, (u32)vals[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (u32)__shfl_xor(mx, o, WAVE));
  if ((threadIdx.x & (WAVE - 1)) == 0 && mx) atomicMax(out, mx);
}

// Range check of cnt values: any value < 0, or >= upper when upper >= 0, sets
// `bit` in *err.  Grid-stride over the 16-byte-aligned body of the array (the
// few values before and after it one by one), 4 groups of 4 values in flight
// per thread, one atomic per wave that found a bad value.
constexpr int VALIDATE_GRID = 4096;
typedef u32 u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_validate_vals(int64_t cnt, const int32_t *__restrict__ vals, int64_t upper,
                                                       u32 *err, u32 bit) {
  // negative values become >= 2^31 as unsigned: one compare covers both ends
  const u32 lim = (upper >= 0 && upper < 0x80000000ll) ? (u32)upper : 0x80000000u;
  const uintptr_t a = reinterpret_cast<uintptr_t>(vals);
  const int64_t head = (a & 3) ? cnt : std::min<int64_t>(cnt, (int64_t)(((16 - (a & 15)) & 15) >> 2));
  const int64_t ng = (cnt - head) >> 2;
  const u32x4 *__restrict__ g4 = reinterpret_cast<const u32x4 *>(vals + head);
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t gt = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool bad = false;
  int64_t i = gt;
  for (; i + 3 * stride < ng; i += 4 * stride) {
    u32x4 q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = __builtin_nontemporal_load(&g4[i + j * stride]);
#pragma unroll
    for (int j = 0; j < 4; ++j) bad |= (q[j].x >= lim) | (q[j].y >= lim) | (q[j].z >= lim) | (q[j].w >= lim);
  }
  for (; i < ng; i += stride) {
    const u32x4 q = __builtin_nontemporal_load(&g4[i]);
    bad |= (q.x >= lim) | (q.y >= lim) | (q.z >= lim) | (q.w >= lim);
  }
  for (int64_t t = gt; t < head; t += stride) bad |= (u32)vals[t] >= lim;
  for (int64_t t = head + (ng << 2) + gt; t < cnt; t += stride) bad |= (u32)vals[t] >= lim;
  if (__ballot(bad) && (threadIdx.x & (WAVE - 1)) == 0) atomicOr(err, bit);
}

// ---------------------------------------------------------------- signature tiers
// A run of consecutive vertices [v0, v1) handled by one workgroup, with the
// run's first entry e0 and its entry count ne, so that a workgroup requests
// its entries without waiting for the row offsets.
struct Range {
  int v0, v1;
  int ne, pad;
  int64_t e0;
};

__device__ inline u64 scale_to(u32 a, u64 n) { return __umul64hi(((u64)a) << 32, n); }

// Exclusive block scan (256 threads) of one u32 per thread; returns the
// thread's prefix and writes the block total to *total.
__device__ inline u32 block_exclusive_scan(u32 mine, u32 *sh_w, u32 *total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  u32 x = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const u32 y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh_w[w] = x;
  __syncthreads();
  u32 base = 0;
  for (int i = 0; i < w; ++i) base += sh_w[i];
  *total = sh_w[0] + sh_w[1] + sh_w[2] + sh_w[3];
  __syncthreads();
  return base + x - mine;
}

// Sum over the workgroup; the result is valid in thread 0.  sh_acc and
// sh_cnt hold one slot per wave.
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

// Range tier: a workgroup takes a run of consecutive vertices holding at most
// EMAX entries (the range capacity, 1024 or 2048) and RANGE_VERTS vertices;
// longer rows go to the row tier.  All entries are gathered at once (EMAX/256
// per thread, loads issued before dependent work, consecutive entries on
// consecutive lanes), then inserted into their vertex's region of an LDS hash
// set (2*deg slots at offset 2*row offset); sums are formed from the set.
// SKIP (work-efficient mode): rows of vertices flagged in skip[] (singleton
// blocks, which cannot split) are left out; the remaining rows are packed,
// so their entries are gathered only after the owner scan.
template <class Src, int EMAX, class K = u64, bool SKIP = false>
__global__ void __launch_bounds__(256) k_sig_range(Src src, const Range *__restrict__ ranges, u64 *__restrict__ H,
                                                   u32 *__restrict__ DC, u64 *table, u64 tmask,
                                                   const u32 *__restrict__ dep, u64 hmask, u64 *zrep, int zfresh,
                                                   const unsigned char *__restrict__ skip) {
  typedef Keys<K> KO;
  constexpr int U = EMAX / 256;
  const u32 epoch = dep[EP_TABLE], zep = dep[EP_ZERO];
  __shared__ K set[2 * EMAX];
  __shared__ u64 acc[RANGE_VERTS];
  __shared__ u32 cnt[RANGE_VERTS];
  __shared__ int roff[RANGE_VERTS + 1];  // CSR row offsets, relative to the range
  __shared__ int coff[SKIP ? RANGE_VERTS + 1 : 1];  // packed offsets (skipped rows empty)
  __shared__ unsigned char owner[EMAX];
  __shared__ u32 wmax[4];
  __shared__ u64 sh_acc[4];
  __shared__ u32 sh_cnt[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const Range rg = ranges[blockIdx.x];
  const int V = rg.v1 - rg.v0;
  const bool single = V == 1;
  const int64_t eb = rg.e0;
  // The addresses of the row offsets, this thread's previous block (V <=
  // blockDim) and the streamed words need only the range, so all three are
  // requested together; the gathers follow, and the offsets reach LDS last.
  const u32 b0 = t <= V ? src.begin_lo(rg.v0 + t) : 0u;
  const u32 b1 = t + 256 <= V ? src.begin_lo(rg.v0 + t + 256) : 0u;
  const u32 own_t = t < V ? src.own(rg.v0 + t) : 0u;
  u32 el[U], er[U];
  if constexpr (!SKIP)
    if (rg.ne > 0) src.template entries<U, 256>(eb, t, rg.ne, el, er);
  K pr[U];
#pragma unroll
  for (int u = 0; u < U; ++u) pr[u] = KO::EMPTY;
  if constexpr (!SKIP) {
    if (rg.ne > 0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const K p = KO::from(src, el[u], er[u]);
        pr[u] = t + u * 256 < rg.ne ? p : KO::EMPTY;
      }
    }
  }
  if (t <= V) roff[t] = (int)(b0 - (u32)eb);
  if (t + 256 <= V) roff[t + 256] = (int)(b1 - (u32)eb);
  for (int i = t; i < V; i += 256) {
    acc[i] = 0;
    cnt[i] = 0;
  }
  if (!single)
    for (int i = t; i < EMAX; i += 256) owner[i] = 0;
  __syncthreads();
  const int *off = roff;  // offsets that place entries and set regions
  bool skipped = false;   // this thread's vertex (t < V) is left out
  if constexpr (SKIP) {
    skipped = t < V && skip[rg.v0 + t];
    const u32 d = (t < V && !skipped) ? (u32)(roff[t + 1] - roff[t]) : 0u;
    u32 total;
    const u32 ex = block_exclusive_scan(d, wmax, &total);
    if (t < V) coff[t] = (int)ex;
    if (t == 0) coff[V] = (int)total;
    __syncthreads();
    off = coff;
  }
  const int E = off[V];
  for (int i = t; i < 2 * E; i += 256) set[i] = KO::EMPTY;
  // the row start of every non-empty vertex marks its index; a max-scan then
  // gives the owner of every entry
  if (!single)
    for (int i = t; i < V; i += 256)
      if (off[i + 1] > off[i]) owner[off[i]] = (unsigned char)i;
  __syncthreads();
  if (!single) {
    constexpr int PER = EMAX / 256;
    u32 run = 0;
    const int j0 = t * PER;
#pragma unroll
    for (int k = 0; k < PER; ++k) run = max(run, (u32)owner[j0 + k]);
    u32 x = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const u32 y = __shfl_up(x, o, WAVE);
      if (lane >= o) x = max(x, y);
    }
    if (lane == 63) wmax[w] = x;
    __syncthreads();
    u32 carry = __shfl_up(x, 1, WAVE);
    if (lane == 0) carry = 0;
    for (int i = 0; i < w; ++i) carry = max(carry, wmax[i]);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      carry = max(carry, (u32)owner[j0 + k]);
      owner[j0 + k] = (unsigned char)carry;
    }
    __syncthreads();
  }
  if constexpr (SKIP) {
    // packed entry j of row lo sits at CSR offset roff[lo] + (j - coff[lo])
    u32 l[U], r[U];
    if (E > 0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = min(t + u * 256, E - 1);
        const int lo = single ? 0 : owner[j];
        src.entry(eb + roff[lo] + (j - coff[lo]), l[u], r[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      K p = KO::EMPTY;
      if (E > 0) p = KO::from(src, l[u], r[u]);
      pr[u] = t + u * 256 < E ? p : KO::EMPTY;
    }
  }
  if (single) {
    // one row: thread-local sums, one block reduction
    u64 a = 0;
    u32 c = 0;
    const u32 sz = 2u * (u32)E;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const K p = pr[u];
      if (p == KO::EMPTY) continue;
      u32 sl = (u32)scale_to(KO::hash(p), sz);
      while (true) {
        const K old = atomicCAS(&set[sl], KO::EMPTY, p);
        if (old == KO::EMPTY) { a += mix_pair(KO::mixin(src, p)); ++c; break; }
        if (old == p) break;
        sl = (sl + 1 == sz) ? 0u : sl + 1;
      }
    }
    block_reduce_2(a, c, sh_acc, sh_cnt);
    bool out = t == 0 && (c || zfresh);
    if constexpr (SKIP) out = out && !skip[rg.v0];
    if (out) {
      const int v = rg.v0;
      const u32 own = own_t;
      const u64 h = finalize_key(a, c, own) & hmask;
      H[v] = h;
      DC[v] = c;
      key_insert(table, tmask, zrep, h, c, own, (u32)v, epoch, zep);
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = t + u * 256;
    if (j < E) {
      const int lo = owner[j];
      const K p = pr[u];
      const int base = 2 * off[lo];
      const u32 sz = 2u * (u32)(off[lo + 1] - off[lo]);
      u32 sl = (u32)scale_to(KO::hash(p), sz);
      while (true) {
        const K old = atomicCAS(&set[base + sl], KO::EMPTY, p);
        if (old == KO::EMPTY || old == p) break;
        sl = (sl + 1 == sz) ? 0u : sl + 1;
      }
    }
  }
  __syncthreads();
  // Sums from the set: thread t reads the 2U consecutive slots from 2Ut on;
  // slot s lies in the region of vertex owner[s / 2].  Runs of one vertex are
  // summed in registers and added to the vertex once per run, so the shared
  // accumulators see a few atomics per vertex instead of one per pair.  Each
  // lane starts at a different slot of its 2U (rotation by lane / (64 / 2U)),
  // so the lanes of one read fall in different LDS banks instead of the few
  // that a stride of 2U words allows; the order of a sum does not matter,
  // and the rotation breaks at most one run.
  {
    constexpr int SL = 2 * U, GRP = WAVE / SL > 0 ? WAVE / SL : 1;
    const int rot = (lane / GRP) & (SL - 1);
    u64 a = 0;
    u32 c = 0;
    int cur = -1;
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      const int sidx = SL * t + ((q + rot) & (SL - 1));
      if (sidx < 2 * E) {
        const int lo = owner[sidx >> 1];
        if (lo != cur) {
          if (c) {
            atomicAdd(&acc[cur], a);
            atomicAdd(&cnt[cur], c);
          }
          cur = lo;
          a = 0;
          c = 0;
        }
        const K p = set[sidx];
        if (p != KO::EMPTY) {
          a += mix_pair(KO::mixin(src, p));
          ++c;
        }
      }
    }
    if (c) {
      atomicAdd(&acc[cur], a);
      atomicAdd(&cnt[cur], c);
    }
  }
  __syncthreads();
  // V <= RANGE_VERTS = blockDim: one vertex per thread.  Vertices with an
  // empty signature keep their representative from the call's first step
  // unless zfresh (their classes never change within a call).
  bool zero = false;
  u32 own = 0;
  const int v = rg.v0 + t;
  if (t < V && !skipped) {
    const u32 c = cnt[t];
    own = own_t;
    if (c) {
      const u64 h = finalize_key(acc[t], c, own) & hmask;
      H[v] = h;
      table_insert(table, tmask, h, (u32)v, epoch);
    } else if (zfresh) {
      zero = true;
    }
    DC[v] = c;
  }
  zero_insert_wave(zrep, zero, own, (u32)v, zep);
}

// Row tier: one workgroup of NT threads per row of more entries than the
// range capacity and at most EMAX.  All entries are gathered at once (EMAX / NT per thread), then
// inserted into an LDS hash set of 2 * deg slots; first insertions add to
// thread-local sums, reduced over the workgroup at the end.
template <class Src, int EMAX, int NT, class K = u64>
__global__ void __launch_bounds__(NT) k_sig_row(Src src, const Range *__restrict__ rows, u64 *__restrict__ H,
                                                u32 *__restrict__ DC, u64 *table, u64 tmask,
                                                const u32 *__restrict__ dep, u64 hmask, u64 *zrep,
                                                const unsigned char *__restrict__ skip) {
  typedef Keys<K> KO;
  constexpr int U = EMAX / NT;
  __shared__ K set[2 * EMAX];
  __shared__ u64 sh_acc[NT / WAVE];
  __shared__ u32 sh_cnt[NT / WAVE];
  const int t = threadIdx.x;
  const Range rw = rows[blockIdx.x];
  const int v = rw.v0;
  if (skip && skip[v]) return;  // singleton block (work-efficient mode)
  const int64_t eb = rw.e0;
  const u32 own0 = t == 0 ? src.own(v) : 0u;  // fetched early, used by thread 0 at the end
  const int E = rw.ne;
  for (int i = t; i < 2 * E; i += NT) set[i] = KO::EMPTY;
  K pr[U];
  if (E > 0) {
    load_keys<K, U, NT>(src, eb, t, E, pr);
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) pr[u] = KO::EMPTY;
  }
  __syncthreads();
  u64 a = 0;
  u32 c = 0;
  const u32 sz = 2u * (u32)E;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const K p = pr[u];
    if (p == KO::EMPTY) continue;
    u32 sl = (u32)scale_to(KO::hash(p), sz);
    while (true) {
      const K old = atomicCAS(&set[sl], KO::EMPTY, p);
      if (old == KO::EMPTY) { a += mix_pair(KO::mixin(src, p)); ++c; break; }
      if (old == p) break;
      sl = (sl + 1 == sz) ? 0u : sl + 1;
    }
  }
  block_reduce_2(a, c, sh_acc, sh_cnt);
  if (t == 0) {
    const u64 h = finalize_key(a, c, own0) & hmask;
    H[v] = h;
    DC[v] = c;
    key_insert(table, tmask, zrep, h, c, own0, (u32)v, dep[EP_TABLE], dep[EP_ZERO]);
  }
}

// Hub tier (deg > BLOCK_MAX), two passes without per-entry global atomics.
//  stage:  a workgroup per chunk of hub_chunk entries removes duplicates
//          inside the chunk (LDS set), splits the chunk's distinct pairs into
//          the hub's P partitions by a partition hash and writes them,
//          grouped by partition, to the chunk's staging area together with
//          the P+1 partition offsets.
//  reduce: a workgroup per (hub, partition) reads that partition's segment
//          of every chunk of the hub, removes duplicates across chunks (LDS
//          set) and adds its distinct count and mix sum to the hub's totals.
struct HubChunk {
  int hub;          // index into the hub arrays
  int parts;        // partitions of this hub (power of two)
  int64_t b, e;     // entry range relative to the start of the hub's row
  int64_t stage;    // offset of the chunk's staging area (hub_chunk slots)
  int64_t poff;     // offset of the chunk's parts+1 partition offsets
};

struct HubPart {
  int hub;
  int part;
  int chunk0;       // first chunk of the hub
  int nchunks;
};

template <class Src, int CHUNK, class K = u64>
__global__ void __launch_bounds__(256) k_hub_stage(Src src, const HubChunk *__restrict__ chunks,
                                                   const int *__restrict__ hubs, K *__restrict__ stage,
                                                   int *__restrict__ poff, u32 *err,
                                                   const unsigned char *__restrict__ skip) {
  typedef Keys<K> KO;
  constexpr int HUB_U = CHUNK / 256;
  __shared__ K set[2 * CHUNK];
  __shared__ int hist[HUB_PMAX + 1];
  __shared__ int wtot[4];
  const HubChunk c = chunks[blockIdx.x];
  if (skip && skip[hubs[c.hub]]) return;  // singleton block (work-efficient mode)
  const int P = c.parts;
  const int64_t row = src.begin(hubs[c.hub]);
  const int E = (int)(c.e - c.b);
  for (int i = threadIdx.x; i < 2 * CHUNK; i += 256) set[i] = KO::EMPTY;
  for (int i = threadIdx.x; i <= P; i += 256) hist[i] = 0;
  K pr[HUB_U];
  if (E > 0) {
    load_keys<K, HUB_U, 256>(src, row + c.b, (int)threadIdx.x, E, pr);
  } else {
#pragma unroll
    for (int u = 0; u < HUB_U; ++u) pr[u] = KO::EMPTY;
  }
  __syncthreads();
  int rank[HUB_U];
#pragma unroll
  for (int u = 0; u < HUB_U; ++u) {
    rank[u] = -1;
    const K p = pr[u];
    if (p == KO::EMPTY) continue;
    u32 sl = KO::hash(p) & (2 * CHUNK - 1);
    while (true) {
      const K old = atomicCAS(&set[sl], KO::EMPTY, p);
      if (old == KO::EMPTY) {
        rank[u] = atomicAdd(&hist[part_hash(p) & (P - 1)], 1);
        break;
      }
      if (old == p) break;
      sl = (sl + 1) & (2 * CHUNK - 1);
    }
  }
  __syncthreads();
  // exclusive scan of hist[0..P) by the whole workgroup (P <= 1024: 4 per thread)
  {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int v4[4];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int idx = t * 4 + k;
      v4[k] = idx < P ? hist[idx] : 0;
      sum += v4[k];
    }
    int x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, WAVE);
      if (lane >= o) x += y;
    }
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    int off = x - sum;
    for (int i = 0; i < w; ++i) off += wtot[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int idx = t * 4 + k;
      if (idx < P) {
        hist[idx] = off;
        poff[c.poff + idx] = off;
      }
      off += v4[k];
    }
    if (t == 255) poff[c.poff + P] = off;
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < HUB_U; ++u) {
    if (rank[u] >= 0) {
      const K p = pr[u];
      stage[c.stage + hist[part_hash(p) & (P - 1)] + rank[u]] = p;
    }
  }
}

template <class Src, class K = u64>
__global__ void __launch_bounds__(256) k_hub_reduce(Src src, const HubPart *__restrict__ parts,
                                                    const HubChunk *__restrict__ chunks,
                                                    const K *__restrict__ stage, const int *__restrict__ poff,
                                                    u64 *hub_acc, u32 *hub_cnt, u32 *err, const int *__restrict__ hubs,
                                                    const unsigned char *__restrict__ skip) {
  typedef Keys<K> KO;
  constexpr int PS = sizeof(K) == 8 ? HUB_PSLOTS_WIDE : HUB_PSLOTS;
  __shared__ K set[PS];
  __shared__ int64_t sbase[HUB_PMAX]; // per chunk: staging position of this partition's segment
  __shared__ int pre[HUB_PMAX + 1];    // exclusive prefix of segment lengths
  __shared__ int wtot[4];
  __shared__ u64 sh_acc[4];
  __shared__ u32 sh_cnt[4];
  __shared__ u32 sh_fill[2];  // distinct keys in the set, overflow flag
  const HubPart hp = parts[blockIdx.x];
  if (skip && skip[hubs[hp.hub]]) return;  // singleton block (work-efficient mode)
  const int C = hp.nchunks;
  for (int i = threadIdx.x; i < PS; i += 256) set[i] = KO::EMPTY;
  // segment lengths, then an exclusive scan over the (at most 1024) chunks
  {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int len4[4];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ci = t * 4 + k;
      len4[k] = 0;
      if (ci < C) {
        const HubChunk c = chunks[hp.chunk0 + ci];
        const int a = poff[c.poff + hp.part], b = poff[c.poff + hp.part + 1];
        sbase[ci] = c.stage + a;
        len4[k] = b - a;
      }
      sum += len4[k];
    }
    int x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, WAVE);
      if (lane >= o) x += y;
    }
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    int off = x - sum;
    for (int i = 0; i < w; ++i) off += wtot[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ci = t * 4 + k;
      if (ci < C) pre[ci] = off;
      off += len4[k];
    }
    if (t == 255) pre[C] = off;
    __syncthreads();
  }
  const int T = pre[C];
  // Distinct keys of this partition, PS slots at a time.  A partition is
  // planned to hold at most PS / 2 of them, but a skewed hub can put more in
  // one partition: then the set stops filling at 3/4 (so probes always end),
  // and the partition is redone in Q sub-passes, each taking the keys whose
  // sub-partition hash (independent of the partition and slot hashes) is q,
  // with Q doubled until every sub-pass fits.  Sub-passes hold disjoint key
  // sets, so their sums and counts add up to the partition's.
  u64 acc = 0;
  u32 cnt = 0;
  u32 Q = 1;
  for (u32 q = 0; q < Q;) {
    if (threadIdx.x == 0) { sh_fill[0] = 0; sh_fill[1] = 0; }
    __syncthreads();
    u64 pacc = 0;
    u32 pcnt = 0;
    for (int t0 = 0; t0 < T; t0 += 4 * 256) {
      K pr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + threadIdx.x + u * 256;
        pr[u] = KO::EMPTY;
        if (t < T) {
          int lo = 0, hi = C - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= t) lo = mid; else hi = mid - 1;
          }
          pr[u] = stage[sbase[lo] + (t - pre[lo])];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const K p = pr[u];
        if (p == KO::EMPTY) continue;
        if (Q > 1 && (sub_hash((u64)p) & (Q - 1)) != q) continue;
        u32 sl = KO::hash(p) & (PS - 1);
        while (true) {
          const K cur = set[sl];
          if (cur == p) break;
          if (cur == KO::EMPTY) {
            // once the pass has overflowed nothing more is inserted (it is redone);
            // at most one insertion per thread lands after the 3/4 mark, so empty
            // slots remain and every probe sequence ends
            if (sh_fill[1]) break;
            const K old = atomicCAS(&set[sl], KO::EMPTY, p);
            if (old == KO::EMPTY) {
              pacc += mix_pair(KO::mixin(src, p));
              ++pcnt;
              if (atomicAdd(&sh_fill[0], 1u) + 1u >= (u32)(PS / 4 * 3)) sh_fill[1] = 1u;
              break;
            }
            if (old == p) break;
          }
          sl = (sl + 1) & (PS - 1);
        }
      }
      __syncthreads();
    }
    __syncthreads();
    const bool over = sh_fill[1] != 0;
    __syncthreads();
    for (int i = threadIdx.x; i < PS; i += 256) set[i] = KO::EMPTY;
    if (over) {
      if (Q >= 4096) {  // 4096 * PS * 3/4 slots exceed any staged hub; not reached
        if (threadIdx.x == 0) atomicOr(err, ERR_VERIFY_OVERFLOW);
        return;
      }
      Q <<= 1;
      q = 0;
      acc = 0;
      cnt = 0;
    } else {
      acc += pacc;
      cnt += pcnt;
      ++q;
    }
    __syncthreads();
  }
  block_reduce_2(acc, cnt, sh_acc, sh_cnt);
  if (threadIdx.x == 0) {
    if (acc) atomicAdd(&hub_acc[hp.hub], acc);
    if (cnt) atomicAdd(&hub_cnt[hp.hub], cnt);
  }
}

// Very large hubs (deg > HUB_STAGED_MAX, or HUB_STAGED_MAX_WIDE with 64-bit
// keys): workgroups of one hub share a
// global hash set of 2*deg slots; slot = pair | (epoch << 62), 0 = unused,
// epochs 1..3.  Pairs are < 2^62.
struct HubGChunk {
  int hub;
  int pad;
  int64_t b, e;      // entry range relative to the start of the hub's row
  int64_t set_off;   // the hub's global set
  int64_t set_size;
};

// Set slots hold key | epoch << 62 and count as empty unless their epoch is
// the current one, so dep[EP_HUB] must be 1..3 (advanced at least once; a
// zeroed set with epoch 0 would have no empty slot) and each set must hold
// more slots than its row has entries.
template <class Src>
__global__ void __launch_bounds__(256) k_sig_hub_global(Src src, const HubGChunk *__restrict__ chunks,
                                                        const int *__restrict__ hubs, u64 *sets, u64 *hub_acc,
                                                        u32 *hub_cnt, const u32 *__restrict__ dep,
                                                        const unsigned char *__restrict__ skip) {
  const u32 hepoch = dep[EP_HUB];
  __shared__ u64 sh_acc[4];
  __shared__ u32 sh_cnt[4];
  const HubGChunk c = chunks[blockIdx.x];
  if (skip && skip[hubs[c.hub]]) return;  // singleton block (work-efficient mode)
  u64 *set = sets + c.set_off;
  const u64 size = (u64)c.set_size;
  const int64_t row = src.begin(hubs[c.hub]);
  u64 acc = 0;
  u32 cnt = 0;
  for (int64_t i = row + c.b + threadIdx.x; i < row + c.e; i += 256) {
    u64 p = src.pair(i);
    if constexpr (Src::HASHED) p = (u64)src.hkey(p);  // the tiers of one graph dedupe the same keys
    const u64 want = p | ((u64)hepoch << 62);
    u64 sl = scale_to(set_hash(p), size);
    while (true) {
      u64 cur = __hip_atomic_load(&set[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      bool done = false;
      while ((cur >> 62) != (u64)hepoch) {
        const u64 old = atomicCAS(&set[sl], cur, want);
        if (old == cur) { acc += mix_pair(p); ++cnt; done = true; break; }
        cur = old;
      }
      if (done || cur == want) break;
      sl = (sl + 1 == size) ? 0 : sl + 1;
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
                            u64 *__restrict__ H, u32 *__restrict__ DC, u64 *table, u64 tmask,
                            const u32 *__restrict__ dep, u64 hmask, u64 *zrep,
                            const unsigned char *__restrict__ skip) {
  const u32 epoch = dep[EP_TABLE], zep = dep[EP_ZERO];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nhub) return;
  const int v = hubs[i];
  const u64 acc = hub_acc[i];
  const u32 cnt = hub_cnt[i];
  hub_acc[i] = 0;
  hub_cnt[i] = 0;
  if (skip && skip[v]) return;  // singleton block (work-efficient mode)
  const u32 own = src.own(v);
  const u64 h = finalize_key(acc, cnt, own) & hmask;
  H[v] = h;
  DC[v] = cnt;
  key_insert(table, tmask, zrep, h, cnt, own, (u32)v, epoch, zep);
}

// ---------------------------------------------------------------- lookup + exact check
// For each vertex: representative r = minimum vertex stored under its key.
// r == v: v heads its block.  Otherwise v joins r's block once the keys are
// shown equal exactly: the previous block, the number of distinct pairs and,
// for rows of at most SMALL_MAX entries, the pair sets here; larger rows go
// to a verification list (k_verify).  Mismatches (hash collisions) go to the
// collision list with rep = -1.  Lists are appended with one atomic per
// wave; they stay short, since device-wide atomics on one counter serialise.
// Updates (dirty != NULL): a vertex and its candidate that are both clean
// (key inputs unchanged) and shared a block in the cached chain (same cached
// name mvc) still have equal keys, so they are accepted without the check.
template <class Src>
__global__ void __launch_bounds__(256) k_lookup(Src src, int count, const int *__restrict__ list,
                                                const u64 *__restrict__ H, const u32 *__restrict__ DC,
                                                const u64 *table, u64 tmask, const u32 *__restrict__ dep,
                                                int *__restrict__ rep, int *vcount, int *vlist, int *ccount,
                                                int *clist, u32 *err, const u64 *zrep, int zfresh,
                                                const unsigned char *__restrict__ skip,
                                                const unsigned char *__restrict__ dirty,
                                                const int32_t *__restrict__ mvc) {
  const u32 epoch = dep[EP_TABLE], zep = dep[EP_ZERO];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool act = i < count;
  const int v = act ? (list ? list[i] : i) : 0;
  bool to_verify = false, collided = false;
  if (act && skip && skip[v]) {
    rep[v] = v;  // a singleton block stays a singleton
  } else if (act) {
    const u32 dcv = DC[v];
    if (dcv == 0) {
      // empty signature: exact grouping by previous block (without zfresh the
      // representative is kept from the call's first step)
      if (zfresh) {
        const u64 z = zrep[src.own(v)];
        if ((u32)(z >> 32) != ~zep) {
          atomicOr(err, ERR_LOOKUP_MISS);
          rep[v] = v;
        } else {
          rep[v] = (int)(u32)z;
        }
      }
    } else {
      const int r = table_lookup(table, tmask, H[v], epoch);
      if (r < 0) {
        atomicOr(err, ERR_LOOKUP_MISS);
        rep[v] = v;
      } else if (r == v) {
        rep[v] = v;
      } else if (src.own(v) != src.own(r) || dcv != DC[r]) {
        rep[v] = -1;
        collided = true;
      } else if (dirty && !dirty[v] && !dirty[r] && mvc[v] == mvc[r]) {
        rep[v] = r;
      } else {
        const int64_t bv = src.begin(v), ev = src.end(v);
        const int64_t br = src.begin(r), er = src.end(r);
        if (ev - bv <= SMALL_MAX && er - br <= SMALL_MAX) {
          // small rows: r's pairs in registers (static indexing); every pair
          // of v must occur among them, and every entry of r must be met by
          // some pair of v (set equality in both directions, so it does not
          // rest on the distinct counts)
          u64 rp[SMALL_MAX];
#pragma unroll
          for (int j = 0; j < SMALL_MAX; ++j) rp[j] = br + j < er ? src.pair(br + j) : EMPTY64;
          const u32 want = (u32)((1ull << (er - br)) - 1ull);
          u32 met = 0;
          bool ok = true;
          for (int64_t j = bv; j < ev && ok; ++j) {
            const u64 p = src.pair(j);
            u32 hit = 0;
#pragma unroll
            for (int q = 0; q < SMALL_MAX; ++q) hit |= (rp[q] == p ? 1u : 0u) << q;
            met |= hit;
            ok = hit != 0;
          }
          ok = ok && met == want;
          if (ok) {
            rep[v] = r;
          } else {
            rep[v] = -1;
            collided = true;
          }
        } else {
          rep[v] = r;  // confirmed or rejected by k_verify
          to_verify = true;
        }
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
__device__ bool wg_subset_one(const Src &src, int v, int r, u32 dcr, u64 *set, int *sh_flag, u32 *err) {
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

// Equal signatures of v and r, given equal distinct counts.  With exact keys
// the counts are the pair counts and one inclusion decides; with hashed keys
// they count distinct keys, so both inclusions are checked.
template <class Src>
__device__ bool wg_subset(const Src &src, int v, int r, u32 dcr, u64 *set, int *sh_flag, u32 *err) {
  if (!wg_subset_one(src, v, r, dcr, set, sh_flag, err)) return false;
  if constexpr (Src::HASHED) return wg_subset_one(src, r, v, dcr, set, sh_flag, err);
  return true;
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
                             u64 *ctable, u64 tmask, const u32 *__restrict__ dep) {
  const u32 epoch = dep[EP_CTABLE];
  const int total = *count;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int v = list[i];
    table_insert(ctable, tmask, H[v], (u32)v, epoch);
  }
}

template <class Src>
__global__ void __launch_bounds__(256) k_res_verify(Src src, const int *__restrict__ count, const int *__restrict__ list,
                                                    const u64 *__restrict__ H, const u32 *__restrict__ DC,
                                                    const u64 *ctable, u64 tmask, const u32 *__restrict__ dep,
                                                    int *__restrict__ rep, int *next_count, int *next_list, u32 *err) {
  const u32 epoch = dep[EP_CTABLE];
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
// Reduce-then-scan over the flags "rep[v] == v" in vertex order (tiles of
// 256 * ITEMS vertices, ITEMS = 8 or 16 per thread): per-tile head counts, one workgroup scans the tile
// counts, then every tile numbers its heads.  A head's exclusive prefix is its
// dense id, so blocks are numbered by their first vertex.  Non-heads get -1
// (k_scan_write lists the heads; the steps number through head words).
template <int ITEMS>
__device__ inline u32 tile_flags(int n, const int *__restrict__ rep, int64_t base) {
  int r[ITEMS];
  if (base + ITEMS <= n) {
    const int4 *p4 = reinterpret_cast<const int4 *>(rep + base);
#pragma unroll
    for (int q = 0; q < ITEMS / 4; ++q) {
      const int4 x = p4[q];
      r[4 * q] = x.x;
      r[4 * q + 1] = x.y;
      r[4 * q + 2] = x.z;
      r[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) r[j] = (base + j < n) ? rep[base + j] : -1;
  }
  u32 bits = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j)
    if (r[j] == (int)(base + j)) bits |= 1u << j;
  return bits;
}


template <int ITEMS>
__global__ void __launch_bounds__(256) k_tile_count(int n, const int *__restrict__ rep, u32 *__restrict__ tile_sum) {
  __shared__ u32 sh_w[4];
  const int64_t base = (int64_t)blockIdx.x * (256 * ITEMS) + (int64_t)threadIdx.x * ITEMS;
  const u32 mine = __popc(tile_flags<ITEMS>(n, rep, base));
  u32 total;
  block_exclusive_scan(mine, sh_w, &total);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One workgroup of 1024 threads: in-place exclusive scan of ntiles counts.
__global__ void __launch_bounds__(1024) k_tile_scan(int ntiles, u32 *tile_sum, int64_t *count_out) {
  __shared__ u32 sh_w[16];
  __shared__ u32 carry;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < ntiles; b0 += 1024 * 8) {
    u32 v8[8];
    u32 sum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = b0 + t * 8 + k;
      v8[k] = i < ntiles ? tile_sum[i] : 0u;
      sum += v8[k];
    }
    u32 x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const u32 y = __shfl_up(x, o, WAVE);
      if (lane >= o) x += y;
    }
    if (lane == 63) sh_w[w] = x;
    __syncthreads();
    u32 off = carry + x - sum;
    for (int i = 0; i < w; ++i) off += sh_w[i];
    u32 all = 0;
    for (int i = 0; i < 16; ++i) all += sh_w[i];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = b0 + t * 8 + k;
      if (i < ntiles) tile_sum[i] = off;
      off += v8[k];
    }
    __syncthreads();
    if (t == 0) carry += all;
    __syncthreads();
  }
  if (t == 0) *count_out = (int64_t)carry;
}

template <int ITEMS>
__global__ void __launch_bounds__(256) k_scan_write(int n, const int *__restrict__ rep, const u32 *__restrict__ tile_pre,
                                                    int *__restrict__ out, int out_aligned) {
  __shared__ u32 sh_w[4];
  const int64_t base = (int64_t)blockIdx.x * (256 * ITEMS) + (int64_t)threadIdx.x * ITEMS;
  const u32 bits = tile_flags<ITEMS>(n, rep, base);
  u32 total;
  u32 id = tile_pre[blockIdx.x] + block_exclusive_scan(__popc(bits), sh_w, &total);
  int o[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    o[j] = (bits & (1u << j)) ? (int)id : -1;
    id += (bits >> j) & 1u;
  }
  if (out_aligned && base + ITEMS <= n) {
    int4 *q4 = reinterpret_cast<int4 *>(out + base);
#pragma unroll
    for (int q = 0; q < ITEMS / 4; ++q) q4[q] = make_int4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
  } else {
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (base + j < n) out[base + j] = o[j];
  }
}

// Head words: the numbering of a step without the scattered write of every
// head's id.  Word w holds one bit per vertex 64w..64w+63 (set for a head,
// rep[v] == v) and the number of heads before the word in its tile (tiles of
// 256 * ITEMS vertices, as k_tile_count; the tile counts go to tile_sum for
// k_tile_scan).  A vertex then reads its dense id from its representative's
// word: tile prefix + word prefix + heads below it in the word.  The words
// (n / 4 bytes) and tile prefixes stay in the caches, unlike a gather of
// every representative's id from the output (n * 4 bytes).
struct HeadWord {
  u64 bits;
  u32 pre;
  u32 pad;
};
struct HeadIds {
  const HeadWord *hw;
  const u32 *tile_pre;  // exclusive prefix of head counts per tile
  int tile_shift;       // log2 of the tile's vertex count
};
__device__ inline int head_id(const HeadIds &h, int r) {
  const u32x4 q = *reinterpret_cast<const u32x4 *>(&h.hw[r >> 6]);
  const u64 bits = (u64)q.x | ((u64)q.y << 32);
  const u64 below = bits & ((1ull << (r & 63)) - 1ull);
  return (int)(h.tile_pre[r >> h.tile_shift] + q.z + (u32)__popcll(below));
}

template <int ITEMS>
__global__ void __launch_bounds__(256) k_head_words(int n, const int *__restrict__ rep, HeadWord *__restrict__ hw,
                                                    u32 *__restrict__ tile_sum) {
  static_assert(64 % ITEMS == 0, "a word spans whole threads");
  constexpr int TPW = 64 / ITEMS;  // threads per word (consecutive lanes of one wave)
  __shared__ u32 sh_w[4];
  const int64_t base = (int64_t)blockIdx.x * (256 * ITEMS) + (int64_t)threadIdx.x * ITEMS;
  const u32 bits = tile_flags<ITEMS>(n, rep, base);
  u32 total;
  const u32 pre = block_exclusive_scan(__popc(bits), sh_w, &total);
  u64 word = 0;
#pragma unroll
  for (int q = 0; q < TPW; ++q) word |= (u64)__shfl_down(bits, q, WAVE) << (q * ITEMS);
  if ((threadIdx.x % TPW) == 0 && base < n)
    *reinterpret_cast<u32x4 *>(&hw[base >> 6]) = u32x4{(u32)word, (u32)(word >> 32), pre, 0u};
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// rep[v] = v for vertices with at least one entry, else -1 (heads of the
// numbering scan, which then lists them in order).
__global__ void k_mark_rows(int n, const int64_t *__restrict__ row_ptr, int *__restrict__ rep) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) rep[v] = row_ptr[v + 1] > row_ptr[v] ? v : -1;
}

// list[pos[v]] = v for every v with pos[v] >= 0.
__global__ void k_list_from_ids(int n, const int *__restrict__ pos, int *__restrict__ list) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && pos[v] >= 0) list[pos[v]] = v;
}

// Every vertex takes its representative's dense id (head words), and the
// new partition is also written in rank order for the next gather (vertices
// no entry names have rank -1 and are left out).
// Work-efficient mode (multi != NULL): every non-head marks its head with the
// step's stamp, so a head left unmarked is a singleton block (k_singletons).
// ASSIGN_V consecutive vertices per thread: representatives, ranks and ids
// move 16 bytes at a time where the arrays' starts allow.
constexpr int ASSIGN_V = 4;
__global__ void __launch_bounds__(256) k_assign(int n, const int *__restrict__ rep, HeadIds ids,
                                                int *__restrict__ out, const int *__restrict__ rank,
                                                int *__restrict__ gpid_next, u32 *multi,
                                                const u32 *__restrict__ dep) {
  const int64_t v0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * ASSIGN_V;
  if (v0 >= n) return;
  const bool vec = v0 + ASSIGN_V <= n && ((reinterpret_cast<uintptr_t>(rep) | reinterpret_cast<uintptr_t>(out) |
                                           reinterpret_cast<uintptr_t>(rank)) & 15) == 0;
  int r[ASSIGN_V], rk[ASSIGN_V], val[ASSIGN_V];
  if (vec) {
    const int4 r4 = *reinterpret_cast<const int4 *>(rep + v0);
    r[0] = r4.x; r[1] = r4.y; r[2] = r4.z; r[3] = r4.w;
    if (rank) {
      const int4 k4 = *reinterpret_cast<const int4 *>(rank + v0);
      rk[0] = k4.x; rk[1] = k4.y; rk[2] = k4.z; rk[3] = k4.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < ASSIGN_V; ++j) {
      r[j] = v0 + j < n ? rep[v0 + j] : -1;
      if (rank) rk[j] = v0 + j < n ? rank[v0 + j] : -1;
    }
  }
#pragma unroll
  for (int j = 0; j < ASSIGN_V; ++j) val[j] = r[j] >= 0 ? head_id(ids, r[j]) : -1;
  if (vec) {
    *reinterpret_cast<int4 *>(out + v0) = make_int4(val[0], val[1], val[2], val[3]);
  } else {
#pragma unroll
    for (int j = 0; j < ASSIGN_V; ++j)
      if (v0 + j < n) out[v0 + j] = val[j];
  }
#pragma unroll
  for (int j = 0; j < ASSIGN_V; ++j) {
    if (v0 + j >= n) break;
    if (multi && r[j] >= 0 && r[j] != (int)(v0 + j)) multi[r[j]] = dep[EP_ZERO];
    if (rank && rk[j] >= 0) gpid_next[rk[j]] = val[j];
  }
}

// single[v] = 1 iff v is alone in its block of the partition just computed.
// A singleton block never splits, so the next step can skip its vertex.
__global__ void k_singletons(int n, const int *__restrict__ rep, const u32 *__restrict__ multi,
                             const u32 *__restrict__ dep, unsigned char *single) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  single[v] = (rep[v] == v && multi[v] != dep[EP_ZERO]) ? 1 : 0;
}

// In-degree histogram, target renumbering and rank-order scatter (create time
// and the start of each call).
// ---------------------------------------------------------------- transpose
// Backward refinement is forward refinement of the transposed graph
// (Def. inverse-schema-element).  Transpose = count entries per target,
// exclusive scan into row offsets, scatter each entry (v, l, w) to row w.

// Exclusive scan of 64-bit values over a 256-thread workgroup.
__device__ inline int64_t block_exclusive_scan64(int64_t mine, int64_t *sh_w, int64_t *total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int64_t x = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, WAVE);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh_w[w] = x;
  __syncthreads();
  int64_t base = 0;
  for (int i = 0; i < w; ++i) base += sh_w[i];
  *total = sh_w[0] + sh_w[1] + sh_w[2] + sh_w[3];
  __syncthreads();
  return base + x - mine;
}

__global__ void __launch_bounds__(256) k_sum_tiles64(int64_t n, const int *__restrict__ cnt, int64_t *tile_sum) {
  __shared__ int64_t sh_w[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t mine = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j)
    if (base + j < n) mine += cnt[base + j];
  int64_t total;
  block_exclusive_scan64(mine, sh_w, &total);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One workgroup of 256 threads: in-place exclusive scan of ntiles sums.
__global__ void __launch_bounds__(256) k_scan_tiles64(int64_t ntiles, int64_t *tile_sum) {
  __shared__ int64_t sh_w[4];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < ntiles; b0 += 256) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t mine = i < ntiles ? tile_sum[i] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan64(mine, sh_w, &total);
    if (i < ntiles) tile_sum[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
}

// out_ptr[i] = sum of cnt[0..i), out_ptr[n] = total; cursor[i] = out_ptr[i] (cursor may be NULL).
__global__ void __launch_bounds__(256) k_write_ptr64(int64_t n, const int *__restrict__ cnt,
                                                     const int64_t *__restrict__ tile_pre, int64_t *out_ptr,
                                                     unsigned long long *cursor) {
  __shared__ int64_t sh_w[4];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t c[SCAN_ITEMS];
  int64_t mine = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    c[j] = base + j < n ? cnt[base + j] : 0;
    mine += c[j];
  }
  int64_t total;
  int64_t off = tile_pre[blockIdx.x] + block_exclusive_scan64(mine, sh_w, &total);
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    if (base + j < n) {
      out_ptr[base + j] = off;
      if (cursor) cursor[base + j] = (unsigned long long)off;
    }
    off += c[j];
    if (base + j + 1 == n) out_ptr[n] = off;
  }
}

// One wave per source row: every entry (v, l, w) takes the next free
// position of row w.  The order inside a transposed row depends on timing;
// signatures are sets, so refinement results do not.
__global__ void __launch_bounds__(256) k_transpose_scatter(int64_t n, const int64_t *__restrict__ row_ptr,
                                                           const int32_t *__restrict__ col,
                                                           const int32_t *__restrict__ elabel,
                                                           unsigned long long *cursor, int32_t *out_col,
                                                           int32_t *out_elabel) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < n; v += waves) {
    const int64_t b = row_ptr[v], e = row_ptr[v + 1];
    for (int64_t i = b + lane; i < e; i += WAVE) {
      const unsigned long long pos = atomicAdd(&cursor[col[i]], 1ULL);
      out_col[pos] = (int32_t)v;
      if (out_elabel) out_elabel[pos] = elabel ? elabel[i] : 0;
    }
  }
}

// Entries per target.  A workgroup counts a chunk of INDEG_CHUNK entries in
// an LDS table (target -> count), then adds one device atomic per distinct
// target, so the many entries of a hot target do not serialise on one
// address across the device.  indeg starts at zero; 256 threads.
constexpr int INDEG_CHUNK = 2048, INDEG_SLOTS = 4096;
__global__ void __launch_bounds__(256) k_indegree(int64_t m, const int *__restrict__ col, int *indeg) {
  __shared__ int key[INDEG_SLOTS];
  __shared__ int val[INDEG_SLOTS];
  for (int64_t base = (int64_t)blockIdx.x * INDEG_CHUNK; base < m; base += (int64_t)gridDim.x * INDEG_CHUNK) {
    for (int i = threadIdx.x; i < INDEG_SLOTS; i += 256) {
      key[i] = -1;
      val[i] = 0;
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(m - base, INDEG_CHUNK);
    for (int i = threadIdx.x; i < cnt; i += 256) {
      const int c = col[base + i];
      u32 sl = ((u32)c * 0x9E3779B1u) >> 20;  // 12 bits: INDEG_SLOTS
      while (true) {
        const int old = atomicCAS(&key[sl], -1, c);
        if (old == -1 || old == c) {
          atomicAdd(&val[sl], 1);
          break;
        }
        sl = (sl + 1) & (INDEG_SLOTS - 1);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < INDEG_SLOTS; i += 256)
      if (key[i] >= 0) atomicAdd(&indeg[key[i]], val[i]);
    __syncthreads();
  }
}
// gcol[e] = rank[col[e]], with the entry's label in the bits above rbits
// when elabel is given (packed form).
__global__ void k_remap(int64_t m, const int *__restrict__ col, const int *__restrict__ rank, int *__restrict__ gcol,
                        const int *__restrict__ elabel, u32 rbits) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    u32 g = (u32)rank[col[e]];
    if (elabel) g |= (u32)elabel[e] << rbits;
    gcol[e] = (int)g;
  }
}
// Order of the entries inside a row.  A signature is a set, so the kernels
// may read a row's entries in any order; with the entries of long rows sorted
// by target rank, the lanes of a wave gather from fewer cache lines (ranks
// put the targets of most edges together).  Packed words (label << rbits |
// rank) are compared with the rank on top: rot(g) = g rotated left by
// 32 - rbits, which keeps the order of ranks and breaks ties by label.
__device__ inline u32 rank_first(u32 g, u32 rbits) { return rbits >= 32 ? g : (g << (32 - rbits)) | (g >> rbits); }
__device__ inline u32 rank_first_inv(u32 x, u32 rbits) { return rbits >= 32 ? x : (x >> (32 - rbits)) | (x << rbits); }

// Sort words[0, len) (len <= N) by rank_first with a bitonic network over N
// LDS slots (padding sorts last); the whole workgroup of NT threads takes
// part.  PAY: labels[0, len) (separate edge labels) move with their words.
template <int N, int NT, bool PAY>
__device__ inline void sort_row_words(u32 *words, u32 *labels, int len, u32 rbits, u32 *sh, u32 *shl) {
  for (int i = threadIdx.x; i < N; i += NT) {
    sh[i] = i < len ? rank_first(words[i], rbits) : 0xFFFFFFFFu;
    if constexpr (PAY) shl[i] = i < len ? labels[i] : 0u;
  }
  __syncthreads();
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N / 2; i += NT) {
        const int lo = 2 * j * (i / j) + (i % j), hi = lo + j;  // pairs (lo, lo + j) with lo & j == 0
        const u32 a = sh[lo], b = sh[hi];
        const bool up = (lo & k) == 0;
        if ((a > b) == up) {
          sh[lo] = b;
          sh[hi] = a;
          if constexpr (PAY) {
            const u32 t = shl[lo];
            shl[lo] = shl[hi];
            shl[hi] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < len; i += NT) {
    words[i] = rank_first_inv(sh[i], rbits);
    if constexpr (PAY) labels[i] = shl[i];
  }
}

static_assert(RANGE_DMAX <= 4096 && ROW_MAX <= 8192 && ROW_MAX_NARROW <= 32768 && HUB_CHUNK_MAX <= 4096,
              "row sort sizes");

// One workgroup of 256 threads per range of at most N entries: each row of
// the range sorted by rank_first in place.  Keys (row << 32 | rank_first) in
// a bitonic network over N LDS slots; the row of an entry is found by
// binary search over the range's row offsets.
template <class Src, int N, bool PAY>
__global__ void __launch_bounds__(256) k_sort_ranges(Src src, u32 *gcol, u32 *labels, const Range *__restrict__ ranges,
                                                     u32 rbits) {
  __shared__ u64 sh[N];
  __shared__ u32 shl[PAY ? N : 1];
  __shared__ int roff[RANGE_VERTS + 1];
  const Range rg = ranges[blockIdx.x];
  const int V = rg.v1 - rg.v0, E = rg.ne;
  u32 *words = gcol + rg.e0;
  u32 *labs = PAY ? labels + rg.e0 : nullptr;
  for (int i = threadIdx.x; i <= V; i += 256) roff[i] = (int)(src.begin_lo(rg.v0 + i) - (u32)rg.e0);
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += 256) {
    u64 key = ~0ULL;
    if (i < E) {
      int lo = 0, hi = V - 1;  // last row whose start is <= i
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (roff[mid] <= i) lo = mid;
        else hi = mid - 1;
      }
      key = ((u64)lo << 32) | rank_first(words[i], rbits);
    }
    sh[i] = key;
    if constexpr (PAY) shl[i] = i < E ? labs[i] : 0u;
  }
  __syncthreads();
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N / 2; i += 256) {
        const int lo = 2 * j * (i / j) + (i % j), hi = lo + j;
        const u64 a = sh[lo], b = sh[hi];
        const bool up = (lo & k) == 0;
        if ((a > b) == up) {
          sh[lo] = b;
          sh[hi] = a;
          if constexpr (PAY) {
            const u32 t = shl[lo];
            shl[lo] = shl[hi];
            shl[hi] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < E; i += 256) {
    words[i] = rank_first_inv((u32)sh[i], rbits);
    if constexpr (PAY) labs[i] = shl[i];
  }
}

// One workgroup per single-row range of at most N entries.
template <int N, bool PAY>
__global__ void __launch_bounds__(1024) k_sort_rows(u32 *gcol, u32 *labels, const Range *__restrict__ rows,
                                                    u32 rbits) {
  __shared__ u32 sh[N];
  __shared__ u32 shl[PAY ? N : 1];
  const Range r = rows[blockIdx.x];
  sort_row_words<N, 1024, PAY>(gcol + r.e0, PAY ? labels + r.e0 : nullptr, r.ne, rbits, sh, shl);
}

// One workgroup per staged hub chunk (entries [b, e) of the hub's row, e - b <= N).
template <int N, bool PAY>
__global__ void __launch_bounds__(1024) k_sort_hub_chunks(u32 *gcol, u32 *labels, const int64_t *__restrict__ row_ptr,
                                                          const int *__restrict__ hubs,
                                                          const HubChunk *__restrict__ chunks, u32 rbits) {
  __shared__ u32 sh[N];
  __shared__ u32 shl[PAY ? N : 1];
  const HubChunk c = chunks[blockIdx.x];
  const int64_t e0 = row_ptr[hubs[c.hub]] + c.b;
  sort_row_words<N, 1024, PAY>(gcol + e0, PAY ? labels + e0 : nullptr, (int)(c.e - c.b), rbits, sh, shl);
}

// gpid[rank[v]] = pid[v] for every vertex some entry names (rank >= 0).
__global__ void k_scatter_rank(int n, const int *__restrict__ pid, const int *__restrict__ rank, int *__restrict__ gpid) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int r = rank[v];
  if (r >= 0) gpid[r] = pid[v];
}

// ---------------------------------------------------------------- batches
// A batch is the disjoint union of G graphs (vertex ranges [first[g],
// first[g+1])).  Blocks never span graphs, so each graph's first vertex heads
// a block and its global id is the number of blocks in earlier graphs:
// per-graph ids are global ids minus that base.
__global__ void k_graph_ids(int G, const int64_t *__restrict__ first, int *__restrict__ gid) {
  const int g = blockIdx.x;
  if (g >= G) return;
  for (int64_t v = first[g] + threadIdx.x; v < first[g + 1]; v += blockDim.x) gid[v] = g;
}

// Every CSR entry must stay inside its row's graph.
__global__ void k_validate_batch(int n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                 const int *__restrict__ gid, u32 *err) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int g = gid[v];
  for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
    if (gid[col[e]] != g) { atomicOr(err, ERR_GRAPH_COL); return; }
}

__global__ void k_rebase(int n, const int *__restrict__ gid, const int64_t *__restrict__ first,
                         const int *__restrict__ global_ids, int *__restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  out[v] = global_ids[v] - global_ids[first[gid[v]]];
}

// counts[g * k + i] for step i; `next[g]` is the first vertex of the next
// non-empty graph after g, or -1 (then the total count closes the range).
__global__ void k_batch_counts(int G, const int64_t *__restrict__ first, const int64_t *__restrict__ next,
                               const int *__restrict__ global_ids, const int64_t *__restrict__ total, int k, int i,
                               int64_t *__restrict__ counts) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  int64_t c = 0;
  if (first[g + 1] > first[g]) {
    const int64_t base = global_ids[first[g]];
    const int64_t end = next[g] >= 0 ? (int64_t)global_ids[next[g]] : *total;
    c = end - base;
  }
  counts[(int64_t)g * k + i] = c;
}

// ---------------------------------------------------------------- summary graph
// The summary (quotient) graph of a refinement chain has one vertex per block
// of P_k and an edge (B, l, C) when the members of B have an l-edge into block
// C of P_{k-1} (Sec. "Graph Summaries for Bisimulation": connected when all
// represented vertices have such an edge; members of one P_k block share
// their (label, P_{k-1} block) sets, so "all" and "some" coincide).  Built by
// packing each CSR entry into one 64-bit key (source block, label, target
// block), sorting the keys (LSD radix, 8-bit digits) and keeping the first of
// every run of equal keys.

struct QKey {
  u32 lb, db;  // bits of the label and target-block fields
};

// Keys are built from the context's gather layout: the target's rank (and
// packed or sorted label) per entry, and the target blocks copied into rank
// order, so the per-entry gather runs over the hot-first array of the
// signature kernels.  One workgroup per range of the degree schedule (owner
// of each entry by a max-scan over row starts, as in k_sig_range), one per
// single-row range, and one per hub chunk; consecutive entries give
// consecutive keys.
template <class Src>
__device__ inline u64 quotient_key(const Src &src, const int32_t *__restrict__ tgt, QKey q, u64 sb, int64_t e) {
  u32 l, r;
  src.entry(e, l, r);
  return sb | ((u64)l << q.db) | (u64)(u32)tgt[r];
}

template <class Src, int EMAX>
__global__ void __launch_bounds__(256) k_quotient_range(Src src, const Range *__restrict__ ranges,
                                                        const int32_t *__restrict__ src_pid,
                                                        const int32_t *__restrict__ tgt, QKey q, u64 *keys) {
  __shared__ int roff[RANGE_VERTS + 1];
  __shared__ unsigned char owner[EMAX];
  __shared__ u64 sbk[RANGE_VERTS];
  __shared__ u32 wmax[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const Range rg = ranges[blockIdx.x];
  const int V = rg.v1 - rg.v0;
  for (int i = t; i <= V; i += 256) roff[i] = (int)(src.begin_lo(rg.v0 + i) - (u32)rg.e0);  // V may be 256
  if (t < V) sbk[t] = (u64)(u32)src_pid[rg.v0 + t] << (q.lb + q.db);
  for (int i = t; i < EMAX; i += 256) owner[i] = 0;
  __syncthreads();
  for (int i = t; i < V; i += 256)
    if (roff[i + 1] > roff[i]) owner[roff[i]] = (unsigned char)i;
  __syncthreads();
  {
    constexpr int PER = EMAX / 256;
    u32 run = 0;
    const int j0 = t * PER;
#pragma unroll
    for (int k = 0; k < PER; ++k) run = max(run, (u32)owner[j0 + k]);
    u32 x = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const u32 y = __shfl_up(x, o, WAVE);
      if (lane >= o) x = max(x, y);
    }
    if (lane == 63) wmax[w] = x;
    __syncthreads();
    u32 carry = __shfl_up(x, 1, WAVE);
    if (lane == 0) carry = 0;
    for (int i = 0; i < w; ++i) carry = max(carry, wmax[i]);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      carry = max(carry, (u32)owner[j0 + k]);
      owner[j0 + k] = (unsigned char)carry;
    }
    __syncthreads();
  }
  for (int j = t; j < rg.ne; j += 256) keys[rg.e0 + j] = quotient_key(src, tgt, q, sbk[owner[j]], rg.e0 + j);
}

// Entry segments of one row each: single-row ranges (v0, e0, ne) ...
template <class Src>
__global__ void __launch_bounds__(256) k_quotient_rows(Src src, const Range *__restrict__ rows,
                                                       const int32_t *__restrict__ src_pid,
                                                       const int32_t *__restrict__ tgt, QKey q, u64 *keys) {
  const Range rw = rows[blockIdx.x];
  const u64 sb = (u64)(u32)src_pid[rw.v0] << (q.lb + q.db);
  for (int j = threadIdx.x; j < rw.ne; j += 256) keys[rw.e0 + j] = quotient_key(src, tgt, q, sb, rw.e0 + j);
}

// ... and hub chunks (entries [b, e) of the hub's row).
template <class Src, class Chunk>
__global__ void __launch_bounds__(256) k_quotient_hubs(Src src, const Chunk *__restrict__ chunks,
                                                       const int *__restrict__ hubs,
                                                       const int32_t *__restrict__ src_pid,
                                                       const int32_t *__restrict__ tgt, QKey q, u64 *keys) {
  const Chunk c = chunks[blockIdx.x];
  const int v = hubs[c.hub];
  const u64 sb = (u64)(u32)src_pid[v] << (q.lb + q.db);
  const int64_t row = src.begin(v);
  for (int64_t e = row + c.b + threadIdx.x; e < row + c.e; e += 256) keys[e] = quotient_key(src, tgt, q, sb, e);
}

constexpr int RADIX_ITEMS = 16;                  // keys per thread per tile
constexpr int RADIX_TILE = 256 * RADIX_ITEMS;    // keys per tile

// Digit histogram of each tile: hist[digit * ntiles + tile].
__global__ void __launch_bounds__(256) k_radix_hist(int64_t m, const u64 *__restrict__ keys, int shift, int64_t ntiles,
                                                    int *__restrict__ hist) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
  // every key of the thread is requested before the first count
  u64 kk[RADIX_ITEMS];
#pragma unroll
  for (int j = 0; j < RADIX_ITEMS; ++j) {
    const int64_t i = base + j * 256 + threadIdx.x;
    kk[j] = i < m ? __builtin_nontemporal_load(&keys[i]) : 0ULL;
  }
#pragma unroll
  for (int j = 0; j < RADIX_ITEMS; ++j)
    if (base + j * 256 + threadIdx.x < m) atomicAdd(&h[(kk[j] >> shift) & 255], 1);
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of a tile.  Keys are ranked chunk by chunk (256 keys, in
// index order); inside a chunk, lanes with equal digits are found with one
// ballot per digit bit, and waves are ordered through per-digit counts.  Each
// key first goes to its digit-sorted place inside the tile, in LDS; then the
// tile is written out in that order, so the keys of one digit leave as one
// run of consecutive addresses (whole lines) instead of one scattered key
// per lane.  hist holds the tile's digit counts (k_radix_hist).
__global__ void __launch_bounds__(256) k_radix_scatter(int64_t m, const u64 *__restrict__ keys, int shift,
                                                       int64_t ntiles, const int64_t *__restrict__ offs,
                                                       const int *__restrict__ hist, u64 *__restrict__ out) {
  __shared__ u64 sk[RADIX_TILE];     // the tile in digit order
  __shared__ int64_t base[256];      // global position of the tile's first key of each digit
  __shared__ int tstart[256];        // tile position of the first key of each digit
  __shared__ int run[256];           // keys of each digit placed so far
  __shared__ int wcnt[4][256];       // per-wave digit counts of the current chunk
  __shared__ u32 sh_w[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  base[t] = offs[(int64_t)t * ntiles + blockIdx.x];
  {
    u32 total;
    tstart[t] = (int)block_exclusive_scan((u32)hist[(int64_t)t * ntiles + blockIdx.x], sh_w, &total);
  }
  run[t] = 0;
  const int64_t tile0 = (int64_t)blockIdx.x * RADIX_TILE;
  const int cnt = (int)min<int64_t>(m - tile0, RADIX_TILE);
  const u64 lt = (1ULL << lane) - 1ULL;
  // the whole tile is requested at once, so its load latency is paid once
  // instead of once per chunk
  u64 kk[RADIX_ITEMS];
#pragma unroll
  for (int j = 0; j < RADIX_ITEMS; ++j) {
    const int i = j * 256 + t;
    kk[j] = i < cnt ? __builtin_nontemporal_load(&keys[tile0 + i]) : 0ULL;
  }
#pragma unroll
  for (int j = 0; j < RADIX_ITEMS; ++j) {
    for (int q = 0; q < 4; ++q) wcnt[q][t] = 0;
    __syncthreads();
    const int i = j * 256 + t;
    const bool valid = i < cnt;
    const u64 key = kk[j];
    const u32 d = (u32)(key >> shift) & 255u;
    u64 peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const u64 ones = __ballot(valid && ((d >> b) & 1u));
      peers &= ((d >> b) & 1u) ? ones : ~ones;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int before = 0;
      for (int q = 0; q < w; ++q) before += wcnt[q][d];
      sk[tstart[d] + run[d] + before + rank] = key;
    }
    __syncthreads();
    run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
  }
  __syncthreads();
  for (int i = t; i < cnt; i += 256) {
    const u64 key = sk[i];
    const u32 d = (u32)(key >> shift) & 255u;
    out[base[d] + (i - tstart[d])] = key;
  }
}

// ---------------------------------------------------------------- degree schedule
// Rows are packed greedily into ranges of consecutive vertices: a range
// closes before a row that would overflow it (range_edges entries), after
// RANGE_VERTS vertices, before a longer row and at the end of its chunk of
// SCHED_CHUNK_V vertices; longer rows go to the row tiers (up to RANGE_DMAX,
// ROW_MAX and row_max entries) or are hubs.  One thread walks one chunk, so
// the schedule depends on n and the degrees only.  The first walk counts per
// chunk (cnt[list * nchunks + chunk], lists: ranges, up to RANGE_DMAX, up to
// ROW_MAX, up to row_max, hubs; sums[5 * chunk + i]: range vertices and
// entries, row-tier rows and entries, non-empty rows); the second writes at
// the scanned offsets off[list * nchunks + chunk], the range lists one after
// another in `ranges` (list starts in base[0..3]) and the hubs in `hubs`.
constexpr int SCHED_CHUNK_V = 16384;

template <bool WRITE>
__global__ void k_sched_walk(const int64_t *__restrict__ ptr, int64_t n, int nchunks, int range_edges,
                             int64_t row_max, int *__restrict__ cnt, int64_t *__restrict__ sums,
                             const int *__restrict__ off, const int *__restrict__ base, Range *__restrict__ ranges,
                             int *__restrict__ hubs) {
  const int ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= nchunks) return;
  const int64_t v0 = (int64_t)ci * SCHED_CHUNK_V, v1 = min(n, v0 + (int64_t)SCHED_CHUNK_V);
  int c[5] = {0, 0, 0, 0, 0};
  int o[5] = {0, 0, 0, 0, 0};
  int b4[4] = {0, 0, 0, 0};
  if constexpr (WRITE) {
#pragma unroll
    for (int l = 0; l < 5; ++l) o[l] = off[(int64_t)l * nchunks + ci];
#pragma unroll
    for (int l = 0; l < 4; ++l) b4[l] = base[l];
  }
  int64_t rv = 0, re = 0, rowv = 0, rowe = 0, nonempty = 0;
  int64_t cur0 = -1, cur_e = 0, cur_b = 0;
  auto emit = [&](int list, int64_t a, int64_t z, int64_t ne, int64_t e0) {
    if constexpr (WRITE) ranges[b4[list] + o[list] + c[list]] = Range{(int)a, (int)z, (int)ne, 0, e0};
    ++c[list];
  };
  auto close = [&](int64_t vend) {
    if (cur0 >= 0) emit(0, cur0, vend, cur_e, cur_b);
    cur0 = -1;
    cur_e = 0;
  };
  constexpr int PF = 16;  // row ends requested together
  int64_t prev = ptr[v0];
  for (int64_t vb = v0; vb < v1; vb += PF) {
    int64_t nx[PF];
#pragma unroll
    for (int j = 0; j < PF; ++j) nx[j] = vb + j < v1 ? ptr[vb + j + 1] : 0;
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int64_t v = vb + j;
      if (v >= v1) break;
      const int64_t b = prev, d = nx[j] - prev;
      prev = nx[j];
      nonempty += d > 0;
      if (d > row_max) {
        close(v);
        if constexpr (WRITE) hubs[o[4] + c[4]] = (int)v;
        ++c[4];
      } else if (d > range_edges) {
        close(v);
        emit(d > ROW_MAX ? 3 : d > RANGE_DMAX ? 2 : 1, v, v + 1, d, b);
        rowv += 1;
        rowe += d;
      } else {
        if (cur0 >= 0 && (cur_e + d > range_edges || v - cur0 == RANGE_VERTS)) close(v);
        if (cur0 < 0) {
          cur0 = v;
          cur_b = b;
        }
        cur_e += d;
        rv += 1;
        re += d;
      }
    }
  }
  close(v1);
  if constexpr (!WRITE) {
#pragma unroll
    for (int l = 0; l < 5; ++l) cnt[(int64_t)l * nchunks + ci] = c[l];
    sums[5 * (int64_t)ci + 0] = rv;
    sums[5 * (int64_t)ci + 1] = re;
    sums[5 * (int64_t)ci + 2] = rowv;
    sums[5 * (int64_t)ci + 3] = rowe;
    sums[5 * (int64_t)ci + 4] = nonempty;
  }
}

// In-degree ranking: key[v] = (RANK_KEYMAX - min(indeg, RANK_KEYMAX)) << 32 | v;
// a stable sort on the high field orders vertices by decreasing in-degree,
// ties by vertex id.
constexpr int RANK_KEYBITS = 20;
constexpr u32 RANK_KEYMAX = (1u << RANK_KEYBITS) - 1u;

__global__ void k_rank_keys(int64_t n, const int *__restrict__ indeg, u64 *keys) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    keys[v] = ((u64)(RANK_KEYMAX - min((u32)indeg[v], RANK_KEYMAX)) << 32) | (u64)v;
}

// Keys (graph of the vertex << 32 | vertex) in the order of `sorted`, for a
// stable sort by graph that keeps the in-degree order inside each graph.
__global__ void k_rank_gid_keys(int64_t n, const u64 *__restrict__ sorted, const int *__restrict__ gid, u64 *keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const u32 v = (u32)sorted[i];
    keys[i] = ((u64)(u32)gid[v] << 32) | (u64)v;
  }
}

// rank[v] = position of v in the sorted order, or -1 when no entry names v:
// such vertices are never gathered, so the rank-order copies skip them.
__global__ void k_rank_from_sorted(int64_t n, const u64 *__restrict__ sorted, const int *__restrict__ indeg,
                                   int *rank) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const u32 v = (u32)sorted[i];
    rank[v] = indeg[v] > 0 ? (int)i : -1;
  }
}

// flag[i] = 1 where a run of equal keys starts.
__global__ void k_run_starts(int64_t m, const u64 *__restrict__ keys, int *__restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// Unpack the run starts into (source block, label, target block) at their rank.
__global__ void k_quotient_write(int64_t m, const u64 *__restrict__ keys, const int *__restrict__ flag,
                                 const int64_t *__restrict__ pos, QKey q, int32_t *out_src, int32_t *out_lab,
                                 int32_t *out_dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) continue;
    const u64 k = keys[i];
    const int64_t o = pos[i];
    out_dst[o] = (int32_t)(k & ((1ULL << q.db) - 1ULL));
    out_lab[o] = q.lb ? (int32_t)((k >> q.db) & ((1ULL << q.lb) - 1ULL)) : 0;
    out_src[o] = (int32_t)(k >> (q.db + q.lb));
  }
}

// ---------------------------------------------------------------- incremental updates
// After edits to a graph, P'_1..P'_k are recomputed from the signatures of the
// vertices whose key inputs changed, with the cached key hashes of the others
// (the paper names incremental computation on evolving graphs as future
// work, Sec. "Discussion").  Blocks are named by their minimum vertex inside
// such chains (a name does not move when other blocks appear or vanish), so
// the key hash of a vertex whose own name and targets' names are unchanged is
// unchanged.  Dense first-vertex ids are still produced for every output.

// A graph read straight from its CSR, with the previous block name of every
// vertex in vertex order: the rows of edited vertices in the edited graph.
template <bool HK>
struct PlainSrcT {
  static constexpr bool GRAPH = true;
  static constexpr bool HASHED = HK;
  const int64_t *row_ptr;
  const int32_t *col;
  const int32_t *elabel;  // null: every edge has label 0
  const int32_t *names;   // previous block name of every vertex
  u32 pb;
  u32 kmask = 0xFFFFFFFFu;
  __device__ inline int64_t begin(int v) const { return row_ptr[v]; }
  __device__ inline int64_t end(int v) const { return row_ptr[v + 1]; }
  __device__ inline u32 pmask() const { return pb >= 31 ? 0x7FFFFFFFu : (1u << pb) - 1u; }
  __device__ inline u32 label(int64_t e) const { return elabel ? (u32)elabel[e] : 0u; }
  __device__ inline u64 pair(int64_t e) const {
    return ((u64)label(e) << 31) | (u64)((u32)names[col[e]] & pmask());
  }
  __device__ inline u32 own(int v) const { return (u32)names[v]; }
  __device__ inline u32 hkey(u64 p) const { return pair_key32(p) & kmask; }
  // the same key forms as GraphSrcT: exact (label << pb) | block, or a hash of the pair
  __device__ inline u32 key32(int64_t e) const {
    if constexpr (HK) return hkey(pair(e));
    else return (label(e) << pb) | ((u32)names[col[e]] & pmask());
  }
  // the row kernels' interface (as GraphSrcT, with targets in vertex order):
  // (label, target) of entries first + min(t + u*STRIDE, count - 1)
  template <int U, int STRIDE>
  __device__ inline void entries(int64_t first, int t, int count, u32 (&l)[U], u32 (&r)[U]) const {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = first + min(t + u * STRIDE, count - 1);
      r[u] = (u32)__builtin_nontemporal_load(&col[e]);
      l[u] = elabel ? (u32)__builtin_nontemporal_load(&elabel[e]) : 0u;
    }
  }
  __device__ inline u64 pair_of(u32 l, u32 r) const { return ((u64)l << 31) | (u64)((u32)names[r] & pmask()); }
  __device__ inline u32 key32_of(u32 l, u32 r) const {
    if constexpr (HK) return hkey(pair_of(l, r));
    else return (l << pb) | ((u32)names[r] & pmask());
  }
  __device__ inline u64 mixin(u32 q) const {
    if constexpr (HK) return (u64)q;
    else return ((u64)(q >> pb) << 31) | (u64)(q & pmask());
  }
};

constexpr int LIST_SMALL = 64;          // rows up to this many entries: one wave per vertex
constexpr int LIST_SET_BYTES = 32768;   // LDS set of the workgroup-per-vertex kernel

constexpr int LIST_BIG = 4096;  // longer rows go to the row and hub tiers, or a global set

// Split a vertex list by row length (rows of `row_ptr`): <= LIST_SMALL entries
// to small[], up to huge_min to large[], longer ones to huge[].  Counters
// start at zero.
__global__ void k_split_list(int count, const int *__restrict__ list, const int64_t *__restrict__ row_ptr,
                             int *nsmall, int *small, int *nlarge, int *large, int64_t huge_min, int *nhuge,
                             int *huge) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = i < count;
  const int v = act ? list[i] : 0;
  const int64_t d = act ? row_ptr[v + 1] - row_ptr[v] : 0;
  wave_append(nsmall, small, act && d <= LIST_SMALL, v);
  wave_append(nlarge, large, act && d > LIST_SMALL && d <= huge_min, v);
  wave_append(nhuge, huge, act && d > huge_min, v);
}

// Key hash of the listed vertices with short rows: one wave per vertex, an
// LDS set of 2 * LIST_SMALL slots per wave.  Writes H and DC and inserts the
// key into the grouping table (or the empty-signature representatives).
template <class Src, class K>
__global__ void __launch_bounds__(256) k_sig_list_small(Src src, const int *__restrict__ count,
                                                        const int *__restrict__ list, u64 *__restrict__ H,
                                                        u32 *__restrict__ DC, u64 *table, u64 tmask,
                                                        const u32 *__restrict__ dep, u64 hmask, u64 *zrep) {
  typedef Keys<K> KO;
  constexpr int SL = 2 * LIST_SMALL;
  __shared__ K set[4][SL];
  const u32 epoch = dep[EP_TABLE], zep = dep[EP_ZERO];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x >> 6;
  const int total = *count;
  const int waves = gridDim.x * 4;
  for (int item = blockIdx.x * 4 + w; item < total; item += waves) {
    const int v = list[item];
    const int64_t b = src.begin(v);
    const int d = (int)(src.end(v) - b);
    set[w][lane] = KO::EMPTY;
    set[w][lane + WAVE] = KO::EMPTY;
    __builtin_amdgcn_wave_barrier();
    u64 a = 0;
    u32 c = 0;
    if (lane < d) {
      const K p = KO::load(src, b + lane);
      u32 sl = KO::hash(p) & (SL - 1);
      while (true) {
        const K old = atomicCAS(&set[w][sl], KO::EMPTY, p);
        if (old == KO::EMPTY) { a = mix_pair(KO::mixin(src, p)); c = 1; break; }
        if (old == p) break;
        sl = (sl + 1) & (SL - 1);
      }
    }
    a = wave_sum_u64(a);
    c = wave_sum_u32(c);
    if (lane == 0) {
      const u32 own = src.own(v);
      const u64 h = finalize_key(a, c, own) & hmask;
      H[v] = h;
      DC[v] = c;
      key_insert(table, tmask, zrep, h, c, own, (u32)v, epoch, zep);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// The same for longer rows: one workgroup per vertex.  The row's distinct keys
// go through an LDS set in Q passes (keys of sub-partition q in pass q), Q a
// power of two doubled whenever a pass fills the set beyond 3/4 (the
// partition is then redone), so any row length works.
template <class Src, class K>
__global__ void __launch_bounds__(256) k_sig_list_large(Src src, const int *__restrict__ count,
                                                        const int *__restrict__ list, u64 *__restrict__ H,
                                                        u32 *__restrict__ DC, u64 *table, u64 tmask,
                                                        const u32 *__restrict__ dep, u64 hmask, u64 *zrep,
                                                        u32 *err) {
  typedef Keys<K> KO;
  constexpr int PS = LIST_SET_BYTES / (int)sizeof(K);
  __shared__ K set[PS];
  __shared__ u64 sh_acc[4];
  __shared__ u32 sh_cnt[4];
  __shared__ u32 sh_fill[2];
  const u32 epoch = dep[EP_TABLE], zep = dep[EP_ZERO];
  const int total = *count;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int v = list[item];
    const int64_t b = src.begin(v), e = src.end(v);
    const int64_t d = e - b;
    u32 Q = 1;
    while ((int64_t)Q * (PS / 2) < d && Q < (1u << 20)) Q <<= 1;
    u64 acc = 0;
    u32 cnt = 0;
    for (int i = threadIdx.x; i < PS; i += 256) set[i] = KO::EMPTY;
    for (u32 q = 0; q < Q;) {
      if (threadIdx.x == 0) { sh_fill[0] = 0; sh_fill[1] = 0; }
      __syncthreads();
      u64 pacc = 0;
      u32 pcnt = 0;
      for (int64_t j = b + threadIdx.x; j < e; j += 256) {
        const K p = KO::load(src, j);
        if (Q > 1 && (sub_hash((u64)p) & (Q - 1)) != q) continue;
        u32 sl = KO::hash(p) & (PS - 1);
        while (true) {
          const K cur = set[sl];
          if (cur == p) break;
          if (cur == KO::EMPTY) {
            if (sh_fill[1]) break;  // overflowed: the pass is redone with more sub-partitions
            const K old = atomicCAS(&set[sl], KO::EMPTY, p);
            if (old == KO::EMPTY) {
              pacc += mix_pair(KO::mixin(src, p));
              ++pcnt;
              if (atomicAdd(&sh_fill[0], 1u) + 1u >= (u32)(PS / 4 * 3)) sh_fill[1] = 1u;
              break;
            }
            if (old == p) break;
          }
          sl = (sl + 1) & (PS - 1);
        }
      }
      __syncthreads();
      const bool over = sh_fill[1] != 0;
      __syncthreads();
      for (int i = threadIdx.x; i < PS; i += 256) set[i] = KO::EMPTY;
      if (over) {
        if (Q >= (1u << 24)) {
          if (threadIdx.x == 0) atomicOr(err, ERR_VERIFY_OVERFLOW);
          break;
        }
        Q <<= 1;
        q = 0;
        acc = 0;
        cnt = 0;
      } else {
        acc += pacc;
        cnt += pcnt;
        ++q;
      }
      __syncthreads();
    }
    block_reduce_2(acc, cnt, sh_acc, sh_cnt);
    if (threadIdx.x == 0) {
      const u32 own = src.own(v);
      const u64 h = finalize_key(acc, cnt, own) & hmask;
      H[v] = h;
      DC[v] = cnt;
      key_insert(table, tmask, zrep, h, cnt, own, (u32)v, epoch, zep);
    }
    __syncthreads();
  }
}

// Vertices whose key inputs did not change take their cached key hash and
// distinct count.  Only some of them are inserted: a clean vertex that headed
// its cached block (mvc[v] == v), and every clean member of a cached block
// whose head changed.  Clean members of one cached block stay together with
// equal keys, so every new block's minimum vertex is inserted (its head if
// clean, else all its clean members; changed vertices insert themselves),
// and the table ends with the same minimum per slot as if all were inserted.
// Empty signatures go by their own block name, the same way.
__global__ void __launch_bounds__(256) k_insert_cached(int n, const unsigned char *__restrict__ dirty,
                                                       const u64 *__restrict__ Hc, const u32 *__restrict__ DCc,
                                                       const int32_t *__restrict__ mvc,
                                                       const int32_t *__restrict__ names, u64 *__restrict__ H,
                                                       u32 *__restrict__ DC, u64 *table, u64 tmask,
                                                       const u32 *__restrict__ dep, u64 *zrep) {
  const u32 epoch = dep[EP_TABLE], zep = dep[EP_ZERO];
  const int v = blockIdx.x * 256 + threadIdx.x;
  const bool act = v < n && !dirty[v];
  bool zero = false;
  u32 own = 0;
  if (act) {
    const u32 c = DCc[v];
    DC[v] = c;
    const int head = mvc[v];
    const bool ins = head == v || dirty[head];
    if (c) {
      const u64 h = Hc[v];
      H[v] = h;
      if (ins) table_insert(table, tmask, h, (u32)v, epoch);
    } else if (ins) {
      zero = true;
      own = (u32)names[v];
    }
  }
  zero_insert_wave(zrep, zero, own, (u32)v, zep);
}

// Every vertex: dense id from its representative (head words), its new
// block name in vertex order and, for the next gather, in rank order.  The name is the representative (the block's minimum
// vertex), or with bname (an update) the name bname[] gives the
// representative's block; vertices whose name differs from the cached
// chain's (old_names) are then listed in changed[].
// list != NULL: only the `count` listed vertices (out may then be NULL).
__global__ void k_assign_names(int n, const int *__restrict__ rep, HeadIds ids, int *__restrict__ out,
                               int32_t *__restrict__ names_out,
                               const int *__restrict__ rank, int *__restrict__ gpid_next,
                               const int32_t *__restrict__ bname, const int32_t *__restrict__ keep,
                               const int32_t *__restrict__ old_names, int *nchanged, int *changed,
                               int count = 0, const int *__restrict__ list = nullptr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = t < (list ? count : n);
  const int v = act ? (list ? list[t] : t) : 0;
  bool moved = false;
  if (act) {
    const int r = rep[v];
    if (out) out[v] = r >= 0 ? head_id(ids, r) : -1;
    int nm = r;
    if (bname) {
      nm = r >= 0 ? bname[r] : -1;
      if (nm >= n && keep[r] < n) nm = keep[r];
    }
    names_out[v] = nm;
    if (rank) {
      const int rk = rank[v];
      if (rk >= 0) gpid_next[rk] = nm;
    }
    moved = old_names && old_names[v] != nm;
  }
  if (old_names) wave_append(nchanged, changed, moved, v);
}

// Update steps with few dirty vertices group only the blocks that can have
// changed.  Clean members of a cached block keep equal keys, so a cached
// block B keeps exactly its members (and its minimum vertex and name) unless
// it holds a dirty vertex (bit "minimum vertex" of touch, set by
// k_update_flags; a bitmap of n bits, so that its reads stay in the caches) or a
// dirty vertex now has B's key.  The second is found by each clean vertex
// looking its own cached key up among the dirty keys already inserted (the
// table, or zrep for an empty signature, whose key is the own name alone):
// every member of B asks with the same key and gets the same answer; a hash
// match whose keys differ only costs work, the exact check sorts it out.
// Dirty vertices and the clean members of such "touched" blocks are listed
// (the clean ones take their cached key hash and distinct count); every other
// vertex keeps its cached block: representative and name = the cached
// minimum vertex.
// A bit filter of the dirty keys lets most clean vertices skip the table
// probe: one of FILTER_BITS bits per key, from bits 36.. of its hash (as the
// table's slot tags), or for an empty signature from a multiplicative hash of
// the own name.  The same filter holds a bit per touched block (another
// multiplicative hash of its minimum vertex), so that most clean vertices
// skip the touch bitmap too.  Copied to LDS by every workgroup of
// k_classify, so the grid strides over vertices.  A clean vertex's bit is fixed by the cached chain
// (its key hash, distinct count and previous name do not change), so it is
// kept per step in the chain (k_filter_keys) and k_classify reads 2 bytes
// per vertex for the test instead of the hash, count and name.
constexpr int FILTER_BITS = 1 << 16;
constexpr int FILTER_WORDS = FILTER_BITS / 32;
constexpr int CLASSIFY_GRID = 2048;
__device__ inline u32 filter_key_bit(u64 h) { return (u32)(h >> 36) & (FILTER_BITS - 1); }
__device__ inline u32 filter_name_bit(u32 name) { return (name * 0x9E3779B1u) >> 16; }
__device__ inline u32 filter_touch_bit(u32 head) { return (head * 0x85EBCA6Bu) >> 16; }
// With many dirty keys the LDS filter fills up; a second, global filter of
// GFILTER_BITS bits (16 MB, held in the L2 and MALL) then keeps most clean
// vertices from a table probe in HBM.  Its key bits come from other hash bits
// than the LDS filter's.
constexpr int64_t GFILTER_BITS = int64_t(1) << 27;
constexpr int64_t GFILTER_WORDS = GFILTER_BITS / 32;
constexpr int GFILTER_MIN_DIRTY = FILTER_BITS / 16;  // fewer dirty keys: the LDS filter suffices
__device__ inline u32 gfilter_key_bit(u64 h) { return (u32)h & (u32)(GFILTER_BITS - 1); }
__device__ inline u32 gfilter_name_bit(u32 name) {
  return (u32)(((u64)name * 0x9E3779B97F4A7C15ull) >> 37) & (u32)(GFILTER_BITS - 1);
}

// Filter bit of every vertex's key at one step of a cached chain.
__global__ void k_filter_keys(int n, const u64 *__restrict__ H, const u32 *__restrict__ DC,
                              const int32_t *__restrict__ names_prev, uint16_t *__restrict__ fk) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  fk[v] = (uint16_t)(DC[v] ? filter_key_bit(H[v]) : filter_name_bit((u32)names_prev[v]));
}

// gfilter: the global filter (cleared), or null.
__global__ void k_build_filter(const int *__restrict__ count, const int *__restrict__ dlist,
                               const u64 *__restrict__ H, const u32 *__restrict__ DC,
                               const int32_t *__restrict__ names, const int32_t *__restrict__ mvc, u32 *filter,
                               u32 *gfilter) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *count) return;
  const int d = dlist[i];
  const u32 dc = DC[d];
  const u64 h = dc ? H[d] : 0ull;
  const u32 nm = (u32)names[d];
  const u32 b = dc ? filter_key_bit(h) : filter_name_bit(nm);
  atomicOr(&filter[b >> 5], 1u << (b & 31));
  const u32 t = filter_touch_bit((u32)mvc[d]);
  atomicOr(&filter[t >> 5], 1u << (t & 31));
  if (gfilter) {
    const u32 g = dc ? gfilter_key_bit(h) : gfilter_name_bit(nm);
    atomicOr(&gfilter[g >> 5], 1u << (g & 31));
  }
}

__global__ void __launch_bounds__(256) k_classify(int n, const int32_t *__restrict__ mvc,
                                                  const unsigned char *__restrict__ dirty,
                                                  const u32 *__restrict__ touch,
                                                  const uint16_t *__restrict__ fkc, const u64 *__restrict__ Hc,
                                                  const u32 *__restrict__ DCc, const int32_t *__restrict__ names,
                                                  const u32 *__restrict__ filter,
                                                  const u32 *__restrict__ gfilter, const u64 *table, u64 tmask,
                                                  const u32 *__restrict__ dep, const u64 *__restrict__ zrep,
                                                  u64 *__restrict__ H, u32 *__restrict__ DC, int *__restrict__ rep,
                                                  int32_t *__restrict__ names_out, int *count, int *list) {
  __shared__ u32 fl[FILTER_WORDS];
  for (int i = threadIdx.x; i < FILTER_WORDS; i += 256) fl[i] = filter[i];
  __syncthreads();
  const u32 epoch = dep[EP_TABLE], zep = dep[EP_ZERO];
  // CV consecutive vertices per thread and round, read and written 4 at a
  // time when every array's start allows (a step's slice of the chain starts
  // at step * n, so with n not a multiple of 4 they are read one by one).
  // Every vertex first gets its cached block as representative and name; a
  // listed vertex's are overwritten by the lookup and naming kernels of the
  // step.  The cached key itself is read only by vertices that pass the touch
  // or filter test.
  constexpr int CV = 4;
  const bool vec = ((reinterpret_cast<uintptr_t>(mvc) | reinterpret_cast<uintptr_t>(rep) |
                     reinterpret_cast<uintptr_t>(names_out)) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(fkc) & 7) == 0 && (reinterpret_cast<uintptr_t>(dirty) & 3) == 0;
  // the list is appended with one atomic per workgroup and round (with many
  // dirty keys most vertices are listed, and per-wave atomics on the one
  // counter would serialise)
  __shared__ u32 sh_w[4];
  __shared__ int sh_base;
  const int64_t stride = (int64_t)gridDim.x * 256 * CV;
  for (int64_t b0 = (int64_t)blockIdx.x * 256 * CV; b0 < n; b0 += stride) {  // uniform in the workgroup
    const int64_t v0 = b0 + (int64_t)threadIdx.x * CV;
    int hd[CV];
    u32 fk[CV], dv[CV];
    const bool full = vec && v0 + CV <= n;
    if (full) {
      const u32 d4 = *reinterpret_cast<const u32 *>(dirty + v0);
      const int4 m4 = *reinterpret_cast<const int4 *>(mvc + v0);
      const uint2 f2 = *reinterpret_cast<const uint2 *>(fkc + v0);
      hd[0] = m4.x; hd[1] = m4.y; hd[2] = m4.z; hd[3] = m4.w;
      fk[0] = f2.x & 0xffffu; fk[1] = f2.x >> 16; fk[2] = f2.y & 0xffffu; fk[3] = f2.y >> 16;
#pragma unroll
      for (int j = 0; j < CV; ++j) dv[j] = (d4 >> (8 * j)) & 0xffu;
      *reinterpret_cast<int4 *>(rep + v0) = m4;
      *reinterpret_cast<int4 *>(names_out + v0) = m4;
    } else {
#pragma unroll
      for (int j = 0; j < CV; ++j) {
        const bool in = v0 + j < n;
        dv[j] = in ? dirty[v0 + j] : 1u;
        hd[j] = in ? mvc[v0 + j] : 0;
        fk[j] = in ? fkc[v0 + j] : 0u;
        if (in) {
          rep[v0 + j] = hd[j];
          names_out[v0 + j] = hd[j];
        }
      }
    }
    u32 tb[CV];
#pragma unroll
    for (int j = 0; j < CV; ++j) {
      // the touch bitmap is read only where the filter says "maybe touched"
      const u32 t = filter_touch_bit((u32)hd[j]);
      if (dv[j]) tb[j] = 1u;
      else if ((fl[t >> 5] >> (t & 31)) & 1u) tb[j] = (touch[hd[j] >> 5] >> (hd[j] & 31)) & 1u;
      else tb[j] = 0u;
    }
    // clean vertices that may share a key with a dirty one (filter hit) or
    // belong to a touched block read their cached key; all such loads are
    // requested before the first is used (with many dirty keys most vertices
    // take this path)
    bool probe[CV], need[CV];
#pragma unroll
    for (int j = 0; j < CV; ++j) {
      const bool clean = v0 + j < n && !dv[j];
      probe[j] = clean && !tb[j] && ((fl[fk[j] >> 5] >> (fk[j] & 31)) & 1u);
      need[j] = clean && (tb[j] || probe[j]);
    }
    u32 dc[CV];
    u64 hv[CV];
#pragma unroll
    for (int j = 0; j < CV; ++j) {
      dc[j] = need[j] ? DCc[v0 + j] : 0u;
      hv[j] = need[j] ? Hc[v0 + j] : 0ull;
    }
    bool listed[CV];
#pragma unroll
    for (int j = 0; j < CV; ++j) {
      const int v = (int)(v0 + j);
      listed[j] = v0 + j < n && dv[j];
      if (need[j]) {
        bool hit = !probe[j];  // touched
        if (probe[j]) {
          const u32 nm = dc[j] == 0 ? (u32)names[v] : 0u;
          bool maybe = true;
          if (gfilter) {
            const u32 g = dc[j] ? gfilter_key_bit(hv[j]) : gfilter_name_bit(nm);
            maybe = (gfilter[g >> 5] >> (g & 31)) & 1u;
          }
          if (maybe) {
            if (dc[j] == 0) hit = (u32)(zrep[nm] >> 32) == ~zep;
            else hit = table_lookup(table, tmask, hv[j], epoch) >= 0;
          }
        }
        if (hit) {
          H[v] = hv[j];
          DC[v] = dc[j];
          listed[j] = true;
        }
      }
    }
    u32 mine = 0;
#pragma unroll
    for (int j = 0; j < CV; ++j) mine += listed[j] ? 1u : 0u;
    if (!__syncthreads_or(mine != 0)) continue;  // most rounds with few dirty keys
    u32 total;
    u32 at = block_exclusive_scan(mine, sh_w, &total);
    if (threadIdx.x == 0) sh_base = atomicAdd(count, (int)total);
    __syncthreads();
    const int base = sh_base;
#pragma unroll
    for (int j = 0; j < CV; ++j)
      if (listed[j]) list[base + (int)at++] = (int)(v0 + j);
    __syncthreads();  // sh_base is rewritten in the next round
  }
}

// Inserts the listed vertices' keys (table, or zrep for empty signatures).
__global__ void __launch_bounds__(256) k_insert_list(int count, const int *__restrict__ list,
                                                     const u64 *__restrict__ H, const u32 *__restrict__ DC,
                                                     const int32_t *__restrict__ names, u64 *table, u64 tmask,
                                                     const u32 *__restrict__ dep, u64 *zrep) {
  const u32 epoch = dep[EP_TABLE], zep = dep[EP_ZERO];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool act = i < count;
  const int v = act ? list[i] : 0;
  const u32 dc = act ? DC[v] : 0;
  if (act && dc) table_insert(table, tmask, H[v], (u32)v, epoch);
  zero_insert_wave(zrep, act && dc == 0, act ? (u32)names[v] : 0u, (u32)v, zep);
}

// Row extents (begin, end) of listed vertices.
__global__ void k_row_extents(int count, const int *__restrict__ list, const int64_t *__restrict__ row_ptr,
                              int64_t *__restrict__ be) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int v = list[i];
  be[2 * i] = row_ptr[v];
  be[2 * i + 1] = row_ptr[v + 1];
}

// Row lengths of listed vertices.
__global__ void k_row_degrees(int count, const int *__restrict__ list, const int64_t *__restrict__ row_ptr,
                              int64_t *__restrict__ deg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int v = list[i];
  deg[i] = row_ptr[v + 1] - row_ptr[v];
}

// Dense id of every vertex: its representative's (head words).
__global__ void __launch_bounds__(256) k_assign_out(int n, const int *__restrict__ rep, HeadIds ids,
                                                    int *__restrict__ out) {
  const int64_t v0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * ASSIGN_V;
  if (v0 >= n) return;
  if (v0 + ASSIGN_V <= n && ((reinterpret_cast<uintptr_t>(rep) | reinterpret_cast<uintptr_t>(out)) & 15) == 0) {
    const int4 r4 = *reinterpret_cast<const int4 *>(rep + v0);
    *reinterpret_cast<int4 *>(out + v0) =
        make_int4(r4.x >= 0 ? head_id(ids, r4.x) : -1, r4.y >= 0 ? head_id(ids, r4.y) : -1,
                  r4.z >= 0 ? head_id(ids, r4.z) : -1, r4.w >= 0 ? head_id(ids, r4.w) : -1);
  } else {
    for (int64_t v = v0; v < v0 + ASSIGN_V && v < n; ++v) {
      const int r = rep[v];
      out[v] = r >= 0 ? head_id(ids, r) : -1;
    }
  }
}

// Block names of an update step.  A new block that keeps an unchanged
// (clean) member takes that member's cached name: clean members of one new
// block shared their cached block (their keys did not change), and no other
// new block holds a member of it, so such names stay distinct.  A block of
// changed vertices only is named n + its minimum vertex, above every cached
// name.  Clean vertices therefore never change names, and renaming does not
// spread through blocks that only gained or lost a few members.
// A block of changed vertices only that holds the vertex which named a cached
// block (old_names[v] == v), and whose cached name no clean member claimed,
// keeps that name (the smallest such vertex, so the choice is
// deterministic): a block whose members all changed keys but stayed
// together, e.g. a singleton, is not renamed.  No other new block can hold
// that vertex, so the name stays distinct.
// Each runs over every vertex, or over the `count` listed ones (list != NULL:
// the vertices of the blocks that can have changed; every other block keeps
// its members and its cached name).
__device__ inline int name_item(int n, int count, const int *list, bool &act) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  act = t < (list ? count : n);
  return act ? (list ? list[t] : t) : 0;
}
__global__ void k_block_names_fresh(int n, const int *__restrict__ rep, int32_t *__restrict__ bname,
                                    int32_t *__restrict__ keep, int count = 0, const int *__restrict__ list = nullptr) {
  bool act;
  const int v = name_item(n, count, list, act);
  if (act && rep[v] == v) {
    bname[v] = n + v;
    keep[v] = 0x7FFFFFFF;
  }
}
__global__ void k_block_names_clean(int n, const int *__restrict__ rep, const unsigned char *__restrict__ dirty,
                                    const int32_t *__restrict__ old_names, int32_t *__restrict__ bname,
                                    unsigned char *__restrict__ claimed, int count = 0,
                                    const int *__restrict__ list = nullptr) {
  bool act;
  const int v = name_item(n, count, list, act);
  if (act && !dirty[v]) {
    const int32_t nm = old_names[v];
    bname[rep[v]] = nm;
    claimed[nm] = 1;
  }
}
__global__ void k_block_names_keep(int n, const int *__restrict__ rep, const unsigned char *__restrict__ dirty,
                                   const int32_t *__restrict__ old_names, const int32_t *__restrict__ bname,
                                   const unsigned char *__restrict__ claimed, int32_t *keep, int count = 0,
                                   const int *__restrict__ list = nullptr) {
  bool act;
  const int v = name_item(n, count, list, act);
  if (act && dirty[v] && old_names[v] == v && !claimed[v]) {
    const int r = rep[v];
    if (bname[r] >= n) atomicMin(&keep[r], v);
  }
}

// Flags for the next step of an update: a vertex whose name changed, and every
// vertex with an edge into it (in-rows of the cached graph; an edge that an
// edit added starts at an edited row, which is recomputed at every step
// anyway).  One wave per changed vertex.
constexpr int MARK_LIGHT = 4096;  // in-rows up to this long are marked by one wave

__global__ void __launch_bounds__(256) k_mark_in_neighbours(const int *__restrict__ count, const int *__restrict__ list,
                                                            const int64_t *__restrict__ tptr,
                                                            const int32_t *__restrict__ tcol,
                                                            unsigned char *flag, int *nheavy, int *heavy) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int total = *count;
  const int waves = (int)((gridDim.x * blockDim.x) >> 6);
  for (int item = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); item < total; item += waves) {
    const int w = list[item];
    const int64_t b = tptr[w], e = tptr[w + 1];
    if (lane == 0) {
      flag[w] = 1;
      if (e - b > MARK_LIGHT) heavy[atomicAdd(nheavy, 1)] = w;
    }
    if (e - b <= MARK_LIGHT)
      for (int64_t j = b + lane; j < e; j += WAVE) flag[tcol[j]] = 1;
  }
}

// In-rows longer than MARK_LIGHT: every workgroup takes its share of each.
__global__ void __launch_bounds__(256) k_mark_heavy(const int *__restrict__ nheavy, const int *__restrict__ heavy,
                                                    const int64_t *__restrict__ tptr,
                                                    const int32_t *__restrict__ tcol, unsigned char *flag) {
  const int total = *nheavy;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int h = 0; h < total; ++h) {
    const int w = heavy[h];
    for (int64_t j = tptr[w] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < tptr[w + 1]; j += stride)
      flag[tcol[j]] = 1;
  }
}

// Per vertex of an update step: dirty = its key inputs may have changed
// (edited row, or flagged by the previous step); skip = not refined by the
// tier kernels (clean, or edited: edited rows are read from the edited graph
// by the list kernels).
// The flagged vertices whose rows were not edited are also listed, split by
// row length (as k_split_list), so that few of them can be signed by the list
// kernels instead of the tier kernels: counts at cnt[0] (short) and cnt[1]
// (up to LIST_BIG entries); longer rows are counted at cnt[2] and left to
// the row and hub tiers (skip[v] = 0 for exactly them).
// Bit mvc[v] of touch is set for every dirty v: its cached block may lose members;
// the dirty vertices are listed in dlist (count at cnt[4]).
constexpr int FLAGS_GROUP = 16;  // vertices per thread in k_update_flags
__global__ void __launch_bounds__(256) k_update_flags(int n, const unsigned char *__restrict__ edited,
                                                      const unsigned char *__restrict__ flag,
                                                      unsigned char *__restrict__ dirty,
                                                      unsigned char *__restrict__ skip,
                                                      const int64_t *__restrict__ row_ptr, int *cnt, int *small,
                                                      int *large, const int32_t *__restrict__ mvc,
                                                      u32 *__restrict__ touch, int *dlist) {
  // FLAGS_GROUP vertices per thread, their bytes moved 16 at a time where the
  // arrays allow.  Most groups are clean (no byte set in either input): one
  // load and one store of each array.  A group with a set byte decides per
  // vertex; its list members are appended once per wave (bit masks).
  const int64_t v0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * FLAGS_GROUP;
  const bool vec = v0 + FLAGS_GROUP <= n &&
                   ((reinterpret_cast<uintptr_t>(edited) | reinterpret_cast<uintptr_t>(flag) |
                     reinterpret_cast<uintptr_t>(dirty) | reinterpret_cast<uintptr_t>(skip)) & 15) == 0;
  u32 eb = 0, fb = 0;  // bit j: vertex v0 + j edited / flagged
  if (vec) {
    const u32x4 e = *reinterpret_cast<const u32x4 *>(edited + v0);
    const u32x4 f = *reinterpret_cast<const u32x4 *>(flag + v0);
#pragma unroll
    for (int j = 0; j < FLAGS_GROUP; ++j) {
      const u32 sh = 8 * (j & 3);
      const u32 ew = j < 4 ? e.x : j < 8 ? e.y : j < 12 ? e.z : e.w;
      const u32 fw = j < 4 ? f.x : j < 8 ? f.y : j < 12 ? f.z : f.w;
      eb |= (((ew >> sh) & 0xffu) != 0u ? 1u : 0u) << j;
      fb |= (((fw >> sh) & 0xffu) != 0u ? 1u : 0u) << j;
    }
  } else {
    for (int j = 0; j < FLAGS_GROUP && v0 + j < n; ++j) {
      eb |= (edited[v0 + j] != 0 ? 1u : 0u) << j;
      fb |= (flag[v0 + j] != 0 ? 1u : 0u) << j;
    }
  }
  const u32 mdirty = eb | fb, mprop = fb & ~eb;
  // row lengths of the flagged unedited vertices, all requested together
  int64_t d[FLAGS_GROUP];
#pragma unroll
  for (int j = 0; j < FLAGS_GROUP; ++j) d[j] = (mprop >> j) & 1u ? row_ptr[v0 + j + 1] - row_ptr[v0 + j] : 0;
  u32 msmall = 0, mlarge = 0, mbig = 0;
#pragma unroll
  for (int j = 0; j < FLAGS_GROUP; ++j) {
    if (!((mprop >> j) & 1u)) continue;
    if (d[j] <= LIST_SMALL) msmall |= 1u << j;
    else if (d[j] <= LIST_BIG) mlarge |= 1u << j;
    else mbig |= 1u << j;
  }
  // dirty = edited or flagged; skip = all but the flagged unedited rows past LIST_BIG
  if (vec) {
    u32 dw[4] = {0u, 0u, 0u, 0u}, sw[4] = {0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u};
#pragma unroll
    for (int j = 0; j < FLAGS_GROUP; ++j) {
      dw[j >> 2] |= ((mdirty >> j) & 1u) << (8 * (j & 3));
      sw[j >> 2] &= ~(((mbig >> j) & 1u) << (8 * (j & 3)));
    }
    *reinterpret_cast<u32x4 *>(dirty + v0) = u32x4{dw[0], dw[1], dw[2], dw[3]};
    *reinterpret_cast<u32x4 *>(skip + v0) = u32x4{sw[0], sw[1], sw[2], sw[3]};
  } else {
    for (int j = 0; j < FLAGS_GROUP && v0 + j < n; ++j) {
      dirty[v0 + j] = (mdirty >> j) & 1u;
      skip[v0 + j] = ((mbig >> j) & 1u) ? 0 : 1;
    }
  }
  // touch: the cached block of every dirty vertex (many share one: set its bit once)
  for (u32 m = mdirty; m; m &= m - 1u) {
    const int h = mvc[v0 + __ffs(m) - 1];
    const u32 bit = 1u << (h & 31);
    if (!(__hip_atomic_load(&touch[h >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit))
      atomicOr(&touch[h >> 5], bit);
  }
  if (!__ballot(mdirty != 0)) return;
  wave_append_mask(&cnt[0], small, msmall, v0);
  wave_append_mask(&cnt[1], large, mlarge, v0);
  wave_append_mask(&cnt[4], dlist, mdirty, v0);
  const u32 nbig = wave_sum_u32((u32)__popc(mbig));
  if ((threadIdx.x & (WAVE - 1)) == 0 && nbig) atomicAdd(&cnt[2], (int)nbig);
}

// Skip flags when every flagged unedited vertex goes to the tier kernels.
__global__ void k_skip_all_flagged(int n, const unsigned char *__restrict__ edited, const unsigned char *__restrict__ flag_dirty,
                                   unsigned char *__restrict__ skip) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) skip[v] = (flag_dirty[v] && !edited[v]) ? 0 : 1;
}

__global__ void k_set_flags(const int *__restrict__ count, const int *__restrict__ list, unsigned char *flag) {
  const int total = *count;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) flag[list[i]] = 1;
}

// ---------------------------------------------------------------- epochs
__global__ void k_advance(u32 *dep, u32 mask) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (mask & ADV_TABLE) {
    dep[EP_TABLE] = dep[EP_TABLE] % 15u + 1u;
    dep[EP_CLR_TABLE] = dep[EP_TABLE] == 1u;
  } else {
    dep[EP_CLR_TABLE] = 0;
  }
  if (mask & ADV_CTABLE) {
    dep[EP_CTABLE] = dep[EP_CTABLE] % 15u + 1u;
    dep[EP_CLR_CTABLE] = dep[EP_CTABLE] == 1u;
  } else {
    dep[EP_CLR_CTABLE] = 0;
  }
  if (mask & ADV_ZERO) dep[EP_ZERO] = dep[EP_ZERO] + 1u;
  if (mask & ADV_HUB) {
    dep[EP_HUB] = dep[EP_HUB] % 3u + 1u;
    dep[EP_CLR_HUB] = dep[EP_HUB] == 1u;
  } else {
    dep[EP_CLR_HUB] = 0;
  }
}

// Clears the tables whose epoch just wrapped (one launch; exits at once when
// nothing wrapped).
__global__ void k_clear_if(const u32 *__restrict__ dep, u64 *table, int64_t tslots, u64 *ctable, u64 *hub_sets,
                           int64_t hub_slots) {
  const bool ct = dep[EP_CLR_TABLE] != 0, cc = dep[EP_CLR_CTABLE] != 0, ch = dep[EP_CLR_HUB] != 0;
  if (!ct && !cc && !ch) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ct)
    for (int64_t i = i0; i < tslots; i += stride) table[i] = 0;
  if (cc)
    for (int64_t i = i0; i < tslots; i += stride) ctable[i] = 0;
  if (ch)
    for (int64_t i = i0; i < hub_slots; i += stride) hub_sets[i] = 0;
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
// One source copied to up to MAX destinations (read once).
struct CopyDsts {
  static constexpr int MAX = 16;
  int32_t *d[MAX];
  int nd;
};
__global__ void k_copy_multi(CopyDsts dst, const int32_t *__restrict__ src, int64_t cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uintptr_t a = reinterpret_cast<uintptr_t>(src);
  for (int q = 0; q < dst.nd; ++q) a |= reinterpret_cast<uintptr_t>(dst.d[q]);
  int64_t done = 0;
  if ((a & 15) == 0) {
    // 16 bytes per thread and step where every start is 16-byte aligned
    const int64_t n4 = cnt >> 2;
    for (int64_t i = t; i < n4; i += stride) {
      const int4 v = reinterpret_cast<const int4 *>(src)[i];
      for (int q = 0; q < dst.nd; ++q) reinterpret_cast<int4 *>(dst.d[q])[i] = v;
    }
    done = n4 << 2;
  }
  for (int64_t i = done + t; i < cnt; i += stride) {
    const int32_t v = src[i];
    for (int q = 0; q < dst.nd; ++q) dst.d[q][i] = v;
  }
}

// Streaming copy, 16 bytes per thread per step (bandwidth probe).
__global__ void k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Gather probe: every CSR entry reads its target's previous block through the
// same index and layout the signature kernels use (one streamed word, one
// random 4-byte gather), and nothing else.  Measures the random-gather rate
// the signature kernels are bounded by; one value per workgroup is written so
// the loads cannot be dropped.
template <class Src>
__global__ void __launch_bounds__(256) k_gather_probe(Src src, int64_t m, u32 *out, u32 omask) {
  u32 acc = 0;
  constexpr int U = 4;
  for (int64_t base = (int64_t)blockIdx.x * 256 * U; base < m; base += (int64_t)gridDim.x * 256 * U) {
    u32 v[U];
    const int cnt = (int)min<int64_t>(m - base, 256 * U);
    load_keys<u32, U, 256>(src, base, (int)threadIdx.x, cnt, v);
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u];
  }
  acc = wave_sum_u32(acc);
  if ((threadIdx.x & (WAVE - 1)) == 0) atomicAdd(&out[blockIdx.x & omask], acc);
}

}  // namespace kb
