/*
 * stepcheck.cpp — property checks of a computed partition chain, for sizes
 * at which the plain reference is too slow.  TEST INFRASTRUCTURE ONLY, like
 * the rest of this directory; it shares no code with the GPU library.
 *
 * It does not compute partitions; it checks a given one against the
 * definition:
 *
 *  check_initial(P0): ids are canonical (numbered by first vertex) and two
 *      vertices share a block iff their vertex-label SETS are equal (base
 *      case of Def. vertex-labeled-bw-bisimulation; no labels: P0 = {V}).
 *
 *  check_step(prev, cur): ids of cur are canonical, and cur is exactly the
 *      partition of V by the key (prev block, signature), the signature being
 *      the SET of (edge label, prev block of target) over the vertex's CSR
 *      entries (Def. edge-labeled-fw-bisimulation, Def. signature):
 *        (a) u, v in one cur block  =>  equal prev block and equal signature;
 *        (b) two different cur blocks  =>  different keys.
 *      (a) and (b) together say that cur is the key partition; canonical ids
 *      then make the array unique.
 *
 * Signatures are materialised per vertex (sorted, duplicates removed), so
 * the memory use is 8 bytes per CSR entry.  Work is spread over OpenMP
 * threads.
 */
#include <omp.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <memory>
#include <vector>

namespace {

enum {
  SC_OK = 0,
  SC_NONCANONICAL = -1,
  SC_NOT_REFINEMENT = -2,
  SC_SPLIT_SIGNATURE = -3,   // one block, two different keys
  SC_DUPLICATE_KEY = -4,     // two blocks, one key
  SC_BAD_INPUT = -5,
};

// Canonical ids: scanning v = 0..n-1, each id is either one already seen or
// exactly the next integer.  Fills first[b] = first vertex of block b.
int canonical(int64_t n, const int32_t *ids, std::vector<int64_t> &first, int64_t *bad) {
  first.clear();
  for (int64_t v = 0; v < n; ++v) {
    const int64_t b = ids[v];
    if (b < 0 || b > (int64_t)first.size()) {
      *bad = v;
      return SC_NONCANONICAL;
    }
    if (b == (int64_t)first.size()) first.push_back(v);
  }
  return SC_OK;
}

uint64_t poly_hash(const uint64_t *p, int64_t len) {
  uint64_t h = 0x6a09e667f3bcc909ull ^ (uint64_t)len;
  for (int64_t i = 0; i < len; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
    h ^= h >> 29;
  }
  return h;
}

// Sorted, duplicate-free item lists per vertex in one flat array.
// (Arrays are left uninitialised and first touched by the parallel fill.)
struct Lists {
  std::unique_ptr<uint64_t[]> vals;
  std::unique_ptr<int64_t[]> begin, len;
  bool same(int64_t a, int64_t b) const {
    return len[a] == len[b] &&
           (len[a] == 0 || std::memcmp(&vals[begin[a]], &vals[begin[b]], 8 * (size_t)len[a]) == 0);
  }
  const uint64_t *at(int64_t v) const { return vals.get() + begin[v]; }
};

template <class Item>
void build_lists(int64_t n, const int64_t *ptr, Item item, Lists &L) {
  const int64_t total = ptr[n] - ptr[0];
  L.vals.reset(new uint64_t[(size_t)std::max<int64_t>(total, 1)]);
  L.begin.reset(new int64_t[(size_t)std::max<int64_t>(n, 1)]);
  L.len.reset(new int64_t[(size_t)std::max<int64_t>(n, 1)]);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    const int64_t b = ptr[v] - ptr[0], e = ptr[v + 1] - ptr[0];
    uint64_t *p = L.vals.get() + b;
    for (int64_t i = b; i < e; ++i) p[i - b] = item(i + ptr[0]);
    std::sort(p, p + (e - b));
    L.begin[v] = b;
    L.len[v] = std::unique(p, p + (e - b)) - p;
  }
}

// The partition `ids` (canonical, first[]) must be exactly the partition by
// (own[v], list(v)); own may be null (then only lists count).
int check_key_partition(int64_t n, const int32_t *ids, const std::vector<int64_t> &first, const int32_t *own,
                        const Lists &L, int64_t *bad) {
  int64_t bad_own = -1, bad_list = -1;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    const int64_t h = first[(size_t)ids[v]];
    if (h == v) continue;
    if (own && own[v] != own[h]) {
#pragma omp critical
      if (bad_own < 0 || v < bad_own) bad_own = v;
    } else if (!L.same(v, h)) {
#pragma omp critical
      if (bad_list < 0 || v < bad_list) bad_list = v;
    }
  }
  if (bad_own >= 0) {
    *bad = bad_own;
    return SC_NOT_REFINEMENT;
  }
  if (bad_list >= 0) {
    *bad = bad_list;
    return SC_SPLIT_SIGNATURE;
  }
  struct K {
    int64_t own;
    uint64_t h;
    int64_t head;
  };
  const int64_t nb = (int64_t)first.size();
  std::vector<K> keys((size_t)nb);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t h = first[(size_t)b];
    keys[(size_t)b] = K{own ? (int64_t)own[h] : 0, poly_hash(L.at(h), L.len[h]), h};
  }
  std::sort(keys.begin(), keys.end(), [](const K &a, const K &b) {
    return a.own != b.own ? a.own < b.own : (a.h != b.h ? a.h < b.h : a.head < b.head);
  });
  // equal (own, hash) runs: every pair inside a run must differ exactly
  int64_t bad_b = -1;
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < nb; ++i) {
    if (i > 0 && keys[i - 1].own == keys[i].own && keys[i - 1].h == keys[i].h) continue;
    int64_t j = i + 1;
    while (j < nb && keys[j].own == keys[i].own && keys[j].h == keys[i].h) ++j;
    for (int64_t a = i; a < j; ++a)
      for (int64_t b = a + 1; b < j; ++b)
        if (L.same(keys[a].head, keys[b].head)) {
#pragma omp critical
          if (bad_b < 0 || keys[b].head < bad_b) bad_b = std::max(keys[a].head, keys[b].head);
        }
  }
  if (bad_b >= 0) {
    *bad = bad_b;
    return SC_DUPLICATE_KEY;
  }
  return SC_OK;
}

}  // namespace

extern "C" {

int stepcheck_threads(int threads) {
  if (threads > 0) omp_set_num_threads(threads);
  return omp_get_max_threads();
}

// Returns the block count (>= 0) if P0 is right, else a negative code; *bad
// receives a vertex where the check failed.
int64_t stepcheck_initial(int64_t n, const int64_t *vlabel_ptr, const int32_t *vlabel, const int32_t *p0,
                          int64_t *bad) {
  *bad = -1;
  if (n < 0 || !p0) return SC_BAD_INPUT;
  std::vector<int64_t> first;
  int rc = canonical(n, p0, first, bad);
  if (rc) return rc;
  Lists L;
  if (vlabel_ptr) {
    build_lists(n, vlabel_ptr, [&](int64_t i) { return (uint64_t)(uint32_t)vlabel[i]; }, L);
  } else if (vlabel) {
    std::vector<int64_t> ptr((size_t)n + 1);
    for (int64_t v = 0; v <= n; ++v) ptr[(size_t)v] = v;
    build_lists(n, ptr.data(), [&](int64_t i) { return (uint64_t)(uint32_t)vlabel[i]; }, L);
  } else {
    std::vector<int64_t> ptr((size_t)n + 1, 0);
    build_lists(n, ptr.data(), [&](int64_t) { return (uint64_t)0; }, L);
  }
  rc = check_key_partition(n, p0, first, nullptr, L, bad);
  return rc ? rc : (int64_t)first.size();
}

// Returns the block count of cur (>= 0) if cur is the refinement step of
// prev, else a negative code.
int64_t stepcheck_step(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *elabel,
                       const int32_t *prev, const int32_t *cur, int64_t *bad) {
  *bad = -1;
  if (n < 0 || !row_ptr || !prev || !cur || (row_ptr[n] > 0 && !col)) return SC_BAD_INPUT;
  std::vector<int64_t> first;
  int rc = canonical(n, cur, first, bad);
  if (rc) return rc;
  Lists L;
  build_lists(n, row_ptr, [&](int64_t i) {
    const uint64_t l = elabel ? (uint64_t)(uint32_t)elabel[i] : 0;
    return (l << 32) | (uint64_t)(uint32_t)prev[col[i]];
  }, L);
  rc = check_key_partition(n, cur, first, prev, L, bad);
  return rc ? rc : (int64_t)first.size();
}

}  // extern "C"
