/*
 * oracle.cpp — plain sequential CPU reference for k-bisimulation partition
 * refinement.  TEST INFRASTRUCTURE ONLY: it is called by the test-suite, by
 * the smoke check and by the benchmark's CPU-baseline leg, never by the GPU
 * library.  It shares no code with the GPU path.
 *
 * What it computes (the plain definition, written out):
 *
 *  P0 — the vertex-labeled base case of Def. vertex-labeled-bw-bisimulation:
 *       u ~0 v iff l_V(u) = l_V(v), with l_V(v) a (possibly empty) SET of
 *       labels (Def. multi-relational-labeled-property-graph).  With no
 *       vertex labels at all, P0 = {V} (the initialisation of
 *       Alg. schaetzle-alg).
 *
 *  P_{i} from P_{i-1} — the step of Def. edge-labeled-fw-bisimulation:
 *       u ~i v iff u ~(i-1) v and the sets of (edge label, target block)
 *       pairs over their out-edges are equal.  That set is the signature of
 *       Def. signature, so the key of v is (block_{i-1}(v), sig_{i-1}(v)),
 *       sig as a sorted, duplicate-free vector (set semantics).
 *
 *  Block ids are dense and numbered by first vertex: scanning v = 0..n-1,
 *  each key not seen before receives the next integer.  The paper names
 *  blocks by hash values (Def. id); dense first-vertex numbering is the
 *  collision-free naming adopted here so that any two correct
 *  implementations produce identical arrays.
 *
 *  Edge semantics: one label per CSR entry (the RDF triple view of the
 *  introduction); parallel entries and self-loops are kept; a missing
 *  edge-label array means all edges share label 0.  Backward refinement is
 *  the same computation on the transposed graph (Def. inverse-schema-element).
 *
 * Every iteration is always computed, also past the fixpoint.
 */
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <map>
#include <utility>
#include <vector>

namespace {

/* Planted-mistake switch for the test-suite's mutation tests (0 = none).
 * Each nonzero value injects one plausible implementation error so that the
 * tests can show that the pins catch it.  Production of reference results
 * always runs with 0.                                                        */
int g_mutation = 0;
enum {
  MUT_NONE = 0,
  MUT_MULTISET = 1,        /* keep duplicate pairs (multiset signature)       */
  MUT_NO_OLD_BLOCK = 2,    /* key without the vertex's own previous block     */
  MUT_NO_EDGE_LABEL = 3,   /* pairs without the edge label                    */
  MUT_SOURCE_BLOCK = 4,    /* pair carries the source's block, not the target's */
  MUT_KEY_ORDER_IDS = 5,   /* ids numbered in key order, not by first vertex  */
  MUT_DROP_LAST_EDGE = 6,  /* off-by-one: last CSR entry of each row skipped  */
  MUT_P0_NO_LABELS = 7,    /* P0 ignores vertex labels                        */
  MUT_P0_FIRST_LABEL = 8,  /* P0 compares only the first label of each set    */
};

int check_csr(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const int32_t *elabel) {
  if (n < 0 || m < 0 || n >= (int64_t(1) << 31)) return -1;
  if (!row_ptr) return -1;
  if (row_ptr[0] != 0 || row_ptr[n] != m) return -2;
  for (int64_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return -2;
  for (int64_t e = 0; e < m; ++e) {
    if (col[e] < 0 || col[e] >= n) return -2;
    if (elabel && elabel[e] < 0) return -2;
  }
  return 0;
}

/* P0 by label-set equality, numbered by first vertex. */
int64_t initial_partition(int64_t n, const int64_t *vlabel_ptr, const int32_t *vlabel, int32_t *out) {
  std::map<std::vector<int32_t>, int32_t> ids;
  for (int64_t v = 0; v < n; ++v) {
    std::vector<int32_t> labels;
    if (vlabel_ptr) {
      for (int64_t j = vlabel_ptr[v]; j < vlabel_ptr[v + 1]; ++j) labels.push_back(vlabel[j]);
    } else if (vlabel) {
      labels.push_back(vlabel[v]);
    }
    if (g_mutation == MUT_P0_NO_LABELS) labels.clear();
    if (g_mutation == MUT_P0_FIRST_LABEL && labels.size() > 1) labels.resize(1);
    std::sort(labels.begin(), labels.end());
    labels.erase(std::unique(labels.begin(), labels.end()), labels.end());
    out[v] = ids.emplace(labels, (int32_t)ids.size()).first->second;
  }
  return (int64_t)ids.size();
}

/* One refinement step: prev -> next, returns the number of blocks. */
int64_t refine_step(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *elabel,
                    const int32_t *prev, int32_t *next) {
  typedef std::pair<int32_t, std::vector<uint64_t>> Key;
  std::map<Key, int32_t> ids;
  for (int64_t v = 0; v < n; ++v) {
    std::vector<uint64_t> sig;
    int64_t end = row_ptr[v + 1];
    if (g_mutation == MUT_DROP_LAST_EDGE && end > row_ptr[v]) --end;
    for (int64_t e = row_ptr[v]; e < end; ++e) {
      uint64_t label = elabel ? (uint64_t)(uint32_t)elabel[e] : 0;
      uint64_t block = (uint64_t)(uint32_t)prev[col[e]];
      if (g_mutation == MUT_NO_EDGE_LABEL) label = 0;
      if (g_mutation == MUT_SOURCE_BLOCK) block = (uint64_t)(uint32_t)prev[v];
      sig.push_back((label << 32) | block);
    }
    std::sort(sig.begin(), sig.end());
    if (g_mutation != MUT_MULTISET) sig.erase(std::unique(sig.begin(), sig.end()), sig.end());
    int32_t own = (g_mutation == MUT_NO_OLD_BLOCK) ? 0 : prev[v];
    next[v] = ids.emplace(Key(own, std::move(sig)), (int32_t)ids.size()).first->second;
  }
  if (g_mutation == MUT_KEY_ORDER_IDS) {
    /* renumber blocks by key order instead of first vertex */
    std::vector<int32_t> rank(ids.size());
    int32_t r = 0;
    for (auto &kv : ids) rank[kv.second] = r++;
    for (int64_t v = 0; v < n; ++v) next[v] = rank[next[v]];
  }
  return (int64_t)ids.size();
}

}  // namespace

extern "C" {

/* Test hook: select a planted mistake (see the MUT_ values); 0 restores the
 * correct reference.  Returns the previous setting.                          */
int oracle_set_mutation(int mutation) {
  int old = g_mutation;
  g_mutation = mutation;
  return old;
}

/* P0 only.  Returns 0 or a negative code. */
int oracle_initial(int64_t n, const int64_t *vlabel_ptr, const int32_t *vlabel, int32_t *out_ids,
                   int64_t *out_count) {
  if (n < 0 || n >= (int64_t(1) << 31) || (n > 0 && !out_ids) || !out_count) return -1;
  if (vlabel_ptr && !vlabel && vlabel_ptr[n] > 0) return -1;
  *out_count = initial_partition(n, vlabel_ptr, vlabel, out_ids);
  return 0;
}

/* Starting from `start` (the caller's P_i, or P0 when start == NULL), compute
 * k further partitions.  out_ids is k*n int32 (partition j+1 at offset j*n),
 * out_counts is k int64, iter_seconds (optional) receives per-iteration wall
 * times.  Returns 0, -1 (bad argument) or -2 (invalid graph).               */
int oracle_refine(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col, const int32_t *elabel,
                  const int64_t *vlabel_ptr, const int32_t *vlabel, const int32_t *start, int k,
                  int32_t *out_ids, int64_t *out_counts, double *iter_seconds) {
  if (k < 0 || (k > 0 && (!out_counts || (n > 0 && !out_ids)))) return -1;
  int rc = check_csr(n, m, row_ptr, col, elabel);
  if (rc) return rc;
  std::vector<int32_t> p0((size_t)n);
  if (start) {
    std::copy(start, start + n, p0.begin());
  } else {
    initial_partition(n, vlabel_ptr, vlabel, p0.data());
  }
  const int32_t *prev = p0.data();
  for (int i = 0; i < k; ++i) {
    auto t0 = std::chrono::steady_clock::now();
    int32_t *next = out_ids + (size_t)i * (size_t)n;
    out_counts[i] = refine_step(n, row_ptr, col, elabel, prev, next);
    auto t1 = std::chrono::steady_clock::now();
    if (iter_seconds) iter_seconds[i] = std::chrono::duration<double>(t1 - t0).count();
    prev = next;
  }
  return 0;
}

}  // extern "C"
