/*
 * graphgen — seeded synthetic multi-relational labeled graphs.
 *
 * This module only produces inputs: vertex ids, edge lists, edge labels and
 * vertex label sets, laid out as CSR arrays.  It holds none of the
 * refinement arithmetic; both the CPU reference and the GPU library read the
 * arrays it writes.
 *
 * Random numbers are counter based: every draw is a pure function of
 * (seed, stream, index), built on the SplitMix64 output function of
 * Steele, Lea and Flood ("Fast splittable pseudorandom number generators",
 * OOPSLA 2014).  Draw i of a stream is mix64(key(seed, stream) + (i+1)*gamma),
 * so every thread count produces bit-identical graphs.
 *
 * Probabilities are turned into integer thresholds once (a 64-bit or 32-bit
 * CDF table) and draws are compared against them as integers, so the same
 * thresholds give the same choices everywhere.
 *
 * The graph data model is the multi-relational labeled graph of the paper's
 * data-structures section (Def. multi-relational-labeled-property-graph):
 * directed edges with one label per edge entry (RDF triple view) and a finite,
 * possibly empty, set of labels per vertex.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Stream key: a mixed function of the seed and a stream tag. */
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return sm_mix(sm_mix(seed + GAMMA) ^ (stream * 0xD1B54A32D192ED03ULL + 0x8CB92BA72F3D8DD7ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t i) { return sm_mix(key + (i + 1) * GAMMA); }

/* Uniform integer in [0, n) by 64x64->128 multiply-high (Lemire). */
static inline uint64_t below(uint64_t r, uint64_t n) {
  return (uint64_t)(((unsigned __int128)r * (unsigned __int128)n) >> 64);
}

/* Stream tags. */
enum {
  ST_RMAT = 1, ST_ER_SRC, ST_ER_DST, ST_ELABEL, ST_VLABEL, ST_VSIZE, ST_VSET,
  ST_SCRAMBLE, ST_BATCH, ST_PERM
};

uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t i) { return draw(stream_key(seed, stream), i); }

/* ------------------------------------------------------------------------- */
/* Vertex-id scrambling: a seeded bijection on [0, 2^bits).                  */
/* Each round is (x*odd + c) mod 2^bits followed by x ^= x >> s; both steps  */
/* are invertible on bits-wide integers, so the composition is a bijection.  */
/* ------------------------------------------------------------------------- */
typedef struct { uint64_t mul[4], add[4]; int bits; uint64_t mask; } scramble_t;

static void scramble_init(scramble_t *s, uint64_t seed, int bits) {
  uint64_t key = stream_key(seed, ST_SCRAMBLE);
  s->bits = bits;
  s->mask = bits >= 64 ? ~0ULL : ((1ULL << bits) - 1);
  for (int r = 0; r < 4; ++r) {
    s->mul[r] = (draw(key, 2 * r) | 1ULL) & s->mask;
    if (s->mul[r] == 0) s->mul[r] = 1;
    s->add[r] = draw(key, 2 * r + 1) & s->mask;
  }
}

static inline uint64_t scramble(const scramble_t *s, uint64_t x) {
  if (s->bits <= 1) return x;
  int sh = (s->bits + 1) / 2;
  for (int r = 0; r < 4; ++r) {
    x = (x * s->mul[r] + s->add[r]) & s->mask;
    x ^= x >> sh;
  }
  return x;
}

uint64_t gg_scramble(uint64_t seed, int bits, uint64_t x) {
  scramble_t s; scramble_init(&s, seed, bits); return scramble(&s, x);
}

/* ------------------------------------------------------------------------- */
/* Edge generators.                                                          */
/* ------------------------------------------------------------------------- */

/* RMAT (Chakrabarti, Zhan, Faloutsos, SDM 2004) without noise: each edge
 * descends `scale` levels; at every level quadrant a/b/c/d is chosen with the
 * given probabilities; c and d set the source bit, b and d the target bit.
 * Two levels are drawn from one 64-bit draw (32 bits each).  If `scramble_ids`
 * is set, both endpoints go through the seeded bijection (Graph500 style).  */
void gg_rmat_edges(uint64_t seed, int scale, int64_t m, double a, double b, double c,
                   int scramble_ids, int32_t *src, int32_t *dst) {
  const double tot = a + b + c + (1.0 - a - b - c);
  (void)tot;
  const uint64_t TA = (uint64_t)llround(a * 4294967296.0);
  const uint64_t TAB = (uint64_t)llround((a + b) * 4294967296.0);
  const uint64_t TABC = (uint64_t)llround((a + b + c) * 4294967296.0);
  const uint64_t key = stream_key(seed, ST_RMAT);
  scramble_t sc; scramble_init(&sc, seed, scale);
  const int per_edge = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t s = 0, t = 0;
    int lvl = 0;
    for (int j = 0; j < per_edge; ++j) {
      uint64_t r = draw(key, (uint64_t)e * (uint64_t)per_edge + (uint64_t)j);
      for (int h = 0; h < 2 && lvl < scale; ++h, ++lvl) {
        uint64_t u = (h == 0) ? (r & 0xFFFFFFFFULL) : (r >> 32);
        int sb, tb;
        if (u < TA) { sb = 0; tb = 0; }
        else if (u < TAB) { sb = 0; tb = 1; }
        else if (u < TABC) { sb = 1; tb = 0; }
        else { sb = 1; tb = 1; }
        s = (s << 1) | (uint64_t)sb;
        t = (t << 1) | (uint64_t)tb;
      }
    }
    if (scramble_ids) { s = scramble(&sc, s); t = scramble(&sc, t); }
    src[e] = (int32_t)s;
    dst[e] = (int32_t)t;
  }
}

/* Uniform random directed edges (Erdos-Renyi G(n, m) with replacement). */
void gg_uniform_edges(uint64_t seed, int64_t n, int64_t m, int32_t *src, int32_t *dst) {
  const uint64_t ks = stream_key(seed, ST_ER_SRC), kd = stream_key(seed, ST_ER_DST);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    src[e] = (int32_t)below(draw(ks, (uint64_t)e), (uint64_t)n);
    dst[e] = (int32_t)below(draw(kd, (uint64_t)e), (uint64_t)n);
  }
}

/* ------------------------------------------------------------------------- */
/* Label distributions.                                                      */
/* ------------------------------------------------------------------------- */

/* Integer CDF for uniform (zipf_s <= 0) or Zipf(s) over L labels: rank i has
 * weight 1/(i+1)^s.  cdf[i] = floor(2^64 * P(X <= i)); cdf[L-1] = UINT64_MAX. */
static uint64_t *make_cdf(int64_t L, double zipf_s) {
  uint64_t *cdf = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)L);
  if (!cdf) return NULL;
  if (zipf_s <= 0.0) {
    for (int64_t i = 0; i < L; ++i) cdf[i] = 0; /* unused: uniform draws use below() */
    return cdf;
  }
  long double total = 0.0L;
  for (int64_t i = 0; i < L; ++i) total += 1.0L / powl((long double)(i + 1), (long double)zipf_s);
  long double acc = 0.0L;
  for (int64_t i = 0; i < L; ++i) {
    acc += 1.0L / powl((long double)(i + 1), (long double)zipf_s);
    long double f = acc / total;
    if (i == L - 1 || f >= 1.0L) cdf[i] = UINT64_MAX;
    else cdf[i] = (uint64_t)(f * 18446744073709551616.0L);
  }
  return cdf;
}

static inline int32_t sample(const uint64_t *cdf, int64_t L, double zipf_s, uint64_t r) {
  if (zipf_s <= 0.0) return (int32_t)below(r, (uint64_t)L);
  int64_t lo = 0, hi = L - 1; /* first i with r <= cdf[i] ... use r < cdf[i] with cdf[L-1]=max */
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (r < cdf[mid]) hi = mid; else lo = mid + 1;
  }
  return (int32_t)lo;
}

/* One label per element i in [0, count): uniform or Zipf(s) over L. */
int gg_labels(uint64_t seed, uint64_t stream, int64_t count, int64_t L, double zipf_s, int32_t *out) {
  uint64_t *cdf = make_cdf(L, zipf_s);
  if (!cdf) return -1;
  const uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) out[i] = sample(cdf, L, zipf_s, draw(key, (uint64_t)i));
  free(cdf);
  return 0;
}

int gg_edge_labels(uint64_t seed, int64_t m, int64_t L, double zipf_s, int32_t *out) {
  return gg_labels(seed, ST_ELABEL, m, L, zipf_s, out);
}

int gg_vertex_labels(uint64_t seed, int64_t n, int64_t L, double zipf_s, int32_t *out) {
  return gg_labels(seed, ST_VLABEL, n, L, zipf_s, out);
}

/* Label-set sizes: size j in [0, nsizes) with probability probs[j]. */
int gg_vertex_set_sizes(uint64_t seed, int64_t n, const double *probs, int nsizes, int64_t *ptr) {
  uint64_t cdf[64];
  if (nsizes < 1 || nsizes > 64) return -1;
  long double acc = 0.0L, tot = 0.0L;
  for (int j = 0; j < nsizes; ++j) tot += probs[j];
  for (int j = 0; j < nsizes; ++j) {
    acc += probs[j];
    long double f = acc / tot;
    cdf[j] = (j == nsizes - 1 || f >= 1.0L) ? UINT64_MAX : (uint64_t)(f * 18446744073709551616.0L);
  }
  const uint64_t key = stream_key(seed, ST_VSIZE);
  ptr[0] = 0;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    uint64_t r = draw(key, (uint64_t)v);
    int j = 0;
    while (j < nsizes - 1 && r >= cdf[j]) ++j;
    ptr[v + 1] = j;
  }
  for (int64_t v = 0; v < n; ++v) ptr[v + 1] += ptr[v];
  return 0;
}

/* Fill each vertex's label set with distinct labels drawn from the
 * uniform/Zipf distribution over L; draws are attempt-indexed so the result
 * does not depend on the thread count.  Sets are written in draw order.      */
int gg_vertex_set_labels(uint64_t seed, int64_t n, const int64_t *ptr, int64_t L, double zipf_s,
                         int32_t *out) {
  uint64_t *cdf = make_cdf(L, zipf_s);
  if (!cdf) return -1;
  const uint64_t key = stream_key(seed, ST_VSET);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t v = 0; v < n; ++v) {
    int64_t b = ptr[v], sz = ptr[v + 1] - ptr[v];
    if (sz > L) { bad = 1; continue; }
    int64_t have = 0;
    for (uint64_t att = 0; have < sz; ++att) {
      int32_t lab = sample(cdf, L, zipf_s, draw(key, (uint64_t)v * 4096ULL + att));
      int dup = 0;
      for (int64_t j = 0; j < have; ++j) if (out[b + j] == lab) { dup = 1; break; }
      if (!dup) out[b + have++] = lab;
      if (att > 100000) { bad = 1; break; }
    }
  }
  free(cdf);
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* CSR construction: stable LSD radix sort of edges by source, so each row   */
/* keeps the edges in generation order.                                      */
/* ------------------------------------------------------------------------- */
int gg_build_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *lbl,
                 int64_t *row_ptr, int32_t *col, int32_t *elabel) {
  memset(row_ptr, 0, sizeof(int64_t) * (size_t)(n + 1));
  if (n <= 0 || m <= 0) return 0;
  int nt = omp_get_max_threads();
  if (nt < 1) nt = 1;
  /* Two-level stable counting sort: first by the high part of src (about
   * 2^14 buckets, each thread handling one contiguous slice of the edge list
   * so the pass is stable), then by src within each bucket.                  */
  int bits = 1;
  while ((1LL << bits) < n) ++bits;
  int shift = bits > 14 ? bits - 14 : 0;
  int64_t nb = ((n - 1) >> shift) + 1;
  int64_t *hist = (int64_t *)calloc((size_t)nb * (size_t)nt, sizeof(int64_t));
  int64_t *bstart = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
  int64_t *tmp_idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
  if (!hist || !bstart || !tmp_idx) { free(hist); free(bstart); free(tmp_idx); return -1; }
  int64_t chunk = (m + nt - 1) / nt;
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int64_t lo = (int64_t)t * chunk, hi = lo + chunk < m ? lo + chunk : m;
    int64_t *h = hist + (size_t)t * (size_t)nb;
    for (int64_t e = lo; e < hi; ++e) h[src[e] >> shift]++;
  }
  int64_t run = 0;
  for (int64_t bkt = 0; bkt < nb; ++bkt) {
    bstart[bkt] = run;
    for (int t = 0; t < nt; ++t) {
      int64_t c = hist[(size_t)t * (size_t)nb + bkt];
      hist[(size_t)t * (size_t)nb + bkt] = run;
      run += c;
    }
  }
  bstart[nb] = run;
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int64_t lo = (int64_t)t * chunk, hi = lo + chunk < m ? lo + chunk : m;
    int64_t *h = hist + (size_t)t * (size_t)nb;
    for (int64_t e = lo; e < hi; ++e) tmp_idx[h[src[e] >> shift]++] = e;
  }
  /* degrees: every vertex belongs to exactly one bucket */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t bkt = 0; bkt < nb; ++bkt)
    for (int64_t i = bstart[bkt]; i < bstart[bkt + 1]; ++i) row_ptr[(int64_t)src[tmp_idx[i]] + 1]++;
  for (int64_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
  /* scatter, stable within each bucket */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t bkt = 0; bkt < nb; ++bkt) {
    int64_t v0 = bkt << shift;
    int64_t v1 = (bkt + 1) << shift;
    if (v1 > n) v1 = n;
    int64_t nv = v1 - v0;
    if (nv <= 0) continue;
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nv);
    for (int64_t v = 0; v < nv; ++v) fill[v] = row_ptr[v0 + v];
    for (int64_t i = bstart[bkt]; i < bstart[bkt + 1]; ++i) {
      int64_t e = tmp_idx[i];
      int64_t pos = fill[src[e] - v0]++;
      col[pos] = dst[e];
      if (elabel) elabel[pos] = lbl ? lbl[e] : 0;
    }
    free(fill);
  }
  free(bstart);
  free(hist);
  free(tmp_idx);
  return 0;
}

/* Degree histogram helper for reporting: counts[d] for d < maxd, counts[maxd] = rest. */
void gg_degree_hist(int64_t n, const int64_t *row_ptr, int64_t maxd, int64_t *counts) {
  for (int64_t d = 0; d <= maxd; ++d) counts[d] = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = row_ptr[v + 1] - row_ptr[v];
    counts[d < maxd ? d : maxd]++;
  }
}

int gg_num_threads(void) { return omp_get_max_threads(); }
