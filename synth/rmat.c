/*
 * rmat.c -- seeded synthetic graph generator (R-MAT / Kronecker-style).
 *
 * Input generation only: it holds none of the clustering method's arithmetic
 * and serves the CPU oracle and the GPU path alike.
 *
 * Each of M edge samples picks one quadrant per level with probabilities
 * (a, b, c, d); the random numbers come from a counter-based generator
 * (SplitMix64's output function applied to key + counter * golden gamma), so a
 * sample depends only on (seed, sample index) and the result does not depend
 * on the thread count.  The graph is made undirected (each sample gives arcs
 * u->v and v->u), self-loops are dropped, every adjacency list is sorted and
 * duplicates are removed.  Output: CSR with int64 offsets and int32 ids.
 *
 * Two passes over the samples (count, then fill) keep the peak memory at the
 * size of the final arc array plus the offsets.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* The j-th 64-bit draw of sample i under `key`. */
static inline uint64_t draw(uint64_t key, uint64_t i, uint64_t j) {
  return sm64_out(key + (i * 32u + j + 1u) * GOLDEN);
}

static inline void sample(uint64_t key, uint64_t i, int scale, uint32_t ta, uint32_t tab,
                          uint32_t tabc, uint32_t* pu, uint32_t* pv) {
  uint32_t u = 0, v = 0;
  uint64_t bits = 0;
  for (int l = 0; l < scale; l++) {
    uint32_t x;
    if ((l & 1) == 0) { bits = draw(key, i, (uint64_t)(l >> 1)); x = (uint32_t)bits; }
    else x = (uint32_t)(bits >> 32);
    u <<= 1; v <<= 1;
    if (x < ta) { /* quadrant a */ }
    else if (x < tab) { v |= 1; }
    else if (x < tabc) { u |= 1; }
    else { u |= 1; v |= 1; }
  }
  *pu = u; *pv = v;
}

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x > y) - (x < y);
}

/*
 * Generate an R-MAT graph with 2^scale vertices from nsamples edge samples.
 * Probabilities a, b, c (d = 1-a-b-c).  On success *off_out (n+1) and
 * *nbr_out (off[n]) are malloc'd and owned by the caller (free with
 * synth_free).  Returns the arc count or -1.
 */
int64_t synth_rmat(int scale, int64_t nsamples, double a, double b, double c, uint64_t seed,
                   int64_t** off_out, int32_t** nbr_out) {
  if (scale < 1 || scale > 31 || nsamples < 0) return -1;
  int64_t n = (int64_t)1 << scale;
  uint64_t key = sm64_out(seed + GOLDEN);
  double s = 4294967296.0;
  uint32_t ta = (uint32_t)(a * s), tab = (uint32_t)((a + b) * s), tabc = (uint32_t)((a + b + c) * s);

  int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!off) return -1;
  int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  if (!cnt) { free(off); return -1; }

#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nsamples; i++) {
    uint32_t u, v;
    sample(key, (uint64_t)i, scale, ta, tab, tabc, &u, &v);
    if (u == v) continue;
#pragma omp atomic
    cnt[u]++;
#pragma omp atomic
    cnt[v]++;
  }
  for (int64_t v = 0; v < n; v++) off[v + 1] = off[v] + cnt[v];
  int64_t arcs = off[n];
  int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(arcs > 0 ? arcs : 1));
  if (!nbr) { free(off); free(cnt); return -1; }
  memcpy(cnt, off, sizeof(int64_t) * (size_t)n); /* fill cursors */

#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nsamples; i++) {
    uint32_t u, v;
    sample(key, (uint64_t)i, scale, ta, tab, tabc, &u, &v);
    if (u == v) continue;
    int64_t pu, pv;
#pragma omp atomic capture
    pu = cnt[u]++;
#pragma omp atomic capture
    pv = cnt[v]++;
    nbr[pu] = (int32_t)v;
    nbr[pv] = (int32_t)u;
  }

  /* Sort and deduplicate each row; cnt[v] becomes the new degree. */
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; v++) {
    int64_t lo = off[v], hi = off[v + 1];
    uint32_t* row = (uint32_t*)(nbr + lo);
    int64_t d = hi - lo;
    if (d > 1) qsort(row, (size_t)d, sizeof(uint32_t), cmp_u32);
    int64_t k = 0;
    for (int64_t j = 0; j < d; j++)
      if (k == 0 || row[j] != row[k - 1]) row[k++] = row[j];
    cnt[v] = k;
  }
  /* Compact rows to the front (new offsets never exceed the old ones). */
  int64_t w = 0;
  for (int64_t v = 0; v < n; v++) {
    int64_t lo = off[v], d = cnt[v];
    if (w != lo && d > 0) memmove(nbr + w, nbr + lo, sizeof(int32_t) * (size_t)d);
    off[v] = w;
    w += d;
  }
  off[n] = w;
  free(cnt);
  int32_t* shrunk = (int32_t*)realloc(nbr, sizeof(int32_t) * (size_t)(w > 0 ? w : 1));
  if (shrunk) nbr = shrunk;
  *off_out = off;
  *nbr_out = nbr;
  return w;
}

void synth_free(void* p) { free(p); }

/* Copy helper so that Python can move the arrays into numpy buffers. */
void synth_copy(void* dst, const void* src, int64_t bytes) { memcpy(dst, src, (size_t)bytes); }
