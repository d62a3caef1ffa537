/*
 * Multicore CPU PR-Nibble + sweep cut: the paper's shared-memory design
 * (round-synchronous push, Sec. 3.3; sweep cut, Sec. 3.1) run with OpenMP on
 * the host's cores.  A measurement baseline reported beside the oracle; it
 * shares no code with the oracle or with the GPU path.
 *
 * Per round: snapshot rho for the frontier, update p and r of the frontier
 * (vertexMap), then every frontier vertex adds (cn rho)/d to its neighbours
 * with an atomic fetch-add (edgeMap); a neighbour whose r crosses eps d in
 * its own add joins the next frontier.  Dense p and r are kept for the
 * graph's lifetime and reset through the touched list after each query.
 * The sweep sorts the support by p/d (ties by id), counts each vertex's
 * earlier-ranked neighbours in parallel and scans for the best prefix.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* growable per-thread list: appends need no shared counter */
struct tlist {
  int32_t* a;
  int64_t n, cap;
};

static inline int tpush(struct tlist* l, int32_t v) {
  if (l->n == l->cap) {
    int64_t c = l->cap ? 2 * l->cap : 4096;
    int32_t* a = (int32_t*)realloc(l->a, sizeof(int32_t) * (size_t)c);
    if (!a) return -1;
    l->a = a;
    l->cap = c;
  }
  l->a[l->n++] = v;
  return 0;
}

typedef struct {
  int64_t n;
  double* p;
  double* r;
  int32_t* rank;
  int32_t* fa;      /* frontier */
  int32_t* fb;      /* next frontier */
  int32_t* touched;
  int32_t* support;
  int32_t* tmp;     /* merge buffer of the sweep sort */
  double* rho;      /* frontier snapshot */
  int64_t* delta;   /* boundary deltas of the sweep */
  int64_t nt, ns;
  int nthr;
  struct tlist* tl; /* per-thread append buffers: 3 per thread */
} cmc_state;

typedef struct {
  int32_t rounds;
  int64_t pushes, edges, support, kstar, cut, vol;
  double phi;
} cmc_result;

void cmc_destroy(cmc_state* s) {
  if (!s) return;
  free(s->p); free(s->r); free(s->rank); free(s->fa); free(s->fb); free(s->touched);
  free(s->support); free(s->tmp); free(s->rho); free(s->delta);
  if (s->tl)
    for (int i = 0; i < 3 * s->nthr; i++) free(s->tl[i].a);
  free(s->tl);
  free(s);
}

cmc_state* cmc_create(int64_t n) {
  cmc_state* s = (cmc_state*)calloc(1, sizeof(cmc_state));
  if (!s) return NULL;
  s->n = n;
  s->p = (double*)calloc((size_t)n, sizeof(double));
  s->r = (double*)calloc((size_t)n, sizeof(double));
  s->rank = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  s->fa = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  s->fb = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  s->touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  s->support = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  s->tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  s->rho = (double*)malloc(sizeof(double) * (size_t)n);
  s->delta = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  s->nthr = omp_get_max_threads();
  s->tl = (struct tlist*)calloc(3 * (size_t)s->nthr, sizeof(struct tlist));
  if (!s->p || !s->r || !s->rank || !s->fa || !s->fb || !s->touched || !s->support || !s->tmp ||
      !s->rho || !s->delta || !s->tl) {
    cmc_destroy(s);
    return NULL;
  }
  return s;
}


/* move every thread's list k onto the end of dst; returns the new length */
static int64_t gather(cmc_state* s, int k, int32_t* dst, int64_t len) {
  for (int t = 0; t < s->nthr; t++) {
    struct tlist* l = &s->tl[3 * t + k];
    memcpy(dst + len, l->a, sizeof(int32_t) * (size_t)l->n);
    len += l->n;
    l->n = 0;
  }
  return len;
}

/* sweep order: p/d descending, ties by ascending id */
static inline int before(const double* p, const int64_t* off, int32_t a, int32_t b) {
  const double ka = p[a] / (double)(off[a + 1] - off[a]);
  const double kb = p[b] / (double)(off[b + 1] - off[b]);
  return ka > kb || (ka == kb && a < b);
}

static void insertion_sort(const double* p, const int64_t* off, int32_t* x, int64_t n) {
  for (int64_t i = 1; i < n; i++) {
    const int32_t v = x[i];
    int64_t j = i;
    while (j > 0 && before(p, off, v, x[j - 1])) { x[j] = x[j - 1]; j--; }
    x[j] = v;
  }
}

static void merge(const double* p, const int64_t* off, const int32_t* a, int64_t na,
                  const int32_t* b, int64_t nb, int32_t* out) {
  int64_t i = 0, j = 0, k = 0;
  while (i < na && j < nb) out[k++] = before(p, off, b[j], a[i]) ? b[j++] : a[i++];
  while (i < na) out[k++] = a[i++];
  while (j < nb) out[k++] = b[j++];
}

/* bottom-up merge sort: runs of 32 by insertion, then passes of parallel merges */
static int32_t* sort_support(const double* p, const int64_t* off, int32_t* x, int32_t* tmp,
                             int64_t n) {
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < n; s += 32) insertion_sort(p, off, x + s, n - s < 32 ? n - s : 32);
  for (int64_t w = 32; w < n; w *= 2) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n; s += 2 * w) {
      const int64_t m = s + w < n ? s + w : n, e = s + 2 * w < n ? s + 2 * w : n;
      merge(p, off, x + s, m - s, x + m, e - m, tmp + s);
    }
    int32_t* t = x; x = tmp; tmp = t;
  }
  return x;
}

/* p/r of the finished query stay in s until the next call (for tests).
   Returns 0, -1 for invalid input, -2 when host memory ran out (the state is
   then unusable: destroy it). */
int cmc_run(cmc_state* s, const int64_t* off, const int32_t* nbr, int32_t seed, double alpha,
            double eps, int32_t rule, int32_t max_rounds, cmc_result* res) {
  const int64_t n = s->n;
  memset(res, 0, sizeof(*res));
  if (seed < 0 || seed >= n || off[seed + 1] == off[seed]) return -1;
  if (!(alpha > 0.0 && alpha < 1.0) || !(eps > 0.0) || !isfinite(eps)) return -1;
  /* reset the previous query through its touched and support lists */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < s->nt; i++) s->r[s->touched[i]] = 0.0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < s->ns; i++) { s->p[s->support[i]] = 0.0; s->rank[s->support[i]] = 0; }
  s->nt = s->ns = 0;
  double cs, cn, keep;
  if (rule == 1) { cs = alpha; cn = (1.0 - alpha) / 2.0; keep = (1.0 - alpha) / 2.0; }
  else { cs = 2.0 * alpha / (1.0 + alpha); cn = (1.0 - alpha) / (1.0 + alpha); keep = 0.0; }
  double* rho = s->rho;
  s->r[seed] = 1.0;
  s->touched[s->nt++] = seed;
  int64_t nf = 1;
  s->fa[0] = seed;
  int oom = 0;
  while (nf > 0 && res->rounds < max_rounds) {
    int64_t edges = 0;
#pragma omp parallel reduction(+ : edges) reduction(| : oom)
    {
      const int t = omp_get_thread_num();
      struct tlist* fr = &s->tl[3 * t];     /* next frontier */
      struct tlist* to = &s->tl[3 * t + 1]; /* newly touched */
      struct tlist* su = &s->tl[3 * t + 2]; /* newly supported */
      /* vertexMap: snapshot, p, r (a pushed vertex keeps -0.0 under the
         optimized rule, so it is not listed as touched again); vertices the
         original rule leaves above the threshold stay in the frontier */
#pragma omp for schedule(static)
      for (int64_t i = 0; i < nf; i++) {
        const int32_t v = s->fa[i];
        const double rv = s->r[v];
        rho[i] = rv;
        if (s->p[v] == 0.0) oom |= tpush(su, v);
        s->p[v] += cs * rv;
        s->r[v] = keep > 0.0 ? keep * rv : -0.0;
        const int64_t d = off[v + 1] - off[v];
        edges += d;
        if (keep > 0.0 && keep * rv >= eps * (double)d) oom |= tpush(fr, v);
      }
      /* edgeMap: fetch-add into r; the add that crosses eps d lists the
         neighbour in the next frontier (contributions are positive, so
         exactly one add crosses) */
#pragma omp for schedule(dynamic, 64) nowait
      for (int64_t i = 0; i < nf; i++) {
        const int32_t v = s->fa[i];
        const int64_t d = off[v + 1] - off[v];
        const double c = (cn * rho[i]) / (double)d;
        for (int64_t e = off[v]; e < off[v + 1]; e++) {
          const int32_t w = nbr[e];
          double old;
#pragma omp atomic capture
          { old = s->r[w]; s->r[w] += c; }
          if (old == 0.0 && !signbit(old)) oom |= tpush(to, w);
          const double thr = eps * (double)(off[w + 1] - off[w]);
          if (old < thr && old + c >= thr) oom |= tpush(fr, w);
        }
      }
    }
    if (oom) return -2;
    res->rounds++;
    res->pushes += nf;
    res->edges += edges;
    nf = gather(s, 0, s->fb, 0);
    s->nt = gather(s, 1, s->touched, s->nt);
    s->ns = gather(s, 2, s->support, s->ns);
    int32_t* t = s->fa; s->fa = s->fb; s->fb = t;
  }
  /* sweep: order, rank, boundary deltas, prefix scan, exact argmin */
  const int64_t N = s->ns;
  res->support = N;
  int32_t* sorted = sort_support(s->p, off, s->support, s->tmp, N);
  if (sorted != s->support) { s->tmp = s->support; s->support = sorted; }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < N; k++) s->rank[s->support[k]] = (int32_t)(k + 1);
  int64_t* delta = s->delta;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < N; k++) {
    const int32_t v = s->support[k];
    int64_t earlier = 0;
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      const int32_t rw = s->rank[nbr[e]];
      earlier += rw > 0 && rw <= k;
    }
    delta[k] = (off[v + 1] - off[v]) - 2 * earlier;
  }
  const int64_t vt = off[n];
  int64_t cut = 0, vol = 0, bc = 0, bd = 1, bv = 0, bk = 0;
  for (int64_t k = 0; k < N; k++) {
    const int32_t v = s->support[k];
    cut += delta[k];
    vol += off[v + 1] - off[v];
    const int64_t den = vol < vt - vol ? vol : vt - vol;
    if (den <= 0) continue;
    if (bk == 0 || (__int128)cut * bd < (__int128)bc * den) { bc = cut; bd = den; bv = vol; bk = k + 1; }
  }
  res->kstar = bk;
  res->cut = bk ? bc : 0;
  res->vol = bk ? bv : 0;
  res->phi = bk ? (double)bc / (double)bd : INFINITY;
  return 0;
}

/* Copies for tests: dense p and r of the last query, and its sweep order. */
void cmc_vectors(const cmc_state* s, double* p, double* r, int32_t* order) {
  memcpy(p, s->p, sizeof(double) * (size_t)s->n);
  memcpy(r, s->r, sizeof(double) * (size_t)s->n);
  memcpy(order, s->support, sizeof(int32_t) * (size_t)s->ns);
}

int cmc_threads(void) { return omp_get_max_threads(); }
