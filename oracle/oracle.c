/*
 * oracle.c -- plain, slow, single-threaded CPU oracle for round-synchronous
 * PR-Nibble and the sweep cut of Shun, Roosta-Khorasani, Fountoulakis and
 * Mahoney, "Parallel Local Graph Clustering" (arXiv 1604.07515).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * helper with the GPU path.
 *
 * Arithmetic: IEEE-754 binary64 throughout, built without fast-math and with
 * -ffp-contract=off so that every multiply and add below rounds separately,
 * in the order written.  Every summation follows one fixed order (ascending
 * frontier ids, then CSR order of each adjacency list), so the oracle is
 * deterministic.
 *
 * Graph format: undirected, unweighted, CSR with int64 row offsets off[n+1]
 * and int32 neighbour ids nbr[off[n]]; every undirected edge appears as two
 * arcs; d(v) = off[v+1]-off[v]  (Sec. 2, "Graph Notation").
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORACLE_OK 0
#define ORACLE_E_INVALID (-1)
#define ORACLE_E_NOMEM (-2)
#define ORACLE_LIMIT 1

#define ORACLE_RULE_OPT 0  /* optimized push rule, Sec. 3.3 "An Optimization" */
#define ORACLE_RULE_ORIG 1 /* original push rule, Sec. 3.3, Fig. alg:pr-nibble */

typedef struct {
  int64_t rounds;      /* iterations of the while loop that pushed something */
  int64_t pushes;      /* sum over rounds of |Frontier|                      */
  int64_t edges;       /* sum over rounds of sum_{v in Frontier} d(v)        */
  int64_t support;     /* |{v : p[v] > 0}| at exit                           */
  double min_rel_gap;  /* min over filter candidates of |r[u]-eps d(u)|/(eps d(u)) */
  int32_t max_frontier;
  int32_t status;      /* ORACLE_OK or ORACLE_LIMIT                          */
} oracle_push_stats;

typedef struct {
  int64_t N;      /* support size |{v : p[v] > 0}|                 */
  int64_t kstar;  /* number of vertices in the best prefix (>= 1)  */
  int64_t cut;    /* |boundary(S_kstar)|                           */
  int64_t vol;    /* vol(S_kstar)                                  */
  int64_t den;    /* min(vol, 2m - vol)                            */
  double phi;     /* cut / den                                     */
  int64_t vol_total; /* 2m                                         */
} oracle_sweep_result;

static int64_t deg_of(const int64_t* off, int64_t v) { return off[v + 1] - off[v]; }

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Push-rule constants (Sec. 3.3).  Original rule: p += alpha r,
 * r[w] += (1-alpha) r / (2 d), r[v] = (1-alpha) r / 2.  Optimized rule:
 * p += (2 alpha/(1+alpha)) r, r[w] += ((1-alpha)/(1+alpha)) r / d, r[v] = 0.
 * Dividing by 2 is exact in binary, so cn*rho/d with cn=(1-alpha)/2 equals
 * (1-alpha)*rho/(2d) bit for bit. */
static void rule_constants(int rule, double alpha, double* cs, double* cn, double* keep) {
  if (rule == ORACLE_RULE_ORIG) {
    *cs = alpha;
    *cn = (1.0 - alpha) / 2.0;
    *keep = (1.0 - alpha) / 2.0;
  } else {
    *cs = 2.0 * alpha / (1.0 + alpha);
    *cn = (1.0 - alpha) / (1.0 + alpha);
    *keep = 0.0;
  }
}

/*
 * Round-synchronous parallel PR-Nibble (Sec. 3.3 "Parallel Implementation",
 * Fig. alg:pr-nibble with the update functions of Fig. alg:pr-nibble2 for the
 * optimized rule), executed one round at a time on one core.
 *
 * Each round: every frontier vertex pushes the residual it held at the start
 * of the round (rho_v); UpdateSelf (vertexMap) is applied to all frontier
 * vertices before any UpdateNgh (edgeMap) contribution lands; the next
 * frontier is {u in F u N(F) : r[u] >= eps d(u)} (the filter).  The seed is
 * placed on the first frontier unconditionally, as the pseudocode does.
 *
 * p and r are dense caller arrays of length n; they are overwritten.
 * round_sizes (optional, length max_rounds) receives |F| of each round.
 * Returns ORACLE_OK, ORACLE_LIMIT (max_rounds reached with a non-empty
 * frontier) or a negative error.
 */
int oracle_prnibble(int64_t n, const int64_t* off, const int32_t* nbr, const int32_t* seeds,
                    int32_t nseeds, double alpha, double eps, int32_t rule, int64_t max_rounds,
                    double* p, double* r, int32_t* round_sizes, oracle_push_stats* st) {
  if (n <= 0 || !off || !nbr || !seeds || nseeds <= 0 || !p || !r || !st) return ORACLE_E_INVALID;
  if (!(alpha > 0.0 && alpha < 1.0) || !(eps > 0.0) || !isfinite(eps)) return ORACLE_E_INVALID;
  if (rule != ORACLE_RULE_OPT && rule != ORACLE_RULE_ORIG) return ORACLE_E_INVALID;
  for (int32_t i = 0; i < nseeds; i++) {
    if (seeds[i] < 0 || seeds[i] >= n || deg_of(off, seeds[i]) <= 0) return ORACLE_E_INVALID;
  }
  double cs, cn, keep;
  rule_constants(rule, alpha, &cs, &cn, &keep);

  memset(st, 0, sizeof(*st));
  st->min_rel_gap = INFINITY;
  for (int64_t v = 0; v < n; v++) { p[v] = 0.0; r[v] = 0.0; }

  int64_t cap = 1024, ccap = 1024;
  if (cap < nseeds) cap = nseeds;
  int32_t* F = (int32_t*)malloc(sizeof(int32_t) * cap);
  double* rho = (double*)malloc(sizeof(double) * cap);
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * ccap);
  uint8_t* mark = (uint8_t*)calloc((size_t)n, 1);
  if (!F || !rho || !cand || !mark) { free(F); free(rho); free(cand); free(mark); return ORACLE_E_NOMEM; }

  /* Initial residual: all mass on the seed (several seeds share it equally). */
  int64_t nf = 0;
  for (int32_t i = 0; i < nseeds; i++) {
    int32_t x = seeds[i];
    if (!mark[x]) { mark[x] = 1; F[nf++] = x; }
  }
  for (int64_t i = 0; i < nf; i++) { mark[F[i]] = 0; r[F[i]] = 1.0 / (double)nf; }
  qsort(F, (size_t)nf, sizeof(int32_t), cmp_i32);

  int status = ORACLE_OK;
  while (nf > 0) {
    if (st->rounds >= max_rounds) { status = ORACLE_LIMIT; break; }
    if (round_sizes) round_sizes[st->rounds] = (int32_t)nf;
    if (nf > st->max_frontier) st->max_frontier = (int32_t)nf;

    /* Snapshot of the residual at the start of the round. */
    for (int64_t i = 0; i < nf; i++) rho[i] = r[F[i]];
    /* vertexMap(Frontier, UpdateSelf). */
    for (int64_t i = 0; i < nf; i++) {
      int32_t v = F[i];
      p[v] = p[v] + cs * rho[i];
      r[v] = keep * rho[i];
    }
    /* edgeMap(G, Frontier, UpdateNgh), in ascending frontier / CSR order. */
    int64_t round_edges = 0;
    for (int64_t i = 0; i < nf; i++) {
      int32_t v = F[i];
      int64_t d = deg_of(off, v);
      double c = (cn * rho[i]) / (double)d;
      for (int64_t e = off[v]; e < off[v + 1]; e++) {
        int32_t w = nbr[e];
        r[w] = r[w] + c;
      }
      round_edges += d;
    }
    st->pushes += nf;
    st->edges += round_edges;
    st->rounds += 1;

    /* Filter over F and its neighbours (the only entries that changed). */
    int64_t nc = 0;
    for (int64_t i = 0; i < nf; i++) {
      int32_t v = F[i];
      int64_t need = nc + 1 + deg_of(off, v);
      if (need > ccap) {
        while (ccap < need) ccap *= 2;
        int32_t* t = (int32_t*)realloc(cand, sizeof(int32_t) * ccap);
        if (!t) { status = ORACLE_E_NOMEM; goto done; }
        cand = t;
      }
      if (!mark[v]) { mark[v] = 1; cand[nc++] = v; }
      for (int64_t e = off[v]; e < off[v + 1]; e++) {
        int32_t w = nbr[e];
        if (!mark[w]) { mark[w] = 1; cand[nc++] = w; }
      }
    }
    int64_t nn = 0;
    for (int64_t i = 0; i < nc; i++) {
      int32_t u = cand[i];
      mark[u] = 0;
      double thr = eps * (double)deg_of(off, u);
      double gap = fabs(r[u] - thr) / thr;
      if (gap < st->min_rel_gap) st->min_rel_gap = gap;
      if (r[u] >= thr) cand[nn++] = u;
    }
    if (nn > cap) {
      while (cap < nn) cap *= 2;
      int32_t* t1 = (int32_t*)realloc(F, sizeof(int32_t) * cap);
      if (t1) F = t1;
      double* t2 = (double*)realloc(rho, sizeof(double) * cap);
      if (t2) rho = t2;
      if (!t1 || !t2) { status = ORACLE_E_NOMEM; goto done; }
    }
    memcpy(F, cand, sizeof(int32_t) * (size_t)nn);
    nf = nn;
    qsort(F, (size_t)nf, sizeof(int32_t), cmp_i32);
  }
  for (int64_t v = 0; v < n; v++) st->support += (p[v] > 0.0);
done:
  st->status = status;
  free(F); free(rho); free(cand); free(mark);
  return status;
}

/* ---------------------------------------------------------------- sweep */

typedef struct { double key; int32_t id; } sweep_item;

/* Non-increasing p[v]/d(v); equal ratios in ascending vertex id. */
static int cmp_sweep(const void* a, const void* b) {
  const sweep_item* x = (const sweep_item*)a;
  const sweep_item* y = (const sweep_item*)b;
  if (x->key > y->key) return -1;
  if (x->key < y->key) return 1;
  return (x->id > y->id) - (x->id < y->id);
}

/* Ordered support {v_1..v_N} of p (Sec. 3.1): vertices with p[v] > 0 sorted by
 * non-increasing p[v]/d(v), ties by ascending id.  Returns N or <0. */
int64_t oracle_sweep_order(int64_t n, const int64_t* off, const double* p, int32_t* order) {
  int64_t N = 0;
  for (int64_t v = 0; v < n; v++) {
    if (p[v] > 0.0) {
      if (deg_of(off, v) <= 0) return ORACLE_E_INVALID;
      N++;
    }
  }
  sweep_item* it = (sweep_item*)malloc(sizeof(sweep_item) * (size_t)(N > 0 ? N : 1));
  if (!it) return ORACLE_E_NOMEM;
  int64_t k = 0;
  for (int64_t v = 0; v < n; v++)
    if (p[v] > 0.0) { it[k].key = p[v] / (double)deg_of(off, v); it[k].id = (int32_t)v; k++; }
  qsort(it, (size_t)N, sizeof(sweep_item), cmp_sweep);
  for (int64_t i = 0; i < N; i++) order[i] = it[i].id;
  free(it);
  return N;
}

/* a/b < c/d for non-negative a, c and positive b, d, exactly. */
static int ratio_less(int64_t a, int64_t b, int64_t c, int64_t d) {
  return (__int128)a * (__int128)d < (__int128)c * (__int128)b;
}

/* Best prefix by exact rational comparison; the first (smallest) k wins ties;
 * prefixes with den = 0 are excluded. */
static void pick_best(int64_t N, const int64_t* cut, const int64_t* vol, int64_t vt,
                      oracle_sweep_result* res) {
  res->N = N;
  res->kstar = 0; res->cut = 0; res->vol = 0; res->den = 0; res->phi = INFINITY;
  res->vol_total = vt;
  for (int64_t k = 0; k < N; k++) {
    int64_t den = vol[k] < vt - vol[k] ? vol[k] : vt - vol[k];
    if (den <= 0) continue;
    if (res->kstar == 0 || ratio_less(cut[k], den, res->cut, res->den)) {
      res->kstar = k + 1; res->cut = cut[k]; res->vol = vol[k]; res->den = den;
    }
  }
  if (res->kstar > 0) res->phi = (double)res->cut / (double)res->den;
}

/*
 * Sequential sweep cut (Sec. 3.1): add v_1, v_2, ... one at a time, keeping
 * vol(S) and |boundary(S)|; for each edge (v_i, w): w already in S decrements
 * the boundary, otherwise increments it.  cut[k-1], vol[k-1] describe S_k.
 */
int oracle_sweep(int64_t n, const int64_t* off, const int32_t* nbr, const double* p,
                 int32_t* order, int64_t* cut, int64_t* vol, oracle_sweep_result* res) {
  int64_t N = oracle_sweep_order(n, off, p, order);
  if (N < 0) return (int)N;
  uint8_t* in = (uint8_t*)calloc((size_t)n, 1);
  if (!in) return ORACLE_E_NOMEM;
  int64_t c = 0, vl = 0;
  for (int64_t k = 0; k < N; k++) {
    int32_t v = order[k];
    vl += deg_of(off, v);
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      if (in[nbr[e]]) c -= 1; else c += 1;
    }
    in[v] = 1;
    cut[k] = c; vol[k] = vl;
  }
  free(in);
  pick_best(N, cut, vol, off[n], res);
  return ORACLE_OK;
}

/*
 * Brute force: every prefix S_k is rebuilt from scratch and its volume and
 * boundary recounted straight from the definitions (Sec. 2).  O(N * vol);
 * for small inputs only.
 */
int oracle_sweep_bruteforce(int64_t n, const int64_t* off, const int32_t* nbr,
                            const int32_t* order, int64_t N, int64_t* cut, int64_t* vol,
                            oracle_sweep_result* res) {
  uint8_t* in = (uint8_t*)malloc((size_t)n);
  if (!in) return ORACLE_E_NOMEM;
  for (int64_t k = 0; k < N; k++) {
    memset(in, 0, (size_t)n);
    for (int64_t i = 0; i <= k; i++) in[order[i]] = 1;
    int64_t c = 0, vl = 0;
    for (int64_t i = 0; i <= k; i++) {
      int32_t v = order[i];
      vl += deg_of(off, v);
      for (int64_t e = off[v]; e < off[v + 1]; e++) c += !in[nbr[e]];
    }
    cut[k] = c; vol[k] = vl;
  }
  free(in);
  pick_best(N, cut, vol, off[n], res);
  return ORACLE_OK;
}

/*
 * The construction in the proof of Theorem 1 (Sec. 3.1), written out: ranks
 * 1..N for the ordered support, N+1 outside; for every arc (v, w) of a support
 * vertex, the pair (1, rank v), (-1, rank w) when rank w > rank v, else
 * (0, rank v), (0, rank w); a stable sort of the pairs by their second value;
 * an inclusive prefix sum of the first values; and the boundary of S_i read
 * at the last pair whose second value is i.
 *
 * Z holds 2*vol(S_N) pairs as zf (first values) and zs (second values); the
 * sorted and summed arrays are returned too so that they can be compared with
 * the worked example.  cut[i-1] receives |boundary(S_i)|.
 */
int oracle_sweep_z(int64_t n, const int64_t* off, const int32_t* nbr, const int32_t* order,
                   int64_t N, int32_t* zf, int64_t* zs, int32_t* zf_sorted, int64_t* zs_sorted,
                   int64_t* z_summed, int64_t* cut) {
  int64_t* rank = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!rank) return ORACLE_E_NOMEM;
  for (int64_t v = 0; v < n; v++) rank[v] = N + 1;
  for (int64_t i = 0; i < N; i++) rank[order[i]] = i + 1;
  int64_t len = 0;
  for (int64_t i = 0; i < N; i++) {
    int32_t v = order[i];
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      int64_t rv = rank[v], rw = rank[nbr[e]];
      if (rw > rv) { zf[len] = 1; zs[len] = rv; zf[len + 1] = -1; zs[len + 1] = rw; }
      else { zf[len] = 0; zs[len] = rv; zf[len + 1] = 0; zs[len + 1] = rw; }
      len += 2;
    }
  }
  /* Stable counting sort by the second value (ranks 1..N+1). */
  int64_t* cnt = (int64_t*)calloc((size_t)(N + 3), sizeof(int64_t));
  if (!cnt) { free(rank); return ORACLE_E_NOMEM; }
  for (int64_t j = 0; j < len; j++) cnt[zs[j] + 1]++;
  for (int64_t k = 1; k < N + 3; k++) cnt[k] += cnt[k - 1];
  for (int64_t j = 0; j < len; j++) {
    int64_t pos = cnt[zs[j]]++;
    zf_sorted[pos] = zf[j]; zs_sorted[pos] = zs[j];
  }
  int64_t acc = 0;
  for (int64_t j = 0; j < len; j++) { acc += zf_sorted[j]; z_summed[j] = acc; }
  for (int64_t i = 0; i < N; i++) cut[i] = 0;
  for (int64_t j = 0; j < len; j++) {
    int64_t rk = zs_sorted[j];
    int last = (j + 1 == len) || (zs_sorted[j + 1] != rk);
    if (last && rk >= 1 && rk <= N) cut[rk - 1] = z_summed[j];
  }
  free(cnt); free(rank);
  return (int)len;
}

/* ------------------------------------------------------------------------
 * Deterministic heat-kernel PageRank, HK-PR (Sec. 3.4, the Kloster-Gleich
 * procedure and Fig. alg:hkpr).  Parameters: seed x, Taylor degree N >= 1,
 * eps > 0, t > 0.
 *
 *   psi_k = sum_{m=0}^{N-k} k!/(m+k)! t^m  (k = 0..N), accumulated term by
 *           term with term_0 = 1, term_m = term_{m-1} * t / (k + m);
 *   threshold at level k for vertex w:  ((e^{-t} * eps) * d(w)) / (2 * N * psi_k);
 *   an entry (v, j) that is processed adds r to p[v]; for j + 1 < N each
 *   neighbour w gets t * r / ((j + 1) d(v)) at level j + 1, and (w, j + 1) is
 *   processed once its residual reaches the level-(j+1) threshold; for
 *   j + 1 == N each neighbour w gets r / d(v) added to p[w] directly.
 *
 * Readings: the pseudocode's loop test "j+1 == N" and its e^{t} contradict
 * the text; the text's "j+1 < N" and e^{-t} are taken.  Threshold and
 * crossing test are inclusive (>=), as for PR-Nibble.  eps > 0: at eps = 0
 * the printed crossing test (r < thr before the update) can never hold and
 * the sequential procedure would stop at the seed, while the filter of the
 * figure would push every touched entry; the two agree for every eps > 0.
 * ------------------------------------------------------------------------ */

typedef struct {
  int64_t levels;      /* levels processed (the last one pushes into p) */
  int64_t pushes;      /* entries processed */
  int64_t edges;       /* sum of d(v) over processed entries */
  int64_t support;     /* vertices with p > 0 */
  double min_rel_gap;  /* closest approach of a threshold decision to its threshold */
} oracle_hk_stats;

static void hk_psi(int32_t N, double t, double* psi) {
  for (int32_t k = 0; k <= N; k++) {
    double term = 1.0, s = 1.0;
    for (int32_t m = 1; m <= N - k; m++) {
      term = term * t / (double)(k + m);
      s += term;
    }
    psi[k] = s;
  }
}

static double hk_thr(double et_eps, int64_t d, int32_t N, double psi_k) {
  return (et_eps * (double)d) / (2.0 * (double)N * psi_k);
}

static void hk_gap(oracle_hk_stats* st, double r, double thr) {
  const double g = fabs(r - thr) / thr;
  if (g < st->min_rel_gap) st->min_rel_gap = g;
}

/*
 * Level-synchronous HK-PR (Fig. alg:hkpr, with the readings above): the
 * frontier of level j pushes; r holds level j (on the vertices that level
 * touched), rn collects level j + 1 with every contribution added (the
 * fetch-and-add of the figure, here in edge order); the next frontier is
 * every vertex whose level-(j+1) residual reached its threshold, and level
 * j's residuals, pushed or not, are dropped.  p dense, length n,
 * overwritten.
 */
int oracle_hkpr(int64_t n, const int64_t* off, const int32_t* nbr, int32_t x, int32_t N,
                double eps, double t, double* p, oracle_hk_stats* st) {
  if (n <= 0 || !off || !nbr || !p || !st || N < 1) return ORACLE_E_INVALID;
  if (x < 0 || x >= n || deg_of(off, x) <= 0) return ORACLE_E_INVALID;
  if (!(eps > 0.0) || !isfinite(eps) || !(t > 0.0) || !isfinite(t)) return ORACLE_E_INVALID;
  double* psi = (double*)malloc(sizeof(double) * (size_t)(N + 1));
  double* r = (double*)calloc((size_t)n, sizeof(double));
  double* rn = (double*)calloc((size_t)n, sizeof(double));
  int32_t* F = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);   /* frontier of level j */
  int32_t* T = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);   /* touched at level j */
  int32_t* G = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);   /* touched at level j + 1 */
  uint8_t* mark = (uint8_t*)calloc((size_t)n, 1);
  if (!psi || !r || !rn || !F || !T || !G || !mark) {
    free(psi); free(r); free(rn); free(F); free(T); free(G); free(mark);
    return ORACLE_E_NOMEM;
  }
  hk_psi(N, t, psi);
  const double et_eps = exp(-t) * eps;
  memset(st, 0, sizeof(*st));
  st->min_rel_gap = INFINITY;
  for (int64_t v = 0; v < n; v++) p[v] = 0.0;
  r[x] = 1.0;
  int64_t nf = 1, nt = 1;
  F[0] = x;
  T[0] = x;
  for (int32_t j = 0; nf > 0; j++) {
    st->levels++;
    /* vertexMap(Frontier, UpdateSelf) */
    for (int64_t i = 0; i < nf; i++) p[F[i]] += r[F[i]];
    st->pushes += nf;
    if (j + 1 == N) {  /* last level: edgeMap with UpdateNghLast */
      for (int64_t i = 0; i < nf; i++) {
        const int32_t v = F[i];
        const int64_t d = deg_of(off, v);
        st->edges += d;
        const double c = r[v] / (double)d;
        for (int64_t e = off[v]; e < off[v + 1]; e++) p[nbr[e]] += c;
      }
      break;
    }
    /* edgeMap(G, Frontier, UpdateNgh) into rn */
    int64_t ng = 0;
    for (int64_t i = 0; i < nf; i++) {
      const int32_t v = F[i];
      const int64_t d = deg_of(off, v);
      st->edges += d;
      const double c = (t * r[v]) / ((double)(j + 1) * (double)d);
      for (int64_t e = off[v]; e < off[v + 1]; e++) {
        const int32_t w = nbr[e];
        rn[w] += c;
        if (!mark[w]) { mark[w] = 1; G[ng++] = w; }
      }
    }
    /* drop level j, move level j + 1 into r, filter the next frontier */
    for (int64_t i = 0; i < nt; i++) r[T[i]] = 0.0;
    nf = 0;
    for (int64_t i = 0; i < ng; i++) {
      const int32_t w = G[i];
      mark[w] = 0;
      r[w] = rn[w];
      rn[w] = 0.0;
      const double thr = hk_thr(et_eps, deg_of(off, w), N, psi[j + 1]);
      hk_gap(st, r[w], thr);
      if (r[w] >= thr) F[nf++] = w;
    }
    qsort(F, (size_t)nf, sizeof(int32_t), cmp_i32);
    int32_t* tmp = T; T = G; G = tmp;
    nt = ng;
  }
  for (int64_t v = 0; v < n; v++) st->support += p[v] > 0.0;
  free(psi); free(r); free(rn); free(F); free(T); free(G); free(mark);
  return ORACLE_OK;
}

/*
 * The sequential procedure of Sec. 3.4 as printed there, for small graphs:
 * residuals keyed by (v, j) in a dense (N + 1) x n table, a FIFO queue of
 * entries; an entry is queued when an update makes its residual cross its
 * level's threshold (r < thr and r + M >= thr), and processing (v, j) adds
 * r[(v, j)] to p[v] and pushes to the neighbours.  An independent second
 * formulation to pin oracle_hkpr against.
 */
int oracle_hkpr_queue(int64_t n, const int64_t* off, const int32_t* nbr, int32_t x, int32_t N,
                      double eps, double t, double* p, oracle_hk_stats* st) {
  if (n <= 0 || !off || !nbr || !p || !st || N < 1) return ORACLE_E_INVALID;
  if (x < 0 || x >= n || deg_of(off, x) <= 0) return ORACLE_E_INVALID;
  if (!(eps > 0.0) || !isfinite(eps) || !(t > 0.0) || !isfinite(t)) return ORACLE_E_INVALID;
  const size_t cells = (size_t)(N + 1) * (size_t)n;
  double* psi = (double*)malloc(sizeof(double) * (size_t)(N + 1));
  double* r = (double*)calloc(cells, sizeof(double));
  int64_t* qv = (int64_t*)malloc(sizeof(int64_t) * (cells + 1));   /* queued cells */
  if (!psi || !r || !qv) { free(psi); free(r); free(qv); return ORACLE_E_NOMEM; }
  hk_psi(N, t, psi);
  const double et_eps = exp(-t) * eps;
  memset(st, 0, sizeof(*st));
  st->min_rel_gap = INFINITY;
  for (int64_t v = 0; v < n; v++) p[v] = 0.0;
  int64_t head = 0, tail = 0;
  r[x] = 1.0;               /* cell (x, 0) */
  qv[tail++] = x;
  int64_t last_level = -1;
  while (head < tail) {
    const int64_t cell = qv[head++];
    const int32_t j = (int32_t)(cell / n);
    const int32_t v = (int32_t)(cell % n);
    if (j != last_level) { st->levels++; last_level = j; }
    const double rv = r[cell];
    const int64_t d = deg_of(off, v);
    st->pushes++;
    st->edges += d;
    p[v] += rv;
    const double M = (t * rv) / ((double)(j + 1) * (double)d);
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      const int32_t w = nbr[e];
      if (j + 1 == N) {
        p[w] += rv / (double)d;
      } else {
        const int64_t cw = (int64_t)(j + 1) * n + w;
        const double thr = hk_thr(et_eps, deg_of(off, w), N, psi[j + 1]);
        if (r[cw] < thr && r[cw] + M >= thr) qv[tail++] = cw;
        r[cw] += M;
      }
    }
  }
  for (int64_t v = 0; v < n; v++) st->support += p[v] > 0.0;
  free(psi); free(r); free(qv);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Nibble (Sec. 3.2, Fig. alg:nibble): the truncated lazy random walk from
 * seed x for up to T iterations.  Iteration t builds p' from p: every
 * frontier vertex v keeps p[v]/2 and sends p[v]/(2 d(v)) to each neighbour
 * (fetch-and-add, here in edge order); the next frontier is every vertex
 * with p'[v] >= eps d(v).  If it is empty the loop stops and p (the previous
 * vector) is returned; otherwise p = p'.  After T iterations p_T is
 * returned.  Readings: the first frontier is {x} whatever its threshold;
 * the returned vector is returned whole (entries below eps d(v) are only
 * not propagated).  p dense, length n, overwritten.
 * ------------------------------------------------------------------------ */

typedef struct {
  int64_t iterations;  /* iterations whose p' was computed */
  int64_t pushes;      /* frontier entries processed */
  int64_t edges;       /* sum of d(v) over them */
  int64_t support;     /* vertices with p > 0 in the returned vector */
  double min_rel_gap;  /* closest approach of a threshold decision to its threshold */
} oracle_nb_stats;

int oracle_nibble(int64_t n, const int64_t* off, const int32_t* nbr, int32_t x, double eps,
                  int32_t T, double* p, oracle_nb_stats* st) {
  if (n <= 0 || !off || !nbr || !p || !st || T < 0) return ORACLE_E_INVALID;
  if (x < 0 || x >= n || deg_of(off, x) <= 0) return ORACLE_E_INVALID;
  if (!(eps > 0.0) || !isfinite(eps)) return ORACLE_E_INVALID;
  double* pn = (double*)calloc((size_t)n, sizeof(double));
  int32_t* F = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);  /* frontier of p */
  int32_t* S = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);  /* support of p */
  int32_t* G = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);  /* support of p' */
  uint8_t* mark = (uint8_t*)calloc((size_t)n, 1);
  if (!pn || !F || !S || !G || !mark) {
    free(pn); free(F); free(S); free(G); free(mark);
    return ORACLE_E_NOMEM;
  }
  memset(st, 0, sizeof(*st));
  st->min_rel_gap = INFINITY;
  for (int64_t v = 0; v < n; v++) p[v] = 0.0;
  p[x] = 1.0;
  int64_t nf = 1, ns = 1;
  F[0] = x;
  S[0] = x;
  for (int32_t t = 1; t <= T; t++) {
    st->iterations++;
    st->pushes += nf;
    /* p' = {}; vertexMap(Frontier, UpdateSelf); edgeMap(G, Frontier, UpdateNgh) */
    int64_t ng = 0;
    for (int64_t i = 0; i < nf; i++) {
      const int32_t v = F[i];
      pn[v] = p[v] / 2.0;
      if (!mark[v]) { mark[v] = 1; G[ng++] = v; }
    }
    for (int64_t i = 0; i < nf; i++) {
      const int32_t v = F[i];
      const int64_t d = deg_of(off, v);
      st->edges += d;
      const double c = p[v] / (2.0 * (double)d);
      for (int64_t e = off[v]; e < off[v + 1]; e++) {
        const int32_t w = nbr[e];
        pn[w] += c;
        if (!mark[w]) { mark[w] = 1; G[ng++] = w; }
      }
    }
    /* Frontier = {v | p'[v] >= d(v) eps} (filter) */
    int64_t k = 0;
    for (int64_t i = 0; i < ng; i++) {
      const int32_t w = G[i];
      mark[w] = 0;
      const double thr = eps * (double)deg_of(off, w);
      const double gap = fabs(pn[w] - thr) / thr;
      if (gap < st->min_rel_gap) st->min_rel_gap = gap;
      if (pn[w] >= thr) F[k++] = w;
    }
    if (k == 0) {  /* return the previous vector */
      for (int64_t i = 0; i < ng; i++) pn[G[i]] = 0.0;
      break;
    }
    /* p = p' */
    for (int64_t i = 0; i < ns; i++) p[S[i]] = 0.0;
    for (int64_t i = 0; i < ng; i++) { p[G[i]] = pn[G[i]]; pn[G[i]] = 0.0; }
    qsort(F, (size_t)k, sizeof(int32_t), cmp_i32);
    nf = k;
    int32_t* tmp = S; S = G; G = tmp;
    ns = ng;
  }
  for (int64_t v = 0; v < n; v++) st->support += p[v] > 0.0;
  free(pn); free(F); free(S); free(G); free(mark);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * PR-Nibble, beta variant (end of Sec. 3.3): each round pushes only the
 * ceil(beta |S|) vertices of the active set S = {v : r[v] >= eps d(v)} with
 * the largest r[v]/d(v) (ties by ascending id), with the round-synchronous
 * updates of Fig. alg:pr-nibble2 among them; every vertex still at or above
 * its threshold afterwards is active in the next round.  beta = 1 is
 * PR-Nibble itself.
 * ------------------------------------------------------------------------ */

typedef struct { double key; int32_t id; } beta_item;

static int cmp_beta(const void* a, const void* b) {
  const beta_item* x = (const beta_item*)a;
  const beta_item* y = (const beta_item*)b;
  if (x->key > y->key) return -1;
  if (x->key < y->key) return 1;
  return x->id < y->id ? -1 : (x->id > y->id);
}

int oracle_prnibble_beta(int64_t n, const int64_t* off, const int32_t* nbr, int32_t x,
                         double alpha, double eps, int32_t rule, double beta, int64_t max_rounds,
                         double* p, double* r, oracle_push_stats* st, double* min_sel_gap) {
  if (n <= 0 || !off || !nbr || !p || !r || !st || !min_sel_gap) return ORACLE_E_INVALID;
  if (x < 0 || x >= n || deg_of(off, x) <= 0) return ORACLE_E_INVALID;
  if (!(alpha > 0.0 && alpha < 1.0) || !(eps > 0.0) || !isfinite(eps)) return ORACLE_E_INVALID;
  if (!(beta > 0.0 && beta <= 1.0)) return ORACLE_E_INVALID;
  if (rule != ORACLE_RULE_OPT && rule != ORACLE_RULE_ORIG) return ORACLE_E_INVALID;
  double cs, cn, keep;
  rule_constants(rule, alpha, &cs, &cn, &keep);
  beta_item* S = (beta_item*)malloc(sizeof(beta_item) * (size_t)n);
  double* rho = (double*)malloc(sizeof(double) * (size_t)n);
  int32_t* act = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);   /* active set */
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t* mark = (uint8_t*)calloc((size_t)n, 1);
  if (!S || !rho || !act || !cand || !mark) {
    free(S); free(rho); free(act); free(cand); free(mark);
    return ORACLE_E_NOMEM;
  }
  memset(st, 0, sizeof(*st));
  st->min_rel_gap = INFINITY;
  *min_sel_gap = INFINITY;
  for (int64_t v = 0; v < n; v++) { p[v] = 0.0; r[v] = 0.0; }
  r[x] = 1.0;
  int64_t na = 1;
  act[0] = x;   /* the seed is active in the first round whatever its threshold */
  int status = ORACLE_OK;
  while (na > 0) {
    if (st->rounds >= max_rounds) { status = ORACLE_LIMIT; break; }
    /* rank the active set by r/d, take the top ceil(beta |S|) */
    for (int64_t i = 0; i < na; i++) {
      S[i].key = r[act[i]] / (double)deg_of(off, act[i]);
      S[i].id = act[i];
    }
    qsort(S, (size_t)na, sizeof(beta_item), cmp_beta);
    int64_t k = (int64_t)ceil(beta * (double)na);
    if (k < 1) k = 1;
    if (k > na) k = na;
    if (k < na && S[k - 1].key > 0.0) {
      const double g = (S[k - 1].key - S[k].key) / S[k - 1].key;
      if (g < *min_sel_gap) *min_sel_gap = g;
    }
    if (k > st->max_frontier) st->max_frontier = (int32_t)k;
    /* round-synchronous push of the chosen k */
    for (int64_t i = 0; i < k; i++) rho[i] = r[S[i].id];
    int64_t nc = 0;
    for (int64_t i = 0; i < k; i++) {
      const int32_t v = S[i].id;
      if (p[v] == 0.0) st->support++;
      p[v] = p[v] + cs * rho[i];
      r[v] = keep * rho[i];
      if (!mark[v]) { mark[v] = 1; cand[nc++] = v; }
    }
    for (int64_t i = 0; i < k; i++) {
      const int32_t v = S[i].id;
      const int64_t d = deg_of(off, v);
      st->edges += d;
      const double c = (cn * rho[i]) / (double)d;
      for (int64_t e = off[v]; e < off[v + 1]; e++) {
        const int32_t w = nbr[e];
        r[w] = r[w] + c;
        if (!mark[w]) { mark[w] = 1; cand[nc++] = w; }
      }
    }
    st->pushes += k;
    st->rounds++;
    /* next active set: the unchosen active vertices (still above threshold)
       and every touched vertex at or above its threshold */
    for (int64_t i = k; i < na; i++) {
      const int32_t v = S[i].id;
      if (!mark[v]) { mark[v] = 1; cand[nc++] = v; }
    }
    int64_t m = 0;
    for (int64_t i = 0; i < nc; i++) {
      const int32_t w = cand[i];
      mark[w] = 0;
      const double thr = eps * (double)deg_of(off, w);
      const double gap = fabs(r[w] - thr) / thr;
      if (gap < st->min_rel_gap) st->min_rel_gap = gap;
      if (r[w] >= thr) act[m++] = w;
    }
    na = m;
  }
  st->status = status;
  free(S); free(rho); free(act); free(cand); free(mark);
  return status;
}
