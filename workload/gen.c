/*
 * Seeded synthetic RDF workload generator: power-law triple sets and
 * random-walk basic graph patterns (BGPs).
 *
 * This module is shared input plumbing for both the CPU oracle and the GPU
 * library.  It only produces inputs (int32 triples and triple patterns) and
 * never evaluates a join: neither side imports anything from here except the
 * generated arrays.  The exact result-size counter below exists to accept or
 * reject candidate queries by size; it is a tree dynamic program (counting
 * homomorphisms of a tree-shaped pattern), not the sparse-matrix join.
 *
 * Randomness is counter based (SplitMix64 finaliser applied to a keyed
 * counter), so every array is a pure function of (parameters, seed) and does
 * not depend on the number of OpenMP threads.  Floating-point reductions are
 * done over fixed-size chunks in a fixed order for the same reason.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC gen.c -o libworkload.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>
#include <stdio.h>

static int wl_verbose(void) {
  const char* e = getenv("WL_VERBOSE");
  return e && e[0] == '1';
}
#define VLOG(...) do { if (wl_verbose()) { fprintf(stderr, __VA_ARGS__); fflush(stderr); } } while (0)

/* ------------------------------------------------------------------ */
/* counter-based random numbers                                        */
/* ------------------------------------------------------------------ */
static inline uint64_t mix64(uint64_t z) {
  z ^= z >> 30; z *= 0xbf58476d1ce4e5b9ULL;
  z ^= z >> 27; z *= 0x94d049bb133111ebULL;
  z ^= z >> 31;
  return z;
}
static inline uint64_t unxorshift(uint64_t y, int k) {
  uint64_t x = y;
  for (int i = 0; i < 64 / k + 1; ++i) x = y ^ (x >> k);
  return x;
}
static uint64_t inv_mul(uint64_t a) { /* inverse of odd a modulo 2^64 (Newton) */
  uint64_t x = a;
  for (int i = 0; i < 6; ++i) x *= 2 - a * x;
  return x;
}
static uint64_t unmix64(uint64_t z) {
  z = unxorshift(z, 31);
  z *= inv_mul(0x94d049bb133111ebULL);
  z = unxorshift(z, 27);
  z *= inv_mul(0xbf58476d1ce4e5b9ULL);
  z = unxorshift(z, 30);
  return z;
}
static inline uint64_t rng(uint64_t seed, uint64_t stream, uint64_t i) {
  return mix64(seed ^ mix64(stream * 0x9E3779B97F4A7C15ULL + i));
}
static inline double u01(uint64_t r) { /* strictly inside (0,1) */
  return ((double)(r >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

uint64_t wl_mix64(uint64_t z) { return mix64(z); }
uint64_t wl_unmix64(uint64_t z) { return unmix64(z); }

enum { S_OUT = 1, S_IN = 2, S_RHO = 3, S_PRED = 4, S_TGT = 5, S_HASH = 6, S_TOPUP = 7 };

/* ------------------------------------------------------------------ */
/* helpers                                                             */
/* ------------------------------------------------------------------ */
static int bits_for(int64_t maxval) { /* bits to hold values in [0, maxval] */
  int b = 1;
  while (b < 63 && ((int64_t)1 << b) <= maxval) ++b;
  return b;
}

/* Stable LSD radix sort of 64-bit keys on their low `nbits` bits. */
static void radix_sort_u64(uint64_t *a, uint64_t *tmp, int64_t n, int nbits) {
  int passes = (nbits + 7) / 8;
  int nt = omp_get_max_threads();
  int64_t *hist = (int64_t *)malloc(sizeof(int64_t) * 256 * nt);
  uint64_t *src = a, *dst = tmp;
  for (int pass = 0; pass < passes; ++pass) {
    int sh = 8 * pass;
    memset(hist, 0, sizeof(int64_t) * 256 * nt);
#pragma omp parallel num_threads(nt)
    {
      int t = omp_get_thread_num();
      int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
      int64_t *h = hist + 256 * t;
      for (int64_t i = lo; i < hi; ++i) h[(src[i] >> sh) & 255]++;
#pragma omp barrier
#pragma omp single
      {
        int64_t run = 0;
        for (int d = 0; d < 256; ++d)
          for (int tt = 0; tt < nt; ++tt) {
            int64_t c = hist[256 * tt + d];
            hist[256 * tt + d] = run;
            run += c;
          }
      }
      for (int64_t i = lo; i < hi; ++i) dst[h[(src[i] >> sh) & 255]++] = src[i];
    }
    uint64_t *sw = src; src = dst; dst = sw;
  }
  if (src != a) memcpy(a, src, sizeof(uint64_t) * n);
  free(hist);
}

/* Stable counting sort of (a, p, b)-packed keys (a<<(pb+vb) | p<<vb | b) by p,
 * writing them repacked as (p, a, b) = p<<2vb | a<<vb | b.  Input sorted by
 * (a, p, b) therefore comes out sorted by (p, a, b). */
static void regroup_by_pred(const uint64_t *in, uint64_t *out, int64_t n, int32_t P, int pb, int vb) {
  int nt = omp_get_max_threads();
  int64_t *hist = (int64_t *)calloc((size_t)P * nt, sizeof(int64_t));
  uint64_t vmask = ((uint64_t)1 << vb) - 1, pmask = ((uint64_t)1 << pb) - 1;
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
    int64_t *h = hist + (size_t)P * t;
    for (int64_t i = lo; i < hi; ++i) h[(in[i] >> vb) & pmask]++;
#pragma omp barrier
#pragma omp single
    {
      int64_t run = 0;
      for (int32_t p = 0; p < P; ++p)
        for (int tt = 0; tt < nt; ++tt) {
          int64_t c = hist[(size_t)P * tt + p];
          hist[(size_t)P * tt + p] = run;
          run += c;
        }
    }
    for (int64_t i = lo; i < hi; ++i) {
      uint64_t x = in[i];
      uint64_t p = (x >> vb) & pmask, a = x >> (pb + vb), b = x & vmask;
      out[h[p]++] = (p << (2 * vb)) | (a << vb) | b;
    }
  }
  free(hist);
}

/* Deterministic sum of doubles: fixed chunks, fixed order. */
#define DCHUNK 65536
static double det_sum(const double *x, int64_t n) {
  int64_t nc = (n + DCHUNK - 1) / DCHUNK;
  double *part = (double *)calloc(nc > 0 ? nc : 1, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; ++c) {
    double s = 0;
    int64_t hi = (c + 1) * DCHUNK < n ? (c + 1) * DCHUNK : n;
    for (int64_t i = c * DCHUNK; i < hi; ++i) s += x[i];
    part[c] = s;
  }
  double s = 0;
  for (int64_t c = 0; c < nc; ++c) s += part[c];
  free(part);
  return s;
}

/* ------------------------------------------------------------------ */
/* graph generator                                                     */
/* ------------------------------------------------------------------ */
/*
 * Out-degree of vertex v: min(floor(xm * q_v), out_cap), q_v = u_v^(-1/(gamma-1))
 * (a discrete power law with exponent gamma); xm solved by bisection so that
 * the total is the wanted number of candidate edges.
 * In-weight of v: min(ym * r_v, in_cap) with r_v = u'_v^(-1/in_alpha), where
 * u'_v = u_v with probability rho (rank-correlated hubs) and fresh otherwise;
 * ym solved so the weights sum to the candidate edge count, so a weight is
 * the vertex's expected in-degree.  Each edge's object is drawn in proportion
 * to in-weight (preferential by expected in-degree, by inverse CDF); its
 * predicate from Zipf(zipf_s) over 0..P-1.
 * Candidates are deduplicated as a set; a keyed bijective hash orders them, and
 * the first T distinct triples in hash order are kept (a uniform subset, in
 * random order).  If fewer than T are distinct, more candidates are drawn.
 */
typedef struct {
  int64_t V; int32_t P; int64_t T;
  double zipf_s, out_exp; int64_t out_cap;
  double in_alpha; int64_t in_cap; double rho;
  uint64_t seed;
} wl_graph_params;

/* Inverse-CDF sampling with a guide table (Chen and Asau's method): C is the
 * inclusive prefix sum of the weights (computed over fixed chunks in a fixed
 * order, so it does not depend on the thread count); guide[k] is the first
 * index whose prefix exceeds k/G of the total.  A draw x in [0, total) then
 * needs a binary search only inside one guide bucket. */
#define GUIDE_BITS 22
static void prefix_sum_det(const double *w, int64_t n, double *C) {
  int64_t nc = (n + DCHUNK - 1) / DCHUNK;
  double *part = (double *)calloc(nc > 0 ? nc : 1, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; ++c) {
    double s = 0;
    int64_t hi = (c + 1) * DCHUNK < n ? (c + 1) * DCHUNK : n;
    for (int64_t i = c * DCHUNK; i < hi; ++i) s += w[i];
    part[c] = s;
  }
  double run = 0;
  for (int64_t c = 0; c < nc; ++c) { double t = part[c]; part[c] = run; run += t; }
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; ++c) {
    double s = part[c];
    int64_t hi = (c + 1) * DCHUNK < n ? (c + 1) * DCHUNK : n;
    for (int64_t i = c * DCHUNK; i < hi; ++i) { s += w[i]; C[i] = s; }
  }
  free(part);
}
static void build_guide(const double *C, int64_t n, int64_t *guide) {
  const int64_t G = (int64_t)1 << GUIDE_BITS;
  const double total = C[n - 1];
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k <= G; ++k) {
    double x = total * (double)k / (double)G;
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) { int64_t m = (lo + hi) / 2; if (C[m] > x) hi = m; else lo = m + 1; }
    guide[k] = lo;
  }
}
static inline int64_t sample_cdf(const double *C, int64_t n, const int64_t *guide, double u) {
  const int64_t G = (int64_t)1 << GUIDE_BITS;
  const double total = C[n - 1];
  double x = u * total;
  int64_t k = (int64_t)(u * (double)G);
  if (k >= G) k = G - 1;
  int64_t lo = guide[k], hi = guide[k + 1];
  if (hi > n - 1) hi = n - 1;
  while (lo < hi) { int64_t m = (lo + hi) / 2; if (C[m] > x) hi = m; else lo = m + 1; }
  /* skip zero-weight entries that share the prefix value */
  while (lo < n - 1 && C[lo] <= x) ++lo;
  return lo;
}

/* Returns number of triples written (== T) or a negative error code. */
int64_t wl_gen_graph(int64_t V, int32_t P, int64_t T, double zipf_s, double out_exp,
                     int64_t out_cap, double in_alpha, int64_t in_cap, double rho,
                     uint64_t seed, int32_t *s_out, int32_t *p_out, int32_t *o_out) {
  if (V < 1 || V > 2147483647LL || P < 1 || T < 0) return -1;
  int vb = bits_for(V - 1), pb = bits_for(P - 1);
  if (2 * vb + pb > 64) return -2;
  if (T == 0) return 0;
  /* a simple upper bound on distinct triples */
  double maxpairs = (double)V * (double)V * (double)P;
  if ((double)T > 0.5 * maxpairs) return -3;

  double *q = (double *)malloc(sizeof(double) * V);
  double *r = (double *)malloc(sizeof(double) * V);
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < V; ++v) {
    double u = u01(rng(seed, S_OUT, v));
    q[v] = pow(u, -1.0 / (out_exp - 1.0));
    /* rho > 0: in-weight rank follows the out-degree draw with probability rho;
     * rho < 0: it follows the reversed rank (anti-correlated) with probability -rho. */
    double coin = u01(rng(seed, S_RHO, v));
    double u2 = coin < fabs(rho) ? (rho > 0 ? u : 1.0 - u) : u01(rng(seed, S_IN, v));
    r[v] = pow(u2, -1.0 / in_alpha);
  }
  /* predicate CDF thresholds */
  uint64_t *thr = (uint64_t *)malloc(sizeof(uint64_t) * P);
  {
    double H = 0;
    for (int32_t k = 0; k < P; ++k) H += pow((double)(k + 1), -zipf_s);
    double c = 0;
    for (int32_t k = 0; k < P; ++k) {
      c += pow((double)(k + 1), -zipf_s) / H;
      double t = c * 18446744073709551616.0;
      thr[k] = (k == P - 1 || t >= 18446744073709551615.0) ? UINT64_MAX : (uint64_t)t;
    }
  }
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * V);
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (V + 1));
  double *w = (double *)malloc(sizeof(double) * V);
  double *C = (double *)malloc(sizeof(double) * V);
  int64_t *guide = (int64_t *)malloc(sizeof(int64_t) * (((int64_t)1 << GUIDE_BITS) + 1));
  uint64_t hseed = mix64(seed ^ 0x5eed5eed5eedULL);
  double over = 1.10;
  int64_t result = -4;
  uint64_t *h = NULL, *tmp = NULL;
  for (int attempt = 0; attempt < 12; ++attempt) {
    double t0 = omp_get_wtime();
    double want = over * (double)T;
    /* solve xm: total out-degree ~= want */
    double lo = 1e-9, hi = 1e9;
    for (int it = 0; it < 64; ++it) {
      double xm = sqrt(lo * hi);
      int64_t tot = 0;
#pragma omp parallel for reduction(+ : tot) schedule(static)
      for (int64_t v = 0; v < V; ++v) {
        double d = floor(xm * q[v]);
        tot += d >= (double)out_cap ? out_cap : (int64_t)d;
      }
      if ((double)tot > want) hi = xm; else lo = xm;
    }
    double xm = hi;
    VLOG("[wl] attempt %d over=%.4f xm solve %.2fs\n", attempt, over, omp_get_wtime() - t0);
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < V; ++v) {
      double d = floor(xm * q[v]);
      deg[v] = d >= (double)out_cap ? out_cap : (int64_t)d;
    }
    off[0] = 0;
    for (int64_t v = 0; v < V; ++v) off[v + 1] = off[v] + deg[v];
    int64_t E = off[V];
    /* solve ym: in-weights sum to E */
    double ylo = 1e-12, yhi = 1e12;
    for (int it = 0; it < 64; ++it) {
      double ym = sqrt(ylo * yhi);
#pragma omp parallel for schedule(static)
      for (int64_t v = 0; v < V; ++v) {
        double x = ym * r[v];
        w[v] = x > (double)in_cap ? (double)in_cap : x;
      }
      if (det_sum(w, V) > (double)E) yhi = ym; else ylo = ym;
    }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < V; ++v) {
      double x = yhi * r[v];
      w[v] = x > (double)in_cap ? (double)in_cap : x;
    }
    VLOG("[wl] ym solve done %.2fs\n", omp_get_wtime() - t0);
    prefix_sum_det(w, V, C);
    build_guide(C, V, guide);
    VLOG("[wl] cdf done %.2fs E=%lld\n", omp_get_wtime() - t0, (long long)E);

    free(h); free(tmp);
    h = (uint64_t *)malloc(sizeof(uint64_t) * (E > 0 ? E : 1));
    tmp = (uint64_t *)malloc(sizeof(uint64_t) * (E > 0 ? E : 1));
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < V; ++v) {
      for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        uint64_t rp = rng(seed, S_PRED, (uint64_t)e + (uint64_t)attempt * 0x100000000000ULL);
        int32_t lo2 = 0, hi2 = P - 1;
        while (lo2 < hi2) { int32_t m = (lo2 + hi2) / 2; if (rp < thr[m]) hi2 = m; else lo2 = m + 1; }
        uint64_t rt = rng(seed, S_TGT, (uint64_t)e + (uint64_t)attempt * 0x100000000000ULL);
        int64_t tgt = sample_cdf(C, V, guide, u01(rt));
        uint64_t key = ((uint64_t)v << (pb + vb)) | ((uint64_t)lo2 << vb) | (uint64_t)tgt;
        h[e] = mix64(key ^ hseed);
      }
    }
    VLOG("[wl] edges done %.2fs\n", omp_get_wtime() - t0);
    radix_sort_u64(h, tmp, E, 64);
    VLOG("[wl] sort done %.2fs\n", omp_get_wtime() - t0);
    /* unique */
    int64_t u = 0;
    for (int64_t i = 0; i < E; ++i)
      if (i == 0 || h[i] != h[i - 1]) h[u++] = h[i];
    VLOG("[wl] unique %lld of %lld (T=%lld) %.2fs\n", (long long)u, (long long)E, (long long)T,
         omp_get_wtime() - t0);
    if (u >= T) {
      uint64_t vmask = ((uint64_t)1 << vb) - 1, pmask = ((uint64_t)1 << pb) - 1;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < T; ++i) {
        uint64_t key = unmix64(h[i]) ^ hseed;
        s_out[i] = (int32_t)(key >> (pb + vb));
        p_out[i] = (int32_t)((key >> vb) & pmask);
        o_out[i] = (int32_t)(key & vmask);
      }
      result = T;
      break;
    }
    over *= 1.02 * (double)T / (double)(u > 0 ? u : 1);
  }
  free(h); free(tmp); free(q); free(r); free(thr); free(deg); free(off); free(w);
  free(C); free(guide);
  return result;
}

/* ------------------------------------------------------------------ */
/* query-side adjacency (generator-private)                            */
/* ------------------------------------------------------------------ */
/*
 * Four sorted views of the triple set, each as (group key, offsets, members):
 *   by subject over all predicates: members (p, o) sorted
 *   by object  over all predicates: members (p, s) sorted
 *   per predicate by subject:       rows s, members o
 *   per predicate by object:        rows o, members s
 */
typedef struct {
  int64_t V; int32_t P; int64_t n;
  int vb, pb;
  /* all-predicate adjacency */
  int64_t *out_off; int32_t *out_p; int32_t *out_o;   /* by subject */
  int64_t *in_off;  int32_t *in_p;  int32_t *in_s;    /* by object  */
  /* per-predicate adjacency: rows, row offsets (global), members */
  int64_t *ps_pred_row; /* [P+1] row range per predicate */
  int32_t *ps_row; int64_t *ps_off; int32_t *ps_nbr;    /* by subject */
  int64_t *po_pred_row;
  int32_t *po_row; int64_t *po_off; int32_t *po_nbr;    /* by object */
  int64_t *deg_total; /* out+in degree per vertex */
  uint64_t *scratch;  /* V zeros between uses (counting program) */
} wl_index;

static void build_grouped(const uint64_t *keys, int64_t n, int64_t ngroups, int sh_group,
                          uint64_t gmask, int64_t *goff) {
  /* keys sorted; group id = (key >> sh_group) & gmask; goff[g] = first index */
  memset(goff, 0, sizeof(int64_t) * (ngroups + 1));
  for (int64_t i = 0; i < n; ++i) goff[((keys[i] >> sh_group) & gmask) + 1]++;
  for (int64_t g = 0; g < ngroups; ++g) goff[g + 1] += goff[g];
}

static void build_pred_view(const uint64_t *keys, int64_t n, int32_t P, int vb,
                            int64_t **pred_row, int32_t **row, int64_t **off, int32_t **nbr) {
  /* keys sorted by (p, a, b) packed as p<<2vb | a<<vb | b */
  uint64_t vmask = ((uint64_t)1 << vb) - 1;
  int64_t nrows = 0;
  for (int64_t i = 0; i < n; ++i)
    if (i == 0 || (keys[i] >> vb) != (keys[i - 1] >> vb)) ++nrows;
  int64_t *pr = (int64_t *)calloc(P + 1, sizeof(int64_t));
  int32_t *rw = (int32_t *)malloc(sizeof(int32_t) * (nrows > 0 ? nrows : 1));
  int64_t *of = (int64_t *)malloc(sizeof(int64_t) * (nrows + 1));
  int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  int64_t r = 0;
  for (int64_t i = 0; i < n; ++i) {
    nb[i] = (int32_t)(keys[i] & vmask);
    if (i == 0 || (keys[i] >> vb) != (keys[i - 1] >> vb)) {
      rw[r] = (int32_t)((keys[i] >> vb) & vmask);
      of[r] = i;
      pr[(keys[i] >> (2 * vb)) + 1]++;
      ++r;
    }
  }
  of[nrows] = n;
  for (int32_t p = 0; p < P; ++p) pr[p + 1] += pr[p];
  *pred_row = pr; *row = rw; *off = of; *nbr = nb;
}

void *wl_index_new(const int32_t *s, const int32_t *p, const int32_t *o, int64_t n, int64_t V,
                   int32_t P) {
  wl_index *ix = (wl_index *)calloc(1, sizeof(wl_index));
  ix->V = V; ix->P = P; ix->n = n;
  ix->vb = bits_for(V - 1); ix->pb = bits_for(P - 1);
  int vb = ix->vb, pb = ix->pb, nb = 2 * vb + pb;
  uint64_t vmask = ((uint64_t)1 << vb) - 1, pmask = ((uint64_t)1 << pb) - 1;
  uint64_t *k = (uint64_t *)malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
  uint64_t *t = (uint64_t *)malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
  for (int side = 0; side < 2; ++side) {
    /* side 0: (s, p, o) -> out adjacency and per-predicate by-subject view;
     * side 1: (o, p, s) -> in adjacency and per-predicate by-object view */
    const int32_t *a1 = side == 0 ? s : o, *a2 = side == 0 ? o : s;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      k[i] = ((uint64_t)a1[i] << (pb + vb)) | ((uint64_t)p[i] << vb) | (uint64_t)a2[i];
    radix_sort_u64(k, t, n, nb);
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (V + 1));
    build_grouped(k, n, V, pb + vb, vmask, off);
    int32_t *pp = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t *mm = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      pp[i] = (int32_t)((k[i] >> vb) & pmask);
      mm[i] = (int32_t)(k[i] & vmask);
    }
    regroup_by_pred(k, t, n, P, pb, vb);
    if (side == 0) {
      ix->out_off = off; ix->out_p = pp; ix->out_o = mm;
      build_pred_view(t, n, P, vb, &ix->ps_pred_row, &ix->ps_row, &ix->ps_off, &ix->ps_nbr);
    } else {
      ix->in_off = off; ix->in_p = pp; ix->in_s = mm;
      build_pred_view(t, n, P, vb, &ix->po_pred_row, &ix->po_row, &ix->po_off, &ix->po_nbr);
    }
  }
  free(k); free(t);
  ix->deg_total = (int64_t *)malloc(sizeof(int64_t) * V);
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < V; ++v)
    ix->deg_total[v] = (ix->out_off[v + 1] - ix->out_off[v]) + (ix->in_off[v + 1] - ix->in_off[v]);
  ix->scratch = (uint64_t *)calloc(V, sizeof(uint64_t));
  return ix;
}

void wl_index_free(void *h) {
  wl_index *ix = (wl_index *)h;
  if (!ix) return;
  free(ix->out_off); free(ix->out_p); free(ix->out_o);
  free(ix->in_off); free(ix->in_p); free(ix->in_s);
  free(ix->ps_pred_row); free(ix->ps_row); free(ix->ps_off); free(ix->ps_nbr);
  free(ix->po_pred_row); free(ix->po_row); free(ix->po_off); free(ix->po_nbr);
  free(ix->deg_total);
  free(ix->scratch);
  free(ix);
}

/* out-degree and in-degree (all predicates) of vertex v */
int64_t wl_out_degree(void *h, int32_t v) { wl_index *ix = h; return ix->out_off[v + 1] - ix->out_off[v]; }
int64_t wl_in_degree(void *h, int32_t v) { wl_index *ix = h; return ix->in_off[v + 1] - ix->in_off[v]; }

/* Vertices whose total degree is at least `min_deg`, into out (cap); returns count. */
int64_t wl_vertices_with_degree(void *h, int64_t min_deg, int32_t *out, int64_t cap) {
  wl_index *ix = h;
  int64_t c = 0;
  for (int64_t v = 0; v < ix->V; ++v)
    if (ix->deg_total[v] >= min_deg) { if (c < cap) out[c] = (int32_t)v; ++c; }
  return c;
}

/* Total-degree histogram helper: number of vertices with total degree <= d. */
int64_t wl_count_degree_le(void *h, int64_t d) {
  wl_index *ix = h;
  int64_t c = 0;
#pragma omp parallel for reduction(+ : c)
  for (int64_t v = 0; v < ix->V; ++v) c += ix->deg_total[v] <= d;
  return c;
}
int64_t wl_max_degree(void *h, int32_t which /*0 total,1 out,2 in*/) {
  wl_index *ix = h;
  int64_t m = 0;
  for (int64_t v = 0; v < ix->V; ++v) {
    int64_t d = which == 0 ? ix->deg_total[v]
              : which == 1 ? ix->out_off[v + 1] - ix->out_off[v]
                           : ix->in_off[v + 1] - ix->in_off[v];
    if (d > m) m = d;
  }
  return m;
}

/* ------------------------------------------------------------------ */
/* exact result size of a tree-shaped BGP (generator-side selection)   */
/* ------------------------------------------------------------------ */
/*
 * Patterns are (s, p, o) int32; an endpoint < 0 is variable -(x+1).
 * The variable graph must be a forest without self loops or repeated
 * variable pairs; otherwise -1 is returned.  The count is saturated at
 * UINT64_MAX/2 (returned as INT64_MAX).
 *
 * For a variable x rooted at r, f_x(v) is the number of assignments of x's
 * subtree with x = v; a child y through pattern (x p y) contributes
 * sum over out-neighbours u of v of f_y(u); through (y p x) the sum runs over
 * in-neighbours.  A constant endpoint contributes a membership indicator.
 */
typedef struct { int64_t n; int32_t *id; uint64_t *val; int one; } sparsef; /* one: f == 1 everywhere */

static const uint64_t SAT = (uint64_t)INT64_MAX;
static inline uint64_t sadd(uint64_t a, uint64_t b) { uint64_t c = a + b; return (c < a || c > SAT) ? SAT : c; }
static inline uint64_t smul(uint64_t a, uint64_t b) {
  if (a == 0 || b == 0) return 0;
  unsigned __int128 c = (unsigned __int128)a * b;
  return c > SAT ? SAT : (uint64_t)c;
}

int cmp32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static int64_t find_row(const int32_t *rows, int64_t lo, int64_t hi, int32_t v) {
  while (lo < hi) { int64_t m = (lo + hi) / 2; if (rows[m] < v) lo = m + 1; else hi = m; }
  return lo;
}

/* message of pattern t (at variable x, `x_is_subject`) as a sparse vector over x */
static sparsef msg_of(wl_index *ix, int32_t p, int x_is_subject, int other_is_const, int32_t cval,
                      const sparsef *child, uint64_t *scratch) {
  sparsef m = {0, NULL, NULL, 0};
  /* view keyed by x's side */
  int64_t *pred_row = x_is_subject ? ix->ps_pred_row : ix->po_pred_row;
  int32_t *row = x_is_subject ? ix->ps_row : ix->po_row;
  int64_t *off = x_is_subject ? ix->ps_off : ix->po_off;
  int32_t *nbr = x_is_subject ? ix->ps_nbr : ix->po_nbr;
  if (p < 0 || p >= ix->P) return m;
  if (other_is_const) {
    /* x ranges over neighbours of the constant in the other view */
    int64_t *pr2 = x_is_subject ? ix->po_pred_row : ix->ps_pred_row;
    int32_t *rw2 = x_is_subject ? ix->po_row : ix->ps_row;
    int64_t *of2 = x_is_subject ? ix->po_off : ix->ps_off;
    int32_t *nb2 = x_is_subject ? ix->po_nbr : ix->ps_nbr;
    if (cval < 0 || cval >= ix->V) return m;
    int64_t r = find_row(rw2, pr2[p], pr2[p + 1], cval);
    if (r >= pr2[p + 1] || rw2[r] != cval) return m;
    int64_t a = of2[r], b = of2[r + 1];
    m.n = b - a;
    m.id = (int32_t *)malloc(sizeof(int32_t) * (m.n > 0 ? m.n : 1));
    m.val = (uint64_t *)malloc(sizeof(uint64_t) * (m.n > 0 ? m.n : 1));
    for (int64_t i = 0; i < m.n; ++i) { m.id[i] = nb2[a + i]; m.val[i] = 1; }
    return m;
  }
  int64_t r0 = pred_row[p], r1 = pred_row[p + 1];
  if (!child->one && child->n * 8 < r1 - r0) {
    /* push: the child's support is small, so sum its values into the
     * neighbours on x's side through the other view (sparse accumulation) */
    int64_t *pr2 = x_is_subject ? ix->po_pred_row : ix->ps_pred_row;
    int32_t *rw2 = x_is_subject ? ix->po_row : ix->ps_row;
    int64_t *of2 = x_is_subject ? ix->po_off : ix->ps_off;
    int32_t *nb2 = x_is_subject ? ix->po_nbr : ix->ps_nbr;
    int64_t cap = 1024, cnt = 0;
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * cap);
    for (int64_t i = 0; i < child->n; ++i) {
      int32_t u = child->id[i];
      int64_t r = find_row(rw2, pr2[p], pr2[p + 1], u);
      if (r >= pr2[p + 1] || rw2[r] != u) continue;
      for (int64_t e = of2[r]; e < of2[r + 1]; ++e) {
        int32_t v = nb2[e];
        if (scratch[v] == 0) {
          if (cnt == cap) { cap *= 2; touched = (int32_t *)realloc(touched, sizeof(int32_t) * cap); }
          touched[cnt++] = v;
        }
        scratch[v] = sadd(scratch[v], child->val[i]);
      }
    }
    /* sort touched ids (radix over 32 bits would do; small lists: insertion via qsort) */
    qsort(touched, (size_t)cnt, sizeof(int32_t), cmp32);
    m.n = cnt;
    m.id = (int32_t *)malloc(sizeof(int32_t) * (cnt > 0 ? cnt : 1));
    m.val = (uint64_t *)malloc(sizeof(uint64_t) * (cnt > 0 ? cnt : 1));
    for (int64_t i = 0; i < cnt; ++i) { m.id[i] = touched[i]; m.val[i] = scratch[touched[i]]; scratch[touched[i]] = 0; }
    free(touched);
    return m;
  }
  m.n = r1 - r0;
  m.id = (int32_t *)malloc(sizeof(int32_t) * (m.n > 0 ? m.n : 1));
  m.val = (uint64_t *)malloc(sizeof(uint64_t) * (m.n > 0 ? m.n : 1));
  if (child->one) {
#pragma omp parallel for schedule(static)
    for (int64_t r = r0; r < r1; ++r) { m.id[r - r0] = row[r]; m.val[r - r0] = (uint64_t)(off[r + 1] - off[r]); }
  } else {
    for (int64_t i = 0; i < child->n; ++i) scratch[child->id[i]] = child->val[i];
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = r0; r < r1; ++r) {
      uint64_t acc = 0;
      for (int64_t e = off[r]; e < off[r + 1]; ++e) acc = sadd(acc, scratch[nbr[e]]);
      m.id[r - r0] = row[r];
      m.val[r - r0] = acc;
    }
    for (int64_t i = 0; i < child->n; ++i) scratch[child->id[i]] = 0;
    /* drop zeros */
    int64_t k = 0;
    for (int64_t i = 0; i < m.n; ++i) if (m.val[i]) { m.id[k] = m.id[i]; m.val[k] = m.val[i]; ++k; }
    m.n = k;
  }
  return m;
}

static void mul_into(sparsef *f, const sparsef *g) {
  /* f *= g (pointwise, both sorted by id); f.one means f == 1 */
  if (f->one) {
    f->one = 0;
    f->n = g->n;
    f->id = (int32_t *)malloc(sizeof(int32_t) * (g->n > 0 ? g->n : 1));
    f->val = (uint64_t *)malloc(sizeof(uint64_t) * (g->n > 0 ? g->n : 1));
    memcpy(f->id, g->id, sizeof(int32_t) * g->n);
    memcpy(f->val, g->val, sizeof(uint64_t) * g->n);
    return;
  }
  int64_t i = 0, j = 0, k = 0;
  while (i < f->n && j < g->n) {
    if (f->id[i] < g->id[j]) ++i;
    else if (f->id[i] > g->id[j]) ++j;
    else { f->id[k] = f->id[i]; f->val[k] = smul(f->val[i], g->val[j]); if (f->val[k]) ++k; ++i; ++j; }
  }
  f->n = k;
}

typedef struct { int32_t s, p, o; } wl_tp;

static sparsef eval_var(wl_index *ix, const wl_tp *tps, int ntp, int32_t x, int parent_tp,
                        uint64_t *scratch) {
  sparsef f = {0, NULL, NULL, 1};
  for (int t = 0; t < ntp; ++t) {
    if (t == parent_tp) continue;
    int32_t s = tps[t].s, o = tps[t].o;
    int xs = (s == -(x + 1)), xo = (o == -(x + 1));
    if (!xs && !xo) continue;
    int32_t other = xs ? o : s;
    sparsef g;
    if (other >= 0) {
      g = msg_of(ix, tps[t].p, xs, 1, other, NULL, scratch);
    } else {
      int32_t y = -other - 1;
      sparsef fy = eval_var(ix, tps, ntp, y, t, scratch);
      g = msg_of(ix, tps[t].p, xs, 0, 0, &fy, scratch);
      free(fy.id); free(fy.val);
    }
    mul_into(&f, &g);
    free(g.id); free(g.val);
  }
  return f;
}

static int64_t count_tree_impl(wl_index *ix, const int32_t *tp3, int32_t ntp, int32_t nvars,
                               uint64_t *scratch);

int64_t wl_count_tree(void *h, const int32_t *tp3, int32_t ntp, int32_t nvars) {
  wl_index *ix = (wl_index *)h;
  return count_tree_impl(ix, tp3, ntp, nvars, ix->scratch);
}

/* Counts nq queries concurrently (one thread per query, private scratch;
 * the per-query loops then run single-threaded).  Query q has ntp[q]
 * patterns starting at tp3 + 3 * off[q]. */
void wl_count_many(void *h, const int32_t *tp3, const int32_t *ntp, const int32_t *nvars,
                   const int64_t *off, int32_t nq, int64_t *out) {
  wl_index *ix = (wl_index *)h;
  int nt = omp_get_max_threads();
  uint64_t **scr = (uint64_t **)calloc(nt, sizeof(uint64_t *));
  /* longest first (cost ~ the predicates' sizes), so no long count is left
   * for the end of the loop */
  int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (nq > 0 ? nq : 1));
  int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (nq > 0 ? nq : 1));
  for (int32_t q = 0; q < nq; ++q) {
    int64_t c = 0;
    for (int32_t t = 0; t < ntp[q]; ++t) {
      int32_t p = tp3[3 * (off[q] + t) + 1];
      if (p >= 0 && p < ix->P) c += ix->ps_off[ix->ps_pred_row[p + 1]] - ix->ps_off[ix->ps_pred_row[p]];
    }
    key[q] = c;
    ord[q] = q;
  }
  for (int32_t i = 1; i < nq; ++i) {  /* insertion sort by descending cost */
    int32_t v = ord[i]; int32_t k = i;
    while (k > 0 && key[ord[k - 1]] < key[v]) { ord[k] = ord[k - 1]; --k; }
    ord[k] = v;
  }
  int lev = omp_get_max_active_levels();
  omp_set_max_active_levels(1);
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
#pragma omp for schedule(dynamic, 1)
    for (int32_t i = 0; i < nq; ++i) {
      int32_t q = ord[i];
      if (!scr[t]) scr[t] = (uint64_t *)calloc(ix->V, sizeof(uint64_t));
      out[q] = count_tree_impl(ix, tp3 + 3 * off[q], ntp[q], nvars[q], scr[t]);
    }
  }
  omp_set_max_active_levels(lev);
  for (int t = 0; t < nt; ++t) free(scr[t]);
  free(scr); free(key); free(ord);
}

static int64_t count_tree_impl(wl_index *ix, const int32_t *tp3, int32_t ntp, int32_t nvars,
                               uint64_t *scratch) {
  const wl_tp *tps = (const wl_tp *)tp3;
  /* validate forest: union-find over variables */
  int32_t *par = (int32_t *)malloc(sizeof(int32_t) * (nvars > 0 ? nvars : 1));
  for (int i = 0; i < nvars; ++i) par[i] = i;
  int ok = 1;
  uint64_t result = 1;
  for (int t = 0; t < ntp && ok; ++t) {
    int32_t s = tps[t].s, o = tps[t].o;
    if (s < 0 && o < 0) {
      int32_t a = -s - 1, b = -o - 1;
      if (a == b) { ok = 0; break; }
      while (par[a] != a) a = par[a];
      while (par[b] != b) b = par[b];
      if (a == b) { ok = 0; break; }
      par[a] = b;
    }
  }
  if (!ok) { free(par); return -1; }
  /* all-constant patterns: membership */
  for (int t = 0; t < ntp; ++t) {
    if (tps[t].s >= 0 && tps[t].o >= 0) {
      sparsef g = msg_of(ix, tps[t].p, 1, 1, tps[t].o, NULL, scratch);
      int found = 0;
      for (int64_t i = 0; i < g.n; ++i) if (g.id[i] == tps[t].s) found = 1;
      free(g.id); free(g.val);
      if (!found) result = 0;
    }
  }
  /* each component rooted at its first variable */
  int32_t *done = (int32_t *)calloc(nvars > 0 ? nvars : 1, sizeof(int32_t));
  for (int32_t x = 0; x < nvars && result; ++x) {
    int32_t rx = x;
    while (par[rx] != rx) rx = par[rx];
    if (done[rx]) continue;
    done[rx] = 1;
    sparsef f = eval_var(ix, tps, ntp, x, -1, scratch);
    uint64_t c;
    if (f.one) c = (uint64_t)ix->V;
    else { c = 0; for (int64_t i = 0; i < f.n; ++i) c = sadd(c, f.val[i]); }
    free(f.id); free(f.val);
    result = smul(result, c);
  }
  free(done); free(par);
  return (int64_t)result;
}

/* ------------------------------------------------------------------ */
/* random-walk query shapes                                            */
/* ------------------------------------------------------------------ */
/*
 * kind 0: chain of n patterns (?x0 p ?x1 . ?x1 p ?x2 ...), following out-edges
 * kind 1: subject star of n patterns around ?x0
 * kind 2: object star of n patterns around ?x0
 * kind 3: snowflake: centre with 2 out-edges, the n-2 remaining patterns are
 *         out-edges of the two branch vertices (at least one each)
 * const_mode k: the k highest-numbered leaf variables are replaced by their
 * witness values (k = 1 on a chain gives a constant object).
 * start >= 0 forces the walk's first vertex (hub-touching queries).
 * bias weights the predicate choice of stars and snowflakes (see below).
 * Returns the number of variables (>0) on success, 0 when this attempt failed.
 * Writes n patterns into tp3 and the witness assignment into witness.
 */
/* Number of distinct predicates in a segment sorted by predicate. */
static int64_t n_pred_runs(const int32_t *pp, int64_t a, int64_t b) {
  int64_t k = 0;
  for (int64_t e = a; e < b; ++e) k += (e == a || pp[e] != pp[e - 1]);
  return k;
}
/* First edge index of the r-th predicate run and its length. */
static int64_t pred_run(const int32_t *pp, int64_t a, int64_t b, int64_t r, int64_t *len) {
  int64_t k = -1, start = a;
  for (int64_t e = a; e < b; ++e) {
    if (e == a || pp[e] != pp[e - 1]) { ++k; if (k == r) start = e; if (k == r + 1) { *len = e - start; return start; } }
  }
  *len = b - start;
  return start;
}
/* Edge chosen by first drawing one of the segment's distinct predicates
 * uniformly, then one of that predicate's edges uniformly. */
static int64_t pick_edge(const int32_t *pp, int64_t a, int64_t b, uint64_t r1, uint64_t r2) {
  int64_t k = n_pred_runs(pp, a, b);
  int64_t len;
  int64_t st = pred_run(pp, a, b, (int64_t)(r1 % (uint64_t)k), &len);
  return st + (int64_t)(r2 % (uint64_t)len);
}
/* k edges with pairwise distinct predicates (fails if fewer predicates).
 * Predicates are drawn without replacement with weight (p+1)^bias among the
 * segment's distinct predicates (bias > 0 favours the rarer, higher-numbered
 * predicates of the Zipf order); the edge is uniform within the predicate. */
static int pick_distinct_preds(const int32_t *pp, int64_t a, int64_t b, int k, double bias,
                               uint64_t seed, uint64_t ctr, int64_t *out) {
  int64_t np = n_pred_runs(pp, a, b);
  if (np < k || k > 40) return 0;
  int64_t *rs = (int64_t *)malloc(sizeof(int64_t) * (np + 1));
  double *w = (double *)malloc(sizeof(double) * np);
  int64_t r = 0;
  for (int64_t e = a; e < b; ++e)
    if (e == a || pp[e] != pp[e - 1]) { rs[r] = e; w[r] = pow((double)pp[e] + 1.0, bias); ++r; }
  rs[np] = b;
  for (int i = 0; i < k; ++i) {
    double tot = 0;
    for (int64_t j = 0; j < np; ++j) tot += w[j];
    double x = u01(rng(seed, 100 + i, ctr)) * tot;
    int64_t j = 0;
    for (; j < np - 1; ++j) { if (w[j] > 0 && x < w[j]) break; x -= w[j]; }
    while (w[j] == 0 && j > 0) --j;
    int64_t len = rs[j + 1] - rs[j];
    out[i] = rs[j] + (int64_t)(rng(seed, 200 + i, ctr) % (uint64_t)len);
    w[j] = 0;
  }
  free(rs); free(w);
  return 1;
}

int32_t wl_walk_query(void *h, int32_t kind, int32_t n, int32_t const_mode, int32_t start,
                      double bias, uint64_t seed, uint64_t ctr, int32_t *tp3, int32_t *witness) {
  wl_index *ix = (wl_index *)h;
  if (n < 1 || n > 32) return 0;
  int64_t V = ix->V;
  (void)V;
  /* stars start at the subject (object) of a uniformly drawn triple, i.e. in
   * proportion to out- (in-) degree; other shapes at a uniform vertex */
  int32_t v0;
  if (start >= 0) v0 = start;
  else if (kind == 1 || kind == 2) {
    int64_t e = (int64_t)(rng(seed, 50, ctr) % (uint64_t)ix->n);
    v0 = kind == 1 ? ix->in_s[e] : ix->out_o[e];
  } else v0 = (int32_t)(rng(seed, 50, ctr) % (uint64_t)V);
  int nv = 0;
  int64_t pick[40];
  if (kind == 0) {
    int32_t v = v0;
    witness[nv++] = v;
    for (int i = 0; i < n; ++i) {
      int64_t d = ix->out_off[v + 1] - ix->out_off[v];
      if (d == 0) return 0;
      int64_t e = pick_edge(ix->out_p, ix->out_off[v], ix->out_off[v + 1], rng(seed, 51 + i, ctr),
                            rng(seed, 81 + i, ctr));
      tp3[3 * i] = -(nv - 1) - 1;
      tp3[3 * i + 1] = ix->out_p[e];
      tp3[3 * i + 2] = -nv - 1;
      v = ix->out_o[e];
      witness[nv++] = v;
    }
  } else if (kind == 1 || kind == 2) {
    int64_t *off = kind == 1 ? ix->out_off : ix->in_off;
    int32_t *pp = kind == 1 ? ix->out_p : ix->in_p;
    int32_t *oo = kind == 1 ? ix->out_o : ix->in_s;
    if (!pick_distinct_preds(pp, off[v0], off[v0 + 1], n, bias, seed, ctr, pick)) return 0;
    witness[nv++] = v0;
    for (int i = 0; i < n; ++i) {
      int64_t e = pick[i];
      if (kind == 1) { tp3[3 * i] = -1; tp3[3 * i + 1] = pp[e]; tp3[3 * i + 2] = -nv - 1; }
      else { tp3[3 * i] = -nv - 1; tp3[3 * i + 1] = pp[e]; tp3[3 * i + 2] = -1; }
      witness[nv++] = oo[e];
    }
  } else if (kind == 3) {
    if (n < 4) return 0;
    if (!pick_distinct_preds(ix->out_p, ix->out_off[v0], ix->out_off[v0 + 1], 2, bias, seed, ctr,
                             pick))
      return 0;
    witness[nv++] = v0;
    int32_t br[2];
    int ti = 0;
    for (int b = 0; b < 2; ++b) {
      int64_t e = pick[b];
      br[b] = ix->out_o[e];
      tp3[3 * ti] = -1; tp3[3 * ti + 1] = ix->out_p[e]; tp3[3 * ti + 2] = -nv - 1;
      witness[nv++] = br[b];
      ++ti;
    }
    /* split the remaining patterns over the two branches, as even as the
     * branch vertices' distinct out-predicates allow (at least one each);
     * what does not fit becomes further leaves of the centre */
    int rest = n - 2;
    int64_t av0 = n_pred_runs(ix->out_p, ix->out_off[br[0]], ix->out_off[br[0] + 1]);
    int64_t av1 = n_pred_runs(ix->out_p, ix->out_off[br[1]], ix->out_off[br[1] + 1]);
    if (av0 < 1 || av1 < 1) return 0;
    int k0 = (rest + 1) / 2, k1 = rest - k0;
    if (k0 > av0) { k1 += k0 - (int)av0; k0 = (int)av0; }
    if (k1 > av1) { int ex = k1 - (int)av1; k1 = (int)av1; int room = (int)av0 - k0; int mv = ex < room ? ex : room; k0 += mv; }
    if (k1 < 1) { k1 = 1; k0 = rest - 1 < k0 ? rest - 1 : k0; }
    int kc = rest - k0 - k1; /* extra centre leaves */
    if (kc < 0) return 0;
    int ks[2] = {k0, k1};
    for (int b = 0; b < 2; ++b) {
      int32_t y = br[b];
      if (!pick_distinct_preds(ix->out_p, ix->out_off[y], ix->out_off[y + 1], ks[b], bias, seed,
                               ctr * 7 + 3 + b, pick))
        return 0;
      for (int i = 0; i < ks[b]; ++i) {
        int64_t e = pick[i];
        tp3[3 * ti] = -(1 + b) - 1; tp3[3 * ti + 1] = ix->out_p[e]; tp3[3 * ti + 2] = -nv - 1;
        witness[nv++] = ix->out_o[e];
        ++ti;
      }
    }
    if (kc > 0) {
      /* further out-edges of the centre with predicates not used by the branches */
      int64_t cpick[40];
      if (!pick_distinct_preds(ix->out_p, ix->out_off[v0], ix->out_off[v0 + 1], 2 + kc, bias, seed,
                               ctr * 7 + 5, cpick))
        return 0;
      int added = 0;
      for (int i = 0; i < 2 + kc && added < kc; ++i) {
        int64_t e = cpick[i];
        if (ix->out_p[e] == tp3[1] || ix->out_p[e] == tp3[4]) continue;
        tp3[3 * ti] = -1; tp3[3 * ti + 1] = ix->out_p[e]; tp3[3 * ti + 2] = -nv - 1;
        witness[nv++] = ix->out_o[e];
        ++ti;
        ++added;
      }
      if (added < kc) return 0;
    }
  } else {
    return 0;
  }
  /* const_mode k > 0: the last k leaf variables (variables used by exactly one
   * pattern, scanned from the highest number down) become their witness
   * values; at least one variable is kept */
  for (int rep = 0; rep < const_mode && nv > 1; ++rep) {
    int32_t pick_var = -1;
    for (int32_t x = nv - 1; x >= 0 && pick_var < 0; --x) {
      int uses = 0;
      for (int i = 0; i < n; ++i) uses += (tp3[3 * i] == -x - 1) + (tp3[3 * i + 2] == -x - 1);
      if (uses == 1) pick_var = x;
    }
    if (pick_var < 0) break;
    int32_t val = witness[pick_var];
    for (int i = 0; i < n; ++i) {
      if (tp3[3 * i] == -pick_var - 1) tp3[3 * i] = val;
      if (tp3[3 * i + 2] == -pick_var - 1) tp3[3 * i + 2] = val;
    }
    /* renumber variables above pick_var down by one */
    for (int i = 0; i < n; ++i) {
      if (tp3[3 * i] < -pick_var - 1) tp3[3 * i] += 1;
      if (tp3[3 * i + 2] < -pick_var - 1) tp3[3 * i + 2] += 1;
    }
    for (int32_t x = pick_var; x < nv - 1; ++x) witness[x] = witness[x + 1];
    --nv;
  }
  return nv;
}
