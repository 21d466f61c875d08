/*
 * mg_oracle.c -- plain FP64 CPU reference of the timestep-splitting
 * Euler-Maruyama (EM) particle step on a metric graph.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The GPU library
 * shares no code with it: no header, helper, table or constant generator.
 *
 * What it follows (Dwaraknath & Ying, "Sampling on Metric Graphs"):
 *   - the EM update on the real line (Sec. 3, Eq. euler_maruyama_real_line);
 *   - Alg. 2 (EM-Step-General, appendix A.5): EM proposal, strict interior
 *     test, hit end chosen by the sign of the proposal, distance to the hit
 *     vertex, solve for the crossing fraction alpha, remaining time
 *     (1-alpha)*dt, new edge drawn from the cumulative jump weights of the
 *     hit vertex, restart at the chosen end of the new edge;
 *   - Alg. 1 (Sec. 3): at a vertex the normal is used by magnitude and points
 *     into the edge, and the step is repeated while time remains;
 *   - Corollary 1 (Sec. 3): the edge a particle leaves a vertex on is the
 *     exit that the exit counts record;
 *   - the uniform-bin histogram of the appendix kernels (A.6).
 * Where the paper is silent or garbled, the reading taken is stated where
 * it is applied below.
 *
 * Floating point: FP64, compiled with -ffp-contract=off; every fused
 * multiply-add is written as fma().  log/sqrt/cos/sin come from libm.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), keyed by the 64-bit seed,
 * counter = (particle, step word, stream word, graph tag):
 *   main stream   ctr = (p, n>>2, 0, tag): (o0,o1) and (o2,o3) are two
 *                 Box-Muller pairs; step n uses pair (n>>1)&1, cosine for
 *                 even n and sine for odd n.  This normal drives the first
 *                 sub-step of step n.
 *   hit stream    ctr = (p, n, k, tag) for the k-th vertex hit (k>=1) of
 *                 step n: o0 is the 32-bit slot draw; the cosine of the
 *                 Box-Muller pair (o1,o2) drives the sub-step after it.
 *   init stream   ctr = (p, 0xFFFFFFFF, 0xFFFFFFFF, tag): o0 picks the edge,
 *                 o1 the position.
 *   vertex stream ctr = (p, n, 0x100 + k, tag) at a Wentzell vertex: for the
 *                 k-th hit of step n (k >= 1), or for a step that starts on
 *                 a sticky vertex (k = 0); o0 decides the killing (the
 *                 holding time is not random: gamma_v times the visit's
 *                 local time).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Philox */
/* Round multipliers and Weyl key increments as published in SC'11. */
#define OR_PHILOX_M0 0xD2511F53u
#define OR_PHILOX_M1 0xCD9E8D57u
#define OR_PHILOX_W0 0x9E3779B9u
#define OR_PHILOX_W1 0xBB67AE85u

static void philox4x32_10(const uint32_t ctr[4], uint32_t k0, uint32_t k1,
                          uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { /* key schedule: bump before every round but the first */
      k0 += OR_PHILOX_W0;
      k1 += OR_PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)OR_PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)OR_PHILOX_M1 * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Batch entry for tests: ctr is [count][4], out is [count][4]. */
void or_philox_batch(const uint32_t *ctr, uint64_t seed, int64_t count,
                     uint32_t *out) {
  for (int64_t i = 0; i < count; ++i)
    philox4x32_10(ctr + 4 * i, (uint32_t)seed, (uint32_t)(seed >> 32),
                  out + 4 * i);
}

/* ----------------------------------------------------------- Box-Muller */
static const double OR_TWO_PI = 6.283185307179586476925286766559;

/* Uniform on (0,1) from 32 bits: (a + 1/2) * 2^-32, exact in FP64. */
static double unit_open(uint32_t a) { return ((double)a + 0.5) * 0x1p-32; }

/* Box-Muller (Box & Muller 1958): R = sqrt(-2 ln u1), angle 2*pi*u2. */
static void box_muller(uint32_t a, uint32_t b, double *w_cos, double *w_sin) {
  double u1 = unit_open(a);
  double u2 = unit_open(b);
  double r = sqrt(-2.0 * log(u1));
  double t = OR_TWO_PI * u2;
  if (w_cos) *w_cos = r * cos(t);
  if (w_sin) *w_sin = r * sin(t);
}

/* Normal that drives the first sub-step of step n of particle p. */
static double main_normal(uint32_t p, uint64_t n, uint32_t tag, uint64_t seed) {
  uint32_t ctr[4] = {p, (uint32_t)(n >> 2), 0u, tag};
  uint32_t o[4];
  philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), o);
  double wc, ws;
  if (((n >> 1) & 1u) == 0) box_muller(o[0], o[1], &wc, &ws);
  else box_muller(o[2], o[3], &wc, &ws);
  return (n & 1u) ? ws : wc;
}

/* Randomness consumed after the k-th vertex hit (k >= 1) of step n. */
static void hit_draw(uint32_t p, uint64_t n, uint32_t k, uint32_t tag,
                     uint64_t seed, uint32_t *slot_bits, double *w_next) {
  uint32_t ctr[4] = {p, (uint32_t)n, k, tag};
  uint32_t o[4];
  philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), o);
  *slot_bits = o[0];
  box_muller(o[1], o[2], w_next, NULL);
}

/* Test entry: main-stream normals for (p[i], n[i]). */
void or_main_normals(const uint32_t *p, const uint64_t *n, int64_t count,
                     uint32_t tag, uint64_t seed, double *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = main_normal(p[i], n[i], tag, seed);
}

/* Test entry: hit-stream draws for (p[i], n[i], k[i]). */
void or_hit_draws(const uint32_t *p, const uint64_t *n, const uint32_t *k,
                  int64_t count, uint32_t tag, uint64_t seed,
                  uint32_t *slot_bits, double *w_next) {
  for (int64_t i = 0; i < count; ++i)
    hit_draw(p[i], n[i], k[i], tag, seed, slot_bits + i, w_next + i);
}

/* ---------------------------------------------------------------- graph */
typedef struct {
  int32_t n_vertices, n_edges;
  const int32_t *edge_init, *edge_term;   /* [E] */
  const double *length;                   /* [E] */
  const double *drift_a, *drift_c;        /* [E] mu_e(x) = a_e + c_e x */
  const double *sigma;                    /* [E] */
  const int32_t *vtx_offsets;             /* [V+1] */
  const int32_t *slot_edge;               /* [nnz] */
  const uint8_t *slot_orient;             /* [nnz] 0: enter at x=0, 1: at x=L */
  const double *slot_jump_prob;           /* [nnz] b_{v,e} */
  const uint8_t *vtx_kind;                /* [V] 0 standard, 1 absorbing,
                                             2 mirror (a reflecting leaf) */
  const double *bin_span;                 /* [E] length the uniform bins cover */
  /* [E] each, or NULL (zero): higher terms of the coefficient functions,
     mu_e(x) = a + c x + c2 x^2 + c3 x^3, sigma_e(x) = sigma + s1 x + s2 x^2
     + s3 x^3 (Sec. 2.2 allows any C^1 coefficients) */
  const double *drift_c2, *drift_c3;
  const double *sigma_c1, *sigma_c2, *sigma_c3;
  /* [V] each, or NULL: a_v and c_v of a Wentzell vertex (kind 3), read
     only at such vertices (Sec. 2.2, the general gluing condition) */
  const double *vtx_kill, *vtx_sticky;
  /* Tabulated coefficients (Sec. 2.2 allows any C^1 drift and diffusion):
     [E+1] offsets, or NULL for none.  Edge e with table_offsets[e+1] -
     table_offsets[e] = K + 1 >= 2 knots has, at x_j = j L / K, the drift
     value and derivative table_mu/table_dmu and the diffusion value and
     derivative table_sigma/table_dsigma (index table_offsets[e] + j); its
     coefficient functions are the cubic Hermite interpolants of these
     (C^1), replacing its drift_a, drift_c, sigma and higher terms. */
  const int32_t *table_offsets;
  const double *table_mu, *table_dmu, *table_sigma, *table_dsigma;
} or_graph;

/* Cubic p0 + p1 x + p2 x^2 + p3 x^3 by Horner's rule; NULL higher arrays
   count as zero, which leaves exactly fma(p1, x, p0). */
static double coef(const double *p2, const double *p3, int32_t e, double p0, double p1,
                   double x) {
  const double c2 = p2 ? p2[e] : 0.0, c3 = p3 ? p3[e] : 0.0;
  return fma(fma(fma(c3, x, c2), x, p1), x, p0);
}
/* Cubic Hermite interpolant at x in [0, L] of values v and derivatives d
   given at the K + 1 knots j h, h = L / K (index k0 + j): on the interval
   j = floor(x / h) (the last one for x = L), with t = x / h - j,
   v_j H00(t) + h d_j H10(t) + v_{j+1} H01(t) + h d_{j+1} H11(t), the
   Hermite basis H00 = 2t^3 - 3t^2 + 1, H10 = t^3 - 2t^2 + t,
   H01 = -2t^3 + 3t^2, H11 = t^3 - t^2.  C^1 on [0, L]. */
static double hermite(const double *v, const double *d, int32_t k0, int32_t K, double L,
                      double x) {
  const double h = L / (double)K;
  const double s = x / h;
  int32_t j = (int32_t)floor(s);
  if (j < 0) j = 0;
  if (j > K - 1) j = K - 1;
  const double t = s - (double)j;
  const double t2 = t * t, t3 = t2 * t;
  const double h00 = 2.0 * t3 - 3.0 * t2 + 1.0;
  const double h10 = t3 - 2.0 * t2 + t;
  const double h01 = -2.0 * t3 + 3.0 * t2;
  const double h11 = t3 - t2;
  return h00 * v[k0 + j] + h10 * h * d[k0 + j] + h01 * v[k0 + j + 1] + h11 * h * d[k0 + j + 1];
}
/* Intervals of edge e's table, 0 if it has none. */
static int32_t table_k(const or_graph *g, int32_t e) {
  if (!g->table_offsets) return 0;
  const int32_t n = g->table_offsets[e + 1] - g->table_offsets[e];
  return n >= 2 ? n - 1 : 0;
}
static double drift_at(const or_graph *g, int32_t e, double x) {
  const int32_t K = table_k(g, e);
  if (K) return hermite(g->table_mu, g->table_dmu, g->table_offsets[e], K, g->length[e], x);
  return coef(g->drift_c2, g->drift_c3, e, g->drift_a[e], g->drift_c[e], x);
}
static double sigma_at(const or_graph *g, int32_t e, double x) {
  const int32_t K = table_k(g, e);
  if (K)
    return hermite(g->table_sigma, g->table_dsigma, g->table_offsets[e], K, g->length[e], x);
  const double s1 = g->sigma_c1 ? g->sigma_c1[e] : 0.0;
  return coef(g->sigma_c2, g->sigma_c3, e, g->sigma[e], s1, x);
}

/*
 * Integer slot thresholds (the reading of the slot draw).  Per
 * vertex, b is divided by its sum, accumulated left to right in FP64 into
 * C_s, and T_s = floor(C_s * 2^32).  From the last slot with b > 0 onward
 * T_s = 2^32, so a trailing zero-probability slot is never drawn.  The slot
 * for a 32-bit draw r is the first s with r < T_s.
 * Returns 0, or -1 if a standard vertex has no positive weight.
 */
int or_thresholds(const or_graph *g, uint64_t *thr) {
  for (int32_t v = 0; v < g->n_vertices; ++v) {
    int32_t s0 = g->vtx_offsets[v], s1 = g->vtx_offsets[v + 1];
    double total = 0.0;
    int32_t last_pos = -1;
    for (int32_t s = s0; s < s1; ++s) {
      total += g->slot_jump_prob[s];
      if (g->slot_jump_prob[s] > 0.0) last_pos = s;
    }
    if (last_pos < 0) {
      for (int32_t s = s0; s < s1; ++s) thr[s] = 0;
      if (s1 > s0 && (!g->vtx_kind || g->vtx_kind[v] != 1)) return -1;
      continue;
    }
    double cum = 0.0;
    for (int32_t s = s0; s < s1; ++s) {
      cum += g->slot_jump_prob[s] / total;
      if (s >= last_pos) {
        thr[s] = (uint64_t)1 << 32;
      } else {
        double t = floor(cum * 4294967296.0);
        thr[s] = t >= 4294967296.0 ? ((uint64_t)1 << 32) : (uint64_t)t;
      }
    }
  }
  return 0;
}

static int32_t pick_slot(const or_graph *g, const uint64_t *thr, int32_t v,
                         uint32_t r) {
  int32_t s0 = g->vtx_offsets[v], s1 = g->vtx_offsets[v + 1];
  for (int32_t s = s0; s < s1; ++s)
    if ((uint64_t)r < thr[s]) return s;
  return s1 - 1;
}

/* -------------------------------------------------- Wentzell vertices */
/*
 * Reading A27 (Sec. 2.2, the Wentzell gluing condition
 * a_v f(v) - sum_e b_ve f'_e(v) + c_v (L f)(v) = 0 with a_v + sum b + c_v = 1;
 * the paper writes the last term as c_v f''(v)/2, the generator of its
 * standard Brownian motion).  With beta_v = sum_e b_ve the process leaves v
 * into edge e with probability b_ve / beta_v, is killed at rate
 * kappa_v = a_v / beta_v per unit of its local time at v, and spends
 * gamma_v = c_v / beta_v units of time on v per unit of that local time
 * (local time in units of length: the reflection term of the distance to v).
 *
 * In the split scheme a visit of v is a hit (or a step that starts on v)
 * followed by the sub-step that leaves v.  The local time of a visit is its
 * share of the reflection term of the distance to v: the overshoot o of the
 * proposal that crossed v (how far past v the free move would have gone)
 * plus the mean local time sigma_v sqrt(2 h'' / pi) of the reflected move
 * of length h'' that leaves v (Levy: the local time of reflected Brownian
 * motion has the law of |B|).  Over many visits these add up to the local
 * time whatever the density next to v looks like.  Per visit:
 *   - the particle first stays on v for gamma_v l, then moves for h'',
 *     with h'' + gamma_v (o + sigma_v sqrt(2 h'' / pi)) = h (the time left
 *     in the step); when gamma_v o >= h it stays on v for all of h and
 *     owes the rest of its stay, which it works off at the start of the
 *     next steps and then leaves v with a visit of its own (o = 0);
 *   - it is killed with probability 1 - exp(-kappa_v l) (o alone while it
 *     stays on v for the rest of the step; the move's part when it leaves).
 * sigma_v is the b-weighted mean of the incident edges' diffusion at v
 * (sigma is continuous at vertices in the paper; then this is its value).
 * A particle owing a stay sits on v; its position field holds the time it
 * still owes as a signed offset beyond the end it sits on (-t at the
 * initial end, L + t at the terminal end).
 */
typedef struct {
  double *kappa;    /* [V] a_v / beta_v (0: no killing) */
  double *gamma;    /* [V] c_v / beta_v (0: not sticky) */
  double *sigma_v;  /* [V] diffusion at v */
} or_wentzell;

static const double OR_PI = 3.14159265358979323846264338327950288;

static int wentzell_params(const or_graph *g, or_wentzell *wz) {
  const int32_t V = g->n_vertices;
  const size_t nv = (size_t)(V > 0 ? V : 1);
  wz->kappa = (double *)calloc(nv, sizeof(double));
  wz->gamma = (double *)calloc(nv, sizeof(double));
  wz->sigma_v = (double *)calloc(nv, sizeof(double));
  if (!wz->kappa || !wz->gamma || !wz->sigma_v) return -2;
  for (int32_t v = 0; v < V; ++v) {
    if (!g->vtx_kind || g->vtx_kind[v] != 3) continue;
    const int32_t s0 = g->vtx_offsets[v], s1 = g->vtx_offsets[v + 1];
    double beta = 0.0, sig = 0.0;
    for (int32_t s = s0; s < s1; ++s) beta += g->slot_jump_prob[s];
    if (!(beta > 0.0)) return -1;
    for (int32_t s = s0; s < s1; ++s) {
      const int32_t e = g->slot_edge[s];
      const double at = g->slot_orient[s] ? g->length[e] : 0.0;
      sig += (g->slot_jump_prob[s] / beta) * sigma_at(g, e, at);
    }
    wz->kappa[v] = (g->vtx_kill ? g->vtx_kill[v] : 0.0) / beta;
    wz->gamma[v] = (g->vtx_sticky ? g->vtx_sticky[v] : 0.0) / beta;
    wz->sigma_v[v] = sig;
  }
  return 0;
}

static void wentzell_free(or_wentzell *wz) {
  free(wz->kappa);
  free(wz->gamma);
  free(wz->sigma_v);
}

/* Vertex-stream draw for visit k (k-th hit, or 0 for a step start). */
static uint32_t vertex_draw(uint32_t p, uint64_t n, uint32_t k, uint32_t tag,
                            uint64_t seed) {
  uint32_t ctr[4] = {p, (uint32_t)n, 0x100u + k, tag};
  uint32_t o[4];
  philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), o);
  return o[0];
}

/*
 * One visit of Wentzell vertex v with overshoot o and time h left in the
 * step.  Returns 1 if the particle is killed.  Otherwise *h_move is the
 * length of the move that leaves v (0: the particle stays on v for the
 * rest of the step) and *owed the stay it still owes after this step.
 */
static int wentzell_visit(const or_wentzell *wz, int32_t v, double o, double h,
                          uint32_t kill_bits, double *h_move, double *owed) {
  const double gam = wz->gamma[v], sig = wz->sigma_v[v];
  const double c = sig * sqrt(2.0 / OR_PI);  /* mean local time of a move: c sqrt(h'') */
  double hm, lt;
  *owed = 0.0;
  if (gam == 0.0) {
    hm = h;
    lt = o + c * sqrt(h);
  } else if (gam * o >= h) {
    hm = 0.0;
    lt = o;
    *owed = gam * o - h;
  } else {
    /* s = sqrt(h'') solves s^2 + gam c s - (h - gam o) = 0 (s >= 0), in the
       cancellation-free form 2 r / (b + sqrt(b^2 + 4 r)) */
    const double b = gam * c, r = h - gam * o;
    const double sq = 2.0 * r / (b + sqrt(b * b + 4.0 * r));
    hm = sq * sq;
    lt = o + c * sq;
  }
  *h_move = hm;
  return wz->kappa[v] > 0.0 && unit_open(kill_bits) < -expm1(-wz->kappa[v] * lt);
}

/* --------------------------------------------------------- crossing time */
/*
 * Smallest u in (0,1] with  C + B u + A u^2 = 0,  C >= 0  (u = sqrt(alpha)).
 * This is Alg. 2's "solve for alpha" written in the distance-to-hit-vertex
 * frame (reading A4: the term end flips the signs of A and B), solved by the
 * cancellation-free form of the quadratic formula (Press et al., Numerical
 * Recipes, Sec. 5.6): q = -(B + sgn(B) sqrt(B^2 - 4AC))/2, roots q/A, C/q.
 * C == 0 (the particle sits on the vertex) has roots 0 and -B/A; the nonzero
 * one is the crossing (reading A5).  Rounding can push the root just past 1;
 * it is clamped to [0, 1].
 */
static double first_root(double A, double B, double C) {
  double u;
  if (C == 0.0) {
    if (A == 0.0) return 0.0;
    u = -B / A;
  } else if (A == 0.0) {
    u = -C / B;
  } else {
    double disc = B * B - 4.0 * A * C;
    if (disc < 0.0) disc = 0.0;
    double sq = sqrt(disc);
    double q = -0.5 * (B >= 0.0 ? B + sq : B - sq);
    double r1 = q / A;
    double r2 = C / q;
    double lo = r1 < r2 ? r1 : r2;
    double hi = r1 < r2 ? r2 : r1;
    u = lo > 0.0 ? lo : hi;
    if (!(u > 0.0)) u = 1.0;
  }
  if (!(u >= 0.0)) u = 0.0;
  if (u > 1.0) u = 1.0;
  return u;
}

/* Test entry for the root solver. */
void or_first_root_batch(const double *A, const double *B, const double *C,
                         int64_t count, double *u) {
  for (int64_t i = 0; i < count; ++i) u[i] = first_root(A[i], B[i], C[i]);
}

/* ------------------------------------------------------------- sequence */
/* Word-wise FNV-1a (Fowler-Noll-Vo) over 32-bit words: records the exact
 * sequence of (step, slot) hits of a particle for parity tests. */
#define OR_FNV_OFFSET 0xcbf29ce484222325ull
#define OR_FNV_PRIME 0x100000001b3ull
static uint64_t fnv_word(uint64_t h, uint32_t w) { return (h ^ w) * OR_FNV_PRIME; }

uint64_t or_fnv_offset(void) { return OR_FNV_OFFSET; }

/* ------------------------------------------------------------ counters */
typedef struct {
  uint64_t *exit_slot;   /* [nnz] */
  uint64_t *absorbed;    /* [V]   */
  uint64_t truncations;
  uint64_t substeps;     /* consumed normals */
  uint64_t hits;
} or_counts;

/* Optional per-hit trace for tests (one particle at a time). */
typedef struct {
  int64_t cap, len;
  uint64_t *step;     /* n */
  int32_t *k;         /* hit index within the step, 1-based */
  int32_t *vertex;    /* hit vertex */
  int32_t *slot;      /* slot drawn, -1 if absorbed */
  double *u;          /* sqrt(alpha) */
  double *h_after;    /* remaining time after the hit */
} or_trace;

/*
 * One particle through steps [n0, n0 + n_steps).  State: edge e, position x
 * measured from e's initial vertex, alive flag.  A position equal to 0 or to
 * L_e means the particle sits on that vertex.
 */
static void run_particle(const or_graph *g, const uint64_t *thr,
                         const or_wentzell *wz, uint32_t p,
                         int32_t *e_io, double *x_io, uint8_t *alive_io,
                         uint64_t *hash_io, uint32_t *hits_io, uint64_t n0,
                         uint64_t n_steps, double dt, uint64_t seed,
                         uint32_t tag, int32_t max_splits, or_counts *cnt,
                         or_trace *tr) {
  int32_t e = *e_io;
  double x = *x_io;
  uint8_t alive = *alive_io;
  uint64_t hash = *hash_io;
  uint32_t hits = *hits_io;

  for (uint64_t n = n0; n < n0 + n_steps && alive; ++n) {
    double h = dt;           /* time left in this step */
    int32_t k = 0;           /* vertex hits in this step */
    int32_t last_slot = -1;  /* slot of the last hit */
    double w = main_normal(p, n, tag, seed);
    /* A step that starts on a Wentzell vertex (reading A27): a particle that
       owes a stay there works it off first; one that sits on the vertex, or
       has just finished its stay, leaves it with a visit of its own.  A step
       that ends where it started (on the vertex, or killed at the visit)
       counts its one sub-step without a move. */
    {
      const double L0 = g->length[e];
      int32_t v0 = -1;
      int init0 = 0;
      double owe = 0.0;
      if (x <= 0.0) {
        v0 = g->edge_init[e];
        init0 = 1;
        owe = -x;
      } else if (x >= L0) {
        v0 = g->edge_term[e];
        owe = x - L0;
      }
      if (v0 >= 0 && g->vtx_kind && g->vtx_kind[v0] == 3) {
        if (owe >= h) {
          owe = owe - h;
          x = init0 ? -owe : L0 + owe;
          cnt->substeps++;
          continue;
        }
        h = h - owe;
        x = init0 ? 0.0 : L0;
        double hm, owed;
        if (wentzell_visit(wz, v0, 0.0, h, vertex_draw(p, n, 0u, tag, seed), &hm, &owed)) {
          alive = 0;
          cnt->absorbed[v0]++;
          cnt->substeps++;
          hash = fnv_word(fnv_word(hash, (uint32_t)n), 0x80000000u | (uint32_t)v0);
          continue;
        }
        if (hm == 0.0) {
          x = init0 ? -owed : L0 + owed;
          cnt->substeps++;
          continue;
        }
        h = hm;
      }
    }
    for (;;) {
      const double L = g->length[e];
      /* At a vertex the normal is used by magnitude, pointing into the edge
         (Alg. 1; reading A3). */
      if (x == 0.0) w = fabs(w);
      else if (x == L) w = -fabs(w);
      /* EM proposal (Alg. 2): x + mu(x) h + sigma(x) sqrt(h) W, both
         coefficients frozen at the sub-step's starting point. */
      const double mu = drift_at(g, e, x);
      const double gsd = sigma_at(g, e, x) * sqrt(h);
      const double xt = fma(gsd, w, fma(mu, h, x));
      cnt->substeps++;
      if (xt > 0.0 && xt < L) { /* strict interior test (reading A6) */
        x = xt;
        break;
      }
      /* Vertex hit: the end is init if the proposal is <= 0 (reading A8). */
      const int hit_init = xt <= 0.0;
      const int32_t v = hit_init ? g->edge_init[e] : g->edge_term[e];
      /* Mirror leaf (reading A25; the far-end reflection of the star-graph
         kernel in the appendix): the mirror image in the vertex ends the
         step when it lies inside the edge; no vertex hit is recorded. */
      if (g->vtx_kind && g->vtx_kind[v] == 2) {
        const double xr = hit_init ? -xt : 2.0 * L - xt;
        if (xr > 0.0 && xr < L) {
          x = xr;
          break;
        }
      }
      const double d = hit_init ? x : L - x;
      const double A = hit_init ? mu * h : -(mu * h);
      const double B = hit_init ? gsd * w : -(gsd * w);
      const double u = first_root(A, B, d);
      const double alpha = u * u;
      h = fma(-alpha, h, h);  /* remaining time (1 - alpha) h */
      k++;
      hits++;
      cnt->hits++;
      /* Wentzell vertex (reading A27): the visit that starts with this hit,
         its overshoot being how far past v the proposal went. */
      const int wentzell = g->vtx_kind && g->vtx_kind[v] == 3;
      double h_move = h, owed = 0.0;
      int killed = 0;
      if (wentzell) {
        const double o = hit_init ? -xt : xt - L;
        killed = wentzell_visit(wz, v, o, h, vertex_draw(p, n, (uint32_t)k, tag, seed),
                                &h_move, &owed);
      }
      if (killed || (g->vtx_kind && g->vtx_kind[v] == 1)) { /* absorbing (reading A17) */
        alive = 0;
        cnt->absorbed[v]++;
        hash = fnv_word(fnv_word(hash, (uint32_t)n), 0x80000000u | (uint32_t)v);
        if (tr && tr->len < tr->cap) {
          tr->step[tr->len] = n; tr->k[tr->len] = k; tr->vertex[tr->len] = v;
          tr->slot[tr->len] = -1; tr->u[tr->len] = u; tr->h_after[tr->len] = h;
          tr->len++;
        }
        break;
      }
      uint32_t r;
      double w_next;
      hit_draw(p, n, (uint32_t)k, tag, seed, &r, &w_next);
      const int32_t s = pick_slot(g, thr, v, r);
      e = g->slot_edge[s];
      x = g->slot_orient[s] ? g->length[e] : 0.0;
      last_slot = s;
      hash = fnv_word(fnv_word(hash, (uint32_t)n), (uint32_t)s);
      if (tr && tr->len < tr->cap) {
        tr->step[tr->len] = n; tr->k[tr->len] = k; tr->vertex[tr->len] = v;
        tr->slot[tr->len] = s; tr->u[tr->len] = u; tr->h_after[tr->len] = h;
        tr->len++;
      }
      if (wentzell) {
        h = h_move;
        if (h == 0.0) {        /* stays on v for the rest of the step */
          x = g->slot_orient[s] ? g->length[e] + owed : -owed;
          break;
        }
      }
      if (h == 0.0) break;     /* the step ended exactly on the vertex */
      if (k == max_splits) {   /* split cap reached: drop the rest (A9) */
        cnt->truncations++;
        break;
      }
      w = w_next;
    }
    /* Exit record of this step (reading A12, Corollary 1). */
    if (k >= 1 && alive) cnt->exit_slot[last_slot]++;
  }
  *e_io = e;
  *x_io = x;
  *alive_io = alive;
  *hash_io = hash;
  *hits_io = hits;
}

/*
 * Advance particles.  pid[i] is the RNG particle index of row i (rows may
 * be any subset).  Counters are added into the caller's arrays.
 */
int or_simulate(const or_graph *g, int64_t count, const uint32_t *pid,
                int32_t *edge, double *x, uint8_t *alive, uint64_t *hash,
                uint32_t *hits, uint64_t n0, uint64_t n_steps, double dt,
                uint64_t seed, uint32_t tag, int32_t max_splits,
                uint64_t *exit_slot, uint64_t *absorbed, uint64_t *scalars,
                int32_t n_threads) {
  const int32_t V = g->n_vertices;
  const int32_t nnz = g->vtx_offsets[V];
  uint64_t *thr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
  if (!thr) return -2;
  if (or_thresholds(g, thr) != 0) { free(thr); return -1; }
  or_wentzell wz;
  const int wrc = wentzell_params(g, &wz);
  if (wrc != 0) { wentzell_free(&wz); free(thr); return wrc; }
  if (n_threads < 1) n_threads = 1;
  int64_t nth = n_threads;
  uint64_t *priv = (uint64_t *)calloc((size_t)nth * (size_t)(nnz + V + 3), sizeof(uint64_t));
  if (!priv) { wentzell_free(&wz); free(thr); return -2; }
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads)
  for (int64_t i = 0; i < count; ++i) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    uint64_t *base = priv + (size_t)tid * (size_t)(nnz + V + 3);
    or_counts c;
    c.exit_slot = base;
    c.absorbed = base + nnz;
    c.truncations = 0; c.substeps = 0; c.hits = 0;
    run_particle(g, thr, &wz, pid[i], &edge[i], &x[i], &alive[i], &hash[i], &hits[i],
                 n0, n_steps, dt, seed, tag, max_splits, &c, NULL);
    base[nnz + V] += c.truncations;
    base[nnz + V + 1] += c.substeps;
    base[nnz + V + 2] += c.hits;
  }
  for (int64_t t = 0; t < nth; ++t) {
    uint64_t *base = priv + (size_t)t * (size_t)(nnz + V + 3);
    for (int32_t s = 0; s < nnz; ++s) exit_slot[s] += base[s];
    for (int32_t v = 0; v < V; ++v) absorbed[v] += base[nnz + v];
    scalars[0] += base[nnz + V];
    scalars[1] += base[nnz + V + 1];
    scalars[2] += base[nnz + V + 2];
  }
  free(priv);
  wentzell_free(&wz);
  free(thr);
  return 0;
}

/* One particle with a per-hit trace (tests only). */
int or_simulate_traced(const or_graph *g, uint32_t pid, int32_t *edge, double *x,
                       uint8_t *alive, uint64_t *hash, uint32_t *hits,
                       uint64_t n0, uint64_t n_steps, double dt, uint64_t seed,
                       uint32_t tag, int32_t max_splits, uint64_t *exit_slot,
                       uint64_t *absorbed, uint64_t *scalars, int64_t cap,
                       uint64_t *t_step, int32_t *t_k, int32_t *t_vertex,
                       int32_t *t_slot, double *t_u, double *t_h,
                       int64_t *t_len) {
  const int32_t nnz = g->vtx_offsets[g->n_vertices];
  uint64_t *thr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
  if (!thr) return -2;
  if (or_thresholds(g, thr) != 0) { free(thr); return -1; }
  or_counts c;
  c.exit_slot = exit_slot; c.absorbed = absorbed;
  c.truncations = 0; c.substeps = 0; c.hits = 0;
  or_wentzell wz;
  const int wrc = wentzell_params(g, &wz);
  if (wrc != 0) { wentzell_free(&wz); free(thr); return wrc; }
  or_trace tr = {cap, 0, t_step, t_k, t_vertex, t_slot, t_u, t_h};
  run_particle(g, thr, &wz, pid, edge, x, alive, hash, hits, n0, n_steps, dt, seed,
               tag, max_splits, &c, &tr);
  wentzell_free(&wz);
  scalars[0] += c.truncations;
  scalars[1] += c.substeps;
  scalars[2] += c.hits;
  *t_len = tr.len;
  free(thr);
  return 0;
}

/* ----------------------------------------------------------------- init */
/*
 * Initial states.  mode 1: every particle starts on vertex `vertex`; its
 * edge is drawn from that vertex's jump probabilities with o0 of the init
 * stream and it sits on the chosen end (reading A20).  mode 2: the edge is
 * drawn with probability proportional to its length (o0 against integer
 * thresholds of the cumulative normalised lengths, built like the slot
 * thresholds) and the position is L_e * (o1 + 1/2) 2^-32.
 */
int or_init(const or_graph *g, int64_t count, const uint32_t *pid, int32_t mode,
            int32_t vertex, uint64_t seed, uint32_t tag, int32_t *edge,
            double *x, uint8_t *alive, uint64_t *hash, uint32_t *hits) {
  const int32_t E = g->n_edges;
  const int32_t nnz = g->vtx_offsets[g->n_vertices];
  uint64_t *thr = NULL;
  if (mode == 1) {
    thr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!thr) return -2;
    if (or_thresholds(g, thr) != 0) { free(thr); return -1; }
  } else if (mode == 2) {
    thr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)E);
    if (!thr) return -2;
    double total = 0.0;
    for (int32_t e = 0; e < E; ++e) total += g->length[e];
    double cum = 0.0;
    for (int32_t e = 0; e < E; ++e) {
      cum += g->length[e];
      if (e == E - 1) {
        thr[e] = (uint64_t)1 << 32;
      } else {
        double t = floor((cum / total) * 4294967296.0);
        thr[e] = t >= 4294967296.0 ? ((uint64_t)1 << 32) : (uint64_t)t;
      }
    }
  } else {
    return -1;
  }
  for (int64_t i = 0; i < count; ++i) {
    uint32_t ctr[4] = {pid[i], 0xFFFFFFFFu, 0xFFFFFFFFu, tag};
    uint32_t o[4];
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), o);
    if (mode == 1) {
      int32_t s = pick_slot(g, thr, vertex, o[0]);
      int32_t e = g->slot_edge[s];
      edge[i] = e;
      x[i] = g->slot_orient[s] ? g->length[e] : 0.0;
    } else {
      int32_t e = E - 1;
      for (int32_t j = 0; j < E; ++j)
        if ((uint64_t)o[0] < thr[j]) { e = j; break; }
      edge[i] = e;
      x[i] = g->length[e] * unit_open(o[1]);
    }
    alive[i] = 1;
    hash[i] = OR_FNV_OFFSET;
    hits[i] = 0;
  }
  free(thr);
  return 0;
}

/*
 * Injection at source vertices (the tracer problem's inlets, Sec. 4.2):
 * particle i starts on a source vertex drawn with probability proportional
 * to its rate, on an incident edge drawn from that vertex's b (the vertex
 * rule of Alg. 1, as for a particle started on one vertex).  Init-stream
 * word 0 draws the source (cumulative rate thresholds built like the slot
 * thresholds: normalised running sum, floor(C 2^32), 2^32 for the last
 * source of positive rate), word 1 the slot.
 */
int or_init_sources(const or_graph *g, int64_t count, const uint32_t *pid,
                    int32_t n_src, const int32_t *src_v, const double *src_rate,
                    uint64_t seed, uint32_t tag, int32_t *edge, double *x,
                    uint8_t *alive, uint64_t *hash, uint32_t *hits) {
  const int32_t nnz = g->vtx_offsets[g->n_vertices];
  if (n_src < 1) return -1;
  double total = 0.0;
  int32_t last_pos = -1;
  for (int32_t j = 0; j < n_src; ++j) {
    if (src_v[j] < 0 || src_v[j] >= g->n_vertices) return -1;
    if (!(src_rate[j] >= 0.0)) return -1;
    total += src_rate[j];
    if (src_rate[j] > 0.0) last_pos = j;
  }
  if (last_pos < 0) return -1;
  uint64_t *sthr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n_src);
  uint64_t *thr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
  if (!sthr || !thr) { free(sthr); free(thr); return -2; }
  double cum = 0.0;
  for (int32_t j = 0; j < n_src; ++j) {
    cum += src_rate[j] / total;
    if (j >= last_pos) {
      sthr[j] = (uint64_t)1 << 32;
    } else {
      double t = floor(cum * 4294967296.0);
      sthr[j] = t >= 4294967296.0 ? ((uint64_t)1 << 32) : (uint64_t)t;
    }
  }
  if (or_thresholds(g, thr) != 0) { free(sthr); free(thr); return -1; }
  for (int64_t i = 0; i < count; ++i) {
    uint32_t ctr[4] = {pid[i], 0xFFFFFFFFu, 0xFFFFFFFFu, tag};
    uint32_t o[4];
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), o);
    int32_t j = n_src - 1;
    for (int32_t k = 0; k < n_src; ++k)
      if ((uint64_t)o[0] < sthr[k]) { j = k; break; }
    const int32_t v = src_v[j];
    const int32_t s = pick_slot(g, thr, v, o[1]);
    const int32_t e = g->slot_edge[s];
    edge[i] = e;
    x[i] = g->slot_orient[s] ? g->length[e] : 0.0;
    alive[i] = 1;
    hash[i] = OR_FNV_OFFSET;
    hits[i] = 0;
  }
  free(sthr);
  free(thr);
  return 0;
}

/* ------------------------------------------------------------ histogram */
/*
 * Uniform-bin histogram of alive particles (appendix kernel; reading A13):
 * bin = min(nb - 1, floor(x * (nb / S_e))), counted into out[e * nb + bin],
 * with S_e the binned length (the edge length unless given otherwise; a
 * semi-infinite edge needs one), so positions beyond S_e land in the last
 * bin.
 */
void or_histogram(const or_graph *g, int64_t count, const int32_t *edge,
                  const double *x, const uint8_t *alive, int32_t nb,
                  uint64_t *out) {
  for (int64_t i = 0; i < count; ++i) {
    if (!alive[i]) continue;
    const int32_t e = edge[i];
    const double inv = (double)nb / g->bin_span[e];
    double f = floor(x[i] * inv);
    int64_t b = f < 0.0 ? 0 : (int64_t)f;
    if (b > nb - 1) b = nb - 1;
    out[(int64_t)e * nb + b]++;
  }
}
