/* Runs every entry point of the FP64 oracle on small graphs that use all of
 * its features (standard, absorbing and mirror vertices, cubic coefficients,
 * a semi-infinite edge, a self-loop, zero jump probabilities, the split cap,
 * injection sources, traced runs that overflow their trace buffer), for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer.  The oracle's
 * source is compiled into this program (one translation unit), without
 * OpenMP.  Exits 0 after checking that particles are conserved. */
#include "../../oracle/mg_oracle.c"

#include <stdio.h>

static int fail(const char *what) {
  fprintf(stderr, "oracle_sanitize: %s\n", what);
  return 1;
}

/* Particles conserved: alive + absorbed = count, histogram total = alive. */
static int run_graph(const or_graph *g, int64_t count, int32_t mode, int32_t vertex,
                     int32_t max_splits, double dt, int64_t steps) {
  const int32_t V = g->n_vertices, E = g->n_edges, nnz = g->vtx_offsets[V];
  uint32_t *pid = malloc(sizeof *pid * (size_t)count);
  int32_t *edge = malloc(sizeof *edge * (size_t)count);
  double *x = malloc(sizeof *x * (size_t)count);
  uint8_t *alive = malloc((size_t)count);
  uint64_t *hash = malloc(sizeof *hash * (size_t)count);
  uint32_t *hits = malloc(sizeof *hits * (size_t)count);
  uint64_t *exit_slot = calloc((size_t)nnz, sizeof(uint64_t));
  uint64_t *absorbed = calloc((size_t)V, sizeof(uint64_t));
  uint64_t sc[3] = {0, 0, 0};
  const int32_t nb = 7;
  uint64_t *hist = calloc((size_t)E * nb, sizeof(uint64_t));
  int rc = 0;
  for (int64_t i = 0; i < count; ++i) pid[i] = (uint32_t)(i * 7 + 3);
  if (or_init(g, count, pid, mode, vertex, 11, 2, edge, x, alive, hash, hits) != 0)
    rc = fail("or_init");
  /* two calls, the second from a step count that is not a multiple of 4 */
  if (!rc && or_simulate(g, count, pid, edge, x, alive, hash, hits, 0, 3, dt, 5, 2,
                         max_splits, exit_slot, absorbed, sc, 1) != 0)
    rc = fail("or_simulate");
  if (!rc && or_simulate(g, count, pid, edge, x, alive, hash, hits, 3, steps, dt, 5, 2,
                         max_splits, exit_slot, absorbed, sc, 1) != 0)
    rc = fail("or_simulate");
  if (!rc) {
    or_histogram(g, count, edge, x, alive, nb, hist);
    uint64_t n_alive = 0, n_abs = 0, n_hist = 0;
    for (int64_t i = 0; i < count; ++i) n_alive += alive[i];
    for (int32_t v = 0; v < V; ++v) n_abs += absorbed[v];
    for (int64_t b = 0; b < (int64_t)E * nb; ++b) n_hist += hist[b];
    if (n_alive + n_abs != (uint64_t)count || n_hist != n_alive) rc = fail("mass");
    printf("graph V=%d E=%d: alive %llu absorbed %llu truncations %llu substeps %llu hits %llu\n",
           V, E, (unsigned long long)n_alive, (unsigned long long)n_abs,
           (unsigned long long)sc[0], (unsigned long long)sc[1], (unsigned long long)sc[2]);
  }
  /* a traced particle whose trace buffer is too short for its hits */
  if (!rc) {
    enum { CAP = 3 };
    uint64_t ts[CAP];
    int32_t tk[CAP], tv[CAP], tsl[CAP];
    double tu[CAP], th[CAP];
    int64_t tlen = 0;
    int32_t e1 = edge[0];
    double x1 = x[0];
    uint8_t a1 = 1;
    uint64_t h1 = OR_FNV_OFFSET;
    uint32_t k1 = 0;
    uint64_t sc1[3] = {0, 0, 0};
    if (or_simulate_traced(g, 5, &e1, &x1, &a1, &h1, &k1, 0, 200, dt, 9, 0, max_splits,
                           exit_slot, absorbed, sc1, CAP, ts, tk, tv, tsl, tu, th, &tlen) != 0)
      rc = fail("or_simulate_traced");
    if (!rc && (tlen < 0 || tlen > CAP)) rc = fail("trace length");
  }
  free(pid); free(edge); free(x); free(alive); free(hash); free(hits);
  free(exit_slot); free(absorbed); free(hist);
  return rc;
}

int main(void) {
  int rc = 0;
  /* 4-edge star: centre 0; leaf 1 standard, 2 absorbing, 3 mirror, edge 3
     a self-loop at the centre; zero b on one centre slot */
  {
    const int32_t ei[4] = {0, 0, 0, 0}, et[4] = {1, 2, 3, 0};
    const double L[4] = {1.0, 0.5, 0.8, 0.3};
    const double a[4] = {-3.0, 2.0, 0.0, 1.0}, c[4] = {0.5, -8.0, 0.0, 0.0};
    const double sg[4] = {1.0, 1.4, 0.7, 1.0};
    const double c2[4] = {0.0, 0.0, 1.5, 0.0}, c3[4] = {0.0, 0.0, -2.0, 0.0};
    const double s1[4] = {0.0, 0.2, 0.0, 0.0}, s2[4] = {0.0, 0.0, 0.1, 0.0};
    const int32_t off[5] = {0, 5, 6, 7, 8};
    const int32_t se[8] = {0, 1, 2, 3, 3, 0, 1, 2};
    const uint8_t so[8] = {0, 0, 0, 0, 1, 1, 1, 1};
    const double b[8] = {0.3, 0.2, 0.0, 0.25, 0.25, 1.0, 1.0, 1.0};
    const uint8_t kind[4] = {0, 0, 1, 2};
    const double span[4] = {1.0, 0.5, 0.8, 0.3};
    or_graph g = {4, 4, ei, et, L, a, c, sg, off, se, so, b, kind, span,
                  c2, c3, s1, s2, NULL};
    rc |= run_graph(&g, 300, 1, 0, 3, 5e-3, 400);
    rc |= run_graph(&g, 300, 2, 0, 8, 1e-2, 250);
  }
  /* the paper's semi-infinite star: three edges [0, inf) whose terminal
     vertices are vertices at infinity */
  {
    const int32_t ei[3] = {0, 0, 0}, et[3] = {1, 2, 3};
    const double L[3] = {INFINITY, INFINITY, INFINITY};
    const double a[3] = {0.0, 0.0, 0.0}, c[3] = {-10.0, -20.0, -30.0};
    const double sg[3] = {1.0, 1.0, 1.0};
    const int32_t off[5] = {0, 3, 4, 5, 6};
    const int32_t se[6] = {0, 1, 2, 0, 1, 2};
    const uint8_t so[6] = {0, 0, 0, 1, 1, 1};
    const double b[6] = {1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0, 1.0, 1.0};
    const double span[3] = {2.0, 2.0, 2.0};
    or_graph g = {4, 3, ei, et, L, a, c, sg, off, se, so, b, NULL, span,
                  NULL, NULL, NULL, NULL, NULL};
    rc |= run_graph(&g, 200, 1, 0, 8, 1e-3, 300);
  }
  /* sources, thresholds, roots and the generator on their own */
  {
    const int32_t ei[2] = {0, 1}, et[2] = {1, 2};
    const double L[2] = {1.0, 2.0}, a[2] = {0.0, 0.0}, c[2] = {0.0, 0.0}, sg[2] = {1.0, 1.0};
    const int32_t off[4] = {0, 1, 3, 4};
    const int32_t se[4] = {0, 0, 1, 1};
    const uint8_t so[4] = {0, 1, 0, 1};
    const double b[4] = {1.0, 0.5, 0.5, 1.0};
    or_graph g = {3, 2, ei, et, L, a, c, sg, off, se, so, b, NULL, L, NULL, NULL, NULL, NULL,
                  NULL};
    const int32_t sv[3] = {0, 2, 1};
    const double sr[3] = {2.0, 0.0, 1.0};
    uint32_t pid[16];
    int32_t edge[16];
    double x[16];
    uint8_t alive[16];
    uint64_t hash[16];
    uint32_t hits[16];
    for (int i = 0; i < 16; ++i) pid[i] = (uint32_t)i;
    if (or_init_sources(&g, 16, pid, 3, sv, sr, 4, 0, edge, x, alive, hash, hits) != 0)
      rc |= fail("or_init_sources");
    uint64_t thr[4];
    if (or_thresholds(&g, thr) != 0) rc |= fail("or_thresholds");
    const double A[6] = {0.0, 1.0, -1.0, 0.0, 2.0, 1e-300};
    const double Bq[6] = {-1.0, 0.5, 3.0, 0.0, -4.0, -1e300};
    const double Cq[6] = {0.5, 0.0, 1.0, 0.0, 1.0, 1e-300};
    double u[6];
    or_first_root_batch(A, Bq, Cq, 6, u);
    for (int i = 0; i < 6; ++i)
      if (!(u[i] >= 0.0 && u[i] <= 1.0)) rc |= fail("root outside [0, 1]");
    uint32_t ctr[8] = {0, 1, 2, 3, 0xFFFFFFFFu, 0xFFFFFFFFu, 0, 7}, out[8];
    or_philox_batch(ctr, 0x123456789abcdefull, 2, out);
    const uint32_t pp[2] = {1, 2};
    const uint64_t nn[2] = {5, 0xFFFFFFFFull};
    const uint32_t kk[2] = {1, 255};
    double w[2];
    uint32_t r[2];
    or_main_normals(pp, nn, 2, 3, 9, w);
    or_hit_draws(pp, nn, kk, 2, 3, 9, r, w);
  }
  if (rc == 0) printf("oracle_sanitize: ok\n");
  return rc;
}
