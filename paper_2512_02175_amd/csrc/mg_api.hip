// mg_api.hip -- host side of the C ABI declared in include/metricgraph.h:
// graph validation and packing, particle-set memory, launch orchestration
// and readback.  All per-particle work runs in the kernels of
// mg_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/metricgraph.h"
#include "mg_internal.h"

using namespace mg;

namespace {

thread_local std::string g_err;

mg_status fail(mg_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

mg_status hip_fail(hipError_t e, const char *what) {
  return fail(MG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define MG_HIP(call, what)                       \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Slot thresholds (the slot draw): per vertex b is divided by its sum and
// accumulated left to right in FP64 into C_s; T_s = floor(C_s 2^32), and
// T_s = 2^32 from the last slot with b > 0 onward.
void slot_thresholds(int32_t V, const int32_t *off, const double *b,
                     std::vector<uint64_t> &thr) {
  thr.assign((size_t)off[V], 0);
  for (int32_t v = 0; v < V; ++v) {
    const int32_t s0 = off[v], s1 = off[v + 1];
    double total = 0.0;
    int32_t last_pos = -1;
    for (int32_t s = s0; s < s1; ++s) {
      total += b[s];
      if (b[s] > 0.0) last_pos = s;
    }
    double cum = 0.0;
    for (int32_t s = s0; s < s1; ++s) {
      if (last_pos < 0) {
        thr[s] = 0;
        continue;
      }
      cum += b[s] / total;
      if (s >= last_pos) {
        thr[s] = 1ull << 32;
      } else {
        const double t = std::floor(cum * 4294967296.0);
        thr[s] = t >= 4294967296.0 ? (1ull << 32) : (uint64_t)t;
      }
    }
  }
}

bool is_finite(double v) { return std::isfinite(v); }

// Iterations of a wave-pool loop between moves of the 32-bit lane tallies
// into 64-bit block totals (1024) and of the block's u32 LDS counters into
// the set's 64-bit ones (2^20; each such move is a round of device-scope
// atomics, which travel past the XCD's L2), or MG_POOL_DRAIN (1 .. 1024) for
// both, from the environment, read at each launch.  Tests lower it to run
// the moves often; the results are the same at any value.
static uint32_t drain_env() {
  const char *v = std::getenv("MG_POOL_DRAIN");
  if (!v || !*v) return 0;
  char *end = nullptr;
  const unsigned long long x = std::strtoull(v, &end, 10);
  return (end && *end == 0 && x >= 1 && x <= kDrainMax) ? (uint32_t)x : 0;
}
// Particle ids a wave of the pool kernels reserves from a set's counter at
// a time, for launches of nsteps steps over sets of about n_typ and at
// most n_max particles.  Every reservation is one atomic on one address
// (about 10 ns each, one after another), and a wave works through its
// reservation alone: reservations of about 1.2e5 / nsteps ids keep the
// atomics under a tenth of the launch's work (64 ids from 2048 steps on),
// and at most about sqrt(0.43 n_typ) ids (the balance of the atomics
// against one wave's work on a one-step launch) keep a small set's ids
// spread over many waves; 64 <= ids <= 1024, a power of two, and small
// enough that the counter, passed by at most one reservation per resident
// wave, cannot wrap.
uint32_t claim_chunk(uint32_t nsteps, int64_t n_typ, int64_t n_max) {
  const double by_steps = 1.2e5 / (double)std::max<uint32_t>(nsteps, 1u);
  const double by_n = std::sqrt(0.43 * (double)std::max<int64_t>(n_typ, 1));
  const double want = std::min(by_steps, by_n);
  uint32_t r = 64;
  while (r < 1024 && (double)r < want) r *= 2;
  const uint64_t waves = (uint64_t)kMaxPersistBlocks * (kBlock / 64);
  const uint64_t room = (0xFFFFFFFFull - (uint64_t)n_max) / waves;
  const uint32_t cap = (uint32_t)std::min<uint64_t>(room, 1024) & ~15u;
  return std::max<uint32_t>(16u, std::min(r, cap));
}

void set_drain(StepArgs &a) {
  const uint32_t d = drain_env();
  a.drain = d ? d : kDrainMax;
  a.drain_lds = d ? d : kLdsDrainMax;
}
// an optional per-edge coefficient array: its entry, or 0 when absent
double higher(const double *p, int32_t e) { return p ? p[e] : 0.0; }

// s0 + s1 x + s2 x^2 + s3 x^3 > 0 on [0, hi]: its minimum is at an end or at
// a real root of the derivative s1 + 2 s2 x + 3 s3 x^2, found with the
// cancellation-free quadratic formula (q = -(b + sgn(b) sqrt(b^2 - 4ac)) / 2,
// roots q/a and c/q) and refined by one Newton step; the cubic is evaluated
// there in FP64 (a minimum within rounding of zero may pass either way).
bool cubic_positive(double s0, double s1, double s2, double s3, double hi) {
  auto val = [&](double x) { return ((s3 * x + s2) * x + s1) * x + s0; };
  auto der = [&](double x) { return (3.0 * s3 * x + 2.0 * s2) * x + s1; };
  auto newton = [&](double x) {
    const double dd = 6.0 * s3 * x + 2.0 * s2;
    return dd != 0.0 ? x - der(x) / dd : x;
  };
  double crit[4] = {0.0, hi, 0.0, 0.0};
  int nc = 2;
  const double qa = 3.0 * s3, qb = 2.0 * s2, qc = s1;
  if (qa != 0.0) {
    const double disc = qb * qb - 4.0 * qa * qc;
    if (disc >= 0.0) {
      const double q = -0.5 * (qb + std::copysign(std::sqrt(disc), qb));
      if (q != 0.0) {
        crit[nc++] = newton(q / qa);
        crit[nc++] = newton(qc / q);
      } else {
        crit[nc++] = 0.0;  // b = c = 0: a double root at 0
      }
    }
  } else if (qb != 0.0) {
    crit[nc++] = -qc / qb;
  }
  for (int i = 0; i < nc; ++i) {
    const double x = crit[i];
    if (x >= 0.0 && x <= hi && !(val(x) > 0.0)) return false;
  }
  return true;
}

// The cubic in t in [0, 1] that interpolates values p0, p1 and slopes d0, d1
// (per unit length) at the ends of an interval of width h (cubic Hermite),
// in powers of t: c0 + c1 t + c2 t^2 + c3 t^3.
void hermite_power(double p0, double d0, double p1, double d1, double h, double c[4]) {
  c[0] = p0;
  c[1] = h * d0;
  c[2] = 3.0 * (p1 - p0) - h * (2.0 * d0 + d1);
  c[3] = 2.0 * (p0 - p1) + h * (d0 + d1);
}

}  // namespace

struct mg_graph {
  int32_t V, E, nnz;
  // FP32 schedule tuning results per dt, shared by the sets on this graph
  mutable std::mutex tune_mu;
  mutable std::vector<std::pair<double, mg_tuning>> tune_cache;
  std::vector<double> length;  // host copy for readback conversion
  std::vector<double> span;    // length binned by the uniform histograms
  std::vector<int32_t> vinit_host, vterm_host;  // end vertices of each edge
  std::vector<uint8_t> wentzell_host;           // [V] Wentzell vertex
  std::vector<VtxBlk> vtx_host;
  // semi-infinite edges (length +infinity): their terminal vertices are
  // the vertices at infinity, which no particle reaches
  bool infinite = false;
  std::vector<uint8_t> at_infinity;  // [V]
  // some edge has higher coefficients (mu beyond affine or sigma(x) not
  // constant), some vertex is a Wentzell vertex; gen: either (the kernels'
  // general instantiation; FP32 sets run the lane schedule or pools of 128
  // with 8-step windows)
  bool poly = false;
  bool wentzell = false;
  bool gen = false;
  // FNV-1a of the packed device tables: names the graph in the tuning file
  uint64_t fingerprint = 0;
  void *dev = nullptr;         // one allocation holding every table
  GraphDev gd{};
};

struct mg_particles {
  const mg_graph *g = nullptr;
  int32_t schedule = MG_SCHED_AUTO;
  // autotuned choice (schedule AUTO): valid for dt == tuned_dt
  bool tuned = false;
  double tuned_dt = 0.0;
  int32_t tuned_kernel = 1;
  int32_t tuned_idle = 8;
  int32_t tuned_spl = 0;  // steps per launch of the tuned choice (0: whole call)
  int64_t n = 0;
  mg_precision prec = MG_FP64;
  int32_t max_splits = 8;
  uint32_t tag = 0;
  bool trace = false;
  int32_t steps_per_launch = 0;
  hipStream_t stream = nullptr;
  bool owns = false;
  void *mem = nullptr;
  SetDev sd{};
  uint64_t step = 0;
  uint64_t obs_start = 0;  // step counter when the streamed histogram started
  void *ev_mem = nullptr;  // event trace: counter, ids and records
  // histogram kernel choice for large E * nb (timed on the first call)
  mutable int32_t hist_nb = 0;
  mutable bool hist_tiled = false;
};

// Sets of a batch whose LDS needs (exit counters, staged tables) keep the
// same number of blocks resident: one launch per group per chunk, each with
// the LDS plan of its own largest graph, so small graphs do not run at the
// occupancy that the largest graph of the batch leaves.
struct BatchGroup {
  int32_t first = 0, count = 0;  // its items in d_items
  int32_t max_nnz = 0;
  int32_t max_stage = 0;  // staged table bytes, 0: tables read from global memory
};

struct mg_batch {
  std::vector<mg_particles *> sets;
  void *dev = nullptr;  // GraphDev[n] + SetDev[n] + BatchItem[items] + item counters
  GraphDev *d_graphs = nullptr;
  SetDev *d_sets = nullptr;
  BatchItem *d_items = nullptr;
  uint32_t *d_claim = nullptr;  // item counters of the persistent launches, one per group
  int32_t n_items = 0;
  int64_t max_n = 0;   // particles of the largest set
  int64_t mean_n = 0;  // and per set
  std::vector<BatchGroup> groups;
  bool gen = false;       // some set's graph has a general method variant
  int32_t gen_level = 0;  // the highest method-variant level of its graphs
  int32_t kernel = 1;     // step schedule fixed at creation (tile size follows it)
  // Per-call set descriptors go up from pinned memory; the launch chain of a
  // call is a HIP graph of kernel nodes, re-instantiated only when the
  // call's shape (steps, dt, seed, schedule) changes.
  SetDev *h_sets = nullptr;
  hipEvent_t uploaded = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t key_steps = -1;
  double key_dt = 0.0;
  uint64_t key_seed = 0;
  int32_t key_idle = -1;
  uint32_t key_chunk = 0;
  uint32_t key_drain = 0, key_drain_lds = 0;
  bool key_obs = false;
};

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct SetLayout {
  size_t ef, pos, hash, hits, exitc, absorbed, totals, err, work, total;
};

SetLayout set_layout(int32_t V, int32_t nnz, int64_t n, mg_precision prec, bool trace) {
  SetLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  L.ef = take((size_t)n * 4);
  L.pos = take((size_t)n * 8);  // double x, or float2 (y, compensation)
  L.hash = trace ? take((size_t)n * 8) : 0;
  L.hits = trace ? take((size_t)n * 4) : 0;
  L.exitc = take((size_t)std::max(nnz, 1) * 8);
  L.absorbed = take((size_t)std::max(V, 1) * 8);
  L.totals = take(4 * 8);
  L.err = take(4);
  L.work = take(4);
  L.total = off;
  return L;
}

mg_status check_device_error(const mg_particles *p) {
  uint32_t err = 0;
  MG_HIP(hipMemcpyAsync(&err, p->sd.err, 4, hipMemcpyDeviceToHost, p->stream),
         "reading the device error word");
  MG_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
  if (err & kErrEdge) return fail(MG_EDEVICE, "a particle's edge id is out of range");
  if (err & kErrPos) return fail(MG_EDEVICE, "a particle's position is outside its edge");
  return MG_OK;
}

bool is_device_pointer(const void *ptr) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice;
}

// Arguments of the general (CSR) histogram: per-edge bins with strictly
// increasing finite upper boundaries from 0, and an output of at least
// bin_offsets[E] counters.  *nbins receives bin_offsets[E].
mg_status check_csr_bins(const mg_particles *p, const int32_t *bin_offsets,
                         const double *bin_upper, const uint64_t *out, int64_t out_len,
                         int64_t *nbins) {
  if (!p || !bin_offsets || !bin_upper || !out) return fail(MG_EINVAL, "NULL argument");
  const int32_t E = p->g->E;
  if (bin_offsets[0] != 0) return fail(MG_EINVAL, "bin_offsets[0] must be 0");
  for (int32_t e = 0; e < E; ++e) {
    if (bin_offsets[e + 1] <= bin_offsets[e])
      return fail(MG_EINVAL, "edge %d has no bins (offsets must increase)", e);
    double prev = 0.0;
    for (int32_t k = bin_offsets[e]; k < bin_offsets[e + 1]; ++k) {
      if (!is_finite(bin_upper[k]) || !(bin_upper[k] > prev))
        return fail(MG_EINVAL, "bin %d of edge %d: upper boundaries must be finite and "
                    "strictly increasing from 0", k - bin_offsets[e], e);
      prev = bin_upper[k];
    }
  }
  *nbins = bin_offsets[E];
  if (out_len < *nbins)
    return fail(MG_EINVAL, "out_len %lld < bin_offsets[E] = %lld", (long long)out_len,
                (long long)*nbins);
  return MG_OK;
}

}  // namespace

// Tuning results kept across processes: with MG_TUNE_CACHE naming a file,
// mg_autotune reads a result from it before probing and appends the result
// of each probe, one JSON object per line.  A line's key: the GPU's
// architecture name and compute-unit count, the graph's table fingerprint,
// the probed particle count, the split cap, dt (its bits) and the probe
// length.  Lines that do not parse, or have another key, are skipped.
struct TuneKey {
  char arch[64];
  int32_t cus;
  uint64_t graph;
  long long n;
  int32_t max_splits;
  uint64_t dt_bits;
  uint32_t probe_steps;
};

bool tune_key(const mg_particles *p, double dt, uint32_t steps, int64_t n, TuneKey &k) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return false;
  std::memset(&k, 0, sizeof k);
  // the name up to the first character the line format cannot hold
  size_t i = 0;
  for (; i + 1 < sizeof k.arch && prop.gcnArchName[i] && prop.gcnArchName[i] != '"' &&
         prop.gcnArchName[i] != '\\' && (unsigned char)prop.gcnArchName[i] > ' ';
       ++i)
    k.arch[i] = prop.gcnArchName[i];
  k.arch[i] = 0;
  k.cus = prop.multiProcessorCount;
  k.graph = p->g->fingerprint;
  k.n = (long long)n;
  k.max_splits = p->max_splits;
  std::memcpy(&k.dt_bits, &dt, 8);
  k.probe_steps = steps;
  return true;
}

#define MG_TUNE_LINE                                                                   \
  "{\"arch\": \"%63[^\"]\", \"cus\": %d, \"graph\": \"%16llx\", \"n\": %lld, "              \
  "\"max_splits\": %d, \"dt_bits\": \"%16llx\", \"probe_steps\": %u, \"schedule\": %d, "      \
  "\"idle_trigger\": %d, \"pool_size\": %d, \"window\": %d, \"steps_per_launch\": %d}"

bool tune_file_read(const char *path, const TuneKey &k, mg_tuning &res) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (!found && std::fgets(line, sizeof line, f)) {
    TuneKey r{};
    unsigned long long gr = 0, dtb = 0;
    mg_tuning t{};
    const int got = std::sscanf(line, MG_TUNE_LINE, r.arch, &r.cus, &gr, &r.n, &r.max_splits,
                                &dtb, &r.probe_steps, &t.schedule, &t.idle_trigger,
                                &t.pool_size, &t.window, &t.steps_per_launch);
    if (got != 12) continue;
    if (std::strcmp(r.arch, k.arch) != 0 || r.cus != k.cus || gr != k.graph || r.n != k.n ||
        r.max_splits != k.max_splits || dtb != k.dt_bits || r.probe_steps != k.probe_steps)
      continue;
    const bool pools = t.schedule == MG_SCHED_POOLS || t.schedule == MG_SCHED_POOLS256 ||
                       t.schedule == MG_SCHED_POOLS_W8;
    if (!(t.schedule == MG_SCHED_LANES || pools) || t.steps_per_launch < 0) continue;
    if (pools && !(t.idle_trigger >= 1 && t.idle_trigger <= 64)) continue;
    res = t;
    found = true;
  }
  std::fclose(f);
  return found;
}

void tune_file_append(const char *path, const TuneKey &k, const mg_tuning &t) {
  char line[512];
  // the writer's format is the reader's with plain conversions
  const int len = std::snprintf(
      line, sizeof line,
      "{\"arch\": \"%s\", \"cus\": %d, \"graph\": \"%016llx\", \"n\": %lld, "
      "\"max_splits\": %d, \"dt_bits\": \"%016llx\", \"probe_steps\": %u, \"schedule\": %d, "
      "\"idle_trigger\": %d, \"pool_size\": %d, \"window\": %d, \"steps_per_launch\": %d}\n",
      k.arch, k.cus, (unsigned long long)k.graph, k.n, k.max_splits,
      (unsigned long long)k.dt_bits, k.probe_steps, t.schedule, t.idle_trigger, t.pool_size,
      t.window, t.steps_per_launch);
  if (len <= 0 || len >= (int)sizeof line) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fwrite(line, 1, (size_t)len, f);
  std::fclose(f);
}

extern "C" {

const char *mg_last_error(void) { return g_err.c_str(); }

mg_status mg_graph_create(const mg_graph_desc *d, mg_graph **out) {
  g_err.clear();
  if (!out) return fail(MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d) return fail(MG_EINVAL, "desc is NULL");
  const int32_t V = d->n_vertices, E = d->n_edges;
  if (V < 1 || E < 1) return fail(MG_EINVAL, "need at least one vertex and one edge");
  if (E > kMaxEdges) return fail(MG_EINVAL, "too many edges");
  if (V > kMaxVertices) return fail(MG_EINVAL, "too many vertices (at most 2^30 - 1)");
  if (!d->edge_init || !d->edge_term || !d->length || !d->sigma || !d->vtx_offsets ||
      !d->slot_edge || !d->slot_orient || !d->slot_jump_prob)
    return fail(MG_EINVAL, "a required array is NULL");
  const int32_t *off = d->vtx_offsets;
  if (off[0] != 0) return fail(MG_EINVAL, "vtx_offsets[0] must be 0");
  for (int32_t v = 0; v < V; ++v)
    if (off[v + 1] < off[v]) return fail(MG_EINVAL, "vtx_offsets decreases at vertex %d", v);
  const int32_t nnz = off[V];
  if ((int64_t)nnz != 2 * (int64_t)E)
    return fail(MG_EINVAL, "nnz = %d, but every edge needs two slots (2E = %d)", nnz, 2 * E);
  bool poly = false;  // some edge has a higher coefficient
  for (int32_t e = 0; e < E; ++e) {
    if (d->edge_init[e] < 0 || d->edge_init[e] >= V || d->edge_term[e] < 0 ||
        d->edge_term[e] >= V)
      return fail(MG_EINVAL, "edge %d has a vertex out of range", e);
    if (std::isnan(d->length[e]) || !(d->length[e] > 0.0))
      return fail(MG_EINVAL, "edge %d: length must be > 0 (finite, or +infinity)", e);
    if (!is_finite(d->sigma[e]) || !(d->sigma[e] > 0.0))
      return fail(MG_EINVAL, "edge %d: sigma must be finite and > 0", e);
    if (d->drift_a && !is_finite(d->drift_a[e])) return fail(MG_EINVAL, "edge %d: drift_a not finite", e);
    if (d->drift_c && !is_finite(d->drift_c[e])) return fail(MG_EINVAL, "edge %d: drift_c not finite", e);
    if (d->bin_span ? !(is_finite(d->bin_span[e]) && d->bin_span[e] > 0.0)
                    : std::isinf(d->length[e]))
      return fail(MG_EINVAL, "edge %d: bin_span must be finite and > 0 (and given for a "
                  "semi-infinite edge)", e);
    const double hi[5] = {higher(d->drift_c2, e), higher(d->drift_c3, e),
                          higher(d->sigma_c1, e), higher(d->sigma_c2, e),
                          higher(d->sigma_c3, e)};
    bool any = false;
    for (double h : hi) {
      if (!is_finite(h)) return fail(MG_EINVAL, "edge %d: higher coefficient not finite", e);
      any |= h != 0.0;
    }
    if (!any) continue;
    poly = true;
    if (std::isinf(d->length[e]))
      return fail(MG_EINVAL, "edge %d: higher coefficients need a finite edge", e);
    // sigma_e(x) > 0 on [0, L]
    if (!cubic_positive(d->sigma[e], hi[2], hi[3], hi[4], d->length[e]))
      return fail(MG_EINVAL, "edge %d: sigma(x) must be > 0 on [0, L]", e);
  }
  // tabulated coefficients: knot counts, finite values, finite edges, no
  // cubic terms beside a table, and sigma > 0 on every interval
  std::vector<TabRec64> tab64;
  std::vector<TabRec32> tab32;
  std::vector<int32_t> tab0(E, 0), tab_k(E, 0);
  if (d->table_offsets) {
    const int32_t *to = d->table_offsets;
    if (to[0] != 0) return fail(MG_EINVAL, "table_offsets[0] must be 0");
    if (!d->table_mu || !d->table_dmu || !d->table_sigma || !d->table_dsigma)
      return fail(MG_EINVAL, "table_offsets needs table_mu, table_dmu, table_sigma and "
                  "table_dsigma");
    for (int32_t e = 0; e < E; ++e) {
      const int32_t n = to[e + 1] - to[e];
      if (n < 0) return fail(MG_EINVAL, "table_offsets decreases at edge %d", e);
      if (n == 0) continue;
      if (n < 2) return fail(MG_EINVAL, "edge %d: a table needs at least 2 knots", e);
      if (std::isinf(d->length[e]))
        return fail(MG_EINVAL, "edge %d: a table needs a finite edge", e);
      for (const double *hp : {d->drift_c2, d->drift_c3, d->sigma_c1, d->sigma_c2, d->sigma_c3})
        if (higher(hp, e) != 0.0)
          return fail(MG_EINVAL, "edge %d: a table replaces the cubic terms, which must be 0", e);
      const int32_t K = n - 1;
      const double h = d->length[e] / K;
      tab0[e] = (int32_t)tab64.size();
      tab_k[e] = K;
      for (int32_t j = to[e]; j < to[e + 1]; ++j)
        if (!is_finite(d->table_mu[j]) || !is_finite(d->table_dmu[j]) ||
            !is_finite(d->table_sigma[j]) || !is_finite(d->table_dsigma[j]))
          return fail(MG_EINVAL, "edge %d: table values must be finite", e);
      for (int32_t j = 0; j < K; ++j) {
        const int32_t k = to[e] + j;
        TabRec64 r{};
        hermite_power(d->table_mu[k], d->table_dmu[k], d->table_mu[k + 1],
                      d->table_dmu[k + 1], h, r.mu);
        hermite_power(d->table_sigma[k], d->table_dsigma[k], d->table_sigma[k + 1],
                      d->table_dsigma[k + 1], h, r.sg);
        if (!cubic_positive(r.sg[0], r.sg[1], r.sg[2], r.sg[3], 1.0))
          return fail(MG_EINVAL, "edge %d: the tabulated sigma(x) must be > 0 on [0, L]", e);
        TabRec32 r32{};
        for (int i = 0; i < 4; ++i) {
          r32.mu[i] = (float)r.mu[i];
          r32.sg[i] = (float)r.sg[i];
        }
        tab64.push_back(r);
        tab32.push_back(r32);
      }
    }
    poly = poly || !tab64.empty();
  }
  // every edge exactly once at each end with the right orientation
  std::vector<uint8_t> seen((size_t)E * 2, 0);
  for (int32_t v = 0; v < V; ++v) {
    double sum = 0.0;
    bool any_pos = false;
    for (int32_t s = off[v]; s < off[v + 1]; ++s) {
      const int32_t e = d->slot_edge[s];
      const uint8_t o = d->slot_orient[s];
      if (e < 0 || e >= E) return fail(MG_EINVAL, "slot %d: edge out of range", s);
      if (o > 1) return fail(MG_EINVAL, "slot %d: orient must be 0 or 1", s);
      const int32_t end_v = o ? d->edge_term[e] : d->edge_init[e];
      if (end_v != v)
        return fail(MG_EINVAL, "slot %d at vertex %d names edge %d, which does not end there", s, v, e);
      if (seen[(size_t)e * 2 + o]++) return fail(MG_EINVAL, "edge %d end %d listed twice", e, o);
      const double b = d->slot_jump_prob[s];
      if (!is_finite(b) || b < 0.0) return fail(MG_EINVAL, "slot %d: jump probability must be >= 0", s);
      sum += b;
      any_pos |= b > 0.0;
    }
    const bool absorbing = d->vtx_kind && d->vtx_kind[v] == MG_VTX_ABSORBING;
    const bool wz = d->vtx_kind && d->vtx_kind[v] == MG_VTX_WENTZELL;
    if (d->vtx_kind && d->vtx_kind[v] > MG_VTX_WENTZELL)
      return fail(MG_EINVAL, "vertex %d: unknown kind", v);
    if (d->vtx_kind && d->vtx_kind[v] == MG_VTX_MIRROR && off[v + 1] - off[v] != 1)
      return fail(MG_EINVAL, "mirror vertex %d must be a leaf (exactly one slot)", v);
    if (wz) {
      // a_v + sum_e b_ve + c_v = 1 (Sec. 2.2) with a_v, c_v >= 0
      const double a = d->vtx_kill ? d->vtx_kill[v] : 0.0;
      const double c = d->vtx_sticky ? d->vtx_sticky[v] : 0.0;
      if (!is_finite(a) || a < 0.0 || !is_finite(c) || c < 0.0)
        return fail(MG_EINVAL, "Wentzell vertex %d: vtx_kill and vtx_sticky must be finite "
                    "and >= 0", v);
      if (!any_pos)
        return fail(MG_EINVAL, "Wentzell vertex %d has no positive jump probability", v);
      if (std::fabs(a + sum + c - 1.0) > 1e-9)
        return fail(MG_EINVAL, "Wentzell vertex %d: a_v + sum b + c_v = %.17g, not 1", v,
                    a + sum + c);
    } else if (!absorbing) {
      if (!any_pos) return fail(MG_EINVAL, "standard vertex %d has no positive jump probability", v);
      if (std::fabs(sum - 1.0) > 1e-9)
        return fail(MG_EINVAL, "vertex %d: jump probabilities sum to %.17g, not 1", v, sum);
    }
  }
  for (size_t i = 0; i < seen.size(); ++i)
    if (!seen[i]) return fail(MG_EINVAL, "edge %zu end %zu is missing from the slot table", i / 2, i % 2);
  // a semi-infinite edge ends at a vertex at infinity: one that holds only
  // that edge's terminal slot
  std::vector<uint8_t> at_inf(V, 0);
  bool infinite = false;
  for (int32_t e = 0; e < E; ++e) {
    if (!std::isinf(d->length[e])) continue;
    infinite = true;
    const int32_t v = d->edge_term[e];
    if (v == d->edge_init[e] || off[v + 1] - off[v] != 1)
      return fail(MG_EINVAL,
                  "edge %d is semi-infinite: its terminal vertex %d must hold only its own end", e, v);
    at_inf[v] = 1;
  }

  // pack
  std::vector<EdgeRec64> e64(E);
  std::vector<EdgeRec32> e32(E);
  auto end_id = [&](int32_t v) {
    const bool mirror = d->vtx_kind && d->vtx_kind[v] == MG_VTX_MIRROR;
    const bool wz = d->vtx_kind && d->vtx_kind[v] == MG_VTX_WENTZELL;
    return (int32_t)((uint32_t)v | (mirror ? kMirrorEnd : 0u) | (wz ? kWentzellEnd : 0u));
  };
  for (int32_t e = 0; e < E; ++e) {
    const double a = d->drift_a ? d->drift_a[e] : 0.0;
    const double c = d->drift_c ? d->drift_c[e] : 0.0;
    const int32_t vi = end_id(d->edge_init[e]), vt = end_id(d->edge_term[e]);
    e64[e] = {d->length[e], a, c, d->sigma[e], vi, vt,
              d->bin_span ? d->bin_span[e] : d->length[e],
              higher(d->drift_c2, e), higher(d->drift_c3, e), higher(d->sigma_c1, e),
              higher(d->sigma_c2, e), higher(d->sigma_c3, e),
              tab_k[e] ? tab_k[e] / d->length[e] : 0.0, tab0[e], tab_k[e]};
    // (a particle never measures from the far end of a semi-infinite edge)
    const double aL = std::isinf(d->length[e]) ? 0.0 : std::fma(c, d->length[e], a);
    const float scale = (float)(std::isinf(d->length[e]) ? d->bin_span[e] : d->length[e]);
    e32[e] = {(float)d->length[e], (float)a, (float)c, (float)d->sigma[e], (float)aL,
              vi, vt, 1e-6f * scale};
  }
  std::vector<uint64_t> thr(nnz);
  slot_thresholds(V, off, d->slot_jump_prob, thr);
  auto eo_of = [&](int32_t s) {
    return ((uint32_t)d->slot_edge[s] << 1) | (uint32_t)d->slot_orient[s] |
           (thr[s] >= (1ull << 32) ? kSatBit : 0u);
  };
  auto t_of = [&](int32_t s) { return thr[s] >= (1ull << 32) ? 0xFFFFFFFFu : (uint32_t)thr[s]; };
  std::vector<SlotRec8> slots(nnz);
  for (int32_t s = 0; s < nnz; ++s) slots[s] = {t_of(s), eo_of(s)};
  std::vector<VtxBlk> vtx(V);
  std::vector<int32_t> guide;
  for (int32_t v = 0; v < V; ++v) {
    const bool absorbing = d->vtx_kind && d->vtx_kind[v] == MG_VTX_ABSORBING;
    const int32_t first = off[v], deg = off[v + 1] - off[v];
    VtxBlk b{};
    b.first = first;
    b.deg = absorbing ? -1 : deg;
    if (!absorbing && deg <= 3) {
      if (deg > 0) b.eo0 = eo_of(first);
      if (deg > 1) { b.t0 = t_of(first); b.eo1 = eo_of(first + 1); }
      if (deg > 2) { b.t1 = t_of(first + 1); b.eo2 = eo_of(first + 2); }
    } else if (!absorbing) {
      // guide table (Chen & Asau): bucket i of the top bits of the draw
      // holds the first slot whose threshold exceeds the bucket's lowest
      // draw, so the scan from there picks the same slot as a scan from 0.
      int32_t bits = 0;
      while ((1 << bits) < deg) ++bits;
      const uint32_t shift = 32u - (uint32_t)bits;
      b.t0 = (uint32_t)guide.size();
      b.t1 = shift;
      int32_t k = 0;
      for (int64_t i = 0; i < (1ll << bits); ++i) {
        const uint64_t lo = (uint64_t)i << shift;
        while (k < deg - 1 && thr[first + k] <= lo) ++k;
        guide.push_back(k);
      }
    }
    vtx[v] = b;
  }
  // Wentzell table: per such vertex, beta = sum_e b_ve, kappa = a_v / beta,
  // gamma = c_v / beta and sigma_v = sum_e (b_ve / beta) sigma_e(v) over
  // its slots in order, sigma_e(v) the cubic by Horner's rule at the edge's
  // end (x = 0 or L), or on a tabulated edge the table's value at that end
  std::vector<WzRec> wzt;
  for (int32_t v = 0; v < V; ++v) {
    if (!(d->vtx_kind && d->vtx_kind[v] == MG_VTX_WENTZELL)) continue;
    double beta = 0.0, sig = 0.0;
    for (int32_t s = off[v]; s < off[v + 1]; ++s) beta += d->slot_jump_prob[s];
    for (int32_t s = off[v]; s < off[v + 1]; ++s) {
      const int32_t e = d->slot_edge[s];
      const double at = d->slot_orient[s] ? d->length[e] : 0.0;
      const double sv =
          tab_k[e] ? d->table_sigma[d->slot_orient[s] ? d->table_offsets[e + 1] - 1
                                                       : d->table_offsets[e]]
                   : std::fma(std::fma(std::fma(higher(d->sigma_c3, e), at,
                                                higher(d->sigma_c2, e)), at,
                                       higher(d->sigma_c1, e)), at, d->sigma[e]);
      sig += (d->slot_jump_prob[s] / beta) * sv;
    }
    WzRec r{};
    r.kappa = (d->vtx_kill ? d->vtx_kill[v] : 0.0) / beta;
    r.gamma = (d->vtx_sticky ? d->vtx_sticky[v] : 0.0) / beta;
    r.lt_per_sqrt = sig * std::sqrt(2.0 / 3.14159265358979323846264338327950288);
    wzt.push_back(r);
    vtx[v].wz = (uint32_t)wzt.size();
  }
  // length-proportional init thresholds, built like the slot thresholds
  // (unused on graphs with semi-infinite edges)
  std::vector<uint64_t> lthr(E);
  if (!infinite) {
    double total = 0.0;
    for (int32_t e = 0; e < E; ++e) total += d->length[e];
    double cum = 0.0;
    for (int32_t e = 0; e < E; ++e) {
      cum += d->length[e];
      if (e == E - 1) {
        lthr[e] = 1ull << 32;
      } else {
        const double t = std::floor((cum / total) * 4294967296.0);
        lthr[e] = t >= 4294967296.0 ? (1ull << 32) : (uint64_t)t;
      }
    }
  }
  mg_graph *g = new mg_graph();
  g->V = V;
  g->E = E;
  g->nnz = nnz;
  g->length.assign(d->length, d->length + E);
  g->vinit_host.assign(d->edge_init, d->edge_init + E);
  g->vterm_host.assign(d->edge_term, d->edge_term + E);
  g->wentzell_host.assign(V, 0);
  for (int32_t v = 0; v < V; ++v)
    g->wentzell_host[v] = d->vtx_kind && d->vtx_kind[v] == MG_VTX_WENTZELL;
  g->span = d->bin_span ? std::vector<double>(d->bin_span, d->bin_span + E) : g->length;
  g->vtx_host = vtx;
  g->infinite = infinite;
  g->at_infinity = at_inf;
  g->poly = poly;
  g->wentzell = !wzt.empty();
  g->gen = g->poly || g->wentzell;
  g->gd.gen = (g->wentzell || !tab64.empty()) ? kGenFull : (g->poly ? kGenCubic : 0);
  const size_t ng = guide.size();
  const size_t o_vtx = 0;
  const size_t o_sl = align_up(o_vtx + sizeof(VtxBlk) * V, 16);
  const size_t o_gd = align_up(o_sl + sizeof(SlotRec8) * nnz, 16);
  const size_t o_32 = align_up(o_gd + 4 * ng, 16);
  const size_t o_64 = align_up(o_32 + sizeof(EdgeRec32) * E, 16);
  const size_t o_lt = align_up(o_64 + sizeof(EdgeRec64) * E, 256);
  const size_t o_wz = align_up(o_lt + 8 * (size_t)E, 256);
  const size_t o_t64 = align_up(o_wz + sizeof(WzRec) * wzt.size(), 256);
  const size_t o_t32 = align_up(o_t64 + sizeof(TabRec64) * tab64.size(), 256);
  const size_t total = align_up(o_t32 + sizeof(TabRec32) * tab32.size(), 256);
  hipError_t he = hipMalloc(&g->dev, total);
  if (he != hipSuccess) {
    delete g;
    return fail(MG_ENOMEM, "hipMalloc of %zu bytes for the graph: %s", total, hipGetErrorString(he));
  }
  char *base = (char *)g->dev;
  std::vector<char> host(total, 0);
  std::memcpy(host.data() + o_vtx, vtx.data(), sizeof(VtxBlk) * V);
  std::memcpy(host.data() + o_sl, slots.data(), sizeof(SlotRec8) * nnz);
  if (ng) std::memcpy(host.data() + o_gd, guide.data(), 4 * ng);
  std::memcpy(host.data() + o_32, e32.data(), sizeof(EdgeRec32) * E);
  std::memcpy(host.data() + o_64, e64.data(), sizeof(EdgeRec64) * E);
  std::memcpy(host.data() + o_lt, lthr.data(), 8 * (size_t)E);
  if (!wzt.empty()) std::memcpy(host.data() + o_wz, wzt.data(), sizeof(WzRec) * wzt.size());
  if (!tab64.empty()) {
    std::memcpy(host.data() + o_t64, tab64.data(), sizeof(TabRec64) * tab64.size());
    std::memcpy(host.data() + o_t32, tab32.data(), sizeof(TabRec32) * tab32.size());
  }
  he = hipMemcpy(base, host.data(), total, hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    (void)hipFree(g->dev);
    delete g;
    return hip_fail(he, "copying the graph tables");
  }
  {
    uint64_t h = 0xcbf29ce484222325ull;
    for (char c : host) h = (h ^ (uint8_t)c) * 0x100000001b3ull;
    g->fingerprint = h;
  }
  g->gd.tables = base;
  g->gd.vtx = (const VtxBlk *)(base + o_vtx);
  g->gd.slots = (const SlotRec8 *)(base + o_sl);
  g->gd.guide = (const int32_t *)(base + o_gd);
  g->gd.e32 = (const EdgeRec32 *)(base + o_32);
  g->gd.e64 = (const EdgeRec64 *)(base + o_64);
  g->gd.len_thr = (const uint64_t *)(base + o_lt);
  g->gd.wz = wzt.empty() ? nullptr : (const WzRec *)(base + o_wz);
  g->gd.tab64 = tab64.empty() ? nullptr : (const TabRec64 *)(base + o_t64);
  g->gd.tab32 = tab32.empty() ? nullptr : (const TabRec32 *)(base + o_t32);
  g->gd.n_guide = (int32_t)ng;
  g->gd.o_vtx = (int32_t)o_vtx;
  g->gd.o_slots = (int32_t)o_sl;
  g->gd.o_guide = (int32_t)o_gd;
  g->gd.o_e32 = (int32_t)o_32;
  g->gd.o_e64 = (int32_t)o_64;
  const size_t st32 = o_32 + sizeof(EdgeRec32) * E;
  const size_t st64 = o_32 + sizeof(EdgeRec64) * E;
  g->gd.stage_bytes32 = st32 <= (size_t)kLdsStageMax ? (int32_t)st32 : 0;
  g->gd.stage_bytes64 = st64 <= (size_t)kLdsStageMax ? (int32_t)st64 : 0;
  g->gd.V = V;
  g->gd.E = E;
  g->gd.nnz = nnz;
  *out = g;
  return MG_OK;
}

void mg_graph_destroy(mg_graph *g) {
  if (!g) return;
  if (g->dev) (void)hipFree(g->dev);
  delete g;
}

int64_t mg_particles_arena_bytes(const mg_graph *g, int64_t n, const mg_options *opt) {
  if (!g || n < 1) return -1;
  const mg_precision prec = opt ? opt->precision : MG_FP64;
  const bool trace = opt && opt->trace;
  return (int64_t)set_layout(g->V, g->nnz, n, prec, trace).total;
}

// Options of a new set on g (NULL: defaults; opt may point to o), with
// the defaults filled in and refused combinations reported.
static mg_status set_options(const mg_graph *g, const mg_options *opt, mg_options &o) {
  o = opt ? *opt : mg_options{};
  if (o.precision != MG_FP64 && o.precision != MG_FP32) return fail(MG_EINVAL, "unknown precision");
  if (o.max_splits < 0 || o.max_splits > 255)
    return fail(MG_EINVAL, "max_splits must be in [0, 255] (0: default)");
  if (o.max_splits == 0) o.max_splits = 8;
  if (o.steps_per_launch < 0) return fail(MG_EINVAL, "steps_per_launch must be >= 0");
  if (o.schedule < MG_SCHED_AUTO || o.schedule > MG_SCHED_POOLS_W8)
    return fail(MG_EINVAL, "unknown schedule");
  if (g->gen && o.precision == MG_FP32 &&
      (o.schedule == MG_SCHED_POOLS || o.schedule == MG_SCHED_POOLS256))
    return fail(MG_EINVAL, "graphs with higher coefficients or Wentzell vertices run the "
                "FP32 lane schedule or MG_SCHED_POOLS_W8 only");
  if (o.precision == MG_FP64 &&
      (o.schedule == MG_SCHED_POOLS || o.schedule == MG_SCHED_POOLS256))
    return fail(MG_EINVAL, "FP64 sets run MG_SCHED_LANES, MG_SCHED_POOLS_W8 or MG_SCHED_AUTO");
  return MG_OK;
}

// Allocates a set of n particles with options o (checked by set_options),
// or places it in the caller's arena, and clears its counters on the set's
// stream; the particle arrays are left for the caller to fill.
static mg_status alloc_set(const mg_graph *g, int64_t n, const mg_options &o,
                           mg_particles **out) {
  const SetLayout L = set_layout(g->V, g->nnz, n, o.precision, o.trace != 0);
  mg_particles *p = new mg_particles();
  p->g = g;
  p->n = n;
  p->prec = o.precision;
  p->max_splits = o.max_splits;
  p->tag = o.graph_tag;
  p->trace = o.trace != 0;
  p->steps_per_launch = o.steps_per_launch;
  p->schedule = o.schedule;
  p->stream = (hipStream_t)o.hip_stream;
  if (o.arena) {
    if (o.arena_bytes < (int64_t)L.total) {
      delete p;
      return fail(MG_ENOMEM, "arena of %lld bytes is smaller than the %zu needed",
                  (long long)o.arena_bytes, L.total);
    }
    if (((uintptr_t)o.arena) % 256) {
      delete p;
      return fail(MG_EINVAL, "arena must be 256-byte aligned");
    }
    p->mem = o.arena;
  } else {
    hipError_t he = hipMalloc(&p->mem, L.total);
    if (he != hipSuccess) {
      delete p;
      return fail(MG_ENOMEM, "hipMalloc of %zu bytes: %s", L.total, hipGetErrorString(he));
    }
    p->owns = true;
  }
  char *base = (char *)p->mem;
  SetDev &s = p->sd;
  s.ef = (uint32_t *)(base + L.ef);
  s.x64 = o.precision == MG_FP64 ? (double *)(base + L.pos) : nullptr;
  s.y32 = o.precision == MG_FP32 ? (float2 *)(base + L.pos) : nullptr;
  s.seqhash = p->trace ? (uint64_t *)(base + L.hash) : nullptr;
  s.hits = p->trace ? (uint32_t *)(base + L.hits) : nullptr;
  s.exit_cnt = (uint64_t *)(base + L.exitc);
  s.absorbed = (uint64_t *)(base + L.absorbed);
  s.totals = (uint64_t *)(base + L.totals);
  s.err = (uint32_t *)(base + L.err);
  s.work = (uint32_t *)(base + L.work);
  s.n = (uint32_t)n;
  s.n0 = 0;
  s.tag = p->tag;
  // counters start at zero (a kernel-free clear: the region is contiguous)
  hipError_t he = hipMemsetAsync(base + L.exitc, 0, L.total - L.exitc, p->stream);
  if (he != hipSuccess) {
    mg_particles_destroy(p);
    return hip_fail(he, "clearing the counters");
  }
  *out = p;
  return MG_OK;
}

// Mode 3 (internal): injection at source vertices.
static mg_status init_impl(const mg_graph *g, int64_t n, int mode, const int32_t *edge,
                           const double *pos, int32_t vertex, int32_t n_src,
                           const int32_t *src_v, const double *src_rate,
                           uint64_t init_seed, const mg_options *opt, mg_particles **out) {
  if (!out) return fail(MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > kMaxParticles) return fail(MG_EINVAL, "n must be in [1, 2^32 - 2^20]");
  if (!g) return fail(MG_EINVAL, "graph is NULL");
  mg_options o;
  mg_status ost = set_options(g, opt, o);
  if (ost != MG_OK) return ost;
  if (mode == MG_INIT_EXPLICIT) {
    if (!edge || !pos) return fail(MG_EINVAL, "explicit init needs edge and pos");
    for (int64_t i = 0; i < n; ++i) {
      if (edge[i] < 0 || edge[i] >= g->E) return fail(MG_EINVAL, "particle %lld: edge out of range", (long long)i);
      if (!(pos[i] >= 0.0 && pos[i] <= g->length[edge[i]]))
        return fail(MG_EINVAL, "particle %lld: position outside [0, L]", (long long)i);
    }
  } else if (mode == MG_INIT_AT_VERTEX) {
    if (vertex < 0 || vertex >= g->V) return fail(MG_EINVAL, "vertex out of range");
    if (g->vtx_host[vertex].deg <= 0)
      return fail(MG_EINVAL, "vertex %d is absorbing or isolated", vertex);
    if (g->at_infinity[vertex]) return fail(MG_EINVAL, "vertex %d is at infinity", vertex);
  } else if (mode == 3) {
    if (n_src < 1 || !src_v || !src_rate) return fail(MG_EINVAL, "need at least one source");
    double total = 0.0;
    for (int32_t j = 0; j < n_src; ++j) {
      const int32_t v = src_v[j];
      if (v < 0 || v >= g->V) return fail(MG_EINVAL, "source %d: vertex out of range", j);
      if (g->vtx_host[v].deg <= 0)
        return fail(MG_EINVAL, "source %d: vertex %d is absorbing or isolated", j, v);
      if (g->at_infinity[v]) return fail(MG_EINVAL, "source %d: vertex %d is at infinity", j, v);
      if (!is_finite(src_rate[j]) || src_rate[j] < 0.0)
        return fail(MG_EINVAL, "source %d: rate must be finite and >= 0", j);
      total += src_rate[j];
    }
    if (!(total > 0.0)) return fail(MG_EINVAL, "the source rates sum to 0");
  } else if (mode != MG_INIT_UNIFORM_LENGTH) {
    return fail(MG_EINVAL, "unknown init mode");
  } else if (g->infinite) {
    return fail(MG_EINVAL, "uniform-by-length init needs finite edges");
  }
  mg_particles *p = nullptr;
  ost = alloc_set(g, n, o, &p);
  if (ost != MG_OK) return ost;
  SetDev &s = p->sd;
  auto bail = [&](mg_status st) {
    mg_particles_destroy(p);
    return st;
  };
  hipError_t he = hipSuccess;
  int32_t *d_edge = nullptr;
  double *d_pos = nullptr;
  void *tmp = nullptr;
  InitSources src{nullptr, nullptr, 0};
  if (mode == 3) {
    std::vector<uint64_t> thr((size_t)n_src);
    const int32_t off[2] = {0, n_src};
    slot_thresholds(1, off, src_rate, thr);
    he = hipMalloc(&tmp, align_up((size_t)n_src * 8, 256) + (size_t)n_src * 4);
    if (he != hipSuccess)
      return bail(fail(MG_ENOMEM, "staging the sources: %s", hipGetErrorString(he)));
    uint64_t *d_thr = (uint64_t *)tmp;
    int32_t *d_v = (int32_t *)((char *)tmp + align_up((size_t)n_src * 8, 256));
    he = hipMemcpy(d_thr, thr.data(), (size_t)n_src * 8, hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(d_v, src_v, (size_t)n_src * 4, hipMemcpyHostToDevice);
    if (he != hipSuccess) {
      (void)hipFree(tmp);
      return bail(hip_fail(he, "copying the sources"));
    }
    src = InitSources{d_thr, d_v, n_src};
  }
  if (mode == MG_INIT_EXPLICIT) {
    he = hipMalloc(&tmp, (size_t)n * 12 + 256);
    if (he != hipSuccess) return bail(fail(MG_ENOMEM, "staging explicit positions: %s", hipGetErrorString(he)));
    d_pos = (double *)tmp;
    d_edge = (int32_t *)((char *)tmp + align_up((size_t)n * 8, 256));
    he = hipMemcpyAsync(d_pos, pos, (size_t)n * 8, hipMemcpyHostToDevice, p->stream);
    if (he == hipSuccess)
      he = hipMemcpyAsync(d_edge, edge, (size_t)n * 4, hipMemcpyHostToDevice, p->stream);
    if (he != hipSuccess) {
      (void)hipFree(tmp);
      return bail(hip_fail(he, "copying explicit positions"));
    }
  }
  he = launch_init(g->gd, s, (int)mode, vertex, (uint32_t)init_seed,
                   (uint32_t)(init_seed >> 32), d_edge, d_pos, src, o.precision == MG_FP64,
                   p->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(p->stream);
  if (tmp) (void)hipFree(tmp);
  if (he != hipSuccess) return bail(hip_fail(he, "initialising particles"));
  *out = p;
  return MG_OK;
}

mg_status mg_particles_init(const mg_graph *g, int64_t n, mg_init_mode mode,
                            const int32_t *edge, const double *pos, int32_t vertex,
                            uint64_t init_seed, const mg_options *opt,
                            mg_particles **out) {
  g_err.clear();
  if (mode != MG_INIT_EXPLICIT && mode != MG_INIT_AT_VERTEX && mode != MG_INIT_UNIFORM_LENGTH) {
    if (out) *out = nullptr;
    return fail(MG_EINVAL, "unknown init mode");
  }
  return init_impl(g, n, (int)mode, edge, pos, vertex, 0, nullptr, nullptr, init_seed, opt,
                   out);
}

mg_status mg_particles_init_sources(const mg_graph *g, int64_t n, int32_t n_sources,
                                    const int32_t *vertices, const double *rates,
                                    uint64_t init_seed, const mg_options *opt,
                                    mg_particles **out) {
  g_err.clear();
  return init_impl(g, n, 3, nullptr, nullptr, 0, n_sources, vertices, rates, init_seed, opt,
                   out);
}

void mg_particles_destroy(mg_particles *p) {
  if (!p) return;
  // a batch may still run the set on its own stream
  if ((p->owns && p->mem) || p->sd.obs || p->ev_mem) (void)hipDeviceSynchronize();
  if (p->owns && p->mem) (void)hipFree(p->mem);
  if (p->sd.obs) (void)hipFree(p->sd.obs);
  if (p->ev_mem) (void)hipFree(p->ev_mem);
  delete p;
}

int64_t mg_particles_step(const mg_particles *p) { return p ? (int64_t)p->step : -1; }

static mg_status check_steps(const mg_particles *p, int64_t n_steps, double dt) {
  if (n_steps < 0) return fail(MG_EINVAL, "n_steps must be >= 0");
  if (!is_finite(dt) || !(dt > 0.0)) return fail(MG_EINVAL, "dt must be finite and > 0");
  if ((uint64_t)p->step + (uint64_t)n_steps > 0xFFFFFFFFull)
    return fail(MG_EINVAL, "the step counter would reach 2^32");
  return MG_OK;
}

// Step kernel (StepArgs::kernel) of an FP32 schedule: 0 one particle per
// lane, 1 / 2 wave pools of 128 / 256 particles, 3 pools of 128 with
// 8-step windows; and back.
static int32_t kernel_of(int32_t schedule) {
  switch (schedule) {
    case MG_SCHED_LANES: return 0;
    case MG_SCHED_POOLS256: return 2;
    case MG_SCHED_POOLS_W8: return 3;
    default: return 1;
  }
}
static int32_t schedule_of(int32_t kernel) {
  static const int32_t s[4] = {MG_SCHED_LANES, MG_SCHED_POOLS, MG_SCHED_POOLS256,
                               MG_SCHED_POOLS_W8};
  return s[kernel];
}

// FP32 step kernel of a set.  Automatic selection takes the autotuned
// choice, or pools of 128 with 8-step windows until tuned (the fastest
// schedule at the hit rates of config 2, the vascular network and the
// batch of config 4).
static int32_t fp32_kernel(const mg_particles *p) {
  // cubic coefficients: the lane schedule or pools of 128 with 8-step
  // windows (FP64 sets ignore this)
  if (p->g->gen && p->prec == MG_FP32) return p->schedule == MG_SCHED_LANES ? 0 : 3;
  if (p->schedule != MG_SCHED_AUTO) return kernel_of(p->schedule);
  return p->tuned ? p->tuned_kernel : 3;
}

// FP64 step kernel of a set: the lane schedule (MG_SCHED_LANES) or wave
// pools of 128 with 8-step windows (MG_SCHED_POOLS_W8, and the automatic
// choice).
static int32_t fp64_kernel(const mg_particles *p) {
  return p->schedule == MG_SCHED_LANES ? 0 : 3;
}

static int32_t step_kernel(const mg_particles *p) {
  return p->prec == MG_FP64 ? fp64_kernel(p) : fp32_kernel(p);
}

static int32_t pool_idle(const mg_particles *p) {
  return (p->schedule == MG_SCHED_AUTO && p->tuned) ? p->tuned_idle : 16;
}

static uint32_t chunk_steps(int32_t spl) {
  // Steps fused per launch, capped at 2^20: a lane of the lane schedule
  // keeps 32-bit tallies of one particle's launch (at most 2^20 (M + 1)
  // sub-steps, M <= 255), the wave pools' drain bound assumes it, and a
  // launch should not run forever.  Block totals are 64-bit and the pools
  // drain their u32 counters, so no count limits a launch otherwise.
  const uint32_t cap = 1u << 20;
  return spl > 0 ? std::min<uint32_t>((uint32_t)spl, cap) : cap;
}

mg_status mg_simulate(mg_particles *p, int64_t n_steps, double dt, uint64_t seed) {
  g_err.clear();
  if (!p) return fail(MG_EINVAL, "particles is NULL");
  mg_status st = check_steps(p, n_steps, dt);
  if (st != MG_OK) return st;
  if (n_steps > 0 && p->prec == MG_FP32 && p->schedule == MG_SCHED_AUTO &&
      !(p->tuned && p->tuned_dt == dt)) {
    st = mg_autotune(p, dt, seed, 0, nullptr);
    if (st != MG_OK) return st;
    g_err.clear();
  }
  StepArgs a{};
  set_drain(a);
  a.max_splits = p->max_splits;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.dt = dt;
  a.kernel = step_kernel(p);
  a.idle = pool_idle(p);
  // a set without a fixed launch length takes the tuned one
  const uint32_t chunk = chunk_steps(
      (p->steps_per_launch == 0 && p->tuned && p->tuned_dt == dt) ? p->tuned_spl
                                                                    : p->steps_per_launch);
  int64_t left = n_steps;
  while (left > 0) {
    const uint32_t now = (uint32_t)std::min<int64_t>(left, chunk);
    a.nsteps = now;
    a.claim_chunk = claim_chunk(now, p->n, p->n);
    p->sd.n0 = (uint32_t)p->step;
    hipError_t he = launch_step(p->g->gd, p->sd, a, p->prec == MG_FP64, p->trace, p->stream);
    if (he != hipSuccess) return hip_fail(he, "launching the step kernel");
    p->step += now;
    left -= now;
  }
  return MG_OK;
}

mg_status mg_histogram(const mg_particles *p, int32_t bins_per_edge, uint64_t *out,
                       int64_t out_len) {
  g_err.clear();
  if (!p || !out) return fail(MG_EINVAL, "NULL argument");
  if (bins_per_edge < 1) return fail(MG_EINVAL, "bins_per_edge must be >= 1");
  const int64_t need = (int64_t)p->g->E * bins_per_edge;
  if (need > 0x7FFFFFFF) return fail(MG_EINVAL, "E * bins_per_edge too large");
  if (out_len < need) return fail(MG_EINVAL, "out_len %lld < E * bins_per_edge = %lld",
                                  (long long)out_len, (long long)need);
  const bool dev_out = is_device_pointer(out);
  uint64_t *d_out = out;
  if (!dev_out) MG_HIP(hipMalloc(&d_out, (size_t)need * 8), "allocating the histogram");
  const bool fp64 = p->prec == MG_FP64;
  hipError_t he = hipSuccess;
  if (need > kLdsHistMax && bins_per_edge <= kLdsHistMax && p->hist_nb != bins_per_edge) {
    // Too large for one LDS copy: time 64-bit global atomics against
    // edge-range LDS tiles once for this bin count and keep the faster.
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    for (hipEvent_t &e : ev)
      if (he == hipSuccess) he = hipEventCreate(&e);
    float t_glob = 0.0f, t_tile = 0.0f;
    if (he == hipSuccess) he = hipMemsetAsync(d_out, 0, (size_t)need * 8, p->stream);
    if (he == hipSuccess) he = hipEventRecord(ev[0], p->stream);
    if (he == hipSuccess)
      he = launch_histogram(p->g->gd, p->sd, bins_per_edge, d_out, fp64, false, p->stream);
    if (he == hipSuccess) he = hipEventRecord(ev[1], p->stream);
    if (he == hipSuccess) he = hipMemsetAsync(d_out, 0, (size_t)need * 8, p->stream);
    if (he == hipSuccess) he = hipEventRecord(ev[2], p->stream);
    if (he == hipSuccess)
      he = launch_histogram(p->g->gd, p->sd, bins_per_edge, d_out, fp64, true, p->stream);
    if (he == hipSuccess) he = hipEventRecord(ev[3], p->stream);
    if (he == hipSuccess) he = hipEventSynchronize(ev[3]);
    if (he == hipSuccess) he = hipEventElapsedTime(&t_glob, ev[0], ev[1]);
    if (he == hipSuccess) he = hipEventElapsedTime(&t_tile, ev[2], ev[3]);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (he == hipSuccess) {
      p->hist_nb = bins_per_edge;
      p->hist_tiled = t_tile < t_glob;
    }
  } else {
    he = hipMemsetAsync(d_out, 0, (size_t)need * 8, p->stream);
    if (he == hipSuccess)
      he = launch_histogram(p->g->gd, p->sd, bins_per_edge, d_out, fp64,
                            p->hist_nb == bins_per_edge && p->hist_tiled, p->stream);
  }
  if (he == hipSuccess && !dev_out)
    he = hipMemcpyAsync(out, d_out, (size_t)need * 8, hipMemcpyDeviceToHost, p->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(p->stream);
  if (!dev_out) (void)hipFree(d_out);
  if (he != hipSuccess) return hip_fail(he, "computing the histogram");
  return check_device_error(p);
}

mg_status mg_histogram_csr(const mg_particles *p, const int32_t *bin_offsets,
                           const double *bin_upper, uint64_t *out, int64_t out_len) {
  g_err.clear();
  int64_t nbins = 0;
  const mg_status vs = check_csr_bins(p, bin_offsets, bin_upper, out, out_len, &nbins);
  if (vs != MG_OK) return vs;
  const int32_t E = p->g->E;
  const bool dev_out = is_device_pointer(out);
  const size_t o_off = 0, o_up = align_up(sizeof(int32_t) * (E + 1), 256),
               o_out = align_up(o_up + sizeof(double) * nbins, 256),
               total = o_out + (dev_out ? 0 : sizeof(uint64_t) * nbins);
  char *mem = nullptr;
  MG_HIP(hipMalloc(&mem, total), "allocating the bin tables");
  int32_t *d_off = (int32_t *)(mem + o_off);
  double *d_up = (double *)(mem + o_up);
  uint64_t *d_out = dev_out ? out : (uint64_t *)(mem + o_out);
  hipError_t he = hipMemcpyAsync(d_off, bin_offsets, sizeof(int32_t) * (E + 1),
                                 hipMemcpyHostToDevice, p->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(d_up, bin_upper, sizeof(double) * nbins, hipMemcpyHostToDevice,
                        p->stream);
  if (he == hipSuccess) he = hipMemsetAsync(d_out, 0, sizeof(uint64_t) * nbins, p->stream);
  if (he == hipSuccess)
    he = launch_histogram_csr(p->g->gd, p->sd, d_off, d_up, (int32_t)nbins, d_out,
                              p->prec == MG_FP64, p->stream);
  if (he == hipSuccess && !dev_out)
    he = hipMemcpyAsync(out, d_out, sizeof(uint64_t) * nbins, hipMemcpyDeviceToHost,
                        p->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(p->stream);
  (void)hipFree(mem);
  if (he != hipSuccess) return hip_fail(he, "computing the histogram");
  return check_device_error(p);
}

mg_status mg_histogram_csr_noalloc(const mg_particles *p, const int32_t *bin_offsets,
                                   const double *bin_upper, uint64_t *out,
                                   int64_t out_len) {
  g_err.clear();
  int64_t nbins = 0;
  const mg_status vs = check_csr_bins(p, bin_offsets, bin_upper, out, out_len, &nbins);
  if (vs != MG_OK) return vs;
  const int32_t E = p->g->E;
  const bool dev_out = is_device_pointer(out);
  // the bin tables (and the counters, for a host `out`) in the fixed
  // workspace of the set's device, laid out as mg_histogram_csr lays out
  // its allocation
  const size_t o_off = 0, o_up = align_up(sizeof(int32_t) * ((size_t)E + 1), 256),
               o_out = align_up(o_up + sizeof(double) * (size_t)nbins, 256),
               total = o_out + (dev_out ? 0 : sizeof(uint64_t) * (size_t)nbins);
  if (total > kNoAllocScratchBytes)
    return fail(MG_EINVAL, "the bin tables need %zu bytes of workspace, more than the %zu "
                "of the allocation-free histogram (use mg_histogram_csr)", total,
                kNoAllocScratchBytes);
  hipPointerAttribute_t attr;
  MG_HIP(hipPointerGetAttributes(&attr, p->sd.ef), "finding the set's device");
  char *mem = nullptr;
  MG_HIP(noalloc_scratch(attr.device, &mem), "looking up the workspace address");
  int32_t *d_off = (int32_t *)(mem + o_off);
  double *d_up = (double *)(mem + o_up);
  uint64_t *d_out = dev_out ? out : (uint64_t *)(mem + o_out);
  hipError_t he = hipMemcpyAsync(d_off, bin_offsets, sizeof(int32_t) * ((size_t)E + 1),
                                 hipMemcpyHostToDevice, p->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(d_up, bin_upper, sizeof(double) * (size_t)nbins,
                        hipMemcpyHostToDevice, p->stream);
  if (he == hipSuccess) he = launch_fill_zero_u64(d_out, nbins, p->stream);
  if (he == hipSuccess)
    he = launch_histogram_csr(p->g->gd, p->sd, d_off, d_up, (int32_t)nbins, d_out,
                              p->prec == MG_FP64, p->stream);
  if (he == hipSuccess && !dev_out)
    he = hipMemcpyAsync(out, d_out, sizeof(uint64_t) * (size_t)nbins, hipMemcpyDeviceToHost,
                        p->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(p->stream);
  if (he != hipSuccess) return hip_fail(he, "computing the histogram");
  return check_device_error(p);
}

mg_status mg_observe_histogram(mg_particles *p, int32_t bins_per_edge, int32_t every) {
  g_err.clear();
  if (!p) return fail(MG_EINVAL, "particles is NULL");
  if (every < 0 || every > (1 << 30)) return fail(MG_EINVAL, "every must be in [0, 2^30]");
  if (every > 0) {
    if (bins_per_edge < 1) return fail(MG_EINVAL, "bins_per_edge must be >= 1");
    if ((int64_t)p->g->E * bins_per_edge > 0x7FFFFFFF)
      return fail(MG_EINVAL, "E * bins_per_edge too large");
  }
  // kernels already queued may still add to the old counters, on the
  // set's stream or, in a batch, on the batch's
  MG_HIP(hipDeviceSynchronize(), "synchronising the device");
  if (p->sd.obs) (void)hipFree(p->sd.obs);
  p->sd.obs = nullptr;
  p->sd.obs_nb = 0;
  p->sd.obs_every = 0;
  if (every == 0) return MG_OK;
  const size_t bytes = (size_t)p->g->E * (size_t)bins_per_edge * 8;
  uint64_t *mem = nullptr;
  hipError_t he = hipMalloc(&mem, bytes);
  if (he != hipSuccess)
    return fail(MG_ENOMEM, "hipMalloc for the streamed histogram: %s", hipGetErrorString(he));
  he = hipMemsetAsync(mem, 0, bytes, p->stream);
  if (he != hipSuccess) {
    (void)hipFree(mem);
    return hip_fail(he, "clearing the streamed histogram");
  }
  p->sd.obs = mem;
  p->sd.obs_nb = bins_per_edge;
  p->sd.obs_every = (uint32_t)every;
  p->obs_start = p->step;
  return MG_OK;
}

mg_status mg_observed_histogram(const mg_particles *p, uint64_t *out, int64_t out_len,
                                int64_t *n_snapshots) {
  g_err.clear();
  if (!p) return fail(MG_EINVAL, "particles is NULL");
  if (!p->sd.obs) return fail(MG_ESTATE, "the streamed histogram is off");
  const int64_t need = (int64_t)p->g->E * p->sd.obs_nb;
  if (out) {
    if (out_len < need)
      return fail(MG_EINVAL, "out_len %lld < E * bins_per_edge = %lld", (long long)out_len,
                  (long long)need);
    MG_HIP(hipMemcpyAsync(out, p->sd.obs, (size_t)need * 8, hipMemcpyDefault, p->stream),
           "copying the streamed histogram");
  }
  MG_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
  if (n_snapshots)
    *n_snapshots = (int64_t)(p->step / p->sd.obs_every - p->obs_start / p->sd.obs_every);
  return check_device_error(p);
}

mg_status mg_density_l2(const mg_graph *g, int32_t bins_per_edge, const uint64_t *counts,
                        double mass, const double *ref_density, double *l2) {
  g_err.clear();
  if (!g || !counts || !ref_density || !l2) return fail(MG_EINVAL, "NULL argument");
  if (bins_per_edge < 1) return fail(MG_EINVAL, "bins_per_edge must be >= 1");
  const int64_t nbins = (int64_t)g->E * bins_per_edge;
  if (nbins > 0x7FFFFFFF) return fail(MG_EINVAL, "E * bins_per_edge too large");
  if (!(mass >= 0.0) || !is_finite(mass)) return fail(MG_EINVAL, "mass must be finite, >= 0");
  std::vector<uint64_t> c((size_t)nbins);
  std::vector<double> ref((size_t)nbins);
  if (is_device_pointer(counts))
    MG_HIP(hipMemcpy(c.data(), counts, (size_t)nbins * 8, hipMemcpyDeviceToHost),
           "copying the counts");
  else
    std::memcpy(c.data(), counts, (size_t)nbins * 8);
  if (is_device_pointer(ref_density))
    MG_HIP(hipMemcpy(ref.data(), ref_density, (size_t)nbins * 8, hipMemcpyDeviceToHost),
           "copying the reference density");
  else
    std::memcpy(ref.data(), ref_density, (size_t)nbins * 8);
  double total = mass;
  if (total == 0.0) {
    uint64_t sum = 0;
    for (uint64_t v : c) sum += v;
    total = (double)sum;
  }
  if (!(total > 0.0)) return fail(MG_EINVAL, "the histogram is empty");
  // Neumaier-compensated sum of w (rho_hat - rho_ref)^2 over all bins
  double acc = 0.0, comp = 0.0;
  for (int32_t e = 0; e < g->E; ++e) {
    const double w = g->span[e] / bins_per_edge;
    for (int32_t k = 0; k < bins_per_edge; ++k) {
      const size_t i = (size_t)e * bins_per_edge + k;
      if (!is_finite(ref[i])) return fail(MG_EINVAL, "reference density %zu not finite", i);
      const double d = (double)c[i] / (total * w) - ref[i];
      const double term = w * d * d;
      const double t = acc + term;
      comp += std::fabs(acc) >= std::fabs(term) ? (acc - t) + term : (term - t) + acc;
      acc = t;
    }
  }
  *l2 = std::sqrt(acc + comp);
  return MG_OK;
}

mg_status mg_exit_counts(const mg_particles *p, uint64_t *slot_counts, uint64_t *absorbed,
                         uint64_t *totals) {
  g_err.clear();
  if (!p) return fail(MG_EINVAL, "particles is NULL");
  if (slot_counts)
    MG_HIP(hipMemcpyAsync(slot_counts, p->sd.exit_cnt, (size_t)p->g->nnz * 8,
                          hipMemcpyDefault, p->stream), "copying exit counts");
  if (absorbed)
    MG_HIP(hipMemcpyAsync(absorbed, p->sd.absorbed, (size_t)p->g->V * 8, hipMemcpyDefault,
                          p->stream), "copying absorbed counts");
  if (totals)
    MG_HIP(hipMemcpyAsync(totals, p->sd.totals, 4 * 8, hipMemcpyDefault, p->stream),
           "copying totals");
  MG_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
  return check_device_error(p);
}

mg_status mg_particles_read(const mg_particles *p, int64_t first, int64_t count,
                            int32_t *edge, double *pos, uint8_t *alive, uint64_t *seqhash,
                            uint32_t *hits) {
  g_err.clear();
  if (!p) return fail(MG_EINVAL, "particles is NULL");
  if (first < 0 || count < 0 || first + count > p->n) return fail(MG_EINVAL, "range out of bounds");
  if ((seqhash || hits) && !p->trace) return fail(MG_ESTATE, "the set was created without trace");
  if (count == 0) return MG_OK;
  std::vector<uint32_t> ef(count);
  MG_HIP(hipMemcpyAsync(ef.data(), p->sd.ef + first, (size_t)count * 4, hipMemcpyDeviceToHost,
                        p->stream), "copying states");
  std::vector<double> x64;
  std::vector<float2> y32;
  if (pos) {
    if (p->prec == MG_FP64) {
      x64.resize(count);
      MG_HIP(hipMemcpyAsync(x64.data(), p->sd.x64 + first, (size_t)count * 8,
                            hipMemcpyDeviceToHost, p->stream), "copying positions");
    } else {
      y32.resize(count);
      MG_HIP(hipMemcpyAsync(y32.data(), p->sd.y32 + first, (size_t)count * 8,
                            hipMemcpyDeviceToHost, p->stream), "copying positions");
    }
  }
  if (seqhash)
    MG_HIP(hipMemcpyAsync(seqhash, p->sd.seqhash + first, (size_t)count * 8, hipMemcpyDefault,
                          p->stream), "copying hashes");
  if (hits)
    MG_HIP(hipMemcpyAsync(hits, p->sd.hits + first, (size_t)count * 4, hipMemcpyDefault,
                          p->stream), "copying hit counts");
  MG_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
  for (int64_t i = 0; i < count; ++i) {
    const int32_t e = (int32_t)(ef[i] & kEdgeMask);
    if (edge) edge[i] = e;
    if (alive) alive[i] = (ef[i] & kDeadBit) ? 0 : 1;
    if (pos) {
      if (p->prec == MG_FP64) {
        pos[i] = x64[i];
      } else {
        const double y = (double)y32[i].x + (double)y32[i].y;
        pos[i] = (ef[i] & kSideBit) ? p->g->length[e] - y : y;
      }
    }
  }
  return check_device_error(p);
}

// ----------------------------------------------------- event trace --
mg_status mg_trace_events(mg_particles *p, int32_t n_ids, const int64_t *ids,
                          int64_t capacity) {
  g_err.clear();
  if (!p) return fail(MG_EINVAL, "particles is NULL");
  if (!p->trace) return fail(MG_ESTATE, "the set was created without trace");
  if (n_ids < 0 || n_ids > 4096) return fail(MG_EINVAL, "n_ids must be in [0, 4096]");
  std::vector<uint32_t> sorted;
  if (n_ids > 0) {
    if (!ids) return fail(MG_EINVAL, "ids is NULL");
    if (capacity < 1 || capacity > (1 << 26))
      return fail(MG_EINVAL, "capacity must be in [1, 2^26]");
    sorted.resize((size_t)n_ids);
    for (int32_t i = 0; i < n_ids; ++i) {
      if (ids[i] < 0 || ids[i] >= p->n) return fail(MG_EINVAL, "id %d out of range", i);
      sorted[i] = (uint32_t)ids[i];
    }
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(MG_EINVAL, "ids must be distinct");
  }
  // kernels already queued may still write the old records, on the set's
  // stream or, in a batch, on the batch's
  MG_HIP(hipDeviceSynchronize(), "synchronising the device");
  if (p->ev_mem) (void)hipFree(p->ev_mem);
  p->ev_mem = nullptr;
  p->sd.ev = nullptr;
  p->sd.ev_cnt = nullptr;
  p->sd.ev_ids = nullptr;
  p->sd.ev_nids = 0;
  p->sd.ev_cap = 0;
  if (n_ids == 0) return MG_OK;
  const size_t o_ids = 256, o_ev = align_up(o_ids + (size_t)n_ids * 4, 256);
  const size_t bytes = o_ev + (size_t)capacity * sizeof(mg_event);
  void *mem = nullptr;
  hipError_t he = hipMalloc(&mem, bytes);
  if (he != hipSuccess)
    return fail(MG_ENOMEM, "hipMalloc for the event trace: %s", hipGetErrorString(he));
  char *base = (char *)mem;
  he = hipMemsetAsync(base, 0, 8, p->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(base + o_ids, sorted.data(), (size_t)n_ids * 4, hipMemcpyHostToDevice,
                        p->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(p->stream);
  if (he != hipSuccess) {
    (void)hipFree(mem);
    return hip_fail(he, "setting up the event trace");
  }
  p->ev_mem = mem;
  p->sd.ev_cnt = (unsigned long long *)base;
  p->sd.ev_ids = (const uint32_t *)(base + o_ids);
  p->sd.ev = (mg_event *)(base + o_ev);
  p->sd.ev_nids = n_ids;
  p->sd.ev_cap = (uint32_t)capacity;
  return MG_OK;
}

mg_status mg_trace_read(const mg_particles *p, mg_event *out, int64_t out_len,
                        int64_t *n_events) {
  g_err.clear();
  if (!p || !n_events) return fail(MG_EINVAL, "NULL argument");
  if (!p->ev_mem) return fail(MG_ESTATE, "the event trace is off");
  if (out_len < 0 || (out_len > 0 && !out)) return fail(MG_EINVAL, "bad output buffer");
  unsigned long long cnt = 0;
  MG_HIP(hipMemcpyAsync(&cnt, p->sd.ev_cnt, 8, hipMemcpyDeviceToHost, p->stream),
         "reading the event count");
  MG_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
  const int64_t kept = (int64_t)std::min<unsigned long long>(cnt, p->sd.ev_cap);
  const int64_t copy = std::min<int64_t>(kept, out_len);
  if (copy > 0) {
    MG_HIP(hipMemcpyAsync(out, p->sd.ev, (size_t)copy * sizeof(mg_event), hipMemcpyDefault,
                          p->stream), "copying the events");
    MG_HIP(hipStreamSynchronize(p->stream), "synchronising the stream");
  }
  *n_events = (int64_t)cnt;
  return check_device_error(p);
}

// ------------------------------------------------------ checkpoints --
// Image of a particle set: mg_image_header, then the sections of
// ckpt_layout at 8-byte aligned offsets, all in the host's byte order.
namespace {

constexpr char kCkptMagic[8] = {'M', 'G', 'S', 'E', 'T', 'I', 'M', 'G'};
constexpr uint32_t kCkptVersion = 1;
static_assert(sizeof(mg_image_header) == 96, "image header layout");
static_assert(sizeof(mg_event) == 40, "event record layout");

struct CkptLayout {
  size_t ef, pos, hash, hits, exitc, absorbed, totals, obs, total;
};

CkptLayout ckpt_layout(int64_t n, int32_t V, int32_t E, int32_t nnz, bool trace,
                       int32_t obs_nb) {
  CkptLayout L{};
  size_t off = sizeof(mg_image_header);
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 8);
    return o;
  };
  L.ef = take((size_t)n * 4);
  L.pos = take((size_t)n * 8);
  L.hash = trace ? take((size_t)n * 8) : 0;
  L.hits = trace ? take((size_t)n * 4) : 0;
  L.exitc = take((size_t)nnz * 8);
  L.absorbed = take((size_t)V * 8);
  L.totals = take(4 * 8);
  L.obs = obs_nb ? take((size_t)E * (size_t)obs_nb * 8) : 0;
  L.total = off;
  return L;
}

CkptLayout ckpt_layout_of(const mg_particles *p) {
  return ckpt_layout(p->n, p->g->V, p->g->E, p->g->nnz, p->trace,
                     p->sd.obs ? p->sd.obs_nb : 0);
}

// A particle state of an image the kernels accept: an edge of the graph,
// the FP32 reference-end flag only in FP32 images, and (alive particles) a
// finite position on the edge, or owing a stay on a Wentzell end (at or
// beyond that end).  The position tests are the step kernels' own.
mg_status check_image_particles(const mg_graph *g, const mg_image_header &h, const char *img,
                                const CkptLayout &L) {
  const bool fp64 = h.precision == MG_FP64;
  auto wz_end = [&](int32_t e, bool term) {
    const int32_t v = term ? g->vterm_host[e] : g->vinit_host[e];
    return g->wentzell_host[v] != 0;
  };
  for (int64_t i = 0; i < h.n; ++i) {
    uint32_t ef;
    std::memcpy(&ef, img + L.ef + (size_t)i * 4, 4);
    const int32_t e = (int32_t)(ef & kEdgeMask);
    if (e >= g->E) return fail(MG_EINVAL, "image particle %lld: edge out of range", (long long)i);
    if (fp64 && (ef & kSideBit))
      return fail(MG_EINVAL, "image particle %lld: FP32 reference-end flag in an FP64 image",
                  (long long)i);
    if (ef & kDeadBit) continue;
    const double Le = g->length[e];
    bool ok;
    if (fp64) {
      double x;
      std::memcpy(&x, img + L.pos + (size_t)i * 8, 8);
      ok = std::isfinite(x) && ((x >= 0.0 && x <= Le) || (x <= 0.0 && wz_end(e, false)) ||
                                (x >= Le && wz_end(e, true)));
    } else {
      float y[2];
      std::memcpy(y, img + L.pos + (size_t)i * 8, 8);
      ok = std::isfinite(y[0]) && std::isfinite(y[1]) &&
           ((y[0] >= 0.0f && y[0] <= (float)Le) ||
            (y[0] < 0.0f && wz_end(e, (ef & kSideBit) != 0)));
    }
    if (!ok)
      return fail(MG_EINVAL, "image particle %lld: position outside its edge", (long long)i);
  }
  return MG_OK;
}

}  // namespace

int64_t mg_particles_image_bytes(const mg_particles *p) {
  if (!p) return -1;
  return (int64_t)ckpt_layout_of(p).total;
}

mg_status mg_particles_save(const mg_particles *p, void *image, int64_t image_bytes) {
  g_err.clear();
  if (!p || !image) return fail(MG_EINVAL, "NULL argument");
  const CkptLayout L = ckpt_layout_of(p);
  if (image_bytes < (int64_t)L.total)
    return fail(MG_EINVAL, "image_bytes %lld < %zu", (long long)image_bytes, L.total);
  if (is_device_pointer(image)) return fail(MG_EINVAL, "the image must be in host memory");
  // waits for every queued step; a set whose error word is set has no
  // state worth keeping
  mg_status st = check_device_error(p);
  if (st != MG_OK) return st;
  char *img = (char *)image;
  const SetDev &s = p->sd;
  const size_t n = (size_t)p->n;
  auto get = [&](size_t off, const void *src, size_t bytes) {
    return hipMemcpyAsync(img + off, src, bytes, hipMemcpyDeviceToHost, p->stream);
  };
  hipError_t he = get(L.ef, s.ef, n * 4);
  if (he == hipSuccess)
    he = get(L.pos, p->prec == MG_FP64 ? (const void *)s.x64 : (const void *)s.y32, n * 8);
  if (he == hipSuccess && p->trace) he = get(L.hash, s.seqhash, n * 8);
  if (he == hipSuccess && p->trace) he = get(L.hits, s.hits, n * 4);
  if (he == hipSuccess) he = get(L.exitc, s.exit_cnt, (size_t)p->g->nnz * 8);
  if (he == hipSuccess) he = get(L.absorbed, s.absorbed, (size_t)p->g->V * 8);
  if (he == hipSuccess) he = get(L.totals, s.totals, 4 * 8);
  if (he == hipSuccess && s.obs) he = get(L.obs, s.obs, (size_t)p->g->E * s.obs_nb * 8);
  if (he == hipSuccess) he = hipStreamSynchronize(p->stream);
  if (he != hipSuccess) return hip_fail(he, "copying the set's state");
  // the bytes between sections are zero, so equal states give equal images
  // (only the u32 sections can end off the 8-byte grid)
  auto pad = [&](size_t end) { std::memset(img + end, 0, align_up(end, 8) - end); };
  pad(L.ef + n * 4);
  if (p->trace) pad(L.hits + n * 4);
  mg_image_header h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = kCkptVersion;
  h.header_bytes = sizeof(mg_image_header);
  h.total_bytes = L.total;
  h.graph = p->g->fingerprint;
  h.n = p->n;
  h.n_vertices = p->g->V;
  h.n_edges = p->g->E;
  h.nnz = p->g->nnz;
  h.precision = p->prec;
  h.max_splits = p->max_splits;
  h.graph_tag = p->tag;
  h.trace = p->trace ? 1 : 0;
  h.obs_bins = s.obs ? s.obs_nb : 0;
  h.obs_every = s.obs ? s.obs_every : 0;
  h.obs_start = s.obs ? p->obs_start : 0;
  h.step = p->step;
  std::memcpy(img, &h, sizeof h);
  return MG_OK;
}

mg_status mg_particles_load(const mg_graph *g, const void *image, int64_t image_bytes,
                            const mg_options *opt, mg_particles **out) {
  g_err.clear();
  if (!out) return fail(MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!g || !image) return fail(MG_EINVAL, "NULL argument");
  if (image_bytes < (int64_t)sizeof(mg_image_header))
    return fail(MG_EINVAL, "image of %lld bytes is shorter than its header",
                (long long)image_bytes);
  if (is_device_pointer(image)) return fail(MG_EINVAL, "the image must be in host memory");
  const char *img = (const char *)image;
  mg_image_header h;
  std::memcpy(&h, img, sizeof h);
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0)
    return fail(MG_EINVAL, "not a particle-set image");
  if (h.version != kCkptVersion || h.header_bytes != sizeof(mg_image_header))
    return fail(MG_EINVAL, "image version %u is not %u", h.version, kCkptVersion);
  if (h.graph != g->fingerprint || h.n_vertices != g->V || h.n_edges != g->E ||
      h.nnz != g->nnz)
    return fail(MG_EINVAL, "the image was saved on another graph");
  if (h.n < 1 || h.n > kMaxParticles) return fail(MG_EINVAL, "image particle count out of range");
  if ((h.precision != MG_FP64 && h.precision != MG_FP32) || h.max_splits < 1 ||
      h.max_splits > 255 || (h.trace != 0 && h.trace != 1) || h.step > 0xFFFFFFFFull)
    return fail(MG_EINVAL, "image header out of range");
  if (h.obs_every == 0 ? (h.obs_bins != 0 || h.obs_start != 0)
                       : (h.obs_every > (1u << 30) || h.obs_bins < 1 ||
                          (int64_t)g->E * h.obs_bins > 0x7FFFFFFF || h.obs_start > h.step))
    return fail(MG_EINVAL, "image streamed-histogram fields out of range");
  const CkptLayout L =
      ckpt_layout(h.n, h.n_vertices, h.n_edges, h.nnz, h.trace != 0, h.obs_bins);
  if (h.total_bytes != L.total || image_bytes < (int64_t)L.total)
    return fail(MG_EINVAL, "image of %lld bytes, %zu expected", (long long)image_bytes, L.total);
  mg_status st = check_image_particles(g, h, img, L);
  if (st != MG_OK) return st;
  // the image fixes what the sample paths depend on; opt gives the rest
  mg_options o = opt ? *opt : mg_options{};
  o.precision = (mg_precision)h.precision;
  o.max_splits = h.max_splits;
  o.graph_tag = h.graph_tag;
  o.trace = h.trace;
  st = set_options(g, &o, o);
  if (st != MG_OK) return st;
  mg_particles *p = nullptr;
  st = alloc_set(g, h.n, o, &p);
  if (st != MG_OK) return st;
  const SetDev &s = p->sd;
  const size_t n = (size_t)h.n;
  auto put = [&](void *dst, size_t off, size_t bytes) {
    return hipMemcpyAsync(dst, img + off, bytes, hipMemcpyHostToDevice, p->stream);
  };
  hipError_t he = put(s.ef, L.ef, n * 4);
  if (he == hipSuccess)
    he = put(p->prec == MG_FP64 ? (void *)s.x64 : (void *)s.y32, L.pos, n * 8);
  if (he == hipSuccess && p->trace) he = put(s.seqhash, L.hash, n * 8);
  if (he == hipSuccess && p->trace) he = put(s.hits, L.hits, n * 4);
  if (he == hipSuccess) he = put(s.exit_cnt, L.exitc, (size_t)h.nnz * 8);
  if (he == hipSuccess) he = put(s.absorbed, L.absorbed, (size_t)h.n_vertices * 8);
  if (he == hipSuccess) he = put(s.totals, L.totals, 4 * 8);
  if (he == hipSuccess) he = hipStreamSynchronize(p->stream);
  if (he != hipSuccess) {
    mg_particles_destroy(p);
    return hip_fail(he, "copying the image's state");
  }
  p->step = h.step;
  if (h.obs_every) {
    st = mg_observe_histogram(p, h.obs_bins, (int32_t)h.obs_every);
    if (st == MG_OK) {
      he = put(p->sd.obs, L.obs, (size_t)h.n_edges * h.obs_bins * 8);
      if (he == hipSuccess) he = hipStreamSynchronize(p->stream);
      if (he != hipSuccess) st = hip_fail(he, "copying the streamed histogram");
    }
    if (st != MG_OK) {
      mg_particles_destroy(p);
      return st;
    }
    p->obs_start = h.obs_start;
  }
  *out = p;
  return MG_OK;
}

mg_status mg_batch_create(int32_t n_sets, mg_particles *const *sets, mg_batch **out) {
  g_err.clear();
  if (!out) return fail(MG_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_sets < 1 || !sets) return fail(MG_EINVAL, "need at least one set");
  for (int32_t i = 0; i < n_sets; ++i) {
    if (!sets[i]) return fail(MG_EINVAL, "set %d is NULL", i);
    if (sets[i]->prec != sets[0]->prec) return fail(MG_EINVAL, "sets differ in precision");
    if (sets[i]->max_splits != sets[0]->max_splits) return fail(MG_EINVAL, "sets differ in max_splits");
    if (sets[i]->trace != sets[0]->trace) return fail(MG_EINVAL, "sets differ in trace");
    if (step_kernel(sets[i]) != step_kernel(sets[0]))
      return fail(MG_EINVAL, "sets differ in schedule");
    // the FP32 general step (cubic coefficients, Wentzell vertices)
    // evaluates the coefficients at the position, the affine one uses
    // per-frame constants: one launch cannot give both sets their own bits
    if (sets[0]->prec == MG_FP32 && sets[i]->g->gen != sets[0]->g->gen)
      return fail(MG_EINVAL, "FP32 sets differ in coefficient form (general variants: cubic "
                  "coefficients or Wentzell vertices, and affine)");
    for (int32_t j = 0; j < i; ++j)
      if (sets[j] == sets[i]) return fail(MG_EINVAL, "set %d appears twice", i);
  }
  mg_batch *b = new mg_batch();
  b->sets.assign(sets, sets + n_sets);
  b->kernel = step_kernel(sets[0]);
  const bool fp64 = sets[0]->prec == MG_FP64;
  const bool trace = sets[0]->trace;
  for (int32_t i = 0; i < n_sets; ++i) {
    b->gen = b->gen || sets[i]->g->gen;
    b->gen_level = std::max(b->gen_level, sets[i]->g->gd.gen);
    b->max_n = std::max(b->max_n, sets[i]->n);
    b->mean_n += sets[i]->n;
  }
  b->mean_n /= n_sets;
  // Group the sets by the blocks per CU that their exit counters leave
  // resident (the tables are staged within a group only where that costs
  // no occupancy), and apart from sets whose graphs have too many exit
  // slots for LDS (a group counts exits in LDS only if all of its graphs
  // can); a group with under 1/32 of the particles joins the next group of
  // larger LDS need with the same exit counting, whose plan covers it.
  StepArgs qa{};
  qa.kernel = b->kernel;
  std::vector<std::pair<int32_t, int32_t>> key(n_sets);  // (global exits, -occupancy)
  int64_t total_n = 0;
  for (int32_t i = 0; i < n_sets; ++i) {
    const int32_t nnz = sets[i]->g->nnz;
    key[i] = {nnz > kLdsExitMax ? 1 : 0,
              -batch_blocks_per_cu(nnz, 0, qa, fp64, trace, b->gen_level, nullptr)};
    total_n += sets[i]->n;
  }
  std::vector<std::pair<int32_t, int32_t>> classes(key);
  std::sort(classes.begin(), classes.end());
  classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
  std::vector<std::vector<int32_t>> members(classes.size());
  for (int32_t i = 0; i < n_sets; ++i)
    members[std::lower_bound(classes.begin(), classes.end(), key[i]) - classes.begin()]
        .push_back(i);
  for (size_t c = 0; c + 1 < members.size(); ++c) {
    if (classes[c + 1].first != classes[c].first) continue;
    int64_t nc = 0;
    for (int32_t i : members[c]) nc += sets[i]->n;
    if (nc * 32 < total_n) {
      members[c + 1].insert(members[c + 1].end(), members[c].begin(), members[c].end());
      members[c].clear();
    }
  }
  std::vector<BatchItem> items;
  const int32_t tile = batch_tile(fp64, b->kernel);
  for (const std::vector<int32_t> &mem : members) {
    if (mem.empty()) continue;
    BatchGroup grp;
    grp.first = (int32_t)items.size();
    bool all_stage = true;
    int32_t max_stage = 0;
    for (int32_t i : mem) {
      for (int64_t f = 0; f < sets[i]->n; f += tile) items.push_back({i, (uint32_t)f});
      grp.max_nnz = std::max(grp.max_nnz, sets[i]->g->nnz);
      const GraphDev &gd = sets[i]->g->gd;
      const int32_t st = fp64 ? gd.stage_bytes64 : gd.stage_bytes32;
      all_stage = all_stage && st > 0;
      max_stage = std::max(max_stage, st);
    }
    if (all_stage && max_stage > 0) {
      bool staged = false;
      const int32_t with = batch_blocks_per_cu(grp.max_nnz, max_stage, qa, fp64, trace,
                                               b->gen_level, &staged);
      const int32_t without =
          batch_blocks_per_cu(grp.max_nnz, 0, qa, fp64, trace, b->gen_level, nullptr);
      if (staged && with >= without) grp.max_stage = max_stage;
    }
    grp.count = (int32_t)items.size() - grp.first;
    // largest sets first, so that each launch ends with small tiles
    std::stable_sort(items.begin() + grp.first, items.end(),
                     [&](const BatchItem &x, const BatchItem &y) {
                       return sets[x.set]->n > sets[y.set]->n;
                     });
    b->groups.push_back(grp);
  }
  b->n_items = (int32_t)items.size();
  const size_t og = 0;
  const size_t os = align_up(sizeof(GraphDev) * n_sets, 256);
  const size_t oi = align_up(os + sizeof(SetDev) * n_sets, 256);
  const size_t oc = align_up(oi + sizeof(BatchItem) * items.size(), 256);
  const size_t total = oc + align_up(sizeof(uint32_t) * b->groups.size(), 256);
  hipError_t he = hipMalloc(&b->dev, total);
  if (he != hipSuccess) {
    delete b;
    return fail(MG_ENOMEM, "hipMalloc for the batch tables: %s", hipGetErrorString(he));
  }
  b->d_graphs = (GraphDev *)((char *)b->dev + og);
  b->d_sets = (SetDev *)((char *)b->dev + os);
  b->d_items = (BatchItem *)((char *)b->dev + oi);
  b->d_claim = (uint32_t *)((char *)b->dev + oc);
  std::vector<GraphDev> gds(n_sets);
  for (int32_t i = 0; i < n_sets; ++i) gds[i] = sets[i]->g->gd;
  he = hipMemcpy(b->d_graphs, gds.data(), sizeof(GraphDev) * n_sets, hipMemcpyHostToDevice);
  if (he == hipSuccess)
    he = hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(),
                   hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipHostMalloc((void **)&b->h_sets, sizeof(SetDev) * n_sets, 0);
  if (he == hipSuccess) he = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
  if (he == hipSuccess) he = hipEventRecord(b->uploaded, sets[0]->stream);
  if (he != hipSuccess) {
    mg_batch_destroy(b);
    return hip_fail(he, "setting up the batch");
  }
  *out = b;
  return MG_OK;
}

static void drop_graph(mg_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->key_steps = -1;
}

// Kernel nodes of one call: per chunk of steps, one launch per group (each
// persistent launch after a node that clears its counters), all chained.
static hipError_t add_group_launch(mg_batch *b, size_t gi, const StepArgs &a0,
                                   hipGraphNode_t &prev) {
  const BatchGroup &grp = b->groups[gi];
  mg_particles *p0 = b->sets[0];
  StepArgs a = a0;
  a.batch_items = (uint32_t)grp.count;
  a.batch_claim = b->d_claim + gi;
  const KernelLaunch k = batch_launch(grp.count, grp.max_nnz, grp.max_stage, a,
                                      p0->prec == MG_FP64, p0->trace, b->key_obs, b->gen_level);
  const GraphDev *g = b->d_graphs;
  const SetDev *sd = b->d_sets;
  const BatchItem *it = b->d_items + grp.first;
  hipError_t he = hipSuccess;
  if (k.persistent) {
    // the sets' particle counters and the group's item counter start at
    // zero (no other group's launch runs meanwhile: the nodes are chained)
    int32_t n_sets = (int32_t)b->sets.size();
    uint32_t *claim = a.batch_claim;
    void *rargs[] = {(void *)&sd, (void *)&n_sets, (void *)&claim};
    hipKernelNodeParams rp{};
    rp.func = (void *)batch_reset_kernel();
    rp.gridDim = dim3((unsigned)((n_sets + 255) / 256));
    rp.blockDim = dim3(256);
    rp.sharedMemBytes = 0;
    rp.kernelParams = rargs;
    rp.extra = nullptr;
    hipGraphNode_t rnode;
    he = hipGraphAddKernelNode(&rnode, b->graph, prev ? &prev : nullptr, prev ? 1 : 0, &rp);
    if (he != hipSuccess) return he;
    prev = rnode;
  }
  void *args[] = {(void *)&g, (void *)&sd, (void *)&it, (void *)&a};
  hipKernelNodeParams np{};
  np.func = (void *)k.func;
  np.gridDim = k.grid;
  np.blockDim = k.block;
  np.sharedMemBytes = (unsigned)k.shm;
  np.kernelParams = args;
  np.extra = nullptr;
  hipGraphNode_t node;
  he = hipGraphAddKernelNode(&node, b->graph, prev ? &prev : nullptr, prev ? 1 : 0, &np);
  if (he == hipSuccess) prev = node;
  return he;
}

static hipError_t build_graph(mg_batch *b, int64_t n_steps, const StepArgs &base,
                              uint32_t chunk) {
  hipError_t he = hipGraphCreate(&b->graph, 0);
  if (he != hipSuccess) return he;
  hipGraphNode_t prev = nullptr;
  uint32_t done = 0;
  int64_t left = n_steps;
  while (left > 0 && he == hipSuccess) {
    StepArgs a = base;
    a.nsteps = (uint32_t)std::min<int64_t>(left, chunk);
    a.claim_chunk = claim_chunk(a.nsteps, b->mean_n, b->max_n);
    a.n0_offset = done;
    for (size_t gi = 0; gi < b->groups.size() && he == hipSuccess; ++gi)
      he = add_group_launch(b, gi, a, prev);
    done += a.nsteps;
    left -= a.nsteps;
  }
  if (he == hipSuccess) he = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  return he;
}

mg_status mg_batch_simulate(mg_batch *b, int64_t n_steps, double dt, uint64_t seed) {
  g_err.clear();
  if (!b) return fail(MG_EINVAL, "batch is NULL");
  for (mg_particles *p : b->sets) {
    mg_status st = check_steps(p, n_steps, dt);
    if (st != MG_OK) return st;
  }
  if (n_steps == 0) return MG_OK;
  mg_particles *p0 = b->sets[0];
  hipStream_t stream = p0->stream;
  StepArgs a{};
  set_drain(a);
  a.max_splits = p0->max_splits;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.dt = dt;
  a.kernel = b->kernel;
  a.idle = pool_idle(p0);
  const uint32_t chunk = chunk_steps(p0->steps_per_launch);
  const int32_t n_sets = (int32_t)b->sets.size();
  // the previous call's upload must have left the pinned buffer
  MG_HIP(hipEventSynchronize(b->uploaded), "waiting for the previous upload");
  for (int32_t i = 0; i < n_sets; ++i) {
    b->h_sets[i] = b->sets[i]->sd;
    b->h_sets[i].n0 = (uint32_t)b->sets[i]->step;
  }
  MG_HIP(hipMemcpyAsync(b->d_sets, b->h_sets, sizeof(SetDev) * n_sets, hipMemcpyHostToDevice,
                        stream), "copying set descriptors");
  MG_HIP(hipEventRecord(b->uploaded, stream), "recording the upload");
  bool obs = false;
  for (mg_particles *p : b->sets) obs = obs || p->sd.obs != nullptr;
  if (!(b->exec && b->key_steps == n_steps && b->key_dt == dt && b->key_seed == seed &&
        b->key_idle == a.idle && b->key_chunk == chunk && b->key_obs == obs &&
        b->key_drain == a.drain && b->key_drain_lds == a.drain_lds)) {
    drop_graph(b);
    b->key_obs = obs;
    hipError_t he = build_graph(b, n_steps, a, chunk);
    if (he != hipSuccess) {
      drop_graph(b);
      return hip_fail(he, "building the batch launch graph");
    }
    b->key_steps = n_steps;
    b->key_dt = dt;
    b->key_seed = seed;
    b->key_idle = a.idle;
    b->key_chunk = chunk;
    b->key_drain = a.drain;
    b->key_drain_lds = a.drain_lds;
  }
  MG_HIP(hipGraphLaunch(b->exec, stream), "launching the batch graph");
  for (mg_particles *p : b->sets) p->step += (uint64_t)n_steps;
  return MG_OK;
}

mg_status mg_autotune(mg_particles *p, double dt, uint64_t seed, int32_t probe_steps,
                      mg_tuning *out) {
  g_err.clear();
  if (!p) return fail(MG_EINVAL, "particles is NULL");
  if (!is_finite(dt) || !(dt > 0.0)) return fail(MG_EINVAL, "dt must be finite and > 0");
  mg_tuning res{};
  if (p->prec == MG_FP32 && p->g->gen) {
    // one pool schedule is built for the general variants: nothing to probe
    res.schedule = MG_SCHED_POOLS_W8;
    res.idle_trigger = pool_idle(p);
    res.pool_size = kPoolSmall;
    res.window = 8;
    if (out) *out = res;
    return MG_OK;
  }
  if (p->prec == MG_FP64) {
    // one FP64 schedule of each kind is built: nothing to probe
    res.schedule = schedule_of(fp64_kernel(p));
    res.idle_trigger = res.schedule == MG_SCHED_LANES ? 0 : pool_idle(p);
    res.pool_size = res.schedule == MG_SCHED_LANES ? 0 : kPoolSmall;
    res.window = 8;
    if (out) *out = res;
    return MG_OK;
  }
  {
    std::lock_guard<std::mutex> lock(p->g->tune_mu);
    for (const auto &c : p->g->tune_cache)
      if (c.first == dt) {
        res = c.second;
        p->tuned = true;
        p->tuned_dt = dt;
        p->tuned_kernel = kernel_of(res.schedule);
        p->tuned_idle = res.idle_trigger;
        p->tuned_spl = res.steps_per_launch;
        if (out) *out = res;
        return MG_OK;
      }
  }
  const int64_t n = std::min<int64_t>(p->n, 1 << 22);
  const uint32_t steps = (uint32_t)(probe_steps > 0 ? probe_steps : 1024);
  if ((uint64_t)p->step + 2ull * steps > 0xFFFFFFFFull)
    return fail(MG_EINVAL, "the probe would pass step 2^32");
  const char *tune_path = std::getenv("MG_TUNE_CACHE");
  if (tune_path && !*tune_path) tune_path = nullptr;
  TuneKey key{};
  if (tune_path && !tune_key(p, dt, steps, n, key)) tune_path = nullptr;
  if (tune_path && tune_file_read(tune_path, key, res)) {
    // a result of an earlier process: no probes
    p->tuned = true;
    p->tuned_dt = dt;
    p->tuned_kernel = kernel_of(res.schedule);
    p->tuned_idle = res.schedule == MG_SCHED_LANES ? 8 : res.idle_trigger;
    p->tuned_spl = res.steps_per_launch;
    {
      std::lock_guard<std::mutex> lock(p->g->tune_mu);
      p->g->tune_cache.emplace_back(dt, res);
    }
    if (out) *out = res;
    return MG_OK;
  }
  const SetLayout L = set_layout(p->g->V, p->g->nnz, n, MG_FP32, false);
  void *mem = nullptr;
  MG_HIP(hipMalloc(&mem, L.total), "allocating the tuning probe");
  char *base = (char *)mem;
  SetDev sd{};
  sd.ef = (uint32_t *)(base + L.ef);
  sd.y32 = (float2 *)(base + L.pos);
  sd.exit_cnt = (uint64_t *)(base + L.exitc);
  sd.absorbed = (uint64_t *)(base + L.absorbed);
  sd.totals = (uint64_t *)(base + L.totals);
  sd.err = (uint32_t *)(base + L.err);
  sd.work = (uint32_t *)(base + L.work);
  sd.n = (uint32_t)n;
  sd.n0 = (uint32_t)p->step;
  sd.tag = p->tag;
  StepArgs a{};
  set_drain(a);
  a.nsteps = steps;
  a.claim_chunk = claim_chunk(steps, n, n);
  a.max_splits = p->max_splits;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.dt = dt;
  a.probe = 1;
  // one particle per lane; pools of 128 (2 per lane) at four idle triggers;
  // pools of 256 (4 per lane) at two; pools of 128 with 8-step windows at
  // three
  constexpr int kCand = 10;
  static_assert(kCand <= (int)(sizeof(mg_tuning::probe_ms) / sizeof(float)), "probe_ms");
  const int32_t cand_kernel[kCand] = {0, 1, 1, 1, 1, 2, 2, 3, 3, 3};
  const int32_t cand_idle[kCand] = {8, 4, 8, 16, 32, 8, 16, 8, 16, 32};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  float best = 0.0f;
  int best_i = -1;
  for (int i = 0; i < kCand && he == hipSuccess; ++i) {
    he = hipMemcpyAsync(sd.ef, p->sd.ef, (size_t)n * 4, hipMemcpyDeviceToDevice, p->stream);
    if (he == hipSuccess)
      he = hipMemcpyAsync(sd.y32, p->sd.y32, (size_t)n * 8, hipMemcpyDeviceToDevice, p->stream);
    if (he == hipSuccess) he = hipEventRecord(e0, p->stream);
    a.kernel = cand_kernel[i];
    a.idle = cand_idle[i];
    if (he == hipSuccess) he = launch_step(p->g->gd, sd, a, false, false, p->stream);
    if (he == hipSuccess) he = hipEventRecord(e1, p->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) break;
    res.probe_ms[i] = ms;
    if (best_i < 0 || ms < best) {
      best = ms;
      best_i = i;
    }
  }
  // steps per launch for the chosen schedule: 2 x steps as one launch
  // against two launches of `steps` (each launch ends with a tail of partly
  // filled waves; the launch count is the only difference)
  a.kernel = cand_kernel[best_i];
  a.idle = cand_idle[best_i];
  for (int i = 0; i < 2 && he == hipSuccess; ++i) {
    he = hipMemcpyAsync(sd.ef, p->sd.ef, (size_t)n * 4, hipMemcpyDeviceToDevice, p->stream);
    if (he == hipSuccess)
      he = hipMemcpyAsync(sd.y32, p->sd.y32, (size_t)n * 8, hipMemcpyDeviceToDevice, p->stream);
    if (he == hipSuccess) he = hipEventRecord(e0, p->stream);
    for (uint32_t done = 0; done < 2 * steps && he == hipSuccess;) {
      a.nsteps = i == 0 ? 2 * steps : steps;
      a.claim_chunk = claim_chunk(a.nsteps, n, n);
      sd.n0 = (uint32_t)p->step + done;
      he = launch_step(p->g->gd, sd, a, false, false, p->stream);
      done += a.nsteps;
    }
    if (he == hipSuccess) he = hipEventRecord(e1, p->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&res.launch_ms[i], e0, e1);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(mem);
  if (he != hipSuccess) return hip_fail(he, "running the tuning probe");
  // fewer launches unless the split is clearly faster
  res.steps_per_launch = res.launch_ms[1] < 0.98f * res.launch_ms[0] ? (int32_t)steps : 0;
  res.n_probes = kCand;
  res.schedule = schedule_of(cand_kernel[best_i]);
  res.idle_trigger = cand_kernel[best_i] ? cand_idle[best_i] : 0;
  res.pool_size = cand_kernel[best_i] ? pool_per_wave(cand_kernel[best_i]) : 0;
  res.window = cand_kernel[best_i] == 3 ? 8 : 4;
  p->tuned = true;
  p->tuned_dt = dt;
  p->tuned_kernel = cand_kernel[best_i];
  p->tuned_idle = cand_idle[best_i];
  p->tuned_spl = res.steps_per_launch;
  {
    std::lock_guard<std::mutex> lock(p->g->tune_mu);
    p->g->tune_cache.emplace_back(dt, res);
  }
  if (tune_path) tune_file_append(tune_path, key, res);
  if (out) *out = res;
  return MG_OK;
}

void mg_batch_destroy(mg_batch *b) {
  if (!b) return;
  if (b->uploaded) (void)hipEventSynchronize(b->uploaded);
  if (!b->sets.empty()) (void)hipStreamSynchronize(b->sets[0]->stream);
  drop_graph(b);
  if (b->uploaded) (void)hipEventDestroy(b->uploaded);
  if (b->h_sets) (void)hipHostFree(b->h_sets);
  if (b->dev) (void)hipFree(b->dev);
  delete b;
}

mg_status mg_valu_rate(int32_t op, int32_t waves_per_simd, uint32_t iters,
                       double *lane_ops_per_s, float *kernel_ms) {
  g_err.clear();
  if (!lane_ops_per_s) return fail(MG_EINVAL, "lane_ops_per_s is NULL");
  if (op < MG_VALU_FMA_F32 || op > MG_VALU_LOG_F32) return fail(MG_EINVAL, "unknown op %d", op);
  if (waves_per_simd < 1 || waves_per_simd > 8)
    return fail(MG_EINVAL, "waves_per_simd must be in 1 .. 8");
  if (iters < 1 || iters > (1u << 20)) return fail(MG_EINVAL, "iters must be in 1 .. 2^20");
  int dev = 0;
  MG_HIP(hipGetDevice(&dev), "querying the device");
  int cus = 0;
  MG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
         "querying the compute units");
  // blocks of four waves: one per CU gives each of its 4 SIMDs one wave
  const uint32_t blocks = (uint32_t)cus * (uint32_t)waves_per_simd;
  const size_t lanes = (size_t)blocks * valu_rate_lanes_per_block();
  uint32_t *out = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipMalloc(&out, lanes * sizeof(uint32_t));
  if (he == hipSuccess) he = hipStreamCreate(&st);
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  // one untimed launch (code load, clocks), then the timed one
  if (he == hipSuccess) he = launch_valu_rate(op, blocks, iters, out, st);
  if (he == hipSuccess) he = hipEventRecord(e0, st);
  if (he == hipSuccess) he = launch_valu_rate(op, blocks, iters, out, st);
  if (he == hipSuccess) he = hipEventRecord(e1, st);
  if (he == hipSuccess) he = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  if (out) (void)hipFree(out);
  if (he != hipSuccess) return hip_fail(he, "running the calibration kernel");
  if (!(ms > 0.0f)) return fail(MG_EDEVICE, "the calibration kernel took no measurable time");
  *lane_ops_per_s = (double)lanes * (double)valu_rate_ops_per_lane(iters) / (ms * 1e-3);
  if (kernel_ms) *kernel_ms = ms;
  return MG_OK;
}

}  // extern "C"
