// mg_kernels.hip -- gfx950 kernels of the timestep-splitting Euler-Maruyama
// particle step on metric graphs (Dwaraknath & Ying, Alg. 2 with Alg. 1's
// vertex rule), the particle initialisation and the per-edge histogram.
//
// One lane owns one particle for all steps of a launch; its edge record
// lives in registers and is reloaded only when a vertex hit changes the
// edge, so the common no-hit step touches no memory.  Random numbers are
// counter-based Philox4x32-10 (Salmon et al., SC'11) keyed by the seed with
// counter (particle, step word, stream word, graph tag):
//   main stream  (p, n>>2, 0, tag): two Box-Muller pairs drive the first
//                sub-steps of steps 4m..4m+3 (cos, sin of pair A; cos, sin
//                of pair B), so one Philox call serves four steps;
//   hit stream   (p, n, k, tag): after the k-th vertex hit of step n, word 0
//                draws the slot and the cosine of pair (word 1, word 2)
//                drives the next sub-step;
//   init stream  (p, 0xFFFFFFFF, 0xFFFFFFFF, tag).
// The FP32 path consumes the same integers as the FP64 path.
//
// Compiled with -ffp-contract=off: every fused multiply-add is explicit.
#include "mg_internal.h"

namespace mg {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;

struct U4 {
  uint32_t x, y, z, w;
};

// Philox4x32-10: ten rounds of two 32x32->64 products and xors, the key
// bumped by the Weyl increments before every round but the first.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2,
                                     uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t t0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t t2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = t0;
    c2 = t2;
  }
  return {c0, c1, c2, c3};
}

// Box-Muller in FP64: R = sqrt(-2 ln u1), angle 2 pi u2, u = (bits + 1/2) 2^-32.
__device__ __forceinline__ void box_muller64(uint32_t a, uint32_t b, double &wc,
                                             double &ws) {
  const double u1 = ((double)a + 0.5) * 0x1p-32;
  const double u2 = ((double)b + 0.5) * 0x1p-32;
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincos(kTwoPi * u2, &s, &c);
  wc = r * c;
  ws = r * s;
}

__device__ __forceinline__ double box_muller64_cos(uint32_t a, uint32_t b) {
  const double u1 = ((double)a + 0.5) * 0x1p-32;
  const double u2 = ((double)b + 0.5) * 0x1p-32;
  return sqrt(-2.0 * log(u1)) * cos(kTwoPi * u2);
}

// Box-Muller in FP32 on the transcendental unit: v_log_f32 is log2 and
// v_sin_f32 / v_cos_f32 take their argument in turns (sin(2 pi t)).
__device__ __forceinline__ void box_muller32(uint32_t a, uint32_t b, float &wc,
                                             float &ws) {
  const float u1 = fmaf((float)a, 0x1p-32f, 0x1p-33f);
  const float u2 = fmaf((float)b, 0x1p-32f, 0x1p-33f);
  const float r =
      __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  wc = r * __builtin_amdgcn_cosf(u2);
  ws = r * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ float box_muller32_cos(uint32_t a, uint32_t b) {
  const float u1 = fmaf((float)a, 0x1p-32f, 0x1p-33f);
  const float u2 = fmaf((float)b, 0x1p-32f, 0x1p-33f);
  return __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1)) *
         __builtin_amdgcn_cosf(u2);
}

// Smallest u in (0, 1] with C + B u + A u^2 = 0 (C >= 0), u = sqrt(alpha):
// Alg. 2's crossing equation in the frame of the distance to the hit
// vertex; cancellation-free quadratic formula q = -(B + sgn(B) sqrt(disc))/2
// with roots q/A and C/q; C = 0 (on the vertex) gives -B/A; clamped to [0,1].
template <typename T>
__device__ __forceinline__ T first_root(T A, T B, T Cc) {
  T u;
  if (Cc == T(0)) {
    if (A == T(0)) return T(0);
    u = -B / A;
  } else if (A == T(0)) {
    u = -Cc / B;
  } else {
    T disc = B * B - T(4) * A * Cc;
    if (disc < T(0)) disc = T(0);
    const T sq = sqrt(disc);
    const T q = T(-0.5) * (B >= T(0) ? B + sq : B - sq);
    const T r1 = q / A;
    const T r2 = Cc / q;
    const T lo = r1 < r2 ? r1 : r2;
    const T hi = r1 < r2 ? r2 : r1;
    u = lo > T(0) ? lo : hi;
    if (!(u > T(0))) u = T(1);
  }
  if (!(u >= T(0))) u = T(0);
  if (u > T(1)) u = T(1);
  return u;
}

__device__ __forceinline__ uint64_t fnv(uint64_t h, uint32_t w) {
  return (h ^ (uint64_t)w) * kFnvPrime;
}

// First slot s of vertex v with r < T_s (the last slot takes the rest).
__device__ __forceinline__ int32_t pick_slot(const SlotRec *slots, VtxRec vr,
                                             uint32_t r) {
  int32_t s = vr.first;
  const int32_t last = vr.first + vr.deg - 1;
  while (s < last && (uint64_t)r >= slots[s].thr) ++s;
  return s;
}

// Per-lane tallies reduced once per block.
struct Tally {
  uint32_t trunc, sub, hits, steps;
};

template <bool LDS>
__device__ __forceinline__ void count_exit(uint32_t *s_exit, uint64_t *g_exit,
                                           int32_t slot) {
  if (LDS)
    atomicAdd(&s_exit[slot], 1u);
  else
    atomicAdd((unsigned long long *)&g_exit[slot], 1ull);
}

// ------------------------------------------------------------ FP64 path --
// The canonical step in FP64, operation for operation.
template <bool TRACE, bool LDS>
__device__ void run64(const GraphDev &G, const SetDev &S, const StepArgs &A,
                      uint32_t pid, uint32_t *s_exit, Tally &t) {
  uint32_t ef = S.ef[pid];
  if (ef & kDeadBit) return;
  int32_t e = (int32_t)(ef & kEdgeMask);
  if (e >= G.E) {
    atomicOr(S.err, kErrEdge);
    return;
  }
  double x = S.x64[pid];
  EdgeRec64 R = G.e64[e];
  if (!(x >= 0.0 && x <= R.L)) {
    atomicOr(S.err, kErrPos);
    return;
  }
  uint64_t hash = TRACE ? S.seqhash[pid] : 0;
  uint32_t nhit = TRACE ? S.hits[pid] : 0;
  bool alive = true;
  const uint32_t n_end = S.n0 + A.nsteps;
  uint32_t n = S.n0;
  while (n < n_end && alive) {
    const uint32_t m = n >> 2;
    const U4 o = philox(pid, m, 0u, S.tag, A.key0, A.key1);
    double W[4];
    box_muller64(o.x, o.y, W[0], W[1]);
    box_muller64(o.z, o.w, W[2], W[3]);
    const uint32_t jb = n & 3u;
    const uint32_t je = min(4u, n_end - (m << 2));
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      if (j < jb || j >= je || !alive) continue;
      const uint32_t step = (m << 2) + j;
      double h = A.dt;
      int32_t k = 0, last = -1;
      double w = W[j];
      t.steps++;
      for (;;) {
        if (x == 0.0)
          w = fabs(w);
        else if (x == R.L)
          w = -fabs(w);
        const double mu = fma(R.c, x, R.a);
        const double g = R.sigma * sqrt(h);
        const double xt = fma(g, w, fma(mu, h, x));
        t.sub++;
        if (xt > 0.0 && xt < R.L) {
          x = xt;
          break;
        }
        const bool at_init = xt <= 0.0;
        const int32_t v = at_init ? R.vinit : R.vterm;
        const double d = at_init ? x : R.L - x;
        const double qa = at_init ? mu * h : -(mu * h);
        const double qb = at_init ? g * w : -(g * w);
        const double u = first_root<double>(qa, qb, d);
        const double alpha = u * u;
        h = fma(-alpha, h, h);
        ++k;
        ++nhit;
        t.hits++;
        const VtxRec vr = G.vtx[v];
        if (vr.deg < 0) {  // absorbing vertex
          alive = false;
          atomicAdd((unsigned long long *)&S.absorbed[v], 1ull);
          if (TRACE) hash = fnv(fnv(hash, step), 0x80000000u | (uint32_t)v);
          break;
        }
        const U4 hd = philox(pid, step, (uint32_t)k, S.tag, A.key0, A.key1);
        const int32_t s = pick_slot(G.slots, vr, hd.x);
        const SlotRec sr = G.slots[s];
        e = sr.edge;
        R = G.e64[e];
        x = sr.orient ? R.L : 0.0;
        last = s;
        if (TRACE) hash = fnv(fnv(hash, step), (uint32_t)s);
        if (h == 0.0) break;
        if (k == A.max_splits) {
          t.trunc++;
          break;
        }
        w = box_muller64_cos(hd.y, hd.z);
      }
      if (k >= 1 && alive) count_exit<LDS>(s_exit, S.exit_cnt, last);
    }
    n = (m << 2) + je;
  }
  S.ef[pid] = (uint32_t)e | (alive ? 0u : kDeadBit);
  S.x64[pid] = x;
  if (TRACE) {
    S.seqhash[pid] = hash;
    S.hits[pid] = nhit;
  }
}

// ------------------------------------------------------------ FP32 path --
// Same step; the position is y = distance from the reference end (bit 30
// of the state word), re-anchored to the nearer end after every interior
// move, so points near a vertex keep full relative precision.  In that
// frame the drift is as + c y with as = a (from the initial end) or
// -(a + c L) (from the terminal end), and the normal's sign flips with the
// end.  The remaining time is a compensated pair (hh, hl); the crossing
// solve runs in FP64 within 1e-6 L of a vertex.
struct Edge32 {
  float L, a, c, sigma, aL;
  int32_t vinit, vterm;
};

__device__ __forceinline__ Edge32 load_edge32(const EdgeRec32 *e32, int32_t e) {
  const EdgeRec32 r = e32[e];
  return {r.L, r.a, r.c, r.sigma, r.aL, r.vinit, r.vterm};
}

template <bool TRACE, bool LDS>
__device__ void run32(const GraphDev &G, const SetDev &S, const StepArgs &A,
                      uint32_t pid, uint32_t *s_exit, Tally &t) {
  uint32_t ef = S.ef[pid];
  if (ef & kDeadBit) return;
  int32_t e = (int32_t)(ef & kEdgeMask);
  if (e >= G.E) {
    atomicOr(S.err, kErrEdge);
    return;
  }
  uint32_t side = (ef & kSideBit) ? 1u : 0u;
  float y = S.y32[pid];
  Edge32 R = load_edge32(G.e32, e);
  if (!(y >= 0.0f && y <= R.L)) {
    atomicOr(S.err, kErrPos);
    return;
  }
  const float dt = (float)A.dt;
  const float sqdt = (float)sqrt(A.dt);
  float as = side ? -R.aL : R.a;
  float g0 = R.sigma * sqdt;
  uint64_t hash = TRACE ? S.seqhash[pid] : 0;
  uint32_t nhit = TRACE ? S.hits[pid] : 0;
  bool alive = true;
  const uint32_t n_end = S.n0 + A.nsteps;
  uint32_t n = S.n0;
  while (n < n_end && alive) {
    const uint32_t m = n >> 2;
    const U4 o = philox(pid, m, 0u, S.tag, A.key0, A.key1);
    float W[4];
    box_muller32(o.x, o.y, W[0], W[1]);
    box_muller32(o.z, o.w, W[2], W[3]);
    const uint32_t jb = n & 3u;
    const uint32_t je = min(4u, n_end - (m << 2));
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      if (j < jb || j >= je || !alive) continue;
      const uint32_t step = (m << 2) + j;
      t.steps++;
      // first sub-step: h = dt
      {
        const float we = (y == 0.0f) ? fabsf(W[j]) : (side ? -W[j] : W[j]);
        const float mu = fmaf(R.c, y, as);
        const float yt = fmaf(g0, we, fmaf(mu, dt, y));
        t.sub++;
        if (yt > 0.0f && yt < R.L) {
          if (yt > 0.5f * R.L) {
            y = R.L - yt;  // exact (Sterbenz)
            side ^= 1u;
            as = side ? -R.aL : R.a;
          } else {
            y = yt;
          }
          continue;
        }
      }
      // minority: the step crosses a vertex; redo the first sub-step's
      // quantities and split
      float hh = dt, hl = 0.0f;
      int32_t k = 0, last = -1;
      float w = W[j];
      bool first = true;
      for (;;) {
        const float we = (y == 0.0f) ? fabsf(w) : (side ? -w : w);
        const float mu = fmaf(R.c, y, as);
        const float g = first ? g0 : R.sigma * __builtin_amdgcn_sqrtf(hh);
        const float yt = fmaf(g, we, fmaf(mu, hh, y));
        if (!first) t.sub++;
        first = false;
        if (yt > 0.0f && yt < R.L) {
          if (yt > 0.5f * R.L) {
            y = R.L - yt;
            side ^= 1u;
            as = side ? -R.aL : R.a;
          } else {
            y = yt;
          }
          break;
        }
        const bool near = yt <= 0.0f;
        const bool at_term = near == (side != 0u);
        const int32_t v = at_term ? R.vterm : R.vinit;
        const float d = near ? y : R.L - y;
        float u;
        if (d < 1e-6f * R.L) {
          // crossing solve in FP64 next to the vertex
          const double hd = (double)hh + (double)hl;
          const double mud = fma((double)R.c, (double)y, (double)as);
          const double gd = (double)R.sigma * sqrt(hd);
          const double qa = near ? mud * hd : -(mud * hd);
          const double qb = near ? gd * (double)we : -(gd * (double)we);
          const double dd = near ? (double)y : (double)R.L - (double)y;
          u = (float)first_root<double>(qa, qb, dd);
        } else {
          const float mh = mu * hh, gw = g * we;
          u = first_root<float>(near ? mh : -mh, near ? gw : -gw, d);
        }
        // remaining time (1 - u^2)(hh + hl), compensated
        {
          const float al = u * u;
          const float p = al * hh;
          const float pe = fmaf(al, hh, -p);
          const float s = hh - p;
          const float bb = s - hh;
          const float se = (hh - (s - bb)) + (-p - bb);
          const float lo = ((se - pe) + hl) - al * hl;
          hh = s + lo;
          hl = lo - (hh - s);
        }
        ++k;
        ++nhit;
        t.hits++;
        const VtxRec vr = G.vtx[v];
        if (vr.deg < 0) {
          alive = false;
          atomicAdd((unsigned long long *)&S.absorbed[v], 1ull);
          if (TRACE) hash = fnv(fnv(hash, step), 0x80000000u | (uint32_t)v);
          break;
        }
        const U4 hd = philox(pid, step, (uint32_t)k, S.tag, A.key0, A.key1);
        const int32_t s = pick_slot(G.slots, vr, hd.x);
        const SlotRec sr = G.slots[s];
        e = sr.edge;
        R = load_edge32(G.e32, e);
        side = sr.orient ? 1u : 0u;
        y = 0.0f;
        as = side ? -R.aL : R.a;
        g0 = R.sigma * sqdt;
        last = s;
        if (TRACE) hash = fnv(fnv(hash, step), (uint32_t)s);
        if (hh == 0.0f) break;
        if (k == A.max_splits) {
          t.trunc++;
          break;
        }
        w = box_muller32_cos(hd.y, hd.z);
      }
      if (k >= 1 && alive) count_exit<LDS>(s_exit, S.exit_cnt, last);
    }
    n = (m << 2) + je;
  }
  S.ef[pid] = (uint32_t)e | (side ? kSideBit : 0u) | (alive ? 0u : kDeadBit);
  S.y32[pid] = y;
  if (TRACE) {
    S.seqhash[pid] = hash;
    S.hits[pid] = nhit;
  }
}

// Block-level reduction of the lane tallies and the LDS exit counters.
__device__ __forceinline__ void flush(const SetDev &S, const Tally &t,
                                      uint32_t *s_tot, uint32_t *s_exit,
                                      int32_t nnz, bool lds) {
  atomicAdd(&s_tot[0], t.trunc);
  atomicAdd(&s_tot[1], t.sub);
  atomicAdd(&s_tot[2], t.hits);
  atomicAdd(&s_tot[3], t.steps);
  __syncthreads();
  if (threadIdx.x < 4 && s_tot[threadIdx.x])
    atomicAdd((unsigned long long *)&S.totals[threadIdx.x],
              (unsigned long long)s_tot[threadIdx.x]);
  if (lds) {
    for (int32_t s = threadIdx.x; s < nnz; s += blockDim.x)
      if (s_exit[s]) atomicAdd((unsigned long long *)&S.exit_cnt[s],
                               (unsigned long long)s_exit[s]);
  }
}

template <bool FP64, bool TRACE, bool LDS>
__global__ __launch_bounds__(kBlock) void k_step(GraphDev G, SetDev S, StepArgs A) {
  extern __shared__ uint32_t s_exit[];
  __shared__ uint32_t s_tot[4];
  if (threadIdx.x < 4) s_tot[threadIdx.x] = 0;
  if (LDS)
    for (int32_t s = threadIdx.x; s < G.nnz; s += blockDim.x) s_exit[s] = 0;
  __syncthreads();
  Tally t{0, 0, 0, 0};
  const uint32_t pid = blockIdx.x * kBlock + threadIdx.x;
  if (pid < S.n) {
    if (FP64)
      run64<TRACE, LDS>(G, S, A, pid, s_exit, t);
    else
      run32<TRACE, LDS>(G, S, A, pid, s_exit, t);
  }
  flush(S, t, s_tot, s_exit, G.nnz, LDS);
}

template <bool FP64, bool TRACE, bool LDS>
__global__ __launch_bounds__(kBlock) void k_batch(const GraphDev *graphs,
                                                  const SetDev *sets,
                                                  const BatchItem *items,
                                                  StepArgs A) {
  extern __shared__ uint32_t s_exit[];
  __shared__ uint32_t s_tot[4];
  const BatchItem it = items[blockIdx.x];
  const SetDev S = sets[it.set];
  const GraphDev G = graphs[it.set];
  if (threadIdx.x < 4) s_tot[threadIdx.x] = 0;
  if (LDS)
    for (int32_t s = threadIdx.x; s < G.nnz; s += blockDim.x) s_exit[s] = 0;
  __syncthreads();
  Tally t{0, 0, 0, 0};
  const uint32_t pid = it.first + threadIdx.x;
  if (pid < S.n) {
    if (FP64)
      run64<TRACE, LDS>(G, S, A, pid, s_exit, t);
    else
      run32<TRACE, LDS>(G, S, A, pid, s_exit, t);
  }
  flush(S, t, s_tot, s_exit, G.nnz, LDS);
}

// ---------------------------------------------------------------- init --
template <bool FP64>
__global__ __launch_bounds__(kBlock) void k_init(GraphDev G, SetDev S, int mode,
                                                 int32_t vertex, uint32_t k0,
                                                 uint32_t k1, const int32_t *edge_in,
                                                 const double *pos_in) {
  const uint32_t pid = blockIdx.x * kBlock + threadIdx.x;
  if (pid >= S.n) return;
  int32_t e;
  double x;
  if (mode == 0) {
    e = edge_in[pid];
    x = pos_in[pid];
  } else {
    const U4 o = philox(pid, 0xFFFFFFFFu, 0xFFFFFFFFu, S.tag, k0, k1);
    if (mode == 1) {
      const VtxRec vr = G.vtx[vertex];
      const int32_t s = pick_slot(G.slots, vr, o.x);
      const SlotRec sr = G.slots[s];
      e = sr.edge;
      x = sr.orient ? G.e64[e].L : 0.0;
    } else {
      // first e with r < T_e (thresholds nondecreasing; T_{E-1} = 2^32)
      int32_t lo = 0, hi = G.E - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if ((uint64_t)o.x < G.len_thr[mid])
          hi = mid;
        else
          lo = mid + 1;
      }
      e = lo;
      x = G.e64[e].L * (((double)o.y + 0.5) * 0x1p-32);
    }
  }
  const double L = G.e64[e].L;
  if (FP64) {
    S.ef[pid] = (uint32_t)e;
    S.x64[pid] = x;
  } else {
    const bool side = x > 0.5 * L;
    S.ef[pid] = (uint32_t)e | (side ? kSideBit : 0u);
    S.y32[pid] = (float)(side ? L - x : x);
  }
  if (S.seqhash) S.seqhash[pid] = 0xcbf29ce484222325ull;
  if (S.hits) S.hits[pid] = 0;
}

// ----------------------------------------------------------- histogram --
template <bool FP64, bool LDS>
__global__ __launch_bounds__(kBlock) void k_hist(GraphDev G, SetDev S, int32_t nb,
                                                 uint64_t *out) {
  extern __shared__ uint32_t s_bin[];
  const int32_t nbins = G.E * nb;
  if (LDS) {
    for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x) s_bin[b] = 0;
    __syncthreads();
  }
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t pid = blockIdx.x * kBlock + threadIdx.x; pid < S.n; pid += stride) {
    const uint32_t ef = S.ef[pid];
    if (ef & kDeadBit) continue;
    const int32_t e = (int32_t)(ef & kEdgeMask);
    const double L = G.e64[e].L;
    double x;
    if (FP64) {
      x = S.x64[pid];
    } else {
      const double y = (double)S.y32[pid];
      x = (ef & kSideBit) ? L - y : y;
    }
    const double inv = (double)nb / L;
    const double f = floor(x * inv);
    int32_t b = f < 0.0 ? 0 : (f > (double)(nb - 1) ? nb - 1 : (int32_t)f);
    const int32_t idx = e * nb + b;
    if (LDS)
      atomicAdd(&s_bin[idx], 1u);
    else
      atomicAdd((unsigned long long *)&out[idx], 1ull);
  }
  if (LDS) {
    __syncthreads();
    for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x)
      if (s_bin[b]) atomicAdd((unsigned long long *)&out[b], (unsigned long long)s_bin[b]);
  }
}

template <bool FP64, bool TRACE>
hipError_t launch_step_t(const GraphDev &g, const SetDev &s, const StepArgs &a,
                         hipStream_t st) {
  const uint32_t blocks = (s.n + kBlock - 1) / kBlock;
  if (g.nnz <= kLdsExitMax) {
    hipLaunchKernelGGL((k_step<FP64, TRACE, true>), dim3(blocks), dim3(kBlock),
                       (size_t)g.nnz * 4, st, g, s, a);
  } else {
    hipLaunchKernelGGL((k_step<FP64, TRACE, false>), dim3(blocks), dim3(kBlock), 0,
                       st, g, s, a);
  }
  return hipGetLastError();
}

template <bool FP64, bool TRACE>
hipError_t launch_batch_t(const GraphDev *graphs, const SetDev *sets,
                          const BatchItem *items, int32_t n_items, int32_t max_nnz,
                          const StepArgs &a, hipStream_t st) {
  if (max_nnz <= kLdsExitMax) {
    hipLaunchKernelGGL((k_batch<FP64, TRACE, true>), dim3(n_items), dim3(kBlock),
                       (size_t)max_nnz * 4, st, graphs, sets, items, a);
  } else {
    hipLaunchKernelGGL((k_batch<FP64, TRACE, false>), dim3(n_items), dim3(kBlock), 0,
                       st, graphs, sets, items, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_init(const GraphDev &g, const SetDev &s, int mode, int32_t vertex,
                       uint32_t key0, uint32_t key1, const int32_t *edge_in,
                       const double *pos_in, bool fp64, hipStream_t st) {
  const uint32_t blocks = (s.n + kBlock - 1) / kBlock;
  if (fp64)
    hipLaunchKernelGGL(k_init<true>, dim3(blocks), dim3(kBlock), 0, st, g, s, mode,
                       vertex, key0, key1, edge_in, pos_in);
  else
    hipLaunchKernelGGL(k_init<false>, dim3(blocks), dim3(kBlock), 0, st, g, s, mode,
                       vertex, key0, key1, edge_in, pos_in);
  return hipGetLastError();
}

hipError_t launch_step(const GraphDev &g, const SetDev &s, const StepArgs &a,
                       bool fp64, bool trace, hipStream_t st) {
  if (fp64) return trace ? launch_step_t<true, true>(g, s, a, st)
                         : launch_step_t<true, false>(g, s, a, st);
  return trace ? launch_step_t<false, true>(g, s, a, st)
               : launch_step_t<false, false>(g, s, a, st);
}

hipError_t launch_batch(const GraphDev *graphs, const SetDev *sets,
                        const BatchItem *items, int32_t n_items, int32_t max_nnz,
                        const StepArgs &a, bool fp64, bool trace, hipStream_t st) {
  if (fp64)
    return trace ? launch_batch_t<true, true>(graphs, sets, items, n_items, max_nnz, a, st)
                 : launch_batch_t<true, false>(graphs, sets, items, n_items, max_nnz, a, st);
  return trace ? launch_batch_t<false, true>(graphs, sets, items, n_items, max_nnz, a, st)
               : launch_batch_t<false, false>(graphs, sets, items, n_items, max_nnz, a, st);
}

hipError_t launch_histogram(const GraphDev &g, const SetDev &s, int32_t nb,
                            uint64_t *out, bool fp64, hipStream_t st) {
  const int64_t nbins = (int64_t)g.E * nb;
  const bool lds = nbins <= kLdsExitMax;
  uint32_t blocks = (s.n + kBlock - 1) / kBlock;
  if (lds && blocks > 1024) blocks = 1024;  // amortise the LDS merge
  if (!lds && blocks > 8192) blocks = 8192;
  const size_t shm = lds ? (size_t)nbins * 4 : 0;
  if (fp64) {
    if (lds) hipLaunchKernelGGL((k_hist<true, true>), dim3(blocks), dim3(kBlock), shm, st, g, s, nb, out);
    else hipLaunchKernelGGL((k_hist<true, false>), dim3(blocks), dim3(kBlock), shm, st, g, s, nb, out);
  } else {
    if (lds) hipLaunchKernelGGL((k_hist<false, true>), dim3(blocks), dim3(kBlock), shm, st, g, s, nb, out);
    else hipLaunchKernelGGL((k_hist<false, false>), dim3(blocks), dim3(kBlock), shm, st, g, s, nb, out);
  }
  return hipGetLastError();
}

}  // namespace mg
