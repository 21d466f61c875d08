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
#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "mg_internal.h"

namespace mg {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Main-stream Philox groups (four steps each) run before the parked lanes
// of a window resolve their vertex hits.
#ifndef MG_WINDOW_GROUPS32
#define MG_WINDOW_GROUPS32 1
#endif
#ifndef MG_WINDOW_GROUPS64
#define MG_WINDOW_GROUPS64 2
#endif
constexpr int kWindowGroups32 = MG_WINDOW_GROUPS32;
constexpr int kWindowGroups64 = MG_WINDOW_GROUPS64;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;

struct U4 {
  uint32_t x, y, z, w;
};

// Three-input exclusive or in one gfx950 instruction (v_bitop3_b32 with
// truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10: ten rounds of two 32x32->64 products (v_mad_u64_u32) and
// three-way xors, the key bumped by the Weyl increments before every round
// but the first.
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
    const uint32_t t0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t t2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = t0;
    c2 = t2;
  }
  return {c0, c1, c2, c3};
}

// Keys of a Philox call in an FP64 kernel.  The FP64 polynomial constants
// fill the scalar registers there, so the round keys, which the compiler
// computes once outside the loops, are spilled to lanes of a vector
// register and read back with a readlane (a vector issue slot) per round.
// Hiding the two keys from the optimiser at the call keeps each Weyl
// increment next to its round, as a scalar add.  FP32 kernels keep their
// round keys in scalar registers and are left as they are.
template <class real>
__device__ __forceinline__ void fresh_keys(uint32_t &k0, uint32_t &k1) {
  if constexpr (sizeof(real) == 8) asm volatile("" : "+s"(k0), "+s"(k1));
}

// Sine and cosine of t in [0, 2 pi) (the Box-Muller angle, t = 2 pi u with
// u in (0, 1)): the argument is reduced by quarter turns, r = t - q pi/2
// with pi/2 in two parts (Cody and Waite); for q <= 4 the first step
// fma(-q, hi, t) is exact, so r carries the error of the second alone.
// On |r| <= pi/4, sin r = r + r^3 P(r^2) and cos r = 1 - r^2/2 + r^4 C(r^2)
// with P of degree 5 and C of degree 5, minimax polynomials for the
// relative error of sine and cosine (Remez exchange; the fit is
// minimax_fit.py beside this file): their approximation errors are below
// 2^-57 and 2^-63 of the value, and Horner's rule with fused multiply-adds
// keeps the result within one ulp of glibc's sin and cos on 2e7 angles
// (the general library routine handles any argument and costs several
// times as much).  The quadrant then picks and signs the two.
__device__ __forceinline__ void sincos_small(double t, double &s_out, double &c_out) {
  const double q = rint(t * 0.6366197723675814);
  double r = fma(-q, 1.5707963267948966, t);
  r = fma(-q, 6.123233995736766e-17, r);
  const double x2 = r * r;
  double ps = 1.5896230157095365e-10;  // P, highest degree first
  ps = fma(ps, x2, -2.5050747762851854e-08);
  ps = fma(ps, x2, 2.755731362138572e-06);
  ps = fma(ps, x2, -0.0001984126982958954);
  ps = fma(ps, x2, 0.008333333333322118);
  ps = fma(ps, x2, -0.1666666666666663);
  const double sn = fma(r * x2, ps, r);
  double pc = -1.1358536524507801e-11;  // C, highest degree first
  pc = fma(pc, x2, 2.087570084203873e-09);
  pc = fma(pc, x2, -2.7557314179297243e-07);
  pc = fma(pc, x2, 2.4801587288851707e-05);
  pc = fma(pc, x2, -0.0013888888888873056);
  pc = fma(pc, x2, 0.041666666666666595);
  pc = fma(pc, x2, -0.5);
  const double cs = fma(pc, x2, 1.0);
  const int iq = (int)q & 3;
  const bool swap = iq & 1;
  const double a = swap ? cs : sn, b = swap ? sn : cs;
  s_out = (iq >= 2) ? -a : a;
  c_out = (iq == 1 || iq == 2) ? -b : b;
}

// Quotient n / d for d in [1, 4) and |n| < 1, where no range scaling,
// overflow or special value can arise: the hardware reciprocal estimate
// refined by two Newton-Raphson steps, the product, and one correction by
// the residual (Markstein's sequence).  These are the device library's
// division steps without its operand scaling and special-value fix-up,
// which leave such operands unchanged, so the quotient is the library's.
__device__ __forceinline__ double div_unit(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  const double q = n * r;
  return fma(fma(-d, q, n), r, q);
}

// Square root of x in [2^-767, 2^1023) (normal, positive, finite): the
// hardware reciprocal square root y refined in Markstein's coupled form
// (g ~ sqrt(x) and h ~ 1/(2 sqrt(x)) updated together, then two residual
// corrections of g).  These are the device library's steps without its
// scaling of tiny arguments and its zero, infinity and NaN checks, which
// leave such arguments unchanged, so the root is the library's.  The
// Box-Muller radius argument -2 ln u lies in [2.3e-10, 44.4].
__device__ __forceinline__ double sqrt_normal(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = y * 0.5;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  double d = fma(-g, g, x);
  h = fma(h, r, h);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

// Natural logarithm of a Box-Muller uniform u in (0, 1) (no zero, infinite
// or negative arguments reach it): u = 2^e m with m in [sqrt(1/2), sqrt(2))
// shifted down by at most 3e-7 of itself (the split is decided on the high
// word of the mantissa),
// f = m - 1 (exact), s = f / (2 + f) (div_unit), and log(1 + f) = 2 atanh(s) written as
// f - (f^2/2 - s (f^2/2 + R)), R = 2 atanh(s)/s - 2 = 2 z/3 + 2 z^2/5 + ...
// in z = s^2 <= 0.0295, here z Q(z) with Q the degree-6 minimax polynomial
// for R (Remez exchange; minimax_fit.py beside this file), whose error is
// below 2^-59 of log(1 + f); e ln 2 with ln 2 in two parts (its first 32
// bits, exact times e, and the rest).  Within 0.80 ulp of the exact value
// on 2e7 draws of (a + 1/2) 2^-32 (the general library routine, with its
// extended-precision steps, costs about twice as many FP64 operations).
__device__ __forceinline__ double log_unit(double u) {
  // exponent and mantissa from the bits: adding 2^20 (1 - sqrt(1/2)) to the
  // high word carries into the exponent exactly when the mantissa's high
  // word is at least sqrt 2's, which picks m in [sqrt(1/2), sqrt(2)) with
  // integer operations alone (u is normal and positive)
  const uint64_t bits = (uint64_t)__double_as_longlong(u);
  const uint32_t hx = (uint32_t)(bits >> 32) + 0x00095f62u;
  const int e = (int)(hx >> 20) - 0x3ff;
  const double m = __longlong_as_double(
      (long long)(((uint64_t)((hx & 0x000fffffu) + 0x3fe6a09eu) << 32) | (bits & 0xffffffffull)));
  const double f = m - 1.0;
  const double s = div_unit(f, 2.0 + f);
  const double z = s * s;
  double r = 0.1479594963458122;  // Q, highest degree first
  r = fma(r, z, 0.15314050559867082);
  r = fma(r, z, 0.18183564325758253);
  r = fma(r, z, 0.22222198573192972);
  r = fma(r, z, 0.2857142874238752);
  r = fma(r, z, 0.3999999999941468);
  r = fma(r, z, 0.6666666666666734);
  r = r * z;
  const double hfsq = 0.5 * f * f;
  const double de = (double)e;
  return fma(de, 0.6931471803691238, f - (hfsq - fma(s, hfsq + r, de * 1.9082149292705877e-10)));
}

// Box-Muller in FP64: R = sqrt(-2 ln u1), angle 2 pi u2, u = (bits + 1/2) 2^-32.
__device__ __forceinline__ void box_muller64(uint32_t a, uint32_t b, double &wc,
                                             double &ws) {
  const double u1 = ((double)a + 0.5) * 0x1p-32;
  const double u2 = ((double)b + 0.5) * 0x1p-32;
  const double r = sqrt_normal(-2.0 * log_unit(u1));
  double s, c;
  sincos_small(kTwoPi * u2, s, c);
  wc = r * c;
  ws = r * s;
}

__device__ __forceinline__ double box_muller64_cos(uint32_t a, uint32_t b) {
  const double u1 = ((double)a + 0.5) * 0x1p-32;
  const double u2 = ((double)b + 0.5) * 0x1p-32;
  double s, c;
  sincos_small(kTwoPi * u2, s, c);
  return sqrt_normal(-2.0 * log_unit(u1)) * c;
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
// with roots q/A and C/q; C = 0 (on the vertex) gives -B/A, A = 0 gives
// -C/B; clamped to [0, 1].  The three cases are computed as one pair of
// divisions whose operands are selected, so no lane branches; in FP64 the
// divisions are IEEE-exact, which keeps the result bit-equal to the plain
// case-by-case evaluation.
__device__ __forceinline__ double first_root64(double A, double B, double Cc) {
  double disc = B * B - 4.0 * A * Cc;
  disc = disc < 0.0 ? 0.0 : disc;
  const double sq = sqrt(disc);
  const double q = -0.5 * (B >= 0.0 ? B + sq : B - sq);
  const bool c0 = Cc == 0.0, a0 = A == 0.0;
  // general: q / A and C / q;  C = 0: -B / A;  A = 0: -C / B
  const double n1 = c0 ? -B : (a0 ? -Cc : q);
  const double d1 = a0 ? B : A;
  const double d2 = (c0 || a0) ? 1.0 : q;
  const double r1 = n1 / d1;
  const double r2 = Cc / d2;
  const double lo = r1 < r2 ? r1 : r2;
  const double hi = r1 < r2 ? r2 : r1;
  double ug = lo > 0.0 ? lo : hi;
  ug = ug > 0.0 ? ug : 1.0;
  double u = (c0 || a0) ? r1 : ug;
  u = (c0 && a0) ? 0.0 : u;
  u = u >= 0.0 ? u : 0.0;  // also maps NaN to 0
  return u > 1.0 ? 1.0 : u;
}

// The same in FP32 with one hardware reciprocal (about one ulp).  In the
// general case the sign of B tells which root is the smallest positive one,
// so only that division is made: with C > 0 and real roots, B < 0 gives
// q > 0 and the root C/q, which is the smaller of two positive roots (A > 0;
// q^2 >= AC) or the positive one (A < 0); B >= 0 gives q <= 0, so C/q <= 0
// and q/A is positive exactly when A < 0.  A negative discriminant (only
// after rounding, next to a double root) is clamped to 0 and gives the
// double root q/A.  No positive root gives the whole sub-step, u = 1.  The
// result equals that of taking both divisions and the smallest positive.
__device__ __forceinline__ float first_root32(float A, float B, float Cc) {
  const float disc0 = fmaf(B, B, -4.0f * A * Cc);
  const bool real2 = disc0 > 0.0f;
  const float sq = __builtin_amdgcn_sqrtf(real2 ? disc0 : 0.0f);
  const bool bneg = B < 0.0f;
  const float q = -0.5f * (bneg ? B - sq : B + sq);
  const bool c0 = Cc == 0.0f, a0 = A == 0.0f;
  const bool cq = bneg & real2;
  // C = 0: -B / A;  A = 0: -C / B;  else C / q or q / A
  const float num = c0 ? -B : (a0 ? -Cc : (cq ? Cc : q));
  const float den = c0 ? A : (a0 ? B : (cq ? q : A));
  const float r = num * __builtin_amdgcn_rcpf(den);
  float u = (c0 || a0) ? r : (r > 0.0f ? r : 1.0f);
  u = (c0 && a0) ? 0.0f : u;
  u = u >= 0.0f ? u : 0.0f;
  return u > 1.0f ? 1.0f : u;
}

__device__ __forceinline__ uint64_t fnv(uint64_t h, uint32_t w) {
  return (h ^ (uint64_t)w) * kFnvPrime;
}

// Event trace: a vertex hit of a chosen particle (ids ascending in S.ev_ids)
// appends its record (step, hit index, vertex, slot or -1 when the particle
// is removed there, u = sqrt(alpha) and the time left after the hit); the
// counter counts every event, records past the capacity are dropped.  Only
// sets with trace call it.
__device__ void trace_hit(const SetDev &S, uint32_t pid, uint32_t step, int32_t k, int32_t v,
                          int32_t slot, double u, double h_after) {
  if (!S.ev) return;
  int32_t lo = 0, hi = S.ev_nids;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (S.ev_ids[mid] < pid)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo == S.ev_nids || S.ev_ids[lo] != pid) return;
  const unsigned long long i = atomicAdd(S.ev_cnt, 1ull);
  if (i < (unsigned long long)S.ev_cap) {
    mg_event &r = S.ev[i];
    r.pid = pid;
    r.step = step;
    r.k = k;
    r.vertex = v;
    r.slot = slot;
    r.reserved = 0;
    r.u = u;
    r.h_after = h_after;
  }
}

// Vertex stream of a Wentzell visit: word 0 of Philox (p, n, 0x100 + k, tag)
// decides the killing at the visit of the k-th hit of step n (k = 0: the
// visit at the start of a step that begins on the vertex).  Hit streams use
// k <= 255 in that word, so the two never share a counter.
__device__ __forceinline__ uint32_t vertex_draw(uint32_t pid, uint32_t step, uint32_t k,
                                                const SetDev &S, const StepArgs &A) {
  return philox(pid, step, 0x100u + k, S.tag, A.key0, A.key1).x;
}

// One visit of a Wentzell vertex (general gluing condition, Sec. 2.2; the
// scheme charges each visit its local time l = o + lt_per_sqrt sqrt(h''),
// the overshoot o of the proposal that crossed the vertex plus the mean
// local time of the move of length h'' that leaves it).  With h left in
// the step, the particle first stays on the vertex for gamma l and then
// moves for h'', where h'' + gamma (o + lt_per_sqrt sqrt(h'')) = h, a
// quadratic in sqrt(h'') solved in cancellation-free form; when gamma o >= h
// it stays for all of h and owes gamma o - h more.  The visit kills with
// probability 1 - exp(-kappa l), decided by the vertex-stream word `bits`
// as a uniform (bits + 1/2) 2^-32.  Returns true if the particle is killed;
// otherwise hm is the move's length (0: it stays for the rest of the step)
// and owed the stay still owed after this step.  FP64 throughout (both
// precisions; visits are rare).
__device__ __forceinline__ bool wz_visit(const WzRec &w, double o, double h, uint32_t bits,
                                         double &hm, double &owed) {
  double lt;
  owed = 0.0;
  if (w.gamma == 0.0) {
    hm = h;
    lt = o + w.lt_per_sqrt * sqrt(h);
  } else if (w.gamma * o >= h) {
    hm = 0.0;
    lt = o;
    owed = w.gamma * o - h;
  } else {
    const double b = w.gamma * w.lt_per_sqrt, r = h - w.gamma * o;
    const double sq = 2.0 * r / (b + sqrt(b * b + 4.0 * r));
    hm = sq * sq;
    lt = o + w.lt_per_sqrt * sq;
  }
  return w.kappa > 0.0 && ((double)bits + 0.5) * 0x1p-32 < -expm1(-w.kappa * lt);
}

// Graph tables as the step kernels see them: global memory, or LDS when the
// block staged them.
struct GView {
  const VtxBlk *vtx;
  const SlotRec8 *slots;
  const int32_t *guide;
  const EdgeRec32 *e32;
  const EdgeRec64 *e64;
  const EdgeRec64 *hi64;  // global FP64 records: the FP32 path reads the
                          // higher coefficient terms from them
  const WzRec *wz;        // global Wentzell table
  const TabRec64 *tab64;  // global tabulated-coefficient intervals
  const TabRec32 *tab32;
};

__device__ __forceinline__ GView global_view(const GraphDev &G) {
  return {G.vtx, G.slots, G.guide, G.e32, G.e64, G.e64, G.wz, G.tab64, G.tab32};
}

struct SlotPick {
  int32_t s;    // global slot id
  uint32_t eo;  // edge << 1 | orient (bit 31: saturated threshold)
};

__device__ __forceinline__ int32_t eo_edge(uint32_t eo) { return (int32_t)((eo & 0x7FFFFFFFu) >> 1); }

// First slot k of the vertex with r < T_k (the last slot takes the rest):
// inline thresholds for degree <= 3, else the guide bucket of r and a short
// scan of the slot table.
__device__ __forceinline__ SlotPick pick_slot(const GView &g, const VtxBlk &vb, uint32_t r) {
  if (vb.deg <= 3) {
    int32_t k = 0;
    uint32_t eo = vb.eo0;
    if (vb.deg > 1 && !(r < vb.t0 || (vb.eo0 & kSatBit))) {
      k = 1;
      eo = vb.eo1;
      if (vb.deg > 2 && !(r < vb.t1 || (vb.eo1 & kSatBit))) {
        k = 2;
        eo = vb.eo2;
      }
    }
    return {vb.first + k, eo};
  }
  int32_t k = g.guide[vb.t0 + (r >> vb.t1)];
  SlotRec8 sr = g.slots[vb.first + k];
  while (k < vb.deg - 1 && !(r < sr.t || (sr.eo & kSatBit))) {
    ++k;
    sr = g.slots[vb.first + k];
  }
  return {vb.first + k, sr.eo};
}

// Per-lane tallies reduced once per block.  A lane of the lane schedule
// holds one particle for a launch of at most 2^20 steps and M <= 255, so
// each field stays below 2^20 (M + 1) = 2^28; the block adds them into
// 64-bit LDS totals.  A lane of the wave pools serves any number of
// particles, so the pools drain their lanes' tallies into the block totals
// periodically (drain_tally).
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

// Bin of position x on an edge binned over [0, span], nb bins per edge: x
// times the FP64 inverse bin width nb / span, rounded down, clamped to
// [0, nb - 1] (the appendix histogram kernel, with x = span and anything
// beyond in the last bin).
__device__ __forceinline__ int32_t bin_of(double x, double span, int32_t nb) {
  const double inv = (double)nb / span;
  const double f = floor(x * inv);
  return f < 0.0 ? 0 : (f > (double)(nb - 1) ? nb - 1 : (int32_t)f);
}

// Streamed histogram.  A snapshot adds every alive particle's bin at each
// step counter value that is a multiple of S.obs_every (the state after
// that many steps).  next_snapshot(n) is the first such value after n; 0
// (never reached: counters after a step are >= 1) when there is none below
// 2^32 or streaming is off.
__device__ __forceinline__ uint32_t next_snapshot(uint32_t n, const SetDev &S) {
  if (!S.obs) return 0u;
  const uint64_t v = ((uint64_t)(n / S.obs_every) + 1u) * S.obs_every;
  return v > 0xFFFFFFFFull ? 0u : (uint32_t)v;
}

// Where snapshots go: LDS bins of the block (lds != null) or the set's
// global counters; e64 is the global FP64 edge table (bins are taken in
// FP64 from the lengths, as the histogram kernel does).
struct ObsSink {
  uint32_t *lds;
  const EdgeRec64 *e64;
};

template <typename P>
__device__ __forceinline__ void observe(const P &q, const SetDev &S, const ObsSink &o) {
  const EdgeRec64 &r = o.e64[q.e];
  const int32_t idx = q.e * S.obs_nb + bin_of(q.pos64(r.L), r.span, S.obs_nb);
  if (o.lds)
    atomicAdd(&o.lds[idx], 1u);
  else
    atomicAdd((unsigned long long *)&S.obs[idx], 1ull);
}

template <typename T, int N>
__device__ __forceinline__ T pickw(const T (&W)[N], uint32_t j) {
  T w = W[0];
#pragma unroll
  for (int i = 1; i < N; ++i) w = (j == (uint32_t)i) ? W[i] : w;
  return w;
}

// Step loop shared by both precisions.  P is a per-lane particle (FP64 or
// FP32) with
//   bool fast(W)                    first sub-step of a step (h = dt); true if
//                                   it stays inside the edge (then applied);
//   void resolve(step, W, ...)      the rest of a step whose first sub-step
//                                   reached a vertex: splits, edge draws,
//                                   further sub-steps, exit record.
// Hits are not resolved where they happen: within one group of four steps
// (one main-stream Philox block) every lane first runs the cheap first
// sub-steps; a lane that reaches a vertex parks there; the parked lanes then
// resolve together and finish their group from the cached normals.  Each
// particle's arithmetic and random numbers are those of the plain order;
// the split code runs once per round for all parked lanes instead of once
// per step for any lane that hit.
template <int NG, bool OBS, typename P>
__device__ __forceinline__ void step_loop(P &q, const SetDev &S, const StepArgs &A,
                                          uint32_t pid, Tally &t, const ObsSink &o) {
  constexpr uint32_t NW = 4 * NG;  // steps per window
  const uint32_t n_end = S.n0 + A.nsteps;
  uint32_t n = S.n0;
  uint32_t snap = OBS ? next_snapshot(n, S) : 0u;
  // after each completed step (and the group-end re-anchoring)
  auto snapshot = [&](uint32_t done) {
    if (OBS && done == snap) {
      observe(q, S, o);
      snap = next_snapshot(done, S);
    }
  };
  while (n < n_end && q.alive) {
    const uint32_t base = n & ~(NW - 1);
    typename P::real W[NW];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      uint32_t k0 = A.key0, k1 = A.key1;
      fresh_keys<typename P::real>(k0, k1);
      const U4 o = philox(pid, (base >> 2) + g, 0u, S.tag, k0, k1);
      P::box_muller(o.x, o.y, W[4 * g + 0], W[4 * g + 1]);
      P::box_muller(o.z, o.w, W[4 * g + 2], W[4 * g + 3]);
    }
    const uint32_t jb = n - base;
    const uint32_t je = min(NW, n_end - base);
    // FP32: the window's normals stay in registers (every access has a
    // compile-time index; the normal of a parked step travels in wp).
    // FP64: the continuation after a hit indexes them at run time, which
    // keeps the eight doubles out of registers (measured faster: one more
    // wave per SIMD).
    int32_t pj = -1;
    typename P::real wp = 0;
    q.prep_window(W, jb);
#pragma unroll
    for (uint32_t j = 0; j < NW; ++j) {
      if (j < jb || j >= je || pj >= 0) continue;
      if (!q.fast_first(W[j])) {
        pj = (int32_t)j;
        wp = W[j];
      } else {
        if ((j & 3u) == 3u) q.reanchor();
        snapshot(base + j + 1u);
      }
    }
    while (pj >= 0) {
      const uint32_t j0 = (uint32_t)pj;
      q.resolve(base + j0, wp, pid, S, A, t);
      if (q.alive) {
        if ((j0 & 3u) == 3u) q.reanchor();
        snapshot(base + j0 + 1u);
      }
      pj = -1;
      if constexpr (sizeof(typename P::real) == 8) {
        for (uint32_t j = j0 + 1; j < je && q.alive; ++j) {
          const typename P::real wj = pickw(W, j);
          if (!q.fast(wj)) {
            pj = (int32_t)j;
            wp = wj;
            break;
          }
          if ((j & 3u) == 3u) q.reanchor();
          snapshot(base + j + 1u);
        }
      } else {
#pragma unroll
        for (uint32_t j = 1; j < NW; ++j) {
          if (j <= j0 || j >= je || !q.alive || pj >= 0) continue;
          if (!q.fast(W[j])) {
            pj = (int32_t)j;
            wp = W[j];
          } else {
            if ((j & 3u) == 3u) q.reanchor();
            snapshot(base + j + 1u);
          }
        }
      }
    }
    n = base + je;
  }
  // every step taken has one first sub-step; resolve() counts the others
  const uint32_t taken = q.alive ? A.nsteps : q.death_step + 1u - S.n0;
  t.steps += taken;
  t.sub += taken;
}

// ------------------------------------------------------------ FP64 path --
// Resolution state of an FP64 step whose sub-step proposal reached a vertex:
// the remaining time, the pending sub-step's normal (as drawn; a sub-step
// from a vertex folds it into the edge), the crossings so far and the last
// slot drawn.
struct Hit64 {
  double h, w;
  int32_t k, last;
};

// The canonical step in FP64, operation for operation.
template <bool TRACE, bool LDS, int GEN>
struct Particle64 {
  using real = double;
  GView G;
  uint32_t *s_exit;
  int32_t e;
  double x;
  EdgeRec64 R;
  bool alive;
  uint64_t hash;
  uint32_t nhit;
  uint32_t death_step;

  __device__ static void box_muller(uint32_t a, uint32_t b, double &c, double &s) {
    box_muller64(a, b, c, s);
  }

  // FP64 positions are always measured from the initial vertex.
  __device__ __forceinline__ void reanchor() {}
  __device__ __forceinline__ void reanchor_if(bool) {}
  __device__ __forceinline__ bool fast_first(double w) { return fast(w); }
  __device__ __forceinline__ double pos64(double) const { return x; }

  // Window preparation of the wave pools: only a window's first active step
  // can start on a vertex (every step that stays inside an edge ends
  // strictly inside it), where the normal points into the edge.
  template <int N>
  __device__ __forceinline__ void prep_window(double (&W)[N], uint32_t jb, bool on = true) const {
    if (on && (x == 0.0 || x == R.L)) {
      const bool init = x == 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i)
        W[i] = (jb == (uint32_t)i) ? (init ? fabs(W[i]) : -fabs(W[i])) : W[i];
    }
  }

  // Drift and diffusion at x: affine and constant, or with GEN the cubics
  // by Horner's rule (with zero higher terms these equal the affine values
  // exactly).
  // A tabulated edge (GEN): its interval at x (the last one at x = L) and
  // the local coordinate t = x K / L - j.
  __device__ __forceinline__ const TabRec64 &interval(double at, double &t) const {
    const double s = at * R.inv_h;
    double j = floor(s);
    j = j < 0.0 ? 0.0 : (j > (double)(R.tab_k - 1) ? (double)(R.tab_k - 1) : j);
    t = s - j;
    return G.tab64[R.tab0 + (int32_t)j];
  }
  __device__ __forceinline__ double drift(double at) const {
    if (!GEN) return fma(R.c, at, R.a);
    if (GEN == kGenFull && R.tab_k) {
      double t;
      const TabRec64 &T = interval(at, t);
      return fma(fma(fma(T.mu[3], t, T.mu[2]), t, T.mu[1]), t, T.mu[0]);
    }
    return fma(fma(fma(R.c3, at, R.c2), at, R.c), at, R.a);
  }
  __device__ __forceinline__ double diffusion(double at) const {
    if (!GEN) return R.sigma;
    if (GEN == kGenFull && R.tab_k) {
      double t;
      const TabRec64 &T = interval(at, t);
      return fma(fma(fma(T.sg[3], t, T.sg[2]), t, T.sg[1]), t, T.sg[0]);
    }
    return fma(fma(fma(R.s3, at, R.s2), at, R.s1), at, R.sigma);
  }

  // GEN: the particle sits on a Wentzell vertex (x <= 0 at the initial
  // end, x >= L at the terminal one; a particle that owes a stay there
  // holds -t or L + t).  Its step starts with a visit, in resolve().
  __device__ __forceinline__ bool on_wentzell() const {
    if constexpr (GEN != kGenFull) return false;
    return (x <= 0.0 && ((uint32_t)R.vinit & kWentzellEnd)) ||
           (x >= R.L && ((uint32_t)R.vterm & kWentzellEnd));
  }

  __device__ __forceinline__ void die(int32_t v, uint32_t step, const SetDev &S) {
    alive = false;
    death_step = step;
    atomicAdd((unsigned long long *)&S.absorbed[v], 1ull);
    if (TRACE) hash = fnv(fnv(hash, step), 0x80000000u | (uint32_t)v);
  }

  __device__ __forceinline__ bool fast(double w) {
    if (on_wentzell()) return false;
    if (x == 0.0)
      w = fabs(w);
    else if (x == R.L)
      w = -fabs(w);
    const double mu = drift(x);
    const double g = diffusion(x) * sqrt(dtv);
    const double xt = fma(g, w, fma(mu, dtv, x));
    if (xt > 0.0 && xt < R.L) {
      x = xt;
      return true;
    }
    return false;
  }

  // The same first sub-step as straight-line code (the wave pools): applied
  // only where `active`; returns whether the proposal stays inside the edge
  // (a step that starts on a Wentzell vertex never does: it is parked for
  // its visit).  The normal is already folded where the step starts on a
  // vertex (prep_window).
  __device__ __forceinline__ bool fast_pred(double w, bool active) {
    const double mu = drift(x);
    const double g = diffusion(x) * sqdt;
    const double xt = fma(g, w, fma(mu, dtv, x));
    const bool in = (xt > 0.0) & (xt < R.L) & !on_wentzell();
    x = (active & in) ? xt : x;
    return in;
  }

  double dtv;
  double sqdt;  // sqrt(dtv)

  // One vertex crossing of a step whose pending sub-step proposal (normal
  // H.w over the remaining time H.h; the step's first sub-step when
  // H.k == 0) reached a vertex: crossing time, edge draw, and the next
  // sub-step's proposal.  Returns true when the step is complete (inside an
  // edge, absorbed, out of time or at the split cap), false when the next
  // proposal reaches a vertex again.  resolve() loops over it; the wave
  // pools run one crossing per lane per pass.  A step that starts on a
  // Wentzell vertex begins here with its visit.
  __device__ bool cross(uint32_t step, Hit64 &H, uint32_t pid, const SetDev &S,
                        const StepArgs &A, Tally &t) {
    double h = H.h;
    bool left_visit = false;  // the move that leaves a start-of-step visit
    if (H.k == 0 && on_wentzell()) {
      // a step that starts on a Wentzell vertex: the stay owed there first,
      // then the visit that leaves it (its own local time only, o = 0); a
      // step spent on the vertex, or ended by the visit's killing, has no
      // move (its one sub-step is counted with the step)
      const bool init = x <= 0.0;
      const int32_t v = (init ? R.vinit : R.vterm) & kVertexMask;
      double owe = init ? -x : x - R.L;
      if (owe >= h) {
        owe = owe - h;
        x = init ? -owe : R.L + owe;
        return true;
      }
      h = h - owe;
      x = init ? 0.0 : R.L;
      double hm, owed;
      if (wz_visit(G.wz[G.vtx[v].wz - 1u], 0.0, h, vertex_draw(pid, step, 0u, S, A), hm, owed)) {
        die(v, step, S);
        return true;
      }
      if (hm == 0.0) {
        x = init ? -owed : R.L + owed;
        return true;
      }
      h = hm;
      H.h = h;
      left_visit = true;
    }
    // the pending proposal, recomputed as it was made
    double w = H.w;
    if (x == 0.0)
      w = fabs(w);
    else if (x == R.L)
      w = -fabs(w);
    const double mu = drift(x);
    const double g = diffusion(x) * sqrt(h);
    const double xt = fma(g, w, fma(mu, h, x));
    bool done = false;
    if (left_visit && xt > 0.0 && xt < R.L) {
      x = xt;
      return true;
    }
    const bool at_init = xt <= 0.0;
    const int32_t vr = at_init ? R.vinit : R.vterm;
    // reflecting leaf: the mirror image ends the step if it lies inside
    // the edge
    const double xr = at_init ? -xt : 2.0 * R.L - xt;
    if (vr < 0 && xr > 0.0 && xr < R.L) {
      x = xr;
      done = true;
    } else {
      const int32_t v = vr & kVertexMask;
      const double d = at_init ? x : R.L - x;
      const double qa = at_init ? mu * h : -(mu * h);
      const double qb = at_init ? g * w : -(g * w);
      const double u = first_root64(qa, qb, d);
      const double alpha = u * u;
      h = fma(-alpha, h, h);
      ++H.k;
      ++nhit;
      t.hits++;
      const VtxBlk vb = G.vtx[v];
      // a Wentzell vertex: the visit this hit starts, its overshoot being
      // how far past the vertex the proposal went
      double h_move = h, owed = 0.0;
      bool killed = false;
      if (GEN == kGenFull && vb.wz) {
        const double o = at_init ? -xt : xt - R.L;
        killed = wz_visit(G.wz[vb.wz - 1u], o, h, vertex_draw(pid, step, (uint32_t)H.k, S, A),
                          h_move, owed);
      }
      if (vb.deg < 0 || killed) {  // absorbing vertex, or killed at the visit
        if (TRACE) trace_hit(S, pid, step, H.k, v, -1, u, h);
        die(v, step, S);
        return true;
      }
      uint32_t k0 = A.key0, k1 = A.key1;
      fresh_keys<double>(k0, k1);
      const U4 hd = philox(pid, step, (uint32_t)H.k, S.tag, k0, k1);
      const SlotPick sp = pick_slot(G, vb, hd.x);
      e = eo_edge(sp.eo);
      R = G.e64[e];
      x = (sp.eo & 1u) ? R.L : 0.0;
      H.last = sp.s;
      if (TRACE) {
        hash = fnv(fnv(hash, step), (uint32_t)sp.s);
        trace_hit(S, pid, step, H.k, v, sp.s, u, h);
      }
      if (GEN == kGenFull && vb.wz) {
        h = h_move;
        if (h == 0.0) {  // stays on the vertex for the rest of the step
          x = (sp.eo & 1u) ? R.L + owed : -owed;
          done = true;
        }
      }
      if (!done) done = h == 0.0;
      if (!done && H.k == A.max_splits) {
        t.trunc++;
        done = true;
      }
      if (!done) {
        // the next sub-step, from the vertex (normal folded into the edge)
        H.w = box_muller64_cos(hd.y, hd.z);
        H.h = h;
        const double w2 = (sp.eo & 1u) ? -fabs(H.w) : fabs(H.w);
        const double mu2 = drift(x);
        const double g2 = diffusion(x) * sqrt(h);
        const double xt2 = fma(g2, w2, fma(mu2, h, x));
        t.sub++;
        if (xt2 > 0.0 && xt2 < R.L) {
          x = xt2;
          done = true;
        }
      }
    }
    if (done && H.k > 0) count_exit<LDS>(s_exit, S.exit_cnt, H.last);
    return done;
  }

  __device__ void resolve(uint32_t step, double w, uint32_t pid, const SetDev &S,
                          const StepArgs &A, Tally &t) {
    Hit64 H{dtv, w, 0, -1};
    while (!cross(step, H, pid, S, A, t)) {
    }
  }
};

template <bool TRACE, bool LDS, bool OBS, int NG, int GEN>
__device__ void run64(const GView &G, int32_t n_edges, const SetDev &S, const StepArgs &A,
                      uint32_t pid, uint32_t *s_exit, Tally &t, const ObsSink &o) {
  const uint32_t ef = S.ef[pid];
  if (ef & kDeadBit) return;
  const int32_t e = (int32_t)(ef & kEdgeMask);
  if (e >= n_edges) {
    atomicOr(S.err, kErrEdge);
    return;
  }
  Particle64<TRACE, LDS, GEN> q{G, s_exit, e, S.x64[pid], G.e64[e], true,
                           TRACE ? S.seqhash[pid] : 0ull, TRACE ? S.hits[pid] : 0u,
                           0u, A.dt, sqrt(A.dt)};
  if (!((q.x >= 0.0 && q.x <= q.R.L) || q.on_wentzell())) {
    atomicOr(S.err, kErrPos);
    return;
  }
  step_loop<NG, OBS>(q, S, A, pid, t, o);
  S.ef[pid] = (uint32_t)q.e | (q.alive ? 0u : kDeadBit);
  S.x64[pid] = q.x;
  if (TRACE) {
    S.seqhash[pid] = q.hash;
    S.hits[pid] = q.nhit;
  }
}

// ------------------------------------------------------------ FP32 path --
// Same step; the position is y = distance from the reference end (bit 30
// of the state word).  The reference end is re-chosen as the nearer end
// after every step that closes a Philox group (step index = 3 mod 4, in
// every schedule alike), so points near a vertex keep full relative
// precision.  In that
// frame the drift is as + c y with as = a (from the initial end) or
// -(a + c L) (from the terminal end), and the normal's sign flips with the
// end.  The position is a compensated pair (y, yl): each move adds its
// increment, computed at the increment's own magnitude, with the rounding
// error of the sum carried in yl (Fast2Sum, Dekker), so positions do not
// collect one rounding of y per step.  The remaining time is a compensated
// pair (hh, hl) too; the crossing solve runs in FP64 when the particle is
// within 1e-6 L of the vertex but not on it (on it the root is one
// division).
struct Edge32 {
  float L, a, c, sigma, aL;
  int32_t vinit, vterm;
};

__device__ __forceinline__ Edge32 load_edge32(const EdgeRec32 *e32, int32_t e) {
  const EdgeRec32 r = e32[e];
  return {r.L, r.a, r.c, r.sigma, r.aL, r.vinit, r.vterm};
}

// Resolution state of an FP32 step whose sub-step reached a vertex:
// remaining time (compensated pair), the pending sub-step's normal, the
// crossings so far and the last slot drawn.
struct Hit32 {
  float hh, hl, w;
  int32_t k, last;
};

// GEN: the graph has a general method variant.  Higher coefficient terms
// (cubic drift or diffusion): the first sub-step evaluates them at the
// particle's position instead of using the per-frame affine constants.
// Wentzell vertices: a step that starts on one begins with a visit (in
// cross()), and a hit there is a visit too; a particle that owes a stay on
// the vertex holds y = -t in the frame of that end.
template <bool TRACE, bool LDS, int GEN = 0>
struct Particle32 {
  using real = float;
  GView G;
  uint32_t *s_exit;
  int32_t e;
  uint32_t side;
  float y, yl;    // distance from the reference end, compensation term
  Edge32 R;
  float as, g0;   // drift constant in the local frame, sigma sqrt(dt)
  float dt, sqdt;
  bool alive;
  uint64_t hash;
  uint32_t nhit;
  uint32_t death_step;
  // First sub-step constants of the current edge and frame: c dt, as dt and
  // g0 with the frame's sign, so that a first sub-step is
  // y + fma(gs, w, fma(cd, y, ad)) with no per-step sign select.
  float cd = 0.0f, ad = 0.0f, gs = 0.0f;
  // Higher terms of the current edge (GEN), x from the initial vertex:
  // drift + c2 x^2 + c3 x^3, diffusion + s1 x + s2 x^2 + s3 x^3.
  float c2 = 0.0f, c3 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  // A tabulated edge (GEN): intervals per unit length and the first
  // interval's row (tab_k = 0: no table).
  float inv_h = 0.0f;
  int32_t tab0 = 0, tab_k = 0;

  // Sets as, g0 and the first sub-step constants for the current edge R and
  // side (after an edge load or a change of reference end).
  __device__ __forceinline__ void frame() {
    as = side ? -R.aL : R.a;
    g0 = R.sigma * sqdt;
    cd = R.c * dt;
    ad = as * dt;
    gs = side ? -g0 : g0;
    if constexpr (GEN) {
      const EdgeRec64 &P = G.hi64[e];
      c2 = (float)P.c2;
      c3 = (float)P.c3;
      s1 = (float)P.s1;
      s2 = (float)P.s2;
      s3 = (float)P.s3;
      if constexpr (GEN == kGenFull) {
        inv_h = (float)P.inv_h;
        tab0 = P.tab0;
        tab_k = P.tab_k;
      }
    }
  }

  // A tabulated edge's interval at x from the initial vertex (the last one
  // at x = L) and the local coordinate t.
  __device__ __forceinline__ const TabRec32 &interval(float x, float &t) const {
    const float s = x * inv_h;
    float j = floorf(s);
    j = j < 0.0f ? 0.0f : (j > (float)(tab_k - 1) ? (float)(tab_k - 1) : j);
    t = s - j;
    return G.tab32[tab0 + (int32_t)j];
  }

  // Drift in the frame (sign of the reference end) and diffusion at
  // distance yy from the reference end.
  __device__ __forceinline__ float fdrift(float yy) const {
    if constexpr (!GEN) {
      return fmaf(R.c, yy, as);
    } else {
      const float x = side ? R.L - yy : yy;
      float m;
      if (GEN == kGenFull && tab_k) {
        float t;
        const TabRec32 &T = interval(x, t);
        m = fmaf(fmaf(fmaf(T.mu[3], t, T.mu[2]), t, T.mu[1]), t, T.mu[0]);
      } else {
        m = fmaf(fmaf(fmaf(c3, x, c2), x, R.c), x, R.a);
      }
      return side ? -m : m;
    }
  }
  __device__ __forceinline__ float fsigma(float yy) const {
    if constexpr (!GEN) {
      return R.sigma;
    } else {
      const float x = side ? R.L - yy : yy;
      if (GEN == kGenFull && tab_k) {
        float t;
        const TabRec32 &T = interval(x, t);
        return fmaf(fmaf(fmaf(T.sg[3], t, T.sg[2]), t, T.sg[1]), t, T.sg[0]);
      }
      return fmaf(fmaf(fmaf(s3, x, s2), x, s1), x, R.sigma);
    }
  }

  __device__ static void box_muller(uint32_t a, uint32_t b, float &c, float &s) {
    box_muller32(a, b, c, s);
  }

  // y + s as a compensated sum (Fast2Sum: exact error when |y| >= |s|,
  // a bounded one otherwise, which happens only within one step of the
  // reference end): returns the rounded sum, err its error.
  __device__ __forceinline__ float add_comp(float s, float &err) const {
    const float yt = y + s;
    err = s - (yt - y);
    return yt;
  }

  // Position from the initial vertex in FP64, as the histogram reads it.
  __device__ __forceinline__ double pos64(double L) const {
    const double v = (double)y + (double)yl;
    return side ? L - v : v;
  }

  // Re-anchor to the nearer end: L - y is exact for y in [L/2, L)
  // (Sterbenz), so the move loses nothing; the compensation flips sign.
  __device__ __forceinline__ void reanchor() {
    reanchor_if(true);
  }
  __device__ __forceinline__ void reanchor_if(bool cond) {
    const bool flip = cond & (y > 0.5f * R.L);
    y = flip ? R.L - y : y;
    yl = flip ? -yl : yl;
    side ^= flip ? 1u : 0u;
    as = flip ? (side ? -R.aL : R.a) : as;
    ad = flip ? as * dt : ad;
    gs = flip ? -gs : gs;
  }

  // GEN: the particle sits on a Wentzell vertex, its reference end (y <= 0:
  // on the vertex, or owing a stay of -y there).
  __device__ __forceinline__ bool on_wentzell() const {
    if constexpr (GEN != kGenFull) return false;
    return y <= 0.0f && ((uint32_t)(side ? R.vterm : R.vinit) & kWentzellEnd);
  }
  // The particle stays on its reference end, a Wentzell vertex, owing a
  // further stay of t there (y = -t as a compensated pair).
  __device__ __forceinline__ void owe_stay(double t) {
    const double yd = -t;
    y = (float)yd;
    yl = (float)(yd - (double)y);
  }
  __device__ __forceinline__ void die(int32_t v, uint32_t step, const SetDev &S) {
    alive = false;
    death_step = step;
    atomicAdd((unsigned long long *)&S.absorbed[v], 1ull);
    if (TRACE) hash = fnv(fnv(hash, step), 0x80000000u | (uint32_t)v);
  }

  // The normal a first sub-step from y = 0 uses: a particle on a vertex
  // moves into its edge, so the noise term is g0 |w| (gs carries the frame's
  // sign, hence |w| with that sign).
  __device__ __forceinline__ float at_vertex(float w) const {
    return copysignf(fabsf(w), gs);
  }
  // A step's first sub-step over dt with normal w; w must already be
  // at_vertex(w) when y = 0.  Returns the proposal and its compensation.
  __device__ __forceinline__ float propose(float w, float &err) const {
    if constexpr (!GEN) {
      return add_comp(fmaf(gs, w, fmaf(cd, y, ad)) + yl, err);
    } else {
      const float sg = fsigma(y) * sqdt;
      return add_comp(fmaf(side ? -sg : sg, w, fdrift(y) * dt) + yl, err);
    }
  }

  // Window preparation of the step loop: the first active step of a window
  // is the only one that can start on a vertex.
  template <int N>
  __device__ __forceinline__ void prep_window(float (&W)[N], uint32_t jb, bool on = true) const {
    if (on && y == 0.0f) {
#pragma unroll
      for (int i = 0; i < N; ++i) W[i] = (jb == (uint32_t)i) ? at_vertex(W[i]) : W[i];
    }
  }
  // First sub-step of a window's first active step after prep_window.
  __device__ __forceinline__ bool fast_first(float w) {
    if (on_wentzell()) return false;
    float err;
    const float yt = propose(w, err);
    if (yt > 0.0f && yt < R.L) {
      y = yt;
      yl = err;
      return true;
    }
    return false;
  }

  __device__ __forceinline__ bool fast(float w) {
    if (on_wentzell()) return false;
    float err;
    const float yt = propose((y == 0.0f) ? at_vertex(w) : w, err);
    if (yt > 0.0f && yt < R.L) {
      y = yt;
      yl = err;
      return true;
    }
    return false;
  }

  // First sub-step as straight-line code: applied only where `active`;
  // returns whether the proposal stays inside the edge.  No y = 0 check:
  // y is positive after every step that stays inside an edge, so only a
  // group's first active step can start on a vertex, and the caller passes
  // at_vertex(w) for it.
  __device__ __forceinline__ bool fast_pred(float w, bool active) {
    float err;
    const float yt = propose(w, err);
    const bool in = (yt > 0.0f) & (yt < R.L) & !on_wentzell();
    const bool upd = active & in;
    y = upd ? yt : y;
    yl = upd ? err : yl;
    return in;
  }

  // One vertex crossing of a step whose current sub-step proposal (normal
  // h.w over the remaining time h.hh + h.hl; the step's first sub-step when
  // h.k == 0) reached a vertex: crossing time, edge draw, and the next
  // sub-step's proposal.  Returns true when the step is complete (inside an
  // edge, absorbed, out of time or at the split cap), false when the next
  // proposal reaches a vertex again.  resolve() loops over it; the wave
  // pools run one crossing per lane per pass.
  __device__ bool cross(uint32_t step, Hit32 &h, uint32_t pid, const SetDev &S,
                        const StepArgs &A, Tally &t) {
    float hh = h.hh, hl = h.hl;
    // the pending sub-step is the step's first, over dt (else over hh + hl)
    bool first = h.k == 0;
    if (first && on_wentzell()) {
      // a step that starts on a Wentzell vertex: the stay owed there first,
      // then the visit that leaves it (o = 0); a step spent on the vertex,
      // or ended by the visit's killing, has no move
      const int32_t v = (side ? R.vterm : R.vinit) & kVertexMask;
      double hd = (double)hh + (double)hl;
      const double owe = -((double)y + (double)yl);
      if (owe >= hd) {
        owe_stay(owe - hd);
        return true;
      }
      hd = hd - owe;
      y = 0.0f;
      yl = 0.0f;
      double hm, owed;
      if (wz_visit(G.wz[G.vtx[v].wz - 1u], 0.0, hd, vertex_draw(pid, step, 0u, S, A), hm,
                   owed)) {
        die(v, step, S);
        return true;
      }
      if (hm == 0.0) {
        owe_stay(owed);
        return true;
      }
      hh = (float)hm;
      hl = (float)(hm - (double)hh);
      h.hh = hh;
      h.hl = hl;
      first = false;
    }
    // the pending proposal, recomputed as it was made
    // (the first sub-step's exactly as propose() made it: g0 we = gs w)
    const float we = (y == 0.0f) ? fabsf(h.w) : (side ? -h.w : h.w);
    const float mu = fdrift(y);
    const float g = first ? (GEN ? fsigma(y) * sqdt : g0)
                          : fsigma(y) * __builtin_amdgcn_sqrtf(hh);
    const float mdt = first ? (GEN ? mu * dt : fmaf(cd, y, ad)) : mu * hh;
    float err;
    const float yt = add_comp(fmaf(g, we, mdt) + yl, err);
    // the move that leaves a start-of-step visit need not reach a vertex
    if (GEN == kGenFull && h.k == 0 && !first && yt > 0.0f && yt < R.L) {
      y = yt;
      yl = err;
      return true;
    }
    const bool near = yt <= 0.0f;
    const bool at_term = near == (side != 0u);
    const int32_t vr = at_term ? R.vterm : R.vinit;
    // reflecting leaf: the mirror image, as a distance from the hit end
    // (-(yt + err) at the reference end; (yt - L) + err at the other, where
    // yt - L is exact for yt <= 2L), renormalised by TwoSum; it ends the
    // step when it lies inside the edge
    const float r0 = near ? -yt : yt - R.L;
    const float r1 = near ? -err : err;
    const float rs = r0 + r1;
    const float rb = rs - r0;
    const float re = (r0 - (rs - rb)) + (r1 - rb);
    bool done;
    if (vr < 0 && rs > 0.0f && rs < R.L) {
      y = rs;
      yl = re;
      if (!near) {
        side ^= 1u;
        frame();
      }
      done = true;
    } else {
      const int32_t v = vr & kVertexMask;
      const float dn = y + yl;
      const float d = fmaxf(near ? dn : (R.L - y) - yl, 0.0f);
      float u;
      if (d > 0.0f && d < G.e32[e].near) {
        // crossing solve in FP64 next to the vertex (on the vertex itself,
        // d = 0, the root is -B/A: one division, no cancellation)
        const double hd = (double)hh + (double)hl;
        const double mud = GEN ? (double)mu : fma((double)R.c, (double)y, (double)as);
        const double gd = (double)fsigma(y) * sqrt(hd);
        const double qa = near ? mud * hd : -(mud * hd);
        const double qb = near ? gd * (double)we : -(gd * (double)we);
        const double yd = (double)y + (double)yl;
        const double dd = fmax(near ? yd : (double)R.L - yd, 0.0);
        u = (float)first_root64(qa, qb, dd);
      } else {
        const float gw = g * we;
        u = first_root32(near ? mdt : -mdt, near ? gw : -gw, d);
      }
      // remaining time (1 - u^2)(hh + hl), compensated (TwoProduct by fma,
      // TwoSum, renormalised)
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
      h.hh = hh;
      h.hl = hl;
      ++h.k;
      ++nhit;
      t.hits++;
      const VtxBlk vb = G.vtx[v];
      // a Wentzell vertex: the visit this hit starts, with the proposal's
      // overshoot past the vertex
      double hm = 0.0, owed = 0.0;
      bool killed = false;
      if (GEN == kGenFull && vb.wz)
        killed = wz_visit(G.wz[vb.wz - 1u], (double)r0 + (double)r1,
                          (double)hh + (double)hl, vertex_draw(pid, step, (uint32_t)h.k, S, A),
                          hm, owed);
      if (vb.deg < 0 || killed) {
        if (TRACE) trace_hit(S, pid, step, h.k, v, -1, u, (double)hh + (double)hl);
        die(v, step, S);
        return true;
      }
      const U4 hd = philox(pid, step, (uint32_t)h.k, S.tag, A.key0, A.key1);
      const SlotPick sp = pick_slot(G, vb, hd.x);
      e = eo_edge(sp.eo);
      R = load_edge32(G.e32, e);
      side = sp.eo & 1u;
      y = 0.0f;
      yl = 0.0f;
      frame();
      h.last = sp.s;
      if (TRACE) {
        hash = fnv(fnv(hash, step), (uint32_t)sp.s);
        trace_hit(S, pid, step, h.k, v, sp.s, u, (double)hh + (double)hl);
      }
      bool stays = false;
      if (GEN == kGenFull && vb.wz) {
        if (hm == 0.0) {  // stays on the vertex for the rest of the step
          owe_stay(owed);
          stays = true;
        } else {
          hh = (float)hm;
          hl = (float)(hm - (double)hh);
          h.hh = hh;
          h.hl = hl;
        }
      }
      done = stays || hh == 0.0f;
      if (!done && h.k == A.max_splits) {
        t.trunc++;
        done = true;
      }
      if (!done) {
        // the next sub-step, from the vertex (normal folded into the edge)
        h.w = box_muller32_cos(hd.y, hd.z);
        const float mu2 = fdrift(y);
        const float g2 = fsigma(y) * __builtin_amdgcn_sqrtf(hh);
        float err2;
        const float yt2 = add_comp(fmaf(g2, fabsf(h.w), mu2 * hh) + yl, err2);
        t.sub++;
        if (yt2 > 0.0f && yt2 < R.L) {
          y = yt2;
          yl = err2;
          done = true;
        }
      }
    }
    if (done && h.k > 0) count_exit<LDS>(s_exit, S.exit_cnt, h.last);
    return done;
  }

  __device__ void resolve(uint32_t step, float w, uint32_t pid, const SetDev &S,
                          const StepArgs &A, Tally &t) {
    Hit32 h{dt, 0.0f, w, 0, -1};
    while (!cross(step, h, pid, S, A, t)) {
    }
  }
};

template <bool TRACE, bool LDS, bool OBS, int NG, int GEN>
__device__ void run32(const GView &G, int32_t n_edges, const SetDev &S, const StepArgs &A,
                      uint32_t pid, uint32_t *s_exit, Tally &t, const ObsSink &o) {
  const uint32_t ef = S.ef[pid];
  if (ef & kDeadBit) return;
  const int32_t e = (int32_t)(ef & kEdgeMask);
  if (e >= n_edges) {
    atomicOr(S.err, kErrEdge);
    return;
  }
  const float sqdt = (float)sqrt(A.dt);
  const Edge32 R = load_edge32(G.e32, e);
  const uint32_t side = (ef & kSideBit) ? 1u : 0u;
  const float2 yy = S.y32[pid];
  Particle32<TRACE, LDS, GEN> q{G, s_exit, e, side, yy.x, yy.y, R,
                           side ? -R.aL : R.a, R.sigma * sqdt, (float)A.dt, sqdt, true,
                           TRACE ? S.seqhash[pid] : 0ull, TRACE ? S.hits[pid] : 0u, 0u};
  q.frame();
  if (!((q.y >= 0.0f && q.y <= R.L) || q.on_wentzell())) {
    atomicOr(S.err, kErrPos);
    return;
  }
  step_loop<NG, OBS>(q, S, A, pid, t, o);
  S.ef[pid] = (uint32_t)q.e | (q.side ? kSideBit : 0u) | (q.alive ? 0u : kDeadBit);
  S.y32[pid] = make_float2(q.y, q.yl);
  if (TRACE) {
    S.seqhash[pid] = q.hash;
    S.hits[pid] = q.nhit;
  }
}

// Block-level reduction of the lane tallies (into the 64-bit LDS totals,
// to which the wave pools' periodic drains have already added) and the LDS
// exit counters.
__device__ __forceinline__ void flush(const SetDev &S, const Tally &t,
                                      unsigned long long *s_tot, uint32_t *s_exit,
                                      int32_t nnz, bool lds) {
  if (t.trunc) atomicAdd(&s_tot[0], (unsigned long long)t.trunc);
  if (t.sub) atomicAdd(&s_tot[1], (unsigned long long)t.sub);
  if (t.hits) atomicAdd(&s_tot[2], (unsigned long long)t.hits);
  if (t.steps) atomicAdd(&s_tot[3], (unsigned long long)t.steps);
  __syncthreads();
  if (threadIdx.x < 4 && s_tot[threadIdx.x])
    atomicAdd((unsigned long long *)&S.totals[threadIdx.x], s_tot[threadIdx.x]);
  if (lds) {
    for (int32_t s = threadIdx.x; s < nnz; s += blockDim.x)
      if (s_exit[s]) atomicAdd((unsigned long long *)&S.exit_cnt[s],
                               (unsigned long long)s_exit[s]);
  }
}

// Adds a block's LDS snapshot bins to the set's counters (after the
// barrier in flush()).
__device__ __forceinline__ void flush_obs(const SetDev &S, const uint32_t *s_obs,
                                          int32_t nbins) {
  for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x)
    if (s_obs[b]) atomicAdd((unsigned long long *)&S.obs[b], (unsigned long long)s_obs[b]);
}

__device__ __forceinline__ int32_t align16(int32_t v) { return (v + 15) & ~15; }

// Shared memory of a step block: [exit counters (LDS)][staged tables]
// [snapshot bins (LDS)].
// Staged tables keep their relative layout: vertex blocks, slot table and
// guide tables, then the edge records of the kernel's precision.
template <bool FP64, bool STAGED>
__device__ __forceinline__ GView block_view(const GraphDev &G, char *smem) {
  if (!STAGED) return global_view(G);
  const int32_t bytes = FP64 ? G.stage_bytes64 : G.stage_bytes32;
  const int32_t head = G.o_e32;
  const uint4 *src_head = (const uint4 *)G.tables;
  const uint4 *src_edge = (const uint4 *)(G.tables + (FP64 ? G.o_e64 : G.o_e32));
  uint4 *dst = (uint4 *)smem;
  for (int32_t i = threadIdx.x; i < head / 16; i += blockDim.x) dst[i] = src_head[i];
  for (int32_t i = threadIdx.x; i < (bytes - head) / 16; i += blockDim.x)
    dst[head / 16 + i] = src_edge[i];
  GView v;
  v.vtx = (const VtxBlk *)(smem + G.o_vtx);
  v.slots = (const SlotRec8 *)(smem + G.o_slots);
  v.guide = (const int32_t *)(smem + G.o_guide);
  v.e32 = (const EdgeRec32 *)(smem + head);
  v.e64 = (const EdgeRec64 *)(smem + head);
  v.hi64 = G.e64;
  v.wz = G.wz;
  v.tab64 = G.tab64;
  v.tab32 = G.tab32;
  return v;
}

__device__ __forceinline__ int32_t exit_bytes(int32_t nnz) { return ((nnz * 4) + 15) & ~15; }

template <bool FP64, bool TRACE, bool LDS, bool STAGED, bool OBS, int GEN>
__device__ __forceinline__ void step_block(const GraphDev &G, const SetDev &S,
                                           const StepArgs &A, uint32_t pid,
                                           unsigned long long *s_tot, char *smem) {
  uint32_t *s_exit = (uint32_t *)smem;
  if (threadIdx.x < 4) s_tot[threadIdx.x] = 0;
  if (LDS)
    for (int32_t s = threadIdx.x; s < G.nnz; s += blockDim.x) s_exit[s] = 0;
  const int32_t ex = LDS ? exit_bytes(G.nnz) : 0;
  const GView view = block_view<FP64, STAGED>(G, smem + ex);
  ObsSink o{nullptr, G.e64};
  if (OBS && A.obs_lds) {
    o.lds = (uint32_t *)(smem + align16(ex + (STAGED ? (FP64 ? G.stage_bytes64
                                                             : G.stage_bytes32) : 0)));
    for (int32_t b = threadIdx.x; b < A.obs_lds; b += blockDim.x) o.lds[b] = 0;
  }
  __syncthreads();
  Tally t{0, 0, 0, 0};
  if (pid < S.n) {
    if (FP64)
      run64<TRACE, LDS, OBS, kWindowGroups64, GEN>(view, G.E, S, A, pid, s_exit, t, o);
    else
      run32<TRACE, LDS, OBS, kWindowGroups32, GEN>(view, G.E, S, A, pid, s_exit, t, o);
  }
  flush(S, t, s_tot, s_exit, G.nnz, LDS);
  if (OBS && A.obs_lds) flush_obs(S, o.lds, A.obs_lds);
}

// GEN: some edge has higher drift or diffusion terms (FP32: lane schedule only).
template <bool FP64, bool TRACE, bool LDS, bool STAGED, bool OBS, int GEN>
__global__ __launch_bounds__(kBlock) void k_step(GraphDev G, SetDev S, StepArgs A) {
  extern __shared__ uint4 smem4[];
  __shared__ unsigned long long s_tot[4];
  step_block<FP64, TRACE, LDS, STAGED, OBS, GEN>(G, S, A, blockIdx.x * kBlock + threadIdx.x,
                                                  s_tot, (char *)smem4);
}

template <bool FP64, bool TRACE, bool LDS, bool STAGED, bool OBS, int GEN>
__global__ __launch_bounds__(kBlock) void k_batch(const GraphDev *graphs,
                                                  const SetDev *sets,
                                                  const BatchItem *items,
                                                  StepArgs A) {
  extern __shared__ uint4 smem4[];
  __shared__ unsigned long long s_tot[4];
  const BatchItem it = items[blockIdx.x];
  SetDev S = sets[it.set];
  S.n0 += A.n0_offset;  // steps already taken by earlier launches of this call
  const GraphDev G = graphs[it.set];
  step_block<FP64, TRACE, LDS, STAGED, OBS, GEN>(G, S, A, it.first + threadIdx.x, s_tot,
                                                  (char *)smem4);
}

// ------------------------------------------------ FP32 wave-pool kernel --
// Each wave owns PW particles (128 or 256): 64 ride in the lanes, the others
// wait in the wave's private LDS home slots.  A lane runs its particle's
// first sub-steps for one window (one or two main-stream Philox groups,
// four or eight steps) per iteration; a particle whose sub-step reaches a
// vertex is parked: its state
// goes to its home slot and its slot id onto the wave's split queue, and the
// lane takes a ready particle instead.  When 64 particles are parked (or
// lanes would idle), one split pass takes them with every lane busy and
// resolves one vertex crossing each: crossing time, Philox hit stream, slot
// draw and the next sub-step's proposal.  A particle whose step is then
// complete goes back on the ready queue (with its exit record); one whose
// proposal reaches a vertex again goes back on the split queue, so a pass
// never waits for the lane with the most crossings.  Each particle still
// consumes exactly the random numbers of its own (step, hit) counters, so the
// results equal the plain per-particle order bit for bit.  Waves never wait
// for one another: the queues and their counters are private to a wave.
constexpr int kWavesPerBlock = kBlock / 64;
#ifndef MG_POOL_CLAIM_MIN
#define MG_POOL_CLAIM_MIN 16
#endif
constexpr int kClaimMin = MG_POOL_CLAIM_MIN;  // free home slots that start a claim
static_assert((kClaimMin & (kClaimMin - 1)) == 0 && kClaimMin <= 64, "claim granularity");
// A batch work item stands for kBatchGens pools' worth of one set's
// particles per wave of a block: the number of items of a set, and so the
// number of blocks that may work on it at once, grows with its size.
constexpr int kBatchGens = 8;

template <bool TRACE, int PW>
struct PoolTrace {
  uint32_t hits[PW];
  uint64_t hash[PW];
};
template <int PW>
struct PoolTrace<false, PW> {};

// A wave's pool in LDS: home slots of its particles, the resolution state
// of parked steps, and the ready and split queues (slot ids).
template <bool TRACE, int PW>
struct PoolLds32 : PoolTrace<TRACE, PW> {
  static_assert(PW % 64 == 0 && PW <= 256, "slot ids are bytes");
  uint32_t ef[PW];
  float y[PW];
  float yl[PW];
  uint32_t n[PW];   // next step (ready) or the step to resolve (parked)
  float w[PW];      // normal of a parked step's pending sub-step
  float hh[PW];     // remaining time of a parked step (when k > 0)
  float hl[PW];
  int32_t last[PW]; // last slot drawn in the parked step
  uint32_t pid[PW];   // particle held by each home slot
  uint8_t k[PW];    // crossings so far in the parked step
  uint8_t ready[PW];
  uint8_t split[PW];
  uint8_t freeq[PW];  // home slots without a particle
};

// The same for FP64 particles: position from the initial vertex, and the
// parked step's normal and remaining time in FP64.
template <bool TRACE, int PW>
struct PoolLds64 : PoolTrace<TRACE, PW> {
  static_assert(PW % 64 == 0 && PW <= 256, "slot ids are bytes");
  uint32_t ef[PW];
  uint32_t n[PW];
  double x[PW];
  double w[PW];
  double h[PW];
  int32_t last[PW];
  uint32_t pid[PW];
  uint8_t k[PW];
  uint8_t ready[PW];
  uint8_t split[PW];
  uint8_t freeq[PW];
};

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// A wave's LDS instructions execute in issue order, so lanes of one wave
// may exchange data through LDS without waiting; only the compiler must not
// move the accesses across each other.
__device__ __forceinline__ void wave_lds_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

// Moving particles between registers, the pool's home slots and the set:
// one overload per precision.
template <bool TRACE, bool LDS, int GEN, int PW>
__device__ __forceinline__ void pool_load(Particle32<TRACE, LDS, GEN> &q,
                                          const PoolLds32<TRACE, PW> &P,
                                          uint32_t s) {
  const uint32_t ef = P.ef[s];
  q.e = (int32_t)(ef & kEdgeMask);
  q.side = (ef & kSideBit) ? 1u : 0u;
  q.y = P.y[s];
  q.yl = P.yl[s];
  q.R = load_edge32(q.G.e32, q.e);
  q.frame();
  q.alive = true;
  if constexpr (TRACE) {
    q.nhit = P.hits[s];
    q.hash = P.hash[s];
  }
}
template <bool TRACE, bool LDS, int GEN, int PW>
__device__ __forceinline__ void pool_load(Particle64<TRACE, LDS, GEN> &q,
                                          const PoolLds64<TRACE, PW> &P,
                                          uint32_t s) {
  q.e = (int32_t)(P.ef[s] & kEdgeMask);
  q.x = P.x[s];
  q.R = q.G.e64[q.e];
  q.alive = true;
  if constexpr (TRACE) {
    q.nhit = P.hits[s];
    q.hash = P.hash[s];
  }
}

template <bool TRACE, bool LDS, int GEN, int PW>
__device__ __forceinline__ void pool_store(const Particle32<TRACE, LDS, GEN> &q,
                                           PoolLds32<TRACE, PW> &P,
                                           uint32_t s, uint32_t n) {
  P.ef[s] = (uint32_t)q.e | (q.side ? kSideBit : 0u);
  P.y[s] = q.y;
  P.yl[s] = q.yl;
  P.n[s] = n;
  if constexpr (TRACE) {
    P.hits[s] = q.nhit;
    P.hash[s] = q.hash;
  }
}
template <bool TRACE, bool LDS, int GEN, int PW>
__device__ __forceinline__ void pool_store(const Particle64<TRACE, LDS, GEN> &q,
                                           PoolLds64<TRACE, PW> &P,
                                           uint32_t s, uint32_t n) {
  P.ef[s] = (uint32_t)q.e;
  P.x[s] = q.x;
  P.n[s] = n;
  if constexpr (TRACE) {
    P.hits[s] = q.nhit;
    P.hash[s] = q.hash;
  }
}

// A parked step's resolution state, to and from its home slot (a fresh
// park, k = 0, has the whole step left: dt, no slot drawn yet).
template <bool TRACE, int PW>
__device__ __forceinline__ Hit32 pool_hit(const PoolLds32<TRACE, PW> &P, uint32_t s,
                                          const StepArgs &A) {
  Hit32 h{(float)A.dt, 0.0f, P.w[s], (int32_t)P.k[s], -1};
  if (h.k > 0) {
    h.hh = P.hh[s];
    h.hl = P.hl[s];
    h.last = P.last[s];
  }
  return h;
}
template <bool TRACE, int PW>
__device__ __forceinline__ void pool_park(PoolLds32<TRACE, PW> &P, uint32_t s, const Hit32 &h) {
  P.w[s] = h.w;
  P.hh[s] = h.hh;
  P.hl[s] = h.hl;
  P.last[s] = h.last;
  P.k[s] = (uint8_t)h.k;
}
template <bool TRACE, int PW>
__device__ __forceinline__ Hit64 pool_hit(const PoolLds64<TRACE, PW> &P, uint32_t s,
                                          const StepArgs &A) {
  Hit64 h{A.dt, P.w[s], (int32_t)P.k[s], -1};
  if (h.k > 0) {
    h.h = P.h[s];
    h.last = P.last[s];
  }
  return h;
}
template <bool TRACE, int PW>
__device__ __forceinline__ void pool_park(PoolLds64<TRACE, PW> &P, uint32_t s, const Hit64 &h) {
  P.w[s] = h.w;
  P.h[s] = h.h;
  P.last[s] = h.last;
  P.k[s] = (uint8_t)h.k;
}

// Reads particle id from the set when a wave claims it: the state word
// and position go to home slot hs.  False for a removed particle, and for
// a corrupt state (the set's error word is raised).
template <bool TRACE, int PW, int GEN>
__device__ __forceinline__ bool pool_claim(const GView &G, const SetDev &S, int32_t n_edges,
                                           uint32_t id, PoolLds32<TRACE, PW> &P, uint32_t hs,
                                           bool mine) {
  bool ok = false;
  uint32_t ef = 0;
  float2 yy = make_float2(0.0f, 0.0f);
  if (mine) {
    ef = S.ef[id];
    yy = S.y32[id];
    const int32_t e = (int32_t)(ef & kEdgeMask);
    if (!(ef & kDeadBit)) {
      if (e >= n_edges) {
        atomicOr(S.err, kErrEdge);
      } else if (!((yy.x >= 0.0f && yy.x <= G.e32[e].L) ||
                   (GEN == kGenFull && yy.x < 0.0f &&
                    ((uint32_t)((ef & kSideBit) ? G.e32[e].vterm : G.e32[e].vinit) &
                     kWentzellEnd)))) {
        atomicOr(S.err, kErrPos);
      } else {
        ok = true;
      }
    }
  }
  if (ok) {
    P.ef[hs] = ef;
    P.y[hs] = yy.x;
    P.yl[hs] = yy.y;
  }
  return ok;
}
template <bool TRACE, int PW, int GEN>
__device__ __forceinline__ bool pool_claim(const GView &G, const SetDev &S, int32_t n_edges,
                                           uint32_t id, PoolLds64<TRACE, PW> &P, uint32_t hs,
                                           bool mine) {
  bool ok = false;
  uint32_t ef = 0;
  double x = 0.0;
  if (mine) {
    ef = S.ef[id];
    x = S.x64[id];
    const int32_t e = (int32_t)(ef & kEdgeMask);
    if (!(ef & kDeadBit)) {
      if (e >= n_edges) {
        atomicOr(S.err, kErrEdge);
      } else {
        const EdgeRec64 &r = G.e64[e];
        if (!((x >= 0.0 && x <= r.L) ||
              (GEN == kGenFull && ((x <= 0.0 && ((uint32_t)r.vinit & kWentzellEnd)) ||
                       (x >= r.L && ((uint32_t)r.vterm & kWentzellEnd)))))) {
          atomicOr(S.err, kErrPos);
        } else {
          ok = true;
        }
      }
    }
  }
  if (ok) {
    P.ef[hs] = ef;
    P.x[hs] = x;
  }
  return ok;
}

// Writes a particle back at the end of its launch and counts the steps it
// took (each has one first sub-step; resolve() counts the others).
template <bool TRACE, bool LDS, int GEN>
__device__ __forceinline__ void pool_finish(const Particle32<TRACE, LDS, GEN> &q, const SetDev &S,
                                            const StepArgs &A, uint32_t pid, Tally &t) {
  S.ef[pid] = (uint32_t)q.e | (q.side ? kSideBit : 0u) | (q.alive ? 0u : kDeadBit);
  S.y32[pid] = make_float2(q.y, q.yl);
  if (TRACE) {
    S.seqhash[pid] = q.hash;
    S.hits[pid] = q.nhit;
  }
  const uint32_t taken = q.alive ? A.nsteps : q.death_step + 1u - S.n0;
  t.steps += taken;
  t.sub += taken;
}
template <bool TRACE, bool LDS, int GEN>
__device__ __forceinline__ void pool_finish(const Particle64<TRACE, LDS, GEN> &q, const SetDev &S,
                                            const StepArgs &A, uint32_t pid, Tally &t) {
  S.ef[pid] = (uint32_t)q.e | (q.alive ? 0u : kDeadBit);
  S.x64[pid] = q.x;
  if (TRACE) {
    S.seqhash[pid] = q.hash;
    S.hits[pid] = q.nhit;
  }
  const uint32_t taken = q.alive ? A.nsteps : q.death_step + 1u - S.n0;
  t.steps += taken;
  t.sub += taken;
}

// A particle of the pool loop, before its first pickup: the graph view,
// exit counters and the launch's dt.
template <bool TRACE, bool LDS, int GEN>
__device__ __forceinline__ void pool_particle(Particle32<TRACE, LDS, GEN> &q, const GView &G,
                                              uint32_t *s_exit, const StepArgs &A) {
  q = Particle32<TRACE, LDS, GEN>{G, s_exit, 0, 0u, 0.0f, 0.0f, Edge32{}, 0.0f, 0.0f,
                                  (float)A.dt, (float)sqrt(A.dt), true, 0ull, 0u, 0u};
}
template <bool TRACE, bool LDS, int GEN>
__device__ __forceinline__ void pool_particle(Particle64<TRACE, LDS, GEN> &q, const GView &G,
                                              uint32_t *s_exit, const StepArgs &A) {
  q = Particle64<TRACE, LDS, GEN>{G, s_exit, 0, 0.0, EdgeRec64{}, true, 0ull, 0u, 0u,
                                  A.dt, sqrt(A.dt)};
}

// Adds a lane's tallies to the block's 64-bit totals and clears them.
__device__ __forceinline__ void drain_tally(Tally &t, unsigned long long *s_tot) {
  if (t.trunc) atomicAdd(&s_tot[0], (unsigned long long)t.trunc);
  if (t.sub) atomicAdd(&s_tot[1], (unsigned long long)t.sub);
  if (t.hits) atomicAdd(&s_tot[2], (unsigned long long)t.hits);
  if (t.steps) atomicAdd(&s_tot[3], (unsigned long long)t.steps);
  t = Tally{0, 0, 0, 0};
}

// Moves a block's u32 LDS counters into their 64-bit counters in the set
// (the lanes of one wave, each counter taken and cleared atomically, so
// counts other waves add meanwhile are kept).
__device__ __forceinline__ void drain_lds(uint32_t *lds, uint64_t *glob, int32_t n) {
  for (int32_t i = (int32_t)(threadIdx.x & 63u); i < n; i += 64) {
    const uint32_t v = atomicExch(&lds[i], 0u);
    if (v) atomicAdd((unsigned long long *)&glob[i], (unsigned long long)v);
  }
}

// A lane of a pool serves any number of particles in a launch, and a
// persistent block any number of particle-steps, so every wave drains its
// lanes' 32-bit tallies into the block's 64-bit totals every A.drain (at
// most kDrainMax = 1024) iterations of its pool loop, and the block's u32
// LDS exit and snapshot counters into the set's 64-bit ones every
// A.drain_lds (at most kLdsDrainMax = 2^20).  Bounds: one iteration
// finishes at most two particles on a lane (its own, and the one of its
// split-pass slot), each adding at most 2^20 steps (a launch's cap), plus
// at most one crossing, so 1024 iterations add at most 2^31 + 1024 to a
// tally.  Between two drains of an LDS counter (by any wave), each of the
// block's four waves runs fewer than A.drain_lds iterations, each adding at
// most 64 exit records and 64 x 9 snapshots (one per step of a window of at
// most 8 steps, and one per split-pass lane): below 4 x 2^20 x 576 < 2^32
// per counter.  The LDS drains are rare because each is a round of
// device-scope atomics on the set's counters, which go past the XCD's L2.

// Where a wave's particles come from: the set's counter.  The grid stays
// resident; every wave reserves the next A.claim_chunk particle ids from the
// counter (one atomic) and moves them into its pool as its home slots free
// up, so pools stay nearly full until the set runs out and a launch ends
// with one short tail instead of one per block.  The reservation is larger
// for short launches (up to 1024 ids): the set's counter is one address
// that every wave of the grid updates, and with 16 ids per update a
// 100-step launch over 1e8 particles spent most of its time on it.  A wave
// that finds the set run out stops reserving, so every wave passes n by at
// most one reservation per set and launch (a batched launch lets a block
// join a set only while its counter is below n, so this holds there too);
// the host bounds the reservation so that the counter cannot wrap.
// Q: the particle type (Particle32 or Particle64, each with its pool type
// in LDS).
template <bool TRACE, bool LDS, bool OBS, int PW, int NG, int GEN, class Q, class Pool>
__device__ void run_pool(const GView &G, int32_t n_edges, const SetDev &S,
                         const StepArgs &A, Pool &P, uint32_t *s_exit, Tally &t,
                         unsigned long long *s_tot, int32_t nnz, const ObsSink &sink) {
  using real = typename Q::real;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n_end = S.n0 + A.nsteps;
  Q q;
  pool_particle(q, G, s_exit, A);
  bool has = false;
  uint32_t slot = 0, n = 0, pid = 0;  // the lane's home slot, next step, particle
  uint32_t snap = 0;  // next snapshot count of the lane's particle
  // Ready, split and free queues: FIFO rings over the pool's slot ids, with
  // wave-uniform head and tail counters.  FIFO keeps the particles of a pool
  // advancing together, so a launch ends without a long tail of stragglers.
  constexpr uint32_t K = (uint32_t)PW;
  uint32_t r_head = 0, r_tail = 0, s_head = 0, s_tail = 0;
  uint32_t f_head = 0, f_tail = K;
  for (uint32_t i = lane; i < K; i += 64u) P.freeq[i] = (uint8_t)i;
  const uint32_t lim = S.n;
  bool exhausted = false;   // the reservation is used up and the set has run out
  bool last_chunk = false;  // the set ran out with the current reservation
  uint32_t res_next = 0, res_end = 0;  // the wave's reserved ids [res_next, res_end)
  uint32_t iter = 0, iter_lds = 0;
  wave_lds_fence();

  for (;;) {
    if (++iter >= A.drain) {
      iter = 0;
      drain_tally(t, s_tot);
    }
    if (++iter_lds >= A.drain_lds) {
      iter_lds = 0;
      if (LDS) drain_lds(s_exit, S.exit_cnt, nnz);
      if (OBS && sink.lds) drain_lds(sink.lds, S.obs, A.obs_lds);
    }
    // Claim more particles: a wave takes as many ids as it has free home
    // slots, in multiples of kClaimMin up to 64, from its reservation, so a
    // pool refills while its first particles finish rather than after half
    // of them have.  Reservations and claims stay multiples of kClaimMin
    // (but for the last ids below n), so every claim starts at a multiple
    // of it: a claim's 128-byte lines of positions belong to one wave (its
    // state words share a line with one neighbouring claim).
    while (!exhausted && f_tail - f_head >= (uint32_t)kClaimMin) {
      if (res_next == res_end) {
        if (last_chunk) {
          exhausted = true;
          break;
        }
        uint32_t v = 0u;
        if (lane == 0u) v = atomicAdd(S.work, A.claim_chunk);
        const uint32_t b = __builtin_amdgcn_readfirstlane(v);
        if (b >= lim) {
          exhausted = true;
          break;
        }
        last_chunk = lim - b <= A.claim_chunk;
        res_next = b;
        res_end = last_chunk ? lim : b + A.claim_chunk;
      }
      const uint32_t want =
          min(min(64u, f_tail - f_head) & ~((uint32_t)kClaimMin - 1u), res_end - res_next);
      const uint32_t id = res_next + lane;
      res_next += want;
      const bool mine = lane < want;
      const uint32_t hs = mine ? P.freeq[(f_head + lane) % K] : 0u;
      const bool ok = pool_claim<TRACE, PW, GEN>(G, S, n_edges, id, P, hs, mine && id < lim);
      f_head += want;
      const uint64_t m_ok = __ballot(ok);
      const uint64_t m_back = __ballot(mine & !ok);
      if (ok) {
        P.n[hs] = S.n0;
        P.pid[hs] = id;
        if constexpr (TRACE) {
          P.hits[hs] = S.hits[id];
          P.hash[hs] = S.seqhash[id];
        }
        P.ready[(r_tail + lane_rank(m_ok)) % K] = (uint8_t)hs;
      } else if (mine) {
        P.freeq[(f_tail + lane_rank(m_back)) % K] = (uint8_t)hs;
      }
      r_tail += (uint32_t)__popcll(m_ok);
      f_tail += (uint32_t)__popcll(m_back);
      wave_lds_fence();
    }
    // lanes without a particle take ready ones
    {
      const uint64_t m_empty = __ballot(!has);
      const uint32_t ready_cnt = r_tail - r_head;
      if (!has) {
        const uint32_t r = lane_rank(m_empty);
        if (r < ready_cnt) {
          slot = P.ready[(r_head + r) % K];
          n = P.n[slot];
          pid = P.pid[slot];
          pool_load(q, P, slot);
          has = true;
          if (OBS) snap = next_snapshot(n, S);
        }
      }
      r_head += min((uint32_t)__popcll(m_empty), ready_cnt);
    }
    bool do_split = false;
    if (__ballot(has) == 0ull) {
      if (s_tail == s_head) {
        if (exhausted) break;
        continue;  // every particle claimed so far was dead: claim more
      }
      do_split = true;
    } else {
      // A window of NG Philox groups of first sub-steps, starting at the
      // group that holds the lane's next step (so a particle resumed after
      // a split skips at most three steps of it).  Every lane runs the same
      // straight-line code; a lane without a particle has no active step.
      constexpr uint32_t NW = 4u * NG;
      const uint32_t base = n & ~3u;
      real W[NW];
#pragma unroll
      for (uint32_t g = 0; g < (uint32_t)NG; ++g) {
        uint32_t k0 = A.key0, k1 = A.key1;
        fresh_keys<real>(k0, k1);
        const U4 o = philox(pid, (base >> 2) + g, 0u, S.tag, k0, k1);
        Q::box_muller(o.x, o.y, W[4 * g + 0], W[4 * g + 1]);
        Q::box_muller(o.z, o.w, W[4 * g + 2], W[4 * g + 3]);
      }
      const uint32_t jb = n & 3u;  // = n - base
      const uint32_t je = has ? min(NW, n_end - base) : 0u;
      q.prep_window(W, jb, has);
      int32_t pj = -1;
      real wp = 0;
      bool go = true;  // no vertex reached yet in this window
#pragma unroll
      for (uint32_t j = 0; j < NW; ++j) {
        const bool act = (j >= jb) & (j < je) & go;
        const bool in = q.fast_pred(W[j], act);
        const bool hit = act & !in;
        pj = hit ? (int32_t)j : pj;
        wp = hit ? W[j] : wp;
        go = go & !hit;
        // a completed group's last step re-anchors
        if ((j & 3u) == 3u) q.reanchor_if(act & in);
        if (OBS && (act & in)) {
          const uint32_t done = base + j + 1u;
          if (done == snap) {
            observe(q, S, sink);
            snap = next_snapshot(done, S);
          }
        }
      }
      const bool parked = pj >= 0;
      n = parked ? base + (uint32_t)pj : (has ? base + je : n);
      const bool done_now = has & !parked & (n == n_end);
      if (done_now) pool_finish(q, S, A, pid, t);
      const uint64_t m_done = __ballot(done_now);
      if (done_now) P.freeq[(f_tail + lane_rank(m_done)) % K] = (uint8_t)slot;
      f_tail += (uint32_t)__popcll(m_done);
      const uint64_t m_park = __ballot(parked);
      if (parked) {
        pool_store(q, P, slot, n);
        P.w[slot] = wp;
        P.k[slot] = 0;  // fresh: the whole step left, no slot drawn yet
        P.split[(s_tail + lane_rank(m_park)) % K] = (uint8_t)slot;
      }
      s_tail += (uint32_t)__popcll(m_park);
      has = has & !parked & !done_now;
      wave_lds_fence();
      const uint32_t empty = (uint32_t)__popcll(__ballot(!has));
      const uint32_t ready_cnt = r_tail - r_head, split_cnt = s_tail - s_head;
      const uint32_t idle = empty > ready_cnt ? empty - ready_cnt : 0u;
      do_split = split_cnt >= 64u || (split_cnt > 0u && idle >= (uint32_t)A.idle);
    }
    if (do_split) {
      // Up to 64 parked particles, one per lane, one crossing each.  The
      // lanes' own particles stay in registers meanwhile.
      const uint32_t B = min(s_tail - s_head, 64u);
      const uint32_t s_base = s_head;
      s_head += B;
      wave_lds_fence();
      bool back = false, again = false, freed = false;
      uint32_t s2 = 0;
      if (lane < B) {
        s2 = P.split[(s_base + lane) % K];
        Q q2;
        pool_particle(q2, G, s_exit, A);
        pool_load(q2, P, s2);
        const uint32_t step = P.n[s2];
        const uint32_t pid2 = P.pid[s2];
        auto h = pool_hit(P, s2, A);
        if (!q2.cross(step, h, pid2, S, A, t)) {
          // reached a vertex again: back on the split queue for a later pass
          pool_store(q2, P, s2, step);
          pool_park(P, s2, h);
          again = true;
        } else {
          if (q2.alive) {
            if ((step & 3u) == 3u) q2.reanchor();
            if (OBS && step + 1u == next_snapshot(step, S)) observe(q2, S, sink);
          }
          const uint32_t n2 = step + 1u;
          if (!q2.alive || n2 == n_end) {
            pool_finish(q2, S, A, pid2, t);
            freed = true;
          } else {
            pool_store(q2, P, s2, n2);
            back = true;
          }
        }
      }
      const uint64_t m_freed = __ballot(freed);
      if (freed) P.freeq[(f_tail + lane_rank(m_freed)) % K] = (uint8_t)s2;
      f_tail += (uint32_t)__popcll(m_freed);
      const uint64_t m_again = __ballot(again);
      if (again) P.split[(s_tail + lane_rank(m_again)) % K] = (uint8_t)s2;
      s_tail += (uint32_t)__popcll(m_again);
      const uint64_t m_back = __ballot(back);
      if (back) P.ready[(r_tail + lane_rank(m_back)) % K] = (uint8_t)s2;
      r_tail += (uint32_t)__popcll(m_back);
      wave_lds_fence();
    }
  }
}

// Shared memory of a pool block: [exit counters][staged tables][pools]
// [snapshot bins].  Stages the set's tables, runs its particles until the
// set's counter has run out and the block's pools are empty, and adds the
// block's counts to the set's counters.
template <int PW, bool FP64, bool TRACE>
using PoolLds = std::conditional_t<FP64, PoolLds64<TRACE, PW>, PoolLds32<TRACE, PW>>;

template <bool FP64, bool TRACE, bool LDS, bool STAGED, bool OBS, int PW, int NG, int GEN>
__device__ __forceinline__ void pool_block(const GraphDev &G, const SetDev &S,
                                           const StepArgs &A, unsigned long long *s_tot,
                                           char *smem) {
  using Pool = PoolLds<PW, FP64, TRACE>;
  using Q = std::conditional_t<FP64, Particle64<TRACE, LDS, GEN>, Particle32<TRACE, LDS, GEN>>;
  uint32_t *s_exit = (uint32_t *)smem;
  if (threadIdx.x < 4) s_tot[threadIdx.x] = 0;
  if (LDS)
    for (int32_t s = threadIdx.x; s < G.nnz; s += blockDim.x) s_exit[s] = 0;
  const int32_t ex = LDS ? exit_bytes(G.nnz) : 0;
  const GView view = block_view<FP64, STAGED>(G, smem + ex);
  const int32_t o_pools =
      align16(ex + (STAGED ? (FP64 ? G.stage_bytes64 : G.stage_bytes32) : 0));
  Pool *pools = (Pool *)(smem + o_pools);
  ObsSink o{nullptr, G.e64};
  if (OBS && A.obs_lds) {
    o.lds = (uint32_t *)(smem + o_pools + (int32_t)sizeof(Pool) * kWavesPerBlock);
    for (int32_t b = threadIdx.x; b < A.obs_lds; b += blockDim.x) o.lds[b] = 0;
  }
  __syncthreads();
  Tally t{0, 0, 0, 0};
  const uint32_t wave = threadIdx.x >> 6;
  run_pool<TRACE, LDS, OBS, PW, NG, GEN, Q>(view, G.E, S, A, pools[wave], s_exit, t, s_tot,
                                            G.nnz, o);
  flush(S, t, s_tot, s_exit, G.nnz, LDS);
  if (OBS && A.obs_lds) flush_obs(S, o.lds, A.obs_lds);
}

#ifndef MG_POOL_WAVES_PER_EU
#define MG_POOL_WAVES_PER_EU 7
#endif

// GEN (cubic coefficients) is instantiated for pools of 128 with two
// Philox groups per window only.
template <bool TRACE, bool LDS, bool STAGED, bool OBS, int PW, int NG, int GEN = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MG_POOL_WAVES_PER_EU)))
void k_pool32(GraphDev G, SetDev S, StepArgs A) {
  extern __shared__ uint4 smem4[];
  __shared__ unsigned long long s_tot[4];
  pool_block<false, TRACE, LDS, STAGED, OBS, PW, NG, GEN>(G, S, A, s_tot, (char *)smem4);
}

// FP64 wave pools: the same schedule over FP64 particles (pools of 128,
// 8-step windows).  Two FP64 particles per lane take more registers: four
// waves per SIMD.
#ifndef MG_POOL64_WAVES_PER_EU
#define MG_POOL64_WAVES_PER_EU 4
#endif
template <bool TRACE, bool LDS, bool STAGED, bool OBS, int GEN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MG_POOL64_WAVES_PER_EU)))
void k_pool64(GraphDev G, SetDev S, StepArgs A) {
  extern __shared__ uint4 smem4[];
  __shared__ unsigned long long s_tot[4];
  pool_block<true, TRACE, LDS, STAGED, OBS, kPoolSmall, 2, GEN>(G, S, A, s_tot, (char *)smem4);
}

// Batched form of the wave pools: a resident grid whose blocks take work
// items (a set index each; A.batch_items of them, largest sets first) from
// the counter A.batch_claim, and for each runs the set's particles with the
// single-set pool code: the block's waves claim ids from the set's own
// counter, alongside every other block working on that set, until it has
// run out.  An item of a set that has run out is passed over at the cost
// of one load.  Both counters are cleared by k_batch_reset before each
// launch.
template <bool TRACE, bool LDS, bool STAGED, bool OBS, int PW, int NG, int GEN = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MG_POOL_WAVES_PER_EU)))
void k_pool32_batch(const GraphDev *graphs, const SetDev *sets, const BatchItem *items,
                    StepArgs A) {
  extern __shared__ uint4 smem4[];
  __shared__ unsigned long long s_tot[4];
  __shared__ int32_t s_set;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t i = atomicAdd(A.batch_claim, 1u);
      int32_t set = -1;  // -1: no items left
      if (i < A.batch_items) {
        set = items[i].set;
        const SetDev &Si = sets[set];
        if (__hip_atomic_load(Si.work, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= Si.n)
          set = -2;  // that set has run out
      }
      s_set = set;
    }
    __syncthreads();
    const int32_t set = s_set;
    __syncthreads();  // every thread has read s_set before thread 0 writes it again
    if (set == -1) break;
    if (set < 0) continue;
    SetDev S = sets[set];
    S.n0 += A.n0_offset;  // steps already taken by earlier launches of this call
    const GraphDev G = graphs[set];
    pool_block<false, TRACE, LDS, STAGED, OBS, PW, NG, GEN>(G, S, A, s_tot, (char *)smem4);
  }
}

// The same over FP64 sets: FP64 wave pools (128 per wave, 8-step windows).
template <bool TRACE, bool LDS, bool STAGED, bool OBS, int GEN = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MG_POOL64_WAVES_PER_EU)))
void k_pool64_batch(const GraphDev *graphs, const SetDev *sets, const BatchItem *items,
                    StepArgs A) {
  extern __shared__ uint4 smem4[];
  __shared__ unsigned long long s_tot[4];
  __shared__ int32_t s_set;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t i = atomicAdd(A.batch_claim, 1u);
      int32_t set = -1;  // -1: no items left
      if (i < A.batch_items) {
        set = items[i].set;
        const SetDev &Si = sets[set];
        if (__hip_atomic_load(Si.work, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= Si.n)
          set = -2;  // that set has run out
      }
      s_set = set;
    }
    __syncthreads();
    const int32_t set = s_set;
    __syncthreads();  // every thread has read s_set before thread 0 writes it again
    if (set == -1) break;
    if (set < 0) continue;
    SetDev S = sets[set];
    S.n0 += A.n0_offset;
    const GraphDev G = graphs[set];
    pool_block<true, TRACE, LDS, STAGED, OBS, kPoolSmall, 2, GEN>(G, S, A, s_tot,
                                                                  (char *)smem4);
  }
}

// Clears the particle counters of a batch's sets and its item counter
// before a launch of k_pool32_batch or k_pool64_batch (a kernel, so that the
// launch chain can be a HIP graph of kernel nodes).
__global__ void k_batch_reset(const SetDev *sets, int32_t n_sets, uint32_t *claim) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_sets) *sets[i].work = 0u;
  if (i == 0) *claim = 0u;
}

// Autotuning probes: the FP32 step kernels under names of their own, so a
// profile tells the probes apart from the launches they tune.
template <bool LDS, bool STAGED, int PW, int NG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MG_POOL_WAVES_PER_EU)))
void k_pool32_probe(GraphDev G, SetDev S, StepArgs A) {
  extern __shared__ uint4 smem4[];
  __shared__ unsigned long long s_tot[4];
  pool_block<false, false, LDS, STAGED, false, PW, NG, false>(G, S, A, s_tot, (char *)smem4);
}

template <bool LDS, bool STAGED>
__global__ __launch_bounds__(kBlock) void k_step32_probe(GraphDev G, SetDev S, StepArgs A) {
  extern __shared__ uint4 smem4[];
  __shared__ unsigned long long s_tot[4];
  step_block<false, false, LDS, STAGED, false, false>(G, S, A, blockIdx.x * kBlock + threadIdx.x,
                                               s_tot, (char *)smem4);
}

// Clears the particle counter of a persistent pool launch (a kernel rather
// than a memset, so that launch chains can be captured in HIP graphs).
__global__ void k_clear_word(uint32_t *w) {
  if (threadIdx.x == 0) *w = 0u;
}

// Blocks of a persistent launch: as many as stay resident at once (CUs x
// blocks per CU for this kernel and LDS size), fewer if the set is small.
uint32_t resident_blocks(const void *func, size_t shm, uint32_t need) {
  // blocks per CU of (device, kernel, LDS bytes) times the device's CU
  // count, queried once and kept: the occupancy query costs microseconds,
  // which short launches would pay on every call
  struct Entry {
    int dev;
    const void *func;
    size_t shm;
    uint32_t blocks;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  uint32_t r = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry &e : cache)
      if (e.dev == dev && e.func == func && e.shm == shm) {
        r = e.blocks;
        break;
      }
  }
  if (r == 0) {
    int cus = 0;
    if (dev < 0 ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, func, kBlock, shm) != hipSuccess ||
        per_cu <= 0)
      per_cu = 1;
    r = (uint32_t)cus * (uint32_t)per_cu;
    if (r > kMaxPersistBlocks) r = kMaxPersistBlocks;  // bounds the claim counter
    std::lock_guard<std::mutex> lock(mu);
    if (cache.size() < 4096) cache.push_back({dev, func, shm, r});
  }
  return need < r ? need : r;
}

// ---------------------------------------------------------------- init --
template <bool FP64>
__global__ __launch_bounds__(kBlock) void k_init(GraphDev G, SetDev S, int mode,
                                                 int32_t vertex, uint32_t k0,
                                                 uint32_t k1, const int32_t *edge_in,
                                                 const double *pos_in, InitSources src) {
  const uint32_t pid = blockIdx.x * kBlock + threadIdx.x;
  if (pid >= S.n) return;
  int32_t e;
  double x;
  if (mode == 0) {
    e = edge_in[pid];
    x = pos_in[pid];
  } else {
    const U4 o = philox(pid, 0xFFFFFFFFu, 0xFFFFFFFFu, S.tag, k0, k1);
    if (mode == 1 || mode == 3) {
      uint32_t r = o.x;
      if (mode == 3) {
        // source: first j with word 0 < T_j (T nondecreasing, last 2^32)
        int32_t lo = 0, hi = src.n - 1;
        while (lo < hi) {
          const int32_t mid = (lo + hi) >> 1;
          if ((uint64_t)o.x < src.thr[mid])
            hi = mid;
          else
            lo = mid + 1;
        }
        vertex = src.vtx[lo];
        r = o.y;
      }
      const SlotPick sp = pick_slot(global_view(G), G.vtx[vertex], r);
      e = eo_edge(sp.eo);
      x = (sp.eo & 1u) ? G.e64[e].L : 0.0;
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
    const double yd = side ? L - x : x;
    const float yh = (float)yd;
    S.ef[pid] = (uint32_t)e | (side ? kSideBit : 0u);
    S.y32[pid] = make_float2(yh, (float)(yd - (double)yh));
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
    const EdgeRec64 &r = G.e64[e];
    double x;
    if (FP64) {
      x = S.x64[pid];
    } else {
      const float2 yy = S.y32[pid];
      const double y = (double)yy.x + (double)yy.y;
      x = (ef & kSideBit) ? r.L - y : y;
    }
    const int32_t idx = e * nb + bin_of(x, r.span, nb);
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

// Histogram too large for one LDS copy, in edge-range tiles: blockIdx.y
// picks a range of whole edges whose bins fit in LDS, and the block counts
// only the particles on those edges (the state word decides; the position
// is read only for them), then merges its u32 counts into the u64 bins.
template <bool FP64>
__global__ __launch_bounds__(kBlock) void k_hist_tiled(GraphDev G, SetDev S, int32_t nb,
                                                       int32_t edges_per_tile, uint64_t *out) {
  extern __shared__ uint32_t s_bin[];
  const int32_t e0 = (int32_t)blockIdx.y * edges_per_tile;
  const int32_t e1 = min(G.E, e0 + edges_per_tile);
  const int32_t nbins = (e1 - e0) * nb;
  for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x) s_bin[b] = 0;
  __syncthreads();
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t pid = blockIdx.x * kBlock + threadIdx.x; pid < S.n; pid += stride) {
    const uint32_t ef = S.ef[pid];
    if (ef & kDeadBit) continue;
    const int32_t e = (int32_t)(ef & kEdgeMask);
    if (e < e0 || e >= e1) continue;
    const EdgeRec64 &r = G.e64[e];
    double x;
    if (FP64) {
      x = S.x64[pid];
    } else {
      const float2 yy = S.y32[pid];
      const double y = (double)yy.x + (double)yy.y;
      x = (ef & kSideBit) ? r.L - y : y;
    }
    atomicAdd(&s_bin[(e - e0) * nb + bin_of(x, r.span, nb)], 1u);
  }
  __syncthreads();
  uint64_t *o = out + (int64_t)e0 * nb;
  for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x)
    if (s_bin[b]) atomicAdd((unsigned long long *)&o[b], (unsigned long long)s_bin[b]);
}

// Histogram over per-edge bins of any widths (the appendix's general
// histogram kernel): the bins of edge e are off[e] .. off[e+1]-1 with upper
// boundaries up[] (FP64, strictly increasing along the edge).  A particle at
// x takes the first bin whose upper boundary is >= x (binary search), or the
// edge's last bin.
template <bool FP64, bool LDS>
__global__ __launch_bounds__(kBlock) void k_hist_csr(GraphDev G, SetDev S, const int32_t *off,
                                                     const double *up, int32_t nbins,
                                                     uint64_t *out) {
  extern __shared__ uint32_t s_bin[];
  if (LDS) {
    for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x) s_bin[b] = 0;
    __syncthreads();
  }
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t pid = blockIdx.x * kBlock + threadIdx.x; pid < S.n; pid += stride) {
    const uint32_t ef = S.ef[pid];
    if (ef & kDeadBit) continue;
    const int32_t e = (int32_t)(ef & kEdgeMask);
    double x;
    if (FP64) {
      x = S.x64[pid];
    } else {
      const float2 yy = S.y32[pid];
      const double y = (double)yy.x + (double)yy.y;
      x = (ef & kSideBit) ? G.e64[e].L - y : y;
    }
    int32_t lo = off[e], hi = off[e + 1] - 1;  // the answer lies in [lo, hi]
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (x <= up[mid])
        hi = mid;
      else
        lo = mid + 1;
    }
    if (LDS)
      atomicAdd(&s_bin[lo], 1u);
    else
      atomicAdd((unsigned long long *)&out[lo], 1ull);
  }
  if (LDS) {
    __syncthreads();
    for (int32_t b = threadIdx.x; b < nbins; b += blockDim.x)
      if (s_bin[b]) atomicAdd((unsigned long long *)&out[b], (unsigned long long)s_bin[b]);
  }
}

// Calls f(std::bool_constant<x>...) for the run-time flags, so one launch
// site covers every compiled variant.
template <typename F>
void with_flags(F &&f) {
  f();
}
template <typename F, typename... Rest>
void with_flags(F &&f, bool x, Rest... rest) {
  if (x)
    with_flags([&](auto... v) { f(std::true_type{}, v...); }, rest...);
  else
    with_flags([&](auto... v) { f(std::false_type{}, v...); }, rest...);
}

// The graph's method-variant level as a compile-time constant: 0 affine
// coefficients, kGenCubic cubic ones, kGenFull tables or Wentzell vertices.
template <typename F>
void with_gen(int32_t level, F &&f) {
  if (level == kGenFull)
    f(std::integral_constant<int, kGenFull>{});
  else if (level == kGenCubic)
    f(std::integral_constant<int, kGenCubic>{});
  else
    f(std::integral_constant<int, 0>{});
}

// Shape of an FP32 wave-pool schedule (StepArgs::kernel 1, 2, 3): particles
// per wave and Philox groups per phase-A window.
template <typename F>
void with_pool(int32_t kernel, F &&f) {
  using I = std::integral_constant<int, 1>;
  if (kernel == 2)
    f(std::integral_constant<int, kPoolLarge>{}, I{});
  else if (kernel == 3)
    f(std::integral_constant<int, kPoolSmall>{}, std::integral_constant<int, 2>{});
  else
    f(std::integral_constant<int, kPoolSmall>{}, I{});
}

// LDS layout of a step block, shared by the host launchers and the
// kernels' offsets: [exit counters][staged tables][pools][snapshot bins].
// Within kLdsBlockMax bytes, exit counters come first (they take an atomic
// per hit-step), staged tables next, snapshot bins last.
struct LdsPlan {
  bool lds_exit;
  bool staged;
  int32_t obs_lds;  // snapshot bins in LDS, 0: global counters
  size_t shm;
};

LdsPlan plan_lds(int32_t nnz, int32_t stage, size_t pools, const SetDev *obs_set,
                 int32_t n_edges) {
  LdsPlan p{};
  p.lds_exit = nnz <= kLdsExitMax;
  p.staged = stage > 0;
  auto size = [&]() {
    const int32_t ex = p.lds_exit ? ((nnz * 4 + 15) & ~15) : 0;
    const size_t b = (size_t)((ex + (p.staged ? stage : 0) + 15) & ~15) + pools;
    return (b + 15) & ~(size_t)15;
  };
  if (size() > (size_t)kLdsBlockMax) p.staged = false;
  if (size() > (size_t)kLdsBlockMax) p.lds_exit = false;
  const size_t base = size();
  p.shm = base;
  if (obs_set && obs_set->obs) {
    const int64_t nbins = (int64_t)n_edges * obs_set->obs_nb;
    if (nbins <= kLdsObsMax && base + (size_t)nbins * 4 <= (size_t)kLdsBlockMax) {
      p.obs_lds = (int32_t)nbins;
      p.shm = base + (size_t)nbins * 4;
    }
  }
  return p;
}

template <bool FP64, bool TRACE>
hipError_t launch_step_t(const GraphDev &g, const SetDev &s, const StepArgs &a0,
                         hipStream_t st) {
  StepArgs a = a0;
  const bool obs = s.obs != nullptr;
  if constexpr (FP64) {
    if (a.kernel == 3) {
      // FP64 wave pools (128 per wave, 8-step windows) on a resident grid
      const LdsPlan lp = plan_lds(g.nnz, g.stage_bytes64,
                                  sizeof(PoolLds64<TRACE, kPoolSmall>) * kWavesPerBlock, &s,
                                  g.E);
      a.obs_lds = lp.obs_lds;
      const uint32_t need = (s.n + kPoolSmall * kWavesPerBlock - 1) / (kPoolSmall * kWavesPerBlock);
      hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, st, s.work);
      with_gen(g.gen, [&](auto Gn) {
        constexpr int gn = decltype(Gn)::value;
        with_flags([&](auto L, auto T, auto O) {
          constexpr bool l = decltype(L)::value, t = decltype(T)::value,
                         o = decltype(O)::value;
          const void *f = (const void *)k_pool64<TRACE, l, t, o, gn>;
          hipLaunchKernelGGL((k_pool64<TRACE, l, t, o, gn>),
                             dim3(resident_blocks(f, lp.shm, need)), dim3(kBlock), lp.shm, st,
                             g, s, a);
        }, lp.lds_exit, lp.staged, obs);
      });
      return hipGetLastError();
    }
  }
  if (!FP64 && a.kernel >= 1 && (!g.gen || a.kernel == 3)) {
    with_pool(a.kernel, [&](auto PWc, auto NGc) {
      constexpr int PW = decltype(PWc)::value, NG = decltype(NGc)::value;
      const int32_t stage = g.stage_bytes32;
      const LdsPlan lp = plan_lds(g.nnz, stage, sizeof(PoolLds32<TRACE, PW>) * kWavesPerBlock,
                                  &s, g.E);
      a.obs_lds = lp.obs_lds;
      const uint32_t need = (s.n + PW * kWavesPerBlock - 1) / (PW * kWavesPerBlock);
      hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, st, s.work);
      if (!TRACE && !obs && a.probe) {
        with_flags([&](auto L, auto T) {
          const void *f =
              (const void *)k_pool32_probe<decltype(L)::value, decltype(T)::value, PW, NG>;
          hipLaunchKernelGGL((k_pool32_probe<decltype(L)::value, decltype(T)::value, PW, NG>),
                             dim3(resident_blocks(f, lp.shm, need)), dim3(kBlock), lp.shm, st,
                             g, s, a);
        }, lp.lds_exit, lp.staged);
        return;
      }
      if constexpr (PW == kPoolSmall && NG == 2) {
        if (g.gen) {
          with_gen(g.gen, [&](auto Gn) {
            constexpr int gn = decltype(Gn)::value;
            if constexpr (gn != 0)
              with_flags([&](auto L, auto T, auto O) {
                const void *f =
                    (const void *)k_pool32<TRACE, decltype(L)::value, decltype(T)::value,
                                           decltype(O)::value, PW, NG, gn>;
                hipLaunchKernelGGL((k_pool32<TRACE, decltype(L)::value, decltype(T)::value,
                                             decltype(O)::value, PW, NG, gn>),
                                   dim3(resident_blocks(f, lp.shm, need)), dim3(kBlock),
                                   lp.shm, st, g, s, a);
              }, lp.lds_exit, lp.staged, obs);
          });
          return;
        }
      }
      with_flags([&](auto L, auto T, auto O) {
        const void *f = (const void *)k_pool32<TRACE, decltype(L)::value, decltype(T)::value,
                                               decltype(O)::value, PW, NG>;
        hipLaunchKernelGGL((k_pool32<TRACE, decltype(L)::value, decltype(T)::value,
                                     decltype(O)::value, PW, NG>),
                           dim3(resident_blocks(f, lp.shm, need)), dim3(kBlock), lp.shm, st,
                           g, s, a);
      }, lp.lds_exit, lp.staged, obs);
    });
    return hipGetLastError();
  }
  const int32_t stage = FP64 ? g.stage_bytes64 : g.stage_bytes32;
  const LdsPlan lp = plan_lds(g.nnz, stage, 0, &s, g.E);
  a.obs_lds = lp.obs_lds;
  const uint32_t blocks = (s.n + kBlock - 1) / kBlock;
  if (!FP64 && !TRACE && !obs && a.probe) {
    with_flags([&](auto L, auto T) {
      hipLaunchKernelGGL((k_step32_probe<decltype(L)::value, decltype(T)::value>),
                         dim3(blocks), dim3(kBlock), lp.shm, st, g, s, a);
    }, lp.lds_exit, lp.staged);
    return hipGetLastError();
  }
  with_gen(g.gen, [&](auto Gn) {
    constexpr int gn = decltype(Gn)::value;
    with_flags([&](auto L, auto T, auto O) {
      hipLaunchKernelGGL((k_step<FP64, TRACE, decltype(L)::value, decltype(T)::value,
                                 decltype(O)::value, gn>),
                         dim3(blocks), dim3(kBlock), lp.shm, st, g, s, a);
    }, lp.lds_exit, lp.staged, obs);
  });
  return hipGetLastError();
}

// Batched launches keep snapshot bins in global memory (the sets differ).
template <bool FP64, bool TRACE>
KernelLaunch batch_launch_t(int32_t n_items, int32_t max_nnz, int32_t max_stage,
                            const StepArgs &a, bool obs, int32_t gen) {
  KernelLaunch k{};
  k.grid = dim3(n_items);
  k.block = dim3(kBlock);
  k.persistent = false;
  // FP32: the wave pools of the set's schedule (only pools of 128 with
  // 8-step windows for the general levels); FP64: its wave pools
  const bool pools = FP64 ? a.kernel == 3 : (a.kernel >= 1 && (!gen || a.kernel == 3));
  with_pool(a.kernel, [&](auto PWc, auto NGc) {
    constexpr int PW = decltype(PWc)::value, NG = decltype(NGc)::value;
    const size_t pool_bytes = FP64 ? sizeof(PoolLds64<TRACE, kPoolSmall>) * kWavesPerBlock
                                   : sizeof(PoolLds32<TRACE, PW>) * kWavesPerBlock;
    const LdsPlan lp = plan_lds(max_nnz, max_stage, pools ? pool_bytes : 0, nullptr, 0);
    k.shm = lp.shm;
    with_gen(gen, [&](auto Gn) {
      constexpr int gn = decltype(Gn)::value;
      with_flags([&](auto L, auto T, auto O) {
        constexpr bool l = decltype(L)::value, t = decltype(T)::value, o = decltype(O)::value;
        if (pools) {
          if constexpr (FP64) {
            k.func = (const void *)k_pool64_batch<TRACE, l, t, o, gn>;
          } else {
            k.func = (const void *)k_pool32_batch<TRACE, l, t, o, PW, NG>;
            if constexpr (PW == kPoolSmall && NG == 2 && gn != 0)
              k.func = (const void *)k_pool32_batch<TRACE, l, t, o, PW, NG, gn>;
          }
          // a resident grid takes the items from the batch's counter
          k.persistent = true;
          k.grid = dim3(resident_blocks(k.func, k.shm, (uint32_t)n_items));
          return;
        }
        k.func = (const void *)k_batch<FP64, TRACE, l, t, o, gn>;
      }, lp.lds_exit, lp.staged, obs);
    });
  });
  return k;
}

}  // namespace

hipError_t launch_init(const GraphDev &g, const SetDev &s, int mode, int32_t vertex,
                       uint32_t key0, uint32_t key1, const int32_t *edge_in,
                       const double *pos_in, const InitSources &src, bool fp64,
                       hipStream_t st) {
  const uint32_t blocks = (s.n + kBlock - 1) / kBlock;
  if (fp64)
    hipLaunchKernelGGL(k_init<true>, dim3(blocks), dim3(kBlock), 0, st, g, s, mode,
                       vertex, key0, key1, edge_in, pos_in, src);
  else
    hipLaunchKernelGGL(k_init<false>, dim3(blocks), dim3(kBlock), 0, st, g, s, mode,
                       vertex, key0, key1, edge_in, pos_in, src);
  return hipGetLastError();
}

hipError_t launch_step(const GraphDev &g, const SetDev &s, const StepArgs &a,
                       bool fp64, bool trace, hipStream_t st) {
  if (fp64) return trace ? launch_step_t<true, true>(g, s, a, st)
                         : launch_step_t<true, false>(g, s, a, st);
  return trace ? launch_step_t<false, true>(g, s, a, st)
               : launch_step_t<false, false>(g, s, a, st);
}

const void *batch_reset_kernel() { return (const void *)k_batch_reset; }

int32_t batch_blocks_per_cu(int32_t max_nnz, int32_t max_stage, const StepArgs &a, bool fp64,
                            bool trace, int32_t gen, bool *staged) {
  const KernelLaunch k = batch_launch(1, max_nnz, max_stage, a, fp64, trace, false, gen);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k.func, kBlock, k.shm) !=
          hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  if (staged) {
    // the plan stages the tables when their bytes are part of its LDS
    const KernelLaunch k0 = batch_launch(1, max_nnz, 0, a, fp64, trace, false, gen);
    *staged = max_stage > 0 && k.shm > k0.shm;
  }
  return per_cu;
}

int32_t batch_tile(bool fp64, int32_t kernel) {
  const bool pools = fp64 ? kernel == 3 : kernel >= 1;
  return pools ? pool_per_wave(kernel) * kWavesPerBlock * kBatchGens : kBlock;
}

KernelLaunch batch_launch(int32_t n_items, int32_t max_nnz, int32_t max_stage,
                          const StepArgs &a, bool fp64, bool trace, bool obs, int32_t gen) {
  if (fp64)
    return trace ? batch_launch_t<true, true>(n_items, max_nnz, max_stage, a, obs, gen)
                 : batch_launch_t<true, false>(n_items, max_nnz, max_stage, a, obs, gen);
  return trace ? batch_launch_t<false, true>(n_items, max_nnz, max_stage, a, obs, gen)
               : batch_launch_t<false, false>(n_items, max_nnz, max_stage, a, obs, gen);
}

hipError_t launch_histogram_csr(const GraphDev &g, const SetDev &s, const int32_t *off,
                                const double *up, int32_t nbins, uint64_t *out, bool fp64,
                                hipStream_t st) {
  const bool lds = nbins <= kLdsHistMax;
  uint32_t blocks = (s.n + kBlock - 1) / kBlock;
  if (lds && blocks > 1024) blocks = 1024;
  if (!lds && blocks > 8192) blocks = 8192;
  const size_t shm = lds ? (size_t)nbins * 4 : 0;
  with_flags([&](auto F, auto L) {
    hipLaunchKernelGGL((k_hist_csr<decltype(F)::value, decltype(L)::value>), dim3(blocks),
                       dim3(kBlock), shm, st, g, s, off, up, nbins, out);
  }, fp64, lds);
  return hipGetLastError();
}

// Clears n 64-bit words (a kernel rather than a memset, so that callers
// may capture the work in a HIP graph).
__global__ __launch_bounds__(kBlock) void k_fill_zero_u64(uint64_t *p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

hipError_t launch_fill_zero_u64(uint64_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero_u64, dim3((uint32_t)blocks), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_histogram(const GraphDev &g, const SetDev &s, int32_t nb,
                            uint64_t *out, bool fp64, bool tiled, hipStream_t st) {
  const int64_t nbins = (int64_t)g.E * nb;
  if (tiled && nbins > kLdsHistMax && nb <= kLdsHistMax) {
    const int32_t ept = kLdsHistMax / nb;
    const uint32_t tiles = (uint32_t)((g.E + ept - 1) / ept);
    uint32_t bx = (s.n + kBlock - 1) / kBlock;
    const uint32_t want = std::max<uint32_t>(1u, 4096u / tiles);  // ~4096 blocks in all
    if (bx > want) bx = want;
    const size_t shm = (size_t)ept * nb * 4;
    if (fp64)
      hipLaunchKernelGGL((k_hist_tiled<true>), dim3(bx, tiles), dim3(kBlock), shm, st, g, s, nb,
                         ept, out);
    else
      hipLaunchKernelGGL((k_hist_tiled<false>), dim3(bx, tiles), dim3(kBlock), shm, st, g, s, nb,
                         ept, out);
    return hipGetLastError();
  }
  const bool lds = nbins <= kLdsHistMax;
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

// Fixed workspace of the allocation-free entry points: one copy per GPU,
// created when the library's code object is loaded on that GPU and held
// until the process ends.  Host code must not take this array's address
// (in host code the name is a host-side stand-in, not a device address):
// it uses the per-device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[mg::kNoAllocScratchBytes];

namespace mg {

hipError_t noalloc_scratch(int device, char **base) {
  static std::mutex mu;
  static char *addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    addr[device] = (char *)ptr;
  }
  *base = addr[device];
  return hipSuccess;
}

}  // namespace mg

