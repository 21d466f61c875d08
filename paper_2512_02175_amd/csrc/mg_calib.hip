// mg_calib.hip -- VALU issue-rate calibration kernels behind mg_valu_rate
// (include/metricgraph.h): long chains of one instruction kind on every
// SIMD, so the step kernels' roofline fraction can be set against a
// measured ceiling as well as the published one.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/metricgraph.h"

namespace {

constexpr int kChains = 8;    // independent chains per lane (hide latency)
constexpr int kUnroll = 16;   // chain rounds per loop trip
constexpr int kBlock = 256;

// One v_bitop3_b32 (truth table 0x6C of its three operands), register
// operands only.
__device__ __forceinline__ uint32_t bitop3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t d;
  asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x6c" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// Each lane runs kChains independent chains of one operation for
// iters x kUnroll rounds; the chains' final values are combined and stored,
// so nothing is dead.  The operands come from the lane id and a runtime
// seed, so nothing folds at compile time.
template <int OP>
__global__ __launch_bounds__(kBlock) void k_valu_rate(uint32_t iters, uint32_t seed,
                                                      uint32_t *out) {
  const uint32_t tid = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t s = seed ^ (tid * 0x9E3779B9u);
  if constexpr (OP == MG_VALU_FMA_F32) {
    float a[kChains];
    const float m = 1.0f - (float)(s & 0xFF) * 0x1p-30f;
    const float c = (float)(s >> 24) * 0x1p-40f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = (float)(s + i) * 0x1p-32f;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = __builtin_fmaf(a[i], m, c);
    }
    float r = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) r += a[i];
    out[tid] = __float_as_uint(r);
  } else if constexpr (OP == MG_VALU_FMA_F64) {
    double a[kChains];
    const double m = 1.0 - (double)(s & 0xFF) * 0x1p-60;
    const double c = (double)(s >> 24) * 0x1p-70;
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = (double)(s + i) * 0x1p-32;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = __builtin_fma(a[i], m, c);
    }
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) r += a[i];
    const uint64_t b = (uint64_t)__double_as_longlong(r);
    out[tid] = (uint32_t)b ^ (uint32_t)(b >> 32);
  } else if constexpr (OP == MG_VALU_MAD_U64_U32) {
    // 32 x 32 -> 64-bit multiply-add: the Philox round's multiply
    uint64_t a[kChains];
    const uint32_t m = s | 1u;
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = (uint64_t)(s + i) << 7;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = (uint64_t)(uint32_t)a[i] * m + a[i];
    }
    uint64_t r = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) r ^= a[i];
    out[tid] = (uint32_t)r ^ (uint32_t)(r >> 32);
  } else if constexpr (OP == MG_VALU_BITOP3) {
    // three-input bitwise function (the Philox round's xor of the key with
    // the other product half and word); each chain takes its neighbours'
    // values.  Written as the instruction itself: left to the compiler, the
    // boolean algebra of consecutive rounds is merged into other forms.
    uint32_t a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = s * (0x85EBCA6Bu + 2u * (uint32_t)i);
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = bitop3(a[i], a[(i + 1) % kChains],
                                                         a[(i + 3) % kChains]);
    }
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) r ^= a[i];
    out[tid] = r;
  } else if constexpr (OP == MG_VALU_LOG_F32) {
    // the transcendental unit's v_log_f32 (base 2), as Box-Muller uses it;
    // chains that leave the positive range run on NaN at the same rate
    float a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = 1.5f + (float)(s + i) * 0x1p-32f;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = __builtin_amdgcn_logf(a[i]);
    }
    float r = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) r += a[i];
    out[tid] = __float_as_uint(r);
  } else {
    // 32-bit integer add (of a neighbouring chain, so no loop folds)
    uint32_t a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = s ^ (uint32_t)i;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = a[i] + a[(i + 1) % kChains];
    }
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) r ^= a[i];
    out[tid] = r;
  }
}

template <int OP>
hipError_t launch(uint32_t blocks, uint32_t iters, uint32_t *out, hipStream_t st) {
  hipLaunchKernelGGL(k_valu_rate<OP>, dim3(blocks), dim3(kBlock), 0, st, iters, 0x2545F491u,
                     out);
  return hipGetLastError();
}

}  // namespace

namespace mg {

uint32_t valu_rate_lanes_per_block() { return kBlock; }
uint64_t valu_rate_ops_per_lane(uint32_t iters) { return (uint64_t)iters * kUnroll * kChains; }

hipError_t launch_valu_rate(int32_t op, uint32_t blocks, uint32_t iters, uint32_t *out,
                            hipStream_t st) {
  switch (op) {
    case MG_VALU_FMA_F32: return launch<MG_VALU_FMA_F32>(blocks, iters, out, st);
    case MG_VALU_FMA_F64: return launch<MG_VALU_FMA_F64>(blocks, iters, out, st);
    case MG_VALU_MAD_U64_U32: return launch<MG_VALU_MAD_U64_U32>(blocks, iters, out, st);
    case MG_VALU_BITOP3: return launch<MG_VALU_BITOP3>(blocks, iters, out, st);
    case MG_VALU_LOG_F32: return launch<MG_VALU_LOG_F32>(blocks, iters, out, st);
    default: return launch<MG_VALU_ADD_U32>(blocks, iters, out, st);
  }
}

}  // namespace mg
