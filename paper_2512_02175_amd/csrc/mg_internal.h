// mg_internal.h -- device table layouts and kernel launchers shared by the
// C ABI (mg_api.hip) and the kernels (mg_kernels.hip).  Library-internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mg {

// Particle state word: edge id in the low 30 bits, bit 30 = the FP32 path's
// reference end (0: position measured from the initial vertex, 1: from the
// terminal vertex), bit 31 = removed at an absorbing vertex.
constexpr uint32_t kEdgeMask = 0x3FFFFFFFu;
constexpr uint32_t kSideBit = 0x40000000u;
constexpr uint32_t kDeadBit = 0x80000000u;
constexpr int32_t kMaxEdges = 0x3FFFFFFF;

// Edge record for the FP64 path: 48 bytes, one per edge.
struct alignas(16) EdgeRec64 {
  double L, a, c, sigma;  // length, drift a + c x, diffusion
  int32_t vinit, vterm;   // end vertices
  int32_t pad0, pad1;
};

// Edge record for the FP32 path: 32 bytes.  aL = a + c L is the drift at
// the terminal end (the constant term of the drift seen from that end).
struct alignas(16) EdgeRec32 {
  float L, a, c, sigma;
  float aL;
  int32_t vinit, vterm;
  float pad;
};

// Slot: T_s as a 33-bit integer (2^32 = take every remaining draw), the
// incident edge and the end the particle enters at.
struct alignas(16) SlotRec {
  uint64_t thr;
  int32_t edge;
  int32_t orient;
};

// Vertex: first slot and degree; degree < 0 marks an absorbing vertex.
struct VtxRec {
  int32_t first;
  int32_t deg;
};

// Device tables of one graph.
struct GraphDev {
  const EdgeRec64 *e64;
  const EdgeRec32 *e32;
  const SlotRec *slots;
  const VtxRec *vtx;
  const uint64_t *len_thr;  // [E] init thresholds, proportional to length
  int32_t V, E, nnz;
};

// Counters of one particle set: exit[nnz], absorbed[V], totals[4]
// {truncations, substeps, hits, steps}, then a device error word.
struct SetDev {
  uint32_t *ef;        // [n] state word
  double *x64;         // [n] FP64 position from the initial vertex
  float *y32;          // [n] FP32 distance from the reference end
  uint64_t *seqhash;   // [n] or null
  uint32_t *hits;      // [n] or null
  uint64_t *exit_cnt;  // [nnz]
  uint64_t *absorbed;  // [V]
  uint64_t *totals;    // [4]
  uint32_t *err;       // [1]
  uint32_t n;
  uint32_t n0;         // first step of this launch (set's step counter)
  uint32_t tag;
};

enum : uint32_t { kErrEdge = 1u, kErrPos = 2u };

struct StepArgs {
  uint32_t nsteps;
  int32_t max_splits;
  uint32_t key0, key1;
  double dt;
};

// Batched form: one work item per (set, tile of particles).
struct BatchItem {
  int32_t set;
  uint32_t first;  // first particle of the tile
};

constexpr int kBlock = 256;
constexpr int kLdsExitMax = 16384;  // slots counted in LDS (64 KiB of u32)

hipError_t launch_init(const GraphDev &g, const SetDev &s, int mode,
                       int32_t vertex, uint32_t key0, uint32_t key1,
                       const int32_t *edge_in, const double *pos_in,
                       bool fp64, hipStream_t st);
hipError_t launch_step(const GraphDev &g, const SetDev &s, const StepArgs &a,
                       bool fp64, bool trace, hipStream_t st);
hipError_t launch_batch(const GraphDev *graphs, const SetDev *sets,
                        const BatchItem *items, int32_t n_items,
                        int32_t max_nnz, const StepArgs &a, bool fp64,
                        bool trace, hipStream_t st);
hipError_t launch_histogram(const GraphDev &g, const SetDev &s, int32_t nb,
                            uint64_t *out, bool fp64, hipStream_t st);
hipError_t launch_read(const GraphDev &g, const SetDev &s, uint32_t first,
                       uint32_t count, int32_t *edge, double *pos,
                       uint8_t *alive, bool fp64, hipStream_t st);

}  // namespace mg
