// mg_internal.h -- device table layouts and kernel launchers shared by the
// C ABI (mg_api.hip) and the kernels (mg_kernels.hip).  Library-internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/metricgraph.h"

namespace mg {

// Particle state word: edge id in the low 30 bits, bit 30 = the FP32 path's
// reference end (0: position measured from the initial vertex, 1: from the
// terminal vertex), bit 31 = removed at an absorbing vertex.
constexpr uint32_t kEdgeMask = 0x3FFFFFFFu;
constexpr uint32_t kSideBit = 0x40000000u;
constexpr uint32_t kDeadBit = 0x80000000u;
constexpr int32_t kMaxEdges = 0x3FFFFFFF;

// Edge record for the FP64 path: 112 bytes, one per edge.  span is the
// length the uniform histograms bin (the edge length unless the caller gave
// another; finite on a semi-infinite edge).  The end vertex ids of both
// records carry kMirrorEnd when that end is a mirror vertex (a reflecting
// leaf: a proposal leaving the edge there takes its mirror image when that
// lies inside the edge), so the step reads the flag with the edge, and
// kWentzellEnd when it is a Wentzell vertex (killing and stickiness), so a
// step that starts on a vertex knows without a table load whether it first
// visits that vertex.
constexpr uint32_t kMirrorEnd = 0x80000000u;
constexpr uint32_t kWentzellEnd = 0x40000000u;
constexpr int32_t kVertexMask = 0x3FFFFFFF;
constexpr int32_t kMaxVertices = 0x3FFFFFFF;
struct alignas(16) EdgeRec64 {
  double L, a, c, sigma;  // length, drift a + c x, diffusion
  int32_t vinit, vterm;   // end vertices (| kMirrorEnd at a mirror vertex)
  double span;
  // higher terms: drift + c2 x^2 + c3 x^3, diffusion + s1 x + s2 x^2 + s3 x^3
  // (all zero for affine drift and constant diffusion, which then evaluate
  // to exactly the affine values)
  double c2, c3, s1, s2, s3;
  // tabulated coefficients: tab_k > 0 intervals of width L / tab_k, the
  // first at row tab0 of the graph's table records; inv_h = tab_k / L
  double inv_h;
  int32_t tab0, tab_k;
  int32_t pad[2];  // explicit, so a packed table's bytes are all defined
};
static_assert(sizeof(EdgeRec64) == 112, "EdgeRec64 has no implicit padding");

// One interval of a tabulated edge: drift and diffusion as cubics in the
// interval's local coordinate t in [0, 1] (c0 + c1 t + c2 t^2 + c3 t^3),
// the cubic Hermite interpolants of the knot values and slopes, written in
// powers of t on the host.
struct alignas(16) TabRec64 {
  double mu[4], sg[4];
};
struct alignas(16) TabRec32 {
  float mu[4], sg[4];
};

// Edge record for the FP32 path: 32 bytes.  aL = a + c L is the drift at
// the terminal end (the constant term of the drift seen from that end);
// near = 1e-6 L (1e-6 times the binned length on a semi-infinite edge): a
// crossing from closer to the vertex than that is solved in FP64.
struct alignas(16) EdgeRec32 {
  float L, a, c, sigma;
  float aL;
  int32_t vinit, vterm;
  float near;
};

// Vertex block, 32 bytes: everything a vertex hit needs in one load.
//   first  global id of the vertex's first CSR slot (slot s = first + k);
//   deg    number of slots, -1 for an absorbing vertex.
// deg <= 3: t0, t1 are the thresholds T_0, T_1 of slots 0 and 1 and eo0..2
//   the slots' (edge << 1 | orient); bit 31 of eo_k flags T_k = 2^32 (a
//   threshold every 32-bit draw lies below).  The last slot needs none.
// deg > 3: t0 = offset of the vertex's guide table, t1 = the shift that maps
//   a draw to its guide bucket; slots are read from the slot table.
//   wz     Wentzell vertex: 1 + its row in the Wentzell table; else 0.
struct alignas(16) VtxBlk {
  int32_t first;
  int32_t deg;
  uint32_t t0, t1;
  uint32_t eo0, eo1, eo2;
  uint32_t wz;
};

// Wentzell vertex v (the general gluing condition a_v f(v) - sum_e b_ve
// f'_e(v) + c_v (L f)(v) = 0, a_v + sum_e b_ve + c_v = 1), with
// beta = sum_e b_ve: a visit of v with local time l kills with probability
// 1 - exp(-kappa l) and holds the particle on v for gamma l.  The local time
// of a visit is its overshoot o plus lt_per_sqrt sqrt(h'') for a move of
// length h'' away from v (the mean local time of a reflected move:
// sigma_v sqrt(2/pi), sigma_v the b-weighted mean of the incident edges'
// diffusion at v).
struct alignas(16) WzRec {
  double kappa;        // a_v / beta
  double gamma;        // c_v / beta
  double lt_per_sqrt;  // sigma_v sqrt(2 / pi)
  double pad;
};

// Slot table entry for vertices of degree > 3 (same encoding as above).
struct SlotRec8 {
  uint32_t t;
  uint32_t eo;
};

constexpr uint32_t kSatBit = 0x80000000u;

// Device tables of one graph.  The tables the step kernels read on a
// vertex hit (vertex blocks, edge records of the kernel's precision, slot
// table, guide tables) are contiguous so that a block can stage them in
// LDS with one copy: stage64/stage32 give the byte range of each
// precision's tables, offsets relative to `tables`.
struct GraphDev {
  const char *tables;
  const EdgeRec64 *e64;
  const EdgeRec32 *e32;
  const VtxBlk *vtx;
  const SlotRec8 *slots;
  const int32_t *guide;
  const uint64_t *len_thr;  // [E] init thresholds, proportional to length
  int32_t V, E, nnz, n_guide;
  // byte offsets of vtx, slots, guide, e32, e64 inside `tables`
  int32_t o_vtx, o_slots, o_guide, o_e32, o_e64;
  int32_t stage_bytes32;  // vtx..e32 (FP32 kernels stage this range)
  int32_t stage_bytes64;  // vtx..guide + e64 (FP64 kernels)
  // method-variant level: 0 affine coefficients and standard, absorbing or
  // mirror vertices; kGenCubic some edge has higher (cubic) drift or
  // diffusion terms; kGenFull some edge is tabulated or some vertex is a
  // Wentzell vertex.  The step kernels run the instantiation of this level
  // (each level's code gives the lower levels' graphs the same bits, except
  // that affine graphs need level 0 in FP32, whose frame constants round
  // differently from the evaluated cubics)
  int32_t gen;
  const WzRec *wz;        // Wentzell table (rows named by VtxBlk::wz), or null
  const TabRec64 *tab64;  // tabulated-coefficient intervals, or null
  const TabRec32 *tab32;
};

// Counters of one particle set: exit[nnz], absorbed[V], totals[4]
// {truncations, substeps, hits, steps}, then a device error word.
struct SetDev {
  uint32_t *ef;        // [n] state word
  double *x64;         // [n] FP64 position from the initial vertex
  float2 *y32;         // [n] FP32 distance from the reference end and its
                       //     compensation term (value = x + y)
  uint64_t *seqhash;   // [n] or null
  uint32_t *hits;      // [n] or null
  uint64_t *exit_cnt;  // [nnz]
  uint64_t *absorbed;  // [V]
  uint64_t *totals;    // [4]
  uint32_t *err;       // [1]
  uint32_t *work;      // [1] next particle id a persistent pool launch hands out
  uint64_t *obs;       // [E * obs_nb] streamed histogram, or null (off)
  int32_t obs_nb;      // its bins per edge
  uint32_t obs_every;  // a snapshot each time the step counter reaches a
                       // multiple of obs_every
  uint32_t n;
  uint32_t n0;         // first step of this launch (set's step counter)
  uint32_t tag;
  // event trace (trace sets only, else null): one record per vertex hit of
  // the particles in ev_ids (ev_nids ids, ascending); ev_cnt counts every
  // event, the first ev_cap are kept
  mg_event *ev;
  unsigned long long *ev_cnt;
  const uint32_t *ev_ids;
  int32_t ev_nids;
  uint32_t ev_cap;
};

enum : uint32_t { kErrEdge = 1u, kErrPos = 2u };

struct StepArgs {
  uint32_t nsteps;
  int32_t max_splits;
  uint32_t key0, key1;
  double dt;
  int32_t kernel;  // FP32 schedule: 0 lane-per-particle windows, 1 / 2 wave
                   // pools of 128 / 256 particles
  int32_t idle;    // wave pools: idle lanes that trigger a partial split pass
  uint32_t n0_offset;  // batched launches: steps taken earlier in the call
  int32_t obs_lds;     // streamed-histogram bins privatised in LDS (0: global)
  int32_t probe;       // autotuning probe: the same kernels under probe names
  uint32_t drain;      // wave pools: iterations between moves of the lanes'
                       // u32 tallies into the block's 64-bit totals
                       // (1 .. 1024; tests lower it)
  uint32_t drain_lds;  // and between moves of the block's u32 LDS exit and
                       // snapshot counters into the set's 64-bit ones
                       // (1 .. 2^20; tests lower it)
  uint32_t claim_chunk;   // wave pools: particle ids a wave reserves from a
                          // set's counter at a time (a multiple of 16)
  uint32_t batch_items;   // batched wave pools: work items (set indices)
  uint32_t *batch_claim;  // and the counter their resident grid takes them from
};

// Largest particle set.  A persistent pool launch hands out particle ids
// from a 32-bit counter; every wave overshoots it by at most one
// reservation, a persistent grid has at most kMaxPersistBlocks blocks of
// four waves, and the host caps a reservation at (2^32 - 1 - n) / 8192 ids
// (at least 112 at this n), so the counter cannot wrap and ids stay below n.
constexpr int64_t kMaxParticles = 0xFFFFFFFFll - 0xFFFFFll;  // 2^32 - 2^20
constexpr uint32_t kMaxPersistBlocks = 2048;
constexpr uint32_t kDrainMax = 1024;
constexpr uint32_t kLdsDrainMax = 1u << 20;

// Batched form: one work item per (set, tile of particles).  The wave-pool
// kernel reads only the set (its waves claim the set's particles from the
// set's counter); the other step kernels run the tile from `first`.
struct BatchItem {
  int32_t set;
  uint32_t first;  // first particle of the tile
};

constexpr int kBlock = 256;
// FP32 wave pools hold 128 or 256 particles per wave (2 or 4 per lane); the
// step schedule (StepArgs::kernel) picks: 0 one particle per lane, 1 pools
// of 128, 2 pools of 256.
constexpr int kPoolSmall = 128, kPoolLarge = 256;
// method-variant levels of the step kernels' instantiations (GraphDev::gen)
constexpr int kGenCubic = 1, kGenFull = 2;
inline int pool_per_wave(int32_t kernel) { return kernel == 2 ? kPoolLarge : kPoolSmall; }
constexpr int kLdsExitMax = 16384;  // slots counted in LDS (64 KiB of u32) when
                                    // the block's LDS budget allows
constexpr int kLdsStageMax = 24576; // graph tables staged in LDS up to this size
constexpr int kLdsHistMax = 16384;  // histogram bins privatised in LDS (64 KiB)
constexpr int kLdsObsMax = 4096;    // streamed-histogram bins privatised in LDS
constexpr int kLdsBlockMax = 65536; // LDS bytes a step block may take

// Injection sources of init mode 3: vertex ids and cumulative rate
// thresholds (device arrays of n entries).
struct InitSources {
  const uint64_t *thr;
  const int32_t *vtx;
  int32_t n;
};

hipError_t launch_init(const GraphDev &g, const SetDev &s, int mode,
                       int32_t vertex, uint32_t key0, uint32_t key1,
                       const int32_t *edge_in, const double *pos_in,
                       const InitSources &src, bool fp64, hipStream_t st);
hipError_t launch_step(const GraphDev &g, const SetDev &s, const StepArgs &a,
                       bool fp64, bool trace, hipStream_t st);
// Particles per batch work item: eight pools per wave for the FP32
// wave-pool kernel (a wave refills its pool from them), a plain block
// otherwise.
int32_t batch_tile(bool fp64, int32_t kernel);

// A kernel and its launch shape, for stream launches and graph nodes.  The
// batch kernels take (const GraphDev*, const SetDev*, const BatchItem*,
// StepArgs).
struct KernelLaunch {
  const void *func;
  dim3 grid, block;
  size_t shm;
  bool persistent;  // a resident grid over the items: k_batch_reset goes first
};
// k_batch_reset(const SetDev *sets, int32_t n_sets, uint32_t *claim): clears
// the sets' particle counters and the item counter of a persistent batch.
const void *batch_reset_kernel();
KernelLaunch batch_launch(int32_t n_items, int32_t max_nnz, int32_t max_stage,
                          const StepArgs &a, bool fp64, bool trace, bool obs, int32_t gen);
// Blocks per CU that a batch launch over graphs with at most max_nnz exit
// slots and max_stage staged table bytes keeps resident (the occupancy of
// its LDS plan), and whether that plan stages the tables.
int32_t batch_blocks_per_cu(int32_t max_nnz, int32_t max_stage, const StepArgs &a, bool fp64,
                            bool trace, int32_t gen, bool *staged);
// tiled: edge-range LDS tiles when E * nb exceeds one LDS copy (else 64-bit
// global atomics); below that size both take the single LDS copy.
hipError_t launch_histogram(const GraphDev &g, const SetDev &s, int32_t nb,
                            uint64_t *out, bool fp64, bool tiled, hipStream_t st);
hipError_t launch_histogram_csr(const GraphDev &g, const SetDev &s, const int32_t *off,
                                const double *up, int32_t nbins, uint64_t *out, bool fp64,
                                hipStream_t st);

// Clears n 64-bit words with a kernel (no memset node in captured work).
hipError_t launch_fill_zero_u64(uint64_t *p, int64_t n, hipStream_t st);

// VALU issue-rate calibration (mg_calib.hip): lanes per block, instructions
// of the measured kind per lane, and the launch of `blocks` blocks.
uint32_t valu_rate_lanes_per_block();
uint64_t valu_rate_ops_per_lane(uint32_t iters);
hipError_t launch_valu_rate(int32_t op, uint32_t blocks, uint32_t iters, uint32_t *out,
                            hipStream_t st);

// Allocation-free entry points stage their tables in one fixed device array
// per GPU of kNoAllocScratchBytes (32 MiB), whose address on `device` is
// looked up once (hipGetSymbolAddress, with that device current) and kept.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, char **base);

}  // namespace mg
