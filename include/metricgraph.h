/*
 * metricgraph.h -- C ABI of the MI355X (gfx950) timestep-splitting
 * Euler-Maruyama particle step on metric graphs.
 *
 * Method: Dwaraknath & Ying, "Sampling on Metric Graphs".  A particle is a
 * pair (edge e, position x in [0, L_e]) with x measured from the edge's
 * initial vertex.  Each step is the EM move x + mu_e(x) dt + sigma_e sqrt(dt) W
 * (Sec. 3, Eq. euler_maruyama_real_line); when the move leaves the edge
 * through a vertex, the step is split at the crossing, a new incident edge
 * is drawn from the vertex-edge jump probabilities b_v of the standard
 * gluing conditions (Def. 4), and the particle continues with the remaining
 * time (Alg. 2; Alg. 1 for the move from a vertex), at most M times per step.
 *
 * Conventions for every call:
 *  - Functions return mg_status; mg_last_error() describes the last failure
 *    of the calling thread (valid until that thread's next call).
 *  - Input arrays are read during the call and copied; the caller keeps
 *    ownership.  Output pointers may be host or device memory (the library
 *    copies with unified addressing); their lengths are checked and a short
 *    buffer gives MG_EINVAL.
 *  - Handles belong to the caller and are released by the matching
 *    *_destroy (NULL is accepted).  A handle must not be used by two threads
 *    at once.
 *  - Work is enqueued on the HIP stream given in mg_options (NULL: the null
 *    stream).  Calls that return results synchronise that stream.  An error
 *    found by a kernel (state out of range, non-finite position) is reported
 *    as MG_EDEVICE by the next call that synchronises.
 */
#ifndef METRICGRAPH_H
#define METRICGRAPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MG_OK = 0,
  MG_EINVAL = 1,   /* invalid argument or graph */
  MG_ENOMEM = 2,   /* device or host allocation failed, or arena too small */
  MG_EDEVICE = 3,  /* HIP runtime error or kernel-reported error */
  MG_ESTATE = 4    /* call not valid in the handle's current state */
} mg_status;

typedef enum { MG_FP64 = 0, MG_FP32 = 1 } mg_precision;

typedef enum {
  MG_VTX_STANDARD = 0, MG_VTX_ABSORBING = 1, MG_VTX_MIRROR = 2, MG_VTX_WENTZELL = 3
} mg_vertex_kind;

typedef struct mg_graph mg_graph;          /* opaque */
typedef struct mg_particles mg_particles;  /* opaque */
typedef struct mg_batch mg_batch;          /* opaque */

/*
 * Graph description (Def. 1 metric graph; Def. 4 jump probabilities;
 * Alg. 2's vertex tables).  All pointers are host memory.
 *   n_vertices, n_edges  1 <= V <= 2^30 - 1, E >= 1.
 *   edge_init/edge_term  [E] vertex ids; x = 0 at edge_init, x = L at edge_term.
 *   length               [E] > 0: finite, or +infinity for a semi-infinite
 *                        edge [0, infinity) (Def. 1 allows l_e = infinity;
 *                        its terminal vertex is a vertex at infinity).  Give
 *                        that vertex an id of its own holding only this
 *                        edge's terminal slot (absorbing, or standard with
 *                        b = 1); no particle reaches it, and it may not be a
 *                        starting or source vertex.  Graphs with such edges
 *                        reject MG_INIT_UNIFORM_LENGTH.
 *   drift_a, drift_c     [E] drift mu_e(x) = a_e + c_e x (NULL: 0); finite.
 *   sigma                [E] finite, > 0 (the paper takes sigma continuous
 *                        at vertices; that is the caller's responsibility).
 *   vtx_offsets          [V+1] CSR offsets, offsets[0] = 0, nondecreasing.
 *   slot_edge            [nnz] incident edge of each slot.
 *   slot_orient          [nnz] 0: the vertex is the edge's initial vertex (a
 *                        particle enters at x = 0); 1: terminal (enters at L).
 *   slot_jump_prob       [nnz] b_{v,e} >= 0, summing to 1 per vertex within
 *                        1e-9 (the library divides by the sum).
 *   vtx_kind             [V] mg_vertex_kind, or NULL for all standard.  An
 *                        absorbing vertex removes a particle that hits it
 *                        (Wentzell killing term a_v = 1, Sec. 2.2).  A
 *                        mirror vertex is a leaf (exactly one slot, b = 1)
 *                        that reflects: a sub-step proposal that leaves the
 *                        edge through it is replaced by its mirror image
 *                        (-x~ at an initial end, 2L - x~ at a terminal end;
 *                        the far-end reflection of the paper's star-graph
 *                        kernel in the appendix) when that image lies strictly
 *                        inside the edge, which ends the step with no vertex
 *                        hit: no split, no hit-stream draw, no exit record of
 *                        its own.  Otherwise (a move longer than the edge, or
 *                        an image on a vertex) the sub-step splits there as at
 *                        a standard leaf.  A Wentzell vertex has the general
 *                        gluing condition of Sec. 2.2, a_v f(v) - sum_e b_ve
 *                        f'_e(v) + c_v (L f)(v) = 0 with a_v + sum_e b_ve +
 *                        c_v = 1 (a_v = vtx_kill[v], c_v = vtx_sticky[v]):
 *                        with beta = sum_e b_ve, a particle leaves it into e
 *                        with probability b_ve / beta, is killed at rate
 *                        a_v / beta per unit of its local time at v and is
 *                        held on v for c_v / beta units of time per unit of
 *                        local time.  The step charges each visit (a hit, or
 *                        a step that starts on v) its local time: the
 *                        overshoot of the proposal that crossed v plus
 *                        sigma_v sqrt(2 h''/pi) for the move of length h''
 *                        that leaves v (sigma_v the b-weighted mean of the
 *                        incident edges' diffusion at v); the visit first
 *                        holds the particle on v, kills it with probability
 *                        1 - exp(-kappa l), and a stay longer than the rest of
 *                        the step carries into the next steps.  A killed
 *                        particle counts in absorbed[v].  Its killing draw is
 *                        word 0 of Philox (p, n, 0x100 + k, tag) for the visit
 *                        of hit k of step n (k = 0: the visit at a step's
 *                        start).  FP32 sets on such a graph run as on graphs
 *                        with higher coefficient terms (below).
 *   bin_span             [E] the length of edge e that the uniform histograms
 *                        (mg_histogram, mg_observe_histogram, mg_density_l2)
 *                        divide into their bins: bin width bin_span[e] / nb,
 *                        positions beyond bin_span[e] counted in the last
 *                        bin.  Finite, > 0.  NULL: the edge lengths (then
 *                        every edge must be finite).
 *   drift_c2, drift_c3   [E] higher drift terms: mu_e(x) = a_e + c_e x +
 *                        c2_e x^2 + c3_e x^3 (NULL: 0); finite.
 *   sigma_c1..sigma_c3   [E] position-dependent diffusion: sigma_e(x) =
 *                        sigma_e + s1_e x + s2_e x^2 + s3_e x^3 (NULL: 0),
 *                        > 0 on all of [0, L_e].  The paper allows any C^1
 *                        coefficients (Sec. 2.2); cubics cover double-well
 *                        potentials and graded diffusivities.  Each sub-step
 *                        freezes both at its starting point (Euler-Maruyama,
 *                        Alg. 2).  Nonzero higher terms need finite edges;
 *                        FP32 sets on such a graph run MG_SCHED_POOLS_W8
 *                        (MG_SCHED_AUTO's choice, no probing) or
 *                        MG_SCHED_LANES; the other pool schedules are
 *                        refused, and an FP32 batch does not mix them with
 *                        sets on affine graphs (FP64 batches may).
 *   vtx_kill, vtx_sticky [V] a_v and c_v of Wentzell vertices (finite, >= 0;
 *                        read only there; NULL: 0).
 *   table_offsets        [E+1] or NULL: tabulated coefficient functions (any
 *                        C^1 drift and diffusion, Sec. 2.2).  Edge e with
 *                        K + 1 = table_offsets[e+1] - table_offsets[e] >= 2
 *                        knots (0: no table) has, at x_j = j L_e / K,
 *                        j = 0..K, the drift value and slope
 *                        table_mu/table_dmu and the diffusion value and
 *                        slope table_sigma/table_dsigma (entry
 *                        table_offsets[e] + j, finite); its mu_e and sigma_e
 *                        are their cubic Hermite interpolants (C^1, exact for
 *                        cubics), which replace drift_a, drift_c, sigma (still
 *                        validated) and require zero higher terms and a
 *                        finite edge; the tabulated sigma must be > 0 on all
 *                        of [0, L_e].  Graphs with tables run like graphs with
 *                        higher terms (FP32 schedules below).
 *   table_mu, table_dmu, table_sigma, table_dsigma  [table_offsets[E]].
 * Every edge must appear exactly once at its initial vertex with orient 0
 * and once at its terminal vertex with orient 1 (a self-loop twice at its
 * vertex).  A standard vertex needs at least one slot with b > 0.
 */
typedef struct {
  int32_t n_vertices, n_edges;
  const int32_t *edge_init, *edge_term;
  const double *length;
  const double *drift_a, *drift_c;
  const double *sigma;
  const int32_t *vtx_offsets;
  const int32_t *slot_edge;
  const uint8_t *slot_orient;
  const double *slot_jump_prob;
  const uint8_t *vtx_kind;
  const double *bin_span;
  const double *drift_c2, *drift_c3;
  const double *sigma_c1, *sigma_c2, *sigma_c3;
  const double *vtx_kill, *vtx_sticky;
  const int32_t *table_offsets;
  const double *table_mu, *table_dmu, *table_sigma, *table_dsigma;
} mg_graph_desc;

/* Validates and packs the graph into device tables (edge records, slot
 * thresholds, vertex records).  *out is NULL on failure. */
mg_status mg_graph_create(const mg_graph_desc *desc, mg_graph **out);
void mg_graph_destroy(mg_graph *g);

/*
 * Options of a particle set.
 *   precision     MG_FP64 (reference arithmetic) or MG_FP32 (positions held
 *                 relative to the nearer edge end, compensated remaining
 *                 time, FP64 crossing solve within 1e-6 L of a vertex,
 *                 off the vertex itself).
 *   max_splits    M in [1, 255], the most vertex hits per step (0: default 8).
 *   graph_tag     fourth Philox counter word; independent streams for sets
 *                 that share seeds (e.g. the members of a batch).
 *   trace         nonzero: keep a per-particle hit-sequence hash and hit
 *                 count, readable with mg_particles_read.
 *   steps_per_launch  steps fused in one kernel launch (0: automatic).
 *   hip_stream    hipStream_t to enqueue on (NULL: null stream).
 *   arena, arena_bytes  optional caller-owned device memory for all of the
 *                 set's device arrays (size from mg_particles_arena_bytes);
 *                 NULL: the library allocates.  The arena must outlive the
 *                 set.
 *   schedule      FP32 kernel schedule: MG_SCHED_AUTO (0), MG_SCHED_LANES
 *                 (1: one particle per lane for a whole launch) or
 *                 MG_SCHED_POOLS (2: each wave cycles 128 particles through
 *                 its lanes and resolves vertex hits in full-width passes),
 *                 MG_SCHED_POOLS256 (3: the same with 256 particles) or
 *                 MG_SCHED_POOLS_W8 (4: pools of 128 whose lanes take
 *                 windows of 8 first sub-steps, two Philox groups, per
 *                 pass instead of 4).
 *                 Results are identical; only the speed differs.  FP64 sets
 *                 run MG_SCHED_LANES or MG_SCHED_POOLS_W8 (FP64 wave pools
 *                 of 128 with 8-step windows, also the automatic choice;
 *                 MG_SCHED_POOLS and MG_SCHED_POOLS256 are refused), with
 *                 identical results, in mg_simulate and in batches.
 *                 On a graph with higher coefficient terms (mg_graph_desc)
 *                 FP32 sets accept only MG_SCHED_AUTO, MG_SCHED_LANES and
 *                 MG_SCHED_POOLS_W8.
 */
typedef enum {
  MG_SCHED_AUTO = 0, MG_SCHED_LANES = 1, MG_SCHED_POOLS = 2, MG_SCHED_POOLS256 = 3,
  MG_SCHED_POOLS_W8 = 4
} mg_schedule;

typedef struct {
  mg_precision precision;
  int32_t max_splits;
  uint32_t graph_tag;
  int32_t trace;
  int32_t steps_per_launch;
  void *hip_stream;
  void *arena;
  int64_t arena_bytes;
  int32_t schedule;
} mg_options;

typedef enum {
  MG_INIT_EXPLICIT = 0,        /* edge[i], pos[i] given (host arrays) */
  MG_INIT_AT_VERTEX = 1,       /* all on `vertex`; edge drawn from b_vertex */
  MG_INIT_UNIFORM_LENGTH = 2   /* edge with prob. L_e / sum L, x ~ U(0, L_e) */
} mg_init_mode;

/* Bytes of device memory a particle set of n particles needs. */
int64_t mg_particles_arena_bytes(const mg_graph *g, int64_t n,
                                 const mg_options *opt);

/*
 * Creates n particles (1 <= n <= 2^32 - 2^20) on graph g.  Random draws of
 * the non-explicit modes use the init stream of Philox keyed by init_seed.
 * EXPLICIT needs 0 <= pos[i] <= L_{edge[i]}; a position on an end means the
 * particle sits on that vertex.  AT_VERTEX needs a standard vertex.  The set
 * keeps a reference to g, which must outlive it.  The step counter starts
 * at 0.
 */
mg_status mg_particles_init(const mg_graph *g, int64_t n, mg_init_mode mode,
                            const int32_t *edge, const double *pos,
                            int32_t vertex, uint64_t init_seed,
                            const mg_options *opt, mg_particles **out);
/*
 * Creates n particles injected at source vertices (the inlets of the
 * tracer problem, Sec. 4.2): particle i starts on source j with probability
 * rates[j] / sum(rates), on an incident edge drawn from that vertex's b
 * (Alg. 1's vertex rule, as in MG_INIT_AT_VERTEX).  Init-stream word 0
 * draws the source (thresholds built like the slot thresholds: normalised
 * running sum, floor(C 2^32), 2^32 for the last source of positive rate),
 * word 1 the slot.  vertices[n_sources] must be standard vertices and
 * rates[n_sources] finite, >= 0, with a positive sum (host arrays).  A
 * continuous injection at these rates has as its steady state the time
 * integral of one such pulse, which the streamed histogram accumulates.
 */
mg_status mg_particles_init_sources(const mg_graph *g, int64_t n, int32_t n_sources,
                                    const int32_t *vertices, const double *rates,
                                    uint64_t init_seed, const mg_options *opt,
                                    mg_particles **out);
/* Frees a set (NULL-safe) once all work on the device has finished. */
void mg_particles_destroy(mg_particles *p);

/*
 * Advances every particle by n_steps steps of size dt > 0 (Alg. 2), using
 * Philox keyed by seed; the set's step counter advances by n_steps, so
 * k calls of n steps equal one call of k*n steps bit for bit.  The step
 * counter must stay below 2^32.  Exit counts, absorbed counts, truncations
 * and sub-step counts accumulate across calls.
 */
mg_status mg_simulate(mg_particles *p, int64_t n_steps, double dt, uint64_t seed);

/*
 * Uniform-bin histogram of the alive particles (appendix kernels):
 * out[e * bins_per_edge + b] = number of particles on e with
 * min(bins_per_edge - 1, floor(x * (bins_per_edge / S_e))) = b, where S_e is
 * the edge's binned length (mg_graph_desc.bin_span; the edge length when
 * none was given), so bins have width S_e / bins_per_edge and positions at
 * or beyond S_e count in the last bin.  The inverse width is formed in FP64.
 * out_len must be >= E * bins_per_edge.  Synchronises the stream.
 */
mg_status mg_histogram(const mg_particles *p, int32_t bins_per_edge,
                       uint64_t *out, int64_t out_len);

/*
 * Histogram over per-edge bins of any count and widths (appendix kernels,
 * the general histogram): edge e owns bins bin_offsets[e] ..
 * bin_offsets[e+1] - 1 (bin_offsets[E+1], bin_offsets[0] = 0, at least one
 * bin per edge), whose upper boundaries bin_upper[] (FP64, measured from the
 * edge's initial vertex) increase strictly from 0 along the edge; the last
 * one is normally L_e.  An alive particle at x goes to the first bin of its
 * edge whose upper boundary is >= x, or to the edge's last bin if x exceeds
 * them all.  bin_offsets and bin_upper are host arrays, copied per call;
 * out[bin_offsets[E]] (host or device).  Allocates device memory for the
 * bin tables; synchronises the stream.
 */
mg_status mg_histogram_csr(const mg_particles *p, const int32_t *bin_offsets,
                           const double *bin_upper, uint64_t *out, int64_t out_len);

/*
 * mg_histogram_csr without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, validation and result as
 * mg_histogram_csr.  The bin tables, and the counters when `out` is host
 * memory, are staged in a fixed workspace of MG_NOALLOC_SCRATCH_BYTES per
 * GPU (a device array of the library, created when the library loads on
 * that GPU and held until the process ends): offsets and boundaries take
 * 256-byte-aligned 4 (E + 1) + 8 bin_offsets[E] bytes, plus
 * 8 bin_offsets[E] for a host `out` (about 2e6 bins with host output).
 * Larger tables give MG_EINVAL.  The call allocates no memory (no hipMalloc,
 * hipFree or allocating library routine), clears the counters with a
 * kernel, and synchronises the set's stream.  Every call on one GPU shares
 * that GPU's workspace: calls that overlap on one GPU (other threads,
 * other streams) race and must be serialised by the caller.
 */
#define MG_NOALLOC_SCRATCH_BYTES (32u << 20)
mg_status mg_histogram_csr_noalloc(const mg_particles *p, const int32_t *bin_offsets,
                                   const double *bin_upper, uint64_t *out,
                                   int64_t out_len);

/*
 * Streamed (time-averaged) histogram, accumulated inside the step kernels.
 * After this call, whenever a step brings the set's step counter to a
 * multiple of `every` (1 <= every <= 2^30), every alive particle adds one
 * count to its bin (binning as in mg_histogram, bins_per_edge per edge) in
 * an accumulator of E * bins_per_edge u64 counters owned by the set.  The
 * sum over a run approximates the time integral of the density (the
 * stationary density after burn-in, Sec. 4.1's error measurement).  The
 * accumulator starts at zero; calling again discards it and starts a new
 * one; every = 0 turns streaming off.  Allocates device memory for the
 * accumulator (outside any arena); first waits for all work on the device
 * (a batch may run the set on another stream).  Batched sets stream too.
 */
mg_status mg_observe_histogram(mg_particles *p, int32_t bins_per_edge, int32_t every);

/*
 * Reads the accumulator into out[E * bins_per_edge] (out may be NULL) and
 * the number of snapshots taken so far into *n_snapshots (may be NULL).
 * MG_ESTATE if streaming is off.  Synchronises the stream.
 */
mg_status mg_observed_histogram(const mg_particles *p, uint64_t *out, int64_t out_len,
                                int64_t *n_snapshots);

/*
 * Empirical L2 distance between the density a histogram estimates and a
 * reference density (the error measure of Sec. 4.1, Fig. "error"):
 *   l2 = sqrt( sum_e sum_k w_e (c_ek / (mass w_e) - ref_ek)^2 ),
 * with w_e = L_e / bins_per_edge the bin width on edge e, c the counts
 * (E * bins_per_edge, edge-major) and ref the reference density averaged
 * over each bin.  mass = 0 takes mass = sum of the counts (the estimate then
 * has total mass 1).  counts and ref_density may be host or device memory.
 * Runs on the host in FP64 with compensated summation.
 */
mg_status mg_density_l2(const mg_graph *g, int32_t bins_per_edge, const uint64_t *counts,
                        double mass, const double *ref_density, double *l2);

/*
 * Accumulated counters (Corollary 1 exit edges): slot_counts[nnz] counts,
 * per slot, the steps whose last vertex hit drew that slot (alive
 * particles); absorbed[V] the particles removed at each vertex;
 * totals[4] = {truncated steps, sub-steps (consumed normals), vertex hits,
 * steps}.  Any pointer may be NULL.  Synchronises the stream.
 */
mg_status mg_exit_counts(const mg_particles *p, uint64_t *slot_counts,
                         uint64_t *absorbed, uint64_t *totals);

/*
 * Copies particles [first, first + count): edge id, position from the
 * edge's initial vertex (FP64; FP32 sets are converted; a particle held on
 * a Wentzell vertex that still owes a stay of t there reads -t at the
 * edge's initial end, L + t at its terminal end), alive flag, and,
 * for traced sets, the hit-sequence hash (FNV-1a over 32-bit words
 * (step, slot) per hit, (step, 0x80000000 | vertex) for an absorption) and
 * the hit count.  Any pointer may be NULL.  Synchronises the stream.
 */
mg_status mg_particles_read(const mg_particles *p, int64_t first, int64_t count,
                            int32_t *edge, double *pos, uint8_t *alive,
                            uint64_t *seqhash, uint32_t *hits);

/* Steps taken so far (the set's step counter). */
int64_t mg_particles_step(const mg_particles *p);

/*
 * Event trace of chosen particles (a parity and debugging aid): with the
 * trace on, every vertex hit of a chosen particle (Alg. 2's crossing: the
 * fraction alpha = u^2 of the sub-step's time, the vertex, the slot drawn
 * there by Alg. 1's rule) appends one record, in every schedule and in
 * batches.
 *
 * mg_trace_events chooses n_ids distinct particle ids (0 <= id < n,
 * n_ids <= 4096, any order) and keeps at most `capacity` records
 * (1 .. 2^26) in device memory the library allocates; n_ids = 0 turns the
 * trace off and frees it.  Every call clears the records and the count.
 * The set must have been created with trace (MG_ESTATE otherwise).  First
 * waits for all work on the device (a batch may run the set on another
 * stream).
 *
 * mg_trace_read copies min(count, out_len) records into host memory out
 * (NULL with out_len 0: count only) and sets *n_events to the number of
 * hits recorded since mg_trace_events (records past the capacity are
 * dropped, so *n_events may exceed it).  Records of one particle come in
 * step and hit order; different particles interleave.  Synchronises the
 * stream.
 */
typedef struct {
  uint32_t pid;       /* particle id */
  uint32_t step;      /* the step counter value of the step */
  int32_t k;          /* hit index within the step, from 1 */
  int32_t vertex;     /* the vertex hit */
  int32_t slot;       /* slot drawn, -1 when the particle was removed there */
  int32_t reserved;
  double u;           /* sqrt(alpha): the crossing root of the sub-step */
  double h_after;     /* time left in the step after the crossing */
} mg_event;

mg_status mg_trace_events(mg_particles *p, int32_t n_ids, const int64_t *ids,
                          int64_t capacity);
mg_status mg_trace_read(const mg_particles *p, mg_event *out, int64_t out_len,
                        int64_t *n_events);

/*
 * Checkpoint and resume.  The appendix's kernels leave every particle's
 * state in global memory between launches; with counter-based draws that
 * state and the step counter are all a later step depends on, so a set
 * saved after k steps and loaded again continues exactly as the original
 * would: the same states, counters and histograms, bit for bit, under any
 * schedule.
 *
 * mg_particles_image_bytes: size of p's image (-1 if p is NULL).
 *
 * mg_particles_save writes the image into caller-owned HOST memory
 * image[0 .. image_bytes) after every step queued on the set's stream has
 * finished (it synchronises the stream).  The image is an mg_image_header
 * (below) followed by, at 8-byte aligned offsets: the state words [n]
 * (u32: edge | FP32 reference-end bit 30 | removed bit 31), positions [n]
 * (FP64: f64 from the initial vertex; FP32: the (distance, compensation)
 * float pair from the reference end), with trace the hashes [n] (u64) and
 * hit counts [n] (u32), exit counts [nnz], absorbed counts [V], the four
 * totals (u64 each), and the streamed histogram [E * bins] (u64) when it is
 * on; all in the host's byte order.  Errors: MG_EINVAL for NULL arguments,
 * a short or device buffer; MG_EDEVICE when the set's device error word is
 * set (its state is not saved).
 *
 * mg_particles_load creates a new set on g from an image.  g must be a
 * graph created from the same description (the header's fingerprint and
 * sizes must match).  The image fixes precision, max_splits, graph_tag and
 * trace (opt's values for them are ignored); opt gives the stream, arena,
 * schedule and steps_per_launch (NULL: defaults).  Every particle is
 * checked on the host as the step kernels would check it (edge in range, a
 * finite position on the edge or owing a stay on a Wentzell end); a bad or
 * truncated image returns MG_EINVAL and creates nothing.  The image stays
 * the caller's.  Tuning results are not part of the image: an automatic
 * FP32 schedule is tuned again (or read from the tuning file) on the first
 * mg_simulate, which changes no result.
 */
typedef struct {
  char magic[8];           /* "MGSETIMG" */
  uint32_t version;        /* 1 */
  uint32_t header_bytes;   /* sizeof(mg_image_header) = 96 */
  uint64_t total_bytes;    /* the whole image */
  uint64_t graph;          /* fingerprint of the graph's packed tables */
  int64_t n;
  int32_t n_vertices, n_edges, nnz;
  int32_t precision, max_splits;
  uint32_t graph_tag;
  int32_t trace;
  int32_t obs_bins;        /* streamed histogram: bins per edge, 0 when off */
  uint64_t obs_every;      /* its period in steps */
  uint64_t obs_start;      /* the step counter when it started */
  uint64_t step;           /* the set's step counter */
} mg_image_header;

int64_t mg_particles_image_bytes(const mg_particles *p);
mg_status mg_particles_save(const mg_particles *p, void *image, int64_t image_bytes);
mg_status mg_particles_load(const mg_graph *g, const void *image, int64_t image_bytes,
                            const mg_options *opt, mg_particles **out);

/*
 * Batch of independent particle sets (possibly on different graphs) that
 * mg_batch_simulate advances in one launch per steps_per_launch chunk and
 * LDS group: mg_batch_create groups the sets by the kernel occupancy that
 * their graphs' per-block exit counters (and staged tables) leave, so that
 * small graphs do not run at the occupancy of the largest one; a group
 * with under 1/32 of the particles joins the next group of larger need.
 * All sets must have the same precision, max_splits, trace flag and
 * schedule; each keeps its own graph_tag, counters and step counter, and
 * every set's results equal those of mg_simulate on that set alone.  The
 * batch references the sets, which must outlive it; it launches on the
 * first set's stream.
 */
mg_status mg_batch_create(int32_t n_sets, mg_particles *const *sets, mg_batch **out);
mg_status mg_batch_simulate(mg_batch *b, int64_t n_steps, double dt, uint64_t seed);
void mg_batch_destroy(mg_batch *b);

/*
 * Autotuning of an FP32 set's kernel schedule.  The candidates (one
 * particle per lane; wave pools of 128 particles (2 per lane) that start a
 * partial split pass at 4, 8, 16 or 32 idle lanes; pools of 256 (4 per
 * lane) at 8 or 16; pools of 128 with 8-step windows at 8, 16 or 32) all
 * give identical results, so tuning changes only
 * speed.  Each candidate advances a scratch copy of the set's first
 * min(n, 2^22) particles by probe_steps steps (<= 0: 1024) of size dt with
 * Philox key seed, timed with HIP events on the set's stream; the set
 * keeps the fastest for its later mg_simulate calls at this dt.  The
 * chosen schedule then runs 2 probe_steps steps as one launch and as two
 * launches; a set created with steps_per_launch 0 takes the faster (0: the
 * whole call per launch, else probe_steps steps per launch).  The
 * result is also kept with the graph: later calls for any set on the same
 * graph at the same dt take it without probing.  With the environment
 * variable MG_TUNE_CACHE naming a file, results also outlive the process:
 * before probing, the call looks there for a line with the same GPU
 * architecture name and compute-unit count, graph (a fingerprint of its
 * packed tables), probed particle count, max_splits, dt and probe_steps,
 * and takes that result (n_probes 0, no probe times); after probing it
 * appends one JSON line with the key and the choice.  Lines that do not
 * parse are skipped; a file that cannot be read or written is ignored.
 * Sets created with
 * schedule MG_SCHED_AUTO are tuned this way on their first mg_simulate at
 * each dt; until then (and in a batch built from untuned sets) they use
 * pools of 128 with 8-step windows.  Fixed pool schedules start a partial
 * pass at 16 idle lanes.  FP64 sets have nothing to probe (their set's FP64 schedule).  `out` (may be
 * NULL) receives the choice and the probe times.  A probe allocates scratch
 * device memory and synchronises the stream.
 */
typedef struct {
  int32_t schedule;      /* MG_SCHED_LANES, _POOLS, _POOLS256 or _POOLS_W8 */
  int32_t idle_trigger;  /* pools: idle lanes that start a partial split pass */
  int32_t pool_size;     /* pools: particles per wave (128 or 256), else 0 */
  int32_t window;        /* first sub-steps per lane and pass (4 or 8) */
  int32_t n_probes;      /* entries used in probe_ms */
  float probe_ms[12];    /* lanes, pools128@4, @8, @16, @32, pools256@8, @16,
                            pools128 8-step windows@8, @16, @32 */
  int32_t steps_per_launch;  /* 0: a whole call per launch; else the chunk */
  float launch_ms[2];    /* the chosen schedule over 2 probe_steps steps: one
                            launch, two launches of probe_steps */
} mg_tuning;

mg_status mg_autotune(mg_particles *p, double dt, uint64_t seed, int32_t probe_steps,
                      mg_tuning *out);

/*
 * Measurement aid, not part of the method: the issue rate of one VALU
 * instruction kind on the calling thread's current GPU, for setting the
 * step kernels' instruction counts against a measured ceiling.  Every SIMD
 * runs waves_per_simd (1 .. 8) waves; each lane runs 8 independent chains
 * of `op` for 128 x iters (1 .. 2^20) rounds.  One untimed launch, then one
 * timed with HIP events on a stream of the call's own.  *lane_ops_per_s
 * gets lanes x rounds x chains / seconds (one lane-op = one lane of one
 * instruction), *kernel_ms (if not NULL) the timed launch.  Allocates a
 * device buffer of 4 bytes per lane for the chains' results and frees it;
 * synchronises.  MG_EINVAL for an unknown op or a count out of range,
 * MG_EDEVICE for a HIP error.
 */
typedef enum {
  MG_VALU_FMA_F32 = 0,      /* v_fma_f32 (not packed) */
  MG_VALU_FMA_F64 = 1,      /* v_fma_f64 */
  MG_VALU_MAD_U64_U32 = 2,  /* v_mad_u64_u32: 32 x 32 -> 64-bit multiply-add */
  MG_VALU_BITOP3 = 3,       /* v_bitop3_b32: any bitwise function of 3 words */
  MG_VALU_ADD_U32 = 4,      /* v_add_u32 */
  MG_VALU_LOG_F32 = 5       /* v_log_f32: the transcendental unit */
} mg_valu_op;

mg_status mg_valu_rate(int32_t op, int32_t waves_per_simd, uint32_t iters,
                       double *lane_ops_per_s, float *kernel_ms);

/* Description of the calling thread's last error ("" if none). */
const char *mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* METRICGRAPH_H */
