/* qedx.h -- C ABI of the batched tree-level QED |M|^2 library (MI355X, gfx950).
 *
 * Process: e-(p) gamma(k) -> e-(p') gamma(k'_1) ... gamma(k'_n), n = 1..6, one
 * electron line, all (n+1)! tree diagrams (Sec. III-A of the paper: the number
 * of orderings in which the photons bind to the electron).  The amplitude is
 * the paper's computation graph (Sec. II-B: base states U, vertices V,
 * propagators S1, joins S2, diagram Sum) after node reduction (App. C),
 * compiled into one straight-line GPU kernel per process variant.
 *
 * Conventions shared by every entry point
 *  - Units hbar = c = 1, electron mass m = 1, metric (+,-,-,-).
 *  - Particle order: [e-_in, gamma_in, e-_out, gamma_out_1..n].
 *  - Momenta are float64 SoA, [4*(n+3)][N] row-major: row 4*i + mu holds
 *    component mu (E, px, py, pz) of particle i for all N points.  The caller
 *    guarantees on-shell momenta and momentum conservation.
 *  - Reported value: reduced |M|^2 = sum over the selected spin/polarisation
 *    configurations of |A|^2 with the coupling e and the overall phase of
 *    (-ie)^(n+1) i^n dropped; the physical value is (4 pi alpha)^(n+1) times it.
 *  - Helicity code (uint32): bit i belongs to particle i; 0 = spin +1/2 (rest
 *    frame z spin boosted to p) or linear polarisation x; 1 = spin -1/2 or
 *    polarisation y; x = (cos t cos f, cos t sin f, -sin t), y = (-sin f, cos f, 0)
 *    in the frame of the given momenta, k-hat = (sin t cos f, sin t sin f, cos t).
 *  - Every device pointer must be a device allocation on the current HIP
 *    device, contiguous, 8-byte aligned (4-byte for helicity codes), and must
 *    not alias an output.  The caller owns all device buffers; the library
 *    owns process and plan handles.
 *  - Calls enqueue work on `stream` (a hipStream_t; NULL = default stream)
 *    and return without synchronising.  Launch failures return QED_ERR_HIP.
 *  - On any error the function returns a nonzero status, writes nothing to
 *    the outputs, and qed_last_error() returns a message (thread-local).
 *  - N == 0 is a valid no-op.  Device memory is allocated only by
 *    qed_batch_plan_create (its tile table, counter and, for FP32C, the
 *    fix-up list), by qed_eval_grad for n >= 4, and by qed_eval of FP32C
 *    per-point processes (workspaces owned by the process handle, grown on
 *    demand and freed by qed_process_destroy).
 */
#ifndef QEDX_H
#define QEDX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qed_process qed_process;       /* immutable after create */
typedef struct qed_batch_plan qed_batch_plan; /* segment table + captured graph */

typedef enum {
  QED_OK = 0,
  QED_ERR_INVALID_ARG = 1,
  QED_ERR_UNSUPPORTED = 2,
  QED_ERR_HIP = 3,
  QED_ERR_COMPILE = 4,
  QED_ERR_OOM = 5
} qed_status;

/* QED_HEL_SUM: sum over all 2^(n+3) spin/polarisation configurations.
 * QED_HEL_PER_POINT: one configuration per point, from a helicity array. */
typedef enum { QED_HEL_SUM = 0, QED_HEL_PER_POINT = 1 } qed_hel_mode;

/* QED_FP64: every step in float64.
 * QED_FP32C: currents, vertices, propagator numerators and diagram values in
 * float32 with compensated (TwoSum) accumulation of the diagram sum;
 * momenta, propagator momenta and denominators, |A|^2 and the helicity sum in
 * float64.  Per-point processes recompute in float64 the points whose diagram
 * sum cancels by more than fix_kappa (qed_variant), which keeps the relative
 * error against float64 below 1e-4 on every point of the stated workloads
 * (measured, not a proof for arbitrary points); helicity sums dilute the
 * cancellation of single configurations and meet the bound without it. */
typedef enum { QED_FP64 = 0, QED_FP32C = 1 } qed_precision;

/* Kernel shape knobs (a zero field = library default for the process).
 * lane_bits:  helicity bits spread over lanes (2^popcount lanes per point),
 *             given as a mask over particle bits; SUM mode only.
 * loop_bits:  helicity bits enumerated by a run-time loop; SUM mode only.
 *             lane_bits = loop_bits = 0 keeps the default coverage.
 * The remaining bits are enumerated inside the graph.  block = threads per
 * workgroup (multiple of 64, <= 1024).  split = photons on the e-_in side
 * of every join (1..n). */
typedef struct {
  uint32_t lane_bits;
  uint32_t loop_bits;
  int32_t block;
  int32_t split;
  int32_t min_waves;    /* minimum waves per SIMD the compiler must allow (0 = free) */
  int32_t order;        /* emission schedule flags (0 = library default) */
  int32_t use_defaults; /* nonzero: ignore the fields above and below */
  int32_t rewrite;      /* 0 = node reduction only (the paper's CDAG optimisation, App. C);
                           1 = node reduction followed by the distributive rewrite the paper
                           proposes (Sec. IV): sums over photon orderings are factored, so the
                           diagram sum becomes one join per photon partition and the currents
                           one per photon subset.  Same result up to rounding.  The fused
                           gradient (n <= 3) uses the node-reduced graph; the split gradient
                           (n = 4, 5) sweeps the process's own graph form. */
  int32_t partial;      /* nonzero: instead of the full pipeline, the paper's unsplit graph
                           after only the first partial_steps single node reductions in the
                           random order seeded by partial_seed (0 steps = unreduced), emitted
                           as one straight-line block; for the reduction experiment of
                           Sec. III-D (kernel time against the number of reductions). */
  int32_t partial_steps;
  uint32_t partial_seed;
  int32_t fixup;        /* FP32C per-point processes: 0 = default (on), < 0 = off.  The FP32C
                           kernel also sums |diagram value|^2; where the square root of that
                           sum exceeds fix_kappa * |A|, the diagram sum cancels beyond what
                           FP32 currents resolve, the point is listed, and a second kernel
                           recomputes the listed points in FP64 (qed_eval launches both on
                           the stream). */
  float fix_kappa;      /* cancellation threshold (0 = library default, 16) */
} qed_variant;

typedef struct {
  int32_t n, mode, precision;
  int64_t nodes_unreduced;   /* CDAG size before node reduction, in-lane graph */
  int64_t nodes_reduced;     /* after reduction and join expansion */
  int64_t n_V, n_S1, n_dot, n_prop;
  double flops_per_point;    /* algorithmic FLOPs per point (add/mul 1, fma 2) */
  int32_t lanes_per_point, block;
  int32_t vgpr, agpr, sgpr, scratch_bytes, lds_bytes; /* from the code object */
  double create_ms_build, create_ms_reduce, create_ms_emit, create_ms_compile, create_ms_load;
  int32_t cache_hit;         /* 1 if the code object came from the cache */
  char kernel_tag[160];      /* kernel shape: process, mode, precision, helicity coverage, schedule */
  char code_hash[24];        /* hash of the eval kernel's source, flags and target (changes with the code) */
  char kernel_name[48];      /* symbol of the eval kernel, qedx_eval_[i<n_in>]n<n>_<sum|pp>_<fp64|fp32c>[_d1][_k<steps>] */
  int32_t n_in;              /* incoming photons (1 unless created by qed_process_create_crossed) */
  int32_t fixup;             /* 1 if the FP32C kernel has the FP64 fix-up pass */
  double fix_kappa;          /* its cancellation threshold */
} qed_info;

/* Build the graph for n outgoing photons (1..6), reduce it, emit and compile
 * (or load from the code-object cache) the kernel.  Loads the module on the
 * current device.  `variant` may be NULL.  Returns QED_ERR_COMPILE if the
 * generated code does not compile, QED_ERR_UNSUPPORTED for n outside 1..6
 * or a mode/precision not built for that n. */
qed_status qed_process_create(int n, qed_hel_mode mode, qed_precision prec, const qed_variant* variant,
                              qed_process** out);
/* The crossed process e-(p) + n_in photons -> e-(p') + n_out photons on one
 * electron line (n_in, n_out >= 1, n_in + n_out <= 7), e.g. the paper's Table I
 * processes e- gamma^n -> e- gamma (n_out = 1).  Same (n_in + n_out)! diagrams
 * and graph; particle order [e-_in, gamma_in_1..n_in, e-_out, gamma_out_1..n_out],
 * so momenta are [4(n_in + n_out + 2)][N] and helicity bit i belongs to
 * particle i.  Incoming photons carry eps, outgoing eps* (equal: real linear
 * polarisations).  qed_eval works as for one incoming photon; qed_rambo,
 * qed_eval_grad and qed_batch_plan_create return UNSUPPORTED for n_in > 1. */
qed_status qed_process_create_crossed(int n_in, int n_out, qed_hel_mode mode, qed_precision prec,
                                      const qed_variant* variant, qed_process** out);
qed_status qed_process_destroy(qed_process* p);
qed_status qed_process_info(const qed_process* p, qed_info* out);

/* |M|^2 for N points (Sec. II-B: the graph takes all four-momenta and returns
 * one real number per point).
 * momenta: device, float64 [4(n+3)][N]; hel: device uint32 [N] in PER_POINT
 * mode and NULL in SUM mode; out: device float64 [N].
 * INVALID_ARG if N < 0, a required pointer is NULL while N > 0, or hel does not
 * match the mode.  FP32C per-point processes with the FP64 fix-up keep a
 * device workspace of 4(N + 1) bytes (allocated, or grown, by the first call
 * with a larger N; freed by qed_process_destroy); calls on one such process
 * must not overlap, and N is limited to 2^32 - 1 for them. */
qed_status qed_eval(const qed_process* p, const double* momenta, const uint32_t* hel, int64_t N, double* out,
                    void* stream);

/* RAMBO phase space (Kleiss, Stirling, Ellis 1986) for this process at
 * centre-of-mass energy sqrt_s > m: writes full momenta [4(n+3)][N] with the
 * incoming pair in its CM frame (photon along +z) and the final state
 * [e-_out (mass 1), n photons] from uniforms [4(n+1)][N] in (0,1) (rows
 * 4j..4j+3 belong to final-state particle j).  INVALID_ARG if sqrt_s <= 1. */
qed_status qed_rambo(const qed_process* p, const double* uniforms, double sqrt_s, int64_t N, double* momenta_out,
                     void* stream);

/* log|M|^2 (SUM mode processes) and its gradient with respect to the RAMBO
 * uniforms: out_logm2 [N], out_grad [4(n+1)][N] (row = uniform index), both
 * float64 device buffers.  The gradient is the reverse sweep of the graph:
 * currents are recomputed from their parents on the way back, not stored.
 * n <= 3: forward RAMBO, forward graph, adjoint graph and adjoint RAMBO in one
 * kernel.  n = 4, 5: per chunk of points, RAMBO into a workspace, one kernel
 * storing every configuration's amplitude A_h and 1/|M|^2 (the adjoint seeds
 * conj(A_h)/|M|^2), one adjoint kernel per photon partition, and the RAMBO
 * adjoint; the workspace (about 2.5 KB per point at n = 4, 320 MB at most)
 * belongs to the process, so calls on one process must not overlap on
 * different streams.  `hel` must be NULL.  UNSUPPORTED for PER_POINT or FP32C
 * processes and for n = 6.  QED_ERR_OOM if the workspace cannot be allocated. */
qed_status qed_eval_grad(const qed_process* p, const double* uniforms, double sqrt_s, const uint32_t* hel,
                         int64_t N, double* out_logm2, double* out_grad, void* stream);

/* Mixed-process batches: segments of different processes evaluated by one
 * persistent kernel launch (captured in a HIP graph at plan creation).
 * All processes of one plan must share the precision (and, for FP32C, the
 * FP64 fix-up setting) and be PER_POINT. */
typedef struct {
  const qed_process* proc;
  const double* momenta; /* device [4(n+3)][N] */
  const uint32_t* hel;   /* device [N] */
  int64_t N;
  double* out;           /* device [N] */
} qed_segment;

/* tile_points = points per work tile, a multiple of 64 (0 = autotuned: a few
 * grid sizes and tile lengths are timed on the given buffers, which are
 * overwritten, after a device synchronisation; the choice is cached by plan
 * signature).  The plan copies the segment table to the device, allocates a
 * 256-byte tile counter, and instantiates a HIP graph of two kernel nodes
 * (counter clear, persistent kernel).  FP32C plans (per-point processes with
 * the FP64 fix-up) also allocate a list of 4(1 + 2 x total points) bytes and
 * add two nodes (list clear, FP64 pass over the listed points); the threshold
 * is the first segment's process's fix_kappa, and the total must stay below
 * 2^31 points.  The segment buffers must stay valid while the plan is
 * launched.  Plans are not thread-safe: launches of one plan on overlapping
 * streams race on its counter. */
qed_status qed_batch_plan_create(const qed_segment* segs, int nseg, int tile_points, qed_batch_plan** out);
qed_status qed_batch_launch(qed_batch_plan* plan, void* stream);
qed_status qed_batch_plan_destroy(qed_batch_plan* plan);
/* Tile layout chosen for a plan: tiles in the tile space, workgroups of the
 * persistent grid, 64-point chunks per tile. */
qed_status qed_batch_info(const qed_batch_plan* plan, int64_t* ntiles, int* grid, int* chunk);
/* Ahead-of-time build of the batch module for the per-point processes
 * n_list[0..count) with default kernel shapes, node-reduced (rewrite = 0) or
 * distributed (rewrite = 1) (no GPU needed). */
qed_status qed_batch_prebuild(const int* n_list, int count, qed_precision prec, int rewrite, double* compile_ms);

/* Last error message of the calling thread ("" if none). */
const char* qed_last_error(void);

/* FP64 pipe probe (measurement tool, not part of the evaluation path).
 * After the distributive factoring of the helicity-summed join (Sec. II-B
 * join task, Sec. IV term rewriting), the join of one photon partition is a
 * small dense complex product that could run on the FP64 matrix pipe
 * (v_mfma_f64_16x16x4) beside the vector code that builds the currents.  This
 * call measures that ceiling: blocks workgroups of 256 lanes, launched on
 * stream (hipStream_t, may be NULL):
 *  kind 0, vector pipe: each lane runs 8 chains a <- fma(a, m, c), iters
 *    steps, from a_j = (lane % 64) + j, j = 0..7; out[lane] = sum of the 8
 *    chains (16 iters FLOPs per lane).
 *  kind 1, matrix pipe: each wave runs 4 chains of iters (a multiple of 8)
 *    v_mfma_f64_16x16x4 on C += A.B, A[i][k] = a[i + 16k], B[k][j] =
 *    b[j + 16k] (a, b: 64 doubles each); out[4 * lane + r] = the sum of the 4
 *    accumulators' item r, which holds C[(lane % 64) / 16 + 4r][lane % 16]
 *    (2048 FLOPs per instruction per wave).
 *  kind 2, both: even waves of each workgroup run kind 0 with iters steps
 *    into out, odd waves kind 1 with iters2 steps into out2.
 * All pointers are device buffers sized blocks * 256 (out of kind 0 and 2)
 * or blocks * 1024 doubles (out of kind 1, out2), owned by the caller.
 * Errors: INVALID_ARG for kind outside 0..2, blocks outside 1..2^24,
 * negative counts, matrix-pipe counts not a multiple of 8, or missing
 * buffers. */
qed_status qed_pipe_probe(int kind, int64_t blocks, int64_t iters, int64_t iters2, double m, double c,
                          const double* a, const double* b, double* out, double* out2, void* stream);
/* Compile the probe's code object into the cache (no GPU). */
qed_status qed_pipe_probe_prebuild(double* compile_ms);

/* Code-object cache directory in use (QEDX_CACHE_DIR or the package default). */
const char* qed_cache_dir(void);

/* Host-side graph tools (no GPU needed), for inspection and tests.
 * qed_graph_counts: node counts of the generated graph for n, enumerated
 * helicity bits `enum_mask` and join split `split`: reduced = 0 gives the
 * paper's unreduced form (one chain per diagram, S2 joins); reduced = 1 the
 * node-reduced, join-expanded form; reduced = 2 that form after the
 * distributive rewrite (see qed_variant.rewrite).  counts[10] = total, data, compute, U, V,
 * S1, S2, Dot, Sum, HelSum. */
qed_status qed_graph_counts(int n, int n_in, uint32_t enum_mask, int split, int reduced, int64_t* counts);
/* Host interpreter of the graph (float64), per point: value of the exit node
 * (sum over enum_mask configurations of |A|^2) with the other bits from hel.
 * reduced as above; mom is host [N][4(n_in+n+2)] (point-major); out host [N]. */
qed_status qed_graph_interpret(int n, int n_in, uint32_t enum_mask, int split, int reduced, const double* mom,
                               const uint32_t* hel, int64_t N, double* out);
/* Canonical structure hash text of the reduced graph reached by (a) the
 * one-pass fixpoint and (b) single reductions in a random order seeded by
 * `seed`; writes at most buflen bytes of each.  Returns the number of single
 * reductions in *steps. */
qed_status qed_graph_reduction_check(int n, int n_in, uint32_t enum_mask, int split, uint64_t seed, char* canon_a,
                                     char* canon_b, int64_t buflen, int64_t* steps);
/* The graph of the reduction experiment (Sec. III-D): the unreduced graph
 * for n outgoing photons, one configuration per point, after the first
 * `steps` single node reductions in the random order seeded by `seed`.
 * Writes counts[10] (as qed_graph_counts) if non-NULL and, for N points
 * (mom host [N][4(n+3)], hel host [N] or NULL), the interpreted |A|^2. */
qed_status qed_graph_partial(int n, int split, int64_t steps, uint64_t seed, const double* mom, const uint32_t* hel,
                             int64_t N, double* out, int64_t* counts);
/* Generated HIP source of the eval kernel for a variant (for inspection and
 * for prebuilding the cache); writes at most buflen bytes, returns the full
 * length in *len. */
qed_status qed_emit_source(int n, qed_hel_mode mode, qed_precision prec, const qed_variant* variant, char* buf,
                           int64_t buflen, int64_t* len);

/* C(DAG) and D(DAG) of the graph (App. B graph metrics): compute effort in
 * FLOPs (add/mul 1, fma 2, div/sqrt 1, per point) and data transfer in bytes,
 * with float32 value sizes if fp32 != 0. */
qed_status qed_graph_metrics(int n, int n_in, uint32_t enum_mask, int split, int reduced, int fp32,
                             double* c_dag, double* d_dag);
/* Emit and compile the kernels of one process variant into the code-object
 * cache without touching the GPU (ahead-of-time build).  with_aux = 1 also
 * builds the RAMBO/gradient module.  *compile_ms receives the compile time
 * (0 on a cache hit). */
qed_status qed_prebuild(int n, qed_hel_mode mode, qed_precision prec, const qed_variant* variant, int with_aux,
                        double* compile_ms);
/* The same for the eval kernel of a crossed process (qed_process_create_crossed
 * arguments); there is no auxiliary module for n_in > 1. */
qed_status qed_prebuild_crossed(int n_in, int n_out, qed_hel_mode mode, qed_precision prec,
                                const qed_variant* variant, double* compile_ms);

/* Host references of the gradient pieces (no GPU), for tests:
 * qed_graph_grad_interpret: F = log(sum over all configurations of |A|^2) and
 * dF/dmom by a reverse sweep over the graph in float64.  mom host [N][4(n+3)]
 * point-major; val [N]; gmom [N][4(n+3)] (rows of the incoming particles 0).
 * qed_rambo_vjp_host: final-state momenta mom [N][4(n+1)] from uniforms
 * u [N][4(n+1)], and gu [N][4(n+1)] = (dk/du)^T gk for given gk [N][4(n+1)]. */
qed_status qed_graph_grad_interpret(int n, int split, int reduced, const double* mom, int64_t N, double* val,
                                    double* gmom);
qed_status qed_rambo_vjp_host(int n, const double* u, double sqrt_s, const double* gk, int64_t N, double* mom,
                              double* gu);

#ifdef __cplusplus
}
#endif

#endif /* QEDX_H */
