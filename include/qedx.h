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
 *  - N == 0 is a valid no-op.  Process handles are read-only after create:
 *    calls on one process from several streams or threads may overlap.
 *    Device memory is allocated, and the device synchronised, only by
 *    create/destroy calls (processes, batch plans); qed_eval, qed_rambo,
 *    qed_eval_grad and qed_batch_launch allocate nothing and do not
 *    synchronise (the split gradient works in a caller-owned workspace).
 *  - Host-side graph tools (inspection, host references for tests) are
 *    declared in qedx_tools.h; they are exported by the same library.
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
 * float64.  Per-point processes recompute in float64 the points whose FP32
 * evaluation the kernel cannot vouch for (fixup, fix_kappa in qed_variant);
 * helicity sums dilute the cancellation of single configurations.  The error
 * against float64 is reported per result by the tests and the benchmark. */
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
  int32_t min_waves;    /* minimum waves per SIMD the compiler must allow (0 = library default) */
  int32_t order;        /* emission schedule flags (0 = library default).  Per-point
                           partition loops (8) may add the one-photon current cache: 256 =
                           2 lanes per point, 512 = 4 lanes per point, 1024 = cache the
                           e-_in side's currents only; qed_process_info reports the
                           resulting lanes_per_point.  Helicity sums with per-partition
                           blocks (4) and the e-_out spin as their one lane bit may add
                           2048 (the two lanes share the e-_in side, each building it for
                           one e-_in spin) and, with it, 4096 (that side's one-photon
                           currents cached in LDS); per-partition blocks may add 8192
                           (each block's momentum loads issued together) */
  int32_t use_defaults; /* nonzero: ignore the fields above and below */
  int32_t rewrite;      /* 0 = node reduction only (the paper's CDAG optimisation, App. C);
                           1 = node reduction followed by the distributive rewrite the paper
                           proposes (Sec. IV): sums over photon orderings are factored, so the
                           diagram sum becomes one join per photon partition and the currents
                           one per photon subset.  Same result up to rounding.  The fused
                           gradient (n <= 3) uses the node-reduced graph; the split gradient
                           (n = 4) sweeps the process's own graph form. */
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
 * match the mode.  FP32C per-point processes with the FP64 fix-up launch two
 * kernels on `stream`: the FP32 pass writes its results and marks the points
 * it cannot vouch for with a negative value in `out`, the FP64 pass
 * recomputes the marked points in place; `out` holds final values once both
 * have run.  No other memory is used. */
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
 * kernel; no workspace (workspace may be NULL).  n = 4: per chunk of points,
 * RAMBO into the workspace, one kernel storing every configuration's
 * amplitude A_h and 1/|M|^2 (the adjoint seeds conj(A_h)/|M|^2), the adjoint
 * kernels of the photon partitions (two per partition: the e-_out-side and
 * the e-_in-side walk), and the RAMBO adjoint.  The workspace is
 * caller-owned device memory, 8-byte aligned, of workspace_bytes bytes: its
 * size sets the chunk (qed_eval_grad_workspace_size gives the size for the
 * largest chunk, about 2.5 KB per point at n = 4, at most 512 MB); less than
 * 64 points' worth (or N's, if smaller) is INVALID_ARG.  Calls that overlap
 * need workspaces of their own.  `hel` must be NULL.  UNSUPPORTED for
 * PER_POINT or FP32C processes and for n >= 5. */
qed_status qed_eval_grad(const qed_process* p, const double* uniforms, double sqrt_s, const uint32_t* hel,
                         int64_t N, double* out_logm2, double* out_grad, void* workspace, int64_t workspace_bytes,
                         void* stream);
/* Workspace bytes qed_eval_grad uses for N points in one chunk (capped at
 * the largest chunk); 0 for processes with the fused gradient kernel. */
qed_status qed_eval_grad_workspace_size(const qed_process* p, int64_t N, int64_t* bytes);

/* qed_eval_grad without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * qed_eval_grad; the n = 4 split gradient runs its chunks through a fixed
 * scratch array the library holds on every GPU it runs on (256 MiB per
 * device, kept until the process ends), which caps a chunk at 2^16 points
 * at n = 4; any N runs, in ceil(N / chunk) passes.  A process whose 64-point
 * chunk would not fit is UNSUPPORTED.  The call allocates nothing and does
 * not synchronise.  All calls on one GPU share that GPU's scratch and the
 * scratch keeps the last call's contents (the kernels initialise what they
 * read): calls that overlap on one GPU (several streams or threads) race and
 * must be serialised by the caller. */
qed_status qed_eval_grad_noalloc(const qed_process* p, const double* uniforms, double sqrt_s, const uint32_t* hel,
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

/* tile_points = lanes per work tile, a multiple of 64: points per tile for
 * processes with one lane per point, half or a quarter of it for processes
 * whose body splits a point over 2 or 4 lanes (0 = autotuned: a few
 * grid sizes and tile lengths are timed on the given buffers, which are
 * overwritten, after a device synchronisation; the choice is cached by plan
 * signature).  The plan copies the segment table to the device, allocates a
 * 256-byte tile counter, and instantiates a HIP graph of two kernel nodes
 * (counter clear, persistent kernel).  FP32C plans (per-point processes with
 * the FP64 fix-up) also allocate 4(64 + total points) bytes (a counter and a
 * point list per segment) and add two nodes (counter clear, FP64 pass over
 * the listed points, segment by segment); the threshold
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

/* Code-object cache directory in use (QEDX_CACHE_DIR or the package default). */
const char* qed_cache_dir(void);

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

#ifdef __cplusplus
}
#endif

#endif /* QEDX_H */
