/* qedx_probe.h -- FP64 pipe probe, a measurement tool kept outside the
 * evaluation library (libqedx_probe.so, which uses libqedx.so's code-object
 * cache and error reporting: qed_last_error() gives its messages).
 */
#ifndef QEDX_PROBE_H
#define QEDX_PROBE_H

#include "qedx.h"

#ifdef __cplusplus
extern "C" {
#endif

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
/* Compile the probe's code objects (this one and the reciprocal probe's)
 * into the cache (no GPU). */
qed_status qed_pipe_probe_prebuild(double* compile_ms);

/* Reciprocal probe (test tool): r[i] = qx::rcp(x[i]) and q[i] =
 * qx::rsqrt(|x[i]|) for i < n, computed by the device functions the
 * generated kernels use for propagator denominators, spinor normalisations
 * and polarisation vectors (the hardware estimates refined by two
 * Newton-Raphson steps).  x, r, q: device buffers of n doubles owned by the
 * caller; x nonzero and well inside the normal range.  Enqueued on stream
 * (hipStream_t, may be NULL).  Errors: INVALID_ARG for n outside 1..2^30
 * or a missing buffer. */
qed_status qed_recip_probe(const double* x, int64_t n, double* r, double* q, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* QEDX_PROBE_H */
