// qedx_emit.hpp -- HIP source generator for the reduced QED computation graph.
#pragma once

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "qedx_dag.hpp"

namespace qedx {

enum Prec : int { PREC_F64 = 0, PREC_F32C = 1 };
enum HelMode : int { HEL_SUM = 0, HEL_PER_POINT = 1 };

// How one kernel instance covers the helicity configurations of a point.
//  - enum_mask: particle bits enumerated inside the graph (shared nodes);
//  - lane_mask: bits taken from the lane index; 2^popcount lanes per point,
//    summed with a wavefront butterfly at the end;
//  - loop_mask: bits enumerated by a run-time loop around the graph body.
// In HEL_PER_POINT mode every bit comes from the per-point input code.
struct Variant {
  int prec = PREC_F64;
  int mode = HEL_SUM;
  uint32_t enum_mask = 0, lane_mask = 0, loop_mask = 0;
  int block = 256;      // threads per workgroup
  int split = 1;        // photons attached on the e-_in side of every join
  int join_side = 1;    // side whose current carries the join propagator
  int order = 0;        // emission order strategy (0 = partition-grouped)
  int min_waves = 0;    // __launch_bounds__ second argument (0 = none)
  int rewrite = 0;      // 0 = node reduction only; 1 = also the distributive rewrite
  int partial = 0;      // 1: unsplit graph after partial_steps single reductions only
  int partial_steps = 0;
  uint32_t partial_seed = 0;
  int fixup = 0;        // 1: FP32C per-point kernel flags ill-conditioned points for an FP64 pass
};

// Lanes of a point that share the one-photon current cache of a per-point
// partition loop and split its partitions: 2 (order flag 256) or 4 (flag
// 512); 1 without the cache.
inline int cache_lanes(const Variant& v) { return (v.order & 512) ? 4 : (v.order & 256) ? 2 : 1; }
// Lanes per phase-space point of an eval kernel: 2^(lane bits) x cache lanes.
inline int lanes_per_point(const Variant& v) { return (1 << __builtin_popcount(v.lane_mask)) * cache_lanes(v); }

// Points scanned by one workgroup of the FP64 fix-up pass.
constexpr int kFixRange = 1024;

struct EmitStats {
  double flops_per_point = 0;   // algorithmic FLOPs per phase-space point
  int64_t n_V = 0, n_S1 = 0, n_dot = 0, n_prop = 0, n_U = 0;
  int64_t lines = 0;
};

// Canonical text of a variant (part of the code-object cache key).
std::string variant_tag(const Variant& v, int n_out, int n_in);

// Build the graph for (process, variant): generate, reduce, expand joins,
// reduce again.  Timings (ms) are written to t_build / t_reduce if non-null.
Dag graph_for(const Process& proc, const Variant& v, double* t_build, double* t_reduce);

// Emit a self-contained HIP translation unit with the device header inlined
// and one kernel
//   extern "C" __global__ void <kname>(const double* mom, const unsigned* hel,
//                                      long long N, double* out)
// mom: [4*npart][N] SoA (row = 4*particle + mu), out: [N].
// With v.fixup (FP32C, per point) the kernel takes one more argument,
// (double fix_kappa), also sums |diagram value|^2 beside the compensated sum,
// and where the square root of that sum exceeds fix_kappa * |A| (a
// cancellation the FP32 currents cannot resolve to the stated bound) writes
// -1 to out[pt] instead of the value.  The module then also holds
//   extern "C" __global__ void <kname>_fix(const double* mom, const unsigned* hel,
//       long long N, double* out)
// launched with ceil(N / kFixRange) workgroups of 256 lanes on the same
// stream: workgroup b scans out[b kFixRange .. (b+1) kFixRange) for negative
// marks and recomputes those points with the FP64 body of the same graph.
// No memory beyond the caller's buffers is used.
std::string emit_eval_kernel(const Dag& d, const Variant& v, const std::string& kname, EmitStats* st);

// Gradient kernel (SUM mode, FP64, partition-local blocks, no loop bits):
//   extern "C" __global__ void <kname>(const double* u, double sqrt_s,
//                                      long long N, double* logm2, double* grad)
// RAMBO forward, forward graph (log |M|^2), adjoint graph and adjoint RAMBO
// in one kernel; u and grad are [4(n+1)][N].  No device header included:
// the caller prepends it.
std::string emit_grad_kernel(const Dag& d, const Variant& v, const std::string& kname, EmitStats* st);

// Split gradient (SUM, FP64), for processes whose fused gradient kernel would
// not fit the register file.  The amplitude kernel stores every
// configuration's amplitude, log |M|^2 and 1/|M|^2:
//   extern "C" __global__ void <kname>(const double* mom, long long N,
//       double* amp /*[2H][N]*/, double* logm2, double* im2)
std::string emit_amp_kernel(const Dag& d, const Variant& v, const std::string& kname, EmitStats* st);
// Kernels <kprefix>_<t>, t = 0..*count-1, launched in order: per photon
// partition the adjoint sweep for every configuration (seeds conj(A_h)/|M|^2
// read from amp), adding its momentum gradient into gm.  A partition whose
// dots factor into per-pattern leaf sums takes two kernels, the e-_out-side
// walk and the e-_in-side walk, each obtaining the other side's leaf sums by
// a forward walk of its own; others take one.
//   extern "C" __global__ void <kprefix>_<t>(const double* mom, const double* amp,
//       const double* im2, long long N, double* gm)
// Only the kernels of partition only_key (~0u: all) and walk only_phase
// (-1: all; 0 = the one-kernel sweep, 1 = e-_out side, 2 = e-_in side) are
// emitted, numbered from t0; *count is the number emitted.
std::string emit_partition_adjoint_kernels(const Dag& d, const Variant& v, const std::string& kprefix, int* count,
                                           EmitStats* st, uint32_t only_key = ~0u, int only_phase = -1, int t0 = 0);
// The (partition, walk) pairs of the adjoint kernels of (d, v) in launch
// order: (key, 1) and (key, 2) for a factored partition, (key, 0) otherwise.
std::vector<std::pair<uint32_t, int>> adjoint_walks(const Dag& d, const Variant& v);

// Device function text of one process body (used by the mixed batch module):
//   __device__ double <fname>(const double* mom, long long N, long long pt,
//                             unsigned hrt)
// returning the per-lane partial sum of |A|^2.  With v.fixup (FP32C, per
// point) it takes (..., int& fixflag, double fix_kappa) and sets fixflag as
// the eval kernel's fix-up test does.
// With pol_param and a partition slot loop (order & 8) the body also takes
// (..., T* qx_pol) after hrt: per-lane LDS of 3 npart x (threads per
// workgroup, 256) values for the photon polarisations, hoisted out of the loop.
// With the one-photon current cache (order & (256 | 512)) the body instead
// takes (..., double* qx_c, int tpt, unsigned sub) after hrt: the calling
// wave's LDS region of body_cache_doubles() values, the point's slot in it
// (lane / cache lanes) and the lane's index among its point's lanes; every
// lane of the point returns the point's |A|^2.
std::string emit_body_function(const Dag& d, const Variant& v, const std::string& fname, EmitStats* st,
                               bool pol_param = false);
// LDS bytes a wave's region may take (4 waves of a 256-lane workgroup share
// the 160 KB of a compute unit).
constexpr int64_t kBodyCacheBytes = 40 * 1024;
// Doubles of a wave's LDS region for a body with the current cache (64 /
// cache lanes points), 0 without it.
int body_cache_doubles(const Dag& d, const Variant& v);

// Element type ("double" or "float") of the per-lane photon polarisation LDS
// of slot-loop kernels and bodies: FP64 unless an FP32C variant turns off its
// FP64 first-step currents (order flag 64).
std::string pol_lds_type(const Variant& v);

// The device header text (inlined into every generated unit).
const std::string& device_header_text();

}  // namespace qedx
