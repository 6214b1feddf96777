// qedx_probe.cpp -- FP64 pipe probe: the vector FMA pipe, the FP64 matrix
// (MFMA) pipe, and both at once on one CU.
//
// Measures the ceiling an MFMA form of the helicity-summed join would work
// under: after the distributive factoring, the join of a photon partition
// (Sec. II-B join task, Sec. IV term rewriting) is a small dense complex
// product of left and right spinor sums, which could run as
// v_mfma_f64_16x16x4 tiles beside the vector code that builds the currents.
// Each kernel's result has a closed form, so the host can check that the work
// was done.
#include <hip/hip_runtime_api.h>

#include <map>
#include <mutex>
#include <string>

#include "../../include/qedx_probe.h"
#include "qedx_emit.hpp"
#include "qedx_internal.hpp"

using namespace qedx_rt;

#define PROBE_HIPCHK(expr)                                                                             \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return fail(QED_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

namespace {

// vector pipe: 8 independent chains a <- a*m + c per lane;
// matrix pipe: 4 independent 16x16x4 accumulations of the same A.B tile;
// mixed: even waves of a workgroup run the vector chains, odd waves the matrix
// chains (two pipes of one SIMD busy at once if the hardware co-issues them).
const char* kProbeSrc = R"HIP(
#include <hip/hip_runtime.h>
typedef double qx_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double valu_chains(long long iters, double m, double c, double seed) {
  double a0 = seed, a1 = seed + 1.0, a2 = seed + 2.0, a3 = seed + 3.0;
  double a4 = seed + 4.0, a5 = seed + 5.0, a6 = seed + 6.0, a7 = seed + 7.0;
  #pragma unroll 4
  for (long long i = 0; i < iters; ++i) {
    a0 = __builtin_fma(a0, m, c); a1 = __builtin_fma(a1, m, c);
    a2 = __builtin_fma(a2, m, c); a3 = __builtin_fma(a3, m, c);
    a4 = __builtin_fma(a4, m, c); a5 = __builtin_fma(a5, m, c);
    a6 = __builtin_fma(a6, m, c); a7 = __builtin_fma(a7, m, c);
  }
  return ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

__device__ __forceinline__ qx_d4 mfma_chains(long long iters, double x, double y) {
  qx_d4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
  // 8 steps per trip (iters is a multiple of 8): the compiler copies the
  // accumulators between AGPRs and VGPRs at the loop's back edge, so the trip
  // is made long enough for those copies not to matter
  for (long long i = 0; i < iters; i += 8) {
    #pragma unroll
    for (int j = 0; j < 8; ++j) {
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c3, 0, 0, 0);
    }
  }
  return (c0 + c1) + (c2 + c3);
}

__device__ __forceinline__ void store4(double* out, size_t g, qx_d4 s) {
  out[4 * g + 0] = s[0]; out[4 * g + 1] = s[1]; out[4 * g + 2] = s[2]; out[4 * g + 3] = s[3];
}

extern "C" __global__ __launch_bounds__(256) void qedx_probe_valu(long long iters, double m, double c,
                                                                  double* __restrict__ out) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  out[g] = valu_chains(iters, m, c, (double)(threadIdx.x & 63));
}

extern "C" __global__ __launch_bounds__(256) void qedx_probe_mfma(long long iters, const double* __restrict__ a,
                                                                  const double* __restrict__ b,
                                                                  double* __restrict__ out) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  store4(out, g, mfma_chains(iters, a[lane], b[lane]));
}

extern "C" __global__ __launch_bounds__(256) void qedx_probe_mixed(long long iters_v, long long iters_m, double m,
                                                                   double c, const double* __restrict__ a,
                                                                   const double* __restrict__ b,
                                                                   double* __restrict__ out_v,
                                                                   double* __restrict__ out_m) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  if (((threadIdx.x >> 6) & 1) == 0)
    out_v[g] = valu_chains(iters_v, m, c, (double)lane);
  else
    store4(out_m, g, mfma_chains(iters_m, a[lane], b[lane]));
}
)HIP";

// the device header's reciprocal and reciprocal square root, lane by lane
const char* kRecipKernel = R"HIP(
extern "C" __global__ __launch_bounds__(256) void qedx_probe_recip(const double* __restrict__ x, long long n,
                                                                    double* __restrict__ r, double* __restrict__ q) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  r[i] = qx::rcp(v);
  q[i] = qx::rsqrt(v < 0.0 ? -v : v);
}
)HIP";

std::mutex g_mu;
std::map<int, hipModule_t> g_mod, g_rmod;

qed_status probe_code(std::string& co, double* ms) {
  KernelMeta meta;
  bool hit = false;
  double t = 0;
  qed_status s = get_code_object("probe_fp64_pipes", kProbeSrc, co, meta, hit, t);
  if (ms) *ms = t;
  return s;
}

qed_status recip_code(std::string& co, double* ms) {
  KernelMeta meta;
  bool hit = false;
  double t = 0;
  qed_status s = get_code_object("probe_recip", "#include <hip/hip_runtime.h>\n" + qedx::device_header_text() + kRecipKernel,
                                 co, meta, hit, t);
  if (ms) *ms = t;
  return s;
}

}  // namespace

extern "C" qed_status qed_pipe_probe_prebuild(double* compile_ms) {
  std::string co;
  double t1 = 0, t2 = 0;
  qed_status s = probe_code(co, &t1);
  if (!s) s = recip_code(co, &t2);
  if (compile_ms) *compile_ms = t1 + t2;
  return s;
}

extern "C" qed_status qed_recip_probe(const double* x, int64_t n, double* r, double* q, void* stream) {
  if (n < 1 || n > ((int64_t)1 << 30)) return fail(QED_ERR_INVALID_ARG, "n must be in 1..2^30");
  if (!x || !r || !q) return fail(QED_ERR_INVALID_ARG, "missing buffer");
  int dev = 0;
  PROBE_HIPCHK(hipGetDevice(&dev));
  hipModule_t mod = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_rmod.find(dev);
    if (it == g_rmod.end()) {
      std::string co;
      qed_status s = recip_code(co, nullptr);
      if (s) return s;
      PROBE_HIPCHK(hipModuleLoadData(&mod, co.data()));
      g_rmod[dev] = mod;
    } else {
      mod = it->second;
    }
  }
  hipFunction_t f = nullptr;
  PROBE_HIPCHK(hipModuleGetFunction(&f, mod, "qedx_probe_recip"));
  long long nn = (long long)n;
  void* args[] = {(void*)&x, (void*)&nn, (void*)&r, (void*)&q};
  PROBE_HIPCHK(hipModuleLaunchKernel(f, (unsigned)((n + 255) / 256), 1, 1, 256, 1, 1, 0, (hipStream_t)stream, args,
                                     nullptr));
  return QED_OK;
}

extern "C" qed_status qed_pipe_probe(int kind, int64_t blocks, int64_t iters, int64_t iters2, double m, double c,
                                     const double* a, const double* b, double* out, double* out2, void* stream) {
  if (kind < 0 || kind > 2) return fail(QED_ERR_INVALID_ARG, "kind must be 0 (vector), 1 (matrix) or 2 (mixed)");
  if (blocks < 1 || blocks > (1 << 24) || iters < 0 || iters2 < 0)
    return fail(QED_ERR_INVALID_ARG, "blocks must be in 1..2^24, iteration counts >= 0");
  if ((kind == 1 && iters % 8) || (kind == 2 && iters2 % 8))
    return fail(QED_ERR_INVALID_ARG, "matrix-pipe iteration counts must be multiples of 8");
  if (!out || (kind != 0 && (!a || !b)) || (kind == 2 && !out2))
    return fail(QED_ERR_INVALID_ARG, "missing buffer");
  int dev = 0;
  PROBE_HIPCHK(hipGetDevice(&dev));
  hipModule_t mod = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_mod.find(dev);
    if (it == g_mod.end()) {
      std::string co;
      qed_status s = probe_code(co, nullptr);
      if (s) return s;
      PROBE_HIPCHK(hipModuleLoadData(&mod, co.data()));
      g_mod[dev] = mod;
    } else {
      mod = it->second;
    }
  }
  static const char* names[3] = {"qedx_probe_valu", "qedx_probe_mfma", "qedx_probe_mixed"};
  hipFunction_t f = nullptr;
  PROBE_HIPCHK(hipModuleGetFunction(&f, mod, names[kind]));
  long long it1 = (long long)iters, it2 = (long long)iters2;
  void* args[8];
  int na = 0;
  if (kind == 0) {
    args[na++] = &it1;
    args[na++] = &m;
    args[na++] = &c;
    args[na++] = &out;
  } else if (kind == 1) {
    args[na++] = &it1;
    args[na++] = &a;
    args[na++] = &b;
    args[na++] = &out;
  } else {
    args[na++] = &it1;
    args[na++] = &it2;
    args[na++] = &m;
    args[na++] = &c;
    args[na++] = &a;
    args[na++] = &b;
    args[na++] = &out;
    args[na++] = &out2;
  }
  PROBE_HIPCHK(hipModuleLaunchKernel(f, (unsigned)blocks, 1, 1, 256, 1, 1, 0, (hipStream_t)stream, args, nullptr));
  return QED_OK;
}
