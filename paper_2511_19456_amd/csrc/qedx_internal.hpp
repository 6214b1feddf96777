// qedx_internal.hpp -- library-internal declarations shared by the runtime
// translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "../../include/qedx.h"
#include "qedx_dag.hpp"
#include "qedx_emit.hpp"

struct KernelMeta {
  int vgpr = -1, agpr = -1, sgpr = -1, scratch = -1, lds = -1, occupancy = -1;
  std::string hash;  // cache key of the code object (hash of source, flags and target)
};

struct qed_process {
  int n = 0;     // outgoing photons
  int n_in = 1;  // incoming photons
  qed_hel_mode mode = QED_HEL_SUM;
  qed_precision prec = QED_FP64;
  qedx::Variant var;
  qedx::Process proc;
  qed_info info{};
  int lanes = 1;
  hipModule_t mod = nullptr;
  hipFunction_t f_eval = nullptr;
  hipFunction_t f_fix = nullptr;  // FP64 pass of FP32C per-point kernels (null if none)
  hipModule_t mod_aux = nullptr;  // RAMBO and gradient kernels
  hipFunction_t f_rambo = nullptr;
  hipFunction_t f_grad = nullptr;
  int grad_block = 256;
  int grad_lanes = 0;
  // split gradient (n = 4): kernels; the workspace is the caller's
  int grad_split = 0, amp_lanes = 0, adj_lanes = 0;
  hipFunction_t f_grambo = nullptr, f_gamp = nullptr, f_grvjp = nullptr;
  std::vector<hipFunction_t> f_gadj;
  std::string eval_src;
  ~qed_process() {
    // launches are asynchronous: wait for any still running before the
    // code objects they execute are unloaded
    if (mod || mod_aux) (void)hipDeviceSynchronize();
    if (mod) (void)hipModuleUnload(mod);
    if (mod_aux) (void)hipModuleUnload(mod_aux);
  }
};

namespace qedx_rt {
qed_status fail(qed_status s, const std::string& msg);
// Compile (or find in the cache) the code object of a generated source.
qed_status get_code_object(const std::string& tag, const std::string& src, std::string& co, KernelMeta& meta,
                           bool& hit, double& ms);
std::string cache_dir();
// Kernel shape the library uses for (n, mode, prec) when the caller gives none.
qed_status default_process_variant(int n, qed_hel_mode mode, qed_precision prec, int rewrite, qedx::Variant& v);
// Launch of the fused gradient kernel (n <= 3).
qed_status grad_fused(const qed_process* p, const double* uniforms, double sqrt_s, int64_t N, double* out_logm2,
                      double* out_grad, void* stream);
}  // namespace qedx_rt
