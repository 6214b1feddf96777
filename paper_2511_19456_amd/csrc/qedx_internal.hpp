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
  hipFunction_t f_fix_zero = nullptr;
  unsigned* fix_ws = nullptr;     // [count, list of N point indices], grown on demand
  size_t fix_bytes = 0;
  hipModule_t mod_aux = nullptr;  // RAMBO and gradient kernels
  hipFunction_t f_rambo = nullptr;
  hipFunction_t f_grad = nullptr;
  int grad_block = 256;
  int grad_lanes = 0;
  // split gradient (n = 4, 5): kernels and a workspace grown on first use
  int grad_split = 0, amp_lanes = 0, adj_lanes = 0;
  hipFunction_t f_grambo = nullptr, f_gamp = nullptr, f_grvjp = nullptr;
  std::vector<hipFunction_t> f_gadj;
  double* ws = nullptr;
  size_t ws_bytes = 0;
  std::string eval_src;
  ~qed_process() {
    if (ws || fix_ws) (void)hipDeviceSynchronize();
    if (ws) (void)hipFree(ws);
    if (fix_ws) (void)hipFree(fix_ws);
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
qed_status default_process_variant(int n, qed_hel_mode mode, qed_precision prec, qedx::Variant& v);
}  // namespace qedx_rt
