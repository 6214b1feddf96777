// qedx_kernels.hpp -- auxiliary generated module: RAMBO and gradient kernels.
#pragma once

#include <string>

#include "qedx_dag.hpp"
#include "qedx_emit.hpp"

namespace qedx {

// Launch shapes of the auxiliary module's gradient kernels.
struct AuxInfo {
  int grad_lanes = 0, grad_block = 0;  // fused gradient kernel (0 if none)
  int split = 0;                       // 1: split gradient kernels instead
  int n_adj = 0;                       // number of per-partition adjoint kernels
  int amp_lanes = 0, adj_lanes = 0;    // lanes per point of the amplitude / adjoint kernels
};

// HIP source with
//   qedx_rambo_n<n>(const double* u, double sqrt_s, long long N, double* mom)
// and, for SUM-mode FP64 processes, the gradient of log |M|^2 with respect to
// the RAMBO uniforms:
//  - n <= 3, fused: qedx_grad_n<n>(const double* u, double sqrt_s, long long N,
//      double* logm2, double* grad);
//  - n = 4, split over a caller workspace (the fused kernel spills heavily):
//      qedx_grambo_n<n>(u, ldu, sqrt_s, N, mom, gm)  RAMBO into the workspace,
//          the final-state momentum-gradient rows of gm zeroed,
//      qedx_gamp_n<n>(mom, N, amp, logm2, im2)  amplitudes of every configuration,
//      qedx_gadj_n<n>_<t>(mom, amp, im2, N, gm)  adjoint of photon partition t,
//      qedx_grvjp_n<n>(u, ldu, sqrt_s, N, gm, grad, ldg)  RAMBO adjoint.
// n >= 5 has RAMBO only (its split gradient module takes tens of minutes of
// compile time and is not built).
std::string emit_aux_module(const Process& proc, const Variant& v, int n, AuxInfo* info);

// Kernel shape of the fused gradient (n <= 3): every photon polarisation and
// as many electron spins as fit on 64 lanes; the rest enumerated in the graph.
Variant grad_variant(const Process& proc);

}  // namespace qedx
