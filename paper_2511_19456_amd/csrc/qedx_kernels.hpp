// qedx_kernels.hpp -- auxiliary generated module: RAMBO and gradient kernels.
#pragma once

#include <string>

#include "qedx_dag.hpp"
#include "qedx_emit.hpp"

namespace qedx {

// HIP source with
//   qedx_rambo_n<n>(const double* u, double sqrt_s, long long N, double* mom)
// and, for SUM-mode FP64 variants, the gradient kernel
//   qedx_grad_n<n>(const double* u, double sqrt_s, long long N, double* logm2, double* grad)
// grad_lanes / grad_block receive the launch shape of qedx_grad_n<n> (0 if the
// module has no gradient kernel).
std::string emit_aux_module(const Process& proc, const Variant& v, int n, int* grad_lanes, int* grad_block);

// Kernel shape of the gradient: every photon polarisation and as many
// electron spins as fit on 64 lanes; the rest enumerated in the graph.
Variant grad_variant(const Process& proc);

}  // namespace qedx
