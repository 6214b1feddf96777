// qedx_kernels.hpp -- auxiliary generated module: RAMBO and gradient kernels.
#pragma once

#include <string>

#include "qedx_dag.hpp"
#include "qedx_emit.hpp"

namespace qedx {

// HIP source with
//   qedx_rambo(const double* u, double sqrt_s, long long N, double* mom)
// and, for SUM-mode FP64 variants, the gradient kernel
//   qedx_grad(const double* u, double sqrt_s, long long N, double* logm2, double* grad)
std::string emit_aux_module(const Process& proc, const Variant& v, int n);

}  // namespace qedx
