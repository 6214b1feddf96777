// qedx_hosttools.cpp -- host-side references of the gradient pieces (graph
// reverse sweep, RAMBO adjoint) for tests; the GPU kernels use the same
// device functions.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/qedx.h"
#include "../../include/qedx_tools.h"
#include "qedx_dag.hpp"

#define QEDX_HD inline
using std::cos;
using std::log;
using std::sin;
using std::sqrt;
#include "qedx_rambo.h"

using namespace qedx;

template <int NF>
static void rambo_host(const double* u, double sqrt_s, const double* gk, double* mom, double* gu) {
  qx::RamboState<NF> S;
  qx::rambo_forward<NF>(u, sqrt_s, 1.0, S);
  for (int j = 0; j < NF; ++j)
    for (int d = 0; d < 4; ++d) mom[4 * j + d] = S.k[j][d];
  double g[NF][4];
  for (int j = 0; j < NF; ++j)
    for (int d = 0; d < 4; ++d) g[j][d] = gk[4 * j + d];
  for (int r = 0; r < 4 * NF; ++r) gu[r] = 0.0;
  qx::rambo_vjp<NF>(u, sqrt_s, 1.0, S, g, gu);
}

extern "C" qed_status qed_rambo_vjp_host(int n, const double* u, double sqrt_s, const double* gk, int64_t N,
                                         double* mom, double* gu) {
  if (n < 1 || n > 6 || N < 0) return QED_ERR_INVALID_ARG;
  const int NF = n + 1;
  for (int64_t i = 0; i < N; ++i) {
    const double* ui = u + 4 * NF * i;
    const double* gi = gk + 4 * NF * i;
    double* mi = mom + 4 * NF * i;
    double* gui = gu + 4 * NF * i;
    switch (n) {
      case 1: rambo_host<2>(ui, sqrt_s, gi, mi, gui); break;
      case 2: rambo_host<3>(ui, sqrt_s, gi, mi, gui); break;
      case 3: rambo_host<4>(ui, sqrt_s, gi, mi, gui); break;
      case 4: rambo_host<5>(ui, sqrt_s, gi, mi, gui); break;
      case 5: rambo_host<6>(ui, sqrt_s, gi, mi, gui); break;
      case 6: rambo_host<7>(ui, sqrt_s, gi, mi, gui); break;
    }
  }
  return QED_OK;
}

extern "C" qed_status qed_graph_grad_interpret(int n, int split, int reduced, const double* mom, int64_t N,
                                               double* val, double* gmom) {
  if (n < 1 || n > 6 || N < 0 || split < 1 || split > n) return QED_ERR_INVALID_ARG;
  Process pr = Process::make(n, 1);
  uint32_t all = (1u << pr.npart) - 1;
  Dag d = build_unreduced(pr, all, split);
  if (reduced) d = compact(reduce_fixpoint(expand_joins(reduce_fixpoint(d), 1)));
  if (reduced == 2) d = distribute(d);
  for (int64_t i = 0; i < N; ++i) val[i] = interpret_grad(d, mom + 4 * pr.npart * i, 0u, gmom + 4 * pr.npart * i);
  return QED_OK;
}
