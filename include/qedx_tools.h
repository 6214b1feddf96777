/* qedx_tools.h -- host-side graph tools of the qedx library (no GPU needed).
 *
 * Inspection of the computation graph the library builds (node counts, the
 * graph metrics of App. B, the reduction fixpoint, the generated kernel
 * source) and host references used by the tests (a float64 interpreter of the
 * graph, its reverse sweep, the RAMBO adjoint).  Exported by libqedx.so beside
 * the evaluation ABI of qedx.h; conventions (particle order, helicity codes,
 * momenta layout, status codes) are those of qedx.h, except that these
 * functions take host buffers, point-major.  None of them touches a GPU.
 */
#ifndef QEDX_TOOLS_H
#define QEDX_TOOLS_H

#include "qedx.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Host-side graph tools (no GPU needed), for inspection and tests.
 * qed_graph_counts: node counts of the generated graph for n, enumerated
 * helicity bits `enum_mask` and join split `split`: reduced = 0 gives the
 * paper's unreduced form (one chain per diagram, S2 joins); reduced = 1 the
 * node-reduced, join-expanded form; reduced = 2 that form after the
 * distributive rewrite (see qed_variant.rewrite).  counts[10] = total, data, compute, U, V,
 * S1, S2, Dot, Sum, HelSum. */
qed_status qed_graph_counts(int n, int n_in, uint32_t enum_mask, int split, int reduced, int64_t* counts);
/* Host interpreter of the graph (float64), per point: value of the exit node
 * (sum over enum_mask configurations of |A|^2) with the other bits from hel.
 * reduced as above; mom is host [N][4(n_in+n+2)] (point-major); out host [N]. */
qed_status qed_graph_interpret(int n, int n_in, uint32_t enum_mask, int split, int reduced, const double* mom,
                               const uint32_t* hel, int64_t N, double* out);
/* Canonical structure hash text of the reduced graph reached by (a) the
 * one-pass fixpoint and (b) single reductions in a random order seeded by
 * `seed`; writes at most buflen bytes of each.  Returns the number of single
 * reductions in *steps. */
qed_status qed_graph_reduction_check(int n, int n_in, uint32_t enum_mask, int split, uint64_t seed, char* canon_a,
                                     char* canon_b, int64_t buflen, int64_t* steps);
/* The graph of the reduction experiment (Sec. III-D): the unreduced graph
 * for n outgoing photons, one configuration per point, after the first
 * `steps` single node reductions in the random order seeded by `seed`.
 * Writes counts[10] (as qed_graph_counts) if non-NULL and, for N points
 * (mom host [N][4(n+3)], hel host [N] or NULL), the interpreted |A|^2. */
qed_status qed_graph_partial(int n, int split, int64_t steps, uint64_t seed, const double* mom, const uint32_t* hel,
                             int64_t N, double* out, int64_t* counts);
/* Generated HIP source of the eval kernel for a variant (for inspection and
 * for prebuilding the cache); writes at most buflen bytes, returns the full
 * length in *len. */
qed_status qed_emit_source(int n, qed_hel_mode mode, qed_precision prec, const qed_variant* variant, char* buf,
                           int64_t buflen, int64_t* len);

/* C(DAG) and D(DAG) of the graph (App. B graph metrics): compute effort in
 * FLOPs (add/mul 1, fma 2, div/sqrt 1, per point) and data transfer in bytes,
 * with float32 value sizes if fp32 != 0. */
qed_status qed_graph_metrics(int n, int n_in, uint32_t enum_mask, int split, int reduced, int fp32,
                             double* c_dag, double* d_dag);
/* Forward C(DAG) (as qed_graph_metrics, float64) and the reverse-mode cost of
 * the same graph (FLOPs per point the adjoint sweep of log sum |A|^2 adds:
 * per node the vector-Jacobian products of the device functions), for the
 * process with one incoming photon; the gradient's algorithmic FLOPs are
 * their sum. */
qed_status qed_graph_adjoint_metrics(int n, uint32_t enum_mask, int split, int reduced, double* c_fwd,
                                     double* c_adj);
/* Host references of the gradient pieces (no GPU), for tests:
 * qed_graph_grad_interpret: F = log(sum over all configurations of |A|^2) and
 * dF/dmom by a reverse sweep over the graph in float64.  mom host [N][4(n+3)]
 * point-major; val [N]; gmom [N][4(n+3)] (rows of the incoming particles 0).
 * qed_rambo_vjp_host: final-state momenta mom [N][4(n+1)] from uniforms
 * u [N][4(n+1)], and gu [N][4(n+1)] = (dk/du)^T gk for given gk [N][4(n+1)]. */
qed_status qed_graph_grad_interpret(int n, int split, int reduced, const double* mom, int64_t N, double* val,
                                    double* gmom);
qed_status qed_rambo_vjp_host(int n, const double* u, double sqrt_s, const double* gk, int64_t N, double* mom,
                              double* gu);

#ifdef __cplusplus
}
#endif

#endif /* QEDX_TOOLS_H */
