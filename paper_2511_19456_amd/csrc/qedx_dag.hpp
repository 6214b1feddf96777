// qedx_dag.hpp -- computable DAG (CDAG) of the n-photon Compton amplitude:
// generator, node reduction, join expansion, cost model and a host
// interpreter used to check that rewrites keep the computation.
//
// CDAG (App. B-B): a bipartite DAG of compute nodes and data nodes; a data
// node has exactly one producer, a compute node one (possibly duplicated)
// result; entry nodes and the single exit node are data nodes.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace qedx {

enum class Kind : uint8_t {
  Entry = 0,  // data node without producer: one external momentum
  Data = 1,   // data node (identity / transfer)
  U = 2,      // base_state: external spinor or polarisation vector
  V = 3,      // vertex: photon state x fermion current
  S1 = 4,     // propagator of an inner electron line
  S2 = 5,     // join: Jbar S(Q) J (paper form, before expansion)
  Dot = 6,    // join after its propagator moved onto one side: Jbar . J
  Sum = 7,    // sum of diagram values of one helicity configuration
  HelSum = 8, // sum over enumerated helicity configurations of |A|^2
  Add = 9     // sum of currents (after the distributive rewrite)
};

const char* kind_name(Kind k);
inline bool is_data(Kind k) { return k == Kind::Entry || k == Kind::Data; }

struct Node {
  Kind kind = Kind::Data;
  int8_t side = -1;      // currents: 0 = from e-_in (column), 1 = from e-_out (row)
  int8_t hel = -1;       // U: 0/1 fixed state, -1 = taken at run time
  int16_t particle = -1; // Entry / U: external particle index
  int16_t photon = -1;   // V: photon number attached (0..P-1)
  uint32_t mask = 0;     // currents: set of photons attached so far
  uint32_t cfg = 0;      // enumerated-helicity bits this value depends on (value)
  uint32_t cfg_dep = 0;  // ... and which enumerated bits those are (mask)
  std::vector<int32_t> in;   // producers (ordered: V = {photon state, current})
  std::vector<int32_t> out;  // consumers
};

// e-(p) + n_in photons -> e-(p') + n_out photons on one electron line.
// Particle order: [e-_in, gamma_in..., e-_out, gamma_out...].
struct Process {
  int n_in = 1, n_out = 1;
  int P = 2;          // photons
  int npart = 4;      // external particles
  int i_ein = 0, i_eout = 2;
  std::vector<int> photon_particle;  // photon j -> particle index
  std::vector<int> photon_sign;      // +1 incoming, -1 outgoing
  static Process make(int n_out, int n_in = 1);
};

struct Dag {
  Process proc;
  std::vector<Node> nodes;
  int exit = -1;            // exit data node
  uint32_t enum_mask = 0;   // particle bits enumerated inside the graph
  int split = 1;            // photons on the e-_in side of every join
  bool expanded = false;    // S2 replaced by S1 + Dot
  int join_side = 1;        // side that carries the join propagator after expansion
  bool distributed = false; // distributive rewrite applied
};

struct Counts {
  int64_t total = 0, data = 0, compute = 0;
  int64_t U = 0, V = 0, S1 = 0, S2 = 0, Dot = 0, Sum = 0, HelSum = 0, Add = 0;
};

// Generator (Sec. II-B, Sec. III-A): one chain per diagram and per enumerated
// helicity configuration, sharing only the external U nodes.  Each diagram
// with ordering sigma attaches sigma(0..split-1) to e-_in and the rest to
// e-_out, and joins the halves with S2.
Dag build_unreduced(const Process& proc, uint32_t enum_mask, int split);

// Node reduction (App. C): merge compute (or data) nodes with the same
// function and the same set of producers; children become the union.
// reduce_fixpoint applies it until no reduction is left (single pass in
// topological order with a canonical key per node).
Dag reduce_fixpoint(const Dag& d);
// One reduction at a time, groups picked in random order (for the
// order-independence check).  Returns the number of reductions applied.
int64_t reduce_random_order(Dag& d, uint64_t seed);
// At most max_steps single reductions (all of them if max_steps < 0), in the
// same seeded random order; the graph is compacted.  Returns the number
// applied.  Partially reduced graphs are what the paper times against the
// number of applied node reductions (Sec. III-D).
int64_t reduce_steps(Dag& d, uint64_t seed, int64_t max_steps);

// Rewrite S2(J, Jbar) = Jbar S(Q) J into Dot(J, S1(Jbar)) (join_side = 1) or
// Dot(S1(J), Jbar) (join_side = 0).  Computationally equivalent (App. B-C).
Dag expand_joins(const Dag& d, int join_side);

// Distributive rewrite (term rewriting the paper proposes next to node
// reduction, Sec. IV / App. C), on a reduced, join-expanded graph:
//  (1) in every diagram Sum, the Dots of one photon partition form the full
//      product {Jbar_r} x {J_l} of the orderings on each side, so
//      sum_{r,l} Jbar_r . J_l = (sum_r Jbar_r) . (sum_l J_l);
//  (2) a sum of currents whose terms share their last linear map (the same
//      vertex photon state, or the propagator of the same photon set) is
//      that map applied to the sum of the inner currents, applied
//      recursively.
// The diagram sum per configuration goes from (n+1)! Dots to one Dot per
// partition, and the currents from one per ordered photon prefix to one per
// photon subset (Berends-Giele recursion).  The result is computationally
// equivalent (App. B-C) and is node-reduced afterwards.
Dag distribute(const Dag& d);

Counts count(const Dag& d);
// Canonical text of a DAG, independent of node numbering.
std::string canonical(const Dag& d);
// Remove nodes not reachable backwards from the exit; renumber topologically.
Dag compact(const Dag& d);

// Cost model (App. B-A): compute effort c(T) in FLOPs (add/mul 1, fma 2,
// div/sqrt 1) of the kernel each node becomes, and data size d(T) in bytes.
struct Cost { double flops = 0; double bytes = 0; };
double node_flops(const Dag& d, int i, bool fp32);
double node_bytes(const Dag& d, int i, bool fp32);
// C(DAG), D(DAG), I(DAG) (App. B, graph metrics).
double compute_effort(const Dag& d, bool fp32);
double data_transfer(const Dag& d, bool fp32);
// Reverse-mode (adjoint) cost of the graph in FLOPs per point, on top of
// compute_effort's forward cost.
double adjoint_effort(const Dag& d);

// Host interpreter in double precision: value of the exit (sum over the
// enumerated configurations of |A|^2) for one point.  mom[4*particle + mu];
// runtime_hel gives the state of every particle not enumerated.
double interpret(const Dag& d, const double* mom, uint32_t runtime_hel);

// Host reverse-mode reference: F = log(value of the exit) and dF/dmom for the
// momenta of the final-state particles (e-_out and outgoing photons; the
// incoming momenta are treated as fixed, their rows stay 0).
double interpret_grad(const Dag& d, const double* mom, uint32_t runtime_hel, double* gmom);

}  // namespace qedx
