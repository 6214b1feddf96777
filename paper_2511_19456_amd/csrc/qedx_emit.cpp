// qedx_emit.cpp -- straight-line HIP code from the reduced QED graph.
//
// One phase-space point per lane (or 2^k lanes per point when helicity bits
// are spread over lanes).  Every compute node becomes one call of the matching
// device function of qedx_device.h; data nodes are renames (App. D: on a
// single device a data node is the identity).  The emission order groups the
// joins by photon partition so that the currents of one partition are live
// together; LLVM allocates registers for the resulting basic block.
#include "qedx_emit.hpp"

#include <algorithm>
#include <array>
#include <chrono>
#include <map>
#include <set>
#include <sstream>
#include <stdexcept>

namespace qedx {

static const char* kDeviceHeaderText =
#include "qedx_device_embed.inc"
    ;

const std::string& device_header_text() {
  static const std::string s(kDeviceHeaderText);
  return s;
}

static int popc(uint32_t x) { return __builtin_popcount(x); }

std::string variant_tag(const Variant& v, int n_out, int n_in) {
  std::ostringstream o;
  o << "nin" << n_in << "_nout" << n_out << "_p" << v.prec << "_m" << v.mode << "_e" << v.enum_mask << "_l"
    << v.lane_mask << "_o" << v.loop_mask << "_b" << v.block << "_s" << v.split << "_j" << v.join_side << "_r"
    << v.order << "_w" << v.min_waves;
  if (v.rewrite) o << "_d" << v.rewrite;
  if (v.partial) o << "_k" << v.partial_steps << "s" << v.partial_seed;
  if (v.fixup) o << "_f" << v.fixup;
  return o.str();
}

std::string pol_lds_type(const Variant& v) {
  return v.prec == PREC_F64 || !(v.order & 64) ? "double" : "float";
}

Dag graph_for(const Process& proc, const Variant& v, double* t_build, double* t_reduce) {
  using clk = std::chrono::steady_clock;
  auto t0 = clk::now();
  Dag d = build_unreduced(proc, v.enum_mask, v.split);
  auto t1 = clk::now();
  if (v.partial) {
    // the paper's form after the first partial_steps single node reductions
    // (seeded random order), joins not split
    reduce_steps(d, v.partial_seed, v.partial_steps);
    if (t_build) *t_build = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (t_reduce) *t_reduce = std::chrono::duration<double, std::milli>(clk::now() - t1).count();
    return d;
  }
  Dag r = reduce_fixpoint(d);
  r = reduce_fixpoint(expand_joins(r, v.join_side));
  r = compact(r);
  if (v.rewrite == 1) r = distribute(r);
  auto t2 = clk::now();
  if (t_build) *t_build = std::chrono::duration<double, std::milli>(t1 - t0).count();
  if (t_reduce) *t_reduce = std::chrono::duration<double, std::milli>(t2 - t1).count();
  return r;
}

namespace {

struct Emitter {
  const Dag& d;
  const Variant& v;
  const Process& pr;
  std::ostringstream os;
  std::vector<char> done;
  std::set<uint32_t> kdone;
  std::set<std::pair<int, uint32_t>> qdone;
  std::map<int, int> acc_of_sum;  // Sum node -> accumulator index
  EmitStats st;
  std::string T;
  std::string ind = "  ";
  int mom_src = 0;  // 0: reload momenta from global memory; 1: opaque copies of registers M<p>_<mu>
  // Partition loop: one block for the canonical partition (photons 0..split-1
  // on the e-_in side) inside a run-time loop over all partitions; photon
  // slot a of iteration `it` is particle slot_tab[it][a], loaded per iteration.
  bool slot = false;
  std::string slot_tab;

  int slot_of(int particle) const {
    for (int a = 0; a < pr.P; ++a)
      if (pr.photon_particle[a] == particle) return a;
    return -1;
  }

  Emitter(const Dag& d_, const Variant& v_) : d(d_), v(v_), pr(d_.proc), done(d_.nodes.size(), 0) {
    T = v.prec == PREC_F64 ? "double" : "float";
    d1 = v.prec != PREC_F64 && !(v.order & 64);
    PT = pol_lds_type(v);
  }

  // FP32C: the first vertex and propagator next to each external electron
  // (U -> V -> S1) are evaluated in FP64 and rounded once.  There
  // (Qslash + m) eps-slash u(p) = eps-slash kslash u + 2 (eps.p) u for
  // Q = p - k, so with eps.p ~ 0 and a soft k the product cancels by
  // ~2E/k; in FP32 that cancellation costs as many digits (likewise
  // ubar(p') eps-slash (p'-slash + kslash + m) on the other side).  Nodes with an
  // FP64 copy are named <name>_d.
  bool d1 = false;
  std::string PT;  // element type of the per-lane polarisation LDS
  std::set<int> has_d;
  std::set<std::pair<int, uint32_t>> qdone_d;

  int producer(int i) const {
    const Node& n = d.nodes[i];
    return n.kind == Kind::Data ? n.in[0] : i;
  }
  std::string name(int i) const {
    auto a = alias.find(producer(i));
    return a != alias.end() ? a->second : "n" + std::to_string(producer(i));
  }
  // LDS staging of the held side of each partition block (order flag 16):
  // the held currents are stored to per-lane LDS slots once and read back,
  // through an address the compiler cannot see through, for every group of
  // kTile streamed currents -- register pressure is then the accumulators,
  // one tile and one held current.
  std::map<int, std::string> alias;
  bool batch_mom = false;  // order flag 8192: block momenta loaded together (see block_momenta)
  bool amp_store = false;  // body() also stores every configuration's amplitude
  bool stage() const { return (v.order & 16) != 0; }
  int lds_slots = 0;
  // partition slot loop: photon polarisation vectors computed once per point
  // (and helicity-loop iteration) before the loop, kept in per-lane LDS and
  // read by slot inside it, instead of once per partition
  bool pol_lds = false;
  static constexpr int kTile = 4;
  // One-photon current cache (order flag 256, per-point FP64 slot loops):
  // the two lanes of a point first compute, for every photon, its
  // polarisation vector and its one-photon currents on both sides,
  // S(Q) eps-slash u and ubar eps-slash S(Q), into per-point LDS; the
  // partition loop, split between the two lanes, reads them there instead of
  // recomputing them in every partition (each photon's one-photon current
  // is otherwise rebuilt once per partition that puts the photon first on a
  // side).  BP = points per workgroup.
  bool cur_cache = false;
  int BP = 0, CL = 1;  // points per workgroup, lanes per point
  bool k_lds = false;  // the signed photon momenta cached too (where LDS allows)
  bool row_only = false;  // order flag 1024: only the e-_in side's currents cached
  // Shared e-_in side (order flag 2048; SUM kernels whose one lane bit is
  // the e-_out spin and whose graph enumerates the e-_in spin): both lanes of
  // a point would build the same e-_in-side currents for both e-_in spins.
  // Instead each lane builds them for one e-_in spin (its lane bit) and takes
  // the other spin's leaves from its partner lane.  Lane 1 thereby swaps the
  // e-_in labels of all its accumulators, which leaves sum |A|^2 unchanged.
  bool coop = false;
  std::map<std::pair<int, int>, int> v_of;  // (photon state, current) -> V node
  std::map<int, int> s1_of;                 // current -> S1 node
  int u_ein0 = -1;                          // U node of e-_in with spin 0
  bool ein1(int x) const {  // an e-_in-side value of e-_in spin 1
    const Node& n = d.nodes[x];
    const uint32_t b = 1u << pr.i_ein;
    return coop && n.side == 0 && (n.kind == Kind::V || n.kind == Kind::S1) && (n.cfg_dep & b) && (n.cfg & b);
  }
  void build_twins() {
    for (size_t i = 0; i < d.nodes.size(); ++i) {
      const Node& n = d.nodes[i];
      if (n.kind == Kind::V) v_of[{producer(n.in[0]), producer(n.in[1])}] = (int)i;
      if (n.kind == Kind::S1) s1_of[producer(n.in[0])] = (int)i;
      if (n.kind == Kind::U && n.particle == pr.i_ein && n.hel == 0) u_ein0 = (int)i;
    }
    if (u_ein0 < 0) throw std::invalid_argument("shared e-_in side: no enumerated e-_in spin");
  }
  // the same value with e-_in spin 0
  int twin(int x) const {
    x = producer(x);
    const Node& n = d.nodes[x];
    if (n.kind == Kind::U) return n.particle == pr.i_ein ? u_ein0 : x;
    if (n.kind == Kind::V) return v_of.at({producer(n.in[0]), twin(n.in[1])});
    if (n.kind == Kind::S1) return s1_of.at(twin(n.in[0]));
    throw std::logic_error("shared e-_in side: unexpected node kind");
  }

  // e-_in-side one-photon currents of a helicity-sum kernel (order flag
  // 4096, with the shared e-_in side): every partition block that puts a
  // photon first on the e-_in side rebuilt S(Q) eps-slash u for each of its
  // polarisation states; they are computed once per point (and loop
  // iteration) into per-lane LDS, [slot][8 words][block], and read there.
  bool r1_cache = false;
  std::map<int, int> r1_slot;  // S1 node -> LDS slot
  std::string r1_ref(int slot, int w) const {
    return "qx_r1[" + std::to_string((8 * slot + w) * v.block) + " + threadIdx.x]";
  }
  void r1_collect() {
    for (size_t i = 0; i < d.nodes.size(); ++i) {
      const Node& n = d.nodes[i];
      if (n.kind == Kind::S1 && n.side == 0 && popc(n.mask) == 1 && !ein1((int)i) && !n.out.empty())
        r1_slot[(int)i] = (int)r1_slot.size();
    }
  }
  void emit_r1_cache() {
    os << ind << "{\n";
    std::string o = ind;
    ind += "  ";
    block_momenta();
    std::fill(done.begin(), done.end(), 0);
    kdone.clear();
    qdone.clear();
    const bool was = r1_cache;
    r1_cache = false;  // compute them here
    for (auto& kv : r1_slot) {
      emit(kv.first);
      for (int k = 0; k < 4; ++k)
        os << ind << r1_ref(kv.second, 2 * k) << " = " << name(kv.first) << ".c[" << k << "].r; "
           << r1_ref(kv.second, 2 * k + 1) << " = " << name(kv.first) << ".c[" << k << "].i;\n";
    }
    r1_cache = was;
    std::fill(done.begin(), done.end(), 0);
    kdone.clear();
    qdone.clear();
    ind = o;
    os << ind << "}\n";
  }

  // a device-function body of the persistent batch kernel: the cache is the
  // wave's own LDS region (BP = points per wave), tpt and sub are arguments,
  // and the wave synchronises only itself
  bool body_mode = false;
  void wave_sync() {
    os << ind << "__builtin_amdgcn_fence(__ATOMIC_RELEASE, \"wavefront\"); __builtin_amdgcn_wave_barrier(); "
       << "__builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"wavefront\");\n";
  }
  std::string ix_tab;  // photon index of every slot: [iteration][P]
  std::string cache_k(const std::string& ix, int mu) const {
    return "qx_k[(4 * " + ix + " + " + std::to_string(mu) + ") * " + std::to_string(BP) + " + tpt]";
  }
  std::string cache_pol(const std::string& ix, int c) const {
    return "qx_pol[(3 * " + ix + " + " + std::to_string(c) + ") * " + std::to_string(BP) + " + tpt]";
  }
  std::string cache_cur(int side, const std::string& ix, int w) const {
    return "qx_cur[(" + std::to_string(side * pr.P * 8 + w) + " + 8 * " + ix + ") * " + std::to_string(BP) + " + tpt]";
  }

  void emitK(uint32_t mask) {
    if (kdone.count(mask)) return;
    int lo = __builtin_ctz(mask);
    uint32_t rest = mask & (mask - 1);
    std::string km = "K" + std::to_string(mask);
    if (rest == 0 && slot && k_lds) {
      for (int mu = 0; mu < 4; ++mu)
        os << ind << "const double " << km << "_" << mu << " = " << cache_k("ix" + std::to_string(lo), mu) << ";\n";
    } else if (rest == 0 && slot) {
      for (int mu = 0; mu < 4; ++mu)
        os << ind << "const double " << km << "_" << mu << " = sg" << lo << " * k" << lo << "_" << mu << ";\n";
      st.flops_per_point += 4;
    } else if (rest == 0) {
      int part = pr.photon_particle[lo];
      const char* sg = pr.photon_sign[lo] > 0 ? "" : "-";
      for (int mu = 0; mu < 4; ++mu)
        os << ind << "const double " << km << "_" << mu << " = " << sg << "m" << part << "_" << mu << ";\n";
    } else {
      emitK(rest);
      emitK(1u << lo);
      std::string kr = "K" + std::to_string(rest), kl = "K" + std::to_string(1u << lo);
      for (int mu = 0; mu < 4; ++mu)
        os << ind << "const double " << km << "_" << mu << " = " << kr << "_" << mu << " + " << kl << "_" << mu
           << ";\n";
      st.flops_per_point += 4;
    }
    kdone.insert(mask);
  }

  std::string qname(int side, uint32_t mask) const {
    return std::string(side == 0 ? "qL" : "qR") + std::to_string(mask);
  }

  void emitQ(int side, uint32_t mask) {
    if (qdone.count({side, mask})) return;
    emitK(mask);
    int pp = side == 0 ? pr.i_ein : pr.i_eout;
    std::string km = "K" + std::to_string(mask);
    os << ind << "const qx::propq<" << T << "> " << qname(side, mask) << " = qx::prop_from<" << T << ">(m" << pp
       << "_0, m" << pp << "_1, m" << pp << "_2, m" << pp << "_3, " << km << "_0, " << km << "_1, " << km << "_2, "
       << km << "_3, " << (side == 0 ? "1.0" : "-1.0") << ", 1.0);\n";
    if (!qdone_d.count({side, mask})) {
      st.flops_per_point += 28;
      ++st.n_prop;
    }
    qdone.insert({side, mask});
  }

  // FP64 propagator coefficients (for the FP32C first-step currents)
  void emitQd(int side, uint32_t mask) {
    if (qdone_d.count({side, mask})) return;
    emitK(mask);
    int pp = side == 0 ? pr.i_ein : pr.i_eout;
    std::string km = "K" + std::to_string(mask);
    os << ind << "const qx::propq<double> " << qname(side, mask) << "_d = qx::prop_from<double>(m" << pp << "_0, m"
       << pp << "_1, m" << pp << "_2, m" << pp << "_3, " << km << "_0, " << km << "_1, " << km << "_2, " << km
       << "_3, " << (side == 0 ? "1.0" : "-1.0") << ", 1.0);\n";
    if (!qdone.count({side, mask})) {
      st.flops_per_point += 28;
      ++st.n_prop;
    }
    qdone_d.insert({side, mask});
  }
  std::string name_d(int i) const { return "n" + std::to_string(producer(i)) + "_d"; }

  std::string hel_expr(const Node& u) const {
    if (coop && u.particle == pr.i_ein) return "(int)((hc >> " + std::to_string(pr.i_eout) + ") & 1u)";
    if (u.hel >= 0) return std::to_string((int)u.hel);
    if (slot && slot_of(u.particle) >= 0) return "hb" + std::to_string(slot_of(u.particle));
    return "(int)((hc >> " + std::to_string(u.particle) + ") & 1u)";
  }

  bool local() const { return (v.order & 4) != 0 && !slot; }
  bool loop_local() const { return (v.order & 32) != 0 && v.loop_mask != 0 && !local() && !slot; }

  // scheduling fence: keeps LLVM's machine scheduler from moving work across
  void fence(int level) {
    if (v.order & level) os << ind << "__builtin_amdgcn_sched_barrier(0);\n";
  }

  void emit(int i) {
    int c = producer(i);
    if (done[c]) return;
    const Node& n = d.nodes[c];
    if (r1_cache && r1_slot.count(c)) {
      os << ind << "const qx::sp4<" << T << "> n" << c << " = {{";
      for (int k = 0; k < 4; ++k)
        os << (k ? ", " : "") << "{" << r1_ref(r1_slot.at(c), 2 * k) << ", " << r1_ref(r1_slot.at(c), 2 * k + 1) << "}";
      os << "}};\n";
      done[c] = 1;
      return;
    }
    if (ein1(c)) {
      // built by the partner lane as its spin-0 twin
      const int t = twin(c);
      emit(t);
      os << ind << "const qx::sp4<" << T << "> n" << c << " = qx::lane_xor1(" << name(t) << ");\n";
      done[c] = 1;
      return;
    }
    if (cur_cache && n.kind == Kind::S1 && popc(n.mask) == 1 && (n.side == 0 || !row_only)) {
      // a one-photon current: read from the per-point cache
      const std::string ix = "ix" + std::to_string(__builtin_ctz(n.mask));
      os << ind << "const qx::sp4<" << T << "> n" << c << " = {{";
      for (int k = 0; k < 4; ++k)
        os << (k ? ", " : "") << "{" << cache_cur(n.side, ix, 2 * k) << ", " << cache_cur(n.side, ix, 2 * k + 1) << "}";
      os << "}};\n";
      done[c] = 1;
      return;
    }
    for (int p : n.in) emit(p);
    std::string nm = "n" + std::to_string(c);
    switch (n.kind) {
      case Kind::Entry: break;
      case Kind::U: {
        int p = n.particle;
        std::string m = "m" + std::to_string(p) + "_";
        // with d1 the state is built in FP64 (name_d) and rounded for the FP32 graph
        const std::string TU = d1 ? "double" : T;
        const std::string nu = d1 ? nm + "_d" : nm;
        if (p == pr.i_ein || p == pr.i_eout) {
          os << ind << "const qx::sp4<" << TU << "> " << nu << " = qx::" << (p == pr.i_ein ? "u_in" : "ubar_out") << "<"
             << TU << ">(" << m << "0, " << m << "1, " << m << "2, " << m << "3, " << hel_expr(n) << ", 1.0);\n";
          if (d1) os << ind << "const qx::sp4<float> " << nm << " = qx::to_f(" << nu << ");\n";
        } else if (cur_cache) {
          // polarisation from the per-point cache, in the graph's type (the
          // FP64 first steps that need it in FP64 are cached themselves)
          os << ind << "const qx::pol3<" << T << "> " << nm << " = {";
          for (int c = 0; c < 3; ++c) os << (c ? ", " : "") << cache_pol("ix" + std::to_string(slot_of(p)), c);
          os << "};\n";
          st.flops_per_point += 16;
          ++st.n_U;
          break;
        } else if (slot && pol_lds) {
          std::string sp = "sp" + std::to_string(slot_of(p));
          os << ind << "const qx::pol3<" << TU << "> " << nu << " = {";
          for (int c = 0; c < 3; ++c)
            os << (c ? ", " : "") << (PT != TU ? "(" + TU + ")" : std::string())
               << "qx_pol[(3 * " << sp << " + " << c << ") * " << v.block << " + threadIdx.x]";
          os << "};\n";
          if (d1) os << ind << "const qx::pol3<float> " << nm << " = qx::to_f(" << nu << ");\n";
        } else {
          if (slot) m = "k" + std::to_string(slot_of(p)) + "_";
          os << ind << "const qx::pol3<" << TU << "> " << nu << " = qx::pol<" << TU << ">(" << m << "1, " << m << "2, "
             << m << "3, " << hel_expr(n) << ");\n";
          if (d1) os << ind << "const qx::pol3<float> " << nm << " = qx::to_f(" << nu << ");\n";
        }
        if (d1) has_d.insert(c);
        st.flops_per_point += 16;
        ++st.n_U;
        break;
      }
      case Kind::V: {
        const Node& ph = d.nodes[producer(n.in[0])];
        bool y = ph.hel == 1;
        const Node& cur = d.nodes[producer(n.in[1])];
        if (d1 && cur.kind == Kind::U && has_d.count(producer(n.in[1])) && has_d.count(producer(n.in[0]))) {
          // first vertex next to an external electron: FP64, rounded once
          os << ind << "const qx::sp4<double> " << nm << "_d = qx::v" << (n.side == 0 ? "L" : "R") << (y ? "_y" : "")
             << "<double>(" << name_d(n.in[1]) << ", " << name_d(n.in[0]) << ");\n";
          os << ind << "const qx::sp4<float> " << nm << " = qx::to_f(" << nm << "_d);\n";
          has_d.insert(c);
        } else {
          os << ind << "const qx::sp4<" << T << "> " << nm << " = qx::v" << (n.side == 0 ? "L" : "R")
             << (y ? "_y" : "") << "<" << T << ">(" << name(n.in[1]) << ", " << name(n.in[0]) << ");\n";
        }
        st.flops_per_point += y ? 24 : 40;
        ++st.n_V;
        break;
      }
      case Kind::S1: {
        if (d1 && d.nodes[producer(n.in[0])].kind == Kind::V && has_d.count(producer(n.in[0]))) {
          // propagator after the first vertex: FP64 on the FP64 current, rounded once
          emitQd(n.side, n.mask);
          os << ind << "const qx::sp4<double> " << nm << "_d = qx::s" << (n.side == 0 ? "L" : "R") << "<double>("
             << name_d(n.in[0]) << ", " << qname(n.side, n.mask) << "_d);\n";
          os << ind << "const qx::sp4<float> " << nm << " = qx::to_f(" << nm << "_d);\n";
          has_d.insert(c);
        } else {
          emitQ(n.side, n.mask);
          os << ind << "const qx::sp4<" << T << "> " << nm << " = qx::s" << (n.side == 0 ? "L" : "R") << "<" << T
             << ">(" << name(n.in[0]) << ", " << qname(n.side, n.mask) << ");\n";
        }
        st.flops_per_point += 56;
        ++st.n_S1;
        break;
      }
      case Kind::Add: {
        std::string e = name(n.in[0]);
        for (size_t t = 1; t < n.in.size(); ++t)
          e = "qx::add4<" + T + ">(" + e + ", " + name(n.in[t]) + ")";
        os << ind << "const qx::sp4<" << T << "> " << nm << " = " << e << ";\n";
        st.flops_per_point += 8.0 * (double)(n.in.size() - 1);
        break;
      }
      case Kind::Dot:
      case Kind::Sum:
      case Kind::HelSum:
      case Kind::S2:
        throw std::logic_error("emit(): joins and sums are emitted by the caller");
      default: break;
    }
    done[c] = 1;
    if (n.kind != Kind::Entry) fence(2);
  }

  // the two operands of a Dot: (column current J, row current B)
  std::pair<int, int> dot_ops(const Node& n) const {
    int a = n.in[0], b = n.in[1];
    if (d.nodes[producer(a)].side != 0) std::swap(a, b);
    return {a, b};
  }

  void emit_dot(int k) {
    const Node& n = d.nodes[k];
    auto ops = dot_ops(n);
    int sum = n.out.empty() ? -1 : d.nodes[n.out[0]].out[0];  // Dot -> Data -> Sum
    int acc = acc_of_sum.at(sum);
    std::string B = name(ops.second);
    if (n.kind == Kind::S2) {
      // join of the paper's form (graphs that were not split): the row
      // current is propagated here, Jbar S(Q) J
      uint32_t mb = d.nodes[producer(ops.second)].mask;
      emitQ(1, mb);
      B = "qx::sR<" + T + ">(" + B + ", " + qname(1, mb) + ")";
      st.flops_per_point += 56;
    }
    if (v.prec == PREC_F64) {
      os << ind << "qx::dot_acc<double>(A" << acc << ", " << B << ", " << name(ops.first) << ");\n";
      st.flops_per_point += 32;
    } else {
      // a join of two FP64 first-step currents (one photon on each side):
      // the dot in FP64 too, the diagram value rounded once
      std::string x = "qx::dot<float>(" + B + ", " + name(ops.first) + ")";
      if (n.kind == Kind::Dot && has_d.count(producer(ops.second)) && has_d.count(producer(ops.first)))
        x = "qx::to_f(qx::dot<double>(" + name_d(ops.second) + ", " + name_d(ops.first) + "))";
      if (abs_sum) {
        os << ind << "{ const qx::cx<float> x_ = " << x << "; qx::comp_acc<float>(A" << acc << ", C" << acc
           << ", x_); S" << acc << " = fmaf(x_.r, x_.r, fmaf(x_.i, x_.i, S" << acc << ")); }\n";
        st.flops_per_point += 30 + 14 + 2;
      } else {
        os << ind << "qx::comp_acc<float>(A" << acc << ", C" << acc << ", " << x << ");\n";
        st.flops_per_point += 30 + 14;
      }
    }
    ++st.n_dot;
    fence(2);
  }

  // FP32C per-point fix-up: sum |diagram value| beside the compensated sum
  // and raise `fixflag` (declared by the kernel) on cancellation
  bool abs_sum = false;

  std::vector<int> sum_nodes() const {
    std::vector<int> sums;
    for (size_t i = 0; i < d.nodes.size(); ++i)
      if (d.nodes[i].kind == Kind::Sum) sums.push_back((int)i);
    return sums;
  }

  // Dots grouped by the photon set on the e-_in side (one group per
  // partition), and an order of the groups in which consecutive partitions
  // share as many photons as possible.
  void partitions(std::map<uint32_t, std::vector<int>>& part, std::vector<uint32_t>& order) const {
    for (size_t i = 0; i < d.nodes.size(); ++i)
      if (d.nodes[i].kind == Kind::Dot || d.nodes[i].kind == Kind::S2) {
        auto ops = dot_ops(d.nodes[i]);
        part[d.nodes[producer(ops.first)].mask].push_back((int)i);
      }
    std::vector<uint32_t> keys;
    for (auto& kv : part) keys.push_back(kv.first);
    std::vector<char> used(keys.size(), 0);
    uint32_t cur = keys.empty() ? 0 : keys[0];
    for (size_t t = 0; t < keys.size(); ++t) {
      int best = -1, bscore = -1;
      for (size_t q = 0; q < keys.size(); ++q) {
        if (used[q]) continue;
        int sc = t == 0 ? (q == 0 ? 1 : 0) : popc(keys[q] & cur);
        if (sc > bscore) {
          bscore = sc;
          best = (int)q;
        }
      }
      used[best] = 1;
      cur = keys[best];
      order.push_back(cur);
    }
  }

  // Partition-local block: momenta reloaded through a value the compiler
  // cannot see through, so nothing computed here is merged with (and kept
  // live from) another partition's block; a uniform branch on an opaque flag
  // puts the block in its own basic block, so instruction selection
  // schedules it on its own.
  std::string open_block() {
    std::string outer = ind;
    os << ind << "{\n" << ind << "  int live = 1;\n" << ind << "  asm volatile(\"\" : \"+s\"(live));\n" << ind
       << "  if (live) {\n";
    ind += "    ";
    block_momenta();
    std::fill(done.begin(), done.end(), 0);
    kdone.clear();
    qdone.clear();
    qdone_d.clear();
    has_d.clear();
    return outer;
  }
  void close_block(const std::string& outer) {
    ind = outer;
    os << ind << "  }\n" << ind << "}\n";
  }

  void forward_block(uint32_t key, const std::vector<int>& dk) {
    fence(1);
    os << ind << "// photons " << key << " | " << (((1u << pr.P) - 1) & ~key) << " on the e-_in | e-_out side\n";
    std::string outer;
    if (local()) outer = open_block();
    forward_block_inner(key, dk);
    if (local()) close_block(outer);
  }

  // opaque per-use LDS index (the base stays visible, so accesses stay ds_*)
  std::string lds_index(int slot) const {
    return "int ix = " + std::to_string(slot * 8 * v.block) + " + (int)threadIdx.x; asm volatile(\"\" : \"+v\"(ix));";
  }

  void staged_block(const std::vector<int>& dk, const std::set<int>& hold, const std::set<int>& stream, bool holdB) {
    std::vector<int> hv(hold.begin(), hold.end()), sv(stream.begin(), stream.end());
    lds_slots = std::max(lds_slots, (int)hv.size());
    for (size_t k = 0; k < hv.size(); ++k) {
      emit(hv[k]);
      os << ind << "{ " << lds_index((int)k) << " qx::lds_put<" << T << ">(qx_lds + ix, " << v.block << ", "
         << name(hv[k]) << "); }\n";
    }
    std::map<std::pair<int, int>, std::vector<int>> dots;  // (held, streamed) -> Dot nodes
    for (int k : dk) {
      auto ops = dot_ops(d.nodes[k]);
      int J = producer(ops.first), B = producer(ops.second);
      dots[holdB ? std::make_pair(B, J) : std::make_pair(J, B)].push_back(k);
    }
    for (size_t t0 = 0; t0 < sv.size(); t0 += kTile) {
      size_t t1 = std::min(sv.size(), t0 + kTile);
      for (size_t t = t0; t < t1; ++t) emit(sv[t]);
      for (size_t k = 0; k < hv.size(); ++k) {
        bool any = false;
        for (size_t t = t0; t < t1 && !any; ++t) any = dots.count({hv[k], sv[t]}) > 0;
        if (!any) continue;
        std::string tmp = "h" + std::to_string(hv[k]) + "_" + std::to_string(t0);
        os << ind << "{\n";
        std::string outer = ind;
        ind += "  ";
        os << ind << lds_index((int)k) << "\n";
        os << ind << "const qx::sp4<" << T << "> " << tmp << " = qx::lds_get<" << T << ">(qx_lds + ix, " << v.block
           << ");\n";
        alias[hv[k]] = tmp;
        for (size_t t = t0; t < t1; ++t) {
          auto it = dots.find({hv[k], sv[t]});
          if (it == dots.end()) continue;
          for (int dkk : it->second) emit_dot(dkk);
        }
        alias.erase(hv[k]);
        ind = outer;
        os << ind << "}\n";
      }
    }
  }

  void forward_block_inner(uint32_t key, const std::vector<int>& dk) {
    (void)key;
    std::set<int> Bs, Js;
    for (int k : dk) {
      auto ops = dot_ops(d.nodes[k]);
      Js.insert(producer(ops.first));
      Bs.insert(producer(ops.second));
    }
    bool holdB = Bs.size() <= Js.size();
    const std::set<int>& hold = holdB ? Bs : Js;
    const std::set<int>& stream = holdB ? Js : Bs;
    if (stage()) {
      staged_block(dk, hold, stream, holdB);
      return;
    }
    for (int h : hold) emit(h);
    auto stream_one = [&](int s) {
      emit(s);
      for (int k : dk) {
        auto ops = dot_ops(d.nodes[k]);
        int sp = producer(holdB ? ops.first : ops.second);
        if (sp == s) emit_dot(k);
      }
    };
    // with the shared e-_in side each spin-1 leaf follows its spin-0 twin
    std::map<int, int> after;
    if (coop && !holdB)
      for (int s : stream)
        if (ein1(s) && stream.count(twin(s))) after[twin(s)] = s;
    for (int s : stream) {
      if (coop && !holdB && ein1(s) && stream.count(twin(s))) continue;
      stream_one(s);
      auto a = after.find(s);
      if (a != after.end()) stream_one(a->second);
    }
  }

  // The partitions of the photons into the two sides of the joins, in the
  // slot order used by slot_loop: iteration t puts photons subsets[t] on the
  // e-_in side; returns the table of particle indices [NIT][P].
  std::vector<int> slot_table() const {
    const int P = pr.P, j = d.split;
    std::vector<int> tab;
    for (uint32_t m = 0; m < (1u << P); ++m) {
      if (popc(m) != j) continue;
      for (int a = 0; a < P; ++a)
        if ((m >> a) & 1) tab.push_back(pr.photon_particle[a]);
      for (int a = 0; a < P; ++a)
        if (!((m >> a) & 1)) tab.push_back(pr.photon_particle[a]);
    }
    return tab;
  }

  void emit_slot_table() {
    std::vector<int> tab = slot_table();
    os << "__constant__ int " << slot_tab << "[" << tab.size() << "] = {";
    for (size_t i = 0; i < tab.size(); ++i) os << (i ? ", " : "") << tab[i];
    os << "};\n";
    if (cur_cache) {
      os << "__constant__ int " << ix_tab << "[" << tab.size() << "] = {";
      for (size_t i = 0; i < tab.size(); ++i) os << (i ? ", " : "") << slot_of(tab[i]);
      os << "};\n";
    }
  }

  void slot_loop(std::map<uint32_t, std::vector<int>>& part) {
    const int P = pr.P;
    const uint32_t key = (1u << d.split) - 1;
    const int nit = (int)(slot_table().size() / P);
    if (!part.count(key)) throw std::logic_error("canonical partition missing");
    for (int p : {pr.i_ein, pr.i_eout})
      for (int mu = 0; mu < 4; ++mu)
        os << ind << "const double m" << p << "_" << mu << " = mom[" << (4 * p + mu) << " * N + ptc];\n";
    if (pol_lds && !cur_cache)
      for (int a = 0; a < P; ++a) {
        int pp = pr.photon_particle[a];
        os << ind << "{ const qx::pol3<" << PT << "> e_ = qx::pol<" << PT << ">(mom[" << (4 * pp + 1) << " * N + ptc], mom["
           << (4 * pp + 2) << " * N + ptc], mom[" << (4 * pp + 3) << " * N + ptc], (int)((hc >> " << pp << ") & 1u));";
        for (int c = 0; c < 3; ++c)
          os << " qx_pol[" << (3 * pp + c) * v.block << " + threadIdx.x] = e_.e" << (c + 1) << ";";
        os << " }\n";
      }
    double pre = 0.0;  // FLOPs per lane before the loop
    if (cur_cache) {
      // photons sub, sub + 2, ... of the point: polarisation vector and the
      // two one-photon currents into the per-point cache (photon index a is
      // particle a + 1 for the n_in incoming photons, a + 2 after e-_out)
      const int ein = pr.i_ein, eout = pr.i_eout, nin = eout - 1;
      auto mref = [&](int p) {
        std::string m = "m" + std::to_string(p) + "_";
        return m + "0, " + m + "1, " + m + "2, " + m + "3";
      };
      if (body_mode)
        wave_sync();  // the previous tile's reads of the region come first
      else
        os << ind << "const int tpt = (int)(threadIdx.x >> " << __builtin_ctz(CL) << ");\n";
      os << ind << "const int q_ = (int)(sub & " << CL - 1 << "u);\n";
      os << ind << "{\n";
      os << ind << "  const qx::sp4<double> ue_ = qx::u_in<double>(" << mref(ein) << ", (int)((hc >> " << ein
         << ") & 1u), 1.0);\n";
      if (!row_only)
        os << ind << "  const qx::sp4<double> ub_ = qx::ubar_out<double>(" << mref(eout) << ", (int)((hc >> " << eout
           << ") & 1u), 1.0);\n";
      os << ind << "  #pragma unroll\n" << ind << "  for (int j = 0; j < " << (P + CL - 1) / CL << "; ++j) {\n";
      os << ind << "    const int a = " << CL << " * j + q_;\n";
      os << ind << "    if (a < " << P << ") {\n";
      os << ind << "      const int pp = a + (a < " << nin << " ? 1 : 2);\n";
      os << ind << "      const double s_ = a < " << nin << " ? 1.0 : -1.0;\n";
      os << ind << "      double k_[4];\n";
      os << ind << "      for (int mu = 0; mu < 4; ++mu) k_[mu] = mom[(4 * pp + mu) * N + ptc];\n";
      os << ind << "      const qx::pol3<double> e_ = qx::pol<double>(k_[1], k_[2], k_[3], (int)((hc >> pp) & 1u));\n";
      for (int c = 0; c < 3; ++c) os << ind << "      " << cache_pol("a", c) << " = (" << T << ")e_.e" << (c + 1) << ";\n";
      if (k_lds)
        for (int mu = 0; mu < 4; ++mu) os << ind << "      " << cache_k("a", mu) << " = s_ * k_[" << mu << "];\n";
      os << ind << "      const qx::sp4<double> r_ = qx::sL<double>(qx::vL<double>(ue_, e_), qx::prop_from<double>("
         << mref(ein) << ", s_ * k_[0], s_ * k_[1], s_ * k_[2], s_ * k_[3], 1.0, 1.0));\n";
      if (!row_only)
        os << ind << "      const qx::sp4<double> c_ = qx::sR<double>(qx::vR<double>(ub_, e_), qx::prop_from<double>("
           << mref(eout) << ", s_ * k_[0], s_ * k_[1], s_ * k_[2], s_ * k_[3], -1.0, 1.0));\n";
      for (int side = 0; side < (row_only ? 1 : 2); ++side)
        for (int k = 0; k < 4; ++k)
          os << ind << "      " << cache_cur(side, "a", 2 * k) << " = (" << T << ")" << (side ? "c_" : "r_") << ".c[" << k
             << "].r; " << cache_cur(side, "a", 2 * k + 1) << " = (" << T << ")" << (side ? "c_" : "r_") << ".c[" << k
             << "].i;\n";
      os << ind << "    }\n" << ind << "  }\n" << ind << "}\n";
      if (body_mode)
        wave_sync();
      else
        os << ind << "__syncthreads();\n";
      pre = (row_only ? 16 : 2 * 16) + (P + CL - 1) / CL * (16 + 4 + (row_only ? 1 : 2) * (40 + 28 + 56));
    }
    std::string outer = ind;
    if (!cur_cache) {
      os << ind << "#pragma unroll 1\n" << ind << "for (int it = 0; it < " << nit << "; ++it) {\n";
      ind += "  ";
      for (int a = 0; a < P; ++a) {
        os << ind << "const int sp" << a << " = " << slot_tab << "[it * " << P << " + " << a << "];\n";
        os << ind << "const double sg" << a << " = sp" << a << " < " << pr.i_eout << " ? 1.0 : -1.0;\n";
        os << ind << "const int hb" << a << " = (int)((hc >> sp" << a << ") & 1u);\n";
        for (int mu = 0; mu < 4; ++mu)
          os << ind << "const double k" << a << "_" << mu << " = mom[(4 * sp" << a << " + " << mu << ") * N + ptc];\n";
      }
    } else {
      // lane q of a point takes partitions CL i2 + q: the loop index stays
      // uniform, so the table entries are scalar loads and each lane selects
      // its own; where the count is not a multiple of CL the last round's
      // spare lanes repeat the last partition and drop their result
      os << ind << "#pragma unroll 1\n" << ind << "for (int i2 = 0; i2 < " << (nit + CL - 1) / CL << "; ++i2) {\n";
      ind += "  ";
      for (int q = 0; q < CL; ++q)
        os << ind << "const int it" << q << " = " << CL << " * i2 + " << q << " < " << nit << " ? " << CL << " * i2 + " << q
           << " : " << nit - 1 << ";\n";
      for (int a = 0; a < P; ++a) {
        for (int q = 0; q < CL; ++q)
          os << ind << "int x" << q << "_" << a << " = " << ix_tab << "[it" << q << " * " << P << " + " << a
             << "]; asm volatile(\"\" : \"+s\"(x" << q << "_" << a << "));\n";
        std::string sel = "x" + std::to_string(CL - 1) + "_" + std::to_string(a);
        for (int q = CL - 2; q >= 0; --q)
          sel = "q_ == " + std::to_string(q) + " ? x" + std::to_string(q) + "_" + std::to_string(a) + " : (" + sel + ")";
        os << ind << "const int ix" << a << " = " << sel << ";\n";
        if (!k_lds) {
          const int nin = pr.i_eout - 1;
          os << ind << "const int sp" << a << " = ix" << a << " + (ix" << a << " < " << nin << " ? 1 : 2);\n";
          os << ind << "const double sg" << a << " = ix" << a << " < " << nin << " ? 1.0 : -1.0;\n";
          os << ind << "const double* const kp" << a << " = mom + (long long)(4 * sp" << a << ") * N + ptc;\n";
          for (int mu = 0; mu < 4; ++mu)
            os << ind << "const double k" << a << "_" << mu << " = kp" << a << "[" << mu << " * N];\n";
        }
      }
      if (nit % CL)
        for (auto& kv : acc_of_sum) {
          const int a = kv.second;
          os << ind << "const qx::cx<" << T << "> As" << a << " = A" << a << ";\n";
          if (v.prec != PREC_F64) os << ind << "const qx::cx<float> Cs" << a << " = C" << a << ";\n";
          if (abs_sum) os << ind << "const float Ss" << a << " = S" << a << ";\n";
        }
    }
    std::fill(done.begin(), done.end(), 0);
    kdone.clear();
    qdone.clear();
    qdone_d.clear();
    has_d.clear();
    double f0 = st.flops_per_point;
    bool was_local = (v.order & 4) != 0;
    (void)was_local;
    forward_block_inner(key, part[key]);
    // per lane: the loop's share of the partitions (the caller multiplies by
    // the lanes of a point)
    st.flops_per_point = f0 + pre + (st.flops_per_point - f0) * ((nit + CL - 1) / CL);
    if (cur_cache && nit % CL) {
      os << ind << "if (" << CL << " * i2 + q_ >= " << nit << ") {";
      for (auto& kv : acc_of_sum) {
        const int a = kv.second;
        os << " A" << a << " = As" << a << ";";
        if (v.prec != PREC_F64) os << " C" << a << " = Cs" << a << ";";
        if (abs_sum) os << " S" << a << " = Ss" << a << ";";
      }
      os << " }\n";
    }
    ind = outer;
    os << ind << "}\n";
    if (cur_cache && v.prec == PREC_F64) {
      // the point's lanes' partial amplitudes
      for (int o = 1; o < CL; o <<= 1)
        for (auto& kv : acc_of_sum)
          os << ind << "A" << kv.second << ".r += __shfl_xor(A" << kv.second << ".r, " << o << "); A" << kv.second
             << ".i += __shfl_xor(A" << kv.second << ".i, " << o << ");\n";
      st.flops_per_point += 2.0 * __builtin_ctz(CL) * (double)acc_of_sum.size();
    }
  }

  // Body: accumulators, all nodes in partition-grouped order, |A|^2 sums
  // added into the double `acc` of the enclosing scope.
  void body() {
    std::vector<int> sums = sum_nodes();
    for (size_t a = 0; a < sums.size(); ++a) {
      acc_of_sum[sums[a]] = (int)a;
      os << ind << "qx::cx<" << T << "> A" << a << " = {" << T << "(0), " << T << "(0)};\n";
      if (v.prec != PREC_F64) os << ind << "qx::cx<float> C" << a << " = {0.0f, 0.0f};\n";
      if (abs_sum) os << ind << "float S" << a << " = 0.0f;\n";
    }
    std::map<uint32_t, std::vector<int>> part;
    std::vector<uint32_t> order;
    partitions(part, order);
    if (mfma_join()) {
      mfma_body(part, order, (int)sums.size());
      return;
    }
    if (slot) {
      slot_loop(part);
    } else {
      if (r1_cache) emit_r1_cache();
      for (uint32_t key : order) forward_block(key, part[key]);
    }
    // |A|^2, summed over the enumerated configurations (HelSum) or single
    for (size_t a = 0; a < sums.size(); ++a) {
      if (amp_store) {
        // staged in per-lane LDS (qx_as) and stored below: stores with
        // their 64-bit addresses held while the accumulators are live spilled
        os << ind << "qx_as[" << (2 * a) * v.block << " + threadIdx.x] = A" << a << ".r; qx_as[" << (2 * a + 1) * v.block
           << " + threadIdx.x] = A" << a << ".i;\n";
      }
      if (v.prec == PREC_F64) {
        os << ind << "acc += A" << a << ".r * A" << a << ".r + A" << a << ".i * A" << a << ".i;\n";
      } else {
        os << ind << "{ double ar = (double)A" << a << ".r + (double)C" << a << ".r, ai = (double)A" << a
           << ".i + (double)C" << a << ".i;";
        if (abs_sum) os << " double sa = (double)S" << a << ";";
        if (cur_cache)
          // the point's lanes' partial sums, combined in FP64
          for (int o = 1; o < CL; o <<= 1) {
            os << " ar += __shfl_xor(ar, " << o << "); ai += __shfl_xor(ai, " << o << ");";
            if (abs_sum) os << " sa += __shfl_xor(sa, " << o << ");";
          }
        os << " acc += ar * ar + ai * ai;";
        if (abs_sum) os << " if (!(sa <= fix_kappa * fix_kappa * (ar * ar + ai * ai))) fixflag = 1;";
        os << " }\n";
      }
      st.flops_per_point += 4;
    }
    if (amp_store) {
      // amplitude of configuration hc | (the Sum's enumerated bits) to
      // amp[2h][N], amp[2h+1][N] (shared e-_in side: lane 1's accumulators
      // carry swapped e-_in labels).  Unguarded: a lane past the end computes
      // point N-1 (ptc) exactly as that point's own lane does and stores the
      // same bytes.
      os << ind << "{\n" << ind << "  const unsigned qx_cf[" << sums.size() << "] = {";
      for (size_t a = 0; a < sums.size(); ++a) os << (a ? ", " : "") << d.nodes[sums[a]].cfg << "u";
      os << "};\n";
      std::string flip = coop ? " ^ (((hc >> " + std::to_string(pr.i_eout) + ") & 1u) << " + std::to_string(pr.i_ein) + ")" : "";
      os << ind << "  #pragma unroll 4\n" << ind << "  for (int a = 0; a < " << sums.size() << "; ++a) {\n";
      os << ind << "    const unsigned hh = hc | (qx_cf[a]" << flip << ");\n";
      os << ind << "    amp[(2 * hh) * N + ptc] = qx_as[2 * a * " << v.block << " + threadIdx.x];\n";
      os << ind << "    amp[(2 * hh + 1) * N + ptc] = qx_as[(2 * a + 1) * " << v.block << " + threadIdx.x];\n";
      os << ind << "  }\n" << ind << "}\n";
    }
  }

  // ---------------------------------------------------------------------
  // Join on the FP64 matrix cores (order flag 128; a measured experiment,
  // not a default).  Graphs whose every photon partition pairs 4 row
  // currents with 4 column currents, each pair the dot of a different one
  // of 16 amplitudes (the distributive helicity-sum graph with 4 photons
  // and the spins on lanes): per partition, each lane stores its row and
  // column currents in the wave's LDS staging area, and the 4 x 4 complex
  // dot matrices of two lanes at a time are computed by two
  // v_mfma_f64_4x4x4 (real part R_re J_re^T - R_im J_im^T and imaginary
  // part R_re J_im^T + R_im J_re^T, K = 4 spinor components).  Every
  // partition maps the 16 amplitudes to the 4 x 4 positions differently; a
  // lane permutation (__shfl) brings them to the first partition's layout
  // before they are accumulated.  The amplitudes are then gathered back to
  // their lanes through LDS for |A|^2.
  // ---------------------------------------------------------------------
  bool mfma_join() const { return (v.order & 128) != 0; }
  std::string mj_tab;  // kernel-name prefix of the per-partition permutation tables

  void mfma_body(std::map<uint32_t, std::vector<int>>& part, const std::vector<uint32_t>& order, int nsum) {
    if (v.prec != PREC_F64 || nsum != 16 || slot || stage())
      throw std::invalid_argument("the matrix-core join takes FP64 graphs with 16 amplitudes per lane");
    // per partition: row and column currents (index = position in the 4 x 4
    // block) and the amplitude of every position
    std::vector<std::array<int, 16>> pos_amp;
    std::vector<std::vector<int>> rows, cols;
    for (uint32_t key : order) {
      std::vector<int> B, J;
      std::array<int, 16> pa;
      pa.fill(-1);
      for (int k : part[key]) {
        const Node& dn = d.nodes[k];
        if (dn.kind != Kind::Dot) throw std::invalid_argument("matrix-core join: split joins only");
        auto ops = dot_ops(dn);
        int j = producer(ops.first), b = producer(ops.second);
        if (std::find(B.begin(), B.end(), b) == B.end()) B.push_back(b);
        if (std::find(J.begin(), J.end(), j) == J.end()) J.push_back(j);
        int r = (int)(std::find(B.begin(), B.end(), b) - B.begin());
        int c = (int)(std::find(J.begin(), J.end(), j) - J.begin());
        if (r > 3 || c > 3) throw std::invalid_argument("matrix-core join: a partition with more than 4 x 4 currents");
        int a = acc_of_sum.at(d.nodes[dn.out[0]].out[0]);
        if (pa[4 * r + c] >= 0) throw std::invalid_argument("matrix-core join: repeated dot");
        pa[4 * r + c] = a;
      }
      for (int x : pa)
        if (x < 0) throw std::invalid_argument("matrix-core join: incomplete 4 x 4 block");
      rows.push_back(B);
      cols.push_back(J);
      pos_amp.push_back(pa);
    }
    // position of every amplitude in the first partition (the accumulator layout)
    std::array<int, 16> pos0;
    for (int q = 0; q < 16; ++q) pos0[pos_amp[0][q]] = q;
    os << ind << "double mj[32];\n" << ind << "#pragma unroll\n" << ind << "for (int t = 0; t < 32; ++t) mj[t] = 0.0;\n";
    os << ind << "double* const mj_stg = qx_mj + (threadIdx.x >> 6) * " << 64 * kMjStride << ";\n";
    os << ind << "const int mj_lane = (int)(threadIdx.x & 63);\n";
    for (size_t p = 0; p < order.size(); ++p) {
      fence(1);
      os << ind << "// photons " << order[p] << " | " << (((1u << pr.P) - 1) & ~order[p])
         << " on the e-_in | e-_out side: 4 x 4 dots on the matrix cores\n";
      for (int b : rows[p]) emit(b);
      for (int j : cols[p]) emit(j);
      os << ind << "{\n";
      std::string o = ind;
      ind += "  ";
      os << ind << "double* const st_ = mj_stg + mj_lane * " << kMjStride << ";\n";
      for (int r = 0; r < 4; ++r)
        for (int k = 0; k < 4; ++k) {
          os << ind << "st_[" << 4 * r + k << "] = " << name(rows[p][r]) << ".c[" << k << "].r; st_[" << 16 + 4 * r + k
             << "] = " << name(rows[p][r]) << ".c[" << k << "].i;\n";
          os << ind << "st_[" << 32 + 4 * r + k << "] = " << name(cols[p][r]) << ".c[" << k << "].r; st_["
             << 48 + 4 * r + k << "] = " << name(cols[p][r]) << ".c[" << k << "].i;\n";
        }
      // source lane (within the lane's block) of the accumulator position
      // (i, j) = ((lane >> 4), lane & 3): where this partition put that amplitude
      os << ind << "const int src_ = " << mj_tab << "[" << p << " * 16 + ((mj_lane >> 4) << 2) + (mj_lane & 3)] + (mj_lane & 12);\n";
      os << ind << "qx::mfma_join4(mj_stg, " << kMjStride << ", src_, mj);\n";
      ind = o;
      os << ind << "}\n";
      st.flops_per_point += 16 * 32;
      st.n_dot += 16;
      (void)pos0;
    }
    // amplitudes back to their lanes, then |A|^2
    os << ind << "#pragma unroll\n" << ind << "for (int t = 0; t < 32; ++t) {\n";
    os << ind << "  const int blk_ = (mj_lane >> 2) & 3;\n";
    os << ind << "  mj_stg[(2 * t + (blk_ >> 1)) * " << kMjStride << " + (blk_ & 1) * 16 + (mj_lane >> 4) * 4 + (mj_lane & 3)] = mj[t];\n";
    os << ind << "}\n";
    os << ind << "#pragma unroll\n" << ind << "for (int q = 0; q < 32; ++q) { const double v_ = mj_stg[mj_lane * " << kMjStride
       << " + q]; acc += v_ * v_; }\n";
    st.flops_per_point += 16 * 4;
    // permutation tables: entry (i0, j0) of partition p is 16 i_p + j_p
    std::ostringstream tab;
    tab << "__constant__ int " << mj_tab << "[" << 16 * order.size() << "] = {";
    for (size_t p = 0; p < order.size(); ++p)
      for (int q0 = 0; q0 < 16; ++q0) {
        int a = pos_amp[0][q0];
        int qp = -1;
        for (int q = 0; q < 16; ++q)
          if (pos_amp[p][q] == a) qp = q;
        tab << (p || q0 ? ", " : "") << 16 * (qp >> 2) + (qp & 3);
      }
    tab << "};\n";
    mj_tables = tab.str();
  }
  std::string mj_tables;
  static constexpr int kMjStride = 65;  // doubles per lane in the staging area (padded against bank conflicts)

  // ---------------------------------------------------------------------
  // Adjoint pass.  Per partition block: the e-_in-side leaves are recomputed
  // and held; the e-_out-side prefix trie is walked depth first, recomputing
  // each current from its parent, taking the dots at its leaves and folding
  // each node's adjoint into its parent on the way back; then the e-_in-side
  // trie is walked the same way with the leaf adjoints gathered at the dots.
  // Only the current path is live: currents are recomputed, not stored.
  // ---------------------------------------------------------------------
  std::set<int> blk;
  std::map<int, std::vector<int>> cons;
  std::set<int> leafJ;

  bool final_particle(int p) const { return p == pr.i_eout || (p > pr.i_eout); }

  // momentum-gradient accumulator of (particle p, component mu): a register,
  // or a per-lane LDS slot when gm_in_lds is set (keeps it out of the
  // register file during the adjoint sweep)
  bool gm_in_lds = false;
  std::string gmref(int p, int mu) const {
    if (!gm_in_lds) return "gm" + std::to_string(p) + "_" + std::to_string(mu);
    if (p < pr.i_eout) throw std::logic_error("gmref(): no gradient slot for an incoming particle");
    return "qx_gm[" + std::to_string((4 * (p - pr.i_eout) + mu) * v.block) + " + threadIdx.x]";
  }

  // Polarisation-vector gradients of the walked side in per-lane LDS slots
  // (ge_in_lds), allocated on first use; a polarisation whose gradient the
  // block never touches gets no slot and no pol_vjp.
  bool ge_in_lds = false;
  const std::string ge_zero_mark = "//@GEZERO@\n";
  std::map<int, int> ge_slot;
  int ge_index(int x) {
    auto it = ge_slot.find(x);
    if (it != ge_slot.end()) return it->second;
    int k = (int)ge_slot.size();
    ge_slot[x] = k;
    return k;
  }
  std::string geref(int slot, int c) const {
    return "qx_ge[" + std::to_string((3 * slot + c) * v.block) + " + threadIdx.x]";
  }
  // vertex gradient with respect to the polarisation vector of node u
  void emit_ge(const std::string& side, const std::string& w, const std::string& X, int u) {
    if (!ge_in_lds) {
      os << ind << "qx::v" << side << "_ge<double>(" << w << ", " << X << ", ge" << u << ");\n";
      return;
    }
    const int k = ge_index(u);
    os << ind << "{ qx::pol3<double> t = {0.0, 0.0, 0.0}; qx::v" << side << "_ge<double>(" << w << ", " << X
       << ", t); " << addto(geref(k, 0), "t.e1") << " " << addto(geref(k, 1), "t.e2") << " " << addto(geref(k, 2), "t.e3")
       << " }\n";
  }

  // Propagator-coefficient gradients accumulated per distinct propagator
  // (side, photon set) in per-lane LDS, across every iteration of the
  // kernel, and mapped to momentum gradients once at its end (the map
  // gq -> (gp, gK) is linear and depends on the momenta only).  Keeps the
  // propagator kinematics out of the registers of the adjoint walk.
  bool gq_in_lds = false;
  std::map<std::pair<int, uint32_t>, int> gq_slot;
  int gq_index(int side, uint32_t mask) {
    auto it = gq_slot.find({side, mask});
    if (it != gq_slot.end()) return it->second;
    int k = (int)gq_slot.size();
    gq_slot[{side, mask}] = k;
    return k;
  }
  std::string gqref(int slot, int c) const {
    return "qx_gq[" + std::to_string((5 * slot + c) * v.block) + " + threadIdx.x]";
  }

  // statement adding val (negated if neg) to the accumulator ref: +=, or,
  // with lds_atomic set, for a per-lane LDS slot (qx_*) an LDS atomic add
  // whose result is not read (ds_add_f64: no read-modify-write round trip
  // for the wave to wait on; each slot belongs to one lane, so the adds keep
  // program order).  Measured per kernel: faster in the e-_out-side walks,
  // slower in the e-_in-side ones (whose repeated adds to one slot the
  // compiler otherwise merges in registers).
  bool lds_atomic = false;
  std::string addto(const std::string& ref, const std::string& val, bool neg = false) const {
    if (!lds_atomic || ref.compare(0, 3, "qx_") != 0) return ref + (neg ? " -= " : " += ") + val + ";";
    return "__hip_atomic_fetch_add(&" + ref + ", " + (neg ? "-(" + val + ")" : val) +
           ", __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);";
  }

  void collect_block(const std::vector<int>& dk) {
    blk.clear();
    cons.clear();
    std::vector<int> stk(dk.begin(), dk.end());
    while (!stk.empty()) {
      int x = stk.back();
      stk.pop_back();
      if (blk.count(x)) continue;
      blk.insert(x);
      for (int p : d.nodes[x].in) {
        int pp = producer(p);
        if (d.nodes[pp].kind == Kind::Entry) continue;
        cons[pp].push_back(x);
        stk.push_back(pp);
      }
    }
  }

  std::string fname(int x) const { return (done[x] ? "n" : "f") + std::to_string(x); }

  // signed photon-momentum sum K of a propagator, in Kl0..Kl3.  opaque: the
  // values pass through an empty asm, so the compiler cannot merge equal
  // sums (and the propagator set-up that follows) across the scopes of an
  // adjoint walk and keep them live from one scope to the next; each scope
  // recomputes its own.
  void emit_K_inline(uint32_t mask, bool opaque = false) {
    for (int mu = 0; mu < 4; ++mu) {
      os << ind << (opaque ? "double Kl" : "const double Kl") << mu << " = 0.0";
      for (int a = 0; a < pr.P; ++a)
        if ((mask >> a) & 1)
          os << (pr.photon_sign[a] > 0 ? " + " : " - ") << "m" << pr.photon_particle[a] << "_" << mu;
      os << ";\n";
    }
    if (opaque) os << ind << "asm volatile(\"\" : \"+v\"(Kl0), \"+v\"(Kl1), \"+v\"(Kl2), \"+v\"(Kl3));\n";
  }

  void prop_grad_to_momenta(int side, uint32_t mask) {
    int pe = side == 0 ? pr.i_ein : pr.i_eout;
    std::string m = "m" + std::to_string(pe) + "_";
    os << ind << "{ double gp[4] = {0.0, 0.0, 0.0, 0.0}, gK[4] = {0.0, 0.0, 0.0, 0.0};\n";
    os << ind << "  qx::prop_from_vjp(" << m << "0, " << m << "1, " << m << "2, " << m << "3, Kl0, Kl1, Kl2, Kl3, "
       << (side == 0 ? "1.0" : "-1.0") << ", 1.0, gq, gp, gK);\n";
    if (final_particle(pe))
      for (int mu = 0; mu < 4; ++mu) os << ind << "  " << addto(gmref(pe, mu), "gp[" + std::to_string(mu) + "]") << "\n";
    for (int a = 0; a < pr.P; ++a)
      if (((mask >> a) & 1) && final_particle(pr.photon_particle[a]))
        for (int mu = 0; mu < 4; ++mu)
          os << ind << "  "
             << addto(gmref(pr.photon_particle[a], mu), "gK[" + std::to_string(mu) + "]", pr.photon_sign[a] < 0) << "\n";
    os << ind << "}\n";
  }

  // momentum gradients of every accumulated propagator (end of the kernel;
  // momenta m<p>_<mu> in scope)
  void flush_gq() {
    for (auto& kv : gq_slot) {
      const int side = kv.first.first;
      const uint32_t mask = kv.first.second;
      os << ind << "{\n";
      std::string o = ind;
      ind += "  ";
      emit_K_inline(mask);
      const char* f[5] = {"qm", "qp", "q1", "q2", "mm"};
      os << ind << "qx::propq<double> gq;\n";
      for (int c = 0; c < 5; ++c) os << ind << "gq." << f[c] << " = " << gqref(kv.second, c) << ";\n";
      prop_grad_to_momenta(side, mask);
      ind = o;
      os << ind << "}\n";
    }
  }

  // Emit the adjoint contribution of consumer c (of current x) into w<x>.
  void rev(int c, int x) {
    const Node& n = d.nodes[c];
    if (n.kind == Kind::Dot) {
      auto ops = dot_ops(n);
      int J = producer(ops.first), B = producer(ops.second);
      int sum = d.nodes[n.out[0]].out[0];
      os << ind << "qx::dot_vjp<double>(c" << acc_of_sum.at(sum) << ", " << fname(B) << ", " << fname(J) << ", w" << B
         << ", w" << J << ");\n";
      st.flops_per_point += 64;
      return;
    }
    const std::string X = fname(x);
    os << ind << "{\n";
    std::string outer = ind;
    ind += "  ";
    const bool leaf = leafJ.count(c) > 0;
    // adjoint of c: its own accumulator, or (factored block, column leaf)
    // the seed shared by the leaves of its configurations
    const std::string wc = (leaf && factored) ? "W" + std::to_string(memJ.at(c)) : "w" + std::to_string(c);
    if (n.kind == Kind::S1) {
      emit_K_inline(n.mask, true);
      int pe = n.side == 0 ? pr.i_ein : pr.i_eout;
      std::string m = "m" + std::to_string(pe) + "_";
      os << ind << "const qx::propq<double> q = qx::prop_from<double>(" << m << "0, " << m << "1, " << m << "2, " << m
         << "3, Kl0, Kl1, Kl2, Kl3, " << (n.side == 0 ? "1.0" : "-1.0") << ", 1.0);\n";
      st.flops_per_point += 28;
    }
    const std::string side = n.side == 0 ? "L" : "R", other = n.side == 0 ? "R" : "L";
    std::string E;
    if (n.kind == Kind::V) E = "n" + std::to_string(producer(n.in[0]));
    if (!leaf) {
      if (n.kind == Kind::V)
        os << ind << "const qx::sp4<double> f" << c << " = qx::v" << side << "<double>(" << X << ", " << E << ");\n";
      else
        os << ind << "const qx::sp4<double> f" << c << " = qx::s" << side << "<double>(" << X << ", q);\n";
      if (factored && memB.count(c)) {
        // row leaf of a factored block: its adjoint is the row seed of its
        // configurations; in the one-kernel sweep it also joins their row
        // sum (the split e-_in-side kernel recomputes those sums itself)
        os << ind << "const qx::sp4<double> w" << c << " = T" << memB.at(c) << ";\n";
        if (grad_phase == 0) {
          os << ind << "qx::add_to(SB" << memB.at(c) << ", f" << c << ");\n";
          st.flops_per_point += 8;
        }
        st.flops_per_point += n.kind == Kind::V ? 40 : 56;
      } else {
        os << ind << "qx::sp4<double> w" << c << " = qx::zero4<double>();\n";
        st.flops_per_point += n.kind == Kind::V ? 40 : 56;
        for (int c2 : cons[c]) rev(c2, c);
      }
    }
    if (n.kind == Kind::V) {
      os << ind << "qx::add_to(w" << x << ", qx::v" << other << "<double>(" << wc << ", " << E << "));\n";
      st.flops_per_point += 40;
      // polarisation gradient, for final-state photons only (the incoming
      // photon's momentum is fixed)
      if (final_particle(d.nodes[producer(n.in[0])].particle)) {
        emit_ge(side, wc, X, producer(n.in[0]));
        st.flops_per_point += 48;
      }
    } else {
      os << ind << "qx::add_to(w" << x << ", qx::s" << other << "<double>(" << wc << ", q));\n";
      os << ind << "qx::propq<double> gq = {0.0, 0.0, 0.0, 0.0, 0.0};\n";
      os << ind << "qx::s" << side << "_gq<double>(" << wc << ", " << X << ", gq);\n";
      if (gq_in_lds) {
        const int k = gq_index(n.side, n.mask);
        const char* f[5] = {"qm", "qp", "q1", "q2", "mm"};
        for (int c = 0; c < 5; ++c) os << ind << addto(gqref(k, c), std::string("gq.") + f[c]) << "\n";
      } else {
        prop_grad_to_momenta(n.side, n.mask);
      }
      st.flops_per_point += 56 + 64 + 60;
    }
    ind = outer;
    os << ind << "}\n";
  }

  // ---------------------------------------------------------------------
  // Adjoint over a distributed graph (subset currents).  Its currents form a
  // DAG (an Add has several parents), so the sweep runs top-down from each
  // join: a node's adjoint is pushed to its inputs, recomputing the forward
  // value of an input where a parameter gradient needs it.  Nothing but the
  // adjoints of the current path is held.
  // ---------------------------------------------------------------------
  int tmpc = 0;
  std::string tmpname(const char* p) { return std::string(p) + std::to_string(tmpc++); }

  // statements computing the value of current node x; returns the variable
  std::string fwd(int x) {
    x = producer(x);
    const Node& n = d.nodes[x];
    std::string v = tmpname("f");
    switch (n.kind) {
      case Kind::U:
        emit(x);
        return name(x);
      case Kind::V: {
        std::string y = fwd(n.in[1]);
        bool yp = d.nodes[producer(n.in[0])].hel == 1;
        os << ind << "const qx::sp4<double> " << v << " = qx::v" << (n.side == 0 ? "L" : "R") << (yp ? "_y" : "")
           << "<double>(" << y << ", " << name(n.in[0]) << ");\n";
        st.flops_per_point += yp ? 24 : 40;
        return v;
      }
      case Kind::S1: {
        std::string y = fwd(n.in[0]);
        os << ind << "qx::sp4<double> " << v << ";\n" << ind << "{\n";
        std::string o = ind;
        ind += "  ";
        emit_K_inline(n.mask);
        int pe = n.side == 0 ? pr.i_ein : pr.i_eout;
        std::string m = "m" + std::to_string(pe) + "_";
        os << ind << "const qx::propq<double> q = qx::prop_from<double>(" << m << "0, " << m << "1, " << m << "2, " << m
           << "3, Kl0, Kl1, Kl2, Kl3, " << (n.side == 0 ? "1.0" : "-1.0") << ", 1.0);\n";
        os << ind << v << " = qx::s" << (n.side == 0 ? "L" : "R") << "<double>(" << y << ", q);\n";
        ind = o;
        os << ind << "}\n";
        st.flops_per_point += 28 + 56;
        return v;
      }
      case Kind::Add: {
        std::string e = fwd(n.in[0]);
        for (size_t t = 1; t < n.in.size(); ++t) e = "qx::add4<double>(" + e + ", " + fwd(n.in[t]) + ")";
        os << ind << "const qx::sp4<double> " << v << " = " << e << ";\n";
        st.flops_per_point += 8.0 * (double)(n.in.size() - 1);
        return v;
      }
      default:
        throw std::logic_error("fwd(): not a current");
    }
  }

  // push adjoint w of current node x to its inputs and to the momentum gradient
  void adj(int x, const std::string& w) {
    x = producer(x);
    const Node& n = d.nodes[x];
    switch (n.kind) {
      case Kind::U:
        if (n.particle == pr.i_eout) {
          std::string m = "m" + std::to_string(pr.i_eout) + "_";
          os << ind << "{ double g[4]; qx::ubar_vjp(" << m << "0, " << m << "1, " << m << "2, " << m << "3, "
             << hel_expr(n) << ", 1.0, " << w << ", g);\n";
          for (int mu = 0; mu < 4; ++mu) os << ind << "  " << addto(gmref(pr.i_eout, mu), "g[" + std::to_string(mu) + "]") << "\n";
          os << ind << "}\n";
        }
        return;
      case Kind::Add:
        for (int y : n.in) adj(y, w);
        return;
      case Kind::V: {
        os << ind << "{\n";
        std::string o = ind;
        ind += "  ";
        const std::string side = n.side == 0 ? "L" : "R", other = n.side == 0 ? "R" : "L";
        std::string y = fwd(n.in[1]);
        os << ind << "qx::v" << side << "_ge<double>(" << w << ", " << y << ", ge" << producer(n.in[0]) << ");\n";
          std::string wy = tmpname("w");
        os << ind << "const qx::sp4<double> " << wy << " = qx::v" << other << "<double>(" << w << ", "
           << name(n.in[0]) << ");\n";
        st.flops_per_point += 48 + 40;
        adj(n.in[1], wy);
        ind = o;
        os << ind << "}\n";
        return;
      }
      case Kind::S1: {
        os << ind << "{\n";
        std::string o = ind;
        ind += "  ";
        const std::string side = n.side == 0 ? "L" : "R", other = n.side == 0 ? "R" : "L";
        std::string y = fwd(n.in[0]);
        emit_K_inline(n.mask);
        int pe = n.side == 0 ? pr.i_ein : pr.i_eout;
        std::string m = "m" + std::to_string(pe) + "_";
        os << ind << "const qx::propq<double> q = qx::prop_from<double>(" << m << "0, " << m << "1, " << m << "2, " << m
           << "3, Kl0, Kl1, Kl2, Kl3, " << (n.side == 0 ? "1.0" : "-1.0") << ", 1.0);\n";
        os << ind << "qx::propq<double> gq = {0.0, 0.0, 0.0, 0.0, 0.0};\n";
        os << ind << "qx::s" << side << "_gq<double>(" << w << ", " << y << ", gq);\n";
        prop_grad_to_momenta(n.side, n.mask);
        std::string wy = tmpname("w");
        os << ind << "const qx::sp4<double> " << wy << " = qx::s" << other << "<double>(" << w << ", q);\n";
        st.flops_per_point += 28 + 64 + 60 + 56;
        adj(n.in[0], wy);
        ind = o;
        os << ind << "}\n";
        return;
      }
      default:
        throw std::logic_error("adj(): not a current");
    }
  }

  void dist_adjoint_block(uint32_t key, const std::vector<int>& dk) {
    os << ind << "// adjoint (subset currents): photons " << key << " | " << (((1u << pr.P) - 1) & ~key) << "\n";
    std::string outer = open_block();
    flush_seeds();
    std::vector<int> pols;
    for (size_t i = 0; i < d.nodes.size(); ++i) {
      const Node& n = d.nodes[i];
      if (n.kind == Kind::U && n.particle != pr.i_ein && n.particle != pr.i_eout) {
        emit((int)i);
        os << ind << "qx::pol3<double> ge" << i << " = {0.0, 0.0, 0.0};\n";
        pols.push_back((int)i);
      }
    }
    for (int k : dk) {
      const Node& dn = d.nodes[k];
      auto ops = dot_ops(dn);
      int sum = d.nodes[dn.out[0]].out[0];
      std::string jv = fwd(ops.first), bv = fwd(ops.second);
      std::string wj = tmpname("w"), wb = tmpname("w");
      os << ind << "qx::sp4<double> " << wj << " = qx::zero4<double>(), " << wb << " = qx::zero4<double>();\n";
      os << ind << "qx::dot_vjp<double>(c" << acc_of_sum.at(sum) << ", " << bv << ", " << jv << ", " << wb << ", " << wj
         << ");\n";
      st.flops_per_point += 64;
      adj(ops.second, wb);
      adj(ops.first, wj);
    }
    for (int u : pols) {
      const Node& n = d.nodes[u];
      if (!final_particle(n.particle)) continue;
      std::string m = "m" + std::to_string(n.particle) + "_";
      os << ind << "{ double g[3]; qx::pol_vjp(" << m << "1, " << m << "2, " << m << "3, " << hel_expr(n) << ", ge" << u
         << ", g);\n";
      for (int mu = 1; mu < 4; ++mu) os << ind << "  " << addto(gmref(n.particle, mu), "g[" + std::to_string(mu - 1) + "]") << "\n";
      os << ind << "}\n";
    }
    close_block(outer);
  }

  // Factored adjoint of a partition block.  For each configuration a the
  // block's dots pair every row leaf B of a with every column leaf J of a
  // (all orderings of the photons on either side), so the block's share of
  // the amplitude is A_a = (sum_B B) . (sum_J J) and its adjoint needs only
  // the sums: w_B = sum_{a: B in a} c_a SJ_a, w_J = sum_{a: J in a} c_a SB_a.
  // No leaf or leaf adjoint is held across the other side's sweep; the
  // sums are kept per membership pattern (the set of configurations a leaf
  // belongs to, a bit mask over the block's accumulators).
  bool factored = false;
  std::map<int, uint32_t> memB, memJ;

  bool factor_block(const std::vector<int>& dk) {
    memB.clear();
    memJ.clear();
    std::map<int, std::set<std::pair<int, int>>> pairs;
    for (int k : dk) {
      const Node& dn = d.nodes[k];
      if (dn.kind != Kind::Dot) return false;
      auto ops = dot_ops(dn);
      int J = producer(ops.first), B = producer(ops.second);
      int a = acc_of_sum.at(d.nodes[dn.out[0]].out[0]);
      if (a >= 32 || !pairs[a].insert({B, J}).second) return false;
      memB[B] |= 1u << a;
      memJ[J] |= 1u << a;
    }
    for (auto& kv : pairs) {
      std::set<int> Bs, Js;
      for (auto& bj : kv.second) {
        Bs.insert(bj.first);
        Js.insert(bj.second);
      }
      if (kv.second.size() != Bs.size() * Js.size()) return false;
    }
    for (auto& kv : memB) {
      const Node& b = d.nodes[kv.first];
      if (b.kind != Kind::S1 && b.kind != Kind::V) return false;
      for (int c2 : cons[kv.first])
        if (d.nodes[c2].kind != Kind::Dot) return false;
    }
    return true;
  }

  // sum over the configurations a in `pat` of c_a times the patterns' sums
  // S<q> of every pattern q containing a
  void emit_seed(const std::string& out, uint32_t pat, const std::string& S, const std::set<uint32_t>& pats,
                 bool declare = true) {
    if (declare) os << ind << "qx::sp4<double> " << out << " = qx::zero4<double>();\n";
    for (int a = 0; a < 32; ++a) {
      if (!((pat >> a) & 1)) continue;
      for (uint32_t q : pats)
        if ((q >> a) & 1) {
          os << ind << "qx::axpy<double>(" << out << ", c" << a << ", " << S << q << ");\n";
          st.flops_per_point += 32;
        }
    }
  }

  // Split adjoint kernels (grad_phase): 0 = the whole partition sweep; 1 =
  // the e-_out-side walk; 2 = the e-_in-side walk.  Each of the two kernels
  // holds only its own walk's state: the seeds of its side come from a
  // forward walk of the other side's trie in a scope of its own (its leaf
  // sums), so nothing passes between the two kernels but the momentum
  // gradients they add.
  int grad_phase = 0;
  // Split kernels whose walked side has no looped photon: the walk's forward
  // currents are the same in every loop iteration and its adjoints are
  // linear in the seeds, so the seeds are summed over the iterations
  // (merge_part 1, inside the loop: the other side's leaf sums and the seed
  // sums) and the side is walked once (merge_part 2, after the loop).
  int merge_part = 0;
  // statements defining the adjoint seeds c<a> (partition adjoint kernels),
  // emitted by the block where it first needs them
  std::string seed_code;
  void flush_seeds() {
    std::istringstream in(seed_code);
    for (std::string line; std::getline(in, line);) os << ind << line << "\n";
    seed_code.clear();
  }

  // forward walk of the leaves `leaves` (node -> pattern) in a scope of its
  // own, summing them per pattern into <S><pattern>; its currents die with
  // the scope (the adjoint walk recomputes what it needs)
  void leaf_sums(const std::map<int, uint32_t>& leaves, const std::string& S, const std::set<uint32_t>& pats) {
    for (uint32_t q : pats) os << ind << "qx::sp4<double> " << S << q << " = qx::zero4<double>();\n";
    os << ind << "{\n";
    std::string o = ind;
    ind += "  ";
    std::vector<char> done0 = done;
    std::set<uint32_t> kdone0 = kdone;
    std::set<std::pair<int, uint32_t>> qdone0 = qdone;
    for (auto& kv : leaves) {
      emit(kv.first);
      os << ind << "qx::add_to(" << S << kv.second << ", " << name(kv.first) << ");\n";
      st.flops_per_point += 8;
    }
    done = done0;
    kdone = kdone0;
    qdone = qdone0;
    ind = o;
    os << ind << "}\n";
  }

  void grad_block(uint32_t key, const std::vector<int>& dk) {
    collect_block(dk);
    os << ind << "// adjoint: photons " << key << " | " << (((1u << pr.P) - 1) & ~key) << "\n";
    std::string outer = open_block();
    // polarisation-gradient accumulators of this block (registers, or LDS
    // slots zeroed at the marker once the walk has allocated them)
    for (int x : blk) {
      const Node& n = d.nodes[x];
      if (n.kind == Kind::U && n.particle != pr.i_ein && n.particle != pr.i_eout) {
        emit(x);
        if (!ge_in_lds && merge_part != 1) os << ind << "qx::pol3<double> ge" << x << " = {0.0, 0.0, 0.0};\n";
      }
    }
    if (ge_in_lds && merge_part != 1) os << ge_zero_mark;
    leafJ.clear();
    for (int k : dk) leafJ.insert(producer(dot_ops(d.nodes[k]).first));
    factored = factor_block(dk);
    std::set<uint32_t> patB, patJ;
    if (factored) {
      for (auto& kv : memB) patB.insert(kv.second);
      for (auto& kv : memJ) patJ.insert(kv.second);
    }
    if (merge_part == 1) {
      // the other side's leaf sums and this iteration's share of the seeds
      if (grad_phase == 2) {
        leaf_sums(memB, "SB", patB);
        flush_seeds();
        for (uint32_t q : patJ) emit_seed("W" + std::to_string(q), q, "SB", patB, false);
      } else {
        leaf_sums(memJ, "SJ", patJ);
        flush_seeds();
        for (uint32_t q : patB) emit_seed("T" + std::to_string(q), q, "SJ", patJ, false);
      }
      close_block(outer);
      return;
    }
    if (merge_part == 2) {
      // seeds summed over the loop (declared by the kernel)
    } else if (factored && grad_phase == 2) {
      // the e-_out side's leaf sums, from a forward walk of the row trie
      leaf_sums(memB, "SB", patB);
      flush_seeds();
    } else if (factored) {
      // column sums per pattern, from a forward walk of the column trie
      leaf_sums(memJ, "SJ", patJ);
      flush_seeds();
      // row seeds, and (one-kernel sweep) the row sums the row sweep
      // accumulates
      for (uint32_t q : patB) emit_seed("T" + std::to_string(q), q, "SJ", patJ);
      if (grad_phase == 0)
        for (uint32_t q : patB) os << ind << "qx::sp4<double> SB" << q << " = qx::zero4<double>();\n";
    } else {
      flush_seeds();
      for (int J : leafJ) {
        emit(J);
        os << ind << "qx::sp4<double> w" << J << " = qx::zero4<double>();\n";
      }
    }
    // e-_out side trie (dots at its leaves), then e-_in side trie
    for (int pass = 0; pass < 2; ++pass) {
      if ((grad_phase == 1 && pass == 1) || (grad_phase == 2 && pass == 0)) continue;
      int root_particle = pass == 0 ? pr.i_eout : pr.i_ein;
      if (pass == 1 && factored && merge_part != 2)
        for (uint32_t q : patJ) emit_seed("W" + std::to_string(q), q, "SB", patB);
      for (int r : blk) {
        const Node& n = d.nodes[r];
        if (n.kind != Kind::U || n.particle != root_particle) continue;
        emit(r);
        os << ind << "qx::sp4<double> w" << r << " = qx::zero4<double>();\n";
        for (int c : cons[r]) rev(c, r);
        if (pass == 0) {
          std::string m = "m" + std::to_string(pr.i_eout) + "_";
          os << ind << "{ double g[4]; qx::ubar_vjp(" << m << "0, " << m << "1, " << m << "2, " << m << "3, "
             << hel_expr(n) << ", 1.0, w" << r << ", g);\n";
          for (int mu = 0; mu < 4; ++mu) os << ind << "  " << addto(gmref(pr.i_eout, mu), "g[" + std::to_string(mu) + "]") << "\n";
          os << ind << "}\n";
        }
      }
    }
    // polarisation vectors -> photon momenta
    for (int x : blk) {
      const Node& n = d.nodes[x];
      if (n.kind == Kind::U && n.particle != pr.i_ein && n.particle != pr.i_eout && final_particle(n.particle)) {
        std::string ge = "ge" + std::to_string(x);
        if (ge_in_lds) {
          auto it = ge_slot.find(x);
          if (it == ge_slot.end()) continue;  // gradient never touched by this block
          ge = "qx::pol3<double>{" + geref(it->second, 0) + ", " + geref(it->second, 1) + ", " +
               geref(it->second, 2) + "}";
        }
        std::string m = "m" + std::to_string(n.particle) + "_";
        os << ind << "{ double g[3]; qx::pol_vjp(" << m << "1, " << m << "2, " << m << "3, " << hel_expr(n) << ", " << ge
           << ", g);\n";
        for (int mu = 1; mu < 4; ++mu)
          os << ind << "  " << addto(gmref(n.particle, mu), "g[" + std::to_string(mu - 1) + "]") << "\n";
        os << ind << "}\n";
      }
    }
    close_block(outer);
  }

  // momenta for a partition-local block, opaque to the compiler
  void block_momenta() {
    if (mom_src == 2) return;  // momenta already in m<p>_<mu> of the enclosing scope
    if (mom_src == 0 && batch_mom) {
      // loaded together: an empty asm takes 16 values at a time (short of
      // registers the compiler otherwise waits for each load in turn)
      os << ind << "long long pq = ptc;\n" << ind << "asm volatile(\"\" : \"+v\"(pq));\n";
      std::vector<std::string> ms;
      for (int p = 0; p < pr.npart; ++p)
        for (int mu = 0; mu < 4; ++mu) {
          ms.push_back("m" + std::to_string(p) + "_" + std::to_string(mu));
          os << ind << "double " << ms.back() << " = mom[" << (4 * p + mu) << " * N + pq];\n";
        }
      for (size_t i0 = 0; i0 < ms.size(); i0 += 16) {
        os << ind << "asm volatile(\"\" :";
        for (size_t i = i0; i < std::min(ms.size(), i0 + 16); ++i) os << (i > i0 ? ", " : " ") << "\"+v\"(" << ms[i] << ")";
        os << ");\n";
      }
    } else if (mom_src == 0) {
      os << ind << "long long pq = ptc;\n" << ind << "asm volatile(\"\" : \"+v\"(pq));\n";
      load_momenta("mom", "N", "pq");
    } else {
      for (int p = 0; p < pr.npart; ++p)
        for (int mu = 0; mu < 4; ++mu)
          os << ind << "double m" << p << "_" << mu << " = M" << p << "_" << mu << "; asm volatile(\"\" : \"+v\"(m" << p
             << "_" << mu << "));\n";
    }
  }

  void load_momenta(const std::string& base, const std::string& N, const std::string& pt) {
    for (int p = 0; p < pr.npart; ++p)
      for (int mu = 0; mu < 4; ++mu)
        os << ind << "const double m" << p << "_" << mu << " = " << base << "[" << (4 * p + mu) << " * " << N
           << " + " << pt << "];\n";
  }

  // deposit the low bits of x into the positions of mask
  static std::string deposit(const std::string& x, uint32_t mask) {
    std::string s;
    int k = 0;
    for (int b = 0; b < 32; ++b)
      if ((mask >> b) & 1) {
        if (!s.empty()) s += " | ";
        s += "(((" + x + " >> " + std::to_string(k) + ") & 1u) << " + std::to_string(b) + ")";
        ++k;
      }
    return s.empty() ? "0u" : s;
  }

  // the per-lane part common to the kernel and the body function: helicity
  // code, loop over loop bits, graph body
  void lane_work(const std::string& hrt_expr) {
    os << ind << "const unsigned hrt = " << hrt_expr << ";\n";
    int nloop = popc(v.loop_mask);
    if (nloop > 0) {
      os << ind << "for (unsigned lp = 0; lp < " << (1u << nloop) << "u; ++lp) {\n";
      ind = "    ";
      os << ind << "const unsigned hc = hrt | " << deposit("lp", v.loop_mask) << ";\n";
      // order flag 32: momenta reloaded per iteration through an opaque index,
      // so nothing is hoisted out of the loop and kept live across it
      if (loop_local()) block_momenta();
      body();
      ind = "  ";
      os << ind << "}\n";
    } else {
      os << ind << "const unsigned hc = hrt;\n";
      body();
    }
  }
};

void check_variant(const Dag& d, const Variant& v) {
  uint32_t all = (1u << d.proc.npart) - 1;
  if (d.enum_mask != v.enum_mask) throw std::invalid_argument("graph/variant enumeration mismatch");
  if ((v.enum_mask & v.lane_mask) || (v.enum_mask & v.loop_mask) || (v.lane_mask & v.loop_mask))
    throw std::invalid_argument("helicity bit classes overlap");
  if (v.mode == HEL_SUM && (v.enum_mask | v.lane_mask | v.loop_mask) != all)
    throw std::invalid_argument("SUM mode must cover every helicity bit");
  if (v.mode == HEL_PER_POINT && (v.enum_mask | v.lane_mask | v.loop_mask) != 0)
    throw std::invalid_argument("PER_POINT mode takes every bit from the input");
  if (popc(v.lane_mask) > 6) throw std::invalid_argument("at most 64 lanes per point");
  if (v.order & 8)
    for (int a = 0; a < d.proc.P; ++a)
      if ((v.enum_mask >> d.proc.photon_particle[a]) & 1)
        throw std::invalid_argument("the partition loop takes photon helicities at run time only");
  if (v.block % 64 != 0 || v.block < 64 || v.block > 1024) throw std::invalid_argument("bad block size");
  if (((v.order & (256 | 512)) &&
       ((v.order & 256 && v.order & 512) || !(v.order & 8) || v.mode != HEL_PER_POINT || (v.order & 64) ||
        v.lane_mask || d.split < 2 || d.proc.P - d.split < 1 || d.distributed)) ||
      ((v.order & 1024) && !(v.order & (256 | 512))) || ((v.order & 8192) && !(v.order & 4)) ||
      ((v.order & 2048) && (v.mode != HEL_SUM || v.lane_mask != (1u << d.proc.i_eout) ||
                            !((v.enum_mask >> d.proc.i_ein) & 1u) || (v.order & (8 | 16 | 128)) || d.distributed)))
    throw std::invalid_argument(
        "the one-photon current cache takes per-point partition loops with split >= 2; the shared e-_in side "
        "takes helicity sums with the e-_out spin as the one lane bit and the e-_in spin in the graph; batched "
        "block momenta take per-partition blocks");
}

// The one-photon current cache of a variant for BP points per LDS region
// whose budget is `budget` bytes: sets e's cache fields; throws if even the
// currents and polarisations do not fit.
void setup_cache(Emitter& e, const Dag& d, const Variant& v, const std::string& kname, int BP, int64_t budget) {
  e.cur_cache = true;
  e.CL = cache_lanes(v);
  e.BP = BP;
  e.ix_tab = kname + "_ix";
  e.row_only = (v.order & 1024) != 0;
  const int64_t per = (int64_t)d.proc.P * BP;                  // photon-points
  const int tsz = v.prec == PREC_F64 ? 8 : 4;                   // currents, polarisations
  const int ncur = e.row_only ? 8 : 16;
  if ((ncur + 3) * tsz * per > budget) throw std::invalid_argument("the current cache does not fit the LDS");
  e.k_lds = ((ncur + 3) * tsz + 4 * 8) * per <= budget;        // momenta in FP64
}

// Bytes of the cache's three arrays for BP points (polarisations and
// currents in the graph's type, momenta in FP64).
int64_t cache_bytes(const Emitter& e, const Dag& d, const Variant& v) {
  const int tsz = v.prec == PREC_F64 ? 8 : 4;
  return (((e.row_only ? 8 : 16) + 3) * tsz + (e.k_lds ? 32 : 0)) * (int64_t)d.proc.P * e.BP;
}

}  // namespace

int body_cache_doubles(const Dag& d, const Variant& v) {
  if (!(v.order & (256 | 512))) return 0;
  Emitter e(d, v);
  setup_cache(e, d, v, "", 64 / cache_lanes(v), kBodyCacheBytes);
  return (int)((cache_bytes(e, d, v) + 7) / 8);
}

std::string emit_eval_kernel(const Dag& d, const Variant& v, const std::string& kname, EmitStats* stats) {
  check_variant(d, v);
  Emitter e(d, v);
  const int G = lanes_per_point(v);
  const int LB = __builtin_ctz(G);
  std::ostringstream& os = e.os;
  os << "// generated by qedx: " << variant_tag(v, d.proc.n_out, d.proc.n_in) << "\n";
  os << "#include <hip/hip_runtime.h>\n";
  os << device_header_text() << "\n";
  if (v.fixup) {
    if (v.prec != PREC_F32C || v.mode != HEL_PER_POINT)
      throw std::invalid_argument("the FP64 fix-up is built for FP32C per-point kernels");
    if (v.order & 16) throw std::invalid_argument("the FP64 fix-up excludes LDS staging");
    e.abs_sum = true;
  }
  if (v.order & 8) {
    e.slot = true;
    e.pol_lds = true;
    e.slot_tab = kname + "_slots";
    if (v.order & (256 | 512)) {
      // polarisations (3), currents (16, or 8 for the e-_in side only) and
      // momenta (4) per photon and point; the momenta only where the
      // workgroups that min_waves asks for still fit the 160 KB of LDS of a
      // compute unit (4 SIMDs)
      const int64_t budget = (int64_t)160 * 1024 * v.block / (256 * std::max(1, v.min_waves));
      setup_cache(e, d, v, kname, v.block / cache_lanes(v), budget);
    }
    e.emit_slot_table();
  }
  if (v.order & 2048) {
    e.coop = true;
    e.build_twins();
  }
  e.batch_mom = (v.order & 8192) != 0;
  if (v.order & 4096) {
    if (!(v.order & 2048) || !(v.order & 4) || v.prec != PREC_F64)
      throw std::invalid_argument("the e-_in-side current cache takes FP64 helicity sums with the shared e-_in side");
    e.r1_cache = true;
    e.r1_collect();
  }
  e.mj_tab = kname + "_mjperm";
  const std::string mj_mark = "//@MJTAB@\n";
  if (e.mfma_join()) {
    if (v.block != 256) throw std::invalid_argument("the matrix-core join takes 256-lane workgroups");
    os << mj_mark;
  }
  os << "extern \"C\" __global__ void __launch_bounds__(" << v.block;
  if (v.min_waves > 0) os << ", " << v.min_waves;
  os << ")\n" << kname
     << "(const double* __restrict__ mom, const unsigned* __restrict__ hel, long long N, double* __restrict__ out"
     << (v.fixup ? ", double fix_kappa" : "") << ")\n{\n";
  const std::string lds_mark = "  //@LDS@\n";
  os << lds_mark;
  os << "  const long long gid = (long long)blockIdx.x * " << v.block << " + threadIdx.x;\n";
  os << "  const long long pt = gid >> " << LB << ";\n";
  os << "  const unsigned sub = (unsigned)(gid & " << (G - 1) << ");\n";
  os << "  const long long ptc = pt < N ? pt : N - 1;\n";
  if (!e.local() && !e.slot && !e.loop_local()) e.load_momenta("mom", "N", "ptc");
  os << "  double acc = 0.0;\n";
  if (v.fixup) os << "  int fixflag = 0;\n";
  std::string hrt = v.mode == HEL_PER_POINT ? "hel[ptc]" : Emitter::deposit("sub", v.lane_mask);
  e.lane_work(hrt);
  // helicity lanes hold parts of the sum (the cache's two lanes hold the
  // same |A|^2, their amplitudes already combined)
  for (int o = e.CL; o < G; o <<= 1) os << "  acc += __shfl_xor(acc, " << o << ");\n";
  if (v.fixup)
    // a point the FP32 pass cannot resolve is marked in place with a negative
    // value (|M|^2 itself is never negative); the FP64 pass below finds it
    os << "  if (pt < N && sub == 0u) out[pt] = fixflag ? -1.0 : acc;\n}\n";
  else
    os << "  if (pt < N && sub == 0u) out[pt] = acc;\n}\n";
  // per point: every lane of the group does the body once per loop iteration
  e.st.flops_per_point *= (double)G * (double)(1 << popc(v.loop_mask));
  std::string src = os.str();
  {
    // per-lane LDS slots for staged currents: [slot][8 words][block]
    std::string decl;
    if (e.lds_slots > 0)
      decl = "  __shared__ " + e.T + " qx_lds[" + std::to_string(e.lds_slots * 8 * v.block) + "];\n";
    if (e.cur_cache) {
      decl += "  __shared__ " + e.T + " qx_pol[" + std::to_string(3 * d.proc.P * e.BP) + "];\n";
      decl += "  __shared__ " + e.T + " qx_cur[" + std::to_string((e.row_only ? 8 : 16) * d.proc.P * e.BP) + "];\n";
      if (e.k_lds) decl += "  __shared__ double qx_k[" + std::to_string(4 * d.proc.P * e.BP) + "];\n";
    } else if (e.pol_lds) {
      decl += "  __shared__ " + e.PT + " qx_pol[" + std::to_string(3 * d.proc.npart * v.block) + "];\n";
    }
    if (e.mfma_join()) decl += "  __shared__ double qx_mj[" + std::to_string(4 * 64 * Emitter::kMjStride) + "];\n";
    if (e.r1_cache) decl += "  __shared__ double qx_r1[" + std::to_string(8 * e.r1_slot.size() * v.block) + "];\n";
    size_t at = src.find(lds_mark);
    src.replace(at, lds_mark.size(), decl);
    if (e.mfma_join()) src.replace(src.find(mj_mark), mj_mark.size(), e.mj_tables);
  }
  if (v.fixup) {
    // FP64 pass over the points the FP32C kernel could not resolve
    Variant v64 = v;
    v64.prec = PREC_F64;
    v64.fixup = 0;
    v64.min_waves = 0;
    EmitStats st64;
    std::ostringstream fx;
    fx << emit_body_function(d, v64, kname + "_b64", &st64) << "\n";
    // with the one-photon current cache the FP64 body takes CL lanes per
    // point and its wave's LDS region
    const int CL = cache_lanes(v64);
    const int W = body_cache_doubles(d, v64);
    // Each workgroup of 256 lanes owns kFixRange consecutive points: it scans
    // their results for the negative marks, compacts the marked offsets in
    // LDS (one LDS atomic per wave: ballot, then each marked lane's rank
    // among the marked lanes below it) and recomputes them 256 / CL at a
    // time, so the FP64 body runs on full waves however sparse the marks are.
    fx << "extern \"C\" __global__ void __launch_bounds__(256)\n"
       << kname << "_fix(const double* __restrict__ mom, const unsigned* __restrict__ hel, long long N, "
       << "double* __restrict__ out)\n{\n"
       << (W ? "  __shared__ double qx_fc[" + std::to_string(4 * W) + "];\n" : std::string())
       << "  __shared__ unsigned fx_list[" << kFixRange << "];\n"
       << "  __shared__ unsigned fx_cnt;\n"
       << "  if (threadIdx.x == 0) fx_cnt = 0u;\n"
       << "  __syncthreads();\n"
       << "  const long long base = (long long)blockIdx.x * " << kFixRange << ";\n"
       << "  const unsigned ln_ = __lane_id();\n"
       << "  for (unsigned i = threadIdx.x; i < " << kFixRange << "u; i += 256u) {\n"
       << "    const long long pt = base + (long long)i;\n"
       << "    const bool f_ = pt < N && out[pt] < 0.0;\n"
       << "    const unsigned long long fm_ = __ballot(f_);\n"
       << "    if (fm_) {\n"
       << "      const unsigned ld_ = (unsigned)__ffsll((unsigned long long)fm_) - 1u;\n"
       << "      unsigned b_ = 0u;\n"
       << "      if (ln_ == ld_) b_ = atomicAdd(&fx_cnt, (unsigned)__popcll(fm_));\n"
       << "      b_ = __shfl(b_, (int)ld_);\n"
       << "      if (f_) fx_list[b_ + (unsigned)__popcll(fm_ & ((1ull << ln_) - 1ull))] = i;\n"
       << "    }\n"
       << "  }\n"
       << "  __syncthreads();\n"
       << "  const unsigned cnt = fx_cnt;\n";
    if (CL == 1) {
      fx << "  for (unsigned j = threadIdx.x; j < cnt; j += 256u) {\n"
         << "    const long long pt = base + (long long)fx_list[j];\n"
         << "    out[pt] = " << kname << "_b64(mom, N, pt, hel[pt]);\n"
         << "  }\n}\n";
    } else {
      // every lane takes part in every round (the body synchronises its wave)
      const int sh = __builtin_ctz(CL);
      fx << "  const unsigned sub = threadIdx.x & " << CL - 1 << "u;\n"
         << "  for (unsigned j0 = 0; j0 < cnt; j0 += " << 256 / CL << "u) {\n"
         << "    const unsigned j = j0 + (threadIdx.x >> " << sh << ");\n"
         << "    const long long pt = base + (long long)fx_list[j < cnt ? j : cnt - 1u];\n"
         << "    const double r = " << kname << "_b64(mom, N, pt, hel[pt], qx_fc + (threadIdx.x >> 6) * " << W
         << ", (int)((threadIdx.x & 63u) >> " << sh << "), sub);\n"
         << "    if (j < cnt && sub == 0u) out[pt] = r;\n"
         << "  }\n}\n";
    }
    src += fx.str();
  }
  e.st.lines = std::count(src.begin(), src.end(), '\n');
  if (stats) *stats = e.st;
  return src;
}

std::string emit_grad_kernel(const Dag& d, const Variant& v, const std::string& kname, EmitStats* stats) {
  check_variant(d, v);
  if (v.mode != HEL_SUM || v.prec != PREC_F64 || !(v.order & 4) || (v.order & 16) || d.distributed)
    throw std::invalid_argument("gradient kernels take SUM, FP64, local blocks, the node-reduced graph");
  Emitter e(d, v);
  e.mom_src = 1;
  const Process& pr = d.proc;
  const int LB = popc(v.lane_mask), G = 1 << LB;
  const int NF = pr.n_out + 1;
  std::ostringstream& os = e.os;
  os << "extern \"C\" __global__ void __launch_bounds__(" << v.block;
  if (v.min_waves > 0) os << ", " << v.min_waves;
  os << ")\n" << kname
     << "(const double* __restrict__ u, double sqrt_s, long long N, double* __restrict__ logm2, double* __restrict__ "
        "grad)\n{\n";
  os << "  const long long gid = (long long)blockIdx.x * " << v.block << " + threadIdx.x;\n";
  os << "  const long long pt = gid >> " << LB << ";\n";
  os << "  const unsigned sub = (unsigned)(gid & " << (G - 1) << ");\n";
  os << "  const long long ptc = pt < N ? pt : N - 1;\n";
  for (int p = 0; p < pr.npart; ++p) os << "  double M" << p << "_0, M" << p << "_1, M" << p << "_2, M" << p << "_3;\n";
  os << "  {\n    double uu[" << 4 * NF << "];\n";
  os << "    for (int r = 0; r < " << 4 * NF << "; ++r) uu[r] = u[r * N + ptc];\n";
  os << "    qx::RamboState<" << NF << "> S;\n    qx::rambo_forward<" << NF << ">(uu, sqrt_s, 1.0, S);\n";
  os << "    double pin[4], kin[4];\n    qx::incoming_cm(sqrt_s, 1.0, pin, kin);\n";
  for (int mu = 0; mu < 4; ++mu) os << "    M0_" << mu << " = pin[" << mu << "]; M1_" << mu << " = kin[" << mu << "];\n";
  for (int j = 0; j < NF; ++j)
    for (int mu = 0; mu < 4; ++mu) os << "    M" << (2 + j) << "_" << mu << " = S.k[" << j << "][" << mu << "];\n";
  os << "  }\n";
  // Helicity bits: lane bits from the lane index, enumerated bits inside the
  // graph, loop bits by a run-time loop.  With loop bits the forward graph
  // runs twice: once over all iterations for |M|^2, then again per iteration
  // for the amplitudes that seed that iteration's adjoint sweep (recomputed,
  // not stored).
  const int nloop = popc(v.loop_mask);
  os << "  const unsigned hrt = " << Emitter::deposit("sub", v.lane_mask) << ";\n";
  os << "  double acc = 0.0;\n";
  std::map<uint32_t, std::vector<int>> part;
  std::vector<uint32_t> order;
  e.partitions(part, order);
  std::vector<int> sums = e.sum_nodes();
  auto seeds_and_adjoint = [&]() {
    for (size_t a = 0; a < sums.size(); ++a)
      os << e.ind << "const qx::cx<double> c" << a << " = {A" << a << ".r * iM2, -A" << a << ".i * iM2};\n";
    for (uint32_t key : order) e.grad_block(key, part[key]);
  };
  auto gm_init = [&]() {
    for (int p = 2; p < pr.npart; ++p)
      for (int mu = 0; mu < 4; ++mu) os << "  double gm" << p << "_" << mu << " = 0.0;\n";
  };
  auto reduce_acc = [&]() {
    for (int o = 1; o < G; o <<= 1) os << "  acc += __shfl_xor(acc, " << o << ");\n";
    os << "  const double iM2 = 1.0 / acc;\n";
  };
  if (nloop == 0) {
    os << "  const unsigned hc = hrt;\n";
    e.body();
    reduce_acc();
    gm_init();
    seeds_and_adjoint();
  } else {
    const std::string loop_head = "  #pragma unroll 1\n  for (unsigned lp = 0; lp < " + std::to_string(1u << nloop) +
                                  "u; ++lp) {\n    const unsigned hc = hrt | " + Emitter::deposit("lp", v.loop_mask) +
                                  ";\n";
    const std::string ind0 = e.ind;
    os << loop_head;
    e.ind = "    ";
    e.body();
    e.ind = ind0;
    os << "  }\n";
    reduce_acc();
    gm_init();
    os << loop_head;
    e.ind = "    ";
    os << e.ind << "double acc = 0.0;\n";  // |A|^2 of the recomputed pass, unused
    e.body();
    os << e.ind << "(void)acc;\n";
    seeds_and_adjoint();
    e.ind = ind0;
    os << "  }\n";
  }
  for (int p = 2; p < pr.npart; ++p)
    for (int mu = 0; mu < 4; ++mu)
      for (int o = 1; o < G; o <<= 1) os << "  gm" << p << "_" << mu << " += __shfl_xor(gm" << p << "_" << mu << ", " << o << ");\n";
  os << "  {\n    double uu[" << 4 * NF << "];\n";
  os << "    for (int r = 0; r < " << 4 * NF << "; ++r) uu[r] = u[r * N + ptc];\n";
  os << "    qx::RamboState<" << NF << "> S;\n    qx::rambo_forward<" << NF << ">(uu, sqrt_s, 1.0, S);\n";
  os << "    double gk[" << NF << "][4] = {";
  for (int j = 0; j < NF; ++j) {
    os << (j ? ", " : "") << "{";
    for (int mu = 0; mu < 4; ++mu) os << (mu ? ", " : "") << "gm" << (2 + j) << "_" << mu;
    os << "}";
  }
  os << "};\n";
  os << "    double gu[" << 4 * NF << "];\n    for (int r = 0; r < " << 4 * NF << "; ++r) gu[r] = 0.0;\n";
  os << "    qx::rambo_vjp<" << NF << ">(uu, sqrt_s, 1.0, S, gk, gu);\n";
  os << "    if (pt < N && sub == 0u) {\n      logm2[pt] = log(acc);\n";
  os << "      for (int r = 0; r < " << 4 * NF << "; ++r) grad[r * N + pt] = gu[r];\n    }\n  }\n}\n";
  e.st.flops_per_point *= (double)G * (double)(1 << popc(v.loop_mask));
  if (stats) *stats = e.st;
  return os.str();
}

// ---------------------------------------------------------------------------
// Split gradient: amplitude kernel + one adjoint kernel per photon partition
// ---------------------------------------------------------------------------
std::string emit_amp_kernel(const Dag& d, const Variant& v, const std::string& kname, EmitStats* stats) {
  check_variant(d, v);
  if (v.mode != HEL_SUM || v.prec != PREC_F64 || (v.order & (8 | 16)) || d.distributed)
    throw std::invalid_argument("amplitude kernels take SUM, FP64, the node-reduced graph, no loop or LDS schedule");
  Emitter e(d, v);
  e.amp_store = true;
  e.batch_mom = (v.order & 8192) != 0;
  if (v.order & 2048) {
    e.coop = true;
    e.build_twins();
  }
  const Process& pr = d.proc;
  const int LB = popc(v.lane_mask), G = 1 << LB;
  std::ostringstream& os = e.os;
  os << "extern \"C\" __global__ void __launch_bounds__(" << v.block << ")\n" << kname
     << "(const double* __restrict__ mom, long long N, double* __restrict__ amp, double* __restrict__ logm2, "
        "double* __restrict__ im2)\n{\n";
  os << "  const long long gid = (long long)blockIdx.x * " << v.block << " + threadIdx.x;\n";
  os << "  const long long pt = gid >> " << LB << ";\n";
  os << "  const unsigned sub = (unsigned)(gid & " << (G - 1) << ");\n";
  os << "  const long long ptc = pt < N ? pt : N - 1;\n";
  {
    // per-lane staging of one iteration's amplitudes
    Emitter probe(d, v);
    os << "  __shared__ double qx_as[" << 2 * probe.sum_nodes().size() * v.block << "];\n";
  }
  if (!e.local()) e.load_momenta("mom", "N", "ptc");
  os << "  double acc = 0.0;\n";
  e.lane_work(Emitter::deposit("sub", v.lane_mask));
  for (int o = 1; o < G; o <<= 1) os << "  acc += __shfl_xor(acc, " << o << ");\n";
  os << "  if (pt < N && sub == 0u) { logm2[pt] = log(acc); im2[pt] = 1.0 / acc; }\n}\n";
  e.st.flops_per_point *= (double)G * (double)(1 << popc(v.loop_mask));
  if (stats) *stats = e.st;
  return os.str();
}

std::vector<std::pair<uint32_t, int>> adjoint_walks(const Dag& d, const Variant& v) {
  std::map<uint32_t, std::vector<int>> part;
  std::vector<uint32_t> order;
  Emitter probe(d, v);
  probe.partitions(part, order);
  std::vector<std::pair<uint32_t, int>> w;
  for (uint32_t key : order) {
    bool split = false;
    if (!d.distributed) {
      Emitter pe(d, v);
      std::vector<int> ps = pe.sum_nodes();
      for (size_t a = 0; a < ps.size(); ++a) pe.acc_of_sum[ps[a]] = (int)a;
      pe.collect_block(part[key]);
      split = pe.factor_block(part[key]);
    }
    if (split) {
      w.push_back({key, 1});
      w.push_back({key, 2});
    } else {
      w.push_back({key, 0});
    }
  }
  return w;
}

std::string emit_partition_adjoint_kernels(const Dag& d, const Variant& v, const std::string& kprefix, int* count,
                                           EmitStats* stats, uint32_t only_key, int only_phase, int t0) {
  check_variant(d, v);
  if (v.mode != HEL_SUM || v.prec != PREC_F64 || !(v.order & 4) || (v.order & (8 | 16)))
    throw std::invalid_argument("adjoint kernels take SUM, FP64, local blocks");
  if (d.distributed && v.enum_mask)
    throw std::invalid_argument("adjoint kernels of the distributed graph take one configuration per iteration");
  const Process& pr = d.proc;
  const int LB = popc(v.lane_mask), G = 1 << LB;
  const int nloop = popc(v.loop_mask);
  std::map<uint32_t, std::vector<int>> part;
  std::vector<uint32_t> order;
  {
    Emitter probe(d, v);
    probe.partitions(part, order);
  }
  std::ostringstream all;
  EmitStats tot;
  int t = t0;
  // per-lane LDS of one workgroup at one wave per SIMD (160 KB per CU)
  const int64_t kLdsBytes = 160 * 1024;
  for (uint32_t key : order) {
    if (only_key != ~0u && key != only_key) continue;
    // factored partitions: two kernels (e-_out-side walk, e-_in-side walk)
    bool split = false;
    if (!d.distributed) {
      Emitter pe(d, v);
      std::vector<int> ps = pe.sum_nodes();
      for (size_t a = 0; a < ps.size(); ++a) pe.acc_of_sum[ps[a]] = (int)a;
      pe.collect_block(part[key]);
      split = pe.factor_block(part[key]);
    }
    for (int phase = split ? 1 : 0; phase <= (split ? 2 : 0); ++phase) {
    if (only_phase >= 0 && phase != only_phase) continue;
    // the split walks keep their polarisation gradients in LDS when they fit
    // beside the momentum and propagator gradients
    for (int ge_lds = phase >= 1 ? 1 : 0; ge_lds >= 0; --ge_lds) {
    Emitter e(d, v);
    e.grad_phase = phase;
    e.ge_in_lds = ge_lds != 0;
    e.lds_atomic = phase == 1;
    e.mom_src = 0;       // momenta reloaded per block from the workspace
    e.gm_in_lds = true;  // gradient accumulators in per-lane LDS slots
    e.gq_in_lds = !d.distributed;  // propagator gradients per propagator, flushed once
    std::vector<int> sums = e.sum_nodes();
    for (size_t a = 0; a < sums.size(); ++a) e.acc_of_sum[sums[a]] = (int)a;
    std::ostringstream& os = e.os;
    os << "extern \"C\" __global__ void __launch_bounds__(" << v.block << ")\n" << kprefix << "_" << t
       << "(const double* __restrict__ mom, const double* __restrict__ amp, const double* __restrict__ im2, "
          "long long N, double* __restrict__ gm)\n{\n";
    const int ngm = 4 * (pr.npart - pr.i_eout);
    os << "  __shared__ double qx_gm[" << ngm * v.block << "];\n";
    const std::string gq_mark = "  //@GQ@\n";
    os << gq_mark;
    os << "  const long long gid = (long long)blockIdx.x * " << v.block << " + threadIdx.x;\n";
    os << "  const long long pt = gid >> " << LB << ";\n";
    os << "  const unsigned sub = (unsigned)(gid & " << (G - 1) << ");\n";
    os << "  const long long ptc = pt < N ? pt : N - 1;\n";
    os << "  const long long NL = N * " << G << ";\n  const long long gidc = gid < NL ? gid : NL - 1;\n";
    for (int p = pr.i_eout; p < pr.npart; ++p)
      for (int mu = 0; mu < 4; ++mu) os << "  " << e.gmref(p, mu) << " = 0.0;\n";
    const std::string gq_zero_mark = "  //@GQZERO@\n";
    os << gq_zero_mark;
    os << "  const double iM2 = im2[ptc];\n";
    os << "  const unsigned hrt = " << Emitter::deposit("sub", v.lane_mask) << ";\n";
    // merge: the walked side (phase 1: e-_out, phase 2: e-_in) holds no
    // looped photon
    uint32_t in_side = 0;
    for (int a = 0; a < pr.P; ++a)
      if ((key >> a) & 1) in_side |= 1u << pr.photon_particle[a];
    const uint32_t photons_all = ((1u << pr.npart) - 1) & ~(1u << pr.i_ein) & ~(1u << pr.i_eout);
    const uint32_t walked = phase == 1 ? (photons_all & ~in_side) : phase == 2 ? in_side : photons_all;
    const bool merge = split && nloop > 0 && (v.loop_mask & walked) == 0;
    if (merge) {
      Emitter pm(d, v);
      std::vector<int> ps = pm.sum_nodes();
      for (size_t a = 0; a < ps.size(); ++a) pm.acc_of_sum[ps[a]] = (int)a;
      pm.collect_block(part[key]);
      pm.factor_block(part[key]);
      std::set<uint32_t> pats;
      for (auto& kv : (phase == 1 ? pm.memB : pm.memJ)) pats.insert(kv.second);
      for (uint32_t q : pats)
        os << "  qx::sp4<double> " << (phase == 1 ? "T" : "W") << q << " = qx::zero4<double>();\n";
    }
    os << "  #pragma unroll 1\n  for (unsigned lp = 0; lp < " << (1u << nloop) << "u; ++lp) {\n";
    os << "    const unsigned hc = hrt | " << Emitter::deposit("lp", v.loop_mask) << ";\n";
    e.ind = "    ";
    // seeds: conj(A_h) / |M|^2 of this iteration's configurations, loaded
    // where the block first needs them (after its leaf-sum walk), 8 at a
    // time behind an empty asm that takes all 16 values at once (otherwise,
    // short of registers, the compiler waits for each load before issuing
    // the next)
    {
      std::ostringstream sc;
      const size_t kBatch = 8;
      for (size_t a0 = 0; a0 < sums.size(); a0 += kBatch) {
        const size_t a1 = std::min(sums.size(), a0 + kBatch);
        for (size_t a = a0; a < a1; ++a)
          sc << "const unsigned h" << a << " = hc | " << d.nodes[sums[a]].cfg << "u; double cr" << a << " = amp[(2 * h"
             << a << ") * N + ptc], ci" << a << " = amp[(2 * h" << a << " + 1) * N + ptc];\n";
        sc << "asm volatile(\"\" :";
        for (size_t a = a0; a < a1; ++a) sc << (a > a0 ? ", " : " ") << "\"+v\"(cr" << a << "), \"+v\"(ci" << a << ")";
        sc << ");\n";
        for (size_t a = a0; a < a1; ++a)
          sc << "const qx::cx<double> c" << a << " = {cr" << a << " * iM2, -ci" << a << " * iM2};\n";
      }
      e.seed_code = sc.str();
    }
    if (d.distributed)
      e.dist_adjoint_block(key, part[key]);
    else {
      e.merge_part = merge ? 1 : 0;
      e.grad_block(key, part[key]);
    }
    e.ind = "  ";
    os << "  }\n";
    if (merge) {
      os << "  {\n    const unsigned hc = hrt;\n";
      e.ind = "    ";
      e.merge_part = 2;
      e.grad_block(key, part[key]);
      e.merge_part = 0;
      e.ind = "  ";
      os << "  }\n";
    }
    if (!e.gq_slot.empty()) {
      // propagator gradients of every iteration -> momentum gradients
      os << "  {\n";
      e.ind = "    ";
      e.load_momenta("mom", "N", "ptc");
      e.flush_gq();
      e.ind = "  ";
      os << "  }\n";
    }
    for (int p = pr.i_eout; p < pr.npart; ++p)
      for (int mu = 0; mu < 4; ++mu) {
        os << "  double gm" << p << "_" << mu << " = " << e.gmref(p, mu) << ";\n";
        for (int o = 1; o < G; o <<= 1)
          os << "  gm" << p << "_" << mu << " += __shfl_xor(gm" << p << "_" << mu << ", " << o << ");\n";
      }
    // all loads of gm before any store (the rows may alias for all the
    // compiler knows, which would otherwise serialise each load-add-store)
    os << "  if (pt < N && sub == 0u) {\n";
    for (int p = pr.i_eout; p < pr.npart; ++p)
      for (int mu = 0; mu < 4; ++mu)
        os << "    const double o" << p << "_" << mu << " = gm[" << (4 * p + mu) << " * N + pt];\n";
    for (int p = pr.i_eout; p < pr.npart; ++p)
      for (int mu = 0; mu < 4; ++mu)
        os << "    gm[" << (4 * p + mu) << " * N + pt] = o" << p << "_" << mu << " + gm" << p << "_" << mu << ";\n";
    os << "  }\n}\n";
    const int ns = (int)e.gq_slot.size(), nge = (int)e.ge_slot.size();
    if (ge_lds && (int64_t)(ngm + 5 * ns + 3 * nge) * v.block * 8 > kLdsBytes) continue;  // registers instead
    tot.flops_per_point += e.st.flops_per_point * (double)G * (double)(1 << nloop);
    std::string ks = os.str();
    {
      std::string decl, zero, gezero;
      if (ns > 0) {
        decl = "  __shared__ double qx_gq[" + std::to_string(5 * ns * v.block) + "];\n";
        for (int k = 0; k < ns; ++k)
          for (int c = 0; c < 5; ++c) zero += "  " + e.gqref(k, c) + " = 0.0;\n";
      }
      if (nge > 0) {
        decl += "  __shared__ double qx_ge[" + std::to_string(3 * nge * v.block) + "];\n";
        for (int k = 0; k < nge; ++k)
          for (int c = 0; c < 3; ++c) gezero += "        " + e.geref(k, c) + " = 0.0;\n";
      }
      ks.replace(ks.find(gq_mark), gq_mark.size(), decl);
      ks.replace(ks.find(gq_zero_mark), gq_zero_mark.size(), zero);
      if (e.ge_in_lds) ks.replace(ks.find(e.ge_zero_mark), e.ge_zero_mark.size(), gezero);
    }
    all << ks;
    ++t;
    break;
    }
    }
  }
  if (count) *count = t - t0;
  if (stats) *stats = tot;
  return all.str();
}

std::string emit_body_function(const Dag& d, const Variant& v, const std::string& fname, EmitStats* stats,
                               bool pol_param) {
  check_variant(d, v);
  if (v.order & 16) throw std::invalid_argument("LDS staging is built for eval kernels only");
  Emitter e(d, v);
  std::ostringstream& os = e.os;
  if (v.order & 8) {
    e.slot = true;
    e.pol_lds = pol_param;
    e.slot_tab = fname + "_slots";
    if (v.order & (256 | 512)) {
      setup_cache(e, d, v, fname, 64 / cache_lanes(v), kBodyCacheBytes);
      e.body_mode = true;
      e.pol_lds = true;
    }
    e.emit_slot_table();
  }
  if (v.fixup) {
    if (v.prec != PREC_F32C || v.mode != HEL_PER_POINT)
      throw std::invalid_argument("the FP64 fix-up is built for FP32C per-point bodies");
    e.abs_sum = true;
  }
  os << "static __device__ double " << fname
     << "(const double* __restrict__ mom, long long N, long long ptc, unsigned hrt_in"
     << (e.cur_cache ? ", double* __restrict__ qx_c, int tpt, unsigned sub"
                     : e.pol_lds ? ", " + e.PT + "* __restrict__ qx_pol" : std::string())
     << (v.fixup ? ", int& fixflag, double fix_kappa" : "") << ")\n{\n";
  if (e.cur_cache) {
    const int P = d.proc.P, ncur = e.row_only ? 8 : 16;
    // (3 + ncur) P BP is even (BP is a multiple of 16), so qx_k stays 8-byte aligned
    os << "  " << e.T << "* const qx_pol = (" << e.T << "*)qx_c;\n";
    os << "  " << e.T << "* const qx_cur = qx_pol + " << 3 * P * e.BP << ";\n";
    if (e.k_lds) os << "  double* const qx_k = (double*)(qx_cur + " << ncur * P * e.BP << ");\n";
  }
  if (!e.local() && !e.slot) e.load_momenta("mom", "N", "ptc");
  os << "  double acc = 0.0;\n";
  e.lane_work("hrt_in");
  os << "  return acc;\n}\n";
  e.st.flops_per_point *= (double)lanes_per_point(v) * (double)(1 << popc(v.loop_mask));
  if (stats) *stats = e.st;
  return os.str();
}

}  // namespace qedx
