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
  return o.str();
}

Dag graph_for(const Process& proc, const Variant& v, double* t_build, double* t_reduce) {
  using clk = std::chrono::steady_clock;
  auto t0 = clk::now();
  Dag d = build_unreduced(proc, v.enum_mask, v.split);
  auto t1 = clk::now();
  Dag r = reduce_fixpoint(d);
  r = reduce_fixpoint(expand_joins(r, v.join_side));
  r = compact(r);
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

  Emitter(const Dag& d_, const Variant& v_) : d(d_), v(v_), pr(d_.proc), done(d_.nodes.size(), 0) {
    T = v.prec == PREC_F64 ? "double" : "float";
  }

  int producer(int i) const {
    const Node& n = d.nodes[i];
    return n.kind == Kind::Data ? n.in[0] : i;
  }
  std::string name(int i) const { return "n" + std::to_string(producer(i)); }

  void emitK(uint32_t mask) {
    if (kdone.count(mask)) return;
    int lo = __builtin_ctz(mask);
    uint32_t rest = mask & (mask - 1);
    std::string km = "K" + std::to_string(mask);
    if (rest == 0) {
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
    st.flops_per_point += 28;
    ++st.n_prop;
    qdone.insert({side, mask});
  }

  std::string hel_expr(const Node& u) const {
    if (u.hel >= 0) return std::to_string((int)u.hel);
    return "(int)((hc >> " + std::to_string(u.particle) + ") & 1u)";
  }

  bool local() const { return (v.order & 4) != 0; }

  // scheduling fence: keeps LLVM's machine scheduler from moving work across
  void fence(int level) {
    if (v.order & level) os << ind << "__builtin_amdgcn_sched_barrier(0);\n";
  }

  void emit(int i) {
    int c = producer(i);
    if (done[c]) return;
    const Node& n = d.nodes[c];
    for (int p : n.in) emit(p);
    std::string nm = "n" + std::to_string(c);
    switch (n.kind) {
      case Kind::Entry: break;
      case Kind::U: {
        int p = n.particle;
        std::string m = "m" + std::to_string(p) + "_";
        if (p == pr.i_ein)
          os << ind << "const qx::sp4<" << T << "> " << nm << " = qx::u_in<" << T << ">(" << m << "0, " << m << "1, "
             << m << "2, " << m << "3, " << hel_expr(n) << ", 1.0);\n";
        else if (p == pr.i_eout)
          os << ind << "const qx::sp4<" << T << "> " << nm << " = qx::ubar_out<" << T << ">(" << m << "0, " << m
             << "1, " << m << "2, " << m << "3, " << hel_expr(n) << ", 1.0);\n";
        else
          os << ind << "const qx::pol3<" << T << "> " << nm << " = qx::pol<" << T << ">(" << m << "1, " << m << "2, "
             << m << "3, " << hel_expr(n) << ");\n";
        st.flops_per_point += 16;
        ++st.n_U;
        break;
      }
      case Kind::V: {
        const Node& ph = d.nodes[producer(n.in[0])];
        bool y = ph.hel == 1;
        os << ind << "const qx::sp4<" << T << "> " << nm << " = qx::v" << (n.side == 0 ? "L" : "R")
           << (y ? "_y" : "") << "<" << T << ">(" << name(n.in[1]) << ", " << name(n.in[0]) << ");\n";
        st.flops_per_point += y ? 24 : 40;
        ++st.n_V;
        break;
      }
      case Kind::S1: {
        emitQ(n.side, n.mask);
        os << ind << "const qx::sp4<" << T << "> " << nm << " = qx::s" << (n.side == 0 ? "L" : "R") << "<" << T
           << ">(" << name(n.in[0]) << ", " << qname(n.side, n.mask) << ");\n";
        st.flops_per_point += 56;
        ++st.n_S1;
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
    if (v.prec == PREC_F64) {
      os << ind << "qx::dot_acc<double>(A" << acc << ", " << name(ops.second) << ", " << name(ops.first) << ");\n";
      st.flops_per_point += 32;
    } else {
      os << ind << "qx::comp_acc<float>(A" << acc << ", C" << acc << ", qx::dot<float>(" << name(ops.second) << ", "
         << name(ops.first) << "));\n";
      st.flops_per_point += 30 + 14;
    }
    ++st.n_dot;
    fence(2);
  }

  // Body: accumulators, all nodes in partition-grouped order, |A|^2 sums
  // added into the double `acc` of the enclosing scope.
  void body() {
    std::vector<int> sums, dots;
    for (size_t i = 0; i < d.nodes.size(); ++i) {
      if (d.nodes[i].kind == Kind::Sum) sums.push_back((int)i);
      if (d.nodes[i].kind == Kind::Dot) dots.push_back((int)i);
    }
    for (size_t a = 0; a < sums.size(); ++a) {
      acc_of_sum[sums[a]] = (int)a;
      os << ind << "qx::cx<" << T << "> A" << a << " = {" << T << "(0), " << T << "(0)};\n";
      if (v.prec != PREC_F64) os << ind << "qx::cx<float> C" << a << " = {0.0f, 0.0f};\n";
    }
    // group dots by the photon set on the e-_in side
    std::map<uint32_t, std::vector<int>> part;
    for (int k : dots) {
      auto ops = dot_ops(d.nodes[k]);
      part[d.nodes[producer(ops.first)].mask].push_back(k);
    }
    // order partitions greedily by overlap with the previous one
    std::vector<uint32_t> keys;
    for (auto& kv : part) keys.push_back(kv.first);
    std::vector<uint32_t> order;
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
    for (uint32_t key : order) {
      std::vector<int>& dk = part[key];
      std::set<int> Bs, Js;
      for (int k : dk) {
        auto ops = dot_ops(d.nodes[k]);
        Js.insert(producer(ops.first));
        Bs.insert(producer(ops.second));
      }
      bool holdB = Bs.size() <= Js.size();
      const std::set<int>& hold = holdB ? Bs : Js;
      const std::set<int>& stream = holdB ? Js : Bs;
      fence(1);
      os << ind << "// photons " << key << " | " << (((1u << pr.P) - 1) & ~key) << " on the e-_in | e-_out side\n";
      std::string outer = ind;
      if (local()) {
        // Partition-local block: momenta reloaded through an index the
        // compiler cannot see through, so nothing computed here is merged
        // with (and kept live from) another partition's block.
        // A uniform branch on an opaque flag puts the block in its own basic
        // block, so instruction selection schedules it on its own.
        os << ind << "{\n" << ind << "  int live = 1;\n" << ind << "  asm volatile(\"\" : \"+s\"(live));\n"
           << ind << "  if (live) {\n";
        ind += "    ";
        os << ind << "long long pq = ptc;\n" << ind << "asm volatile(\"\" : \"+v\"(pq));\n";
        load_momenta("mom", "N", "pq");
        std::fill(done.begin(), done.end(), 0);
        kdone.clear();
        qdone.clear();
      }
      for (int h : hold) emit(h);
      for (int s : stream) {
        emit(s);
        for (int k : dk) {
          auto ops = dot_ops(d.nodes[k]);
          int sp = producer(holdB ? ops.first : ops.second);
          if (sp == s) emit_dot(k);
        }
      }
      if (local()) {
        ind = outer;
        os << ind << "  }\n" << ind << "}\n";
      }
    }
    // |A|^2, summed over the enumerated configurations (HelSum) or single
    for (size_t a = 0; a < sums.size(); ++a) {
      if (v.prec == PREC_F64) {
        os << ind << "acc += A" << a << ".r * A" << a << ".r + A" << a << ".i * A" << a << ".i;\n";
      } else {
        os << ind << "{ const double ar = (double)A" << a << ".r + (double)C" << a << ".r, ai = (double)A" << a
           << ".i + (double)C" << a << ".i; acc += ar * ar + ai * ai; }\n";
      }
      st.flops_per_point += 4;
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
  if (v.block % 64 != 0 || v.block < 64 || v.block > 1024) throw std::invalid_argument("bad block size");
}

}  // namespace

std::string emit_eval_kernel(const Dag& d, const Variant& v, const std::string& kname, EmitStats* stats) {
  check_variant(d, v);
  Emitter e(d, v);
  const int LB = popc(v.lane_mask);
  const int G = 1 << LB;
  std::ostringstream& os = e.os;
  os << "// generated by qedx: " << variant_tag(v, d.proc.n_out, d.proc.n_in) << "\n";
  os << "#include <hip/hip_runtime.h>\n";
  os << device_header_text() << "\n";
  os << "extern \"C\" __global__ void __launch_bounds__(" << v.block;
  if (v.min_waves > 0) os << ", " << v.min_waves;
  os << ")\n" << kname
     << "(const double* __restrict__ mom, const unsigned* __restrict__ hel, long long N, double* __restrict__ out)\n{\n";
  os << "  const long long gid = (long long)blockIdx.x * " << v.block << " + threadIdx.x;\n";
  os << "  const long long pt = gid >> " << LB << ";\n";
  os << "  const unsigned sub = (unsigned)(gid & " << (G - 1) << ");\n";
  os << "  const long long ptc = pt < N ? pt : N - 1;\n";
  if (!e.local()) e.load_momenta("mom", "N", "ptc");
  os << "  double acc = 0.0;\n";
  std::string hrt = v.mode == HEL_PER_POINT ? "hel[ptc]" : Emitter::deposit("sub", v.lane_mask);
  e.lane_work(hrt);
  for (int o = 1; o < G; o <<= 1) os << "  acc += __shfl_xor(acc, " << o << ");\n";
  os << "  if (pt < N && sub == 0u) out[pt] = acc;\n}\n";
  // per point: every lane of the group does the body once per loop iteration
  e.st.flops_per_point *= (double)G * (double)(1 << popc(v.loop_mask));
  std::string src = os.str();
  e.st.lines = std::count(src.begin(), src.end(), '\n');
  if (stats) *stats = e.st;
  return src;
}

std::string emit_body_function(const Dag& d, const Variant& v, const std::string& fname, EmitStats* stats) {
  check_variant(d, v);
  Emitter e(d, v);
  std::ostringstream& os = e.os;
  os << "static __device__ double " << fname
     << "(const double* __restrict__ mom, long long N, long long ptc, unsigned hrt_in)\n{\n";
  if (!e.local()) e.load_momenta("mom", "N", "ptc");
  os << "  double acc = 0.0;\n";
  e.lane_work("hrt_in");
  os << "  return acc;\n}\n";
  e.st.flops_per_point *= (double)(1 << popc(v.lane_mask)) * (double)(1 << popc(v.loop_mask));
  if (stats) *stats = e.st;
  return os.str();
}

}  // namespace qedx
