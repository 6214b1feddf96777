// qedx_dag.cpp -- CDAG generator, node reduction, join expansion, cost model
// and host interpreter for the n-photon Compton amplitude.
#include "qedx_dag.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <map>
#include <random>
#include <set>
#include <tuple>
#include <stdexcept>
#include <unordered_map>

#define QEDX_HD inline
#include "qedx_device.h"

namespace qedx {

const char* kind_name(Kind k) {
  switch (k) {
    case Kind::Entry: return "Entry";
    case Kind::Data: return "Data";
    case Kind::U: return "U";
    case Kind::V: return "V";
    case Kind::S1: return "S1";
    case Kind::S2: return "S2";
    case Kind::Dot: return "Dot";
    case Kind::Sum: return "Sum";
    case Kind::HelSum: return "HelSum";
    case Kind::Add: return "Add";
  }
  return "?";
}

Process Process::make(int n_out, int n_in) {
  Process p;
  p.n_in = n_in;
  p.n_out = n_out;
  p.P = n_in + n_out;
  p.npart = p.P + 2;
  p.i_ein = 0;
  p.i_eout = 1 + n_in;
  for (int j = 0; j < n_in; ++j) {
    p.photon_particle.push_back(1 + j);
    p.photon_sign.push_back(+1);
  }
  for (int j = 0; j < n_out; ++j) {
    p.photon_particle.push_back(2 + n_in + j);
    p.photon_sign.push_back(-1);
  }
  return p;
}

namespace {

int add_node(Dag& d, Node n) {
  int id = (int)d.nodes.size();
  for (int p : n.in) d.nodes[p].out.push_back(id);
  d.nodes.push_back(std::move(n));
  return id;
}

// data node carrying the result of compute node c (copies its attributes)
int add_data(Dag& d, int c) {
  Node n = d.nodes[c];
  n.kind = Kind::Data;
  n.in = {c};
  n.out.clear();
  return add_node(d, std::move(n));
}

int add_compute(Dag& d, Kind k, std::vector<int32_t> in, int8_t side, uint32_t mask, int16_t photon) {
  Node n;
  n.kind = k;
  n.side = side;
  n.mask = mask;
  n.photon = photon;
  for (int p : in) {
    n.cfg |= d.nodes[p].cfg;
    n.cfg_dep |= d.nodes[p].cfg_dep;
  }
  n.in = std::move(in);
  int c = add_node(d, std::move(n));
  return add_data(d, c);
}

}  // namespace

Dag build_unreduced(const Process& proc, uint32_t enum_mask, int split) {
  if (split < 1 || split > proc.P - 1)
    throw std::invalid_argument("split must leave at least one photon on each side");
  Dag d;
  d.proc = proc;
  d.enum_mask = enum_mask;
  d.split = split;
  const int P = proc.P;
  // entries
  std::vector<int> entry(proc.npart);
  for (int i = 0; i < proc.npart; ++i) {
    Node n;
    n.kind = Kind::Entry;
    n.particle = (int16_t)i;
    entry[i] = add_node(d, n);
  }
  // base states, one per particle and spin/polarisation state
  std::vector<std::array<int, 2>> state(proc.npart);
  for (int i = 0; i < proc.npart; ++i) {
    bool en = (enum_mask >> i) & 1;
    for (int h = 0; h < (en ? 2 : 1); ++h) {
      Node n;
      n.kind = Kind::U;
      n.particle = (int16_t)i;
      n.hel = en ? (int8_t)h : (int8_t)-1;
      n.in = {entry[i]};
      if (en) {
        n.cfg_dep = 1u << i;
        n.cfg = (uint32_t)h << i;
      }
      if (i == proc.i_ein) n.side = 0;
      if (i == proc.i_eout) n.side = 1;
      int c = add_node(d, n);
      state[i][h] = add_data(d, c);
    }
  }
  auto st = [&](int particle, uint32_t cfg) {
    bool en = (enum_mask >> particle) & 1;
    return state[particle][en ? ((cfg >> particle) & 1) : 0];
  };
  std::vector<int> perm(P);
  std::vector<int32_t> sums;
  uint32_t cfg = 0;
  while (true) {
    for (int a = 0; a < P; ++a) perm[a] = a;
    std::vector<int32_t> diagrams;
    do {
      // e-_in side: sigma(0) .. sigma(split-1)
      int J = st(proc.i_ein, cfg);
      uint32_t mask = 0;
      for (int t = 0; t < split; ++t) {
        int a = perm[t];
        mask |= 1u << a;
        J = add_compute(d, Kind::V, {st(proc.photon_particle[a], cfg), J}, 0, mask, (int16_t)a);
        if (t < split - 1) J = add_compute(d, Kind::S1, {J}, 0, mask, -1);
      }
      // e-_out side: sigma(P-1) down to sigma(split)
      int Jb = st(proc.i_eout, cfg);
      uint32_t maskb = 0;
      for (int t = 0; t < P - split; ++t) {
        int a = perm[P - 1 - t];
        maskb |= 1u << a;
        Jb = add_compute(d, Kind::V, {st(proc.photon_particle[a], cfg), Jb}, 1, maskb, (int16_t)a);
        if (t < P - split - 1) Jb = add_compute(d, Kind::S1, {Jb}, 1, maskb, -1);
      }
      diagrams.push_back(add_compute(d, Kind::S2, {J, Jb}, -1, 0, -1));
    } while (std::next_permutation(perm.begin(), perm.end()));
    sums.push_back(add_compute(d, Kind::Sum, diagrams, -1, 0, -1));
    if (cfg == enum_mask) break;
    cfg = (cfg - enum_mask) & enum_mask;  // next subset of enum_mask
  }
  if (sums.size() == 1) {
    d.exit = sums[0];
  } else {
    d.exit = add_compute(d, Kind::HelSum, sums, -1, 0, -1);
  }
  return d;
}

// ---------------------------------------------------------------------------
// Node reduction
// ---------------------------------------------------------------------------
namespace {

struct Key {
  Kind kind;
  int8_t side, hel;
  int16_t particle, photon;
  uint32_t mask;
  std::vector<int32_t> in;  // sorted canonical producers
  bool operator==(const Key& o) const {
    return kind == o.kind && side == o.side && hel == o.hel && particle == o.particle && photon == o.photon &&
           mask == o.mask && in == o.in;
  }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    mix((uint64_t)k.kind);
    mix((uint64_t)(uint8_t)k.side);
    mix((uint64_t)(uint8_t)k.hel);
    mix((uint64_t)(uint16_t)k.particle);
    mix((uint64_t)(uint16_t)k.photon);
    mix(k.mask);
    for (int32_t v : k.in) mix((uint64_t)(uint32_t)v);
    return (size_t)h;
  }
};

Key key_of(const Node& n, const std::vector<int32_t>& canon_in) {
  Key k;
  k.kind = n.kind;
  k.side = n.side;
  k.hel = n.hel;
  k.particle = n.particle;
  k.photon = n.photon;
  k.mask = n.mask;
  k.in = canon_in;
  // a compute node's producers form a set (App. C); V keeps its two typed
  // operands, which can never coincide, so sorting loses nothing
  std::sort(k.in.begin(), k.in.end());
  return k;
}

}  // namespace

Dag reduce_fixpoint(const Dag& d) {
  // Nodes are stored producers-first, so one pass in index order sees every
  // producer's representative before its consumers: this is the fixpoint of
  // repeated node reductions (the fixpoint is unique, Sec. III-D).
  Dag r;
  r.proc = d.proc;
  r.enum_mask = d.enum_mask;
  r.split = d.split;
  r.expanded = d.expanded;
  r.join_side = d.join_side;
  r.distributed = d.distributed;
  std::vector<int32_t> rep(d.nodes.size(), -1);
  std::unordered_map<Key, int32_t, KeyHash> seen;
  seen.reserve(d.nodes.size());
  for (size_t i = 0; i < d.nodes.size(); ++i) {
    const Node& n = d.nodes[i];
    std::vector<int32_t> cin;
    cin.reserve(n.in.size());
    for (int p : n.in) cin.push_back(rep[p]);
    Key k = key_of(n, cin);
    auto it = seen.find(k);
    if (it != seen.end()) {
      rep[i] = it->second;
      continue;
    }
    Node m = n;
    m.in = cin;
    m.out.clear();
    int id = add_node(r, std::move(m));
    seen.emplace(std::move(k), id);
    rep[i] = id;
  }
  r.exit = rep[d.exit];
  return r;
}

int64_t reduce_random_order(Dag& d, uint64_t seed) { return reduce_steps(d, seed, -1); }

int64_t reduce_steps(Dag& d, uint64_t seed, int64_t max_steps) {
  std::mt19937_64 rng(seed);
  std::vector<char> alive(d.nodes.size(), 1);
  int64_t steps = 0;
  while (max_steps < 0 || steps < max_steps) {
    std::unordered_map<Key, std::vector<int32_t>, KeyHash> groups;
    for (size_t i = 0; i < d.nodes.size(); ++i) {
      if (!alive[i]) continue;
      groups[key_of(d.nodes[i], d.nodes[i].in)].push_back((int32_t)i);
    }
    std::vector<const std::vector<int32_t>*> cand;
    for (auto& kv : groups)
      if (kv.second.size() >= 2) cand.push_back(&kv.second);
    if (cand.empty()) break;
    std::sort(cand.begin(), cand.end(), [](auto a, auto b) { return (*a)[0] < (*b)[0]; });
    const std::vector<int32_t>& g = *cand[rng() % cand.size()];
    int32_t keep = g[0];
    for (size_t t = 1; t < g.size(); ++t) {
      int32_t gone = g[t];
      for (int32_t c : d.nodes[gone].out) {
        for (auto& p : d.nodes[c].in)
          if (p == gone) p = keep;
        d.nodes[keep].out.push_back(c);
      }
      for (int32_t p : d.nodes[gone].in) {
        auto& o = d.nodes[p].out;
        o.erase(std::remove(o.begin(), o.end(), gone), o.end());
      }
      d.nodes[gone].out.clear();
      alive[gone] = 0;
      if (d.exit == gone) d.exit = keep;
    }
    ++steps;
  }
  d = compact(d);
  return steps;
}

Dag compact(const Dag& d) {
  std::vector<char> live(d.nodes.size(), 0);
  std::vector<int32_t> stack{d.exit};
  live[d.exit] = 1;
  while (!stack.empty()) {
    int v = stack.back();
    stack.pop_back();
    for (int p : d.nodes[v].in)
      if (!live[p]) {
        live[p] = 1;
        stack.push_back(p);
      }
  }
  // topological renumbering (Kahn, smallest old index first for stability)
  std::vector<int> indeg(d.nodes.size(), 0);
  for (size_t i = 0; i < d.nodes.size(); ++i)
    if (live[i]) indeg[i] = (int)d.nodes[i].in.size();
  std::vector<int32_t> order;
  std::vector<int32_t> ready;
  for (size_t i = 0; i < d.nodes.size(); ++i)
    if (live[i] && indeg[i] == 0) ready.push_back((int32_t)i);
  std::make_heap(ready.begin(), ready.end(), std::greater<int32_t>());
  std::vector<std::vector<int32_t>> cons(d.nodes.size());
  for (size_t i = 0; i < d.nodes.size(); ++i)
    if (live[i])
      for (int p : d.nodes[i].in) cons[p].push_back((int32_t)i);
  while (!ready.empty()) {
    std::pop_heap(ready.begin(), ready.end(), std::greater<int32_t>());
    int32_t v = ready.back();
    ready.pop_back();
    order.push_back(v);
    for (int32_t c : cons[v])
      if (--indeg[c] == 0) {
        ready.push_back(c);
        std::push_heap(ready.begin(), ready.end(), std::greater<int32_t>());
      }
  }
  std::vector<int32_t> nid(d.nodes.size(), -1);
  for (size_t t = 0; t < order.size(); ++t) nid[order[t]] = (int32_t)t;
  Dag r;
  r.proc = d.proc;
  r.enum_mask = d.enum_mask;
  r.split = d.split;
  r.expanded = d.expanded;
  r.join_side = d.join_side;
  r.distributed = d.distributed;
  for (int32_t v : order) {
    Node m = d.nodes[v];
    for (auto& p : m.in) p = nid[p];
    m.out.clear();
    add_node(r, std::move(m));
  }
  r.exit = nid[d.exit];
  return r;
}

Dag expand_joins(const Dag& d, int join_side) {
  Dag r;
  r.proc = d.proc;
  r.enum_mask = d.enum_mask;
  r.split = d.split;
  r.expanded = true;
  r.join_side = join_side;
  std::vector<int32_t> nid(d.nodes.size(), -1);
  for (size_t i = 0; i < d.nodes.size(); ++i) {
    const Node& n = d.nodes[i];
    std::vector<int32_t> in;
    for (int p : n.in) in.push_back(nid[p]);
    if (n.kind == Kind::S2) {
      int J = in[0], Jb = in[1];
      if (r.nodes[J].side != 0) std::swap(J, Jb);
      int prop_src = join_side == 1 ? Jb : J;
      const Node& ps = r.nodes[prop_src];
      int s1 = add_compute(r, Kind::S1, {prop_src}, ps.side, ps.mask, -1);
      // the S1's data node is s1; the dot takes it in place of prop_src
      std::vector<int32_t> din = join_side == 1 ? std::vector<int32_t>{J, s1} : std::vector<int32_t>{s1, Jb};
      Node dn;
      dn.kind = Kind::Dot;
      for (int p : din) {
        dn.cfg |= r.nodes[p].cfg;
        dn.cfg_dep |= r.nodes[p].cfg_dep;
      }
      dn.in = din;
      nid[i] = add_node(r, std::move(dn));
      continue;
    }
    Node m = n;
    m.in = in;
    m.out.clear();
    nid[i] = add_node(r, std::move(m));
  }
  r.exit = nid[d.exit];
  return r;
}

// ---------------------------------------------------------------------------
// Distributive rewrite
// ---------------------------------------------------------------------------
namespace {

struct Distributor {
  const Dag& d;
  Dag r;
  std::vector<int32_t> copied;                     // old node -> new node (data nodes and entries)
  std::map<std::vector<int32_t>, int32_t> sums;    // sorted old terms -> new data node

  explicit Distributor(const Dag& d_) : d(d_), copied(d_.nodes.size(), -1) {
    r.proc = d.proc;
    r.enum_mask = d.enum_mask;
    r.split = d.split;
    r.expanded = d.expanded;
    r.join_side = d.join_side;
  r.distributed = d.distributed;
    r.distributed = true;
  }

  // copy an old entry or data node (and what it depends on) unchanged
  int32_t copy(int32_t i) {
    if (copied[i] >= 0) return copied[i];
    const Node& n = d.nodes[i];
    int32_t id;
    if (n.kind == Kind::Entry) {
      Node m = n;
      m.in.clear();
      m.out.clear();
      id = add_node(r, std::move(m));
    } else if (n.kind == Kind::Data) {
      const Node& c = d.nodes[n.in[0]];
      std::vector<int32_t> in;
      for (int p : c.in) in.push_back(copy(p));
      Node m = c;
      m.in = in;
      m.out.clear();
      int32_t cid = add_node(r, std::move(m));
      Node dn = n;
      dn.in = {cid};
      dn.out.clear();
      id = add_node(r, std::move(dn));
    } else {
      throw std::logic_error("distribute: copy() takes entry and data nodes");
    }
    copied[i] = id;
    return id;
  }

  // new data node holding the sum of the old current values `terms`
  int32_t sum_of(std::vector<int32_t> terms) {
    std::sort(terms.begin(), terms.end());
    terms.erase(std::unique(terms.begin(), terms.end()), terms.end());
    if (terms.size() == 1) return copy(terms[0]);
    auto it = sums.find(terms);
    if (it != sums.end()) return it->second;
    // group the terms by their last linear map: vertex with one photon state,
    // or propagator of one (side, photon set); anything else stays a term
    std::map<std::tuple<int, int, int64_t>, std::vector<int32_t>> groups;
    std::vector<std::tuple<int, int, int64_t>> order;
    for (int32_t t : terms) {
      const Node& c = d.nodes[d.nodes[t].in[0]];
      std::tuple<int, int, int64_t> key;
      if (c.kind == Kind::V)
        key = {(int)Kind::V, c.side, (int64_t)c.in[0]};
      else if (c.kind == Kind::S1)
        key = {(int)Kind::S1, c.side, (int64_t)c.mask};
      else
        key = {(int)c.kind, c.side, -1 - (int64_t)t};
      if (!groups.count(key)) order.push_back(key);
      groups[key].push_back(t);
    }
    std::vector<int32_t> parts;
    for (auto& key : order) {
      const std::vector<int32_t>& g = groups[key];
      if (g.size() == 1) {
        parts.push_back(copy(g[0]));
        continue;
      }
      const Node& c0 = d.nodes[d.nodes[g[0]].in[0]];
      std::vector<int32_t> inner;
      for (int32_t t : g) {
        const Node& c = d.nodes[d.nodes[t].in[0]];
        inner.push_back(c.kind == Kind::V ? c.in[1] : c.in[0]);
      }
      int32_t x = sum_of(inner);
      std::vector<int32_t> in = c0.kind == Kind::V ? std::vector<int32_t>{copy(c0.in[0]), x} : std::vector<int32_t>{x};
      parts.push_back(add_compute(r, c0.kind, in, c0.side, c0.mask, c0.photon));
    }
    const Node& t0 = d.nodes[terms[0]];
    int32_t id = parts.size() == 1 ? parts[0] : add_compute(r, Kind::Add, parts, t0.side, t0.mask, -1);
    sums.emplace(terms, id);
    return id;
  }

  int32_t side_op(const Node& dot, int side) const {
    for (int p : dot.in)
      if (d.nodes[p].side == side) return p;
    throw std::logic_error("distribute: Dot without an operand of each side");
  }

  // new data node of a diagram Sum (old data node s)
  int32_t diagram_sum(int32_t s) {
    const Node& sc = d.nodes[d.nodes[s].in[0]];
    // Dots by photon partition (photon set on the e-_in side)
    std::map<uint32_t, std::vector<int32_t>> part;
    for (int p : sc.in) {
      const Node& dot = d.nodes[d.nodes[p].in[0]];
      if (dot.kind != Kind::Dot) throw std::logic_error("distribute: Sum input is not a Dot");
      part[d.nodes[side_op(dot, 0)].mask].push_back(p);
    }
    std::vector<int32_t> terms;
    for (auto& kv : part) {
      std::set<std::pair<int32_t, int32_t>> pairs;
      std::set<int32_t> Js, Bs;
      for (int p : kv.second) {
        const Node& dot = d.nodes[d.nodes[p].in[0]];
        int32_t J = side_op(dot, 0), B = side_op(dot, 1);
        pairs.insert({J, B});
        Js.insert(J);
        Bs.insert(B);
      }
      if (pairs.size() == kv.second.size() && pairs.size() == Js.size() * Bs.size()) {
        int32_t J = sum_of(std::vector<int32_t>(Js.begin(), Js.end()));
        int32_t B = sum_of(std::vector<int32_t>(Bs.begin(), Bs.end()));
        terms.push_back(add_compute(r, Kind::Dot, {J, B}, -1, 0, -1));
      } else {
        for (int p : kv.second) terms.push_back(copy(p));  // not a full product: kept as it is
      }
    }
    return add_compute(r, Kind::Sum, terms, -1, 0, -1);
  }

  void run() {
    const Node& ex = d.nodes[d.exit];
    const Node& top = d.nodes[ex.in[0]];
    if (top.kind == Kind::Sum) {
      r.exit = diagram_sum(d.exit);
    } else if (top.kind == Kind::HelSum) {
      std::vector<int32_t> in;
      for (int p : top.in) in.push_back(diagram_sum(p));
      r.exit = add_compute(r, Kind::HelSum, in, -1, 0, -1);
    } else {
      throw std::logic_error("distribute: exit is not a Sum or HelSum");
    }
  }
};

}  // namespace

Dag distribute(const Dag& d) {
  if (!d.expanded) throw std::invalid_argument("distribute() takes a join-expanded graph");
  Distributor w(d);
  w.run();
  return compact(reduce_fixpoint(w.r));
}

Counts count(const Dag& d) {
  Counts c;
  for (const Node& n : d.nodes) {
    ++c.total;
    if (is_data(n.kind)) {
      ++c.data;
      continue;
    }
    ++c.compute;
    switch (n.kind) {
      case Kind::U: ++c.U; break;
      case Kind::V: ++c.V; break;
      case Kind::S1: ++c.S1; break;
      case Kind::S2: ++c.S2; break;
      case Kind::Dot: ++c.Dot; break;
      case Kind::Sum: ++c.Sum; break;
      case Kind::HelSum: ++c.HelSum; break;
      case Kind::Add: ++c.Add; break;
      default: break;
    }
  }
  return c;
}

std::string canonical(const Dag& d) {
  // Structural hash of every node from its kind, attributes and the hashes of
  // its producers; the sorted list of (hash, #consumers) is numbering-free.
  std::vector<uint64_t> h(d.nodes.size());
  for (size_t i = 0; i < d.nodes.size(); ++i) {
    const Node& n = d.nodes[i];
    std::vector<uint64_t> ph;
    for (int p : n.in) ph.push_back(h[p]);
    std::sort(ph.begin(), ph.end());
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
      x ^= v + 0x9e3779b97f4a7c15ull + (x << 6) + (x >> 2);
      x *= 1099511628211ull;
    };
    mix((uint64_t)n.kind);
    mix((uint64_t)(uint8_t)n.side);
    mix((uint64_t)(uint8_t)n.hel);
    mix((uint64_t)(uint16_t)n.particle);
    mix((uint64_t)(uint16_t)n.photon);
    mix(n.mask);
    for (uint64_t v : ph) mix(v);
    h[i] = x;
  }
  std::vector<std::pair<uint64_t, size_t>> sig;
  for (size_t i = 0; i < d.nodes.size(); ++i) sig.push_back({h[i], d.nodes[i].out.size()});
  std::sort(sig.begin(), sig.end());
  std::string s;
  char buf[48];
  for (auto& p : sig) {
    snprintf(buf, sizeof buf, "%016llx:%zu;", (unsigned long long)p.first, p.second);
    s += buf;
  }
  snprintf(buf, sizeof buf, "exit=%016llx", (unsigned long long)h[d.exit]);
  s += buf;
  return s;
}

// ---------------------------------------------------------------------------
// Cost model (App. B-A).  FLOPs follow the device functions of qedx_device.h.
// ---------------------------------------------------------------------------
static bool photon_state_is_y(const Dag& d, const Node& v) {
  const Node& ph = d.nodes[v.in[0]];
  return ph.hel == 1;
}

double node_flops(const Dag& d, int i, bool fp32) {
  const Node& n = d.nodes[i];
  switch (n.kind) {
    case Kind::Entry:
    case Kind::Data: return 0.0;
    case Kind::U: return 16.0;
    case Kind::V: return photon_state_is_y(d, n) ? 24.0 : 40.0;
    case Kind::S1: return 56.0;
    case Kind::S2: return 56.0 + 30.0;
    case Kind::Dot: return 30.0;
    case Kind::Sum: {
      double k = (double)n.in.size();
      return fp32 ? 14.0 * k : 2.0 * (k - 1.0);
    }
    case Kind::HelSum: return 4.0 * (double)n.in.size() - 1.0;
    case Kind::Add: return 8.0 * ((double)n.in.size() - 1.0);
  }
  return 0.0;
}

static double value_bytes(const Dag& d, const Node& n, bool fp32) {
  double w = fp32 ? 4.0 : 8.0;
  switch (n.kind) {
    case Kind::Entry: return 32.0;
    case Kind::U: {
      bool ph = n.particle != d.proc.i_ein && n.particle != d.proc.i_eout;
      return ph ? 3 * w : 8 * w;
    }
    case Kind::V:
    case Kind::S1:
    case Kind::Add: return 8 * w;
    case Kind::S2:
    case Kind::Dot:
    case Kind::Sum: return 2 * w;
    case Kind::HelSum: return 8.0;
    default: return 0.0;
  }
}

double node_bytes(const Dag& d, int i, bool fp32) {
  const Node& n = d.nodes[i];
  if (n.kind == Kind::Entry) return 32.0;
  if (n.kind != Kind::Data) return 0.0;
  return value_bytes(d, d.nodes[n.in[0]], fp32);
}

// Propagator set-up (K = sum of signed photon momenta, D = +-2p.K + K^2, five
// scaled coefficients) once per distinct (side, photon set).
static const double kPropSetupFlops = 26.0;

double compute_effort(const Dag& d, bool fp32) {
  double c = 0.0;
  std::map<std::pair<int, uint32_t>, int> props;
  for (size_t i = 0; i < d.nodes.size(); ++i) {
    c += node_flops(d, (int)i, fp32);
    const Node& n = d.nodes[i];
    if (n.kind == Kind::S1) props[{n.side, n.mask}] = 1;
    if (n.kind == Kind::S2) props[{1, d.nodes[n.in[1]].mask}] = 1;
  }
  return c + kPropSetupFlops * (double)props.size();
}

// Reverse-mode cost of the same graph (the adjoint sweep of F = log sum |A|^2
// that a gradient adds to the forward evaluation), per node, following the
// vector-Jacobian products of qedx_device.h: V its forward map on the
// adjoint (40 or 24) plus the polarisation gradient 60; S1 56 plus the
// propagator-coefficient gradient 69; external spinor 96, polarisation
// vector 40; 2 per amplitude for its seed conj(A)/|M|^2; 8 per extra
// consumer of a current (adjoint accumulation); 50 per distinct propagator
// set-up (its gradient into the electron momentum and the photon sum).
// Dots: the dots of one amplitude within one photon partition pair every
// row leaf with every column leaf, so their adjoint is taken from the two
// leaf sums: 8 per leaf for the sums and 2 x 32 for the two seeds, in place
// of 2 x 32 per dot.
double adjoint_effort(const Dag& d) {
  double c = 0.0;
  std::map<std::pair<int, uint32_t>, int> props;
  // (column leaf's photon set, amplitude) -> distinct row and column leaves
  std::map<std::pair<uint32_t, int>, std::pair<std::set<int>, std::set<int>>> groups;
  auto prod = [&](int x) { return d.nodes[x].kind == Kind::Data ? d.nodes[x].in[0] : x; };
  for (size_t i = 0; i < d.nodes.size(); ++i) {
    const Node& n = d.nodes[i];
    if (n.kind == Kind::Dot) {
      int a = prod(n.in[0]), b = prod(n.in[1]);
      if (d.nodes[a].side != 0) std::swap(a, b);
      int sum = n.out.empty() ? -1 : d.nodes[n.out[0]].out.empty() ? -1 : d.nodes[n.out[0]].out[0];
      auto& g = groups[{d.nodes[a].mask, sum}];
      g.first.insert(b);
      g.second.insert(a);
    }
    switch (n.kind) {
      case Kind::U: {
        bool ph = n.particle != d.proc.i_ein && n.particle != d.proc.i_eout;
        c += ph ? 40.0 : 96.0;
        break;
      }
      case Kind::V: c += (photon_state_is_y(d, n) ? 24.0 : 40.0) + 60.0; break;
      case Kind::S1: c += 56.0 + 69.0; props[{n.side, n.mask}] = 1; break;
      case Kind::S2: c += 56.0 + 69.0 + 64.0; props[{1, d.nodes[n.in[1]].mask}] = 1; break;
      case Kind::Sum: c += 2.0; break;
      default: break;
    }
    if (n.kind == Kind::Data && !n.in.empty() && n.out.size() > 1) {
      const Node& src = d.nodes[n.in[0]];
      if (src.kind == Kind::V || src.kind == Kind::S1 || src.kind == Kind::Add ||
          (src.kind == Kind::U && (src.particle == d.proc.i_ein || src.particle == d.proc.i_eout)))
        c += 8.0 * (double)(n.out.size() - 1);
    }
  }
  for (auto& g : groups) c += 64.0 + 8.0 * (double)(g.second.first.size() + g.second.second.size());
  return c + 50.0 * (double)props.size();
}

double data_transfer(const Dag& d, bool fp32) {
  double t = 0.0;
  for (size_t i = 0; i < d.nodes.size(); ++i)
    if (is_data(d.nodes[i].kind)) t += node_bytes(d, (int)i, fp32) * (double)d.nodes[i].out.size();
  return t;
}

// ---------------------------------------------------------------------------
// Host interpreter (double precision)
// ---------------------------------------------------------------------------
namespace {
struct Val {
  double m[4];
  qx::sp4<double> j;
  qx::pol3<double> e;
  qx::cx<double> z;
  double r;
};
}  // namespace

static qx::propq<double> prop_for(const Process& pr, const double* mom, int side, uint32_t mask) {
  double K[4] = {0, 0, 0, 0};
  for (int a = 0; a < pr.P; ++a)
    if ((mask >> a) & 1) {
      const double* k = mom + 4 * pr.photon_particle[a];
      for (int mu = 0; mu < 4; ++mu) K[mu] += pr.photon_sign[a] * k[mu];
    }
  const double* p = mom + 4 * (side == 0 ? pr.i_ein : pr.i_eout);
  double pK = p[0] * K[0] - p[1] * K[1] - p[2] * K[2] - p[3] * K[3];
  double KK = K[0] * K[0] - K[1] * K[1] - K[2] * K[2] - K[3] * K[3];
  double s = side == 0 ? 1.0 : -1.0;
  // Q = p + K (left) or p' - K (right); Q^2 - m^2 = +-2 p.K + K^2 exactly
  double Q[4];
  for (int mu = 0; mu < 4; ++mu) Q[mu] = p[mu] + s * K[mu];
  double D = 2.0 * s * pK + KK;
  return qx::prop_coeffs<double>(Q[0], Q[1], Q[2], Q[3], D, 1.0);
}

double interpret(const Dag& d, const double* mom, uint32_t runtime_hel) {
  const Process& pr = d.proc;
  std::vector<Val> v(d.nodes.size());
  for (size_t i = 0; i < d.nodes.size(); ++i) {
    const Node& n = d.nodes[i];
    Val& o = v[i];
    switch (n.kind) {
      case Kind::Entry:
        for (int mu = 0; mu < 4; ++mu) o.m[mu] = mom[4 * n.particle + mu];
        break;
      case Kind::Data: o = v[n.in[0]]; break;
      case Kind::U: {
        const double* p = v[n.in[0]].m;
        int h = n.hel >= 0 ? n.hel : (int)((runtime_hel >> n.particle) & 1);
        if (n.particle == pr.i_ein)
          o.j = qx::u_in<double>(p[0], p[1], p[2], p[3], h, 1.0);
        else if (n.particle == pr.i_eout)
          o.j = qx::ubar_out<double>(p[0], p[1], p[2], p[3], h, 1.0);
        else
          o.e = qx::pol<double>(p[1], p[2], p[3], h);
        break;
      }
      case Kind::V: {
        const qx::pol3<double>& e = v[n.in[0]].e;
        const qx::sp4<double>& J = v[n.in[1]].j;
        o.j = n.side == 0 ? qx::vL<double>(J, e) : qx::vR<double>(J, e);
        break;
      }
      case Kind::S1: {
        qx::propq<double> q = prop_for(pr, mom, n.side, n.mask);
        const qx::sp4<double>& J = v[n.in[0]].j;
        o.j = n.side == 0 ? qx::sL<double>(J, q) : qx::sR<double>(J, q);
        break;
      }
      case Kind::S2: {
        const Node& a = d.nodes[n.in[0]];
        int iJ = a.side == 0 ? n.in[0] : n.in[1];
        int iB = a.side == 0 ? n.in[1] : n.in[0];
        qx::propq<double> q = prop_for(pr, mom, 1, d.nodes[iB].mask);
        o.z = qx::dot<double>(qx::sR<double>(v[iB].j, q), v[iJ].j);
        break;
      }
      case Kind::Dot: {
        const Node& a = d.nodes[n.in[0]];
        int iJ = a.side == 0 ? n.in[0] : n.in[1];
        int iB = a.side == 0 ? n.in[1] : n.in[0];
        o.z = qx::dot<double>(v[iB].j, v[iJ].j);
        break;
      }
      case Kind::Sum: {
        o.z = {0.0, 0.0};
        for (int p : n.in) {
          o.z.r += v[p].z.r;
          o.z.i += v[p].z.i;
        }
        break;
      }
      case Kind::HelSum: {
        o.r = 0.0;
        for (int p : n.in) o.r += v[p].z.r * v[p].z.r + v[p].z.i * v[p].z.i;
        break;
      }
      case Kind::Add: {
        o.j = qx::zero4<double>();
        for (int p : n.in) qx::add_to(o.j, v[p].j);
        break;
      }
    }
  }
  const Node& ex = d.nodes[d.exit];
  const Node& pr_ex = d.nodes[ex.kind == Kind::Data ? ex.in[0] : d.exit];
  const Val& r = v[d.exit];
  if (pr_ex.kind == Kind::HelSum) return r.r;
  return r.z.r * r.z.r + r.z.i * r.z.i;
}

double interpret_grad(const Dag& d, const double* mom, uint32_t runtime_hel, double* gmom) {
  const Process& pr = d.proc;
  const size_t Nn = d.nodes.size();
  std::vector<Val> v(Nn);
  // forward (same as interpret)
  for (size_t i = 0; i < Nn; ++i) {
    const Node& n = d.nodes[i];
    Val& o = v[i];
    switch (n.kind) {
      case Kind::Entry:
        for (int mu = 0; mu < 4; ++mu) o.m[mu] = mom[4 * n.particle + mu];
        break;
      case Kind::Data: o = v[n.in[0]]; break;
      case Kind::U: {
        const double* p = v[n.in[0]].m;
        int h = n.hel >= 0 ? n.hel : (int)((runtime_hel >> n.particle) & 1);
        if (n.particle == pr.i_ein)
          o.j = qx::u_in<double>(p[0], p[1], p[2], p[3], h, 1.0);
        else if (n.particle == pr.i_eout)
          o.j = qx::ubar_out<double>(p[0], p[1], p[2], p[3], h, 1.0);
        else
          o.e = qx::pol<double>(p[1], p[2], p[3], h);
        break;
      }
      case Kind::V: {
        const qx::pol3<double>& e = v[n.in[0]].e;
        const qx::sp4<double>& J = v[n.in[1]].j;
        o.j = n.side == 0 ? qx::vL<double>(J, e) : qx::vR<double>(J, e);
        break;
      }
      case Kind::S1: {
        qx::propq<double> q = prop_for(pr, mom, n.side, n.mask);
        o.j = n.side == 0 ? qx::sL<double>(v[n.in[0]].j, q) : qx::sR<double>(v[n.in[0]].j, q);
        break;
      }
      case Kind::S2:
      case Kind::Dot: {
        const Node& a = d.nodes[n.in[0]];
        int iJ = a.side == 0 ? n.in[0] : n.in[1];
        int iB = a.side == 0 ? n.in[1] : n.in[0];
        qx::sp4<double> B = v[iB].j;
        if (n.kind == Kind::S2) B = qx::sR<double>(B, prop_for(pr, mom, 1, d.nodes[iB].mask));
        o.z = qx::dot<double>(B, v[iJ].j);
        break;
      }
      case Kind::Sum:
        o.z = {0.0, 0.0};
        for (int p : n.in) {
          o.z.r += v[p].z.r;
          o.z.i += v[p].z.i;
        }
        break;
      case Kind::HelSum:
        o.r = 0.0;
        for (int p : n.in) o.r += v[p].z.r * v[p].z.r + v[p].z.i * v[p].z.i;
        break;
      case Kind::Add:
        o.j = qx::zero4<double>();
        for (int p : n.in) qx::add_to(o.j, v[p].j);
        break;
    }
  }
  double M2 = 0.0;
  for (size_t i = 0; i < Nn; ++i)
    if (d.nodes[i].kind == Kind::Sum) M2 += v[i].z.r * v[i].z.r + v[i].z.i * v[i].z.i;
  // reverse
  struct Adj {
    qx::sp4<double> w;
    qx::cx<double> z;
    qx::pol3<double> ge;
  };
  std::vector<Adj> a(Nn);
  for (auto& x : a) {
    x.w = qx::zero4<double>();
    x.z = {0.0, 0.0};
    x.ge = {0.0, 0.0, 0.0};
  }
  for (int k = 0; k < 4 * pr.npart; ++k) gmom[k] = 0.0;
  auto fixed = [&](int particle) { return particle == pr.i_ein || particle == 1; };
  auto add_prop_grad = [&](int side, uint32_t mask, const qx::propq<double>& gq) {
    double K[4] = {0, 0, 0, 0};
    for (int b = 0; b < pr.P; ++b)
      if ((mask >> b) & 1) {
        const double* kk = mom + 4 * pr.photon_particle[b];
        for (int mu = 0; mu < 4; ++mu) K[mu] += pr.photon_sign[b] * kk[mu];
      }
    int pe = side == 0 ? pr.i_ein : pr.i_eout;
    const double* p = mom + 4 * pe;
    double gp[4] = {0, 0, 0, 0}, gK[4] = {0, 0, 0, 0};
    qx::prop_from_vjp(p[0], p[1], p[2], p[3], K[0], K[1], K[2], K[3], side == 0 ? 1.0 : -1.0, 1.0, gq, gp, gK);
    if (!fixed(pe))
      for (int mu = 0; mu < 4; ++mu) gmom[4 * pe + mu] += gp[mu];
    for (int b = 0; b < pr.P; ++b)
      if ((mask >> b) & 1) {
        int part = pr.photon_particle[b];
        if (!(pr.photon_sign[b] > 0 && part == 1))
          for (int mu = 0; mu < 4; ++mu) gmom[4 * part + mu] += pr.photon_sign[b] * gK[mu];
      }
  };
  for (size_t ii = Nn; ii-- > 0;) {
    const Node& n = d.nodes[ii];
    Adj& w = a[ii];
    switch (n.kind) {
      case Kind::HelSum:
        break;
      case Kind::Add:
        for (int p : n.in) qx::add_to(a[p].w, w.w);
        break;
      case Kind::Sum: {
        qx::cx<double> c = {v[ii].z.r / M2, -v[ii].z.i / M2};
        for (int p : n.in) {
          a[p].z.r += c.r;
          a[p].z.i += c.i;
        }
        break;
      }
      case Kind::Data: {
        int p = n.in[0];
        qx::add_to(a[p].w, w.w);
        a[p].z.r += w.z.r;
        a[p].z.i += w.z.i;
        a[p].ge.e1 += w.ge.e1;
        a[p].ge.e2 += w.ge.e2;
        a[p].ge.e3 += w.ge.e3;
        break;
      }
      case Kind::S2:
      case Kind::Dot: {
        const Node& an = d.nodes[n.in[0]];
        int iJ = an.side == 0 ? n.in[0] : n.in[1];
        int iB = an.side == 0 ? n.in[1] : n.in[0];
        qx::sp4<double> B = v[iB].j;
        qx::propq<double> q{};
        if (n.kind == Kind::S2) {
          q = prop_for(pr, mom, 1, d.nodes[iB].mask);
          B = qx::sR<double>(B, q);
        }
        qx::sp4<double> wB = qx::zero4<double>();
        qx::dot_vjp(w.z, B, v[iJ].j, wB, a[iJ].w);
        if (n.kind == Kind::S2) {
          qx::add_to(a[iB].w, qx::sL<double>(wB, q));
          qx::propq<double> gq = {0, 0, 0, 0, 0};
          qx::sR_gq(wB, v[iB].j, gq);
          add_prop_grad(1, d.nodes[iB].mask, gq);
        } else {
          qx::add_to(a[iB].w, wB);
        }
        break;
      }
      case Kind::S1: {
        qx::propq<double> q = prop_for(pr, mom, n.side, n.mask);
        qx::propq<double> gq = {0, 0, 0, 0, 0};
        const qx::sp4<double>& J = v[n.in[0]].j;
        if (n.side == 0) {
          qx::add_to(a[n.in[0]].w, qx::sR<double>(w.w, q));
          qx::sL_gq(w.w, J, gq);
        } else {
          qx::add_to(a[n.in[0]].w, qx::sL<double>(w.w, q));
          qx::sR_gq(w.w, J, gq);
        }
        add_prop_grad(n.side, n.mask, gq);
        break;
      }
      case Kind::V: {
        const qx::pol3<double>& e = v[n.in[0]].e;
        const qx::sp4<double>& J = v[n.in[1]].j;
        qx::pol3<double>& ge = a[n.in[0]].ge;
        if (n.side == 0) {
          qx::add_to(a[n.in[1]].w, qx::vR<double>(w.w, e));
          qx::vL_ge(w.w, J, ge);
        } else {
          qx::add_to(a[n.in[1]].w, qx::vL<double>(w.w, e));
          qx::vR_ge(w.w, J, ge);
        }
        break;
      }
      case Kind::U: {
        int part = n.particle;
        if (fixed(part)) break;
        const double* p = v[n.in[0]].m;
        int h = n.hel >= 0 ? n.hel : (int)((runtime_hel >> n.particle) & 1);
        if (part == pr.i_eout) {
          double g[4];
          qx::ubar_vjp(p[0], p[1], p[2], p[3], h, 1.0, w.w, g);
          for (int mu = 0; mu < 4; ++mu) gmom[4 * part + mu] += g[mu];
        } else {
          double g[3];
          qx::pol_vjp(p[1], p[2], p[3], h, w.ge, g);
          for (int mu = 0; mu < 3; ++mu) gmom[4 * part + 1 + mu] += g[mu];
        }
        break;
      }
      default: break;
    }
  }
  return log(M2);
}

}  // namespace qedx
