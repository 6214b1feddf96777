// qedx_runtime.cpp -- the C ABI of include/qedx.h: process creation (graph
// build, node reduction, code generation, code-object cache, module load),
// launches, and the host-side graph tools.
#include <dlfcn.h>
#include <fcntl.h>
#include <signal.h>
#include <hip/hip_runtime_api.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/qedx.h"
#include "../../include/qedx_tools.h"
#include "qedx_dag.hpp"
#include "qedx_emit.hpp"
#include "qedx_internal.hpp"
#include "qedx_scratch.hpp"
#include "qedx_kernels.hpp"

extern char** environ;

using namespace qedx;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static qed_status fail(qed_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

extern "C" const char* qed_last_error(void) { return g_err.c_str(); }

#define HIPCHK(expr)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return fail(QED_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// cache directory and compiler
// ---------------------------------------------------------------------------
static std::string lib_dir() {
  Dl_info info;
  if (dladdr((void*)&qed_last_error, &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    auto s = p.rfind('/');
    if (s != std::string::npos) return p.substr(0, s);
  }
  return ".";
}

static std::string& cache_dir_str() {
  static std::string dir = [] {
    const char* e = getenv("QEDX_CACHE_DIR");
    std::string d = e && *e ? std::string(e) : lib_dir() + "/kcache";
    mkdir(d.c_str(), 0755);
    return d;
  }();
  return dir;
}

extern "C" const char* qed_cache_dir(void) { return cache_dir_str().c_str(); }

static uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

static std::string hex64(uint64_t v) {
  char b[20];
  snprintf(b, sizeof b, "%016llx", (unsigned long long)v);
  return b;
}

static const char* kArch = "gfx950";

static std::vector<std::string> compile_flags() {
  std::vector<std::string> f = {"--offload-arch=gfx950",
                                "-O3",
                                "--genco",
                                "-std=c++17",
                                "-ffp-contract=fast",
                                "-Xclang",
                                "-target-feature",
                                "-Xclang",
                                "-packed-fp32-ops",
                                "-Rpass-analysis=kernel-resource-usage"};
  if (const char* x = getenv("QEDX_EXTRA_FLAGS")) {
    std::istringstream is(x);
    std::string t;
    while (is >> t) f.push_back(t);
  }
  return f;
}

static std::string hipcc_path() {
  const char* r = getenv("ROCM_PATH");
  std::string base = r && *r ? r : "/opt/rocm";
  return base + "/bin/hipcc";
}

static bool read_file(const std::string& path, std::string& out) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  std::ostringstream ss;
  ss << f.rdbuf();
  out = ss.str();
  return true;
}

static bool write_file(const std::string& path, const std::string& data) {
  std::string tmp = path + ".tmp" + std::to_string(getpid()) + "_" +
                    std::to_string(std::hash<std::thread::id>()(std::this_thread::get_id()));
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return false;
    f.write(data.data(), (std::streamsize)data.size());
    if (!f) return false;
  }
  return rename(tmp.c_str(), path.c_str()) == 0;
}

// Run hipcc as a child process (never replaces this process).
static int run_hipcc(const std::string& src, const std::string& out, const std::string& log, double timeout_s) {
  std::vector<std::string> args = {hipcc_path()};
  for (auto& f : compile_flags()) args.push_back(f);
  args.push_back(src);
  args.push_back("-o");
  args.push_back(out);
  std::vector<char*> argv;
  for (auto& a : args) argv.push_back((char*)a.c_str());
  argv.push_back(nullptr);
  posix_spawn_file_actions_t fa;
  posix_spawn_file_actions_init(&fa);
  posix_spawn_file_actions_addopen(&fa, 1, log.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
  posix_spawn_file_actions_adddup2(&fa, 1, 2);
  pid_t pid;
  int rc = posix_spawn(&pid, argv[0], &fa, nullptr, argv.data(), environ);
  posix_spawn_file_actions_destroy(&fa);
  if (rc != 0) return -1000 - rc;
  auto t0 = std::chrono::steady_clock::now();
  int status = 0;
  while (true) {
    pid_t w = waitpid(pid, &status, WNOHANG);
    if (w == pid) break;
    if (w < 0) return -2000;
    double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (el > timeout_s) {
      kill(pid, SIGKILL);
      waitpid(pid, &status, 0);
      return -3000;
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(20));
  }
  return WIFEXITED(status) ? WEXITSTATUS(status) : -4000;
}


static KernelMeta parse_meta(const std::string& log) {
  KernelMeta m;
  auto grab = [&](const char* key, int& v) {
    auto p = log.find(key);
    if (p != std::string::npos) v = atoi(log.c_str() + p + strlen(key));
  };
  grab(" VGPRs: ", m.vgpr);
  grab(" AGPRs: ", m.agpr);
  grab(" SGPRs: ", m.sgpr);
  grab("ScratchSize [bytes/lane]: ", m.scratch);
  grab("LDS Size [bytes/block]: ", m.lds);
  grab("Occupancy [waves/SIMD]: ", m.occupancy);
  return m;
}

// Compile (or find) the code object for a generated source.  Thread-safe.
// Returns the code object bytes; *hit = cache hit; *ms = compile time.
static std::mutex g_cache_mu;

static qed_status get_code_object(const std::string& tag, const std::string& src, std::string& co,
                                  KernelMeta& meta, bool& hit, double& ms) {
  std::string key_material = src;
  for (auto& f : compile_flags()) key_material += "\n" + f;
  key_material += std::string("\n") + kArch;
  std::string h = hex64(fnv1a(key_material.data(), key_material.size()));
  std::string base = cache_dir_str() + "/" + tag + "-" + h;
  std::string path = base + ".hsaco", sum = base + ".sum", log = base + ".log";
  hit = false;
  ms = 0;
  {
    std::string s, chk;
    if (read_file(path, co) && read_file(sum, chk) && chk == hex64(fnv1a(co.data(), co.size()))) {
      std::string lg;
      read_file(log, lg);
      meta = parse_meta(lg);
      meta.hash = h;
      hit = true;
      return QED_OK;
    }
  }
  std::string srcp = base + ".hip";
  if (!write_file(srcp, src)) return fail(QED_ERR_COMPILE, "cannot write " + srcp);
  if (getenv("QEDX_NO_COMPILE"))
    return fail(QED_ERR_COMPILE, "code object " + path + " missing or corrupt and QEDX_NO_COMPILE is set (source in " +
                                     srcp + ")");
  std::string tmpo = base + ".o.tmp" + std::to_string(getpid()) + "_" +
                     std::to_string(std::hash<std::thread::id>()(std::this_thread::get_id()));
  std::string tmpl = log + ".tmp" + std::to_string(getpid()) + "_" +
                     std::to_string(std::hash<std::thread::id>()(std::this_thread::get_id()));
  double tmo = 3600.0;
  if (const char* t = getenv("QEDX_COMPILE_TIMEOUT")) tmo = atof(t);
  auto t0 = std::chrono::steady_clock::now();
  int rc = run_hipcc(srcp, tmpo, tmpl, tmo);
  ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  std::string lg;
  read_file(tmpl, lg);
  if (rc != 0 || !read_file(tmpo, co) || co.empty()) {
    unlink(tmpo.c_str());
    unlink(tmpl.c_str());
    return fail(QED_ERR_COMPILE, "hipcc failed (rc " + std::to_string(rc) + ") for " + srcp + ":\n" +
                                     lg.substr(0, 4000));
  }
  std::lock_guard<std::mutex> lk(g_cache_mu);
  rename(tmpl.c_str(), log.c_str());
  rename(tmpo.c_str(), path.c_str());
  write_file(sum, hex64(fnv1a(co.data(), co.size())));
  meta = parse_meta(lg);
  meta.hash = h;
  return QED_OK;
}

// ---------------------------------------------------------------------------
// processes
// ---------------------------------------------------------------------------

static void default_variant(int n, int nin, qed_hel_mode mode, qed_precision prec, int rewrite, Variant& v) {
  v = Variant();
  v.prec = prec == QED_FP64 ? PREC_F64 : PREC_F32C;
  v.mode = mode == QED_HEL_SUM ? HEL_SUM : HEL_PER_POINT;
  const int P = n + nin, npart = P + 2, i_eout = 1 + nin;
  // photons on the e-_in side of every join: half; one more for per-point
  // kernels with an odd photon count >= 5, whose partition loop then
  // recomputes fewer currents (measured: 8 % faster at 5 photons, 6 % at 7)
  v.split = (mode == QED_HEL_PER_POINT && P >= 5) ? (P + 1) / 2 : P / 2;
  v.block = 256;
  v.join_side = 1;
  // P <= 4 photons: one shared graph per lane (few partitions, registers
  // suffice).  P >= 5: per photon partition, its currents recomputed
  // (bounded live set): helicity sums use one basic block per partition;
  // per-point kernels a run-time loop over the partitions around one
  // canonical block (compact code, seconds to compile even at P = 7).
  v.order = P >= 5 ? (mode == QED_HEL_PER_POINT ? 8 : 4) : 0;
  // One configuration per point, FP64, node-reduced, 5..7 photons: the
  // partition loop with the one-photon current cache (each photon's
  // one-photon currents computed once per point into LDS, the partitions
  // split between the lanes of a point).  Measured on 2^20 points (2^18 at
  // 7 photons) against the loop without it: 5 photons, 2 lanes, the e-_in
  // side cached (170 VGPRs, 77 KB LDS: two waves per SIMD) 0.445 against
  // 0.548 ms (both sides cached: 0.512 ms, one wave per SIMD; 4 lanes:
  // 0.63-0.74 ms); 6 photons, 4 lanes, both sides (218 VGPRs, two waves per
  // SIMD) 1.53 against 1.82 ms (2 lanes 1.62; e-_in side only 1.67);
  // 7 photons, 4 lanes, both sides 2.02 against 2.19 ms (2 lanes 2.12).
  // FP32C (currents and polarisations cached rounded to FP32, computed in
  // FP64 as the first steps are), same shapes: 0.444 against 0.554 ms, 1.46
  // against 1.86 ms, 2.22 against 2.93 ms
  v.min_waves = 0;
  if (mode == QED_HEL_PER_POINT && !rewrite && P >= 5 && P <= 7) {
    v.order = P == 5 ? (8 | 256 | 1024) : (8 | 512);
    v.min_waves = P == 5 || (P == 6 && prec == QED_FP64) ? 2 : 0;
  }
  if (mode == QED_HEL_SUM) {
    uint32_t all = (1u << npart) - 1;
    // electron spins over lanes; photon polarisations shared in the graph
    // for few photons, partly looped for more
    v.lane_mask = (1u << 0) | (1u << i_eout);
    uint32_t photons = all & ~v.lane_mask;
    if (P == 4 && prec == QED_FP64 && !rewrite) {
      // 4 photons, node-reduced FP64: only the e-_out spin over lanes (2 per
      // point), everything else in the graph, one basic block per partition:
      // no scratch (202 AGPRs instead of 256 + 360 B spill) and 6 % faster
      // than 4 spin lanes with one shared block; FP32C and the distributive
      // rewrite keep the shared block, where it measured faster
      v.lane_mask = 1u << i_eout;
      v.enum_mask = all & ~v.lane_mask;
      // the two lanes share the e-_in side (each builds it for one e-_in
      // spin): 1.73 against 1.79 ms on 2^20 points; and the e-_in side's
      // one-photon currents are computed once per point into LDS (131 KB per
      // workgroup, 160 AGPRs instead of 198): 1.63 against 1.73 ms (at five
      // photons the same cache measured slower, 5.21 against 5.12 ms)
      v.order = 4 | 2048 | 4096;
    } else if (P <= 4) {
      v.enum_mask = photons;
    } else {
      // keep 2^3 photon configurations inside the graph, loop over the rest;
      // with 5 photons in FP64 (node-reduced) the e-_in spin also moves into
      // the graph and only the e-_out spin stays on lanes (27 % faster)
      if (P == 5 && prec == QED_FP64 && !rewrite) {
        v.lane_mask = 1u << i_eout;
        photons = all & ~v.lane_mask & ~1u;
        // shared e-_in side: 5.16 against 5.23 ms on 2^18 points; each
        // block's momentum loads issued together: 5.09 against 5.14 ms (at
        // 4 photons the same measured slower, 1.65 against 1.62 ms)
        v.order |= 2048 | 8192;
      }
      uint32_t e = (v.lane_mask & 1u) ? 0u : 1u;
      int k = 0;
      for (int b = 0; b < npart && k < 3; ++b)
        if ((photons >> b) & 1) {
          e |= 1u << b;
          ++k;
        }
      v.enum_mask = e;
      v.loop_mask = photons & ~e;
    }
  }
}

static const double kFixKappa = 16.0;

static qed_status make_variant_shape(int n, int nin, qed_hel_mode mode, qed_precision prec, const qed_variant* qv,
                                     Variant& v);

// Kernel shape plus the FP64 fix-up flag of FP32C per-point kernels.
static qed_status make_variant(int n, int nin, qed_hel_mode mode, qed_precision prec, const qed_variant* qv,
                               Variant& v, double* fix_kappa = nullptr) {
  qed_status s = make_variant_shape(n, nin, mode, prec, qv, v);
  if (s) return s;
  bool custom = qv && !qv->use_defaults;
  v.fixup = (prec == QED_FP32C && mode == QED_HEL_PER_POINT && !(v.order & 16) && !v.partial &&
             !(custom && qv->fixup < 0))
                ? 1
                : 0;
  double k = custom && qv->fix_kappa != 0.0f ? (double)qv->fix_kappa : kFixKappa;
  if (!(k >= 1.0) || !std::isfinite(k)) return fail(QED_ERR_INVALID_ARG, "fix_kappa must be >= 1");
  if (fix_kappa) *fix_kappa = k;
  return QED_OK;
}

static qed_status make_variant_shape(int n, int nin, qed_hel_mode mode, qed_precision prec, const qed_variant* qv,
                                     Variant& v) {
  default_variant(n, nin, mode, prec, qv && !qv->use_defaults ? qv->rewrite : 0, v);
  const int P = n + nin, npart = P + 2;
  if (qv && !qv->use_defaults) {
    if (qv->block) v.block = qv->block;
    if (qv->split) v.split = qv->split;
    if (qv->order) {
      // an explicit schedule drops the default's occupancy hint (made for the
      // default schedule) unless one is given
      v.order = qv->order;
      v.min_waves = 0;
    }
    if (qv->min_waves) v.min_waves = qv->min_waves;
    if (qv->rewrite < 0 || qv->rewrite > 1) return fail(QED_ERR_INVALID_ARG, "rewrite must be 0 or 1");
    v.rewrite = qv->rewrite;
    if (qv->partial) {
      // partially reduced graph of the paper's form: whole graph in one
      // straight-line block (the partition loop assumes identical partitions)
      if (v.rewrite) return fail(QED_ERR_INVALID_ARG, "partial reduction excludes the rewrite");
      if (qv->partial_steps < 0) return fail(QED_ERR_INVALID_ARG, "partial_steps must be >= 0");
      v.partial = 1;
      v.partial_steps = qv->partial_steps;
      v.partial_seed = qv->partial_seed;
      v.order = 0;
      v.min_waves = qv->min_waves;
      if (!qv->split) v.split = P / 2;  // the join position of the Table I graphs
    }
    if (mode == QED_HEL_SUM && (qv->lane_bits || qv->loop_bits)) {
      // both zero keeps the default helicity coverage
      uint32_t all = (1u << npart) - 1;
      v.lane_mask = qv->lane_bits & all;
      v.loop_mask = qv->loop_bits & all & ~v.lane_mask;
      v.enum_mask = all & ~v.lane_mask & ~v.loop_mask;
      // an explicit coverage with at most 4 photons keeps the shared block
      // unless an order is given (the 4-photon default above pairs its own
      // coverage with per-partition blocks)
      if (!qv->order && P <= 4) v.order = 0;
    } else if (mode != QED_HEL_SUM && (qv->lane_bits || qv->loop_bits)) {
      return fail(QED_ERR_INVALID_ARG, "lane_bits/loop_bits apply to SUM mode only");
    }
  }
  // FP32C with one photon on the e-_in side of every join: the join's
  // propagator goes onto that side, where it follows the first vertex and is
  // evaluated in FP64 with it (the product next to the external electron can
  // cancel; see the emitter's first-step currents)
  v.join_side = (v.prec == PREC_F32C && v.split == 1) ? 0 : 1;
  if (v.block % 64 || v.block < 64 || v.block > 1024) return fail(QED_ERR_INVALID_ARG, "block must be 64..1024, multiple of 64");
  if (v.split < 1 || v.split > P - 1) return fail(QED_ERR_INVALID_ARG, "split must be in 1..(photons - 1)");
  if (__builtin_popcount(v.lane_mask) > 6) return fail(QED_ERR_INVALID_ARG, "at most 6 lane bits");
  return QED_OK;
}

// Symbol of the eval kernel: one name per (process, mode, precision, rewrite),
// so profiles tell the kernels of different processes apart.
static std::string eval_kernel_name(int n, int nin, qed_hel_mode mode, qed_precision prec, const Variant& v) {
  std::string k = "qedx_eval_" + (nin != 1 ? "i" + std::to_string(nin) : std::string()) + "n" + std::to_string(n) +
                  (mode == QED_HEL_SUM ? "_sum" : "_pp") + (prec == QED_FP64 ? "_fp64" : "_fp32c");
  if (v.rewrite) k += "_d" + std::to_string(v.rewrite);
  if (v.partial) k += "_k" + std::to_string(v.partial_steps);
  if (v.order & 128) k += "_mfma";
  return k;
}

// The auxiliary module (RAMBO, gradient) depends on the process, mode and
// precision only, not on the eval kernel's shape: one cache entry per process.
static std::string aux_tag(int n, qed_hel_mode mode, qed_precision prec, int rewrite) {
  return "aux_n" + std::to_string(n) + (mode == QED_HEL_SUM ? "_sum" : "_pp") + (prec == QED_FP64 ? "_fp64" : "_fp32c") +
         (rewrite ? "_d" + std::to_string(rewrite) : "");
}

static qed_status build_source(int n, int nin, qed_hel_mode mode, qed_precision prec, const qed_variant* qv,
                               Variant& v, Process& proc, std::string& src, qed_info& info) {
  if (n < 1 || nin < 1 || n + nin > 7) return fail(QED_ERR_UNSUPPORTED, "need n_out >= 1, n_in >= 1, n_in + n_out <= 7");
  if (mode != QED_HEL_SUM && mode != QED_HEL_PER_POINT) return fail(QED_ERR_INVALID_ARG, "bad helicity mode");
  if (prec != QED_FP64 && prec != QED_FP32C) return fail(QED_ERR_INVALID_ARG, "bad precision");
  double fk = 0;
  qed_status s = make_variant(n, nin, mode, prec, qv, v, &fk);
  if (s) return s;
  info.fixup = v.fixup;
  info.fix_kappa = v.fixup ? fk : 0.0;
  proc = Process::make(n, nin);
  try {
    double tb = 0, tr = 0;
    Dag un = build_unreduced(proc, v.enum_mask, v.split);
    info.nodes_unreduced = (int64_t)un.nodes.size();
    un = Dag();
    Dag d = graph_for(proc, v, &tb, &tr);
    info.create_ms_build = tb;
    info.create_ms_reduce = tr;
    info.nodes_reduced = (int64_t)d.nodes.size();
    auto t0 = std::chrono::steady_clock::now();
    EmitStats st;
    src = emit_eval_kernel(d, v, eval_kernel_name(n, nin, mode, prec, v), &st);
    info.create_ms_emit = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info.n_V = st.n_V;
    info.n_S1 = st.n_S1;
    info.n_dot = st.n_dot;
    info.n_prop = st.n_prop;
    info.flops_per_point = st.flops_per_point;
  } catch (const std::exception& e) {
    return fail(QED_ERR_INVALID_ARG, std::string("graph/emit: ") + e.what());
  }
  info.n = n;
  info.mode = mode;
  info.precision = prec;
  info.lanes_per_point = lanes_per_point(v);
  info.block = v.block;
  std::string tag = variant_tag(v, n, nin);
  snprintf(info.kernel_tag, sizeof info.kernel_tag, "%s", tag.c_str());
  snprintf(info.kernel_name, sizeof info.kernel_name, "%s", eval_kernel_name(n, nin, mode, prec, v).c_str());
  info.n_in = nin;
  return QED_OK;
}

extern "C" qed_status qed_emit_source(int n, qed_hel_mode mode, qed_precision prec, const qed_variant* variant,
                                      char* buf, int64_t buflen, int64_t* len) {
  Variant v;
  Process proc;
  std::string src;
  qed_info info{};
  qed_status s = build_source(n, 1, mode, prec, variant, v, proc, src, info);
  if (s) return s;
  if (len) *len = (int64_t)src.size();
  if (buf && buflen > 0) {
    size_t m = std::min<size_t>((size_t)buflen - 1, src.size());
    memcpy(buf, src.data(), m);
    buf[m] = 0;
  }
  return QED_OK;
}

// Emit + compile into the cache without touching the GPU (used to prebuild).
static qed_status prebuild(int nin, int n, qed_hel_mode mode, qed_precision prec, const qed_variant* variant,
                           int with_aux, double* compile_ms) {
  Variant v;
  Process proc;
  std::string src;
  qed_info info{};
  qed_status s = build_source(n, nin, mode, prec, variant, v, proc, src, info);
  if (s) return s;
  std::string co;
  KernelMeta meta;
  bool hit;
  double ms = 0, ms2 = 0;
  s = get_code_object(info.kernel_tag, src, co, meta, hit, ms);
  if (s) return s;
  if (with_aux && nin == 1) {
    std::string asrc;
    try {
      asrc = emit_aux_module(proc, v, n, nullptr);
    } catch (const std::exception& e) {
      return fail(QED_ERR_INVALID_ARG, std::string("aux emit: ") + e.what());
    }
    std::string atag = aux_tag(n, mode, prec, v.rewrite);
    s = get_code_object(atag, asrc, co, meta, hit, ms2);
    if (s) return s;
  }
  if (compile_ms) *compile_ms = ms + ms2;
  return QED_OK;
}

extern "C" qed_status qed_prebuild(int n, qed_hel_mode mode, qed_precision prec, const qed_variant* variant,
                                   int with_aux, double* compile_ms) {
  return prebuild(1, n, mode, prec, variant, with_aux, compile_ms);
}

extern "C" qed_status qed_prebuild_crossed(int n_in, int n_out, qed_hel_mode mode, qed_precision prec,
                                           const qed_variant* variant, double* compile_ms) {
  return prebuild(n_in, n_out, mode, prec, variant, 0, compile_ms);
}

static qed_status process_create(int nin, int n, qed_hel_mode mode, qed_precision prec, const qed_variant* variant,
                                 qed_process** out) {
  if (!out) return fail(QED_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  auto p = std::make_unique<qed_process>();
  qed_status s = build_source(n, nin, mode, prec, variant, p->var, p->proc, p->eval_src, p->info);
  if (s) return s;
  p->n = n;
  p->n_in = nin;
  p->mode = mode;
  p->prec = prec;
  p->lanes = p->info.lanes_per_point;
  std::string co;
  KernelMeta meta;
  bool hit = false;
  double ms = 0;
  s = get_code_object(p->info.kernel_tag, p->eval_src, co, meta, hit, ms);
  if (s) return s;
  p->info.create_ms_compile = ms;
  p->info.cache_hit = hit ? 1 : 0;
  p->info.vgpr = meta.vgpr;
  p->info.agpr = meta.agpr;
  p->info.sgpr = meta.sgpr;
  p->info.scratch_bytes = meta.scratch;
  p->info.lds_bytes = meta.lds;
  snprintf(p->info.code_hash, sizeof p->info.code_hash, "%s", meta.hash.c_str());
  auto t0 = std::chrono::steady_clock::now();
  HIPCHK(hipModuleLoadData(&p->mod, co.data()));
  HIPCHK(hipModuleGetFunction(&p->f_eval, p->mod, p->info.kernel_name));
  if (p->var.fixup) {
    std::string fx = std::string(p->info.kernel_name) + "_fix";
    HIPCHK(hipModuleGetFunction(&p->f_fix, p->mod, fx.c_str()));
  }
  if (nin != 1) {  // RAMBO and the gradient are built for one incoming photon
    p->info.create_ms_load = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = p.release();
    return QED_OK;
  }
  // auxiliary module: RAMBO (all processes) and the gradient kernel
  std::string asrc;
  try {
    AuxInfo ai;
    asrc = emit_aux_module(p->proc, p->var, n, &ai);
    p->grad_lanes = ai.grad_lanes;
    p->grad_block = ai.grad_block ? ai.grad_block : 256;
    p->grad_split = ai.split;
    p->amp_lanes = ai.amp_lanes;
    p->adj_lanes = ai.adj_lanes;
    p->f_gadj.assign(ai.n_adj, nullptr);
  } catch (const std::exception& e) {
    return fail(QED_ERR_INVALID_ARG, std::string("aux emit: ") + e.what());
  }
  std::string aco;
  KernelMeta am;
  bool ahit;
  double ams;
  s = get_code_object(aux_tag(n, mode, prec, p->var.rewrite), asrc, aco, am, ahit, ams);
  if (s) return s;
  p->info.create_ms_compile += ams;
  HIPCHK(hipModuleLoadData(&p->mod_aux, aco.data()));
  const std::string ns = std::to_string(n);
  HIPCHK(hipModuleGetFunction(&p->f_rambo, p->mod_aux, ("qedx_rambo_n" + ns).c_str()));
  if (hipModuleGetFunction(&p->f_grad, p->mod_aux, ("qedx_grad_n" + ns).c_str()) != hipSuccess) p->f_grad = nullptr;
  if (p->grad_split) {
    HIPCHK(hipModuleGetFunction(&p->f_grambo, p->mod_aux, ("qedx_grambo_n" + ns).c_str()));
    HIPCHK(hipModuleGetFunction(&p->f_gamp, p->mod_aux, ("qedx_gamp_n" + ns).c_str()));
    HIPCHK(hipModuleGetFunction(&p->f_grvjp, p->mod_aux, ("qedx_grvjp_n" + ns).c_str()));
    for (size_t t = 0; t < p->f_gadj.size(); ++t)
      HIPCHK(hipModuleGetFunction(&p->f_gadj[t], p->mod_aux, ("qedx_gadj_n" + ns + "_" + std::to_string(t)).c_str()));
  }
  (void)hipGetLastError();
  p->info.create_ms_load = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = p.release();
  return QED_OK;
}

extern "C" qed_status qed_process_create(int n, qed_hel_mode mode, qed_precision prec, const qed_variant* variant,
                                         qed_process** out) {
  return process_create(1, n, mode, prec, variant, out);
}

extern "C" qed_status qed_process_create_crossed(int n_in, int n_out, qed_hel_mode mode, qed_precision prec,
                                                 const qed_variant* variant, qed_process** out) {
  return process_create(n_in, n_out, mode, prec, variant, out);
}

extern "C" qed_status qed_process_destroy(qed_process* p) {
  delete p;  // unloads its modules
  return QED_OK;
}

extern "C" qed_status qed_process_info(const qed_process* p, qed_info* out) {
  if (!p || !out) return fail(QED_ERR_INVALID_ARG, "NULL argument");
  *out = p->info;
  return QED_OK;
}

static qed_status launch(hipFunction_t f, int64_t threads, int block, void* stream, void** args) {
  int64_t grid = (threads + block - 1) / block;
  if (grid > 0x7fffffff) return fail(QED_ERR_INVALID_ARG, "N too large for one launch");
  HIPCHK(hipModuleLaunchKernel(f, (unsigned)grid, 1, 1, (unsigned)block, 1, 1, 0, (hipStream_t)stream, args,
                               nullptr));
  return QED_OK;
}

extern "C" qed_status qed_eval(const qed_process* p, const double* momenta, const uint32_t* hel, int64_t N,
                               double* out, void* stream) {
  if (!p) return fail(QED_ERR_INVALID_ARG, "process is NULL");
  if (N < 0) return fail(QED_ERR_INVALID_ARG, "N < 0");
  if (p->mode == QED_HEL_SUM && hel) return fail(QED_ERR_INVALID_ARG, "hel must be NULL in SUM mode");
  if (N == 0) return QED_OK;
  if (!momenta || !out) return fail(QED_ERR_INVALID_ARG, "NULL buffer");
  if (p->mode == QED_HEL_PER_POINT && !hel) return fail(QED_ERR_INVALID_ARG, "hel required in PER_POINT mode");
  if (N > (int64_t)1 << 40) return fail(QED_ERR_INVALID_ARG, "N too large");
  long long n = (long long)N;
  if (!p->f_fix) {
    void* args[] = {(void*)&momenta, (void*)&hel, (void*)&n, (void*)&out};
    return launch(p->f_eval, N * (int64_t)p->lanes, p->var.block, stream, args);
  }
  // FP32C pass, which marks the points it cannot resolve with a negative
  // value in `out`, then the FP64 pass over those marks (one workgroup per
  // kFixRange points); no memory beyond the caller's buffers
  double kappa = p->info.fix_kappa;
  void* args[] = {(void*)&momenta, (void*)&hel, (void*)&n, (void*)&out, (void*)&kappa};
  qed_status s = launch(p->f_eval, N * (int64_t)p->lanes, p->var.block, stream, args);
  if (s) return s;
  void* fargs[] = {(void*)&momenta, (void*)&hel, (void*)&n, (void*)&out};
  const int64_t fix_groups = (N + kFixRange - 1) / kFixRange;
  return launch(p->f_fix, fix_groups * 256, 256, stream, fargs);
}

extern "C" qed_status qed_rambo(const qed_process* p, const double* uniforms, double sqrt_s, int64_t N,
                                double* momenta_out, void* stream) {
  if (!p) return fail(QED_ERR_INVALID_ARG, "process is NULL");
  if (!p->f_rambo) return fail(QED_ERR_UNSUPPORTED, "RAMBO is built for one incoming photon");
  if (N < 0) return fail(QED_ERR_INVALID_ARG, "N < 0");
  if (!(sqrt_s > 1.0) || !std::isfinite(sqrt_s)) return fail(QED_ERR_INVALID_ARG, "sqrt_s must exceed m = 1");
  if (N == 0) return QED_OK;
  if (!uniforms || !momenta_out) return fail(QED_ERR_INVALID_ARG, "NULL buffer");
  long long n = (long long)N;
  void* args[] = {(void*)&uniforms, (void*)&sqrt_s, (void*)&n, (void*)&momenta_out};
  return launch(p->f_rambo, N, 256, stream, args);
}

// Split gradient: bytes of workspace per point (momenta and momentum
// gradient [4 npart] each, amplitudes [2 H], 1/|M|^2) and the largest chunk
// of points one pass takes (a power of two, at most 2^20 and 512 MB).
static int64_t grad_ws_per_point(const qed_process* p) {
  const int npart = p->n + p->n_in + 2;
  const int64_t H = (int64_t)1 << npart;
  return 8 * (2 * 4 * (int64_t)npart + 2 * H + 1);
}

static int64_t grad_max_chunk(const qed_process* p) {
  int64_t C = (int64_t)1 << 20;
  while (C > 256 && C * grad_ws_per_point(p) > ((int64_t)512 << 20)) C >>= 1;
  return C;
}

extern "C" qed_status qed_eval_grad_workspace_size(const qed_process* p, int64_t N, int64_t* bytes) {
  if (!p || !bytes) return fail(QED_ERR_INVALID_ARG, "NULL argument");
  if (N < 0) return fail(QED_ERR_INVALID_ARG, "N < 0");
  *bytes = p->grad_split ? grad_ws_per_point(p) * std::min<int64_t>(N, grad_max_chunk(p)) : 0;
  return QED_OK;
}

// The split gradient over chunks of C points through a workspace of
// C * grad_ws_per_point bytes (any device memory of that size: the caller's
// workspace, or the allocation-free entry point's static buffer).
static qed_status grad_split_chunks(const qed_process* p, const double* uniforms, double sqrt_s, int64_t N,
                                    double* out_logm2, double* out_grad, double* ws, int64_t C, void* stream) {
  const int npart = p->n + p->n_in + 2;
  const int64_t H = (int64_t)1 << npart;
  for (int64_t off = 0; off < N; off += C) {
    long long cnt = (long long)std::min<int64_t>(C, N - off);
    long long ldu = (long long)N;
    double* mom = ws;
    double* gm = mom + 4 * (int64_t)npart * cnt;
    double* amp = gm + 4 * (int64_t)npart * cnt;
    double* im2 = amp + 2 * H * cnt;
    const double* u = uniforms + off;
    double* lg = out_logm2 + off;
    double* gr = out_grad + off;
    qed_status st;
    void* a1[] = {(void*)&u, (void*)&ldu, (void*)&sqrt_s, (void*)&cnt, (void*)&mom, (void*)&gm};
    if ((st = launch(p->f_grambo, cnt, 256, stream, a1))) return st;
    void* a2[] = {(void*)&mom, (void*)&cnt, (void*)&amp, (void*)&lg, (void*)&im2};
    if ((st = launch(p->f_gamp, cnt * (int64_t)p->amp_lanes, 256, stream, a2))) return st;
    for (hipFunction_t f : p->f_gadj) {
      void* a3[] = {(void*)&mom, (void*)&amp, (void*)&im2, (void*)&cnt, (void*)&gm};
      if ((st = launch(f, cnt * (int64_t)p->adj_lanes, 256, stream, a3))) return st;
    }
    void* a4[] = {(void*)&u, (void*)&ldu, (void*)&sqrt_s, (void*)&cnt, (void*)&gm, (void*)&gr, (void*)&ldu};
    if ((st = launch(p->f_grvjp, cnt, 256, stream, a4))) return st;
  }
  return QED_OK;
}

static qed_status grad_check(const qed_process* p, const double* uniforms, double sqrt_s, const uint32_t* hel,
                             int64_t N, double* out_logm2, double* out_grad) {
  if (!p) return fail(QED_ERR_INVALID_ARG, "process is NULL");
  if (p->mode != QED_HEL_SUM || p->prec != QED_FP64 || p->n_in != 1)
    return fail(QED_ERR_UNSUPPORTED, "gradient is built for SUM-mode FP64 processes with one incoming photon");
  if (!p->f_grad && !p->grad_split) return fail(QED_ERR_UNSUPPORTED, "no gradient kernel for this process (n > 4)");
  if (hel) return fail(QED_ERR_INVALID_ARG, "hel must be NULL");
  if (N < 0) return fail(QED_ERR_INVALID_ARG, "N < 0");
  if (!(sqrt_s > 1.0) || !std::isfinite(sqrt_s)) return fail(QED_ERR_INVALID_ARG, "sqrt_s must exceed m = 1");
  if (N > 0 && (!uniforms || !out_logm2 || !out_grad)) return fail(QED_ERR_INVALID_ARG, "NULL buffer");
  if (N > (int64_t)1 << 40) return fail(QED_ERR_INVALID_ARG, "N too large");
  return QED_OK;
}

extern "C" qed_status qed_eval_grad(const qed_process* p, const double* uniforms, double sqrt_s,
                                    const uint32_t* hel, int64_t N, double* out_logm2, double* out_grad,
                                    void* workspace, int64_t workspace_bytes, void* stream) {
  qed_status s = grad_check(p, uniforms, sqrt_s, hel, N, out_logm2, out_grad);
  if (s || N == 0) return s;
  if (!p->grad_split) return qedx_rt::grad_fused(p, uniforms, sqrt_s, N, out_logm2, out_grad, stream);
  const int64_t per_pt = grad_ws_per_point(p);
  const int64_t need_min = per_pt * std::min<int64_t>(N, 64);
  if (!workspace || workspace_bytes < need_min)
    return fail(QED_ERR_INVALID_ARG, "workspace of at least " + std::to_string(need_min) +
                                         " bytes required (qed_eval_grad_workspace_size gives the full size)");
  if ((uintptr_t)workspace % 8) return fail(QED_ERR_INVALID_ARG, "workspace must be 8-byte aligned");
  const int64_t C = std::min(N, std::min(workspace_bytes / per_pt, grad_max_chunk(p)));
  return grad_split_chunks(p, uniforms, sqrt_s, N, out_logm2, out_grad, (double*)workspace, C, stream);
}

// The same gradient with the library's fixed per-device scratch in place of
// the caller's workspace: no allocation, no synchronisation.  The scratch
// bounds the chunk of points per pass, not N.
extern "C" qed_status qed_eval_grad_noalloc(const qed_process* p, const double* uniforms, double sqrt_s,
                                            const uint32_t* hel, int64_t N, double* out_logm2, double* out_grad,
                                            void* stream) {
  qed_status s = grad_check(p, uniforms, sqrt_s, hel, N, out_logm2, out_grad);
  if (s || N == 0) return s;
  if (!p->grad_split) return qedx_rt::grad_fused(p, uniforms, sqrt_s, N, out_logm2, out_grad, stream);
  const int64_t per_pt = grad_ws_per_point(p);
  if (per_pt * 64 > qedx_rt::kScratchBytes)
    return fail(QED_ERR_UNSUPPORTED, "a 64-point chunk of this process needs " + std::to_string(per_pt * 64) +
                                         " bytes, more than the " + std::to_string(qedx_rt::kScratchBytes) +
                                         "-byte scratch");
  void* ws = nullptr;
  hipError_t e = qedx_rt::scratch_address(&ws);
  if (e != hipSuccess) return fail(QED_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  const int64_t C = std::min(N, std::min(qedx_rt::kScratchBytes / per_pt, grad_max_chunk(p)));
  return grad_split_chunks(p, uniforms, sqrt_s, N, out_logm2, out_grad, (double*)ws, C, stream);
}

// ---------------------------------------------------------------------------
// host graph tools
// ---------------------------------------------------------------------------
static Dag tool_graph(int n, int n_in, uint32_t enum_mask, int split, int reduced) {
  Process pr = Process::make(n, n_in);
  Dag d = build_unreduced(pr, enum_mask, split);
  if (reduced) {
    d = reduce_fixpoint(d);
    d = compact(reduce_fixpoint(expand_joins(d, 1)));
  }
  if (reduced == 2) d = distribute(d);
  return d;
}

static qed_status check_tool_args(int n, int n_in, uint32_t enum_mask, int split) {
  if (n < 1 || n_in < 1 || n + n_in > 9) return fail(QED_ERR_INVALID_ARG, "need n >= 1, n_in >= 1, n + n_in <= 9");
  if (split < 1 || split >= n + n_in) return fail(QED_ERR_INVALID_ARG, "split must be in 1..P-1");
  if (enum_mask >> (n + n_in + 2)) return fail(QED_ERR_INVALID_ARG, "enum_mask has bits beyond the particles");
  return QED_OK;
}

extern "C" qed_status qed_graph_counts(int n, int n_in, uint32_t enum_mask, int split, int reduced,
                                       int64_t* counts) {
  if (!counts) return fail(QED_ERR_INVALID_ARG, "counts is NULL");
  qed_status s = check_tool_args(n, n_in, enum_mask, split);
  if (s) return s;
  try {
    Dag d = tool_graph(n, n_in, enum_mask, split, reduced);
    Counts c = count(d);
    int64_t v[10] = {c.total, c.data, c.compute, c.U, c.V, c.S1, c.S2, c.Dot, c.Sum, c.HelSum};
    memcpy(counts, v, sizeof v);
  } catch (const std::bad_alloc&) {
    return fail(QED_ERR_OOM, "graph too large");
  }
  return QED_OK;
}

extern "C" qed_status qed_graph_interpret(int n, int n_in, uint32_t enum_mask, int split, int reduced,
                                          const double* mom, const uint32_t* hel, int64_t N, double* out) {
  qed_status s = check_tool_args(n, n_in, enum_mask, split);
  if (s) return s;
  if (N < 0 || (N > 0 && (!mom || !out))) return fail(QED_ERR_INVALID_ARG, "bad buffers");
  Dag d = tool_graph(n, n_in, enum_mask, split, reduced);
  int np = n + n_in + 2;
  for (int64_t i = 0; i < N; ++i) out[i] = interpret(d, mom + 4 * np * i, hel ? hel[i] : 0u);
  return QED_OK;
}

extern "C" qed_status qed_graph_partial(int n, int split, int64_t steps, uint64_t seed, const double* mom,
                                        const uint32_t* hel, int64_t N, double* out, int64_t* counts) {
  qed_status s = check_tool_args(n, 1, 0, split);
  if (s) return s;
  if (steps < 0 || N < 0 || (N > 0 && (!mom || !out))) return fail(QED_ERR_INVALID_ARG, "bad arguments");
  Process pr = Process::make(n, 1);
  Dag d = build_unreduced(pr, 0, split);
  reduce_steps(d, seed, steps);
  if (counts) {
    Counts c = count(d);
    int64_t v[10] = {c.total, c.data, c.compute, c.U, c.V, c.S1, c.S2, c.Dot, c.Sum, c.HelSum};
    memcpy(counts, v, sizeof v);
  }
  for (int64_t i = 0; i < N; ++i) out[i] = interpret(d, mom + 4 * pr.npart * i, hel ? hel[i] : 0u);
  return QED_OK;
}

extern "C" qed_status qed_graph_reduction_check(int n, int n_in, uint32_t enum_mask, int split, uint64_t seed,
                                                char* canon_a, char* canon_b, int64_t buflen, int64_t* steps) {
  qed_status s = check_tool_args(n, n_in, enum_mask, split);
  if (s) return s;
  Process pr = Process::make(n, n_in);
  Dag u = build_unreduced(pr, enum_mask, split);
  Dag a = compact(reduce_fixpoint(u));
  Dag b = u;
  int64_t k = reduce_random_order(b, seed);
  if (steps) *steps = k;
  std::string ca = canonical(a), cb = canonical(b);
  auto put = [&](char* dst, const std::string& src) {
    if (!dst || buflen <= 0) return;
    size_t m = std::min<size_t>((size_t)buflen - 1, src.size());
    memcpy(dst, src.data(), m);
    dst[m] = 0;
  };
  put(canon_a, ca);
  put(canon_b, cb);
  return QED_OK;
}

extern "C" qed_status qed_graph_metrics(int n, int n_in, uint32_t enum_mask, int split, int reduced, int fp32,
                                        double* c_dag, double* d_dag) {
  qed_status s = check_tool_args(n, n_in, enum_mask, split);
  if (s) return s;
  Dag d = tool_graph(n, n_in, enum_mask, split, reduced);
  if (c_dag) *c_dag = compute_effort(d, fp32 != 0);
  if (d_dag) *d_dag = data_transfer(d, fp32 != 0);
  return QED_OK;
}

extern "C" qed_status qed_graph_adjoint_metrics(int n, uint32_t enum_mask, int split, int reduced, double* c_fwd,
                                                double* c_adj) {
  qed_status s = check_tool_args(n, 1, enum_mask, split);
  if (s) return s;
  Dag d = tool_graph(n, 1, enum_mask, split, reduced);
  if (c_fwd) *c_fwd = compute_effort(d, false);
  if (c_adj) *c_adj = adjoint_effort(d);
  return QED_OK;
}

// ---------------------------------------------------------------------------
// mixed-process batches (persistent kernel) -- see qedx_batch.cpp
// ---------------------------------------------------------------------------

namespace qedx_rt {
qed_status fail(qed_status s, const std::string& msg) { return ::fail(s, msg); }
qed_status get_code_object(const std::string& tag, const std::string& src, std::string& co, KernelMeta& meta,
                           bool& hit, double& ms) {
  return ::get_code_object(tag, src, co, meta, hit, ms);
}
std::string cache_dir() { return cache_dir_str(); }
qed_status grad_fused(const qed_process* p, const double* uniforms, double sqrt_s, int64_t N, double* out_logm2,
                      double* out_grad, void* stream) {
  long long n = (long long)N;
  void* args[] = {(void*)&uniforms, (void*)&sqrt_s, (void*)&n, (void*)&out_logm2, (void*)&out_grad};
  return launch(p->f_grad, N * (int64_t)p->grad_lanes, p->grad_block, stream, args);
}
qed_status default_process_variant(int n, qed_hel_mode mode, qed_precision prec, int rewrite, qedx::Variant& v) {
  if (!rewrite) return make_variant(n, 1, mode, prec, nullptr, v);
  qed_variant q;
  std::memset(&q, 0, sizeof q);
  q.rewrite = 1;
  return make_variant(n, 1, mode, prec, &q, v);
}
}  // namespace qedx_rt
