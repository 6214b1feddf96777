// qedx_device.h -- per-lane building blocks of the QED matrix-element kernels.
//
// These are the compute tasks of the paper's QED computation graph (Sec. II-B:
// base_state U, vertex V, propagator S1, join S2 and Sum), written for one
// phase-space point per lane.  Generated kernels include this header verbatim
// and call these functions once per graph node; the host-side graph
// interpreter uses the same functions on the CPU.
//
// Representation.  Chiral (Weyl) basis, gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]]
// with sigma = (1, sigma_vec), sigmabar = (1, -sigma_vec), so that
//   a-slash = [[0, a0 - a.sigma], [a0 + a.sigma, 0]].
// A fermion current from the incoming-electron side is a column 4-spinor
// (L0, L1, R0, R1); one from the outgoing-electron side is a row spinor
// (ubar-side, same component order).  The physical states are the Dirac-basis
// ones -- rest-frame z spin boosted to p -- mapped by the unitary
// (1/sqrt2)[[1,-1],[1,1]], which leaves every amplitude unchanged.
//
// Polarisation vectors are linear (x, y), real, with eps^0 = 0 in the frame
// of the input momenta, so eps-slash = [[0, -E], [E, 0]] with
// E = eps_vec . sigma = [[e3, e1 - i e2], [e1 + i e2, -e3]].
//
// Propagator S(Q) = (Q-slash + m) / (Q^2 - m^2) (Sec. I-D, i and i*epsilon
// dropped).  Callers pass Q/D and m/D precomputed in double precision:
//   qm = (Q0 - Q3)/D, qp = (Q0 + Q3)/D, q1 = Q1/D, q2 = Q2/D, mm = m/D.
//
// FLOP counts (add/mul = 1, fma = 2) are stated per function; the host cost
// model uses the same numbers.
#pragma once

#ifndef QEDX_HD
#define QEDX_HD __host__ __device__ inline
#endif

namespace qx {

template <class T> struct cx { T r, i; };
template <class T> struct sp4 { cx<T> c[4]; };          // L0 L1 R0 R1
template <class T> struct pol3 { T e1, e2, e3; };        // eps_vec, eps^0 = 0
template <class T> struct propq { T qm, qp, q1, q2, mm; };

// Round an FP64 current or polarisation vector to FP32 (one rounding per entry).
QEDX_HD sp4<float> to_f(const sp4<double>& x) {
  sp4<float> o;
  for (int k = 0; k < 4; ++k) o.c[k] = {(float)x.c[k].r, (float)x.c[k].i};
  return o;
}
QEDX_HD pol3<float> to_f(const pol3<double>& e) { return {(float)e.e1, (float)e.e2, (float)e.e3}; }
QEDX_HD cx<float> to_f(const cx<double>& z) { return {(float)z.r, (float)z.i}; }

// ---------------------------------------------------------------------------
// 2x2 blocks.  E x and x E for E = [[e3, e1 - i e2], [e1 + i e2, -e3]].
// y0 = e3 x0 + (e1 - i e2) x1 ; y1 = (e1 + i e2) x0 - e3 x1.     20 FLOPs
// With e3 == 0 (the y polarisation) use the *_y forms.            12 FLOPs
// ---------------------------------------------------------------------------
template <class T>
QEDX_HD void Ex(const pol3<T>& e, const cx<T>& x0, const cx<T>& x1, T s, cx<T>& y0, cx<T>& y1) {
  // s = +1 or -1 folds a sign into the result (free: source modifiers)
  y0.r = s * (e.e3 * x0.r + e.e1 * x1.r + e.e2 * x1.i);
  y0.i = s * (e.e3 * x0.i + e.e1 * x1.i - e.e2 * x1.r);
  y1.r = s * (e.e1 * x0.r - e.e2 * x0.i - e.e3 * x1.r);
  y1.i = s * (e.e1 * x0.i + e.e2 * x0.r - e.e3 * x1.i);
}
template <class T>
QEDX_HD void Ex_y(const pol3<T>& e, const cx<T>& x0, const cx<T>& x1, T s, cx<T>& y0, cx<T>& y1) {
  y0.r = s * (e.e1 * x1.r + e.e2 * x1.i);
  y0.i = s * (e.e1 * x1.i - e.e2 * x1.r);
  y1.r = s * (e.e1 * x0.r - e.e2 * x0.i);
  y1.i = s * (e.e1 * x0.i + e.e2 * x0.r);
}
// row x times E: (x0 e3 + x1 (e1 + i e2), x0 (e1 - i e2) - x1 e3)
template <class T>
QEDX_HD void xE(const pol3<T>& e, const cx<T>& x0, const cx<T>& x1, T s, cx<T>& y0, cx<T>& y1) {
  y0.r = s * (e.e3 * x0.r + e.e1 * x1.r - e.e2 * x1.i);
  y0.i = s * (e.e3 * x0.i + e.e1 * x1.i + e.e2 * x1.r);
  y1.r = s * (e.e1 * x0.r + e.e2 * x0.i - e.e3 * x1.r);
  y1.i = s * (e.e1 * x0.i - e.e2 * x0.r - e.e3 * x1.i);
}
template <class T>
QEDX_HD void xE_y(const pol3<T>& e, const cx<T>& x0, const cx<T>& x1, T s, cx<T>& y0, cx<T>& y1) {
  y0.r = s * (e.e1 * x1.r - e.e2 * x1.i);
  y0.i = s * (e.e1 * x1.i + e.e2 * x1.r);
  y1.r = s * (e.e1 * x0.r + e.e2 * x0.i);
  y1.i = s * (e.e1 * x0.i - e.e2 * x0.r);
}

// ---------------------------------------------------------------------------
// V: vertex.  Left current:  J' = eps-slash J   = (-E R, E L).       40 FLOPs
//             Right current: J'bar = Jbar eps-slash = (b E, -a E).    40 FLOPs
// ("_y" variants for e3 == 0: 24 FLOPs.)
// ---------------------------------------------------------------------------
template <class T> QEDX_HD sp4<T> vL(const sp4<T>& J, const pol3<T>& e) {
  sp4<T> o;
  Ex<T>(e, J.c[2], J.c[3], T(-1), o.c[0], o.c[1]);
  Ex<T>(e, J.c[0], J.c[1], T(1), o.c[2], o.c[3]);
  return o;
}
template <class T> QEDX_HD sp4<T> vL_y(const sp4<T>& J, const pol3<T>& e) {
  sp4<T> o;
  Ex_y<T>(e, J.c[2], J.c[3], T(-1), o.c[0], o.c[1]);
  Ex_y<T>(e, J.c[0], J.c[1], T(1), o.c[2], o.c[3]);
  return o;
}
template <class T> QEDX_HD sp4<T> vR(const sp4<T>& J, const pol3<T>& e) {
  sp4<T> o;
  xE<T>(e, J.c[2], J.c[3], T(1), o.c[0], o.c[1]);
  xE<T>(e, J.c[0], J.c[1], T(-1), o.c[2], o.c[3]);
  return o;
}
template <class T> QEDX_HD sp4<T> vR_y(const sp4<T>& J, const pol3<T>& e) {
  sp4<T> o;
  xE_y<T>(e, J.c[2], J.c[3], T(1), o.c[0], o.c[1]);
  xE_y<T>(e, J.c[0], J.c[1], T(-1), o.c[2], o.c[3]);
  return o;
}

// ---------------------------------------------------------------------------
// S1: propagator.  Left:  (Q-slash + m) J / D = (mm L + Qs R, Qb L + mm R)
//                  Right: Jbar (Q-slash + m) / D = (mm a + b Qb, a Qs + mm b)
// Qs = Q.sigma/D = [[qm, -q1 + i q2], [-q1 - i q2, qp]],
// Qb = Q.sigmabar/D = [[qp, q1 - i q2], [q1 + i q2, qm]].        56 FLOPs each
// ---------------------------------------------------------------------------
template <class T> QEDX_HD sp4<T> sL(const sp4<T>& J, const propq<T>& q) {
  const cx<T>&L0 = J.c[0], &L1 = J.c[1], &R0 = J.c[2], &R1 = J.c[3];
  sp4<T> o;
  o.c[0].r = q.mm * L0.r + q.qm * R0.r - q.q1 * R1.r - q.q2 * R1.i;
  o.c[0].i = q.mm * L0.i + q.qm * R0.i - q.q1 * R1.i + q.q2 * R1.r;
  o.c[1].r = q.mm * L1.r - q.q1 * R0.r + q.q2 * R0.i + q.qp * R1.r;
  o.c[1].i = q.mm * L1.i - q.q1 * R0.i - q.q2 * R0.r + q.qp * R1.i;
  o.c[2].r = q.mm * R0.r + q.qp * L0.r + q.q1 * L1.r + q.q2 * L1.i;
  o.c[2].i = q.mm * R0.i + q.qp * L0.i + q.q1 * L1.i - q.q2 * L1.r;
  o.c[3].r = q.mm * R1.r + q.q1 * L0.r - q.q2 * L0.i + q.qm * L1.r;
  o.c[3].i = q.mm * R1.i + q.q1 * L0.i + q.q2 * L0.r + q.qm * L1.i;
  return o;
}
template <class T> QEDX_HD sp4<T> sR(const sp4<T>& J, const propq<T>& q) {
  const cx<T>&a0 = J.c[0], &a1 = J.c[1], &b0 = J.c[2], &b1 = J.c[3];
  sp4<T> o;
  // (mm a + b Qb): b Qb = (b0 qp + b1 (q1 + i q2), b0 (q1 - i q2) + b1 qm)
  o.c[0].r = q.mm * a0.r + q.qp * b0.r + q.q1 * b1.r - q.q2 * b1.i;
  o.c[0].i = q.mm * a0.i + q.qp * b0.i + q.q1 * b1.i + q.q2 * b1.r;
  o.c[1].r = q.mm * a1.r + q.q1 * b0.r + q.q2 * b0.i + q.qm * b1.r;
  o.c[1].i = q.mm * a1.i + q.q1 * b0.i - q.q2 * b0.r + q.qm * b1.i;
  // (a Qs + mm b): a Qs = (a0 qm + a1 (-q1 - i q2), a0 (-q1 + i q2) + a1 qp)
  o.c[2].r = q.mm * b0.r + q.qm * a0.r - q.q1 * a1.r + q.q2 * a1.i;
  o.c[2].i = q.mm * b0.i + q.qm * a0.i - q.q1 * a1.i - q.q2 * a1.r;
  o.c[3].r = q.mm * b1.r - q.q1 * a0.r - q.q2 * a0.i + q.qp * a1.r;
  o.c[3].i = q.mm * b1.i - q.q1 * a0.i + q.q2 * a0.r + q.qp * a1.i;
  return o;
}

// ---------------------------------------------------------------------------
// Dot (the join after its propagator has been moved onto one side):
// acc += Jbar . J = sum_k Jbar_k J_k.                                 32 FLOPs
// ---------------------------------------------------------------------------
template <class T> QEDX_HD void dot_acc(cx<T>& acc, const sp4<T>& B, const sp4<T>& J) {
  T r = acc.r, i = acc.i;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r = r + B.c[k].r * J.c[k].r;
    i = i + B.c[k].r * J.c[k].i;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r = r - B.c[k].i * J.c[k].i;
    i = i + B.c[k].i * J.c[k].r;
  }
  acc.r = r;
  acc.i = i;
}
template <class T> QEDX_HD cx<T> dot(const sp4<T>& B, const sp4<T>& J) {
  cx<T> a{T(0), T(0)};
  dot_acc(a, B, J);
  return a;
}

// Error-free transformation of a sum (Knuth TwoSum): s + e == a + b exactly.
template <class T> QEDX_HD void two_sum(T a, T b, T& s, T& e) {
  s = a + b;
  T bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
// Compensated accumulation of a complex value (FP32 path): 12 FLOPs.
template <class T> QEDX_HD void comp_acc(cx<T>& s, cx<T>& c, const cx<T>& x) {
  T e;
  two_sum(s.r, x.r, s.r, e);
  c.r = c.r + e;
  two_sum(s.i, x.i, s.i, e);
  c.i = c.i + e;
}

// ---------------------------------------------------------------------------
// Join on the FP64 matrix cores (experiment): the 4 x 4 complex dot matrices
// D[i][j] = sum_k R_i[k] J_j[k] of the 64 lanes of a wave, two lanes per
// pair of v_mfma_f64_4x4x4 (4 blocks of 4 x 4 x 4).  stg holds, per lane
// (stride doubles apart), R_re[i][k] at 4i+k, R_im at 16+4i+k, J_re[j][k] at
// 32+4j+k, J_im at 48+4j+k.  Block b of pair t: lane 2t + (b >> 1), real
// part for even b (R_re J_re^T - R_im J_im^T), imaginary for odd b
// (R_re J_im^T + R_im J_re^T).  Operand lanes: A[b][i][k] at 16k + 4b + i,
// B[b][k][j] at 16k + 4b + j; result C[b][i][j] at 16i + 4b + j.  mj[t] +=
// the result of lane src (the caller's permutation into its accumulator
// layout).  Device only; all 64 lanes of the wave must be active.
// ---------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__)
// The current held by the partner lane (lane ^ 1): the two lanes of a point
// that build the e-_in-side currents for one e-_in spin each exchange them,
// through DPP (quad_perm [1,0,3,2]: one VALU move per 32 bits; measured
// faster than the LDS permute of __shfl_xor in the helicity-sum kernels).
// Device only; both lanes of the pair must be active.
__device__ inline float lane_xor1(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}
__device__ inline double lane_xor1(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <class T> __device__ inline sp4<T> lane_xor1(const sp4<T>& a) {
  sp4<T> o;
#pragma unroll
  for (int k = 0; k < 4; ++k) o.c[k] = {lane_xor1(a.c[k].r), lane_xor1(a.c[k].i)};
  return o;
}

__device__ inline void mfma_join4(const double* stg, int stride, int src, double (&mj)[32]) {
  const int l = (int)(threadIdx.x & 63);
  const int k = l >> 4, b = (l >> 2) & 3, r = l & 3;
  const bool im = (b & 1) != 0;
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const double* q = stg + (2 * t + (b >> 1)) * stride;
    const double a1 = q[4 * r + k];
    const double b1 = q[(im ? 48 : 32) + 4 * r + k];
    const double a2 = im ? q[16 + 4 * r + k] : -q[16 + 4 * r + k];
    const double b2 = q[(im ? 32 : 48) + 4 * r + k];
    double c = __builtin_amdgcn_mfma_f64_4x4x4f64(a1, b1, 0.0, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_4x4x4f64(a2, b2, c, 0, 0, 0);
    mj[t] += __shfl(c, src);
  }
}
#endif

// ---------------------------------------------------------------------------
// Reciprocal and reciprocal square root of a positive (rcp: nonzero) double
// well inside the normal range -- propagator denominators, |k|^2, 2(E+m).
// In the kernels: the hardware estimate (v_rcp_f64, v_rsq_f64) refined by two
// Newton-Raphson steps, r <- r + r (1 - x r) and y <- y + (y/2)(1 - x y^2),
// each of which squares the relative error: within about an ulp of the exact
// value, not correctly rounded, in 5 and 7 instructions where the correctly
// rounded division and square root take about 10 each.  On the host: plain
// arithmetic.
// ---------------------------------------------------------------------------
QEDX_HD double rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return r;
#else
  return 1.0 / x;
#endif
}
QEDX_HD double rsqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(x);
  y = __builtin_fma(0.5 * y, __builtin_fma(-(x * y), y, 1.0), y);
  y = __builtin_fma(0.5 * y, __builtin_fma(-(x * y), y, 1.0), y);
  return y;
#else
  return 1.0 / sqrt(x);
#endif
}

// ---------------------------------------------------------------------------
// U: external states (base_state) from momenta, double precision.
// u(p, s): psi_L = ((E+m) - p.sigma) chi / sqrt(2(E+m)),
//          psi_R = ((E+m) + p.sigma) chi / sqrt(2(E+m)),  chi_0 = (1,0), chi_1 = (0,1).
// ubar(p, s) = (conj psi_R, conj psi_L) as a row.
// ---------------------------------------------------------------------------
template <class T> QEDX_HD sp4<T> u_in(double E, double px, double py, double pz, int s, double m) {
  double c = E + m;
  double nrm = rsqrt(2.0 * c);
  // spin 0: (c - pz, -px - i py, c + pz, px + i py) nrm
  // spin 1: (-px + i py, c + pz, px - i py, c - pz) nrm
  // (selects, not branches: the spin may be a run-time lane bit)
  const double a = (c - pz) * nrm, b = (c + pz) * nrm, x = px * nrm, y = py * nrm;
  const bool up = s == 0;
  sp4<T> o;
  o.c[0] = {T(up ? a : -x), T(up ? 0.0 : y)};
  o.c[1] = {T(up ? -x : b), T(up ? -y : 0.0)};
  o.c[2] = {T(up ? b : x), T(up ? 0.0 : -y)};
  o.c[3] = {T(up ? x : a), T(up ? y : 0.0)};
  return o;
}
template <class T> QEDX_HD sp4<T> ubar_out(double E, double px, double py, double pz, int s, double m) {
  sp4<T> u = u_in<T>(E, px, py, pz, s, m);
  sp4<T> o;
  o.c[0] = {u.c[2].r, -u.c[2].i};
  o.c[1] = {u.c[3].r, -u.c[3].i};
  o.c[2] = {u.c[0].r, -u.c[0].i};
  o.c[3] = {u.c[1].r, -u.c[1].i};
  return o;
}
// Linear polarisation in the theta/phi basis of k-hat:
// eps_x = (cos t cos f, cos t sin f, -sin t), eps_y = (-sin f, cos f, 0);
// k_T = 0: f = 0 and cos t = sign(k_z).
template <class T> QEDX_HD pol3<T> pol(double kx, double ky, double kz, int lam) {
  double kt2 = kx * kx + ky * ky;
  // k_T = 0 (along the z axis): phi = 0, cos theta = sign kz.  Written with
  // selects rather than branches so the surrounding straight-line code stays
  // one basic block.
  const bool flat = !(kt2 > 0.0);
  const double ikt = rsqrt(flat ? 1.0 : kt2);
  const double ikk = rsqrt(flat ? 1.0 : kt2 + kz * kz);
  const double kt = kt2 * ikt;
  const double sgn = kz > 0.0 ? 1.0 : (kz < 0.0 ? -1.0 : 0.0);
  const double cf = flat ? 1.0 : kx * ikt;
  const double sf = flat ? 0.0 : ky * ikt;
  const double ct = flat ? sgn : kz * ikk;
  const double st = flat ? 0.0 : kt * ikk;
  const bool x = lam == 0;
  pol3<T> e;
  e.e1 = T(x ? ct * cf : -sf);
  e.e2 = T(x ? ct * sf : cf);
  e.e3 = T(x ? -st : 0.0);
  return e;
}

// Propagator coefficients from Q and D = Q^2 - m^2 (double precision).
template <class T> QEDX_HD propq<T> prop_coeffs(double Q0, double Q1, double Q2, double Q3, double D, double m) {
  double id = rcp(D);
  propq<T> q;
  q.qm = T((Q0 - Q3) * id);
  q.qp = T((Q0 + Q3) * id);
  q.q1 = T(Q1 * id);
  q.q2 = T(Q2 * id);
  q.mm = T(m * id);
  return q;
}

// Propagator coefficients for Q = p + s K with p on shell and s = +-1:
// Q^2 - m^2 = 2 s p.K + K^2, free of the cancellation in Q.Q - m^2.  28 FLOPs.
template <class T>
QEDX_HD propq<T> prop_from(double p0, double p1, double p2, double p3, double K0, double K1, double K2, double K3,
                           double s, double m) {
  double pK = p0 * K0 - p1 * K1 - p2 * K2 - p3 * K3;
  double KK = K0 * K0 - K1 * K1 - K2 * K2 - K3 * K3;
  double D = 2.0 * s * pK + KK;
  return prop_coeffs<T>(p0 + s * K0, p1 + s * K1, p2 + s * K2, p3 + s * K3, D, m);
}

// ---------------------------------------------------------------------------
// Vector-Jacobian products for the adjoint (reverse) sweep.
//
// For a complex intermediate z the adjoint weight w is defined by
//   dF = 2 Re sum_k w_k dz_k,
// so for F = log(sum_h |A_h|^2) the seed of amplitude A_h is conj(A_h)/|M|^2.
// A linear map J' = M J then gives w_J += M^T w_J' (transpose, no conjugate),
// which for the slash-type maps here is the same map applied from the other
// side: adjoint of vL is vR, of sL is sR and vice versa.
// ---------------------------------------------------------------------------
template <class T> QEDX_HD void add_to(sp4<T>& w, const sp4<T>& x) {
  for (int k = 0; k < 4; ++k) {
    w.c[k].r = w.c[k].r + x.c[k].r;
    w.c[k].i = w.c[k].i + x.c[k].i;
  }
}
// A current in per-lane LDS slots: component k at p[k * stride] (stride =
// threads per block, so a wavefront's accesses are consecutive words).
template <class T> QEDX_HD void lds_put(T* p, int stride, const sp4<T>& x) {
  for (int k = 0; k < 4; ++k) {
    p[(2 * k) * stride] = x.c[k].r;
    p[(2 * k + 1) * stride] = x.c[k].i;
  }
}
template <class T> QEDX_HD sp4<T> lds_get(const T* p, int stride) {
  sp4<T> x;
  for (int k = 0; k < 4; ++k) {
    x.c[k].r = p[(2 * k) * stride];
    x.c[k].i = p[(2 * k + 1) * stride];
  }
  return x;
}
// sum of two currents (Add node, after the distributive rewrite): 8 FLOPs
template <class T> QEDX_HD sp4<T> add4(const sp4<T>& a, const sp4<T>& b) {
  sp4<T> o;
  for (int k = 0; k < 4; ++k) {
    o.c[k].r = a.c[k].r + b.c[k].r;
    o.c[k].i = a.c[k].i + b.c[k].i;
  }
  return o;
}
template <class T> QEDX_HD sp4<T> zero4() {
  sp4<T> z;
  for (int k = 0; k < 4; ++k) z.c[k] = {T(0), T(0)};
  return z;
}
// w += c * x (complex scalar times spinor)
template <class T> QEDX_HD void axpy(sp4<T>& w, const cx<T>& c, const sp4<T>& x) {
  for (int k = 0; k < 4; ++k) {
    w.c[k].r = w.c[k].r + c.r * x.c[k].r - c.i * x.c[k].i;
    w.c[k].i = w.c[k].i + c.r * x.c[k].i + c.i * x.c[k].r;
  }
}
// Dot A = sum_k B_k J_k with seed c: w_B += c J, w_J += c B.
template <class T> QEDX_HD void dot_vjp(const cx<T>& c, const sp4<T>& B, const sp4<T>& J, sp4<T>& wB, sp4<T>& wJ) {
  axpy(wB, c, J);
  axpy(wJ, c, B);
}
// 2 Re(x^T sigma_i y) for the three Pauli matrices, x, y 2-spinors.
template <class T> QEDX_HD void re_pauli(const cx<T>& x0, const cx<T>& x1, const cx<T>& y0, const cx<T>& y1, T s,
                                         T& g1, T& g2, T& g3) {
  // sigma1: x0 y1 + x1 y0; sigma2: -i x0 y1 + i x1 y0; sigma3: x0 y0 - x1 y1
  T a01r = x0.r * y1.r - x0.i * y1.i, a01i = x0.r * y1.i + x0.i * y1.r;
  T a10r = x1.r * y0.r - x1.i * y0.i, a10i = x1.r * y0.i + x1.i * y0.r;
  T a00r = x0.r * y0.r - x0.i * y0.i;
  T a11r = x1.r * y1.r - x1.i * y1.i;
  g1 = g1 + s * T(2) * (a01r + a10r);
  g2 = g2 + s * T(2) * (a01i - a10i);  // Re(-i z) = Im z
  g3 = g3 + s * T(2) * (a00r - a11r);
}
// Polarisation gradient of a left vertex J' = (-E R, E L), E = e . sigma:
// 2 Re(w . J') = 2 Re(-wa^T E R + wb^T E L).
template <class T> QEDX_HD void vL_ge(const sp4<T>& w, const sp4<T>& J, pol3<T>& g) {
  re_pauli(w.c[0], w.c[1], J.c[2], J.c[3], T(-1), g.e1, g.e2, g.e3);
  re_pauli(w.c[2], w.c[3], J.c[0], J.c[1], T(1), g.e1, g.e2, g.e3);
}
// Right vertex Jb' = (b E, -a E): 2 Re(b^T E wa - a^T E wb).
template <class T> QEDX_HD void vR_ge(const sp4<T>& w, const sp4<T>& J, pol3<T>& g) {
  re_pauli(J.c[2], J.c[3], w.c[0], w.c[1], T(1), g.e1, g.e2, g.e3);
  re_pauli(J.c[0], J.c[1], w.c[2], w.c[3], T(-1), g.e1, g.e2, g.e3);
}
template <class T> QEDX_HD T re_mul(const cx<T>& a, const cx<T>& b) { return a.r * b.r - a.i * b.i; }
template <class T> QEDX_HD T im_mul(const cx<T>& a, const cx<T>& b) { return a.r * b.i + a.i * b.r; }
// Propagator-coefficient gradient of a left S1: J' = (mm L + Qs R, Qb L + mm R).
template <class T> QEDX_HD void sL_gq(const sp4<T>& w, const sp4<T>& J, propq<T>& g) {
  const cx<T>&a0 = w.c[0], &a1 = w.c[1], &b0 = w.c[2], &b1 = w.c[3];
  const cx<T>&L0 = J.c[0], &L1 = J.c[1], &R0 = J.c[2], &R1 = J.c[3];
  g.mm = g.mm + T(2) * (re_mul(a0, L0) + re_mul(a1, L1) + re_mul(b0, R0) + re_mul(b1, R1));
  g.qm = g.qm + T(2) * (re_mul(a0, R0) + re_mul(b1, L1));
  g.qp = g.qp + T(2) * (re_mul(a1, R1) + re_mul(b0, L0));
  g.q1 = g.q1 + T(2) * (-re_mul(a0, R1) - re_mul(a1, R0) + re_mul(b0, L1) + re_mul(b1, L0));
  // Re(i z) = -Im z
  g.q2 = g.q2 + T(2) * (-im_mul(a0, R1) + im_mul(a1, R0) + im_mul(b0, L1) - im_mul(b1, L0));
}
// Right S1: Jb' = (mm a + b Qb, a Qs + mm b) with w = (wa, wb), J = (a, b).
template <class T> QEDX_HD void sR_gq(const sp4<T>& w, const sp4<T>& J, propq<T>& g) {
  const cx<T>&wa0 = w.c[0], &wa1 = w.c[1], &wb0 = w.c[2], &wb1 = w.c[3];
  const cx<T>&a0 = J.c[0], &a1 = J.c[1], &b0 = J.c[2], &b1 = J.c[3];
  g.mm = g.mm + T(2) * (re_mul(wa0, a0) + re_mul(wa1, a1) + re_mul(wb0, b0) + re_mul(wb1, b1));
  g.qm = g.qm + T(2) * (re_mul(b1, wa1) + re_mul(a0, wb0));
  g.qp = g.qp + T(2) * (re_mul(b0, wa0) + re_mul(a1, wb1));
  g.q1 = g.q1 + T(2) * (re_mul(b0, wa1) + re_mul(b1, wa0) - re_mul(a0, wb1) - re_mul(a1, wb0));
  g.q2 = g.q2 + T(2) * (im_mul(b0, wa1) - im_mul(b1, wa0) - im_mul(a0, wb1) + im_mul(a1, wb0));
}
// Gradient of 2 Re(w . ubar(p, s)) with respect to p = (E, px, py, pz).
QEDX_HD void ubar_vjp(double E, double px, double py, double pz, int s, double m, const sp4<double>& w,
                      double g[4]) {
  // ubar = (conj psi_R, conj psi_L); psi components are nrm * (affine in p),
  // nrm = (2c)^(-1/2), c = E + m.  Write u_k = nrm * v_k(p); then
  // d u_k = nrm dv_k + v_k dnrm, dnrm/dE = -nrm / (2c).
  double c = E + m;
  double nrm = 1.0 / sqrt(2.0 * c);
  double dn = -nrm / (2.0 * c);
  // v for psi_L (index 0,1) and psi_R (index 2,3) as complex (re, im);
  // dv/dp columns: E, px, py, pz
  double vr[4], vi[4], dvr[4][4], dvi[4][4];
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) dvr[k][j] = dvi[k][j] = 0.0;
  if (s == 0) {
    vr[0] = c - pz; vi[0] = 0;   dvr[0][0] = 1; dvr[0][3] = -1;
    vr[1] = -px;    vi[1] = -py; dvr[1][1] = -1; dvi[1][2] = -1;
    vr[2] = c + pz; vi[2] = 0;   dvr[2][0] = 1; dvr[2][3] = 1;
    vr[3] = px;     vi[3] = py;  dvr[3][1] = 1; dvi[3][2] = 1;
  } else {
    vr[0] = -px;    vi[0] = py;  dvr[0][1] = -1; dvi[0][2] = 1;
    vr[1] = c + pz; vi[1] = 0;   dvr[1][0] = 1; dvr[1][3] = 1;
    vr[2] = px;     vi[2] = -py; dvr[2][1] = 1; dvi[2][2] = -1;
    vr[3] = c - pz; vi[3] = 0;   dvr[3][0] = 1; dvr[3][3] = -1;
  }
  // ubar component k = conj(u_{perm k}), perm = (2,3,0,1)
  const int perm[4] = {2, 3, 0, 1};
  for (int j = 0; j < 4; ++j) g[j] = 0.0;
  for (int k = 0; k < 4; ++k) {
    int q = perm[k];
    // d(conj u_q) = nrm conj(dv_q) + conj(v_q) dnrm
    for (int j = 0; j < 4; ++j) {
      double dr = nrm * dvr[q][j] + (j == 0 ? vr[q] * dn : 0.0);
      double di = -(nrm * dvi[q][j] + (j == 0 ? vi[q] * dn : 0.0));
      g[j] += 2.0 * (w.c[k].r * dr - w.c[k].i * di);
    }
  }
}
// Gradient of ge . eps(k, lam) with respect to (kx, ky, kz).
QEDX_HD void pol_vjp(double kx, double ky, double kz, int lam, const pol3<double>& ge, double g[3]) {
  double kt2 = kx * kx + ky * ky;
  double kt = sqrt(kt2);
  double kk2 = kt2 + kz * kz;
  double kk = sqrt(kk2);
  // along the z axis (measure zero) the derivative is not defined: zero,
  // with selects instead of an early return (one basic block)
  const bool flat = !(kt > 0.0);
  if (flat) {
    kt = 1.0;
    kt2 = 1.0;
    kk = 1.0;
    kk2 = 1.0;
  }
  double cf = kx / kt, sf = ky / kt, ct = kz / kk, st = kt / kk;
  double kt3 = kt2 * kt, kk3 = kk2 * kk;
  // partial derivatives of cf, sf, ct, st
  double dcf[3] = {ky * ky / kt3, -kx * ky / kt3, 0.0};
  double dsf[3] = {-kx * ky / kt3, kx * kx / kt3, 0.0};
  double dct[3] = {-kz * kx / kk3, -kz * ky / kk3, kt2 / kk3};
  double dst[3] = {cf * kz * kz / kk3, sf * kz * kz / kk3, -kt * kz / kk3};
  for (int j = 0; j < 3; ++j) {
    // lam 0: eps = (ct cf, ct sf, -st); lam 1: (-sf, cf, 0)
    const double gx = ge.e1 * (dct[j] * cf + ct * dcf[j]) + ge.e2 * (dct[j] * sf + ct * dsf[j]) - ge.e3 * dst[j];
    const double gy = -ge.e1 * dsf[j] + ge.e2 * dcf[j];
    g[j] = flat ? 0.0 : (lam == 0 ? gx : gy);
  }
}
// Gradient through prop_from: given g over (qm, qp, q1, q2, mm), accumulate
// into gp (the electron momentum) and gK (the photon sum).
QEDX_HD void prop_from_vjp(double p0, double p1, double p2, double p3, double K0, double K1, double K2, double K3,
                           double s, double m, const propq<double>& g, double gp[4], double gK[4]) {
  double pK = p0 * K0 - p1 * K1 - p2 * K2 - p3 * K3;
  double KK = K0 * K0 - K1 * K1 - K2 * K2 - K3 * K3;
  double D = 2.0 * s * pK + KK;
  double id = 1.0 / D;
  double Q0 = p0 + s * K0, Q1 = p1 + s * K1, Q2 = p2 + s * K2, Q3 = p3 + s * K3;
  double gQ0 = (g.qm + g.qp) * id, gQ3 = (g.qp - g.qm) * id, gQ1 = g.q1 * id, gQ2 = g.q2 * id;
  double gid = g.qm * (Q0 - Q3) + g.qp * (Q0 + Q3) + g.q1 * Q1 + g.q2 * Q2 + g.mm * m;
  double gD = -gid * id * id;
  const double eta[4] = {1.0, -1.0, -1.0, -1.0};
  const double gQ[4] = {gQ0, gQ1, gQ2, gQ3};
  const double pp[4] = {p0, p1, p2, p3};
  const double KKv[4] = {K0, K1, K2, K3};
  for (int mu = 0; mu < 4; ++mu) {
    gp[mu] += gQ[mu] + gD * 2.0 * s * eta[mu] * KKv[mu];
    gK[mu] += s * gQ[mu] + gD * (2.0 * s * eta[mu] * pp[mu] + 2.0 * eta[mu] * KKv[mu]);
  }
}

}  // namespace qx
