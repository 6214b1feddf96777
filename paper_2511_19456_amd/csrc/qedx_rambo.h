// qedx_rambo.h -- RAMBO phase-space generation for one point per lane.
//
// RAMBO (Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359):
// NF isotropic massless momenta with exponential energies are boosted and
// scaled so that they sum to (sqrt_s, 0); the three-momenta are then scaled
// by a common factor xi so that the energies on the mass shells sum to sqrt_s.
// Here the final state is [e-_out (mass m), NF-1 photons]; the incoming pair
// sits in its CM frame with the photon along +z.
//
// Uniform layout: u[4 j + r] for final-state particle j, r = 0..3:
//   c = 2 u0 - 1, phi = 2 pi u1, q0 = -ln(u2 u3).
#pragma once

namespace qx {

template <int NF>
struct RamboState {
  // massless intermediate quantities kept for the adjoint
  double q[NF][4];
  double Q[4], M, b[3], gam, a, x;
  double p[NF][4];  // massless momenta summing to (sqrt_s, 0)
  double xi;
  double k[NF][4];  // final momenta
};

// Newton solve of f(xi) = sqrt(m^2 + xi^2 E0^2) + xi sum_{i>0} E_i - sqrt_s = 0
// (massive first particle, massless rest); stops when |dxi| <= 4 eps xi.
QEDX_HD double rambo_xi(double E0, double Erest, double sqrt_s, double m) {
  double xi = sqrt(1.0 - (m / sqrt_s) * (m / sqrt_s));
  for (int it = 0; it < 50; ++it) {
    double e0 = sqrt(m * m + xi * xi * E0 * E0);
    double f = e0 + xi * Erest - sqrt_s;
    double fp = xi * E0 * E0 / e0 + Erest;
    double dxi = f / fp;
    xi -= dxi;
    if (fabs(dxi) <= 4.0 * 2.220446049250313e-16 * fabs(xi)) break;
  }
  return xi;
}

template <int NF>
QEDX_HD void rambo_forward(const double* u, double sqrt_s, double m, RamboState<NF>& S) {
  for (int d = 0; d < 4; ++d) S.Q[d] = 0.0;
  for (int j = 0; j < NF; ++j) {
    double c = 2.0 * u[4 * j] - 1.0;
    double phi = 6.283185307179586 * u[4 * j + 1];
    double sphi = sin(phi), cphi = cos(phi);
    double q0 = -log(u[4 * j + 2] * u[4 * j + 3]);
    double st = sqrt(1.0 - c * c);
    S.q[j][0] = q0;
    S.q[j][1] = q0 * st * cphi;
    S.q[j][2] = q0 * st * sphi;
    S.q[j][3] = q0 * c;
    for (int d = 0; d < 4; ++d) S.Q[d] += S.q[j][d];
  }
  S.M = sqrt(S.Q[0] * S.Q[0] - S.Q[1] * S.Q[1] - S.Q[2] * S.Q[2] - S.Q[3] * S.Q[3]);
  for (int d = 0; d < 3; ++d) S.b[d] = -S.Q[d + 1] / S.M;
  S.gam = S.Q[0] / S.M;
  S.a = 1.0 / (1.0 + S.gam);
  S.x = sqrt_s / S.M;
  for (int j = 0; j < NF; ++j) {
    double bq = S.b[0] * S.q[j][1] + S.b[1] * S.q[j][2] + S.b[2] * S.q[j][3];
    S.p[j][0] = S.x * (S.gam * S.q[j][0] + bq);
    for (int d = 0; d < 3; ++d) S.p[j][d + 1] = S.x * (S.q[j][d + 1] + S.b[d] * S.q[j][0] + S.a * bq * S.b[d]);
  }
  double Erest = 0.0;
  for (int j = 1; j < NF; ++j) Erest += S.p[j][0];
  S.xi = rambo_xi(S.p[0][0], Erest, sqrt_s, m);
  S.k[0][0] = sqrt(m * m + S.xi * S.xi * S.p[0][0] * S.p[0][0]);
  for (int j = 1; j < NF; ++j) S.k[j][0] = S.xi * S.p[j][0];
  for (int j = 0; j < NF; ++j)
    for (int d = 1; d < 4; ++d) S.k[j][d] = S.xi * S.p[j][d];
}

// Adjoint of rambo_forward: given gk = dF/dk (final momenta), accumulate
// gu = dF/du.  xi is differentiated implicitly through f(xi, p0) = 0:
// dxi/dp0_j = -(df/dp0_j) / (df/dxi).  S must hold the forward state.
template <int NF>
QEDX_HD void rambo_vjp(const double* u, double sqrt_s, double m, const RamboState<NF>& S, const double gk[NF][4],
                       double* gu) {
  const double xi = S.xi;
  // --- mass rescaling: k_0 = (sqrt(m^2 + xi^2 E0^2), xi p_0), k_j = xi p_j
  double E0 = S.p[0][0];
  double e0 = S.k[0][0];
  double gxi = gk[0][0] * xi * E0 * E0 / e0;
  double gp[NF][4];
  gp[0][0] = gk[0][0] * xi * xi * E0 / e0;
  for (int j = 1; j < NF; ++j) {
    gxi += gk[j][0] * S.p[j][0];
    gp[j][0] = gk[j][0] * xi;
  }
  for (int j = 0; j < NF; ++j)
    for (int d = 1; d < 4; ++d) {
      gxi += gk[j][d] * S.p[j][d];
      gp[j][d] = gk[j][d] * xi;
    }
  double Erest = 0.0;
  for (int j = 1; j < NF; ++j) Erest += S.p[j][0];
  double dfdxi = xi * E0 * E0 / e0 + Erest;
  gp[0][0] += gxi * (-(xi * xi * E0 / e0) / dfdxi);
  for (int j = 1; j < NF; ++j) gp[j][0] += gxi * (-xi / dfdxi);
  // --- boost and scale: p0 = x (gam q0 + b.q), p = x (q + b q0 + a (b.q) b)
  double gx = 0.0, ggam = 0.0, ga = 0.0, gb[3] = {0.0, 0.0, 0.0};
  double gq[NF][4];
  for (int j = 0; j < NF; ++j) {
    const double* q = S.q[j];
    double bq = S.b[0] * q[1] + S.b[1] * q[2] + S.b[2] * q[3];
    double g0 = gp[j][0];
    double gvb = gp[j][1] * S.b[0] + gp[j][2] * S.b[1] + gp[j][3] * S.b[2];
    gx += g0 * (S.gam * q[0] + bq);
    for (int d = 0; d < 3; ++d) gx += gp[j][d + 1] * (q[d + 1] + S.b[d] * q[0] + S.a * bq * S.b[d]);
    ggam += g0 * S.x * q[0];
    double gbq = g0 * S.x + S.x * S.a * gvb;
    ga += S.x * bq * gvb;
    for (int d = 0; d < 3; ++d) gb[d] += S.x * (q[0] + S.a * bq) * gp[j][d + 1] + gbq * q[d + 1];
    gq[j][0] = g0 * S.x * S.gam + S.x * gvb;
    for (int d = 0; d < 3; ++d) gq[j][d + 1] = S.x * gp[j][d + 1] + gbq * S.b[d];
  }
  // --- Q stage: M = sqrt(Q^2), b = -Qv/M, gam = Q0/M, a = 1/(1+gam), x = sqrt_s/M
  ggam += ga * (-S.a * S.a);
  double M = S.M, M2 = M * M;
  double gM = gx * (-sqrt_s / M2) + ggam * (-S.Q[0] / M2);
  for (int d = 0; d < 3; ++d) gM += gb[d] * (S.Q[d + 1] / M2);
  double gQ[4];
  gQ[0] = ggam / M + gM * S.Q[0] / M;
  for (int d = 0; d < 3; ++d) gQ[d + 1] = -gb[d] / M - gM * S.Q[d + 1] / M;
  // --- isotropic massless momenta q_j = q0 (st cos phi, st sin phi, c)
  for (int j = 0; j < NF; ++j) {
    double g0 = gq[j][0] + gQ[0];
    double gx1 = gq[j][1] + gQ[1], gy1 = gq[j][2] + gQ[2], gz1 = gq[j][3] + gQ[3];
    double c = 2.0 * u[4 * j] - 1.0;
    double phi = 6.283185307179586 * u[4 * j + 1];
    double sphi = sin(phi), cphi = cos(phi);
    double q0 = S.q[j][0];
    double st = sqrt(1.0 - c * c);
    double gq0 = g0 + gx1 * st * cphi + gy1 * st * sphi + gz1 * c;
    double dst = -c / st;
    double gc = gx1 * q0 * cphi * dst + gy1 * q0 * sphi * dst + gz1 * q0;
    double gphi = -gx1 * q0 * st * sphi + gy1 * q0 * st * cphi;
    gu[4 * j + 0] += 2.0 * gc;
    gu[4 * j + 1] += 6.283185307179586 * gphi;
    gu[4 * j + 2] += -gq0 / u[4 * j + 2];
    gu[4 * j + 3] += -gq0 / u[4 * j + 3];
  }
}

// Incoming pair in the CM frame: p = (E, 0, 0, -kap), k = (kap, 0, 0, kap).
QEDX_HD void incoming_cm(double sqrt_s, double m, double p[4], double k[4]) {
  double s = sqrt_s * sqrt_s;
  double kap = (s - m * m) / (2.0 * sqrt_s);
  double E = (s + m * m) / (2.0 * sqrt_s);
  p[0] = E;
  p[1] = 0.0;
  p[2] = 0.0;
  p[3] = -kap;
  k[0] = kap;
  k[1] = 0.0;
  k[2] = 0.0;
  k[3] = kap;
}

}  // namespace qx
