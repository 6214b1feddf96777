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
    double sphi, cphi;
    sincospi(2.0 * u[4 * j + 1], &sphi, &cphi);
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
