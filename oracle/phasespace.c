/* Massless phase space by sequential two-body splittings, and the top
 * width from its three-body decay (test infrastructure of the oracle).
 *
 * Phase-space measure (Sec. 1 after Eq. 3): dPhi_n = (2 pi)^4 delta^4(P -
 * sum p_i) prod d^3p_i / ((2 pi)^3 2 E_i).  It factorises as
 *   dPhi_n(P; p_1..p_n) = dPhi_2(P; p_1, Q) dQ^2 / (2 pi) dPhi_{n-1}(Q; p_2..p_n),
 * with, for a massless p_1 and an invariant mass m of Q,
 *   dPhi_2 = |p*| / (16 pi^2 M) dOmega*,   |p*| = (M^2 - m^2) / (2 M).
 * A point draws Q^2 uniformly in [0, M^2] at each splitting and the
 * directions uniformly; its weight is the product of the Phi_2 factors
 * |p*| / (4 pi M) and of M^2 / (2 pi) per Q^2 draw, so the weights average to
 * the phase-space volume.  Uniforms come from the oracle's Philox stream. */
#include <math.h>
#include <string.h>

#include "oracle.h"

/* p1 (massless) and p2 (mass m) from P (mass M) with p1 along (c, phi) in
 * P's rest frame, both boosted to P's frame; returns |p*| */
static double split(const double* P, double M, double m, double c, double phi, double* p1, double* p2)
{
  const double pst = (M * M - m * m) / (2.0 * M);
  const double s = sqrt(fmax(0.0, 1.0 - c * c));
  double q1[4] = {pst, pst * s * cos(phi), pst * s * sin(phi), pst * c};
  double q2[4] = {sqrt(pst * pst + m * m), -q1[1], -q1[2], -q1[3]};
  /* boost from P's rest frame: beta = P / E */
  const double bx = P[1] / P[0], by = P[2] / P[0], bz = P[3] / P[0];
  const double b2 = bx * bx + by * by + bz * bz;
  const double g = P[0] / M;
  double* in[2] = {q1, q2};
  double* out[2] = {p1, p2};
  for (int k = 0; k < 2; ++k) {
    const double* q = in[k];
    double bp = bx * q[1] + by * q[2] + bz * q[3];
    double g2 = b2 > 0.0 ? (g - 1.0) / b2 : 0.0;
    out[k][0] = g * (q[0] + bp);
    out[k][1] = q[1] + (g2 * bp + g * q[0]) * bx;
    out[k][2] = q[2] + (g2 * bp + g * q[0]) * by;
    out[k][3] = q[3] + (g2 * bp + g * q[0]) * bz;
  }
  return pst;
}

/* One point of massless n-body phase space (2 <= n <= 6) of a system of
 * mass M at rest, from 3n - 4 uniforms; momenta to p[4n]; returns the
 * weight. */
static double ps_point(int n, double M, const double* u, double* p)
{
  double Q[4] = {M, 0.0, 0.0, 0.0};
  double mQ = M, w = 1.0;
  int iu = 0;
  for (int k = 0; k < n - 1; ++k) {
    double m = 0.0;
    if (k < n - 2) {
      /* invariant mass of the remaining n - 1 - k particles */
      m = mQ * sqrt(u[iu++]);
      w *= mQ * mQ / (2.0 * M_PI);
    }
    const double c = 2.0 * u[iu++] - 1.0, phi = 2.0 * M_PI * u[iu++];
    double rest[4];
    const double pst = split(Q, mQ, m, c, phi, p + 4 * k, rest);
    w *= pst / (4.0 * M_PI * mQ);
    memcpy(Q, rest, sizeof(Q));
    mQ = m;
  }
  memcpy(p + 4 * (n - 1), Q, sizeof(Q));
  return w;
}

double or_ps_volume(int n, double sqrt_s, uint64_t seed, int64_t n_points, double* err)
{
  double s1 = 0.0, s2 = 0.0;
  double u[16], p[24];
  for (int64_t k = 0; k < n_points; ++k) {
    or_uniforms(seed, (uint32_t)k, 0u, 0u, (uint32_t)n, 3 * n - 4, u);
    const double w = ps_point(n, sqrt_s, u, p);
    s1 += w;
    s2 += w * w;
  }
  const double N = (double)n_points, I = s1 / N;
  if (err) *err = sqrt(fmax(0.0, s2 / N - I * I) / (N - 1.0));
  return I;
}

/* Gamma(t -> b l+ nu) of an on-shell top at rest: (1 / (2 m_t)) (1/2)
 * sum_spins int dPhi_3 |M|^2 with |M|^2 = or_decay_w_factor(W virtuality)
 * x or_top_decay_spinsum (the W chain of the oracle's matrix element).  The
 * W virtuality is drawn through the Breit-Wigner tan map over [0, m_t^2]
 * (its Jacobian times the Breit-Wigner factor is constant), the two
 * splittings' directions uniformly. */
double or_top_width(const or_params* p, uint64_t seed, int64_t n_points, double* err)
{
  const double mt = p->m_t, mw = p->m_w, gw = p->w_w;
  const double th0 = atan(-mw * mw / (mw * gw)), th1 = atan((mt * mt - mw * mw) / (mw * gw));
  const double pt[4] = {mt, 0.0, 0.0, 0.0};
  double s1 = 0.0, s2 = 0.0;
  double u[5];
  for (int64_t k = 0; k < n_points; ++k) {
    or_uniforms(seed, (uint32_t)k, 0u, 0u, 7u, 5, u);
    const double th = th0 + u[0] * (th1 - th0);
    const double q2 = mw * mw + mw * gw * tan(th);
    if (!(q2 > 0.0 && q2 < mt * mt)) continue;
    const double mq = sqrt(q2);
    double b[4], W[4], lp[4], nu[4];
    const double ps1 = split(pt, mt, mq, 2.0 * u[1] - 1.0, 2.0 * M_PI * u[2], b, W);
    const double ps2 = split(W, mq, 0.0, 2.0 * u[3] - 1.0, 2.0 * M_PI * u[4], lp, nu);
    /* dq2 / (2 pi) with dq2 = (th1 - th0) du / (M Gamma bw): the tan map's
     * Jacobian, which the matrix element's Breit-Wigner factor bw cancels */
    const double d = q2 - mw * mw, bw = 1.0 / (d * d + mw * mw * gw * gw);
    const double dq2 = (th1 - th0) / (mw * gw * bw);
    const double phase = dq2 / (2.0 * M_PI) * (ps1 / (4.0 * M_PI * mt)) * (ps2 / (4.0 * M_PI * mq));
    const double me = or_decay_w_factor(p, q2) * or_top_decay_spinsum(mt, pt, b, lp, nu);
    const double w = phase * me / (2.0 * mt) * 0.5;
    s1 += w;
    s2 += w * w;
  }
  const double N = (double)n_points, I = s1 / N;
  if (err) *err = sqrt(fmax(0.0, s2 / N - I * I) / (N - 1.0));
  return I;
}
