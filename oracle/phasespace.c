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

/* Partonic cross section of g g (channel 0) or q qbar (channel 1) ->
 * t tbar -> b l+ nu bbar l- nubar at fixed sqrt(shat), beams along z:
 *   sigma = (1 / (2 shat)) int dPhi_6 |M|^2,
 * with |M|^2 the oracle's decayed matrix element (or_tt_me2_gg / _qq: spin
 * and colour averaged, couplings and the four Breit-Wigner factors
 * included).  dPhi_6 is generated by the exact recursion
 *   dPhi_6 = dPhi_2(shat; t, tbar) (dq_t^2 / 2 pi) (dq_tbar^2 / 2 pi)
 *            dPhi_2(t; b, W+) (dq_W+^2 / 2 pi) dPhi_2(W+; l+, nu) x (tbar side),
 * each virtuality through the Breit-Wigner tan map of its propagator over
 * its kinematic range, each direction uniformly; dPhi_2 = |p*| / (4 pi M)
 * after the angular integration.  Points outside the kinematic limits
 * weigh 0. */
static double tan_map(double u, double m, double w, double hi, double* q2)
{
  const double mw = m * w;
  const double t0 = atan(-m * m / mw), t1 = atan((hi - m * m) / mw);
  const double th = t0 + u * (t1 - t0);
  *q2 = m * m + mw * tan(th);
  const double d = *q2 - m * m;
  return (t1 - t0) * (d * d + mw * mw) / mw;     /* dq2 / du */
}

double or_tt_decayed_sigma(const or_params* p, int channel, double sqrt_shat, uint64_t seed, int64_t n_points,
                           double* err)
{
  const double rs = sqrt_shat, shat = rs * rs;
  const double k1[4] = {0.5 * rs, 0.0, 0.0, 0.5 * rs}, k2[4] = {0.5 * rs, 0.0, 0.0, -0.5 * rs};
  double s1 = 0.0, s2 = 0.0;
  for (int64_t k = 0; k < n_points; ++k) {
    double u[16];
    or_uniforms(seed, (uint32_t)k, 0u, 0u, 9u, 16, u);
    double q2t, q2tb, q2wp, q2wm;
    double jac = tan_map(u[0], p->m_t, p->w_t, shat, &q2t) * tan_map(u[1], p->m_t, p->w_t, shat, &q2tb);
    const double mt1 = sqrt(fmax(q2t, 0.0)), mt2 = sqrt(fmax(q2tb, 0.0));
    double w = 0.0;
    if (q2t > 0.0 && q2tb > 0.0 && mt1 + mt2 < rs) {
      jac *= tan_map(u[2], p->m_w, p->w_w, q2t, &q2wp) * tan_map(u[3], p->m_w, p->w_w, q2tb, &q2wm);
      if (q2wp > 0.0 && q2wm > 0.0 && q2wp < q2t && q2wm < q2tb) {
        /* t tbar in the partonic frame */
        const double lam = (shat - (mt1 + mt2) * (mt1 + mt2)) * (shat - (mt1 - mt2) * (mt1 - mt2));
        const double pst = sqrt(lam) / (2.0 * rs);
        const double c = 2.0 * u[4] - 1.0, sn = sqrt(fmax(0.0, 1.0 - c * c)), phi = 2.0 * M_PI * u[5];
        const double pt[4] = {sqrt(pst * pst + q2t), pst * sn * cos(phi), pst * sn * sin(phi), pst * c};
        const double ptb[4] = {sqrt(pst * pst + q2tb), -pt[1], -pt[2], -pt[3]};
        double mom[24], W[4], Wb[4];
        const double mw1 = sqrt(q2wp), mw2 = sqrt(q2wm);
        const double p1 = split(pt, mt1, mw1, 2.0 * u[6] - 1.0, 2.0 * M_PI * u[7], mom + 0, W);
        const double p2 = split(W, mw1, 0.0, 2.0 * u[8] - 1.0, 2.0 * M_PI * u[9], mom + 4, mom + 8);
        const double p3 = split(ptb, mt2, mw2, 2.0 * u[10] - 1.0, 2.0 * M_PI * u[11], mom + 12, Wb);
        const double p4 = split(Wb, mw2, 0.0, 2.0 * u[12] - 1.0, 2.0 * M_PI * u[13], mom + 16, mom + 20);
        const double phase = (pst / (4.0 * M_PI * rs)) * (p1 / (4.0 * M_PI * mt1)) * (p2 / (4.0 * M_PI * mw1))
                           * (p3 / (4.0 * M_PI * mt2)) * (p4 / (4.0 * M_PI * mw2))
                           * jac / pow(2.0 * M_PI, 4.0);
        const double me = channel == 0 ? or_tt_me2_gg(p, k1, k2, mom) : or_tt_me2_qq(p, k1, k2, mom);
        w = phase * me / (2.0 * shat);
      }
    }
    s1 += w;
    s2 += w * w;
  }
  const double N = (double)n_points, I = s1 / N;
  if (err) *err = sqrt(fmax(0.0, s2 / N - I * I) / (N - 1.0));
  return I;
}
