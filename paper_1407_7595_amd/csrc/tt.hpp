// ttbar dilepton integrand: Sec. 3, Eq. integrand, with the change of
// variables to the top and W virtualities (Eq. dilepsolv) and the per-point
// missing transverse momentum of Sec. 4, extended by a transverse recoil of
// the hard system drawn from a Gaussian prior.
//
// Integration variables x in [0,1]^8:
//   x0, x1  r = E_meas/E of the b (from t) and bbar jets, linear in r
//   x2..x5  q2_t, q2_tbar, q2_W+, q2_W- by tan maps aligned with the
//           Breit-Wigner poles (their Jacobians cancel the propagators,
//           leaving (theta1 - theta0)/(M Gamma) each)
//   x6, x7  recoil k_T by a Box-Muller map (prior density x Jacobian = 1)
// Per neutrino solution the final state is boosted transversely to zero
// total p_T; x_{1,2} = (E' +- P_z)/sqrt(S) there, and the integrand picks
// up E_lab/E' from the energy delta function.  FP64: maps, solve, boost,
// Jacobians.  T (FP32 or FP64): matrix element, PDFs, TFs.
#pragma once
#include "device_common.hpp"
#include "dy.hpp"
#include "process.hpp"
#include "tt_me.hpp"
#include "tt_solve.hpp"

namespace memk {

struct TTEvent {
  double n[2][3];      // unit directions of the two jets
  double em[2];        // measured jet energies
  double sin_th[2];
  v4 lp, lm;           // exact leptons
  double lep_fac;      // 1 / (2E_l+ 2E_l-)
};

__device__ __forceinline__ void tt_load(const EventsView& ev, int e, int perm, TTEvent& t)
{
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    int obj = perm ? 1 - k : k;
    double E, x, y, z;
    ev.load(obj, e, E, x, y, z);
    double p = sqrt(x * x + y * y + z * z);
    t.em[k] = E;
    t.n[k][0] = x / p; t.n[k][1] = y / p; t.n[k][2] = z / p;
    t.sin_th[k] = sqrt(x * x + y * y) / p;
  }
  ev.load(2, e, t.lp.e, t.lp.x, t.lp.y, t.lp.z);
  ev.load(3, e, t.lm.e, t.lm.x, t.lm.y, t.lm.z);
  t.lep_fac = 1.0 / (4.0 * t.lp.e * t.lm.e);
}

template <class T>
__device__ __forceinline__ T tf_r(T r, const TFParams& tf)
{
  const T inv_sqrt_2pi = T(0.39894228040143267794);
  const T d = r - T(1);
  const T ic = T(tf.i_core), dc = d * ic;
  T g = exp(T(-0.5) * dc * dc) * ic;
  if (tf.f_tail > 0.0) {
    const T it = T(tf.i_tail), f = T(tf.f_tail), dt = d * it;
    g = (T(1) - f) * g + f * exp(T(-0.5) * dt * dt) * it;
  }
  return inv_sqrt_2pi * g;
}

// transverse boost removing the total transverse momentum P_T
struct TBoost {
  double bx, by, g, g2;
  __device__ __forceinline__ TBoost(const v4& P)
  {
    const double ie = fast_rcp(P.e);
    bx = P.x * ie; by = P.y * ie;
    const double b2 = bx * bx + by * by;
    g = fast_rsqrt(1.0 - b2);
    g2 = g * g * fast_rcp(g + 1.0);     // (g - 1) / b2 without the cancellation
  }
  template <class T>
  __device__ __forceinline__ mom<T> apply(const v4& v) const
  {
    double bp = bx * v.x + by * v.y;
    return mom<T>{T(g * (v.e - bp)), T(v.x + (g2 * bp - g * v.e) * bx),
                  T(v.y + (g2 * bp - g * v.e) * by), T(v.z)};
  }
  __device__ __forceinline__ v4 apply64(const v4& v) const
  {
    double bp = bx * v.x + by * v.y;
    return v4{g * (v.e - bp), v.x + (g2 * bp - g * v.e) * bx, v.y + (g2 * bp - g * v.e) * by, v.z};
  }
};

template <class T>
__device__ __forceinline__ double tt_integrand(const ProcParams& pp, const TTEvent& ev, const double (&x)[8],
                                               int* nsol_out)
{
  const TFParams& tf = pp.tf_b;
  v4 bq[2];
  T jetf = T(1);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double r = tf.r_lo + x[k] * (tf.r_hi - tf.r_lo), ir = fast_rcp(r);
    const double E = ev.em[k] * ir;
    bq[k] = v4{E, E * ev.n[k][0], E * ev.n[k][1], E * ev.n[k][2]};
    // E^2 sin dE T / (2E): the true energy cancels against the TF
    jetf *= T(ev.sin_th[k] * (tf.r_hi - tf.r_lo) * E * ir * 0.5) * tf_r<T>(T(r), tf);
  }
  const double mtg = pp.m_t * pp.w_t, mwg = pp.m_w * pp.w_w;
  const double q2t = pp.m_t * pp.m_t + mtg * tan(pp.th0_t + x[2] * (pp.th1_t - pp.th0_t));
  const double q2tb = pp.m_t * pp.m_t + mtg * tan(pp.th0_t + x[3] * (pp.th1_t - pp.th0_t));
  const double q2wp = pp.m_w * pp.m_w + mwg * tan(pp.th0_w + x[4] * (pp.th1_w - pp.th0_w));
  const double q2wm = pp.m_w * pp.m_w + mwg * tan(pp.th0_w + x[5] * (pp.th1_w - pp.th0_w));
  const double rho = pp.sigma_k * sqrt(-2.0 * log(1.0 - x[6]));
  const double phi = 2.0 * M_PI * x[7];
  const double sphi = sin(phi), cphi = cos(phi);
  const double metx = rho * cphi - (bq[0].x + bq[1].x + ev.lp.x + ev.lm.x);
  const double mety = rho * sphi - (bq[0].y + bq[1].y + ev.lp.y + ev.lm.y);

  NuSet sols;
  solve_dilepton(bq[0], bq[1], ev.lp, ev.lm, metx, mety, q2wp, q2t, q2wm, q2tb, sols);
  const int ns = sols.n;

  // matrix element stage: only the solutions are live here
  const T mt = T(pp.m_t);
  const double isqs = pp.inv_sqrt_s;
  double acc = 0.0;
  for (int k = 0; k < ns; ++k) {
    const NuSol sk = sols.get(k);
    v4 nu{0.0, sk.nx, sk.ny, sk.nz}, nb{0.0, sk.bx, sk.by, sk.bz};
    nu.e = norm3(nu);
    nb.e = norm3(nb);
    v4 P = add(add(add(bq[0], bq[1]), add(ev.lp, ev.lm)), add(nu, nb));
    double Eh = sqrt(P.e * P.e - P.x * P.x - P.y * P.y);
    double x1 = (Eh + P.z) * isqs, x2 = (Eh - P.z) * isqs;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    TBoost B(P);
    v4 hb = B.apply64(bq[0]), hl = B.apply64(ev.lp), hn = B.apply64(nu);
    v4 hbb = B.apply64(bq[1]), hlm = B.apply64(ev.lm), hnb = B.apply64(nb);
    v4 tp = add(add(hb, hl), hn), tm = add(add(hbb, hlm), hnb);
    mom<T> pt{T(tp.e), T(tp.x), T(tp.y), T(tp.z)}, ptb{T(tm.e), T(tm.x), T(tm.y), T(tm.z)};
    drow<T> R, C;
    decay_rows<T>(hb, hl, hn, hbb, hlm, hnb, pt, ptb, mt, R, C);
    double a = 0.5 * x1 * pp.sqrt_s, bm = 0.5 * x2 * pp.sqrt_s;
    T mgg = gg_sum<T>(R, C, pt, T(a), T(bm), mt);
    v4 k1{a, 0.0, 0.0, a}, k2{bm, 0.0, 0.0, -bm};
    T mq1 = qq_sum<T>(R, C, k1, k2);
    T mq2 = qq_sum<T>(R, C, k2, k1);
    // toy densities x f(x) (configuration) and x g(x) = 3 (1-x)^5
    double o1 = 1.0 - x1, o2 = 1.0 - x2;
    T g1 = T(3.0 * o1 * o1 * o1 * o1 * o1), g2 = T(3.0 * o2 * o2 * o2 * o2 * o2);
    T q1 = T(xfu(x1, o1) + xfd(x1, o1)), q2 = T(xfu(x2, o2) + xfd(x2, o2));
    T qb1 = T(xfq(o1)), qb2 = T(xfq(o2));
    T me = g1 * g2 * mgg * T(1.0 / 256.0) + (q1 * qb2 * mq1 + qb1 * q2 * mq2) * T(1.0 / 36.0);
    double shat = x1 * x2 * pp.S;
    acc += P.e * (double)me * fast_rcp(Eh * shat * x1 * x2 * sk.adet * nu.e * nb.e);
  }
  if (nsol_out) *nsol_out = ns;
  return acc * pp.tt_const * ev.lep_fac * (double)jetf;
}

}  // namespace memk
