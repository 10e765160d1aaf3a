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
  // boosted and in matrix-element units (kMeScale, exact)
  __device__ __forceinline__ v4 apply_me(const v4& v) const
  {
    const v4 h = apply64(v);
    return v4{h.e * kMeScale, h.x * kMeScale, h.y * kMeScale, h.z * kMeScale};
  }
};

// The integrand in stages.  tt_maps: per point, the jet energies, TFs,
// virtualities and recoil; the neutrino solve (solve_dilepton, or its
// stages dilep_prepare / quartic_real_roots / dilep_accept); tt_solution:
// per neutrino solution, the boost, |M|^2, PDFs and the weight.  The
// solutions of a point are summed in order, then times the point factors.
template <class T>
struct TTMaps {
  v4 bq[2];          // the two jets (parton energies)
  T jetf;            // jet factors (TF, phase-space density)
  double q2t, q2tb, q2wp, q2wm, metx, mety;
};

template <class T>
__device__ __forceinline__ void tt_maps(const ProcParams& pp, const TTEvent& ev, const double (&x)[8], TTMaps<T>& m)
{
  const TFParams& tf = pp.tf_b;
  T jetf = T(1);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double r = tf.r_lo + x[k] * (tf.r_hi - tf.r_lo), ir = fast_rcp(r);
    const double E = ev.em[k] * ir;
    m.bq[k] = v4{E, E * ev.n[k][0], E * ev.n[k][1], E * ev.n[k][2]};
    // E^2 sin dE T / (2E): the true energy cancels against the TF
    jetf *= T(ev.sin_th[k] * (tf.r_hi - tf.r_lo) * E * ir * 0.5) * tf_r<T>(T(r), tf);
  }
  m.jetf = jetf;
  const double mtg = pp.m_t * pp.w_t, mwg = pp.m_w * pp.w_w;
  m.q2t = pp.m_t * pp.m_t + mtg * tan_halfpi(pp.th0_t + x[2] * (pp.th1_t - pp.th0_t));
  m.q2tb = pp.m_t * pp.m_t + mtg * tan_halfpi(pp.th0_t + x[3] * (pp.th1_t - pp.th0_t));
  m.q2wp = pp.m_w * pp.m_w + mwg * tan_halfpi(pp.th0_w + x[4] * (pp.th1_w - pp.th0_w));
  m.q2wm = pp.m_w * pp.m_w + mwg * tan_halfpi(pp.th0_w + x[5] * (pp.th1_w - pp.th0_w));
  const double rho = pp.sigma_k * sqrt(-2.0 * log(1.0 - x[6]));
  double sphi, cphi;
  sincospi(2.0 * x[7], &sphi, &cphi);     // angle 2 pi x7
  m.metx = rho * cphi - (m.bq[0].x + m.bq[1].x + ev.lp.x + ev.lm.x);
  m.mety = rho * sphi - (m.bq[0].y + m.bq[1].y + ev.lp.y + ev.lm.y);
}

// jet of event slot k with parton energy E
__device__ __forceinline__ v4 tt_jet(const TTEvent& ev, int k, double E)
{
  return v4{E, E * ev.n[k][0], E * ev.n[k][1], E * ev.n[k][2]};
}

// Luminosities in x f form at (x1, x2): gg = xg xg, qq12 = sum_q xq(x1)
// xqbar(x2), qq21 = sum_q xqbar(x1) xq(x2).  Toy densities: u + d against
// the common sea; with a grid, the sums over d, u, s, c, b at m_t.
template <class T>
__device__ __forceinline__ void tt_lumis(const ProcParams& pp, double x1, double x2, T& gg, T& qq12, T& qq21)
{
#ifndef MEM_HOST_COUNT      // the host operation count covers the toy densities
  if (pp.pdf_xf) {
    pdf_grid_tt_lumis<T>(pp, x1, x2, gg, qq12, qq21);
    return;
  }
#endif
  const double o1 = 1.0 - x1, o2 = 1.0 - x2;
  const T g1 = T(3.0 * o1 * o1 * o1 * o1 * o1), g2 = T(3.0 * o2 * o2 * o2 * o2 * o2);
  const T q1 = T(xfu(x1, o1) + xfd(x1, o1)), q2 = T(xfu(x2, o2) + xfd(x2, o2));
  const T qb1 = T(xfq(o1)), qb2 = T(xfq(o2));
  gg = g1 * g2;
  qq12 = q1 * qb2;
  qq21 = qb1 * q2;
}

// |M|^2 x PDFs of a final state given in the lab (b, l+, nu from the top;
// bbar, l-, nubar from the antitop): boost to zero transverse momentum,
// x1, x2 = (E' +- P_z) / sqrt(S), the gg and q qbar channels with the toy
// densities.  Returns false (me = 0) when x1 or x2 falls outside (0, 1];
// P.e and E' (Eh) are returned for the energy delta function.
template <class T>
__device__ __forceinline__ bool tt_me_pdf(const ProcParams& pp, const v4& b0, const v4& lp, const v4& nu,
                                          const v4& b1, const v4& lm, const v4& nb, double& me_out, double& Pe,
                                          double& Eh, double& x1, double& x2)
{
  me_out = 0.0;
  const v4 P = add(add(add(b0, b1), add(lp, lm)), add(nu, nb));
  Pe = P.e;
  Eh = sqrt(P.e * P.e - P.x * P.x - P.y * P.y);
  x1 = (Eh + P.z) * pp.inv_sqrt_s;
  x2 = (Eh - P.z) * pp.inv_sqrt_s;
  if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) return false;
  // densities x f: toy (configuration) or from the grid; formed before the
  // matrix element so that only the three luminosities stay live across it
  T gg, qq12, qq21;
  tt_lumis<T>(pp, x1, x2, gg, qq12, qq21);
  // |M|^2 in the hard frame, in matrix-element units
  const T mt = T(pp.m_t * kMeScale);
  TBoost B(P);
  const v4 hb = B.apply_me(b0), hl = B.apply_me(lp), hn = B.apply_me(nu);
  const v4 hbb = B.apply_me(b1), hlm = B.apply_me(lm), hnb = B.apply_me(nb);
  const v4 tp = add(add(hb, hl), hn), tm = add(add(hbb, hlm), hnb);
  drow<T> R, C;
  decay_rows<T>(hb, hl, hn, hbb, hlm, hnb, tp, tm, mt, R, C);
  const double a = 0.5 * x1 * pp.sqrt_s * kMeScale, bm = 0.5 * x2 * pp.sqrt_s * kMeScale;
  const T mgg = gg_sum<T>(R, C, tp, a, bm, mt);
  // q qbar: the same |M|^2 for the quark from either beam
  const T mqq = qq_beams<T>(R, C, T(a), T(bm));
  const T me = gg * mgg * T(1.0 / 256.0) + (qq12 + qq21) * mqq * T(1.0 / 36.0);
  me_out = (double)me * kMeDeg8;
  return true;
}

// Weight of one neutrino solution sk of a point whose jets have parton
// energies E0, E1 (0 when x1 or x2 falls outside (0, 1]).
template <class T>
__device__ __forceinline__ double tt_solution(const ProcParams& pp, const TTEvent& ev, double E0, double E1,
                                              const NuSol& sk)
{
  const v4 b0 = tt_jet(ev, 0, E0), b1 = tt_jet(ev, 1, E1);
  v4 nu{0.0, sk.nx, sk.ny, sk.nz}, nb{0.0, sk.bx, sk.by, sk.bz};
  nu.e = norm3(nu);
  nb.e = norm3(nb);
  double me, Pe, Eh, x1, x2;
  if (!tt_me_pdf<T>(pp, b0, ev.lp, nu, b1, ev.lm, nb, me, Pe, Eh, x1, x2)) return 0.0;
  const double shat = x1 * x2 * pp.S;
  return Pe * me * fast_rcp(Eh * shat * x1 * x2 * sk.adet * nu.e * nb.e);
}

// Breit-Wigner factor 1 / ((q2 - m^2)^2 + m^2 Gamma^2)
__device__ __forceinline__ double bw_factor(double q2, double m, double w)
{
  const double d = q2 - m * m;
  return fast_rcp(d * d + m * m * w * w);
}

// Parton-level weight of one assignment (transfer functions are delta
// functions; Sec. 4's parton-level timing): the energy and longitudinal
// momentum delta functions (2/S) (E / E'), the flux 1/(2 shat) and the
// complete |M|^2 times the densities f(x1) f(x2).  tt_me_pdf works with
// x f(x) and leaves out the couplings and the four top and W Breit-Wigner
// factors (in the integrand the maps' Jacobians cancel those):
// me_const / (x1 x2) and the factors at the partons' virtualities restore
// them.
template <class T>
__device__ __forceinline__ double tt_parton(const ProcParams& pp, const v4& b0, const v4& lp, const v4& nu,
                                           const v4& b1, const v4& lm, const v4& nb)
{
  double me, Pe, Eh, x1, x2;
  if (!tt_me_pdf<T>(pp, b0, lp, nu, b1, lm, nb, me, Pe, Eh, x1, x2)) return 0.0;
  const v4 wp = add(lp, nu), wm = add(lm, nb), t = add(b0, wp), tb = add(b1, wm);
  const double bw = bw_factor(mdot(t, t), pp.m_t, pp.w_t) * bw_factor(mdot(tb, tb), pp.m_t, pp.w_t)
                  * bw_factor(mdot(wp, wp), pp.m_w, pp.w_w) * bw_factor(mdot(wm, wm), pp.m_w, pp.w_w);
  const double shat = x1 * x2 * pp.S;
  return (2.0 * pp.inv_sqrt_s * pp.inv_sqrt_s) * (Pe * fast_rcp(Eh)) * pp.me_const * bw * me
         * fast_rcp(2.0 * shat * x1 * x2);
}

// The point's value from the sum of its solution weights.
template <class T>
__device__ __forceinline__ double tt_point(const ProcParams& pp, const TTEvent& ev, double acc, T jetf)
{
  return acc * pp.tt_const * ev.lep_fac * (double)jetf;
}

template <class T>
__device__ __forceinline__ double tt_integrand(const ProcParams& pp, const TTEvent& ev, const double (&x)[8],
                                               int* nsol_out)
{
  TTMaps<T> m;
  tt_maps<T>(pp, ev, x, m);
  NuSet sols;
  solve_dilepton(m.bq[0], m.bq[1], ev.lp, ev.lm, m.metx, m.mety, m.q2wp, m.q2t, m.q2wm, m.q2tb, sols, polish_tol<T>());
  const int ns = sols.n;
  double acc = 0.0;
  for (int k = 0; k < ns; ++k) acc += tt_solution<T>(pp, ev, m.bq[0].e, m.bq[1].e, sols.get(k));
  if (nsol_out) *nsol_out = ns;
  return tt_point<T>(pp, ev, acc, m.jetf);
}

}  // namespace memk
