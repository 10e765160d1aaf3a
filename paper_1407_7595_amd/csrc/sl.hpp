// ttbar semileptonic integrand (one W -> q qbar'): Sec. 3, Eq. integrand
// with the hadronic W, the hadronic top and the leptonic W aligned with
// integration variables, and the per-point missing transverse momentum of
// Sec. 4 shifted by the transverse recoil of the hard system.
//
// Assignment perm in [0,12): the ordered pair (b of the leptonic top, b of
// the hadronic top) of distinct jets, b_l-major; the other two jets, in
// ascending order (a, b), are the W -> q qbar' pair and both orderings of
// quark and antiquark are summed inside the integrand.
//
// Variables x in [0,1]^7:
//   x0      r = E_meas/E of light jet a
//   x1      q2 of the hadronic W (tan map) -> E_b = q2 / (2 E_a (1 - cos))
//   x2      q2 of the hadronic top (tan map) -> E_bh linear in q2
//   x3      r of the leptonic b
//   x4, x5  recoil k_T (Box-Muller)
//   x6      q2 of the leptonic W (tan map) -> nu_z from a quadratic
// The three aligned Breit-Wigner factors cancel against the map
// Jacobians; the leptonic top's is evaluated.
#pragma once
#include "device_common.hpp"
#include "dy.hpp"
#include "process.hpp"
#include "tt.hpp"
#include "tt_me.hpp"

namespace memk {

// Jets in role order for one assignment: 0 = light jet a, 1 = light jet b,
// 2 = b of the hadronic top, 3 = b of the leptonic top (static indexing).
struct SLEvent {
  double n[4][3];     // unit jet directions
  double em[4];       // measured jet energies
  double sin_th[4];
  v4 l;               // exact lepton
  int charge;         // +1: l+ (the top decays leptonically), -1: l-
};

// jet slots of assignment perm: (b_l, b_h) ordered pair, b_l-major; the
// remaining two ascending
__device__ __forceinline__ void sl_roles(int perm, int (&slot)[4])
{
  const int ibl = perm / 3, r3 = perm - 3 * ibl;
  const int ibh = r3 < ibl ? r3 : r3 + 1;
  int ja = 0;
  while (ja == ibl || ja == ibh) ++ja;
  int jb = ja + 1;
  while (jb == ibl || jb == ibh) ++jb;
  slot[0] = ja; slot[1] = jb; slot[2] = ibh; slot[3] = ibl;
}

__device__ __forceinline__ void sl_load(const EventsView& ev, const int32_t* charge, int e, int perm, SLEvent& s)
{
  int slot[4];
  sl_roles(perm, slot);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double E, x, y, z;
    ev.load(slot[k], e, E, x, y, z);
    double p = sqrt(x * x + y * y + z * z);
    s.em[k] = E;
    s.n[k][0] = x / p; s.n[k][1] = y / p; s.n[k][2] = z / p;
    s.sin_th[k] = sqrt(x * x + y * y) / p;
  }
  ev.load(4, e, s.l.e, s.l.x, s.l.y, s.l.z);
  s.charge = charge ? (charge[e] < 0 ? -1 : 1) : 1;
}

template <int K>
__device__ __forceinline__ v4 sl_jet(const SLEvent& s, double E)
{
  return v4{E, E * s.n[K][0], E * s.n[K][1], E * s.n[K][2]};
}

template <class T>
__device__ __forceinline__ double sl_integrand(const ProcParams& pp, const SLEvent& ev, const double (&x)[7],
                                               int* nsol_out)
{
  if (nsol_out) *nsol_out = 0;
  const TFParams& tb = pp.tf_b;
  const TFParams& tl = pp.tf_lj;
  // light jet a from its r
  const double ema = ev.em[0];
  const double ra = tl.r_lo + x[0] * (tl.r_hi - tl.r_lo), ira = fast_rcp(ra);
  const v4 qa = sl_jet<0>(ev, ema * ira);
  // hadronic W: q2 = 2 E_a E_b (1 - cos(a, b))
  const double mwg = pp.m_w * pp.w_w, mtg = pp.m_t * pp.w_t;
  const double q2wh = pp.m_w * pp.m_w + mwg * tan_halfpi(pp.th0_w + x[1] * (pp.th1_w - pp.th0_w));
  const v4 ua = sl_jet<0>(ev, 1.0), ub = sl_jet<1>(ev, 1.0);
  const double omc = 1.0 - (ua.x * ub.x + ua.y * ub.y + ua.z * ub.z);
  if (!(omc > 0.0)) return 0.0;
  const double dEb = fast_rcp(2.0 * qa.e * omc);          // dE_b / dq2
  const double Eb = q2wh * dEb;
  const v4 qb = sl_jet<1>(ev, Eb);
  // hadronic top: q2 = q2_W + 2 E_bh (E_W - n_bh . p_W)
  const double q2th = pp.m_t * pp.m_t + mtg * tan_halfpi(pp.th0_t + x[2] * (pp.th1_t - pp.th0_t));
  const v4 W = add(qa, qb);
  const v4 uh = sl_jet<2>(ev, 1.0);
  const double den = 2.0 * (W.e - (uh.x * W.x + uh.y * W.y + uh.z * W.z));
  if (!(den > 0.0)) return 0.0;
  const double dEh = fast_rcp(den);
  const double Ebh = (q2th - q2wh) * dEh;
  if (!(Ebh > 0.0)) return 0.0;
  const v4 bh = sl_jet<2>(ev, Ebh);
  // leptonic b from its r
  const double eml = ev.em[3];
  const double rl = tb.r_lo + x[3] * (tb.r_hi - tb.r_lo), irl = fast_rcp(rl);
  const v4 bl = sl_jet<3>(ev, eml * irl);
  // solved energies must lie inside their TF windows
  const double rb = ev.em[1] * fast_rcp(Eb), rh = ev.em[2] * fast_rcp(Ebh);
  if (rb < tl.r_lo || rb > tl.r_hi || rh < tb.r_lo || rh > tb.r_hi) return 0.0;
  // jet factors E^2 sin dE T / (2E): sin/2 tf_r(r) times dE per unit variable
  T jetf = T(0.5 * ev.sin_th[0] * (tl.r_hi - tl.r_lo) * ema * ira * ira) * tf_r<T>(T(ra), tl);
  jetf *= T(0.5 * ev.sin_th[1] * dEb) * tf_r<T>(T(rb), tl);
  jetf *= T(0.5 * ev.sin_th[2] * dEh) * tf_r<T>(T(rh), tb);
  jetf *= T(0.5 * ev.sin_th[3] * (tb.r_hi - tb.r_lo) * eml * irl * irl) * tf_r<T>(T(rl), tb);
  // neutrino transverse momentum from the recoil
  const double rho = pp.sigma_k * sqrt(-2.0 * log(1.0 - x[4]));
  double sphi, cphi;
  sincospi(2.0 * x[5], &sphi, &cphi);     // angle 2 pi x5
  const double nx = rho * cphi - (qa.x + qb.x + bh.x + bl.x + ev.l.x);
  const double ny = rho * sphi - (qa.y + qb.y + bh.y + bl.y + ev.l.y);
  // leptonic W: 2 l.nu = q2 at fixed nu_T -> l_T^2 nu_z^2 - 2 a l_z nu_z + E_l^2 nu_T^2 - a^2 = 0
  const double q2wl = pp.m_w * pp.m_w + mwg * tan_halfpi(pp.th0_w + x[6] * (pp.th1_w - pp.th0_w));
  const v4& l = ev.l;
  const double lt2 = l.x * l.x + l.y * l.y;
  const double a = 0.5 * q2wl + l.x * nx + l.y * ny;
  const double disc = a * a - lt2 * (nx * nx + ny * ny);
  if (!(a > 0.0) || disc < 0.0 || !(lt2 > 0.0)) return 0.0;
  const double sq = l.e * sqrt(disc), ilt2 = fast_rcp(lt2);
  const T mt = T(pp.m_t * kMeScale);      // matrix-element units
  const double isqs = pp.inv_sqrt_s;
  const v4 vis = add(add(add(qa, qb), add(bh, bl)), l);
  double acc = 0.0;
  int ns = 0;
  for (int s = 0; s < 2; ++s) {
    const double nz = (a * l.z + (s ? -sq : sq)) * ilt2;
    v4 nu{0.0, nx, ny, nz};
    nu.e = norm3(nu);
    const double dq = fabs(2.0 * (l.e * nz * fast_rcp(nu.e) - l.z));
    if (!(dq > 0.0)) continue;
    ++ns;
    const v4 P = add(vis, nu);
    const double Eh = sqrt(P.e * P.e - P.x * P.x - P.y * P.y);
    const double x1 = (Eh + P.z) * isqs, x2 = (Eh - P.z) * isqs;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    // the leptonic top's Breit-Wigner (its virtuality is not a variable)
    const v4 tl4 = add(add(bl, l), nu);
    const double dtl = mdot(tl4, tl4) - pp.m_t * pp.m_t;
    const double bwtl = fast_rcp(dtl * dtl + mtg * mtg);
    TBoost B(P);
    const v4 hqa = B.apply_me(qa), hqb = B.apply_me(qb), hbh = B.apply_me(bh);
    const v4 hbl = B.apply_me(bl), hl = B.apply_me(l), hn = B.apply_me(nu);
    const double ak = 0.5 * x1 * pp.sqrt_s * kMeScale, bk = 0.5 * x2 * pp.sqrt_s * kMeScale;
    T gg, qq12, qq21;
    tt_lumis<T>(pp, x1, x2, gg, qq12, qq21);
    T me = T(0);
    for (int o = 0; o < 2; ++o) {
      // ordering o: (quark, antiquark) of the hadronic W
      const v4& qk = o == 0 ? hqa : hqb;
      const v4& qbk = o == 0 ? hqb : hqa;
      // W+ current ubar(f) .. v(fbar) on the top side, W- current on the
      // antitop side: leptonic top (l+ nu) or hadronic top (u dbar)
      const bool lp = ev.charge > 0;
      const v4& tb_ = lp ? hbl : hbh;
      const v4& tf1b = lp ? hl : qbk;     // antifermion of the W+
      const v4& tf1 = lp ? hn : qk;       // fermion of the W+
      const v4& ab_ = lp ? hbh : hbl;
      const v4& af2 = lp ? qk : hl;       // fermion of the W-
      const v4& af2b = lp ? qbk : hn;     // antifermion of the W-
      const v4 tp = add(add(tb_, tf1b), tf1), tm = add(add(ab_, af2), af2b);
      drow<T> R, C;
      decay_rows<T>(tb_, tf1b, tf1, ab_, af2, af2b, tp, tm, mt, R, C);
      const T mgg = gg_sum<T>(R, C, tp, ak, bk, mt);
      const T mqq = qq_beams<T>(R, C, T(ak), T(bk));
      me += gg * mgg * T(1.0 / 256.0) + (qq12 + qq21) * mqq * T(1.0 / 36.0);
    }
    const double shat = x1 * x2 * pp.S;
    acc += P.e * ((double)me * kMeDeg8) * bwtl * fast_rcp(Eh * shat * x1 * x2 * dq * nu.e);
  }
  if (nsol_out) *nsol_out = ns;
  return acc * pp.sl_const * (double)jetf * fast_rcp(2.0 * l.e);
}

}  // namespace memk
