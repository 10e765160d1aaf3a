// gg -> t tbar H integrand, H -> b bbar, one W -> l nu and one W -> q qbar'
// (Sec. 3, Eq. integrand; Sec. 4 with the missing transverse momentum
// shifted by the transverse recoil of the hard system).
//
// Event objects: four b-tagged jets (rows 0-3), two light jets (rows 4, 5),
// the lepton (row 6); the lepton charge comes with the events.
// Assignment perm in [0, 24): o = perm % 2 makes light jet 0 (o = 0) or
// light jet 1 (o = 1) the quark of the hadronic W; perm / 2 selects the b
// pair of the Higgs (6 pairs, ascending) and which of the remaining two
// b-jets comes from the leptonic top (the lower one for an even value).
//
// Variables x in [0,1]^9:
//   x0      r of light jet 0
//   x1      q2 of the hadronic W (tan map) -> energy of light jet 1
//   x2      q2 of the hadronic top (tan map) -> energy of its b
//   x3      r of the leptonic b
//   x4, x5  recoil k_T (Box-Muller)
//   x6      q2 of the leptonic W (tan map) -> nu_z from a quadratic
//   x7      r of the first b of the Higgs pair
//   x8      q2 of the Higgs (tan map) -> energy of the second b
// Four Breit-Wigner factors (hadronic W and top, leptonic W, Higgs) cancel
// against the map Jacobians; the leptonic top's is evaluated.
#pragma once
#include "device_common.hpp"
#include "dy.hpp"
#include "process.hpp"
#include "tt.hpp"
#include "tt_me.hpp"

namespace memk {

// Jets in role order: 0 light jet 0, 1 light jet 1, 2 b of the hadronic
// top, 3 b of the leptonic top, 4 and 5 the Higgs pair.
struct TTHEvent {
  double n[6][3];
  double em[6];
  double sin_th[6];
  v4 l;
  int charge;
  int o;          // 0: light jet 0 is the quark, 1: light jet 1 is
};

__device__ __forceinline__ void tth_roles(int perm, int (&row)[6], int& o)
{
  o = perm & 1;
  const int bp = perm >> 1, hp = bp >> 1;
  // pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
  const int h1 = hp < 3 ? 0 : hp < 5 ? 1 : 2;
  const int h2 = hp < 3 ? hp + 1 : hp < 5 ? hp - 1 : 3;
  int r0 = 0;
  while (r0 == h1 || r0 == h2) ++r0;
  int r1 = r0 + 1;
  while (r1 == h1 || r1 == h2) ++r1;
  const bool odd = bp & 1;
  row[0] = 4; row[1] = 5;
  row[2] = odd ? r0 : r1;   // b of the hadronic top
  row[3] = odd ? r1 : r0;   // b of the leptonic top
  row[4] = h1; row[5] = h2;
}

__device__ __forceinline__ void tth_load(const EventsView& ev, const int32_t* charge, int e, int perm, TTHEvent& s)
{
  int row[6];
  tth_roles(perm, row, s.o);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double E, x, y, z;
    ev.load(row[k], e, E, x, y, z);
    const double p = sqrt(x * x + y * y + z * z);
    s.em[k] = E;
    s.n[k][0] = x / p; s.n[k][1] = y / p; s.n[k][2] = z / p;
    s.sin_th[k] = sqrt(x * x + y * y) / p;
  }
  ev.load(6, e, s.l.e, s.l.x, s.l.y, s.l.z);
  s.charge = charge ? (charge[e] < 0 ? -1 : 1) : 1;
}

template <int K>
__device__ __forceinline__ v4 tth_jet(const TTHEvent& s, double E)
{
  return v4{E, E * s.n[K][0], E * s.n[K][1], E * s.n[K][2]};
}

template <class T>
__device__ __forceinline__ double tth_integrand(const ProcParams& pp, const TTHEvent& ev, const double (&x)[9],
                                                int* nsol_out)
{
  if (nsol_out) *nsol_out = 0;
  const TFParams& tb = pp.tf_b;
  const TFParams& tl = pp.tf_lj;
  const double mwg = pp.m_w * pp.w_w, mtg = pp.m_t * pp.w_t, mhg = pp.m_h * pp.w_h;
  // light jet 0 from its r; light jet 1 from the hadronic W virtuality
  const double ra = tl.r_lo + x[0] * (tl.r_hi - tl.r_lo);
  const v4 qa = tth_jet<0>(ev, ev.em[0] / ra);
  const double q2wh = pp.m_w * pp.m_w + mwg * tan(pp.th0_w + x[1] * (pp.th1_w - pp.th0_w));
  const double omc = 1.0 - (ev.n[0][0] * ev.n[1][0] + ev.n[0][1] * ev.n[1][1] + ev.n[0][2] * ev.n[1][2]);
  if (!(omc > 0.0)) return 0.0;
  const double dEb = fast_rcp(2.0 * qa.e * omc);
  const double Eb = q2wh * dEb;
  const v4 qb = tth_jet<1>(ev, Eb);
  // b of the hadronic top from the top virtuality
  const double q2th = pp.m_t * pp.m_t + mtg * tan(pp.th0_t + x[2] * (pp.th1_t - pp.th0_t));
  const v4 W = add(qa, qb);
  const double den = 2.0 * (W.e - (ev.n[2][0] * W.x + ev.n[2][1] * W.y + ev.n[2][2] * W.z));
  if (!(den > 0.0)) return 0.0;
  const double dEh = fast_rcp(den);
  const double Ebh = (q2th - q2wh) * dEh;
  if (!(Ebh > 0.0)) return 0.0;
  const v4 bh = tth_jet<2>(ev, Ebh);
  // leptonic b and the first Higgs b from their r
  const double rl = tb.r_lo + x[3] * (tb.r_hi - tb.r_lo);
  const v4 bl = tth_jet<3>(ev, ev.em[3] / rl);
  const double r1 = tb.r_lo + x[7] * (tb.r_hi - tb.r_lo);
  const v4 h1 = tth_jet<4>(ev, ev.em[4] / r1);
  // second Higgs b from the Higgs virtuality
  const double q2h = pp.m_h * pp.m_h + mhg * tan(pp.th0_h + x[8] * (pp.th1_h - pp.th0_h));
  const double omh = 1.0 - (ev.n[4][0] * ev.n[5][0] + ev.n[4][1] * ev.n[5][1] + ev.n[4][2] * ev.n[5][2]);
  if (!(omh > 0.0)) return 0.0;
  const double dE2 = fast_rcp(2.0 * h1.e * omh);
  const double E2 = q2h * dE2;
  const v4 h2 = tth_jet<5>(ev, E2);
  const double rb = ev.em[1] / Eb, rh = ev.em[2] / Ebh, r2 = ev.em[5] / E2;
  if (rb < tl.r_lo || rb > tl.r_hi || rh < tb.r_lo || rh > tb.r_hi || r2 < tb.r_lo || r2 > tb.r_hi) return 0.0;
  // jet factors E^2 sin dE T / (2E)
  T jetf = T(0.5 * ev.sin_th[0] * (tl.r_hi - tl.r_lo) * ev.em[0] / (ra * ra)) * tf_r<T>(T(ra), tl);
  jetf *= T(0.5 * ev.sin_th[1] * dEb) * tf_r<T>(T(rb), tl);
  jetf *= T(0.5 * ev.sin_th[2] * dEh) * tf_r<T>(T(rh), tb);
  jetf *= T(0.5 * ev.sin_th[3] * (tb.r_hi - tb.r_lo) * ev.em[3] / (rl * rl)) * tf_r<T>(T(rl), tb);
  jetf *= T(0.5 * ev.sin_th[4] * (tb.r_hi - tb.r_lo) * ev.em[4] / (r1 * r1)) * tf_r<T>(T(r1), tb);
  jetf *= T(0.5 * ev.sin_th[5] * dE2) * tf_r<T>(T(r2), tb);
  // neutrino transverse momentum from the recoil
  const double rho = pp.sigma_k * sqrt(-2.0 * log(1.0 - x[4]));
  const double phi = 2.0 * M_PI * x[5];
  const v4 vis = add(add(add(qa, qb), add(bh, bl)), add(add(h1, h2), ev.l));
  const double nx = rho * cos(phi) - vis.x;
  const double ny = rho * sin(phi) - vis.y;
  // leptonic W: nu_z from the quadratic
  const double q2wl = pp.m_w * pp.m_w + mwg * tan(pp.th0_w + x[6] * (pp.th1_w - pp.th0_w));
  const v4& l = ev.l;
  const double lt2 = l.x * l.x + l.y * l.y;
  const double aq = 0.5 * q2wl + l.x * nx + l.y * ny;
  const double disc = aq * aq - lt2 * (nx * nx + ny * ny);
  if (!(aq > 0.0) || disc < 0.0 || !(lt2 > 0.0)) return 0.0;
  const double sq = l.e * sqrt(disc), ilt2 = fast_rcp(lt2);
  const T mt = T(pp.m_t);
  const double isqs = 1.0 / pp.sqrt_s;
  double acc = 0.0;
  int ns = 0;
  for (int s = 0; s < 2; ++s) {
    const double nz = (aq * l.z + (s ? -sq : sq)) * ilt2;
    v4 nu{0.0, nx, ny, nz};
    nu.e = norm3(nu);
    const double dq = fabs(2.0 * (l.e * nz / nu.e - l.z));
    if (!(dq > 0.0)) continue;
    ++ns;
    const v4 P = add(vis, nu);
    const double Eh = sqrt(P.e * P.e - P.x * P.x - P.y * P.y);
    const double x1 = (Eh + P.z) * isqs, x2 = (Eh - P.z) * isqs;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    const v4 tl4 = add(add(bl, l), nu);
    const double dtl = mdot(tl4, tl4) - pp.m_t * pp.m_t;
    const double bwtl = fast_rcp(dtl * dtl + mtg * mtg);
    TBoost B(P);
    const v4 hqa = B.apply64(qa), hqb = B.apply64(qb), hbh = B.apply64(bh);
    const v4 hbl = B.apply64(bl), hl = B.apply64(l), hn = B.apply64(nu);
    const v4 hh = add(B.apply64(h1), B.apply64(h2));
    const double ak = 0.5 * x1 * pp.sqrt_s, bk = 0.5 * x2 * pp.sqrt_s;
    const double o1 = 1.0 - x1, o2 = 1.0 - x2;
    const T g1 = T(3.0 * o1 * o1 * o1 * o1 * o1), g2 = T(3.0 * o2 * o2 * o2 * o2 * o2);
    const v4& qk = ev.o == 0 ? hqa : hqb;     // quark of the hadronic W
    const v4& qbk = ev.o == 0 ? hqb : hqa;
    const bool lp = ev.charge > 0;
    const v4& tb_ = lp ? hbl : hbh;
    const v4& tf1b = lp ? hl : qbk;
    const v4& tf1 = lp ? hn : qk;
    const v4& ab_ = lp ? hbh : hbl;
    const v4& af2 = lp ? qk : hl;
    const v4& af2b = lp ? qbk : hn;
    const v4 tp = add(add(tb_, tf1b), tf1), tm = add(add(ab_, af2), af2b);
    drow<T> R, C;
    decay_rows<T>(tb_, tf1b, tf1, ab_, af2, af2b, tp, tm, mt, R, C);
    const T me = g1 * g2 * gg_tth_sum<T>(R, C, tp, tm, hh, ak, bk, mt) * T(1.0 / 256.0);
    const double shat = x1 * x2 * pp.S;
    acc += (P.e / Eh) * (double)me * bwtl / (shat * x1 * x2 * dq * nu.e);
  }
  if (nsol_out) *nsol_out = ns;
  return acc * q2h * pp.tth_const * (double)jetf / (2.0 * l.e);
}

}  // namespace memk
