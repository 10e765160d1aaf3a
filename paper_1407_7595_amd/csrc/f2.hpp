// The t tbar H (H -> b bbar) signal and the t tbar b bbar background in the
// dilepton channel, each tt decaying to b l+ nu bbar l- nubar: Sec. 4's
// analysis with its 8-dimensional integration (Eq. integrand).
//
// Event objects: four b-jets (rows 0-3), l+ (row 4), l- (row 5).
// Assignments (the outer sum of Eq. integrand), rows of (b, bbar, pair 1,
// pair 2):
//   t tbar H, 12: perm = 2 hp + s; the Higgs pair is the hp-th of the six
//     ascending jet pairs; the other two jets, ascending, go to (b, bbar)
//     for s = 0 and to (bbar, b) for s = 1;
//   t tbar b bbar, 24: the perm-th permutation, lexicographic, of the four
//     jets onto (b, bbar, b', bbar').
// Variables x in [0,1]^8:
//   x0, x1  r = E_meas / E of the b and bbar jets
//   x2..x5  q2 of t, tbar, W+, W- (tan maps; the four Breit-Wigner
//           factors cancel against the map Jacobians), Eq. dilepsolv
//   x6      r of pair jet 1
//   x7      t tbar H: q2 of the Higgs (tan map, Eq. mhsolve) giving the
//           energy of pair jet 2 (its Breit-Wigner cancels as well);
//           t tbar b bbar: r of pair jet 2.
// All four jets carry the b-jet transfer function.  The two neutrinos'
// transverse momenta add up to minus that of the visible objects
// (transverse momentum balance; no recoil integration).  gg initial state.
#pragma once
#include "device_common.hpp"
#include "process.hpp"
#include "tt.hpp"
#include "tt_me.hpp"
#include "tt_solve.hpp"
#include "ttbb_me.hpp"

namespace memk {

struct F2Event {
  double n[4][3];      // unit directions of the jets in role order
  double em[4];        // measured energies
  double sin_th[4];
  v4 lp, lm;
  double lep_fac;      // 1 / (2E_l+ 2E_l-)
};

__device__ __forceinline__ void f2_rows(bool tth, int perm, int (&rows)[4])
{
  if (tth) {
    const int hp = perm >> 1, s = perm & 1;
    // pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
    const int h1 = hp < 3 ? 0 : hp < 5 ? 1 : 2;
    const int h2 = hp < 3 ? hp + 1 : hp < 5 ? hp - 1 : 3;
    int o0 = -1, o1 = -1;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j != h1 && j != h2) { if (o0 < 0) o0 = j; else o1 = j; }
    rows[0] = s ? o1 : o0;
    rows[1] = s ? o0 : o1;
    rows[2] = h1;
    rows[3] = h2;
    return;
  }
  // factorial number system: digits 3! 2! 1! 0! pick from the remaining jets
  int avail = 0x3210, r = perm;
  const int fact[4] = {6, 2, 1, 1};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = r / fact[k];
    r -= q * fact[k];
    rows[k] = (avail >> (4 * q)) & 0xF;
    // drop digit q
    const int low = avail & ((1 << (4 * q)) - 1);
    avail = low | ((avail >> (4 * (q + 1))) << (4 * q));
  }
}

__device__ __forceinline__ void f2_load(const EventsView& ev, bool tth, int e, int perm, F2Event& t)
{
  int rows[4];
  f2_rows(tth, perm, rows);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double E, x, y, z;
    ev.load(rows[k], e, E, x, y, z);
    const double p = sqrt(x * x + y * y + z * z);
    t.em[k] = E;
    t.n[k][0] = x / p; t.n[k][1] = y / p; t.n[k][2] = z / p;
    t.sin_th[k] = sqrt(x * x + y * y) / p;
  }
  ev.load(4, e, t.lp.e, t.lp.x, t.lp.y, t.lp.z);
  ev.load(5, e, t.lm.e, t.lm.x, t.lm.y, t.lm.z);
  t.lep_fac = 1.0 / (4.0 * t.lp.e * t.lm.e);
}

// |M|^2 units: the momenta enter in units of 256 GeV (kMeScale).  Without
// its Breit-Wigner denominators, |M|^2 is homogeneous in momenta and masses
// of degree 6 for t tbar H (one top propagator more than t tbar: 256^6 =
// 2^48) and of degree 4 for t tbar b bbar (a top propagator and the b
// pair's current over a gluon propagator more: 256^4 = 2^32).
constexpr double kMeDeg6 = 0x1p48;
constexpr double kMeDeg4 = 0x1p32;

template <class T, bool TTH>
__device__ __forceinline__ double f2_integrand(const ProcParams& pp, const F2Event& ev, const double (&x)[8],
                                               int* nsol_out)
{
  if (nsol_out) *nsol_out = 0;
  const TFParams& tf = pp.tf_b;
  double E[4];
  T jetf = T(1);
  const int xr[3] = {0, 1, 6};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double r = tf.r_lo + x[xr[k]] * (tf.r_hi - tf.r_lo), ir = fast_rcp(r);
    E[k] = ev.em[k] * ir;
    jetf *= T(ev.sin_th[k] * (tf.r_hi - tf.r_lo) * E[k] * ir * 0.5) * tf_r<T>(T(r), tf);
  }
  double q2h = 1.0;
  if constexpr (TTH) {
    // Eq. mhsolve: the second Higgs jet's energy from the Higgs virtuality
    const double mhg = pp.m_h * pp.w_h;
    q2h = pp.m_h * pp.m_h + mhg * tan_halfpi(pp.th0_h + x[7] * (pp.th1_h - pp.th0_h));
    const double omc = 1.0 - (ev.n[2][0] * ev.n[3][0] + ev.n[2][1] * ev.n[3][1] + ev.n[2][2] * ev.n[3][2]);
    if (!(omc > 0.0)) return 0.0;
    const double dE = fast_rcp(2.0 * E[2] * omc);
    E[3] = q2h * dE;
    const double r3 = ev.em[3] / E[3];
    if (r3 < tf.r_lo || r3 > tf.r_hi) return 0.0;
    jetf *= T(0.5 * ev.sin_th[3] * dE) * tf_r<T>(T(r3), tf);
  } else {
    const double r = tf.r_lo + x[7] * (tf.r_hi - tf.r_lo), ir = fast_rcp(r);
    E[3] = ev.em[3] * ir;
    jetf *= T(ev.sin_th[3] * (tf.r_hi - tf.r_lo) * E[3] * ir * 0.5) * tf_r<T>(T(r), tf);
  }
  v4 j[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) j[k] = v4{E[k], E[k] * ev.n[k][0], E[k] * ev.n[k][1], E[k] * ev.n[k][2]};
  const double mtg = pp.m_t * pp.w_t, mwg = pp.m_w * pp.w_w;
  const double q2t = pp.m_t * pp.m_t + mtg * tan_halfpi(pp.th0_t + x[2] * (pp.th1_t - pp.th0_t));
  const double q2tb = pp.m_t * pp.m_t + mtg * tan_halfpi(pp.th0_t + x[3] * (pp.th1_t - pp.th0_t));
  const double q2wp = pp.m_w * pp.m_w + mwg * tan_halfpi(pp.th0_w + x[4] * (pp.th1_w - pp.th0_w));
  const double q2wm = pp.m_w * pp.m_w + mwg * tan_halfpi(pp.th0_w + x[5] * (pp.th1_w - pp.th0_w));
  const v4 vis = add(add(add(j[0], j[1]), add(j[2], j[3])), add(ev.lp, ev.lm));
  NuSet sols;
  solve_dilepton(j[0], j[1], ev.lp, ev.lm, -vis.x, -vis.y, q2wp, q2t, q2wm, q2tb, sols, polish_tol<T>());
  const int ns = sols.n;
  const T mt = T(pp.m_t * kMeScale);
  double acc = 0.0;
  for (int s = 0; s < ns; ++s) {
    const NuSol sk = sols.get(s);
    v4 nu{0.0, sk.nx, sk.ny, sk.nz}, nb{0.0, sk.bx, sk.by, sk.bz};
    nu.e = norm3(nu);
    nb.e = norm3(nb);
    const v4 P = add(vis, add(nu, nb));
    const double Eh = sqrt(P.e * P.e - P.x * P.x - P.y * P.y);
    const double x1 = (Eh + P.z) * pp.inv_sqrt_s, x2 = (Eh - P.z) * pp.inv_sqrt_s;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    T gg, qq12, qq21;
    tt_lumis<T>(pp, x1, x2, gg, qq12, qq21);
    TBoost B(P);
    const v4 hb = B.apply_me(j[0]), hl = B.apply_me(ev.lp), hn = B.apply_me(nu);
    const v4 hbb = B.apply_me(j[1]), hlm = B.apply_me(ev.lm), hnb = B.apply_me(nb);
    const v4 h1 = B.apply_me(j[2]), h2 = B.apply_me(j[3]);
    const v4 tp = add(add(hb, hl), hn), tm = add(add(hbb, hlm), hnb);
    drow<T> R, C;
    decay_rows<T>(hb, hl, hn, hbb, hlm, hnb, tp, tm, mt, R, C);
    const double a = 0.5 * x1 * pp.sqrt_s * kMeScale, bm = 0.5 * x2 * pp.sqrt_s * kMeScale;
    double me;
    if constexpr (TTH)
      me = (double)(gg * gg_tth_sum<T>(R, C, tp, tm, add(h1, h2), a, bm, mt)) * kMeDeg6;
    else
      me = (double)(gg * gg_ttbb_sum<T>(R, C, tp, tm, h1, h2, a, bm, mt)) * kMeDeg4;
    const double shat = x1 * x2 * pp.S;
    acc += P.e * me * fast_rcp(Eh * shat * x1 * x2 * sk.adet * nu.e * nb.e);
  }
  if (nsol_out) *nsol_out = ns;
  return acc * pp.f2_const * q2h * ev.lep_fac * (double)jetf;
}

// Parton level (Sec. 4's Table 2 workload): the transfer functions are
// delta functions, so the weight of an assignment is (2/S) (E / E') times
// the complete |M|^2 and densities over 2 shat x1 x2 (x f form); the four
// top and W Breit-Wigner factors (and the Higgs one with its q2_H) are
// evaluated, f2_parton_const holds the couplings.  o: b quarks 0-3, l+, l-,
// nu, nubar; the weight is the mean over the assignments.
__device__ __forceinline__ v4 pick4(const v4& a, const v4& b, const v4& c, const v4& d, int r)
{
  return r == 0 ? a : r == 1 ? b : r == 2 ? c : d;
}

template <class T, bool TTH>
__device__ __forceinline__ double f2_parton(const ProcParams& pp, const v4 (&o)[8])
{
  constexpr int n = TTH ? 12 : 24;
  const T mt = T(pp.m_t * kMeScale);
  double sum = 0.0;
#pragma unroll 1
  for (int perm = 0; perm < n; ++perm) {
    int rows[4];
    f2_rows(TTH, perm, rows);
    const v4 b0 = pick4(o[0], o[1], o[2], o[3], rows[0]), b1 = pick4(o[0], o[1], o[2], o[3], rows[1]);
    const v4 q1 = pick4(o[0], o[1], o[2], o[3], rows[2]), q2 = pick4(o[0], o[1], o[2], o[3], rows[3]);
    const v4 P = add(add(add(b0, b1), add(q1, q2)), add(add(o[4], o[5]), add(o[6], o[7])));
    const double Eh = sqrt(P.e * P.e - P.x * P.x - P.y * P.y);
    const double x1 = (Eh + P.z) * pp.inv_sqrt_s, x2 = (Eh - P.z) * pp.inv_sqrt_s;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    T gg, qq12, qq21;
    tt_lumis<T>(pp, x1, x2, gg, qq12, qq21);
    TBoost B(P);
    const v4 hb = B.apply_me(b0), hl = B.apply_me(o[4]), hn = B.apply_me(o[6]);
    const v4 hbb = B.apply_me(b1), hlm = B.apply_me(o[5]), hnb = B.apply_me(o[7]);
    const v4 h1 = B.apply_me(q1), h2 = B.apply_me(q2);
    const v4 tp = add(add(hb, hl), hn), tm = add(add(hbb, hlm), hnb);
    drow<T> R, C;
    decay_rows<T>(hb, hl, hn, hbb, hlm, hnb, tp, tm, mt, R, C);
    const double a = 0.5 * x1 * pp.sqrt_s * kMeScale, bm = 0.5 * x2 * pp.sqrt_s * kMeScale;
    const v4 wp = add(o[4], o[6]), wm = add(o[5], o[7]), t = add(b0, wp), tb = add(b1, wm);
    double bw = bw_factor(mdot(t, t), pp.m_t, pp.w_t) * bw_factor(mdot(tb, tb), pp.m_t, pp.w_t)
              * bw_factor(mdot(wp, wp), pp.m_w, pp.w_w) * bw_factor(mdot(wm, wm), pp.m_w, pp.w_w);
    double me;
    if constexpr (TTH) {
      // massless b quarks: (p1 + p2)^2 = 2 p1.p2
      const double q2h = 2.0 * (q1.e * q2.e - q1.x * q2.x - q1.y * q2.y - q1.z * q2.z);
      bw *= q2h * bw_factor(q2h, pp.m_h, pp.w_h);
      me = (double)(gg * gg_tth_sum<T>(R, C, tp, tm, add(h1, h2), a, bm, mt)) * kMeDeg6;
    } else {
      me = (double)(gg * gg_ttbb_sum<T>(R, C, tp, tm, h1, h2, a, bm, mt)) * kMeDeg4;
    }
    const double shat = x1 * x2 * pp.S;
    sum += P.e * me * bw * fast_rcp(Eh * 2.0 * shat * x1 * x2);
  }
  return sum * (2.0 * pp.inv_sqrt_s * pp.inv_sqrt_s) * pp.f2_parton_const / n;
}

}  // namespace memk
