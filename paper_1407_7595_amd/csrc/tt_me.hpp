// Tree-level |M|^2 of gg, q qbar -> t tbar -> b l+ nu bbar l- nubar with
// full spin correlations, in two-component (Weyl) spinor form.
//
// The paper evaluates the matrix element inside the integrand kernel for
// every phase-space point (Sec. 4) with generated HELAS-style code.  Here
// the amplitudes are written by hand for this process, exploiting its
// structure:
//  * massless b, l, nu with V-A couplings: each decay chain has a single
//    helicity configuration, and the W current contracted with sigma-bar is
//    the rank-one matrix 2 (eps^T nu*)(l^T eps) (Fierz), so the decayed top
//    acts on the production vertex as one Dirac row
//        R = (m r, r (p_t.sigma)),  r = 2 <b|eps^T|nu*> (eps^T l)^T
//    and the decayed antitop as one Dirac column
//        C = (-(p_tbar.sigma) c, m c),  c = 2 (eps^T lbar*) (nubar^T eps bbar);
//  * gluons along +-z in the frame where the hard system has no transverse
//    momentum: the helicity polarisations make eps.sigma and eps.sigma-bar
//    single-entry 2x2 matrices, and the s-channel triple-gluon term reduces
//    to (eps1.eps2) R (k1 - k2)-slash C / s.
// Colour: A = T^aT^b A12 + T^bT^a A21, summed |A|^2 =
// 16/3 (|A12|^2 + |A21|^2) - 4/3 Re(A12 A21*); q qbar: 2 |A|^2.
// The four Breit-Wigner denominators are NOT included: they cancel against
// the Jacobians of the propagator-aligned maps (Sec. 3).
#pragma once
#include "device_common.hpp"

namespace memk {

// Unit of the momenta and masses that enter |M|^2: 256 GeV.  Without its
// Breit-Wigner denominators the six-fermion |M|^2 is homogeneous of degree
// 8 in momenta and masses.  In GeV its values exceed the FP32 range when a
// neutrino carries several TeV (a far off-shell leptonic W), while in units
// of 256 GeV they sit near 1.  The unit is a power of two, so the rescaling
// is exact and FP64 results do not change.
constexpr double kMeScale = 1.0 / 256.0;       // GeV -> matrix-element units
constexpr double kMeDeg8 = 0x1p64;             // 256^8: |M|^2 back to GeV units

template <class T> struct cx { T re, im; };
template <class T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <class T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <class T> __device__ __forceinline__ T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }

template <class T> struct sp { cx<T> a, b; };   // two-component spinor

// lambda(p): (p.sigma-bar) lambda = 0, lambda lambda^dagger = p.sigma
// (the left-handed massless solution, normalised to |lambda|^2 = 2E).
// E + |p_z| is formed in FP64 (no cancellation); for p_z >= 0
//   lambda = (-p_x n, p_y n; (E + p_z) n, 0),
// otherwise ((E - p_z) n, 0; -p_x n, -p_y n), n = 1/sqrt(E + |p_z|): one
// reciprocal square root and selects, so that the lanes of a wavefront
// with either sign share one path.
template <class T>
__device__ __forceinline__ sp<T> lam(const v4& p)
{
  const bool up = p.z >= 0.0;
  const double ep = p.e + fabs(p.z);
  const double n = fast_rsqrt(ep);
  const T q = T(ep * n), xn = T(-p.x * n), yn = T(p.y * n);
  return up ? sp<T>{{xn, yn}, {q, T(0)}} : sp<T>{{q, T(0)}, {xn, -yn}};
}
// eps^T v with eps = [[0,1],[-1,0]]: (-v_b, v_a)
template <class T> __device__ __forceinline__ sp<T> epsT(sp<T> v) { return sp<T>{-v.b, v.a}; }
template <class T> __device__ __forceinline__ sp<T> cj(sp<T> v) { return sp<T>{conj(v.a), conj(v.b)}; }

// row times (p.sigma) and (p.sigma) times column; p.sigma =
// [[p0-p3, -(p1 - i p2)], [-(p1 + i p2), p0+p3]]
template <class T> struct mom { T e, x, y, z; };
template <class T>
__device__ __forceinline__ sp<T> row_psig(sp<T> r, const mom<T>& p)
{
  cx<T> m00{p.e - p.z, T(0)}, m01{-p.x, p.y}, m10{-p.x, -p.y}, m11{p.e + p.z, T(0)};
  return sp<T>{r.a * m00 + r.b * m10, r.a * m01 + r.b * m11};
}
template <class T>
__device__ __forceinline__ sp<T> psig_col(const mom<T>& p, sp<T> c)
{
  cx<T> m00{p.e - p.z, T(0)}, m01{-p.x, p.y}, m10{-p.x, -p.y}, m11{p.e + p.z, T(0)};
  return sp<T>{m00 * c.a + m01 * c.b, m10 * c.a + m11 * c.b};
}
// (p.sigma-bar) entries: [[p0+p3, p1 - i p2], [p1 + i p2, p0-p3]]

// A momentum by its light-cone components p0 + p3, p0 - p3 and p1, p2,
// formed in FP64 before the rounding to T: for a top far off its mass shell
// p0 - p3 (or p0 + p3) is much smaller than p0, and forming it from
// components already rounded to FP32 loses the digits the amplitudes need.
template <class T> struct lcm { T p, m, x, y; };
template <class T> __device__ __forceinline__ lcm<T> to_lc(const v4& v)
{
  return lcm<T>{T(v.e + v.z), T(v.e - v.z), T(v.x), T(v.y)};
}
template <class T>
__device__ __forceinline__ sp<T> row_psig(sp<T> r, const lcm<T>& p)
{
  cx<T> m00{p.m, T(0)}, m01{-p.x, p.y}, m10{-p.x, -p.y}, m11{p.p, T(0)};
  return sp<T>{r.a * m00 + r.b * m10, r.a * m01 + r.b * m11};
}
template <class T>
__device__ __forceinline__ sp<T> psig_col(const lcm<T>& p, sp<T> c)
{
  cx<T> m00{p.m, T(0)}, m01{-p.x, p.y}, m10{-p.x, -p.y}, m11{p.p, T(0)};
  return sp<T>{m00 * c.a + m01 * c.b, m10 * c.a + m11 * c.b};
}

// Dirac row / column in chiral blocks (L, R)
template <class T> struct drow { sp<T> L, R; };

// Decayed top row and antitop column (see header comment); pt, ptb: the
// top and antitop momenta (FP64, matrix-element units).
template <class T>
__device__ __forceinline__ void decay_rows(const v4& b, const v4& lp, const v4& nu, const v4& bb,
                                           const v4& lm, const v4& nub, const v4& pt64,
                                           const v4& ptb64, T mt, drow<T>& R, drow<T>& C)
{
  const lcm<T> pt = to_lc<T>(pt64), ptb = to_lc<T>(ptb64);
  sp<T> lb = lam<T>(b), ll = lam<T>(lp), ln = lam<T>(nu);
  sp<T> lbb = lam<T>(bb), llm = lam<T>(lm), lnb = lam<T>(nub);
  // r = 2 (lambda_b^dagger eps^T lambda_nu^*) (eps^T lambda_l)^T
  sp<T> al = epsT(cj(ln));
  cx<T> st = T(2) * (conj(lb.a) * al.a + conj(lb.b) * al.b);
  sp<T> be = epsT(ll);
  sp<T> r{st * be.a, st * be.b};
  R.L = sp<T>{mt * r.a, mt * r.b};
  R.R = row_psig(r, pt);
  // c = 2 (eps^T lambda_lm^*) (lambda_nub^T eps lambda_bb)
  sp<T> bq = epsT(lnb);
  cx<T> sb = T(2) * (bq.a * lbb.a + bq.b * lbb.b);
  sp<T> al2 = epsT(cj(llm));
  sp<T> c{sb * al2.a, sb * al2.b};
  sp<T> pc = psig_col(ptb, c);
  C.L = sp<T>{-pc.a, -pc.b};
  C.R = sp<T>{mt * c.a, mt * c.b};
}

template <class T> __device__ __forceinline__ cx<T> dot2(sp<T> r, sp<T> c) { return r.a * c.a + r.b * c.b; }

// R (q-slash + m) ... amplitude of one ordering for gluon helicity labels
// (h1 on the top side, h2 on the antitop side): R e1-slash (q-slash + m)
// e2-slash C.  eps(+) = (0,1,i,0)/sqrt2, eps(-) = (0,1,-i,0)/sqrt2.
template <class T>
__device__ __forceinline__ cx<T> chain_amp(const drow<T>& R, const drow<T>& C, const lcm<T>& q, T mt,
                                           int h1, int h2)
{
  const T s2 = T(1.41421356237309504880);
  // w1 = R_L (e1.sigma), w2 = R_R (e1.sigma-bar): one nonzero entry each
  //  h = +: e.sigma = [[0,-s2],[0,0]], e.sigma-bar = [[0,s2],[0,0]]
  //  h = -: e.sigma = [[0,0],[-s2,0]], e.sigma-bar = [[0,0],[s2,0]]
  // u1 = (e2.sigma-bar) C_L, u2 = (e2.sigma) C_R
  // A = w1 . (m u1 + Qbar u2) + w2 . (Q u1 + m u2)
  cx<T> w1, w2;       // the single nonzero entry; index = (h1 == + ? 1 : 0)
  cx<T> u1, u2;       // single nonzero entry; index = (h2 == + ? 0 : 1)
  if (h1 == 0) { w1 = -s2 * R.L.a; w2 = s2 * R.R.a; } else { w1 = -s2 * R.L.b; w2 = s2 * R.R.b; }
  if (h2 == 0) { u1 = s2 * C.L.b; u2 = -s2 * C.R.b; } else { u1 = s2 * C.L.a; u2 = -s2 * C.R.a; }
  const int iw = (h1 == 0) ? 1 : 0;   // column of w
  const int iu = (h2 == 0) ? 0 : 1;   // row of u
  // Q = q.sigma, Qbar = q.sigma-bar, entry [iw][iu]
  cx<T> Q, Qb;
  if (iw == 0 && iu == 0) { Q = cx<T>{q.m, T(0)}; Qb = cx<T>{q.p, T(0)}; }
  else if (iw == 0 && iu == 1) { Q = cx<T>{-q.x, q.y}; Qb = cx<T>{q.x, -q.y}; }
  else if (iw == 1 && iu == 0) { Q = cx<T>{-q.x, -q.y}; Qb = cx<T>{q.x, q.y}; }
  else { Q = cx<T>{q.p, T(0)}; Qb = cx<T>{q.m, T(0)}; }
  // w . (m u1 e_iu + Qbar[:,iu] u2): only component iw of the vector matters
  cx<T> v1 = (iw == iu) ? (mt * u1 + Qb * u2) : (Qb * u2);
  cx<T> v2 = (iw == iu) ? (Q * u1 + mt * u2) : (Q * u1);
  return w1 * v1 + w2 * v2;
}

// sum over gluon helicities and colours of |A|^2 for g(k1) g(k2) -> t tbar
// (k1 = (a,0,0,a), k2 = (bm,0,0,-bm)); R, C from decay_rows; pt the top
// momentum (FP64).  The internal top momenta p_t - k_i and their propagator
// denominators (p_t - k_i)^2 - m^2 = (p_t^2 - m^2) - 2 p_t.k_i are formed in
// FP64: far off the top's mass shell single diagrams grow while their sum
// does not, and FP32 rounding of these inputs would show in the sum.
template <class T>
__device__ __forceinline__ T gg_sum(const drow<T>& R, const drow<T>& C, const v4& pt, double a, double bm, T mt)
{
  const double pp = pt.e + pt.z, pm = pt.e - pt.z;
  const lcm<T> q1{T(pp - 2.0 * a), T(pm), T(pt.x), T(pt.y)};     // p_t - k1
  const lcm<T> q2{T(pp), T(pm - 2.0 * bm), T(pt.x), T(pt.y)};    // p_t - k2
  const double off = mdot(pt, pt) - (double)mt * (double)mt;
  const T iDt = rcp_t(T(off - 2.0 * a * pm)), iDu = rcp_t(T(off - 2.0 * bm * pp));
  const T s = T(4.0 * a * bm);
  // R (k1-k2)-slash C = R_L (K.sigma) C_R + R_R (K.sigma-bar) C_L,
  // K.sigma = diag(-2bm, 2a), K.sigma-bar = diag(2a, -2bm)
  const T a2 = T(2.0 * a), b2 = T(-2.0 * bm);
  cx<T> rkc = b2 * (R.L.a * C.R.a) + a2 * (R.L.b * C.R.b) + a2 * (R.R.a * C.L.a) + b2 * (R.R.b * C.L.b);
  cx<T> sch = rcp_t(s) * rkc;
  T sum = T(0);
#pragma unroll
  for (int h1 = 0; h1 < 2; ++h1)
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      cx<T> at = iDt * chain_amp(R, C, q1, mt, h1, h2);
      cx<T> au = iDu * chain_amp(R, C, q2, mt, h2, h1);
      // eps1.eps2 = -1 for opposite labels, 0 for equal ones
      cx<T> a12 = (h1 != h2) ? at - sch : at;
      cx<T> a21 = (h1 != h2) ? au + sch : au;
      cx<T> x = a12 * conj(a21);
      sum += T(16.0 / 3.0) * (abs2(a12) + abs2(a21)) - T(4.0 / 3.0) * x.re;
    }
  return sum;
}

// q qbar -> t tbar through one s-channel gluon, summed over the two
// non-vanishing quark helicities and colours (factor 2), for beams along
// +-z: k1 = (a,0,0,a), k2 = (bm,0,0,-bm).  The quark currents are
//   left:  J.sigma-bar = 2 (eps^T lqb*)(lq^T eps),  J.sigma = 2 lq lqb^dagger
//   right: J.sigma = 2 (eps^T ltqb*)(ltq^T eps),    J.sigma-bar = 2 ltq ltqb^dagger
// and R J-slash C = R_L (J.sigma) C_R + R_R (J.sigma-bar) C_L.  With the
// beam spinors written out (lambda(k1) = (0, al), lambda~(k1) = (al, 0),
// lambda(k2) = (be, 0), lambda~(k2) = (0, be), al = sqrt(2a), be = sqrt(2bm))
// the two helicity amplitudes of a quark along +z are
//   A_L = 2 al be X,  X = R_L.b C_R.a - R_R.b C_L.a,
//   A_R = 2 al be Y,  Y = R_R.a C_L.b - R_L.a C_R.b,
// and for the quark along -z they are -A_R and -A_L: both orderings give
//   2 (|A_L|^2 + |A_R|^2) / s^2 = 8 (|X|^2 + |Y|^2) / s,  s = 4 a bm,
// with no square roots.
template <class T>
__device__ __forceinline__ T qq_beams(const drow<T>& R, const drow<T>& C, T a, T bm)
{
  const cx<T> X = R.L.b * C.R.a - R.R.b * C.L.a;
  const cx<T> Y = R.R.a * C.L.b - R.L.a * C.R.b;
  return T(8) * (abs2(X) + abs2(Y)) * rcp_t(T(4) * a * bm);
}

// ------------------------------------------------------------ t tbar H --
// Generic Dirac-row operations for chains with a Higgs insertion.
// p.sigma-bar = [[p0+p3, p1 - i p2], [p1 + i p2, p0-p3]]
template <class T>
__device__ __forceinline__ sp<T> row_psigbar(sp<T> r, const mom<T>& p)
{
  cx<T> m00{p.e + p.z, T(0)}, m01{p.x, -p.y}, m10{p.x, p.y}, m11{p.e - p.z, T(0)};
  return sp<T>{r.a * m00 + r.b * m10, r.a * m01 + r.b * m11};
}
// R (q-slash + m)
template <class T>
__device__ __forceinline__ drow<T> row_prop(const drow<T>& R, const mom<T>& q, T m)
{
  sp<T> l = row_psigbar(R.R, q), r = row_psig(R.L, q);
  return drow<T>{{m * R.L.a + l.a, m * R.L.b + l.b}, {r.a + m * R.R.a, r.b + m * R.R.b}};
}
template <class T>
__device__ __forceinline__ drow<T> row_scale(const drow<T>& R, T f)
{
  return drow<T>{{f * R.L.a, f * R.L.b}, {f * R.R.a, f * R.R.b}};
}
// R eps-slash for a gluon along +-z with helicity label h (0: +, 1: -):
// (R_R (e.sigma-bar), R_L (e.sigma)), one nonzero entry each
template <class T>
__device__ __forceinline__ drow<T> row_eps(const drow<T>& R, int h)
{
  const T s2 = T(1.41421356237309504880);
  const cx<T> z{T(0), T(0)};
  if (h == 0) return drow<T>{{z, s2 * R.R.a}, {z, -s2 * R.L.a}};
  return drow<T>{{s2 * R.R.b, z}, {-s2 * R.L.b, z}};
}
// R (k1 - k2)-slash, k1 = (a,0,0,a), k2 = (bm,0,0,-bm)
template <class T>
__device__ __forceinline__ drow<T> row_kslash(const drow<T>& R, T a, T bm)
{
  return drow<T>{{(T(2) * a) * R.R.a, (T(-2) * bm) * R.R.b}, {(T(-2) * bm) * R.L.a, (T(2) * a) * R.L.b}};
}
template <class T> __device__ __forceinline__ cx<T> row_col(const drow<T>& R, const drow<T>& C)
{
  return dot2(R.L, C.L) + dot2(R.R, C.R);
}
template <class T> __device__ __forceinline__ T mom2(const mom<T>& q) { return q.e * q.e - q.x * q.x - q.y * q.y - q.z * q.z; }
template <class T> __device__ __forceinline__ mom<T> madd(const mom<T>& a, const mom<T>& b, T f)
{
  return mom<T>{a.e + f * b.e, a.x + f * b.x, a.y + f * b.y, a.z + f * b.z};
}

// Sum over gluon helicities and colours of |A|^2 for g(k1) g(k2) -> t tbar H
// with unit Yukawa vertex: the Higgs at every position of the top line of
// the three gg -> t tbar diagrams (8 diagrams), colour orderings as gg_sum.
// pt, ptb: top and antitop momenta; ph: Higgs momentum (FP64: the internal
// momenta and their propagator denominators are formed in FP64, where
// (p_t + p_H)^2 - m_t^2 would lose digits to cancellation in FP32).
template <class T>
__device__ __forceinline__ T gg_tth_sum(const drow<T>& R, const drow<T>& C, const v4& pt, const v4& ptb,
                                        const v4& ph, double a, double bm, T mt)
{
  const double m2 = (double)mt * (double)mt;
  const v4 qa = add(pt, ph);                                      // H next to the top
  const v4 qc{-ptb.e - ph.e, -ptb.x - ph.x, -ptb.y - ph.y, -ptb.z - ph.z};   // H next to the antitop
  const v4 q1{pt.e - a, pt.x, pt.y, pt.z - a}, q2{pt.e - bm, pt.x, pt.y, pt.z + bm};   // pt - k_i
  const v4 q1h = add(q1, ph), q2h = add(q2, ph);                  // pt - k_i + ph
  auto to = [](const v4& v) { return mom<T>{T(v.e), T(v.x), T(v.y), T(v.z)}; };
  const T iDa = T(fast_rcp(mdot(qa, qa) - m2)), iDc = T(fast_rcp(mdot(qc, qc) - m2));
  const T iD1 = T(fast_rcp(mdot(q1, q1) - m2)), iD2 = T(fast_rcp(mdot(q2, q2) - m2));
  const T iD1h = T(fast_rcp(mdot(q1h, q1h) - m2)), iD2h = T(fast_rcp(mdot(q2h, q2h) - m2));
  const T s = T(4.0 * a * bm);
  const T ta = T(a), tbm = T(bm);
  const mom<T> qaT = to(qa), qcT = to(qc), q1T = to(q1), q2T = to(q2), q1hT = to(q1h), q2hT = to(q2h);
  const drow<T> Sa = row_scale(row_prop(R, qaT, mt), iDa);     // R S(pt + ph)
  // s-channel current with the Higgs on either side of it
  const cx<T> sch = rcp_t(s) * (row_col(row_kslash(Sa, ta, tbm), C)
                                 + iDc * row_col(row_prop(row_kslash(R, ta, tbm), qcT, mt), C));
  T sum = T(0);
#pragma unroll
  for (int h1 = 0; h1 < 2; ++h1)
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      // ordering 12: gluon 1 next to the top
      const drow<T> e1 = row_eps(R, h1);
      const drow<T> e1q = row_prop(e1, q1T, mt);                // R e1 (pt - k1 + m)
      cx<T> a12 = (iD1h) * row_col(row_eps(row_prop(row_eps(Sa, h1), q1hT, mt), h2), C);
      a12 = a12 + (iD1 * iD1h) * row_col(row_eps(row_prop(e1q, q1hT, mt), h2), C);
      a12 = a12 + (iD1 * iDc) * row_col(row_prop(row_eps(e1q, h2), qcT, mt), C);
      // ordering 21: gluon 2 next to the top
      const drow<T> e2 = row_eps(R, h2);
      const drow<T> e2q = row_prop(e2, q2T, mt);
      cx<T> a21 = (iD2h) * row_col(row_eps(row_prop(row_eps(Sa, h2), q2hT, mt), h1), C);
      a21 = a21 + (iD2 * iD2h) * row_col(row_eps(row_prop(e2q, q2hT, mt), h1), C);
      a21 = a21 + (iD2 * iDc) * row_col(row_prop(row_eps(e2q, h1), qcT, mt), C);
      // eps1.eps2 = -1 for opposite labels, 0 for equal ones
      if (h1 != h2) { a12 = a12 - sch; a21 = a21 + sch; }
      const cx<T> x = a12 * conj(a21);
      sum += T(16.0 / 3.0) * (abs2(a12) + abs2(a21)) - T(4.0 / 3.0) * x.re;
    }
  return sum;
}

}  // namespace memk
