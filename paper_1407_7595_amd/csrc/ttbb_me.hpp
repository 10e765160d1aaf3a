// Tree-level |M|^2 of g(k1, a) g(k2, b) -> t(i) tbar(j) b(k) bbar(l), the
// irreducible background of the t tbar H (H -> b bbar) analysis (Sec. 4),
// with decayed tops (the Dirac row R and column C of decay_rows) and
// massless b quarks, in two-component (Weyl) form.
//
// Feynman rules (couplings stripped): quark-gluon vertex i gamma^mu T^a,
// quark propagator i (pslash + m)/(p^2 - m^2), gluon propagator
// -i g_mu_nu / q^2, triple-gluon vertex f^abc V^{mu nu rho}(k1, k2, k3)
// with V = g^mu_nu (k1-k2)^rho + g^nu_rho (k2-k3)^mu + g^rho_mu (k3-k1)^nu
// (momenta incoming), four-gluon vertex -i [f f (g g - g g) x 3].  The 36
// diagrams fall into six classes: the b pair radiated from the top line
// with both gluons on it (A, 6 orderings) and the mirror image (B, 6); one
// gluon on each line and a gluon exchanged (C, 8); g g -> g* on either line
// (D, 4); one gluon joining the exchanged gluon (E1, 8); both gluons on the
// exchanged gluon, through two triple vertices, one triple vertex after
// g g -> g*, or the four-gluon vertex (E2, 4, the last as its three colour
// terms).
//
// Colour: with T^c_ij T^c_kl = (delta_il delta_kj - delta_ij delta_kl / N)/2
// and f^abc T^c = -i [T^a, T^b], every diagram's colour factor is a
// combination of twelve tensors
//   [P|Q]x = P_il Q_kj  (P, Q) = (ab,1) (ba,1) (1,ab) (1,ba) (a,b) (b,a)  0-5
//   [P|Q]= = P_ij Q_kl  in the same order                                 6-11
// (a = T^a, ab = T^a T^b).  Per helicity the twelve partial sums J_m give
// the colour-summed |A|^2 = sum_mn conj(J_m) G_mn J_n with G the colour
// matrix of the tensors (kColTTBB, filled on the host from explicit SU(3)
// generators).  Helicities: two per gluon, two for the massless b line
// (b and bbar of opposite helicity), one for each V-A top decay chain.
#pragma once
#include "tt_me.hpp"

namespace memk {

__constant__ double kColTTBB[144];
__constant__ float kColTTBBf[144];
template <class T> __device__ __forceinline__ T col_ttbb(int q);
template <> __device__ __forceinline__ double col_ttbb<double>(int q) { return kColTTBB[q]; }
template <> __device__ __forceinline__ float col_ttbb<float>(int q) { return kColTTBBf[q]; }

template <class T> struct cv { cx<T> t, x, y, z; };   // complex four-vector, upper index

template <class T> __device__ __forceinline__ cx<T> mul_i(cx<T> z) { return cx<T>{-z.im, z.re}; }
template <class T> __device__ __forceinline__ cv<T> cvs(cx<T> f, const cv<T>& v)
{
  return cv<T>{f * v.t, f * v.x, f * v.y, f * v.z};
}
template <class T> __device__ __forceinline__ cv<T> cvs(T f, const cv<T>& v)
{
  return cv<T>{f * v.t, f * v.x, f * v.y, f * v.z};
}
template <class T> __device__ __forceinline__ cv<T> cvadd(const cv<T>& a, const cv<T>& b)
{
  return cv<T>{a.t + b.t, a.x + b.x, a.y + b.y, a.z + b.z};
}
template <class T> __device__ __forceinline__ cv<T> cvsub(const cv<T>& a, const cv<T>& b)
{
  return cv<T>{a.t - b.t, a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class T> __device__ __forceinline__ cv<T> cvmom(const mom<T>& p)
{
  return cv<T>{{p.e, T(0)}, {p.x, T(0)}, {p.y, T(0)}, {p.z, T(0)}};
}
template <class T> __device__ __forceinline__ cx<T> cdot(const cv<T>& a, const cv<T>& b)
{
  return a.t * b.t - a.x * b.x - a.y * b.y - a.z * b.z;
}
template <class T> __device__ __forceinline__ cx<T> cdot(const cv<T>& a, const mom<T>& p)
{
  return cx<T>{a.t.re * p.e - a.x.re * p.x - a.y.re * p.y - a.z.re * p.z,
               a.t.im * p.e - a.x.im * p.x - a.y.im * p.y - a.z.im * p.z};
}

// R J-slash for a complex J: (R_R (J.sigma-bar), R_L (J.sigma)) with
// J.sigma = [[J0 - Jz, -Jx + i Jy], [-Jx - i Jy, J0 + Jz]] and
// J.sigma-bar = [[J0 + Jz, Jx - i Jy], [Jx + i Jy, J0 - Jz]]
template <class T>
__device__ __forceinline__ drow<T> row_slash(const drow<T>& R, const cv<T>& J)
{
  const cx<T> iy = mul_i(J.y);
  const cx<T> s00 = J.t - J.z, s01 = iy - J.x, s10 = -(J.x + iy), s11 = J.t + J.z;
  const cx<T> b00 = J.t + J.z, b01 = J.x - iy, b10 = J.x + iy, b11 = J.t - J.z;
  return drow<T>{{R.R.a * b00 + R.R.b * b10, R.R.a * b01 + R.R.b * b11},
                 {R.L.a * s00 + R.L.b * s10, R.L.a * s01 + R.L.b * s11}};
}
// J-slash C: ((J.sigma) C_R, (J.sigma-bar) C_L)
template <class T>
__device__ __forceinline__ drow<T> slash_col(const cv<T>& J, const drow<T>& C)
{
  const cx<T> iy = mul_i(J.y);
  const cx<T> s00 = J.t - J.z, s01 = iy - J.x, s10 = -(J.x + iy), s11 = J.t + J.z;
  const cx<T> b00 = J.t + J.z, b01 = J.x - iy, b10 = J.x + iy, b11 = J.t - J.z;
  return drow<T>{{s00 * C.R.a + s01 * C.R.b, s10 * C.R.a + s11 * C.R.b},
                 {b00 * C.L.a + b01 * C.L.b, b10 * C.L.a + b11 * C.L.b}};
}
// (q-slash + m) C
template <class T>
__device__ __forceinline__ drow<T> prop_col(const mom<T>& q, T m, const drow<T>& C)
{
  const sp<T> l = psig_col(q, C.R);
  const cx<T> b00{q.e + q.z, T(0)}, b01{q.x, -q.y}, b10{q.x, q.y}, b11{q.e - q.z, T(0)};
  return drow<T>{{l.a + m * C.L.a, l.b + m * C.L.b},
                 {b00 * C.L.a + b01 * C.L.b + m * C.R.a, b10 * C.L.a + b11 * C.L.b + m * C.R.b}};
}
// V^mu = R gamma^mu C = R_L sigma^mu C_R + R_R sigma-bar^mu C_L
template <class T>
__device__ __forceinline__ cv<T> vec_rc(const drow<T>& R, const drow<T>& C)
{
  const sp<T> l = R.L, r = R.R, cr = C.R, cl = C.L;
  cv<T> v;
  v.t = (l.a * cr.a + l.b * cr.b) + (r.a * cl.a + r.b * cl.b);
  v.x = (l.a * cr.b + l.b * cr.a) - (r.a * cl.b + r.b * cl.a);
  v.y = mul_i((l.b * cr.a - l.a * cr.b) - (r.b * cl.a - r.a * cl.b));
  v.z = (l.a * cr.a - l.b * cr.b) - (r.a * cl.a - r.b * cl.b);
  return v;
}

// triple-gluon vertex with legs (J1, k1), (J2, k2) and the third leg open
// (incoming momentum k3 = -k1 - k2)
template <class T>
__device__ __forceinline__ cv<T> vertex3(const cv<T>& J1, const mom<T>& k1, const cv<T>& J2, const mom<T>& k2)
{
  const mom<T> d12{k1.e - k2.e, k1.x - k2.x, k1.y - k2.y, k1.z - k2.z};
  const mom<T> d23{k1.e + T(2) * k2.e, k1.x + T(2) * k2.x, k1.y + T(2) * k2.y, k1.z + T(2) * k2.z};
  const mom<T> d31{-T(2) * k1.e - k2.e, -T(2) * k1.x - k2.x, -T(2) * k1.y - k2.y, -T(2) * k1.z - k2.z};
  const cx<T> j12 = cdot(J1, J2), a = cdot(J1, d23), b = cdot(J2, d31);
  return cvadd(cvadd(cvs(j12, cvmom(d12)), cvs(a, J2)), cvs(b, J1));
}

// A fermion line between row R and column C with three, two or one
// current insertions; P1, P2 the internal momenta (outgoing quark momentum
// minus the momenta entered so far), iD their propagator reciprocals.  The
// factors i of the vertices and propagators are included: i, -i and i.
template <class T>
__device__ __forceinline__ cx<T> line3(const drow<T>& R, const drow<T>& C, const cv<T>& J1, const mom<T>& P1,
                                       const cv<T>& J2, const mom<T>& P2, const cv<T>& J3, T m, T iD12)
{
  const drow<T> r = row_prop(row_slash(row_prop(row_slash(R, J1), P1, m), J2), P2, m);
  return mul_i(iD12 * row_col(row_slash(r, J3), C));
}
template <class T>
__device__ __forceinline__ cx<T> line2(const drow<T>& R, const drow<T>& C, const cv<T>& J1, const mom<T>& P1,
                                       const cv<T>& J2, T m, T iD1)
{
  return -mul_i(iD1 * row_col(row_slash(row_prop(row_slash(R, J1), P1, m), J2), C));
}

template <class T>
__device__ __forceinline__ mom<T> tomom(const v4& v) { return mom<T>{T(v.e), T(v.x), T(v.y), T(v.z)}; }

// Colour- and helicity-summed |A|^2 (no couplings, no average).  R, C:
// decayed top row and antitop column; pt, ptb, p5, p6: top, antitop, b and
// bbar momenta (FP64: the propagator denominators are formed in FP64 and
// rounded once); beams k1 = (a,0,0,a), k2 = (bm,0,0,-bm).
template <class T>
__device__ __forceinline__ T gg_ttbb_sum(const drow<T>& R, const drow<T>& C, const v4& pt, const v4& ptb,
                                         const v4& p5, const v4& p6, double a, double bm, T mt)
{
  const double m2 = (double)mt * (double)mt;
  const v4 K1{a, 0.0, 0.0, a}, K2{bm, 0.0, 0.0, -bm};
  const v4 Pb = add(p5, p6), Pt = add(pt, ptb);
  auto sub = [](const v4& u, const v4& w) { return v4{u.e - w.e, u.x - w.x, u.y - w.y, u.z - w.z}; };
  auto neg = [](const v4& u) { return v4{-u.e, -u.x, -u.y, -u.z}; };
  // top line internal momenta: p3-k1, p3-k2, p3+Pb, -p4-Pb, -p4+k2, -p4+k1
  const v4 tq[6] = {sub(pt, K1), sub(pt, K2), add(pt, Pb), sub(neg(ptb), Pb), add(neg(ptb), K2),
                    add(neg(ptb), K1)};
  // b line: p5-k1, p5-k2, p5+Pt, -p6-Pt, -p6+k2, -p6+k1
  const v4 bq[6] = {sub(p5, K1), sub(p5, K2), add(p5, Pt), sub(neg(p6), Pt), add(neg(p6), K2),
                    add(neg(p6), K1)};
  T it[6], ib[6];
  mom<T> tm[6], bmo[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    it[q] = T(fast_rcp(mdot(tq[q], tq[q]) - m2));
    ib[q] = T(fast_rcp(mdot(bq[q], bq[q])));
    tm[q] = tomom<T>(tq[q]);
    bmo[q] = tomom<T>(bq[q]);
  }
  // gluon propagators: Pb^2, Pt^2, (k1+k2)^2, (k_x - Pb)^2, (k_x - Pt)^2
  const T iPb = T(fast_rcp(mdot(Pb, Pb))), iPt = T(fast_rcp(mdot(Pt, Pt))), iS = T(fast_rcp(4.0 * a * bm));
  const v4 qb1 = sub(K1, Pb), qb2 = sub(K2, Pb), qt1 = sub(K1, Pt), qt2 = sub(K2, Pt);
  const T iQb[2] = {T(fast_rcp(mdot(qb1, qb1))), T(fast_rcp(mdot(qb2, qb2)))};
  const T iQt[2] = {T(fast_rcp(mdot(qt1, qt1))), T(fast_rcp(mdot(qt2, qt2)))};
  const mom<T> k[2] = {tomom<T>(K1), tomom<T>(K2)};
  const mom<T> mPb = tomom<T>(neg(Pb)), mPt = tomom<T>(neg(Pt));
  const mom<T> Qb[2] = {tomom<T>(qb1), tomom<T>(qb2)};
  const mom<T> Kt = tomom<T>(add(K1, K2));
  // the top pair's gluon current (1/Pt^2) R gamma C: helicity independent
  const cv<T> Gt = cvs(iPt, vec_rc(R, C));
  // massless b spinors: lambda lambda^dagger = p.sigma; mu = eps^T lambda^*
  const sp<T> l5 = lam<T>(p5), l6 = lam<T>(p6);
  const T s2 = T(0.70710678118654752440);
  const cx<T> zc{T(0), T(0)};
  const sp<T> z2{zc, zc};
  const T h = T(0.5), hn = T(0.5 / 3.0);
  T sum = T(0);
  // helicity loops kept rolled: one copy of the 38 diagrams in registers
#pragma unroll 1
  for (int hb = 0; hb < 2; ++hb) {
    // (U, V) = (ubar_1, v_1) = ((0, lambda5^*), (lambda6, 0)) or
    //          (ubar_2, v_2) = ((eps^T lambda5, 0), (0, eps^T lambda6^*))
    const drow<T> U = hb == 0 ? drow<T>{z2, cj(l5)} : drow<T>{epsT(l5), z2};
    const drow<T> V = hb == 0 ? drow<T>{l6, z2} : drow<T>{z2, epsT(cj(l6))};
    const cv<T> Gb = cvs(iPb, vec_rc(U, V));
#pragma unroll 1
    for (int hh = 0; hh < 4; ++hh) {
      // gluon polarisations (0, 1, +-i, 0)/sqrt2
      const T sy1 = (hh & 1) ? -s2 : s2, sy2 = (hh & 2) ? -s2 : s2;
      const cv<T> e[2] = {cv<T>{zc, {s2, T(0)}, {T(0), sy1}, zc}, cv<T>{zc, {s2, T(0)}, {T(0), sy2}, zc}};
      cx<T> J[12];
#pragma unroll
      for (int m = 0; m < 12; ++m) J[m] = zc;
      // ---- A: orders of (g1, g2, Gb) on the top line
      {
        const cx<T> A0 = line3(R, C, e[0], tm[0], e[1], tm[3], Gb, mt, it[0] * it[3]);   // abc
        const cx<T> A1 = line3(R, C, e[0], tm[0], Gb, tm[4], e[1], mt, it[0] * it[4]);   // acb
        const cx<T> A2 = line3(R, C, e[1], tm[1], e[0], tm[3], Gb, mt, it[1] * it[3]);   // bac
        const cx<T> A3 = line3(R, C, e[1], tm[1], Gb, tm[5], e[0], mt, it[1] * it[5]);   // bca
        const cx<T> A4 = line3(R, C, Gb, tm[2], e[0], tm[4], e[1], mt, it[2] * it[4]);   // cab
        const cx<T> A5 = line3(R, C, Gb, tm[2], e[1], tm[5], e[0], mt, it[2] * it[5]);   // cba
        J[0] = J[0] + h * A0; J[4] = J[4] + h * A1; J[1] = J[1] + h * A2;
        J[5] = J[5] + h * A3; J[2] = J[2] + h * A4; J[3] = J[3] + h * A5;
        J[6] = J[6] - hn * (A0 + A1 + A4);
        J[7] = J[7] - hn * (A2 + A3 + A5);
      }
      // ---- B: orders of (g1, g2, Gt) on the b line
      {
        const cx<T> B0 = line3(U, V, e[0], bmo[0], e[1], bmo[3], Gt, T(0), ib[0] * ib[3]);
        const cx<T> B1 = line3(U, V, e[0], bmo[0], Gt, bmo[4], e[1], T(0), ib[0] * ib[4]);
        const cx<T> B2 = line3(U, V, e[1], bmo[1], e[0], bmo[3], Gt, T(0), ib[1] * ib[3]);
        const cx<T> B3 = line3(U, V, e[1], bmo[1], Gt, bmo[5], e[0], T(0), ib[1] * ib[5]);
        const cx<T> B4 = line3(U, V, Gt, bmo[2], e[0], bmo[4], e[1], T(0), ib[2] * ib[4]);
        const cx<T> B5 = line3(U, V, Gt, bmo[2], e[1], bmo[5], e[0], T(0), ib[2] * ib[5]);
        J[2] = J[2] + h * B0; J[5] = J[5] + h * B1; J[3] = J[3] + h * B2;
        J[4] = J[4] + h * B3; J[0] = J[0] + h * B4; J[1] = J[1] + h * B5;
        J[8] = J[8] - hn * (B0 + B1 + B4);
        J[9] = J[9] - hn * (B2 + B3 + B5);
      }
      // ---- C: gluon x on the top line, y on the b line, a gluon exchanged
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int y = 1 - x;
        // exchanged gluon from the b line, order (y, slot) then (slot, y):
        // -(1/(Q^2 D)) vec(U ey (p5 - k_y), V) / vec(U, (k_y - p6) ey V)
        const int by = y == 0 ? 0 : 1, bs = y == 0 ? 5 : 4;    // p5 - k_y; -p6 + k_y
        const T iQ = iQb[y];
        const cv<T> G0 = cvs(-iQ * ib[by], vec_rc(row_prop(row_slash(U, e[y]), bmo[by], T(0)), V));
        const cv<T> G1 = cvs(-iQ * ib[bs], vec_rc(U, prop_col(bmo[bs], T(0), slash_col(e[y], V))));
        // top line: (x, G): p3 - k_x;  (G, x): -p4 + k_x
        const int tx = x == 0 ? 0 : 1, tg = x == 0 ? 5 : 4;
        const cx<T> C00 = line2(R, C, e[x], tm[tx], G0, mt, it[tx]);
        const cx<T> C01 = line2(R, C, e[x], tm[tx], G1, mt, it[tx]);
        const cx<T> C10 = line2(R, C, G0, tm[tg], e[x], mt, it[tg]);
        const cx<T> C11 = line2(R, C, G1, tm[tg], e[x], mt, it[tg]);
        if (x == 0) {
          J[4] = J[4] + h * C00; J[0] = J[0] + h * C01; J[3] = J[3] + h * C10; J[5] = J[5] + h * C11;
          J[10] = J[10] - hn * (C00 + C01 + C10 + C11);
        } else {
          J[5] = J[5] + h * C00; J[1] = J[1] + h * C01; J[2] = J[2] + h * C10; J[4] = J[4] + h * C11;
          J[11] = J[11] - hn * (C00 + C01 + C10 + C11);
        }
      }
      // ---- D: g g -> g* (G12) with the other pair's gluon, on either line
      const cv<T> G12 = cvs(mul_i(cx<T>{-iS, T(0)}), vertex3(e[0], k[0], e[1], k[1]));
      {
        const cx<T> D0 = mul_i(-line2(R, C, G12, tm[3], Gb, mt, it[3]));          // -i (top: ec)
        const cx<T> D1 = mul_i(-line2(R, C, Gb, tm[2], G12, mt, it[2]));          // -i (top: ce)
        const cx<T> D2 = mul_i(-line2(U, V, G12, bmo[3], Gt, T(0), ib[3]));       // -i (b: ec)
        const cx<T> D3 = mul_i(-line2(U, V, Gt, bmo[2], G12, T(0), ib[2]));       // -i (b: ce)
        J[0] = J[0] + h * (D0 + D3); J[1] = J[1] - h * (D0 + D3);
        J[2] = J[2] + h * (D1 + D2); J[3] = J[3] - h * (D1 + D2);
        J[6] = J[6] - hn * (D0 + D1); J[7] = J[7] + hn * (D0 + D1);
        J[8] = J[8] - hn * (D2 + D3); J[9] = J[9] + hn * (D2 + D3);
      }
      // ---- E1: gluon x joins the exchanged gluon, y on the top / b line
      cv<T> Gxb[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int y = 1 - x;
        Gxb[x] = cvs(mul_i(cx<T>{-iQb[x], T(0)}), vertex3(e[x], k[x], Gb, mPb));
        const cv<T> Gxt = cvs(mul_i(cx<T>{-iQt[x], T(0)}), vertex3(e[x], k[x], Gt, mPt));
        // top line (y, G): p3 - k_y; (G, y): -p4 + k_y
        const int ty = y == 0 ? 0 : 1, tg = y == 0 ? 5 : 4;
        const cx<T> E0 = mul_i(-line2(R, C, e[y], tm[ty], Gxb[x], mt, it[ty]));
        const cx<T> E1 = mul_i(-line2(R, C, Gxb[x], tm[tg], e[y], mt, it[tg]));
        const cx<T> E2 = mul_i(-line2(U, V, e[y], bmo[ty], Gxt, T(0), ib[ty]));
        const cx<T> E3 = mul_i(-line2(U, V, Gxt, bmo[tg], e[y], T(0), ib[tg]));
        if (x == 0) {   // -i h: (X1 - X5), (X4 - X2), (X3 - X4), (X5 - X0)
          J[1] = J[1] + h * E0; J[5] = J[5] - h * E0;
          J[4] = J[4] + h * E1; J[2] = J[2] - h * E1;
          J[3] = J[3] + h * E2; J[4] = J[4] - h * E2;
          J[5] = J[5] + h * E3; J[0] = J[0] - h * E3;
        } else {        // -i h: (X0 - X4), (X5 - X3), (X2 - X5), (X4 - X1)
          J[0] = J[0] + h * E0; J[4] = J[4] - h * E0;
          J[5] = J[5] + h * E1; J[3] = J[3] - h * E1;
          J[2] = J[2] + h * E2; J[5] = J[5] - h * E2;
          J[4] = J[4] + h * E3; J[1] = J[1] - h * E3;
        }
      }
      // ---- E2: one insertion on the top line carrying Pt
      {
        const cx<T> mi_pt{T(0), -iPt};   // -i / Pt^2
        // x then y along the exchanged gluon
        const cv<T> J0 = cvs(mi_pt, vertex3(e[1], k[1], Gxb[0], Qb[0]));   // x = a, y = b
        const cv<T> J1 = cvs(mi_pt, vertex3(e[0], k[0], Gxb[1], Qb[1]));   // x = b, y = a
        // g g -> g* joining the exchanged gluon
        const cv<T> J2 = cvs(mi_pt, vertex3(G12, Kt, Gb, mPb));
        // four-gluon vertex, three colour terms: -i [...] then -i/Pt^2
        const cx<T> e1Gb = cdot(e[0], Gb), e2Gb = cdot(e[1], Gb), e1e2 = cdot(e[0], e[1]);
        const cv<T> X0 = cvsub(cvs(e1Gb, e[1]), cvs(e2Gb, e[0]));
        const cv<T> X1 = cvsub(cvs(e1e2, Gb), cvs(e2Gb, e[0]));
        const cv<T> X2 = cvsub(cvs(e1e2, Gb), cvs(e1Gb, e[1]));
        const T m_pt = -iPt;
        const cx<T> F0 = mul_i(row_col(row_slash(R, J0), C));
        const cx<T> F1 = mul_i(row_col(row_slash(R, J1), C));
        const cx<T> F2 = mul_i(row_col(row_slash(R, J2), C));
        const cx<T> F3 = mul_i(m_pt * row_col(row_slash(R, X0), C));
        const cx<T> F4 = mul_i(m_pt * row_col(row_slash(R, X1), C));
        const cx<T> F5 = mul_i(m_pt * row_col(row_slash(R, X2), C));
        // F0: -h (X1 - X5 - X4 + X2); F1: -h (X0 - X4 - X5 + X3);
        // F2, F3: -h (X0 - X1 - X2 + X3); F4: h (X1 - X5 - X4 + X2);
        // F5: h (X0 - X4 - X5 + X3)
        const cx<T> u = F4 - F0, v = F5 - F1, w = F2 + F3;
        J[0] = J[0] + h * (v - w); J[1] = J[1] + h * (u + w);
        J[2] = J[2] + h * (u + w); J[3] = J[3] + h * (v - w);
        J[4] = J[4] - h * (u + v); J[5] = J[5] - h * (u + v);
      }
      // colour sum
#pragma unroll
      for (int m = 0; m < 12; ++m) {
        cx<T> t = zc;
#pragma unroll
        for (int n = 0; n < 12; ++n) t = t + col_ttbb<T>(m * 12 + n) * J[n];
        sum += J[m].re * t.re + J[m].im * t.im;
      }
    }
  }
  return sum;
}

}  // namespace memk
