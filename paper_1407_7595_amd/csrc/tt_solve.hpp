// FP64 solution of the dilepton constraint system (Sec. 3, Eq. dilepsolv).
//
// Given the b and lepton momenta, the two W and two top virtualities and the
// transverse momentum carried by the neutrino pair, each top side gives two
// linear equations in (E, p) of its (massless) neutrino, so E and p_z are
// affine in (p_x, p_y) and the mass shell is a conic.  The antineutrino's
// (p_x, p_y) is the transverse balance minus the neutrino's, so both conics
// live in the same plane; eliminating p_y with their resultant leaves a
// quartic in p_x (the analytic route of Sonnenschein).  Real roots are
// isolated between the real roots of the derivative (themselves isolated by
// the second derivative) and refined by bracketed Newton; each candidate is
// polished by two Newton steps on the full 4x4 system.  Everything runs in
// FP64: the coefficients cancel strongly (Sec. 4).
#pragma once
#include "device_common.hpp"

namespace memk {

// p(t) = c0 + c1 t + ... + cN t^N
template <int N>
__device__ __forceinline__ double horner(const double (&c)[N + 1], double t)
{
  double r = c[N];
#pragma unroll
  for (int i = N - 1; i >= 0; --i) r = __fma_rn(r, t, c[i]);
  return r;
}
template <int N>
__device__ __forceinline__ void horner_d(const double (&c)[N + 1], double t, double& f, double& df)
{
  f = c[N];
  df = 0.0;
#pragma unroll
  for (int i = N - 1; i >= 0; --i) { df = __fma_rn(df, t, f); f = __fma_rn(f, t, c[i]); }
}

// Root of a polynomial that is monotone on [lo, hi] with a sign change:
// Newton steps, falling back to bisection whenever a step leaves the bracket.
template <int N>
__device__ __forceinline__ double bracketed_root(const double (&c)[N + 1], double lo, double hi, double flo)
{
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 80; ++it) {
    double f, df;
    horner_d<N>(c, x, f, df);
    if (f == 0.0) return x;
    if ((f < 0.0) == (flo < 0.0)) lo = x; else hi = x;
    double xn = x - f / df;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (fabs(xn - x) <= 4e-16 * fabs(x) + 1e-300 || !(hi > lo)) return xn;
    x = xn;
  }
  return x;
}

// Real roots of a quartic (c4 != 0), ascending; returns the count.
__device__ __forceinline__ int quartic_real_roots(const double (&c_in)[5], double (&root)[4])
{
  double inv = 1.0 / c_in[4];
  double c[5] = {c_in[0] * inv, c_in[1] * inv, c_in[2] * inv, c_in[3] * inv, 1.0};
  double bound = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) bound = fmax(bound, fabs(c[i]));
  bound += 1.0;
  // derivatives
  double d1[4] = {c[1], 2.0 * c[2], 3.0 * c[3], 4.0};
  double d2[3] = {2.0 * c[2], 6.0 * c[3], 12.0};
  // roots of the second derivative (closed form, stable)
  double s[2];
  int ns = 0;
  {
    double disc = d2[1] * d2[1] - 4.0 * d2[2] * d2[0];
    if (disc > 0.0) {
      double q = -0.5 * (d2[1] + copysign(sqrt(disc), d2[1]));
      double a = q / d2[2], b = (q != 0.0) ? d2[0] / q : a;
      s[0] = fmin(a, b); s[1] = fmax(a, b);
      ns = 2;
    }
  }
  // the first derivative is monotone between consecutive points of
  // {-bound, s.., bound}: at most one critical point of the quartic each
  double crit[3];
  int nc = 0;
  {
    double pts[4];
    int np = 0;
    pts[np++] = -bound;
    for (int i = 0; i < ns; ++i) if (s[i] > -bound && s[i] < bound) pts[np++] = s[i];
    pts[np++] = bound;
    double fprev = horner<3>(d1, pts[0]);
    for (int i = 0; i + 1 < np; ++i) {
      double fnext = horner<3>(d1, pts[i + 1]);
      if (fprev == 0.0) crit[nc++] = pts[i];
      else if ((fprev < 0.0) != (fnext < 0.0) && fnext != 0.0)
        crit[nc++] = bracketed_root<3>(d1, pts[i], pts[i + 1], fprev);
      fprev = fnext;
    }
  }
  // the quartic is monotone between consecutive critical points
  int nr = 0;
  double pts[5];
  int np = 0;
  pts[np++] = -bound;
  for (int i = 0; i < nc; ++i) pts[np++] = crit[i];
  pts[np++] = bound;
  double fprev = horner<4>(c, pts[0]);
  for (int i = 0; i + 1 < np; ++i) {
    double fnext = horner<4>(c, pts[i + 1]);
    if (fprev == 0.0) { if (nr < 4) root[nr++] = pts[i]; }
    else if ((fprev < 0.0) != (fnext < 0.0) && fnext != 0.0) {
      if (nr < 4) root[nr++] = bracketed_root<4>(c, pts[i], pts[i + 1], fprev);
    }
    fprev = fnext;
  }
  return nr;
}

// Neutrino energy and p_z as affine functions of (p_x, p_y) from
// 2 l.nu = q2w and 2 b.nu = q2t - q2w - 2 b.l (massless b, l, nu).
struct Affine { double e0, e1, e2, z0, z1, z2; };

__device__ __forceinline__ bool nu_affine(const v4& b, const v4& l, double q2w, double q2t, Affine& a)
{
  double h1 = 0.5 * q2w;
  double h2 = 0.5 * (q2t - q2w) - mdot(b, l);
  double det = l.z * b.e - l.e * b.z;
  if (det == 0.0) return false;
  double id = 1.0 / det;
  a.e0 = (l.z * h2 - b.z * h1) * id;
  a.e1 = (l.z * b.x - b.z * l.x) * id;
  a.e2 = (l.z * b.y - b.z * l.y) * id;
  a.z0 = (l.e * h2 - b.e * h1) * id;
  a.z1 = (l.e * b.x - b.e * l.x) * id;
  a.z2 = (l.e * b.y - b.e * l.y) * id;
  return true;
}

// 4x4 Gaussian elimination with partial pivoting, all indexing static.
// Returns det(A); if solve, overwrites r with A^-1 r.
__device__ __forceinline__ double det_solve4(double (&A)[4][4], double (&r)[4], bool solve)
{
  double det = 1.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    // pivot: bring the largest |A[k][c]|, k >= c, to row c
#pragma unroll
    for (int k = c + 1; k < 4; ++k) {
      if (fabs(A[k][c]) > fabs(A[c][c])) {
#pragma unroll
        for (int j = 0; j < 4; ++j) { double t = A[c][j]; A[c][j] = A[k][j]; A[k][j] = t; }
        double t = r[c]; r[c] = r[k]; r[k] = t;
        det = -det;
      }
    }
    double piv = A[c][c];
    det *= piv;
    if (piv == 0.0) return 0.0;
    double ip = 1.0 / piv;
#pragma unroll
    for (int k = c + 1; k < 4; ++k) {
      double f = A[k][c] * ip;
#pragma unroll
      for (int j = c; j < 4; ++j) A[k][j] -= f * A[c][j];
      r[k] -= f * r[c];
    }
  }
  if (solve) {
#pragma unroll
    for (int c = 3; c >= 0; --c) {
      double s = r[c];
#pragma unroll
      for (int j = c + 1; j < 4; ++j) s -= A[c][j] * r[j];
      r[c] = s / A[c][c];
    }
  }
  return det;
}

// Virtualities (q2_W+, q2_t, q2_W-, q2_tbar) at v = (nu_x, nu_y, nu_z,
// nubar_z) with nubar_xy = met - nu_xy, and their Jacobian w.r.t. v.
__device__ __forceinline__ void dilep_eval(const v4& lp, const v4& wt, const v4& lm, const v4& wtb,
                                           double wt2, double wtb2, double mx, double my,
                                           const double (&v)[4], double (&F)[4], double (&J)[4][4])
{
  v4 nu{0.0, v[0], v[1], v[2]};
  v4 nb{0.0, mx - v[0], my - v[1], v[3]};
  nu.e = norm3(nu);
  nb.e = norm3(nb);
  F[0] = 2.0 * mdot(lp, nu);
  F[1] = wt2 + 2.0 * mdot(wt, nu);
  F[2] = 2.0 * mdot(lm, nb);
  F[3] = wtb2 + 2.0 * mdot(wtb, nb);
  double inu = 1.0 / nu.e, inb = 1.0 / nb.e;
  double n3[3] = {nu.x * inu, nu.y * inu, nu.z * inu};
  double b3[3] = {nb.x * inb, nb.y * inb, nb.z * inb};
  double l3[3] = {lp.x, lp.y, lp.z}, t3[3] = {wt.x, wt.y, wt.z};
  double m3[3] = {lm.x, lm.y, lm.z}, u3[3] = {wtb.x, wtb.y, wtb.z};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    J[0][i] = 2.0 * (lp.e * n3[i] - l3[i]);
    J[1][i] = 2.0 * (wt.e * n3[i] - t3[i]);
  }
  J[0][3] = 0.0; J[1][3] = 0.0;
  double gl[3], gt[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) { gl[i] = 2.0 * (lm.e * b3[i] - m3[i]); gt[i] = 2.0 * (wtb.e * b3[i] - u3[i]); }
  J[2][0] = -gl[0]; J[2][1] = -gl[1]; J[2][2] = 0.0; J[2][3] = gl[2];
  J[3][0] = -gt[0]; J[3][1] = -gt[1]; J[3][2] = 0.0; J[3][3] = gt[2];
}

// Enumerates every accepted (nu, nubar) solution, calling
// sink(nu, nubar, |det J|) in lab units.  Inputs in GeV / GeV^2.
template <class Sink>
__device__ __forceinline__ int solve_dilepton(const v4& b_in, const v4& bb_in, const v4& lp_in, const v4& lm_in,
                                              double metx, double mety, double q2wp, double q2t,
                                              double q2wm, double q2tb, Sink&& sink)
{
  // scale to O(1) numbers
  const double lam = 0.25 * (b_in.e + bb_in.e + lp_in.e + lm_in.e);
  const double il = 1.0 / lam, il2 = il * il;
  v4 b{b_in.e * il, b_in.x * il, b_in.y * il, b_in.z * il};
  v4 bb{bb_in.e * il, bb_in.x * il, bb_in.y * il, bb_in.z * il};
  v4 lp{lp_in.e * il, lp_in.x * il, lp_in.y * il, lp_in.z * il};
  v4 lm{lm_in.e * il, lm_in.x * il, lm_in.y * il, lm_in.z * il};
  const double mx = metx * il, my = mety * il;
  const double tq[4] = {q2wp * il2, q2t * il2, q2wm * il2, q2tb * il2};

  Affine A1, A2;
  if (!nu_affine(b, lp, tq[0], tq[1], A1)) return 0;
  if (!nu_affine(bb, lm, tq[2], tq[3], A2)) return 0;
  // conic E^2 - p^2 = 0 of each side: {xx, xy, yy, x, y, 1}
  double c1[6] = {A1.e1 * A1.e1 - 1.0 - A1.z1 * A1.z1, 2.0 * (A1.e1 * A1.e2 - A1.z1 * A1.z2),
                  A1.e2 * A1.e2 - 1.0 - A1.z2 * A1.z2, 2.0 * (A1.e0 * A1.e1 - A1.z0 * A1.z1),
                  2.0 * (A1.e0 * A1.e2 - A1.z0 * A1.z2), A1.e0 * A1.e0 - A1.z0 * A1.z0};
  double cb[6] = {A2.e1 * A2.e1 - 1.0 - A2.z1 * A2.z1, 2.0 * (A2.e1 * A2.e2 - A2.z1 * A2.z2),
                  A2.e2 * A2.e2 - 1.0 - A2.z2 * A2.z2, 2.0 * (A2.e0 * A2.e1 - A2.z0 * A2.z1),
                  2.0 * (A2.e0 * A2.e2 - A2.z0 * A2.z2), A2.e0 * A2.e0 - A2.z0 * A2.z0};
  // substitute nubar_xy = met - nu_xy
  double c2[6] = {cb[0], cb[1], cb[2],
                  -2.0 * mx * cb[0] - my * cb[1] - cb[3],
                  -2.0 * my * cb[2] - mx * cb[1] - cb[4],
                  (cb[0] * mx + cb[1] * my + cb[3]) * mx + (cb[2] * my + cb[4]) * my + cb[5]};
  // as polynomials in py: a py^2 + (b0 + b1 px) py + (g0 + g1 px + g2 px^2)
  const double a1 = c1[2], a2 = c2[2];
  const double P0 = a1 * c2[5] - a2 * c1[5], P1 = a1 * c2[3] - a2 * c1[3], P2 = a1 * c2[0] - a2 * c1[0];
  const double Q0 = a1 * c2[4] - a2 * c1[4], Q1 = a1 * c2[1] - a2 * c1[1];
  // R = B1 C2 - B2 C1 (cubic)
  const double R0 = c1[4] * c2[5] - c2[4] * c1[5];
  const double R1 = c1[4] * c2[3] + c1[1] * c2[5] - c2[4] * c1[3] - c2[1] * c1[5];
  const double R2 = c1[4] * c2[0] + c1[1] * c2[3] - c2[4] * c1[0] - c2[1] * c1[3];
  const double R3 = c1[1] * c2[0] - c2[1] * c1[0];
  // resultant P^2 - Q R
  double quart[5] = {P0 * P0 - Q0 * R0,
                     2.0 * P0 * P1 - Q0 * R1 - Q1 * R0,
                     P1 * P1 + 2.0 * P0 * P2 - Q0 * R2 - Q1 * R1,
                     2.0 * P1 * P2 - Q0 * R3 - Q1 * R2,
                     P2 * P2 - Q1 * R3};
  if (quart[4] == 0.0) return 0;
  double roots[4];
  const int nr = quartic_real_roots(quart, roots);

  const v4 wt = add(b, lp), wtb = add(bb, lm);
  const double wt2 = mdot(wt, wt), wtb2 = mdot(wtb, wtb);
  int ns = 0;
  const double l4 = lam * lam * lam * lam;
  for (int k = 0; k < nr; ++k) {
    const double px = roots[k];
    const double q = Q0 + Q1 * px;
    if (!(fabs(q) > 1e-12 * (fabs(Q0) + fabs(Q1 * px)))) continue;
    const double py = -(P0 + (P1 + P2 * px) * px) / q;
    const double E1 = A1.e0 + A1.e1 * px + A1.e2 * py;
    const double bx = mx - px, by = my - py;
    const double E2 = A2.e0 + A2.e1 * bx + A2.e2 * by;
    if (!(E1 > 0.0 && E2 > 0.0)) continue;
    double v[4] = {px, py, A1.z0 + A1.z1 * px + A1.z2 * py, A2.z0 + A2.z1 * bx + A2.z2 * by};
    double F[4], J[4][4];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      dilep_eval(lp, wt, lm, wtb, wt2, wtb2, mx, my, v, F, J);
      double r[4] = {F[0] - tq[0], F[1] - tq[1], F[2] - tq[2], F[3] - tq[3]};
      if (det_solve4(J, r, true) == 0.0) break;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] -= r[i];
    }
    dilep_eval(lp, wt, lm, wtb, wt2, wtb2, mx, my, v, F, J);
    double worst = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) worst = fmax(worst, fabs(F[i] - tq[i]) / fabs(tq[i]));
    if (!(worst < 1e-6)) continue;
    double dummy[4] = {0, 0, 0, 0};
    double det = det_solve4(J, dummy, false);
    if (det == 0.0) continue;
    v4 nu{0.0, v[0] * lam, v[1] * lam, v[2] * lam};
    v4 nb{0.0, (mx - v[0]) * lam, (my - v[1]) * lam, v[3] * lam};
    nu.e = norm3(nu);
    nb.e = norm3(nb);
    sink(nu, nb, fabs(det) * l4);
    ++ns;
  }
  return ns;
}

}  // namespace memk
