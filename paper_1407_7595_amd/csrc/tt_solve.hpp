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
//
// The root finder runs in lockstep across a wavefront, so its cost is the
// slowest lane's iteration count.  Two things keep that short: every
// bracketed search starts from a model estimate (the closed-form cubic for
// the critical points, the local quadratic at a critical point for the
// quartic roots), and it stops as soon as the residual is within the
// rounding error of its own evaluation instead of waiting for the step to
// vanish, which near a root with condition number above a few never
// happens and left the search bisecting to the last bit.
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

// Reciprocal for a Newton step: the hardware estimate refined once (an
// error of the step's size times ~1e-15 changes no iterate that matters:
// the step is recomputed from the new residual every iteration).
__device__ __forceinline__ double step_rcp(double d)
{
#ifdef MEM_HOST_COUNT
  return 1.0 / d;
#else
  const double r = __builtin_amdgcn_rcp(d);
  return __fma_rn(r, __fma_rn(-d, r, 1.0), r);
#endif
}

// Root of a polynomial that is monotone on [lo, hi] with a sign change,
// starting at x0 (the midpoint when x0 is not inside): Newton steps, with
// bisection whenever a step leaves the bracket.  Stops when |p(x)| is at
// most 1e-15 sum |c_i| |x|^i (x is then the exact root of a polynomial
// whose coefficients differ from c by ~1e-15 relative; the degree-4 Horner
// rounding bound is 8 u = 8.9e-16) or when the step vanishes.  TEST0 =
// false skips that test at the starting point (the quartic's model
// estimates are never within rounding of a root).
template <int N, bool TEST0 = true>
__device__ __forceinline__ double bracketed_root(const double (&c)[N + 1], double lo, double hi, double flo,
                                                 double x0)
{
  double x = (x0 > lo && x0 < hi) ? x0 : 0.5 * (lo + hi);
  for (int it = 0; it < 80; ++it) {
    double f, df;
    horner_d<N>(c, x, f, df);
    if (TEST0 || it > 0) {
      const double ax = fabs(x);
      double fa = fabs(c[N]);
#pragma unroll
      for (int i = N - 1; i >= 0; --i) fa = __fma_rn(fa, ax, fabs(c[i]));
      if (fabs(f) <= 1e-15 * fa) return x;
    }
    if ((f < 0.0) == (flo < 0.0)) lo = x; else hi = x;
    double xn = x - f * step_rcp(df);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (fabs(xn - x) <= 4e-16 * fabs(x) + 1e-300 || !(hi > lo)) return xn;
    x = xn;
  }
  return x;
}

// Up to four doubles with a count; filled and read through select chains so
// that the values stay in registers (no dynamically indexed arrays).
struct Four {
  double v0, v1, v2, v3;
  int n;
  __device__ __forceinline__ void put(double x)
  {
    v0 = n == 0 ? x : v0;
    v1 = n == 1 ? x : v1;
    v2 = n == 2 ? x : v2;
    v3 = n >= 3 ? x : v3;
    ++n;
  }
  __device__ __forceinline__ double get(int k) const { return k == 0 ? v0 : k == 1 ? v1 : k == 2 ? v2 : v3; }
};

// Roots of a polynomial in each of `NI` consecutive intervals of pts
// (monotone on each), appended ascending to out; guess(i, lo, hi, flo, fhi)
// gives the starting point in interval i.
template <int N, int NI, bool TEST0, class Guess>
__device__ __forceinline__ void roots_on_intervals(const double (&c)[N + 1], const double (&pts)[NI + 1], Four& out,
                                                   Guess guess)
{
  double fprev = horner<N>(c, pts[0]);
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const double lo = pts[i], hi = pts[i + 1];
    const double fnext = horner<N>(c, hi);
    if (hi > lo) {
      if (fprev == 0.0) out.put(lo);
      else if ((fprev < 0.0) != (fnext < 0.0) && fnext != 0.0)
        out.put(bracketed_root<N, TEST0>(c, lo, hi, fprev, guess(i, lo, hi, fprev, fnext)));
    }
    fprev = fnext;
  }
}

// Real roots of the monic cubic t^3 + A t^2 + B t + C in closed form
// (trigonometric form for three real roots, Cardano's with the
// non-cancelling cube root otherwise; the single root is repeated).  Used
// only as starting points: accuracy is lost near a double root.
__device__ __forceinline__ void cubic_estimates(double A, double B, double C, double (&r)[3])
{
  const double a3 = A * (1.0 / 3.0);
  const double p = B - A * a3, q = C + a3 * (2.0 * a3 * a3 - B);
  const double D = 0.25 * q * q + p * p * p * (1.0 / 27.0);
  if (D <= 0.0 && p < 0.0) {
    const double m = sqrt(-p * (1.0 / 3.0));
    const double cphi = fmin(1.0, fmax(-1.0, -0.5 * q * fast_rcp(m * m * m)));
    double st, ct;
    sincos(acos(cphi) * (1.0 / 3.0), &st, &ct);
    r[0] = 2.0 * m * ct - a3;
    r[1] = m * (-ct + 1.7320508075688772 * st) - a3;
    r[2] = m * (-ct - 1.7320508075688772 * st) - a3;
  } else {
    const double u = cbrt(-0.5 * q - copysign(sqrt(fmax(D, 0.0)), q));
    r[0] = r[1] = r[2] = (u != 0.0 ? u - p * fast_rcp(3.0 * u) : 0.0) - a3;
  }
}

// The real roots of a quartic (c4 != 0) in two steps.  quartic_isolate:
// the monic coefficients and the intervals between consecutive critical
// points (and the root bound) across which the quartic changes sign,
// ascending, each with the starting point of its search (hi == lo: a root
// exactly at lo).  quartic_root: the root of one such interval.  The work
// queue kernel runs the second step on the intervals of a whole wavefront
// gathered in LDS, so that the bracketed searches run in lockstep over
// full lanes; quartic_real_roots runs both per lane.  Either way a root
// comes out of the same function with the same inputs.
struct QuartIso {
  double c[5];        // monic coefficients
  Four lo, hi, x0;    // the intervals (lo.n of them) and their starting points
};

__device__ __forceinline__ void quartic_isolate(const double (&c_in)[5], QuartIso& q)
{
  const double inv = fast_rcp(c_in[4]);
  const double c[5] = {c_in[0] * inv, c_in[1] * inv, c_in[2] * inv, c_in[3] * inv, 1.0};
#pragma unroll
  for (int i = 0; i < 5; ++i) q.c[i] = c[i];
  double bound = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) bound = fmax(bound, fabs(c[i]));
  bound += 1.0;
  const double d1[4] = {c[1], 2.0 * c[2], 3.0 * c[3], 4.0};
  const double d2[3] = {2.0 * c[2], 6.0 * c[3], 12.0};
  // roots of the second derivative (closed form, stable); when absent both
  // collapse onto -bound and the corresponding intervals are empty
  double s0 = -bound, s1 = -bound;
  const double disc = d2[1] * d2[1] - 4.0 * d2[2] * d2[0];
  if (disc > 0.0) {
    const double qq = -0.5 * (d2[1] + copysign(sqrt(disc), d2[1]));
    const double a = qq * (1.0 / 12.0), b = (qq != 0.0) ? d2[0] * fast_rcp(qq) : a;
    s0 = fmin(fmax(fmin(a, b), -bound), bound);
    s1 = fmin(fmax(fmax(a, b), -bound), bound);
  }
  // the first derivative is monotone between consecutive points; its roots
  // start from the closed form (the estimate that falls inside)
  double est[3];
  cubic_estimates(0.75 * c[3], 0.5 * c[2], 0.25 * c[1], est);
  Four crit;
  crit.n = 0;
  const double p3[4] = {-bound, s0, s1, bound};
  // a closed-form estimate inside a derivative sign-change interval is its
  // root to a few ulp away from double roots of p' (where the quartic is
  // locally flat and its roots ill-conditioned anyway); only an interval
  // without one runs the bracketed search
  {
    double fprev = horner<3>(d1, p3[0]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double lo = p3[i], hi = p3[i + 1];
      const double fnext = horner<3>(d1, hi);
      if (hi > lo) {
        if (fprev == 0.0) crit.put(lo);
        else if ((fprev < 0.0) != (fnext < 0.0) && fnext != 0.0) {
          const bool in0 = est[0] > lo && est[0] < hi, in1 = est[1] > lo && est[1] < hi;
          const bool in2 = est[2] > lo && est[2] < hi;
          crit.put(in0 ? est[0] : in1 ? est[1] : in2 ? est[2]
                                            : bracketed_root<3, true>(d1, lo, hi, fprev, 0.5 * (lo + hi)));
        }
      }
      fprev = fnext;
    }
  }
  // the quartic is monotone between consecutive critical points; a root
  // starts from the quadratic model p(e) + p''(e) d^2 / 2 at the critical
  // end e with the smaller |p| (interior intervals have two)
  const double p4[5] = {-bound, crit.n > 0 ? crit.v0 : bound, crit.n > 1 ? crit.v1 : bound,
                        crit.n > 2 ? crit.v2 : bound, bound};
  q.lo.n = q.hi.n = q.x0.n = 0;
  double fprev = horner<4>(c, p4[0]);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double lo = p4[i], hi = p4[i + 1];
    const double fnext = horner<4>(c, hi);
    if (hi > lo) {
      if (fprev == 0.0) {
        q.lo.put(lo); q.hi.put(lo); q.x0.put(lo);
      } else if ((fprev < 0.0) != (fnext < 0.0) && fnext != 0.0) {
        const bool lo_crit = i > 0, hi_crit = hi < bound;
        const bool use_lo = lo_crit && (!hi_crit || fabs(fprev) <= fabs(fnext));
        const double e = use_lo ? lo : hi, fe = use_lo ? fprev : fnext;
        const double d = sqrt(fabs(2.0 * fe * fast_rcp(horner<2>(d2, e))));
        q.lo.put(lo); q.hi.put(hi); q.x0.put(use_lo ? lo + d : hi - d);
      }
    }
    fprev = fnext;
  }
}

__device__ __forceinline__ double quartic_root(const double (&c)[5], double lo, double hi, double x0)
{
  return hi == lo ? lo : bracketed_root<4, false>(c, lo, hi, horner<4>(c, lo), x0);
}

// Real roots of a quartic (c4 != 0), ascending.
__device__ __forceinline__ void quartic_real_roots(const double (&c_in)[5], Four& roots)
{
  QuartIso q;
  quartic_isolate(c_in, q);
  roots.n = 0;
  for (int k = 0; k < q.lo.n; ++k) roots.put(quartic_root(q.c, q.lo.get(k), q.hi.get(k), q.x0.get(k)));
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
  const double id = fast_rcp(det);
  a.e0 = (l.z * h2 - b.z * h1) * id;
  a.e1 = (l.z * b.x - b.z * l.x) * id;
  a.e2 = (l.z * b.y - b.z * l.y) * id;
  a.z0 = (l.e * h2 - b.e * h1) * id;
  a.z1 = (l.e * b.x - b.e * l.x) * id;
  a.z2 = (l.e * b.y - b.e * l.y) * id;
  return true;
}

// Virtualities (q2_W+, q2_t, q2_W-, q2_tbar) at v = (nu_x, nu_y, nu_z,
// nubar_z), with nubar_xy = met - nu_xy.
struct DilepGeom {
  v4 lp, wt, lm, wtb;      // l+, b + l+, l-, bbar + l- (scaled units)
  double wt2, wtb2, mx, my;
};

__device__ __forceinline__ void dilep_F(const DilepGeom& g, const double (&v)[4], double (&F)[4], v4& nu, v4& nb)
{
  nu = v4{0.0, v[0], v[1], v[2]};
  nb = v4{0.0, g.mx - v[0], g.my - v[1], v[3]};
  nu.e = norm3(nu);
  nb.e = norm3(nb);
  F[0] = 2.0 * mdot(g.lp, nu);
  F[1] = g.wt2 + 2.0 * mdot(g.wt, nu);
  F[2] = 2.0 * mdot(g.lm, nb);
  F[3] = g.wtb2 + 2.0 * mdot(g.wtb, nb);
}

// The Jacobian of F w.r.t. v has two zeros per row pair:
//   rows W+, t   depend on (nu_x, nu_y, nu_z)     : a = dF0, b = dF1
//   rows W-, tbar depend on (nu_x, nu_y, nubar_z) : c = dF2, d = dF3
// (nubar_x,y = met - nu_x,y).  Eliminating nu_z and nubar_z leaves the 2x2
// system [[E0, E1], [G0, G1]] in (nu_x, nu_y) with
//   E = a_z b_xy - b_z a_xy,  G = c_z d_xy - d_z c_xy,
// and det J = -(E0 G1 - E1 G0): no pivoting, no division.
struct DilepJac { double a[3], b[3], c[3], d[3]; };

__device__ __forceinline__ void dilep_J(const DilepGeom& g, const v4& nu, const v4& nb, DilepJac& J)
{
  const double inu = fast_rcp(nu.e), inb = fast_rcp(nb.e);
  const double n3[3] = {nu.x * inu, nu.y * inu, nu.z * inu};
  const double b3[3] = {nb.x * inb, nb.y * inb, nb.z * inb};
  const double l3[3] = {g.lp.x, g.lp.y, g.lp.z}, t3[3] = {g.wt.x, g.wt.y, g.wt.z};
  const double m3[3] = {g.lm.x, g.lm.y, g.lm.z}, u3[3] = {g.wtb.x, g.wtb.y, g.wtb.z};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    J.a[i] = 2.0 * (g.lp.e * n3[i] - l3[i]);
    J.b[i] = 2.0 * (g.wt.e * n3[i] - t3[i]);
    // d/dnu_{x,y} = -d/dnubar_{x,y}; the third entry is d/dnubar_z
    const double sgn = i < 2 ? -1.0 : 1.0;
    J.c[i] = sgn * 2.0 * (g.lm.e * b3[i] - m3[i]);
    J.d[i] = sgn * 2.0 * (g.wtb.e * b3[i] - u3[i]);
  }
}

__device__ __forceinline__ double dilep_det(const DilepJac& J)
{
  const double E0 = J.a[2] * J.b[0] - J.b[2] * J.a[0], E1 = J.a[2] * J.b[1] - J.b[2] * J.a[1];
  const double G0 = J.c[2] * J.d[0] - J.d[2] * J.c[0], G1 = J.c[2] * J.d[1] - J.d[2] * J.c[1];
  return -(E0 * G1 - E1 * G0);
}

// Newton step: solve J dv = r by the block elimination above.
__device__ __forceinline__ bool dilep_step(const DilepJac& J, const double (&r)[4], double (&dv)[4])
{
  const double E0 = J.a[2] * J.b[0] - J.b[2] * J.a[0], E1 = J.a[2] * J.b[1] - J.b[2] * J.a[1];
  const double G0 = J.c[2] * J.d[0] - J.d[2] * J.c[0], G1 = J.c[2] * J.d[1] - J.d[2] * J.c[1];
  const double h0 = J.a[2] * r[1] - J.b[2] * r[0], h1 = J.c[2] * r[3] - J.d[2] * r[2];
  const double D = E0 * G1 - E1 * G0;
  if (D == 0.0) return false;
  const double iD = fast_rcp(D);
  dv[0] = (h0 * G1 - E1 * h1) * iD;
  dv[1] = (E0 * h1 - h0 * G0) * iD;
  // back-substitute through the better conditioned row of each pair
  const bool ua = fabs(J.a[2]) >= fabs(J.b[2]);
  const double pz = ua ? J.a[2] : J.b[2];
  const double rz = (ua ? r[0] : r[1]) - (ua ? J.a[0] : J.b[0]) * dv[0] - (ua ? J.a[1] : J.b[1]) * dv[1];
  const bool uc = fabs(J.c[2]) >= fabs(J.d[2]);
  const double pb = uc ? J.c[2] : J.d[2];
  const double rb = (uc ? r[2] : r[3]) - (uc ? J.c[0] : J.d[0]) * dv[0] - (uc ? J.c[1] : J.d[1]) * dv[1];
  if (pz == 0.0 || pb == 0.0) return false;
  dv[2] = rz * fast_rcp(pz);
  dv[3] = rb * fast_rcp(pb);
  return true;
}

// Relative constraint residual above which a root is polished by Newton on
// the full system: near the FP64 rounding level when the matrix element
// runs in FP64; 1e-10 when it runs in FP32, whose rounding (~1e-7) the
// remaining solve error then stays far below.
template <class T> constexpr double polish_tol() { return sizeof(T) == 4 ? 1e-10 : 1e-13; }

// Accepted (nu, nubar) solutions of one point, held in four static slots
// so that they stay in registers.
struct NuSol { double nx, ny, nz, bx, by, bz, adet; };
// Field-wise selects: an if-chain over whole records gets merged by the
// compiler into a dynamically indexed (scratch) array.
__device__ __forceinline__ NuSol sel(bool c, const NuSol& a, const NuSol& b)
{
  return NuSol{c ? a.nx : b.nx, c ? a.ny : b.ny, c ? a.nz : b.nz, c ? a.bx : b.bx,
               c ? a.by : b.by, c ? a.bz : b.bz, c ? a.adet : b.adet};
}
struct NuSet {
  NuSol s0, s1, s2, s3;
  int n;
  __device__ __forceinline__ void put(const NuSol& v)
  {
    s0 = sel(n == 0, v, s0);
    s1 = sel(n == 1, v, s1);
    s2 = sel(n == 2, v, s2);
    s3 = sel(n >= 3, v, s3);
    ++n;
  }
  __device__ __forceinline__ NuSol get(int k) const
  {
    return sel(k == 0, s0, sel(k == 1, s1, sel(k == 2, s2, s3)));
  }
};

// Per-point state of the solve once the resultant is formed (scaled units:
// momenta / lam, virtualities / lam^2).
struct DilepPoint {
  Affine A1, A2;                  // E, p_z of nu (A1) and nubar (A2), affine in p_x, p_y
  double P0, P1, P2, Q0, Q1;      // p_y = -(P0 + P1 px + P2 px^2) / (Q0 + Q1 px)
  double tq[4], itq[4];           // target virtualities and their reciprocals
  double lam, mx, my;             // scale; missing transverse momentum
};

// Scaling, the affine neutrino kinematics, the two conics and their
// resultant (quartic in p_x, quart[0..4]).  false: no solution possible.
__device__ __forceinline__ bool dilep_prepare(const v4& b_in, const v4& bb_in, const v4& lp_in, const v4& lm_in,
                                              double metx, double mety, double q2wp, double q2t, double q2wm,
                                              double q2tb, DilepPoint& s, double (&quart)[5])
{
  // scale to O(1) numbers
  const double lam = 0.25 * (b_in.e + bb_in.e + lp_in.e + lm_in.e);
  const double il = fast_rcp(lam), il2 = il * il;
  const v4 b{b_in.e * il, b_in.x * il, b_in.y * il, b_in.z * il};
  const v4 bb{bb_in.e * il, bb_in.x * il, bb_in.y * il, bb_in.z * il};
  const v4 lp{lp_in.e * il, lp_in.x * il, lp_in.y * il, lp_in.z * il};
  const v4 lm{lm_in.e * il, lm_in.x * il, lm_in.y * il, lm_in.z * il};
  const double mx = metx * il, my = mety * il;
  s.lam = lam; s.mx = mx; s.my = my;
  s.tq[0] = q2wp * il2; s.tq[1] = q2t * il2; s.tq[2] = q2wm * il2; s.tq[3] = q2tb * il2;
#pragma unroll
  for (int i = 0; i < 4; ++i) s.itq[i] = fast_rcp(s.tq[i]);

  Affine& A1 = s.A1;
  Affine& A2 = s.A2;
  if (!nu_affine(b, lp, s.tq[0], s.tq[1], A1)) return false;
  if (!nu_affine(bb, lm, s.tq[2], s.tq[3], A2)) return false;
  // conic E^2 - p^2 = 0 of each side: {xx, xy, yy, x, y, 1}
  const double c1[6] = {A1.e1 * A1.e1 - 1.0 - A1.z1 * A1.z1, 2.0 * (A1.e1 * A1.e2 - A1.z1 * A1.z2),
                        A1.e2 * A1.e2 - 1.0 - A1.z2 * A1.z2, 2.0 * (A1.e0 * A1.e1 - A1.z0 * A1.z1),
                        2.0 * (A1.e0 * A1.e2 - A1.z0 * A1.z2), A1.e0 * A1.e0 - A1.z0 * A1.z0};
  const double cb[6] = {A2.e1 * A2.e1 - 1.0 - A2.z1 * A2.z1, 2.0 * (A2.e1 * A2.e2 - A2.z1 * A2.z2),
                        A2.e2 * A2.e2 - 1.0 - A2.z2 * A2.z2, 2.0 * (A2.e0 * A2.e1 - A2.z0 * A2.z1),
                        2.0 * (A2.e0 * A2.e2 - A2.z0 * A2.z2), A2.e0 * A2.e0 - A2.z0 * A2.z0};
  // substitute nubar_xy = met - nu_xy
  const double c2[6] = {cb[0], cb[1], cb[2],
                        -2.0 * mx * cb[0] - my * cb[1] - cb[3],
                        -2.0 * my * cb[2] - mx * cb[1] - cb[4],
                        (cb[0] * mx + cb[1] * my + cb[3]) * mx + (cb[2] * my + cb[4]) * my + cb[5]};
  // as polynomials in py: a py^2 + (b0 + b1 px) py + (g0 + g1 px + g2 px^2)
  const double a1 = c1[2], a2 = c2[2];
  const double P0 = a1 * c2[5] - a2 * c1[5], P1 = a1 * c2[3] - a2 * c1[3], P2 = a1 * c2[0] - a2 * c1[0];
  const double Q0 = a1 * c2[4] - a2 * c1[4], Q1 = a1 * c2[1] - a2 * c1[1];
  s.P0 = P0; s.P1 = P1; s.P2 = P2; s.Q0 = Q0; s.Q1 = Q1;
  // R = B1 C2 - B2 C1 (cubic)
  const double R0 = c1[4] * c2[5] - c2[4] * c1[5];
  const double R1 = c1[4] * c2[3] + c1[1] * c2[5] - c2[4] * c1[3] - c2[1] * c1[5];
  const double R2 = c1[4] * c2[0] + c1[1] * c2[3] - c2[4] * c1[0] - c2[1] * c1[3];
  const double R3 = c1[1] * c2[0] - c2[1] * c1[0];
  // resultant P^2 - Q R
  quart[0] = P0 * P0 - Q0 * R0;
  quart[1] = 2.0 * P0 * P1 - Q0 * R1 - Q1 * R0;
  quart[2] = P1 * P1 + 2.0 * P0 * P2 - Q0 * R2 - Q1 * R1;
  quart[3] = 2.0 * P1 * P2 - Q0 * R3 - Q1 * R2;
  quart[4] = P2 * P2 - Q1 * R3;
  return quart[4] != 0.0;
}

// Scaled geometry of the two top sides from the unscaled inputs.
__device__ __forceinline__ void dilep_geom(const v4& b_in, const v4& bb_in, const v4& lp_in, const v4& lm_in,
                                           const DilepPoint& s, DilepGeom& g)
{
  const double il = fast_rcp(s.lam);
  const v4 b{b_in.e * il, b_in.x * il, b_in.y * il, b_in.z * il};
  const v4 bb{bb_in.e * il, bb_in.x * il, bb_in.y * il, bb_in.z * il};
  g.lp = v4{lp_in.e * il, lp_in.x * il, lp_in.y * il, lp_in.z * il};
  g.lm = v4{lm_in.e * il, lm_in.x * il, lm_in.y * il, lm_in.z * il};
  g.wt = add(b, g.lp);
  g.wtb = add(bb, g.lm);
  g.wt2 = mdot(g.wt, g.wt);
  g.wtb2 = mdot(g.wtb, g.wtb);
  g.mx = s.mx;
  g.my = s.my;
}

// One real root px of the resultant: p_y from the conics, positive
// energies, conditional Newton polish on the full system (when the largest
// relative residual exceeds polish_tol), residual test; on acceptance the
// solution in lab units (GeV) with |det J| (GeV^4).
__device__ __forceinline__ bool dilep_accept(const DilepPoint& s, const DilepGeom& g, double px, NuSol& out,
                                             double polish_tol)
{
  const Affine& A1 = s.A1;
  const Affine& A2 = s.A2;
  const double q = s.Q0 + s.Q1 * px;
  if (!(fabs(q) > 1e-12 * (fabs(s.Q0) + fabs(s.Q1 * px)))) return false;
  const double py = -(s.P0 + (s.P1 + s.P2 * px) * px) * fast_rcp(q);
  const double E1 = A1.e0 + A1.e1 * px + A1.e2 * py;
  const double bx = s.mx - px, by = s.my - py;
  const double E2 = A2.e0 + A2.e1 * bx + A2.e2 * by;
  if (!(E1 > 0.0 && E2 > 0.0)) return false;
  double v[4] = {px, py, A1.z0 + A1.z1 * px + A1.z2 * py, A2.z0 + A2.z1 * bx + A2.z2 * by};
  double F[4];
  v4 nu, nb;
  dilep_F(g, v, F, nu, nb);
  double worst = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) worst = fmax(worst, fabs((F[i] - s.tq[i]) * s.itq[i]));
  // the resultant loses digits near degenerate configurations: polish by
  // Newton on the full system only where the residual shows it
  for (int it = 0; it < 2 && worst > polish_tol; ++it) {
    DilepJac J;
    dilep_J(g, nu, nb, J);
    double r[4] = {F[0] - s.tq[0], F[1] - s.tq[1], F[2] - s.tq[2], F[3] - s.tq[3]}, dv[4];
    if (!dilep_step(J, r, dv)) break;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] -= dv[i];
    dilep_F(g, v, F, nu, nb);
    worst = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) worst = fmax(worst, fabs((F[i] - s.tq[i]) * s.itq[i]));
  }
  if (!(worst < 1e-6)) return false;
  DilepJac J;
  dilep_J(g, nu, nb, J);
  const double det = dilep_det(J);
  if (det == 0.0) return false;
  const double lam = s.lam, l4 = lam * lam * lam * lam;
  out = NuSol{v[0] * lam, v[1] * lam, v[2] * lam, (s.mx - v[0]) * lam, (s.my - v[1]) * lam, v[3] * lam,
              fabs(det) * l4};
  return true;
}

// Every accepted (nu, nubar) solution, in lab units (GeV) with |det J|
// (GeV^4).  Inputs in GeV / GeV^2.
__device__ __forceinline__ void solve_dilepton(const v4& b_in, const v4& bb_in, const v4& lp_in, const v4& lm_in,
                                               double metx, double mety, double q2wp, double q2t, double q2wm,
                                               double q2tb, NuSet& out, double polish_tol)
{
  out.n = 0;
  DilepPoint s;
  double quart[5];
  if (!dilep_prepare(b_in, bb_in, lp_in, lm_in, metx, mety, q2wp, q2t, q2wm, q2tb, s, quart)) return;
  Four roots;
  quartic_real_roots(quart, roots);
  DilepGeom g;
  dilep_geom(b_in, bb_in, lp_in, lm_in, s, g);
  for (int k = 0; k < roots.n; ++k) {
    NuSol sol;
    if (dilep_accept(s, g, roots.get(k), sol, polish_tol)) out.put(sol);
  }
}

}  // namespace memk
