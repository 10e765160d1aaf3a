/*
 * Oracle: phase-space maps, constraint solves and the two integrands.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Drell-Yan: Eq. mem_def with the n-body phase space below it, the TF
 * convolution of Eq. 3 and a Gaussian momentum TF (Sec. 1).
 * ttbar dilepton: Eq. integrand of Sec. 3 with the change of variables to
 * the top and W propagator virtualities, Eq. dilepsolv, and the per-point
 * missing transverse momentum of Sec. 4 (extended by a transverse recoil).
 */
#include "oracle.h"
#include <math.h>
#include <string.h>

static double mdot(const double* a, const double* b)
{
  return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}
static double norm3(const double* p) { return sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]); }

/* -------------------------------------------------------- toy densities -- */
double or_xf_u(double x) { return 2.0 * sqrt(x) * pow(1.0 - x, 3); }
double or_xf_d(double x) { return sqrt(x) * pow(1.0 - x, 4); }
double or_xf_qbar(double x) { return 0.2 * pow(1.0 - x, 7); }
double or_xf_g(double x) { return 3.0 * pow(1.0 - x, 5); }

/* densities f = x f / x of the 11 flavours at (x, Q) from the grid */
static void grid_f(const or_params* p, double x, double Q, double* f)
{
  for (int k = 0; k < 11; ++k) f[k] = or_pdf_interp(p->pdf, k - 5, x, Q) / x;
}

/* Parton luminosities of the top processes at (x1, x2) (Eq. mem_def: the
 * densities of both beams): gg = f_g f_g, qq12 = sum_q f_q(x1) f_qbar(x2),
 * qq21 = sum_q f_qbar(x1) f_q(x2), the sums over d, u, s, c, b.  Toy
 * densities: u + d against the common sea antiquark. */
typedef struct { double gg, qq12, qq21; } tt_lumi;
static tt_lumi tt_lumis(const or_params* p, double x1, double x2)
{
  tt_lumi L;
  if (!p->pdf) {
    double g1 = or_xf_g(x1) / x1, g2 = or_xf_g(x2) / x2;
    double q1 = (or_xf_u(x1) + or_xf_d(x1)) / x1, qb1 = or_xf_qbar(x1) / x1;
    double q2 = (or_xf_u(x2) + or_xf_d(x2)) / x2, qb2 = or_xf_qbar(x2) / x2;
    L.gg = g1 * g2;
    L.qq12 = q1 * qb2;
    L.qq21 = qb1 * q2;
    return L;
  }
  double f1[11], f2[11];
  grid_f(p, x1, p->m_t, f1);
  grid_f(p, x2, p->m_t, f2);
  L.gg = f1[5] * f2[5];
  L.qq12 = L.qq21 = 0.0;
  for (int q = 1; q <= 5; ++q) {
    L.qq12 += f1[5 + q] * f2[5 - q];
    L.qq21 += f1[5 - q] * f2[5 + q];
  }
  return L;
}

/* Drell-Yan luminosity sum_q e_q^2 (f_q(x1) f_qbar(x2) + f_qbar(x1) f_q(x2))
 * at the scale Q (grid densities only; charges -1/3, 2/3, -1/3, 2/3, -1/3
 * for d, u, s, c, b) */
static double dy_grid_lumi(const or_params* p, double x1, double x2, double Q)
{
  static const double e2[6] = {0.0, 1.0 / 9.0, 4.0 / 9.0, 1.0 / 9.0, 4.0 / 9.0, 1.0 / 9.0};
  double f1[11], f2[11];
  grid_f(p, x1, Q, f1);
  grid_f(p, x2, Q, f2);
  double lum = 0.0;
  for (int q = 1; q <= 5; ++q) lum += e2[q] * (f1[5 + q] * f2[5 - q] + f1[5 - q] * f2[5 + q]);
  return lum;
}

double or_gauss_tf(double meas, double truth, double rel_sigma)
{
  double s = rel_sigma * truth;
  double z = (meas - truth) / s;
  return exp(-0.5 * z * z) / (sqrt(2.0 * M_PI) * s);
}

/* ----------------------------------------------------------- Drell-Yan -- */
/* Collins-Soper polar angle of the mu- in the pair rest frame */
static double cos_cs(const double* m1, const double* m2)
{
  double P[4];
  for (int i = 0; i < 4; ++i) P[i] = m1[i] + m2[i];
  double M2 = mdot(P, P), pt2 = P[1] * P[1] + P[2] * P[2];
  double p1p = (m1[0] + m1[3]) / sqrt(2.0), p1m = (m1[0] - m1[3]) / sqrt(2.0);
  double p2p = (m2[0] + m2[3]) / sqrt(2.0), p2m = (m2[0] - m2[3]) / sqrt(2.0);
  return 2.0 * (p1p * p2m - p1m * p2p) / (sqrt(M2) * sqrt(M2 + pt2));
}

double or_dy_integrand(const or_params* p, const double* ev, const double* x)
{
  const double S = p->sqrt_s * p->sqrt_s;
  double mu[2][4];
  double factor = 1.0;
  for (int k = 0; k < 2; ++k) {
    const double* m = ev + 4 * k;
    double pm = norm3(m);
    double r = p->r_lo + x[k] * (p->r_hi - p->r_lo);
    double pt = pm / r;                      /* true |p| */
    double jac = (p->r_hi - p->r_lo) * pm / (r * r);
    for (int i = 1; i < 4; ++i) mu[k][i] = m[i] / pm * pt;
    mu[k][0] = pt;
    double sin_th = sqrt(m[1] * m[1] + m[2] * m[2]) / pm;
    /* d^3p/((2pi)^3 2E) with delta functions on the direction:
     * p^2 sin(theta) dp / (2E), times the TF (the (2pi) powers are
     * collected below) */
    factor *= pt * pt * sin_th / (2.0 * pt) * or_gauss_tf(pm, pt, p->tf_sigma) * jac;
  }
  double P[4];
  for (int i = 0; i < 4; ++i) P[i] = mu[0][i] + mu[1][i];
  double M2 = mdot(P, P);
  if (M2 <= 0.0) return 0.0;
  double M = sqrt(M2);
  if (M < p->m_lo || M > p->m_hi) return 0.0;
  double x1 = (P[0] + P[3]) / p->sqrt_s, x2 = (P[0] - P[3]) / p->sqrt_s;
  if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) return 0.0;
  double c = cos_cs(mu[0], mu[1]);
  double e2 = 4.0 * M_PI * p->alpha;
  double me_unit = e2 * e2 * (1.0 + c * c) / 3.0;   /* for Q_q^2 = 1 */
  double lum;
  if (p->pdf) {
    lum = dy_grid_lumi(p, x1, x2, M);
  } else {
    double fu1 = or_xf_u(x1) / x1, fd1 = or_xf_d(x1) / x1, fq1 = or_xf_qbar(x1) / x1;
    double fu2 = or_xf_u(x2) / x2, fd2 = or_xf_d(x2) / x2, fq2 = or_xf_qbar(x2) / x2;
    lum = 4.0 / 9.0 * (fu1 * fq2 + fq1 * fu2) + 1.0 / 9.0 * (fd1 * fq2 + fq1 * fd2);
  }
  double shat = x1 * x2 * S;
  double flux = 1.0 / (2.0 * shat);
  double two_pi_pow = pow(2.0 * M_PI, 4.0 - 3.0 * 2.0);
  return two_pi_pow * (2.0 / S) * lum * me_unit * flux * factor;
}

/* Gauss-Legendre nodes on [-1,1] by Newton on the Legendre recurrence */
static void gauss_legendre(int n, double* xs, double* ws)
{
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int j = 0; j < n; ++j) { double p2 = p1; p1 = p0; p0 = ((2.0 * j + 1.0) * z * p1 - j * p2) / (j + 1.0); }
      pp = n * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / pp;
      z -= dz;
      if (fabs(dz) < 1e-15) break;
    }
    xs[i] = z;
    ws[i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

static double dy_lumi_sigma(const or_params* p, double x1, double x2)
{
  double fu1 = or_xf_u(x1) / x1, fd1 = or_xf_d(x1) / x1, fq1 = or_xf_qbar(x1) / x1;
  double fu2 = or_xf_u(x2) / x2, fd2 = or_xf_d(x2) / x2, fq2 = or_xf_qbar(x2) / x2;
  double lum = 4.0 / 9.0 * (fu1 * fq2 + fq1 * fu2) + 1.0 / 9.0 * (fd1 * fq2 + fq1 * fd2);
  double shat = x1 * x2 * p->sqrt_s * p->sqrt_s;
  /* partonic sigma(q qbar -> mu mu) for unit charge, colour averaged:
   * 4 pi alpha^2 / (3 shat) / 3 */
  return lum * 4.0 * M_PI * p->alpha * p->alpha / (9.0 * shat);
}

double or_dy_sigma_2d(const or_params* p, int nodes)
{
  /* integrate over (ln tau, y) with x1 = sqrt(tau) e^y, x2 = sqrt(tau) e^-y,
   * dx1 dx2 = tau d(ln tau) dy */
  double xs[4096], ws[4096];
  if (nodes > 4096) nodes = 4096;
  gauss_legendre(nodes, xs, ws);
  double S = p->sqrt_s * p->sqrt_s;
  double lt0 = log(p->m_lo * p->m_lo / S), lt1 = log(p->m_hi * p->m_hi / S);
  double total = 0.0;
  for (int i = 0; i < nodes; ++i) {
    double lt = 0.5 * (lt1 - lt0) * xs[i] + 0.5 * (lt1 + lt0);
    double tau = exp(lt);
    double ymax = -0.5 * lt;
    double inner = 0.0;
    for (int j = 0; j < nodes; ++j) {
      double y = ymax * xs[j];
      double x1 = sqrt(tau) * exp(y), x2 = sqrt(tau) * exp(-y);
      if (x1 >= 1.0 || x2 >= 1.0) continue;
      inner += ws[j] * ymax * dy_lumi_sigma(p, x1, x2);
    }
    total += ws[i] * 0.5 * (lt1 - lt0) * tau * inner;
  }
  return total;
}

double or_dy_sigma_tau(const or_params* p, int nodes)
{
  /* sigma = int dtau/tau * tau * L(tau) sigmahat, L(tau) = int_tau^1 dx/x f(x) f(tau/x);
   * substitute x = tau^v, v in (0,1): dx/x = -ln(tau) dv */
  double xs[4096], ws[4096];
  if (nodes > 4096) nodes = 4096;
  gauss_legendre(nodes, xs, ws);
  double S = p->sqrt_s * p->sqrt_s;
  double lt0 = log(p->m_lo * p->m_lo / S), lt1 = log(p->m_hi * p->m_hi / S);
  double total = 0.0;
  for (int i = 0; i < nodes; ++i) {
    double lt = 0.5 * (lt1 - lt0) * xs[i] + 0.5 * (lt1 + lt0);
    double tau = exp(lt);
    double lum = 0.0;
    for (int j = 0; j < nodes; ++j) {
      double v = 0.5 * xs[j] + 0.5;
      double x1 = exp(v * lt), x2 = tau / x1;
      double f = 4.0 / 9.0 * (or_xf_u(x1) * or_xf_qbar(x2) + or_xf_qbar(x1) * or_xf_u(x2))
               + 1.0 / 9.0 * (or_xf_d(x1) * or_xf_qbar(x2) + or_xf_qbar(x1) * or_xf_d(x2));
      /* f_a(x1) f_b(x2) = xf_a xf_b / (x1 x2) = xf xf / tau;  dx1/x1 = -lt dv */
      lum += 0.5 * ws[j] * (-lt) * f / tau;
    }
    double shat = tau * S;
    total += ws[i] * 0.5 * (lt1 - lt0) * tau * lum * 4.0 * M_PI * p->alpha * p->alpha / (9.0 * shat);
  }
  return total;
}

/* ------------------------------------------------- dilepton solutions --- */
/* Polynomial helpers, coefficients in ascending order. */
static double peval(const double* c, int n, double x)
{
  double r = c[n];
  for (int i = n - 1; i >= 0; --i) r = r * x + c[i];
  return r;
}

/* Real roots of a polynomial of degree n <= 4, found by isolating each
 * root between consecutive real roots of the derivative (where the
 * polynomial is monotone) and bisecting to the last representable bit.
 * Returns the count; roots ascending. */
static int real_roots(const double* c_in, int n, double* roots)
{
  double c[5];
  memcpy(c, c_in, sizeof(double) * (n + 1));
  while (n > 0 && c[n] == 0.0) --n;
  if (n == 0) return 0;
  if (n == 1) { roots[0] = -c[0] / c[1]; return 1; }
  double dc[4] = {0, 0, 0, 0};
  for (int i = 1; i <= n; ++i) dc[i - 1] = i * c[i];
  double crit[4];
  int nc = real_roots(dc, n - 1, crit);
  double bound = 0.0;
  for (int i = 0; i < n; ++i) bound = fmax(bound, fabs(c[i] / c[n]));
  bound = 1.0 + bound;
  double pts[6];
  int np = 0;
  pts[np++] = -bound;
  for (int i = 0; i < nc; ++i) if (crit[i] > -bound && crit[i] < bound) pts[np++] = crit[i];
  pts[np++] = bound;
  int nr = 0;
  for (int i = 0; i + 1 < np; ++i) {
    double lo = pts[i], hi = pts[i + 1];
    double flo = peval(c, n, lo), fhi = peval(c, n, hi);
    if (flo == 0.0) {                       /* exact root at the left end */
      if (nr == 0 || roots[nr - 1] != lo) roots[nr++] = lo;
      continue;
    }
    if (fhi == 0.0) {                       /* recorded as the next left end */
      if (i + 2 == np) roots[nr++] = hi;
      continue;
    }
    if ((flo < 0) == (fhi < 0)) continue;   /* monotone, no sign change */
    for (int it = 0; it < 2000; ++it) {
      double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      double fm = peval(c, n, mid);
      if (fm == 0.0) { lo = hi = mid; break; }
      if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
    }
    roots[nr++] = 0.5 * (lo + hi);
  }
  return nr;
}

/* Linear part of the neutrino constraints for one top: with E = |p|,
 * 2 l.nu = q2w and 2 b.nu = q2t - q2w - 2 b.l give E and p_z as affine
 * functions of (p_x, p_y): E = e0 + e1 px + e2 py, pz = z0 + z1 px + z2 py. */
static int nu_affine(const double* b, const double* l, double q2w, double q2t,
                     double e[3], double z[3])
{
  double h1 = 0.5 * q2w;
  double h2 = 0.5 * (q2t - q2w - 2.0 * mdot(b, l));
  double det = -l[0] * b[3] + l[3] * b[0];
  if (det == 0.0) return 0;
  e[0] = (-b[3] * h1 + l[3] * h2) / det;
  e[1] = (-b[3] * l[1] + l[3] * b[1]) / det;
  e[2] = (-b[3] * l[2] + l[3] * b[2]) / det;
  z[0] = (l[0] * h2 - b[0] * h1) / det;
  z[1] = (l[0] * b[1] - b[0] * l[1]) / det;
  z[2] = (l[0] * b[2] - b[0] * l[2]) / det;
  return 1;
}

/* conic coefficients {xx, xy, yy, x, y, 1} of E^2 - px^2 - py^2 - pz^2 = 0 */
static void conic_of(const double e[3], const double z[3], double c[6])
{
  c[0] = e[1] * e[1] - 1.0 - z[1] * z[1];
  c[1] = 2.0 * (e[1] * e[2] - z[1] * z[2]);
  c[2] = e[2] * e[2] - 1.0 - z[2] * z[2];
  c[3] = 2.0 * (e[0] * e[1] - z[0] * z[1]);
  c[4] = 2.0 * (e[0] * e[2] - z[0] * z[2]);
  c[5] = e[0] * e[0] - z[0] * z[0];
}

static void residuals(const double* b, const double* bb, const double* lp, const double* lm,
                      double mx, double my, const double v[4], double F[4], double Jm[16])
{
  double nu[4], nb[4];
  nu[1] = v[0]; nu[2] = v[1]; nu[3] = v[2];
  nb[1] = mx - v[0]; nb[2] = my - v[1]; nb[3] = v[3];
  nu[0] = norm3(nu); nb[0] = norm3(nb);
  double wt[4], wtb[4];
  for (int i = 0; i < 4; ++i) { wt[i] = b[i] + lp[i]; wtb[i] = bb[i] + lm[i]; }
  /* F = (q2_W+, q2_t, q2_W-, q2_tbar) at (nu, nubar) */
  F[0] = 2.0 * mdot(lp, nu);
  F[1] = mdot(wt, wt) + 2.0 * mdot(wt, nu);
  F[2] = 2.0 * mdot(lm, nb);
  F[3] = mdot(wtb, wtb) + 2.0 * mdot(wtb, nb);
  if (!Jm) return;
  /* d(a.nu)/d(nu_i) = a_E nu_i / E - a_i ;  nubar_x,y = met - nu_x,y */
  for (int i = 0; i < 3; ++i) {
    double dl = lp[0] * nu[i + 1] / nu[0] - lp[i + 1];
    double dw = wt[0] * nu[i + 1] / nu[0] - wt[i + 1];
    Jm[0 * 4 + i] = 2.0 * dl;
    Jm[1 * 4 + i] = 2.0 * dw;
  }
  Jm[0 * 4 + 3] = 0.0;
  Jm[1 * 4 + 3] = 0.0;
  double dlm[3], dwm[3];
  for (int i = 0; i < 3; ++i) {
    dlm[i] = 2.0 * (lm[0] * nb[i + 1] / nb[0] - lm[i + 1]);
    dwm[i] = 2.0 * (wtb[0] * nb[i + 1] / nb[0] - wtb[i + 1]);
  }
  Jm[2 * 4 + 0] = -dlm[0]; Jm[2 * 4 + 1] = -dlm[1]; Jm[2 * 4 + 2] = 0.0; Jm[2 * 4 + 3] = dlm[2];
  Jm[3 * 4 + 0] = -dwm[0]; Jm[3 * 4 + 1] = -dwm[1]; Jm[3 * 4 + 2] = 0.0; Jm[3 * 4 + 3] = dwm[2];
}

/* Gaussian elimination with partial pivoting; returns det and, if rhs is
 * given, solves A x = rhs in place. */
static double lu_det_solve(double A_in[16], double* rhs)
{
  double A[16];
  memcpy(A, A_in, sizeof(A));
  double det = 1.0;
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r) if (fabs(A[r * 4 + c]) > fabs(A[piv * 4 + c])) piv = r;
    if (A[piv * 4 + c] == 0.0) return 0.0;
    if (piv != c) {
      for (int k = 0; k < 4; ++k) { double t = A[c * 4 + k]; A[c * 4 + k] = A[piv * 4 + k]; A[piv * 4 + k] = t; }
      if (rhs) { double t = rhs[c]; rhs[c] = rhs[piv]; rhs[piv] = t; }
      det = -det;
    }
    det *= A[c * 4 + c];
    for (int r = c + 1; r < 4; ++r) {
      double f = A[r * 4 + c] / A[c * 4 + c];
      for (int k = c; k < 4; ++k) A[r * 4 + k] -= f * A[c * 4 + k];
      if (rhs) rhs[r] -= f * rhs[c];
    }
  }
  if (rhs)
    for (int r = 3; r >= 0; --r) {
      double s = rhs[r];
      for (int k = r + 1; k < 4; ++k) s -= A[r * 4 + k] * rhs[k];
      rhs[r] = s / A[r * 4 + r];
    }
  return det;
}

void or_dilepton_residual(const double* b, const double* bb, const double* lp,
                          const double* lm, const double* nu, const double* nub,
                          double* q2)
{
  double wt[4], wtb[4], wp[4], wm[4];
  for (int i = 0; i < 4; ++i) {
    wp[i] = lp[i] + nu[i]; wm[i] = lm[i] + nub[i];
    wt[i] = wp[i] + b[i]; wtb[i] = wm[i] + bb[i];
  }
  q2[0] = mdot(wp, wp); q2[1] = mdot(wt, wt); q2[2] = mdot(wm, wm); q2[3] = mdot(wtb, wtb);
}

int or_solve_dilepton(const double* b_in, const double* bb_in, const double* lp_in,
                      const double* lm_in, double metx, double mety,
                      double q2wp, double q2t, double q2wm, double q2tb,
                      double* nu_out, double* nub_out, double* detj_out)
{
  /* work in units of lam so that all polynomial coefficients are O(1) */
  double lam = 0.25 * (b_in[0] + bb_in[0] + lp_in[0] + lm_in[0]);
  double b[4], bb[4], lp[4], lm[4];
  for (int i = 0; i < 4; ++i) { b[i] = b_in[i] / lam; bb[i] = bb_in[i] / lam; lp[i] = lp_in[i] / lam; lm[i] = lm_in[i] / lam; }
  double mx = metx / lam, my = mety / lam, l2 = lam * lam;
  double qwp = q2wp / l2, qt = q2t / l2, qwm = q2wm / l2, qtb = q2tb / l2;

  double e1[3], z1[3], e2[3], z2[3];
  if (!nu_affine(b, lp, qwp, qt, e1, z1)) return 0;
  if (!nu_affine(bb, lm, qwm, qtb, e2, z2)) return 0;
  double c1[6], cb[6], c2[6];
  conic_of(e1, z1, c1);
  conic_of(e2, z2, cb);
  /* the nubar conic in (nubar_x, nubar_y) -> in (nu_x, nu_y) */
  c2[0] = cb[0]; c2[1] = cb[1]; c2[2] = cb[2];
  c2[3] = -2.0 * mx * cb[0] - my * cb[1] - cb[3];
  c2[4] = -2.0 * my * cb[2] - mx * cb[1] - cb[4];
  c2[5] = cb[0] * mx * mx + cb[1] * mx * my + cb[2] * my * my + cb[3] * mx + cb[4] * my + cb[5];
  /* each conic as A py^2 + B(px) py + C(px); resultant in py */
  double A1 = c1[2], A2 = c2[2];
  double B1[2] = {c1[4], c1[1]}, B2[2] = {c2[4], c2[1]};
  double C1[3] = {c1[5], c1[3], c1[0]}, C2[3] = {c2[5], c2[3], c2[0]};
  double P[3], Q[2], R[4] = {0, 0, 0, 0};
  for (int i = 0; i < 3; ++i) P[i] = A1 * C2[i] - A2 * C1[i];
  for (int i = 0; i < 2; ++i) Q[i] = A1 * B2[i] - A2 * B1[i];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) R[i + j] += B1[i] * C2[j] - B2[i] * C1[j];
  double res[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) res[i + j] += P[i] * P[j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 4; ++j) if (i + j <= 4) res[i + j] -= Q[i] * R[j];
  double roots[4];
  int nr = real_roots(res, 4, roots);
  int ns = 0;
  for (int k = 0; k < nr; ++k) {
    double px = roots[k];
    double q = Q[0] + Q[1] * px;
    double py;
    double pval = P[0] + P[1] * px + P[2] * px * px;
    if (fabs(q) > 1e-12 * (fabs(Q[0]) + fabs(Q[1] * px)) && q != 0.0) {
      py = -pval / q;
    } else {
      /* degenerate elimination: take the root of conic 1 that best
       * satisfies conic 2 */
      double a = A1, bq = B1[0] + B1[1] * px, cq = C1[0] + C1[1] * px + C1[2] * px * px;
      double disc = bq * bq - 4 * a * cq;
      if (disc < 0 || a == 0.0) continue;
      double y1 = (-bq + sqrt(disc)) / (2 * a), y2 = (-bq - sqrt(disc)) / (2 * a);
      double r1 = fabs(c2[0] * px * px + c2[1] * px * y1 + c2[2] * y1 * y1 + c2[3] * px + c2[4] * y1 + c2[5]);
      double r2 = fabs(c2[0] * px * px + c2[1] * px * y2 + c2[2] * y2 * y2 + c2[3] * px + c2[4] * y2 + c2[5]);
      py = r1 < r2 ? y1 : y2;
    }
    double E1 = e1[0] + e1[1] * px + e1[2] * py;
    double pz1 = z1[0] + z1[1] * px + z1[2] * py;
    double pbx = mx - px, pby = my - py;
    double E2 = e2[0] + e2[1] * pbx + e2[2] * pby;
    double pz2 = z2[0] + z2[1] * pbx + z2[2] * pby;
    if (!(E1 > 0.0 && E2 > 0.0)) continue;
    double v[4] = {px, py, pz1, pz2};
    double target[4] = {qwp, qt, qwm, qtb};
    double F[4], Jm[16];
    for (int it = 0; it < 2; ++it) {
      residuals(b, bb, lp, lm, mx, my, v, F, Jm);
      double rhs[4];
      for (int i = 0; i < 4; ++i) rhs[i] = F[i] - target[i];
      if (lu_det_solve(Jm, rhs) == 0.0) break;
      for (int i = 0; i < 4; ++i) v[i] -= rhs[i];
    }
    residuals(b, bb, lp, lm, mx, my, v, F, Jm);
    double worst = 0.0;
    for (int i = 0; i < 4; ++i) worst = fmax(worst, fabs(F[i] - target[i]) / fabs(target[i]));
    if (!(worst < 1e-6)) continue;
    double det = lu_det_solve(Jm, NULL);
    if (det == 0.0) continue;
    double* nu = nu_out + 4 * ns;
    double* nb = nub_out + 4 * ns;
    nu[1] = v[0] * lam; nu[2] = v[1] * lam; nu[3] = v[2] * lam;
    nb[1] = (mx - v[0]) * lam; nb[2] = (my - v[1]) * lam; nb[3] = v[3] * lam;
    nu[0] = norm3(nu); nb[0] = norm3(nb);
    /* the Jacobian has dimension GeV^4 (q2 per momentum) */
    detj_out[ns] = det * lam * lam * lam * lam;
    ++ns;
  }
  return ns;
}

/* ------------------------------------------------------ ttbar dilepton -- */
/* Breit-Wigner (tan) map of x onto q2 in [lo, hi]; returns the Jacobian */
double or_bw_map(double x, double m, double w, double lo, double hi, double* q2)
{
  double mw = m * w;
  double t0 = atan((lo - m * m) / mw), t1 = atan((hi - m * m) / mw);
  double th = t0 + x * (t1 - t0);
  *q2 = m * m + mw * tan(th);
  double d = *q2 - m * m;
  return (t1 - t0) * (d * d + mw * mw) / mw;
}

/* transverse boost that removes the total transverse momentum P_T */
static void boost_transverse(const double* P, const double* in, double* out)
{
  double bx = P[1] / P[0], by = P[2] / P[0];
  double b2 = bx * bx + by * by;
  double g = 1.0 / sqrt(1.0 - b2);
  double bp = bx * in[1] + by * in[2];
  double g2 = b2 > 0.0 ? (g - 1.0) / b2 : 0.0;
  out[0] = g * (in[0] - bp);
  out[1] = in[1] + g2 * bp * bx - g * bx * in[0];
  out[2] = in[2] + g2 * bp * by - g * by * in[0];
  out[3] = in[3];
}

int or_dims(int kind)
{
  return (kind == OR_KIND_DY || kind == OR_KIND_STEP) ? 2 : kind == OR_KIND_GENZ ? 4
       : (kind == OR_KIND_TT_SL || kind == OR_KIND_TT_SL_DIRECT) ? 7 : kind == OR_KIND_TTH ? 9 : 8;
}
int or_nperm(int kind)
{
  return (kind == OR_KIND_TT || kind == OR_KIND_TT_DIRECT) ? 2
       : (kind == OR_KIND_TT_SL || kind == OR_KIND_TT_SL_DIRECT) ? 12 : kind == OR_KIND_TTH ? 24
       : (kind == OR_KIND_TTH_LL || kind == OR_KIND_TTH_LL_DIRECT) ? 12 : kind == OR_KIND_TTBB_LL ? 24 : 1;
}

double or_genz_integrand(const double* x)
{
  double f = 1.0;
  for (int d = 0; d < 4; ++d) {
    double c = 0.3 + 0.1 * d, a = 20.0;
    f *= a / (1.0 + a * a * (x[d] - c) * (x[d] - c));
  }
  return f;
}

double or_genz_exact(void)
{
  double v = 1.0;
  for (int d = 0; d < 4; ++d) {
    double c = 0.3 + 0.1 * d, a = 20.0;
    v *= atan(a * (1.0 - c)) + atan(a * c);
  }
  return v;
}

double or_tt_integrand(const or_params* p, const double* ev, int perm,
                       const double* x, int* nsol_out)
{
  const double S = p->sqrt_s * p->sqrt_s;
  const double* jet[2] = {ev + (perm ? 4 : 0), ev + (perm ? 0 : 4)};
  const double* lp = ev + 8;
  const double* lm = ev + 12;
  if (nsol_out) *nsol_out = 0;
  /* jet energies through r = E_meas / E_true, directions fixed */
  double bq[2][4];
  double jetf = 1.0;
  for (int k = 0; k < 2; ++k) {
    const double* m = jet[k];
    double em = m[0], pm = norm3(m);
    double r = p->r_lo + x[k] * (p->r_hi - p->r_lo);
    double E = em / r;
    double jac = (p->r_hi - p->r_lo) * em / (r * r);
    bq[k][0] = E;
    for (int i = 1; i < 4; ++i) bq[k][i] = m[i] / pm * E;
    double sin_th = sqrt(m[1] * m[1] + m[2] * m[2]) / pm;
    /* E^2 sin(theta) dE T(E_meas | E) / (2E), massless partons */
    jetf *= E * E * sin_th * or_gauss_tf(em, E, p->tf_sigma) / (2.0 * E) * jac;
  }
  double q2t, q2tb, q2wp, q2wm;
  double jbw = or_bw_map(x[2], p->m_t, p->w_t, 0.0, S, &q2t)
             * or_bw_map(x[3], p->m_t, p->w_t, 0.0, S, &q2tb)
             * or_bw_map(x[4], p->m_w, p->w_w, 0.0, S, &q2wp)
             * or_bw_map(x[5], p->m_w, p->w_w, 0.0, S, &q2wm);
  /* recoil k_T drawn from its Gaussian prior: the prior density times the
   * Jacobian of this (Box-Muller) map is one */
  double rho = p->sigma_k * sqrt(-2.0 * log(1.0 - x[6]));
  double phi = 2.0 * M_PI * x[7];
  double kx = rho * cos(phi), ky = rho * sin(phi);
  /* missing transverse momentum at this point (Sec. 4), shifted by k_T */
  double metx = kx - (bq[0][1] + bq[1][1] + lp[1] + lm[1]);
  double mety = ky - (bq[0][2] + bq[1][2] + lp[2] + lm[2]);
  double nu[16], nub[16], detj[4];
  int ns = or_solve_dilepton(bq[0], bq[1], lp, lm, metx, mety, q2wp, q2t, q2wm, q2tb, nu, nub, detj);
  if (nsol_out) *nsol_out = ns;
  double sum = 0.0;
  for (int s = 0; s < ns; ++s) {
    const double* v = nu + 4 * s;
    const double* vb = nub + 4 * s;
    double lab[6][4];
    memcpy(lab[0], bq[0], sizeof(lab[0])); memcpy(lab[1], lp, sizeof(lab[1]));
    memcpy(lab[2], v, sizeof(lab[2]));     memcpy(lab[3], bq[1], sizeof(lab[3]));
    memcpy(lab[4], lm, sizeof(lab[4]));    memcpy(lab[5], vb, sizeof(lab[5]));
    double P[4] = {0, 0, 0, 0};
    for (int k = 0; k < 6; ++k) for (int i = 0; i < 4; ++i) P[i] += lab[k][i];
    double hard[24];
    for (int k = 0; k < 6; ++k) boost_transverse(P, lab[k], hard + 4 * k);
    double Eh = sqrt(P[0] * P[0] - P[1] * P[1] - P[2] * P[2]);
    double x1 = (Eh + P[3]) / p->sqrt_s, x2 = (Eh - P[3]) / p->sqrt_s;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    double k1[4] = {0.5 * x1 * p->sqrt_s, 0, 0, 0.5 * x1 * p->sqrt_s};
    double k2[4] = {0.5 * x2 * p->sqrt_s, 0, 0, -0.5 * x2 * p->sqrt_s};
    const tt_lumi L = tt_lumis(p, x1, x2);
    double me = L.gg * or_tt_me2_gg(p, k1, k2, hard)
              + L.qq12 * or_tt_me2_qq(p, k1, k2, hard)
              + L.qq21 * or_tt_me2_qq(p, k2, k1, hard);
    double shat = x1 * x2 * S;
    double f = (2.0 / S) * (P[0] / Eh) * me / (2.0 * shat)
             / fabs(detj[s]) / (2.0 * v[0] * 2.0 * vb[0]);
    sum += f;
  }
  double two_pi_pow = pow(2.0 * M_PI, 4.0 - 3.0 * 6.0);
  double lep = 1.0 / (2.0 * lp[0] * 2.0 * lm[0]);
  return sum * two_pi_pow * lep * jetf * jbw;
}

/* ------------------------------------------------- ttbar semileptonic -- */
/* The weight of one assignment: jets b (from t) and bb, the leptons and
 * neutrinos as given (Eq. integrand with every transfer function a delta
 * function: only the flux, the x1, x2 delta functions and |M|^2 x PDFs
 * remain). */
static double parton_assignment(const or_params* p, const double* b, const double* bb, const double* lp,
                                const double* lm, const double* nu, const double* nub)
{
  const double S = p->sqrt_s * p->sqrt_s;
  double lab[6][4];
  memcpy(lab[0], b, sizeof(lab[0]));   memcpy(lab[1], lp, sizeof(lab[1]));
  memcpy(lab[2], nu, sizeof(lab[2]));  memcpy(lab[3], bb, sizeof(lab[3]));
  memcpy(lab[4], lm, sizeof(lab[4]));  memcpy(lab[5], nub, sizeof(lab[5]));
  double P[4] = {0, 0, 0, 0};
  for (int k = 0; k < 6; ++k) for (int i = 0; i < 4; ++i) P[i] += lab[k][i];
  double hard[24];
  for (int k = 0; k < 6; ++k) boost_transverse(P, lab[k], hard + 4 * k);
  double Eh = sqrt(P[0] * P[0] - P[1] * P[1] - P[2] * P[2]);
  double x1 = (Eh + P[3]) / p->sqrt_s, x2 = (Eh - P[3]) / p->sqrt_s;
  if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) return 0.0;
  double k1[4] = {0.5 * x1 * p->sqrt_s, 0, 0, 0.5 * x1 * p->sqrt_s};
  double k2[4] = {0.5 * x2 * p->sqrt_s, 0, 0, -0.5 * x2 * p->sqrt_s};
  const tt_lumi L = tt_lumis(p, x1, x2);
  double me = L.gg * or_tt_me2_gg(p, k1, k2, hard)
            + L.qq12 * or_tt_me2_qq(p, k1, k2, hard)
            + L.qq21 * or_tt_me2_qq(p, k2, k1, hard);
  double shat = x1 * x2 * S;
  return (2.0 / S) * (P[0] / Eh) * me / (2.0 * shat);
}

double or_tt_parton_weight(const or_params* p, const double* ev)
{
  const double *b = ev, *bb = ev + 4, *lp = ev + 8, *lm = ev + 12, *nu = ev + 16, *nub = ev + 20;
  return 0.5 * (parton_assignment(p, b, bb, lp, lm, nu, nub) + parton_assignment(p, bb, b, lp, lm, nu, nub));
}

double or_dgauss_tf(double meas, double truth, double core, double tail, double ftail)
{
  return (1.0 - ftail) * or_gauss_tf(meas, truth, core) + ftail * or_gauss_tf(meas, truth, tail);
}

void or_semilep_perm(int perm, int* i_bl, int* i_bh, int* i_ja, int* i_jb)
{
  int bl = perm / 3, r = perm % 3;
  int bh = r < bl ? r : r + 1;          /* the r-th jet other than bl */
  int rest[2], n = 0;
  for (int j = 0; j < 4; ++j) if (j != bl && j != bh) rest[n++] = j;
  *i_bl = bl; *i_bh = bh; *i_ja = rest[0]; *i_jb = rest[1];
}

/* The jet-energy part of the semileptonic map: x0 -> E_a (r map of light
 * jet a), x1 -> q2 of the hadronic W -> E_b = q2/(2 E_a (1 - cos)),
 * x2 -> q2 of the hadronic top -> E_bh linear in q2, x3 -> E_bl (r map).
 * Writes (E_a, E_b, E_bh, E_bl); returns the Jacobian
 * |d(E_a, E_b, E_bh, E_bl)/d(x0..x3)| or 0 outside the TF windows. */
double or_semilep_map(const or_params* p, const double* ev, int perm, const double* x, double* E4)
{
  const double S = p->sqrt_s * p->sqrt_s;
  int ibl, ibh, ja, jb;
  or_semilep_perm(perm, &ibl, &ibh, &ja, &jb);
  double dir[4][3], em[4];
  for (int k = 0; k < 4; ++k) {
    const double* m = ev + 4 * k;
    double pm = norm3(m);
    em[k] = m[0];
    for (int i = 0; i < 3; ++i) dir[k][i] = m[i + 1] / pm;
  }
  double jac = 1.0;
  double ra = p->lj_r_lo + x[0] * (p->lj_r_hi - p->lj_r_lo);
  double Ea = em[ja] / ra;
  jac *= (p->lj_r_hi - p->lj_r_lo) * em[ja] / (ra * ra);
  double q2wh;
  jac *= or_bw_map(x[1], p->m_w, p->w_w, 0.0, S, &q2wh);
  double ca = dir[ja][0] * dir[jb][0] + dir[ja][1] * dir[jb][1] + dir[ja][2] * dir[jb][2];
  if (!(1.0 - ca > 0.0)) return 0.0;
  double Eb = q2wh / (2.0 * Ea * (1.0 - ca));
  jac *= 1.0 / (2.0 * Ea * (1.0 - ca));
  double q2th;
  jac *= or_bw_map(x[2], p->m_t, p->w_t, 0.0, S, &q2th);
  double W[4] = {Ea + Eb, Ea * dir[ja][0] + Eb * dir[jb][0], Ea * dir[ja][1] + Eb * dir[jb][1],
                 Ea * dir[ja][2] + Eb * dir[jb][2]};
  double den = 2.0 * (W[0] - (dir[ibh][0] * W[1] + dir[ibh][1] * W[2] + dir[ibh][2] * W[3]));
  if (!(den > 0.0)) return 0.0;
  double Ebh = (q2th - q2wh) / den;
  if (!(Ebh > 0.0)) return 0.0;
  jac *= 1.0 / den;
  double rb = p->r_lo + x[3] * (p->r_hi - p->r_lo);
  double Ebl = em[ibl] / rb;
  jac *= (p->r_hi - p->r_lo) * em[ibl] / (rb * rb);
  double rr_b = em[jb] / Eb, rr_h = em[ibh] / Ebh;
  if (rr_b < p->lj_r_lo || rr_b > p->lj_r_hi || rr_h < p->r_lo || rr_h > p->r_hi) return 0.0;
  E4[0] = Ea; E4[1] = Eb; E4[2] = Ebh; E4[3] = Ebl;
  return jac;
}

/* nu_z from 2 l.nu = q2 at fixed nu_T (massless l, nu): squaring gives
 * l_T^2 nu_z^2 - 2 a l_z nu_z + E_l^2 nu_T^2 - a^2 = 0, a = q2/2 + l_T.nu_T;
 * both roots satisfy the unsquared equation iff a > 0.  Returns the count. */
int or_semilep_nu_z(const double* l, double nx, double ny, double q2, double* nz)
{
  double lt2 = l[1] * l[1] + l[2] * l[2];
  double a = 0.5 * q2 + l[1] * nx + l[2] * ny;
  double disc = a * a - lt2 * (nx * nx + ny * ny);
  if (!(a > 0.0) || disc < 0.0 || !(lt2 > 0.0)) return 0;
  double sq = l[0] * sqrt(disc);
  nz[0] = (a * l[3] + sq) / lt2;
  nz[1] = (a * l[3] - sq) / lt2;
  return 2;
}

/* Variables: x0..x3 jet energies (or_semilep_map); x4, x5 recoil k_T;
 * x6 q2 of the leptonic W (-> nu_z).  Sec. 3 / Eq. integrand with one
 * hadronic W. */
double or_tt_semilep_integrand(const or_params* p, const double* ev, int lep_charge, int perm,
                               const double* x, int* nsol_out)
{
  const double S = p->sqrt_s * p->sqrt_s;
  if (lep_charge == 0) lep_charge = ev[20] > 0 ? 1 : -1;
  int ibl, ibh, ja, jb;
  or_semilep_perm(perm, &ibl, &ibh, &ja, &jb);
  const double* l = ev + 16;
  if (nsol_out) *nsol_out = 0;
  double E4[4];
  double jac = or_semilep_map(p, ev, perm, x, E4);
  if (jac == 0.0) return 0.0;
  double qa[4], qb[4], bh[4], bl[4];
  const int idx[4] = {ja, jb, ibh, ibl};
  double* dst[4] = {qa, qb, bh, bl};
  double tf = 1.0;
  for (int k = 0; k < 4; ++k) {
    const double* m = ev + 4 * idx[k];
    double pm = norm3(m), E = E4[k];
    dst[k][0] = E;
    for (int i = 0; i < 3; ++i) dst[k][i + 1] = E * m[i + 1] / pm;
    double sin_th = sqrt(m[1] * m[1] + m[2] * m[2]) / pm;
    double T = k < 2 ? or_dgauss_tf(m[0], E, p->lj_core, p->lj_tail, p->lj_ftail)
                     : or_gauss_tf(m[0], E, p->tf_sigma);
    /* E^2 sin dE T / (2E) */
    tf *= E * E * sin_th * T / (2.0 * E);
  }
  /* recoil and neutrino transverse momentum */
  double rho = p->sigma_k * sqrt(-2.0 * log(1.0 - x[4]));
  double phi = 2.0 * M_PI * x[5];
  double nx = rho * cos(phi) - (qa[1] + qb[1] + bh[1] + bl[1] + l[1]);
  double ny = rho * sin(phi) - (qa[2] + qb[2] + bh[2] + bl[2] + l[2]);
  /* leptonic W: 2 l.nu = q2 -> quadratic in nu_z */
  double q2wl;
  jac *= or_bw_map(x[6], p->m_w, p->w_w, 0.0, S, &q2wl);
  double nzs[2];
  int nroot = or_semilep_nu_z(l, nx, ny, q2wl, nzs);
  double sum = 0.0;
  int ns = 0;
  for (int s = 0; s < nroot; ++s) {
    double nz = nzs[s];
    double nu[4] = {sqrt(nx * nx + ny * ny + nz * nz), nx, ny, nz};
    double dq = fabs(2.0 * (l[0] * nz / nu[0] - l[3]));
    if (!(dq > 0.0)) continue;
    ++ns;
    double P[4];
    for (int i = 0; i < 4; ++i) P[i] = qa[i] + qb[i] + bh[i] + bl[i] + l[i] + nu[i];
    double Eh = sqrt(P[0] * P[0] - P[1] * P[1] - P[2] * P[2]);
    double x1 = (Eh + P[3]) / p->sqrt_s, x2 = (Eh - P[3]) / p->sqrt_s;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    double k1[4] = {0.5 * x1 * p->sqrt_s, 0, 0, 0.5 * x1 * p->sqrt_s};
    double k2[4] = {0.5 * x2 * p->sqrt_s, 0, 0, -0.5 * x2 * p->sqrt_s};
    double hq[2][4], hbh[4], hbl[4], hl[4], hn[4];
    boost_transverse(P, qa, hq[0]);
    boost_transverse(P, qb, hq[1]);
    boost_transverse(P, bh, hbh);
    boost_transverse(P, bl, hbl);
    boost_transverse(P, l, hl);
    boost_transverse(P, nu, hn);
    const tt_lumi L = tt_lumis(p, x1, x2);
    double me = 0.0;
    for (int o = 0; o < 2; ++o) {
      /* light-jet ordering o: (quark, antiquark) of the hadronic W */
      const double* qk = hq[o];
      const double* qbk = hq[1 - o];
      double mom[24];
      if (lep_charge > 0) {
        /* t -> b l+ nu, tbar -> bbar d ubar: W- current ubar(d) .. v(ubar) */
        memcpy(mom, hbl, 32); memcpy(mom + 4, hl, 32); memcpy(mom + 8, hn, 32);
        memcpy(mom + 12, hbh, 32); memcpy(mom + 16, qk, 32); memcpy(mom + 20, qbk, 32);
      } else {
        /* t -> b u dbar, tbar -> bbar l- nubar: W+ current ubar(u) .. v(dbar) */
        memcpy(mom, hbh, 32); memcpy(mom + 4, qbk, 32); memcpy(mom + 8, qk, 32);
        memcpy(mom + 12, hbl, 32); memcpy(mom + 16, hl, 32); memcpy(mom + 20, hn, 32);
      }
      me += L.gg * or_tt_me2_gg(p, k1, k2, mom) + L.qq12 * or_tt_me2_qq(p, k1, k2, mom)
          + L.qq21 * or_tt_me2_qq(p, k2, k1, mom);
    }
    me *= 3.0 * 2.0;   /* colour of the hadronic W, two quark generations */
    double shat = x1 * x2 * S;
    sum += (2.0 / S) * (P[0] / Eh) * me / (2.0 * shat) / dq / (2.0 * nu[0]);
  }
  if (nsol_out) *nsol_out = ns;
  double two_pi_pow = pow(2.0 * M_PI, 4.0 - 3.0 * 6.0);
  return sum * two_pi_pow * tf * jac / (2.0 * l[0]);
}

/* -------------------------------------------------------------- ttbar H -- */
/* Event rows: four b-tagged jets b0..b3, two light jets l0, l1, the lepton,
 * then (charge, 0, 0, 0).  Assignment perm in [0, 24): o = perm % 2 picks
 * the quark of the hadronic W (l0 for o = 0, l1 for o = 1); perm / 2 in
 * [0, 12) picks the b pair of the Higgs (6 pairs, ascending) and which of
 * the two remaining b-jets comes from the leptonic top (the lower one for
 * an even value). */
void or_tth_perm(int perm, int* i_h1, int* i_h2, int* i_bl, int* i_bh, int* o)
{
  static const int pairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  *o = perm & 1;
  int bp = perm >> 1, hp = bp >> 1;
  *i_h1 = pairs[hp][0];
  *i_h2 = pairs[hp][1];
  int rest[2], n = 0;
  for (int j = 0; j < 4; ++j) if (j != *i_h1 && j != *i_h2) rest[n++] = j;
  *i_bl = (bp & 1) ? rest[1] : rest[0];
  *i_bh = (bp & 1) ? rest[0] : rest[1];
}

/* Jet energies of the ttH map (all jets double-Gaussian, one r window):
 * x0 -> E(l0) (r map), x1 -> hadronic W q2 -> E(l1), x2 -> hadronic top q2
 * -> E(b_h), x3 -> E(b_l) (r map), x7 -> E(h1) (r map), x8 -> Higgs q2 ->
 * E(h2) = q2 / (2 E(h1) (1 - cos)).  E6 = (l0, l1, b_h, b_l, h1, h2);
 * returns the Jacobian or 0 outside the windows. */
double or_tth_map(const or_params* p, const double* ev, int perm, const double* x, double* E6)
{
  const double S = p->sqrt_s * p->sqrt_s;
  int ih1, ih2, ibl, ibh, o;
  or_tth_perm(perm, &ih1, &ih2, &ibl, &ibh, &o);
  const int rows[6] = {4, 5, ibh, ibl, ih1, ih2};
  double dir[6][3], em[6];
  for (int k = 0; k < 6; ++k) {
    const double* m = ev + 4 * rows[k];
    double pm = norm3(m);
    em[k] = m[0];
    for (int i = 0; i < 3; ++i) dir[k][i] = m[i + 1] / pm;
  }
  const double rlo = p->lj_r_lo, rhi = p->lj_r_hi;
  double jac = 1.0;
  double ra = rlo + x[0] * (rhi - rlo);
  double Ea = em[0] / ra;
  jac *= (rhi - rlo) * em[0] / (ra * ra);
  double q2wh;
  jac *= or_bw_map(x[1], p->m_w, p->w_w, 0.0, S, &q2wh);
  double ca = dir[0][0] * dir[1][0] + dir[0][1] * dir[1][1] + dir[0][2] * dir[1][2];
  if (!(1.0 - ca > 0.0)) return 0.0;
  double Eb = q2wh / (2.0 * Ea * (1.0 - ca));
  jac *= 1.0 / (2.0 * Ea * (1.0 - ca));
  double q2th;
  jac *= or_bw_map(x[2], p->m_t, p->w_t, 0.0, S, &q2th);
  double W[4] = {Ea + Eb, Ea * dir[0][0] + Eb * dir[1][0], Ea * dir[0][1] + Eb * dir[1][1],
                 Ea * dir[0][2] + Eb * dir[1][2]};
  double den = 2.0 * (W[0] - (dir[2][0] * W[1] + dir[2][1] * W[2] + dir[2][2] * W[3]));
  if (!(den > 0.0)) return 0.0;
  double Ebh = (q2th - q2wh) / den;
  if (!(Ebh > 0.0)) return 0.0;
  jac *= 1.0 / den;
  double rl = rlo + x[3] * (rhi - rlo);
  double Ebl = em[3] / rl;
  jac *= (rhi - rlo) * em[3] / (rl * rl);
  double r1 = rlo + x[7] * (rhi - rlo);
  double E1 = em[4] / r1;
  jac *= (rhi - rlo) * em[4] / (r1 * r1);
  double q2h;
  jac *= or_bw_map(x[8], p->m_h, p->w_h, 0.0, S, &q2h);
  double c12 = dir[4][0] * dir[5][0] + dir[4][1] * dir[5][1] + dir[4][2] * dir[5][2];
  if (!(1.0 - c12 > 0.0)) return 0.0;
  double E2 = q2h / (2.0 * E1 * (1.0 - c12));
  jac *= 1.0 / (2.0 * E1 * (1.0 - c12));
  const double rs[3] = {em[1] / Eb, em[2] / Ebh, em[5] / E2};
  for (int k = 0; k < 3; ++k)
    if (rs[k] < rlo || rs[k] > rhi) return 0.0;
  E6[0] = Ea; E6[1] = Eb; E6[2] = Ebh; E6[3] = Ebl; E6[4] = E1; E6[5] = E2;
  return jac;
}

/* Variables: x0..x3, x7, x8 jet energies (or_tth_map); x4, x5 recoil k_T;
 * x6 leptonic W q2 (-> nu_z).  gg -> t tbar H, H -> b bbar, one W -> l nu,
 * one W -> q qbar'. */
double or_tth_integrand(const or_params* p, const double* ev, int lep_charge, int perm, const double* x,
                        int* nsol_out)
{
  const double S = p->sqrt_s * p->sqrt_s;
  if (lep_charge == 0) lep_charge = ev[28] > 0 ? 1 : -1;
  int ih1, ih2, ibl, ibh, o;
  or_tth_perm(perm, &ih1, &ih2, &ibl, &ibh, &o);
  const double* l = ev + 24;
  if (nsol_out) *nsol_out = 0;
  double E6[6];
  double jac = or_tth_map(p, ev, perm, x, E6);
  if (jac == 0.0) return 0.0;
  const int rows[6] = {4, 5, ibh, ibl, ih1, ih2};
  double j4[6][4];
  double tf = 1.0;
  for (int k = 0; k < 6; ++k) {
    const double* m = ev + 4 * rows[k];
    double pm = norm3(m), E = E6[k];
    j4[k][0] = E;
    for (int i = 0; i < 3; ++i) j4[k][i + 1] = E * m[i + 1] / pm;
    double sin_th = sqrt(m[1] * m[1] + m[2] * m[2]) / pm;
    double T = or_dgauss_tf(m[0], E, p->lj_core, p->lj_tail, p->lj_ftail);
    tf *= E * E * sin_th * T / (2.0 * E);
  }
  double rho = p->sigma_k * sqrt(-2.0 * log(1.0 - x[4]));
  double phi = 2.0 * M_PI * x[5];
  double vx = 0.0, vy = 0.0;
  for (int k = 0; k < 6; ++k) { vx += j4[k][1]; vy += j4[k][2]; }
  double nx = rho * cos(phi) - (vx + l[1]);
  double ny = rho * sin(phi) - (vy + l[2]);
  double q2wl;
  jac *= or_bw_map(x[6], p->m_w, p->w_w, 0.0, S, &q2wl);
  double nzs[2];
  int nroot = or_semilep_nu_z(l, nx, ny, q2wl, nzs);
  double sum = 0.0;
  int ns = 0;
  for (int s = 0; s < nroot; ++s) {
    double nz = nzs[s];
    double nu[4] = {sqrt(nx * nx + ny * ny + nz * nz), nx, ny, nz};
    double dq = fabs(2.0 * (l[0] * nz / nu[0] - l[3]));
    if (!(dq > 0.0)) continue;
    ++ns;
    double P[4];
    for (int i = 0; i < 4; ++i) {
      P[i] = l[i] + nu[i];
      for (int k = 0; k < 6; ++k) P[i] += j4[k][i];
    }
    double Eh = sqrt(P[0] * P[0] - P[1] * P[1] - P[2] * P[2]);
    double x1 = (Eh + P[3]) / p->sqrt_s, x2 = (Eh - P[3]) / p->sqrt_s;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    double k1[4] = {0.5 * x1 * p->sqrt_s, 0, 0, 0.5 * x1 * p->sqrt_s};
    double k2[4] = {0.5 * x2 * p->sqrt_s, 0, 0, -0.5 * x2 * p->sqrt_s};
    double h[6][4], hl[4], hn[4];
    for (int k = 0; k < 6; ++k) boost_transverse(P, j4[k], h[k]);
    boost_transverse(P, l, hl);
    boost_transverse(P, nu, hn);
    const double* qk = h[o];
    const double* qbk = h[1 - o];
    double mom[24];
    if (lep_charge > 0) {
      memcpy(mom, h[3], 32); memcpy(mom + 4, hl, 32); memcpy(mom + 8, hn, 32);
      memcpy(mom + 12, h[2], 32); memcpy(mom + 16, qk, 32); memcpy(mom + 20, qbk, 32);
    } else {
      memcpy(mom, h[2], 32); memcpy(mom + 4, qbk, 32); memcpy(mom + 8, qk, 32);
      memcpy(mom + 12, h[3], 32); memcpy(mom + 16, hl, 32); memcpy(mom + 20, hn, 32);
    }
    double g1, g2;
    if (p->pdf) {
      g1 = or_pdf_interp(p->pdf, 0, x1, p->m_t) / x1;
      g2 = or_pdf_interp(p->pdf, 0, x2, p->m_t) / x2;
    } else {
      g1 = or_xf_g(x1) / x1;
      g2 = or_xf_g(x2) / x2;
    }
    double me = g1 * g2 * or_tth_me2_gg(p, k1, k2, mom, h[4], h[5]) * 3.0 * 2.0;
    double shat = x1 * x2 * S;
    sum += (2.0 / S) * (P[0] / Eh) * me / (2.0 * shat) / dq / (2.0 * nu[0]);
  }
  if (nsol_out) *nsol_out = ns;
  double two_pi_pow = pow(2.0 * M_PI, 4.0 - 3.0 * 8.0);
  return sum * two_pi_pow * tf * jac / (2.0 * l[0]);
}

/* ------------------------------------- t tbar H against t tbar b bbar -- */
/* Sec. 4's analysis in the dilepton channel: four b-jets (event rows 0-3),
 * l+ (row 4), l- (row 5).  Jet assignments (the outer sum of Eq.
 * integrand):
 *   OR_KIND_TTH_LL, 12: perm = 2 hp + s; the Higgs pair is the hp-th of the
 *     six ascending jet pairs, the other two jets (ascending) go to b and
 *     bbar of the tops in that order for s = 0 and swapped for s = 1;
 *   OR_KIND_TTBB_LL, 24: the perm-th permutation in lexicographic order of
 *     the four jets onto (b, bbar, b', bbar'), b' bbar' the gluon's pair.
 * rows[0..3] = event rows of (b, bbar, pair jet 1, pair jet 2). */
void or_f2_perm(int kind, int perm, int* rows)
{
  if (kind == OR_KIND_TTH_LL) {
    static const int pairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    int hp = perm >> 1, s = perm & 1;
    rows[2] = pairs[hp][0];
    rows[3] = pairs[hp][1];
    int rest[2], n = 0;
    for (int j = 0; j < 4; ++j) if (j != rows[2] && j != rows[3]) rest[n++] = j;
    rows[0] = rest[s];
    rows[1] = rest[1 - s];
    return;
  }
  /* lexicographic permutation number perm of (0, 1, 2, 3) */
  int avail[4] = {0, 1, 2, 3}, na = 4, r = perm;
  static const int fact[4] = {6, 2, 1, 1};
  for (int k = 0; k < 4; ++k) {
    int q = r / fact[k];
    r %= fact[k];
    rows[k] = avail[q];
    for (int j = q; j < na - 1; ++j) avail[j] = avail[j + 1];
    --na;
  }
}

/* Variables x in [0,1]^8 (the paper's eight: four jet energies, four
 * propagator virtualities of Eq. dilepsolv):
 *   x0, x1  r = E_meas / E of the b and bbar jets
 *   x2..x5  q2 of t, tbar, W+, W- (tan maps over [0, S])
 *   x6      r of pair jet 1
 *   x7      t tbar H: q2 of the Higgs (tan map; Eq. mhsolve) giving the
 *           energy of pair jet 2; t tbar b bbar: r of pair jet 2.
 * All four jets carry the Gaussian TF of the b-jets.  The neutrinos'
 * transverse momenta add up to minus that of the visible objects (the
 * transverse momentum balance of Sec. 3; no recoil).  Only the gg initial
 * state. */
/* direct_e4: x7 is the r map of pair jet 2 for either kind (the direct
 * parametrisation of the t tbar H integral, a closure check). */
static double f2_integrand_me(int kind, int direct_e4, const or_params* p, const double* ev, int perm,
                              const double* x, int* nsol_out)
{
  const double S = p->sqrt_s * p->sqrt_s;
  int rows[4];
  or_f2_perm(kind, perm, rows);
  const double* lp = ev + 16;
  const double* lm = ev + 20;
  if (nsol_out) *nsol_out = 0;
  double dir[4][3], em[4], sin_th[4];
  for (int k = 0; k < 4; ++k) {
    const double* m = ev + 4 * rows[k];
    double pm = norm3(m);
    em[k] = m[0];
    for (int i = 0; i < 3; ++i) dir[k][i] = m[i + 1] / pm;
    sin_th[k] = sqrt(m[1] * m[1] + m[2] * m[2]) / pm;
  }
  const double rlo = p->r_lo, rhi = p->r_hi;
  double E[4], jac = 1.0;
  const int xr[3] = {0, 1, 6};
  for (int k = 0; k < 3; ++k) {
    double r = rlo + x[xr[k]] * (rhi - rlo);
    E[k] = em[k] / r;
    jac *= (rhi - rlo) * em[k] / (r * r);
  }
  double q2h = 0.0;
  if (kind == OR_KIND_TTH_LL && !direct_e4) {
    jac *= or_bw_map(x[7], p->m_h, p->w_h, 0.0, S, &q2h);
    double c12 = dir[2][0] * dir[3][0] + dir[2][1] * dir[3][1] + dir[2][2] * dir[3][2];
    if (!(1.0 - c12 > 0.0)) return 0.0;
    E[3] = q2h / (2.0 * E[2] * (1.0 - c12));
    jac *= 1.0 / (2.0 * E[2] * (1.0 - c12));
    double r3 = em[3] / E[3];
    if (r3 < rlo || r3 > rhi) return 0.0;
  } else {
    double r = rlo + x[7] * (rhi - rlo);
    E[3] = em[3] / r;
    jac *= (rhi - rlo) * em[3] / (r * r);
  }
  double j4[4][4];
  double jetf = 1.0;
  for (int k = 0; k < 4; ++k) {
    j4[k][0] = E[k];
    for (int i = 0; i < 3; ++i) j4[k][i + 1] = E[k] * dir[k][i];
    /* E^2 sin(theta) T(E_meas | E) / (2E) */
    jetf *= E[k] * E[k] * sin_th[k] * or_gauss_tf(em[k], E[k], p->tf_sigma) / (2.0 * E[k]);
  }
  double q2t, q2tb, q2wp, q2wm;
  jac *= or_bw_map(x[2], p->m_t, p->w_t, 0.0, S, &q2t) * or_bw_map(x[3], p->m_t, p->w_t, 0.0, S, &q2tb)
       * or_bw_map(x[4], p->m_w, p->w_w, 0.0, S, &q2wp) * or_bw_map(x[5], p->m_w, p->w_w, 0.0, S, &q2wm);
  double metx = -(lp[1] + lm[1]), mety = -(lp[2] + lm[2]);
  for (int k = 0; k < 4; ++k) { metx -= j4[k][1]; mety -= j4[k][2]; }
  double nu[16], nub[16], detj[4];
  int ns = or_solve_dilepton(j4[0], j4[1], lp, lm, metx, mety, q2wp, q2t, q2wm, q2tb, nu, nub, detj);
  if (nsol_out) *nsol_out = ns;
  double sum = 0.0;
  for (int s = 0; s < ns; ++s) {
    const double* v = nu + 4 * s;
    const double* vb = nub + 4 * s;
    double lab[8][4];
    memcpy(lab[0], j4[0], 32); memcpy(lab[1], lp, 32); memcpy(lab[2], v, 32);
    memcpy(lab[3], j4[1], 32); memcpy(lab[4], lm, 32); memcpy(lab[5], vb, 32);
    memcpy(lab[6], j4[2], 32); memcpy(lab[7], j4[3], 32);
    double P[4] = {0, 0, 0, 0};
    for (int k = 0; k < 8; ++k) for (int i = 0; i < 4; ++i) P[i] += lab[k][i];
    double hard[32];
    for (int k = 0; k < 8; ++k) boost_transverse(P, lab[k], hard + 4 * k);
    double Eh = sqrt(P[0] * P[0] - P[1] * P[1] - P[2] * P[2]);
    double x1 = (Eh + P[3]) / p->sqrt_s, x2 = (Eh - P[3]) / p->sqrt_s;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    double k1[4] = {0.5 * x1 * p->sqrt_s, 0, 0, 0.5 * x1 * p->sqrt_s};
    double k2[4] = {0.5 * x2 * p->sqrt_s, 0, 0, -0.5 * x2 * p->sqrt_s};
    double g1, g2;
    if (p->pdf) {
      g1 = or_pdf_interp(p->pdf, 0, x1, p->m_t) / x1;
      g2 = or_pdf_interp(p->pdf, 0, x2, p->m_t) / x2;
    } else {
      g1 = or_xf_g(x1) / x1;
      g2 = or_xf_g(x2) / x2;
    }
    double me = kind == OR_KIND_TTH_LL ? or_tth_me2_gg(p, k1, k2, hard, hard + 24, hard + 28)
                                       : or_ttbb_me2_gg(p, k1, k2, hard, hard + 24, hard + 28);
    double shat = x1 * x2 * S;
    sum += (2.0 / S) * (P[0] / Eh) * g1 * g2 * me / (2.0 * shat) / fabs(detj[s]) / (2.0 * v[0] * 2.0 * vb[0]);
  }
  double two_pi_pow = pow(2.0 * M_PI, 4.0 - 3.0 * 8.0);
  double lep = 1.0 / (2.0 * lp[0] * 2.0 * lm[0]);
  return sum * two_pi_pow * lep * jetf * jac;
}

double or_tthll_integrand(const or_params* p, const double* ev, int perm, const double* x, int* nsol_out)
{
  return f2_integrand_me(OR_KIND_TTH_LL, 0, p, ev, perm, x, nsol_out);
}
double or_ttbbll_integrand(const or_params* p, const double* ev, int perm, const double* x, int* nsol_out)
{
  return f2_integrand_me(OR_KIND_TTBB_LL, 0, p, ev, perm, x, nsol_out);
}

/* Parton level for Sec. 4's processes (its Table 2 workload): the transfer
 * functions are delta functions, so only the energy and longitudinal
 * momentum delta functions, the flux, the densities and the complete
 * |M|^2 remain; the weight is the mean over the jet assignments (the four b
 * quarks placed as in or_f2_perm).  ev: 8 x {E,px,py,pz}: b quarks 0-3 (any
 * order), l+, l-, nu, nubar. */
double or_f2_parton_weight(int kind, const or_params* p, const double* ev)
{
  const double S = p->sqrt_s * p->sqrt_s;
  const double *lp = ev + 16, *lm = ev + 20, *nu = ev + 24, *nub = ev + 28;
  const int n = or_nperm(kind);
  double sum = 0.0;
  for (int perm = 0; perm < n; ++perm) {
    int rows[4];
    or_f2_perm(kind, perm, rows);
    double lab[8][4];
    memcpy(lab[0], ev + 4 * rows[0], 32); memcpy(lab[1], lp, 32); memcpy(lab[2], nu, 32);
    memcpy(lab[3], ev + 4 * rows[1], 32); memcpy(lab[4], lm, 32); memcpy(lab[5], nub, 32);
    memcpy(lab[6], ev + 4 * rows[2], 32); memcpy(lab[7], ev + 4 * rows[3], 32);
    double P[4] = {0, 0, 0, 0};
    for (int k = 0; k < 8; ++k) for (int i = 0; i < 4; ++i) P[i] += lab[k][i];
    double hard[32];
    for (int k = 0; k < 8; ++k) boost_transverse(P, lab[k], hard + 4 * k);
    double Eh = sqrt(P[0] * P[0] - P[1] * P[1] - P[2] * P[2]);
    double x1 = (Eh + P[3]) / p->sqrt_s, x2 = (Eh - P[3]) / p->sqrt_s;
    if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) continue;
    double k1[4] = {0.5 * x1 * p->sqrt_s, 0, 0, 0.5 * x1 * p->sqrt_s};
    double k2[4] = {0.5 * x2 * p->sqrt_s, 0, 0, -0.5 * x2 * p->sqrt_s};
    double g1, g2;
    if (p->pdf) {
      g1 = or_pdf_interp(p->pdf, 0, x1, p->m_t) / x1;
      g2 = or_pdf_interp(p->pdf, 0, x2, p->m_t) / x2;
    } else {
      g1 = or_xf_g(x1) / x1;
      g2 = or_xf_g(x2) / x2;
    }
    double me = kind == OR_KIND_TTH_LL ? or_tth_me2_gg(p, k1, k2, hard, hard + 24, hard + 28)
                                       : or_ttbb_me2_gg(p, k1, k2, hard, hard + 24, hard + 28);
    double shat = x1 * x2 * S;
    sum += (2.0 / S) * (P[0] / Eh) * g1 * g2 * me / (2.0 * shat);
  }
  return sum / n;
}

/* ------------------------------------------- direct parametrisations -- */
/* Eq. integrand written in the unmeasured momenta themselves: no
 * propagator-aligned variables, no constraint solve, the Breit-Wigner
 * factors left inside |M|^2.  They exist to check the mapped integrands
 * above by closure (the two parametrisations of one integral must agree);
 * the driver integrates them as kinds of their own.
 *
 * A momentum component p is drawn by the Cauchy map p = c + s tan(pi (x -
 * 1/2)), dp/dx = pi s (1 + ((p - c)/s)^2). */
static double cauchy_map(double x, double c, double s, double* jac)
{
  const double t = tan(M_PI * (x - 0.5));
  *jac *= M_PI * s * (1.0 + t * t);
  return c + s * t;
}

/* ttbar dilepton: x0, x1 jet energies and x6, x7 recoil exactly as in
 * or_tt_integrand; x2..x5 -> (nu_x, nu_y, nu_z, nubar_z), nubar_T = MET -
 * nu_T (the transverse delta function), measure d^3nu/(2E) d^3nubar/(2E)
 * reduced by it to d^3nu dnubar_z / (2E 2E). */
double or_tt_direct_integrand(const or_params* p, const double* ev, int perm, const double* x)
{
  const double S = p->sqrt_s * p->sqrt_s;
  const double* jet[2] = {ev + (perm ? 4 : 0), ev + (perm ? 0 : 4)};
  const double* lp = ev + 8;
  const double* lm = ev + 12;
  double bq[2][4];
  double jetf = 1.0;
  for (int k = 0; k < 2; ++k) {
    const double* m = jet[k];
    double em = m[0], pm = norm3(m);
    double r = p->r_lo + x[k] * (p->r_hi - p->r_lo);
    double E = em / r;
    double jac = (p->r_hi - p->r_lo) * em / (r * r);
    bq[k][0] = E;
    for (int i = 1; i < 4; ++i) bq[k][i] = m[i] / pm * E;
    double sin_th = sqrt(m[1] * m[1] + m[2] * m[2]) / pm;
    jetf *= E * E * sin_th * or_gauss_tf(em, E, p->tf_sigma) / (2.0 * E) * jac;
  }
  double rho = p->sigma_k * sqrt(-2.0 * log(1.0 - x[6]));
  double phi = 2.0 * M_PI * x[7];
  double metx = rho * cos(phi) - (bq[0][1] + bq[1][1] + lp[1] + lm[1]);
  double mety = rho * sin(phi) - (bq[0][2] + bq[1][2] + lp[2] + lm[2]);
  double jnu = 1.0;
  double v[4], vb[4];
  v[1] = cauchy_map(x[2], 0.5 * metx, 60.0, &jnu);
  v[2] = cauchy_map(x[3], 0.5 * mety, 60.0, &jnu);
  v[3] = cauchy_map(x[4], 0.0, 100.0, &jnu);
  vb[3] = cauchy_map(x[5], 0.0, 100.0, &jnu);
  vb[1] = metx - v[1];
  vb[2] = mety - v[2];
  v[0] = norm3(v);
  vb[0] = norm3(vb);
  double lab[6][4];
  memcpy(lab[0], bq[0], sizeof(lab[0])); memcpy(lab[1], lp, sizeof(lab[1]));
  memcpy(lab[2], v, sizeof(lab[2]));     memcpy(lab[3], bq[1], sizeof(lab[3]));
  memcpy(lab[4], lm, sizeof(lab[4]));    memcpy(lab[5], vb, sizeof(lab[5]));
  double P[4] = {0, 0, 0, 0};
  for (int k = 0; k < 6; ++k) for (int i = 0; i < 4; ++i) P[i] += lab[k][i];
  double hard[24];
  for (int k = 0; k < 6; ++k) boost_transverse(P, lab[k], hard + 4 * k);
  double Eh = sqrt(P[0] * P[0] - P[1] * P[1] - P[2] * P[2]);
  double x1 = (Eh + P[3]) / p->sqrt_s, x2 = (Eh - P[3]) / p->sqrt_s;
  if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) return 0.0;
  double k1[4] = {0.5 * x1 * p->sqrt_s, 0, 0, 0.5 * x1 * p->sqrt_s};
  double k2[4] = {0.5 * x2 * p->sqrt_s, 0, 0, -0.5 * x2 * p->sqrt_s};
  const tt_lumi L = tt_lumis(p, x1, x2);
  double me = L.gg * or_tt_me2_gg(p, k1, k2, hard)
            + L.qq12 * or_tt_me2_qq(p, k1, k2, hard)
            + L.qq21 * or_tt_me2_qq(p, k2, k1, hard);
  double shat = x1 * x2 * S;
  double f = (2.0 / S) * (P[0] / Eh) * me / (2.0 * shat) / (2.0 * v[0] * 2.0 * vb[0]);
  double two_pi_pow = pow(2.0 * M_PI, 4.0 - 3.0 * 6.0);
  double lep = 1.0 / (2.0 * lp[0] * 2.0 * lm[0]);
  return f * two_pi_pow * lep * jetf * jnu;
}

/* ttbar semileptonic: (2/S)(E/E') sum |M|^2 x PDFs / (2 shat) of one
 * configuration of the six final-state momenta (zero when x1 or x2 leaves
 * (0, 1]); the body of or_tt_semilep_integrand's solution loop. */
static double sl_config_weight(const or_params* p, int lep_charge, const double* qa, const double* qb,
                               const double* bh, const double* bl, const double* l, const double* nu)
{
  const double S = p->sqrt_s * p->sqrt_s;
  double P[4];
  for (int i = 0; i < 4; ++i) P[i] = qa[i] + qb[i] + bh[i] + bl[i] + l[i] + nu[i];
  double Eh = sqrt(P[0] * P[0] - P[1] * P[1] - P[2] * P[2]);
  double x1 = (Eh + P[3]) / p->sqrt_s, x2 = (Eh - P[3]) / p->sqrt_s;
  if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) return 0.0;
  double k1[4] = {0.5 * x1 * p->sqrt_s, 0, 0, 0.5 * x1 * p->sqrt_s};
  double k2[4] = {0.5 * x2 * p->sqrt_s, 0, 0, -0.5 * x2 * p->sqrt_s};
  double hq[2][4], hbh[4], hbl[4], hl[4], hn[4];
  boost_transverse(P, qa, hq[0]);
  boost_transverse(P, qb, hq[1]);
  boost_transverse(P, bh, hbh);
  boost_transverse(P, bl, hbl);
  boost_transverse(P, l, hl);
  boost_transverse(P, nu, hn);
  const tt_lumi L = tt_lumis(p, x1, x2);
  double me = 0.0;
  for (int o = 0; o < 2; ++o) {
    const double* qk = hq[o];
    const double* qbk = hq[1 - o];
    double mom[24];
    if (lep_charge > 0) {
      memcpy(mom, hbl, 32); memcpy(mom + 4, hl, 32); memcpy(mom + 8, hn, 32);
      memcpy(mom + 12, hbh, 32); memcpy(mom + 16, qk, 32); memcpy(mom + 20, qbk, 32);
    } else {
      memcpy(mom, hbh, 32); memcpy(mom + 4, qbk, 32); memcpy(mom + 8, qk, 32);
      memcpy(mom + 12, hbl, 32); memcpy(mom + 16, hl, 32); memcpy(mom + 20, hn, 32);
    }
    me += L.gg * or_tt_me2_gg(p, k1, k2, mom) + L.qq12 * or_tt_me2_qq(p, k1, k2, mom)
        + L.qq21 * or_tt_me2_qq(p, k2, k1, mom);
  }
  me *= 3.0 * 2.0;
  double shat = x1 * x2 * S;
  return (2.0 / S) * (P[0] / Eh) * me / (2.0 * shat);
}

/* ttbar semileptonic with parts of the parametrisation made direct.
 * mode & OR_SL_DIRECT_EB: x1 is the r map of light jet b (over its TF
 * window) instead of the hadronic W virtuality; mode & OR_SL_DIRECT_EBH: x2
 * is the r map of the hadronic top's b instead of the hadronic top
 * virtuality; mode & OR_SL_DIRECT_NU: x6 -> nu_z (Cauchy map; nu_T = MET,
 * the measure d^3nu/(2E) with the transverse delta function leaving
 * dnu_z/(2E)) instead of the leptonic W virtuality and the nu_z quadratic.
 * x0, x3 (r maps of light jet a and of the leptonic top's b) and x4, x5
 * (recoil) as in or_tt_semilep_integrand, which mode 0 reproduces. */
double or_tt_semilep_direct_integrand(const or_params* p, const double* ev, int lep_charge, int perm,
                                      const double* x, int mode)
{
  const double S = p->sqrt_s * p->sqrt_s;
  if (lep_charge == 0) lep_charge = ev[20] > 0 ? 1 : -1;
  int ibl, ibh, ja, jb;
  or_semilep_perm(perm, &ibl, &ibh, &ja, &jb);
  const double* l = ev + 16;
  const int idx[4] = {ja, jb, ibh, ibl};
  double dir[4][3], em[4];
  for (int k = 0; k < 4; ++k) {
    const double* m = ev + 4 * idx[k];
    const double pm = norm3(m);
    em[k] = m[0];
    for (int i = 0; i < 3; ++i) dir[k][i] = m[i + 1] / pm;
  }
  double E4[4], jac = 1.0;
  /* r = E_meas / E over [lo, hi] */
  #define R_MAP(k, xv, lo, hi) do { const double r_ = (lo) + (xv) * ((hi) - (lo)); \
      E4[k] = em[k] / r_; jac *= ((hi) - (lo)) * em[k] / (r_ * r_); } while (0)
  R_MAP(0, x[0], p->lj_r_lo, p->lj_r_hi);
  R_MAP(3, x[3], p->r_lo, p->r_hi);
  const double ca = dir[0][0] * dir[1][0] + dir[0][1] * dir[1][1] + dir[0][2] * dir[1][2];
  if (!(1.0 - ca > 0.0)) return 0.0;
  double q2wh;
  if (mode & OR_SL_DIRECT_EB) {
    R_MAP(1, x[1], p->lj_r_lo, p->lj_r_hi);
    q2wh = 2.0 * E4[0] * E4[1] * (1.0 - ca);
  } else {
    jac *= or_bw_map(x[1], p->m_w, p->w_w, 0.0, S, &q2wh);
    E4[1] = q2wh / (2.0 * E4[0] * (1.0 - ca));
    jac *= 1.0 / (2.0 * E4[0] * (1.0 - ca));
    const double rr = em[1] / E4[1];
    if (rr < p->lj_r_lo || rr > p->lj_r_hi) return 0.0;
  }
  if (mode & OR_SL_DIRECT_EBH) {
    R_MAP(2, x[2], p->r_lo, p->r_hi);
  } else {
    double q2th;
    jac *= or_bw_map(x[2], p->m_t, p->w_t, 0.0, S, &q2th);
    const double W[4] = {E4[0] + E4[1], E4[0] * dir[0][0] + E4[1] * dir[1][0],
                         E4[0] * dir[0][1] + E4[1] * dir[1][1], E4[0] * dir[0][2] + E4[1] * dir[1][2]};
    const double den = 2.0 * (W[0] - (dir[2][0] * W[1] + dir[2][1] * W[2] + dir[2][2] * W[3]));
    if (!(den > 0.0)) return 0.0;
    E4[2] = (q2th - q2wh) / den;
    if (!(E4[2] > 0.0)) return 0.0;
    jac *= 1.0 / den;
    const double rr = em[2] / E4[2];
    if (rr < p->r_lo || rr > p->r_hi) return 0.0;
  }
  #undef R_MAP
  double qa[4], qb[4], bh[4], bl[4];
  double* dst[4] = {qa, qb, bh, bl};
  double tf = 1.0;
  for (int k = 0; k < 4; ++k) {
    const double* m = ev + 4 * idx[k];
    double pm = norm3(m), E = E4[k];
    dst[k][0] = E;
    for (int i = 0; i < 3; ++i) dst[k][i + 1] = E * m[i + 1] / pm;
    double sin_th = sqrt(m[1] * m[1] + m[2] * m[2]) / pm;
    double T = k < 2 ? or_dgauss_tf(m[0], E, p->lj_core, p->lj_tail, p->lj_ftail)
                     : or_gauss_tf(m[0], E, p->tf_sigma);
    tf *= E * E * sin_th * T / (2.0 * E);
  }
  double rho = p->sigma_k * sqrt(-2.0 * log(1.0 - x[4]));
  double phi = 2.0 * M_PI * x[5];
  double nx = rho * cos(phi) - (qa[1] + qb[1] + bh[1] + bl[1] + l[1]);
  double ny = rho * sin(phi) - (qa[2] + qb[2] + bh[2] + bl[2] + l[2]);
  double sum = 0.0;
  if (mode & OR_SL_DIRECT_NU) {
    double nu[4] = {0.0, nx, ny, 0.0};
    nu[3] = cauchy_map(x[6], 0.0, 100.0, &jac);
    nu[0] = norm3(nu);
    sum = sl_config_weight(p, lep_charge, qa, qb, bh, bl, l, nu) / (2.0 * nu[0]);
  } else {
    double q2wl;
    jac *= or_bw_map(x[6], p->m_w, p->w_w, 0.0, S, &q2wl);
    double nzs[2];
    int nroot = or_semilep_nu_z(l, nx, ny, q2wl, nzs);
    for (int s = 0; s < nroot; ++s) {
      double nu[4] = {sqrt(nx * nx + ny * ny + nzs[s] * nzs[s]), nx, ny, nzs[s]};
      double dq = fabs(2.0 * (l[0] * nzs[s] / nu[0] - l[3]));
      if (!(dq > 0.0)) continue;
      sum += sl_config_weight(p, lep_charge, qa, qb, bh, bl, l, nu) / dq / (2.0 * nu[0]);
    }
  }
  double two_pi_pow = pow(2.0 * M_PI, 4.0 - 3.0 * 6.0);
  return sum * two_pi_pow * tf * jac / (2.0 * l[0]);
}

/* t tbar H dilepton (Sec. 4): as or_tthll_integrand, but x7 is the r map of
 * the second Higgs jet's energy (as for t tbar b bbar) instead of the Higgs
 * virtuality of Eq. mhsolve; the Higgs Breit-Wigner factor stays in
 * |M|^2. */
double or_tthll_direct_integrand(const or_params* p, const double* ev, int perm, const double* x)
{
  /* the t tbar b bbar branch of f2_integrand maps x7 that way; only the
   * matrix element differs */
  return f2_integrand_me(OR_KIND_TTH_LL, 1, p, ev, perm, x, NULL);
}
