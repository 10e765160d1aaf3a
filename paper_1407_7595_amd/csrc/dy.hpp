// Drell-Yan q qbar -> gamma* -> mu- mu+ integrand (FP64).
//
// Eq. mem_def with the two true muon momenta |p1|, |p2| integrated against a
// Gaussian momentum TF (Eq. 3), directions fixed by delta functions (Sec. 1).
// Parton fractions come from the true pair, x_{1,2} = (E +- p_z)/sqrt(S),
// the transverse momentum of the pair is not constrained, and the matrix
// element is the spin/colour averaged (4 pi alpha)^2 Q^2 (1 + cos^2)/3 in
// the Collins-Soper angle.
#pragma once
#include "device_common.hpp"
#include "pdf.hpp"
#include "process.hpp"

namespace memk {

struct DYEvent {
  double n[2][3];     // unit directions of mu-, mu+
  double pm[2];       // measured |p|
  double sin_th[2];
};

__device__ __forceinline__ void dy_load(const EventsView& ev, int e, DYEvent& d)
{
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double E, x, y, z;
    ev.load(k, e, E, x, y, z);
    double p = sqrt(x * x + y * y + z * z);
    d.pm[k] = p;
    d.n[k][0] = x / p; d.n[k][1] = y / p; d.n[k][2] = z / p;
    d.sin_th[k] = sqrt(x * x + y * y) / p;
  }
}

// relative-energy TF density times the true energy: sum_k w_k N(r; 1, s_k)
__device__ __forceinline__ double tf_r64(double r, const TFParams& tf)
{
  const double inv_sqrt_2pi = 0.39894228040143267794;
  double d = r - 1.0;
  double g = exp(-0.5 * d * d / (tf.s_core * tf.s_core)) / tf.s_core;
  if (tf.f_tail > 0.0)
    g = (1.0 - tf.f_tail) * g + tf.f_tail * exp(-0.5 * d * d / (tf.s_tail * tf.s_tail)) / tf.s_tail;
  return inv_sqrt_2pi * g;
}

// toy densities x f(x) of the configuration (omx = 1 - x): u and d
// valence-like, the common sea antiquark, the gluon x g(x) = 3 (1-x)^5
__host__ __device__ inline double xfu(double x, double omx) { double o = omx * omx * omx; return 2.0 * sqrt(x) * o; }
__host__ __device__ inline double xfd(double x, double omx) { double o = omx * omx; return sqrt(x) * o * o; }
__host__ __device__ inline double xfq(double omx) { double o2 = omx * omx, o4 = o2 * o2; return 0.2 * o4 * o2 * omx; }
__host__ __device__ inline double xfg(double omx) { return 3.0 * omx * omx * omx * omx * omx; }

__device__ __forceinline__ double dy_integrand(const ProcParams& pp, const DYEvent& ev, const double (&x)[2])
{
  const TFParams& tf = pp.tf_mu;
  v4 mu[2];
  double w = pp.dy_const;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double r = tf.r_lo + x[k] * (tf.r_hi - tf.r_lo);
    double p = ev.pm[k] / r;
    mu[k] = v4{p, p * ev.n[k][0], p * ev.n[k][1], p * ev.n[k][2]};
    // p^2 sin dp T/(2E) with dp = (r_hi - r_lo) p_meas / r^2 dx:
    // the true |p| cancels against the TF normalisation
    w *= ev.sin_th[k] * (tf.r_hi - tf.r_lo) * ev.pm[k] / (r * r) * 0.5 * tf_r64(r, tf);
  }
  v4 P = add(mu[0], mu[1]);
  double m2 = mdot(P, P);
  if (!(m2 >= pp.m_lo * pp.m_lo && m2 <= pp.m_hi * pp.m_hi)) return 0.0;
  double x1 = (P.e + P.z) / pp.sqrt_s, x2 = (P.e - P.z) / pp.sqrt_s;
  if (!(x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) return 0.0;
  double pt2 = P.x * P.x + P.y * P.y;
  double c = 2.0 * (mu[0].z * mu[1].e - mu[0].e * mu[1].z) / (sqrt(m2) * sqrt(m2 + pt2));
  // parton densities f = xf / x; the 1/(x1 x2) joins 1/shat below
  double lum;
#ifndef MEM_HOST_COUNT
  if (pp.pdf_xf) {
    lum = pdf_grid_dy_lumi(pp, x1, x2, m2);
  } else
#endif
  {
    double o1 = 1.0 - x1, o2 = 1.0 - x2;
    double u1 = xfu(x1, o1), d1 = xfd(x1, o1), q1 = xfq(o1);
    double u2 = xfu(x2, o2), d2 = xfd(x2, o2), q2 = xfq(o2);
    lum = (4.0 / 9.0) * (u1 * q2 + q1 * u2) + (1.0 / 9.0) * (d1 * q2 + q1 * d2);
  }
  double shat = x1 * x2 * pp.S;
  return w * lum * (1.0 + c * c) / (shat * x1 * x2);
}

}  // namespace memk
