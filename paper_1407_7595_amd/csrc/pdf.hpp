// Parton densities from a grid in (ln x, ln Q) (Sec. 4: the densities of
// each flavour are tabulated once and interpolated bilinearly inside the
// integrand).
//
// A node holds x f of the 11 flavours and a zero pad: 48 bytes, three
// 16-byte loads, so one set of cell weights serves every flavour.  With the scale fixed (the top processes, Q = m_t) only the two
// grid rows around m_t are read: 2 x nx x 48 B, cache-resident.  The cell
// position is formed in FP64 (an FP32 ln x would move the interpolated
// value by up to ~1e-5 at x = 1e-5); the blend runs in the matrix-element
// type T.
#pragma once
#include "device_common.hpp"
#include "process.hpp"

#ifndef MEM_HOST_COUNT
namespace memk {

// cell index and fraction of position s on n nodes (edge cells continue
// linearly outside the grid); the index stays in [0, n - 2] for any s,
// NaN included
__device__ __forceinline__ int pdf_cell(double s, int n, double& frac)
{
  double c = s >= 0.0 ? floor(s) : 0.0;
  c = c > (double)(n - 2) ? (double)(n - 2) : c;
  frac = s - c;
  return (int)c;
}

// Node layout on the device: three 16-byte groups (g, 0, d, dbar),
// (u, ubar, s, sbar), (c, cbar, b, bbar), so that a quark and its antiquark
// arrive in one load and a luminosity is accumulated group by group with
// few values live.
constexpr int kPdfNode = 12;
__host__ __device__ inline int pdf_slot(int fl)     // device slot of flavour fl = -5..5
{
  return fl == 0 ? 0 : 2 * (fl < 0 ? -fl : fl) + (fl < 0 ? 1 : 0);
}

// the grid cell of one x (and the Q cell) with its four corner weights
template <class T>
struct PdfCell {
  const float4* n00;     // corner (ix, iq); (ix+1, iq) is 3 groups on, (ix, iq+1) one row on
  int64_t row;           // groups per Q row
  T w00, w10, w01, w11;
};

template <class T>
__device__ __forceinline__ PdfCell<T> pdf_locate(const ProcParams& pp, double x, int iq, double uq)
{
  double tx;
  const int ix = pdf_cell((log(x) - pp.pdf_lx0) * pp.pdf_ihx, pp.pdf_nx, tx);
  const T t = T(tx), u = T(uq);
  PdfCell<T> c;
  c.n00 = reinterpret_cast<const float4*>(pp.pdf_xf + ((int64_t)iq * pp.pdf_nx + ix) * kPdfNode);
  c.row = 3 * (int64_t)pp.pdf_nx;
  c.w00 = (T(1) - t) * (T(1) - u);
  c.w10 = t * (T(1) - u);
  c.w01 = (T(1) - t) * u;
  c.w11 = t * u;
  return c;
}

// bilinear blend of group k (0..2) of the four corners
template <class T>
__device__ __forceinline__ void pdf_group(const PdfCell<T>& c, int k, T (&v)[4])
{
  const float4 a = c.n00[k], b = c.n00[k + 3], d = c.n00[c.row + k], e = c.n00[c.row + k + 3];
  v[0] = c.w00 * T(a.x) + c.w10 * T(b.x) + c.w01 * T(d.x) + c.w11 * T(e.x);
  v[1] = c.w00 * T(a.y) + c.w10 * T(b.y) + c.w01 * T(d.y) + c.w11 * T(e.y);
  v[2] = c.w00 * T(a.z) + c.w10 * T(b.z) + c.w01 * T(d.z) + c.w11 * T(e.z);
  v[3] = c.w00 * T(a.w) + c.w10 * T(b.w) + c.w01 * T(d.w) + c.w11 * T(e.w);
}

// Luminosities of the top processes from the grid at the fixed scale m_t,
// in x f form: gg = xg(x1) xg(x2), qq12 = sum_q xq(x1) xqbar(x2), qq21 =
// sum_q xqbar(x1) xq(x2) over d, u, s, c, b (in that order).
template <class T>
__device__ __forceinline__ void pdf_grid_tt_lumis(const ProcParams& pp, double x1, double x2, T& gg, T& qq12, T& qq21)
{
  const PdfCell<T> c1 = pdf_locate<T>(pp, x1, pp.pdf_iq_mt, pp.pdf_uq_mt);
  const PdfCell<T> c2 = pdf_locate<T>(pp, x2, pp.pdf_iq_mt, pp.pdf_uq_mt);
  T a[4], b[4];
  pdf_group(c1, 0, a);
  pdf_group(c2, 0, b);
  gg = a[0] * b[0];
  qq12 = a[2] * b[3];
  qq21 = a[3] * b[2];
#pragma unroll 1
  for (int k = 1; k < 3; ++k) {
    pdf_group(c1, k, a);
    pdf_group(c2, k, b);
    qq12 += a[0] * b[1];
    qq21 += a[1] * b[0];
    qq12 += a[2] * b[3];
    qq21 += a[3] * b[2];
  }
}

// Drell-Yan luminosity sum_q e_q^2 (xq(x1) xqbar(x2) + xqbar(x1) xq(x2))
// at the scale Q = the pair mass (FP64); charges squared 1/9 (d, s, b)
// and 4/9 (u, c)
__device__ __forceinline__ double pdf_grid_dy_lumi(const ProcParams& pp, double x1, double x2, double m2)
{
  double uq;
  const int iq = pdf_cell((0.5 * log(m2) - pp.pdf_lq0) * pp.pdf_ihq, pp.pdf_nq, uq);
  const PdfCell<double> c1 = pdf_locate<double>(pp, x1, iq, uq), c2 = pdf_locate<double>(pp, x2, iq, uq);
  const double e_d = 1.0 / 9.0, e_u = 4.0 / 9.0;
  double a[4], b[4];
  pdf_group(c1, 0, a);
  pdf_group(c2, 0, b);
  double lum = e_d * (a[2] * b[3] + a[3] * b[2]);
#pragma unroll 1
  for (int k = 1; k < 3; ++k) {
    pdf_group(c1, k, a);
    pdf_group(c2, k, b);
    lum += e_u * (a[0] * b[1] + a[1] * b[0]);     // u (k = 1), c (k = 2)
    lum += e_d * (a[2] * b[3] + a[3] * b[2]);                      // s (k = 1), b (k = 2)
  }
  return lum;
}

}  // namespace memk
#endif  // MEM_HOST_COUNT
