/* Parton densities from a grid in (ln x, ln Q), bilinear interpolation
 * (test infrastructure of the oracle).
 *
 * Sec. 4: the densities of each flavour are queried once, stored on an
 * (x, Q) grid and interpolated bilinearly inside the integrand.  Written
 * from the definition of bilinear interpolation on a rectangle: with the
 * cell [a0, a1] x [b0, b1] and t = (a - a0)/(a1 - a0), u = (b - b0)/(b1 - b0),
 *   f = (1 - t)(1 - u) f00 + t (1 - u) f10 + (1 - t) u f01 + t u f11,
 * which reproduces every function of the form c0 + c1 a + c2 b + c3 a b. */
#include <math.h>
#include <stddef.h>

#include "oracle.h"

/* index of the cell that holds coordinate v on n nodes from v0 with step h,
 * clamped to the first and last cell */
static int cell(double v, double v0, double h, int n)
{
  double c = floor((v - v0) / h);
  if (c < 0.0) return 0;
  if (c > (double)(n - 2)) return n - 2;
  return (int)c;
}

double or_pdf_interp(const or_pdf_grid* g, int fl, double x, double Q)
{
  if (fl < -5 || fl > 5) return 0.0;
  const double hx = (g->lx_max - g->lx_min) / (g->nx - 1);
  const double hq = (g->lq_max - g->lq_min) / (g->nq - 1);
  const double a = log(x), b = log(Q);
  const int i = cell(a, g->lx_min, hx, g->nx), j = cell(b, g->lq_min, hq, g->nq);
  const double a0 = g->lx_min + i * hx, b0 = g->lq_min + j * hq;
  const double t = (a - a0) / hx, u = (b - b0) / hq;
  const int k = fl + 5;
  const double f00 = g->xf[((size_t)j * g->nx + i) * 11 + k];
  const double f10 = g->xf[((size_t)j * g->nx + i + 1) * 11 + k];
  const double f01 = g->xf[((size_t)(j + 1) * g->nx + i) * 11 + k];
  const double f11 = g->xf[((size_t)(j + 1) * g->nx + i + 1) * 11 + k];
  return (1.0 - t) * (1.0 - u) * f00 + t * (1.0 - u) * f10 + (1.0 - t) * u * f01 + t * u * f11;
}

void or_pdf_tabulate_toy(const or_pdf_grid* g, float* xf_out)
{
  const double hx = (g->lx_max - g->lx_min) / (g->nx - 1);
  for (int j = 0; j < g->nq; ++j)
    for (int i = 0; i < g->nx; ++i) {
      const double x = exp(g->lx_min + i * hx);
      float* v = xf_out + ((size_t)j * g->nx + i) * 11;
      for (int k = 0; k < 11; ++k) v[k] = 0.0f;
      if (x >= 1.0) continue;
      v[5 + 2] = (float)or_xf_u(x);
      v[5 + 1] = (float)or_xf_d(x);
      v[5 - 2] = (float)or_xf_qbar(x);
      v[5 - 1] = (float)or_xf_qbar(x);
      v[5] = (float)or_xf_g(x);
    }
}
