/*
 * Oracle: counter-based random numbers and the VEGAS grid.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The MC estimator S_N and its error (Sec. 2, Eq. for S_N and the error
 * estimate below it) are driven by VEGAS (Sec. 2, Lepage 1978/1980), here
 * written from Lepage's published description of the adaptive map.
 */
#include "oracle.h"
#include <math.h>
#include <string.h>

/* Philox4x32-10, Salmon et al. SC'11: the round multipliers are the two
 * constants the paper lists for N=4, W=32; the key increments are the
 * 32-bit golden-ratio and sqrt(3)-1 Weyl constants. */
#define PH_M0 0xD2511F53u
#define PH_M1 0xCD9E8D57u
#define PH_W0 0x9E3779B9u
#define PH_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += PH_W0; k1 += PH_W1; }
    uint64_t prod0 = (uint64_t)PH_M0 * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)PH_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u53(uint32_t hi, uint32_t lo)
{
  uint64_t bits = ((uint64_t)hi << 32) | (uint64_t)lo;
  return (double)(bits >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
}

void or_uniforms(uint64_t seed, uint32_t k, uint32_t iter, uint32_t event,
                 uint32_t perm, int D, double* u)
{
  or_uniforms_block(seed, k, iter, event, perm, 0u, D, u);
}

/* The same stream with the counter's last word perm*16 + block0 + b: the
 * learned proposal draws its base points from blocks 8.. of a permutation. */
void or_uniforms_block(uint64_t seed, uint32_t k, uint32_t iter, uint32_t event,
                       uint32_t perm, uint32_t block0, int D, double* u)
{
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int b = 0; 2 * b < D; ++b) {
    uint32_t ctr[4] = {k, iter, event, perm * 16u + block0 + (uint32_t)b};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    u[2 * b] = u53(w[0], w[1]);
    if (2 * b + 1 < D) u[2 * b + 1] = u53(w[2], w[3]);
  }
}

/* ------------------------------------------------------------------------
 * VEGAS map.  Each dimension has OR_NBINS bins of unequal width between
 * edges e_0 = 0 < ... < e_64 = 1.  A uniform u selects bin i = floor(64u)
 * and the position inside it linearly; the Jacobian is 64 * width.
 * The position is formed with a fused multiply-add so that the result is
 * the correctly rounded value of e_i + frac * width.
 * ---------------------------------------------------------------------- */
void or_vegas_uniform_grid(double* grid, int D)
{
  for (int d = 0; d < D; ++d)
    for (int i = 0; i <= OR_NBINS; ++i)
      grid[d * (OR_NBINS + 1) + i] = (double)i / (double)OR_NBINS;
}

double or_vegas_map(const double* grid, int D, const double* u, double* x, int* bins)
{
  double jac = 1.0;
  for (int d = 0; d < D; ++d) {
    const double* e = grid + d * (OR_NBINS + 1);
    double t = u[d] * (double)OR_NBINS;
    int i = (int)t;
    if (i > OR_NBINS - 1) i = OR_NBINS - 1;
    double frac = t - (double)i;
    double width = e[i + 1] - e[i];
    x[d] = fma(frac, width, e[i]);
    jac *= (double)OR_NBINS * width;
    if (bins) bins[d] = i;
  }
  return jac;
}

/* Damped rebinning (Lepage 1978): the per-bin sums of w^2 are smoothed by a
 * three-point average (two points at the ends), normalised to rho_i, turned
 * into importances m_i = ((1 - rho_i) / ln(1/rho_i))^alpha, and the new
 * edges are placed so that every new bin holds an equal share of sum m,
 * interpolating linearly inside the old bins.  A dimension whose sums are
 * all zero keeps its grid. */
void or_vegas_refine_dim(const double* d_in, double alpha, double* edges)
{
  const int n = OR_NBINS;
  double s[OR_NBINS], m[OR_NBINS], old[OR_NBINS + 1];
  s[0] = (d_in[0] + d_in[1]) / 2.0;
  for (int i = 1; i < n - 1; ++i) s[i] = (d_in[i - 1] + d_in[i] + d_in[i + 1]) / 3.0;
  s[n - 1] = (d_in[n - 2] + d_in[n - 1]) / 2.0;
  double total = 0.0;
  for (int i = 0; i < n; ++i) total += s[i];
  if (!(total > 0.0)) return;
  double msum = 0.0;
  for (int i = 0; i < n; ++i) {
    double rho = s[i] / total;
    if (rho <= 0.0) m[i] = 0.0;
    else if (rho >= 1.0) m[i] = 1.0; /* limit of (1-rho)/ln(1/rho) */
    else m[i] = pow((1.0 - rho) / log(1.0 / rho), alpha);
    msum += m[i];
  }
  memcpy(old, edges, sizeof(old));
  double share = msum / (double)n;
  int i = 0;
  double acc = 0.0; /* sum of m over old bins before bin i */
  for (int k = 1; k < n; ++k) {
    double target = share * (double)k;
    while (i < n && acc + m[i] < target) { acc += m[i]; ++i; }
    if (i >= n) { edges[k] = 1.0; continue; }
    edges[k] = old[i] + (target - acc) / m[i] * (old[i + 1] - old[i]);
  }
  edges[0] = 0.0;
  edges[n] = 1.0;
}
