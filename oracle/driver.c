/*
 * Oracle: the per-integral VEGAS loop and the per-event result.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Sec. 2: S_N = V (1/N) sum f(x_i) and its error V sigma_f / sqrt(N), with
 * sigma_f read as the standard deviation (the printed bracket defines the
 * variance).  Iterations are combined by inverse-variance weighting, the
 * first one (uniform grid) discarded.  Sec. 3 / Sec. 4: the event density
 * averages the integrals over the jet-parton assignments.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double integrand(int kind, const or_params* p, const double* ev, int perm, const double* x)
{
  if (kind == OR_KIND_DY) return or_dy_integrand(p, ev, x);
  if (kind == OR_KIND_GENZ) return or_genz_integrand(x);
  if (kind == OR_KIND_STEP) return 1.0 + floor(4.0 * x[0]) + 3.0 * floor(4.0 * x[1]);
  if (kind == OR_KIND_TT_SL) return or_tt_semilep_integrand(p, ev, 0, perm, x, NULL);
  if (kind == OR_KIND_TTH) return or_tth_integrand(p, ev, 0, perm, x, NULL);
  if (kind == OR_KIND_TTH_LL) return or_tthll_integrand(p, ev, perm, x, NULL);
  if (kind == OR_KIND_TTBB_LL) return or_ttbbll_integrand(p, ev, perm, x, NULL);
  if (kind == OR_KIND_TT_DIRECT) return or_tt_direct_integrand(p, ev, perm, x);
  if (kind == OR_KIND_TT_SL_DIRECT) return or_tt_semilep_direct_integrand(p, ev, 0, perm, x, OR_SL_DIRECT_EB | OR_SL_DIRECT_EBH | OR_SL_DIRECT_NU);
  if (kind == OR_KIND_TTH_LL_DIRECT) return or_tthll_direct_integrand(p, ev, perm, x);
  return or_tt_integrand(p, ev, perm, x, NULL);
}

double or_weight_at(int kind, const or_params* p, const double* ev, int perm,
                    const double* grid, const double* u)
{
  int D = or_dims(kind);
  double x[16];
  double jac = or_vegas_map(grid, D, u, x, NULL);
  return integrand(kind, p, ev, perm, x) * jac;
}

void or_vegas_iteration(int kind, const or_params* p, const double* ev, int perm,
                        uint64_t seed, uint32_t event_index, uint32_t iter,
                        int64_t n_points, const double* grid,
                        double* s1_out, double* s2_out, double* bins)
{
  int D = or_dims(kind);
  double s1 = 0.0, s2 = 0.0;
  memset(bins, 0, sizeof(double) * D * OR_NBINS);
  for (int64_t k = 0; k < n_points; ++k) {
    double u[16], x[16];
    int bi[16];
    or_uniforms(seed, (uint32_t)k, iter, event_index, (uint32_t)perm, D, u);
    double jac = or_vegas_map(grid, D, u, x, bi);
    double w = integrand(kind, p, ev, perm, x) * jac;
    s1 += w;
    s2 += w * w;
    for (int d = 0; d < D; ++d) bins[d * OR_NBINS + bi[d]] += w * w;
  }
  *s1_out = s1;
  *s2_out = s2;
}

void or_integrate_one(int kind, const or_params* p, const double* ev, int perm,
                      uint64_t seed, uint32_t event_index, int64_t n_points,
                      int n_iter, double alpha, double* grid_io,
                      double* iter_I, double* iter_var, or_result* res)
{
  int D = or_dims(kind);
  double* grid = (double*)malloc(sizeof(double) * D * (OR_NBINS + 1));
  double* bins = (double*)malloc(sizeof(double) * D * OR_NBINS);
  if (grid_io) memcpy(grid, grid_io, sizeof(double) * D * (OR_NBINS + 1));
  else or_vegas_uniform_grid(grid, D);
  double wsum = 0.0, wIsum = 0.0;
  double* Is = (double*)malloc(sizeof(double) * (n_iter > 0 ? n_iter : 1));
  double* Vs = (double*)malloc(sizeof(double) * (n_iter > 0 ? n_iter : 1));
  for (int j = 0; j < n_iter; ++j) {
    double s1, s2;
    or_vegas_iteration(kind, p, ev, perm, seed, event_index, (uint32_t)j, n_points, grid, &s1, &s2, bins);
    double N = (double)n_points;
    double I = s1 / N;
    double var = (s2 / N - I * I) / (N - 1.0);
    if (var < 0.0) var = 0.0;
    Is[j] = I; Vs[j] = var;
    if (iter_I) iter_I[j] = I;
    if (iter_var) iter_var[j] = var;
    if (j >= 1 && var > 0.0) { wsum += 1.0 / var; wIsum += I / var; }
    for (int d = 0; d < D; ++d)
      or_vegas_refine_dim(bins + d * OR_NBINS, alpha, grid + d * (OR_NBINS + 1));
  }
  res->n_iter_used = n_iter;
  if (wsum > 0.0) {
    res->I = wIsum / wsum;
    res->sigma = sqrt(1.0 / wsum);
    double chi2 = 0.0;
    int n = 0;
    for (int j = 1; j < n_iter; ++j)
      if (Vs[j] > 0.0) { chi2 += (Is[j] - res->I) * (Is[j] - res->I) / Vs[j]; ++n; }
    res->chi2dof = n > 1 ? chi2 / (n - 1) : 0.0;
  } else {
    /* no iteration with a positive variance: every weight was equal (in
     * practice, all zero) */
    double m = 0.0;
    int n = 0;
    for (int j = 1; j < n_iter; ++j) { m += Is[j]; ++n; }
    res->I = n ? m / n : (n_iter ? Is[0] : 0.0);
    res->sigma = 0.0;
    res->chi2dof = 0.0;
  }
  if (grid_io) memcpy(grid_io, grid, sizeof(double) * D * (OR_NBINS + 1));
  free(grid); free(bins); free(Is); free(Vs);
}

/* Events integrated independently; event e runs n_iter_ev[e] iterations
 * when that array is given, else n_iter.  OpenMP over (event, assignment)
 * integrals, handed out longest first (by iteration count) so that the
 * threads finish together; every integral's arithmetic is the same in any
 * order. */
static const int32_t* g_iter_key;
static int by_iters_desc(const void* a, const void* b)
{
  const int ia = *(const int*)a, ib = *(const int*)b;
  const int32_t ka = g_iter_key[ia], kb = g_iter_key[ib];
  return ka != kb ? (ka < kb ? 1 : -1) : (ia > ib) - (ia < ib);
}

void or_integrate_events_iters(int kind, const or_params* p, const double* events,
                               int n_events, int n_obj, uint64_t seed, int64_t n_points,
                               int n_iter, const int32_t* n_iter_ev, double alpha, double sigma_norm,
                               double* P, double* err, int32_t* status)
{
  int np = or_nperm(kind);
  int64_t per = (n_points + np - 1) / np;   /* points per permutation */
  int n_int = n_events * np;
  or_result* r = (or_result*)malloc(sizeof(or_result) * (n_int > 0 ? n_int : 1));
  int* order = (int*)malloc(sizeof(int) * (n_int > 0 ? n_int : 1));
  int32_t* key = (int32_t*)malloc(sizeof(int32_t) * (n_int > 0 ? n_int : 1));
  for (int i = 0; i < n_int; ++i) {
    order[i] = i;
    key[i] = n_iter_ev ? n_iter_ev[i / np] : n_iter;
  }
  g_iter_key = key;
  qsort(order, (size_t)n_int, sizeof(int), by_iters_desc);
  #pragma omp parallel for schedule(dynamic, 1)
  for (int q = 0; q < n_int; ++q) {
    int i = order[q];
    int e = i / np, perm = i % np;
    int it = n_iter_ev ? n_iter_ev[e] : n_iter;
    or_integrate_one(kind, p, events + (size_t)e * n_obj * 4, perm, seed, (uint32_t)e,
                     per, it, alpha, NULL, NULL, NULL, &r[i]);
  }
  double norm = sigma_norm > 0.0 ? 1.0 / sigma_norm : 1.0;
  for (int e = 0; e < n_events; ++e) {
    double s = 0.0, v = 0.0;
    int bad = 0;
    for (int k = 0; k < np; ++k) {
      s += r[e * np + k].I;
      v += r[e * np + k].sigma * r[e * np + k].sigma;
      if (!isfinite(r[e * np + k].I)) bad = 1;
    }
    P[e] = norm * s / np;
    err[e] = norm * sqrt(v) / np;
    status[e] = bad ? 3 : (s == 0.0 ? 1 : 0);
  }
  free(r);
  free(order);
  free(key);
}

void or_integrate_events(int kind, const or_params* p, const double* events,
                         int n_events, int n_obj, uint64_t seed, int64_t n_points,
                         int n_iter, double alpha, double sigma_norm,
                         double* P, double* err, int32_t* status)
{
  or_integrate_events_iters(kind, p, events, n_events, n_obj, seed, n_points, n_iter, NULL, alpha,
                            sigma_norm, P, err, status);
}

/* OpenMP thread count of later calls (n < 1: the runtime's default) and the
 * count a parallel region would use now. */
void or_set_threads(int n)
{
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}

int or_max_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------- combining the iterations -- */
/* The estimate of one integral from its iterations' I_j and sigma_j^2,
 * iterations first_kept, first_kept + 1, ... (the first ones only adapt the
 * grid).  mode 0, Lepage's weighting (Sec. 2's VEGAS): I = sum (I_j /
 * sigma_j^2) / sum (1 / sigma_j^2), sigma^2 = 1 / sum (1 / sigma_j^2) over
 * the iterations with sigma_j^2 > 0; with none, the plain mean of the kept
 * I_j and sigma = 0.  mode 1, equal weights: I = mean of the kept I_j,
 * sigma^2 = sum sigma_j^2 / n^2.  Each I_j is unbiased given its grid,
 * which the earlier iterations fixed, so the mean is unbiased; the
 * weighted form is not where a low I_j comes with a low sigma_j^2 (an
 * iteration that missed the large weights). */
void or_combine_iterations(const double* Is, const double* Vs, int n_iter, int first_kept, int mode, double* I,
                           double* sigma)
{
  int n = 0;
  double m = 0.0, vs = 0.0, wsum = 0.0, wIsum = 0.0;
  for (int j = first_kept; j < n_iter; ++j) {
    m += Is[j];
    vs += Vs[j];
    ++n;
    if (Vs[j] > 0.0) { wsum += 1.0 / Vs[j]; wIsum += Is[j] / Vs[j]; }
  }
  if (n == 0) { *I = 0.0; *sigma = 0.0; return; }
  if (mode == 1) {
    *I = m / n;
    *sigma = sqrt(vs) / n;
  } else if (wsum > 0.0) {
    *I = wIsum / wsum;
    *sigma = sqrt(1.0 / wsum);
  } else {
    *I = m / n;
    *sigma = 0.0;
  }
}

/* ------------------------------------------ adaptive stratified VEGAS -- */
/* VEGAS with adaptive stratified sampling (Lepage, "Adaptive
 * multidimensional integration: VEGAS enhanced", J. Comput. Phys. 439
 * (2021) 110386), on top of the importance-sampling grid of Sec. 2's
 * VEGAS.  The unit cube of the map's input is cut into H = n_s^D equal
 * hypercubes; hypercube h (digits c_d of h in base n_s, dimension 0 the
 * least significant) gets n_h points of the N of an iteration, taken in
 * hypercube order: point k of the iteration belongs to the hypercube whose
 * cumulative range holds k, and its input is y_d = (c_d + u_d) / n_s with u
 * the point stream's k-th uniforms.  With w = f(x) J(y):
 *   I = sum_h (1/H) mean_h(w),   var I = sum_h (1/H^2) s_h^2 / n_h,
 * s_h^2 the sample variance of w in h.  The grid adapts from the per-bin
 * sums of w^2 / (H n_h) (each point stands for 1/(H n_h) of the volume).
 * Allocation: the first iteration splits N equally (floor(N/H) each, one
 * more to the first N mod H hypercubes); afterwards every hypercube keeps 2
 * points and the other N - 2H go out in proportion to s_h^beta (beta =
 * 0.75), rounded down, the remainder one each to the first hypercubes in
 * index order (equal split when every s_h is 0).  n_s is the largest
 * integer with 2 n_s^D <= N and n_s^D <= OR_STRAT_HMAX. */
int or_strat_ns(int D, int64_t N)
{
  int ns = 1;
  for (;;) {
    int64_t h = 1;
    for (int d = 0; d < D; ++d) h *= (ns + 1);
    if (2 * h > N || h > OR_STRAT_HMAX) break;
    ++ns;
  }
  return ns;
}

void or_strat_allocate(int64_t H, int64_t N, const double* sig, int first, int64_t* nh)
{
  double tot = 0.0;
  if (!first)
    for (int64_t h = 0; h < H; ++h) tot += sqrt(sig[h] * sqrt(sig[h]));    /* sig^0.75 */
  int64_t used = 0;
  if (first || !(tot > 0.0)) {
    for (int64_t h = 0; h < H; ++h) nh[h] = N / H;
    used = (N / H) * H;
  } else {
    const int64_t R = N - 2 * H;
    for (int64_t h = 0; h < H; ++h) {
      nh[h] = 2 + (int64_t)floor((double)R * (sqrt(sig[h] * sqrt(sig[h])) / tot));
      used += nh[h];
    }
  }
  for (int64_t h = 0; used < N; h = (h + 1) % H) { nh[h] += 1; ++used; }
}

void or_strat_iteration(int kind, const or_params* p, const double* ev, int perm, uint64_t seed,
                        uint32_t event_index, uint32_t iter, int64_t N, const double* grid, int ns,
                        const int64_t* nh, double* I_out, double* var_out, double* sig_out, double* bins,
                        double* w_out)
{
  const int D = or_dims(kind);
  int64_t H = 1;
  for (int d = 0; d < D; ++d) H *= ns;
  memset(bins, 0, sizeof(double) * D * OR_NBINS);
  double I = 0.0, var = 0.0;
  int64_t k = 0;
  for (int64_t h = 0; h < H; ++h) {
    int c[16];
    int64_t r = h;
    for (int d = 0; d < D; ++d) { c[d] = (int)(r % ns); r /= ns; }
    double s1 = 0.0, s2 = 0.0;
    for (int64_t j = 0; j < nh[h]; ++j, ++k) {
      double u[16], y[16], x[16];
      int bi[16];
      or_uniforms(seed, (uint32_t)k, iter, event_index, (uint32_t)perm, D, u);
      for (int d = 0; d < D; ++d) y[d] = ((double)c[d] + u[d]) / (double)ns;
      const double jac = or_vegas_map(grid, D, y, x, bi);
      const double w = integrand(kind, p, ev, perm, x) * jac;
      if (w_out) w_out[k] = w;
      s1 += w;
      s2 += w * w;
      for (int d = 0; d < D; ++d) bins[d * OR_NBINS + bi[d]] += w * w / ((double)H * (double)nh[h]);
    }
    const double n = (double)nh[h];
    const double mean = s1 / n;
    double v = (s2 / n - mean * mean) * n / (n - 1.0);
    if (v < 0.0) v = 0.0;
    I += mean / (double)H;
    var += v / ((double)H * (double)H * n);
    if (sig_out) sig_out[h] = sqrt(v);
  }
  *I_out = I;
  *var_out = var;
}

/* One integral with adaptive stratified VEGAS: n_iter iterations of N
 * points; allocation, estimate and grid refinement as above; iterations
 * combined by inverse variance from the second on (the first adapts
 * only), as or_integrate_one. iter_I, iter_var (may be NULL) per
 * iteration. */
void or_integrate_one_strat(int kind, const or_params* p, const double* ev, int perm, uint64_t seed,
                            uint32_t event_index, int64_t N, int n_iter, double alpha, double* iter_I,
                            double* iter_var, or_result* res)
{
  const int D = or_dims(kind);
  const int ns = or_strat_ns(D, N);
  int64_t H = 1;
  for (int d = 0; d < D; ++d) H *= ns;
  double* grid = (double*)malloc(sizeof(double) * D * (OR_NBINS + 1));
  double* bins = (double*)malloc(sizeof(double) * D * OR_NBINS);
  double* sig = (double*)calloc((size_t)H, sizeof(double));
  int64_t* nh = (int64_t*)malloc(sizeof(int64_t) * (size_t)H);
  double* Is = (double*)malloc(sizeof(double) * (n_iter > 0 ? n_iter : 1));
  double* Vs = (double*)malloc(sizeof(double) * (n_iter > 0 ? n_iter : 1));
  or_vegas_uniform_grid(grid, D);
  double wsum = 0.0, wIsum = 0.0;
  for (int j = 0; j < n_iter; ++j) {
    or_strat_allocate(H, N, sig, j == 0, nh);
    double I, var;
    or_strat_iteration(kind, p, ev, perm, seed, event_index, (uint32_t)j, N, grid, ns, nh, &I, &var, sig, bins,
                       NULL);
    Is[j] = I;
    Vs[j] = var;
    if (iter_I) iter_I[j] = I;
    if (iter_var) iter_var[j] = var;
    if (j >= 1 && var > 0.0) { wsum += 1.0 / var; wIsum += I / var; }
    for (int d = 0; d < D; ++d) or_vegas_refine_dim(bins + d * OR_NBINS, alpha, grid + d * (OR_NBINS + 1));
  }
  res->n_iter_used = n_iter;
  if (wsum > 0.0) {
    res->I = wIsum / wsum;
    res->sigma = sqrt(1.0 / wsum);
    double chi2 = 0.0;
    int n = 0;
    for (int j = 1; j < n_iter; ++j)
      if (Vs[j] > 0.0) { chi2 += (Is[j] - res->I) * (Is[j] - res->I) / Vs[j]; ++n; }
    res->chi2dof = n > 1 ? chi2 / (n - 1) : 0.0;
  } else {
    double m = 0.0;
    int n = 0;
    for (int j = 1; j < n_iter; ++j) { m += Is[j]; ++n; }
    res->I = n ? m / n : (n_iter ? Is[0] : 0.0);
    res->sigma = 0.0;
    res->chi2dof = 0.0;
  }
  free(grid); free(bins); free(sig); free(nh); free(Is); free(Vs);
}
