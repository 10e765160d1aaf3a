// libmem: C ABI of the MI355X matrix element method integrator.
//
// One call to mem_integrate_events runs the whole per-event MC integration
// (Sec. 2 estimator, VEGAS adaptation, Sec. 3/4 integrands) on the device:
// the host only validates, lays out the work list and launches.  Control
// returns to the host once per iteration at most (in target-accuracy mode,
// to read the number of integrals still running).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/mem.h"
#include "flow_kernels.hpp"
#include "flow_sample.hpp"
#include "kernels.hpp"
#include "process_params.hpp"

using namespace memk;

// ---------------------------------------------------------------- errors --
static thread_local std::string g_last_error;

static mem_status fail(mem_status s, const std::string& msg)
{
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(e_ == hipErrorOutOfMemory ? MEM_ENOMEM : MEM_EDEVICE,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

// ------------------------------------------------------------- processes --
struct mem_process_s {
  mem_process_desc desc;
  mem_tf_desc tf[5];
  ProcParams pp;
  int32_t chunk_points = 0;   // tuned points per work-queue chunk (0: library default)
  int32_t waves = 0;          // tuned waves-per-SIMD variant of its queue kernel (0: the default)
  // parton-density grid on the device (null: toy densities) and its shape
  float* pdf_dev = nullptr;
  int pdf_device = -1;        // the device that holds pdf_dev
  int32_t pdf_nx = 0, pdf_nq = 0;
  double pdf_bounds[4] = {0.0, 0.0, 0.0, 0.0};
  // default learned proposal of integrations of this process (null: VEGAS)
  mem_flow proposal = nullptr;
  ~mem_process_s() { if (pdf_dev) (void)hipFree(pdf_dev); }
};

// grid fields of the process parameters from the process's grid
static void apply_pdf(mem_process_s* p)
{
  ProcParams& pp = p->pp;
  pp.pdf_xf = p->pdf_dev;
  if (!p->pdf_dev) return;
  pp.pdf_nx = p->pdf_nx;
  pp.pdf_nq = p->pdf_nq;
  pp.pdf_lx0 = p->pdf_bounds[0];
  pp.pdf_ihx = (p->pdf_nx - 1) / (p->pdf_bounds[1] - p->pdf_bounds[0]);
  pp.pdf_lq0 = p->pdf_bounds[2];
  pp.pdf_ihq = (p->pdf_nq - 1) / (p->pdf_bounds[3] - p->pdf_bounds[2]);
  const double s = (std::log(p->desc.m_top) - pp.pdf_lq0) * pp.pdf_ihq;
  double c = std::floor(s);
  c = c < 0.0 ? 0.0 : c > (double)(p->pdf_nq - 2) ? (double)(p->pdf_nq - 2) : c;
  pp.pdf_iq_mt = (int32_t)c;
  pp.pdf_uq_mt = s - c;
}

static void derive(mem_process_s* p)
{
  p->pp = derive_params(p->desc, p->tf);
  apply_pdf(p);
}

extern "C" mem_status mem_create_process(const mem_process_desc* d, mem_process* out)
{
  if (!d || !out) return fail(MEM_EINVAL, "null argument");
  if (d->kind != MEM_DY_QQ_GAMMA_MUMU && d->kind != MEM_TT_DILEPTON && d->kind != MEM_TT_SEMILEPTON &&
      d->kind != MEM_TTH_SEMILEPTON && d->kind != MEM_TTH_DILEPTON && d->kind != MEM_TTBB_DILEPTON)
    return fail(MEM_EINVAL, "unknown process kind");
  if ((d->kind == MEM_TTH_SEMILEPTON || d->kind == MEM_TTH_DILEPTON) &&
      !(d->m_h > 0.0 && d->w_h > 0.0 && d->m_b >= 0.0))
    return fail(MEM_EINVAL, "Higgs mass and width must be positive");
  if (!(d->sqrt_s > 0.0)) return fail(MEM_EINVAL, "sqrt_s must be positive");
  if (d->precision != MEM_FP64 && d->precision != MEM_FP32) return fail(MEM_EINVAL, "bad precision");
  if (d->kind == MEM_DY_QQ_GAMMA_MUMU) {
    if (!(d->alpha > 0.0)) return fail(MEM_EINVAL, "alpha must be positive");
    if (!(d->m_hi > d->m_lo && d->m_lo >= 0.0)) return fail(MEM_EINVAL, "bad mass window");
    if (d->precision != MEM_FP64) return fail(MEM_EUNSUPPORTED, "Drell-Yan runs in FP64 only");
  } else {
    if (!(d->m_top > 0 && d->w_top > 0 && d->m_w > 0 && d->w_w > 0 && d->alpha_s > 0 && d->g_fermi > 0 &&
          d->sigma_k > 0))
      return fail(MEM_EINVAL, "masses, widths, couplings and sigma_k must be positive");
  }
  if (!(d->sigma_norm >= 0.0)) return fail(MEM_EINVAL, "sigma_norm must be >= 0");
  mem_process_s* p = new (std::nothrow) mem_process_s;
  if (!p) return fail(MEM_ENOMEM, "host allocation");
  p->desc = *d;
  default_tfs(d->kind, p->tf);
  derive(p);
  *out = p;
  return MEM_OK;
}

extern "C" mem_status mem_set_transfer_functions(mem_process p, const mem_tf_desc* tf, int32_t n)
{
  if (!p || (!tf && n > 0) || n < 0) return fail(MEM_EINVAL, "null argument or negative count");
  for (int i = 0; i < n; ++i) {
    const mem_tf_desc& t = tf[i];
    if (t.obj_class < 0 || t.obj_class > MEM_OBJ_NEUTRINO) return fail(MEM_EINVAL, "unknown object class");
    if (t.kind < MEM_TF_DELTA || t.kind > MEM_TF_DGAUSS) return fail(MEM_EINVAL, "unknown TF kind");
    if (t.kind >= MEM_TF_GAUSS && !(t.sigma_core > 0.0)) return fail(MEM_EINVAL, "sigma_core must be > 0");
    if (t.kind == MEM_TF_DGAUSS && !(t.sigma_tail > 0.0)) return fail(MEM_EINVAL, "sigma_tail must be > 0");
    if (t.kind == MEM_TF_DGAUSS && !(t.f_tail >= 0.0 && t.f_tail <= 1.0)) return fail(MEM_EINVAL, "f_tail outside [0,1]");
    if (!(t.window > 0.0) || !(t.r_min >= 0.0)) return fail(MEM_EINVAL, "window must be > 0 and r_min >= 0");
    // the integrated classes need an energy-resolving TF
    if ((t.obj_class == MEM_OBJ_MUON && p->desc.kind == MEM_DY_QQ_GAMMA_MUMU) ||
        (t.obj_class == MEM_OBJ_BJET && p->desc.kind != MEM_DY_QQ_GAMMA_MUMU) ||
        (t.obj_class == MEM_OBJ_LJET && p->desc.kind == MEM_TT_SEMILEPTON))
      if (t.kind < MEM_TF_GAUSS) return fail(MEM_EINVAL, "integrated objects need a (double) Gaussian TF");
  }
  for (int i = 0; i < n; ++i) p->tf[tf[i].obj_class] = tf[i];
  derive(p);
  return MEM_OK;
}

extern "C" void mem_destroy_process(mem_process p) { delete p; }

// Colour matrix of the twelve colour tensors of g g -> t tbar b bbar
// (ttbb_me.hpp), [P|Q]x = P_il Q_kj and [P|Q]= = P_ij Q_kl over (P, Q) =
// (ab,1) (ba,1) (1,ab) (1,ba) (a,b) (b,a), from explicit generators
// T^a = lambda^a / 2: G_mn = sum over a, b, i, j, k, l of t_m conj(t_n).
static void ttbb_colour_matrix(double* G)
{
  typedef std::complex<double> C;
  C T[8][3][3] = {};
  const C I(0.0, 1.0);
  T[0][0][1] = T[0][1][0] = 0.5;
  T[1][0][1] = -0.5 * I; T[1][1][0] = 0.5 * I;
  T[2][0][0] = 0.5; T[2][1][1] = -0.5;
  T[3][0][2] = T[3][2][0] = 0.5;
  T[4][0][2] = -0.5 * I; T[4][2][0] = 0.5 * I;
  T[5][1][2] = T[5][2][1] = 0.5;
  T[6][1][2] = -0.5 * I; T[6][2][1] = 0.5 * I;
  T[7][0][0] = T[7][1][1] = 0.5 / std::sqrt(3.0); T[7][2][2] = -1.0 / std::sqrt(3.0);
  for (int q = 0; q < 144; ++q) G[q] = 0.0;
  std::vector<C> t(12 * 81);
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      // the five matrices 1, T^a, T^b, T^a T^b, T^b T^a
      C M[5][3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          M[0][i][j] = i == j ? 1.0 : 0.0;
          M[1][i][j] = T[a][i][j];
          M[2][i][j] = T[b][i][j];
          C ab = 0.0, ba = 0.0;
          for (int k = 0; k < 3; ++k) { ab += T[a][i][k] * T[b][k][j]; ba += T[b][i][k] * T[a][k][j]; }
          M[3][i][j] = ab;
          M[4][i][j] = ba;
        }
      static const int PQ[6][2] = {{3, 0}, {4, 0}, {0, 3}, {0, 4}, {1, 2}, {2, 1}};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
              const int o = ((i * 3 + j) * 3 + k) * 3 + l;
              for (int m = 0; m < 6; ++m) {
                t[m * 81 + o] = M[PQ[m][0]][i][l] * M[PQ[m][1]][k][j];
                t[(6 + m) * 81 + o] = M[PQ[m][0]][i][j] * M[PQ[m][1]][k][l];
              }
            }
      for (int m = 0; m < 12; ++m)
        for (int n = 0; n < 12; ++n) {
          C s = 0.0;
          for (int o = 0; o < 81; ++o) s += t[m * 81 + o] * std::conj(t[n * 81 + o]);
          G[m * 12 + n] += s.real();
        }
    }
}

// The colour matrix in each device's constant memory, once per device.
static mem_status ensure_ttbb_colour()
{
  static bool done[64] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(MEM_EDEVICE, "hipGetDevice");
  if (done[dev]) return MEM_OK;
  double G[144];
  float Gf[144];
  ttbb_colour_matrix(G);
  for (int q = 0; q < 144; ++q) Gf[q] = (float)G[q];
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(kColTTBB), G, sizeof(G)));
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(kColTTBBf), Gf, sizeof(Gf)));
  done[dev] = true;
  return MEM_OK;
}

// Device state a process needs before a launch: its PDF grid lives on the
// current device; the t tbar b bbar colour matrix is in place.
static mem_status check_pdf_device(const mem_process_s* p)
{
  if (p->desc.kind == MEM_TTBB_DILEPTON) {
    mem_status st = ensure_ttbb_colour();
    if (st != MEM_OK) return st;
  }
  if (!p->pdf_dev) return MEM_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(MEM_EDEVICE, "hipGetDevice");
  if (dev != p->pdf_device)
    return fail(MEM_EINVAL, "the process's PDF grid lives on device " + std::to_string(p->pdf_device) +
                                ", the current device is " + std::to_string(dev));
  return MEM_OK;
}

static mem_status check_pdf_shape(int32_t nx, int32_t nq, const double* b)
{
  if (!b) return fail(MEM_EINVAL, "null bounds");
  if (nx < 2 || nq < 2) return fail(MEM_EINVAL, "the grid needs at least 2 x 2 nodes");
  if ((int64_t)nx * nq > (int64_t)1 << 22) return fail(MEM_EINVAL, "grid above 2^22 nodes");
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(b[k])) return fail(MEM_EINVAL, "bounds must be finite");
  if (!(b[1] > b[0] && b[3] > b[2])) return fail(MEM_EINVAL, "bounds must increase");
  return MEM_OK;
}

extern "C" mem_status mem_set_pdf_grid(mem_process p, const float* xf, int32_t nx, int32_t nq, const double* bounds)
{
  if (!p) return fail(MEM_EINVAL, "null process");
  if (!xf) {
    if (p->pdf_dev) (void)hipFree(p->pdf_dev);
    p->pdf_dev = nullptr;
    apply_pdf(p);
    return MEM_OK;
  }
  if (p->desc.kind == MEM_TTH_SEMILEPTON) return fail(MEM_EUNSUPPORTED, "t tbar H keeps the toy gluon density");
  mem_status st = check_pdf_shape(nx, nq, bounds);
  if (st != MEM_OK) return st;
  const size_t nodes = (size_t)nx * nq;
  // device node layout: quark / antiquark pairs in 16-byte groups
  std::vector<float> pad(nodes * kPdfNode, 0.0f);
  for (size_t n = 0; n < nodes; ++n)
    for (int fl = -5; fl <= 5; ++fl) {
      const float v = xf[n * 11 + fl + 5];
      if (!std::isfinite(v)) return fail(MEM_EINVAL, "non-finite table entry");
      pad[n * kPdfNode + pdf_slot(fl)] = v;
    }
  float* d = nullptr;
  if (hipMalloc(&d, pad.size() * sizeof(float)) != hipSuccess) return fail(MEM_ENOMEM, "device allocation of the grid");
  if (hipMemcpy(d, pad.data(), pad.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return fail(MEM_EDEVICE, "copy of the grid");
  }
  if (p->pdf_dev) (void)hipFree(p->pdf_dev);
  p->pdf_dev = d;
  if (hipGetDevice(&p->pdf_device) != hipSuccess) p->pdf_device = -1;
  p->pdf_nx = nx;
  p->pdf_nq = nq;
  for (int k = 0; k < 4; ++k) p->pdf_bounds[k] = bounds[k];
  apply_pdf(p);
  return MEM_OK;
}

extern "C" mem_status mem_toy_pdf_table(float* xf, int32_t nx, int32_t nq, const double* bounds)
{
  if (!xf) return fail(MEM_EINVAL, "null table");
  mem_status st = check_pdf_shape(nx, nq, bounds);
  if (st != MEM_OK) return st;
  const double hx = (bounds[1] - bounds[0]) / (nx - 1);
  for (int j = 0; j < nq; ++j)
    for (int i = 0; i < nx; ++i) {
      const double x = std::exp(bounds[0] + i * hx), o = 1.0 - x;
      float* v = xf + ((size_t)j * nx + i) * 11;
      for (int k = 0; k < 11; ++k) v[k] = 0.0f;
      if (!(x < 1.0)) continue;
      v[5 + 2] = (float)xfu(x, o);
      v[5 + 1] = (float)xfd(x, o);
      v[5 - 2] = v[5 - 1] = (float)xfq(o);
      v[5] = (float)xfg(o);
    }
  return MEM_OK;
}

extern "C" mem_status mem_process_shape(mem_process p, int32_t* dims, int32_t* n_perm)
{
  if (!p) return fail(MEM_EINVAL, "null process");
  if (dims) *dims = p->pp.dims;
  if (n_perm) *n_perm = p->pp.n_perm;
  return MEM_OK;
}

// ------------------------------------------------------------ kernels ----
__global__ void init_grids_kernel(double* grids, const IntegralDesc* ints, int n_int)
{
  int ig = blockIdx.x;
  if (ig >= n_int) return;
  const IntegralDesc in = ints[ig];
  for (int i = threadIdx.x; i < in.dims * (kBins + 1); i += blockDim.x)
    grids[in.grid_off + i] = (double)(i % (kBins + 1)) / (double)kBins;
}

// Start of an iteration: clear the queue heads and the running count
// (a kernel, not a memset, so that it can live in a captured graph).
__global__ void iter_begin_kernel(Control* ctl, uint32_t* heads, int n_heads)
{
  int i = threadIdx.x;
  if (i < n_heads) heads[i] = 0u;
  if (i == 0) ctl->n_running = 0;
}

__global__ void iter_end_kernel(Control* ctl)
{
  if (threadIdx.x == 0) ctl->iter += 1u;
}

__global__ void fill_kernel(double* p, int64_t n, double v)
{
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v)
{
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Sum the chunk partials of each integral in chunk order, form the
// iteration estimate and its variance, fold it into the inverse-variance
// combination (iterations >= 1) and refine the grid.  One workgroup per
// integral: integral blockIdx.x, or ig_list[blockIdx.x] once the host has
// listed the running events' integrals (late iterations of target mode).
__global__ __launch_bounds__(kBlock) void finish_iter_kernel(const int32_t* __restrict__ ig_list,
                                                             const IntegralDesc* __restrict__ ints,
                                                             const Chunk* __restrict__ chunks,
                                                             const double* __restrict__ parts,
                                                             double* __restrict__ grids,
                                                             double* __restrict__ state,
                                                             const int32_t* __restrict__ active,
                                                             double alpha, const Control* __restrict__ ctl,
                                                             int n_int, double* __restrict__ iter_out,
                                                             const int64_t* __restrict__ alloc,
                                                             double* __restrict__ n_evals, uint32_t first_kept,
                                                             const double* __restrict__ strat_iv)
{
  __shared__ double sb[kMaxDims * kBins];
  __shared__ double scratch[kBlock / kWave][3 * (kBins + 1)];
  const int ig = ig_list ? ig_list[blockIdx.x] : (int)blockIdx.x;
  if (!active[ig]) return;
  const uint32_t iter = ctl->iter;
  const IntegralDesc in = ints[ig];
  const int D = in.dims;
  // this iteration's points: the equal share, or the allocation (its chunks
  // are the first ones of the integral)
  const int64_t npts = alloc ? alloc[ig] : in.n_points;
  int nch = in.n_chunks;
  if (alloc)
    while (nch > 0 && chunks[in.chunk0 + nch - 1].start >= npts) --nch;
  for (int i = threadIdx.x; i < D * kBins; i += kBlock) {
    double acc = 0.0;
    for (int c = 0; c < nch; ++c) acc += parts[chunks[in.chunk0 + c].part_off + 2 + i];
    sb[i] = acc;
  }
  if (threadIdx.x == 0) {
    double s1 = 0.0, s2 = 0.0;
    for (int c = 0; c < nch; ++c) {
      const double* p = parts + chunks[in.chunk0 + c].part_off;
      s1 += p[0];
      s2 += p[1];
    }
    const double N = (double)npts;
    atomicAdd(n_evals, N);
    double I = s1 / N;
    double var = (s2 / N - I * I) / (N - 1.0);
    if (var < 0.0) var = 0.0;
    if (strat_iv) {
      // stratified: the estimate over the hypercubes
      I = strat_iv[2 * ig];
      var = strat_iv[2 * ig + 1];
    }
    double* st = state + (int64_t)ig * ST_SIZE;
    if (!isfinite(s1) || !isfinite(s2) || !isfinite(I) || !isfinite(var)) st[ST_NONFINITE] = 1.0;
    if (iter >= first_kept) {
      if (var > 0.0) { st[ST_WSUM] += 1.0 / var; st[ST_WISUM] += I / var; }
      st[ST_ISUM] += I;
      st[ST_NITER] += 1.0;
      st[ST_VSUM] += var;
    }
    st[ST_LAST_I] = I;
    st[ST_LAST_V] = var;
    if (iter_out) {
      iter_out[((int64_t)iter * n_int + ig) * 2 + 0] = I;
      iter_out[((int64_t)iter * n_int + ig) * 2 + 1] = var;
    }
  }
  __syncthreads();
  const int wave = threadIdx.x / kWave;
  for (int d0 = 0; d0 < D; d0 += kBlock / kWave) {
    const int d = d0 + wave;
    const bool valid = d < D;
    refine_dim_wave(sb + (valid ? d : 0) * kBins, grids + in.grid_off + (valid ? d : 0) * (kBins + 1), alpha,
                    valid, scratch[wave], scratch[wave] + (kBins + 1), scratch[wave] + 2 * (kBins + 1));
  }
}

// Combined estimate of one integral from its running state: inverse-
// variance weights (MEM_COMBINE_WEIGHTED), or equal weights
// (MEM_COMBINE_MEAN: mean of the kept I_j, variance sum sigma_j^2 / n^2).
__device__ __forceinline__ void integral_estimate(const double* st, int combine, double& I, double& var)
{
  if (combine == MEM_COMBINE_MEAN && st[ST_NITER] > 0.0) {
    I = st[ST_ISUM] / st[ST_NITER];
    var = st[ST_VSUM] / (st[ST_NITER] * st[ST_NITER]);
  } else if (st[ST_WSUM] > 0.0) {
    I = st[ST_WISUM] / st[ST_WSUM];
    var = 1.0 / st[ST_WSUM];
  } else {
    I = st[ST_NITER] > 0.0 ? st[ST_ISUM] / st[ST_NITER] : st[ST_LAST_I];
    var = 0.0;
  }
}

// Per event: average over permutations (Sec. 3/4), normalise by sigma, and
// either retire converged events (target mode, during the iterations) or
// write the outputs (final pass).
__global__ void event_kernel(const int64_t* __restrict__ ev_int0, const int32_t* __restrict__ ev_nperm,
                             const double* __restrict__ ev_norm, const double* __restrict__ state,
                             int32_t* __restrict__ active, int n_events, double target, Control* ctl,
                             int final_pass, double* P, double* err, int32_t* status, int32_t* n_iter_used,
                             int32_t* ev_done, uint32_t first_kept, int combine)
{
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_events) return;
  const uint32_t iter = ctl->iter;
  const int64_t i0 = ev_int0[e];
  const int np = ev_nperm[e];
  double s = 0.0, v = 0.0;
  bool bad = false;
  for (int k = 0; k < np; ++k) {
    double I, var;
    const double* st = state + (i0 + k) * ST_SIZE;
    integral_estimate(st, combine, I, var);
    s += I;
    v += var;
    if (st[ST_NONFINITE] != 0.0 || !isfinite(I)) bad = true;
  }
  const double norm = ev_norm[e];
  const double p = norm * s / np, sd = norm * sqrt(v) / np;
  if (!final_pass) {
    if (!ev_done[e] && iter >= first_kept + 1 && (p > 0.0 && sd <= target * p)) {
      ev_done[e] = (int32_t)iter + 1;
      for (int k = 0; k < np; ++k) active[i0 + k] = 0;
    }
    if (!ev_done[e]) atomicAdd(&ctl->n_running, 1);
    return;
  }
  P[e] = p;
  err[e] = sd;
  int32_t stt = MEM_EV_OK;
  if (bad) stt = MEM_EV_NONFINITE;
  else if (s == 0.0) stt = MEM_EV_ZERO_INTEGRAND;
  else if (target > 0.0 && !ev_done[e]) stt = MEM_EV_NOT_CONVERGED;
  status[e] = stt;
  if (n_iter_used) n_iter_used[e] = ev_done[e] ? ev_done[e] : (int32_t)iter;
}

// Neyman allocation of each running event's points among its permutations
// for the next iteration.  sigma_k, the standard deviation of permutation
// k's weights, comes from the last iteration's variance of its mean times
// its points.  The permutation average's variance sum sigma_k^2 / n_k is
// smallest for n_k proportional to sigma_k under a fixed total; here every
// permutation keeps a floor (1/8 of the equal share, so that its grid keeps
// adapting and its variance stays estimated) and the rest of the event's
// budget (n_perm equal shares) goes by sigma_k, water-filled under each
// integral's chunk coverage: a permutation above its cap gets the cap and
// the others share what is left.
constexpr int kMaxPerm = 24;
__global__ void neyman_kernel(const int64_t* __restrict__ ev_int0, const int32_t* __restrict__ ev_nperm,
                              const IntegralDesc* __restrict__ ints, const double* __restrict__ state,
                              const int32_t* __restrict__ active, const int64_t* __restrict__ cap,
                              int64_t* __restrict__ alloc, int n_events)
{
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_events) return;
  const int64_t i0 = ev_int0[e];
  const int np = ev_nperm[e];
  if (np < 2 || np > kMaxPerm || !active[i0]) return;   // retired events keep their allocation
  const int64_t per = ints[i0].n_points;
  const int64_t floor_pts = per / 8 > 2 ? per / 8 : 2;
  double sig[kMaxPerm];
  bool capped[kMaxPerm];
  double ssum = 0.0;
  for (int k = 0; k < np; ++k) {
    const double v = state[(i0 + k) * ST_SIZE + ST_LAST_V];
    sig[k] = sqrt(v * (double)alloc[i0 + k]);
    capped[k] = false;
    ssum += sig[k];
  }
  if (!(ssum > 0.0) || !isfinite(ssum)) return;          // nothing to go by: keep the split
  double rest = (double)(per * np);                       // points for the uncapped permutations
  int n_free = np;
  for (int round = 0; round < np; ++round) {
    double s_free = 0.0;
    for (int k = 0; k < np; ++k) if (!capped[k]) s_free += sig[k];
    const double share = rest - (double)(n_free * floor_pts);
    bool changed = false;
    for (int k = 0; k < np; ++k) {
      if (capped[k]) continue;
      const double want = (double)floor_pts + (s_free > 0.0 ? share * (sig[k] / s_free) : share / n_free);
      if (want > (double)cap[i0 + k]) {
        capped[k] = true;
        rest -= (double)cap[i0 + k];
        --n_free;
        changed = true;
      }
    }
    if (!changed || n_free == 0) {
      for (int k = 0; k < np; ++k) {
        int64_t n;
        if (capped[k]) n = cap[i0 + k];
        else n = floor_pts + (int64_t)(s_free > 0.0 ? share * (sig[k] / s_free) : share / n_free);
        alloc[i0 + k] = n < 2 ? 2 : n > cap[i0 + k] ? cap[i0 + k] : n;
      }
      return;
    }
  }
}

// ---- adaptive stratified sampling (Lepage 2021) ----
// The hypercube of the first point of each chunk of one integral: the
// largest h with cum[h] <= start.  Called by the whole workgroup once the
// integral's cumulative counts are in device memory (written by this
// workgroup before its last barrier).
__device__ void strat_chunk_starts(const int32_t* cum, int H, const Chunk* __restrict__ chunks,
                                   const IntegralDesc& in, int32_t* __restrict__ h0)
{
  for (int i = threadIdx.x; i < in.n_chunks; i += kBlock) {
    const int64_t start = chunks[in.chunk0 + i].start;
    int lo = 0, hi = H - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((int64_t)cum[mid] <= start) lo = mid; else hi = mid - 1;
    }
    h0[in.chunk0 + i] = lo;
  }
}

// First iteration: N split equally over the H hypercubes, floor(N / H)
// each and one more to the first N mod H.
__global__ __launch_bounds__(kBlock) void strat_init_kernel(const IntegralDesc* __restrict__ ints, StratView sv,
                                                            int32_t* __restrict__ cum, const Chunk* __restrict__ chunks,
                                                            int32_t* __restrict__ h0)
{
  const IntegralDesc in = ints[blockIdx.x];
  const StratDesc sd = sv.sd[blockIdx.x];
  const int64_t q = in.n_points / sd.H, r = in.n_points % sd.H;
  int32_t* c = cum + sd.cum_off;
  for (int h = threadIdx.x; h <= sd.H; h += kBlock) c[h] = (int32_t)(h * q + (h < r ? h : r));
  __syncthreads();
  strat_chunk_starts(c, sd.H, chunks, in, h0);
}

// inclusive prefix sum of an int across the workgroup (every thread
// calls it; wsum: kBlock / kWave ints of LDS); *total gets the sum
__device__ __forceinline__ int block_scan_int(int v, int* wsum, int* total)
{
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  if (lane == kWave - 1) wsum[wave] = v;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    before += w < wave ? wsum[w] : 0;
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return v + before;
}

// After an iteration's integrand launches, per running integral (one
// workgroup, thread t taking hypercubes t, t + 256, ... so that a
// wavefront's reads are neighbours): each hypercube's mean and sample
// variance of its weights, summed in point order
// (s^2 = (sum w^2 / n - mean^2) n / (n - 1), clipped at 0); the iteration
// estimate sum_h mean_h / H and its variance sum_h s_h^2 / (H^2 n_h) are the
// threads' partial sums added in thread order, so the result does not
// depend on scheduling.  The next iteration's allocation: 2 points per
// hypercube plus floor((N - 2H) s_h^0.75 / sum_h s_h^0.75), the remainder
// one each to the first hypercubes in index order (equal split when the sum
// is 0 or not finite), turned into cumulative counts in place.  s_h^0.75 is
// formed as sqrt(s sqrt(s)).
__global__ __launch_bounds__(kBlock) void strat_finish_kernel(const IntegralDesc* __restrict__ ints, StratView sv,
                                                              int32_t* __restrict__ cum, double* __restrict__ sigb,
                                                              const int32_t* __restrict__ active,
                                                              const Chunk* __restrict__ chunks,
                                                              int32_t* __restrict__ h0, double* __restrict__ strat_iv)
{
  __shared__ double pI[kBlock], pV[kBlock], pS[kBlock];
  __shared__ int64_t pN[kBlock];
  __shared__ double tot[3];
  __shared__ int64_t used_all;
  __shared__ int wsum[kBlock / kWave];
  const int ig = blockIdx.x;
  if (!active[ig]) return;
  const IntegralDesc in = ints[ig];
  const StratDesc sd = sv.sd[ig];
  const int H = sd.H;
  const int64_t N = in.n_points;
  int32_t* c = cum + sd.cum_off;
  const double* w = sv.w + sd.w_off;
  double* sg = sigb + sd.cum_off;
  const double Hd = (double)H;
  double Ip = 0.0, Vp = 0.0, Sp = 0.0;
  for (int h = threadIdx.x; h < H; h += kBlock) {
    const int32_t k0 = c[h], k1 = c[h + 1];
    double s1 = 0.0, s2 = 0.0;
#pragma unroll 4
    for (int32_t k = k0; k < k1; ++k) {
      const double x = w[k];
      s1 += x;
      s2 += x * x;
    }
    const double n = (double)(k1 - k0);
    const double mean = s1 / n;
    double v = (s2 / n - mean * mean) * n / (n - 1.0);
    if (v < 0.0) v = 0.0;
    Ip += mean / Hd;
    Vp += v / (Hd * Hd * n);
    const double sig = sqrt(v);
    const double b = sqrt(sig * sqrt(sig));
    sg[h] = b;
    Sp += b;
  }
  pI[threadIdx.x] = Ip;
  pV[threadIdx.x] = Vp;
  pS[threadIdx.x] = Sp;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, v = 0.0, d = 0.0;
    for (int t = 0; t < kBlock; ++t) { a += pI[t]; v += pV[t]; d += pS[t]; }
    tot[0] = a; tot[1] = v; tot[2] = d;
    strat_iv[2 * ig] = a;
    strat_iv[2 * ig + 1] = v;
  }
  __syncthreads();     // every read of this iteration's counts is done
  const double S = tot[2];
  const bool equal = !(S > 0.0) || !isfinite(S);
  const int64_t R = N - 2 * (int64_t)H;
  // the counts before the remainder, in place of the cumulative counts
  int64_t u = 0;
  for (int h = threadIdx.x; h < H; h += kBlock) {
    const int64_t n = equal ? N / H : 2 + (int64_t)floor((double)R * (sg[h] / S));
    c[h] = (int32_t)n;
    u += n;
  }
  pN[threadIdx.x] = u;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t a = 0;
    for (int t = 0; t < kBlock; ++t) a += pN[t];
    used_all = a;
  }
  __syncthreads();
  const int64_t rem = N - used_all;       // 0 <= rem <= H
  // exclusive prefix sums in tiles of kBlock hypercubes (counts < 2^31)
  int off = 0;
  for (int base = 0; base < H; base += kBlock) {
    const int h = base + threadIdx.x;
    const int n = h < H ? c[h] + (h < rem ? 1 : 0) : 0;
    int tile = 0;
    const int incl = block_scan_int(n, wsum, &tile);
    if (h < H) c[h] = off + incl - n;
    off += tile;
  }
  if (threadIdx.x == 0) c[H] = off;
  __syncthreads();
  strat_chunk_starts(c, H, chunks, in, h0);
}

template <int KIND, int D, class T>
__global__ __launch_bounds__(kBlock) void eval_points_kernel(ProcParams pp, EventsView ev, int event, int perm,
                                                             const double* __restrict__ xs, int64_t n,
                                                             double* __restrict__ f, int32_t* __restrict__ nsol)
{
  int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  double x[D];
#pragma unroll
  for (int d = 0; d < D; ++d) x[d] = xs[k * D + d];
  int ns = 0;
  if constexpr (KIND == kDY) {
    DYEvent e;
    dy_load(ev, event, e);
    f[k] = dy_integrand(pp, e, x);
  } else if constexpr (KIND == kTT) {
    TTEvent e;
    tt_load(ev, event, perm, e);
    f[k] = tt_integrand<T>(pp, e, x, &ns);
  } else if constexpr (KIND == kSL) {
    SLEvent e;
    sl_load(ev, ev.charge, event, perm, e);
    f[k] = sl_integrand<T>(pp, e, x, &ns);
  } else if constexpr (KIND == kTHL || KIND == kTBB) {
    F2Event e;
    f2_load(ev, KIND == kTHL, event, perm, e);
    f[k] = f2_integrand<T, KIND == kTHL>(pp, e, x, &ns);
  } else {
    TTHEvent e;
    tth_load(ev, ev.charge, event, perm, e);
    f[k] = tth_integrand<T>(pp, e, x, &ns);
  }
  if (nsol) nsol[k] = ns;
}

__global__ void uniforms_kernel(uint64_t seed, uint32_t iter, uint32_t event, uint32_t perm, int D, int64_t n,
                                double* __restrict__ u)
{
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  for (int b = 0; 2 * b < D; ++b) {
    u32x4 w = philox10(u32x4{(uint32_t)k, iter, event, perm * 16u + (uint32_t)b}, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
    u[k * D + 2 * b] = u53(w.x, w.y);
    if (2 * b + 1 < D) u[k * D + 2 * b + 1] = u53(w.z, w.w);
  }
}

__global__ __launch_bounds__(kBlock) void refine_only_kernel(const double* __restrict__ bins,
                                                             double* __restrict__ grids, int D, double alpha)
{
  __shared__ double scratch[kBlock / kWave][3 * (kBins + 1)];
  __shared__ double sb[kMaxDims * kBins];
  const int ig = blockIdx.x;
  for (int i = threadIdx.x; i < D * kBins; i += kBlock) sb[i] = bins[(int64_t)ig * D * kBins + i];
  __syncthreads();
  const int wave = threadIdx.x / kWave;
  for (int d0 = 0; d0 < D; d0 += kBlock / kWave) {
    const int d = d0 + wave;
    const bool valid = d < D;
    refine_dim_wave(sb + (valid ? d : 0) * kBins, grids + ((int64_t)ig * D + (valid ? d : 0)) * (kBins + 1),
                    alpha, valid, scratch[wave], scratch[wave] + (kBins + 1), scratch[wave] + 2 * (kBins + 1));
  }
}

// ------------------------------------------------------------ helpers ----
namespace {

// Device memory of one call's work buffers: hipMalloc / hipFree, the
// caller's allocator hook, or a fixed arena handed in by the caller of the
// no-allocation entry point.  Blocks go back (hook, hipFree) when the
// workspace is destroyed, after the call has synchronised its stream.
class Workspace {
 public:
  Workspace() = default;
  Workspace(mem_alloc_fn a, mem_free_fn f, void* user, hipStream_t s) : afn_(a), ffn_(f), user_(user), s_(s) {}
  Workspace(char* arena, size_t cap) : arena_(arena), cap_(cap) {}
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  ~Workspace()
  {
    // a call that returns early may still have work queued on the caller's
    // stream: the hook's memory may be handed out again at once
    if (afn_ && !blocks_.empty()) (void)hipStreamSynchronize(s_);
    for (auto& b : blocks_) {
      if (afn_) ffn_(b.first, b.second, (void*)s_, user_);
      else (void)hipFree(b.first);
    }
  }
  bool arena() const { return arena_ != nullptr; }
  size_t used() const { return used_; }
  size_t capacity() const { return cap_; }
  // bytes the call has asked the arena for, the refused requests included
  size_t requested() const { return need_; }
  hipError_t get(void** p, size_t bytes)
  {
    bytes = bytes ? (bytes + 255) / 256 * 256 : 256;
    *p = nullptr;
    if (arena_) {
      need_ += bytes;
      if (need_ > cap_) return hipErrorOutOfMemory;
      *p = arena_ + used_;
      used_ += bytes;
      return hipSuccess;
    }
    if (afn_) {
      void* q = afn_(bytes, (void*)s_, user_);
      if (!q) return hipErrorOutOfMemory;
      *p = q;
    } else {
      hipError_t e = hipMalloc(p, bytes);
      if (e != hipSuccess) return e;
    }
    blocks_.emplace_back(*p, bytes);
    used_ += bytes;
    return hipSuccess;
  }

 private:
  mem_alloc_fn afn_ = nullptr;
  mem_free_fn ffn_ = nullptr;
  void* user_ = nullptr;
  hipStream_t s_ = nullptr;
  char* arena_ = nullptr;
  size_t cap_ = 0, used_ = 0, need_ = 0;
  std::vector<std::pair<void*, size_t>> blocks_;
};

// A device buffer: its own hipMalloc block, or a block of a workspace
// (released with the workspace).
struct DevBuf {
  void* p = nullptr;
  Workspace* w = nullptr;
  DevBuf() = default;
  explicit DevBuf(Workspace* ws) : w(ws) {}
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { if (p && !w) (void)hipFree(p); }
  hipError_t alloc(size_t bytes) { return w ? w->get(&p, bytes) : hipMalloc(&p, bytes ? bytes : 8); }
  template <class X> X* as() const { return (X*)p; }
};

constexpr int64_t kDefaultChunk = 4096;   // points per work-queue chunk

int n_obj_of(int kind)
{
  return kind == MEM_DY_QQ_GAMMA_MUMU ? 2 : kind == MEM_TT_SEMILEPTON ? 5 : kind == MEM_TTH_SEMILEPTON ? 7
       : (kind == MEM_TTH_DILEPTON || kind == MEM_TTBB_DILEPTON) ? 6 : 4;
}
bool is_f2(int kind) { return kind == MEM_TTH_DILEPTON || kind == MEM_TTBB_DILEPTON; }

// relative cost of one evaluation (for the longest-first queue order)
double eval_cost(int kind)
{
  return kind == MEM_DY_QQ_GAMMA_MUMU ? 1.0 : kind == MEM_TT_SEMILEPTON ? 12.0 : kind == MEM_TTH_SEMILEPTON ? 30.0
       : kind == MEM_TTH_DILEPTON ? 40.0 : kind == MEM_TTBB_DILEPTON ? 200.0 : 30.0;
}

int kind_mask(int kind)
{
  return kind == MEM_DY_QQ_GAMMA_MUMU ? kMaskDY : kind == MEM_TT_DILEPTON ? kMaskTT
       : kind == MEM_TT_SEMILEPTON ? kMaskSL : kind == MEM_TTH_DILEPTON ? kMaskTHL
       : kind == MEM_TTBB_DILEPTON ? kMaskTBB : kMaskTTH;
}

mem_status check_event_arrays(const mem_events* ev)
{
  if (!ev) return fail(MEM_EINVAL, "null events");
  if (ev->n_events < 0 || ev->n_obj <= 0) return fail(MEM_EINVAL, "bad event sizes");
  if (ev->n_events > 0 && (!ev->E || !ev->px || !ev->py || !ev->pz)) return fail(MEM_EINVAL, "null event arrays");
  return MEM_OK;
}

// Host-side events: every object the event's process uses must be finite
// with a positive energy; charges must be +-1.
mem_status check_host_event(const mem_events* ev, int e, int n_obj_used)
{
  if (ev->on_device) return MEM_OK;
  for (int o = 0; o < n_obj_used; ++o) {
    int64_t i = (int64_t)o * ev->n_events + e;
    double E = ev->E[i], x = ev->px[i], y = ev->py[i], z = ev->pz[i];
    if (!std::isfinite(E) || !std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
      return fail(MEM_EINVAL, "non-finite event component");
    if (!(E > 0.0)) return fail(MEM_EINVAL, "non-positive object energy");
  }
  if (ev->charge && !(ev->charge[e] == 1 || ev->charge[e] == -1)) return fail(MEM_EINVAL, "charge must be +1 or -1");
  return MEM_OK;
}

// Events resident on the device for the duration of a call.
struct DevEvents {
  DevBuf buf, cbuf;
  EventsView view{};
  DevEvents() = default;
  explicit DevEvents(Workspace* w) : buf(w), cbuf(w) {}
  mem_status make(const mem_events* ev, hipStream_t s)
  {
    view.n_events = ev->n_events;
    view.n_obj = ev->n_obj;
    if (ev->on_device) {
      view.E = ev->E; view.px = ev->px; view.py = ev->py; view.pz = ev->pz;
      view.charge = ev->charge;
      return MEM_OK;
    }
    size_t n = (size_t)ev->n_events * ev->n_obj;
    HIP_TRY(buf.alloc(4 * n * sizeof(double)));
    double* d = buf.as<double>();
    HIP_TRY(hipMemcpyAsync(d, ev->E, n * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d + n, ev->px, n * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d + 2 * n, ev->py, n * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d + 3 * n, ev->pz, n * sizeof(double), hipMemcpyHostToDevice, s));
    view.E = d; view.px = d + n; view.py = d + 2 * n; view.pz = d + 3 * n;
    view.charge = nullptr;
    if (ev->charge) {
      HIP_TRY(cbuf.alloc((size_t)ev->n_events * sizeof(int32_t)));
      HIP_TRY(hipMemcpyAsync(cbuf.p, ev->charge, (size_t)ev->n_events * sizeof(int32_t), hipMemcpyHostToDevice, s));
      view.charge = cbuf.as<int32_t>();
    }
    return MEM_OK;
  }
};

// Persistent grid: enough workgroups to fill every CU at the kernel's
// occupancy (never more than there are chunks).
// The queue kernel instance for a precision and a set of kinds.
typedef void (*QueueKernel)(const ProcParams*, EventsView, const Chunk*, int64_t, const IntegralDesc*,
                            const double*, const int32_t*, uint64_t, Control*, uint32_t*, double*,
                            const int64_t*, QueueHooks, StratView);
// Waves-per-SIMD variants compiled per process kind (the first is the
// default): Drell-Yan also at 2 and 4, the top kinds at 1 and 2 (spills
// beyond), t tbar H at 2 only.
int waves_variants(int kind, int* out)
{
  switch (kind) {
    case MEM_DY_QQ_GAMMA_MUMU: out[0] = 1; out[1] = 2; out[2] = 4; return 3;
    case MEM_TTH_SEMILEPTON: out[0] = 2; return 1;
    default: out[0] = 1; out[1] = 2; return 2;
  }
}
bool waves_supported(int kind, int waves)
{
  int v[4];
  const int n = waves_variants(kind, v);
  for (int i = 0; i < n; ++i) if (v[i] == waves) return true;
  return false;
}
// The queue kernel instance for a precision, a set of kinds and a waves
// variant (0: the default; a launch of several kinds takes the default).
template <class T>
QueueKernel queue_kernel_for(int mask, int waves)
{
  switch (mask) {
    case kMaskDY:
      return waves == 2 ? vegas_queue_kernel<T, kMaskDY, 2> : waves == 4 ? vegas_queue_kernel<T, kMaskDY, 4>
                                                                          : vegas_queue_kernel<T, kMaskDY>;
    case kMaskTT: return waves == 2 ? vegas_queue_kernel<T, kMaskTT, 2> : vegas_queue_kernel<T, kMaskTT>;
    case kMaskSL: return waves == 2 ? vegas_queue_kernel<T, kMaskSL, 2> : vegas_queue_kernel<T, kMaskSL>;
    case kMaskTTH: return vegas_queue_kernel<T, kMaskTTH>;
    case kMaskTHL: return waves == 2 ? vegas_queue_kernel<T, kMaskTHL, 2> : vegas_queue_kernel<T, kMaskTHL>;
    case kMaskTBB: return waves == 2 ? vegas_queue_kernel<T, kMaskTBB, 2> : vegas_queue_kernel<T, kMaskTBB>;
    case kMaskTHL | kMaskTBB: return vegas_queue_kernel<T, kMaskTHL | kMaskTBB>;
    default:
      if (!(mask & kMaskTTH)) return vegas_queue_kernel<T, kMaskDY | kMaskTT | kMaskSL>;
      return vegas_queue_kernel<T, kMaskDY | kMaskTT | kMaskSL | kMaskTTH>;
  }
}

// Persistent grid: enough workgroups to fill every CU at the kernel's
// occupancy (never more than there are chunks).
int persistent_blocks(QueueKernel k, int64_t n_chunks)
{
  int dev = 0, cus = 256, per_cu = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  int64_t b = (int64_t)cus * per_cu;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, n_chunks));
}

// One launch group: chunks whose processes share the matrix-element
// precision (Drell-Yan, always FP64, joins the first group).
struct Group {
  int prec;
  std::vector<int32_t> queue;   // chunk indices, longest first
  int mask = 0;                 // kinds present
  int blocks = 0;
  QueueKernel kernel = nullptr;
  int waves = -1;               // the processes' waves variant (0: they differ)
};

}  // namespace

// ------------------------------------------------------ checkpoints ----
// The state of a VEGAS integration between calls, in host memory: what
// identifies the integration (so that a resume can be refused when the
// call differs) and everything the device iterates on.
struct mem_checkpoint_s {
  bool has = false;
  // identity
  int32_t n_ev = 0, n_int = 0, allocation = 0;
  uint64_t seed = 0;
  double alpha = 0.0;
  std::vector<uint64_t> ev_key;       // per event: hash of its process's description and TFs
  std::vector<int64_t> int_key;       // per integral: event, perm, dims, points per iteration
  // state
  uint32_t iter = 0;
  std::vector<double> grids, state;
  std::vector<int32_t> active, done;
  std::vector<int64_t> alloc;
};

namespace {

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull)
{
  const unsigned char* c = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  return h;
}

uint64_t process_key(const mem_process_s* p)
{
  uint64_t h = fnv1a(&p->desc, sizeof(p->desc));
  h = fnv1a(p->tf, sizeof(p->tf), h);
  h = fnv1a(&p->pdf_dev, sizeof(p->pdf_dev), h);
  return h;
}

}  // namespace

extern "C" mem_status mem_checkpoint_create(mem_checkpoint* out)
{
  if (!out) return fail(MEM_EINVAL, "null argument");
  *out = new (std::nothrow) mem_checkpoint_s();
  return *out ? MEM_OK : fail(MEM_ENOMEM, "checkpoint allocation failed");
}

extern "C" void mem_checkpoint_destroy(mem_checkpoint c) { delete c; }

extern "C" mem_status mem_checkpoint_iterations(mem_checkpoint c, int32_t* n_iter)
{
  if (!c || !n_iter) return fail(MEM_EINVAL, "null argument");
  *n_iter = c->has ? (int32_t)c->iter : 0;
  return MEM_OK;
}

namespace {

constexpr char kCkptMagic[8] = {'M', 'E', 'M', 'C', 'K', 'P', 'T', '1'};

template <class V>
bool put_vec(std::FILE* f, const std::vector<V>& v)
{
  const uint64_t n = v.size();
  return std::fwrite(&n, sizeof(n), 1, f) == 1 && (n == 0 || std::fwrite(v.data(), sizeof(V), n, f) == n);
}
template <class V>
bool get_vec(std::FILE* f, std::vector<V>& v)
{
  uint64_t n = 0;
  if (std::fread(&n, sizeof(n), 1, f) != 1 || n > ((uint64_t)1 << 36) / sizeof(V)) return false;
  v.resize(n);
  return n == 0 || std::fread(v.data(), sizeof(V), n, f) == n;
}

}  // namespace

extern "C" mem_status mem_checkpoint_save(mem_checkpoint c, const char* path)
{
  if (!c || !path) return fail(MEM_EINVAL, "null argument");
  if (!c->has) return fail(MEM_EINVAL, "empty checkpoint");
  std::FILE* f = std::fopen(path, "wb");
  if (!f) return fail(MEM_EINVAL, std::string("cannot write ") + path);
  bool ok = std::fwrite(kCkptMagic, 1, 8, f) == 8;
  ok = ok && std::fwrite(&c->n_ev, sizeof(int32_t), 1, f) == 1 && std::fwrite(&c->n_int, sizeof(int32_t), 1, f) == 1;
  ok = ok && std::fwrite(&c->allocation, sizeof(int32_t), 1, f) == 1 && std::fwrite(&c->iter, sizeof(uint32_t), 1, f) == 1;
  ok = ok && std::fwrite(&c->seed, sizeof(uint64_t), 1, f) == 1 && std::fwrite(&c->alpha, sizeof(double), 1, f) == 1;
  ok = ok && put_vec(f, c->ev_key) && put_vec(f, c->int_key) && put_vec(f, c->grids) && put_vec(f, c->state);
  ok = ok && put_vec(f, c->active) && put_vec(f, c->done) && put_vec(f, c->alloc);
  ok = (std::fclose(f) == 0) && ok;
  return ok ? MEM_OK : fail(MEM_EINVAL, std::string("write failed: ") + path);
}

extern "C" mem_status mem_checkpoint_load(const char* path, mem_checkpoint* out)
{
  if (!path || !out) return fail(MEM_EINVAL, "null argument");
  std::FILE* f = std::fopen(path, "rb");
  if (!f) return fail(MEM_EINVAL, std::string("cannot read ") + path);
  mem_checkpoint_s c;
  char magic[8];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kCkptMagic, 8) == 0;
  ok = ok && std::fread(&c.n_ev, sizeof(int32_t), 1, f) == 1 && std::fread(&c.n_int, sizeof(int32_t), 1, f) == 1;
  ok = ok && std::fread(&c.allocation, sizeof(int32_t), 1, f) == 1 && std::fread(&c.iter, sizeof(uint32_t), 1, f) == 1;
  ok = ok && std::fread(&c.seed, sizeof(uint64_t), 1, f) == 1 && std::fread(&c.alpha, sizeof(double), 1, f) == 1;
  ok = ok && get_vec(f, c.ev_key) && get_vec(f, c.int_key) && get_vec(f, c.grids) && get_vec(f, c.state);
  ok = ok && get_vec(f, c.active) && get_vec(f, c.done) && get_vec(f, c.alloc);
  std::fclose(f);
  ok = ok && c.n_ev >= 0 && c.n_int >= 0 && (int64_t)c.ev_key.size() == c.n_ev &&
       (int64_t)c.int_key.size() == 4 * (int64_t)c.n_int && (int64_t)c.state.size() == (int64_t)c.n_int * ST_SIZE &&
       (int64_t)c.active.size() == c.n_int && (int64_t)c.done.size() == c.n_ev &&
       (c.alloc.empty() || (int64_t)c.alloc.size() == c.n_int);
  if (!ok) return fail(MEM_EINVAL, std::string("malformed checkpoint file ") + path);
  c.has = true;
  *out = new (std::nothrow) mem_checkpoint_s(std::move(c));
  return *out ? MEM_OK : fail(MEM_ENOMEM, "checkpoint allocation failed");
}

static mem_status integrate_flow(const mem_events* ev, const mem_process* hyp, int32_t n_hyp,
                                 const int64_t* n_points, int32_t n_np, int32_t iters, const mem_integrate_opts& o,
                                 double* p_out, double* err_out, int32_t* status_out, Workspace& work);

static mem_status integrate_vegas(const mem_events* ev, const mem_process* hyp, int32_t n_hyp,
                                  const int64_t* n_points, int32_t n_np, int32_t iters, const mem_integrate_opts& o,
                                  double* p_out, double* err_out, int32_t* status_out, const int32_t* ev_mask,
                                  Workspace& work, mem_flow seed_flow = nullptr);
static mem_status seed_grids_from_flow(mem_flow f, const EventsView& view, const std::vector<IntegralDesc>& ints,
                                       const IntegralDesc* d_ints, double* grids, uint64_t seed, Workspace& work,
                                       hipStream_t s);

// ---------------------------------------------------------- integrate ----
// arena: null (work buffers from hipMalloc or the caller's allocator), or
// the no-allocation entry point's scratch of arena_bytes
static mem_status integrate_entry(const mem_events* ev, const mem_process* hyp, int32_t n_hyp,
                                  const int64_t* n_points, int32_t n_np, int32_t n_iter,
                                  const mem_integrate_opts* opt, double* p_out, double* err_out,
                                  int32_t* status_out, void* arena, size_t arena_bytes)
{
  mem_status st = check_event_arrays(ev);
  if (st != MEM_OK) return st;
  const int n_ev = ev->n_events;
  if (!hyp || !n_points) return fail(MEM_EINVAL, "null argument");
  if (n_ev > 0 && (!p_out || !err_out || !status_out)) return fail(MEM_EINVAL, "null output");
  if (!(n_hyp == 1 || n_hyp == n_ev)) return fail(MEM_EINVAL, "n_hyp must be 1 or n_events");
  if (!(n_np == 1 || n_np == n_ev)) return fail(MEM_EINVAL, "n_np must be 1 or n_events");
  mem_integrate_opts o{};
  o.seed = 0x14077595ull;
  o.alpha = 1.5;
  o.max_iter = 64;
  o.use_graph = 1;
  if (opt) o = *opt;
  if (!(o.alpha > 0.0)) return fail(MEM_EINVAL, "alpha must be positive");
  if (o.allocation != MEM_ALLOC_EQUAL && o.allocation != MEM_ALLOC_NEYMAN) return fail(MEM_EINVAL, "unknown allocation");
  if (o.flow_mode != MEM_FLOW_SAMPLE && o.flow_mode != MEM_FLOW_SEED_GRID) return fail(MEM_EINVAL, "unknown flow_mode");
  if (o.stratify != MEM_STRATIFY_OFF && o.stratify != MEM_STRATIFY_ADAPTIVE) return fail(MEM_EINVAL, "unknown stratify");
  if (o.combine != MEM_COMBINE_WEIGHTED && o.combine != MEM_COMBINE_MEAN) return fail(MEM_EINVAL, "unknown combine");
  if (o.tail_chunk_points != 0) {
    if (o.tail_chunk_points < 0 || o.tail_chunk_points % kBlock != 0 || o.tail_chunk_points > 65536)
      return fail(MEM_EINVAL, "tail_chunk_points must be 0 or a multiple of 256 <= 65536");
    if (o.tail_iter < 1) return fail(MEM_EINVAL, "tail_iter must be at least 1");
    if (o.stratify) return fail(MEM_EUNSUPPORTED, "tail chunking of stratified integrations");
  }
  if (o.stratify) {
    if (o.allocation == MEM_ALLOC_NEYMAN) return fail(MEM_EINVAL, "stratified sampling takes the equal split across permutations");
    if (o.flow) return fail(MEM_EUNSUPPORTED, "stratified sampling is VEGAS-only");
    if (o.checkpoint) return fail(MEM_EUNSUPPORTED, "no checkpoints of stratified integrations");
  }
  const bool target_mode = o.target_rel_err > 0.0;
  const int iters = target_mode ? o.max_iter : n_iter;
  const bool resume = o.checkpoint && o.checkpoint->has;
  if (iters < (resume ? 1 : 2)) return fail(MEM_EINVAL, "at least two iterations are needed (one when resuming)");
  if (iters > 100000) return fail(MEM_EINVAL, "too many iterations");
  int64_t chunk_pts = o.chunk_points > 0 ? o.chunk_points : kDefaultChunk;
  if (chunk_pts % kBlock != 0 || chunk_pts > 65536) return fail(MEM_EINVAL, "chunk_points must be a multiple of 256 <= 65536");
  if ((o.alloc_fn == nullptr) != (o.free_fn == nullptr)) return fail(MEM_EINVAL, "alloc_fn and free_fn go together");
  if (o.hooks & ~(uint32_t)MEM_HOOK_NONFINITE) return fail(MEM_EINVAL, "unknown hook");
  if ((o.hooks & MEM_HOOK_NONFINITE) && (o.hook_event < 0 || o.hook_event >= n_ev))
    return fail(MEM_EINVAL, "hook_event outside the events");
  if (!o.flow && !o.stratify && n_ev > 0) {
    // the processes' own proposal (mem_set_proposal), when they share one
    mem_flow pf = hyp[0] ? hyp[0]->proposal : nullptr;
    for (int i = 1; i < n_hyp && pf; ++i)
      if (!hyp[i] || hyp[i]->proposal != pf) pf = nullptr;
    o.flow = pf;
  }
  if (o.flow && (o.weights_out || o.checkpoint || o.hooks))
    return fail(MEM_EUNSUPPORTED, "weights_out, checkpoints and hooks are VEGAS-only");
  if (n_ev == 0) return MEM_OK;
  if (arena) {
    if (o.flow) return fail(MEM_EUNSUPPORTED, "the no-allocation entry point integrates with VEGAS only");
    if (o.timing_out) return fail(MEM_EUNSUPPORTED, "timing_out creates events: not in the no-allocation entry point");
    if (o.alloc_fn) return fail(MEM_EINVAL, "the no-allocation entry point takes no allocator");
    if (!ev->on_device || !o.outputs_on_device)
      return fail(MEM_EINVAL, "the no-allocation entry point needs events and outputs in device memory");
    // direct launches on the caller's stream: no graph, no stream of its own
    o.use_graph = 0;
    Workspace work((char*)arena, arena_bytes);
    return integrate_vegas(ev, hyp, n_hyp, n_points, n_np, iters, o, p_out, err_out, status_out, nullptr, work);
  }
  Workspace work(o.alloc_fn, o.free_fn, o.alloc_user, (hipStream_t)o.stream);
  if (o.flow && o.flow_mode == MEM_FLOW_SEED_GRID) {
    for (int i = 0; i < n_hyp; ++i)
      if (!hyp[i] || hyp[i]->desc.kind != MEM_TT_DILEPTON)
        return fail(MEM_EUNSUPPORTED, "flow-seeded grids cover ttbar dilepton only");
    return integrate_vegas(ev, hyp, n_hyp, n_points, n_np, iters, o, p_out, err_out, status_out, nullptr, work,
                           o.flow);
  }
  if (o.flow) return integrate_flow(ev, hyp, n_hyp, n_points, n_np, iters, o, p_out, err_out, status_out, work);
  return integrate_vegas(ev, hyp, n_hyp, n_points, n_np, iters, o, p_out, err_out, status_out, nullptr, work);
}

extern "C" mem_status mem_integrate_events(const mem_events* ev, const mem_process* hyp, int32_t n_hyp,
                                           const int64_t* n_points, int32_t n_np, int32_t n_iter,
                                           const mem_integrate_opts* opt, double* p_out, double* err_out,
                                           int32_t* status_out)
{
  return integrate_entry(ev, hyp, n_hyp, n_points, n_np, n_iter, opt, p_out, err_out, status_out, nullptr, 0);
}

// ------------------------------------------------------- no allocation ----
// The work buffers of mem_integrate_events_noalloc live in this array: one
// copy per device, held until the process ends.  In host code its name is
// not a device address; the address of the current device's copy comes
// from hipGetSymbolAddress, once per device, and only that address is
// handed to kernels and copies.
static __device__ __align__(256) char scratch[MEM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

mem_status scratch_of_current_device(void** out)
{
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(MEM_EDEVICE, "device number outside the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(MEM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MEM_OK;
}
}  // namespace

extern "C" mem_status mem_integrate_events_noalloc(const mem_events* ev, const mem_process* hyp, int32_t n_hyp,
                                                   const int64_t* n_points, int32_t n_np, int32_t n_iter,
                                                   const mem_integrate_opts* opt, double* p_out, double* err_out,
                                                   int32_t* status_out)
{
  if (!opt) return fail(MEM_EINVAL, "the no-allocation entry point needs options (device outputs, stream)");
  void* base = nullptr;
  const mem_status st = scratch_of_current_device(&base);
  if (st != MEM_OK) return st;
  return integrate_entry(ev, hyp, n_hyp, n_points, n_np, n_iter, opt, p_out, err_out, status_out, base,
                         (size_t)MEM_NOALLOC_SCRATCH_BYTES);
}

// VEGAS over every event, or over the events with ev_mask[e] != 0 (host
// array; the others are skipped and their outputs are undefined).
// seed_flow: the proposal whose samples seed every integral's grid (then
// every iteration enters the estimate), or null (uniform grids, the first
// iteration only adapts).
static mem_status integrate_vegas(const mem_events* ev, const mem_process* hyp, int32_t n_hyp,
                                  const int64_t* n_points, int32_t n_np, int32_t iters, const mem_integrate_opts& o,
                                  double* p_out, double* err_out, int32_t* status_out, const int32_t* ev_mask,
                                  Workspace& work, mem_flow seed_flow)
{
  const uint32_t first_kept = seed_flow ? 0u : 1u;
  const bool strat = o.stratify == MEM_STRATIFY_ADAPTIVE;
  mem_status st = MEM_OK;
  const int n_ev = ev->n_events;
  const bool target_mode = o.target_rel_err > 0.0;

  // ---- processes, integrals (event x permutation) and chunks ----
  std::vector<const mem_process_s*> procs;
  std::vector<int> ev_proc(n_ev);
  for (int e = 0; e < n_ev; ++e) {
    const mem_process p = hyp[n_hyp == 1 ? 0 : e];
    if (!p) return fail(MEM_EINVAL, "null process handle");
    if (ev->n_obj < n_obj_of(p->desc.kind)) return fail(MEM_EINVAL, "n_obj too small for the process kind");
    st = check_host_event(ev, e, n_obj_of(p->desc.kind));
    if (st != MEM_OK) return st;
    int pi = -1;
    for (size_t k = 0; k < procs.size(); ++k) if (procs[k] == p) pi = (int)k;
    if (pi < 0) { procs.push_back(p); pi = (int)procs.size() - 1; }
    ev_proc[e] = pi;
  }
  int n_f2 = 0;
  for (const auto* pr : procs) {
    mem_status ps = check_pdf_device(pr);
    if (ps != MEM_OK) return ps;
    n_f2 += is_f2(pr->desc.kind) ? 1 : 0;
  }
  if (n_f2 > 0 && n_f2 < (int)procs.size())
    return fail(MEM_EUNSUPPORTED, "t tbar H / t tbar b bbar dilepton integrate in a batch of their own");
  std::vector<ProcParams> ptab(procs.size());
  for (size_t k = 0; k < procs.size(); ++k) ptab[k] = procs[k]->pp;
  std::vector<IntegralDesc> ints;
  std::vector<int> int_proc;
  std::vector<int64_t> ev_int0(n_ev);
  std::vector<int32_t> ev_np(n_ev);
  std::vector<double> ev_norm(n_ev);
  int64_t grid_total = 0;
  for (int e = 0; e < n_ev; ++e) {
    const mem_process_s* p = procs[ev_proc[e]];
    const int64_t npts = n_points[n_np == 1 ? 0 : e];
    const int np = p->pp.n_perm;
    const int64_t per = (npts + np - 1) / np;
    if (per < 2) return fail(MEM_EINVAL, "n_points too small");
    if (per > (int64_t)0xFFFFFFFF) return fail(MEM_EINVAL, "n_points exceeds 2^32 per permutation");
    if (o.allocation == MEM_ALLOC_NEYMAN && per * std::min(np, 4) > (int64_t)0xFFFFFFFF)
      return fail(MEM_EINVAL, "n_points exceeds 2^32 per permutation under Neyman allocation");
    ev_int0[e] = (int64_t)ints.size();
    ev_np[e] = np;
    ev_norm[e] = p->desc.sigma_norm > 0.0 ? 1.0 / p->desc.sigma_norm : 1.0;
    for (int k = 0; k < np; ++k) {
      IntegralDesc d{};
      d.event = e; d.perm = k; d.dims = p->pp.dims; d.n_points = per;
      d.grid_off = grid_total;
      grid_total += (int64_t)p->pp.dims * (kBins + 1);
      ints.push_back(d);
      int_proc.push_back(ev_proc[e]);
    }
  }
  const int n_int = (int)ints.size();
  // Neyman allocation: an integral may take up to min(n_perm, 4) equal
  // shares in an iteration, so its chunks cover that many points
  const bool neyman = o.allocation == MEM_ALLOC_NEYMAN;
  std::vector<int64_t> cover(n_int);
  for (int ig = 0; ig < n_int; ++ig) {
    const int np = ev_np[ints[ig].event];
    cover[ig] = neyman ? ints[ig].n_points * std::min(np, 4) : ints[ig].n_points;
  }
  std::vector<Chunk> chunks;
  int64_t part_total = 0;
  for (int ig = 0; ig < n_int; ++ig) {
    IntegralDesc& d = ints[ig];
    // the call's chunk size, else the process's tuned one, else the default
    const int tuned = procs[int_proc[ig]]->chunk_points;
    int64_t chunk_pts = o.chunk_points > 0 ? o.chunk_points : tuned > 0 ? tuned : kDefaultChunk;
    // a stratified chunk's cumulative counts are staged in LDS
    if (strat) chunk_pts = std::min<int64_t>(chunk_pts, kStratChunkMax);
    d.chunk0 = (int64_t)chunks.size();
    d.n_chunks = 0;
    for (int64_t s0 = 0; s0 < cover[ig]; s0 += chunk_pts) {
      Chunk c{};
      c.integral = ig; c.event = d.event; c.perm = d.perm;
      c.count = (int32_t)std::min<int64_t>(chunk_pts, cover[ig] - s0);
      c.start = s0;
      c.part_off = part_total;
      c.proc = int_proc[ig];
      c.id = (int32_t)chunks.size();
      part_total += 2 + (int64_t)d.dims * kBins;
      chunks.push_back(c);
      d.n_chunks++;
    }
  }
  if ((int64_t)chunks.size() > (int64_t)0x7FFFFFFF) return fail(MEM_EINVAL, "too many chunks");
  // stratification: hypercubes per integral, offsets of their cumulative
  // counts and of the point weights
  std::vector<StratDesc> sdesc;
  int64_t cum_total = 0, w_total = 0;
  if (strat) {
    sdesc.resize(n_int);
    for (int ig = 0; ig < n_int; ++ig) {
      const int64_t N = ints[ig].n_points;
      if (N > (int64_t)0x7FFFFFFF) return fail(MEM_EINVAL, "stratified sampling takes below 2^31 points per permutation");
      const int D = ints[ig].dims;
      int ns = 1;
      for (;;) {
        int64_t h = 1;
        for (int d = 0; d < D; ++d) h *= ns + 1;
        if (2 * h > N || h > kStratHMax) break;
        ++ns;
      }
      int64_t H = 1;
      for (int d = 0; d < D; ++d) H *= ns;
      sdesc[ig] = StratDesc{ns, (int32_t)H, cum_total, w_total};
      cum_total += H + 1;
      w_total += N;
    }
  }
  QueueHooks hooks{nullptr, 0, -1, -1};
  if (o.weights_out) {
    if (o.weights_integral < 0 || o.weights_integral >= n_int) return fail(MEM_EINVAL, "weights_integral outside the integrals");
    if (o.weights_stride < cover[o.weights_integral]) return fail(MEM_EINVAL, "weights_stride below the integral's points");
    hooks.wout = o.weights_out;
    hooks.w_stride = o.weights_stride;
    hooks.w_int = o.weights_integral;
  }
  if (o.hooks & MEM_HOOK_NONFINITE) hooks.nan_event = o.hook_event;
  // checkpoint: what identifies this integration, and the state to resume from
  mem_checkpoint_s* ck = o.checkpoint;
  std::vector<uint64_t> ev_key(n_ev);
  std::vector<int64_t> int_key(4 * (size_t)n_int);
  if (ck) {
    for (int e = 0; e < n_ev; ++e) ev_key[e] = process_key(procs[ev_proc[e]]);
    for (int ig = 0; ig < n_int; ++ig) {
      int_key[4 * ig] = ints[ig].event; int_key[4 * ig + 1] = ints[ig].perm;
      int_key[4 * ig + 2] = ints[ig].dims; int_key[4 * ig + 3] = ints[ig].n_points;
    }
    if (ck->has) {
      if (ev_mask) return fail(MEM_EUNSUPPORTED, "checkpoints of masked integrations");
      if (ck->n_ev != n_ev || ck->n_int != n_int || ck->seed != o.seed || ck->alpha != o.alpha ||
          ck->allocation != o.allocation || ck->ev_key != ev_key || ck->int_key != int_key ||
          (int64_t)ck->grids.size() != grid_total)
        return fail(MEM_EINVAL, "the checkpoint holds a different integration");
    }
  }
  const bool resume = ck && ck->has;
  const uint32_t iter0 = resume ? ck->iter : 0u;
  // iterations this call runs: n_iter more, or up to max_iter in total
  const int run_iters = target_mode ? std::max<int>(0, iters - (int)iter0) : iters;
  // the queue kernel writes row `iteration index` of weights_out
  if (o.weights_out && (int64_t)iter0 + run_iters > (int64_t)o.weights_rows)
    return fail(MEM_EINVAL, "weights_rows below the iterations the call can reach");
  // tail chunking: a second chunk table (chunks of tail_chunk_points, their
  // own partial slots after the first table's) that the iterations from
  // tail_iter on use; built only when the call can reach tail_iter
  const size_t n_main = chunks.size();
  const bool tail = o.tail_chunk_points > 0 && (int64_t)iter0 + run_iters > (int64_t)o.tail_iter;
  std::vector<IntegralDesc> ints_tail;
  if (tail) {
    ints_tail = ints;
    for (int ig = 0; ig < n_int; ++ig) {
      IntegralDesc& d = ints_tail[ig];
      d.chunk0 = (int64_t)chunks.size();
      d.n_chunks = 0;
      for (int64_t s0 = 0; s0 < cover[ig]; s0 += o.tail_chunk_points) {
        Chunk c{};
        c.integral = ig; c.event = d.event; c.perm = d.perm;
        c.count = (int32_t)std::min<int64_t>(o.tail_chunk_points, cover[ig] - s0);
        c.start = s0;
        c.part_off = part_total;
        c.proc = int_proc[ig];
        c.id = (int32_t)chunks.size();
        part_total += 2 + (int64_t)d.dims * kBins;
        chunks.push_back(c);
        d.n_chunks++;
      }
    }
    if ((int64_t)chunks.size() > (int64_t)0x7FFFFFFF) return fail(MEM_EINVAL, "too many chunks");
  }
  // launch groups by matrix-element precision; queue order longest first
  std::vector<Group> groups;
  auto group_of = [&](int prec) {
    for (size_t g = 0; g < groups.size(); ++g) if (groups[g].prec == prec) return (int)g;
    groups.push_back(Group{prec, {}, 0, 0, nullptr});
    return (int)groups.size() - 1;
  };
  int first_prec = -1;
  for (const auto* p : procs) if (p->desc.kind != MEM_DY_QQ_GAMMA_MUMU) { first_prec = p->desc.precision; break; }
  if (first_prec < 0) first_prec = MEM_FP64;
  std::vector<double> cost(chunks.size());
  std::vector<int> int_group(n_int, 0);
  for (size_t c = 0; c < chunks.size(); ++c)
    cost[c] = chunks[c].count * eval_cost(procs[chunks[c].proc]->desc.kind);
  for (size_t c = 0; c < n_main; ++c) {
    const mem_process_s* p = procs[chunks[c].proc];
    int prec = p->desc.kind == MEM_DY_QQ_GAMMA_MUMU ? first_prec : p->desc.precision;
    const int gi = group_of(prec);
    int_group[chunks[c].integral] = gi;
    Group& G = groups[gi];
    G.queue.push_back((int32_t)c);
    G.mask |= kind_mask(p->desc.kind);
    G.waves = G.waves < 0 ? p->waves : G.waves == p->waves ? G.waves : 0;
  }
  for (auto& G : groups)
    std::stable_sort(G.queue.begin(), G.queue.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });

  // ---- stream: the caller's, or a private one (graphs cannot capture the null stream) ----
  hipStream_t s = (hipStream_t)o.stream;
  hipStream_t own = nullptr;
  const bool want_graph = o.use_graph != 0 && o.timing_out == nullptr;
  if (!s && want_graph) HIP_TRY(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
  struct StreamGuard { hipStream_t& s; ~StreamGuard() { if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); } } } sg{own};
  hipStream_t ws = own ? own : s;

  DevEvents dev(&work);
  st = dev.make(ev, ws);
  if (st != MEM_OK) return st;
  DevBuf b_procs(&work), b_ints(&work), b_chunks(&work), b_queue(&work), b_grids(&work), b_parts(&work),
      b_state(&work), b_active(&work), b_evi0(&work), b_evnp(&work), b_evnorm(&work), b_done(&work), b_ctl(&work),
      b_heads(&work), b_P(&work), b_err(&work), b_status(&work), b_alloc(&work), b_cover(&work), b_nev(&work),
      b_sd(&work), b_cum(&work), b_sigb(&work), b_h0(&work), b_wpt(&work), b_siv(&work), b_finlist(&work);
  size_t qtotal = 0;
  for (auto& G : groups) qtotal += G.queue.size();
  // every work buffer is taken before the first copy or launch; the chunk
  // table in queue order (the queue kernel reads it instead of gathering
  // through the queue) included
  DevBuf b_chunks_q(&work);
  {
    hipError_t ae = hipSuccess;
    auto A = [&](DevBuf& b, size_t bytes) {
      hipError_t e = b.alloc(bytes);
      if (ae == hipSuccess) ae = e;
    };
    A(b_procs, ptab.size() * sizeof(ProcParams));
    A(b_ints, ints.size() * sizeof(IntegralDesc));
    A(b_chunks, chunks.size() * sizeof(Chunk));
    A(b_queue, qtotal * sizeof(int32_t));
    A(b_grids, grid_total * sizeof(double));
    A(b_parts, part_total * sizeof(double));
    A(b_state, (size_t)n_int * ST_SIZE * sizeof(double));
    A(b_active, (size_t)n_int * sizeof(int32_t));
    A(b_evi0, (size_t)n_ev * sizeof(int64_t));
    A(b_evnp, (size_t)n_ev * sizeof(int32_t));
    A(b_evnorm, (size_t)n_ev * sizeof(double));
    A(b_done, (size_t)n_ev * sizeof(int32_t));
    A(b_ctl, sizeof(Control));
    A(b_heads, groups.size() * sizeof(uint32_t));
    A(b_nev, sizeof(double));
    A(b_chunks_q, std::max(qtotal, chunks.size() - n_main) * sizeof(Chunk));
    A(b_finlist, (size_t)n_int * sizeof(int32_t));
    if (neyman) {
      A(b_alloc, (size_t)n_int * sizeof(int64_t));
      A(b_cover, (size_t)n_int * sizeof(int64_t));
    }
    if (strat) {
      A(b_sd, (size_t)n_int * sizeof(StratDesc));
      A(b_cum, (size_t)cum_total * sizeof(int32_t));
      A(b_sigb, (size_t)cum_total * sizeof(double));
      A(b_h0, chunks.size() * sizeof(int32_t));
      A(b_wpt, (size_t)w_total * sizeof(double));
      A(b_siv, (size_t)n_int * 2 * sizeof(double));
    }
    if (o.outputs_on_device == 0) {
      A(b_P, n_ev * sizeof(double));
      A(b_err, n_ev * sizeof(double));
      A(b_status, n_ev * sizeof(int32_t));
    }
    if (ae != hipSuccess && work.arena())
      return fail(MEM_ENOMEM, "the work buffers of this call take " + std::to_string(work.requested()) +
                                  " bytes, more than the " + std::to_string(work.capacity()) +
                                  "-byte scratch of the no-allocation entry point: integrate fewer events, "
                                  "assignments or points per call");
    HIP_TRY(ae);
  }
  const bool out_dev = o.outputs_on_device != 0;
  std::vector<int32_t> flat;
  std::vector<size_t> gq0;
  for (auto& G : groups) { gq0.push_back(flat.size()); flat.insert(flat.end(), G.queue.begin(), G.queue.end()); }
  HIP_TRY(hipMemcpyAsync(b_procs.p, ptab.data(), ptab.size() * sizeof(ProcParams), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_ints.p, ints.data(), ints.size() * sizeof(IntegralDesc), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_chunks.p, chunks.data(), chunks.size() * sizeof(Chunk), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_queue.p, flat.data(), flat.size() * sizeof(int32_t), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_evi0.p, ev_int0.data(), n_ev * sizeof(int64_t), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_evnp.p, ev_np.data(), n_ev * sizeof(int32_t), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_evnorm.p, ev_norm.data(), n_ev * sizeof(double), hipMemcpyHostToDevice, ws));
  std::vector<int64_t> alloc0;
  if (neyman) {
    // the first iteration splits equally
    alloc0.resize(n_int);
    for (int ig = 0; ig < n_int; ++ig) alloc0[ig] = ints[ig].n_points;
    HIP_TRY(hipMemcpyAsync(b_alloc.p, alloc0.data(), n_int * sizeof(int64_t), hipMemcpyHostToDevice, ws));
    HIP_TRY(hipMemcpyAsync(b_cover.p, cover.data(), n_int * sizeof(int64_t), hipMemcpyHostToDevice, ws));
  }
  const Control ctl0{0u, 0u, 0, 0u};
  HIP_TRY(hipMemcpyAsync(b_ctl.p, &ctl0, sizeof(Control), hipMemcpyHostToDevice, ws));
  {
    const int64_t ns = (int64_t)n_int * ST_SIZE;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, ws, b_state.as<double>(), ns, 0.0);
    // chunk partials start at zero (the buffer may hold an earlier call's)
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((part_total + 255) / 256)), dim3(256), 0, ws,
                       b_parts.as<double>(), part_total, 0.0);
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n_int + 255) / 256)), dim3(256), 0, ws,
                       b_active.as<int32_t>(), (int64_t)n_int, 1);
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n_ev + 255) / 256)), dim3(256), 0, ws,
                       b_done.as<int32_t>(), (int64_t)n_ev, 0);
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, ws, b_nev.as<double>(), (int64_t)1, 0.0);
    hipLaunchKernelGGL(init_grids_kernel, dim3(n_int), dim3(kBlock), 0, ws, b_grids.as<double>(),
                       b_ints.as<IntegralDesc>(), n_int);
    HIP_TRY(hipGetLastError());
  }
  StratView sview{nullptr, nullptr, nullptr, nullptr};
  if (strat) {
    HIP_TRY(hipMemcpyAsync(b_sd.p, sdesc.data(), n_int * sizeof(StratDesc), hipMemcpyHostToDevice, ws));
    sview = StratView{b_sd.as<StratDesc>(), b_cum.as<int32_t>(), b_h0.as<int32_t>(), b_wpt.as<double>()};
    hipLaunchKernelGGL(strat_init_kernel, dim3(n_int), dim3(kBlock), 0, ws, b_ints.as<IntegralDesc>(), sview,
                       b_cum.as<int32_t>(), b_chunks.as<Chunk>(), b_h0.as<int32_t>());
    HIP_TRY(hipGetLastError());
  }
  if (seed_flow) {
    st = seed_grids_from_flow(seed_flow, dev.view, ints, b_ints.as<IntegralDesc>(), b_grids.as<double>(), o.seed,
                              work, ws);
    if (st != MEM_OK) return st;
  }
  if (resume) {
    // the state of the earlier call; the host vectors live in the handle
    const Control ctlr{iter0, 0u, 0, 0u};
    HIP_TRY(hipMemcpyAsync(b_ctl.p, &ctlr, sizeof(Control), hipMemcpyHostToDevice, ws));
    HIP_TRY(hipMemcpyAsync(b_grids.p, ck->grids.data(), grid_total * sizeof(double), hipMemcpyHostToDevice, ws));
    HIP_TRY(hipMemcpyAsync(b_state.p, ck->state.data(), ck->state.size() * sizeof(double), hipMemcpyHostToDevice, ws));
    HIP_TRY(hipMemcpyAsync(b_active.p, ck->active.data(), n_int * sizeof(int32_t), hipMemcpyHostToDevice, ws));
    HIP_TRY(hipMemcpyAsync(b_done.p, ck->done.data(), n_ev * sizeof(int32_t), hipMemcpyHostToDevice, ws));
    if (neyman && (int64_t)ck->alloc.size() == n_int)
      HIP_TRY(hipMemcpyAsync(b_alloc.p, ck->alloc.data(), n_int * sizeof(int64_t), hipMemcpyHostToDevice, ws));
    HIP_TRY(hipStreamSynchronize(ws));
  }
  if (ev_mask) {
    // skipped events: integrals inactive and the event retired from the start
    std::vector<int32_t> act(n_int), dn(n_ev);
    for (int ig = 0; ig < n_int; ++ig) act[ig] = ev_mask[ints[ig].event] ? 1 : 0;
    for (int e = 0; e < n_ev; ++e) dn[e] = ev_mask[e] ? 0 : 1;
    HIP_TRY(hipMemcpyAsync(b_active.p, act.data(), n_int * sizeof(int32_t), hipMemcpyHostToDevice, ws));
    HIP_TRY(hipMemcpyAsync(b_done.p, dn.data(), n_ev * sizeof(int32_t), hipMemcpyHostToDevice, ws));
    HIP_TRY(hipStreamSynchronize(ws));
  }
  for (auto& G : groups) {
    const int wv = G.waves > 0 ? G.waves : 0;
    G.kernel = G.prec == MEM_FP32 ? queue_kernel_for<float>(G.mask, wv) : queue_kernel_for<double>(G.mask, wv);
    G.blocks = persistent_blocks(G.kernel, (int64_t)G.queue.size());
  }
  // chunk order through the queue: the kernel reads chunks[queue[c]]; the
  // queue kernel takes the chunk table permuted on the device instead
  // (one gather per call)
  std::vector<size_t> gqn(groups.size());     // queue length per group
  {
    std::vector<Chunk> perm_chunks(flat.size());
    for (size_t i = 0; i < flat.size(); ++i) perm_chunks[i] = chunks[flat[i]];
    HIP_TRY(hipMemcpyAsync(b_chunks_q.p, perm_chunks.data(), flat.size() * sizeof(Chunk), hipMemcpyHostToDevice, ws));
    HIP_TRY(hipStreamSynchronize(ws));   // perm_chunks goes out of scope
    for (size_t g = 0; g < groups.size(); ++g) gqn[g] = groups[g].queue.size();
  }

  const int ev_blocks = (n_ev + 255) / 256;
  Control* ctl = b_ctl.as<Control>();
  // the integrals the finish step visits: every one, until a queue rebuild
  // lists the running events' integrals
  int n_fin = n_int;
  bool fin_list = false;
  auto list_running = [&](const std::vector<int32_t>& dn) -> mem_status {
    std::vector<int32_t> l;
    for (int e = 0; e < n_ev; ++e)
      if (!dn[e])
        for (int k = 0; k < ev_np[e]; ++k) l.push_back((int32_t)(ev_int0[e] + k));
    if (l.empty()) return MEM_OK;     // nothing runs: the full grid, every workgroup returns at once
    HIP_TRY(hipMemcpy(b_finlist.p, l.data(), l.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    n_fin = (int)l.size();
    fin_list = true;
    return MEM_OK;
  };
  // one iteration: begin -> queue kernel(s) -> finish -> [events] -> end
  auto enqueue_iteration = [&](bool time_kernels, std::vector<hipEvent_t>* tev) -> mem_status {
    hipLaunchKernelGGL(iter_begin_kernel, dim3(1), dim3(64), 0, ws, ctl, b_heads.as<uint32_t>(), (int)groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
      const Group& G = groups[g];
      const Chunk* cq = b_chunks_q.as<Chunk>() + gq0[g];
      if (time_kernels) {
        hipEvent_t a, b;
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        tev->push_back(a);
        tev->push_back(b);
        HIP_TRY(hipEventRecord(a, ws));
      }
      hipLaunchKernelGGL(G.kernel, dim3(G.blocks), dim3(kBlock), 0, ws, b_procs.as<ProcParams>(), dev.view, cq,
                         (int64_t)gqn[g], b_ints.as<IntegralDesc>(), b_grids.as<double>(),
                         b_active.as<int32_t>(), o.seed, ctl, b_heads.as<uint32_t>() + g, b_parts.as<double>(),
                         neyman ? b_alloc.as<int64_t>() : nullptr, hooks, sview);
      HIP_TRY(hipGetLastError());
      if (time_kernels) HIP_TRY(hipEventRecord(tev->back(), ws));
    }
    if (strat)
      hipLaunchKernelGGL(strat_finish_kernel, dim3(n_int), dim3(kBlock), 0, ws, b_ints.as<IntegralDesc>(), sview,
                         b_cum.as<int32_t>(), b_sigb.as<double>(), b_active.as<int32_t>(), b_chunks.as<Chunk>(),
                         b_h0.as<int32_t>(), b_siv.as<double>());
    hipLaunchKernelGGL(finish_iter_kernel, dim3(n_fin), dim3(kBlock), 0, ws, fin_list ? b_finlist.as<int32_t>() : nullptr,
                       b_ints.as<IntegralDesc>(),
                       b_chunks.as<Chunk>(), b_parts.as<double>(), b_grids.as<double>(), b_state.as<double>(),
                       b_active.as<int32_t>(), o.alpha, ctl, n_int, o.iter_out,
                       neyman ? b_alloc.as<int64_t>() : nullptr, b_nev.as<double>(), first_kept,
                       strat ? b_siv.as<double>() : nullptr);
    if (target_mode)
      hipLaunchKernelGGL(event_kernel, dim3(ev_blocks), dim3(256), 0, ws, b_evi0.as<int64_t>(), b_evnp.as<int32_t>(),
                         b_evnorm.as<double>(), b_state.as<double>(), b_active.as<int32_t>(), n_ev,
                         o.target_rel_err, ctl, 0, nullptr, nullptr, nullptr, nullptr, b_done.as<int32_t>(),
                         first_kept, o.combine);
    if (neyman)
      hipLaunchKernelGGL(neyman_kernel, dim3(ev_blocks), dim3(256), 0, ws, b_evi0.as<int64_t>(), b_evnp.as<int32_t>(),
                         b_ints.as<IntegralDesc>(), b_state.as<double>(), b_active.as<int32_t>(),
                         b_cover.as<int64_t>(), b_alloc.as<int64_t>(), n_ev);
    hipLaunchKernelGGL(iter_end_kernel, dim3(1), dim3(64), 0, ws, ctl);
    HIP_TRY(hipGetLastError());
    return MEM_OK;
  };

  std::vector<hipEvent_t> tev;
  struct EventsGuard { std::vector<hipEvent_t>& v; ~EventsGuard() { for (auto e : v) (void)hipEventDestroy(e); } } eg{tev};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct GraphGuard {
    hipGraph_t& g; hipGraphExec_t& x;
    ~GraphGuard() { if (x) (void)hipGraphExecDestroy(x); if (g) (void)hipGraphDestroy(g); }
  } gg{graph, gexec};
  const bool use_graph = want_graph && ws != nullptr;
  auto capture = [&]() -> mem_status {
    if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
    if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
    HIP_TRY(hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal));
    mem_status cs = enqueue_iteration(false, nullptr);
    hipGraph_t gcap = nullptr;
    hipError_t ce = hipStreamEndCapture(ws, &gcap);
    graph = gcap;
    if (cs != MEM_OK) return cs;
    if (ce != hipSuccess) return fail(MEM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    HIP_TRY(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    return MEM_OK;
  };
  if (use_graph) {
    mem_status cs = capture();
    if (cs != MEM_OK) return cs;
  }
  // Target mode: once the running events have halved since the queue was
  // last built, the queue is rebuilt from the running events' chunks only
  // (same order), so that late iterations do not pop the retired events'
  // chunks one by one.  Partial sums live in per-chunk slots and are summed
  // per integral in chunk order, so the results do not change.
  std::vector<int32_t> qhost(flat.begin(), flat.end());
  int64_t running_at_build = n_ev;
  if (target_mode && resume && run_iters > 0) {
    // events retired before the checkpoint leave the queue at once
    int64_t running = 0;
    for (int e = 0; e < n_ev; ++e) running += ck->done[e] == 0 ? 1 : 0;
    if (running == 0) running_at_build = 0;
  }
  auto compact = [&]() -> mem_status {
    std::vector<int32_t> dn(n_ev);
    HIP_TRY(hipMemcpy(dn.data(), b_done.p, n_ev * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> nq;
    std::vector<size_t> ng(groups.size());
    size_t pos = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
      const size_t start = nq.size();
      for (size_t i = 0; i < gqn[g]; ++i) {
        const int32_t c = qhost[pos + i];
        if (!dn[chunks[c].event]) nq.push_back(c);
      }
      pos += gqn[g];
      ng[g] = nq.size() - start;
    }
    std::vector<Chunk> pc(nq.size());
    for (size_t i = 0; i < nq.size(); ++i) pc[i] = chunks[nq[i]];
    if (!pc.empty())
      HIP_TRY(hipMemcpy(b_chunks_q.p, pc.data(), pc.size() * sizeof(Chunk), hipMemcpyHostToDevice));
    size_t off = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
      gq0[g] = off;
      gqn[g] = ng[g];
      off += ng[g];
      groups[g].blocks = persistent_blocks(groups[g].kernel, (int64_t)ng[g]);
    }
    qhost.swap(nq);
    mem_status ls = list_running(dn);
    if (ls != MEM_OK) return ls;
    return use_graph ? capture() : MEM_OK;
  };
  // tail chunking: before iteration tail_iter the running integrals move to
  // the tail table (their chunk table entries and partial slots), the queue
  // is rebuilt from it and the iteration graph recaptured
  bool tail_pending = tail;
  auto switch_to_tail = [&]() -> mem_status {
    HIP_TRY(hipStreamSynchronize(ws));
    std::vector<int32_t> dn(n_ev);
    HIP_TRY(hipMemcpy(dn.data(), b_done.p, n_ev * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(b_ints.p, ints_tail.data(), n_int * sizeof(IntegralDesc), hipMemcpyHostToDevice));
    std::vector<std::vector<int32_t>> q(groups.size());
    for (size_t c = n_main; c < chunks.size(); ++c)
      if (!dn[chunks[c].event]) q[int_group[chunks[c].integral]].push_back((int32_t)c);
    std::vector<int32_t> nq;
    int64_t running = 0;
    for (int e = 0; e < n_ev; ++e) running += dn[e] == 0 ? 1 : 0;
    for (size_t g = 0; g < groups.size(); ++g) {
      std::stable_sort(q[g].begin(), q[g].end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
      gq0[g] = nq.size();
      gqn[g] = q[g].size();
      nq.insert(nq.end(), q[g].begin(), q[g].end());
      groups[g].blocks = persistent_blocks(groups[g].kernel, (int64_t)q[g].size());
    }
    std::vector<Chunk> pc(nq.size());
    for (size_t i = 0; i < nq.size(); ++i) pc[i] = chunks[nq[i]];
    if (!pc.empty())
      HIP_TRY(hipMemcpy(b_chunks_q.p, pc.data(), pc.size() * sizeof(Chunk), hipMemcpyHostToDevice));
    qhost.swap(nq);
    if (target_mode) running_at_build = running;
    mem_status ls = list_running(dn);
    if (ls != MEM_OK) return ls;
    return use_graph ? capture() : MEM_OK;
  };
  auto wall0 = std::chrono::steady_clock::now();
  for (int j = 0; j < run_iters && running_at_build > 0; ++j) {
    if (tail_pending && (int64_t)iter0 + j >= (int64_t)o.tail_iter) {
      tail_pending = false;
      mem_status ts = switch_to_tail();
      if (ts != MEM_OK) return ts;
      if (running_at_build == 0) break;     // target mode: every event retired
    }
    if (use_graph) HIP_TRY(hipGraphLaunch(gexec, ws));
    else {
      mem_status es = enqueue_iteration(o.timing_out != nullptr, &tev);
      if (es != MEM_OK) return es;
    }
    if (j == 0) {
      // a launch that failed on the device surfaces here, before the
      // remaining iterations run on its results
      HIP_TRY(hipStreamSynchronize(ws));
      HIP_TRY(hipGetLastError());
    }
    if (target_mode) {
      Control hc{};
      HIP_TRY(hipMemcpyAsync(&hc, ctl, sizeof(Control), hipMemcpyDeviceToHost, ws));
      HIP_TRY(hipStreamSynchronize(ws));
      if (hc.n_running == 0) break;
      if (2 * (int64_t)hc.n_running <= running_at_build && n_ev >= 64) {
        running_at_build = hc.n_running;
        mem_status cs = compact();
        if (cs != MEM_OK) return cs;
      }
    }
  }
  double* P = out_dev ? p_out : b_P.as<double>();
  double* E = out_dev ? err_out : b_err.as<double>();
  int32_t* S = out_dev ? status_out : b_status.as<int32_t>();
  // the final pass reads ctl->iter == iterations run
  hipLaunchKernelGGL(event_kernel, dim3(ev_blocks), dim3(256), 0, ws, b_evi0.as<int64_t>(), b_evnp.as<int32_t>(),
                     b_evnorm.as<double>(), b_state.as<double>(), b_active.as<int32_t>(), n_ev,
                     target_mode ? o.target_rel_err : 0.0, ctl, 1, P, E, S, o.n_iter_out, b_done.as<int32_t>(),
                     first_kept, o.combine);
  HIP_TRY(hipGetLastError());
  if (o.grid_out)
    HIP_TRY(hipMemcpyAsync(o.grid_out, b_grids.p, grid_total * sizeof(double), hipMemcpyDeviceToDevice, ws));
  if (!out_dev) {
    HIP_TRY(hipMemcpyAsync(p_out, P, n_ev * sizeof(double), hipMemcpyDeviceToHost, ws));
    HIP_TRY(hipMemcpyAsync(err_out, E, n_ev * sizeof(double), hipMemcpyDeviceToHost, ws));
    HIP_TRY(hipMemcpyAsync(status_out, S, n_ev * sizeof(int32_t), hipMemcpyDeviceToHost, ws));
  }
  // the work buffers are freed on return: wait for the stream
  HIP_TRY(hipStreamSynchronize(ws));
  if (ck) {
    // the final state into the handle
    Control hc{};
    std::vector<double> grids(grid_total), state((size_t)n_int * ST_SIZE);
    std::vector<int32_t> act(n_int), dn(n_ev);
    std::vector<int64_t> al(neyman ? n_int : 0);
    HIP_TRY(hipMemcpy(&hc, ctl, sizeof(Control), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(grids.data(), b_grids.p, grid_total * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(state.data(), b_state.p, state.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(act.data(), b_active.p, n_int * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dn.data(), b_done.p, n_ev * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (neyman) HIP_TRY(hipMemcpy(al.data(), b_alloc.p, n_int * sizeof(int64_t), hipMemcpyDeviceToHost));
    ck->n_ev = n_ev; ck->n_int = n_int; ck->allocation = o.allocation; ck->seed = o.seed; ck->alpha = o.alpha;
    ck->ev_key.swap(ev_key); ck->int_key.swap(int_key);
    ck->iter = hc.iter;
    ck->grids.swap(grids); ck->state.swap(state); ck->active.swap(act); ck->done.swap(dn); ck->alloc.swap(al);
    ck->has = true;
  }
  if (o.timing_out) {
    double ms = 0.0;
    for (size_t i = 0; i + 1 < tev.size(); i += 2) {
      float t = 0.0f;
      HIP_TRY(hipEventElapsedTime(&t, tev[i], tev[i + 1]));
      ms += t;
    }
    // evaluations, counted on the device: every active integral's points
    // of every iteration (converged events stop; events outside the mask
    // run none)
    double n_evals = 0.0;
    HIP_TRY(hipMemcpy(&n_evals, b_nev.p, sizeof(double), hipMemcpyDeviceToHost));
    o.timing_out[0] = ms;
    o.timing_out[1] = (double)(tev.size() / 2);
    o.timing_out[2] = n_evals;
    o.timing_out[3] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
    for (int i = 4; i < 8; ++i) o.timing_out[i] = 0.0;
  }
  return MEM_OK;
}

// ------------------------------------------------------ building blocks ----
extern "C" mem_status mem_uniforms(uint64_t seed, uint32_t iter, uint32_t event, uint32_t perm, int32_t D,
                                   int64_t n, double* u, void* stream)
{
  if (!u || D <= 0 || D > kMaxDims || n < 0) return fail(MEM_EINVAL, "bad arguments");
  if (n > (int64_t)0xFFFFFFFF) return fail(MEM_EINVAL, "n exceeds 2^32");
  if (n == 0) return MEM_OK;
  hipLaunchKernelGGL(uniforms_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, seed,
                     iter, event, perm, D, n, u);
  HIP_TRY(hipGetLastError());
  return MEM_OK;
}

extern "C" mem_status mem_eval_points(mem_process p, const mem_events* ev, int32_t event, int32_t perm,
                                      const double* x, int64_t n, double* f, int32_t* nsol, void* stream)
{
  if (!p || !x || !f) return fail(MEM_EINVAL, "null argument");
  mem_status st = check_pdf_device(p);
  if (st != MEM_OK) return st;
  st = check_event_arrays(ev);
  if (st != MEM_OK) return st;
  if (event < 0 || event >= ev->n_events) return fail(MEM_EINVAL, "event index out of range");
  if (perm < 0 || perm >= p->pp.n_perm) return fail(MEM_EINVAL, "permutation out of range");
  if (ev->n_obj < n_obj_of(p->desc.kind)) return fail(MEM_EINVAL, "n_obj too small for the process kind");
  st = check_host_event(ev, event, n_obj_of(p->desc.kind));
  if (st != MEM_OK) return st;
  if (n < 0) return fail(MEM_EINVAL, "negative n");
  if (n == 0) return MEM_OK;
  hipStream_t s = (hipStream_t)stream;
  DevEvents dev;
  st = dev.make(ev, s);
  if (st != MEM_OK) return st;
  dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
  if (p->desc.kind == MEM_DY_QQ_GAMMA_MUMU)
    hipLaunchKernelGGL((eval_points_kernel<kDY, 2, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event, perm,
                       x, n, f, nsol);
  else if (p->desc.kind == MEM_TTH_DILEPTON && p->desc.precision == MEM_FP32)
    hipLaunchKernelGGL((eval_points_kernel<kTHL, 8, float>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                       perm, x, n, f, nsol);
  else if (p->desc.kind == MEM_TTH_DILEPTON)
    hipLaunchKernelGGL((eval_points_kernel<kTHL, 8, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                       perm, x, n, f, nsol);
  else if (p->desc.kind == MEM_TTBB_DILEPTON && p->desc.precision == MEM_FP32)
    hipLaunchKernelGGL((eval_points_kernel<kTBB, 8, float>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                       perm, x, n, f, nsol);
  else if (p->desc.kind == MEM_TTBB_DILEPTON)
    hipLaunchKernelGGL((eval_points_kernel<kTBB, 8, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                       perm, x, n, f, nsol);
  else if (p->desc.kind == MEM_TTH_SEMILEPTON && p->desc.precision == MEM_FP32)
    hipLaunchKernelGGL((eval_points_kernel<kTTH, 9, float>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                       perm, x, n, f, nsol);
  else if (p->desc.kind == MEM_TTH_SEMILEPTON)
    hipLaunchKernelGGL((eval_points_kernel<kTTH, 9, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                       perm, x, n, f, nsol);
  else if (p->desc.kind == MEM_TT_SEMILEPTON && p->desc.precision == MEM_FP32)
    hipLaunchKernelGGL((eval_points_kernel<kSL, 7, float>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event, perm,
                       x, n, f, nsol);
  else if (p->desc.kind == MEM_TT_SEMILEPTON)
    hipLaunchKernelGGL((eval_points_kernel<kSL, 7, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                       perm, x, n, f, nsol);
  else if (p->desc.precision == MEM_FP32)
    hipLaunchKernelGGL((eval_points_kernel<kTT, 8, float>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event, perm,
                       x, n, f, nsol);
  else
    hipLaunchKernelGGL((eval_points_kernel<kTT, 8, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                       perm, x, n, f, nsol);
  HIP_TRY(hipGetLastError());
  if (!ev->on_device) HIP_TRY(hipStreamSynchronize(s));   // the staged copy is freed on return
  return MEM_OK;
}

// Event discriminant of Sec. 4: D = log10(p_signal / p_background).
__global__ void discriminant_kernel(const double* __restrict__ ps, const double* __restrict__ pb, int64_t n,
                                    double* __restrict__ d)
{
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double s = ps[k], b = pb[k];
  double v;
  if (s > 0.0 && b > 0.0) v = log10(s) - log10(b);
  else if (s > 0.0 && b == 0.0) v = HUGE_VAL;
  else if (s == 0.0 && b > 0.0) v = -HUGE_VAL;
  else v = __builtin_nan("");
  d[k] = v;
}

extern "C" mem_status mem_discriminant(const double* p_sig, const double* p_bkg, int64_t n, double* d_out,
                                       void* stream)
{
  if (n < 0) return fail(MEM_EINVAL, "negative n");
  if (n == 0) return MEM_OK;
  if (!p_sig || !p_bkg || !d_out) return fail(MEM_EINVAL, "null argument");
  if (n > ((int64_t)1 << 40)) return fail(MEM_EINVAL, "n too large");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(discriminant_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p_sig,
                     p_bkg, n, d_out);
  HIP_TRY(hipGetLastError());
  return MEM_OK;
}

// Parton-level weights: one thread per event, the two b assignments in
// order (objects b, bbar, l+, l-, nu, nubar; assignment 1 swaps the b's).
template <class T>
__global__ __launch_bounds__(kBlock, MEM_TT_WAVES) void parton_kernel(ProcParams pp, EventsView ev,
                                                                      double* __restrict__ w)
{
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= ev.n_events) return;
  v4 o[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) ev.load(k, e, o[k].e, o[k].x, o[k].y, o[k].z);
  const double w0 = tt_parton<T>(pp, o[0], o[2], o[4], o[1], o[3], o[5]);
  const double w1 = tt_parton<T>(pp, o[1], o[2], o[4], o[0], o[3], o[5]);
  w[e] = 0.5 * (w0 + w1);
}

// Parton-level weights of the four-b dilepton kinds: one thread per event,
// the 12 or 24 assignments in order (objects: b quarks 0-3, l+, l-, nu,
// nubar).
template <class T, bool TTH>
__global__ __launch_bounds__(kBlock, 1) void f2_parton_kernel(ProcParams pp, EventsView ev, double* __restrict__ w)
{
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= ev.n_events) return;
  v4 o[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) ev.load(k, e, o[k].e, o[k].x, o[k].y, o[k].z);
  w[e] = f2_parton<T, TTH>(pp, o);
}

extern "C" mem_status mem_parton_weights(mem_process p, const mem_events* ev, double* w_out, void* stream)
{
  if (!p) return fail(MEM_EINVAL, "null argument");
  mem_status st = check_pdf_device(p);
  if (st != MEM_OK) return st;
  st = check_event_arrays(ev);
  if (st != MEM_OK) return st;
  if (!w_out && ev->n_events > 0) return fail(MEM_EINVAL, "null argument");
  const bool four_b = is_f2(p->desc.kind);
  if (p->desc.kind != MEM_TT_DILEPTON && !four_b)
    return fail(MEM_EUNSUPPORTED, "parton-level weights: ttbar dilepton and the four-b dilepton kinds");
  const int n_obj = four_b ? 8 : 6;
  if (ev->n_obj < n_obj) return fail(MEM_EINVAL, "parton-level events need 6 objects (8 for the four-b kinds)");
  for (int e = 0; e < ev->n_events; ++e) {
    st = check_host_event(ev, e, n_obj);
    if (st != MEM_OK) return st;
  }
  if (ev->n_events == 0) return MEM_OK;
  hipStream_t s = (hipStream_t)stream;
  DevEvents dev;
  st = dev.make(ev, s);
  if (st != MEM_OK) return st;
  DevBuf wbuf;
  double* w = w_out;
  if (!ev->on_device) {
    HIP_TRY(wbuf.alloc((size_t)ev->n_events * sizeof(double)));
    w = wbuf.as<double>();
  }
  dim3 grid((unsigned)((ev->n_events + kBlock - 1) / kBlock));
  const bool f32 = p->desc.precision == MEM_FP32;
  if (p->desc.kind == MEM_TTH_DILEPTON && f32)
    hipLaunchKernelGGL((f2_parton_kernel<float, true>), grid, dim3(kBlock), 0, s, p->pp, dev.view, w);
  else if (p->desc.kind == MEM_TTH_DILEPTON)
    hipLaunchKernelGGL((f2_parton_kernel<double, true>), grid, dim3(kBlock), 0, s, p->pp, dev.view, w);
  else if (p->desc.kind == MEM_TTBB_DILEPTON && f32)
    hipLaunchKernelGGL((f2_parton_kernel<float, false>), grid, dim3(kBlock), 0, s, p->pp, dev.view, w);
  else if (p->desc.kind == MEM_TTBB_DILEPTON)
    hipLaunchKernelGGL((f2_parton_kernel<double, false>), grid, dim3(kBlock), 0, s, p->pp, dev.view, w);
  else if (f32)
    hipLaunchKernelGGL(parton_kernel<float>, grid, dim3(kBlock), 0, s, p->pp, dev.view, w);
  else
    hipLaunchKernelGGL(parton_kernel<double>, grid, dim3(kBlock), 0, s, p->pp, dev.view, w);
  HIP_TRY(hipGetLastError());
  if (!ev->on_device) {
    HIP_TRY(hipMemcpyAsync(w_out, w, (size_t)ev->n_events * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return MEM_OK;
}

extern "C" mem_status mem_vegas_refine(const double* bins, double* grids, int32_t n_int, int32_t D, double alpha,
                                       void* stream)
{
  if (!bins || !grids || n_int < 0 || D <= 0 || D > kMaxDims || !(alpha > 0.0))
    return fail(MEM_EINVAL, "bad arguments");
  if (n_int == 0) return MEM_OK;
  hipLaunchKernelGGL(refine_only_kernel, dim3(n_int), dim3(kBlock), 0, (hipStream_t)stream, bins, grids, D, alpha);
  HIP_TRY(hipGetLastError());
  return MEM_OK;
}

// -------------------------------------------------------------- autotuner ----
namespace {
std::string device_arch()
{
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string tuning_key(const std::string& arch, const mem_process_s* p)
{
  return arch + " " + std::to_string(p->desc.kind) + " " + std::to_string(p->desc.precision);
}

bool valid_chunk(int64_t c) { return c > 0 && c % kBlock == 0 && c <= 65536; }
}  // namespace

extern "C" mem_status mem_autotune(mem_process p, const mem_events* ev, int64_t n_points, int32_t n_iter,
                                   const mem_integrate_opts* base, const int32_t* candidates, int32_t n_cand,
                                   const int32_t* waves, int32_t n_waves, const char* table_path, int32_t* best_out,
                                   int32_t* best_waves_out, double* rate_out)
{
  if (!p) return fail(MEM_EINVAL, "null process");
  mem_status st = check_event_arrays(ev);
  if (st != MEM_OK) return st;
  if (ev->n_events < 1) return fail(MEM_EINVAL, "the tuner needs at least one event");
  static const int32_t kDefaults[] = {1024, 2048, 4096, 8192, 16384};
  if (!candidates) { candidates = kDefaults; n_cand = 5; }
  if (n_cand < 1) return fail(MEM_EINVAL, "no candidates");
  for (int i = 0; i < n_cand; ++i)
    if (!valid_chunk(candidates[i])) return fail(MEM_EINVAL, "candidates must be multiples of 256 <= 65536");
  int32_t wdef[4];
  if (!waves) { n_waves = waves_variants(p->desc.kind, wdef); waves = wdef; }
  if (n_waves < 1) return fail(MEM_EINVAL, "no waves candidates");
  for (int i = 0; i < n_waves; ++i)
    if (!waves_supported(p->desc.kind, waves[i])) return fail(MEM_EINVAL, "a waves candidate not compiled for this kind");
  // the timed call: the caller's options (outputs to the host, no
  // recording, no checkpoint, chunk size from the candidate), else a
  // 2-iteration integration with the defaults
  mem_integrate_opts base_opts{};
  base_opts.seed = 0x5EEDu;
  base_opts.alpha = 1.5;
  base_opts.max_iter = 64;
  base_opts.use_graph = 1;
  if (base) base_opts = *base;
  else n_iter = 2;
  base_opts.outputs_on_device = 0;
  base_opts.iter_out = nullptr;
  base_opts.grid_out = nullptr;
  base_opts.n_iter_out = nullptr;
  base_opts.timing_out = nullptr;
  base_opts.weights_out = nullptr;
  base_opts.hooks = 0;
  base_opts.checkpoint = nullptr;
  const int n_ev = ev->n_events;
  std::vector<double> P(n_ev), E(n_ev);
  std::vector<int32_t> S(n_ev);
  const int32_t keep_chunk = p->chunk_points, keep_waves = p->waves;
  double best_rate = -1.0;
  int32_t best = candidates[0], best_w = waves[0];
  for (int iw = 0; iw < n_waves; ++iw) {
    p->waves = waves[iw];
    for (int i = 0; i < n_cand; ++i) {
      double rate = 0.0;
      for (int rep = 0; rep < 2; ++rep) {   // the better of two runs
        mem_integrate_opts o = base_opts;
        o.seed = base_opts.seed + (uint64_t)rep;
        o.chunk_points = candidates[i];
        const auto t0 = std::chrono::steady_clock::now();
        st = mem_integrate_events(ev, &p, 1, &n_points, 1, n_iter, &o, P.data(), E.data(), S.data());
        const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (st != MEM_OK) { p->chunk_points = keep_chunk; p->waves = keep_waves; return st; }
        if (sec > 0.0) rate = std::max(rate, (double)n_ev / sec);
      }
      if (rate > best_rate) { best_rate = rate; best = candidates[i]; best_w = waves[iw]; }
    }
  }
  p->chunk_points = best;
  p->waves = best_w;
  if (best_out) *best_out = best;
  if (best_waves_out) *best_waves_out = best_w;
  if (rate_out) *rate_out = best_rate;
  if (table_path) {
    const std::string arch = device_arch();
    if (arch.empty()) return fail(MEM_EDEVICE, "cannot read the device architecture");
    const std::string key = tuning_key(arch, p);
    std::vector<std::string> lines;
    if (FILE* fh = std::fopen(table_path, "r")) {
      char buf[512];
      while (std::fgets(buf, sizeof buf, fh)) {
        std::string ln(buf);
        while (!ln.empty() && (ln.back() == '\n' || ln.back() == '\r')) ln.pop_back();
        if (ln.empty() || ln.compare(0, key.size() + 1, key + " ") == 0) continue;
        lines.push_back(ln);
      }
      std::fclose(fh);
    }
    char row[256];
    std::snprintf(row, sizeof row, "%s %d %d %.6g", key.c_str(), best, best_w, best_rate);
    lines.push_back(row);
    FILE* fo = std::fopen(table_path, "w");
    if (!fo) return fail(MEM_EINVAL, std::string("cannot write ") + table_path);
    std::fputs("# arch kind precision chunk_points waves_per_simd events_per_s\n", fo);
    for (const auto& ln : lines)
      if (ln[0] != '#') { std::fputs(ln.c_str(), fo); std::fputc('\n', fo); }
    std::fclose(fo);
  }
  return MEM_OK;
}

extern "C" mem_status mem_tuning_load(mem_process p, const char* table_path, const char* arch, int32_t* found)
{
  if (!p || !table_path) return fail(MEM_EINVAL, "null argument");
  if (found) *found = 0;
  const std::string a = arch ? std::string(arch) : device_arch();
  if (a.empty()) return fail(MEM_EDEVICE, "cannot read the device architecture");
  FILE* fh = std::fopen(table_path, "r");
  if (!fh) return fail(MEM_EINVAL, std::string("cannot read ") + table_path);
  const std::string key = tuning_key(a, p);
  char buf[512];
  mem_status st = MEM_OK;
  while (std::fgets(buf, sizeof buf, fh)) {
    std::string ln(buf);
    if (ln.compare(0, key.size() + 1, key + " ") != 0) continue;
    char* end = nullptr;
    const long c = std::strtol(ln.c_str() + key.size() + 1, &end, 10);
    const long w = std::strtol(end, nullptr, 10);
    if (!valid_chunk(c) || !waves_supported(p->desc.kind, (int)w)) { st = fail(MEM_EINVAL, "malformed tuning entry"); break; }
    p->chunk_points = (int32_t)c;
    p->waves = (int32_t)w;
    if (found) *found = 1;
  }
  std::fclose(fh);
  return st;
}

extern "C" mem_status mem_process_set_launch(mem_process p, int32_t chunk_points, int32_t waves)
{
  if (!p) return fail(MEM_EINVAL, "null process");
  if (chunk_points != 0 && !valid_chunk(chunk_points)) return fail(MEM_EINVAL, "chunk_points must be 0 or a multiple of 256 <= 65536");
  if (waves != 0 && !waves_supported(p->desc.kind, waves)) return fail(MEM_EINVAL, "waves variant not compiled for this kind");
  p->chunk_points = chunk_points;
  p->waves = waves;
  return MEM_OK;
}

extern "C" mem_status mem_process_waves(mem_process p, int32_t* waves)
{
  if (!p || !waves) return fail(MEM_EINVAL, "null argument");
  int32_t v[4];
  waves_variants(p->desc.kind, v);
  *waves = p->waves > 0 ? p->waves : v[0];
  return MEM_OK;
}

extern "C" mem_status mem_process_chunk_points(mem_process p, int32_t* chunk_points)
{
  if (!p || !chunk_points) return fail(MEM_EINVAL, "null argument");
  *chunk_points = p->chunk_points > 0 ? p->chunk_points : (int32_t)kDefaultChunk;
  return MEM_OK;
}

// ------------------------------------------------------- training data ----
extern "C" mem_status mem_vegas_capture(mem_process p, const mem_events* ev, const int32_t* event,
                                        const int32_t* perm, int32_t n_int, const double* grids, int64_t n_per,
                                        uint64_t seed, uint32_t iter, int32_t normalise, float* x_out,
                                        float* w_out, void* stream)
{
  if (!p || !event || !perm || !grids || !x_out || !w_out) return fail(MEM_EINVAL, "null argument");
  mem_status st = check_pdf_device(p);
  if (st != MEM_OK) return st;
  st = check_event_arrays(ev);
  if (st != MEM_OK) return st;
  if (n_int < 0 || n_per < 1 || n_per > (int64_t)0xFFFFFFFF) return fail(MEM_EINVAL, "bad sizes");
  if (ev->n_obj < n_obj_of(p->desc.kind)) return fail(MEM_EINVAL, "n_obj too small for the process kind");
  if (n_int == 0) return MEM_OK;
  // the kernels index events through event[]: check them on the host
  std::vector<int32_t> he(n_int), hp(n_int);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(he.data(), event, n_int * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hp.data(), perm, n_int * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < n_int; ++i) {
    if (he[i] < 0 || he[i] >= ev->n_events) return fail(MEM_EINVAL, "event index out of range");
    if (hp[i] < 0 || hp[i] >= p->pp.n_perm) return fail(MEM_EINVAL, "permutation out of range");
    st = check_host_event(ev, he[i], n_obj_of(p->desc.kind));
    if (st != MEM_OK) return st;
  }
  DevEvents dev;
  st = dev.make(ev, s);
  if (st != MEM_OK) return st;
  const int64_t tot = (int64_t)n_int * n_per;
  dim3 grid((unsigned)((tot + kBlock - 1) / kBlock));
  const bool f32 = p->desc.precision == MEM_FP32;
  switch (p->desc.kind) {
    case MEM_DY_QQ_GAMMA_MUMU:
      hipLaunchKernelGGL((capture_kernel<kDY, 2, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event, perm,
                         n_int, grids, n_per, seed, iter, x_out, w_out);
      break;
    case MEM_TT_SEMILEPTON:
      if (f32)
        hipLaunchKernelGGL((capture_kernel<kSL, 7, float>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event, perm,
                           n_int, grids, n_per, seed, iter, x_out, w_out);
      else
        hipLaunchKernelGGL((capture_kernel<kSL, 7, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                           perm, n_int, grids, n_per, seed, iter, x_out, w_out);
      break;
    case MEM_TTH_SEMILEPTON:
      if (f32)
        hipLaunchKernelGGL((capture_kernel<kTTH, 9, float>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                           perm, n_int, grids, n_per, seed, iter, x_out, w_out);
      else
        hipLaunchKernelGGL((capture_kernel<kTTH, 9, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                           perm, n_int, grids, n_per, seed, iter, x_out, w_out);
      break;
    case MEM_TT_DILEPTON:
      if (f32)
        hipLaunchKernelGGL((capture_kernel<kTT, 8, float>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event, perm,
                           n_int, grids, n_per, seed, iter, x_out, w_out);
      else
        hipLaunchKernelGGL((capture_kernel<kTT, 8, double>), grid, dim3(kBlock), 0, s, p->pp, dev.view, event,
                           perm, n_int, grids, n_per, seed, iter, x_out, w_out);
      break;
    case MEM_TTH_DILEPTON:
    case MEM_TTBB_DILEPTON:
      return fail(MEM_EUNSUPPORTED, "training capture covers the single-top-pair kinds");
    default:
      return fail(MEM_EINVAL, "unknown process kind");
  }
  HIP_TRY(hipGetLastError());
  if (normalise) {
    hipLaunchKernelGGL(normalise_kernel, dim3(n_int), dim3(kBlock), 0, s, w_out, n_per);
    HIP_TRY(hipGetLastError());
  }
  if (!ev->on_device) HIP_TRY(hipStreamSynchronize(s));
  return MEM_OK;
}

// ------------------------------------------------------------------ flow ----
struct mem_flow_s {
  float* P = nullptr;       // FP32 master parameters
  float* grad = nullptr;
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  uint16_t* Wb = nullptr;   // BF16 operand copies of the 128-wide layers
  uint16_t* Wf = nullptr;   // the same in matrix-core fragment order (sampling)
  float* tape = nullptr;    // training tape, tape_cap samples
  float* lq = nullptr;      // log q of the training samples
  int64_t tape_cap = 0;
  double* loss_parts = nullptr;
  float* part = nullptr;    // per-workgroup gradient slots of the backward pass
  int part_slots = 0;
  int64_t step = 0;
  int32_t mode = MEM_FLOW_BF16;
  ~mem_flow_s()
  {
    for (void* q : {(void*)P, (void*)grad, (void*)m, (void*)v, (void*)Wb, (void*)Wf, (void*)tape, (void*)lq,
                    (void*)loss_parts, (void*)part})
      if (q) (void)hipFree(q);
  }
};

namespace {
constexpr int kLossBlocks = 256;
// backward workgroups (and gradient slots) of a training step: one per CU
constexpr unsigned kGradSlots = 256;

__global__ void fill_f32_kernel(float* p, int64_t n, float v)
{
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void fill_f32(float* p, int64_t n, float v, hipStream_t s)
{
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
}

mem_status flow_convert(mem_flow f, hipStream_t s)
{
  const int64_t n = (int64_t)FLAYERS * FB_PER;
  hipLaunchKernelGGL(flow_convert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f->P, f->Wb);
  const int64_t nf = (int64_t)FLAYERS * FS_PER;
  hipLaunchKernelGGL(flow_swizzle_kernel, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, f->P, f->Wf);
  HIP_TRY(hipGetLastError());
  return MEM_OK;
}

mem_status flow_tape(mem_flow f, int64_t n)
{
  const int64_t need = (n + FP - 1) / FP * FP;
  if (need <= f->tape_cap) return MEM_OK;
  if (f->tape) { (void)hipFree(f->tape); f->tape = nullptr; }
  if (f->lq) { (void)hipFree(f->lq); f->lq = nullptr; }
  f->tape_cap = 0;
  HIP_TRY(hipMalloc(&f->tape, (size_t)need * FLAYERS * FTAPE * sizeof(float)));
  HIP_TRY(hipMalloc(&f->lq, (size_t)need * sizeof(float)));
  f->tape_cap = need;
  return MEM_OK;
}

// the first layer's context part of n contexts
mem_status flow_cvec(mem_flow f, const float* ctx, int n, float* cvec, hipStream_t s)
{
  const int64_t t = (int64_t)n * FLAYERS * FH;
  hipLaunchKernelGGL(flow_cvec_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, f->P, ctx, n, cvec);
  HIP_TRY(hipGetLastError());
  return MEM_OK;
}

// range [min, max] of the context rows a sample set uses (read back and
// checked on the host: the kernels index the context table with them)
mem_status sint_range(const int32_t* sint, int64_t n, hipStream_t s, int32_t* lo, int32_t* hi)
{
  std::vector<int32_t> h(n);
  HIP_TRY(hipMemcpyAsync(h.data(), sint, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int32_t mn = h[0], mx = h[0];
  for (int64_t i = 0; i < n; ++i) {
    if (h[i] < 0) return fail(MEM_EINVAL, "negative context index");
    mn = std::min(mn, h[i]);
    mx = std::max(mx, h[i]);
  }
  *lo = mn;
  *hi = mx;
  return MEM_OK;
}
}  // namespace

extern "C" mem_status mem_flow_create(int32_t mode, mem_flow* out)
{
  if (!out) return fail(MEM_EINVAL, "null argument");
  *out = nullptr;
  if (mode != MEM_FLOW_BF16 && mode != MEM_FLOW_BF16X2) return fail(MEM_EINVAL, "unknown flow mode");
  mem_flow f = new (std::nothrow) mem_flow_s;
  if (!f) return fail(MEM_ENOMEM, "host allocation");
  f->mode = mode;
  auto bad = [&](mem_status st) { delete f; return st; };
  for (float** q : {&f->P, &f->grad, &f->m, &f->v}) {
    if (hipMalloc(q, (size_t)FNP * sizeof(float)) != hipSuccess) return bad(fail(MEM_ENOMEM, "flow parameters"));
    if (hipMemset(*q, 0, (size_t)FNP * sizeof(float)) != hipSuccess) return bad(fail(MEM_EDEVICE, "hipMemset"));
  }
  if (hipMalloc(&f->Wb, (size_t)FLAYERS * FB_PER * sizeof(uint16_t)) != hipSuccess ||
      hipMalloc(&f->Wf, (size_t)FLAYERS * FS_PER * sizeof(uint16_t)) != hipSuccess ||
      hipMalloc(&f->loss_parts, kLossBlocks * sizeof(double)) != hipSuccess)
    return bad(fail(MEM_ENOMEM, "flow buffers"));
  mem_status st = flow_convert(f, nullptr);
  if (st != MEM_OK) return bad(st);
  if (hipDeviceSynchronize() != hipSuccess) return bad(fail(MEM_EDEVICE, "hipDeviceSynchronize"));
  *out = f;
  return MEM_OK;
}

extern "C" void mem_flow_destroy(mem_flow f)
{
  if (!f) return;
  (void)hipDeviceSynchronize();
  delete f;
}

extern "C" mem_status mem_flow_set_params(mem_flow f, const float* params, int64_t n, int32_t on_device)
{
  if (!f || !params) return fail(MEM_EINVAL, "null argument");
  if (n != FNP) return fail(MEM_EINVAL, "parameter count must be 192552");
  HIP_TRY(hipMemcpy(f->P, params, (size_t)FNP * sizeof(float),
                    on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(f->m, 0, (size_t)FNP * sizeof(float)));
  HIP_TRY(hipMemset(f->v, 0, (size_t)FNP * sizeof(float)));
  f->step = 0;
  mem_status st = flow_convert(f, nullptr);
  if (st != MEM_OK) return st;
  HIP_TRY(hipDeviceSynchronize());
  return MEM_OK;
}

extern "C" mem_status mem_flow_get_params(mem_flow f, float* params, int64_t n, int32_t on_device)
{
  if (!f || !params) return fail(MEM_EINVAL, "null argument");
  if (n != FNP) return fail(MEM_EINVAL, "parameter count must be 192552");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(params, f->P, (size_t)FNP * sizeof(float),
                    on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  return MEM_OK;
}

extern "C" mem_status mem_flow_context(const mem_events* ev, const int32_t* event, const int32_t* perm, int32_t n,
                                       float* ctx, void* stream)
{
  if (!event || !perm || !ctx) return fail(MEM_EINVAL, "null argument");
  mem_status st = check_event_arrays(ev);
  if (st != MEM_OK) return st;
  if (n < 0) return fail(MEM_EINVAL, "negative n");
  if (ev->n_obj < 4) return fail(MEM_EINVAL, "n_obj too small for ttbar dilepton");
  if (n == 0) return MEM_OK;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> he(n), hp(n);
  HIP_TRY(hipMemcpyAsync(he.data(), event, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hp.data(), perm, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i) {
    if (he[i] < 0 || he[i] >= ev->n_events) return fail(MEM_EINVAL, "event index out of range");
    if (hp[i] < 0 || hp[i] > 1) return fail(MEM_EINVAL, "permutation out of range");
    st = check_host_event(ev, he[i], 4);
    if (st != MEM_OK) return st;
  }
  DevEvents dev;
  st = dev.make(ev, s);
  if (st != MEM_OK) return st;
  hipLaunchKernelGGL(flow_ctx_kernel, dim3((n + 255) / 256), dim3(256), 0, s, dev.view, event, perm, n, ctx);
  HIP_TRY(hipGetLastError());
  if (!ev->on_device) HIP_TRY(hipStreamSynchronize(s));
  return MEM_OK;
}

extern "C" mem_status mem_flow_sample(mem_flow f, const float* ctx, const int32_t* event, const int32_t* perm,
                                      int32_t n_int, int64_t n_per, uint64_t seed, uint32_t iter, float* x_out,
                                      float* logq_out, void* stream)
{
  if (!f || !ctx || !event || !perm || !x_out || !logq_out) return fail(MEM_EINVAL, "null argument");
  if (n_int < 0 || n_per < 1 || n_per > (int64_t)0xFFFFFFFF) return fail(MEM_EINVAL, "bad sizes");
  if (n_int == 0) return MEM_OK;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> he(n_int), hp(n_int);
  HIP_TRY(hipMemcpyAsync(he.data(), event, n_int * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hp.data(), perm, n_int * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<FlowChunk> ch;
  for (int i = 0; i < n_int; ++i)
    for (int64_t s0 = 0; s0 < n_per; s0 += FP)
      ch.push_back(FlowChunk{i, he[i], hp[i], (int32_t)std::min<int64_t>(FP, n_per - s0), s0, (int64_t)i * n_per + s0});
  if ((int64_t)ch.size() > (int64_t)0x7FFFFFFF) return fail(MEM_EINVAL, "too many points");
  DevBuf b_cvec, b_ch;
  HIP_TRY(b_cvec.alloc((size_t)n_int * FLAYERS * FH * sizeof(float)));
  HIP_TRY(b_ch.alloc(ch.size() * sizeof(FlowChunk)));
  HIP_TRY(hipMemcpyAsync(b_ch.p, ch.data(), ch.size() * sizeof(FlowChunk), hipMemcpyHostToDevice, s));
  mem_status st = flow_cvec(f, ctx, n_int, b_cvec.as<float>(), s);
  if (st != MEM_OK) return st;
  hipLaunchKernelGGL(f->mode == MEM_FLOW_BF16X2 ? flow_sample2_kernel<true> : flow_sample2_kernel<false>,
                     dim3((unsigned)ch.size()), dim3(FT), 0, s, f->P, f->Wf, b_cvec.as<float>(),
                     b_ch.as<FlowChunk>(), seed, iter, (const uint32_t*)nullptr, (const int32_t*)nullptr, x_out,
                     logq_out);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));   // the chunk table is freed on return
  return MEM_OK;
}

extern "C" mem_status mem_flow_log_prob(mem_flow f, const float* ctx, const int32_t* sint, const float* x, int64_t n,
                                        float* logq_out, void* stream)
{
  if (!f || !ctx || !sint || !x || !logq_out) return fail(MEM_EINVAL, "null argument");
  if (n < 0 || n > (int64_t)0x7FFFFFFF) return fail(MEM_EINVAL, "bad size");
  if (n == 0) return MEM_OK;
  hipStream_t s = (hipStream_t)stream;
  int32_t c_lo = 0, c_hi = 0;
  mem_status st = sint_range(sint, n, s, &c_lo, &c_hi);
  if (st != MEM_OK) return st;
  const int n_ctx = c_hi - c_lo + 1;
  st = flow_tape(f, n);
  if (st != MEM_OK) return st;
  DevBuf b_cvec;
  HIP_TRY(b_cvec.alloc((size_t)n_ctx * FLAYERS * FH * sizeof(float)));
  st = flow_cvec(f, ctx + (int64_t)c_lo * FCTX, n_ctx, b_cvec.as<float>(), s);
  if (st != MEM_OK) return st;
  hipLaunchKernelGGL(f->mode == MEM_FLOW_BF16X2 ? flow_train_fwd_kernel<true> : flow_train_fwd_kernel<false>,
                     dim3((unsigned)((n + FP - 1) / FP)), dim3(FT), 0, s, f->P, f->Wb,
                     b_cvec.as<float>(), sint, c_lo, x, (int)n, f->tape, logq_out);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return MEM_OK;
}

// One training step once the arguments are checked: the minibatch's context
// rows are [c_lo, c_lo + n_ctx); cvec holds n_ctx first-layer projections.
// Enqueues on s; synchronises only for loss_out.
static mem_status flow_train_core(mem_flow f, const float* ctx, const int32_t* sint, const float* x,
                                  const float* wt, int64_t n, double lr, double* loss_out, float* grad_out,
                                  hipStream_t s, int32_t c_lo, int n_ctx, float* cvec)
{
  mem_status st = flow_tape(f, n);
  if (st != MEM_OK) return st;
  st = flow_cvec(f, ctx + (int64_t)c_lo * FCTX, n_ctx, cvec, s);
  if (st != MEM_OK) return st;
  const unsigned nb = (unsigned)((n + FP - 1) / FP);
  // one gradient slot per backward workgroup, summed in slot order
  const int slots = (int)std::min<unsigned>(nb, (unsigned)kGradSlots);
  if (slots > f->part_slots) {
    if (f->part) { (void)hipFree(f->part); f->part = nullptr; f->part_slots = 0; }
    HIP_TRY(hipMalloc(&f->part, (size_t)slots * FNP * sizeof(float)));
    f->part_slots = slots;
  }
  hipLaunchKernelGGL(f->mode == MEM_FLOW_BF16X2 ? flow_train_fwd_kernel<true> : flow_train_fwd_kernel<false>,
                     dim3(nb), dim3(FT), 0, s, f->P, f->Wb, cvec, sint, c_lo, x, (int)n, f->tape, f->lq);
  hipLaunchKernelGGL(flow_train_bwd_kernel, dim3(slots), dim3(FT), 0, s, f->P, f->Wb, ctx, sint, wt, (int)n,
                     f->tape, f->part);
  hipLaunchKernelGGL(flow_grad_reduce_kernel, dim3((FNP + 255) / 256), dim3(256), 0, s, f->part, slots, f->grad);
  HIP_TRY(hipGetLastError());
  if (grad_out) HIP_TRY(hipMemcpyAsync(grad_out, f->grad, (size_t)FNP * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (loss_out) {
    hipLaunchKernelGGL(flow_loss_kernel, dim3(kLossBlocks), dim3(kBlock), 0, s, wt, f->lq, n, f->loss_parts);
    HIP_TRY(hipGetLastError());
    double h[kLossBlocks];
    HIP_TRY(hipMemcpyAsync(h, f->loss_parts, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double L = 0.0;
    for (int i = 0; i < kLossBlocks; ++i) L += h[i];
    *loss_out = L;
  }
  if (lr > 0.0) {
    f->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)f->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)f->step)));
    hipLaunchKernelGGL(flow_adam_kernel, dim3((FNP + 255) / 256), dim3(256), 0, s, f->P, f->grad, f->m, f->v, FNP,
                       (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    HIP_TRY(hipGetLastError());
    st = flow_convert(f, s);
    if (st != MEM_OK) return st;
  }
  return MEM_OK;
}

extern "C" mem_status mem_flow_train_step(mem_flow f, const float* ctx, const int32_t* sint, const float* x,
                                          const float* wt, int64_t n, double lr, double* loss_out, float* grad_out,
                                          void* stream)
{
  if (!f || !ctx || !sint || !x || !wt) return fail(MEM_EINVAL, "null argument");
  if (n < 1 || n > (int64_t)0x7FFFFFFF) return fail(MEM_EINVAL, "bad size");
  if (!(lr >= 0.0)) return fail(MEM_EINVAL, "lr must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  int32_t c_lo = 0, c_hi = 0;
  mem_status st = sint_range(sint, n, s, &c_lo, &c_hi);
  if (st != MEM_OK) return st;
  const int n_ctx = c_hi - c_lo + 1;
  DevBuf b_cvec;
  HIP_TRY(b_cvec.alloc((size_t)n_ctx * FLAYERS * FH * sizeof(float)));
  st = flow_train_core(f, ctx, sint, x, wt, n, lr, loss_out, grad_out, s, c_lo, n_ctx, b_cvec.as<float>());
  if (st != MEM_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));   // the context projection is freed on return
  return MEM_OK;
}

// ------------------------------------------------ proposal training ----
namespace {
__global__ void integral_of_sample_kernel(int32_t* sint, int64_t n, int32_t per)
{
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) sint[i] = (int32_t)(i / per);
}
__global__ void event_perm_kernel(int32_t* ev, int32_t* pm, int32_t n_int)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_int) { ev[i] = i >> 1; pm[i] = i & 1; }
}
// splitmix64 (Steele, Lea, Flood, OOPSLA 2014): the minibatch order
uint64_t splitmix64(uint64_t& st)
{
  uint64_t z = (st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
}  // namespace

extern "C" mem_status mem_train_proposal(mem_process p, const mem_events* train, const mem_flow_desc* fd,
                                         mem_flow* out)
{
  if (!p || !train || !out) return fail(MEM_EINVAL, "null argument");
  *out = nullptr;
  if (p->desc.kind != MEM_TT_DILEPTON) return fail(MEM_EUNSUPPORTED, "the proposal is defined for ttbar dilepton");
  mem_flow_desc d{};
  d.mode = MEM_FLOW_BF16;
  if (fd) d = *fd;
  const int64_t vpts = d.vegas_points > 0 ? d.vegas_points : 8192;
  const int32_t viter = d.vegas_iter > 0 ? d.vegas_iter : 4;
  const int32_t cap = d.capture > 0 ? d.capture : 168;
  const int32_t batch = d.batch > 0 ? d.batch : 65536;
  const int32_t epochs = d.epochs > 0 ? d.epochs : 24;
  const double lr_max = d.lr_max > 0.0 ? d.lr_max : 2e-3, lr_min = d.lr_min > 0.0 ? d.lr_min : 1e-4;
  if (d.mode != MEM_FLOW_BF16 && d.mode != MEM_FLOW_BF16X2) return fail(MEM_EINVAL, "unknown flow mode");
  if (viter < 2) return fail(MEM_EINVAL, "vegas_iter must be at least 2");
  if (!(lr_min <= lr_max)) return fail(MEM_EINVAL, "lr_min above lr_max");
  mem_status st = check_event_arrays(train);
  if (st != MEM_OK) return st;
  const int n_ev = train->n_events;
  if (train->n_obj < 4) return fail(MEM_EINVAL, "n_obj too small for ttbar dilepton");
  const int64_t n_int = 2 * (int64_t)n_ev;
  const int64_t n_s = n_int * cap;
  if (n_int < 1 || n_s > (int64_t)0x7FFFFFFF) return fail(MEM_EINVAL, "training set size out of range");
  if (batch < 1 || batch > n_s) return fail(MEM_EINVAL, "batch must be between 1 and the number of samples");
  hipStream_t s = (hipStream_t)d.stream;
  // events on the device once (VEGAS, capture and context all read them)
  DevEvents dev;
  st = dev.make(train, s);
  if (st != MEM_OK) return st;
  mem_events ed = *train;
  ed.E = dev.view.E; ed.px = dev.view.px; ed.py = dev.view.py; ed.pz = dev.view.pz;
  ed.charge = dev.view.charge;
  ed.on_device = 1;
  // 1. VEGAS on the training events; their adapted grids
  DevBuf b_grid, b_P, b_err, b_st, b_ev, b_pm;
  HIP_TRY(b_grid.alloc((size_t)n_int * 8 * (kBins + 1) * sizeof(double)));
  HIP_TRY(b_P.alloc((size_t)n_ev * sizeof(double)));
  HIP_TRY(b_err.alloc((size_t)n_ev * sizeof(double)));
  HIP_TRY(b_st.alloc((size_t)n_ev * sizeof(int32_t)));
  HIP_TRY(b_ev.alloc((size_t)n_int * sizeof(int32_t)));
  HIP_TRY(b_pm.alloc((size_t)n_int * sizeof(int32_t)));
  {
    mem_integrate_opts o{};
    o.seed = d.seed;
    o.alpha = 1.5;
    o.max_iter = 64;
    o.use_graph = 1;
    o.stream = d.stream;
    o.outputs_on_device = 1;
    o.grid_out = b_grid.as<double>();
    const mem_process hyp[1] = {p};
    st = mem_integrate_events(&ed, hyp, 1, &vpts, 1, viter, &o, b_P.as<double>(), b_err.as<double>(),
                              b_st.as<int32_t>());
    if (st != MEM_OK) return st;
  }
  hipLaunchKernelGGL(event_perm_kernel, dim3((unsigned)((n_int + 255) / 256)), dim3(256), 0, s, b_ev.as<int32_t>(),
                     b_pm.as<int32_t>(), (int32_t)n_int);
  HIP_TRY(hipGetLastError());
  // 2. samples of the adapted grids (x, f J normalised per integral) and contexts
  DevBuf b_x, b_w, b_ctx, b_sint;
  HIP_TRY(b_x.alloc((size_t)n_s * 8 * sizeof(float)));
  HIP_TRY(b_w.alloc((size_t)n_s * sizeof(float)));
  HIP_TRY(b_ctx.alloc((size_t)n_int * FCTX * sizeof(float)));
  HIP_TRY(b_sint.alloc((size_t)n_s * sizeof(int32_t)));
  st = mem_vegas_capture(p, &ed, b_ev.as<int32_t>(), b_pm.as<int32_t>(), (int32_t)n_int, b_grid.as<double>(), cap,
                         d.seed, 99u, 1, b_x.as<float>(), b_w.as<float>(), d.stream);
  if (st != MEM_OK) return st;
  st = mem_flow_context(&ed, b_ev.as<int32_t>(), b_pm.as<int32_t>(), (int32_t)n_int, b_ctx.as<float>(), d.stream);
  if (st != MEM_OK) return st;
  hipLaunchKernelGGL(integral_of_sample_kernel, dim3((unsigned)((n_s + 255) / 256)), dim3(256), 0, s,
                     b_sint.as<int32_t>(), n_s, cap);
  HIP_TRY(hipGetLastError());
  // 3. the flow, trained on shuffled minibatches (contiguous slices of the
  //    samples: each holds whole integrals' samples), cosine learning rate
  mem_flow f = nullptr;
  st = mem_flow_create(d.mode, &f);
  if (st != MEM_OK) return st;
  struct FlowGuard { mem_flow& f; ~FlowGuard() { if (f) mem_flow_destroy(f); } } fg{f};
  const int64_t n_b = n_s / batch;
  const int max_ctx = (int)((batch + cap - 1) / cap) + 1;
  DevBuf b_cvec;
  HIP_TRY(b_cvec.alloc((size_t)max_ctx * FLAYERS * FH * sizeof(float)));
  std::vector<int64_t> order(n_b);
  uint64_t rs = d.seed ^ 0x5EEDF10Aull;
  const int64_t total = (int64_t)epochs * n_b;
  int64_t k = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = 0; i < n_b; ++i) order[i] = i;
    for (int64_t i = n_b - 1; i > 0; --i) std::swap(order[i], order[(int64_t)(splitmix64(rs) % (uint64_t)(i + 1))]);
    for (int64_t j = 0; j < n_b; ++j, ++k) {
      const int64_t b = order[j];
      const double lr = lr_min + 0.5 * (lr_max - lr_min) * (1.0 + std::cos(M_PI * (double)k / (double)total));
      const int64_t s0 = b * batch;
      const int32_t c_lo = (int32_t)(s0 / cap), c_hi = (int32_t)((s0 + batch - 1) / cap);
      double L = 0.0;
      const bool want = d.loss_out != nullptr && j == 0;
      st = flow_train_core(f, b_ctx.as<float>(), b_sint.as<int32_t>() + s0, b_x.as<float>() + s0 * 8,
                           b_w.as<float>() + s0, batch, lr, want ? &L : nullptr, nullptr, s, c_lo,
                           c_hi - c_lo + 1, b_cvec.as<float>());
      if (st != MEM_OK) return st;
      if (want) d.loss_out[ep] = L / ((double)batch / (double)cap);
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  *out = f;
  f = nullptr;
  return MEM_OK;
}

extern "C" mem_status mem_set_proposal(mem_process p, mem_flow f)
{
  if (!p) return fail(MEM_EINVAL, "null process");
  if (f && p->desc.kind != MEM_TT_DILEPTON) return fail(MEM_EUNSUPPORTED, "the proposal is defined for ttbar dilepton");
  p->proposal = f;
  return MEM_OK;
}

// File layout of a saved flow: "MEMFLOW1", int32 mode, int32 0, int64 Adam
// step, int64 parameter count, then the FP32 parameters and the two Adam
// moments (little-endian, as in memory).
extern "C" mem_status mem_flow_save(mem_flow f, const char* path)
{
  if (!f || !path) return fail(MEM_EINVAL, "null argument");
  std::vector<float> h(3 * (size_t)FNP);
  HIP_TRY(hipMemcpy(h.data(), f->P, (size_t)FNP * sizeof(float), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(h.data() + FNP, f->m, (size_t)FNP * sizeof(float), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(h.data() + 2 * (size_t)FNP, f->v, (size_t)FNP * sizeof(float), hipMemcpyDeviceToHost));
  FILE* fp = std::fopen(path, "wb");
  if (!fp) return fail(MEM_EINVAL, std::string("cannot write ") + path);
  const int32_t hdr[2] = {f->mode, 0};
  const int64_t nums[2] = {f->step, (int64_t)FNP};
  bool ok = std::fwrite("MEMFLOW1", 1, 8, fp) == 8 && std::fwrite(hdr, sizeof(hdr), 1, fp) == 1 &&
            std::fwrite(nums, sizeof(nums), 1, fp) == 1 && std::fwrite(h.data(), sizeof(float), h.size(), fp) == h.size();
  ok = (std::fclose(fp) == 0) && ok;
  if (!ok) return fail(MEM_EINVAL, std::string("write failed: ") + path);
  return MEM_OK;
}

extern "C" mem_status mem_flow_load(const char* path, mem_flow* out)
{
  if (!path || !out) return fail(MEM_EINVAL, "null argument");
  *out = nullptr;
  FILE* fp = std::fopen(path, "rb");
  if (!fp) return fail(MEM_EINVAL, std::string("cannot read ") + path);
  char magic[8];
  int32_t hdr[2];
  int64_t nums[2];
  std::vector<float> h(3 * (size_t)FNP);
  bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "MEMFLOW1", 8) == 0 &&
            std::fread(hdr, sizeof(hdr), 1, fp) == 1 && std::fread(nums, sizeof(nums), 1, fp) == 1 &&
            nums[1] == (int64_t)FNP && nums[0] >= 0 && std::fread(h.data(), sizeof(float), h.size(), fp) == h.size();
  char extra;
  ok = ok && std::fread(&extra, 1, 1, fp) == 0;
  std::fclose(fp);
  if (!ok) return fail(MEM_EINVAL, std::string("not a saved flow: ") + path);
  mem_flow f = nullptr;
  mem_status st = mem_flow_create(hdr[0], &f);
  if (st != MEM_OK) return st;
  st = mem_flow_set_params(f, h.data(), FNP, 0);
  if (st == MEM_OK) {
    if (hipMemcpy(f->m, h.data() + FNP, (size_t)FNP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(f->v, h.data() + 2 * (size_t)FNP, (size_t)FNP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
      st = fail(MEM_EDEVICE, "hipMemcpy of the Adam moments");
  }
  if (st != MEM_OK) { mem_flow_destroy(f); return st; }
  f->step = nums[0];
  *out = f;
  return MEM_OK;
}

// Flow-proposal integration (see mem_integrate_opts.flow).
// ------------------------------------------------ flow-seeded grids ----
namespace {
constexpr int64_t kSeedPoints = 1024;        // proposal samples per integral
constexpr int kSeedHist = 512;               // histogram bins per dimension
constexpr double kSeedUniform = 0.2;         // share of the uniform density in the seeded grid
constexpr uint32_t kSeedIter = 0xFFFFFFF0u;  // iteration index of the seeding draws

// Grid of integral blockIdx.x from M proposal samples x[ig][M][8]: per
// dimension the edges at the quantiles k/64 of the mixture
// (1 - eps) F_samples + eps F_uniform, the sample CDF read from a
// kSeedHist-bin histogram and linear inside a bin.  The uniform share keeps
// every bin wider than eps / 64 of the unit interval, where the proposal
// underweights the integrand.  One wavefront per dimension.
__global__ __launch_bounds__(256) void seed_grids_kernel(const float* __restrict__ x, int64_t M,
                                                         const IntegralDesc* __restrict__ ints,
                                                         double* __restrict__ grids, double eps)
{
  __shared__ uint32_t hist[4][kSeedHist];
  const int ig = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const IntegralDesc in = ints[ig];
  for (int d0 = 0; d0 < 8; d0 += 4) {
    const int d = d0 + w;
    for (int b = lane; b < kSeedHist; b += 64) hist[w][b] = 0u;
    __syncthreads();
    for (int64_t k = lane; k < M; k += 64) {
      const float v = x[((int64_t)ig * M + k) * 8 + d];
      const int b = min(kSeedHist - 1, max(0, (int)(v * (float)kSeedHist)));
      atomicAdd(&hist[w][b], 1u);
    }
    __syncthreads();
    if (lane == 0 && d < in.dims) {
      double* e = grids + in.grid_off + (int64_t)d * (kBins + 1);
      const double inv = 1.0 / (double)M, hw = 1.0 / kSeedHist;
      double cum = 0.0;
      int b = 0;
      e[0] = 0.0;
      for (int k = 1; k < kBins; ++k) {
        const double t = (double)k / kBins;
        while (b < kSeedHist - 1 && (1.0 - eps) * (cum + hist[w][b] * inv) + eps * (b + 1) * hw < t) {
          cum += hist[w][b] * inv;
          ++b;
        }
        const double g0 = (1.0 - eps) * cum + eps * b * hw;
        const double g1 = (1.0 - eps) * (cum + hist[w][b] * inv) + eps * (b + 1) * hw;
        e[k] = fmin(1.0, (b + (t - g0) / (g1 - g0)) * hw);
      }
      e[kBins] = 1.0;
    }
    __syncthreads();
  }
}
}  // namespace

// Seed the grids of ttbar dilepton integrals from a proposal: kSeedPoints
// samples of each integral (the flow's own point stream at iteration
// kSeedIter, apart from VEGAS's), then seed_grids_kernel.
static mem_status seed_grids_from_flow(mem_flow f, const EventsView& view, const std::vector<IntegralDesc>& ints,
                                       const IntegralDesc* d_ints, double* grids, uint64_t seed, Workspace& work,
                                       hipStream_t s)
{
  const int n_int = (int)ints.size();
  std::vector<int32_t> iev(n_int), ipm(n_int);
  std::vector<FlowChunk> sch;
  for (int ig = 0; ig < n_int; ++ig) {
    if (ints[ig].dims != 8) return fail(MEM_EUNSUPPORTED, "flow-seeded grids cover ttbar dilepton only");
    iev[ig] = ints[ig].event;
    ipm[ig] = ints[ig].perm;
    for (int64_t s0 = 0; s0 < kSeedPoints; s0 += FP)
      sch.push_back(FlowChunk{ig, iev[ig], ipm[ig], (int32_t)std::min<int64_t>(FP, kSeedPoints - s0), s0,
                              (int64_t)ig * kSeedPoints + s0});
  }
  DevBuf b_ev(&work), b_pm(&work), b_ctx(&work), b_cvec(&work), b_sch(&work), b_x(&work), b_lq(&work);
  HIP_TRY(b_ev.alloc(n_int * sizeof(int32_t)));
  HIP_TRY(b_pm.alloc(n_int * sizeof(int32_t)));
  HIP_TRY(b_ctx.alloc((size_t)n_int * FCTX * sizeof(float)));
  HIP_TRY(b_cvec.alloc((size_t)n_int * FLAYERS * FH * sizeof(float)));
  HIP_TRY(b_sch.alloc(sch.size() * sizeof(FlowChunk)));
  HIP_TRY(b_x.alloc((size_t)n_int * kSeedPoints * 8 * sizeof(float)));
  HIP_TRY(b_lq.alloc((size_t)n_int * kSeedPoints * sizeof(float)));
  HIP_TRY(hipMemcpyAsync(b_ev.p, iev.data(), n_int * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b_pm.p, ipm.data(), n_int * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b_sch.p, sch.data(), sch.size() * sizeof(FlowChunk), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(flow_ctx_kernel, dim3((n_int + 255) / 256), dim3(256), 0, s, view, b_ev.as<int32_t>(),
                     b_pm.as<int32_t>(), n_int, b_ctx.as<float>());
  HIP_TRY(hipGetLastError());
  mem_status st = flow_cvec(f, b_ctx.as<float>(), n_int, b_cvec.as<float>(), s);
  if (st != MEM_OK) return st;
  hipLaunchKernelGGL(f->mode == MEM_FLOW_BF16X2 ? flow_sample2_kernel<true> : flow_sample2_kernel<false>,
                     dim3((unsigned)sch.size()), dim3(FT), 0, s, f->P, f->Wf, b_cvec.as<float>(),
                     b_sch.as<FlowChunk>(), seed, kSeedIter, (const uint32_t*)nullptr, (const int32_t*)nullptr,
                     b_x.as<float>(), b_lq.as<float>());
  hipLaunchKernelGGL(seed_grids_kernel, dim3(n_int), dim3(256), 0, s, b_x.as<float>(), kSeedPoints, d_ints, grids,
                     kSeedUniform);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));   // the samples are freed on return
  return MEM_OK;
}

static mem_status integrate_flow(const mem_events* ev, const mem_process* hyp, int32_t n_hyp,
                                 const int64_t* n_points, int32_t n_np, int32_t iters, const mem_integrate_opts& o,
                                 double* p_out, double* err_out, int32_t* status_out, Workspace& work)
{
  const int n_ev = ev->n_events;
  mem_flow fl = o.flow;
  const double thr = o.ess_threshold > 0.0 ? o.ess_threshold : 0.3;
  const bool target_mode = o.target_rel_err > 0.0;
  std::vector<const mem_process_s*> procs;
  std::vector<int> ev_proc(n_ev);
  int prec = -1;
  for (int e = 0; e < n_ev; ++e) {
    const mem_process p = hyp[n_hyp == 1 ? 0 : e];
    if (!p) return fail(MEM_EINVAL, "null process handle");
    if (p->desc.kind != MEM_TT_DILEPTON) return fail(MEM_EUNSUPPORTED, "the flow proposal covers ttbar dilepton only");
    if (prec < 0) prec = p->desc.precision;
    if (p->desc.precision != prec) return fail(MEM_EINVAL, "one precision per flow call");
    if (ev->n_obj < 4) return fail(MEM_EINVAL, "n_obj too small for the process kind");
    mem_status st = check_host_event(ev, e, 4);
    if (st != MEM_OK) return st;
    int pi = -1;
    for (size_t k = 0; k < procs.size(); ++k) if (procs[k] == p) pi = (int)k;
    if (pi < 0) { procs.push_back(p); pi = (int)procs.size() - 1; }
    ev_proc[e] = pi;
  }
  for (const auto* pr : procs) {
    mem_status ps = check_pdf_device(pr);
    if (ps != MEM_OK) return ps;
  }
  std::vector<ProcParams> ptab(procs.size());
  for (size_t k = 0; k < procs.size(); ++k) ptab[k] = procs[k]->pp;
  // integrals, sampling chunks (FP points), weight chunks (FW points)
  std::vector<FlowIntegral> ints;
  std::vector<int32_t> int_proc, int_ev, int_perm;
  std::vector<int64_t> ev_int0(n_ev);
  std::vector<int32_t> ev_np(n_ev);
  std::vector<double> ev_norm(n_ev);
  std::vector<FlowChunk> sch, wch;
  int64_t tot = 0;
  for (int e = 0; e < n_ev; ++e) {
    const mem_process_s* p = procs[ev_proc[e]];
    const int np = p->pp.n_perm;
    const int64_t per = (n_points[n_np == 1 ? 0 : e] + np - 1) / np;
    if (per < 2) return fail(MEM_EINVAL, "n_points too small");
    if (per > (int64_t)0xFFFFFFFF) return fail(MEM_EINVAL, "n_points exceeds 2^32 per permutation");
    ev_int0[e] = (int64_t)ints.size();
    ev_np[e] = np;
    ev_norm[e] = p->desc.sigma_norm > 0.0 ? 1.0 / p->desc.sigma_norm : 1.0;
    for (int k = 0; k < np; ++k) {
      const int ig = (int)ints.size();
      FlowIntegral d{(int32_t)wch.size(), 0, per};
      for (int64_t s0 = 0; s0 < per; s0 += FP)
        sch.push_back(FlowChunk{ig, e, k, (int32_t)std::min<int64_t>(FP, per - s0), s0, tot + s0});
      for (int64_t s0 = 0; s0 < per; s0 += FW) {
        wch.push_back(FlowChunk{ig, e, k, (int32_t)std::min<int64_t>(FW, per - s0), s0, tot + s0});
        d.n_wchunks++;
      }
      tot += per;
      ints.push_back(d);
      int_proc.push_back(ev_proc[e]);
      int_ev.push_back(e);
      int_perm.push_back(k);
    }
  }
  if (tot > ((int64_t)1 << 28)) return fail(MEM_EINVAL, "a flow batch is limited to 2^28 points");
  const int n_int = (int)ints.size();

  hipStream_t s = (hipStream_t)o.stream;
  hipStream_t own = nullptr;
  const bool want_graph = o.use_graph != 0 && o.timing_out == nullptr;
  if (!s && want_graph) HIP_TRY(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
  struct StreamGuard { hipStream_t& s; ~StreamGuard() { if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); } } } sg{own};
  hipStream_t ws = own ? own : s;
  DevEvents dev(&work);
  mem_status st = dev.make(ev, ws);
  if (st != MEM_OK) return st;
  DevBuf b_procs(&work), b_iproc(&work), b_iev(&work), b_iperm(&work), b_ctx(&work), b_cvec(&work), b_ints(&work), b_sch(&work), b_wch(&work), b_parts(&work), b_state(&work), b_active(&work), b_evi0(&work), b_evnp(&work), b_evnorm(&work), b_done(&work), b_ctl(&work), b_x(&work), b_lq(&work), b_P(&work), b_err(&work), b_status(&work);
  HIP_TRY(b_procs.alloc(ptab.size() * sizeof(ProcParams)));
  HIP_TRY(b_iproc.alloc(n_int * sizeof(int32_t)));
  HIP_TRY(b_iev.alloc(n_int * sizeof(int32_t)));
  HIP_TRY(b_iperm.alloc(n_int * sizeof(int32_t)));
  HIP_TRY(b_ctx.alloc((size_t)n_int * FCTX * sizeof(float)));
  HIP_TRY(b_cvec.alloc((size_t)n_int * FLAYERS * FH * sizeof(float)));
  HIP_TRY(b_ints.alloc(ints.size() * sizeof(FlowIntegral)));
  HIP_TRY(b_sch.alloc(sch.size() * sizeof(FlowChunk)));
  HIP_TRY(b_wch.alloc(wch.size() * sizeof(FlowChunk)));
  HIP_TRY(b_parts.alloc(wch.size() * 2 * sizeof(double)));
  HIP_TRY(b_state.alloc((size_t)n_int * FS_SIZE * sizeof(double)));
  HIP_TRY(b_active.alloc(n_int * sizeof(int32_t)));
  HIP_TRY(b_evi0.alloc(n_ev * sizeof(int64_t)));
  HIP_TRY(b_evnp.alloc(n_ev * sizeof(int32_t)));
  HIP_TRY(b_evnorm.alloc(n_ev * sizeof(double)));
  HIP_TRY(b_done.alloc(n_ev * sizeof(int32_t)));
  HIP_TRY(b_ctl.alloc(sizeof(Control)));
  HIP_TRY(b_x.alloc((size_t)tot * 8 * sizeof(float)));
  HIP_TRY(b_lq.alloc((size_t)tot * sizeof(float)));
  const bool out_dev = o.outputs_on_device != 0;
  if (!out_dev) {
    HIP_TRY(b_P.alloc(n_ev * sizeof(double)));
    HIP_TRY(b_err.alloc(n_ev * sizeof(double)));
    HIP_TRY(b_status.alloc(n_ev * sizeof(int32_t)));
  }
  HIP_TRY(hipMemcpyAsync(b_procs.p, ptab.data(), ptab.size() * sizeof(ProcParams), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_iproc.p, int_proc.data(), n_int * sizeof(int32_t), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_iev.p, int_ev.data(), n_int * sizeof(int32_t), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_iperm.p, int_perm.data(), n_int * sizeof(int32_t), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_ints.p, ints.data(), ints.size() * sizeof(FlowIntegral), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_sch.p, sch.data(), sch.size() * sizeof(FlowChunk), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_wch.p, wch.data(), wch.size() * sizeof(FlowChunk), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_evi0.p, ev_int0.data(), n_ev * sizeof(int64_t), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_evnp.p, ev_np.data(), n_ev * sizeof(int32_t), hipMemcpyHostToDevice, ws));
  HIP_TRY(hipMemcpyAsync(b_evnorm.p, ev_norm.data(), n_ev * sizeof(double), hipMemcpyHostToDevice, ws));
  const Control ctl0{0u, 0u, 0, 0u};
  HIP_TRY(hipMemcpyAsync(b_ctl.p, &ctl0, sizeof(Control), hipMemcpyHostToDevice, ws));
  {
    const int64_t ns = (int64_t)n_int * FS_SIZE;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, ws, b_state.as<double>(), ns, 0.0);
    hipLaunchKernelGGL(fill_i32_kernel, dim3((n_int + 255) / 256), dim3(256), 0, ws, b_active.as<int32_t>(),
                       (int64_t)n_int, 1);
    hipLaunchKernelGGL(fill_i32_kernel, dim3((n_ev + 255) / 256), dim3(256), 0, ws, b_done.as<int32_t>(),
                       (int64_t)n_ev, 0);
    hipLaunchKernelGGL(flow_ctx_kernel, dim3((n_int + 255) / 256), dim3(256), 0, ws, dev.view,
                       b_iev.as<int32_t>(), b_iperm.as<int32_t>(), n_int, b_ctx.as<float>());
    HIP_TRY(hipGetLastError());
  }
  st = flow_cvec(fl, b_ctx.as<float>(), n_int, b_cvec.as<float>(), ws);
  if (st != MEM_OK) return st;

  Control* ctl = b_ctl.as<Control>();
  const int ev_blocks = (n_ev + 255) / 256;
  auto wkernel = prec == MEM_FP32 ? flow_weight_kernel<float> : flow_weight_kernel<double>;
  std::vector<hipEvent_t> tev_s, tev_w;
  auto timed = [&](std::vector<hipEvent_t>* tv, bool on, auto&& launch) -> mem_status {
    hipEvent_t a = nullptr, b = nullptr;
    if (on) {
      HIP_TRY(hipEventCreate(&a));
      HIP_TRY(hipEventCreate(&b));
      tv->push_back(a);
      tv->push_back(b);
      HIP_TRY(hipEventRecord(a, ws));
    }
    launch();
    HIP_TRY(hipGetLastError());
    if (on) HIP_TRY(hipEventRecord(b, ws));
    return MEM_OK;
  };
  auto enqueue_iteration = [&](bool time_kernels) -> mem_status {
    hipLaunchKernelGGL(flow_iter_begin_kernel, dim3(1), dim3(64), 0, ws, &ctl->n_running);
    mem_status es = timed(&tev_s, time_kernels, [&] {
      hipLaunchKernelGGL(fl->mode == MEM_FLOW_BF16X2 ? flow_sample2_kernel<true> : flow_sample2_kernel<false>,
                         dim3((unsigned)sch.size()), dim3(FT), 0, ws, fl->P, fl->Wf,
                         b_cvec.as<float>(), b_sch.as<FlowChunk>(), o.seed, 0u, &ctl->iter, b_active.as<int32_t>(),
                         b_x.as<float>(), b_lq.as<float>());
    });
    if (es != MEM_OK) return es;
    es = timed(&tev_w, time_kernels, [&] {
      hipLaunchKernelGGL(wkernel, dim3((unsigned)wch.size()), dim3(kBlock), 0, ws, b_procs.as<ProcParams>(),
                         b_iproc.as<int32_t>(), dev.view, b_wch.as<FlowChunk>(), b_active.as<int32_t>(),
                         b_x.as<float>(), b_lq.as<float>(), (double*)nullptr, b_parts.as<double>());
    });
    if (es != MEM_OK) return es;
    hipLaunchKernelGGL(flow_finish_kernel, dim3((n_int + 255) / 256), dim3(256), 0, ws, b_ints.as<FlowIntegral>(),
                       b_parts.as<double>(), b_state.as<double>(), b_active.as<int32_t>(), &ctl->iter, n_int, thr,
                       o.iter_out);
    hipLaunchKernelGGL(flow_event_kernel, dim3(ev_blocks), dim3(256), 0, ws, b_evi0.as<int64_t>(),
                       b_evnp.as<int32_t>(), b_evnorm.as<double>(), b_state.as<double>(), b_active.as<int32_t>(), n_ev,
                       target_mode ? o.target_rel_err : 0.0, &ctl->iter, &ctl->n_running, 0, nullptr, nullptr,
                       nullptr, nullptr, b_done.as<int32_t>());
    hipLaunchKernelGGL(flow_iter_end_kernel, dim3(1), dim3(64), 0, ws, &ctl->iter);
    HIP_TRY(hipGetLastError());
    return MEM_OK;
  };

  struct EventsGuard {
    std::vector<hipEvent_t>& a; std::vector<hipEvent_t>& b;
    ~EventsGuard() { for (auto e : a) (void)hipEventDestroy(e); for (auto e : b) (void)hipEventDestroy(e); }
  } eg{tev_s, tev_w};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct GraphGuard {
    hipGraph_t& g; hipGraphExec_t& x;
    ~GraphGuard() { if (x) (void)hipGraphExecDestroy(x); if (g) (void)hipGraphDestroy(g); }
  } gg{graph, gexec};
  const bool use_graph = want_graph && ws != nullptr;
  if (use_graph) {
    HIP_TRY(hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal));
    mem_status cs = enqueue_iteration(false);
    hipGraph_t gcap = nullptr;
    hipError_t ce = hipStreamEndCapture(ws, &gcap);
    graph = gcap;
    if (cs != MEM_OK) return cs;
    if (ce != hipSuccess) return fail(MEM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    HIP_TRY(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
  }
  auto wall0 = std::chrono::steady_clock::now();
  for (int j = 0; j < iters; ++j) {
    if (use_graph) HIP_TRY(hipGraphLaunch(gexec, ws));
    else {
      mem_status es = enqueue_iteration(o.timing_out != nullptr);
      if (es != MEM_OK) return es;
    }
    if (target_mode || j == 0) {
      Control hc{};
      HIP_TRY(hipMemcpyAsync(&hc, ctl, sizeof(Control), hipMemcpyDeviceToHost, ws));
      HIP_TRY(hipStreamSynchronize(ws));
      if (hc.n_running == 0) break;
    }
  }
  double* P = out_dev ? p_out : b_P.as<double>();
  double* E = out_dev ? err_out : b_err.as<double>();
  int32_t* S = out_dev ? status_out : b_status.as<int32_t>();
  hipLaunchKernelGGL(flow_event_kernel, dim3(ev_blocks), dim3(256), 0, ws, b_evi0.as<int64_t>(), b_evnp.as<int32_t>(),
                     b_evnorm.as<double>(), b_state.as<double>(), b_active.as<int32_t>(), n_ev,
                     target_mode ? o.target_rel_err : 0.0, &ctl->iter, &ctl->n_running, 1, P, E, S, o.n_iter_out,
                     b_done.as<int32_t>());
  HIP_TRY(hipGetLastError());
  double n_evals = 0.0;
  {
    std::vector<double> hs((size_t)n_int * FS_SIZE);
    HIP_TRY(hipMemcpyAsync(hs.data(), b_state.p, hs.size() * sizeof(double), hipMemcpyDeviceToHost, ws));
    HIP_TRY(hipStreamSynchronize(ws));
    // the pooled points of every integral plus its pilot batch
    for (int i = 0; i < n_int; ++i) n_evals += hs[(size_t)i * FS_SIZE + FS_N] + (double)ints[i].n_points;
  }
  // events below the ESS threshold: VEGAS on a compact copy
  std::vector<int32_t> done(n_ev);
  HIP_TRY(hipMemcpyAsync(done.data(), b_done.p, n_ev * sizeof(int32_t), hipMemcpyDeviceToHost, ws));
  HIP_TRY(hipStreamSynchronize(ws));
  std::vector<int32_t> fb;
  for (int e = 0; e < n_ev; ++e) if (done[e] < 0) fb.push_back(e);
  double fb_timing[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (!fb.empty()) {
    // VEGAS on the same event set with every other event masked, so that a
    // fallback event sees the point stream of a plain VEGAS call
    const int nf = (int)fb.size();
    std::vector<int32_t> mask(n_ev, 0);
    for (int e : fb) mask[e] = 1;
    DevBuf b_idx(&work), b_fP(&work), b_fE(&work), b_fS(&work), b_fN(&work);
    HIP_TRY(b_idx.alloc(nf * sizeof(int32_t)));
    HIP_TRY(b_fP.alloc(n_ev * sizeof(double)));
    HIP_TRY(b_fE.alloc(n_ev * sizeof(double)));
    HIP_TRY(b_fS.alloc(n_ev * sizeof(int32_t)));
    HIP_TRY(b_fN.alloc(n_ev * sizeof(int32_t)));
    HIP_TRY(hipMemcpyAsync(b_idx.p, fb.data(), nf * sizeof(int32_t), hipMemcpyHostToDevice, ws));
    mem_integrate_opts o2 = o;
    o2.flow = nullptr;
    o2.stream = ws;
    o2.outputs_on_device = 1;
    o2.iter_out = nullptr;
    o2.grid_out = nullptr;
    o2.n_iter_out = b_fN.as<int32_t>();
    o2.timing_out = o.timing_out ? fb_timing : nullptr;
    st = integrate_vegas(ev, hyp, n_hyp, n_points, n_np, iters, o2, b_fP.as<double>(), b_fE.as<double>(),
                         b_fS.as<int32_t>(), mask.data(), work);
    if (st != MEM_OK) return st;
    hipLaunchKernelGGL(scatter_fallback_kernel, dim3((nf + 255) / 256), dim3(256), 0, ws, b_idx.as<int32_t>(), nf,
                       b_fP.as<double>(), b_fE.as<double>(), b_fS.as<int32_t>(), b_fN.as<int32_t>(), P, E, S,
                       o.n_iter_out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(ws));
  }
  if (!out_dev) {
    HIP_TRY(hipMemcpyAsync(p_out, P, n_ev * sizeof(double), hipMemcpyDeviceToHost, ws));
    HIP_TRY(hipMemcpyAsync(err_out, E, n_ev * sizeof(double), hipMemcpyDeviceToHost, ws));
    HIP_TRY(hipMemcpyAsync(status_out, S, n_ev * sizeof(int32_t), hipMemcpyDeviceToHost, ws));
  }
  HIP_TRY(hipStreamSynchronize(ws));
  if (o.timing_out) {
    double ms_w = 0.0, ms_s = 0.0;
    for (size_t i = 0; i + 1 < tev_w.size(); i += 2) {
      float t = 0.0f;
      HIP_TRY(hipEventElapsedTime(&t, tev_w[i], tev_w[i + 1]));
      ms_w += t;
    }
    for (size_t i = 0; i + 1 < tev_s.size(); i += 2) {
      float t = 0.0f;
      HIP_TRY(hipEventElapsedTime(&t, tev_s[i], tev_s[i + 1]));
      ms_s += t;
    }
    o.timing_out[0] = ms_w + fb_timing[0];
    o.timing_out[1] = (double)(tev_w.size() / 2) + fb_timing[1];
    o.timing_out[2] = n_evals + fb_timing[2];
    o.timing_out[3] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
    o.timing_out[4] = ms_s;
    o.timing_out[5] = (double)(tev_s.size() / 2);
    o.timing_out[6] = n_evals;
    o.timing_out[7] = fb_timing[2];
  }
  return MEM_OK;
}

extern "C" const char* mem_status_string(mem_status s)
{
  switch (s) {
    case MEM_OK: return "ok";
    case MEM_EINVAL: return "invalid argument";
    case MEM_ENOMEM: return "out of memory";
    case MEM_EDEVICE: return "device error";
    case MEM_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

extern "C" mem_status mem_last_error(char* buf, size_t n)
{
  if (!buf || n == 0) return MEM_EINVAL;
  std::snprintf(buf, n, "%s", g_last_error.c_str());
  return MEM_OK;
}
