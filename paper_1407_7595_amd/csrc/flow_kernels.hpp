// Kernels of the learned proposal: context features, the per-integral
// projection of the context through the first layer, BF16 operand copies,
// sampling (inverse pass, x = T^-1(z) with log q), proposal weights
// f(x)/q(x), training forward with a tape, training backward, Adam.
//
// Work unit of the sampling and training kernels: 128 points (a 4-wave
// workgroup, 32 points per wave).  Per coupling layer: the first layer's
// 4 conditioning inputs on VALU (the 24 context inputs are folded into a
// per-integral bias), the two 128-wide layers on MFMA from LDS, the spline
// on VALU with two threads per point.
#pragma once
#include "device_common.hpp"
#include "flow.hpp"
#include "process.hpp"
#include "kernels.hpp"
#include "sl.hpp"
#include "tt.hpp"
#include "../../include/mem.h"

namespace memk {

constexpr int FP = 128;            // points per workgroup
constexpr int FT = 256;            // threads per workgroup

struct FlowChunk {
  int32_t integral;   // index into the context / point tables
  int32_t event;
  int32_t perm;
  int32_t count;      // <= FP
  int64_t start;      // first point index inside the integral
  int64_t out;        // first output slot
};

// ------------------------------------------------------------- setup --
__global__ void flow_ctx_kernel(EventsView ev, const int32_t* __restrict__ event, const int32_t* __restrict__ perm,
                                int n, float* __restrict__ ctx)
{
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double o[4][4];
  const int e = event[i], pm = perm[i];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int obj = k < 2 ? (pm ? 1 - k : k) : k;
    ev.load(obj, e, o[k][0], o[k][1], o[k][2], o[k][3]);
  }
  flow_context(o[0], o[1], o[2], o[3], ctx + (int64_t)i * FCTX);
}

// cvec[i][l][o] = b1_l[o] + sum_j W1_l[o][4 + j] ctx_i[j]
__global__ void flow_cvec_kernel(const float* __restrict__ P, const float* __restrict__ ctx, int n,
                                 float* __restrict__ cvec)
{
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * FLAYERS * FH) return;
  const int o = (int)(t % FH), l = (int)((t / FH) % FLAYERS);
  const int64_t i = t / (FH * FLAYERS);
  const float* W1 = P + (int64_t)l * FPER + F_W1;
  float s = P[(int64_t)l * FPER + F_B1 + o];
#pragma unroll
  for (int j = 0; j < FCTX; ++j) s += W1[o * FIN + 4 + j] * ctx[i * FCTX + j];
  cvec[t] = s;
}

// bf16 operand copies of W2 and W3 (and their transposes), W3 padded to 96
__global__ void flow_convert_kernel(const float* __restrict__ P, uint16_t* __restrict__ Wb)
{
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)FLAYERS * FB_PER) return;
  const int l = (int)(t / FB_PER), r = (int)(t % FB_PER);
  const float* L = P + (int64_t)l * FPER;
  float v = 0.0f;
  if (r < FB_W2T) { int n = r / FH, k = r % FH; v = L[F_W2 + n * FH + k]; }
  else if (r < FB_W3) { int q = r - FB_W2T, k = q / FH, n = q % FH; v = L[F_W2 + n * FH + k]; }
  else if (r < FB_W3T) { int q = r - FB_W3, n = q / FH, k = q % FH; v = n < FOUT ? L[F_W3 + n * FH + k] : 0.0f; }
  else { int q = r - FB_W3T, k = q / FOUTP, n = q % FOUTP; v = n < FOUT ? L[F_W3 + n * FH + k] : 0.0f; }
  Wb[t] = f2bf(v);
}

// ----------------------------------------------------- shared layer --
// LDS of the sampling / forward kernels.  h1 is dead once the second
// layer has been formed, so theta shares its space.  X2: every activation
// is held as two BF16 terms, hi = bf16(h) and lo = bf16(h - hi) (second
// half of h1 / h2), and each product is formed from both.
template <bool X2>
struct __align__(16) FlowSmem {
  static constexpr int NA = X2 ? 2 : 1;
  float v[FP][8];
  float logq[FP];
  int32_t sint[FP];         // integral of each point (training)
  union {
    uint16_t h1[NA * FP * FH];   // [part][p][k]
    float th[FP * FOUTP];        // [p][n]
  };
  uint16_t h2[NA * FP * FH];     // [part][p][k]
  float cv[FH];                  // this layer's context bias (one integral per workgroup)
};

template <bool X2>
__device__ __forceinline__ void store_act(uint16_t* h, int idx, float v)
{
  const uint16_t hi = f2bf(v);
  h[idx] = hi;
  if constexpr (X2) h[FP * FH + idx] = f2bf(v - bf2f(hi));
}

// h1 = silu(cvec + W1[:, :4] v_B) for all points of the workgroup.  cvec_l
// (training, points of many integrals): the layer's rows, indexed by
// S.sint; null: the LDS copy S.cv.
template <bool X2>
__device__ __forceinline__ void layer_h1(const float* __restrict__ L, const int (&B)[4], FlowSmem<X2>& S,
                                         const float* __restrict__ cvec_l, float* a1_tape, int64_t tape_stride)
{
  // thread t: hidden unit o = t % 128, points p = t / 128 + 2 q
  const int o = threadIdx.x % FH;
  const float w0 = L[F_W1 + o * FIN + 0], w1 = L[F_W1 + o * FIN + 1];
  const float w2 = L[F_W1 + o * FIN + 2], w3 = L[F_W1 + o * FIN + 3];
  for (int q = 0; q < FP / 2; ++q) {
    const int p = threadIdx.x / FH + 2 * q;
    const float c = cvec_l ? cvec_l[(int64_t)S.sint[p] * FLAYERS * FH + o] : S.cv[o];
    const float a = c + w0 * S.v[p][B[0]] + w1 * S.v[p][B[1]] + w2 * S.v[p][B[2]] + w3 * S.v[p][B[3]];
    if (a1_tape) a1_tape[(int64_t)p * tape_stride + o] = a;
    store_act<X2>(S.h1, p * FH + o, silu(a));
  }
}

// acc += act x W (act from LDS, one or two BF16 parts)
template <bool X2>
__device__ __forceinline__ void act_tile(const uint16_t* act, const uint16_t* Wt, int ldw, int m0, int n0, int K,
                                         f32x16& acc)
{
  mfma_tile(act, FH, Wt, ldw, m0, n0, K, acc);
  if constexpr (X2) mfma_tile(act + FP * FH, FH, Wt, ldw, m0, n0, K, acc);
}

// h2 = silu(W2 h1 + b2) and theta = W3 h2 + b3 on MFMA; wave w owns points
// [32 w, 32 w + 32).
template <bool X2>
__device__ __forceinline__ void layer_mlp_mfma(const float* __restrict__ L, const uint16_t* __restrict__ Wb,
                                               FlowSmem<X2>& S, float* a2_tape, int64_t tape_stride)
{
  const int w = threadIdx.x / kWave;
  const int m0 = 32 * w;
  f32x16 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) { zero16(acc[t]); act_tile<X2>(S.h1, Wb + FB_W2, FH, m0, 32 * t, FH, acc[t]); }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int p = m0 + mfma_row(r), n = 32 * t + mfma_col();
      const float a = acc[t][r] + L[F_B2 + n];
      if (a2_tape) a2_tape[(int64_t)p * tape_stride + n] = a;
      store_act<X2>(S.h2, p * FH + n, silu(a));
    }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 3; ++t) { zero16(acc[t]); act_tile<X2>(S.h2, Wb + FB_W3, FH, m0, 32 * t, FH, acc[t]); }
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int p = m0 + mfma_row(r), n = 32 * t + mfma_col();
      S.th[p * FOUTP + n] = n < FOUT ? acc[t][r] + L[F_B3 + n] : 0.0f;
    }
  __syncthreads();
}

// w = f(x) / q(x|c) for flow points of the ttbar dilepton process; per
// chunk (up to FW points of one integral) sum w and sum w^2.  A point at
// x_d = 1 (the spline's upper edge in FP32) is moved just inside the cube.
constexpr int FW = 2048;
template <class T>
__global__ __launch_bounds__(kBlock, MEM_TT_WAVES) void flow_weight_kernel(
    const ProcParams* __restrict__ pp_tab, const int32_t* __restrict__ int_proc, EventsView ev,
    const FlowChunk* __restrict__ chunks, const int32_t* __restrict__ active, const float* __restrict__ x,
    const float* __restrict__ lq, double* __restrict__ w_out, double* __restrict__ parts)
{
  __shared__ double red[2 * kBlock / kWave];
  const FlowChunk ch = chunks[blockIdx.x];
  if (active && !active[ch.integral]) return;
  const ProcParams pp = pp_tab[int_proc[ch.integral]];
  TTEvent e;
  tt_load(ev, ch.event, ch.perm, e);
  double s1 = 0.0, s2 = 0.0;
  for (int k = threadIdx.x; k < ch.count; k += kBlock) {
    double xx[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) xx[d] = fmin((double)x[(ch.out + k) * 8 + d], 0.99999994);
    const double f = tt_integrand<T>(pp, e, xx, nullptr);
    const double w = f == 0.0 ? 0.0 : f * exp(-(double)lq[ch.out + k]);
    if (w_out) w_out[ch.out + k] = w;
    s1 += w;
    s2 += w * w;
  }
  block_reduce2<0>(s1, s2, red);
  if (threadIdx.x == 0) { parts[2 * blockIdx.x] = s1; parts[2 * blockIdx.x + 1] = s2; }
}

// Per-integral state of a flow integration (FP64).
enum { FS_S1 = 0, FS_S2, FS_N, FS_NONFINITE, FS_ESS, FS_FALLBACK, FS_SIZE = 8 };

struct FlowIntegral {
  int32_t wchunk0, n_wchunks;   // weight chunks of the integral
  int64_t n_points;             // per batch
};

// Fold one batch into every active integral (chunk partials in a fixed
// order).  The first batch is a pilot: its ESS/N = (sum w)^2 / (N sum w^2)
// decides whether the integral stays with the proposal (below the threshold
// it is handed to VEGAS), and its sums are left out of the estimate.  A
// batch that passed the test is more likely to have missed the large
// weights, so pooling it would bias the kept integrals low; the later
// batches are independent of the decision.
__global__ void flow_finish_kernel(const FlowIntegral* __restrict__ ints, const double* __restrict__ parts,
                                   double* __restrict__ state, int32_t* __restrict__ active,
                                   const uint32_t* __restrict__ iter_p, int n_int, double ess_thr,
                                   double* __restrict__ iter_out)
{
  const int ig = blockIdx.x * blockDim.x + threadIdx.x;
  if (ig >= n_int || !active[ig]) return;
  const FlowIntegral in = ints[ig];
  double s1 = 0.0, s2 = 0.0;
  for (int c = 0; c < in.n_wchunks; ++c) { s1 += parts[2 * (in.wchunk0 + c)]; s2 += parts[2 * (in.wchunk0 + c) + 1]; }
  double* st = state + (int64_t)ig * FS_SIZE;
  const double N = (double)in.n_points;
  if (!isfinite(s1) || !isfinite(s2)) st[FS_NONFINITE] = 1.0;
  const uint32_t iter = *iter_p;
  if (iter == 0) {
    const double ess = s2 > 0.0 ? s1 * s1 / (N * s2) : 0.0;
    st[FS_ESS] = ess;
    if (!(ess >= ess_thr)) { st[FS_FALLBACK] = 1.0; active[ig] = 0; }
  } else {
    st[FS_S1] += s1;
    st[FS_S2] += s2;
    st[FS_N] += N;
  }
  if (iter_out) {
    const double I = s1 / N;
    double var = (s2 / N - I * I) / (N - 1.0);
    iter_out[((int64_t)iter * n_int + ig) * 2 + 0] = I;
    iter_out[((int64_t)iter * n_int + ig) * 2 + 1] = var > 0.0 ? var : 0.0;
  }
}

// Pooled estimate of one flow integral: every batch after the pilot is
// drawn from the same proposal, so their points enter one mean and one
// variance.
__device__ __forceinline__ void flow_estimate(const double* st, double& I, double& var)
{
  const double N = st[FS_N];
  I = N > 0.0 ? st[FS_S1] / N : 0.0;
  var = N > 1.0 ? (st[FS_S2] / N - I * I) / (N - 1.0) : 0.0;
  if (var < 0.0) var = 0.0;
}

// Per event: an event with a permutation below the ESS threshold goes to
// VEGAS as a whole (done = -1); otherwise it stops once err <= target P
// (from the second batch on) -- or writes the outputs (final pass).
__global__ void flow_event_kernel(const int64_t* __restrict__ ev_int0, const int32_t* __restrict__ ev_nperm,
                                  const double* __restrict__ ev_norm, const double* __restrict__ state,
                                  int32_t* __restrict__ active, int n_events, double target,
                                  uint32_t* __restrict__ iter_p, int32_t* __restrict__ n_running, int final_pass,
                                  double* P, double* err, int32_t* status, int32_t* n_iter_used,
                                  int32_t* __restrict__ ev_done)
{
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_events) return;
  const uint32_t iter = *iter_p;
  const int64_t i0 = ev_int0[e];
  const int np = ev_nperm[e];
  double s = 0.0, v = 0.0;
  bool bad = false, fb = false;
  for (int k = 0; k < np; ++k) {
    const double* st = state + (i0 + k) * FS_SIZE;
    double I, var;
    flow_estimate(st, I, var);
    s += I;
    v += var;
    if (st[FS_NONFINITE] != 0.0 || !isfinite(I)) bad = true;
    if (st[FS_FALLBACK] != 0.0) fb = true;
  }
  const double norm = ev_norm[e];
  const double p = norm * s / np, sd = norm * sqrt(v) / np;
  if (!final_pass) {
    if (ev_done[e] == 0) {
      if (fb) {
        ev_done[e] = -1;
        for (int k = 0; k < np; ++k) active[i0 + k] = 0;
      } else if (target > 0.0 && iter >= 1 && p > 0.0 && sd <= target * p) {
        ev_done[e] = (int32_t)iter + 1;
        for (int k = 0; k < np; ++k) active[i0 + k] = 0;
      }
    }
    if (ev_done[e] == 0) atomicAdd(n_running, 1);
    return;
  }
  int32_t stt = MEM_EV_OK;
  if (ev_done[e] < 0) { P[e] = 0.0; err[e] = 0.0; stt = MEM_EV_FLOW_FALLBACK; }
  else {
    P[e] = p;
    err[e] = sd;
    if (bad) stt = MEM_EV_NONFINITE;
    else if (s == 0.0) stt = MEM_EV_ZERO_INTEGRAND;
    else if (target > 0.0 && ev_done[e] == 0) stt = MEM_EV_NOT_CONVERGED;
  }
  status[e] = stt;
  if (n_iter_used) n_iter_used[e] = ev_done[e] > 0 ? ev_done[e] : (int32_t)iter;
}

__global__ void flow_iter_begin_kernel(int32_t* n_running) { if (threadIdx.x == 0) *n_running = 0; }
__global__ void flow_iter_end_kernel(uint32_t* iter_p) { if (threadIdx.x == 0) *iter_p += 1u; }

// ------------------------------------------------ training samples --
// Points of an adapted VEGAS grid with their weights w = f(x) J(x): the
// density of x is 1/J, so w/sum(w) weights each point by its share of the
// integrand (the flow's training target).  Thread per point.
template <int KIND, int D, class T>
__global__ __launch_bounds__(kBlock, KIND == kTTH ? 2 : MEM_TT_WAVES) void capture_kernel(
    ProcParams pp, EventsView ev, const int32_t* __restrict__ event, const int32_t* __restrict__ perm,
    int n_int, const double* __restrict__ grids, int64_t n_per, uint64_t seed, uint32_t iter,
    float* __restrict__ xo, float* __restrict__ wo)
{
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= (int64_t)n_int * n_per) return;
  const int ig = (int)(idx / n_per);
  const int64_t k = idx - (int64_t)ig * n_per;
  const int e = event[ig], pm = perm[ig];
  double u[D], x[D];
  int bin[D];
  point_uniforms<D>(seed, (uint32_t)k, iter, (uint32_t)e, (uint32_t)pm, u);
  const double jac = vegas_map<D>(grids + (int64_t)ig * D * (kBins + 1), u, x, bin);
  double f = 0.0;
  if constexpr (KIND == kTT) {
    TTEvent te;
    tt_load(ev, e, pm, te);
    f = tt_integrand<T>(pp, te, x, nullptr);
  } else if constexpr (KIND == kSL) {
    SLEvent se;
    sl_load(ev, ev.charge, e, pm, se);
    f = sl_integrand<T>(pp, se, x, nullptr);
  } else if constexpr (KIND == kTTH) {
    TTHEvent he;
    tth_load(ev, ev.charge, e, pm, he);
    f = tth_integrand<T>(pp, he, x, nullptr);
  } else {
    DYEvent de;
    dy_load(ev, e, de);
    f = dy_integrand(pp, de, x);
  }
#pragma unroll
  for (int d = 0; d < D; ++d) xo[idx * D + d] = (float)x[d];
  wo[idx] = (float)(f * jac);
}

// w /= sum of the integral's w (one workgroup per integral; zero sums stay 0)
__global__ __launch_bounds__(kBlock) void normalise_kernel(float* __restrict__ w, int64_t n_per)
{
  __shared__ double red[2 * kBlock / kWave];
  float* wi = w + (int64_t)blockIdx.x * n_per;
  double s = 0.0, dummy = 0.0;
  for (int64_t k = threadIdx.x; k < n_per; k += kBlock) s += (double)wi[k];
  block_reduce2<0>(s, dummy, red);
  __shared__ double tot;
  if (threadIdx.x == 0) tot = s;
  __syncthreads();
  const double t = tot;
  if (t > 0.0)
    for (int64_t k = threadIdx.x; k < n_per; k += kBlock) wi[k] = (float)((double)wi[k] / t);
}

// loss = -sum_i wt_i log q_i (FP64 partial per workgroup, summed on the host)
__global__ __launch_bounds__(kBlock) void flow_loss_kernel(const float* __restrict__ wt, const float* __restrict__ lq,
                                                           int64_t n, double* __restrict__ parts)
{
  __shared__ double red[2 * kBlock / kWave];
  double s = 0.0, dummy = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    s -= (double)wt[i] * (double)lq[i];
  block_reduce2<0>(s, dummy, red);
  if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

// VEGAS results (full-size arrays) of the fallback events into the outputs
__global__ void scatter_fallback_kernel(const int32_t* __restrict__ idx, int n, const double* __restrict__ Pf,
                                        const double* __restrict__ Ef, const int32_t* __restrict__ Sf,
                                        const int32_t* __restrict__ Nf, double* P, double* err, int32_t* status,
                                        int32_t* n_iter_used)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e = idx[i];
  P[e] = Pf[e];
  err[e] = Ef[e];
  status[e] = Sf[e] == MEM_EV_OK ? MEM_EV_FLOW_FALLBACK : Sf[e];
  if (n_iter_used) n_iter_used[e] = Nf[e];
}

// ---------------------------------------------------------- training --
// Tape per sample and layer: layer input vector (8), a1 (128), a2 (128),
// theta (96).
constexpr int FTAPE = 8 + FH + FH + FOUTP;

// Forward T(x) for training samples (any integrals), writing the tape and
// log q.  cvec holds the context projections of contexts ctx0, ctx0 + 1, ..
template <bool X2>
__global__ __launch_bounds__(FT) void flow_train_fwd_kernel(const float* __restrict__ P,
                                                            const uint16_t* __restrict__ Wb,
                                                            const float* __restrict__ cvec,
                                                            const int32_t* __restrict__ sint, int32_t ctx0,
                                                            const float* __restrict__ xs, int n,
                                                            float* __restrict__ tape, float* __restrict__ lq)
{
  __shared__ FlowSmem<X2> S;
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * FP;
  if (t < FP) {
    const int64_t i = base + t;
#pragma unroll
    for (int d = 0; d < 8; ++d) S.v[t][d] = i < n ? xs[i * 8 + d] : 0.5f;
    S.logq[t] = 0.0f;
    S.sint[t] = (i < n ? sint[i] : sint[0]) - ctx0;
  }
  __syncthreads();
  for (int l = 0; l < FLAYERS; ++l) {
    if (l == 3 && t < FP) {
#pragma unroll
      for (int d = 0; d < 4; ++d) { float x = S.v[t][d]; S.v[t][d] = S.v[t][7 - d]; S.v[t][7 - d] = x; }
    }
    __syncthreads();
    int A[4], B[4];
    flow_masks(l, A, B);
    const float* L = P + (int64_t)l * FPER;
    float* tp = tape + (base * FLAYERS + l) * FTAPE;   // sample p at tp + p * FLAYERS * FTAPE
    const int64_t stride = (int64_t)FLAYERS * FTAPE;
    if (t < FP) {
#pragma unroll
      for (int d = 0; d < 8; ++d) tp[t * stride + d] = S.v[t][d];
    }
    layer_h1(L, B, S, cvec + l * FH, tp + 8, stride);
    __syncthreads();
    layer_mlp_mfma(L, Wb + (int64_t)l * FB_PER, S, tp + 8 + FH, stride);
    for (int q = t; q < FP * FOUTP; q += FT) {
      const int p = q / FOUTP, nn = q % FOUTP;
      tp[p * stride + 8 + 2 * FH + nn] = S.th[q];
    }
    {
      const int p = t >> 1, j0 = 2 * (t & 1);
      float lsum = 0.0f;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        Spline sp;
        spline_make(&S.th[p * FOUTP + 23 * (j0 + jj)], sp);
        float ld;
        const int a = A[j0 + jj];
        S.v[p][a] = spline_fwd(sp, S.v[p][a], ld);
        lsum += ld;
      }
      lsum += __shfl_xor(lsum, 1, kWave);
      if ((t & 1) == 0) S.logq[p] += lsum;
    }
    __syncthreads();
  }
  if (t < FP && base + t < n) lq[base + t] = S.logq[t];
}

// d(y, log dy/dx) of one spline position w.r.t. its 23 logits and x.
__device__ __forceinline__ void spline_backward(const float* th, float x, float gy, float gl, float* gth,
                                                float& gx)
{
  const float m = 1e-3f, cw = 1.0f - FK * 1e-3f, c0 = 0.53974242f;
  float mw = th[0], mh = th[FK];
#pragma unroll
  for (int k = 1; k < FK; ++k) { mw = fmaxf(mw, th[k]); mh = fmaxf(mh, th[FK + k]); }
  float pw[FK], ph[FK], sw = 0.0f, sh = 0.0f;
#pragma unroll
  for (int k = 0; k < FK; ++k) { pw[k] = __expf(th[k] - mw); sw += pw[k]; ph[k] = __expf(th[FK + k] - mh); sh += ph[k]; }
  // knots exactly as the forward pass forms them (same bin for x)
  const float kiw = cw * frcp(sw), kih = cw * frcp(sh);
  float xk[FK + 1], yk[FK + 1], d[FK + 1];
  xk[0] = 0.0f;
  yk[0] = 0.0f;
#pragma unroll
  for (int k = 0; k < FK; ++k) { xk[k + 1] = xk[k] + m + pw[k] * kiw; yk[k + 1] = yk[k] + m + ph[k] * kih; }
  xk[FK] = 1.0f;
  yk[FK] = 1.0f;
  const float isw = frcp(sw), ish = frcp(sh);
#pragma unroll
  for (int k = 0; k < FK; ++k) { pw[k] *= isw; ph[k] *= ish; }
  d[0] = 1.0f; d[FK] = 1.0f;
#pragma unroll
  for (int k = 1; k < FK; ++k) d[k] = m + softplus(th[2 * FK + k - 1] + c0);
  int kb = 0;
#pragma unroll
  for (int k = 1; k < FK; ++k) if (x >= xk[k]) kb = k;
  float w = 0, h = 0, x0 = 0, d0 = 0, d1 = 0;
#pragma unroll
  for (int k = 0; k < FK; ++k)
    if (k == kb) { w = xk[k + 1] - xk[k]; h = yk[k + 1] - yk[k]; x0 = xk[k]; d0 = d[k]; d1 = d[k + 1]; }
  const float iw = frcp(w);
  const float t = (x - x0) * iw, omt = 1.0f - t, sk = h * iw;
  const float g = d1 + d0 - 2.0f * sk;
  const float den = sk + g * t * omt, nu = sk * t * t + d0 * t * omt;
  const float nd = d1 * t * t + 2.0f * sk * t * omt + d0 * omt * omt;
  const float iden = frcp(den), ind = frcp(nd);
  const float id2 = iden * iden;
  const float dy_dt = h * ((2.0f * sk * t + d0 * (1.0f - 2.0f * t)) * den - nu * g * (1.0f - 2.0f * t)) * id2;
  const float dy_dsk = h * (t * t * den - nu * (1.0f - 2.0f * t * omt)) * id2;
  const float dy_dh = nu * iden;
  const float dy_dd0 = h * (t * omt * den - nu * t * omt) * id2;
  const float dy_dd1 = -h * nu * t * omt * id2;
  const float dl_dt = (2.0f * d1 * t + 2.0f * sk * (1.0f - 2.0f * t) - 2.0f * d0 * omt) * ind
                    - 2.0f * g * (1.0f - 2.0f * t) * iden;
  const float dl_dsk = 2.0f * frcp(sk) + 2.0f * t * omt * ind - 2.0f * (1.0f - 2.0f * t * omt) * iden;
  const float dl_dd0 = omt * omt * ind - 2.0f * t * omt * iden;
  const float dl_dd1 = t * t * ind - 2.0f * t * omt * iden;
  // combine the two outputs with their incoming gradients
  const float c_t = gy * dy_dt + gl * dl_dt, c_sk = gy * dy_dsk + gl * dl_dsk;
  gx = c_t * iw;
  const float g_w = c_t * (-t * iw) + c_sk * (-h * iw * iw);
  const float g_x0 = -c_t * iw;
  const float g_h = gy * dy_dh + c_sk * iw;
  float gw[FK], gh[FK];
#pragma unroll
  for (int k = 0; k < FK; ++k) {
    gw[k] = (k == kb ? g_w : 0.0f) + (k < kb ? g_x0 : 0.0f);
    gh[k] = (k == kb ? g_h : 0.0f) + (k < kb ? gy : 0.0f);
  }
  float aw = 0.0f, ah = 0.0f;
#pragma unroll
  for (int k = 0; k < FK; ++k) { aw += gw[k] * pw[k]; ah += gh[k] * ph[k]; }
#pragma unroll
  for (int k = 0; k < FK; ++k) { gth[k] = cw * pw[k] * (gw[k] - aw); gth[FK + k] = cw * ph[k] * (gh[k] - ah); }
#pragma unroll
  for (int k = 1; k < FK; ++k) {
    const float sg = frcp(1.0f + __expf(-(th[2 * FK + k - 1] + c0)));
    const float gd = (k == kb ? gy * dy_dd0 + gl * dl_dd0 : 0.0f) + (k == kb + 1 ? gy * dy_dd1 + gl * dl_dd1 : 0.0f);
    gth[2 * FK + k - 1] = gd * sg;
  }
}

// LDS of the backward kernel (phases reuse one region)
constexpr int FHP = FH + 1;   // padded row of the first-layer gradient (bank spread)
constexpr int FW1S = FIN + 1; // first-layer gradient terms per unit: W1 row and b1
// row of the transposed activations h1T, h2T [unit][sample]: padded by 8 so
// that the transposing writes (consecutive units, one sample) spread over
// the banks while rows stay 16-byte aligned for the matrix-core loads
constexpr int FPT = FP + 8;
struct __align__(16) FlowBwdSmem {
  float gv[FP][8];          // dL/d(layer output vector)
  float gl[FP];             // dL/d(log q) per sample (= -weight)
  float ctx_in[FP][4];      // the layer's conditioning inputs
  float ctx[FP][FCTX];      // the samples' contexts
  float gb2[FT / kWave][FH];  // per-wave partial sums of the second-layer bias gradient
  union {
    struct { uint16_t g[FP * FOUTP]; uint16_t gT[FOUTP * FP]; uint16_t h2T[FH * FPT]; } a;  // 82 KB
    struct { uint16_t g[FP * FH]; uint16_t gT[FH * FP]; uint16_t h1T[FH * FPT]; } b;        // 98 KB
    struct { float ga1[FP * FHP]; float w1[FH * FW1S]; } c;                               // 81 KB
  } u;
};

// hT[k][p] = bf16(silu(a[p][k])) for the tile's FP samples and FH units,
// a[p][k] = src[p * stride + k] in the tape.  Consecutive threads read one
// sample's consecutive units (coalesced); each thread first issues eight
// independent loads, then converts and stores them, so that one wave
// waits for the memory once per eight values.
__device__ __forceinline__ void transpose_act(const float* __restrict__ src, int64_t stride, uint16_t* hT)
{
  static_assert((FH * FP) % (8 * FT) == 0, "whole rounds of eight loads per thread");
  for (int q0 = threadIdx.x; q0 < FH * FP; q0 += 8 * FT) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * FT, p = q / FH, k = q % FH;
      v[u] = src[p * stride + k];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * FT, p = q / FH, k = q % FH;
      hT[k * FPT + p] = f2bf(silu(v[u]));
    }
  }
}

// The gradient slot of a workgroup is written by exactly one thread per
// entry, in the same order on every run: plain stores on the workgroup's
// first tile, additions on the later ones.
__device__ __forceinline__ void slot_add(float* g, float v, bool first) { *g = first ? v : *g + v; }

__device__ __forceinline__ void store_tile(float* dst, int ld, int m0, int n0, int mmax, int nmax, const f32x16& acc,
                                           bool first)
{
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + mfma_row(r), n = n0 + mfma_col();
    if (m < mmax && n < nmax) slot_add(dst + m * ld + n, acc[r], first);
  }
}

// Backward of L = -sum_i wt_i log q(x_i|c_i) through every layer (tape from
// flow_train_fwd_kernel).  Workgroup g takes the tiles of FP samples g,
// g + G, g + 2G, ... (G = gridDim.x) and accumulates their parameter
// gradient in its own slot part[g][FNP]; flow_grad_reduce_kernel then sums
// the slots in slot order, so the gradient is the same on every run (no
// atomics).
__global__ __launch_bounds__(FT) void flow_train_bwd_kernel(const float* __restrict__ P,
                                                            const uint16_t* __restrict__ Wb,
                                                            const float* __restrict__ ctx,
                                                            const int32_t* __restrict__ sint,
                                                            const float* __restrict__ wt, int n,
                                                            const float* __restrict__ tape,
                                                            float* __restrict__ part)
{
  __shared__ FlowBwdSmem S;
  const int t = threadIdx.x;
  const int n_tiles = (n + FP - 1) / FP;
  const int64_t stride = (int64_t)FLAYERS * FTAPE;
  const int wv = t / kWave, m0 = 32 * wv;
  float* slot = part + (int64_t)blockIdx.x * FNP;
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
  const bool first = tile == (int)blockIdx.x;
  const int64_t base = (int64_t)tile * FP;
  if (t < FP) {
#pragma unroll
    for (int d = 0; d < 8; ++d) S.gv[t][d] = 0.0f;
    S.gl[t] = base + t < n ? -wt[base + t] : 0.0f;
  }
  for (int q = t; q < FP * FCTX; q += FT) {
    const int p = q / FCTX, j = q % FCTX;
    S.ctx[p][j] = base + p < n ? ctx[(int64_t)sint[base + p] * FCTX + j] : 0.0f;
  }
  __syncthreads();
  for (int l = FLAYERS - 1; l >= 0; --l) {
    int A[4], B[4];
    flow_masks(l, A, B);
    const float* L = P + (int64_t)l * FPER;
    const uint16_t* W = Wb + (int64_t)l * FB_PER;
    float* G = slot + (int64_t)l * FPER;
    const float* tp = tape + (base * FLAYERS + l) * FTAPE;
    // ---- spline backward: g theta (bf16, both layouts) and the input gradient
    for (int q = t; q < FP * FOUTP; q += FT) { S.u.a.g[q] = 0; }
    for (int q = t; q < FOUTP * FP; q += FT) { S.u.a.gT[q] = 0; }
    __syncthreads();
    {
      const int p = t >> 1, j0 = 2 * (t & 1);
      const float* th = tp + p * stride + 8 + 2 * FH;
      float gin[2];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int j = j0 + jj, a = A[j];
        float gth[23], gx;
        spline_backward(th + 23 * j, tp[p * stride + a], S.gv[p][a], S.gl[p], gth, gx);
#pragma unroll
        for (int m = 0; m < 23; ++m) {
          const uint16_t b = f2bf(gth[m]);
          S.u.a.g[p * FOUTP + 23 * j + m] = b;
          S.u.a.gT[(23 * j + m) * FP + p] = b;
        }
        gin[jj] = gx;
      }
      __syncthreads();
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) S.gv[p][A[j0 + jj]] = gin[jj];
    }
    // h2 transposed (bf16) from the tape: consecutive threads read one
    // sample's consecutive units (coalesced) and write a column of h2T
    transpose_act(tp + 8 + FH, stride, S.u.a.h2T);
    __syncthreads();
    // gb3[n] = sum_p g[p][n] (rows of the transposed copy)
    if (t < FOUT) {
      float sb = 0.0f;
      for (int p = 0; p < FP; ++p) sb += bf2f(S.u.a.gT[t * FP + p]);
      slot_add(&G[F_B3 + t], sb, first);
    }
    // ---- gW3[n][k] += sum_p g[p][n] h2[p][k]: 3 x 4 tiles over the 4 waves
    for (int tile3 = wv; tile3 < 12; tile3 += 4) {
      const int tm = tile3 / 4, tn = tile3 % 4;
      f32x16 acc;
      zero16(acc);
      mfma_tile(S.u.a.gT, FP, S.u.a.h2T, FPT, 32 * tm, 32 * tn, FP, acc);
      store_tile(G + F_W3, FH, 32 * tm, 32 * tn, FOUT, FH, acc, first);
    }
    // ---- gh2[p][k] = sum_n g[p][n] W3[n][k]; ga2 = gh2 silu'(a2)
    f32x16 gh[4];
#pragma unroll
    for (int tn = 0; tn < 4; ++tn) { zero16(gh[tn]); mfma_tile(S.u.a.g, FOUTP, W + FB_W3T, FOUTP, m0, 32 * tn, FOUTP, gh[tn]); }
    __syncthreads();
    // (region b overwrites region a from here on)
#pragma unroll
    for (int tn = 0; tn < 4; ++tn) {
      float sb = 0.0f;   // this lane's column k over its 16 rows
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int p = m0 + mfma_row(r), k = 32 * tn + mfma_col();
        const float ga = gh[tn][r] * dsilu(tp[p * stride + 8 + FH + k]);
        const uint16_t b = f2bf(ga);
        S.u.b.g[p * FH + k] = b;
        S.u.b.gT[k * FP + p] = b;
        sb += ga;
      }
      sb += __shfl_xor(sb, 32, kWave);
      if ((t & 63) < 32) S.gb2[wv][32 * tn + mfma_col()] = sb;
    }
    transpose_act(tp + 8, stride, S.u.b.h1T);
    __syncthreads();
    // gb2: the four waves' sums in wave order
    if (t < FH) slot_add(&G[F_B2 + t], ((S.gb2[0][t] + S.gb2[1][t]) + S.gb2[2][t]) + S.gb2[3][t], first);
    // ---- gW2[o][k] += sum_p ga2[p][o] h1[p][k]: 4 x 4 tiles
    for (int tile2 = wv; tile2 < 16; tile2 += 4) {
      const int tm = tile2 / 4, tn = tile2 % 4;
      f32x16 acc;
      zero16(acc);
      mfma_tile(S.u.b.gT, FP, S.u.b.h1T, FPT, 32 * tm, 32 * tn, FP, acc);
      store_tile(G + F_W2, FH, 32 * tm, 32 * tn, FH, FH, acc, first);
    }
    // ---- gh1[p][k] = sum_o ga2[p][o] W2[o][k]
#pragma unroll
    for (int tn = 0; tn < 4; ++tn) { zero16(gh[tn]); mfma_tile(S.u.b.g, FH, W + FB_W2T, FH, m0, 32 * tn, FH, gh[tn]); }
    __syncthreads();
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int p = m0 + mfma_row(r), k = 32 * tn + mfma_col();
        S.u.c.ga1[p * FHP + k] = gh[tn][r] * dsilu(tp[p * stride + 8 + k]);
      }
    if (t < FP) {
#pragma unroll
      for (int j = 0; j < 4; ++j) S.ctx_in[t][j] = tp[t * stride + B[j]];
    }
    __syncthreads();
    // ---- first layer (VALU): gb1, gW1 (each unit's sums over the two
    //      halves of the samples, added in half order) and the
    //      conditioning-input gradient
    {
      const int o = t % FH, half = t / FH;
      float sb = 0.0f, sw[FIN];
#pragma unroll
      for (int j = 0; j < FIN; ++j) sw[j] = 0.0f;
      for (int p = half; p < FP; p += 2) {
        const float g1 = S.u.c.ga1[p * FHP + o];
        sb += g1;
#pragma unroll
        for (int j = 0; j < 4; ++j) sw[j] += g1 * S.ctx_in[p][j];
#pragma unroll
        for (int j = 0; j < FCTX; ++j) sw[4 + j] += g1 * S.ctx[p][j];
      }
      if (half == 1) {
#pragma unroll
        for (int j = 0; j < FIN; ++j) S.u.c.w1[o * FW1S + j] = sw[j];
        S.u.c.w1[o * FW1S + FIN] = sb;
      }
      __syncthreads();
      if (half == 0) {
#pragma unroll
        for (int j = 0; j < FIN; ++j) slot_add(&G[F_W1 + o * FIN + j], sw[j] + S.u.c.w1[o * FW1S + j], first);
        slot_add(&G[F_B1 + o], sb + S.u.c.w1[o * FW1S + FIN], first);
      }
    }
    if (t < FP) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float s = 0.0f;
#pragma unroll 8
        for (int o = 0; o < FH; ++o) s += S.u.c.ga1[t * FHP + o] * L[F_W1 + o * FIN + j];
        S.gv[t][B[j]] += s;
      }
    }
    __syncthreads();
    if (l == 3 && t < FP) {
#pragma unroll
      for (int d = 0; d < 4; ++d) { float x = S.gv[t][d]; S.gv[t][d] = S.gv[t][7 - d]; S.gv[t][7 - d] = x; }
    }
    __syncthreads();
  }
  }
}

// grad[i] = sum over the workgroup slots g = 0, 1, ... of part[g][i], in
// slot order.
__global__ void flow_grad_reduce_kernel(const float* __restrict__ part, int n_slots, float* __restrict__ grad)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= FNP) return;
  float s = 0.0f;
  for (int g = 0; g < n_slots; ++g) s += part[(int64_t)g * FNP + i];
  grad[i] = s;
}

// Adam on the FP32 master parameters (bias-corrected moments).
__global__ void flow_adam_kernel(float* __restrict__ P, float* __restrict__ g, float* __restrict__ m,
                                 float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                                 float c2)
{
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace memk
