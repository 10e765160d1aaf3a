// Learned importance-sampling proposal: a conditional rational-quadratic
// spline flow on [0,1]^8 (Durkan et al. 2019), trained and evaluated by
// BF16 MFMA kernels with FP32 accumulation.  The estimator f(x)/q(x) is
// unbiased for any proposal, so the flow only changes the variance; plain
// VEGAS (Sec. 2) remains the fallback.
//
// Definition (the same on every side by specification):
//  * T: x -> z in [0,1]^8 through 6 coupling layers; the coordinate order is
//    reversed before layer 3.  Layer l transforms positions {1,3,5,7}
//    (l even) or {0,2,4,6} (l odd), conditioned on the other four and on a
//    24-value event context.
//  * per layer an MLP 28 -> 128 -> 128 -> 92 (SiLU), input [conditioning
//    values ascending, context]; output per transformed position j: 8
//    width logits, 8 height logits, 7 interior-derivative logits at 23 j.
//  * widths, heights = 1e-3 + (1 - 8e-3) softmax; derivatives = 1e-3 +
//    softplus(logit + c0) with c0 = ln(e^(1-1e-3) - 1) (a zero output is
//    the identity); boundary derivatives 1.
//  * log q(x|c) = sum of log dz/dx over layers and transformed positions.
//  * parameters per layer, row-major (out x in): W1[128][28], b1, W2, b2,
//    W3[92][128], b3 (32 092 per layer).
//
// MFMA: v_mfma_f32_32x32x16_bf16.  A wave multiplies a 32-row tile of
// activations by a 32-column tile of weights; operands come from LDS (or
// L2) in bf16 with k contiguous.
#pragma once
#include "device_common.hpp"

namespace memk {

constexpr int FK = 8, FH = 128, FIN = 28, FOUT = 92, FOUTP = 96, FLAYERS = 6;
constexpr int FPER = FH * FIN + FH + FH * FH + FH + FOUT * FH + FOUT;   // 32 092
constexpr int FNP = FLAYERS * FPER;                                     // 192 552
constexpr int FCTX = 24;
// offsets inside one layer's parameters
constexpr int F_W1 = 0, F_B1 = FH * FIN, F_W2 = F_B1 + FH, F_B2 = F_W2 + FH * FH, F_W3 = F_B2 + FH,
              F_B3 = F_W3 + FOUT * FH;
// bf16 operand copies per layer: W2 [n][k], W2^T [k][n], W3 [n(96)][k], W3^T [k][n(96)]
constexpr int FB_W2 = 0, FB_W2T = FH * FH, FB_W3 = 2 * FH * FH, FB_W3T = 2 * FH * FH + FOUTP * FH,
              FB_PER = 2 * FH * FH + 2 * FOUTP * FH;

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float v)
{
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Reciprocal by the hardware approximation (1 ulp): the activations are
// rounded to BF16 (or split into two BF16 terms, ~2^-17), far coarser than
// the correctly rounded division this replaces (about ten instructions).
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float silu(float a) { return a * frcp(1.0f + __expf(-a)); }
__device__ __forceinline__ float dsilu(float a)
{
  const float s = frcp(1.0f + __expf(-a));
  return s * (1.0f + a * (1.0f - s));
}
__device__ __forceinline__ float softplus(float v) { return v > 20.0f ? v : log1pf(__expf(v)); }

// Row and column of accumulator register r of this lane in a 32x32 tile.
__device__ __forceinline__ int mfma_row(int r) { return 8 * (r >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (r & 3); }
__device__ __forceinline__ int mfma_col() { return threadIdx.x & 31; }

// acc += A[m0.., 0..K) x B[0..K, n0..): A(m, k) = A[m * lda + k],
// B(k, n) = Bt[n * ldb + k] (bf16, k contiguous), i.e.
// acc += A[m0:m0+32][0:K] Bt[n0:n0+32][0:K]^T on v_mfma_f32_32x32x16_bf16
// (K a multiple of 16, rows 16-byte aligned): lane i < 32 supplies row m0 + i
// (n0 + i) with k in [k0, k0 + 8), lane 32 + i the same row with k in
// [k0 + 8, k0 + 16).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short short8_t __attribute__((ext_vector_type(8)));
__device__ __forceinline__ void mfma_tile(const uint16_t* A, int lda, const uint16_t* Bt, int ldb, int m0, int n0,
                                          int K, f32x16& acc)
{
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, kq = (lane >> 5) * 8;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x8_t a = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const short8_t*>(A + (m0 + i) * lda + k0 + kq));
    const bf16x8_t b = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const short8_t*>(Bt + (n0 + i) * ldb + k0 + kq));
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
}

__device__ __forceinline__ void zero16(f32x16& a)
{
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = 0.0f;
}

// ------------------------------------------------------------ spline --
struct Spline {
  float xk[FK + 1], yk[FK + 1], d[FK + 1];
};

__device__ __forceinline__ void spline_make(const float* th, Spline& s)
{
  const float m = 1e-3f, cw = 1.0f - FK * 1e-3f;
  const float c0 = 0.53974242f;     // ln(e^(1-1e-3) - 1)
  float mw = th[0], mh = th[FK];
#pragma unroll
  for (int k = 1; k < FK; ++k) { mw = fmaxf(mw, th[k]); mh = fmaxf(mh, th[FK + k]); }
  float ew[FK], eh[FK], sw = 0.0f, sh = 0.0f;
#pragma unroll
  for (int k = 0; k < FK; ++k) { ew[k] = __expf(th[k] - mw); sw += ew[k]; eh[k] = __expf(th[FK + k] - mh); sh += eh[k]; }
  const float iw = cw * frcp(sw), ih = cw * frcp(sh);
  s.xk[0] = 0.0f; s.yk[0] = 0.0f;
#pragma unroll
  for (int k = 0; k < FK; ++k) { s.xk[k + 1] = s.xk[k] + m + ew[k] * iw; s.yk[k + 1] = s.yk[k] + m + eh[k] * ih; }
  s.xk[FK] = 1.0f; s.yk[FK] = 1.0f;
  s.d[0] = 1.0f; s.d[FK] = 1.0f;
#pragma unroll
  for (int k = 1; k < FK; ++k) s.d[k] = m + softplus(th[2 * FK + k - 1] + c0);
}

// bin parameters of the bin holding v among the given knots
struct Bin { float x0, w, y0, h, d0, d1; };
__device__ __forceinline__ Bin spline_bin(const Spline& s, float v, bool by_y)
{
  Bin b{s.xk[0], s.xk[1] - s.xk[0], s.yk[0], s.yk[1] - s.yk[0], s.d[0], s.d[1]};
#pragma unroll
  for (int k = 1; k < FK; ++k) {
    const float edge = by_y ? s.yk[k] : s.xk[k];
    if (v >= edge) b = Bin{s.xk[k], s.xk[k + 1] - s.xk[k], s.yk[k], s.yk[k + 1] - s.yk[k], s.d[k], s.d[k + 1]};
  }
  return b;
}

// forward: y(x), log dy/dx
__device__ __forceinline__ float spline_fwd(const Spline& s, float x, float& ld)
{
  const Bin b = spline_bin(s, x, false);
  const float iw = frcp(b.w);
  const float sk = b.h * iw, t = (x - b.x0) * iw, omt = 1.0f - t;
  const float g = b.d1 + b.d0 - 2.0f * sk;
  const float den = sk + g * t * omt;
  const float nd = b.d1 * t * t + 2.0f * sk * t * omt + b.d0 * omt * omt;
  ld = __logf(sk * sk * nd * frcp(den * den));
  return b.y0 + b.h * (sk * t * t + b.d0 * t * omt) * frcp(den);
}

// inverse: x(y) from the quadratic in t; log dy/dx at the returned x
__device__ __forceinline__ float spline_inv(const Spline& s, float y, float& ld)
{
  const Bin b = spline_bin(s, y, true);
  const float sk = b.h * frcp(b.w), dy = y - b.y0;
  const float g = b.d1 + b.d0 - 2.0f * sk;
  const float qa = b.h * (sk - b.d0) + dy * g;
  const float qb = b.h * b.d0 - dy * g;
  const float qc = -sk * dy;
  const float disc = fmaxf(qb * qb - 4.0f * qa * qc, 0.0f);
  const float t = fminf(fmaxf((2.0f * qc) * frcp(-qb - sqrtf(disc)), 0.0f), 1.0f);
  const float omt = 1.0f - t;
  const float den = sk + g * t * omt;
  const float nd = b.d1 * t * t + 2.0f * sk * t * omt + b.d0 * omt * omt;
  ld = __logf(sk * sk * nd * frcp(den * den));
  return fminf(fmaxf(b.x0 + t * b.w, 0.0f), 1.0f);
}

// ---------------------------------------------------------- context --
// Dilepton event context for assignment perm: jets in assignment order,
// l+, l-, their sum as (log(E/100), p/100), then -sum p_T as
// (log((|MET|+1)/100), MET_x/100, MET_y/100, 0).
__device__ __forceinline__ void flow_context(const double* o0, const double* o1, const double* o2,
                                             const double* o3, float* ctx)
{
  const double* o[4] = {o0, o1, o2, o3};
  double S[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int i = 0; i < 4; ++i) S[i] += o[k][i];
    ctx[4 * k] = (float)log(o[k][0] / 100.0);
#pragma unroll
    for (int i = 1; i < 4; ++i) ctx[4 * k + i] = (float)(o[k][i] / 100.0);
  }
  ctx[16] = (float)log(S[0] / 100.0);
#pragma unroll
  for (int i = 1; i < 4; ++i) ctx[16 + i] = (float)(S[i] / 100.0);
  const double mx = -S[1], my = -S[2];
  ctx[20] = (float)log((sqrt(mx * mx + my * my) + 1.0) / 100.0);
  ctx[21] = (float)(mx / 100.0);
  ctx[22] = (float)(my / 100.0);
  ctx[23] = 0.0f;
}

__device__ __forceinline__ void flow_masks(int l, int (&A)[4], int (&B)[4])
{
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    A[j] = (l & 1) ? 2 * j : 2 * j + 1;
    B[j] = (l & 1) ? 2 * j + 1 : 2 * j;
  }
}

}  // namespace memk
