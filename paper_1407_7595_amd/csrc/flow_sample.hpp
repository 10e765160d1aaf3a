// Sampling kernel of the learned proposal, laid out for CDNA4.
//
// One workgroup (4 wavefronts) maps 128 base points z to x = T^-1(z; c)
// with log q, one coupling layer at a time (inverse order):
//  1. h1 = silu(W1 [v_B, c] + b1) on VALU (the context part of W1 c + b1 is
//     a per-integral bias computed once), BF16 into a padded LDS tile;
//  2. a2 = W2 h1 on v_mfma_f32_32x32x16_bf16, split by output column: wave w
//     owns columns [32w, 32w + 32) for all 128 points, with its W2 slice
//     held in registers; A fragments are conflict-free 16-byte LDS reads;
//  3. h2 = silu(a2 + b2) back into the same LDS tile;
//  4. theta^T = W3 h2^T, split by point: wave w owns points [32w, 32w + 32)
//     and all 96 (92 used) rows; W3 fragments stream from L2 in fragment
//     order (one coalesced 16-byte load per lane);
//  5. the two lane halves of a column hold complementary rows of one
//     point's theta: one swap across the halves gives each lane the 46
//     logits of its two transformed positions, and the spline inverse runs
//     in registers (theta never touches LDS).
// LDS: 39 KB (BF16) / 73 KB (BF16X2), so two workgroups share a CU and one
// workgroup's matrix products overlap the other's VALU work.
#pragma once
#include "flow.hpp"
#include "flow_kernels.hpp"

namespace memk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short8 __attribute__((ext_vector_type(8)));

constexpr int HP = FH + 8;                      // padded LDS row (bf16): 272 B
// fragment-ordered weight copies per layer: W2 [n-tile 4][k-step 8][lane 64][8],
// W3 [m-tile 3][k-step 8][lane 64][8] (rows >= 92 zero)
constexpr int FS_W2 = 0, FS_W3 = 4 * 8 * 64 * 8, FS_PER = FS_W3 + 3 * 8 * 64 * 8;

// fragment-ordered copies: element e of lane l of block (tile, ks) is
// W[32 tile + (l & 31)][16 ks + 8 (l >> 5) + e]
__global__ void flow_swizzle_kernel(const float* __restrict__ P, uint16_t* __restrict__ Wf)
{
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)FLAYERS * FS_PER) return;
  const int l = (int)(t / FS_PER), r = (int)(t % FS_PER);
  const float* L = P + (int64_t)l * FPER;
  const bool w3 = r >= FS_W3;
  const int q = w3 ? r - FS_W3 : r;
  const int e = q & 7, lane = (q >> 3) & 63, ks = (q >> 9) & 7, tile = q >> 12;
  const int row = 32 * tile + (lane & 31), k = 16 * ks + 8 * (lane >> 5) + e;
  float v;
  if (w3) v = row < FOUT ? L[F_W3 + row * FH + k] : 0.0f;
  else v = L[F_W2 + row * FH + k];
  Wf[t] = f2bf(v);
}

template <bool X2>
struct __align__(16) FlowSampleSmem {
  static constexpr int NA = X2 ? 2 : 1;
  float v[FP][8];
  float logq[FP];
  float cv[FH];
  uint16_t h[NA][FP * HP];       // h1, then h2 (same tile)
};

__device__ __forceinline__ bf16x8 lds_frag(const uint16_t* base)
{
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const short8*>(base));
}

__device__ __forceinline__ bf16x8 glb_frag(const uint16_t* __restrict__ base)
{
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const short8*>(base));
}

template <bool X2>
__device__ __forceinline__ void put_act(FlowSampleSmem<X2>& S, int idx, float v)
{
  const __bf16 hi = (__bf16)v;
  S.h[0][idx] = __builtin_bit_cast(uint16_t, hi);
  if constexpr (X2) S.h[X2 ? 1 : 0][idx] = __builtin_bit_cast(uint16_t, (__bf16)(v - (float)hi));
}

template <bool X2>
__global__ __launch_bounds__(FT, 2) void flow_sample2_kernel(const float* __restrict__ P,
                                                              const uint16_t* __restrict__ Wf,
                                                              const float* __restrict__ cvec,
                                                              const FlowChunk* __restrict__ chunks, uint64_t seed,
                                                              uint32_t iter, const uint32_t* __restrict__ iter_p,
                                                              const int32_t* __restrict__ active,
                                                              float* __restrict__ xout, float* __restrict__ lqout)
{
  __shared__ FlowSampleSmem<X2> S;
  const FlowChunk ch = chunks[blockIdx.x];
  if (active && !active[ch.integral]) return;
  if (iter_p) iter = *iter_p;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6, col = lane & 31, half = lane >> 5;
  if (t < FP) {
    double u[8];
    point_uniforms<8>(seed, (uint32_t)(ch.start + t), iter, (uint32_t)ch.event, (uint32_t)ch.perm, u, 8u);
#pragma unroll
    for (int d = 0; d < 8; ++d) S.v[t][d] = fminf((float)u[d], 0.99999994f);
    S.logq[t] = 0.0f;
  }
  for (int l = FLAYERS - 1; l >= 0; --l) {
    int A[4], B[4];
    flow_masks(l, A, B);
    const float* L = P + (int64_t)l * FPER;
    const uint16_t* W = Wf + (int64_t)l * FS_PER;
    if (t < FH) S.cv[t] = cvec[((int64_t)ch.integral * FLAYERS + l) * FH + t];
    // this wave's W2 column slice (kept for the whole product)
    bf16x8 wb[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) wb[ks] = glb_frag(W + FS_W2 + ((w * 8 + ks) * 64 + lane) * 8);
    __syncthreads();
    // ---- 1. first layer (VALU): unit o, points p = t/128 + 2q
    {
      const int o = t & (FH - 1);
      const float w0 = L[F_W1 + o * FIN + 0], w1 = L[F_W1 + o * FIN + 1];
      const float w2 = L[F_W1 + o * FIN + 2], w3 = L[F_W1 + o * FIN + 3];
      const float c = S.cv[o];
#pragma unroll 4
      for (int q = 0; q < FP / 2; ++q) {
        const int p = (t >> 7) + 2 * q;
        const float a = c + w0 * S.v[p][B[0]] + w1 * S.v[p][B[1]] + w2 * S.v[p][B[2]] + w3 * S.v[p][B[3]];
        put_act<X2>(S, p * HP + o, silu(a));
      }
    }
    __syncthreads();
    // ---- 2. a2 = W2 h1: columns 32w + col, all points
    f32x16 acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      zero16(acc[mt]);
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        const int off = (32 * mt + col) * HP + 16 * ks + 8 * half;
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lds_frag(&S.h[0][off]), wb[ks], acc[mt], 0, 0, 0);
        if constexpr (X2)
          acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lds_frag(&S.h[X2 ? 1 : 0][off]), wb[ks], acc[mt], 0, 0, 0);
      }
    }
    __syncthreads();
    // ---- 3. h2 = silu(a2 + b2) into the same tile
    {
      const int n = 32 * w + col;
      const float b2 = L[F_B2 + n];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) put_act<X2>(S, (32 * mt + mfma_row(r)) * HP + n, silu(acc[mt][r] + b2));
    }
    __syncthreads();
    // ---- 4. theta^T = W3 h2^T: rows 32mt + mfma_row(r), point 32w + col
    f32x16 th[3];
#pragma unroll
    for (int mt = 0; mt < 3; ++mt) {
      zero16(th[mt]);
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        const bf16x8 a = glb_frag(W + FS_W3 + ((mt * 8 + ks) * 64 + lane) * 8);
        const int off = (32 * w + col) * HP + 16 * ks + 8 * half;
        th[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, lds_frag(&S.h[0][off]), th[mt], 0, 0, 0);
        if constexpr (X2)
          th[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, lds_frag(&S.h[X2 ? 1 : 0][off]), th[mt], 0, 0, 0);
      }
    }
    // ---- 5. logits of this lane's two positions (2 half + jj), spline inverse
    // own[mt][r] is row 32mt + 8(r>>2) + 4 half + (r&3); oth[] the partner half's
    float own[3][16], oth[3][16];
#pragma unroll
    for (int mt = 0; mt < 3; ++mt)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * mt + mfma_row(r);
        own[mt][r] = th[mt][r] + (row < FOUT ? L[F_B3 + row] : 0.0f);
        oth[mt][r] = __shfl_xor(own[mt][r], 32, kWave);
      }
    const int p = 32 * w + col;
    float lsum = 0.0f;
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      float tl[23];
#pragma unroll
      for (int m = 0; m < 23; ++m) {
        // row q of half h lives in half ((q % 32) >> 2) & 1 at (q / 32, 4 ((q % 32) >> 3) + (q % 4))
        const int q0 = 23 * jj + m, q1 = 23 * (2 + jj) + m;
        const int g0 = ((q0 & 31) >> 2) & 1, g1 = ((q1 & 31) >> 2) & 1;
        const int r0 = 4 * ((q0 & 31) >> 3) + (q0 & 3), r1 = 4 * ((q1 & 31) >> 3) + (q1 & 3);
        const float v0 = g0 == 0 ? own[q0 >> 5][r0] : oth[q0 >> 5][r0];   // value for half 0
        const float v1 = g1 == 1 ? own[q1 >> 5][r1] : oth[q1 >> 5][r1];   // value for half 1
        tl[m] = half ? v1 : v0;
      }
      Spline sp;
      spline_make(tl, sp);
      float ld;
      const int a = A[2 * half + jj];
      S.v[p][a] = spline_inv(sp, S.v[p][a], ld);
      lsum += ld;
    }
    lsum += __shfl_xor(lsum, 32, kWave);
    if (half == 0) S.logq[p] += lsum;
    __syncthreads();
    if (l == 3 && t < FP) {
#pragma unroll
      for (int d = 0; d < 4; ++d) { float x = S.v[t][d]; S.v[t][d] = S.v[t][7 - d]; S.v[t][7 - d] = x; }
    }
  }
  __syncthreads();
  if (t < ch.count) {
#pragma unroll
    for (int d = 0; d < 8; ++d) xout[(ch.out + t) * 8 + d] = S.v[t][d];
    lqout[ch.out + t] = S.logq[t];
  }
}

}  // namespace memk
