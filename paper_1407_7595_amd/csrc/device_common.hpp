// Device building blocks shared by the MEM kernels: counter-based random
// numbers, the VEGAS map, wavefront reductions and small vector helpers.
//
// The MC estimator S_N = V mean f(x_i) and its error (Sec. 2) are fed by a
// Philox4x32-10 point stream (Salmon et al., SC'11) mapped through a VEGAS
// grid (Lepage 1978).  Points are generated in registers, never stored.
#pragma once
#if !defined(MEM_HOST_COUNT) && !defined(MEM_HOST_EMU)
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

namespace memk {

constexpr int kBins = 64;          // VEGAS bins per dimension
constexpr int kMaxDims = 12;       // largest integration dimension supported
constexpr int kWave = 64;          // CDNA wavefront width

// ---------------------------------------------------------------- Philox --
// One Philox4x32-10 block: ten rounds of two 32x32 -> 64 products whose
// halves are mixed with the other two words and a Weyl-sequence key.
struct u32x4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u32x4 philox10(u32x4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint32_t lo0 = m0 * c.x, hi0 = __umulhi(m0, c.x);
    uint32_t lo1 = m1 * c.z, hi1 = __umulhi(m1, c.z);
    c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// 53-bit uniform in [0,1) from a (hi, lo) word pair.
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo)
{
  uint64_t bits = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
  return (double)bits * 0x1.0p-53;
}

// Uniforms of point k: dims (2b, 2b+1) from counter {k, iter, event, perm*16+b}.
// block0 offsets the counter block (the learned proposal draws its base
// points from blocks 8..11 of the same stream).
template <int D>
__device__ __forceinline__ void point_uniforms(uint64_t seed, uint32_t k, uint32_t iter,
                                               uint32_t event, uint32_t perm, double (&u)[D],
                                               uint32_t block0 = 0u)
{
#pragma unroll
  for (int b = 0; 2 * b < D; ++b) {
    u32x4 w = philox10(u32x4{k, iter, event, perm * 16u + block0 + (uint32_t)b},
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    u[2 * b] = u53(w.x, w.y);
    if (2 * b + 1 < D) u[2 * b + 1] = u53(w.z, w.w);
  }
}

// ------------------------------------------------------------ VEGAS map --
// x = e_i + frac * width through a fused multiply-add (correctly rounded),
// Jacobian = prod 64 * width.  `grid` points at D rows of 65 edges (LDS).
template <int D>
__device__ __forceinline__ double vegas_map(const double* __restrict__ grid, const double (&u)[D],
                                            double (&x)[D], int (&bin)[D])
{
  double jac = 1.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    double t = u[d] * (double)kBins;
    int i = (int)t;
    i = i > kBins - 1 ? kBins - 1 : i;
    double frac = t - (double)i;
    double e0 = grid[d * (kBins + 1) + i];
    double width = grid[d * (kBins + 1) + i + 1] - e0;
    x[d] = __fma_rn(frac, width, e0);
    jac *= (double)kBins * width;
    bin[d] = i;
  }
  return jac;
}

// ----------------------------------------------------------- reductions --
#ifndef MEM_HOST_COUNT
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// inclusive prefix sum across a wavefront
__device__ __forceinline__ double wave_scan(double v)
{
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    double o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  return v;
}

// Orders the LDS accesses of the lanes of one wavefront around this point
// (a wavefront-scope fence pair around a code-motion barrier; no block
// barrier, so wavefronts of a block may run different trip counts).
__device__ __forceinline__ void wave_sync()
{
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#endif  // MEM_HOST_COUNT

// FP64 reciprocal: hardware estimate refined by two Newton steps (full
// double accuracy for normal operands, without the scaling and fix-up of
// an IEEE division; 0 gives a non-finite result).
__device__ __forceinline__ double fast_rcp(double d)
{
#ifdef MEM_HOST_COUNT
  return 1.0 / d;
#else
  double r = __builtin_amdgcn_rcp(d);
  double e = __fma_rn(-d, r, 1.0);
  r = __fma_rn(r, e, r);
  e = __fma_rn(-d, r, 1.0);
  return __fma_rn(r, e, r);
#endif
}

// FP64 1/sqrt(d), d > 0: hardware estimate refined by two Newton steps
// r <- r + r (1 - d r^2) / 2.
__device__ __forceinline__ double fast_rsqrt(double d)
{
#ifdef MEM_HOST_COUNT
  return 1.0 / sqrt(d);
#else
  double r = __builtin_amdgcn_rsq(d);
  double e = __fma_rn(-d * r, r, 1.0);
  r = __fma_rn(0.5 * r, e, r);
  e = __fma_rn(-d * r, r, 1.0);
  return __fma_rn(0.5 * r, e, r);
#endif
}

// tan(theta) for |theta| < pi/2 in FP64 (within 3 ulp; the Breit-Wigner
// maps stay inside that range).  Above pi/4, tan(a) = 1 / tan(pi/2 - a)
// with pi/2 in two parts, so that pi/2 - a is exact to an ulp next to the
// pole.  On [0, pi/4], Lambert's continued fraction
// tan x = x / (1 - x^2 / (3 - x^2 / (5 - ...))) cut after the term 17,
// written as x N(x^2) / D(x^2) (the exact rational coefficients rounded to
// double, normalised to N(0) = D(0) = 1); its truncation error on [0, pi/4]
// is below 1e-18.
__device__ __forceinline__ double tan_halfpi(double theta)
{
#ifdef MEM_HOST_COUNT
  return tan(theta);        // counted as one transcendental, like the library call
#endif
  const double a = fabs(theta);
  const bool big = a > 0.78539816339744831;
  const double x = big ? (1.5707963267948966 - a) + 6.123233995736766e-17 : a;
  const double y = x * x;
  double n = 2.901963686277412e-08;
  n = __fma_rn(n, y, -2.8729440494146376e-05);
  n = __fma_rn(n, y, 0.00392156862745098);
  n = __fma_rn(n, y, -0.13725490196078433);
  n = __fma_rn(n, y, 1.0);
  double d = 1.3058836588248353e-06;
  d = __fma_rn(d, y, -0.00040221216691804925);
  d = __fma_rn(d, y, 0.027450980392156862);
  d = __fma_rn(d, y, -0.47058823529411764);
  d = __fma_rn(d, y, 1.0);
  const double num = x * n;
  const double t = big ? d * fast_rcp(num) : num * fast_rcp(d);
  return copysign(t, theta);
}

// Reciprocal in the matrix-element type: the hardware v_rcp_f32 (1 ulp) in
// FP32, fast_rcp in FP64.
#ifdef MEM_HOST_COUNT
template <class T> inline T rcp_t(T x) { return T(1) / x; }
#else
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return fast_rcp(x); }
#endif

// ------------------------------------------------------ four-vector math --
struct v4 { double e, x, y, z; };
__device__ __forceinline__ double mdot(const v4& a, const v4& b)
{
  return a.e * b.e - a.x * b.x - a.y * b.y - a.z * b.z;
}
__device__ __forceinline__ v4 add(const v4& a, const v4& b) { return v4{a.e + b.e, a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ double norm3(const v4& a) { return sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }

}  // namespace memk
