// Host execution of the device headers for checking: a workgroup of 256
// lanes runs as 256 host threads.  The qualifiers become plain C++,
// __shared__ variables become function statics (one workgroup runs at a
// time, so they stand for its LDS), __syncthreads is a barrier over the
// workgroup, and the cross-lane operations of a wavefront (shuffles,
// ballots, the wavefront barrier) exchange values through a per-wavefront
// slot array between two barriers over its 64 lanes.  The hardware
// reciprocal estimates become exact divisions.  Built with the sanitizers,
// this runs the queue kernel's own code (chunk loop, LDS queues, ballots,
// reductions) under AddressSanitizer, UndefinedBehaviorSanitizer or
// ThreadSanitizer; it is a checking tool, not a model of the GPU's timing.
#pragma once
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __constant__

struct __attribute__((aligned(16))) float4 { float x, y, z, w; };
struct emu_dim3 { unsigned x = 0, y = 0, z = 0; };
inline thread_local emu_dim3 threadIdx;
inline thread_local emu_dim3 blockIdx;
inline emu_dim3 blockDim{256, 1, 1};
inline emu_dim3 gridDim{1, 1, 1};

namespace emu {
constexpr int kLanes = 64;
constexpr int kThreads = 256;
struct Wave {
  std::barrier<> bar{kLanes};
  uint64_t slot[kLanes];
};
struct Block {
  std::barrier<> bar{kThreads};
  Wave waves[kThreads / kLanes];
};
inline Block* g_block = nullptr;
inline Wave& wave() { return g_block->waves[threadIdx.x / kLanes]; }
inline int lane() { return (int)(threadIdx.x % kLanes); }

template <class V>
inline V exchange(V v, int src)
{
  static_assert(sizeof(V) <= 8, "one slot per lane");
  Wave& w = wave();
  uint64_t bits = 0;
  std::memcpy(&bits, &v, sizeof(V));
  w.slot[lane()] = bits;
  w.bar.arrive_and_wait();
  V out = v;
  if (src >= 0 && src < kLanes) std::memcpy(&out, &w.slot[src], sizeof(V));
  w.bar.arrive_and_wait();
  return out;
}

// runs kernel() on `blocks` workgroups of 256 lanes, one workgroup at a time
inline void launch(unsigned blocks, const std::function<void()>& kernel)
{
  gridDim = emu_dim3{blocks, 1, 1};
  for (unsigned b = 0; b < blocks; ++b) {
    auto blk = std::make_unique<Block>();
    g_block = blk.get();
    std::vector<std::thread> ts;
    ts.reserve(kThreads);
    for (int t = 0; t < kThreads; ++t)
      ts.emplace_back([b, t, &kernel] {
        threadIdx = emu_dim3{(unsigned)t, 0, 0};
        blockIdx = emu_dim3{b, 0, 0};
        kernel();
      });
    for (auto& th : ts) th.join();
    g_block = nullptr;
  }
}
}  // namespace emu

inline void __syncthreads() { emu::g_block->bar.arrive_and_wait(); }

template <class V> inline V __shfl_xor(V v, int m, int = 64) { return emu::exchange(v, emu::lane() ^ m); }
template <class V> inline V __shfl_up(V v, unsigned d, int = 64)
{
  const int src = emu::lane() - (int)d;
  return emu::exchange(v, src >= 0 ? src : emu::lane());
}
template <class V> inline V __shfl(V v, int src, int = 64) { return emu::exchange(v, src); }

inline uint64_t __ballot(int pred)
{
  emu::Wave& w = emu::wave();
  w.slot[emu::lane()] = pred ? 1u : 0u;
  w.bar.arrive_and_wait();
  uint64_t m = 0;
  for (int i = 0; i < emu::kLanes; ++i) m |= (w.slot[i] ? 1ull : 0ull) << i;
  w.bar.arrive_and_wait();
  return m;
}
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }

// wavefront barrier; the fences around it become the barrier's own ordering
#define __builtin_amdgcn_fence(order, scope) ((void)0)
#define __builtin_amdgcn_wave_barrier() (emu::wave().bar.arrive_and_wait())
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt(x))
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))

inline double __fma_rn(double a, double b, double c) { return std::fma(a, b, c); }
inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
inline void sincospi(double a, double* s, double* c)
{
  *s = std::sin(M_PI * a);
  *c = std::cos(M_PI * a);
}

inline double atomicAdd(double* p, double v)
{
  uint64_t* q = reinterpret_cast<uint64_t*>(p);
  uint64_t old = __atomic_load_n(q, __ATOMIC_RELAXED);
  for (;;) {
    double o;
    std::memcpy(&o, &old, 8);
    const double n = o + v;
    uint64_t nb;
    std::memcpy(&nb, &n, 8);
    if (__atomic_compare_exchange_n(q, &old, nb, false, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED)) return o;
  }
}
inline uint32_t atomicAdd(uint32_t* p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_ACQ_REL); }
inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_ACQ_REL); }
