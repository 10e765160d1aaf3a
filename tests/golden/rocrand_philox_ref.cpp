// Reference Philox4x32-10 stream from ROCm's rocRAND (host execution).
// Reads lines "seed k iter event sub" from stdin and prints the four
// 32-bit words of Philox4x32-10 at counter {k, iter, event, sub} with key
// {seed_lo, seed_hi}, using rocRAND's engine seeded at subsequence
// (event | sub << 32) and offset 4 * (k | iter << 32).
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main()
{
  unsigned long long seed, k, it, ev, sub;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &k, &it, &ev, &sub) == 5) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, ev | (sub << 32), 4ull * (k | (it << 32)), &st);
    unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
