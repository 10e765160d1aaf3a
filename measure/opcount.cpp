// Algorithmic operation count of the ttbar dilepton integrand.
//
// Compiles the device integrand headers for the host with counting scalar
// types in place of double (FP64) and of the matrix-element type T (FP32),
// runs a small VEGAS integration of a few events with the same point
// stream, maps and grid refinement as the GPU path, and reports the number
// of arithmetic operations per integrand evaluation: add/sub, mul, fma
// (2 FLOP), div, sqrt and transcendental calls (1 FLOP each), separately
// for FP64 and FP32.  Integer work (Philox) is not counted.
//
// Input (stdin, binary): int32 n_events, then n_events x 4 objects x 4
// float64 (E, px, py, pz) in the ttbar dilepton order.  Arguments:
// n_points_per_iteration n_iterations n_events_to_use.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

struct Tally {
  double add[2], mul[2], fma[2], div[2], sqr[2], trans[2];
};
static Tally g_t;
enum { F64 = 0, F32 = 1 };

struct CF;
struct CD {
  double v;
  constexpr CD() : v(0) {}
  constexpr CD(double x) : v(x) {}
  CD(float x) : v(x) {}
  CD(int x) : v(x) {}
  CD(unsigned x) : v(x) {}
  CD(long x) : v((double)x) {}
  CD(unsigned long x) : v((double)x) {}
  CD(long long x) : v((double)x) {}
  CD(unsigned long long x) : v((double)x) {}
  CD(const CF& f);
  explicit operator int() const { return (int)v; }
};
struct CF {
  float v;
  CF() : v(0) {}
  CF(double x) : v((float)x) {}
  CF(float x) : v(x) {}
  CF(int x) : v((float)x) {}
  CF(const CD& d) : v((float)d.v) {}
};
inline CD::CD(const CF& f) : v(f.v) {}

#define ARITH(TY, K)                                                                              \
  inline TY operator+(TY a, TY b) { g_t.add[K]++; return TY(a.v + b.v); }                        \
  inline TY operator-(TY a, TY b) { g_t.add[K]++; return TY(a.v - b.v); }                        \
  inline TY operator*(TY a, TY b) { g_t.mul[K]++; return TY(a.v * b.v); }                        \
  inline TY operator/(TY a, TY b) { g_t.div[K]++; return TY(a.v / b.v); }                        \
  inline TY operator-(TY a) { return TY(-a.v); }                                                 \
  inline TY& operator+=(TY& a, TY b) { a = a + b; return a; }                                    \
  inline TY& operator-=(TY& a, TY b) { a = a - b; return a; }                                    \
  inline TY& operator*=(TY& a, TY b) { a = a * b; return a; }                                    \
  inline bool operator<(TY a, TY b) { return a.v < b.v; }                                       \
  inline bool operator>(TY a, TY b) { return a.v > b.v; }                                        \
  inline bool operator<=(TY a, TY b) { return a.v <= b.v; }                                      \
  inline bool operator>=(TY a, TY b) { return a.v >= b.v; }                                      \
  inline bool operator==(TY a, TY b) { return a.v == b.v; }                                      \
  inline bool operator!=(TY a, TY b) { return a.v != b.v; }                                      \
  inline TY sqrt(TY a) { g_t.sqr[K]++; return TY(std::sqrt(a.v)); }                              \
  inline TY exp(TY a) { g_t.trans[K]++; return TY(std::exp(a.v)); }                              \
  inline TY log(TY a) { g_t.trans[K]++; return TY(std::log(a.v)); }                              \
  inline TY tan(TY a) { g_t.trans[K]++; return TY(std::tan(a.v)); }                              \
  inline TY atan(TY a) { g_t.trans[K]++; return TY(std::atan(a.v)); }                            \
  inline TY acos(TY a) { g_t.trans[K]++; return TY(std::acos(a.v)); }                            \
  inline TY cbrt(TY a) { g_t.trans[K]++; return TY(std::cbrt(a.v)); }                            \
  inline TY sin(TY a) { g_t.trans[K]++; return TY(std::sin(a.v)); }                              \
  inline TY cos(TY a) { g_t.trans[K]++; return TY(std::cos(a.v)); }                              \
  inline TY pow(TY a, TY b) { g_t.trans[K]++; return TY(std::pow(a.v, b.v)); }                   \
  inline TY fabs(TY a) { return TY(std::fabs(a.v)); }                                            \
  inline TY fmax(TY a, TY b) { return TY(std::fmax(a.v, b.v)); }                                 \
  inline TY fmin(TY a, TY b) { return TY(std::fmin(a.v, b.v)); }                                 \
  inline TY copysign(TY a, TY b) { return TY(std::copysign(a.v, b.v)); }                         \
  inline bool isfinite(TY a) { return std::isfinite(a.v); }
ARITH(CD, F64)
ARITH(CF, F32)
// mixed operands with plain literals
#define MIX(TY, LIT)                                                                              \
  inline TY operator+(TY a, LIT b) { return a + TY(b); }                                         \
  inline TY operator+(LIT a, TY b) { return TY(a) + b; }                                         \
  inline TY operator-(TY a, LIT b) { return a - TY(b); }                                         \
  inline TY operator-(LIT a, TY b) { return TY(a) - b; }                                         \
  inline TY operator*(TY a, LIT b) { return a * TY(b); }                                         \
  inline TY operator*(LIT a, TY b) { return TY(a) * b; }                                         \
  inline TY operator/(TY a, LIT b) { return a / TY(b); }                                         \
  inline TY operator/(LIT a, TY b) { return TY(a) / b; }                                         \
  inline bool operator<(TY a, LIT b) { return a.v < b; }                                         \
  inline bool operator>(TY a, LIT b) { return a.v > b; }                                         \
  inline bool operator<=(TY a, LIT b) { return a.v <= b; }                                       \
  inline bool operator>=(TY a, LIT b) { return a.v >= b; }                                       \
  inline bool operator==(TY a, LIT b) { return a.v == b; }                                       \
  inline bool operator!=(TY a, LIT b) { return a.v != b; }
MIX(CD, double)
MIX(CD, int)
MIX(CF, float)
MIX(CF, int)
inline CD operator*(CD a, CF b) { return a * CD(b); }
inline CD operator*(CF a, CD b) { return CD(a) * b; }
inline void sincos(CD a, CD* s, CD* c) { g_t.trans[F64] += 2; *s = CD(std::sin(a.v)); *c = CD(std::cos(a.v)); }
inline void sincospi(CD a, CD* s, CD* c)
{
  g_t.trans[F64] += 2;
  *s = CD(std::sin(M_PI * a.v));
  *c = CD(std::cos(M_PI * a.v));
}
inline CD __fma_rn(CD a, CD b, CD c) { g_t.fma[F64]++; return CD(std::fma(a.v, b.v, c.v)); }
inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }

#define MEM_HOST_COUNT 1
#define __device__
#define __host__
#define __forceinline__ inline
#define __global__
#define __launch_bounds__(x)
#define double CD
#include "device_common.hpp"
#include "process.hpp"
#include "tt.hpp"
#undef double

using namespace memk;

// sequential form of the damped rebinning (same rule as the device)
static void refine(const std::vector<double>& d, double alpha, double* e)
{
  const int n = kBins;
  double s[kBins], m[kBins], old[kBins + 1];
  s[0] = 0.5 * (d[0] + d[1]);
  for (int i = 1; i < n - 1; ++i) s[i] = (d[i - 1] + d[i] + d[i + 1]) / 3.0;
  s[n - 1] = 0.5 * (d[n - 2] + d[n - 1]);
  double tot = 0;
  for (int i = 0; i < n; ++i) tot += s[i];
  if (!(tot > 0)) return;
  double ms = 0;
  for (int i = 0; i < n; ++i) {
    double r = s[i] / tot;
    m[i] = r <= 0 ? 0 : r >= 1 ? 1 : std::pow((1 - r) / std::log(1 / r), alpha);
    ms += m[i];
  }
  std::memcpy(old, e, sizeof(old));
  int i = 0;
  double acc = 0;
  for (int k = 1; k < n; ++k) {
    double t = ms / n * k;
    while (i < n && acc + m[i] < t) acc += m[i++];
    e[k] = i >= n ? 1.0 : old[i] + (t - acc) / m[i] * (old[i + 1] - old[i]);
  }
}

int main(int argc, char** argv)
{
  if (argc < 4) { std::fprintf(stderr, "usage: opcount n_points n_iter n_events [first_event] < events.bin\n"); return 2; }
  const long npts = std::atol(argv[1]);
  const int nit = std::atoi(argv[2]);
  int nuse = std::atoi(argv[3]);
  // index of the first event in the whole sample (the point stream's event counter)
  const int e0 = argc > 4 ? std::atoi(argv[4]) : 0;
  int32_t n_ev = 0;
  if (std::fread(&n_ev, 4, 1, stdin) != 1) return 3;
  std::vector<double> ev((size_t)n_ev * 16);
  if (std::fread(ev.data(), 8, ev.size(), stdin) != ev.size()) return 3;
  if (nuse > n_ev) nuse = n_ev;
  // events as SoA [4 comps][4 obj][n_ev] for EventsView
  std::vector<CD> comp(4 * 4 * (size_t)n_ev);
  for (int e = 0; e < n_ev; ++e)
    for (int o = 0; o < 4; ++o)
      for (int c = 0; c < 4; ++c) comp[((size_t)c * 4 + o) * n_ev + e] = CD(ev[((size_t)e * 4 + o) * 4 + c]);
  EventsView view;
  view.E = comp.data(); view.px = comp.data() + 4 * n_ev; view.py = comp.data() + 8 * n_ev;
  view.pz = comp.data() + 12 * n_ev; view.n_events = n_ev; view.n_obj = 4;
  // process parameters as the library derives them for the default process
  ProcParams pp{};
  const double sqs = 13000.0, mt = 172.5, wt = 1.4, mw = 80.4, ww = 2.1, as = 0.118, gf = 1.1663787e-5;
  pp.kind = kTT; pp.precision = 1; pp.dims = 8; pp.n_perm = 2;
  pp.sqrt_s = sqs; pp.S = sqs * sqs; pp.inv_sqrt_s = 1.0 / sqs; pp.m_t = mt; pp.w_t = wt; pp.m_w = mw; pp.w_w = ww; pp.sigma_k = 20.0;
  pp.tf_b.s_core = 0.15; pp.tf_b.s_tail = 0.15; pp.tf_b.f_tail = 0.0; pp.tf_b.r_lo = 0.25; pp.tf_b.r_hi = 1.75;
  pp.tf_b.i_core = 1.0 / 0.15; pp.tf_b.i_tail = 1.0 / 0.15;
  const double S = sqs * sqs;
  pp.th0_t = std::atan(-mt * mt / (mt * wt)); pp.th1_t = std::atan((S - mt * mt) / (mt * wt));
  pp.th0_w = std::atan(-mw * mw / (mw * ww)); pp.th1_w = std::atan((S - mw * mw) / (mw * ww));
  pp.tt_const = 1.0;
  Tally zero{};
  double n_evals = 0, n_nonzero = 0, n_sol = 0;
  std::vector<double> per_iter_flops(nit, 0.0);
  for (int e = 0; e < nuse; ++e)
    for (int perm = 0; perm < 2; ++perm) {
      TTEvent tev;
      tt_load(view, e, perm, tev);
      std::vector<double> grid(8 * 65);
      for (int d = 0; d < 8; ++d)
        for (int i = 0; i <= 64; ++i) grid[d * 65 + i] = i / 64.0;
      for (int j = 0; j < nit; ++j) {
        std::vector<CD> cg(grid.begin(), grid.end());
        std::vector<double> bins(8 * 64, 0.0);
        Tally before = g_t;
        for (long k = 0; k < npts; ++k) {
          CD u[8], x[8];
          int bin[8];
          point_uniforms<8>(0x14077595ull, (uint32_t)k, (uint32_t)j, (uint32_t)(e0 + e), (uint32_t)perm, u);
          CD jac = vegas_map<8>(cg.data(), u, x, bin);
          int ns = 0;
          CD f = tt_integrand<CF>(pp, tev, x, &ns);
          double w = (f * jac).v;
          n_evals += 1;
          n_sol += ns;
          if (w != 0) {
            n_nonzero += 1;
            for (int d = 0; d < 8; ++d) bins[d * 64 + bin[d]] += w * w;
          }
        }
        Tally& a = g_t;
        double fl = 0;
        for (int p = 0; p < 2; ++p)
          fl += (a.add[p] - before.add[p]) + (a.mul[p] - before.mul[p]) + 2 * (a.fma[p] - before.fma[p]) +
                (a.div[p] - before.div[p]) + (a.sqr[p] - before.sqr[p]) + (a.trans[p] - before.trans[p]);
        per_iter_flops[j] += fl;
        for (int d = 0; d < 8; ++d) {
          std::vector<double> dd(bins.begin() + d * 64, bins.begin() + d * 64 + 64);
          refine(dd, 1.5, grid.data() + d * 65);
        }
      }
    }
  (void)zero;
  const char* nm[2] = {"fp64", "fp32"};
  std::printf("{\"evaluations\": %.0f, \"nonzero_fraction\": %.6f, \"solutions_per_eval\": %.6f", n_evals,
              n_nonzero / n_evals, n_sol / n_evals);
  double tot64 = 0, tot32 = 0;
  for (int p = 0; p < 2; ++p) {
    const Tally& a = g_t;
    double flops = a.add[p] + a.mul[p] + 2 * a.fma[p] + a.div[p] + a.sqr[p] + a.trans[p];
    (p == 0 ? tot64 : tot32) = flops / n_evals;
    std::printf(", \"%s\": {\"add\": %.4f, \"mul\": %.4f, \"fma\": %.4f, \"div\": %.4f, \"sqrt\": %.4f, "
                "\"transcendental\": %.4f, \"flop\": %.4f}",
                nm[p], a.add[p] / n_evals, a.mul[p] / n_evals, a.fma[p] / n_evals, a.div[p] / n_evals,
                a.sqr[p] / n_evals, a.trans[p] / n_evals, flops / n_evals);
  }
  std::printf(", \"flop_fp32_equivalent\": %.4f, \"per_iteration_flop\": [", tot32 + 2 * tot64);
  for (int j = 0; j < nit; ++j) std::printf("%s%.4f", j ? ", " : "", per_iter_flops[j] / (nuse * 2.0 * npts));
  std::printf("]}\n");
  return 0;
}
