// One iteration of the persistent work-queue kernel (vegas_queue_kernel)
// executed on the host through hip_host_emu.hpp, on the uniform grid, for
// every (event, assignment) integral of the given events; prints each
// integral's sum of w, sum of w^2 and per-(dimension, bin) sums of w^2 (the
// chunk partials summed in chunk order), for comparison with the oracle's
// iteration on the same point stream.
//
//   host_queue DESC_FILE EVENTS_FILE VARIANT N_POINTS SEED CHUNK BLOCKS [NS]
//
// With NS (hypercubes per dimension), the iteration is stratified with the
// first iteration's equal split of N_POINTS over NS^D hypercubes, and each
// integral's line carries its N_POINTS point weights after the bin sums.
// DESC_FILE: a mem_process_desc as bytes.  EVENTS_FILE: int32 n_events,
// int32 n_obj, then E, px, py, pz planes [n_obj][n_events] of doubles,
// optionally followed by one int32 lepton charge per event.  VARIANT: tt1f,
// tt2f, tt1d (dilepton at one or two waves per SIMD, FP32 or FP64 matrix
// element), dy (Drell-Yan), sl1f (semileptonic), tth2f (t tbar H in the
// instance that carries every kind, as launches with t tbar H chunks run).
#include "hip_host_emu.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

using std::max;
using std::min;

#include "kernels.hpp"
#include "process_params.hpp"

using namespace memk;

typedef void (*Kernel)(const ProcParams*, EventsView, const Chunk*, int64_t, const IntegralDesc*, const double*,
                       const int32_t*, uint64_t, Control*, uint32_t*, double*, const int64_t*, QueueHooks, StratView);

static Kernel pick(const std::string& v)
{
  if (v == "tt1f") return vegas_queue_kernel<float, kMaskTT, 1>;
  if (v == "tt2f") return vegas_queue_kernel<float, kMaskTT, 2>;
  if (v == "tt1d") return vegas_queue_kernel<double, kMaskTT, 1>;
  if (v == "dy") return vegas_queue_kernel<double, kMaskDY, 1>;
  if (v == "sl1f") return vegas_queue_kernel<float, kMaskSL, 1>;
  if (v == "tth2f") return vegas_queue_kernel<float, kMaskDY | kMaskTT | kMaskSL | kMaskTTH, 2>;
  return nullptr;
}

static std::vector<char> slurp(const char* path)
{
  std::vector<char> b;
  FILE* f = std::fopen(path, "rb");
  if (!f) return b;
  char buf[65536];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) b.insert(b.end(), buf, buf + n);
  std::fclose(f);
  return b;
}

int main(int argc, char** argv)
{
  if (argc != 8 && argc != 9) {
    std::fprintf(stderr, "usage: host_queue DESC EVENTS VARIANT N_POINTS SEED CHUNK BLOCKS [NS]\n");
    return 2;
  }
  const int ns = argc == 9 ? std::atoi(argv[8]) : 0;
  const std::vector<char> db = slurp(argv[1]), eb = slurp(argv[2]);
  Kernel kern = pick(argv[3]);
  const int64_t N = std::atoll(argv[4]);
  const uint64_t seed = std::strtoull(argv[5], nullptr, 0);
  const int64_t chunk = std::atoll(argv[6]);
  const unsigned blocks = (unsigned)std::atoi(argv[7]);
  if (db.size() != sizeof(mem_process_desc) || eb.size() < 8 || !kern || N < 2 || chunk < 1 || blocks < 1) {
    std::fprintf(stderr, "bad arguments\n");
    return 2;
  }
  mem_process_desc d;
  std::memcpy(&d, db.data(), sizeof d);
  int32_t n_ev, n_obj;
  std::memcpy(&n_ev, eb.data(), 4);
  std::memcpy(&n_obj, eb.data() + 4, 4);
  const size_t plane = (size_t)n_ev * n_obj;
  const size_t body = 8 + 4 * plane * sizeof(double);
  const bool charged = eb.size() == body + (size_t)n_ev * 4;
  if (n_ev < 1 || n_obj < 1 || (eb.size() != body && !charged)) {
    std::fprintf(stderr, "bad events file\n");
    return 2;
  }
  std::vector<double> comp(4 * plane);
  std::memcpy(comp.data(), eb.data() + 8, comp.size() * sizeof(double));
  std::vector<int32_t> charge(charged ? n_ev : 0);
  if (charged) std::memcpy(charge.data(), eb.data() + body, (size_t)n_ev * 4);
  mem_tf_desc tf[5];
  default_tfs(d.kind, tf);
  const ProcParams pp = derive_params(d, tf);
  const EventsView ev{comp.data(), comp.data() + plane, comp.data() + 2 * plane, comp.data() + 3 * plane,
                      charged ? charge.data() : nullptr, n_ev, n_obj};
  const int D = pp.dims, np = pp.n_perm;
  std::vector<IntegralDesc> ints;
  std::vector<Chunk> chunks;
  int64_t part_total = 0;
  for (int e = 0; e < n_ev; ++e)
    for (int k = 0; k < np; ++k) {
      IntegralDesc in{};
      in.event = e; in.perm = k; in.dims = D; in.n_points = N;
      in.grid_off = (int64_t)ints.size() * D * (kBins + 1);
      in.chunk0 = (int64_t)chunks.size();
      for (int64_t s0 = 0; s0 < N; s0 += chunk) {
        Chunk c{};
        c.integral = (int32_t)ints.size(); c.event = e; c.perm = k;
        c.count = (int32_t)std::min<int64_t>(chunk, N - s0);
        c.start = s0;
        c.part_off = part_total;
        c.proc = 0;
        c.id = (int32_t)chunks.size();
        part_total += 2 + (int64_t)D * kBins;
        chunks.push_back(c);
        in.n_chunks++;
      }
      ints.push_back(in);
    }
  std::vector<double> grids(ints.size() * D * (kBins + 1));
  for (size_t i = 0; i < grids.size(); ++i) grids[i] = (double)(i % (kBins + 1)) / (double)kBins;
  std::vector<int32_t> active(ints.size(), 1);
  std::vector<double> parts(part_total, 0.0);
  Control ctl{0u, 0u, 0, 0u};
  uint32_t head = 0;
  const QueueHooks hk{nullptr, 0, -1, -1};
  // stratification: every integral's equal split and each chunk's first
  // hypercube, as the library's first iteration sets them
  std::vector<StratDesc> sd;
  std::vector<int32_t> cum, h0(chunks.size(), 0);
  std::vector<double> wpt;
  if (ns > 0) {
    int64_t H = 1;
    for (int dd = 0; dd < D; ++dd) H *= ns;
    if (2 * H > N || H > kStratHMax || chunk > kStratChunkMax) {
      std::fprintf(stderr, "bad stratification\n");
      return 2;
    }
    const int64_t q = N / H, r = N % H;
    for (size_t ig = 0; ig < ints.size(); ++ig) {
      sd.push_back(StratDesc{ns, (int32_t)H, (int64_t)cum.size(), (int64_t)(ig * N)});
      const int64_t base = (int64_t)cum.size();
      for (int64_t h = 0; h <= H; ++h) cum.push_back((int32_t)(h * q + (h < r ? h : r)));
      for (int c = 0; c < ints[ig].n_chunks; ++c) {
        const int64_t start = chunks[ints[ig].chunk0 + c].start;
        int64_t h = 0;
        while (h + 1 < H && cum[base + h + 1] <= start) ++h;
        h0[ints[ig].chunk0 + c] = (int32_t)h;
      }
    }
    wpt.assign(ints.size() * N, 0.0);
  }
  const StratView sv = ns > 0 ? StratView{sd.data(), cum.data(), h0.data(), wpt.data()}
                              : StratView{nullptr, nullptr, nullptr, nullptr};
  emu::launch(blocks, [&] {
    kern(&pp, ev, chunks.data(), (int64_t)chunks.size(), ints.data(), grids.data(), active.data(), seed, &ctl, &head,
         parts.data(), nullptr, hk, sv);
  });
  for (const IntegralDesc& in : ints) {
    double s1 = 0.0, s2 = 0.0;
    std::vector<double> bins((size_t)D * kBins, 0.0);
    for (int c = 0; c < in.n_chunks; ++c) {
      const double* p = parts.data() + chunks[in.chunk0 + c].part_off;
      s1 += p[0];
      s2 += p[1];
      for (int i = 0; i < D * kBins; ++i) bins[i] += p[2 + i];
    }
    std::printf("%d %d %.17g %.17g", in.event, in.perm, s1, s2);
    for (double b : bins) std::printf(" %.17g", b);
    if (ns > 0) {
      const double* w = wpt.data() + (size_t)(&in - ints.data()) * N;
      for (int64_t k = 0; k < N; ++k) std::printf(" %.17g", w[k]);
    }
    std::printf("\n");
  }
  return 0;
}
