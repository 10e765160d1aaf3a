// Kernels of one VEGAS iteration over many independent integrals.
//
// Integration unit: one (event, jet-parton assignment) integral.  Its points
// of one iteration are split into chunks that form a device work queue.  A
// persistent grid of workgroups pops chunks from an atomic head until the
// queue is exhausted; for each chunk a workgroup stages the integral's VEGAS
// grid in LDS, generates each point in registers (Philox -> VEGAS map),
// evaluates the fused integrand of the chunk's process (phase-space map,
// constraint solve, |M|^2, PDFs, TFs, weight), and accumulates sum w, sum w^2
// (wavefront shuffles) and the per-(dimension, bin) sums of w^2 (LDS
// atomics).  Processes of different kinds, dimensions and budgets share one
// launch.  The chunk's partial sums go to HBM; a second kernel sums them in a
// fixed order per integral, forms I_j and sigma_j^2, updates the
// inverse-variance combination and refines the grid (one wavefront per
// dimension, one lane per bin).  The iteration index and the queue head live
// in device memory, so an iteration can be captured once as a graph and
// replayed.
#pragma once
#include "device_common.hpp"
#include "dy.hpp"
#include "process.hpp"
#include "sl.hpp"
#include "tt.hpp"
#include "tth.hpp"
#include "f2.hpp"

namespace memk {

constexpr int kBlock = 256;
// Waves per SIMD the integrand kernels are compiled for.  One: a lone wave
// owns the whole 512-entry register file (256 VGPRs plus 256 AGPRs), which
// holds the FP64 solve and the matrix element without scratch spills; at
// two waves per SIMD the dilepton kernel spilled 166 VGPRs to scratch and
// ran 1.3x slower, the semileptonic one 1.7x.
#ifndef MEM_TT_WAVES
#define MEM_TT_WAVES 1
#endif

struct Chunk {
  int32_t integral;
  int32_t event;
  int32_t perm;
  int32_t count;
  int64_t start;      // first point index of the chunk inside its integral
  int64_t part_off;   // offset of its partial sums (2 + D*64 doubles)
  int32_t proc;       // index into the launch's process table
  int32_t id;         // index in the call's chunk table
};

// device control block of one integration
struct Control {
  uint32_t iter;          // current iteration
  uint32_t head;          // work-queue head
  int32_t n_running;      // events still iterating (target mode)
  uint32_t pad;
};

struct IntegralDesc {
  int32_t event;
  int32_t perm;
  int32_t dims;
  int32_t n_chunks;
  int64_t n_points;   // per iteration
  int64_t grid_off;   // offset of its D x 65 grid
  int64_t chunk0;     // first chunk
};

// Checks: the weights of one integral recorded per iteration, and a forced
// non-finite weight for one event (the host-forced failure of the status
// path).  Zero-initialised = off.
struct QueueHooks {
  double* wout;        // [iteration][w_stride] weights of integral w_int (null: off)
  int64_t w_stride;
  int32_t w_int;
  int32_t nan_event;   // event whose weights become NaN (-1: none)
};

// Adaptive stratified sampling (Lepage 2021): per integral, n_s^D = H
// equal hypercubes of the map's input cube; the iteration's points are
// handed out in hypercube order by the cumulative counts cum[0..H]
// (cum[0] = 0, cum[H] = N), so point k lies in the h with
// cum[h] <= k < cum[h + 1] and enters the map as y_d = (c_d + u_d) / n_s,
// c_d the base-n_s digits of h (dimension 0 least significant).
constexpr int kStratHMax = 16384;
constexpr int kStratChunkMax = 4096;
// cumulative counts a chunk can touch: every hypercube holds at least two
// points, so a chunk of c points spans at most c / 2 + 1 of them
constexpr int kStratSeg = kStratChunkMax / 2 + 2;
struct StratDesc {
  int32_t ns;         // hypercubes per dimension
  int32_t H;          // ns^D
  int64_t cum_off;    // its H + 1 cumulative counts in StratView::cum
  int64_t w_off;      // its N point weights in StratView::w
};
struct StratView {
  const StratDesc* sd;     // per integral; null: no stratification
  const int32_t* cum;
  const int32_t* h0;       // per chunk (Chunk::id): hypercube of its first point
  double* w;               // this iteration's weight of every point
};
// A chunk's view: the cumulative counts it touches, staged in LDS.
struct StratChunk {
  const int32_t* seg;      // cum[h0 .. h0 + nseg)
  int32_t nseg, h0, ns, H;
  double* w;               // the integral's point weights
};

// Point k of a stratified chunk: moves the uniforms u into the point's
// hypercube and returns H n_h (the bins take w^2 / (H n_h)).
__device__ __forceinline__ int strat_find(const StratChunk& sc, int64_t k)
{
  int lo = 0, hi = sc.nseg - 2;      // the i with seg[i] <= k < seg[i + 1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)sc.seg[mid] <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}
// H n_h of the hypercube holding point k
__device__ __forceinline__ double strat_hn(const StratChunk& sc, int64_t k)
{
  const int i = strat_find(sc, k);
  return (double)sc.H * (double)(sc.seg[i + 1] - sc.seg[i]);
}
template <int D>
__device__ __forceinline__ double strat_point(const StratChunk& sc, int64_t k, double (&u)[D])
{
  const int lo = strat_find(sc, k);
  int r = sc.h0 + lo;
  const double hn = (double)sc.H * (double)(sc.seg[lo + 1] - sc.seg[lo]);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int c = r % sc.ns;
    r /= sc.ns;
    u[d] = ((double)c + u[d]) / (double)sc.ns;
  }
  return hn;
}

// per-integral running state
// (sums over the kept iterations: 1/sigma_j^2, I_j/sigma_j^2, I_j, their
// count, sigma_j^2; a non-finite flag; the last iteration's I_j, sigma_j^2)
enum { ST_WSUM = 0, ST_WISUM, ST_ISUM, ST_NITER, ST_NONFINITE, ST_LAST_I, ST_LAST_V, ST_VSUM, ST_SIZE = 8 };

template <int D>
__device__ __forceinline__ void block_reduce2(double& a, double& b, double* red)
{
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) { red[2 * wave] = a; red[2 * wave + 1] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0; b = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) { a += red[2 * w]; b += red[2 * w + 1]; }
  }
}

// Points [start, start + count) of one chunk: sum w, sum w^2 and the
// per-bin sums of w^2 (LDS atomics into the calling wavefront's own bins).
// F(x) is the integrand.
// wrec: null, or where point k's weight is recorded (wrec[k]); poison:
// every weight becomes NaN (test hook).
template <int D, class F>
__device__ __forceinline__ void chunk_points(const Chunk& ch, uint64_t seed, uint32_t iter, const double* sgrid,
                                             double* sbins, double& s1, double& s2, double* wrec, bool poison,
                                             bool strat, const StratChunk& sc, F&& f)
{
  for (int k = threadIdx.x; k < ch.count; k += kBlock) {
    double u[D], x[D];
    int bin[D];
    point_uniforms<D>(seed, (uint32_t)(ch.start + k), iter, (uint32_t)ch.event, (uint32_t)ch.perm, u);
    const double hn = strat ? strat_point<D>(sc, ch.start + k, u) : 1.0;
    double jac = vegas_map<D>(sgrid, u, x, bin);
    double w = f(x) * jac;
    if (poison) w = __builtin_nan("");
    if (wrec) wrec[k] = w;
    s1 += w;
    s2 += w * w;
    if (strat) sc.w[ch.start + k] = w;
    if (w != 0.0) {
      const double q = strat ? w * w / hn : w * w;
#pragma unroll
      for (int d = 0; d < D; ++d) atomicAdd(&sbins[d * kBins + bin[d]], q);
    }
  }
}

// Dilepton chunk with the root searches and the per-root work of each
// wavefront compacted.  Every lane maps a point, forms the resultant
// quartic and isolates its real roots (0 to 4 sign-change intervals between
// critical points); the lane's solve state and monic quartic go to an LDS
// record and its intervals to an LDS queue (exclusive prefix sum of the
// counts from three ballots).  Every lane then takes queue entries lane,
// lane + 64, ...: first it runs the bracketed search of that interval
// (the searches of a wavefront run in lockstep, so a lane no longer waits
// for the slowest of its own up to four intervals), then, on the found
// root, it rebuilds the owner's geometry from the record, polishes and
// tests the root (dilep_accept) and evaluates the matrix element stage
// (tt_solution); each point sums its own entries in root order.  Both
// stages run in rounds of 64 entries instead of max(roots) times.
//
// Rounds on few lanes are put off: after the whole rounds of a batch, a
// remainder of at most kTTDefer entries stays at the front of the queue
// for the next batch.  The lanes that own those entries keep their point
// (record, Jacobian, bins, partial sum) and take no new point in that
// batch; the other lanes take the wavefront's next points (its 64-point
// segment of every 256-point block, the same points as a fixed lane per
// point, handed out in order).  Once the wavefront's points are handed out
// the queue is drained.  Each root still runs the same functions on the
// same inputs and a point adds its solutions in root order, so its weight
// does not depend on the batching; the order in which finished points
// enter s1 and s2 does.  Same functions, inputs and order as tt_integrand
// (a rejected root adds +0); the compiler contracts the two instances'
// arithmetic differently, which leaves relative differences of about 1e-11
// in FP64 and 1e-7 with the FP32 matrix element.  ON = false compiles to
// nothing (no LDS) for launches without dilepton chunks.
constexpr int kTTRec = 34;       // DilepPoint (28 doubles), the two jet energies, the monic quartic c0..c3
#ifndef MEM_TT_DEFER
#define MEM_TT_DEFER 32
#endif
constexpr int kTTDefer = MEM_TT_DEFER;               // largest remainder put off to the next batch
static_assert(kTTDefer >= 0 && kTTDefer < kWave, "a remainder is below one round");
constexpr int kTTQueue = 4 * kWave + kTTDefer;        // entries: the deferred ones and up to 4 per lane
template <class T, bool ON>
__device__ __forceinline__ void chunk_points_tt(const Chunk& ch, uint64_t seed, uint32_t iter, const double* sgrid,
                                                double* sbins, double& s1, double& s2, double* wrec, bool poison,
                                                bool strat, const StratChunk& sc, const ProcParams& pp,
                                                const TTEvent& ev)
{
  if constexpr (ON) {
    __shared__ double srec[kBlock / kWave][kTTRec][kWave];
    __shared__ double spx[kBlock / kWave][kTTQueue];
    __shared__ double slo[kBlock / kWave][kTTQueue];
    __shared__ double shi[kBlock / kWave][kTTQueue];
    __shared__ double sres[kBlock / kWave][kTTQueue];
    __shared__ int sown[kBlock / kWave][kTTQueue];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    double (*rec)[kWave] = srec[wv];
    double* qpx = spx[wv];
    double* qlo = slo[wv];
    double* qhi = shi[wv];
    double* qres = sres[wv];
    int* qown = sown[wv];
    const uint64_t lt = lane ? (~0ull >> (kWave - lane)) : 0ull;     // lanes below this one
    // the wavefront's points: 64 of every 256-point block, and its share of
    // a ragged last block
    const int n_wave = (ch.count / kBlock) * kWave + min(max(ch.count % kBlock - wv * kWave, 0), kWave);
    int t = 0;         // the wavefront's points handed out so far
    int ndef = 0;      // deferred entries at the front of the queue
    // the lane's point while entries of it are queued (busy)
    bool busy = false;
    int k = 0, off = 0, left = 0;
    double jac = 0.0, acc = 0.0;
    T jetf = T(0);
    uint32_t bins0 = 0, bins1 = 0;    // the point's 8 bin indices, 6 bits each
    // wavefront-uniform control: every decision below comes from ballots
    for (;;) {
      const int avail = n_wave - t;
      if (avail <= 0 && ndef == 0) break;
      const uint64_t freem = __ballot(!busy);
      const int rank = __popcll(freem & lt);
      const bool take = !busy && rank < avail;
      QuartIso qi;
      qi.lo.n = 0;
      if (take) {
        const int s = t + rank;
        k = (s / kWave) * kBlock + wv * kWave + (s & (kWave - 1));
        double u[8], x[8];
        point_uniforms<8>(seed, (uint32_t)(ch.start + k), iter, (uint32_t)ch.event, (uint32_t)ch.perm, u);
        if (strat) (void)strat_point<8>(sc, ch.start + k, u);
        int bin[8];
        jac = vegas_map<8>(sgrid, u, x, bin);
        static_assert(kBins <= 64, "bin indices are packed in 6 bits");
        bins0 = (uint32_t)bin[0] | (uint32_t)bin[1] << 6 | (uint32_t)bin[2] << 12 | (uint32_t)bin[3] << 18 |
                (uint32_t)bin[4] << 24;
        bins1 = (uint32_t)bin[5] | (uint32_t)bin[6] << 6 | (uint32_t)bin[7] << 12;
        TTMaps<T> m;
        tt_maps<T>(pp, ev, x, m);
        jetf = m.jetf;
        acc = 0.0;
        DilepPoint sp;
        double quart[5];
        if (dilep_prepare(m.bq[0], m.bq[1], ev.lp, ev.lm, m.metx, m.mety, m.q2wp, m.q2t, m.q2wm, m.q2tb, sp, quart)) {
          // the solve state goes to the lane's LDS record before the root
          // isolation, so that it is not held in registers across it (its
          // last reader finished before the previous batch's last wave_sync)
          const double r[30] = {sp.A1.e0, sp.A1.e1, sp.A1.e2, sp.A1.z0, sp.A1.z1, sp.A1.z2,
                                sp.A2.e0, sp.A2.e1, sp.A2.e2, sp.A2.z0, sp.A2.z1, sp.A2.z2,
                                sp.P0, sp.P1, sp.P2, sp.Q0, sp.Q1,
                                sp.tq[0], sp.tq[1], sp.tq[2], sp.tq[3], sp.itq[0], sp.itq[1], sp.itq[2], sp.itq[3],
                                sp.lam, sp.mx, sp.my, m.bq[0].e, m.bq[1].e};
#pragma unroll
          for (int f = 0; f < 30; ++f) rec[f][lane] = r[f];
          quartic_isolate(quart, qi);
#pragma unroll
          for (int f = 0; f < 4; ++f) rec[30 + f][lane] = qi.c[f];
        }
      }
      t += min(__popcll(freem), max(avail, 0));
      // the new entries go after the deferred ones, in lane order
      const int nr = qi.lo.n;
      int o = 0, total = ndef;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const uint64_t msk = __ballot((nr >> b) & 1);
        o += __popcll(msk & lt) << b;
        total += __popcll(msk) << b;
      }
      o += ndef;
      if (nr > 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (j < nr) {
            qpx[o + j] = qi.x0.get(j);
            qlo[o + j] = qi.lo.get(j);
            qhi[o + j] = qi.hi.get(j);
            qown[o + j] = lane;
          }
        }
      }
      if (take) {
        busy = true;
        off = o;
        left = nr;
      }
      wave_sync();
      // entries run in this batch: whole rounds, and the remainder when it
      // exceeds kTTDefer or the wavefront has no points left to hand out
      int done = total;
      if (t < n_wave && total % kWave <= kTTDefer) done = total - total % kWave;
      // the root searches, one interval per lane
      for (int i = lane; i < done; i += kWave) {
        const int ow = qown[i];
        const double c[5] = {rec[30][ow], rec[31][ow], rec[32][ow], rec[33][ow], 1.0};
        qpx[i] = quartic_root(c, qlo[i], qhi[i], qpx[i]);
      }
      wave_sync();
      // the roots' acceptance and matrix elements, one root per lane
      for (int i = lane; i < done; i += kWave) {
        const int ow = qown[i];
        DilepPoint sp;
        sp.A1 = Affine{rec[0][ow], rec[1][ow], rec[2][ow], rec[3][ow], rec[4][ow], rec[5][ow]};
        sp.A2 = Affine{rec[6][ow], rec[7][ow], rec[8][ow], rec[9][ow], rec[10][ow], rec[11][ow]};
        sp.P0 = rec[12][ow]; sp.P1 = rec[13][ow]; sp.P2 = rec[14][ow]; sp.Q0 = rec[15][ow]; sp.Q1 = rec[16][ow];
#pragma unroll
        for (int c = 0; c < 4; ++c) { sp.tq[c] = rec[17 + c][ow]; sp.itq[c] = rec[21 + c][ow]; }
        sp.lam = rec[25][ow]; sp.mx = rec[26][ow]; sp.my = rec[27][ow];
        const double E0 = rec[28][ow], E1 = rec[29][ow];
        DilepGeom g;
        dilep_geom(tt_jet(ev, 0, E0), tt_jet(ev, 1, E1), ev.lp, ev.lm, sp, g);
        NuSol sol;
        qres[i] = dilep_accept(sp, g, qpx[i], sol, polish_tol<T>()) ? tt_solution<T>(pp, ev, E0, E1, sol) : 0.0;
      }
      wave_sync();
      if (busy) {
        // this batch's entries of the lane's point, in root order
        const int p = min(max(done - off, 0), left);
        for (int j = 0; j < p; ++j) acc += qres[off + j];
        left -= p;
        off += p - done;
        if (left == 0) {
          busy = false;
          double w = tt_point<T>(pp, ev, acc, jetf) * jac;
          if (poison) w = __builtin_nan("");
          if (wrec) wrec[k] = w;
          s1 += w;
          s2 += w * w;
          if (strat) sc.w[ch.start + k] = w;
          if (w != 0.0) {
            // H n_h found again rather than held in registers across the solve
            const double q = strat ? w * w / strat_hn(sc, ch.start + k) : w * w;
#pragma unroll
            for (int d = 0; d < 8; ++d)
              atomicAdd(&sbins[d * kBins + (int)(((d < 5 ? bins0 : bins1) >> (6 * (d < 5 ? d : d - 5))) & 63u)], q);
          }
        }
      }
      // the deferred entries to the front of the queue (at most one per lane)
      const int nd = total - done;
      if (done > 0 && nd > 0) {
        double dpx = 0.0, dlo = 0.0, dhi = 0.0;
        int down = 0;
        if (lane < nd) { dpx = qpx[done + lane]; dlo = qlo[done + lane]; dhi = qhi[done + lane]; down = qown[done + lane]; }
        wave_sync();
        if (lane < nd) { qpx[lane] = dpx; qlo[lane] = dlo; qhi[lane] = dhi; qown[lane] = down; }
      }
      wave_sync();     // the next batch appends to the queue
      ndef = nd;
    }
  }
}

// Persistent work-queue kernel: every workgroup loops until the shared head
// passes n_chunks (each iteration of the loop reads the head once, so every
// workgroup reaches the exit).  KINDS is the set of process kinds compiled
// in (bit 1 DY, 2 dilepton, 4 semileptonic, 8 t tbar H, 16 t tbar H
// dilepton, 32 t tbar b bbar dilepton): a launch carries only the
// integrands its chunks need, and with them only their register demand.
enum { kMaskDY = 1, kMaskTT = 2, kMaskSL = 4, kMaskTTH = 8, kMaskTHL = 16, kMaskTBB = 32 };
// Instances that carry the t tbar H integrand stay at two waves per SIMD:
// compiled at one, the FP32 instance returned wrong iteration sums (zero or
// infinite for every integral) although the same integrand evaluated point
// by point was right, and host builds of the integrand run clean under
// MemorySanitizer and UBSan.  The cause is not known; at two waves the
// instance matches the oracle.
template <int KINDS> constexpr int queue_waves()
{
  return (KINDS & kMaskTTH) ? 2 : MEM_TT_WAVES;
}
// WAVES: waves per SIMD the instance is compiled for (its register budget
// is 512 / WAVES per lane); the tuner picks among the compiled variants.
template <class T, int KINDS, int WAVES = queue_waves<KINDS>()>
__global__ __launch_bounds__(kBlock, WAVES) void vegas_queue_kernel(
    const ProcParams* __restrict__ procs, EventsView ev, const Chunk* __restrict__ chunks, int64_t n_chunks,
    const IntegralDesc* __restrict__ ints, const double* __restrict__ grids, const int32_t* __restrict__ active,
    uint64_t seed, Control* __restrict__ ctl, uint32_t* __restrict__ head, double* __restrict__ parts,
    const int64_t* __restrict__ alloc, QueueHooks hk, StratView sv)
{
  static_assert(!(KINDS & kMaskTTH) || WAVES >= 2, "t tbar H instances run at two or more waves per SIMD");
  __shared__ double sgrid[kMaxDims * (kBins + 1)];
  __shared__ int32_t sseg[kStratSeg];
  // per-wavefront bin sums, combined in wavefront order: the result does not
  // depend on how the wavefronts interleave
  __shared__ double sbins[kBlock / kWave][kMaxDims * kBins];
  __shared__ double red[2 * kBlock / kWave];
  __shared__ int64_t s_next;
  const uint32_t iter = ctl->iter;
  for (;;) {
    if (threadIdx.x == 0) s_next = (int64_t)atomicAdd(head, 1u);
    __syncthreads();
    const int64_t c = s_next;
    __syncthreads();
    if (c >= n_chunks) break;
    Chunk ch = chunks[c];
    if (!active[ch.integral]) continue;
    if (alloc) {
      // this iteration's points of the integral (Neyman allocation): the
      // chunks past them are skipped, the one across the end is cut
      const int64_t na = alloc[ch.integral];
      if (ch.start >= na) continue;
      if (ch.start + ch.count > na) ch.count = (int32_t)(na - ch.start);
    }
    const IntegralDesc in = ints[ch.integral];
    const int D = in.dims;
    for (int i = threadIdx.x; i < D * (kBins + 1); i += kBlock) sgrid[i] = grids[in.grid_off + i];
    for (int i = threadIdx.x; i < D * kBins; i += kBlock)
#pragma unroll
      for (int w = 0; w < kBlock / kWave; ++w) sbins[w][i] = 0.0;
    const bool strat = sv.sd != nullptr;
    StratChunk sc{sseg, 2, 0, 1, 1, nullptr};
    if (strat) {
      const StratDesc sd = sv.sd[ch.integral];
      const int32_t h0 = sv.h0[ch.id];
      const int nseg = min(min(ch.count / 2 + 2, sd.H + 1 - h0), kStratSeg);
      for (int i = threadIdx.x; i < nseg; i += kBlock) sseg[i] = sv.cum[sd.cum_off + h0 + i];
      sc = StratChunk{sseg, nseg, h0, sd.ns, sd.H, sv.w + sd.w_off};
    }
    __syncthreads();
    const ProcParams& pp = procs[ch.proc];
    double* wbins = sbins[threadIdx.x / kWave];
    double s1 = 0.0, s2 = 0.0;
    double* wrec = (hk.wout && ch.integral == hk.w_int) ? hk.wout + (int64_t)iter * hk.w_stride + ch.start : nullptr;
    const bool poison = ch.event == hk.nan_event;
    if ((KINDS & kMaskDY) && pp.kind == kDY) {
      DYEvent e;
      dy_load(ev, ch.event, e);
      chunk_points<2>(ch, seed, iter, sgrid, wbins, s1, s2, wrec, poison, strat, sc,
                      [&](const double (&x)[2]) { return dy_integrand(pp, e, x); });
    } else if ((KINDS & kMaskTT) && pp.kind == kTT) {
      TTEvent e;
      tt_load(ev, ch.event, ch.perm, e);
      // instances at two or more waves per SIMD (every launch that also
      // carries t tbar H chunks, and the tuner's variants), where the 80 KB
      // of queues would not fit twice: per-lane root loop
      if constexpr (WAVES == 1)
        chunk_points_tt<T, (KINDS & kMaskTT) != 0>(ch, seed, iter, sgrid, wbins, s1, s2, wrec, poison, strat, sc, pp, e);
      else
        chunk_points<8>(ch, seed, iter, sgrid, wbins, s1, s2, wrec, poison, strat, sc,
                        [&](const double (&x)[8]) { return tt_integrand<T>(pp, e, x, nullptr); });
    } else if ((KINDS & kMaskSL) && pp.kind == kSL) {
      SLEvent e;
      sl_load(ev, ev.charge, ch.event, ch.perm, e);
      chunk_points<7>(ch, seed, iter, sgrid, wbins, s1, s2, wrec, poison, strat, sc,
                      [&](const double (&x)[7]) { return sl_integrand<T>(pp, e, x, nullptr); });
    } else if ((KINDS & kMaskTTH) && pp.kind == kTTH) {
      TTHEvent e;
      tth_load(ev, ev.charge, ch.event, ch.perm, e);
      chunk_points<9>(ch, seed, iter, sgrid, wbins, s1, s2, wrec, poison, strat, sc,
                      [&](const double (&x)[9]) { return tth_integrand<T>(pp, e, x, nullptr); });
    } else if ((KINDS & (kMaskTHL | kMaskTBB)) && (pp.kind == kTHL || pp.kind == kTBB)) {
      // the chunk's event is the same for the whole workgroup: one copy in
      // LDS instead of 58 registers per lane across the matrix element
      __shared__ F2Event sf2;
      const bool tth = pp.kind == kTHL;
      if (threadIdx.x == 0) f2_load(ev, tth, ch.event, ch.perm, sf2);
      __syncthreads();
      if ((KINDS & kMaskTHL) && tth)
        chunk_points<8>(ch, seed, iter, sgrid, wbins, s1, s2, wrec, poison, strat, sc,
                        [&](const double (&x)[8]) { return f2_integrand<T, true>(pp, sf2, x, nullptr); });
      else if (KINDS & kMaskTBB)
        chunk_points<8>(ch, seed, iter, sgrid, wbins, s1, s2, wrec, poison, strat, sc,
                        [&](const double (&x)[8]) { return f2_integrand<T, false>(pp, sf2, x, nullptr); });
    }
    block_reduce2<0>(s1, s2, red);
    __syncthreads();
    double* out = parts + ch.part_off;
    if (threadIdx.x == 0) { out[0] = s1; out[1] = s2; }
    for (int i = threadIdx.x; i < D * kBins; i += kBlock) {
      double b = 0.0;
#pragma unroll
      for (int w = 0; w < kBlock / kWave; ++w) b += sbins[w][i];
      out[2 + i] = b;
    }
    __syncthreads();
  }
}

// Damped rebinning of one dimension by one wavefront (lane i = bin i):
// three-point smoothing of the per-bin sums of w^2, importances
// m_i = ((1 - rho_i)/ln(1/rho_i))^alpha, then new edges at equal shares of
// sum m, interpolated linearly inside the old bins (Lepage 1978).  Every
// wavefront of the block must call this (valid = false for idle ones): it
// contains block barriers.  d: the 64 sums; e: the 65 edges, updated in
// place; C, E, M: per-wavefront LDS scratch of 65, 65 and 64 doubles.
__device__ __forceinline__ void refine_dim_wave(const double* d, double* e, double alpha, bool valid,
                                                double* C, double* E, double* M)
{
  const int i = threadIdx.x & (kWave - 1);
  double s = 0.0;
  if (valid) {
    double di = d[i];
    double dm = d[i > 0 ? i - 1 : 0], dp = d[i < kBins - 1 ? i + 1 : kBins - 1];
    if (i == 0) s = 0.5 * (di + dp);
    else if (i == kBins - 1) s = 0.5 * (dm + di);
    else s = (dm + di + dp) / 3.0;
  }
  const double total = wave_sum(s);
  const bool go = valid && total > 0.0;
  double m = 0.0;
  if (go) {
    double rho = s / total;
    if (rho <= 0.0) m = 0.0;
    else if (rho >= 1.0) m = 1.0;
    else m = pow((1.0 - rho) / log(1.0 / rho), alpha);
  }
  const double cum = wave_scan(m);
  const double msum = __shfl(cum, kBins - 1, kWave);
  if (go) {
    C[i + 1] = cum;
    M[i] = m;
    E[i] = e[i];
    if (i == 0) { C[0] = 0.0; E[kBins] = e[kBins]; }
  }
  __syncthreads();
  if (go) {
    if (i >= 1) {
      const double target = msum / (double)kBins * (double)i;
      double edge = 1.0;
      if (C[kBins] >= target) {
        // smallest bin j whose cumulative importance reaches the target
        int lo = 0, hi = kBins - 1;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (C[mid + 1] >= target) hi = mid; else lo = mid + 1;
        }
        edge = E[lo] + (target - C[lo]) / M[lo] * (E[lo + 1] - E[lo]);
      }
      e[i] = edge;
    } else {
      e[0] = 0.0;
      e[kBins] = 1.0;
    }
  }
  __syncthreads();
}

}  // namespace memk
