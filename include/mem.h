/*
 * mem.h - C ABI of the MI355X matrix element method (MEM) integrator.
 *
 * The library computes, for each observed event X and hypothesis i, the
 * MEM density of Schouten, DeAbreu & Stelzer (CPC 2014):
 *   P_i(X) = (1/sigma_i) (1/|perm|) sum_perm sum_flavour
 *            int |M_i|^2 f1 f2 / flux  dPhi_n  T(X|Y) dY
 * (Sec. 1, Eq. mem_def and Eq. 3; Sec. 3, Eq. integrand), estimated by
 * VEGAS Monte Carlo (Sec. 2, Eq. for S_N and its error) entirely on one GPU.
 *
 * Conventions for every call:
 *  - four-vectors are (E, px, py, pz) in GeV, metric (+,-,-,-);
 *  - "device pointer" means memory allocated on the current HIP device;
 *    the library never takes ownership of caller memory;
 *  - a call either completes or returns a status != MEM_OK before it has
 *    written any output; no C++ exception crosses this interface;
 *  - calls that take a stream are stream-ordered: outputs are valid once
 *    the stream has reached the call (unless stated otherwise);
 *  - handles are thread-compatible: concurrent calls are allowed when they
 *    use different streams and different output buffers.
 */
#ifndef MEM_H
#define MEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MEM_OK = 0,
  MEM_EINVAL = 1,       /* invalid argument (null pointer, bad size, NaN input) */
  MEM_ENOMEM = 2,       /* device or host allocation failed */
  MEM_EDEVICE = 3,      /* a HIP runtime call failed */
  MEM_EUNSUPPORTED = 4  /* valid request that the library does not implement */
} mem_status;

/* Process kinds (hypotheses).  Object order expected in mem_events:
 *  MEM_DY_QQ_GAMMA_MUMU  q qbar -> gamma* -> mu- mu+          : mu-, mu+
 *  MEM_TT_DILEPTON       gg/qqbar -> t tbar -> b l+ nu bbar l- nubar
 *                                                   : jet, jet, l+, l-
 *  MEM_TT_SEMILEPTON     gg/qqbar -> t tbar, one W -> l nu, one W -> q qbar'
 *                                   : jet, jet, jet, jet, lepton (charge in
 *                                     mem_events.charge; +1 when null)
 *  MEM_TTH_SEMILEPTON    gg -> t tbar H, H -> b bbar, one W -> l nu, one
 *                        W -> q qbar': b-jet x 4, light jet x 2, lepton
 *                                   (charge as above)
 *  MEM_TTH_DILEPTON      gg -> t tbar H, H -> b bbar, both tops -> b l nu
 *                        (Sec. 4's signal, Eqs. integrand, dilepsolv and
 *                        mhsolve; 8 dimensions, 12 assignments)
 *                                   : b-jet x 4, l+, l-
 *  MEM_TTBB_DILEPTON     gg -> t tbar b bbar, both tops -> b l nu (Sec. 4's
 *                        background; 36 tree-level QCD diagrams; 8
 *                        dimensions, 24 assignments): b-jet x 4, l+, l-
 *  The two dilepton four-b kinds use the b-jet transfer function for all
 *  four jets, take the neutrinos' summed transverse momentum as minus that
 *  of the visible objects (no recoil; sigma_k unused), and integrate in
 *  batches that hold no other kind (MEM_EUNSUPPORTED otherwise); flow
 *  proposals, training capture and parton-level weights do not cover them. */
typedef enum {
  MEM_DY_QQ_GAMMA_MUMU = 1,
  MEM_TT_DILEPTON = 2,
  MEM_TT_SEMILEPTON = 3,
  MEM_TTH_SEMILEPTON = 4,
  MEM_TTH_DILEPTON = 5,
  MEM_TTBB_DILEPTON = 6
} mem_kind;

typedef enum { MEM_FP64 = 0, MEM_FP32 = 1 } mem_precision;

/* Physics description of one hypothesis (Sec. 4: "model parameters").
 * Masses and widths in GeV; alpha, alpha_s dimensionless; g_fermi GeV^-2.
 * sigma_k: width (GeV) of each component of the Gaussian transverse recoil
 * of the hard system (tt kinds).  m_lo, m_hi: Drell-Yan window on the true
 * pair mass.  sigma_norm: the 1/sigma_i of Eq. mem_def; 0 = unnormalised.
 * precision: arithmetic of the matrix element / PDF / TF stage
 * (MEM_FP64 for Drell-Yan, MEM_FP32 or MEM_FP64 for tt).  m_h, w_h: the
 * Higgs; m_b: the b mass in the H -> b bbar coupling (0: 4.18 GeV; the b
 * quarks are massless in the kinematics). */
typedef struct {
  int32_t kind;
  int32_t precision;
  double sqrt_s;
  double m_top, w_top, m_w, w_w, m_h, w_h;
  double alpha, alpha_s, g_fermi;
  double sigma_k;
  double m_lo, m_hi;
  double sigma_norm;
  double m_b;
} mem_process_desc;

typedef struct mem_process_s* mem_process;

/* Transfer functions (Sec. 1, after Eq. 3): a delta for well measured
 * objects, uniform for neutrinos, (double) Gaussian in energy for jets.
 * T(E_meas | E) = sum_k w_k N(E_meas; E, (s_k E)^2) with w = (1-f, f),
 * s = (sigma_core, sigma_tail).  The energy is integrated over
 * r = E_meas / E in [max(r_min, 1 - window s_max), 1 + window s_max]. */
typedef enum { MEM_TF_DELTA = 0, MEM_TF_UNIFORM = 1, MEM_TF_GAUSS = 2, MEM_TF_DGAUSS = 3 } mem_tf_kind;
typedef enum {
  MEM_OBJ_MUON = 0, MEM_OBJ_LEPTON = 1, MEM_OBJ_BJET = 2, MEM_OBJ_LJET = 3, MEM_OBJ_NEUTRINO = 4
} mem_obj_class;
typedef struct {
  int32_t obj_class;    /* mem_obj_class */
  int32_t kind;         /* mem_tf_kind */
  double sigma_core;    /* relative width of the core Gaussian (> 0) */
  double sigma_tail;    /* relative width of the tail Gaussian (DGAUSS) */
  double f_tail;        /* tail fraction in [0,1] (DGAUSS) */
  double window;        /* half width of the r window in units of the widest sigma */
  double r_min;         /* lower floor of r */
} mem_tf_desc;

/* Observed events, SoA: component arrays [n_obj][n_events] (object-major,
 * event index fastest), FP64.  n_obj is the stride: an event uses the first
 * objects its process kind needs (padding objects are ignored).  charge:
 * optional int32 per event, the lepton charge (+1 / -1) of semileptonic
 * events.  on_device != 0: all arrays are device pointers, else host
 * pointers (copied in by the call). */
typedef struct {
  int32_t n_events;
  int32_t n_obj;
  const double* E;
  const double* px;
  const double* py;
  const double* pz;
  const int32_t* charge;
  int32_t on_device;
} mem_events;

/* A learned importance-sampling proposal: a conditional rational-quadratic
 * spline flow on [0,1]^8 for the ttbar dilepton integrand (definition at
 * mem_flow_create).  Owned by the library until mem_flow_destroy. */
typedef struct mem_flow_s* mem_flow;

/* Options of mem_integrate_events; pass NULL for the defaults listed.
 *  seed            Philox key (default: the process seed 0x14077595)
 *  alpha           VEGAS damping exponent (1.5)
 *  target_rel_err  0: run exactly n_iter iterations.  > 0: per event, stop
 *                  once err/P <= target (checked after every iteration from
 *                  the third on) or at max_iter
 *  max_iter        cap in target mode (64)
 *  stream          hipStream_t of the caller (NULL: the null stream)
 *  outputs_on_device  p_out, err_out, status_out are device pointers
 *  iter_out        optional device pointer, [n_iter][n_integrals][2]:
 *                  I_j and sigma_j^2 of every integral and iteration
 *  grid_out        optional device pointer, [n_integrals][D][65]: the VEGAS
 *                  grids after the last refinement
 *  n_iter_out      optional device pointer [n_events]: iterations used
 *  timing_out      optional HOST pointer, 8 doubles: milliseconds spent in
 *                  the integrand kernel (HIP events around every launch on
 *                  `stream`), its number of launches, the number of
 *                  integrand evaluations it performed, the wall time of
 *                  the call in milliseconds, then for a flow: milliseconds
 *                  spent in its sampling kernel, its launches, the points
 *                  it sampled, and the integrand evaluations of the VEGAS
 *                  fallback (all 0 without a flow)
 *  chunk_points    points per work-queue chunk for every process of the
 *                  call (0: each process's tuned value, see mem_autotune,
 *                  else 4096); a multiple of 256 up to 65536
 *  use_graph       0: launch every iteration; 1 (default when the options
 *                  are NULL): capture one iteration as a hipGraph and
 *                  replay it
 *  flow            NULL: the processes' proposal when they share one
 *                  (mem_set_proposal), else VEGAS (Sec. 2).  A flow:
 *                  importance sampling from it instead (ttbar dilepton
 *                  events only).  Batch j of an
 *                  integral draws n_points/n_perm base points z from the
 *                  point stream (counter blocks perm*16 + 8 + d/2,
 *                  iteration j), maps them to x = T^-1(z; c) and weighs
 *                  them by w = f(x)/q(x|c).  The first batch is a pilot:
 *                  every permutation must have ESS/N =
 *                  (sum w)^2/(N sum w^2) >= ess_threshold on it, else the
 *                  whole event is integrated by VEGAS with the same
 *                  arguments (status MEM_EV_FLOW_FALLBACK when that
 *                  converges); its weights do not enter the estimate
 *                  (selected on them, it would bias it).  Batches 2, 3, ...
 *                  of an integral are pooled into one mean and one
 *                  variance; in target mode the stopping test runs after
 *                  each of them.
 *  ess_threshold   flow fallback threshold on ESS/N (0: 0.3)
 *  allocation      how an event's points are shared among its permutations
 *                  (VEGAS, a flow's VEGAS fallback included; the flow's own
 *                  batches ignore it).  MEM_ALLOC_EQUAL (0, the
 *                  default): every iteration gives each permutation
 *                  ceil(n_points / n_perm) points.  MEM_ALLOC_NEYMAN (1): the
 *                  first iteration splits equally; from then on permutation k
 *                  gets a floor of 1/8 of the equal share plus a part of the
 *                  rest proportional to the standard deviation of its weights
 *                  in the previous iteration (Neyman allocation, which
 *                  minimises the variance of the permutation average for a
 *                  fixed total), at most min(n_perm, 4) equal shares; the
 *                  event's total per iteration stays n_perm equal shares up
 *                  to that cap.  Same point stream (point k of an integral is
 *                  the same u in either mode); estimates differ from equal
 *                  splitting by MC fluctuation only.  Other values:
 *                  MEM_EINVAL.
 *  weights_out     optional device pointer [weights_rows][weights_stride]
 *                  doubles: the weight w = f(x) J(x) of every point the
 *                  integrand kernel evaluates for integral weights_integral
 *                  (integral index = sum of the earlier events'
 *                  permutation counts + permutation), at
 *                  [iteration][point index k], iterations counted from the
 *                  start of the integration (a resumed checkpoint's
 *                  iterations included).  Entries an iteration does not
 *                  evaluate are left as they were.  weights_stride must be
 *                  at least the integral's points per iteration (its equal
 *                  share, times min(n_perm, 4) under Neyman allocation) and
 *                  weights_rows at least the last iteration index the call
 *                  can reach plus one (n_iter, or max_iter in target mode,
 *                  plus a resumed checkpoint's iterations in fixed mode);
 *                  otherwise MEM_EINVAL before any launch.  VEGAS only
 *                  (MEM_EUNSUPPORTED with a flow).
 *  hooks, hook_event  test hooks (MEM_HOOK_*; 0 = none)
 *  checkpoint      NULL, or a handle from mem_checkpoint_create (VEGAS only;
 *                  MEM_EUNSUPPORTED with a flow).  An empty handle: the
 *                  integration starts afresh.  A handle holding the state
 *                  of an earlier call over the same events, processes,
 *                  n_points, seed, alpha and allocation: the integration
 *                  resumes from it (grids, cumulative sums, iteration
 *                  count, retired events, allocations) and runs n_iter
 *                  more iterations (fixed mode) or continues to the target
 *                  or to max_iter iterations in total (target mode); the
 *                  result equals that of one uninterrupted call bit for
 *                  bit.  A handle whose state does not match: MEM_EINVAL.
 *                  In every case the handle holds the final state when the
 *                  call returns MEM_OK (unchanged otherwise).
 *  alloc_fn, free_fn, alloc_user  optional allocator for the call's
 *                  device work buffers (both or neither); NULL: hipMalloc
 *                  and hipFree.
 *  flow_mode       how a flow (given or the processes' proposal) is used:
 *                  MEM_FLOW_SAMPLE (0): importance sampling from it, as
 *                  described under `flow`;
 *                  MEM_FLOW_SEED_GRID: VEGAS whose grids start from the
 *                  flow instead of uniform ones: 1024 flow samples of each
 *                  integral (the flow's point stream at iteration
 *                  0xFFFFFFF0) give, per dimension, edges at the quantiles
 *                  k/64 of 0.8 x (sample CDF) + 0.2 x (uniform CDF); every
 *                  iteration then enters the estimate (the first one too)
 *                  and the stopping test runs from the second iteration.
 *                  Each iteration is still VEGAS importance sampling on
 *                  its own grid, so the estimate stays unbiased; ttbar
 *                  dilepton processes only (MEM_EUNSUPPORTED), no
 *                  ess_threshold.  Other values: MEM_EINVAL.
 *  stratify        MEM_STRATIFY_OFF (0, the default): plain VEGAS
 *                  importance sampling (Sec. 2).  MEM_STRATIFY_ADAPTIVE (1):
 *                  adaptive stratified sampling on top of the grid (Lepage,
 *                  J. Comput. Phys. 439 (2021) 110386).  Per integral of N
 *                  points per iteration and D dimensions, the map's input
 *                  cube is cut into H = n_s^D equal hypercubes, n_s the
 *                  largest integer with 2 n_s^D <= N and n_s^D <= 16384;
 *                  hypercube h (digits c_d of h in base n_s, dimension 0
 *                  least significant) gets n_h of the N points, taken in
 *                  hypercube order: point k of the iteration (the k-th
 *                  draw of the point stream, as without stratification)
 *                  lies in the hypercube whose cumulative range holds k
 *                  and enters the map as y_d = (c_d + u_d) / n_s.  The
 *                  iteration estimate is sum_h mean_h(w) / H with variance
 *                  sum_h s_h^2 / (H^2 n_h) (s_h^2 the sample variance of
 *                  the weights in h); the grid adapts from the per-bin sums
 *                  of w^2 / (H n_h).  The first iteration splits N equally
 *                  (floor(N / H) each, one more to the first N mod H
 *                  hypercubes); afterwards every hypercube keeps 2 points
 *                  and the other N - 2H go out in proportion to s_h^0.75,
 *                  rounded down, the remainder one each to the first
 *                  hypercubes in index order (equal split again when every
 *                  s_h is 0 or their sum is not finite).  Iterations are
 *                  combined as without stratification.  Work-queue chunks
 *                  are capped at 4096 points.  Requires the equal split
 *                  across permutations (MEM_EINVAL with MEM_ALLOC_NEYMAN);
 *                  no flow and no checkpoint (MEM_EUNSUPPORTED).  Device
 *                  memory on top of plain VEGAS: 8 bytes per point of an
 *                  iteration and 12 per hypercube.  Other values:
 *                  MEM_EINVAL.
 *  combine         how an integral's kept iterations (the second on; the
 *                  first on with flow-seeded grids) form its estimate
 *                  (VEGAS; a flow's own batches are pooled regardless).
 *                  MEM_COMBINE_WEIGHTED (0, the default): inverse-variance
 *                  weights, I = sum(I_j / s_j^2) / sum(1 / s_j^2), error^2
 *                  = 1 / sum(1 / s_j^2) (Lepage 1978).  MEM_COMBINE_MEAN
 *                  (1): equal weights, I = mean of the I_j, error^2 =
 *                  sum s_j^2 / n^2.  Every I_j is unbiased given its grid,
 *                  which earlier iterations fixed, so the mean is unbiased;
 *                  the weighted form runs low where budgets are small
 *                  against the integrand's peaks (an iteration that missed
 *                  the large weights has a low I_j and a low s_j^2 and so
 *                  the larger weight), at the price of a larger error when
 *                  the grid is still improving.  The stopping test of
 *                  target mode uses the chosen estimate.  Other values:
 *                  MEM_EINVAL.
 *  tail_chunk_points, tail_iter
 *                  work-queue chunks of the late iterations: 0 (the
 *                  default) keeps every iteration at the call's chunk size;
 *                  otherwise, from iteration tail_iter (>= 1, counted from
 *                  the integration's start, a resumed checkpoint's
 *                  iterations included) on, every integral's points are cut
 *                  into chunks of tail_chunk_points (a multiple of 256, at
 *                  most 65536) instead.  In target mode the late iterations
 *                  carry few events, whose few long chunks leave most of
 *                  the GPU idle; shorter chunks spread them.  The chunking
 *                  of an iteration depends only on its index, so a target-
 *                  mode event equals a fixed run with the same options bit
 *                  for bit; a different chunking changes the order of the
 *                  partial sums, hence the last bits of the grids and the
 *                  points drawn after them.  Work buffers grow by the tail
 *                  table (chunk table and partials).  Not with stratify
 *                  (MEM_EUNSUPPORTED).  Invalid values: MEM_EINVAL.     */
enum { MEM_ALLOC_EQUAL = 0, MEM_ALLOC_NEYMAN = 1 };
enum { MEM_FLOW_SAMPLE = 0, MEM_FLOW_SEED_GRID = 1 };
enum { MEM_STRATIFY_OFF = 0, MEM_STRATIFY_ADAPTIVE = 1 };
enum { MEM_COMBINE_WEIGHTED = 0, MEM_COMBINE_MEAN = 1 };

/* Per-integral state of a VEGAS integration, owned by the library (see
 * mem_checkpoint_create). */
typedef struct mem_checkpoint_s* mem_checkpoint;

/* Device memory for the work buffers of a call, supplied by the caller
 * (for instance a caching allocator).  alloc_fn returns `bytes` of device
 * memory on the current device usable on `stream` (NULL: failure, the call
 * returns MEM_ENOMEM); free_fn gets back every block alloc_fn returned,
 * with its size, once the call's work on `stream` has completed and before
 * the call returns.  `user` is passed through. */
typedef void* (*mem_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*mem_free_fn)(void* ptr, size_t bytes, void* stream, void* user);

/* Test hooks (mem_integrate_opts.hooks): conditions forced from the host so
 * that failure handling can be exercised with valid inputs.
 *  MEM_HOOK_NONFINITE  every integrand weight of event hook_event is
 *                      replaced by a quiet NaN (VEGAS: the event ends with
 *                      status MEM_EV_NONFINITE; its grids stay unrefined) */
enum { MEM_HOOK_NONFINITE = 1 };

typedef struct {
  uint64_t seed;
  double alpha;
  double target_rel_err;
  int32_t max_iter;
  void* stream;
  int32_t outputs_on_device;
  double* iter_out;
  double* grid_out;
  int32_t* n_iter_out;
  double* timing_out;
  int32_t chunk_points;
  int32_t use_graph;
  mem_flow flow;
  double ess_threshold;
  int32_t allocation;
  double* weights_out;
  int64_t weights_stride;
  int32_t weights_integral;
  int32_t weights_rows;
  uint32_t hooks;
  int32_t hook_event;
  mem_checkpoint checkpoint;
  mem_alloc_fn alloc_fn;
  mem_free_fn free_fn;
  void* alloc_user;
  int32_t flow_mode;
  int32_t stratify;
  int32_t combine;
  int32_t tail_chunk_points;
  int32_t tail_iter;
} mem_integrate_opts;

/* Per-event status codes written to status_out. */
enum {
  MEM_EV_OK = 0,
  MEM_EV_ZERO_INTEGRAND = 1,   /* every sampled weight was zero: P = err = 0 */
  MEM_EV_NOT_CONVERGED = 2,    /* target mode: max_iter reached */
  MEM_EV_NONFINITE = 3,        /* a non-finite weight was produced */
  MEM_EV_FLOW_FALLBACK = 4     /* flow proposal below the ESS threshold; the
                                  event was integrated by VEGAS instead */
};

/* Create a hypothesis (Sec. 1: process i).  Errors: MEM_EINVAL for a null
 * pointer, unknown kind, non-positive sqrt_s/masses/widths or
 * m_hi <= m_lo for Drell-Yan; MEM_EUNSUPPORTED for Drell-Yan in FP32;
 * MEM_ENOMEM.  The handle is owned by the library until
 * mem_destroy_process.  Default TFs: muon Gaussian 5 %, b-jet Gaussian 15 %
 * (double Gaussian 10 %/25 %, tail 0.2 for t tbar H), light jet double
 * Gaussian 10 %/25 %, tail 0.2; window 5, r_min 0.1. */
mem_status mem_create_process(const mem_process_desc* d, mem_process* out);

/* Replace the TF of the listed object classes (copied in).  MEM_EINVAL on
 * unknown class or kind, sigma <= 0, f_tail outside [0,1], window <= 0. */
mem_status mem_set_transfer_functions(mem_process p, const mem_tf_desc* tf, int32_t n);

void mem_destroy_process(mem_process p);

/* Parton densities from a table (Sec. 4: the densities of d, u, s, c, b,
 * their antiquarks and the gluon are stored on (x, Q) grids and
 * interpolated bilinearly inside the integrand).
 *  xf      host array [nq][nx][11] float: x f(x, Q) of flavour fl = -5..5
 *          (PDG codes: 1 d, 2 u, 3 s, 4 c, 5 b, negative for antiquarks,
 *          0 the gluon) at index fl + 5, at node (ix, iq) with
 *            ln x = bounds[0] + ix (bounds[1] - bounds[0]) / (nx - 1),
 *            ln Q = bounds[2] + iq (bounds[3] - bounds[2]) / (nq - 1);
 *          copied to the current device; every later call with this
 *          process returns MEM_EINVAL on another current device.  NULL
 *          restores the built-in toy densities.
 *  nx, nq  >= 2 each; nx * nq <= 2^22
 *  bounds  ln x and ln Q ranges (natural logarithms), increasing; the
 *          first and last nodes sit on them.  A table laid out for a reader
 *          that steps by (max - min)/n (nodes at min + i (max - min)/n,
 *          i < n, as the paper's interpolation listing does) is the same
 *          grid with the upper bound min + (n - 1)(max - min)/n: pass that.
 * Outside the grid the edge cells extrapolate linearly.  Factorisation
 * scale (not stated in the paper): the muon pair mass for Drell-Yan, m_t
 * for the top processes.  Errors: MEM_EINVAL for a null process or bounds,
 * nx or nq < 2, a grid above the size limit, bounds not increasing or not
 * finite, a non-finite table entry; MEM_EUNSUPPORTED for t tbar H (its
 * integrand keeps the toy gluon density); MEM_ENOMEM. */
mem_status mem_set_pdf_grid(mem_process p, const float* xf, int32_t nx, int32_t nq, const double* bounds);

/* The library's toy densities tabulated at the nodes of such a grid into
 * the caller's host array xf [nq][nx][11] (u and d valence-like, a common
 * sea for ubar and dbar, the gluon; s, c, b and their antiquarks zero;
 * zero at x >= 1).  MEM_EINVAL as for mem_set_pdf_grid. */
mem_status mem_toy_pdf_table(float* xf, int32_t nx, int32_t nq, const double* bounds);

/* Event discriminant of Sec. 4, D = log10(p_sig / p_bkg), per event: for
 * the t tbar H and t tbar b bbar densities of mem_integrate_events on the
 * same events.  p_sig, p_bkg, d_out: device arrays of n doubles (caller
 * owned; d_out may alias neither input).  p_sig > 0 with p_bkg == 0 gives
 * +inf, the reverse -inf, both zero NaN.  Asynchronous on stream.
 * MEM_EINVAL for n < 0 or null arrays with n > 0. */
mem_status mem_discriminant(const double* p_sig, const double* p_bkg, int64_t n, double* d_out, void* stream);

/* Integration dimension and number of jet-parton assignments of a process. */
mem_status mem_process_shape(mem_process p, int32_t* dims, int32_t* n_perm);

/* The MEM density of every event (Sec. 1 Eq. mem_def, Sec. 3 Eq. integrand).
 *  ev        events (see mem_events); n_obj must match the process kind
 *  hyp       one process per event (n_hyp == n_events), or one for all
 *            (n_hyp == 1)
 *  n_points  VEGAS points per event per iteration, split equally over the
 *            permutations (ceil); one per event (n_np == n_events) or one
 *            for all (n_np == 1); each >= 2
 *  n_iter    iterations (>= 2; the first adapts the grid only)
 *  p_out, err_out   P_i and its MC error per event
 *  status_out       MEM_EV_* per event
 * Errors: MEM_EINVAL (null pointers, sizes, non-finite or non-positive
 * energies in host-side events), MEM_ENOMEM, MEM_EDEVICE.  Device-resident
 * events are not scanned for NaNs; a NaN gives status MEM_EV_NONFINITE. */
mem_status mem_integrate_events(const mem_events* ev, const mem_process* hyp, int32_t n_hyp,
                                const int64_t* n_points, int32_t n_np, int32_t n_iter,
                                const mem_integrate_opts* opt,
                                double* p_out, double* err_out, int32_t* status_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * mem_integrate_events with every work buffer (process table, work queue,
 * grids, chunk partials, running state) placed in a fixed scratch array of
 * MEM_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
 * on, from the first call on that device until the process ends.  The call
 * allocates no device memory, creates no stream, graph or event, and runs
 * the iterations as direct launches on opt->stream (NULL: the null stream)
 * of the current device.
 *   Arguments and results as mem_integrate_events, with these limits: opt
 *   is required, events (ev->on_device) and outputs (opt->outputs_on_device)
 *   are device memory, VEGAS only (opt->flow or the processes' proposal:
 *   MEM_EUNSUPPORTED), no
 *   timing_out (MEM_EUNSUPPORTED), no allocator hook (MEM_EINVAL).  A call
 *   whose work buffers exceed the scratch returns MEM_ENOMEM before any copy
 *   or launch, with the bytes it would need in mem_last_error (the buffers
 *   grow with the number of integrals and of work-queue chunks: about
 *   2 + 64 D doubles per chunk of chunk_points points, some 75 KB per
 *   dilepton event at 65 536 points per iteration under the equal split
 *   and twice that under Neyman allocation).
 *   Every call on a device shares that device's scratch, which keeps the
 *   last call's contents (the call initialises what it reads).  Calls that
 *   overlap in time on one device (other host threads, other streams) race
 *   on it: the caller serialises them.  Returns after opt->stream has
 *   completed the call's work. */
#define MEM_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
mem_status mem_integrate_events_noalloc(const mem_events* ev, const mem_process* hyp, int32_t n_hyp,
                                        const int64_t* n_points, int32_t n_np, int32_t n_iter,
                                        const mem_integrate_opts* opt, double* p_out, double* err_out,
                                        int32_t* status_out);

/* Checkpoints of VEGAS integrations (per-integral grids, cumulative sums,
 * iteration counter, retired events and allocations, held in host memory).
 * create: an empty handle.  save: write the state to a file (MEM_EINVAL for
 * an empty handle or an unwritable path).  load: a new handle from a file
 * written by save (MEM_EINVAL for an unreadable or malformed file).  A
 * handle is used by one call at a time. */
mem_status mem_checkpoint_create(mem_checkpoint* out);
void mem_checkpoint_destroy(mem_checkpoint c);
mem_status mem_checkpoint_save(mem_checkpoint c, const char* path);
mem_status mem_checkpoint_load(const char* path, mem_checkpoint* out);
/* Iterations the state holds (0 for an empty handle). */
mem_status mem_checkpoint_iterations(mem_checkpoint c, int32_t* n_iter);

/* ---- autotuner ----
 * The launch configuration of a process's integrand kernel, per device:
 *  - points per work-queue chunk (the tile one workgroup of 256 threads
 *    integrates, so chunk_points / 256 points per thread): queue overhead
 *    and per-chunk partial sums against load balance and tail effects;
 *  - waves per SIMD the kernel is compiled for (its launch bounds: a
 *    register budget of 512 / waves per lane), i.e. latency hiding
 *    against register spills.  Compiled variants: Drell-Yan 1, 2, 4; t tbar
 *    H 2; the other kinds 1 and 2 (the first of each list is the
 *    default).  At one wave per SIMD the dilepton kernel compacts its root
 *    searches through LDS; at two it runs them per lane (the same
 *    arithmetic, contracted differently by the compiler).
 *    A launch that mixes kinds uses their default variant.
 * mem_autotune times an integration of the given events (n_points per
 * event per iteration) with every pair of a chunk candidate (NULL: 1024,
 * 2048, 4096, 8192, 16384; each a multiple of 256 <= 65536) and a waves
 * candidate (NULL: every compiled variant of the kind), the better of two
 * runs (seeds base seed and base seed + 1), by the host clock around the
 * call.  The timed call is mem_integrate_events with `base`'s options
 * (target mode, allocation, stratification, stream, ...; its outputs go to
 * host memory and its recording options, hooks and checkpoint are
 * ignored) and n_iter iterations; base NULL: n_iter = 2 with the default
 * options.  Tune with the options the process will run with: a target-mode
 * run spends its late iterations on a few events, where smaller chunks
 * balance better than a fixed-budget run shows.  The fastest pair is kept
 * in the process (used by every later mem_integrate_events call whose
 * options do not set chunk_points) and reported in best_out,
 * best_waves_out and rate_out (events per second of the timed call; all
 * optional).  table_path (optional): a text table of lines "arch kind
 * precision chunk_points waves_per_simd events_per_s", created or updated
 * in place for this device and process.  Errors: MEM_EINVAL (null
 * process, no events, bad candidates, a waves candidate not compiled for
 * the kind, unwritable table), the errors of mem_integrate_events. */
mem_status mem_autotune(mem_process p, const mem_events* ev, int64_t n_points, int32_t n_iter,
                        const mem_integrate_opts* base, const int32_t* candidates, int32_t n_cand,
                        const int32_t* waves, int32_t n_waves, const char* table_path, int32_t* best_out,
                        int32_t* best_waves_out, double* rate_out);

/* Look up the tuned launch configuration of a process in a table written
 * by mem_autotune, for architecture `arch` (e.g. "gfx950"; NULL: the
 * current device's).  found (optional) is set to 1 when the entry exists;
 * a missing entry is not an error.  MEM_EINVAL for an unreadable table or
 * a malformed entry (including a waves value not compiled for the kind). */
mem_status mem_tuning_load(mem_process p, const char* table_path, const char* arch, int32_t* found);

/* Set the launch configuration directly: chunk_points 0 or a multiple of
 * 256 <= 65536 (0: the library default, 4096), waves 0 or a compiled
 * variant of the kind (0: the default).  MEM_EINVAL otherwise. */
mem_status mem_process_set_launch(mem_process p, int32_t chunk_points, int32_t waves);

/* The waves-per-SIMD variant integrations of this process use. */
mem_status mem_process_waves(mem_process p, int32_t* waves);

/* The chunk size integrations of this process use by default. */
mem_status mem_process_chunk_points(mem_process p, int32_t* chunk_points);

/* ---- building blocks of the path, exposed for checks and custom drivers ---- */

/* Uniform point stream of the estimator (Sec. 2): for k = 0..n-1 writes
 * u[k*D + d] in [0,1), 53-bit, from Philox4x32-10 with key = seed and
 * counter {k, iter, event, perm*16 + d/2}.  u: device pointer, n*D doubles. */
mem_status mem_uniforms(uint64_t seed, uint32_t iter, uint32_t event, uint32_t perm,
                        int32_t D, int64_t n, double* u, void* stream);

/* Integrand f(x) of one (event, permutation) at n points x in [0,1]^D (no
 * VEGAS Jacobian).  x: device [n][D]; f: device [n]; nsol: optional device
 * [n], number of accepted neutrino solutions (tt kinds).  ev as in
 * mem_integrate_events; event indexes it. */
mem_status mem_eval_points(mem_process p, const mem_events* ev, int32_t event, int32_t perm,
                           const double* x, int64_t n, double* f, int32_t* nsol, void* stream);

/* Parton-level weights (Sec. 4's parton-level timing: transfer functions
 * are delta functions, so nothing is integrated and the method reduces to
 * the matrix element at the given momenta).  ttbar dilepton processes
 * only.  Event e holds six objects in this order: b, bbar, l+, l-, nu,
 * nubar (massless, GeV).  Per assignment of the two b partons (as given,
 * then swapped), the final state is boosted to zero transverse momentum,
 * x1, x2 = (E' +- P_z) / sqrt(S), and
 *   w = (2 / S) (E / E') sum_channels f(x1) f(x2) |M|^2 / (2 shat)
 * (gg and the two q qbar orderings; |M|^2 with its couplings, the top and
 * W Breit-Wigner propagators at the partons' virtualities, spin and colour
 * averages); w_out[e] is the average over the two assignments, 0
 * where x1 or x2 leaves (0, 1].  FP32 or FP64 per the process precision.
 * w_out: n_events doubles, device memory when ev->on_device, else host
 * (may be null when n_events is 0).
 * MEM_TTH_DILEPTON and MEM_TTBB_DILEPTON (Sec. 4's parton-level timing,
 * its Table 2): objects b quarks 0-3 (any order), l+, l-, nu, nubar; the
 * same formula with the gg channel, the complete t tbar H (with H -> b bbar
 * and the Higgs Breit-Wigner) or t tbar b bbar |M|^2, averaged over the 12
 * or 24 placements of the four b quarks.
 * MEM_EUNSUPPORTED for other kinds; MEM_EINVAL for null pointers, fewer
 * than 6 objects (8 for the four-b kinds), or (host events) non-finite or
 * non-positive-energy objects. */
mem_status mem_parton_weights(mem_process p, const mem_events* ev, double* w_out, void* stream);

/* VEGAS damped rebinning (Lepage 1978) of n_int x D grids in place from
 * per-bin sums of w^2.  bins: device [n_int][D][64]; grids: device
 * [n_int][D][65]; alpha > 0. */
mem_status mem_vegas_refine(const double* bins, double* grids, int32_t n_int, int32_t D,
                            double alpha, void* stream);

/* Points of adapted VEGAS grids and their weights, the training samples of
 * the flow.  For integral i = (event[i], perm[i]) with grid
 * grids[i][D][65] (as written by mem_integrate_events' grid_out) and
 * k < n_per: u from the point stream (seed, iter), x = VEGAS map of u, and
 * w = f(x) J(x) (Sec. 2: the weight of x is its share of the integral).
 * x_out: device float [n_int][n_per][D]; w_out: device float
 * [n_int][n_per]; normalise != 0 divides each integral's weights by their
 * sum.  event, perm: device int32 [n_int].  Every process kind (D = 2, 8,
 * 7, 9 for Drell-Yan, dilepton, semileptonic, t tbar H); w is rounded to
 * FP32 (t tbar H weights, ~1e-40 with the physical constants, come out
 * subnormal or zero).  MEM_EINVAL on null pointers or n_per < 1. */
mem_status mem_vegas_capture(mem_process p, const mem_events* ev, const int32_t* event, const int32_t* perm,
                             int32_t n_int, const double* grids, int64_t n_per, uint64_t seed, uint32_t iter,
                             int32_t normalise, float* x_out, float* w_out, void* stream);

/* ---- learned proposal (conditional rational-quadratic spline flow) ----
 * Density of x in [0,1]^8 given an event context c (24 floats):
 * q(x|c) = |det dT/dx| with T = 6 coupling layers (Durkan et al. 2019
 * splines, 8 bins, minimum bin width/height/derivative 1e-3, boundary
 * derivative 1).  Coordinates are reversed before layer 3; layer l
 * transforms positions {1,3,5,7} (l even) or {0,2,4,6} (l odd) given the
 * other four and c, through an MLP 28 -> 128 -> 128 -> 92 with SiLU whose
 * output at 23 j holds 8 width, 8 height and 7 derivative logits of the
 * j-th transformed position (derivative = 1e-3 + softplus(logit + c0),
 * c0 = ln(e^0.999 - 1), so zero logits give the identity).  Parameters:
 * FP32 master copy, per layer row-major W1[128][28], b1[128],
 * W2[128][128], b2[128], W3[92][128], b3[92] (192 552 floats); the two
 * 128-wide layers run as BF16 matrix products with FP32 accumulation.
 * Context of (event, perm), ttbar dilepton objects jet, jet, l+, l- with
 * the jets swapped when perm = 1: for each of the four objects and for
 * their sum (log(E/100), px/100, py/100, pz/100), then (log((|m|+1)/100),
 * m_x/100, m_y/100, 0) of m = -(sum p_T). */
#define MEM_FLOW_NPARAMS 192552
#define MEM_FLOW_CONTEXT 24

/* Arithmetic of the two 128-wide layers of every coupling MLP (forward
 * passes; products always accumulate in FP32):
 *  MEM_FLOW_BF16    activations rounded to BF16 (one matrix-core product)
 *  MEM_FLOW_BF16X2  activations split into two BF16 terms, hi = bf16(h) and
 *                   lo = bf16(h - hi) (about 16 significant bits; two
 *                   products per layer)
 * Weights are always the BF16 copies of the FP32 master parameters. */
enum { MEM_FLOW_BF16 = 0, MEM_FLOW_BF16X2 = 1 };

/* New flow with every parameter zero (the identity map, q = 1).
 * MEM_EINVAL for an unknown mode. */
mem_status mem_flow_create(int32_t mode, mem_flow* out);
void mem_flow_destroy(mem_flow f);
/* Copy all MEM_FLOW_NPARAMS parameters in (set; resets the Adam state) or
 * out (get).  on_device: params is a device pointer, else host.  n must be
 * MEM_FLOW_NPARAMS.  Synchronous. */
mem_status mem_flow_set_params(mem_flow f, const float* params, int64_t n, int32_t on_device);
mem_status mem_flow_get_params(mem_flow f, float* params, int64_t n, int32_t on_device);

/* Contexts of n (event, perm) pairs of ttbar dilepton events.  event, perm:
 * device int32 [n]; ctx: device float [n][24]. */
mem_status mem_flow_context(const mem_events* ev, const int32_t* event, const int32_t* perm, int32_t n,
                            float* ctx, void* stream);

/* Sample n_per points of each of n_int contexts: z_k from the point stream
 * (seed, iter, event[i], counter blocks perm[i]*16 + 8 + d/2; float of the
 * 53-bit uniform, at most 1 - 2^-24), x = T^-1(z; c_i) and log q(x|c_i).
 * ctx: device [n_int][24]; event, perm: device int32 [n_int]; x_out:
 * device float [n_int][n_per][8]; logq_out: device float [n_int][n_per]. */
mem_status mem_flow_sample(mem_flow f, const float* ctx, const int32_t* event, const int32_t* perm, int32_t n_int,
                           int64_t n_per, uint64_t seed, uint32_t iter, float* x_out, float* logq_out,
                           void* stream);

/* log q(x_i | ctx[sint_i]) of n points (x: device float [n][8]; sint:
 * device int32 [n], rows of ctx; logq_out: device float [n]). */
mem_status mem_flow_log_prob(mem_flow f, const float* ctx, const int32_t* sint, const float* x, int64_t n,
                             float* logq_out, void* stream);

/* One training step on the weighted negative log-likelihood
 * L = -sum_i wt_i log q(x_i | ctx[sint_i]): gradient by the flow's own
 * backward kernels (FP32 accumulation of BF16 products), then, if lr > 0,
 * one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master
 * parameters.  loss_out: optional HOST double (L; synchronises);
 * grad_out: optional device float [MEM_FLOW_NPARAMS] (dL/dparams).
 * Arrays as in mem_flow_log_prob; wt: device float [n].  Calls on one flow
 * are serialised by the caller. */
mem_status mem_flow_train_step(mem_flow f, const float* ctx, const int32_t* sint, const float* x, const float* wt,
                               int64_t n, double lr, double* loss_out, float* grad_out, void* stream);

/* Training of the proposal on one call (the learned importance sampling
 * of the integrand; the method's own sampling idea is Sec. 2's importance
 * sampling, the flow is this library's): VEGAS runs over the training
 * events (vegas_iter iterations of vegas_points points per event), the
 * adapted grids give `capture` samples (x, f(x) J(x) normalised per
 * integral) of every (event, assignment) integral, and the flow is fitted
 * to them by minimising -sum w log q(x|c) over shuffled minibatches of
 * `batch` consecutive samples (whole integrals' samples), `epochs` passes,
 * Adam with a cosine learning rate from lr_max to lr_min.  Zero fields take
 * the defaults in brackets. */
typedef struct {
  int32_t mode;            /* MEM_FLOW_BF16 or MEM_FLOW_BF16X2 */
  int32_t vegas_iter;      /* [4] adaptation iterations, >= 2 */
  int64_t vegas_points;    /* [8192] VEGAS points per training event and iteration */
  int32_t capture;         /* [168] samples per training integral */
  int32_t batch;           /* [65536] samples per minibatch */
  int32_t epochs;          /* [24] */
  int32_t pad;
  double lr_max, lr_min;   /* [2e-3, 1e-4] */
  uint64_t seed;           /* point streams (VEGAS and capture) and minibatch order */
  void* stream;            /* hipStream_t (NULL: the null stream) */
  double* loss_out;        /* optional host [epochs]: the loss per integral of each epoch's first minibatch */
} mem_flow_desc;

/* Train a proposal for process p (MEM_TT_DILEPTON; other kinds
 * MEM_EUNSUPPORTED) on the events `train` (host or device, as in
 * mem_integrate_events); f: NULL for the defaults.  On MEM_OK *out is a new
 * flow owned by the caller (mem_flow_destroy).  Deterministic for fixed
 * inputs.  MEM_EINVAL: bad sizes (fewer samples than a batch, more than
 * 2^31), unknown mode, lr_min > lr_max. */
mem_status mem_train_proposal(mem_process p, const mem_events* train, const mem_flow_desc* f, mem_flow* out);

/* Default proposal of integrations of process p: mem_integrate_events uses
 * f when its options name no flow and every process of the call has the
 * same proposal (NULL clears it: VEGAS).  The flow stays owned by the
 * caller and must outlive its use.  MEM_EUNSUPPORTED for kinds other than
 * MEM_TT_DILEPTON. */
mem_status mem_set_proposal(mem_process p, mem_flow f);

/* A flow to a file and back: parameters, Adam moments and step count
 * (mode included).  save: MEM_EINVAL for an unwritable path.  load: a new
 * flow (caller-owned); MEM_EINVAL for an unreadable or malformed file. */
mem_status mem_flow_save(mem_flow f, const char* path);
mem_status mem_flow_load(const char* path, mem_flow* out);

const char* mem_status_string(mem_status s);
/* Copies the message of the last failed call on this thread (may be empty). */
mem_status mem_last_error(char* buf, size_t n);

#ifdef __cplusplus
}
#endif
#endif
