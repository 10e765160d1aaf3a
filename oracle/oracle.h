/*
 * Oracle for the matrix element method (MEM) integration path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, double-precision CPU
 * implementation of what the GPU library computes.  It shares no code,
 * header, table or constant generator with the HIP library; only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  Every function cites the passage of Schouten, DeAbreu & Stelzer,
 * "Accelerated Matrix Element Method with Parallel Computing" (CPC 2014)
 * that it follows, or names the published method it writes out.
 *
 * Conventions (fixed here, stated once):
 *   metric (+,-,-,-); four-vectors are double[4] = {E, px, py, pz};
 *   Dirac representation for gamma matrices; sums over spins use complete
 *   bases of Dirac spinors, sums over gluon polarisations use the two
 *   linear transverse polarisations.
 */
#ifndef MEM_ORACLE_H
#define MEM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ RNG -- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its
 * published definition: 10 rounds of two 32x32->64 multiplications with a
 * Weyl-sequence key schedule. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The point stream of the MC estimator (Sec. 2, Eq. for S_N): uniform
 * u in [0,1)^D for point k of iteration `iter` of integral (event, perm).
 * Dimension pair (2b, 2b+1) comes from one Philox call with counter
 * {k, iter, event, perm*16 + b}; each 64-bit half (w0<<32|w1, w2<<32|w3)
 * is shifted right by 11 and scaled by 2^-53. */
void or_uniforms(uint64_t seed, uint32_t k, uint32_t iter, uint32_t event,
                 uint32_t perm, int D, double* u);
void or_uniforms_block(uint64_t seed, uint32_t k, uint32_t iter, uint32_t event,
                       uint32_t perm, uint32_t block0, int D, double* u);

/* ---------------------------------------------------------------- VEGAS -- */
#define OR_NBINS 64
/* Lepage's VEGAS map (J. Comput. Phys. 27 (1978) 192): grid holds D rows of
 * 65 edges.  Returns the Jacobian, writes x. */
double or_vegas_map(const double* grid, int D, const double* u, double* x, int* bins);
void   or_vegas_uniform_grid(double* grid, int D);
/* damped rebinning of one dimension from its per-bin sums of w^2 */
void   or_vegas_refine_dim(const double* d_in, double alpha, double* edges);

/* -------------------------------------------------------------- physics -- */
typedef struct {
  double sqrt_s;
  double m_t, w_t, m_w, w_w;
  double alpha;        /* QED coupling (Drell-Yan) */
  double alpha_s;      /* strong coupling, fixed */
  double g_fermi;      /* G_F in GeV^-2 */
  double sigma_k;      /* Gaussian width of each component of the recoil k_T */
  double tf_sigma;     /* relative width of the Gaussian energy TF */
  double r_lo, r_hi;   /* integration window of r = E_meas / E_true */
  double m_lo, m_hi;   /* Drell-Yan truth window on m_mumu */
  /* light-jet double-Gaussian TF and its r window (semileptonic) */
  double lj_core, lj_tail, lj_ftail, lj_r_lo, lj_r_hi;
  /* Higgs mass and width, b mass in the H -> b bbar coupling (ttH) */
  double m_h, w_h, m_b;
  /* parton densities from a grid (or_pdf_grid below); NULL: the toy
   * densities */
  const struct or_pdf_grid_s* pdf;
} or_params;

/* ------------------------------------------------------------ PDF grids -- */
/* Parton densities from a table (Sec. 4: the densities of d, u, s, c, b,
 * their antiquarks and the gluon are stored on grids in (x, Q) and
 * evaluated by bilinear interpolation).  Readings: the grid is uniform in
 * (ln x, ln Q) with its first and last nodes on the bounds,
 *   ln x_i = lx_min + i (lx_max - lx_min) / (nx - 1),  i = 0 .. nx - 1,
 * ln Q likewise, and holds x f(x, Q) of the 11 flavours fl = -5 .. 5
 * (PDG codes: 1 d, 2 u, 3 s, 4 c, 5 b, negative for the antiquarks, 0 for
 * the gluon) at index fl + 5, laid out [nq][nx][11]. */
typedef struct or_pdf_grid_s {
  int nx, nq;
  double lx_min, lx_max, lq_min, lq_max;
  const float* xf;
} or_pdf_grid;
/* x f(x, Q) of flavour fl: bilinear interpolation in (ln x, ln Q) over the
 * grid cell that holds the point; outside the grid the edge cell's
 * bilinear function continues (linear extrapolation).  0 for |fl| > 5. */
double or_pdf_interp(const or_pdf_grid* g, int fl, double x, double Q);
/* The toy densities tabulated at the nodes of g (u, d, ubar = dbar, g;
 * s, c, b and their antiquarks zero) into xf_out [nq][nx][11]. */
void or_pdf_tabulate_toy(const or_pdf_grid* g, float* xf_out);
/* Factorisation scales (the paper does not state them): the pair mass for
 * Drell-Yan, m_t for the top processes. */

/* toy parton densities x*f(x) of the configuration, and the gluon choice */
double or_xf_u(double x);
double or_xf_d(double x);
double or_xf_qbar(double x);
double or_xf_g(double x);

/* Drell-Yan qqbar -> gamma* -> mu mu, integrand over the two true |p|
 * (Eq. mem_def + Eq. 3 with a Gaussian momentum TF). ev = mu-, mu+ as
 * 2 x {E,px,py,pz}.  x in [0,1]^2.  No VEGAS Jacobian. */
double or_dy_integrand(const or_params* p, const double* ev, const double* x);
/* spin- and colour-averaged |M|^2 for q qbar -> mu- mu+ computed from
 * explicit Dirac spinors and gamma matrices (p1 = quark, p2 = antiquark,
 * p3 = mu-, p4 = mu+), charges in units of e. */
double or_qq_mumu_me2(const double* p1, const double* p2, const double* p3,
                      const double* p4, double Qq, double alpha);
/* LO sigma(q qbar -> gamma* -> mu mu) in the window [m_lo, m_hi] by 2D
 * Gauss-Legendre quadrature over (x1, x2); in GeV^-2. */
double or_dy_sigma_2d(const or_params* p, int nodes);
/* the same as a 1D integral over tau of the parton luminosity */
double or_dy_sigma_tau(const or_params* p, int nodes);

/* ttbar dilepton (Eqs. integrand and dilepsolv).  ev = b-jet 0, b-jet 1,
 * l+, l- as 4 x {E,px,py,pz}.  perm 0: jet 0 is the b (from t), perm 1:
 * swapped.  x in [0,1]^8.  Writes the number of accepted neutrino
 * solutions when nsol != 0. */
double or_tt_integrand(const or_params* p, const double* ev, int perm,
                       const double* x, int* nsol);

/* One W chain of the top decays in the ttbar matrix element: the two W
 * vertices squared, (g_W^2 / 2)^2 with g_W^2 = 8 G_F M_W^2 / sqrt 2, times
 * the W Breit-Wigner factor 1 / ((w2 - M_W^2)^2 + M_W^2 Gamma_W^2). */
double or_decay_w_factor(const or_params* p, double w2);

/* Volume of massless n-body phase space (2 <= n <= 6) at sqrt(s), by Monte
 * Carlo over sequential two-body splittings (n_points Philox points);
 * writes the MC error to err. */
double or_ps_volume(int n, double sqrt_s, uint64_t seed, int64_t n_points, double* err);

/* Width Gamma(t -> b l+ nu) of an on-shell top from its three-body decay
 * phase space with the matrix element's W chain (or_decay_w_factor x
 * or_top_decay_spinsum); writes the MC error to err. */
double or_top_width(const or_params* p, uint64_t seed, int64_t n_points, double* err);

/* Partonic cross section of g g (channel 0) or q qbar (channel 1) -> t tbar
 * -> b l+ nu bbar l- nubar at fixed sqrt(shat) from the decayed matrix
 * element over the full six-body phase space (MC, n_points Philox points);
 * writes the MC error to err.  In units of GeV^-2. */
double or_tt_decayed_sigma(const or_params* p, int channel, double sqrt_shat, uint64_t seed, int64_t n_points,
                           double* err);

/* Parton-level weight of a ttbar dilepton event whose six final-state
 * partons are all known (transfer functions are delta functions, Sec. 4's
 * parton-level timing).  ev = b, bbar, l+, l-, nu, nubar as 6 x
 * {E,px,py,pz}.  For each assignment of the two b partons (as given, then
 * swapped): boost to zero transverse momentum, x1, x2 = (E' +- P_z)/sqrt(S),
 * w = (2/S) (E/E') [f_g f_g |M_gg|^2 + f_q f_qbar |M_qq|^2 (both beam
 * orderings)] / (2 shat); 0 when x1 or x2 leaves (0, 1].  Returns the
 * average over the two assignments. */
double or_tt_parton_weight(const or_params* p, const double* ev);

/* ttbar semileptonic (one W -> q qbar').  ev = jets j0..j3, lepton as
 * 5 x {E,px,py,pz}, then a sixth row {charge, 0, 0, 0} with the lepton
 * charge +1 (l+: the top decays leptonically) or -1 (read when lep_charge
 * is 0).  perm in [0,12): the ordered pair (b from the leptonic top, b from the
 * hadronic top) of distinct jets, enumerated b_l-major; the remaining two
 * jets are the W -> q qbar' pair, both orderings summed inside the
 * integrand.  x in [0,1]^7. */
double or_tt_semilep_integrand(const or_params* p, const double* ev, int lep_charge, int perm,
                               const double* x, int* nsol);
void or_semilep_perm(int perm, int* i_bl, int* i_bh, int* i_ja, int* i_jb);
double or_semilep_map(const or_params* p, const double* ev, int perm, const double* x, double* E4);
int or_semilep_nu_z(const double* l, double nx, double ny, double q2, double* nz);
double or_dgauss_tf(double meas, double truth, double core, double tail, double ftail);

/* Building blocks exposed for tests. */
/* all real (nu, nubar) solutions of Eq. dilepsolv; returns the count (<= 4),
 * writes nu[4*i], nub[4*i] and the 4x4 Jacobian determinant of
 * (q2_W+, q2_t, q2_W-, q2_tbar) w.r.t. (nu_x, nu_y, nu_z, nubar_z). */
int or_solve_dilepton(const double* b, const double* bb, const double* lp,
                      const double* lm, double metx, double mety,
                      double q2wp, double q2t, double q2wm, double q2tb,
                      double* nu, double* nub, double* detj);
/* residuals of Eq. dilepsolv at (nu, nubar) */
void or_dilepton_residual(const double* b, const double* bb, const double* lp,
                          const double* lm, const double* nu, const double* nub,
                          double* q2_out /* wp, t, wm, tb */);
/* |M|^2 summed over all spins and colours (no averaging, no couplings), for
 * gg -> t tbar -> b l+ nu bbar l- nubar.  k1, k2 gluons along +z, -z.
 * mom = b, l+, nu, bbar, l-, nubar. Includes the four Breit-Wigner
 * propagators.  Returns the colour/spin sum times g_s^4 g_W^8/16 / (avg). */
double or_tt_me2_gg(const or_params* p, const double* k1, const double* k2, const double* mom);
double or_tt_me2_qq(const or_params* p, const double* kq, const double* kqb, const double* mom);
/* on-shell production only, spin/colour averaged, couplings g_s = 1 */
double or_gg_ttbar_prod(double mt, const double* k1, const double* k2,
                        const double* pt, const double* ptb);
double or_qq_ttbar_prod(double mt, const double* k1, const double* k2,
                        const double* pt, const double* ptb);
/* Ward test: replace gluon 1's polarisation by its momentum; returns the
 * largest |amplitude| over spins and the other gluon's polarisation */
double or_gg_ttbar_ward(double mt, const double* k1, const double* k2,
                        const double* pt, const double* ptb);
/* t -> b l+ nu, summed over all spins, without couplings or W propagator */
double or_top_decay_spinsum(double mt, const double* pt, const double* b,
                            const double* lp, const double* nu);

/* pieces of the tt map exposed for tests */
double or_bw_map(double x, double m, double w, double lo, double hi, double* q2);
double or_gauss_tf(double meas, double truth, double rel_sigma);
/* Genz product-peak test integrand on [0,1]^4 (kind OR_KIND_GENZ):
 * prod_d a / (1 + a^2 (x_d - c_d)^2), a = 20, c_d = 0.3 + 0.1 d */
double or_genz_integrand(const double* x);
double or_genz_exact(void);

/* ---------------------------------------------------- learned proposal -- */
/* Conditional rational-quadratic spline flow on [0,1]^8 (definition in
 * flow.c).  forward: x -> z, returns log q(x|c); inverse: z -> x, returns
 * log q(x|c) at the returned x. */
int or_flow_nparams(void);
double or_flow_forward(const double* params, const double* ctx, const double* x, double* z);
double or_flow_inverse(const double* params, const double* ctx, const double* z, double* x);
void or_flow_context(const double* ev, int perm, double* ctx);
double or_flow_nll_grad(const double* params, int n, const double* x, const double* ctx, const double* wt,
                        double* grad);

/* -------------------------------------------------------------- driver -- */
enum { OR_KIND_DY = 1, OR_KIND_TT = 2, OR_KIND_GENZ = 3, OR_KIND_TT_SL = 4, OR_KIND_TTH = 5,
       OR_KIND_TTH_LL = 6, OR_KIND_TTBB_LL = 7,
       /* the same integrals in direct parametrisations (closure checks) */
       OR_KIND_TT_DIRECT = 8, OR_KIND_TT_SL_DIRECT = 9, OR_KIND_TTH_LL_DIRECT = 10,
       /* 1 + floor(4 x0) + 3 floor(4 x1) on [0,1]^2 (integral 7): constant on
        * a 4 x 4 lattice, a check of stratified sampling */
       OR_KIND_STEP = 11 };
/* Direct parametrisations of the t tbar dilepton, t tbar semileptonic and
 * t tbar H dilepton integrands (integrands.c): the unmeasured momenta
 * themselves as variables, no constraint solve, Breit-Wigner factors left
 * in |M|^2.  Same events, assignments and dimensions as the mapped kinds;
 * their integrals over [0,1]^D are the same numbers. */
double or_tt_direct_integrand(const or_params* p, const double* ev, int perm, const double* x);
enum { OR_SL_DIRECT_EB = 1, OR_SL_DIRECT_NU = 2, OR_SL_DIRECT_EBH = 4 };
double or_tt_semilep_direct_integrand(const or_params* p, const double* ev, int lep_charge, int perm,
                                      const double* x, int mode);
double or_tthll_direct_integrand(const or_params* p, const double* ev, int perm, const double* x);
/* t tbar H (H -> b bbar) and t tbar b bbar, both tops decaying to b l nu
 * (Sec. 4's analysis): events b-jets 0-3, l+, l- as 6 x {E,px,py,pz};
 * assignments and variables in integrands.c (or_f2_perm: the event rows of
 * b, bbar and the pair jets for an assignment). */
void or_f2_perm(int kind, int perm, int* rows);
double or_tthll_integrand(const or_params* p, const double* ev, int perm, const double* x, int* nsol_out);
double or_ttbbll_integrand(const or_params* p, const double* ev, int perm, const double* x, int* nsol_out);
/* parton level (transfer functions delta functions): ev = 8 x {E,px,py,pz},
 * b quarks 0-3, l+, l-, nu, nubar; mean over the jet assignments */
double or_f2_parton_weight(int kind, const or_params* p, const double* ev);
typedef struct {
  double I, sigma;          /* combined estimate over iterations >= 2 */
  double chi2dof;
  int    n_iter_used;
} or_result;
/* Full VEGAS integration of one (event, permutation) integral.  iter_I and
 * iter_var (may be NULL) receive I_j, sigma_j^2 of every iteration.
 * grid_io (may be NULL): if non-NULL it is the starting grid and receives
 * the final grid. */
/* Combined estimate from per-iteration I_j, sigma_j^2 (driver.c): mode 0
 * inverse-variance weights, mode 1 equal weights. */
void or_combine_iterations(const double* Is, const double* Vs, int n_iter, int first_kept, int mode, double* I,
                           double* sigma);
void or_integrate_one(int kind, const or_params* p, const double* ev, int perm,
                      uint64_t seed, uint32_t event_index, int64_t n_points,
                      int n_iter, double alpha, double* grid_io,
                      double* iter_I, double* iter_var, or_result* res);
/* one VEGAS iteration with a given grid; returns sum w, sum w^2 and the
 * per-(dim,bin) sums of w^2 (D x 64) */
void or_vegas_iteration(int kind, const or_params* p, const double* ev, int perm,
                        uint64_t seed, uint32_t event_index, uint32_t iter,
                        int64_t n_points, const double* grid,
                        double* s1, double* s2, double* bins);
/* integrand value at u (maps through the grid, multiplies the Jacobian) */
double or_weight_at(int kind, const or_params* p, const double* ev, int perm,
                    const double* grid, const double* u);
/* P and its error per event (Eq. mem_def with the permutation average),
 * events laid out [n_events][n_obj][4]; OpenMP over integrals. */
void or_integrate_events(int kind, const or_params* p, const double* events,
                         int n_events, int n_obj, uint64_t seed, int64_t n_points,
                         int n_iter, double alpha, double sigma_norm,
                         double* P, double* err, int32_t* status);
void or_integrate_events_iters(int kind, const or_params* p, const double* events,
                               int n_events, int n_obj, uint64_t seed, int64_t n_points,
                               int n_iter, const int32_t* n_iter_ev, double alpha, double sigma_norm,
                               double* P, double* err, int32_t* status);
/* Adaptive stratified VEGAS (driver.c): hypercubes per dimension for D
 * dimensions and N points, the allocation of N points over H hypercubes
 * (first iteration, or from the per-hypercube standard deviations sig),
 * one iteration (estimate, variance, per-hypercube deviations, per-bin
 * sums, optionally every point's weight in iteration order), and a whole
 * integration. */
#define OR_STRAT_HMAX 16384
int or_strat_ns(int D, int64_t N);
void or_strat_allocate(int64_t H, int64_t N, const double* sig, int first, int64_t* nh);
void or_strat_iteration(int kind, const or_params* p, const double* ev, int perm, uint64_t seed,
                        uint32_t event_index, uint32_t iter, int64_t N, const double* grid, int ns,
                        const int64_t* nh, double* I_out, double* var_out, double* sig_out, double* bins,
                        double* w_out);
void or_integrate_one_strat(int kind, const or_params* p, const double* ev, int perm, uint64_t seed,
                            uint32_t event_index, int64_t N, int n_iter, double alpha, double* iter_I,
                            double* iter_var, or_result* res);
void or_set_threads(int n);
int or_max_threads(void);
int or_dims(int kind);
int or_nperm(int kind);

#ifdef __cplusplus
}
#endif
/* ----------------------------------------------------------- ttbar H -- */
/* g g -> t tbar H (Higgs at every position of the top line of the three
 * gg -> t tbar diagrams; unit Yukawa): spin/colour-summed |M|^2 of on-shell
 * tops averaged over initial states; the Ward-identity residual (e1 -> k1,
 * relative); the soft-Higgs check against d/dm of the t tbar amplitude
 * (relative deviation); the decayed |M|^2 with couplings and Breit-Wigner
 * factors (see dirac.c). */
double or_gg_tth_prod(double mt, const double* k1, const double* k2, const double* pt, const double* ptb,
                      const double* ph);
double or_gg_tth_ward(double mt, const double* k1, const double* k2, const double* pt, const double* ptb,
                      const double* ph);
double or_tth_soft_check(double mt, const double* mom, double delta);
/* g g -> t tbar b bbar (the t tbar H analysis' background, Sec. 4): 36
 * tree-level QCD diagrams with explicit SU(3) colour sums.  _prod: on-shell
 * tops of mass mt, massless b, spin and colour summed and averaged, no
 * couplings; _ward: the Ward identity for gluon g (0/1), |M|^2 with that
 * gluon's polarisation replaced by its momentum relative to the physical
 * one; _me2_gg: decayed tops (mom as or_tt_me2_gg), couplings, top and W
 * Breit-Wigner factors included.  or_colour_matrix_ttbb: the colour matrix
 * of the 38 colour terms; or_colour_fabc: f^abc from the generators. */
double or_gg_ttbb_prod(double mt, const double* k1, const double* k2, const double* p3, const double* p4,
                       const double* p5, const double* p6);
double or_gg_ttbb_prod_explicit(double mt, const double* k1, const double* k2, const double* p3,
                                const double* p4, const double* p5, const double* p6);
double or_gg_ttbb_ward(double mt, const double* k1, const double* k2, const double* p3, const double* p4,
                       const double* p5, const double* p6, int g);
double or_ttbb_me2_gg(const or_params* p, const double* k1, const double* k2, const double* mom, const double* p5,
                      const double* p6);
double or_colour_matrix_ttbb(int d, int e);
double or_colour_fabc(int a, int b, int c);
double or_tth_me2_gg(const or_params* p, const double* k1, const double* k2, const double* mom, const double* hb,
                     const double* hbb);

/* c3 event rows b0..b3, l0, l1, lepton, (charge,0,0,0); 24 assignments */
void or_tth_perm(int perm, int* i_h1, int* i_h2, int* i_bl, int* i_bh, int* o);
double or_tth_map(const or_params* p, const double* ev, int perm, const double* x, double* E6);
double or_tth_integrand(const or_params* p, const double* ev, int lep_charge, int perm, const double* x,
                        int* nsol_out);

#endif
