/*
 * Oracle: explicit Dirac algebra and the tree-level squared matrix elements.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The |M|^2 of Eq. mem_def is evaluated here the plain way: 4x4 gamma
 * matrices in the Dirac representation, Dirac-basis spinors whose outer
 * products sum to (pslash +- m), explicit sums over every external spin,
 * linear gluon polarisations and explicit colour factors.  The ME code of
 * the paper came from a generator (Sec. 4); nothing of it is reproduced.
 */
#include "oracle.h"
#include <complex.h>
#include <math.h>
#include <string.h>

typedef double complex cx;
typedef struct { cx m[16]; } mat4;   /* row-major */
typedef struct { cx s[4]; } spin4;

static mat4 G[4];   /* gamma^mu, upper index */
static mat4 G5;
static mat4 ID4;
static int g_ready = 0;

static void init_gamma(void)
{
  if (g_ready) return;
  memset(G, 0, sizeof(G));
  memset(&G5, 0, sizeof(G5));
  memset(&ID4, 0, sizeof(ID4));
  for (int i = 0; i < 4; ++i) ID4.m[i * 5] = 1.0;
  /* gamma^0 = diag(1,1,-1,-1) */
  G[0].m[0] = 1; G[0].m[5] = 1; G[0].m[10] = -1; G[0].m[15] = -1;
  /* gamma^i = [[0, sigma_i], [-sigma_i, 0]] */
  const cx sig[3][4] = {{0, 1, 1, 0}, {0, -I, I, 0}, {1, 0, 0, -1}};
  for (int k = 0; k < 3; ++k)
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        G[k + 1].m[r * 4 + (c + 2)] = sig[k][r * 2 + c];
        G[k + 1].m[(r + 2) * 4 + c] = -sig[k][r * 2 + c];
      }
  /* gamma^5 = [[0, 1], [1, 0]] */
  G5.m[2] = 1; G5.m[7] = 1; G5.m[8] = 1; G5.m[13] = 1;
  g_ready = 1;
}

static mat4 mmul(mat4 a, mat4 b)
{
  mat4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cx s = 0;
      for (int k = 0; k < 4; ++k) s += a.m[i * 4 + k] * b.m[k * 4 + j];
      r.m[i * 4 + j] = s;
    }
  return r;
}
static mat4 madd(mat4 a, mat4 b, cx fb)
{
  mat4 r;
  for (int i = 0; i < 16; ++i) r.m[i] = a.m[i] + fb * b.m[i];
  return r;
}
static mat4 mscale(mat4 a, cx f)
{
  mat4 r;
  for (int i = 0; i < 16; ++i) r.m[i] = f * a.m[i];
  return r;
}
static spin4 mvec(mat4 a, spin4 v)
{
  spin4 r;
  for (int i = 0; i < 4; ++i) {
    cx s = 0;
    for (int k = 0; k < 4; ++k) s += a.m[i * 4 + k] * v.s[k];
    r.s[i] = s;
  }
  return r;
}
static spin4 rowmat(spin4 row, mat4 a)
{
  spin4 r;
  for (int j = 0; j < 4; ++j) {
    cx s = 0;
    for (int k = 0; k < 4; ++k) s += row.s[k] * a.m[k * 4 + j];
    r.s[j] = s;
  }
  return r;
}
static cx rowcol(spin4 row, spin4 col)
{
  cx s = 0;
  for (int k = 0; k < 4; ++k) s += row.s[k] * col.s[k];
  return s;
}
/* a-slash = gamma^mu a_mu = g0 a^0 - g1 a^1 - g2 a^2 - g3 a^3 (a given
 * with upper indices, possibly complex) */
static mat4 slash(const cx* a)
{
  mat4 r = mscale(G[0], a[0]);
  for (int k = 1; k < 4; ++k) r = madd(r, G[k], -a[k]);
  return r;
}
static mat4 slash_r(const double* p)
{
  cx a[4] = {p[0], p[1], p[2], p[3]};
  return slash(a);
}
static mat4 proj_left(void) { return mscale(madd(ID4, G5, -1.0), 0.5); }
static double mdot(const double* a, const double* b)
{
  return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}
/* Dirac-basis spinors: u = [sqrt(E+m) xi ; (sigma.p) xi / sqrt(E+m)],
 * v = [(sigma.p) eta / sqrt(E+m) ; sqrt(E+m) eta], xi, eta in {(1,0),(0,1)}.
 * Their outer products sum to pslash + m and pslash - m. */
static void sigma_dot_p(const double* p, int s, cx out[2])
{
  /* (sigma.p) applied to the basis vector s */
  cx col0[2] = {p[3], p[1] + I * p[2]};
  cx col1[2] = {p[1] - I * p[2], -p[3]};
  out[0] = s ? col1[0] : col0[0];
  out[1] = s ? col1[1] : col0[1];
}
static spin4 spinor_u(const double* p, double m, int s)
{
  double n = sqrt(p[0] + m);
  cx sp[2];
  sigma_dot_p(p, s, sp);
  spin4 r;
  r.s[0] = s ? 0 : n; r.s[1] = s ? n : 0;
  r.s[2] = sp[0] / n; r.s[3] = sp[1] / n;
  return r;
}
static spin4 spinor_v(const double* p, double m, int s)
{
  double n = sqrt(p[0] + m);
  cx sp[2];
  sigma_dot_p(p, s, sp);
  spin4 r;
  r.s[0] = sp[0] / n; r.s[1] = sp[1] / n;
  r.s[2] = s ? 0 : n; r.s[3] = s ? n : 0;
  return r;
}
/* psi-bar = psi^dagger gamma^0 as a row */
static spin4 dbar(spin4 v)
{
  spin4 r;
  for (int i = 0; i < 4; ++i) r.s[i] = conj(v.s[i]) * G[0].m[i * 5];
  return r;
}
/* current bar(a) gamma^mu P_L b, upper index */
static void current_L(spin4 abar, spin4 b, cx* J)
{
  mat4 PL = proj_left();
  for (int mu = 0; mu < 4; ++mu) J[mu] = rowcol(abar, mvec(mmul(G[mu], PL), b));
}
static void current_V(spin4 abar, spin4 b, cx* J)
{
  for (int mu = 0; mu < 4; ++mu) J[mu] = rowcol(abar, mvec(G[mu], b));
}

/* ---------------------------------------------------------------- DY ---- */
double or_qq_mumu_me2(const double* p1, const double* p2, const double* p3,
                      const double* p4, double Qq, double alpha)
{
  init_gamma();
  /* M = e^2 Qq [vbar(p2) g^mu u(p1)] [ubar(p3) g_mu v(p4)] / s,
   * lepton charge -1 (the overall sign drops out of |M|^2). */
  double P[4] = {p1[0] + p2[0], p1[1] + p2[1], p1[2] + p2[2], p1[3] + p2[3]};
  double s = mdot(P, P);
  double e2 = 4.0 * M_PI * alpha;
  double sum = 0.0;
  for (int s1 = 0; s1 < 2; ++s1)
    for (int s2 = 0; s2 < 2; ++s2) {
      cx Jq[4];
      current_V(dbar(spinor_v(p2, 0.0, s2)), spinor_u(p1, 0.0, s1), Jq);
      for (int s3 = 0; s3 < 2; ++s3)
        for (int s4 = 0; s4 < 2; ++s4) {
          cx Jl[4];
          current_V(dbar(spinor_u(p3, 0.0, s3)), spinor_v(p4, 0.0, s4), Jl);
          cx a = Jq[0] * Jl[0] - Jq[1] * Jl[1] - Jq[2] * Jl[2] - Jq[3] * Jl[3];
          a *= e2 * Qq / s;
          sum += creal(a * conj(a));
        }
    }
  /* colour: sum over i,j of |delta_ij|^2 = 3, averaged over 9; spins / 4 */
  return sum * 3.0 / 9.0 / 4.0;
}

/* -------------------------------------------------------------- ttbar --- */
/* Production kernels with generic top "wave functions": row R (replaces
 * ubar(t)) and column C (replaces v(tbar)).  p_t, p_tb are the (possibly
 * off-shell) top momenta entering the internal propagators. */
typedef struct {
  mat4 g12[2][2], g21[2][2];   /* gluon polarisation pairs (lin. x / y) */
} gg_vertices;

static void lin_pol(int which, double eps[4])
{
  eps[0] = 0; eps[1] = which == 0 ? 1 : 0; eps[2] = which == 1 ? 1 : 0; eps[3] = 0;
}

/* Gluon-gluon fusion into a top pair: three diagrams (t-, u-channel top
 * exchange and the s-channel triple-gluon vertex), decomposed in the two
 * colour orderings T^a T^b and T^b T^a.  The s-channel part enters the two
 * orderings with opposite signs (f^abc T^c = -i [T^a, T^b]). */
static void build_gg(double mt, const double* k1, const double* k2, const double* pt,
                     const double* eps1_in, const double* eps2_in, int use_given,
                     gg_vertices* out)
{
  double q1[4], q2[4], K[4], s;
  for (int i = 0; i < 4; ++i) { q1[i] = pt[i] - k1[i]; q2[i] = pt[i] - k2[i]; K[i] = k1[i] + k2[i]; }
  s = mdot(K, K);
  double Dt = mdot(q1, q1) - mt * mt;
  double Du = mdot(q2, q2) - mt * mt;
  mat4 prop1 = madd(slash_r(q1), ID4, mt);
  mat4 prop2 = madd(slash_r(q2), ID4, mt);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      double e1[4], e2[4];
      if (use_given) { memcpy(e1, eps1_in, sizeof(e1)); memcpy(e2, eps2_in, sizeof(e2)); if (b) lin_pol(1, e2); else lin_pol(0, e2); }
      else { lin_pol(a, e1); lin_pol(b, e2); }
      mat4 s1 = slash_r(e1), s2 = slash_r(e2);
      double V[4];
      double e1e2 = mdot(e1, e2), k2e1 = mdot(k2, e1), k1e2 = mdot(k1, e2);
      for (int i = 0; i < 4; ++i)
        V[i] = e1e2 * (k1[i] - k2[i]) + 2.0 * k2e1 * e2[i] - 2.0 * k1e2 * e1[i];
      mat4 sV = mscale(slash_r(V), 1.0 / s);
      mat4 t12 = mscale(mmul(mmul(s1, prop1), s2), 1.0 / Dt);
      mat4 t21 = mscale(mmul(mmul(s2, prop2), s1), 1.0 / Du);
      out->g12[a][b] = madd(t12, sV, 1.0);
      out->g21[a][b] = madd(t21, sV, -1.0);
    }
}

/* colour-summed |.|^2 of T^aT^b A12 + T^bT^a A21 */
static double colour_gg(cx a12, cx a21)
{
  return 16.0 / 3.0 * (creal(a12 * conj(a12)) + creal(a21 * conj(a21)))
       + 2.0 * (-2.0 / 3.0) * creal(a12 * conj(a21));
}

double or_gg_ttbar_prod(double mt, const double* k1, const double* k2,
                        const double* pt, const double* ptb)
{
  init_gamma();
  gg_vertices gv;
  build_gg(mt, k1, k2, pt, NULL, NULL, 0, &gv);
  double sum = 0.0;
  for (int st = 0; st < 2; ++st)
    for (int sb = 0; sb < 2; ++sb) {
      spin4 R = dbar(spinor_u(pt, mt, st));
      spin4 C = spinor_v(ptb, mt, sb);
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          sum += colour_gg(rowcol(R, mvec(gv.g12[a][b], C)), rowcol(R, mvec(gv.g21[a][b], C)));
    }
  return sum / 256.0;  /* 4 polarisations x 64 colours */
}

double or_gg_ttbar_ward(double mt, const double* k1, const double* k2,
                        const double* pt, const double* ptb)
{
  init_gamma();
  gg_vertices gv;
  double e1[4] = {k1[0], k1[1], k1[2], k1[3]};
  build_gg(mt, k1, k2, pt, e1, e1, 1, &gv);
  double worst = 0.0;
  for (int st = 0; st < 2; ++st)
    for (int sb = 0; sb < 2; ++sb) {
      spin4 R = dbar(spinor_u(pt, mt, st));
      spin4 C = spinor_v(ptb, mt, sb);
      for (int b = 0; b < 2; ++b) {
        /* the full colour-dressed amplitude vanishes iff A12 + A21 = 0 and
         * the commutator part does; with eps1 -> k1 each ordering must be
         * separately zero */
        cx a12 = rowcol(R, mvec(gv.g12[0][b], C));
        cx a21 = rowcol(R, mvec(gv.g21[0][b], C));
        double m = fmax(cabs(a12), cabs(a21));
        if (m > worst) worst = m;
      }
    }
  return worst;
}

double or_qq_ttbar_prod(double mt, const double* k1, const double* k2,
                        const double* pt, const double* ptb)
{
  init_gamma();
  double K[4];
  for (int i = 0; i < 4; ++i) K[i] = k1[i] + k2[i];
  double s = mdot(K, K);
  double sum = 0.0;
  for (int s1 = 0; s1 < 2; ++s1)
    for (int s2 = 0; s2 < 2; ++s2) {
      cx Jq[4];
      current_V(dbar(spinor_v(k2, 0.0, s2)), spinor_u(k1, 0.0, s1), Jq);
      for (int st = 0; st < 2; ++st)
        for (int sb = 0; sb < 2; ++sb) {
          cx Jt[4];
          current_V(dbar(spinor_u(pt, mt, st)), spinor_v(ptb, mt, sb), Jt);
          cx a = (Jq[0] * Jt[0] - Jq[1] * Jt[1] - Jq[2] * Jt[2] - Jq[3] * Jt[3]) / s;
          sum += 2.0 * creal(a * conj(a));  /* colour: Tr(T^aT^b)Tr(T^aT^b) = 2 */
        }
    }
  return sum / 36.0;  /* 4 spins x 9 colours */
}

double or_top_decay_spinsum(double mt, const double* pt, const double* b,
                            const double* lp, const double* nu)
{
  init_gamma();
  mat4 PL = proj_left();
  double sum = 0.0;
  for (int sn = 0; sn < 2; ++sn)
    for (int sl = 0; sl < 2; ++sl) {
      cx J[4];
      current_L(dbar(spinor_u(nu, 0.0, sn)), spinor_v(lp, 0.0, sl), J);
      mat4 Js = slash(J);
      for (int sbq = 0; sbq < 2; ++sbq)
        for (int st = 0; st < 2; ++st) {
          spin4 row = rowmat(dbar(spinor_u(b, 0.0, sbq)), mmul(Js, PL));
          cx a = rowcol(row, spinor_u(pt, mt, st));
          sum += creal(a * conj(a));
        }
    }
  return sum;
}

/* Decayed top rows R = ubar(b) Jslash+ P_L (pslash_t + m) and decayed
 * antitop columns C = (-pslash_tbar + m) Jslash- P_L v(bbar), one per
 * combination of the three decay-product spins. */
static void decay_wavefunctions(double mt, const double* mom, spin4 R[8], spin4 C[8],
                                double* pt_out, double* ptb_out)
{
  const double *b = mom, *lp = mom + 4, *nu = mom + 8;
  const double *bb = mom + 12, *lm = mom + 16, *nub = mom + 20;
  double pt[4], ptb[4];
  for (int i = 0; i < 4; ++i) { pt[i] = b[i] + lp[i] + nu[i]; ptb[i] = bb[i] + lm[i] + nub[i]; }
  mat4 PL = proj_left();
  mat4 topnum = madd(slash_r(pt), ID4, mt);
  mat4 atopnum = madd(mscale(slash_r(ptb), -1.0), ID4, mt);
  int n = 0;
  for (int sb = 0; sb < 2; ++sb)
    for (int sn = 0; sn < 2; ++sn)
      for (int sl = 0; sl < 2; ++sl) {
        cx J[4];
        current_L(dbar(spinor_u(nu, 0.0, sn)), spinor_v(lp, 0.0, sl), J);
        R[n] = rowmat(rowmat(dbar(spinor_u(b, 0.0, sb)), mmul(slash(J), PL)), topnum);
        cx Jm[4];
        current_L(dbar(spinor_u(lm, 0.0, sl)), spinor_v(nub, 0.0, sn), Jm);
        C[n] = mvec(atopnum, mvec(mmul(slash(Jm), PL), spinor_v(bb, 0.0, sb)));
        ++n;
      }
  memcpy(pt_out, pt, sizeof(pt));
  memcpy(ptb_out, ptb, sizeof(ptb));
}

static double bw2(double q2, double m, double w)
{
  double d = q2 - m * m;
  return 1.0 / (d * d + m * m * w * w);
}

/* One W chain of a top decay: the two W vertices (g_W / sqrt 2)^2 each,
 * squared, with g_W^2 = 8 G_F M_W^2 / sqrt 2, times the W Breit-Wigner
 * factor at virtuality w2. */
double or_decay_w_factor(const or_params* p, double w2)
{
  double gw2 = 8.0 * p->g_fermi * p->m_w * p->m_w / sqrt(2.0);
  return (gw2 / 2.0) * (gw2 / 2.0) * bw2(w2, p->m_w, p->w_w);
}

static double decay_couplings(const or_params* p, const double* mom, const double* pt, const double* ptb)
{
  const double *b = mom, *lp = mom + 4, *nu = mom + 8;
  const double *bb = mom + 12, *lm = mom + 16, *nub = mom + 20;
  (void)b; (void)bb;
  double wp[4], wm[4];
  for (int i = 0; i < 4; ++i) { wp[i] = lp[i] + nu[i]; wm[i] = lm[i] + nub[i]; }
  double gs2 = 4.0 * M_PI * p->alpha_s;
  return gs2 * gs2 * or_decay_w_factor(p, mdot(wp, wp)) * or_decay_w_factor(p, mdot(wm, wm))
         * bw2(mdot(pt, pt), p->m_t, p->w_t) * bw2(mdot(ptb, ptb), p->m_t, p->w_t);
}

double or_tt_me2_gg(const or_params* p, const double* k1, const double* k2, const double* mom)
{
  init_gamma();
  spin4 R[8], C[8];
  double pt[4], ptb[4];
  decay_wavefunctions(p->m_t, mom, R, C, pt, ptb);
  gg_vertices gv;
  build_gg(p->m_t, k1, k2, pt, NULL, NULL, 0, &gv);
  double sum = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int j = 0; j < 8; ++j) {
        spin4 c12 = mvec(gv.g12[a][b], C[j]);
        spin4 c21 = mvec(gv.g21[a][b], C[j]);
        for (int i = 0; i < 8; ++i)
          sum += colour_gg(rowcol(R[i], c12), rowcol(R[i], c21));
      }
  return sum * decay_couplings(p, mom, pt, ptb) / 256.0;
}

double or_tt_me2_qq(const or_params* p, const double* kq, const double* kqb, const double* mom)
{
  init_gamma();
  spin4 R[8], C[8];
  double pt[4], ptb[4];
  decay_wavefunctions(p->m_t, mom, R, C, pt, ptb);
  double K[4];
  for (int i = 0; i < 4; ++i) K[i] = kq[i] + kqb[i];
  double s = mdot(K, K);
  double sum = 0.0;
  for (int s1 = 0; s1 < 2; ++s1)
    for (int s2 = 0; s2 < 2; ++s2) {
      cx Jq[4];
      current_V(dbar(spinor_v(kqb, 0.0, s2)), spinor_u(kq, 0.0, s1), Jq);
      mat4 Jslash = slash(Jq);
      for (int j = 0; j < 8; ++j) {
        spin4 cj = mvec(Jslash, C[j]);
        for (int i = 0; i < 8; ++i) {
          cx a = rowcol(R[i], cj) / s;
          sum += 2.0 * creal(a * conj(a));
        }
      }
    }
  return sum * decay_couplings(p, mom, pt, ptb) / 36.0;
}

/* ---------------------------------------------------------- ttbar H --- */
/* g(k1) g(k2) -> t tbar H: the Higgs (unit Yukawa vertex, the coupling
 * m_t/v is applied by the caller) is inserted at every position of the top
 * line of each gg -> t tbar diagram.  Between the top row R and the
 * antitop column C, for the colour ordering T^a T^b (gluon 1 next to the
 * top):
 *   H S(pt+pH) e1 S(pt+pH-k1) e2  +  e1 S(pt-k1) H S(pt-k1+pH) e2
 *   + e1 S(pt-k1) e2 S(-ptb-pH) H
 * and the s-channel current V (as in gg -> t tbar) with the Higgs on either
 * side of it, entering the two orderings with opposite signs;
 * S(q) = (qslash + m)/(q^2 - m^2). */
static mat4 prop_m(const double* q, double mt)
{
  return mscale(madd(slash_r(q), ID4, mt), 1.0 / (mdot(q, q) - mt * mt));
}

static void build_ggh(double mt, const double* k1, const double* k2, const double* pt, const double* ptb,
                      const double* ph, const double* e1, const double* e2, mat4* m12, mat4* m21)
{
  double qa[4], qb1[4], qb2[4], qc[4], ra1[4], rb1[4], rb2[4], K[4];
  for (int i = 0; i < 4; ++i) {
    qa[i] = pt[i] + ph[i];                  /* after H next to the top */
    qc[i] = -ptb[i] - ph[i];                /* before H next to the antitop */
    qb1[i] = pt[i] - k1[i];                 /* ordering 12 */
    qb2[i] = pt[i] + ph[i] - k1[i];
    rb1[i] = pt[i] - k2[i];                 /* ordering 21 */
    rb2[i] = pt[i] + ph[i] - k2[i];
    ra1[i] = pt[i] - k1[i] + ph[i];
    K[i] = k1[i] + k2[i];
  }
  double rb2b[4];
  for (int i = 0; i < 4; ++i) rb2b[i] = pt[i] - k2[i] + ph[i];
  mat4 s1 = slash_r(e1), s2 = slash_r(e2);
  mat4 Sa = prop_m(qa, mt), Sc = prop_m(qc, mt);
  /* ordering 12 */
  mat4 t12 = mmul(mmul(mmul(Sa, s1), prop_m(qb2, mt)), s2);
  t12 = madd(t12, mmul(mmul(mmul(s1, prop_m(qb1, mt)), prop_m(ra1, mt)), s2), 1.0);
  t12 = madd(t12, mmul(mmul(mmul(s1, prop_m(qb1, mt)), s2), Sc), 1.0);
  /* ordering 21 */
  mat4 t21 = mmul(mmul(mmul(Sa, s2), prop_m(rb2, mt)), s1);
  t21 = madd(t21, mmul(mmul(mmul(s2, prop_m(rb1, mt)), prop_m(rb2b, mt)), s1), 1.0);
  t21 = madd(t21, mmul(mmul(mmul(s2, prop_m(rb1, mt)), s1), Sc), 1.0);
  /* s-channel */
  double s = mdot(K, K);
  double V[4];
  double e1e2 = mdot(e1, e2), k2e1 = mdot(k2, e1), k1e2 = mdot(k1, e2);
  for (int i = 0; i < 4; ++i) V[i] = e1e2 * (k1[i] - k2[i]) + 2.0 * k2e1 * e2[i] - 2.0 * k1e2 * e1[i];
  mat4 sV = mscale(slash_r(V), 1.0 / s);
  mat4 sch = madd(mmul(Sa, sV), mmul(sV, Sc), 1.0);
  *m12 = madd(t12, sch, 1.0);
  *m21 = madd(t21, sch, -1.0);
}

/* spin- and colour-summed |M|^2 of g g -> t tbar H for on-shell tops, with
 * unit Yukawa coupling, averaged over the 256 initial colours and
 * polarisations */
double or_gg_tth_prod(double mt, const double* k1, const double* k2, const double* pt, const double* ptb,
                      const double* ph)
{
  init_gamma();
  double sum = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      double e1[4], e2[4];
      lin_pol(a, e1);
      lin_pol(b, e2);
      mat4 m12, m21;
      build_ggh(mt, k1, k2, pt, ptb, ph, e1, e2, &m12, &m21);
      for (int st = 0; st < 2; ++st)
        for (int sb = 0; sb < 2; ++sb) {
          spin4 R = dbar(spinor_u(pt, mt, st));
          spin4 C = spinor_v(ptb, mt, sb);
          sum += colour_gg(rowcol(R, mvec(m12, C)), rowcol(R, mvec(m21, C)));
        }
    }
  return sum / 256.0;
}

/* Ward identity: with e1 -> k1 every colour-ordered amplitude vanishes.
 * Returns the largest |A| relative to the largest amplitude with physical
 * polarisations. */
double or_gg_tth_ward(double mt, const double* k1, const double* k2, const double* pt, const double* ptb,
                      const double* ph)
{
  init_gamma();
  double worst = 0.0, scale = 0.0;
  for (int b = 0; b < 2; ++b) {
    double e2[4], ex[4];
    lin_pol(b, e2);
    lin_pol(0, ex);
    mat4 g12, g21, p12, p21;
    build_ggh(mt, k1, k2, pt, ptb, ph, k1, e2, &g12, &g21);
    build_ggh(mt, k1, k2, pt, ptb, ph, ex, e2, &p12, &p21);
    for (int st = 0; st < 2; ++st)
      for (int sb = 0; sb < 2; ++sb) {
        spin4 R = dbar(spinor_u(pt, mt, st));
        spin4 C = spinor_v(ptb, mt, sb);
        worst = fmax(worst, fmax(cabs(rowcol(R, mvec(g12, C))), cabs(rowcol(R, mvec(g21, C)))));
        scale = fmax(scale, fmax(cabs(rowcol(R, mvec(p12, C))), cabs(rowcol(R, mvec(p21, C)))));
      }
  }
  return scale > 0.0 ? worst / scale : worst;
}

/* Decayed top line with zero-width propagators, for the soft-Higgs check:
 * ubar(b) J+slash P_L S(pt) [production] S(-ptb) J-slash P_L v(bbar). */
static void ord_amps_tt(double mt, const double* k1, const double* k2, const double* mom, int i_sp, int a, int b,
                        cx* a12, cx* a21)
{
  const double *bq = mom, *lp = mom + 4, *nu = mom + 8;
  const double *bb = mom + 12, *lm = mom + 16, *nub = mom + 20;
  double pt[4], ptb[4], mptb[4];
  for (int i = 0; i < 4; ++i) { pt[i] = bq[i] + lp[i] + nu[i]; ptb[i] = bb[i] + lm[i] + nub[i]; mptb[i] = -ptb[i]; }
  mat4 PL = proj_left();
  int sb = (i_sp >> 2) & 1, sn = (i_sp >> 1) & 1, sl = i_sp & 1;
  cx J[4], Jm[4];
  current_L(dbar(spinor_u(nu, 0.0, sn)), spinor_v(lp, 0.0, sl), J);
  current_L(dbar(spinor_u(lm, 0.0, sl)), spinor_v(nub, 0.0, sn), Jm);
  spin4 R = rowmat(rowmat(dbar(spinor_u(bq, 0.0, sb)), mmul(slash(J), PL)), prop_m(pt, mt));
  spin4 C = mvec(prop_m(mptb, mt), mvec(mmul(slash(Jm), PL), spinor_v(bb, 0.0, sb)));
  gg_vertices gv;
  build_gg(mt, k1, k2, pt, NULL, NULL, 0, &gv);
  *a12 = rowcol(R, mvec(gv.g12[a][b], C));
  *a21 = rowcol(R, mvec(gv.g21[a][b], C));
}

static void ord_amps_tth(double mt, const double* k1, const double* k2, const double* mom, const double* ph,
                         int i_sp, int a, int b, cx* a12, cx* a21)
{
  const double *bq = mom, *lp = mom + 4, *nu = mom + 8;
  const double *bb = mom + 12, *lm = mom + 16, *nub = mom + 20;
  double pt[4], ptb[4], mptb[4];
  for (int i = 0; i < 4; ++i) { pt[i] = bq[i] + lp[i] + nu[i]; ptb[i] = bb[i] + lm[i] + nub[i]; mptb[i] = -ptb[i]; }
  mat4 PL = proj_left();
  int sb = (i_sp >> 2) & 1, sn = (i_sp >> 1) & 1, sl = i_sp & 1;
  cx J[4], Jm[4];
  current_L(dbar(spinor_u(nu, 0.0, sn)), spinor_v(lp, 0.0, sl), J);
  current_L(dbar(spinor_u(lm, 0.0, sl)), spinor_v(nub, 0.0, sn), Jm);
  spin4 R = rowmat(rowmat(dbar(spinor_u(bq, 0.0, sb)), mmul(slash(J), PL)), prop_m(pt, mt));
  spin4 C = mvec(prop_m(mptb, mt), mvec(mmul(slash(Jm), PL), spinor_v(bb, 0.0, sb)));
  double e1[4], e2[4];
  lin_pol(a, e1);
  lin_pol(b, e2);
  mat4 m12, m21;
  build_ggh(mt, k1, k2, pt, ptb, ph, e1, e2, &m12, &m21);
  *a12 = rowcol(R, mvec(m12, C));
  *a21 = rowcol(R, mvec(m21, C));
}

/* Soft-Higgs theorem: a zero-momentum scalar with unit coupling inserted
 * into a fermion line turns each propagator S into S S = dS/dm, so the
 * t tbar H amplitude at pH -> 0 equals d/dm of the t tbar amplitude (top
 * mass in every propagator, the two decay propagators included, momenta
 * fixed).  mom: the six decay momenta (massless); the gluons are placed
 * along +-z to balance the t tbar system plus pH = delta (1, 0, 0, 1).
 * Returns the largest relative deviation over spins, polarisations and the
 * two colour orderings. */
double or_tth_soft_check(double mt, const double* mom, double delta)
{
  init_gamma();
  double P[4] = {0, 0, 0, 0};
  for (int k = 0; k < 6; ++k)
    for (int i = 0; i < 4; ++i) P[i] += mom[4 * k + i];
  double ph[4] = {delta, 0.0, 0.0, delta};
  /* gluons with zero p_T balancing P (+ ph); P must have P_T = 0 */
  double E = P[0], Z = P[3];
  double k1t[4] = {0.5 * (E + Z), 0, 0, 0.5 * (E + Z)}, k2t[4] = {0.5 * (E - Z), 0, 0, -0.5 * (E - Z)};
  double Eh = E + ph[0], Zh = Z + ph[3];
  double k1h[4] = {0.5 * (Eh + Zh), 0, 0, 0.5 * (Eh + Zh)}, k2h[4] = {0.5 * (Eh - Zh), 0, 0, -0.5 * (Eh - Zh)};
  double worst = 0.0;
  const double h = 1e-4 * mt;
  for (int isp = 0; isp < 8; ++isp)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        cx p12, p21, m12, m21, h12, h21;
        ord_amps_tt(mt + h, k1t, k2t, mom, isp, a, b, &p12, &p21);
        ord_amps_tt(mt - h, k1t, k2t, mom, isp, a, b, &m12, &m21);
        ord_amps_tth(mt, k1h, k2h, mom, ph, isp, a, b, &h12, &h21);
        cx d12 = (p12 - m12) / (2.0 * h), d21 = (p21 - m21) / (2.0 * h);
        double sc = fmax(cabs(d12), cabs(d21));
        if (sc == 0.0) continue;
        worst = fmax(worst, fmax(cabs(h12 - d12), cabs(h21 - d21)) / sc);
      }
  return worst;
}

/* g g -> t tbar H with decayed tops (massless decay products, V-A W
 * couplings), H -> b bbar: the spin- and colour-summed |M|^2 averaged over
 * initial states, times the top and W Breit-Wigner factors and couplings
 * (as or_tt_me2_gg), the Yukawa coupling (m_t/v)^2, the H -> b bbar decay
 * (m_b/v)^2 3 Tr(pb pbbar) = 6 (m_b/v)^2 (pb+pbbar)^2, and the Higgs
 * Breit-Wigner factor.  mom: 6 decay momenta as or_tt_me2_gg; hb, hbb: the
 * Higgs decay b quarks. */
double or_tth_me2_gg(const or_params* p, const double* k1, const double* k2, const double* mom, const double* hb,
                     const double* hbb)
{
  init_gamma();
  spin4 R[8], C[8];
  double pt[4], ptb[4], ph[4];
  decay_wavefunctions(p->m_t, mom, R, C, pt, ptb);
  for (int i = 0; i < 4; ++i) ph[i] = hb[i] + hbb[i];
  double sum = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      double e1[4], e2[4];
      lin_pol(a, e1);
      lin_pol(b, e2);
      mat4 m12, m21;
      build_ggh(p->m_t, k1, k2, pt, ptb, ph, e1, e2, &m12, &m21);
      for (int j = 0; j < 8; ++j) {
        spin4 c12 = mvec(m12, C[j]);
        spin4 c21 = mvec(m21, C[j]);
        for (int i = 0; i < 8; ++i) sum += colour_gg(rowcol(R[i], c12), rowcol(R[i], c21));
      }
    }
  double v2 = 1.0 / (sqrt(2.0) * p->g_fermi);
  double yt2 = p->m_t * p->m_t / v2, yb2 = p->m_b * p->m_b / v2;
  /* massless b quarks: (pb + pbbar)^2 = 2 pb.pbbar, which avoids the
   * cancellation in E^2 - p^2 of the pair (the Higgs width is 4 MeV) */
  double q2h = 2.0 * mdot(hb, hbb);
  return sum * decay_couplings(p, mom, pt, ptb) / 256.0 * yt2 * 6.0 * yb2 * q2h * bw2(q2h, p->m_h, p->w_h);
}

/* ------------------------------------------------------ ttbar b bbar --- */
/* g(k1, a) g(k2, b) -> t(p3, i) tbar(p4, j) b(p5, k) bbar(p6, l), the
 * irreducible background of Sec. 4's t tbar H analysis.  Tree level QCD
 * only: 36 Feynman diagrams, written out one by one with the Feynman rules
 * in one fixed convention (couplings g_s stripped, put back as g_s^8 in
 * |M|^2):
 *   quark-gluon vertex  i gamma^mu T^a,   quark propagator i (pslash+m)/(p^2-m^2),
 *   gluon propagator    -i g_mu_nu delta^ab / q^2,
 *   triple-gluon vertex (all momenta incoming, legs (k1,a,mu) (k2,b,nu) (k3,c,rho))
 *     f^abc [g^mu_nu (k1-k2)^rho + g^nu_rho (k2-k3)^mu + g^rho_mu (k3-k1)^nu],
 *   four-gluon vertex   -i [f^abe f^cde (g^mu_rho g^nu_sigma - g^mu_sigma g^nu_rho)
 *                          + f^ace f^bde (g^mu_nu g^rho_sigma - g^mu_sigma g^nu_rho)
 *                          + f^ade f^bce (g^mu_nu g^rho_sigma - g^mu_rho g^nu_sigma)].
 * Each diagram is a Lorentz factor A_d times a colour tensor c_d(a,b,i,j,k,l)
 * built from explicit Gell-Mann matrices; the colour sum is
 *   sum_colours |sum_d c_d A_d|^2 = sum_dd' A_d CM_dd' conj(A_d'),
 * CM_dd' = sum over all 5184 colour assignments of c_d conj(c_d').
 * The four-gluon diagram is kept as its three colour terms: 38 terms. */

#define NTB 38
static cx TG[8][3][3];
static double FABC[8][8][8];
static cx CMAT[NTB][NTB];
static cx TENS[NTB][5184];
static int ttbb_ready = 0;

/* colour words: symbols 'a', 'b' (the two gluons), 'c', 'e', 'g', 'h'
 * (internal, summed); tw and bw are the ordered generator products along the
 * top and the bottom line (from the quark end), f the structure constants,
 * up to two triples separated by '|' */
typedef struct { const char *tw, *bw, *f; } ttbb_colour;
static const ttbb_colour TTBB_COL[NTB] = {
  /* A: the b pair from a gluon off the top line, both gluons on the top line */
  {"abc", "c", ""}, {"acb", "c", ""}, {"bac", "c", ""}, {"bca", "c", ""}, {"cab", "c", ""}, {"cba", "c", ""},
  /* B: the top pair from a gluon off the b line, both gluons on the b line */
  {"c", "abc", ""}, {"c", "acb", ""}, {"c", "bac", ""}, {"c", "bca", ""}, {"c", "cab", ""}, {"c", "cba", ""},
  /* C: gluon x on the top line, y on the b line, a gluon exchanged; (x, y) =
   * (a, b) then (b, a); t order (x, exchange) / (exchange, x), b order
   * (y, exchange) / (exchange, y) */
  {"ac", "bc", ""}, {"ac", "cb", ""}, {"ca", "bc", ""}, {"ca", "cb", ""},
  {"bc", "ac", ""}, {"bc", "ca", ""}, {"cb", "ac", ""}, {"cb", "ca", ""},
  /* D: g g -> g* (e), on the top line with the b pair gluon (c) / on the b line */
  {"ec", "c", "abe"}, {"ce", "c", "abe"}, {"c", "ec", "abe"}, {"c", "ce", "abe"},
  /* E1: gluon x on the exchanged gluon, y on the top line / on the b line */
  {"be", "c", "ace"}, {"eb", "c", "ace"}, {"c", "be", "ace"}, {"c", "eb", "ace"},
  {"ae", "c", "bce"}, {"ea", "c", "bce"}, {"c", "ae", "bce"}, {"c", "ea", "bce"},
  /* E2: both gluons on the exchanged gluon: x then y from the b line, the
   * g g -> g* gluon joining it, the four-gluon vertex (three terms) */
  {"g", "c", "ace|beg"}, {"g", "c", "bce|aeg"}, {"g", "c", "abe|ecg"},
  {"g", "c", "abh|cgh"}, {"g", "c", "ach|bgh"}, {"g", "c", "agh|bch"},
};

static void init_colour(void)
{
  memset(TG, 0, sizeof(TG));
  /* T^a = lambda^a / 2 */
  TG[0][0][1] = TG[0][1][0] = 0.5;
  TG[1][0][1] = -0.5 * I; TG[1][1][0] = 0.5 * I;
  TG[2][0][0] = 0.5; TG[2][1][1] = -0.5;
  TG[3][0][2] = TG[3][2][0] = 0.5;
  TG[4][0][2] = -0.5 * I; TG[4][2][0] = 0.5 * I;
  TG[5][1][2] = TG[5][2][1] = 0.5;
  TG[6][1][2] = -0.5 * I; TG[6][2][1] = 0.5 * I;
  TG[7][0][0] = TG[7][1][1] = 0.5 / sqrt(3.0); TG[7][2][2] = -1.0 / sqrt(3.0);
  /* f^abc = -2i Tr([T^a, T^b] T^c) */
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      for (int c = 0; c < 8; ++c) {
        cx t = 0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
              t += (TG[a][i][j] * TG[b][j][k] - TG[b][i][j] * TG[a][j][k]) * TG[c][k][i];
        FABC[a][b][c] = creal(-2.0 * I * t);
      }
}

/* product of the generators named by word w (symbol values in v) */
static void word_mat(const char* w, const int* v, cx out[3][3])
{
  cx m[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (const char* s = w; *s; ++s) {
    const int g = v[(int)*s];
    cx r[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cx t = 0;
        for (int k = 0; k < 3; ++k) t += m[i][k] * TG[g][k][j];
        r[i][j] = t;
      }
    memcpy(m, r, sizeof(m));
  }
  memcpy(out, m, sizeof(m));
}

/* colour tensor of term d: t[a][b][i][j][k][l] (5184 entries) */
static void colour_tensor(int d, cx* t)
{
  const ttbb_colour* c = &TTBB_COL[d];
  static const char internal[4] = {'c', 'e', 'g', 'h'};
  int used[4] = {0, 0, 0, 0}, n_used = 0;
  for (int q = 0; q < 4; ++q) {
    used[q] = strchr(c->tw, internal[q]) != NULL || strchr(c->bw, internal[q]) != NULL
              || strchr(c->f, internal[q]) != NULL;
    n_used += used[q];
  }
  memset(t, 0, sizeof(cx) * 5184);
  int v[128];
  int n_int = 1;
  for (int q = 0; q < n_used; ++q) n_int *= 8;
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      for (int it = 0; it < n_int; ++it) {
        v['a'] = a; v['b'] = b;
        int r = it;
        for (int q = 0; q < 4; ++q)
          if (used[q]) { v[(int)internal[q]] = r % 8; r /= 8; }
        double f = 1.0;
        for (const char* s = c->f; *s; s += (s[3] == '|') ? 4 : 3) {
          f *= FABC[v[(int)s[0]]][v[(int)s[1]]][v[(int)s[2]]];
          if (s[3] == 0) break;
        }
        if (f == 0.0) continue;
        cx mt[3][3], mb[3][3];
        word_mat(c->tw, v, mt);
        word_mat(c->bw, v, mb);
        cx* o = t + (a * 8 + b) * 81;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
              for (int l = 0; l < 3; ++l) o[((i * 3 + j) * 3 + k) * 3 + l] += f * mt[i][j] * mb[k][l];
      }
}

static void init_ttbb(void)
{
  if (ttbb_ready) return;
  init_gamma();
  init_colour();
  for (int d = 0; d < NTB; ++d) colour_tensor(d, TENS[d]);
  for (int d = 0; d < NTB; ++d)
    for (int e = 0; e < NTB; ++e) {
      cx s = 0;
      for (int q = 0; q < 5184; ++q) s += TENS[d][q] * conj(TENS[e][q]);
      CMAT[d][e] = s;
    }
  ttbb_ready = 1;
}

double or_colour_matrix_ttbb(int d, int e)
{
  init_ttbb();
  return creal(CMAT[d][e]);
}
double or_colour_fabc(int a, int b, int c)
{
  init_ttbb();
  return FABC[a][b][c];
}

static cx cdot4(const cx* a, const cx* b) { return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]; }
static cx cdotr(const cx* a, const double* p) { return a[0] * p[0] - a[1] * p[1] - a[2] * p[2] - a[3] * p[3]; }

/* triple-gluon vertex contracted with two legs (J1, k1), (J2, k2), momenta
 * incoming; the third leg (incoming momentum k3 = -k1-k2) is left open:
 * W^rho = (J1.J2)(k1-k2)^rho + J2^rho J1.(k2-k3) + J1^rho J2.(k3-k1) */
static void vertex3(const cx* J1, const double* k1, const cx* J2, const double* k2, cx* W)
{
  double k3[4], d12[4], d23[4], d31[4];
  for (int i = 0; i < 4; ++i) {
    k3[i] = -k1[i] - k2[i];
    d12[i] = k1[i] - k2[i]; d23[i] = k2[i] - k3[i]; d31[i] = k3[i] - k1[i];
  }
  cx j12 = cdot4(J1, J2), a = cdotr(J1, d23), b = cdotr(J2, d31);
  for (int i = 0; i < 4; ++i) W[i] = j12 * d12[i] + a * J2[i] + b * J1[i];
}
/* the current of an internal gluon of momentum Q whose far end gives W:
 * (-i / Q^2) W */
static void gluon_current(const cx* W, const double* Q, cx* J)
{
  cx f = -I / mdot(Q, Q);
  for (int i = 0; i < 4; ++i) J[i] = f * W[i];
}

/* fermion line between its quark row and antiquark column, insertions in
 * order from the quark end: (i J1-slash) S(p - q1) (i J2-slash) ...
 * (i Jn-slash); p the outgoing quark momentum, q_k the momentum entering
 * at insertion k, S(p) = i (pslash + m) / (p^2 - m^2) */
static mat4 line_mat(double m, const double* pout, int n, cx J[][4], double q[][4])
{
  mat4 M = mscale(slash(J[0]), I);
  double p[4];
  memcpy(p, pout, sizeof(p));
  for (int k = 1; k < n; ++k) {
    for (int i = 0; i < 4; ++i) p[i] -= q[k - 1][i];
    mat4 S = mscale(madd(slash_r(p), ID4, m), I / (mdot(p, p) - m * m));
    M = mmul(mmul(M, S), mscale(slash(J[k]), I));
  }
  return M;
}

/* the top line's matrix when the top pair attaches through one gluon whose
 * other end is fn(J) for the gluon's current J (linear in J):
 * sum_nu fn(e_nu) (-i/Pt^2) i gamma^nu = (1/Pt^2) sum_nu fn(e_nu) gamma^nu */
typedef cx (*ttbb_rest_fn)(const cx* Jt, const void* ctx);

typedef struct {
  const double *k1, *k2, *p5, *p6, *Pt, *Pb;
  const cx *e1, *e2, *Gb;
  spin4 U, V;
  int x, y;        /* gluon indices 0/1 for the E1 terms */
  int order;       /* insertion order on the b line */
} bctx;

static const double* kk(const bctx* c, int g) { return g ? c->k2 : c->k1; }
static const cx* ee(const bctx* c, int g) { return g ? c->e2 : c->e1; }

static cx bline(const bctx* c, int n, cx J[][4], double q[][4])
{
  return rowcol(c->U, mvec(line_mat(0.0, c->p5, n, J, q), c->V));
}

/* B: b line with the two gluons and the top pair's gluon in one of 6 orders */
static const int PERM3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static cx rest_B(const cx* Jt, const void* vc)
{
  const bctx* c = vc;
  cx J[3][4];
  double q[3][4];
  for (int s = 0; s < 3; ++s) {
    int w = PERM3[c->order][s];
    for (int i = 0; i < 4; ++i) {
      J[s][i] = w == 0 ? c->e1[i] : w == 1 ? c->e2[i] : Jt[i];
      q[s][i] = w == 0 ? c->k1[i] : w == 1 ? c->k2[i] : -c->Pt[i];
    }
  }
  return bline(c, 3, J, q);
}
/* D on the b line: g g -> g* and the top pair's gluon */
static cx rest_Db(const cx* Jt, const void* vc)
{
  const bctx* c = vc;
  cx W[4], G12[4], J[2][4];
  double K[4], q[2][4];
  for (int i = 0; i < 4; ++i) K[i] = c->k1[i] + c->k2[i];
  vertex3(c->e1, c->k1, c->e2, c->k2, W);
  gluon_current(W, K, G12);
  for (int i = 0; i < 4; ++i) {
    J[c->order][i] = G12[i];     q[c->order][i] = K[i];
    J[1 - c->order][i] = Jt[i];  q[1 - c->order][i] = -c->Pt[i];
  }
  return bline(c, 2, J, q);
}
/* E1 on the b line: gluon x joins the top pair's gluon, gluon y on the b line */
static cx rest_E1b(const cx* Jt, const void* vc)
{
  const bctx* c = vc;
  const double* kx = kk(c, c->x);
  double mPt[4], Q[4], q[2][4];
  for (int i = 0; i < 4; ++i) { mPt[i] = -c->Pt[i]; Q[i] = kx[i] - c->Pt[i]; }
  cx W[4], G[4], J[2][4];
  vertex3(ee(c, c->x), kx, Jt, mPt, W);
  gluon_current(W, Q, G);
  const int sy = c->order == 0 ? 0 : 1;      /* order 0: (y, e), 1: (e, y) */
  for (int i = 0; i < 4; ++i) {
    J[sy][i] = ee(c, c->y)[i];  q[sy][i] = kk(c, c->y)[i];
    J[1 - sy][i] = G[i];        q[1 - sy][i] = Q[i];
  }
  return bline(c, 2, J, q);
}
static mat4 top_from_rest(ttbb_rest_fn fn, const bctx* c)
{
  mat4 M;
  memset(&M, 0, sizeof(M));
  for (int nu = 0; nu < 4; ++nu) {
    cx e[4] = {0, 0, 0, 0};
    e[nu] = 1.0;
    M = madd(M, G[nu], fn(e, c));
  }
  return mscale(M, 1.0 / mdot(c->Pt, c->Pt));
}

/* the 38 top-line matrices M_d (amplitude_d = R M_d C) for gluon
 * polarisations e1, e2 (complex, upper index) and b spinors U (row), V */
static void ttbb_mats(double mt, const double* k1, const double* k2, const double* p3, const double* p4,
                      const double* p5, const double* p6, const cx* e1, const cx* e2, spin4 U, spin4 V,
                      mat4* M)
{
  double Pb[4], Pt[4], mPb[4];
  for (int i = 0; i < 4; ++i) { Pb[i] = p5[i] + p6[i]; Pt[i] = p3[i] + p4[i]; mPb[i] = -Pb[i]; }
  /* the b pair's gluon current (1/Pb^2) ubar gamma V... from the rules:
   * (-i/Pb^2) U (i gamma^mu) V */
  cx Xb[4], Gb[4];
  for (int mu = 0; mu < 4; ++mu) Xb[mu] = I * rowcol(U, mvec(G[mu], V));
  gluon_current(Xb, Pb, Gb);
  const cx* E[2] = {e1, e2};
  const double* K[2] = {k1, k2};
  int d = 0;
  /* A */
  for (int o = 0; o < 6; ++o) {
    cx J[3][4];
    double q[3][4];
    for (int s = 0; s < 3; ++s) {
      int w = PERM3[o][s];
      for (int i = 0; i < 4; ++i) {
        J[s][i] = w < 2 ? E[w][i] : Gb[i];
        q[s][i] = w < 2 ? K[w][i] : mPb[i];
      }
    }
    M[d++] = line_mat(mt, p3, 3, J, q);
  }
  bctx c = {k1, k2, p5, p6, Pt, Pb, e1, e2, Gb, U, V, 0, 1, 0};
  /* B */
  for (int o = 0; o < 6; ++o) { c.order = o; M[d++] = top_from_rest(rest_B, &c); }
  /* C */
  for (int xy = 0; xy < 2; ++xy) {
    const int x = xy, y = 1 - xy;
    for (int to = 0; to < 2; ++to)
      for (int bo = 0; bo < 2; ++bo) {
        /* exchanged gluon: the b line with gluon y and an open index */
        double Q[4], qb[2][4];
        for (int i = 0; i < 4; ++i) Q[i] = Pb[i] - K[y][i];
        cx X[4];
        for (int mu = 0; mu < 4; ++mu) {
          cx Jb[2][4];
          cx eo[4] = {0, 0, 0, 0};
          eo[mu] = 1.0;
          const int sy = bo;     /* bo 0: (y, exchange), 1: (exchange, y) */
          for (int i = 0; i < 4; ++i) {
            Jb[sy][i] = E[y][i];  qb[sy][i] = K[y][i];
            Jb[1 - sy][i] = eo[i]; qb[1 - sy][i] = Q[i];
          }
          /* open upper index mu: slash(e_mu) = g_mumu gamma^mu */
          X[mu] = (mu == 0 ? 1.0 : -1.0) * rowcol(U, mvec(line_mat(0.0, p5, 2, Jb, qb), V));
        }
        cx Gx[4];
        gluon_current(X, Q, Gx);
        cx J[2][4];
        double q[2][4];
        const int sx = to;       /* to 0: (x, exchange), 1: (exchange, x) */
        for (int i = 0; i < 4; ++i) {
          J[sx][i] = E[x][i];   q[sx][i] = K[x][i];
          J[1 - sx][i] = Gx[i]; q[1 - sx][i] = -Q[i];
        }
        M[d++] = line_mat(mt, p3, 2, J, q);
      }
  }
  /* D */
  {
    cx W[4], G12[4];
    double Kt[4];
    for (int i = 0; i < 4; ++i) Kt[i] = k1[i] + k2[i];
    vertex3(e1, k1, e2, k2, W);
    gluon_current(W, Kt, G12);
    for (int o = 0; o < 2; ++o) {
      cx J[2][4];
      double q[2][4];
      for (int i = 0; i < 4; ++i) {
        J[o][i] = G12[i];    q[o][i] = Kt[i];
        J[1 - o][i] = Gb[i]; q[1 - o][i] = mPb[i];
      }
      M[d++] = line_mat(mt, p3, 2, J, q);
    }
    for (int o = 0; o < 2; ++o) { c.order = o; M[d++] = top_from_rest(rest_Db, &c); }
  }
  /* E1: x = gluon 1 (a) then x = gluon 2 (b) */
  for (int x = 0; x < 2; ++x) {
    const int y = 1 - x;
    double Q[4];
    for (int i = 0; i < 4; ++i) Q[i] = K[x][i] - Pb[i];
    cx W[4], Gxb[4];
    vertex3(E[x], K[x], Gb, mPb, W);
    gluon_current(W, Q, Gxb);
    for (int o = 0; o < 2; ++o) {    /* o 0: (y, e), 1: (e, y) */
      cx J[2][4];
      double q[2][4];
      for (int i = 0; i < 4; ++i) {
        J[o][i] = E[y][i];    q[o][i] = K[y][i];
        J[1 - o][i] = Gxb[i]; q[1 - o][i] = Q[i];
      }
      M[d++] = line_mat(mt, p3, 2, J, q);
    }
    c.x = x; c.y = y;
    for (int o = 0; o < 2; ++o) { c.order = o; M[d++] = top_from_rest(rest_E1b, &c); }
  }
  /* E2: single insertion on the top line, carrying Pt */
  {
    cx Jt[6][4];
    for (int xy = 0; xy < 2; ++xy) {
      const int x = xy, y = 1 - xy;
      double Q[4], mQ[4];
      for (int i = 0; i < 4; ++i) { Q[i] = K[x][i] - Pb[i]; mQ[i] = Q[i]; }
      cx W[4], Gxb[4], W2[4];
      vertex3(E[x], K[x], Gb, mPb, W);
      gluon_current(W, Q, Gxb);
      vertex3(E[y], K[y], Gxb, mQ, W2);
      gluon_current(W2, Pt, Jt[xy]);
    }
    {
      cx W[4], G12[4], W2[4];
      double Kt[4];
      for (int i = 0; i < 4; ++i) Kt[i] = k1[i] + k2[i];
      vertex3(e1, k1, e2, k2, W);
      gluon_current(W, Kt, G12);
      vertex3(G12, Kt, Gb, mPb, W2);
      gluon_current(W2, Pt, Jt[2]);
    }
    {
      /* four-gluon vertex, legs (e1, mu) (e2, nu) (Gb, rho), open sigma */
      cx e1Gb = cdot4(e1, Gb), e2Gb = cdot4(e2, Gb), e1e2 = cdot4(e1, e2);
      cx X[3][4];
      for (int i = 0; i < 4; ++i) {
        X[0][i] = -I * (e1Gb * e2[i] - e1[i] * e2Gb);
        X[1][i] = -I * (e1e2 * Gb[i] - e1[i] * e2Gb);
        X[2][i] = -I * (e1e2 * Gb[i] - e1Gb * e2[i]);
      }
      for (int t = 0; t < 3; ++t) gluon_current(X[t], Pt, Jt[3 + t]);
    }
    for (int t = 0; t < 6; ++t) M[d++] = mscale(slash(Jt[t]), I);
  }
}

/* colour-summed |sum_d c_d R M_d C|^2 */
static double ttbb_colour_sum(spin4 R, spin4 C, const mat4* M)
{
  cx A[NTB];
  for (int d = 0; d < NTB; ++d) A[d] = rowcol(R, mvec(M[d], C));
  double s = 0.0;
  for (int d = 0; d < NTB; ++d) {
    cx t = 0;
    for (int e = 0; e < NTB; ++e) t += CMAT[d][e] * conj(A[e]);
    s += creal(A[d] * t);
  }
  return s;
}

/* the same sum with the colour-dressed amplitude formed for each of the
 * 5184 colour assignments (no cancellation between linearly dependent
 * colour terms: the form used where the sum is expected to vanish) */
static double ttbb_colour_sum_explicit(spin4 R, spin4 C, const mat4* M)
{
  cx A[NTB];
  for (int d = 0; d < NTB; ++d) A[d] = rowcol(R, mvec(M[d], C));
  double s = 0.0;
  for (int q = 0; q < 5184; ++q) {
    cx t = 0;
    for (int d = 0; d < NTB; ++d) t += TENS[d][q] * A[d];
    s += creal(t * conj(t));
  }
  return s;
}

static void pol_vec(int which, cx e[4])
{
  double r[4];
  lin_pol(which, r);
  for (int i = 0; i < 4; ++i) e[i] = r[i];
}

/* spin- and colour-summed |M|^2 of g g -> t tbar b bbar for on-shell tops of
 * mass mt (massless b), without couplings, averaged over the 256 initial
 * colours and polarisations */
static double gg_ttbb_prod(double mt, const double* k1, const double* k2, const double* p3, const double* p4,
                           const double* p5, const double* p6, int explicit_colour)
{
  init_ttbb();
  double sum = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int s5 = 0; s5 < 2; ++s5)
        for (int s6 = 0; s6 < 2; ++s6) {
          cx e1[4], e2[4];
          pol_vec(a, e1);
          pol_vec(b, e2);
          mat4 M[NTB];
          ttbb_mats(mt, k1, k2, p3, p4, p5, p6, e1, e2, dbar(spinor_u(p5, 0.0, s5)), spinor_v(p6, 0.0, s6), M);
          for (int st = 0; st < 2; ++st)
            for (int sb = 0; sb < 2; ++sb)
              sum += explicit_colour
                         ? ttbb_colour_sum_explicit(dbar(spinor_u(p3, mt, st)), spinor_v(p4, mt, sb), M)
                         : ttbb_colour_sum(dbar(spinor_u(p3, mt, st)), spinor_v(p4, mt, sb), M);
        }
  return sum / 256.0;
}
double or_gg_ttbb_prod(double mt, const double* k1, const double* k2, const double* p3, const double* p4,
                       const double* p5, const double* p6)
{
  return gg_ttbb_prod(mt, k1, k2, p3, p4, p5, p6, 0);
}
/* the same with the colour sum taken over explicit colour assignments */
double or_gg_ttbb_prod_explicit(double mt, const double* k1, const double* k2, const double* p3,
                                const double* p4, const double* p5, const double* p6)
{
  return gg_ttbb_prod(mt, k1, k2, p3, p4, p5, p6, 1);
}

/* Ward identity: with the polarisation of gluon g (0 or 1) replaced by its
 * momentum and the other gluon physical, the colour-summed |M|^2 vanishes.
 * Returns that sum relative to the one with physical polarisations. */
double or_gg_ttbb_ward(double mt, const double* k1, const double* k2, const double* p3, const double* p4,
                       const double* p5, const double* p6, int g)
{
  init_ttbb();
  double bad = 0.0, good = 0.0;
  for (int b = 0; b < 2; ++b)
    for (int s5 = 0; s5 < 2; ++s5)
      for (int s6 = 0; s6 < 2; ++s6) {
        cx ek[4], ep[4], eo[4];
        const double* kg = g ? k2 : k1;
        for (int i = 0; i < 4; ++i) ek[i] = kg[i];
        pol_vec(0, ep);
        pol_vec(b, eo);
        mat4 Mk[NTB], Mp[NTB];
        spin4 U = dbar(spinor_u(p5, 0.0, s5)), V = spinor_v(p6, 0.0, s6);
        if (g == 0) {
          ttbb_mats(mt, k1, k2, p3, p4, p5, p6, ek, eo, U, V, Mk);
          ttbb_mats(mt, k1, k2, p3, p4, p5, p6, ep, eo, U, V, Mp);
        } else {
          ttbb_mats(mt, k1, k2, p3, p4, p5, p6, eo, ek, U, V, Mk);
          ttbb_mats(mt, k1, k2, p3, p4, p5, p6, eo, ep, U, V, Mp);
        }
        for (int st = 0; st < 2; ++st)
          for (int sb = 0; sb < 2; ++sb) {
            spin4 R = dbar(spinor_u(p3, mt, st)), C = spinor_v(p4, mt, sb);
            bad += ttbb_colour_sum_explicit(R, C, Mk);
            good += ttbb_colour_sum_explicit(R, C, Mp);
          }
      }
  return good > 0.0 ? fabs(bad) / good : fabs(bad);
}

/* g g -> t tbar b bbar with decayed tops (as or_tt_me2_gg): spin- and
 * colour-summed |M|^2 averaged over initial states, times the top and W
 * Breit-Wigner factors and all couplings (g_s^8 for the production).
 * mom: the six top decay momenta; p5, p6: the b and bbar of the gluon. */
double or_ttbb_me2_gg(const or_params* p, const double* k1, const double* k2, const double* mom, const double* p5,
                      const double* p6)
{
  init_ttbb();
  spin4 R[8], C[8];
  double pt[4], ptb[4];
  decay_wavefunctions(p->m_t, mom, R, C, pt, ptb);
  double sum = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int s5 = 0; s5 < 2; ++s5)
        for (int s6 = 0; s6 < 2; ++s6) {
          cx e1[4], e2[4];
          pol_vec(a, e1);
          pol_vec(b, e2);
          mat4 M[NTB];
          ttbb_mats(p->m_t, k1, k2, pt, ptb, p5, p6, e1, e2, dbar(spinor_u(p5, 0.0, s5)), spinor_v(p6, 0.0, s6), M);
          for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) sum += ttbb_colour_sum(R[i], C[j], M);
        }
  double gs2 = 4.0 * M_PI * p->alpha_s;
  return sum * decay_couplings(p, mom, pt, ptb) * gs2 * gs2 / 256.0;
}
