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
