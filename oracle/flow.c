/*
 * Oracle: the learned importance-sampling proposal (conditional
 * rational-quadratic spline flow on the unit cube).
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper's integration uses VEGAS (Sec. 2); the proposal is an
 * additional importance sampler whose estimator f(x)/q(x) stays unbiased.
 * Spline: Durkan, Bekasov, Murray, Papamakarios (2019), monotone
 * rational-quadratic segments on K bins with boundary derivatives 1.
 *
 * Definition (shared with the GPU side by specification, not by code):
 *  - T maps x in [0,1]^8 to z in [0,1]^8 through 6 coupling layers; before
 *    layer 3 the coordinate order is reversed.  Layer l transforms the
 *    positions {1,3,5,7} (l even) or {0,2,4,6} (l odd), conditioned on the
 *    other four and on a 24-value event context.
 *  - per layer an MLP 28 -> 128 -> 128 -> 92 with SiLU, input
 *    [conditioning values ascending, context]; output per transformed
 *    position j (ascending): 8 width logits, 8 height logits, 7 interior
 *    derivative logits at theta[23 j ..].
 *  - widths = m + (1 - K m) softmax, same for heights, m = 1e-3;
 *    derivatives = m + softplus(logit + c0), c0 = ln(e^(1-m) - 1), so a
 *    zero output gives the identity map; boundary derivatives 1.
 *  - log q(x|c) = sum over layers and transformed positions of
 *    log dz/dx (the base density on the cube is 1).
 *  - parameters per layer, row-major (out x in): W1[128][28], b1, W2[128][128],
 *    b2, W3[92][128], b3; 32 092 per layer, 192 552 in total.
 */
#include "oracle.h"
#include <math.h>
#include <string.h>
#include <stdlib.h>

#define FK 8
#define FMIN 1e-3
#define FH 128
#define FIN 28
#define FOUT 92
#define FLAYERS 6
#define FPER (FH * FIN + FH + FH * FH + FH + FOUT * FH + FOUT)

int or_flow_nparams(void) { return FLAYERS * FPER; }

static double softplus(double v) { return v > 30.0 ? v : log1p(exp(v)); }
static double sigmoid(double v) { return 1.0 / (1.0 + exp(-v)); }
static double silu(double v) { return v * sigmoid(v); }

/* spline knots from the 23 logits of one transformed position */
typedef struct { double xk[FK + 1], yk[FK + 1], d[FK + 1], w[FK], h[FK]; } spline_t;

static void spline_from_logits(const double* th, spline_t* s)
{
  double mw = -1e300, mh = -1e300;
  for (int k = 0; k < FK; ++k) { mw = fmax(mw, th[k]); mh = fmax(mh, th[FK + k]); }
  double sw = 0.0, sh = 0.0, ew[FK], eh[FK];
  for (int k = 0; k < FK; ++k) { ew[k] = exp(th[k] - mw); sw += ew[k]; eh[k] = exp(th[FK + k] - mh); sh += eh[k]; }
  s->xk[0] = 0.0; s->yk[0] = 0.0;
  for (int k = 0; k < FK; ++k) {
    s->w[k] = FMIN + (1.0 - FK * FMIN) * ew[k] / sw;
    s->h[k] = FMIN + (1.0 - FK * FMIN) * eh[k] / sh;
    s->xk[k + 1] = s->xk[k] + s->w[k];
    s->yk[k + 1] = s->yk[k] + s->h[k];
  }
  s->xk[FK] = 1.0; s->yk[FK] = 1.0;
  const double c0 = log(exp(1.0 - FMIN) - 1.0);
  s->d[0] = 1.0; s->d[FK] = 1.0;
  for (int k = 1; k < FK; ++k) s->d[k] = FMIN + softplus(th[2 * FK + k - 1] + c0);
}

static int spline_bin(const double* edges, double v)
{
  int k = 0;
  while (k < FK - 1 && v >= edges[k + 1]) ++k;
  return k;
}

/* forward spline: y and log dy/dx at x in [0,1] */
static double spline_fwd(const spline_t* s, double x, double* logdet)
{
  int k = spline_bin(s->xk, x);
  double w = s->w[k], h = s->h[k], sk = h / w;
  double t = (x - s->xk[k]) / w, omt = 1.0 - t;
  double den = sk + (s->d[k + 1] + s->d[k] - 2.0 * sk) * t * omt;
  double y = s->yk[k] + h * (sk * t * t + s->d[k] * t * omt) / den;
  double num = sk * sk * (s->d[k + 1] * t * t + 2.0 * sk * t * omt + s->d[k] * omt * omt);
  *logdet = log(num) - 2.0 * log(den);
  return y;
}

/* inverse spline: the x whose forward image is y, by the quadratic in t */
static double spline_inv(const spline_t* s, double y, double* logdet)
{
  int k = spline_bin(s->yk, y);
  double w = s->w[k], h = s->h[k], sk = h / w;
  double dy = y - s->yk[k];
  double g = s->d[k + 1] + s->d[k] - 2.0 * sk;
  double a = h * (sk - s->d[k]) + dy * g;
  double b = h * s->d[k] - dy * g;
  double c = -sk * dy;
  double disc = b * b - 4.0 * a * c;
  if (disc < 0.0) disc = 0.0;
  double t = (2.0 * c) / (-b - sqrt(disc));
  double x = s->xk[k] + t * w;
  if (x < 0.0) x = 0.0;
  if (x > 1.0) x = 1.0;
  spline_fwd(s, x, logdet);
  return x;
}

static void layer_mlp(const double* P, const double* in28, double* out92, double* h1, double* h2, double* a1,
                      double* a2)
{
  const double *W1 = P, *b1 = W1 + FH * FIN, *W2 = b1 + FH, *b2 = W2 + FH * FH, *W3 = b2 + FH, *b3 = W3 + FOUT * FH;
  for (int o = 0; o < FH; ++o) {
    double s = b1[o];
    for (int i = 0; i < FIN; ++i) s += W1[o * FIN + i] * in28[i];
    a1[o] = s;
    h1[o] = silu(s);
  }
  for (int o = 0; o < FH; ++o) {
    double s = b2[o];
    for (int i = 0; i < FH; ++i) s += W2[o * FH + i] * h1[i];
    a2[o] = s;
    h2[o] = silu(s);
  }
  for (int o = 0; o < FOUT; ++o) {
    double s = b3[o];
    for (int i = 0; i < FH; ++i) s += W3[o * FH + i] * h2[i];
    out92[o] = s;
  }
}

static void masks(int l, int* A, int* B)
{
  for (int j = 0; j < 4; ++j) {
    A[j] = (l % 2 == 0) ? 2 * j + 1 : 2 * j;
    B[j] = (l % 2 == 0) ? 2 * j : 2 * j + 1;
  }
}

static void reverse8(double* v)
{
  for (int i = 0; i < 4; ++i) { double t = v[i]; v[i] = v[7 - i]; v[7 - i] = t; }
}

double or_flow_forward(const double* params, const double* ctx, const double* x_in, double* z_out)
{
  double v[8], logq = 0.0;
  memcpy(v, x_in, sizeof(v));
  for (int l = 0; l < FLAYERS; ++l) {
    if (l == 3) reverse8(v);
    int A[4], B[4];
    masks(l, A, B);
    double in[FIN], th[FOUT], h1[FH], h2[FH], a1[FH], a2[FH];
    for (int j = 0; j < 4; ++j) in[j] = v[B[j]];
    for (int j = 0; j < 24; ++j) in[4 + j] = ctx[j];
    layer_mlp(params + (size_t)l * FPER, in, th, h1, h2, a1, a2);
    for (int j = 0; j < 4; ++j) {
      spline_t s;
      spline_from_logits(th + 23 * j, &s);
      double ld;
      v[A[j]] = spline_fwd(&s, v[A[j]], &ld);
      logq += ld;
    }
  }
  if (z_out) memcpy(z_out, v, sizeof(v));
  return logq;
}

double or_flow_inverse(const double* params, const double* ctx, const double* z_in, double* x_out)
{
  double v[8], logq = 0.0;
  memcpy(v, z_in, sizeof(v));
  for (int l = FLAYERS - 1; l >= 0; --l) {
    int A[4], B[4];
    masks(l, A, B);
    double in[FIN], th[FOUT], h1[FH], h2[FH], a1[FH], a2[FH];
    for (int j = 0; j < 4; ++j) in[j] = v[B[j]];
    for (int j = 0; j < 24; ++j) in[4 + j] = ctx[j];
    layer_mlp(params + (size_t)l * FPER, in, th, h1, h2, a1, a2);
    for (int j = 0; j < 4; ++j) {
      spline_t s;
      spline_from_logits(th + 23 * j, &s);
      double ld;
      v[A[j]] = spline_inv(&s, v[A[j]], &ld);
      logq += ld;
    }
    if (l == 3) reverse8(v);
  }
  memcpy(x_out, v, sizeof(v));
  return logq;
}

/* Event context for the dilepton flow: jets in assignment order, l+, l-,
 * their sum, each as (log(E/100), px/100, py/100, pz/100), then the missing
 * transverse momentum -sum p_T as (log((|MET|+1)/100), MET_x/100,
 * MET_y/100, 0).  ev = jet, jet, l+, l- as 4 x {E,px,py,pz}. */
void or_flow_context(const double* ev, int perm, double* ctx)
{
  const double* o[4] = {ev + (perm ? 4 : 0), ev + (perm ? 0 : 4), ev + 8, ev + 12};
  double S[4] = {0, 0, 0, 0};
  for (int k = 0; k < 4; ++k) {
    for (int i = 0; i < 4; ++i) S[i] += o[k][i];
    ctx[4 * k] = log(o[k][0] / 100.0);
    for (int i = 1; i < 4; ++i) ctx[4 * k + i] = o[k][i] / 100.0;
  }
  ctx[16] = log(S[0] / 100.0);
  for (int i = 1; i < 4; ++i) ctx[16 + i] = S[i] / 100.0;
  double mx = -S[1], my = -S[2];
  ctx[20] = log((sqrt(mx * mx + my * my) + 1.0) / 100.0);
  ctx[21] = mx / 100.0;
  ctx[22] = my / 100.0;
  ctx[23] = 0.0;
}

/* ----------------------------------------------------------- backward --- */
/* d log(dy/dx) and d y w.r.t. the spline inputs: the 23 logits and x, by
 * the chain rule through knots, widths, heights and derivatives. */
static void spline_grad(const double* th, double x, double* y_out, double* ld_out, double* dy_dth,
                        double* dld_dth, double* dy_dx, double* dld_dx)
{
  /* forward quantities */
  spline_t s;
  spline_from_logits(th, &s);
  int k = spline_bin(s.xk, x);
  /* parameters of the bin as functions of (w_j, h_j, d_j) */
  double w = s.w[k], h = s.h[k], xk = s.xk[k], yk = s.yk[k], d0 = s.d[k], d1 = s.d[k + 1];
  double t = (x - xk) / w, omt = 1.0 - t, sk = h / w;
  double g = d1 + d0 - 2.0 * sk;
  double den = sk + g * t * omt;
  double numy = sk * t * t + d0 * t * omt;
  double y = yk + h * numy / den;
  double nd = d1 * t * t + 2.0 * sk * t * omt + d0 * omt * omt;
  double ld = 2.0 * log(sk) + log(nd) - 2.0 * log(den);
  *y_out = y;
  *ld_out = ld;
  /* partial derivatives w.r.t. the local variables (t, sk, h, yk, d0, d1) */
  double dy_dt = h * ((2.0 * sk * t + d0 * (1.0 - 2.0 * t)) * den - numy * g * (1.0 - 2.0 * t)) / (den * den);
  double dy_dsk = h * ((t * t) * den - numy * (1.0 - 2.0 * t * omt)) / (den * den);
  double dy_dh = numy / den;
  double dy_dyk = 1.0;
  double dy_dd0 = h * ((t * omt) * den - numy * t * omt) / (den * den);
  double dy_dd1 = h * (-numy * t * omt) / (den * den);
  double dld_dt = (2.0 * d1 * t + 2.0 * sk * (1.0 - 2.0 * t) - 2.0 * d0 * omt) / nd - 2.0 * g * (1.0 - 2.0 * t) / den;
  double dld_dsk = 2.0 / sk + 2.0 * t * omt / nd - 2.0 * (1.0 - 2.0 * t * omt) / den;
  double dld_dd0 = omt * omt / nd - 2.0 * t * omt / den;
  double dld_dd1 = t * t / nd - 2.0 * t * omt / den;
  /* t = (x - xk)/w, sk = h/w */
  *dy_dx = dy_dt / w;
  *dld_dx = dld_dt / w;
  double dy_dw = dy_dt * (-t / w) + dy_dsk * (-h / (w * w));
  double dld_dw = dld_dt * (-t / w) + dld_dsk * (-h / (w * w));
  double dy_dxk = -dy_dt / w, dld_dxk = -dld_dt / w;
  double dy_dhh = dy_dh + dy_dsk / w, dld_dh = dld_dsk / w;
  /* gradients w.r.t. every width / height / derivative */
  double gw[FK], gh[FK], gd[FK + 1];
  double lw[FK], lh[FK], ldd[FK + 1];
  for (int j = 0; j < FK; ++j) { gw[j] = gh[j] = lw[j] = lh[j] = 0.0; }
  for (int j = 0; j <= FK; ++j) { gd[j] = ldd[j] = 0.0; }
  gw[k] += dy_dw; lw[k] += dld_dw;
  gh[k] += dy_dhh; lh[k] += dld_dh;
  for (int j = 0; j < k; ++j) { gw[j] += dy_dxk; lw[j] += dld_dxk; gh[j] += dy_dyk; }
  gd[k] += dy_dd0; gd[k + 1] += dy_dd1;
  ldd[k] += dld_dd0; ldd[k + 1] += dld_dd1;
  /* through softmax (widths, heights) and softplus (interior derivatives) */
  double mw = -1e300, mh = -1e300;
  for (int j = 0; j < FK; ++j) { mw = fmax(mw, th[j]); mh = fmax(mh, th[FK + j]); }
  double sw = 0.0, sh = 0.0, pw[FK], ph[FK];
  for (int j = 0; j < FK; ++j) { pw[j] = exp(th[j] - mw); sw += pw[j]; ph[j] = exp(th[FK + j] - mh); sh += ph[j]; }
  for (int j = 0; j < FK; ++j) { pw[j] /= sw; ph[j] /= sh; }
  double cw = 1.0 - FK * FMIN;
  double aw = 0.0, ah = 0.0, law = 0.0, lah = 0.0;
  for (int j = 0; j < FK; ++j) { aw += gw[j] * pw[j]; ah += gh[j] * ph[j]; law += lw[j] * pw[j]; lah += lh[j] * ph[j]; }
  for (int j = 0; j < FK; ++j) {
    dy_dth[j] = cw * pw[j] * (gw[j] - aw);
    dld_dth[j] = cw * pw[j] * (lw[j] - law);
    dy_dth[FK + j] = cw * ph[j] * (gh[j] - ah);
    dld_dth[FK + j] = cw * ph[j] * (lh[j] - lah);
  }
  const double c0 = log(exp(1.0 - FMIN) - 1.0);
  for (int j = 1; j < FK; ++j) {
    double sg = sigmoid(th[2 * FK + j - 1] + c0);
    dy_dth[2 * FK + j - 1] = gd[j] * sg;
    dld_dth[2 * FK + j - 1] = ldd[j] * sg;
  }
}

/* Weighted negative log-likelihood L = -sum_i wt_i log q(x_i | c_i) and its
 * gradient (added into grad, length or_flow_nparams()).  x: [n][8],
 * ctx: [n][24], wt: [n].  Reverse-mode through every layer. */
double or_flow_nll_grad(const double* params, int n, const double* x, const double* ctx, const double* wt,
                        double* grad)
{
  double loss = 0.0;
  /* per-sample tape */
  typedef struct {
    double vin[8];            /* layer input vector (after the reversal at l == 3) */
    double in[FIN], a1[FH], h1[FH], a2[FH], h2[FH], th[FOUT];
  } tape_t;
  tape_t* T = (tape_t*)malloc(sizeof(tape_t) * FLAYERS);
  for (int i = 0; i < n; ++i) {
    double v[8], logq = 0.0;
    memcpy(v, x + 8 * i, sizeof(v));
    for (int l = 0; l < FLAYERS; ++l) {
      if (l == 3) reverse8(v);
      memcpy(T[l].vin, v, sizeof(v));
      int A[4], B[4];
      masks(l, A, B);
      for (int j = 0; j < 4; ++j) T[l].in[j] = v[B[j]];
      for (int j = 0; j < 24; ++j) T[l].in[4 + j] = ctx[24 * i + j];
      layer_mlp(params + (size_t)l * FPER, T[l].in, T[l].th, T[l].h1, T[l].h2, T[l].a1, T[l].a2);
      for (int j = 0; j < 4; ++j) {
        spline_t s;
        spline_from_logits(T[l].th + 23 * j, &s);
        double ld;
        v[A[j]] = spline_fwd(&s, v[A[j]], &ld);
        logq += ld;
      }
    }
    loss -= wt[i] * logq;
    /* backward: gv = dL/d(layer output vector) */
    double gv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double gl = -wt[i];      /* dL/d(logq) */
    for (int l = FLAYERS - 1; l >= 0; --l) {
      int A[4], B[4];
      masks(l, A, B);
      const double* P = params + (size_t)l * FPER;
      double* G = grad + (size_t)l * FPER;
      const double *W1 = P, *W2 = W1 + FH * FIN + FH, *W3 = W2 + FH * FH + FH;
      double *gW1 = G, *gb1 = gW1 + FH * FIN, *gW2 = gb1 + FH, *gb2 = gW2 + FH * FH, *gW3 = gb2 + FH,
             *gb3 = gW3 + FOUT * FH;
      double gth[FOUT];
      double gvin[8];
      for (int d = 0; d < 8; ++d) gvin[d] = gv[d];     /* identity part */
      for (int j = 0; j < 4; ++j) {
        double y, ld, dyt[23], dldt[23], dydx, dlddx;
        spline_grad(T[l].th + 23 * j, T[l].vin[A[j]], &y, &ld, dyt, dldt, &dydx, &dlddx);
        double gy = gv[A[j]];
        for (int m = 0; m < 23; ++m) gth[23 * j + m] = gy * dyt[m] + gl * dldt[m];
        gvin[A[j]] = gy * dydx + gl * dlddx;
      }
      /* MLP backward */
      double gh2[FH], ga2[FH], gh1[FH], ga1[FH], gin[FIN];
      for (int o = 0; o < FOUT; ++o) {
        gb3[o] += gth[o];
        for (int q = 0; q < FH; ++q) gW3[o * FH + q] += gth[o] * T[l].h2[q];
      }
      for (int q = 0; q < FH; ++q) {
        double s = 0.0;
        for (int o = 0; o < FOUT; ++o) s += W3[o * FH + q] * gth[o];
        gh2[q] = s;
        double sg = sigmoid(T[l].a2[q]);
        ga2[q] = s * (sg * (1.0 + T[l].a2[q] * (1.0 - sg)));
      }
      for (int o = 0; o < FH; ++o) {
        gb2[o] += ga2[o];
        for (int q = 0; q < FH; ++q) gW2[o * FH + q] += ga2[o] * T[l].h1[q];
      }
      for (int q = 0; q < FH; ++q) {
        double s = 0.0;
        for (int o = 0; o < FH; ++o) s += W2[o * FH + q] * ga2[o];
        gh1[q] = s;
        double sg = sigmoid(T[l].a1[q]);
        ga1[q] = s * (sg * (1.0 + T[l].a1[q] * (1.0 - sg)));
      }
      for (int o = 0; o < FH; ++o) {
        gb1[o] += ga1[o];
        for (int q = 0; q < FIN; ++q) gW1[o * FIN + q] += ga1[o] * T[l].in[q];
      }
      for (int q = 0; q < 4; ++q) {
        double s = 0.0;
        for (int o = 0; o < FH; ++o) s += W1[o * FIN + q] * ga1[o];
        gin[q] = s;
      }
      for (int j = 0; j < 4; ++j) gvin[B[j]] += gin[j];
      (void)gh2; (void)gh1;
      memcpy(gv, gvin, sizeof(gv));
      if (l == 3) reverse8(gv);
    }
  }
  free(T);
  return loss;
}
