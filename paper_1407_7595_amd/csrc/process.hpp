// Process parameters as the kernels see them, and the per-event view.
#pragma once
#include <stdint.h>

namespace memk {

enum Kind : int32_t { kDY = 1, kTT = 2, kSL = 3, kTTH = 4, kTHL = 5, kTBB = 6 };

// One transfer function for the energy of a measured object, Gaussian or
// double Gaussian in r = E_meas / E_true (Sec. 1, after Eq. 3).
struct TFParams {
  double s_core, s_tail, f_tail;  // relative widths and tail fraction
  double r_lo, r_hi;              // integration window in r
  double i_core, i_tail;          // 1 / s_core, 1 / s_tail
};

// Everything the integrand needs about a hypothesis, precomputed on the host.
struct ProcParams {
  int32_t kind;
  int32_t precision;               // 0: FP64 matrix element stage, 1: FP32
  int32_t dims;
  int32_t n_perm;
  double sqrt_s, S, inv_sqrt_s;
  double m_t, w_t, m_w, w_w;
  double alpha, alpha_s, g_fermi;
  double sigma_k;
  double m_lo, m_hi;
  double sigma_norm;
  TFParams tf_mu;                  // Drell-Yan muons
  TFParams tf_b;                   // tt b-jets
  TFParams tf_lj;                  // light jets (semileptonic)
  // Breit-Wigner tan maps q2 = M^2 + M Gamma tan(theta), theta in [th0, th1]
  double th0_t, th1_t, th0_w, th1_w;
  double m_h, w_h, th0_h, th1_h;   // Higgs (t tbar H)
  // constant factors of the tt weight: couplings, (2 pi) powers, the
  // product of the four (th1 - th0)/(M Gamma) that remain after the
  // propagators cancel against the map Jacobians
  double tt_const;
  // Drell-Yan: (2 pi)^-2 (2/S) (4 pi alpha)^2 / 3 / 2
  double dy_const;
  // semileptonic: as tt_const with three aligned propagators and the
  // hadronic W's colour and generation factor
  double sl_const;
  // t tbar H: as sl_const with the Higgs map, the Yukawa coupling and the
  // H -> b bbar decay (times q2_H per point)
  double tth_const;
  // couplings of the t tbar |M|^2: g_s^4 (g_W^2 / 2)^4
  double me_const;
  // t tbar H and t tbar b bbar, dilepton: (2 pi)^-20 (2/S) / (2 shat)
  // / (2E_nu 2E_nubar), the couplings, the initial-state average 1/256 and
  // the (th1 - th0)/(M Gamma) of the aligned propagators (for t tbar H with
  // the Yukawa and H -> b bbar factors; times q2_H per point)
  double f2_const;
  // their parton-level weights: the couplings and 1/256 (Breit-Wigner
  // factors per point)
  double f2_parton_const;
  // parton densities from a grid (null: the toy densities): x f of the
  // 11 flavours in nodes of 12 floats (layout in pdf.hpp), [nq][nx][12],
  // uniform in ln x and ln Q; position = (ln v - v0) * inverse step
  const float* pdf_xf;
  int32_t pdf_nx, pdf_nq;
  double pdf_lx0, pdf_ihx, pdf_lq0, pdf_ihq;
  // the top processes' fixed scale m_t: its Q cell and weight
  int32_t pdf_iq_mt;
  double pdf_uq_mt;
};

struct EventsView {
  const double* E;
  const double* px;
  const double* py;
  const double* pz;
  const int32_t* charge;   // lepton charge per event (semileptonic), may be null
  int32_t n_events;
  int32_t n_obj;
  __device__ __forceinline__ void load(int obj, int ev, double& e, double& x, double& y, double& z) const
  {
    int64_t i = (int64_t)obj * n_events + ev;
    e = E[i]; x = px[i]; y = py[i]; z = pz[i];
  }
};

}  // namespace memk
