// Process parameters as the kernels see them, derived on the host from a
// process description and its transfer functions (couplings, Breit-Wigner
// map ranges, the constant factors of each integrand).  Host code only.
#pragma once
#include <algorithm>
#include <cmath>

#include "../../include/mem.h"
#include "process.hpp"

namespace memk {

// The transfer functions a new process starts with: muons Gaussian 5 %,
// b-jets Gaussian 15 % (double Gaussian 10 %/25 %, tail 0.2, for t tbar H,
// semileptonic), light jets double Gaussian 10 %/25 %, tail 0.2; window 5,
// r_min 0.1; leptons exact.
inline void default_tfs(int32_t kind, mem_tf_desc (&tf)[5])
{
  for (int c = 0; c < 5; ++c) tf[c] = mem_tf_desc{c, MEM_TF_DELTA, 0.0, 0.0, 0.0, 5.0, 0.1};
  tf[MEM_OBJ_MUON] = mem_tf_desc{MEM_OBJ_MUON, MEM_TF_GAUSS, 0.05, 0.05, 0.0, 5.0, 0.1};
  tf[MEM_OBJ_BJET] = mem_tf_desc{MEM_OBJ_BJET, MEM_TF_GAUSS, 0.15, 0.15, 0.0, 5.0, 0.1};
  tf[MEM_OBJ_LJET] = mem_tf_desc{MEM_OBJ_LJET, MEM_TF_DGAUSS, 0.10, 0.25, 0.2, 5.0, 0.1};
  tf[MEM_OBJ_NEUTRINO] = mem_tf_desc{MEM_OBJ_NEUTRINO, MEM_TF_UNIFORM, 0.0, 0.0, 0.0, 5.0, 0.1};
  if (kind == MEM_TTH_SEMILEPTON)   // every jet double-Gaussian
    tf[MEM_OBJ_BJET] = mem_tf_desc{MEM_OBJ_BJET, MEM_TF_DGAUSS, 0.10, 0.25, 0.2, 5.0, 0.1};
}

// A transfer function's kernel form: widths, reciprocal widths, and the
// integration window in r = E_meas / E (window x the wider width, r >= r_min).
inline TFParams tf_params(const mem_tf_desc& t)
{
  TFParams p{};
  p.s_core = t.sigma_core;
  p.s_tail = t.kind == MEM_TF_DGAUSS ? t.sigma_tail : t.sigma_core;
  p.f_tail = t.kind == MEM_TF_DGAUSS ? t.f_tail : 0.0;
  double smax = std::max(p.s_core, p.s_tail);
  p.r_lo = std::max(t.r_min, 1.0 - t.window * smax);
  p.r_hi = 1.0 + t.window * smax;
  p.i_core = 1.0 / p.s_core;
  p.i_tail = 1.0 / p.s_tail;
  return p;
}

// The kernel parameters of a process (the grid fields of ProcParams are left
// empty: the library fills them from the process's PDF grid).
inline ProcParams derive_params(const mem_process_desc& d, const mem_tf_desc (&tf)[5])
{
  ProcParams pp{};
  pp.kind = d.kind;
  pp.precision = d.precision;
  pp.sqrt_s = d.sqrt_s;
  pp.S = d.sqrt_s * d.sqrt_s;
  pp.inv_sqrt_s = 1.0 / d.sqrt_s;
  pp.m_t = d.m_top; pp.w_t = d.w_top; pp.m_w = d.m_w; pp.w_w = d.w_w;
  pp.alpha = d.alpha; pp.alpha_s = d.alpha_s; pp.g_fermi = d.g_fermi;
  pp.sigma_k = d.sigma_k;
  pp.m_lo = d.m_lo; pp.m_hi = d.m_hi;
  pp.sigma_norm = d.sigma_norm;
  pp.tf_mu = tf_params(tf[MEM_OBJ_MUON]);
  pp.tf_b = tf_params(tf[MEM_OBJ_BJET]);
  pp.tf_lj = tf_params(tf[MEM_OBJ_LJET]);
  const double two_pi = 2.0 * M_PI;
  if (d.kind == MEM_DY_QQ_GAMMA_MUMU) {
    pp.dims = 2;
    pp.n_perm = 1;
    double e2 = 4.0 * M_PI * d.alpha;
    pp.dy_const = std::pow(two_pi, -2.0) * (2.0 / pp.S) * e2 * e2 / 3.0 * 0.5;
  } else {
    pp.dims = d.kind == MEM_TT_SEMILEPTON ? 7 : d.kind == MEM_TTH_SEMILEPTON ? 9 : 8;
    pp.n_perm = d.kind == MEM_TT_SEMILEPTON ? 12 : d.kind == MEM_TTH_SEMILEPTON ? 24
              : d.kind == MEM_TTH_DILEPTON ? 12 : d.kind == MEM_TTBB_DILEPTON ? 24 : 2;
    double mtg = d.m_top * d.w_top, mwg = d.m_w * d.w_w;
    pp.th0_t = std::atan((0.0 - d.m_top * d.m_top) / mtg);
    pp.th1_t = std::atan((pp.S - d.m_top * d.m_top) / mtg);
    pp.th0_w = std::atan((0.0 - d.m_w * d.m_w) / mwg);
    pp.th1_w = std::atan((pp.S - d.m_w * d.m_w) / mwg);
    double kbw = std::pow((pp.th1_t - pp.th0_t) / mtg, 2) * std::pow((pp.th1_w - pp.th0_w) / mwg, 2);
    double gs2 = 4.0 * M_PI * d.alpha_s;
    double gw2 = 8.0 * d.g_fermi * d.m_w * d.m_w / std::sqrt(2.0);
    double coup = gs2 * gs2 * std::pow(gw2 / 2.0, 4);
    pp.me_const = coup;
    // (2 pi)^(4 - 3*6) (2/S) / (2 shat) / (2E_nu 2E_nubar): shat, E's per point
    pp.tt_const = std::pow(two_pi, -14.0) * (2.0 / pp.S) * 0.5 * 0.25 * coup * kbw;
    // semileptonic: hadronic W, hadronic top and leptonic W aligned; the
    // 1/(2 E_nu) of the neutrino; colour 3 x two generations of the W -> q q'
    double kbw3 = (pp.th1_t - pp.th0_t) / mtg * std::pow((pp.th1_w - pp.th0_w) / mwg, 2);
    pp.sl_const = std::pow(two_pi, -14.0) * (2.0 / pp.S) * 0.5 * 0.5 * coup * kbw3 * 6.0;
    if (d.kind == MEM_TTH_SEMILEPTON) {
      // Higgs map aligned with its Breit-Wigner; Yukawa (m_t/v)^2 and the
      // H -> b bbar factor 6 (m_b/v)^2 q2_H (q2_H applied per point);
      // two more final-state particles: (2 pi)^-6
      const double mhg = d.m_h * d.w_h;
      pp.m_h = d.m_h; pp.w_h = d.w_h;
      pp.th0_h = std::atan((0.0 - d.m_h * d.m_h) / mhg);
      pp.th1_h = std::atan((pp.S - d.m_h * d.m_h) / mhg);
      const double v2 = 1.0 / (std::sqrt(2.0) * d.g_fermi);
      const double mb = d.m_b > 0.0 ? d.m_b : 4.18;
      pp.tth_const = pp.sl_const * std::pow(two_pi, -6.0) * (pp.th1_h - pp.th0_h) / mhg
                   * (d.m_top * d.m_top / v2) * 6.0 * (mb * mb / v2);
    }
    if (d.kind == MEM_TTH_DILEPTON || d.kind == MEM_TTBB_DILEPTON) {
      // eight final-state particles: (2 pi)^(4 - 24); all four top and W
      // propagators aligned
      const double base = std::pow(two_pi, -20.0) * (2.0 / pp.S) * 0.5 * 0.25 * std::pow(gw2 / 2.0, 4) * kbw / 256.0;
      const double pbase = std::pow(gw2 / 2.0, 4) / 256.0;
      if (d.kind == MEM_TTBB_DILEPTON) {
        pp.f2_const = base * gs2 * gs2 * gs2 * gs2;
        pp.f2_parton_const = pbase * gs2 * gs2 * gs2 * gs2;
      } else {
        const double mhg = d.m_h * d.w_h;
        pp.m_h = d.m_h; pp.w_h = d.w_h;
        pp.th0_h = std::atan((0.0 - d.m_h * d.m_h) / mhg);
        pp.th1_h = std::atan((pp.S - d.m_h * d.m_h) / mhg);
        const double v2 = 1.0 / (std::sqrt(2.0) * d.g_fermi);
        const double mb = d.m_b > 0.0 ? d.m_b : 4.18;
        pp.f2_const = base * gs2 * gs2 * (pp.th1_h - pp.th0_h) / mhg * (d.m_top * d.m_top / v2) * 6.0
                    * (mb * mb / v2);
        pp.f2_parton_const = pbase * gs2 * gs2 * (d.m_top * d.m_top / v2) * 6.0 * (mb * mb / v2);
      }
    }
  }
  return pp;
}


}  // namespace memk
