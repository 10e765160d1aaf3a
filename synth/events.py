"""Seeded synthetic collision events for the matrix element method.

This module is the only piece shared by the oracle side and the GPU side:
it draws input events and holds none of the method's arithmetic (no matrix
element, parton density, transfer-function density or phase-space weight).
Events are produced by sampling production and decay kinematics directly
(Breit-Wigner masses, isotropic two-body decays, a Gaussian transverse
recoil) and smearing energies with the detector resolution, so their shapes
match the processes of the paper's benchmark (Sec. 3 and 4) without being
weighted by any |M|^2.

Layouts: `obs` is float64 [n_events, n_obj, 4] with rows (E, px, py, pz).
  Drell-Yan:       mu-, mu+
  ttbar dilepton:  jet_a, jet_b, l+, l-    (b/bbar order random)
  ttbar semileptonic: j0..j3 (random order), lepton, (charge, 0, 0, 0)
  ttbar H:         b0..b3 (b-tagged, random order), l0, l1 (random order),
                   lepton, (charge, 0, 0, 0)
  ttbar H and ttbar b bbar, dilepton: b0..b3 (random order), l+, l-
"""
import numpy as np

SQRT_S = 13000.0
M_T, W_T = 172.5, 1.4
M_W, W_W = 80.4, 2.1
M_H = 125.0


def _rng(seed):
    return np.random.Generator(np.random.Philox(key=seed))


def _bw(rng, n, m, w, lo, hi):
    """Breit-Wigner (Cauchy) masses truncated to [lo, hi] by inverse CDF."""
    a0 = np.arctan((lo - m) / (0.5 * w))
    a1 = np.arctan((hi - m) / (0.5 * w))
    return m + 0.5 * w * np.tan(a0 + rng.random(n) * (a1 - a0))


def _iso(rng, n):
    c = 2.0 * rng.random(n) - 1.0
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    phi = 2.0 * np.pi * rng.random(n)
    return np.stack([s * np.cos(phi), s * np.sin(phi), c], axis=-1)


def _two_body(M, m1, m2, nhat):
    """momenta of a two-body decay at rest; returns p1, p2 as (n,4)"""
    p = np.sqrt(np.maximum(0.0, (M * M - (m1 + m2) ** 2) * (M * M - (m1 - m2) ** 2))) / (2.0 * M)
    e1 = np.sqrt(p * p + m1 * m1)
    e2 = np.sqrt(p * p + m2 * m2)
    v1 = np.concatenate([e1[:, None], p[:, None] * nhat], axis=1)
    v2 = np.concatenate([e2[:, None], -p[:, None] * nhat], axis=1)
    return v1, v2


def _boost(p, P):
    """boost four-vectors p (n,4) from the rest frame of P (n,4) to the lab"""
    M = np.sqrt(np.maximum(P[:, 0] ** 2 - np.sum(P[:, 1:] ** 2, axis=1), 1e-300))
    b = P[:, 1:] / P[:, :1]
    b2 = np.sum(b * b, axis=1)
    g = P[:, 0] / M
    bp = np.sum(b * p[:, 1:], axis=1)
    g2 = np.where(b2 > 0, (g - 1.0) / np.where(b2 > 0, b2, 1.0), 0.0)
    E = g * (p[:, 0] + bp)
    vec = p[:, 1:] + (g2 * bp + g * p[:, 0])[:, None] * b
    return np.concatenate([E[:, None], vec], axis=1)


def _massless(E, direction_from):
    n = direction_from[:, 1:] / np.linalg.norm(direction_from[:, 1:], axis=1, keepdims=True)
    return np.concatenate([E[:, None], E[:, None] * n], axis=1)


def _smear(rng, E, rel):
    """E (1 + rel z), redrawn while non-positive (the resolution model)"""
    out = E * (1.0 + rel * rng.standard_normal(E.shape))
    bad = out <= 0.0
    while np.any(bad):
        out[bad] = E[bad] * (1.0 + rel * rng.standard_normal(int(bad.sum())))
        bad = out <= 0.0
    return out


def drell_yan(n_events, seed, m_lo=60.0, m_hi=120.0, rel_sigma=0.05):
    """q qbar -> gamma* -> mu- mu+ at sqrt(S) = 13 TeV.  The pair mass has a
    falling m^-3 shape in [m_lo, m_hi], the pair rapidity is uniform inside
    |y| < 2.5 (and the kinematic limit), the decay angle follows 1 + cos^2,
    and each muon |p| is smeared by a Gaussian of relative width rel_sigma
    with its direction kept."""
    rng = _rng(seed)
    u = rng.random(n_events)
    m = 1.0 / np.sqrt(m_lo ** -2 + u * (m_hi ** -2 - m_lo ** -2))
    ymax = np.minimum(2.5, np.log(SQRT_S / m))
    y = (2.0 * rng.random(n_events) - 1.0) * ymax
    cth = np.empty(n_events)
    filled = 0
    while filled < n_events:
        c = 2.0 * rng.random(2 * n_events) - 1.0
        keep = c[rng.random(2 * n_events) * 2.0 < 1.0 + c * c]
        take = min(len(keep), n_events - filled)
        cth[filled:filled + take] = keep[:take]
        filled += take
    phi = 2.0 * np.pi * rng.random(n_events)
    s = np.sqrt(1.0 - cth * cth)
    nhat = np.stack([s * np.cos(phi), s * np.sin(phi), cth], axis=1)
    mu1, mu2 = _two_body(m, np.zeros(n_events), np.zeros(n_events), nhat)
    P = np.stack([m * np.cosh(y), np.zeros(n_events), np.zeros(n_events), m * np.sinh(y)], axis=1)
    mu1 = _boost(mu1, P)
    mu2 = _boost(mu2, P)
    truth = np.stack([mu1, mu2], axis=1)
    obs = np.empty_like(truth)
    for k in range(2):
        pm = _smear(rng, truth[:, k, 0], rel_sigma)
        obs[:, k] = _massless(pm, truth[:, k])
    return {"obs": obs, "truth": truth, "m": m}


def ttbar_dilepton(n_events, seed, rel_sigma=0.15, sigma_k=20.0):
    """pp -> t tbar -> b l+ nu bbar l- nubar.  Top and W masses are
    Breit-Wigner distributed, sqrt(shat) rises from threshold with a
    Gamma(2, 80 GeV) excess, the pair rapidity is Gaussian (width 1) within
    the kinematic limit, all decays are isotropic, the system receives a
    Gaussian transverse recoil k_T (sigma_k per component), b-jet energies
    are smeared by rel_sigma, leptons are exact, and the two b-jets are
    stored in random order."""
    rng = _rng(seed)
    n = n_events
    mt1 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mt2 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mw1 = _bw(rng, n, M_W, W_W, 65.0, 95.0)
    mw2 = _bw(rng, n, M_W, W_W, 65.0, 95.0)
    mtt = mt1 + mt2 + rng.gamma(2.0, 80.0, n)
    ymax = np.log(SQRT_S / mtt)
    y = np.clip(rng.standard_normal(n), -1.0, 1.0) * np.minimum(2.0, 0.9 * ymax)
    t, tb = _two_body(mtt, mt1, mt2, _iso(rng, n))
    b, wp = _two_body(mt1, np.zeros(n), mw1, _iso(rng, n))
    bb, wm = _two_body(mt2, np.zeros(n), mw2, _iso(rng, n))
    lp, nu = _two_body(mw1, np.zeros(n), np.zeros(n), _iso(rng, n))
    lm, nub = _two_body(mw2, np.zeros(n), np.zeros(n), _iso(rng, n))
    lp, nu = _boost(lp, wp), _boost(nu, wp)
    lm, nub = _boost(lm, wm), _boost(nub, wm)
    b, lp, nu = (_boost(v, t) for v in (b, lp, nu))
    bb, lm, nub = (_boost(v, tb) for v in (bb, lm, nub))
    # longitudinal boost of the pair, then the transverse recoil
    k = sigma_k * rng.standard_normal((n, 2))
    E_cm = np.sqrt(mtt ** 2 + np.sum(k * k, axis=1)) * np.cosh(y)
    P = np.stack([E_cm, k[:, 0], k[:, 1], np.sqrt(mtt ** 2 + np.sum(k * k, axis=1)) * np.sinh(y)], axis=1)
    parts = [_boost(v, P) for v in (b, lp, nu, bb, lm, nub)]
    b, lp, nu, bb, lm, nub = parts
    Eb = _smear(rng, b[:, 0], rel_sigma)
    Ebb = _smear(rng, bb[:, 0], rel_sigma)
    jb = _massless(Eb, b)
    jbb = _massless(Ebb, bb)
    swap = rng.random(n) < 0.5
    j0 = np.where(swap[:, None], jbb, jb)
    j1 = np.where(swap[:, None], jb, jbb)
    obs = np.stack([j0, j1, lp, lm], axis=1)
    truth = {"b": b, "bb": bb, "lp": lp, "lm": lm, "nu": nu, "nub": nub, "k": k,
             "swap": swap, "mt1": mt1, "mt2": mt2, "mw1": mw1, "mw2": mw2}
    return {"obs": obs, "truth": truth}


def ttbar_dilepton_partons(n_events, seed, sigma_k=20.0):
    """parton-level ttbar dilepton events (every transfer function a delta
    function): the generator of ttbar_dilepton without smearing; rows b-quark
    0, b-quark 1 (the b and the bbar in random order), l+, l-, nu, nubar"""
    d = ttbar_dilepton(n_events, seed, rel_sigma=0.0, sigma_k=sigma_k)
    t = d["truth"]
    swap = t["swap"][:, None]
    q0 = np.where(swap, t["bb"], t["b"])
    q1 = np.where(swap, t["b"], t["bb"])
    return {"obs": np.stack([q0, q1, t["lp"], t["lm"], t["nu"], t["nub"]], axis=1), "truth": t}


def _smear_dgauss(rng, E, core, tail, ftail):
    """E (1 + s z) with s = tail for a fraction ftail of the draws, else
    core, redrawn while non-positive"""
    out = np.empty_like(E)
    todo = np.ones(E.shape, dtype=bool)
    while np.any(todo):
        n = int(todo.sum())
        s = np.where(rng.random(n) < ftail, tail, core)
        v = E[todo] * (1.0 + s * rng.standard_normal(n))
        idx = np.flatnonzero(todo)
        ok = v > 0.0
        out[idx[ok]] = v[ok]
        todo[idx[ok]] = False
    return out


def ttbar_semileptonic(n_events, seed, rel_sigma_b=0.15, lj=(0.10, 0.25, 0.2), sigma_k=20.0):
    """pp -> t tbar with one W -> l nu and one W -> q qbar'.  Kinematics as
    in ttbar_dilepton; the lepton charge is random (+1: the top decays
    leptonically).  b-jet energies are smeared by rel_sigma_b, light-jet
    energies by a double Gaussian (core, tail, tail fraction), the lepton is
    exact, and the four jets are stored in random order.  Layout: jets
    j0..j3, lepton, then a row (charge, 0, 0, 0)."""
    rng = _rng(seed)
    n = n_events
    mt1 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mt2 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mw1 = _bw(rng, n, M_W, W_W, 65.0, 95.0)
    mw2 = _bw(rng, n, M_W, W_W, 65.0, 95.0)
    mtt = mt1 + mt2 + rng.gamma(2.0, 80.0, n)
    ymax = np.log(SQRT_S / mtt)
    y = np.clip(rng.standard_normal(n), -1.0, 1.0) * np.minimum(2.0, 0.9 * ymax)
    t, tb = _two_body(mtt, mt1, mt2, _iso(rng, n))
    b, wp = _two_body(mt1, np.zeros(n), mw1, _iso(rng, n))
    bb, wm = _two_body(mt2, np.zeros(n), mw2, _iso(rng, n))
    f1, f1b = _two_body(mw1, np.zeros(n), np.zeros(n), _iso(rng, n))   # W+ decay products
    f2, f2b = _two_body(mw2, np.zeros(n), np.zeros(n), _iso(rng, n))   # W- decay products
    f1, f1b = _boost(f1, wp), _boost(f1b, wp)
    f2, f2b = _boost(f2, wm), _boost(f2b, wm)
    b, f1, f1b = (_boost(v, t) for v in (b, f1, f1b))
    bb, f2, f2b = (_boost(v, tb) for v in (bb, f2, f2b))
    k = sigma_k * rng.standard_normal((n, 2))
    mT = np.sqrt(mtt ** 2 + np.sum(k * k, axis=1))
    P = np.stack([mT * np.cosh(y), k[:, 0], k[:, 1], mT * np.sinh(y)], axis=1)
    b, f1, f1b, bb, f2, f2b = (_boost(v, P) for v in (b, f1, f1b, bb, f2, f2b))
    charge = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    plus = charge[:, None] > 0
    # l+ : top leptonic (W+ -> l+ nu), W- -> q qbar'; l- : the reverse
    lep = np.where(plus, f1b, f2)
    nu = np.where(plus, f1, f2b)
    q1 = np.where(plus, f2, f1)
    q2 = np.where(plus, f2b, f1b)
    b_lep = np.where(plus, b, bb)
    b_had = np.where(plus, bb, b)
    jets = [_massless(_smear(rng, b_lep[:, 0], rel_sigma_b), b_lep),
            _massless(_smear(rng, b_had[:, 0], rel_sigma_b), b_had),
            _massless(_smear_dgauss(rng, q1[:, 0], *lj), q1),
            _massless(_smear_dgauss(rng, q2[:, 0], *lj), q2)]
    jets = np.stack(jets, axis=1)                     # order: b_lep, b_had, q, qbar
    order = np.argsort(rng.random((n, 4)), axis=1)    # random jet order
    obs_jets = np.take_along_axis(jets, order[:, :, None], axis=1)
    crow = np.zeros((n, 4))
    crow[:, 0] = charge
    obs = np.concatenate([obs_jets, lep[:, None, :], crow[:, None, :]], axis=1)
    pos = np.argsort(order, axis=1)                   # pos[i, parton] = jet slot
    truth = {"b_lep": b_lep, "b_had": b_had, "q": q1, "qbar": q2, "lep": lep, "nu": nu, "k": k,
             "charge": charge, "slot": pos}
    return {"obs": obs, "truth": truth}


def ttbar_higgs(n_events, seed, lj=(0.10, 0.25, 0.2), sigma_k=20.0):
    """gg -> t tbar H with H -> b bbar (narrow, 125 GeV), one W -> l nu and
    one W -> q qbar'.  The t tbar H mass rises from threshold with a
    Gamma(2, 100 GeV) excess, the t tbar subsystem mass is uniform between
    its threshold and the kinematic limit, all decays are isotropic, the
    system gets a Gaussian recoil k_T and a Gaussian rapidity; all six jet
    energies are smeared by the double Gaussian `lj`, the lepton is exact.
    The four b-jets and the two light jets are stored in random order."""
    rng = _rng(seed)
    n = n_events
    mt1 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mt2 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mw1 = _bw(rng, n, M_W, W_W, 65.0, 95.0)
    mw2 = _bw(rng, n, M_W, W_W, 65.0, 95.0)
    mh = np.full(n, M_H)
    mtth = mt1 + mt2 + mh + rng.gamma(2.0, 100.0, n)
    mtt = mt1 + mt2 + rng.random(n) * (mtth - mh - mt1 - mt2)
    ymax = np.log(SQRT_S / mtth)
    y = np.clip(rng.standard_normal(n), -1.0, 1.0) * np.minimum(2.0, 0.9 * ymax)
    tt, h = _two_body(mtth, mtt, mh, _iso(rng, n))
    t, tb = _two_body(mtt, mt1, mt2, _iso(rng, n))
    t, tb = _boost(t, tt), _boost(tb, tt)
    hb, hbb = _two_body(mh, np.zeros(n), np.zeros(n), _iso(rng, n))
    hb, hbb = _boost(hb, h), _boost(hbb, h)
    b, wp = _two_body(mt1, np.zeros(n), mw1, _iso(rng, n))
    bb, wm = _two_body(mt2, np.zeros(n), mw2, _iso(rng, n))
    f1, f1b = _two_body(mw1, np.zeros(n), np.zeros(n), _iso(rng, n))
    f2, f2b = _two_body(mw2, np.zeros(n), np.zeros(n), _iso(rng, n))
    f1, f1b = _boost(f1, wp), _boost(f1b, wp)
    f2, f2b = _boost(f2, wm), _boost(f2b, wm)
    b, f1, f1b = (_boost(v, t) for v in (b, f1, f1b))
    bb, f2, f2b = (_boost(v, tb) for v in (bb, f2, f2b))
    k = sigma_k * rng.standard_normal((n, 2))
    mT = np.sqrt(mtth ** 2 + np.sum(k * k, axis=1))
    P = np.stack([mT * np.cosh(y), k[:, 0], k[:, 1], mT * np.sinh(y)], axis=1)
    b, f1, f1b, bb, f2, f2b, hb, hbb = (_boost(v, P) for v in (b, f1, f1b, bb, f2, f2b, hb, hbb))
    charge = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    plus = charge[:, None] > 0
    lep = np.where(plus, f1b, f2)
    nu = np.where(plus, f1, f2b)
    q1 = np.where(plus, f2, f1)
    q2 = np.where(plus, f2b, f1b)
    b_lep = np.where(plus, b, bb)
    b_had = np.where(plus, bb, b)
    bjets = np.stack([_massless(_smear_dgauss(rng, v[:, 0], *lj), v) for v in (b_lep, b_had, hb, hbb)], axis=1)
    ljets = np.stack([_massless(_smear_dgauss(rng, v[:, 0], *lj), v) for v in (q1, q2)], axis=1)
    border = np.argsort(rng.random((n, 4)), axis=1)
    lorder = np.argsort(rng.random((n, 2)), axis=1)
    crow = np.zeros((n, 4))
    crow[:, 0] = charge
    obs = np.concatenate([np.take_along_axis(bjets, border[:, :, None], axis=1),
                          np.take_along_axis(ljets, lorder[:, :, None], axis=1),
                          lep[:, None, :], crow[:, None, :]], axis=1)
    truth = {"b_lep": b_lep, "b_had": b_had, "hb": hb, "hbb": hbb, "q": q1, "qbar": q2, "lep": lep, "nu": nu,
             "k": k, "charge": charge, "bslot": np.argsort(border, axis=1), "lslot": np.argsort(lorder, axis=1)}
    return {"obs": obs, "truth": truth}


def _dilepton_tops(rng, n, t, tb, mt1, mt2):
    """b l+ nu from the top and bbar l- nubar from the antitop, isotropic
    decays with Breit-Wigner W masses, in the frame of t and tb"""
    mw1 = _bw(rng, n, M_W, W_W, 65.0, 95.0)
    mw2 = _bw(rng, n, M_W, W_W, 65.0, 95.0)
    b, wp = _two_body(mt1, np.zeros(n), mw1, _iso(rng, n))
    bb, wm = _two_body(mt2, np.zeros(n), mw2, _iso(rng, n))
    lp, nu = _two_body(mw1, np.zeros(n), np.zeros(n), _iso(rng, n))
    lm, nub = _two_body(mw2, np.zeros(n), np.zeros(n), _iso(rng, n))
    lp, nu = _boost(lp, wp), _boost(nu, wp)
    lm, nub = _boost(lm, wm), _boost(nub, wm)
    b, lp, nu = (_boost(v, t) for v in (b, lp, nu))
    bb, lm, nub = (_boost(v, tb) for v in (bb, lm, nub))
    return b, lp, nu, bb, lm, nub


def _four_b_dilepton(rng, n, M, y, parts, rel_sigma):
    """boost the hard system (mass M, rapidity y, no transverse recoil) to
    the lab, smear the four b energies, store the b-jets in random order"""
    P = np.stack([M * np.cosh(y), np.zeros(n), np.zeros(n), M * np.sinh(y)], axis=1)
    b, lp, nu, bb, lm, nub, p1, p2 = (_boost(v, P) for v in parts)
    quarks = (b, bb, p1, p2)
    jets = np.stack([_massless(_smear(rng, v[:, 0], rel_sigma), v) for v in quarks], axis=1)
    order = np.argsort(rng.random((n, 4)), axis=1)
    obs = np.concatenate([np.take_along_axis(jets, order[:, :, None], axis=1), lp[:, None, :], lm[:, None, :]], axis=1)
    truth = {"b": b, "bb": bb, "p1": p1, "p2": p2, "lp": lp, "lm": lm, "nu": nu, "nub": nub,
             "slot": np.argsort(order, axis=1)}
    return {"obs": obs, "truth": truth}


def ttbar_higgs_dilepton(n_events, seed, rel_sigma=0.15):
    """gg -> t tbar H, H -> b bbar (125 GeV, narrow), both tops to b l nu
    (Sec. 4's signal).  Masses and decays as ttbar_higgs, no transverse
    recoil (the hard system's transverse momentum is zero, as the
    integrand's transverse momentum balance assumes); the four b-jet
    energies are smeared by the Gaussian rel_sigma, the leptons are exact.
    truth slot[:, q] is the jet row of quark q in (b, bbar, b of H, bbar of H)."""
    rng = _rng(seed)
    n = n_events
    mt1 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mt2 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mh = np.full(n, M_H)
    M = mt1 + mt2 + mh + rng.gamma(2.0, 100.0, n)
    mtt = mt1 + mt2 + rng.random(n) * (M - mh - mt1 - mt2)
    y = np.clip(rng.standard_normal(n), -1.0, 1.0) * np.minimum(2.0, 0.9 * np.log(SQRT_S / M))
    tt, h = _two_body(M, mtt, mh, _iso(rng, n))
    t, tb = _two_body(mtt, mt1, mt2, _iso(rng, n))
    t, tb = _boost(t, tt), _boost(tb, tt)
    hb, hbb = _two_body(mh, np.zeros(n), np.zeros(n), _iso(rng, n))
    hb, hbb = _boost(hb, h), _boost(hbb, h)
    parts = _dilepton_tops(rng, n, t, tb, mt1, mt2) + (hb, hbb)
    return _four_b_dilepton(rng, n, M, y, parts, rel_sigma)


def ttbar_bbbar_dilepton(n_events, seed, rel_sigma=0.15):
    """gg -> t tbar b bbar with both tops to b l nu (Sec. 4's background):
    the extra b bbar pair has a mass 20 GeV + Gamma(1.5, 60 GeV), the t tbar
    b bbar mass rises from threshold with a Gamma(2, 120 GeV) excess and the
    t tbar mass is uniform in between; decays isotropic, no recoil, jets as
    ttbar_higgs_dilepton (slot order b, bbar, b', bbar')."""
    rng = _rng(seed)
    n = n_events
    mt1 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mt2 = _bw(rng, n, M_T, W_T, 160.0, 185.0)
    mbb = 20.0 + rng.gamma(1.5, 60.0, n)
    M = mt1 + mt2 + mbb + rng.gamma(2.0, 120.0, n)
    mtt = mt1 + mt2 + rng.random(n) * (M - mbb - mt1 - mt2)
    y = np.clip(rng.standard_normal(n), -1.0, 1.0) * np.minimum(2.0, 0.9 * np.log(SQRT_S / M))
    tt, g = _two_body(M, mtt, mbb, _iso(rng, n))
    t, tb = _two_body(mtt, mt1, mt2, _iso(rng, n))
    t, tb = _boost(t, tt), _boost(tb, tt)
    p1, p2 = _two_body(mbb, np.zeros(n), np.zeros(n), _iso(rng, n))
    p1, p2 = _boost(p1, g), _boost(p2, g)
    parts = _dilepton_tops(rng, n, t, tb, mt1, mt2) + (p1, p2)
    return _four_b_dilepton(rng, n, M, y, parts, rel_sigma)


def four_b_partons(d, seed):
    """parton-level events from a four-b dilepton sample's truth: the four
    b quarks in random order, then l+, l-, nu, nubar (exact momenta)"""
    t = d["truth"]
    rng = _rng(seed)
    quarks = np.stack([t["b"], t["bb"], t["p1"], t["p2"]], axis=1)
    order = np.argsort(rng.random((quarks.shape[0], 4)), axis=1)
    rest = np.stack([t["lp"], t["lm"], t["nu"], t["nub"]], axis=1)
    return np.concatenate([np.take_along_axis(quarks, order[:, :, None], axis=1), rest], axis=1)


def budgets(n_events, seed, lo=16384, hi=262144):
    """per-event point budgets drawn uniformly from [lo, hi)"""
    rng = _rng(seed)
    return (lo + np.floor(rng.random(n_events) * (hi - lo))).astype(np.int64)
