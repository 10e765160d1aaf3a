"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: a
library routine (rocRAND's Philox), textbook closed forms (Ellis-Stirling-
Webber heavy-quark production, the V-A decay spin sum, e+e- -> mu+mu-),
gauge invariance, symmetries, exact integrals and brute-force quadrature.
"""
import ctypes
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from synth import events

HERE = os.path.dirname(os.path.abspath(__file__))


def mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


# ----------------------------------------------------------------- RNG ----
@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(tmp_path):
    """Philox4x32-10 equals rocRAND's engine word for word (host run)."""
    exe = tmp_path / "philox_ref"
    subprocess.run(["hipcc", "-O1", os.path.join(HERE, "golden", "rocrand_philox_ref.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    rng = np.random.default_rng(5)
    rows = []
    for _ in range(200):
        rows.append((int(rng.integers(0, 2**63)), int(rng.integers(0, 2**32)),
                     int(rng.integers(0, 64)), int(rng.integers(0, 2**20)), int(rng.integers(0, 400))))
    rows.append((0, 0, 0, 0, 0))
    # the reference maps the counter through a 64-bit offset 4*(k | iter<<32),
    # so iter stays below 2^30 there
    rows.append((2**64 - 1, 2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1))
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    for r, want in zip(rows, ref):
        seed, k, it, ev, sub = r
        got = oracle.philox([k, it, ev, sub], [seed & 0xFFFFFFFF, seed >> 32])
        assert np.array_equal(got.astype(np.uint64), want), r


def test_uniforms_are_53bit_and_uniform():
    u = np.array([oracle.uniforms(7, k, 0, 3, 0, 2) for k in range(20000)]).ravel()
    assert np.all(u >= 0.0) and np.all(u < 1.0)
    scaled = u * 2.0**53
    assert np.all(scaled == np.floor(scaled))
    hist, _ = np.histogram(u, bins=50, range=(0, 1))
    expect = len(u) / 50
    chi2 = np.sum((hist - expect) ** 2 / expect)
    assert chi2 < 100.0  # 49 dof, p ~ 1e-5
    from scipy import stats
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_uniforms_word_layout():
    """dims (2b, 2b+1) come from words (0,1) and (2,3) of counter block b"""
    seed = 0x1407759512345
    u = oracle.uniforms(seed, 11, 2, 5, 1, 5)
    for b in range(3):
        w = oracle.philox([11, 2, 5, 16 + b], [seed & 0xFFFFFFFF, seed >> 32]).astype(np.uint64)
        hi = int((w[0] << np.uint64(32)) | w[1]) >> 11
        assert u[2 * b] == hi * 2.0**-53
        if 2 * b + 1 < 5:
            lo = int((w[2] << np.uint64(32)) | w[3]) >> 11
            assert u[2 * b + 1] == lo * 2.0**-53


def test_uniforms_block_offset():
    """the counter-block offset addresses the same stream: blocks 16.. of
    permutation p are blocks 0.. of permutation p + 1, and blocks 8.. are
    disjoint from both"""
    seed = 0x1407759577
    for k, it, ev, perm in ((0, 0, 0, 0), (123, 4, 9, 3), (2**31, 7, 2**20, 5)):
        a = oracle.uniforms(seed, k, it, ev, perm, 8, block0=16)
        b = oracle.uniforms(seed, k, it, ev, perm + 1, 8)
        assert np.array_equal(a, b)
        z = oracle.uniforms(seed, k, it, ev, perm, 8, block0=8)
        assert not np.any(np.isin(z, oracle.uniforms(seed, k, it, ev, perm, 8)))


# --------------------------------------------------------------- VEGAS ----
def test_uniform_grid_map_is_identity():
    g = oracle.uniform_grid(3)
    rng = np.random.default_rng(1)
    for _ in range(100):
        u = np.floor(rng.random(3) * 2**53) * 2.0**-53
        x, jac, bins = oracle.vegas_map(g, u)
        assert np.all(x == u) and jac == 1.0
        assert np.all(bins == np.floor(u * 64))


def test_map_monotone_and_jacobian():
    rng = np.random.default_rng(2)
    edges = np.concatenate([[0.0], np.sort(rng.random(63)), [1.0]])
    g = edges[None, :]
    us = np.sort(rng.random(2000))
    xs = [oracle.vegas_map(g, [u])[0][0] for u in us]
    assert np.all(np.diff(xs) >= 0)
    for u in us[:50]:
        x, jac, b = oracle.vegas_map(g, [u])
        i = int(u * 64)
        assert edges[i] <= x[0] <= edges[i + 1]
        assert jac == 64 * (edges[i + 1] - edges[i])


def test_refine_flat_keeps_uniform_and_peak_concentrates():
    e = np.linspace(0, 1, 65)
    assert np.allclose(oracle.refine_dim(np.ones(64), 1.5, e), e, atol=1e-15)
    d = np.zeros(64)
    d[20] = 1.0
    new = oracle.refine_dim(d, 1.5, e)
    assert new[0] == 0.0 and new[64] == 1.0
    assert np.all(np.diff(new) > 0)
    # smoothing spreads bin 20 over 19..21; those bins take most new bins
    inside = np.sum((new[1:] <= e[22]) & (new[:-1] >= e[19]))
    assert inside > 40
    zero = oracle.refine_dim(np.zeros(64), 1.5, e)
    assert np.array_equal(zero, e)


def test_refine_matches_damped_rebinning_by_hand():
    """one refinement step checked against the written-out Lepage rule"""
    rng = np.random.default_rng(3)
    d = rng.random(64) ** 3
    e = np.concatenate([[0.0], np.sort(rng.random(63)), [1.0]])
    s = np.empty(64)
    s[0] = (d[0] + d[1]) / 2
    s[1:-1] = (d[:-2] + d[1:-1] + d[2:]) / 3
    s[-1] = (d[-2] + d[-1]) / 2
    rho = s / s.sum()
    m = ((1 - rho) / np.log(1 / rho)) ** 1.5
    cum = np.concatenate([[0.0], np.cumsum(m)])
    targets = cum[-1] * np.arange(1, 64) / 64
    # inverse of the piecewise-linear cumulative importance
    want = np.interp(targets, cum, e)
    got = oracle.refine_dim(d, 1.5, e)
    assert np.allclose(got[1:64], want, rtol=0, atol=1e-13)


def test_refine_converges_to_inverse_cdf():
    """Iterated refinement on a separable product peak prod_d g_d(x_d),
    g_d = a / (1 + a^2 (x - c_d)^2): each bin of the adapted grid ends up
    holding an equal share of int |g_d| (the map's density follows |g_d|),
    so the edges approach the inverse CDF
        G_d^-1(k/64) = c_d + tan(k/64 (atan(a (1 - c_d)) + atan(a c_d)) - atan(a c_d)) / a,
    to a fraction of the local bin width, and the weights' spread falls by
    two orders of magnitude.  Lepage's damping only sets how fast the grid
    gets there; a rule that misplaced the new edges (interpolation inside
    the old bins, the cumulative importance, the smoothing's indices) ends
    elsewhere."""
    p = oracle.dy_params()
    g0 = oracle.uniform_grid(4)
    r, Is, Vs, g = oracle.integrate_one(oracle.KIND_GENZ, p, np.zeros(4), 0, 7, 0, 200000, 15, grid=g0)
    a = 20.0
    k = np.arange(65) / 64
    for d in range(4):
        c = 0.3 + 0.1 * d
        tot = math.atan(a * (1 - c)) + math.atan(a * c)
        inv = c + np.tan(k * tot - math.atan(a * c)) / a
        w = np.diff(inv)
        local = np.concatenate([[w[0]], np.minimum(w[:-1], w[1:]), [w[-1]]])
        dev = np.abs(g[d] - inv) / local
        assert dev.max() < 0.3, (d, dev.max())
    rel = np.sqrt(Vs) / Is
    assert rel[-1] < 0.02 * rel[0], rel


def test_vegas_genz_product_peak():
    """VEGAS on a separable product peak: estimate within 3 sigma of the
    exact integral, and the adapted error far below plain MC."""
    exact = oracle.lib().or_genz_exact()
    p = oracle.dy_params()
    r, Is, Vs, _ = oracle.integrate_one(oracle.KIND_GENZ, p, np.zeros(4), 0, 99, 0, 20000, 8)
    pull = (r.I - exact) / r.sigma
    assert abs(pull) < 3.0, (r.I, exact, r.sigma)
    assert r.sigma / exact < 0.2 * math.sqrt(Vs[0]) / exact


def test_vegas_pull_distribution_genz():
    exact = oracle.lib().or_genz_exact()
    p = oracle.dy_params()
    pulls = []
    for seed in range(30):
        r, _, _, _ = oracle.integrate_one(oracle.KIND_GENZ, p, np.zeros(4), 0, 1000 + seed, 0, 4000, 6)
        pulls.append((r.I - exact) / r.sigma)
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 0.6 and 0.5 < pulls.std() < 1.6


# ------------------------------------------------- stratified VEGAS ----
def test_strat_hypercubes_and_allocation():
    """n_s is the largest count with 2 n_s^D <= N (and H within the cap);
    every allocation uses exactly N points, at least 2 per hypercube; after
    the first iteration the points beyond 2 per hypercube follow
    sigma^0.75 (to rounding)"""
    assert oracle.strat_ns(2, 4096) == 45 and oracle.strat_ns(8, 32768) == 3 and oracle.strat_ns(8, 511) == 1
    assert oracle.strat_ns(2, 31) == 3 and oracle.strat_ns(2, 32) == 4
    assert oracle.strat_ns(2, 10 ** 9) ** 2 <= oracle.STRAT_HMAX
    nh = oracle.strat_allocate(16, 100, first=True)
    assert nh.sum() == 100 and list(nh[:4]) == [7, 7, 7, 7] and nh[4] == 6
    rng = np.random.default_rng(8)
    sig = rng.random(81) ** 3
    sig[5] = 0.0
    nh = oracle.strat_allocate(81, 5000, sig)
    assert nh.sum() == 5000 and nh.min() >= 2 and nh[5] <= 3
    share = sig ** 0.75 / np.sum(sig ** 0.75) * (5000 - 2 * 81)
    assert np.all(np.abs((nh - 2) - share) <= 2.0)
    # every deviation zero: the equal split
    assert np.array_equal(oracle.strat_allocate(81, 5000, np.zeros(81)), oracle.strat_allocate(81, 5000, first=True))


def test_strat_exact_on_aligned_steps():
    """a function constant on the hypercubes (1 + floor(4 x0) + 3 floor(4 x1),
    n_s = 4 for N in [32, 50)) is integrated exactly with zero variance;
    with n_s = 2 the steps inside a hypercube give a positive variance
    that is the textbook stratified one, (1/H^2) sum s_h^2 / n_h"""
    p = oracle.dy_params()
    g = oracle.uniform_grid(2)
    for N in (32, 40, 49):
        ns = oracle.strat_ns(2, N)
        assert ns == 4
        nh = oracle.strat_allocate(16, N, first=True)
        I, var, sig, bins, w = oracle.strat_iteration(oracle.KIND_STEP, p, np.zeros(2), 0, 3, 0, 0, N, g, ns, nh)
        assert I == pytest.approx(7.0, rel=1e-14) and var == 0.0 and np.all(sig == 0.0)
    N = 16
    ns = oracle.strat_ns(2, N)
    assert ns == 2
    nh = oracle.strat_allocate(4, N, first=True)
    I, var, sig, bins, w = oracle.strat_iteration(oracle.KIND_STEP, p, np.zeros(2), 0, 3, 0, 0, N, g, ns, nh)
    # hypercube h holds points [4h, 4h + 4) in iteration order
    want_var = sum(np.var(w[4 * h:4 * h + 4], ddof=1) / 4 for h in range(4)) / 16
    assert var == pytest.approx(want_var, rel=1e-12)
    assert I == pytest.approx(np.mean(w), rel=1e-12)


def test_strat_vegas_genz_and_pulls():
    """stratified VEGAS on the Genz product peak: the estimate within 3
    sigma of the exact integral, the second iteration's error below plain
    VEGAS's on the same budget, and a 30-seed pull distribution"""
    exact = oracle.lib().or_genz_exact()
    p = oracle.dy_params()
    r, Is, Vs = oracle.integrate_one_strat(oracle.KIND_GENZ, p, np.zeros(4), 0, 99, 0, 20000, 8)
    assert abs(r.I - exact) < 3 * r.sigma
    _, Is2, Vs2, _ = oracle.integrate_one(oracle.KIND_GENZ, p, np.zeros(4), 0, 99, 0, 20000, 8)
    assert math.sqrt(Vs[1]) / Is[1] < 0.6 * math.sqrt(Vs2[1]) / Is2[1]
    pulls = []
    for seed in range(30):
        r, _, _ = oracle.integrate_one_strat(oracle.KIND_GENZ, p, np.zeros(4), 0, 2000 + seed, 0, 4000, 6)
        pulls.append((r.I - exact) / r.sigma)
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 0.6 and 0.5 < pulls.std() < 1.6


# ------------------------------------------------------------- physics ----
def _on_shell_tt(rng, mt, rs):
    k1 = np.array([rs / 2, 0, 0, rs / 2])
    k2 = np.array([rs / 2, 0, 0, -rs / 2])
    p = math.sqrt(rs * rs / 4 - mt * mt)
    c = 2 * rng.random() - 1
    ph = 2 * math.pi * rng.random()
    sn = math.sqrt(1 - c * c)
    pt = np.array([rs / 2, p * sn * math.cos(ph), p * sn * math.sin(ph), p * c])
    ptb = np.array([rs / 2, -pt[1], -pt[2], -pt[3]])
    return k1, k2, pt, ptb


def test_heavy_quark_production_closed_forms():
    """gg -> QQbar and qqbar -> QQbar spin/colour averaged |M|^2 / g^4
    (Ellis-Stirling-Webber, tau_i = 2 p_i.p_3 / s, rho = 4 m^2 / s)"""
    rng = np.random.default_rng(4)
    mt = 172.5
    for _ in range(20):
        rs = 2 * mt + 2000 * rng.random()
        k1, k2, pt, ptb = _on_shell_tt(rng, mt, rs)
        s = rs * rs
        t1, t2, rho = 2 * mdot(k1, pt) / s, 2 * mdot(k2, pt) / s, 4 * mt * mt / s
        gg = (1 / (6 * t1 * t2) - 3 / 8) * (t1 * t1 + t2 * t2 + rho - rho * rho / (4 * t1 * t2))
        qq = 4 / 9 * (t1 * t1 + t2 * t2 + rho / 2)
        assert oracle.call4("or_gg_ttbar_prod", mt, k1, k2, pt, ptb) == pytest.approx(gg, rel=1e-12)
        assert oracle.call4("or_qq_ttbar_prod", mt, k1, k2, pt, ptb) == pytest.approx(qq, rel=1e-12)


def test_gg_ward_identity():
    rng = np.random.default_rng(5)
    for _ in range(10):
        k1, k2, pt, ptb = _on_shell_tt(rng, 172.5, 400 + 1000 * rng.random())
        assert oracle.call4("or_gg_ttbar_ward", 172.5, k1, k2, pt, ptb) < 1e-10


def _massless(rng, scale=60.0):
    v = rng.normal(size=3) * scale
    return np.array([np.linalg.norm(v), *v])


def test_top_decay_spin_sum():
    """sum over spins of |ubar(b) J P_L u(t)|^2 = 16 (t.l)(b.nu) (V-A)"""
    rng = np.random.default_rng(6)
    for _ in range(10):
        b, lp, nu = _massless(rng), _massless(rng), _massless(rng)
        pt = b + lp + nu
        m = math.sqrt(mdot(pt, pt))
        v = oracle.call4("or_top_decay_spinsum", m, pt, b, lp, nu)
        assert v == pytest.approx(16 * mdot(pt, lp) * mdot(b, nu), rel=1e-12)


def test_qq_mumu_me_and_cross_section():
    """|M|^2 = (4 pi alpha)^2 Q^2 (1 + cos^2)/3 and, by exact quadrature
    over dPhi_2 = dOmega / (32 pi^2), sigma(e+e- -> mu+mu-) = 4 pi alpha^2/(3s)"""
    a = 1 / 137.0
    rs = 91.0
    s = rs * rs
    p1 = np.array([rs / 2, 0, 0, rs / 2])
    p2 = np.array([rs / 2, 0, 0, -rs / 2])
    xs, ws = np.polynomial.legendre.leggauss(6)
    sig = 0.0
    L = oracle.lib()
    for c, w in zip(xs, ws):
        sn = math.sqrt(1 - c * c)
        p3 = np.array([rs / 2, rs / 2 * sn * 0.6, rs / 2 * sn * 0.8, rs / 2 * c])
        p4 = np.array([rs / 2, -p3[1], -p3[2], -p3[3]])
        args = [np.ascontiguousarray(v) for v in (p1, p2, p3, p4)]
        me = L.or_qq_mumu_me2(*[oracle._ptr(v) for v in args], 1.0, a) * 3.0  # undo colour avg
        assert me == pytest.approx((4 * math.pi * a) ** 2 * (1 + c * c), rel=1e-12)
        sig += w * 2 * math.pi * me / (32 * math.pi**2) / (2 * s)
    assert sig == pytest.approx(4 * math.pi * a * a / (3 * s), rel=1e-12)


def _tt_point(rng):
    """random 2->6 kinematics with gluons along the beam"""
    parts = [_massless(rng, 70.0) for _ in range(6)]
    P = sum(parts)
    # transverse boost to zero pT, then read x1, x2 from E +- pz
    bx, by = P[1] / P[0], P[2] / P[0]
    b2 = bx * bx + by * by
    g = 1 / math.sqrt(1 - b2)
    out = []
    for v in parts:
        bp = bx * v[1] + by * v[2]
        g2 = (g - 1) / b2
        out.append(np.array([g * (v[0] - bp), v[1] + g2 * bp * bx - g * bx * v[0],
                             v[2] + g2 * bp * by - g * by * v[0], v[3]]))
    P = sum(out)
    k1 = np.array([(P[0] + P[3]) / 2, 0, 0, (P[0] + P[3]) / 2])
    k2 = np.array([(P[0] - P[3]) / 2, 0, 0, -(P[0] - P[3]) / 2])
    return k1, k2, np.concatenate(out)


def _zboost(v, eta):
    ch, sh = math.cosh(eta), math.sinh(eta)
    return np.array([ch * v[0] + sh * v[3], v[1], v[2], sh * v[0] + ch * v[3]])


def _zrot(v, a):
    c, s = math.cos(a), math.sin(a)
    return np.array([v[0], c * v[1] - s * v[2], s * v[1] + c * v[2], v[3]])


def test_full_me_invariance_and_cp():
    """the 2->6 |M|^2 is unchanged by boosts along and rotations about the
    beam, and by CP (particles <-> antiparticles, momenta reflected, the
    two beams exchanged)"""
    p = oracle.tt_params()
    rng = np.random.default_rng(7)
    for _ in range(5):
        k1, k2, mom = _tt_point(rng)
        m6 = mom.reshape(6, 4)
        gg = oracle.call4("or_tt_me2_gg", p, k1, k2, mom)
        qq = oracle.call4("or_tt_me2_qq", p, k1, k2, mom)
        assert gg > 0 and qq > 0
        eta, ang = rng.normal(), rng.random() * 6.28
        tr = lambda v: _zrot(_zboost(v, eta), ang)
        mom2 = np.concatenate([tr(v) for v in m6])
        assert oracle.call4("or_tt_me2_gg", p, tr(k1), tr(k2), mom2) == pytest.approx(gg, rel=1e-9)
        assert oracle.call4("or_tt_me2_qq", p, tr(k1), tr(k2), mom2) == pytest.approx(qq, rel=1e-9)
        par = lambda v: np.array([v[0], -v[1], -v[2], -v[3]])
        b, lp, nu, bb, lm, nub = m6
        cp = np.concatenate([par(v) for v in (bb, lm, nub, b, lp, nu)])
        assert oracle.call4("or_tt_me2_gg", p, par(k2), par(k1), cp) == pytest.approx(gg, rel=1e-9)
        # qqbar: the quark becomes an antiquark; the beam it came from is reflected
        assert oracle.call4("or_tt_me2_qq", p, par(k2), par(k1), cp) == pytest.approx(qq, rel=1e-9)


def test_dilepton_solutions_round_trip():
    """the generator's true (nu, nubar) is among the solutions of
    Eq. dilepsolv for its own propagator virtualities and MET"""
    d = events.ttbar_dilepton(40, 21)
    t = d["truth"]
    for i in range(40):
        b, bb, lp, lm, nu, nub = (t[k][i] for k in ("b", "bb", "lp", "lm", "nu", "nub"))
        q2 = oracle.dilepton_q2(b, bb, lp, lm, nu, nub)
        met = nu[1:3] + nub[1:3]
        sols, solsb, det = oracle.solve_dilepton(b, bb, lp, lm, met, q2)
        assert len(sols) in (2, 4) or len(sols) >= 1
        err = [max(np.max(np.abs(s - nu)), np.max(np.abs(sb - nub))) / nu[0] for s, sb in zip(sols, solsb)]
        assert min(err) < 1e-9
        for s, sb in zip(sols, solsb):
            assert np.allclose(oracle.dilepton_q2(b, bb, lp, lm, s, sb), q2, rtol=1e-9)


def test_dilepton_jacobian_finite_difference():
    d = events.ttbar_dilepton(10, 22)
    t = d["truth"]
    for i in range(10):
        b, bb, lp, lm, nu, nub = (t[k][i] for k in ("b", "bb", "lp", "lm", "nu", "nub"))
        q2 = oracle.dilepton_q2(b, bb, lp, lm, nu, nub)
        met = nu[1:3] + nub[1:3]
        sols, solsb, det = oracle.solve_dilepton(b, bb, lp, lm, met, q2)
        for s, sb, dj in zip(sols, solsb, det):
            v0 = np.array([s[1], s[2], s[3], sb[3]])

            def F(v):
                n = np.array([0, v[0], v[1], v[2]])
                n[0] = np.linalg.norm(n[1:])
                m = np.array([0, met[0] - v[0], met[1] - v[1], v[3]])
                m[0] = np.linalg.norm(m[1:])
                return oracle.dilepton_q2(b, bb, lp, lm, n, m)

            J = np.zeros((4, 4))
            for j in range(4):
                h = 1e-4 * max(1.0, abs(v0[j]))
                e = np.zeros(4)
                e[j] = h
                J[:, j] = (F(v0 + e) - F(v0 - e)) / (2 * h)
            assert np.linalg.det(J) == pytest.approx(dj, rel=1e-5)


def test_bw_map_and_tf_normalisation():
    """Jacobian x Breit-Wigner is the constant (theta1-theta0)/(M Gamma), and
    the Gaussian TF integrates to one over the measured energy"""
    L = oracle.lib()
    m, w, lo, hi = 172.5, 1.4, 0.0, 13000.0**2
    t0, t1 = math.atan((lo - m * m) / (m * w)), math.atan((hi - m * m) / (m * w))
    for x in np.linspace(0.01, 0.99, 13):
        q2 = ctypes.c_double()
        jac = L.or_bw_map(float(x), m, w, lo, hi, ctypes.byref(q2))
        bw = 1.0 / ((q2.value - m * m) ** 2 + m * m * w * w)
        assert jac * bw == pytest.approx((t1 - t0) / (m * w), rel=1e-9)
    from scipy import integrate
    for truth, sig in ((50.0, 0.15), (300.0, 0.05)):
        val, _ = integrate.quad(lambda e: L.or_gauss_tf(e, truth, sig), truth * (1 - 12 * sig), truth * (1 + 12 * sig), epsabs=0, epsrel=1e-12)
        assert val == pytest.approx(1.0, abs=1e-10)


def test_dy_sigma_two_ways():
    p = oracle.dy_params()
    L = oracle.lib()
    a = L.or_dy_sigma_2d(ctypes.byref(p), 300)
    b = L.or_dy_sigma_tau(ctypes.byref(p), 300)
    assert a == pytest.approx(b, rel=1e-10)
    assert a > 0


def _dy_quadrature(p, ev, n=400):
    """brute-force tensor Gauss-Legendre over the 2D unit square (the
    integrand has a hard mass window, so use many nodes)"""
    xs, ws = np.polynomial.legendre.leggauss(n)
    xs = 0.5 * (xs + 1)
    ws = 0.5 * ws
    tot = 0.0
    for x0, w0 in zip(xs, ws):
        for x1, w1 in zip(xs, ws):
            tot += w0 * w1 * oracle.dy_integrand(p, ev, [x0, x1])
    return tot


def test_dy_vegas_vs_quadrature():
    """VEGAS estimate of the Drell-Yan integral within 3 sigma of brute-force
    quadrature (pins the VEGAS driver on the real integrand)"""
    p = oracle.dy_params()
    d = events.drell_yan(3, 31)
    for i in range(3):
        ev = d["obs"][i]
        q = _dy_quadrature(p, ev, 300)
        r, _, _, _ = oracle.integrate_one(oracle.KIND_DY, p, ev, 0, 5, i, 4096, 10)
        assert abs(r.I - q) < 3.5 * r.sigma + 1e-3 * q, (r.I, q, r.sigma)


def tt_truth_x(p, obs, tr, i):
    """invert the tt map at the generator's truth: r windows, BW tan maps and
    the Box-Muller recoil map"""
    S = p.sqrt_s ** 2
    b, bb = tr["b"][i], tr["bb"][i]
    jb, jbb = (obs[1], obs[0]) if tr["swap"][i] else (obs[0], obs[1])
    perm = 1 if tr["swap"][i] else 0
    x = np.zeros(8)
    x[0] = (jb[0] / b[0] - p.r_lo) / (p.r_hi - p.r_lo)
    x[1] = (jbb[0] / bb[0] - p.r_lo) / (p.r_hi - p.r_lo)
    q2 = oracle.dilepton_q2(b, bb, tr["lp"][i], tr["lm"][i], tr["nu"][i], tr["nub"][i])
    for j, (q, m, w) in enumerate(((q2[1], p.m_t, p.w_t), (q2[3], p.m_t, p.w_t),
                                   (q2[0], p.m_w, p.w_w), (q2[2], p.m_w, p.w_w))):
        t0, t1 = math.atan((0 - m * m) / (m * w)), math.atan((S - m * m) / (m * w))
        x[2 + j] = (math.atan((q - m * m) / (m * w)) - t0) / (t1 - t0)
    k = tr["k"][i]
    x[6] = 1 - math.exp(-(k @ k) / (2 * p.sigma_k ** 2))
    x[7] = (math.atan2(k[1], k[0]) / (2 * math.pi)) % 1.0
    return x, perm


def test_tt_integrand_positive_at_truth():
    """at the truth point the map reproduces the event and one neutrino
    solution exists; elsewhere the integrand is finite and non-negative"""
    p = oracle.tt_params()
    d = events.ttbar_dilepton(8, 41)
    rng = np.random.default_rng(9)
    for i in range(8):
        ev = d["obs"][i]
        x, perm = tt_truth_x(p, ev, d["truth"], i)
        v, ns = oracle.tt_integrand(p, ev, perm, x)
        assert ns >= 1 and v > 0
        vals = np.array([oracle.tt_integrand(p, ev, rng.integers(2), rng.random(8))[0] for _ in range(100)])
        assert np.all(np.isfinite(vals)) and np.all(vals >= 0)


# ------------------------------------------------------ semileptonic ----
def test_semilep_permutations_cover_assignments():
    seen = set()
    for perm in range(12):
        bl, bh, ja, jb = oracle.sl_perm(perm)
        assert len({bl, bh, ja, jb}) == 4 and ja < jb
        seen.add((bl, bh))
    assert len(seen) == 12


def test_semilep_map_jacobian_finite_difference():
    """|d(E_a, E_b, E_bh, E_bl)/d(x0..x3)| of the jet-energy map by central
    differences"""
    p = oracle.sl_params()
    d = events.ttbar_semileptonic(6, 51)
    rng = np.random.default_rng(4)
    checked = 0
    for e in range(6):
        for _ in range(40):
            perm = int(rng.integers(12))
            x = 0.05 + 0.9 * rng.random(7)
            jac, E = oracle.sl_map(p, d["obs"][e], perm, x)
            if jac == 0.0:
                continue
            J = np.zeros((4, 4))
            ok = True
            for j in range(4):
                h = 1e-6
                xp, xm = x.copy(), x.copy()
                xp[j] += h
                xm[j] -= h
                jp, Ep = oracle.sl_map(p, d["obs"][e], perm, xp)
                jm, Em = oracle.sl_map(p, d["obs"][e], perm, xm)
                if jp == 0.0 or jm == 0.0:
                    ok = False
                    break
                J[:, j] = (Ep - Em) / (2 * h)
            if not ok:
                continue
            assert abs(np.linalg.det(J)) == pytest.approx(jac, rel=1e-5)
            checked += 1
    assert checked > 20


def test_semilep_nu_z_roots():
    """the generator's nu_z is a root of the leptonic W constraint, both
    roots satisfy 2 l.nu = q2, and they agree with numpy's roots of the
    squared quadratic"""
    d = events.ttbar_semileptonic(30, 52)
    t = d["truth"]
    for i in range(30):
        l, nu = t["lep"][i], t["nu"][i]
        q2 = 2 * mdot(l, nu)
        nz = oracle.sl_nu_z(l, nu[1], nu[2], q2)
        assert len(nz) == 2
        assert min(abs(nz - nu[3])) < 1e-9 * nu[0]
        for z in nz:
            n4 = np.array([math.sqrt(nu[1] ** 2 + nu[2] ** 2 + z * z), nu[1], nu[2], z])
            assert 2 * mdot(l, n4) == pytest.approx(q2, rel=1e-10)
        a = 0.5 * q2 + l[1] * nu[1] + l[2] * nu[2]
        lt2 = l[1] ** 2 + l[2] ** 2
        ref = np.roots([lt2, -2 * a * l[3], l[0] ** 2 * (nu[1] ** 2 + nu[2] ** 2) - a * a])
        assert np.allclose(np.sort(nz), np.sort(ref.real), rtol=1e-8)


def test_double_gaussian_tf_normalisation():
    from scipy import integrate
    L = oracle.lib()
    for truth in (40.0, 250.0):
        val, _ = integrate.quad(lambda e: L.or_dgauss_tf(e, truth, 0.10, 0.25, 0.2), truth * (1 - 4), truth * (1 + 4),
                                epsabs=0, epsrel=1e-12, limit=200)
        assert val == pytest.approx(1.0, abs=1e-9)


def sl_truth_x(p, obs, tr, i):
    """invert the semileptonic map at the generator's truth"""
    S = p.sqrt_s ** 2
    slot = tr["slot"][i]                       # parton -> jet slot: b_lep, b_had, q, qbar
    bl, bh = int(slot[0]), int(slot[1])
    perm = [k for k in range(12) if oracle.sl_perm(k)[:2] == (bl, bh)][0]
    _, _, ja, jb = oracle.sl_perm(perm)
    part = {int(slot[2]): tr["q"][i], int(slot[3]): tr["qbar"][i]}
    qa, qb = part[ja], part[jb]
    x = np.zeros(7)
    x[0] = (obs[ja][0] / qa[0] - p.lj_r_lo) / (p.lj_r_hi - p.lj_r_lo)

    def inv_bw(q, m, w):
        t0, t1 = math.atan((0 - m * m) / (m * w)), math.atan((S - m * m) / (m * w))
        return (math.atan((q - m * m) / (m * w)) - t0) / (t1 - t0)

    W = qa + qb
    x[1] = inv_bw(mdot(W, W), p.m_w, p.w_w)
    T = W + tr["b_had"][i]
    x[2] = inv_bw(mdot(T, T), p.m_t, p.w_t)
    x[3] = (obs[bl][0] / tr["b_lep"][i][0] - p.r_lo) / (p.r_hi - p.r_lo)
    k = tr["k"][i]
    x[4] = 1 - math.exp(-(k @ k) / (2 * p.sigma_k ** 2))
    x[5] = (math.atan2(k[1], k[0]) / (2 * math.pi)) % 1.0
    Wl = tr["lep"][i] + tr["nu"][i]
    x[6] = inv_bw(mdot(Wl, Wl), p.m_w, p.w_w)
    return x, perm


def test_semilep_integrand_positive_at_truth():
    p = oracle.sl_params()
    d = events.ttbar_semileptonic(8, 53)
    for i in range(8):
        x, perm = sl_truth_x(p, d["obs"][i], d["truth"], i)
        jac, E = oracle.sl_map(p, d["obs"][i], perm, x)
        tr = d["truth"]
        if jac == 0.0:       # a truth energy outside a 5-sigma window: skip
            continue
        assert E[3] == pytest.approx(tr["b_lep"][i][0], rel=1e-9)
        assert E[2] == pytest.approx(tr["b_had"][i][0], rel=1e-9)
        v, ns = oracle.sl_integrand(p, d["obs"][i], perm, x)
        assert ns >= 1 and v > 0


# ------------------------------------------------------------ ttbar H ----
def tth_kinematics(n, seed, mt=172.5):
    """on-shell t, tbar, H in the partonic CM with gluons along z"""
    rng = events._rng(seed)
    roots = 700.0 + 300.0 * rng.random(n)
    mtt = 2 * mt + rng.random(n) * (roots - 125.0 - 2 * mt)
    tt, h = events._two_body(roots, mtt, np.full(n, 125.0), events._iso(rng, n))
    t, tb = events._two_body(mtt, np.full(n, mt), np.full(n, mt), events._iso(rng, n))
    return roots, events._boost(t, tt), events._boost(tb, tt), h


def test_gg_tth_gauge_lorentz_bose():
    """e1 -> k1 annihilates both colour orderings (all 8 diagrams); |M|^2 is
    invariant under a boost along and a rotation about the beam, and
    symmetric under exchange of the two gluons"""
    mt = 172.5
    roots, t, tb, h = tth_kinematics(8, 5)
    B = np.array([[np.cosh(0.7), 0, 0, np.sinh(0.7)], [0, 1, 0, 0], [0, 0, 1, 0], [np.sinh(0.7), 0, 0, np.cosh(0.7)]])
    c, s = np.cos(1.1), np.sin(1.1)
    L = B @ np.array([[1, 0, 0, 0], [0, c, -s, 0], [0, s, c, 0], [0, 0, 0, 1]])
    for i in range(8):
        k1 = np.array([roots[i] / 2, 0, 0, roots[i] / 2])
        k2 = np.array([roots[i] / 2, 0, 0, -roots[i] / 2])
        m0 = oracle.gg_tth_prod(mt, k1, k2, t[i], tb[i], h[i])
        assert m0 > 0
        assert oracle.gg_tth_ward(mt, k1, k2, t[i], tb[i], h[i]) < 1e-10
        assert oracle.gg_tth_prod(mt, k2, k1, t[i], tb[i], h[i]) == pytest.approx(m0, rel=1e-13)
        assert oracle.gg_tth_prod(mt, L @ k1, L @ k2, L @ t[i], L @ tb[i], L @ h[i]) == pytest.approx(m0, rel=1e-11)


def test_tth_soft_higgs_theorem():
    """A(gg -> t tbar H) at p_H -> 0 equals d/dm A(gg -> t tbar) for the
    decayed tops (the scalar vertex is the identity and every top propagator
    takes one insertion): the deviation falls linearly with p_H"""
    rng = events._rng(9)
    for _ in range(3):
        M = 420.0 + 200.0 * rng.random(1)
        t1, t2 = events._two_body(M, np.array([162.0]), np.array([184.0]), events._iso(rng, 1))
        b, wp = events._two_body(np.array([162.0]), np.zeros(1), np.array([79.0]), events._iso(rng, 1))
        bb, wm = events._two_body(np.array([184.0]), np.zeros(1), np.array([81.0]), events._iso(rng, 1))
        lp, nu = events._two_body(np.array([79.0]), np.zeros(1), np.zeros(1), events._iso(rng, 1))
        lm, nub = events._two_body(np.array([81.0]), np.zeros(1), np.zeros(1), events._iso(rng, 1))
        lp, nu = events._boost(lp, wp), events._boost(nu, wp)
        lm, nub = events._boost(lm, wm), events._boost(nub, wm)
        b, lp, nu = (events._boost(v, t1) for v in (b, lp, nu))
        bb, lm, nub = (events._boost(v, t2) for v in (bb, lm, nub))
        Pz = np.array([[np.sqrt(M[0] ** 2 + 150.0 ** 2), 0, 0, 150.0]])
        mom = np.concatenate([events._boost(v, Pz) for v in (b, lp, nu, bb, lm, nub)])
        d3, d4, d5 = (oracle.tth_soft_check(172.5, mom, dl) for dl in (1e-3, 1e-4, 1e-5))
        assert 5.0 < d3 / d4 < 20.0 and 5.0 < d4 / d5 < 20.0 and d5 < 1e-4, (d3, d4, d5)


def tth_truth_x(p, obs, tr, i):
    """invert the ttH map at the generator's truth"""
    S = p.sqrt_s ** 2
    bs, ls = tr["bslot"][i], tr["lslot"][i]          # parton -> slot
    bl, bh, h1, h2 = (int(v) for v in bs)
    hpair = tuple(sorted((h1, h2)))
    perm = [k for k in range(24) if oracle.tth_perm(k)[:4] == hpair + (bl, bh)
            and oracle.tth_perm(k)[4] == (0 if int(ls[0]) == 0 else 1)][0]
    ih1 = hpair[0]
    part_b = {bl: tr["b_lep"][i], bh: tr["b_had"][i], h1: tr["hb"][i], h2: tr["hbb"][i]}
    part_l = {int(ls[0]): tr["q"][i], int(ls[1]): tr["qbar"][i]}
    x = np.zeros(9)
    r = lambda meas, true: (meas / true - p.lj_r_lo) / (p.lj_r_hi - p.lj_r_lo)

    def inv_bw(q, m, w):
        t0, t1 = math.atan((0 - m * m) / (m * w)), math.atan((S - m * m) / (m * w))
        return (math.atan((q - m * m) / (m * w)) - t0) / (t1 - t0)

    x[0] = r(obs[4][0], part_l[0][0])
    W = part_l[0] + part_l[1]
    x[1] = inv_bw(mdot(W, W), p.m_w, p.w_w)
    T = W + tr["b_had"][i]
    x[2] = inv_bw(mdot(T, T), p.m_t, p.w_t)
    x[3] = r(obs[bl][0], tr["b_lep"][i][0])
    k = tr["k"][i]
    x[4] = 1 - math.exp(-(k @ k) / (2 * p.sigma_k ** 2))
    x[5] = (math.atan2(k[1], k[0]) / (2 * math.pi)) % 1.0
    Wl = tr["lep"][i] + tr["nu"][i]
    x[6] = inv_bw(mdot(Wl, Wl), p.m_w, p.w_w)
    x[7] = r(obs[ih1][0], part_b[ih1][0])
    H = tr["hb"][i] + tr["hbb"][i]
    x[8] = inv_bw(mdot(H, H), p.m_h, p.w_h)
    return x, perm


def test_tth_integrand_positive_at_truth():
    p = oracle.tt_params()
    d = events.ttbar_higgs(10, 71)
    n_ok = 0
    for i in range(10):
        x, perm = tth_truth_x(p, d["obs"][i], d["truth"], i)
        if np.any(x <= 0) or np.any(x >= 1):
            continue
        jac, E = oracle.tth_map(p, d["obs"][i], perm, x)
        if jac == 0.0:       # a truth energy outside the r window: skip
            continue
        tr = d["truth"]
        assert E[2] == pytest.approx(tr["b_had"][i][0], rel=1e-8)
        assert E[3] == pytest.approx(tr["b_lep"][i][0], rel=1e-8)
        v, ns = oracle.tth_integrand(p, d["obs"][i], perm, x)
        assert ns >= 1 and v > 0
        n_ok += 1
    assert n_ok >= 5


# ------------------------------------------------------------ flow -----
def test_flow_context_permutation_and_balance():
    """perm = 1 swaps the two jet slots and leaves the rest; the sum slot
    holds the four objects' sum; MET balances the visible transverse
    momentum"""
    from synth import events
    d = events.ttbar_dilepton(6, 41)
    for e in range(6):
        ev = d["obs"][e]
        c0, c1 = oracle.flow_context(ev, 0), oracle.flow_context(ev, 1)
        assert np.array_equal(c0[0:4], c1[4:8]) and np.array_equal(c0[4:8], c1[0:4])
        assert np.array_equal(c0[8:], c1[8:])
        S = ev[:4].sum(axis=0)
        assert c0[16] == pytest.approx(np.log(S[0] / 100.0), rel=1e-14)
        assert np.allclose(c0[17:20] * 100.0, S[1:], rtol=1e-13)
        assert np.allclose(c0[21:23] * 100.0, -S[1:3], rtol=1e-13)
        met = np.hypot(S[1], S[2])
        assert c0[20] == pytest.approx(np.log((met + 1.0) / 100.0), rel=1e-13)
        for k in range(4):
            assert np.exp(c0[4 * k]) * 100.0 == pytest.approx(ev[k, 0], rel=1e-13)


def test_flow_identity_at_init():
    """zero last layer: the flow is the identity up to the fixed reversal
    of the coordinate order, with log q = 0"""
    p = oracle.flow_init(3, 0.0)
    rng = np.random.default_rng(0)
    for _ in range(20):
        c, x = rng.standard_normal(24), rng.random(8)
        z, lq = oracle.flow_forward(p, c, x)
        assert np.allclose(z, x[::-1], atol=1e-14) and abs(lq) < 1e-13


def test_flow_inverse_and_logdet():
    """inverse(forward(x)) = x; log q equals log|det dz/dx| by central
    differences"""
    p = oracle.flow_init(4, 0.3)
    rng = np.random.default_rng(1)
    for _ in range(10):
        c, x = rng.standard_normal(24), 0.02 + 0.96 * rng.random(8)
        z, lq = oracle.flow_forward(p, c, x)
        x2, lq2 = oracle.flow_inverse(p, c, z)
        assert np.allclose(x2, x, atol=1e-12) and lq2 == pytest.approx(lq, abs=1e-10)
        J = np.zeros((8, 8))
        for j in range(8):
            h = 1e-6
            e = np.zeros(8)
            e[j] = h
            J[:, j] = (oracle.flow_forward(p, c, x + e)[0] - oracle.flow_forward(p, c, x - e)[0]) / (2 * h)
        assert np.log(abs(np.linalg.det(J))) == pytest.approx(lq, abs=1e-6)


def test_flow_density_normalised():
    """int q(x) dx = 1 over the cube: mean of q at uniform x"""
    p = oracle.flow_init(5, 0.25)
    rng = np.random.default_rng(2)
    c = rng.standard_normal(24)
    q = np.array([np.exp(oracle.flow_forward(p, c, rng.random(8))[1]) for _ in range(40000)])
    assert abs(q.mean() - 1.0) < 4 * q.std() / np.sqrt(len(q))


def test_flow_nll_gradient_finite_difference():
    p = oracle.flow_init(6, 0.2)
    rng = np.random.default_rng(3)
    n = 5
    x = 0.05 + 0.9 * rng.random((n, 8))
    ctx = rng.standard_normal((n, 24))
    wt = rng.random(n)
    loss, g = oracle.flow_nll_grad(p, x, ctx, wt)
    per = oracle.FLOW_PER_LAYER
    # parameters from every block of every layer: W1, b1, W2, b2, W3, b3
    offs = [0, 128 * 28, 128 * 28 + 128, 128 * 28 + 128 + 128 * 128, 128 * 28 + 256 + 128 * 128,
            128 * 28 + 256 + 128 * 128 + 92 * 128]
    sizes = [128 * 28, 128, 128 * 128, 128, 92 * 128, 92]
    idx = []
    for l in range(6):
        for o, s in zip(offs, sizes):
            idx += list(l * per + o + rng.integers(0, s, 2))
    for i in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (oracle.flow_nll_grad(pp, x, ctx, wt)[0] - oracle.flow_nll_grad(pm, x, ctx, wt)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-7), (i, g[i], fd)


# ------------------------------------------------------ parton-level weight --
def _boost_z_axis_rotation(mom, phi):
    c, s = np.cos(phi), np.sin(phi)
    out = mom.copy()
    out[:, 1] = c * mom[:, 1] - s * mom[:, 2]
    out[:, 2] = s * mom[:, 1] + c * mom[:, 2]
    return out


def _transverse_boost(mom, bx, by):
    b2 = bx * bx + by * by
    g = 1.0 / np.sqrt(1.0 - b2)
    out = mom.copy()
    bp = bx * mom[:, 1] + by * mom[:, 2]
    out[:, 0] = g * (mom[:, 0] + bp)
    k = (g - 1.0) * bp / b2 + g * mom[:, 0]
    out[:, 1] = mom[:, 1] + k * bx
    out[:, 2] = mom[:, 2] + k * by
    return out


def test_parton_weight_symmetries():
    """the parton-level weight depends on the final state only through its
    zero-transverse-momentum frame and the beam axis: unchanged by a common
    transverse boost or a rotation about the beam, and by the reflection
    z -> -z, which exchanges the beams (x1 <-> x2, gg and q qbar channels
    mapped onto themselves); averaged over the b assignments it does not
    depend on the order of the b partons; positive for generated events"""
    p = oracle.tt_params()
    d = events.ttbar_dilepton_partons(40, 5)
    rng = np.random.default_rng(3)
    for ev in d["obs"]:
        w = oracle.tt_parton_weight(p, ev)
        assert w > 0.0
        rot = _boost_z_axis_rotation(ev, rng.uniform(0, 2 * np.pi))
        assert oracle.tt_parton_weight(p, rot) == pytest.approx(w, rel=1e-11)
        bx, by = rng.uniform(-0.3, 0.3, 2)
        bst = _transverse_boost(ev, bx, by)
        assert oracle.tt_parton_weight(p, bst) == pytest.approx(w, rel=1e-9)
        refl = ev.copy()
        refl[:, 3] = -refl[:, 3]
        assert oracle.tt_parton_weight(p, refl) == pytest.approx(w, rel=1e-11)
        sw = ev[[1, 0, 2, 3, 4, 5]]
        assert oracle.tt_parton_weight(p, sw) == pytest.approx(w, rel=1e-14)


def test_parton_weight_limits():
    """an event whose mass in its zero-transverse-momentum frame exceeds
    sqrt(S) needs x1 x2 > 1 and weighs 0; scaling every momentum of an event
    by s (below that limit) scales the weight as the flux, the densities and
    the dimensionless |M|^2 dictate, so it is finite and positive"""
    p = oracle.tt_params()
    ev = events.ttbar_dilepton_partons(3, 8)["obs"][0]
    P = ev.sum(axis=0)
    m = np.sqrt(P[0] ** 2 - P[1] ** 2 - P[2] ** 2 - P[3] ** 2)
    big = ev * (1.01 * p.sqrt_s / m)
    assert oracle.tt_parton_weight(p, big) == 0.0
    mid = ev * (0.5 * p.sqrt_s / m)
    w = oracle.tt_parton_weight(p, mid)
    assert np.isfinite(w) and w >= 0.0


# ------------------------------------------------------------ phase space --
@pytest.mark.parametrize("n", [2, 3, 4])
def test_massless_phase_space_volumes(n):
    """massless n-body phase space: Phi_2 = 1/(8 pi), Phi_3 = s/(256 pi^3),
    Phi_4 = s^2/(24576 pi^5), i.e. (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) /
    ((n-1)! (n-2)!)"""
    rs = 500.0
    s = rs * rs
    exact = (2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2) / (
        math.factorial(n - 1) * math.factorial(n - 2))
    v, err = oracle.ps_volume(n, rs, 0x5eed, 200000)
    if n == 2:
        assert v == pytest.approx(1 / (8 * math.pi), rel=1e-14) and err < 1e-15 * v
    else:
        assert abs(v - exact) < 4 * err and err < 0.01 * exact, (v, exact, err)
    if n == 3:
        assert exact == pytest.approx(s / (256 * math.pi ** 3), rel=1e-14)


def test_top_width_from_decay_phase_space():
    """Gamma(t -> b l+ nu) integrated over the three-body decay phase space with
    the matrix element's W chain equals, in the narrow-width limit,
    Gamma(t -> bW) Gamma(W -> l nu) / Gamma_W with the closed forms
    Gamma(t -> bW) = G_F m_t^3 / (8 sqrt2 pi) (1 - r)^2 (1 + 2r), r = M_W^2/m_t^2,
    and Gamma(W -> l nu) = G_F M_W^3 / (6 sqrt2 pi): this fixes the
    normalisation of the decay vertices and of the W Breit-Wigner factor"""
    gw = 0.01
    p = oracle.tt_params(w_w=gw)
    gf, mt, mw = p.g_fermi, p.m_t, p.m_w
    r = mw * mw / (mt * mt)
    g_tbw = gf * mt ** 3 / (8 * math.sqrt(2) * math.pi) * (1 - r) ** 2 * (1 + 2 * r)
    g_wlnu = gf * mw ** 3 / (6 * math.sqrt(2) * math.pi)
    want = g_tbw * g_wlnu / gw
    v, err = oracle.top_width(p, 0x70b, 400000)
    assert abs(v - want) < 4 * err + 2e-3 * want, (v, want, err)
    assert err < 3e-3 * want


@pytest.mark.parametrize("channel", [0, 1])
def test_decayed_me_narrow_width_factorisation(channel):
    """The decayed t tbar matrix element integrated over the full six-body
    phase space, sigma = (1/(2 shat)) int dPhi_6 |M|^2 (or_tt_me2_gg / _qq),
    tends for Gamma/M -> 0 to the on-shell production cross section times
    the two decay branching fractions:
      sigma -> sigma(ij -> t tbar) [Gamma(t -> bW) Gamma(W -> l nu) / (Gamma_W Gamma_t)]^2,
    with Ellis-Stirling-Webber's closed forms
      sigma_gg = pi a_s^2/(3 s) [(1 + rho + rho^2/16) ln((1+b)/(1-b)) - b (7/4 + 31 rho/16)],
      sigma_qq = 8 pi a_s^2/(27 s) b (1 + rho/2),     rho = 4 m_t^2/s, b = sqrt(1 - rho),
    and the decay widths' closed forms.  Every factor of the decayed matrix
    element enters: couplings, the spin sums of production and decays, the
    initial-state averages and the four Breit-Wigner factors.  Widths scaled
    by 1e-2 put the off-shell corrections (O(Gamma/M)) below the MC error."""
    eps = 1e-2
    p = oracle.tt_params(w_t=1.4 * eps, w_w=2.1 * eps)
    gf, mt, mw, a_s = p.g_fermi, p.m_t, p.m_w, p.alpha_s
    r = mw * mw / (mt * mt)
    g_tbw = gf * mt ** 3 / (8 * math.sqrt(2) * math.pi) * (1 - r) ** 2 * (1 + 2 * r)
    g_wlnu = gf * mw ** 3 / (6 * math.sqrt(2) * math.pi)
    br = g_tbw * g_wlnu / (p.w_t * p.w_w)
    for rs in (400.0, 700.0):
        s = rs * rs
        rho = 4 * mt * mt / s
        b = math.sqrt(1 - rho)
        if channel == 0:
            prod = math.pi * a_s ** 2 / (3 * s) * ((1 + rho + rho * rho / 16) * math.log((1 + b) / (1 - b))
                                                   - b * (7 / 4 + 31 * rho / 16))
        else:
            prod = 8 * math.pi * a_s ** 2 / (27 * s) * b * (1 + rho / 2)
        want = prod * br * br
        v, err = oracle.tt_decayed_sigma(p, channel, rs, 0xa11 + channel, 60000)
        assert err < 5e-3 * want
        assert abs(v - want) < 4 * err + 5e-4 * want, (rs, v / want, err / want)


# ------------------------------------------- closure of the integrands ----
# Eq. integrand is one integral over the unmeasured momenta; the mapped
# integrands write it in propagator-aligned variables with the constraint
# solves (Eq. dilepsolv, the nu_z quadratic, Eq. mhsolve) and their
# Jacobians.  The same integral written directly in the momenta (the
# oracle's direct kinds: no solve, no Breit-Wigner maps, the Breit-Wigner
# factors left in |M|^2) must give the same number: any dropped or extra
# factor of the change of variables (a Jacobian, its power, a 1/(2E), a
# missing solution) breaks the equality.
def test_closure_dilepton_direct_parametrisation():
    """t tbar dilepton: the 8D mapped integral (Eq. dilepsolv solve) equals
    the 8D integral over (nu_x, nu_y, nu_z, nubar_z) with the transverse
    delta function, per (event, assignment), within the combined VEGAS
    errors.  Widths of 20 (top) and 15 GeV (W) let plain VEGAS converge on
    the direct side; the identity holds for any width."""
    from concurrent.futures import ThreadPoolExecutor
    p = oracle.tt_params(w_t=20.0, w_w=15.0)
    obs = events.ttbar_dilepton(4, 0xc105e)["obs"]
    jobs = [(e, pm) for e in range(4) for pm in (0, 1)]

    def run(args):
        kind, n, (e, pm) = args
        r, _, _, _ = oracle.integrate_one(kind, p, obs[e], pm, 11, e, n, 8)
        return r.I, r.sigma

    with ThreadPoolExecutor(8) as ex:
        mapped = list(ex.map(run, [(oracle.KIND_TT, 30000, j) for j in jobs]))
        direct = list(ex.map(run, [(oracle.KIND_TT_DIRECT, 80000, j) for j in jobs]))
    rel = []
    for j, (a, sa), (b, sb) in zip(jobs, mapped, direct):
        assert a > 0 and b > 0, j
        pull = (a - b) / math.hypot(sa, sb)
        assert abs(pull) < 4.0, (j, a, b, sa / a, sb / b)
        rel.append((a - b) / b)
    assert abs(np.mean(rel)) < 0.02, rel


def _slices(fn_pairs, n_found, rng, draw, axis):
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        _slices_quad(fn_pairs, n_found, rng, draw, axis)


def _slices_quad(fn_pairs, n_found, rng, draw, axis):
    from scipy import integrate
    done = 0
    tries = 0
    while done < n_found:
        tries += 1
        assert tries < 400
        ev, perm, x = draw(rng)
        fa, fb = fn_pairs(ev, perm)

        def on(f):
            def g(t):
                y = x.copy()
                y[axis] = t
                return f(y)
            return g

        if max(on(fa)(t) for t in np.linspace(0.02, 0.98, 25)) == 0.0:
            continue
        a = integrate.quad(on(fa), 0, 1, limit=500, epsabs=0, epsrel=1e-10)[0]
        b = integrate.quad(on(fb), 0, 1, limit=500, epsabs=0, epsrel=1e-10)[0]
        assert abs(a - b) <= 1e-6 * abs(a), (axis, perm, a, b)
        done += 1


def test_closure_semileptonic_slices():
    """t tbar semileptonic, one change of variables at a time, each checked
    as a 1D integral at fixed values of the other variables (adaptive
    quadrature to 1e-10):
      nu_z:  the leptonic W virtuality with the nu_z quadratic (both roots,
             Jacobian |d q^2 / d nu_z|) against nu_z itself;
      E_bh:  the hadronic top virtuality against the hadronic b's energy
             (at a fixed hadronic W virtuality);
      E_b:   the hadronic W virtuality against light jet b's energy (at a
             fixed hadronic b energy).
    The three changes compose the semileptonic map; mode 0 of the direct
    integrand is the mapped integrand itself."""
    p = oracle.tt_params()
    obs = events.ttbar_semileptonic(4, 0xc1060)["obs"]
    rng = np.random.default_rng(5)
    for _ in range(100):
        e, perm, x = int(rng.integers(4)), int(rng.integers(12)), rng.random(7)
        a = oracle.sl_integrand(p, obs[e], perm, x)[0]
        b = oracle.sl_direct_integrand(p, obs[e], perm, x, 0)
        assert abs(a - b) <= 1e-14 * abs(a)
    E, N, H = oracle.SL_DIRECT_EB, oracle.SL_DIRECT_NU, oracle.SL_DIRECT_EBH

    def draw(r):
        return obs[int(r.integers(4))], int(r.integers(12)), r.random(7)

    for axis, m1, m2 in ((6, 0, N), (2, 0, H), (1, H, E | H)):
        pairs = (lambda ev, pm, m1=m1, m2=m2: (lambda y: oracle.sl_direct_integrand(p, ev, pm, y, m1),
                                               lambda y: oracle.sl_direct_integrand(p, ev, pm, y, m2)))
        _slices(pairs, 3, rng, draw, axis)


def test_closure_tth_mhsolve_slices():
    """t tbar H dilepton (Sec. 4): the Higgs virtuality of Eq. mhsolve (the
    second Higgs jet's energy solved from it, Jacobian 1/(2 E_1 (1 -
    cos w12))) against that jet's energy itself, as 1D integrals at fixed
    values of the other seven variables.  Higgs width 1 GeV for the
    quadrature; the identity holds for any width."""
    p = oracle.tt_params(w_h=1.0)
    obs = events.ttbar_higgs_dilepton(4, 0xc1061)["obs"]
    rng = np.random.default_rng(6)

    def draw(r):
        return obs[int(r.integers(4))], int(r.integers(12)), r.random(8)

    pairs = (lambda ev, pm: (lambda y: oracle.tthll_integrand(p, ev, pm, y)[0],
                             lambda y: oracle.tthll_direct_integrand(p, ev, pm, y)))
    _slices(pairs, 4, rng, draw, 7)


# ----------------------------------------------------------- PDF grids ----
PDF_BOUNDS = (math.log(1e-5), 0.0, math.log(10.0), math.log(13000.0))


def _grid_from(tables, nx=320, nq=16, bounds=PDF_BOUNDS, qfac=None):
    """grid whose flavour fl holds tables[fl] (a function of x), times
    qfac(ln Q) when given"""
    lx = np.linspace(bounds[0], bounds[1], nx)
    lq = np.linspace(bounds[2], bounds[3], nq)
    xf = np.zeros((nq, nx, 11))
    x = np.exp(lx)
    for fl, f in tables.items():
        col = np.array([f(v) if v < 1.0 else 0.0 for v in x])
        for j in range(nq):
            xf[j, :, fl + 5] = col * (qfac(lq[j]) if qfac else 1.0)
    return oracle.PdfGrid(xf.astype(np.float32), bounds)


def _toy_tables():
    L = oracle.lib()
    return {2: L.or_xf_u, 1: L.or_xf_d, -2: L.or_xf_qbar, -1: L.or_xf_qbar, 0: L.or_xf_g}


def test_pdf_grid_bilinear_exact():
    """the interpolant reproduces c0 + c1 ln x + c2 ln Q + c3 ln x ln Q (a
    different one per flavour) inside the grid and, by linear
    extrapolation of the edge cells, outside it; node values exact"""
    b = (-8.0, 0.0, 1.0, 5.0)                 # unit node spacing, exact in FP32
    nx, nq = 9, 5
    coef = {fl: (fl + 7.0, 0.5 * fl - 1.0, 2.0 - 0.25 * fl, 0.125 * (fl + 2)) for fl in range(-5, 6)}
    lx, lq = np.linspace(b[0], b[1], nx), np.linspace(b[2], b[3], nq)
    xf = np.zeros((nq, nx, 11))
    for fl, (c0, c1, c2, c3) in coef.items():
        xf[:, :, fl + 5] = c0 + c1 * lx[None, :] + c2 * lq[:, None] + c3 * lx[None, :] * lq[:, None]
    g = oracle.PdfGrid(xf.astype(np.float32), b)
    assert np.array_equal(g.xf, xf)
    rng = np.random.default_rng(5)
    for a, q in zip(rng.uniform(-10.0, 1.0, 300), rng.uniform(0.0, 6.5, 300)):
        for fl in (-5, -2, 0, 1, 5):
            c0, c1, c2, c3 = coef[fl]
            want = c0 + c1 * a + c2 * q + c3 * a * q
            got = oracle.pdf_interp(g, fl, math.exp(a), math.exp(q))
            assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (fl, a, q, got, want)
    for i in (0, 3, 8):
        for j in (0, 2, 4):
            assert oracle.pdf_interp(g, 2, math.exp(lx[i]), math.exp(lq[j])) == pytest.approx(xf[j, i, 7], rel=1e-14)
    assert oracle.pdf_interp(g, 6, 0.1, 100.0) == 0.0 and oracle.pdf_interp(g, -6, 0.1, 100.0) == 0.0


def test_pdf_grid_listing_spacing():
    """The paper's interpolation listing (Sec. 4) steps the grid by
    (max - min)/n, so its nodes sit at min + i (max - min)/n, i < n, and the
    last one falls a step short of the stated maximum; outside the range it
    continues the edge cell.  A table laid out for that reader is the
    oracle's grid with the upper bound min + (n - 1)(max - min)/n: the
    oracle's interpolation of it with that bound equals the listing's rule
    (written here from its description: the cell index from the offset over
    the step, clamped to [0, n - 2], bilinear weights over the cell area)
    inside and outside the grid."""
    nx, nq = 37, 9
    lx0, lx1, lq0, lq1 = math.log(1e-4), 0.0, math.log(20.0), math.log(5000.0)
    rng = np.random.default_rng(21)
    xf = rng.random((nq, nx, 11)).astype(np.float32)
    dx, dq = (lx1 - lx0) / nx, (lq1 - lq0) / nq
    g = oracle.PdfGrid(xf, (lx0, lx0 + (nx - 1) * dx, lq0, lq0 + (nq - 1) * dq))

    def listing(fl, x, Q):
        lx, lq = math.log(x), math.log(Q)
        ix = int((lx - lx0) / dx) if lx > lx0 else 0
        ix = min(ix, nx - 2)
        iq = int((lq - lq0) / dq) if lq > lq0 else 0
        iq = min(iq, nq - 2)
        c1x, c1q = lx0 + dx * ix, lq0 + dq * iq
        c2x, c2q = lx0 + dx * (ix + 1), lq0 + dq * (iq + 1)
        t = xf[:, :, fl + 5].astype(np.float64)
        return (t[iq, ix] * (c2x - lx) * (c2q - lq) + t[iq, ix + 1] * (lx - c1x) * (c2q - lq)
                + t[iq + 1, ix] * (c2x - lx) * (lq - c1q) + t[iq + 1, ix + 1] * (lx - c1x) * (lq - c1q)) / (dx * dq)

    for _ in range(400):
        x = math.exp(rng.uniform(lx0 - 0.5, lx1 + 0.3))
        Q = math.exp(rng.uniform(lq0 - 0.3, lq1 + 0.3))
        fl = int(rng.integers(-5, 6))
        want = listing(fl, x, Q)
        assert oracle.pdf_interp(g, fl, x, Q) == pytest.approx(want, rel=1e-9, abs=1e-9)


def test_pdf_grid_toy_accuracy():
    """Sec. 4 states interpolated densities within 1 % of the directly
    queried ones: the toy densities tabulated on 320 x 16 nodes, x in
    [1e-5, 1], Q in [10, 13000] GeV, meet that on x in [1e-4, 0.5] (the
    range the top processes sample); s, c, b are zero"""
    g = oracle.pdf_tabulate_toy(320, 16, PDF_BOUNDS)
    ref = _grid_from(_toy_tables())
    assert np.array_equal(g.xf, ref.xf)
    rng = np.random.default_rng(6)
    for fl, f in _toy_tables().items():
        for x in np.exp(rng.uniform(math.log(1e-4), math.log(0.5), 400)):
            Q = math.exp(rng.uniform(PDF_BOUNDS[2], PDF_BOUNDS[3]))
            assert abs(oracle.pdf_interp(g, fl, x, Q) / f(x) - 1.0) < 0.01, (fl, x)
    for fl in (3, 4, 5, -3, -4, -5):
        assert oracle.pdf_interp(g, fl, 0.01, 100.0) == 0.0


def _dy_points(p, ev, n, rng):
    """points of the Drell-Yan map inside the mass window, with their pair mass"""
    out = []
    while len(out) < n:
        x = rng.random(2)
        mu = []
        for k in range(2):
            r = p.r_lo + x[k] * (p.r_hi - p.r_lo)
            pm = np.linalg.norm(ev[k][1:])
            pk = pm / r
            mu.append(np.concatenate([[pk], pk * ev[k][1:] / pm]))
        P = mu[0] + mu[1]
        m2 = mdot(P, P)
        if p.m_lo ** 2 <= m2 <= p.m_hi ** 2:
            out.append((x, math.sqrt(m2)))
    return out


def test_pdf_grid_drell_yan_flavours_and_scale():
    """Drell-Yan with grid densities: the luminosity weights each flavour by
    its charge squared (c as u, d and s a quarter of u), pairs a quark with
    its own antiquark, and takes the pair mass as the scale (a grid scaled
    by a linear function of ln Q scales the integrand by its square at M)"""
    p = oracle.dy_params()
    L = oracle.lib()
    ev = events.drell_yan(1, 71)["obs"][0]
    pts = _dy_points(p, ev, 40, np.random.default_rng(7))
    U, Q = L.or_xf_u, L.or_xf_qbar
    gu = _grid_from({2: U, -2: Q})
    gc = _grid_from({4: U, -4: Q})
    gs = _grid_from({3: U, -3: Q})
    gx = _grid_from({2: U, -1: Q})                      # u against dbar: no pair
    qf = lambda lq: 0.5 + 0.3 * lq
    gq = _grid_from({2: U, -2: Q}, qfac=qf)
    for x, M in pts:
        vu = oracle.dy_integrand(oracle.with_pdf(p, gu), ev, x)
        assert vu > 0
        assert oracle.dy_integrand(oracle.with_pdf(p, gc), ev, x) == pytest.approx(vu, rel=1e-12)
        assert oracle.dy_integrand(oracle.with_pdf(p, gs), ev, x) == pytest.approx(0.25 * vu, rel=1e-12)
        assert oracle.dy_integrand(oracle.with_pdf(p, gx), ev, x) == 0.0
        vq = oracle.dy_integrand(oracle.with_pdf(p, gq), ev, x)
        assert vq == pytest.approx(vu * qf(math.log(M)) ** 2, rel=2e-6)
    # the full toy tables reproduce the toy integrand within the 1 % of the tables
    gt = oracle.pdf_tabulate_toy(320, 16, PDF_BOUNDS)
    for x, _ in pts:
        assert oracle.dy_integrand(oracle.with_pdf(p, gt), ev, x) == pytest.approx(
            oracle.dy_integrand(p, ev, x), rel=0.01)


def test_pdf_grid_top_flavours_and_scale():
    """ttbar dilepton with grid densities: q qbar -> t tbar is flavour-blind
    (u and b tables give the same value), a quark pairs only with its own
    antiquark (u against dbar leaves the gg channel alone), the scale is
    m_t (a ln Q-linear factor enters squared at m_t), and the toy tables
    reproduce the toy integrand within 1 %"""
    p = oracle.tt_params()
    L = oracle.lib()
    d = events.ttbar_dilepton(3, 41)
    U, Q, G = L.or_xf_u, L.or_xf_qbar, L.or_xf_g
    gu = _grid_from({2: U, -2: Q, 0: G})
    gb = _grid_from({5: U, -5: Q, 0: G})
    gx = _grid_from({2: U, -1: Q, 0: G})
    gg = _grid_from({0: G})
    qf = lambda lq: 0.5 + 0.3 * lq
    gq = _grid_from({2: U, -2: Q, 0: G}, qfac=qf)
    gt = oracle.pdf_tabulate_toy(320, 16, PDF_BOUNDS)
    rng = np.random.default_rng(8)
    n = 0
    for i in range(3):
        ev = d["obs"][i]
        xt, perm = tt_truth_x(p, ev, d["truth"], i)
        for x in np.clip(xt + 0.002 * rng.standard_normal((30, 8)), 1e-6, 1 - 1e-6):
            vu = oracle.tt_integrand(oracle.with_pdf(p, gu), ev, perm, x)[0]
            if vu == 0.0:
                continue
            n += 1
            assert oracle.tt_integrand(oracle.with_pdf(p, gb), ev, perm, x)[0] == pytest.approx(vu, rel=1e-12)
            vx = oracle.tt_integrand(oracle.with_pdf(p, gx), ev, perm, x)[0]
            assert vx == pytest.approx(oracle.tt_integrand(oracle.with_pdf(p, gg), ev, perm, x)[0], rel=1e-12)
            assert vx < vu
            vq = oracle.tt_integrand(oracle.with_pdf(p, gq), ev, perm, x)[0]
            assert vq == pytest.approx(vu * qf(math.log(p.m_t)) ** 2, rel=2e-6)
            assert oracle.tt_integrand(oracle.with_pdf(p, gt), ev, perm, x)[0] == pytest.approx(
                oracle.tt_integrand(p, ev, perm, x)[0], rel=0.01)
    assert n > 30


def test_pdf_grid_tth_gluon_and_scale():
    """gg -> ttbar H with grid densities: only the gluon table enters, at the
    scale m_t; the toy gluon table reproduces the toy integrand within 1 %"""
    p = oracle.tt_params()
    L = oracle.lib()
    d = events.ttbar_higgs(10, 71)
    G = L.or_xf_g
    gg = _grid_from({0: G})
    gq = _grid_from({0: G, 2: L.or_xf_u, -2: L.or_xf_qbar})
    qf = lambda lq: 0.5 + 0.3 * lq
    gs = _grid_from({0: G}, qfac=qf)
    gt = oracle.pdf_tabulate_toy(320, 16, PDF_BOUNDS)
    n = 0
    for i in range(10):
        x, perm = tth_truth_x(p, d["obs"][i], d["truth"], i)
        if np.any(x <= 0) or np.any(x >= 1):
            continue
        v = oracle.tth_integrand(oracle.with_pdf(p, gg), d["obs"][i], perm, x)[0]
        if v == 0.0:
            continue
        n += 1
        assert oracle.tth_integrand(oracle.with_pdf(p, gq), d["obs"][i], perm, x)[0] == v
        assert oracle.tth_integrand(oracle.with_pdf(p, gs), d["obs"][i], perm, x)[0] == pytest.approx(
            v * qf(math.log(p.m_t)) ** 2, rel=2e-6)
        assert oracle.tth_integrand(oracle.with_pdf(p, gt), d["obs"][i], perm, x)[0] == pytest.approx(
            oracle.tth_integrand(p, d["obs"][i], perm, x)[0], rel=0.01)
    assert n >= 5


# ------------------------------------------ t tbar b bbar and Sec. 4 (f2) --
def _ttbb_kin(rng, mt, mb=0.0, spread=150.0):
    """g(k1) g(k2) -> p3 p4 p5 p6 in the partonic rest frame, masses (mt, mt,
    mb, mb), gluons along +-z"""
    ps = rng.normal(0.0, spread, (3, 3))
    P = np.vstack([ps, -ps.sum(0)])
    m = np.array([mt, mt, mb, mb])
    E = np.sqrt((P ** 2).sum(1) + m ** 2)
    mom = np.column_stack([E, P])
    W = E.sum()
    return np.array([W / 2, 0, 0, W / 2]), np.array([W / 2, 0, 0, -W / 2]), mom


def test_ttbb_colour_closed_forms():
    """SU(3) pins of the colour machinery: f^123 = 1, f^acd f^bcd = N
    delta^ab, and diagonal colour-matrix entries of four diagram classes
    worked out by hand with Tr(T^a T^b) = delta^ab / 2 and sum_a T^a T^a = C_F:
    (T^aT^bT^c)_ij T^c_kl: C_F^3 N / 2 = 32/9; (T^aT^c)_ij (T^bT^c)_kl: 2 C_F^2
    = 32/9; f^abe (T^eT^c)_ij T^c_kl: N^2 C_F^2 / 2 = 8; f^ace f^beg T^g_ij
    T^c_kl: N^2 (N^2 - 1) / 4 = 18."""
    F = oracle.colour_fabc()
    assert F[0, 1, 2] == pytest.approx(1.0, abs=1e-14)
    assert np.allclose(np.einsum("acd,bcd->ab", F, F), 3.0 * np.eye(8), atol=1e-13)
    assert np.allclose(F, -np.transpose(F, (1, 0, 2)), atol=1e-14)
    CM = oracle.colour_matrix_ttbb()
    assert np.allclose(CM, CM.T, atol=1e-12)
    assert np.min(np.linalg.eigvalsh(CM)) > -1e-10            # a Gram matrix
    for d, v in ((0, 32 / 9), (6, 32 / 9), (12, 32 / 9), (20, 8.0), (32, 18.0)):
        assert CM[d, d] == pytest.approx(v, rel=1e-12), d


@pytest.mark.parametrize("mt", [172.5, 0.0])
def test_ttbb_ward_identity(mt):
    """with either gluon's polarisation replaced by its momentum (the other
    physical) the colour-summed |M|^2 vanishes: every diagram, colour factor
    and relative sign enters"""
    rng = np.random.default_rng(11)
    for _ in range(3):
        k1, k2, m = _ttbb_kin(rng, mt)
        for g in (0, 1):
            assert oracle.gg_ttbb_ward(mt, k1, k2, *m, g) < 1e-20


def test_ttbb_symmetries():
    """Bose symmetry (k1 <-> k2); with massless tops the t tbar <-> b bbar
    exchange; the colour quadratic form equals the explicit colour sum"""
    rng = np.random.default_rng(12)
    for _ in range(3):
        k1, k2, m = _ttbb_kin(rng, 172.5)
        v = oracle.gg_ttbb_prod(172.5, k1, k2, *m)
        assert v > 0.0
        assert oracle.gg_ttbb_prod(172.5, k2, k1, *m) == pytest.approx(v, rel=1e-12)
        assert oracle.gg_ttbb_prod_explicit(172.5, k1, k2, *m) == pytest.approx(v, rel=1e-10)
        k1, k2, m = _ttbb_kin(rng, 0.0)
        v0 = oracle.gg_ttbb_prod(0.0, k1, k2, *m)
        assert oracle.gg_ttbb_prod(0.0, k1, k2, m[2], m[3], m[0], m[1]) == pytest.approx(v0, rel=1e-12)


def test_f2_assignments():
    """every assignment is a distinct placement of the four jets: 12 for
    t tbar H (the Higgs pair unordered), 24 for t tbar b bbar"""
    L = oracle.lib()
    assert L.or_nperm(oracle.KIND_TTH_LL) == 12 and L.or_nperm(oracle.KIND_TTBB_LL) == 24
    assert L.or_dims(oracle.KIND_TTH_LL) == 8 and L.or_dims(oracle.KIND_TTBB_LL) == 8
    seen = set()
    for q in range(12):
        r = oracle.f2_perm(oracle.KIND_TTH_LL, q)
        assert sorted(r) == [0, 1, 2, 3] and r[2] < r[3]
        seen.add((r[0], r[1], frozenset(r[2:])))
    assert len(seen) == 12
    perms = [oracle.f2_perm(oracle.KIND_TTBB_LL, q) for q in range(24)]
    assert perms == sorted(perms) and len(set(perms)) == 24


def _inv_bw(q2, m, w, S=13000.0 ** 2):
    mw = m * w
    t0, t1 = math.atan(-m * m / mw), math.atan((S - m * m) / mw)
    return (math.atan((q2 - m * m) / mw) - t0) / (t1 - t0)


def f2_truth_x(po, kind, d, e):
    """the assignment and the point x of the generated partons of event e"""
    t, obs, slot = d["truth"], d["obs"][e], d["truth"]["slot"][e]
    m2 = lambda v: v[0] ** 2 - v[1] ** 2 - v[2] ** 2 - v[3] ** 2
    for perm in range(oracle.lib().or_nperm(kind)):
        rows = oracle.f2_perm(kind, perm)
        if kind == oracle.KIND_TTH_LL:
            ok = rows[:2] == tuple(slot[:2]) and sorted(rows[2:]) == sorted(slot[2:])
        else:
            ok = rows == tuple(slot)
        if ok:
            break
    q = {slot[0]: t["b"][e], slot[1]: t["bb"][e], slot[2]: t["p1"][e], slot[3]: t["p2"][e]}
    r = lambda row: (obs[row][0] / q[row][0] - po.r_lo) / (po.r_hi - po.r_lo)
    x = np.zeros(8)
    x[0], x[1], x[6] = r(rows[0]), r(rows[1]), r(rows[2])
    x[2] = _inv_bw(m2(t["b"][e] + t["lp"][e] + t["nu"][e]), po.m_t, po.w_t)
    x[3] = _inv_bw(m2(t["bb"][e] + t["lm"][e] + t["nub"][e]), po.m_t, po.w_t)
    x[4] = _inv_bw(m2(t["lp"][e] + t["nu"][e]), po.m_w, po.w_w)
    x[5] = _inv_bw(m2(t["lm"][e] + t["nub"][e]), po.m_w, po.w_w)
    if kind == oracle.KIND_TTH_LL:
        h1, h2 = q[rows[2]], q[rows[3]]
        x[7] = _inv_bw(2.0 * (h1[0] * h2[0] - h1[1:] @ h2[1:]), po.m_h, po.w_h)
    else:
        x[7] = r(rows[3])
    return x, perm


@pytest.mark.parametrize("kind", [oracle.KIND_TTH_LL, oracle.KIND_TTBB_LL])
def test_f2_integrand_truth_and_relabelling(kind):
    """at the generated partons' point the integrand is positive and its
    neutrino solve has a solution; relabelling the event's jets and
    following them with the assignment leaves every value unchanged"""
    po = oracle.tt_params()
    gen = events.ttbar_higgs_dilepton if kind == oracle.KIND_TTH_LL else events.ttbar_bbbar_dilepton
    f = oracle.tthll_integrand if kind == oracle.KIND_TTH_LL else oracle.ttbbll_integrand
    d = gen(4, 21)
    n = oracle.lib().or_nperm(kind)
    for e in range(4):
        x, perm = f2_truth_x(po, kind, d, e)
        assert np.all((x > 0) & (x < 1))
        v, ns = f(po, d["obs"][e], perm, x)
        assert v > 0.0 and ns >= 1
        # swap two jet rows (t tbar H: the b and bbar jets, which keeps the
        # Higgs pair's order) and find the assignment with the same partons
        rows = oracle.f2_perm(kind, perm)
        i, j = (rows[0], rows[1]) if kind == oracle.KIND_TTH_LL else (0, 3)
        ev2 = d["obs"][e].copy()
        ev2[[i, j]] = ev2[[j, i]]
        sw = {i: j, j: i}
        want = tuple(sw.get(r, r) for r in rows)
        p2 = [q for q in range(n) if oracle.f2_perm(kind, q) == want][0]
        assert f(po, ev2, p2, x)[0] == v


@pytest.mark.parametrize("kind", [oracle.KIND_TTH_LL, oracle.KIND_TTBB_LL])
def test_f2_parton_weight_invariances(kind):
    """the parton-level weight (mean over every placement of the four b
    quarks) does not depend on the order the b quarks are stored in, and is
    invariant under a rotation about the beam"""
    po = oracle.tt_params()
    gen = events.ttbar_higgs_dilepton if kind == oracle.KIND_TTH_LL else events.ttbar_bbbar_dilepton
    ev = events.four_b_partons(gen(2, 41), 42)
    c, s = math.cos(0.7), math.sin(0.7)
    for e in ev:
        w = oracle.f2_parton_weight(kind, po, e)
        assert w > 0.0
        sh = e.copy()
        sh[:4] = e[[2, 0, 3, 1]]
        assert oracle.f2_parton_weight(kind, po, sh) == pytest.approx(w, rel=1e-12)
        rot = e.copy()
        rot[:, 1], rot[:, 2] = c * e[:, 1] - s * e[:, 2], s * e[:, 1] + c * e[:, 2]
        assert oracle.f2_parton_weight(kind, po, rot) == pytest.approx(w, rel=1e-9)


def test_four_b_generators():
    """Sec. 4's synthetic samples: no recoil (the partons' transverse
    momenta sum to zero), the t tbar H sample's Higgs pair at 125 GeV, the
    t tbar b bbar pair above its 20 GeV floor, the measured jets along the
    quarks and the truth slots a permutation"""
    for gen, key in ((events.ttbar_higgs_dilepton, "tth"), (events.ttbar_bbbar_dilepton, "ttbb")):
        d = gen(200, 51)
        t = d["truth"]
        parts = [t[k] for k in ("b", "bb", "p1", "p2", "lp", "lm", "nu", "nub")]
        P = sum(parts)
        assert np.max(np.abs(P[:, 1:3])) < 1e-8 * np.max(P[:, 0])
        q = t["p1"] + t["p2"]
        m = np.sqrt(np.maximum(q[:, 0] ** 2 - np.sum(q[:, 1:] ** 2, axis=1), 0.0))
        if key == "tth":
            assert np.allclose(m, 125.0, rtol=1e-9)
        else:
            assert np.all(m > 20.0 - 1e-9)
        obs = d["obs"]
        assert obs.shape == (200, 6, 4)
        for e in range(5):
            slot = t["slot"][e]
            assert sorted(slot) == [0, 1, 2, 3]
            for quark, row in zip((t["b"][e], t["bb"][e], t["p1"][e], t["p2"][e]), slot):
                j = obs[e, row]
                cosang = (j[1:] @ quark[1:]) / (np.linalg.norm(j[1:]) * np.linalg.norm(quark[1:]))
                assert cosang == pytest.approx(1.0, abs=1e-12)
        pe = events.four_b_partons(d, 52)
        assert pe.shape == (200, 8, 4)
        assert np.allclose(np.sort(pe[:, :4, 0], axis=1),
                           np.sort(np.stack([t["b"][:, 0], t["bb"][:, 0], t["p1"][:, 0], t["p2"][:, 0]], 1), axis=1))


def test_combine_iterations():
    """the two combinations of VEGAS iterations: the weighted one equals
    the driver's own result bit for bit; equal weights worked by hand; on
    the Genz product peak at 128 points x 6 iterations over 300 seeds the
    equal-weight estimate is unbiased (its seed average within 3 standard
    errors of the exact integral) while the inverse-variance one runs low
    (an iteration that missed the peak has both a low I_j and a low
    sigma_j^2, and so the larger weight)"""
    I, s = oracle.combine_iterations([9.0, 1.0, 2.0, 3.0], [5.0, 1.0, 4.0, 9.0], 1, 1)
    assert I == 2.0 and s == pytest.approx(math.sqrt(14.0) / 3.0, rel=1e-15)
    I, s = oracle.combine_iterations([9.0, 1.0, 2.0, 3.0], [5.0, 1.0, 4.0, 9.0], 1, 0)
    w = np.array([1.0, 0.25, 1.0 / 9.0])
    assert I == pytest.approx((1.0 * 1 + 2.0 * 0.25 + 3.0 / 9.0) / w.sum(), rel=1e-15)
    assert s == pytest.approx(math.sqrt(1.0 / w.sum()), rel=1e-15)
    assert oracle.combine_iterations([4.0, 0.0, 0.0], [1.0, 0.0, 0.0], 1, 0) == (0.0, 0.0)
    p = oracle.dy_params()
    exact = oracle.lib().or_genz_exact()
    wt, eq = [], []
    for seed in range(300):
        r, Is, Vs, _ = oracle.integrate_one(oracle.KIND_GENZ, p, np.zeros(4), 0, 1000 + seed, 0, 128, 6)
        a, sa = oracle.combine_iterations(Is, Vs, 1, 0)
        assert a == r.I and sa == r.sigma
        wt.append(a / exact)
        eq.append(oracle.combine_iterations(Is, Vs, 1, 1)[0] / exact)
    wt, eq = np.array(wt), np.array(eq)
    se_eq, se_wt = eq.std(ddof=1) / math.sqrt(len(eq)), wt.std(ddof=1) / math.sqrt(len(wt))
    assert abs(eq.mean() - 1.0) < 3.0 * se_eq
    assert wt.mean() < 1.0 - 10.0 * se_wt
