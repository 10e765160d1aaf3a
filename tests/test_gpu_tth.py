"""gg -> t tbar H (H -> b bbar, semileptonic tops) on the GPU vs the FP64
oracle: the integrand on identical points (FP32 matrix element within 1e-5
relative, FP64 mode within 1e-9; points whose oracle value moves by more
than a tenth of the bar under 1-ulp input changes are counted and
excluded), the first iteration's sums on the uniform grid, full estimates
by a pull test on the oracle's point stream, and the FP32 error estimate
against an independent FP64 reference."""
import sys

import numpy as np
import pytest

import oracle
from synth import events

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mem():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1407_7595_amd as m
    m.lib()
    return m


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def ill_conditioned(po, ev, perm, x, f0, rel):
    """the oracle's own value moves by more than rel under 1-ulp input
    changes (the Higgs tan map, M Gamma = 0.5 GeV^2, amplifies the angle's
    rounding far from the pole)"""
    for k in range(3):
        xp = np.nextafter(x, 1.0) if k == 0 else np.nextafter(x, 0.0) if k == 1 else x * (1 + 2e-16)
        xp = np.clip(xp, 0.0, 1.0 - 2 ** -53)
        f1 = oracle.tth_integrand(po, ev, perm, xp)[0]
        if abs(f1 - f0) > rel * max(abs(f0), 1e-300):
            return True
    return False


def tth_split(obs):
    """oracle layout (7 objects + a charge row) -> GPU components + charges"""
    comps = torch.as_tensor(np.ascontiguousarray(obs[:, :7, :]), dtype=torch.float64).permute(2, 1, 0).contiguous()
    charge = torch.as_tensor(obs[:, 7, 0].astype(np.int32))
    return comps.cuda(), charge.cuda()


@pytest.mark.parametrize("precision,tol", [(1, 1e-5), (0, 1e-9)])
def test_tth_integrand(mem, precision, tol):
    from test_oracle_pins import tth_truth_x
    p = mem.Process(mem.MEM_TTH_SEMILEPTON, precision=precision)
    po = oracle.tt_params()
    d = events.ttbar_higgs(4, 91)
    comps, charge = tth_split(d["obs"])
    rng = np.random.default_rng(5)
    n_cmp = n_flag = 0
    worst = 0.0
    for e in range(4):
        xt, tperm = tth_truth_x(po, d["obs"][e], d["truth"], e)
        near = np.clip(xt + 0.003 * rng.standard_normal((150, 9)), 1e-6, 1 - 1e-6)
        for perm in sorted({tperm, int(rng.integers(24)), int(rng.integers(24))}):
            x = near if perm == tperm else rng.random((300, 9))
            say(f"tth integrand precision={precision} event={e} perm={perm}")
            f = torch.empty(len(x), dtype=torch.float64, device="cuda")
            ns = torch.empty(len(x), dtype=torch.int32, device="cuda")
            mem.eval_points(p, comps, e, perm, dev(x), f, ns, charge=charge)
            torch.cuda.synchronize()
            got, gns = f.cpu().numpy(), ns.cpu().numpy()
            assert np.all(np.isfinite(got)), (e, perm)
            for k, xi in enumerate(x):
                want, wns = oracle.tth_integrand(po, d["obs"][e], perm, xi)
                if want == 0.0 and got[k] == 0.0:
                    continue
                r = abs(got[k] - want) / max(abs(want), 1e-300)
                if (r > tol or gns[k] != wns) and ill_conditioned(po, d["obs"][e], perm, xi, want, 0.1 * tol):
                    n_flag += 1
                    continue
                assert r <= tol and gns[k] == wns, (e, perm, k, got[k], want, gns[k], wns)
                n_cmp += 1
                worst = max(worst, r)
    say(f"tth compared {n_cmp} nonzero points, worst rel {worst:.3g}, flagged ill-conditioned {n_flag}")
    assert n_cmp > 150 and n_flag <= 0.01 * n_cmp + 2


def test_tth_iteration0_sums(mem):
    p = mem.Process(mem.MEM_TTH_SEMILEPTON, precision=mem.MEM_FP32)
    po = oracle.tt_params()
    d = events.ttbar_higgs(2, 92)
    comps, charge = tth_split(d["obs"])
    n_per, seed = 600, 23                 # one ragged chunk per assignment
    it_out = torch.zeros(2 * 48 * 2, dtype=torch.float64, device="cuda")
    say("tth integrate 2 events x 24 x 600 points x 2 iterations")
    mem.integrate_events(comps, p, 24 * n_per, 2, seed=seed, iter_out=it_out, charge=charge)
    torch.cuda.synchronize()
    rec = it_out.cpu().numpy().reshape(2, 48, 2)
    g0 = oracle.uniform_grid(9)
    n_nz = 0
    for e in range(2):
        for perm in (0, 7, 13, 22):
            s1, s2, _ = oracle.vegas_iteration(oracle.KIND_TTH, po, d["obs"][e], perm, seed, e, 0, n_per, g0)
            I0 = s1 / n_per
            n_nz += I0 > 0
            assert rec[0, 24 * e + perm, 0] == pytest.approx(I0, rel=2e-5, abs=1e-300), (e, perm)
    assert n_nz >= 2


def test_tth_estimates_pull(mem):
    p = mem.Process(mem.MEM_TTH_SEMILEPTON, precision=mem.MEM_FP32)
    po = oracle.tt_params()
    n_ev, n_pts, n_it = 3, 24 * 1500, 4
    d = events.ttbar_higgs(n_ev, 93)
    comps, charge = tth_split(d["obs"])
    say(f"tth integrate {n_ev} events x {n_pts} x {n_it}")
    P, err, st = mem.integrate_events(comps, p, n_pts, n_it, seed=77, charge=charge)
    torch.cuda.synchronize()
    P, err, st = P.cpu().numpy(), err.cpu().numpy(), st.cpu().numpy()
    assert np.all(np.isfinite(P)) and np.all(P > 0) and np.all(st == 0)
    Po, Eo, So = oracle.integrate_events(oracle.KIND_TTH, po, d["obs"], 77, n_pts, n_it)
    pl = (P - Po) / np.sqrt(err ** 2 + Eo ** 2)
    say("tth P", P, "oracle", Po, "pulls", np.round(pl, 3))
    assert np.all(np.abs(pl) < 3.0)


def test_tth_pulls_independent_streams(mem):
    """the FP32 estimates and their errors against an independent FP64
    reference (48 events, 24 x 262 144 points x 12 iterations, seed 7).
    With calibrated errors the pulls (difference over the combined error)
    are standard normal.  At the configured budget (262 144 points per event
    and iteration, 10 iterations) VEGAS's inverse-variance combination runs
    about 20 % low with error estimates of 3.5 %, in FP32 and FP64 alike
    (printed, not asserted): an iteration that missed the large weights has
    a low I_j and a low sigma_j^2 and so the larger weight.  Asserted: the
    equal-weight combination (MEM_COMBINE_MEAN) at that budget, and the
    weighted one at 16 times the points, where it has converged, both with
    pulls of median within 0.75 of 0, median |pull| in (0.3, 1.5) and at
    most 5 of 48 beyond 3"""
    n_ev = 48
    d = events.ttbar_higgs(n_ev, 94)
    comps, charge = tth_split(d["obs"])
    p32 = mem.Process(mem.MEM_TTH_SEMILEPTON, precision=mem.MEM_FP32)
    p64 = mem.Process(mem.MEM_TTH_SEMILEPTON, precision=mem.MEM_FP64)
    say(f"tth pulls: {n_ev} events against FP64 24 x 262144 x 12")
    Pr, Er, Sr = (t.cpu().numpy() for t in mem.integrate_events(comps, p64, 24 * 262144, 12, seed=7, charge=charge))
    assert np.all(Sr == 0)
    for name, per, comb, checked in (("weighted", 10923, mem.MEM_COMBINE_WEIGHTED, False),
                                     ("mean", 10923, mem.MEM_COMBINE_MEAN, True),
                                     ("weighted", 174763, mem.MEM_COMBINE_WEIGHTED, True)):
        P, E, S = (t.cpu().numpy() for t in mem.integrate_events(comps, p32, 24 * per, 10, seed=5, charge=charge,
                                                                 combine=comb))
        assert np.all(S == 0)
        pull = (P - Pr) / np.sqrt(E ** 2 + Er ** 2)
        a = np.abs(pull)
        say(f"{name} 24 x {per} x 10: median P/Pref {np.median(P / Pr):.4f}, median err/P {np.median(E / P):.4f}, "
            f"median pull {np.median(pull):.3f}, median |pull| {np.median(a):.3f}, |pull| > 3: {int(np.sum(a > 3))}")
        if checked:
            assert abs(np.median(pull)) < 0.75
            assert 0.3 < np.median(a) < 1.5
            assert np.sum(a > 3) <= 5
