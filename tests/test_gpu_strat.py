"""Adaptive stratified sampling on the GPU (mem_integrate_opts.stratify)
against the oracle's stratified VEGAS (Lepage 2021 on top of the grid of
Sec. 2): same hypercube count, same point-to-hypercube assignment, same
per-hypercube estimate, variance and allocation, same grid refinement.

Covered: FP64 Drell-Yan (2D, 2025 hypercubes) and FP64 ttbar dilepton (8D,
256 hypercubes, two assignments) iteration by iteration over several
iterations, so that every allocation after the first is exercised (an
allocation that differed by one point would move every later point of the
integral to other uniforms and break the per-iteration agreement); FP32
ttbar dilepton point by point in the first iteration and its I, sigma^2;
target mode (deterministic, converged, consistent with a high-statistics
plain VEGAS reference); and the refused combinations.  Bars: Drell-Yan
1e-9 relative on I_j and 1e-6 on sigma_j^2 (the per-hypercube variances
come from sums over a few points and cancel); dilepton FP64 1e-6 on I_j and
1e-4 on sigma_j^2: the two sides' grids agree to rounding, which moves a
point's x by ulps, and near the edges of the solvable region the
integrand amplifies that (measured 3e-8 on I_j), while one point of
allocation moved would shift every later point to other uniforms and
change I_j by its MC error, 1e-2 and more; FP32 per point 1e-5 as the
hot-path tests, I_0 1e-5 and sigma_0^2 1e-3.
"""
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


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def test_strat_dy_every_iteration(mem):
    """FP64 Drell-Yan, 4 events x 4096 points x 6 iterations: I_j and
    sigma_j^2 of every iteration, the combined P and its error"""
    n_ev, N, iters, seed = 4, 4096, 6, 31
    d = events.drell_yan(n_ev, 0x51)
    comps = mem.to_components(d["obs"]).cuda()
    dy = mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64)
    rec = torch.zeros((iters, n_ev, 2), dtype=torch.float64, device="cuda")
    P, E, S = mem.integrate_events(comps, dy, N, iters, seed=seed, iter_out=rec, stratify=mem.MEM_STRATIFY_ADAPTIVE)
    rec = rec.cpu().numpy()
    P, E, S = P.cpu().numpy(), E.cpu().numpy(), S.cpu().numpy()
    assert np.all(S == 0)
    assert oracle.strat_ns(2, N) == 45
    ratios = []
    for e in range(n_ev):
        r, Is, Vs = oracle.integrate_one_strat(oracle.KIND_DY, oracle.dy_params(), d["obs"][e], 0, seed, e, N, iters)
        say(f"dy event {e}: I_j rel {rel(rec[:, e, 0], Is).max():.3g}, var_j rel {rel(rec[:, e, 1], Vs).max():.3g}")
        assert rel(rec[:, e, 0], Is).max() < 1e-9
        assert rel(rec[:, e, 1], Vs).max() < 1e-6
        ratios.append((P[e] / r.I, E[e] / r.sigma))
    ratios = np.array(ratios)
    # P = I / sigma_norm for every event: one constant
    assert rel(ratios[:, 0], ratios[0, 0]).max() < 1e-9 and rel(ratios[:, 1], ratios[0, 0]).max() < 1e-6
    # the plain VEGAS call with the same points differs (stratification is on)
    Pp, _, _ = mem.integrate_events(comps, dy, N, iters, seed=seed)
    assert not np.array_equal(Pp.cpu().numpy(), P)


@pytest.mark.parametrize("n_points", [8192, 8192 + 2 * 700])
def test_strat_tt_fp64_every_iteration(mem, n_points):
    """FP64 ttbar dilepton, 3 events x 2 assignments x 4 iterations (the
    second size leaves a ragged chunk and unequal first-iteration counts)"""
    n_ev, iters, seed = 3, 4, 17
    t = events.ttbar_dilepton(n_ev, 0x52)
    comps = mem.to_components(t["obs"]).cuda()
    tt = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP64)
    n_int = 2 * n_ev
    N = n_points // 2
    rec = torch.zeros((iters, n_int, 2), dtype=torch.float64, device="cuda")
    _, _, S = mem.integrate_events(comps, tt, n_points, iters, seed=seed, iter_out=rec,
                                   stratify=mem.MEM_STRATIFY_ADAPTIVE)
    rec = rec.cpu().numpy()
    assert np.all(S.cpu().numpy() == 0)
    assert oracle.strat_ns(8, N) == 2
    po = oracle.tt_params()
    for ig in range(n_int):
        e, perm = divmod(ig, 2)
        _, Is, Vs = oracle.integrate_one_strat(oracle.KIND_TT, po, t["obs"][e], perm, seed, e, N, iters)
        ri, rv = rel(rec[:, ig, 0], Is).max(), rel(rec[:, ig, 1], Vs).max()
        say(f"tt fp64 N={N} integral {ig}: I_j rel {ri:.3g}, var_j rel {rv:.3g}")
        assert ri < 1e-6 and rv < 1e-4


def test_strat_tt_fp32_first_iteration(mem):
    """FP32 ttbar dilepton: every point's weight in the first (equal-split)
    iteration, and its I_0 and sigma_0^2"""
    n_ev, N, seed = 2, 4096, 23
    t = events.ttbar_dilepton(n_ev, 0x53)
    comps = mem.to_components(t["obs"]).cuda()
    tt = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    po = oracle.tt_params()
    ns = oracle.strat_ns(8, N)
    H = ns ** 8
    nh = oracle.strat_allocate(H, N, first=True)
    for ig in (1, 2):
        e, perm = divmod(ig, 2)
        wout = torch.full((2, N), -1.0, dtype=torch.float64, device="cuda")
        rec = torch.zeros((2, 2 * n_ev, 2), dtype=torch.float64, device="cuda")
        mem.integrate_events(comps, tt, 2 * N, 2, seed=seed, iter_out=rec, weights_out=wout, weights_integral=ig,
                             stratify=mem.MEM_STRATIFY_ADAPTIVE)
        got = wout.cpu().numpy()[0]
        I0, V0, _, _, want = oracle.strat_iteration(oracle.KIND_TT, po, t["obs"][e], perm, seed, e, 0, N,
                                                    oracle.uniform_grid(8), ns, nh)
        both_zero = (got == 0.0) & (want == 0.0)
        r = np.where(both_zero, 0.0, rel(got, want))
        say(f"tt fp32 integral {ig}: {int((~both_zero).sum())} nonzero of {N}, worst rel {r.max():.3g}")
        assert np.all(np.isfinite(got)) and r.max() < 1e-5
        r0 = rec.cpu().numpy()[0, ig]
        say(f"  I_0 rel {rel(r0[0], I0):.3g}, var_0 rel {rel(r0[1], V0):.3g}")
        assert rel(r0[0], I0) < 1e-5 and rel(r0[1], V0) < 1e-3


def test_strat_target_mode(mem):
    """target mode with stratification: deterministic, every event converged
    to 1 %, estimates consistent with a high-statistics plain VEGAS
    reference; the stratified errors at a fixed budget against plain
    VEGAS's are printed"""
    n_ev = 48
    t = events.ttbar_dilepton(n_ev, 0x54)
    comps = mem.to_components(t["obs"]).cuda()
    tt = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    kw = dict(seed=7, target_rel_err=0.01, max_iter=64, stratify=mem.MEM_STRATIFY_ADAPTIVE)
    a = [x.cpu().numpy() for x in mem.integrate_events(comps, tt, 65536, 64, **kw)]
    b = [x.cpu().numpy() for x in mem.integrate_events(comps, tt, 65536, 64, **kw)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    P, E, S = a
    ok = S == 0
    say(f"converged {ok.sum()} of {n_ev}")
    assert np.all((S == 0) | (S == 2)) and ok.mean() >= 0.9 and np.all(E[ok] <= 0.01 * P[ok])
    say("reference: plain VEGAS 262144 x 10")
    Pr, Er, Sr = (x.cpu().numpy() for x in mem.integrate_events(comps, tt, 262144, 10, seed=8))
    assert np.all(Sr == 0)
    pull = (P - Pr) / np.sqrt(E ** 2 + Er ** 2)
    say(f"target-mode pulls: median {np.median(pull):.2f}, median |pull| {np.median(np.abs(pull)):.2f}")
    assert abs(np.median(pull)) < 1.0 and np.median(np.abs(pull)) < 1.5
    fixed = {}
    for name, st in (("plain", 0), ("stratified", 1)):
        Pf, Ef, Sf = (x.cpu().numpy() for x in mem.integrate_events(comps, tt, 32768, 6, seed=9, stratify=st))
        assert np.all(Sf == 0)
        fixed[name] = float(np.median(Ef / Pf))
    say("median err/P at 32768 x 6", fixed)
    assert fixed["stratified"] < 1.5 * fixed["plain"]


def test_strat_refused(mem):
    """stratification with Neyman allocation, a flow, a checkpoint, or an
    unknown mode is refused before any launch"""
    t = events.ttbar_dilepton(2, 0x55)
    comps = mem.to_components(t["obs"]).cuda()
    tt = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    with pytest.raises(mem.MemError):
        mem.integrate_events(comps, tt, 4096, 2, stratify=7)
    with pytest.raises(mem.MemError):
        mem.integrate_events(comps, tt, 4096, 2, stratify=1, allocation=mem.MEM_ALLOC_NEYMAN)
    with pytest.raises(mem.MemError):
        mem.integrate_events(comps, tt, 4096, 2, stratify=1, flow=mem.Flow())
    with pytest.raises(mem.MemError):
        mem.integrate_events(comps, tt, 4096, 2, stratify=1, checkpoint=mem.Checkpoint())


def test_strat_mixed_batch_and_noalloc(mem):
    """one call with Drell-Yan (2D, FP64) and dilepton (8D, FP64) events and
    uneven budgets, so integrals of different dimensions and hypercube
    counts share the work queue: every integral's I_j and sigma_j^2 against
    the oracle's stratified driver (event index = position in the batch);
    the no-allocation entry point gives the same outputs bit for bit"""
    dy = mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64)
    tt = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP64)
    dd = events.drell_yan(2, 0x56)["obs"]
    dt = events.ttbar_dilepton(2, 0x57)["obs"]
    kinds = ["dy", "tt", "dy", "tt"]
    src = {"dy": iter(dd), "tt": iter(dt)}
    full, obs = [], np.zeros((len(kinds), 4, 4))
    for i, k in enumerate(kinds):
        o = next(src[k])
        full.append(o)
        n = 2 if k == "dy" else 4
        obs[i, :n] = o[:n]
    budgets = [4096, 8192 + 1400, 2500, 8192]
    procs = [dy if k == "dy" else tt for k in kinds]
    comps = mem.to_components(obs).cuda()
    iters, seed = 4, 29
    n_int = 1 + 2 + 1 + 2
    rec = torch.zeros((iters, n_int, 2), dtype=torch.float64, device="cuda")
    out = mem.integrate_events(comps, procs, budgets, iters, seed=seed, iter_out=rec,
                               stratify=mem.MEM_STRATIFY_ADAPTIVE)
    rec = rec.cpu().numpy()
    out = [t.cpu().numpy() for t in out]
    assert np.all(out[2] == 0)
    ig = 0
    for i, k in enumerate(kinds):
        kind, po, npm = (oracle.KIND_DY, oracle.dy_params(), 1) if k == "dy" else (oracle.KIND_TT, oracle.tt_params(), 2)
        N = -(-budgets[i] // npm)
        for perm in range(npm):
            _, Is, Vs = oracle.integrate_one_strat(kind, po, full[i], perm, seed, i, N, iters)
            ri, rv = rel(rec[:, ig, 0], Is).max(), rel(rec[:, ig, 1], Vs).max()
            say(f"mixed event {i} ({k}) perm {perm}, N={N}: I_j rel {ri:.3g}, var_j rel {rv:.3g}")
            bar_i, bar_v = (1e-9, 1e-6) if k == "dy" else (1e-6, 1e-4)
            assert ri < bar_i and rv < bar_v
            ig += 1
    outs = (torch.empty(4, dtype=torch.float64, device="cuda"), torch.empty(4, dtype=torch.float64, device="cuda"),
            torch.empty(4, dtype=torch.int32, device="cuda"))
    na = mem.integrate_events_noalloc(comps, procs, budgets, iters, outputs=outs, seed=seed,
                                      stratify=mem.MEM_STRATIFY_ADAPTIVE)
    for a, b in zip(out, na):
        assert np.array_equal(a, b.cpu().numpy())
