"""Autotuner on the GPU: the launch configuration of a process's integrand
kernel (points per chunk, waves per SIMD the kernel is compiled for).  The
tuner picks one of the candidates, records it in the table, a new process
loads it; every compiled waves variant gives the same weights as the
default on the same points, and the tuned configuration's weights match the
oracle point by point (1e-5, the hot-path bar)."""
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


def first_iteration_weights(mem, comps, proc, n_points, ig, charge=None):
    """the weights of integral ig's points in the first iteration (uniform
    grid), through weights_out"""
    n_int_pts = -(-n_points // proc.shape()[1])
    w = torch.full((2, n_int_pts), -1.0, dtype=torch.float64, device="cuda")
    mem.integrate_events(comps, proc, n_points, 2, seed=3, weights_out=w, weights_integral=ig, charge=charge)
    torch.cuda.synchronize()
    return w.cpu().numpy()[0]


def test_autotune_table_and_use(mem, tmp_path):
    d = events.ttbar_dilepton(24, 61)
    comps = mem.to_components(d["obs"]).cuda()
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    table = tmp_path / "tune.txt"
    say("autotune 24 tt events x 16384, chunks 1024, 4096 x waves 1, 2")
    best, bw, rate = p.autotune(comps, 16384, candidates=[1024, 4096], waves=[1, 2], table_path=str(table))
    say(f"best chunk {best}, {bw} waves per SIMD, {rate:.3g} events/s")
    assert best in (1024, 4096) and bw in (1, 2) and rate > 0
    assert p.chunk_points() == best and p.waves() == bw
    rows = [ln.split() for ln in table.read_text().splitlines() if not ln.startswith("#")]
    assert len(rows) == 1 and rows[0][0].startswith("gfx") and rows[0][1:5] == ["2", "1", str(best), str(bw)]
    q = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    assert q.waves() == 1 and q.load_tuning(str(table)) and q.chunk_points() == best and q.waves() == bw
    # tuned vs the defaults (4096 points, one wave): same estimates within the MC error
    P1, E1, S1 = mem.integrate_events(comps, q, 8192, 4, seed=3)
    q.set_launch(0, 0)
    assert q.chunk_points() == 4096 and q.waves() == 1
    P2, E2, S2 = mem.integrate_events(comps, q, 8192, 4, seed=3)
    torch.cuda.synchronize()
    P1, E1, P2, E2 = (t.cpu().numpy() for t in (P1, E1, P2, E2))
    assert np.all(S1.cpu().numpy() == 0) and np.all(S2.cpu().numpy() == 0)
    # other chunk sums reorder FP64 additions, so the refined grids and the
    # points differ in the last bits: far inside the MC error
    assert np.all(np.abs(P1 - P2) <= 1e-3 * np.sqrt(E1 ** 2 + E2 ** 2))


CASES = [  # kind, precision, events, points per event, waves variants, per-point bar between variants
    ("dy", 0, 8, 4096, (1, 2, 4), 1e-14),
    ("tt", 0, 3, 8192, (1, 2), 1e-10),
    ("tt", 1, 3, 8192, (1, 2), 1e-6),
    ("sl", 1, 2, 12 * 1024, (1, 2), 2e-6),
]


@pytest.mark.parametrize("kind,prec,n_ev,n_points,variants,bar", CASES)
def test_waves_variants_same_weights(mem, kind, prec, n_ev, n_points, variants, bar):
    """every compiled waves variant evaluates the first iteration's points
    (same uniforms, same grid) to the default's weights, with the same zero
    pattern.  Drell-Yan and the semileptonic kernel agree bit for bit; the
    dilepton's one-wave variant runs its root searches from the LDS queue,
    the two-wave one per lane, and the compiler contracts their arithmetic
    differently (measured 1e-11 relative in FP64, 8e-8 with the FP32 matrix
    element, both far inside the oracle bars of 1e-9 and 1e-5)"""
    if kind == "dy":
        d, k = events.drell_yan(n_ev, 62), mem.MEM_DY_QQ_GAMMA_MUMU
    elif kind == "tt":
        d, k = events.ttbar_dilepton(n_ev, 63), mem.MEM_TT_DILEPTON
    else:
        d, k = events.ttbar_semileptonic(n_ev, 64), mem.MEM_TT_SEMILEPTON
    comps = mem.to_components(d["obs"]).cuda()
    charge = torch.as_tensor(d["charge"], dtype=torch.int32).cuda() if "charge" in d else None
    p = mem.Process(k, precision=prec)
    n_perm = p.shape()[1]
    ig = n_perm * (n_ev - 1) + (n_perm - 1)
    ref = None
    for wv in variants:
        p.set_launch(4096, wv)
        w = first_iteration_weights(mem, comps, p, n_points, ig, charge)
        if ref is None:
            ref = w
            continue
        nz = (ref != 0) | (w != 0)
        r = np.abs(w - ref) / np.maximum(np.abs(ref), 1e-300)
        say(f"{kind} prec {prec} waves {wv}: {int(nz.sum())} nonzero, bit-equal {np.array_equal(w, ref)}, "
            f"worst rel {r[nz].max() if nz.any() else 0.0:.3g}")
        assert np.array_equal(w == 0, ref == 0)
        assert (r[nz].max() if nz.any() else 0.0) <= bar


def test_tuned_launch_matches_oracle(mem, tmp_path):
    """the configuration the tuner picks (and the other waves variant),
    point by point against the oracle on the first iteration's points of a
    two-chunk dilepton integral"""
    d = events.ttbar_dilepton(8, 65)
    comps = mem.to_components(d["obs"]).cuda()
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    best, bw, _ = p.autotune(comps, 16384, candidates=[2048, 4096], waves=[1, 2])
    say(f"tuned: chunk {best}, waves {bw}")
    po = oracle.tt_params()
    e, perm, N = 5, 1, 8192
    g0 = oracle.uniform_grid(8)
    want = np.zeros(N)
    for k in range(N):
        u = oracle.uniforms(3, k, 0, e, perm, 8)
        x, jac, _ = oracle.vegas_map(g0, u)
        want[k] = oracle.tt_integrand(po, d["obs"][e], perm, x)[0] * jac
    for wv in (bw, 3 - bw):
        p.set_launch(best, wv)
        got = first_iteration_weights(mem, comps, p, 2 * N, 2 * e + perm)
        both_zero = (got == 0) & (want == 0)
        r = np.where(both_zero, 0.0, np.abs(got - want) / np.maximum(np.abs(want), 1e-300))
        say(f"waves {wv}: {int((~both_zero).sum())} nonzero of {N}, worst rel {r.max():.3g}")
        assert r.max() < 1e-5


def test_autotune_target_mode(mem):
    """tuning on a target-mode call (the options the process will run
    with): a valid pair, the rate in events per second of that call"""
    d = events.ttbar_dilepton(64, 67)
    comps = mem.to_components(d["obs"]).cuda()
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    best, bw, rate = p.autotune(comps, 16384, candidates=[1024, 4096], waves=[1, 2], target_rel_err=0.02,
                                max_iter=16, allocation=mem.MEM_ALLOC_NEYMAN)
    say(f"target mode: chunk {best}, waves {bw}, {rate:.4g} events/s")
    assert best in (1024, 4096) and bw in (1, 2) and 0 < rate < 1e9
    assert p.chunk_points() == best and p.waves() == bw


def test_tuning_refusals(mem, tmp_path):
    tt = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    tth = mem.Process(mem.MEM_TTH_SEMILEPTON, precision=mem.MEM_FP32)
    for proc, args in ((tt, (4096, 4)), (tt, (1000, 1)), (tth, (4096, 1))):
        with pytest.raises(mem.MemError):
            proc.set_launch(*args)
    assert tth.waves() == 2
    comps = mem.to_components(events.ttbar_dilepton(2, 66)["obs"]).cuda()
    with pytest.raises(mem.MemError):
        tt.autotune(comps, 4096, candidates=[4096], waves=[3])
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 2 1 4096 3 1e9\n")
    with pytest.raises(mem.MemError):
        tt.load_tuning(str(bad), arch="gfx950")
