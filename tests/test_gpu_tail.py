"""Tail chunking (mem_integrate_opts.tail_chunk_points / tail_iter): from a
given iteration on, the integrals' points run in chunks of another size.
The chunking of an iteration depends only on its index, so a target-mode
event equals a fixed run with the same options bit for bit, and iterations
before tail_iter equal a run without the option bit for bit.  After the
switch every point's weight still matches the oracle (FP32 1e-5), the
estimates agree with plain runs within their errors, the no-allocation entry
point gives the same results, and invalid settings are refused."""
import sys

import numpy as np
import pytest

import oracle
from synth import events

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TAIL = dict(tail_chunk_points=1024, tail_iter=3)


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


def fixed(mem, comps, p, npts, n_it, **kw):
    P, E, S = mem.integrate_events(comps, p, npts, n_it, **kw)
    torch.cuda.synchronize()
    return P.cpu().numpy(), E.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("alloc", [0, 1])
def test_tail_target_matches_fixed_runs(mem, alloc):
    """160 dilepton events to 3 % with chunks of 1024 points from the third
    iteration on (4096 before): an event retired after n iterations equals a
    fixed n-iteration run with the same options; runs that end before the
    switch equal runs without the option"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    d = events.ttbar_dilepton(160, 106)
    comps = mem.to_components(d["obs"]).cuda()
    n_it = torch.zeros(160, dtype=torch.int32, device="cuda")
    say(f"tail chunking: target 3 %, allocation {alloc}, 160 events")
    P, E, S = mem.integrate_events(comps, p, 8192, 0, seed=79, target_rel_err=0.03, max_iter=30,
                                   allocation=alloc, n_iter_out=n_it, **TAIL)
    torch.cuda.synchronize()
    P, E, S, n = P.cpu().numpy(), E.cpu().numpy(), S.cpu().numpy(), n_it.cpu().numpy()
    ok = S == 0
    assert ok.sum() >= 150
    counts = np.unique(n[ok], return_counts=True)
    say(f"  iterations used: {dict(zip(counts[0].tolist(), counts[1].tolist()))}")
    assert counts[0].max() > TAIL["tail_iter"], "some events run past the switch"
    checked = late = 0
    for it in counts[0][:5]:
        Pf, Ef, _ = fixed(mem, comps, p, 8192, int(it), seed=79, allocation=alloc, **TAIL)
        sel = ok & (n == it)
        assert np.array_equal(P[sel], Pf[sel]) and np.array_equal(E[sel], Ef[sel]), it
        checked += int(sel.sum())
        late += int(sel.sum()) if it > TAIL["tail_iter"] else 0
    say(f"  {checked} events equal to fixed runs, {late} of them retired after the switch")
    assert checked >= 100 and late >= 10
    # before the switch the tail table is not in use
    n_pre = int(TAIL["tail_iter"])
    Pa, Ea, _ = fixed(mem, comps, p, 8192, n_pre, seed=79, allocation=alloc, **TAIL)
    Pb, Eb, _ = fixed(mem, comps, p, 8192, n_pre, seed=79, allocation=alloc)
    assert np.array_equal(Pa, Pb) and np.array_equal(Ea, Eb)


def test_tail_weights_match_oracle(mem):
    """every point of an integral in iterations past the switch (chunks of
    1024 points, a ragged last one) against the oracle on the grid the
    shorter run leaves"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    d = events.ttbar_dilepton(2, 0x5eed2)
    comps = mem.to_components(d["obs"]).cuda()
    npts, n_iter, ig = 2 * 9000, 5, 1
    per = npts // 2
    wout = torch.full((n_iter, per), float("nan"), dtype=torch.float64, device="cuda")
    mem.integrate_events(comps, p, npts, n_iter, seed=5, weights_out=wout, weights_integral=ig, **TAIL)
    grids = torch.zeros((4, 8, 65), dtype=torch.float64, device="cuda")
    mem.integrate_events(comps, p, npts, n_iter - 1, seed=5, grid_out=grids, **TAIL)
    torch.cuda.synchronize()
    got = wout.cpu().numpy()[n_iter - 1]
    assert not np.any(np.isnan(got))
    g = grids.cpu().numpy()[ig]
    po = oracle.tt_params()
    e, perm = ig // 2, ig % 2
    want = np.zeros(per)
    for k in range(per):
        u = oracle.uniforms(5, k, n_iter - 1, e, perm, 8)
        x, jac, _ = oracle.vegas_map(g, u)
        want[k] = oracle.tt_integrand(po, d["obs"][e], perm, x)[0] * jac
    both_zero = (got == 0) & (want == 0)
    rel = np.where(both_zero, 0.0, np.abs(got - want) / np.maximum(np.abs(want), 1e-300))
    say(f"tail weights, iteration {n_iter - 1}: {int((~both_zero).sum())} nonzero of {per}, worst rel {rel.max():.3g}")
    assert (~both_zero).sum() > 100
    assert rel.max() < 1e-5


def test_tail_estimates_agree_with_plain(mem):
    """the same events to 2 % with and without tail chunking: every event
    converges and the estimates agree within the combined errors"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    comps = mem.to_components(events.ttbar_dilepton(96, 111)["obs"]).cuda()
    kw = dict(seed=7, target_rel_err=0.02, max_iter=40, allocation=mem.MEM_ALLOC_NEYMAN)
    Pa, Ea, Sa = fixed(mem, comps, p, 16384, 0, **kw)
    Pb, Eb, Sb = fixed(mem, comps, p, 16384, 0, tail_chunk_points=2048, tail_iter=4, **kw)
    pull = (Pb - Pa) / np.sqrt(Ea ** 2 + Eb ** 2)
    say(f"tail vs plain: median |pull| {np.median(np.abs(pull)):.3f}, max {np.abs(pull).max():.2f}")
    assert np.all(Sa == 0) and np.all(Sb == 0)
    assert np.median(np.abs(pull)) < 0.5 and np.abs(pull).max() < 4.0


def test_tail_noalloc_equals_integrate(mem):
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    comps = mem.to_components(events.ttbar_dilepton(24, 112)["obs"]).cuda()
    kw = dict(seed=8, target_rel_err=0.03, max_iter=12, allocation=mem.MEM_ALLOC_NEYMAN, **TAIL)
    ref = mem.integrate_events(comps, p, 8192, 0, **kw)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = mem.integrate_events_noalloc(comps, p, 8192, 0, stream=s, **kw)
    s.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)


def test_tail_refusals(mem):
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    comps = mem.to_components(events.ttbar_dilepton(2, 113)["obs"]).cuda()
    for kw in (dict(tail_chunk_points=1000, tail_iter=3), dict(tail_chunk_points=-256, tail_iter=3),
               dict(tail_chunk_points=1024, tail_iter=0), dict(tail_chunk_points=1 << 17, tail_iter=3),
               dict(tail_chunk_points=1024, tail_iter=2, stratify=mem.MEM_STRATIFY_ADAPTIVE)):
        with pytest.raises(mem.MemError):
            mem.integrate_events(comps, p, 4096, 4, **kw)
