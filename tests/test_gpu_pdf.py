"""Parton densities from (ln x, ln Q) grids (Sec. 4): the HIP integrands
with a grid set (mem_set_pdf_grid) against the oracle with the same grid.

Grids come from the oracle's tabulation (test infrastructure) or from
closed-form tables written here; the GPU receives the same float32 table.
Bars: those of the toy-density parity tests (FP64 Drell-Yan 1e-11, FP64
top processes 1e-9, FP32 1e-5 on every point the oracle does not flag as
ill-conditioned); parton weights as in their own test.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from synth import events

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BOUNDS = (math.log(1e-5), 0.0, math.log(10.0), math.log(13000.0))


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


def flavour_grid(nx=320, nq=16):
    """every flavour non-zero with its own shape and a ln Q dependence, so
    that the flavour sums, the quark/antiquark pairing and the scale all
    matter"""
    L = oracle.lib()
    lx = np.linspace(BOUNDS[0], BOUNDS[1], nx)
    lq = np.linspace(BOUNDS[2], BOUNDS[3], nq)
    x = np.exp(lx)
    xf = np.zeros((nq, nx, 11))
    for fl in range(-5, 6):
        if fl == 0:
            col = np.array([L.or_xf_g(v) for v in x])
        elif fl > 0:
            col = np.array([(L.or_xf_u(v) if fl % 2 == 0 else L.or_xf_d(v)) for v in x]) * (1.0 - 0.15 * (fl - 1))
        else:
            col = np.array([L.or_xf_qbar(v) for v in x]) * (1.0 + 0.2 * (-fl - 1))
        for j in range(nq):
            xf[j, :, fl + 5] = col * (0.6 + 0.1 * lq[j] + 0.02 * fl * lq[j])
    xf[:, -1, :] = 0.0
    return oracle.PdfGrid(xf.astype(np.float32), BOUNDS)


def grids():
    return {"toy": oracle.pdf_tabulate_toy(320, 16, BOUNDS), "flavours": flavour_grid()}


@pytest.mark.parametrize("which", ["toy", "flavours"])
def test_dy_grid_fp64(mem, which):
    g = grids()[which]
    p = mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64)
    p.set_pdf_grid(g.xf, g.bounds)
    po = oracle.with_pdf(oracle.dy_params(), g)
    d = events.drell_yan(4, 3)
    comps = mem.to_components(d["obs"]).cuda()
    x = np.random.default_rng(1).random((600, 2))
    for e in range(4):
        say(f"dy grid={which} event {e}")
        f = torch.empty(len(x), dtype=torch.float64, device="cuda")
        mem.eval_points(p, comps, e, 0, dev(x), f)
        torch.cuda.synchronize()
        got = f.cpu().numpy()
        want = np.array([oracle.dy_integrand(po, d["obs"][e], xi) for xi in x])
        assert np.sum(want > 0) > 50
        assert np.allclose(got, want, rtol=1e-11, atol=0), np.max(np.abs(got - want) / np.maximum(want, 1e-300))


@pytest.mark.parametrize("which", ["toy", "flavours"])
@pytest.mark.parametrize("precision,tol", [(1, 1e-5), (0, 1e-9)])
def test_tt_grid(mem, which, precision, tol):
    from test_gpu_parity import ill_conditioned, tt_points
    g = grids()[which]
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=precision)
    p.set_pdf_grid(g.xf, g.bounds)
    po = oracle.with_pdf(oracle.tt_params(), g)
    d = events.ttbar_dilepton(3, 17)
    comps = mem.to_components(d["obs"]).cuda()
    rng = np.random.default_rng(2)
    n_cmp = n_flag = 0
    worst = 0.0
    for e in range(3):
        x, _ = tt_points(po, d, 400, rng, e)
        for perm in (0, 1):
            say(f"tt grid={which} precision={precision} event={e} perm={perm}")
            f = torch.empty(len(x), dtype=torch.float64, device="cuda")
            ns = torch.empty(len(x), dtype=torch.int32, device="cuda")
            mem.eval_points(p, comps, e, perm, dev(x), f, ns)
            torch.cuda.synchronize()
            got, gns = f.cpu().numpy(), ns.cpu().numpy()
            assert np.all(np.isfinite(got))
            for k, xi in enumerate(x):
                want, wns = oracle.tt_integrand(po, d["obs"][e], perm, xi)
                if want == 0.0 and got[k] == 0.0:
                    continue
                r = abs(got[k] - want) / max(abs(want), 1e-300)
                if r > tol or gns[k] != wns:
                    if ill_conditioned(po, d["obs"][e], perm, xi, want):
                        n_flag += 1
                        continue
                    assert r <= tol and gns[k] == wns, (e, perm, k, got[k], want, gns[k], wns)
                n_cmp += 1
                worst = max(worst, r)
    say(f"compared {n_cmp}, worst rel {worst:.3g}, flagged {n_flag}")
    assert n_cmp > 200 and n_flag <= 0.01 * n_cmp + 2


def test_sl_grid_fp32(mem):
    from test_gpu_parity import sl_split
    from test_oracle_pins import sl_truth_x
    g = flavour_grid()
    p = mem.Process(mem.MEM_TT_SEMILEPTON, precision=mem.MEM_FP32)
    p.set_pdf_grid(g.xf, g.bounds)
    po = oracle.with_pdf(oracle.sl_params(), g)
    d = events.ttbar_semileptonic(3, 61)
    comps, charge = sl_split(d["obs"])
    comps, charge = comps.cuda(), charge.cuda()
    rng = np.random.default_rng(3)
    n_cmp, worst = 0, 0.0
    for e in range(3):
        xt, tperm = sl_truth_x(po, d["obs"][e], d["truth"], e)
        x = np.clip(xt + 0.003 * rng.standard_normal((200, 7)), 1e-6, 1 - 1e-6)
        say(f"sl grid event={e} perm={tperm}")
        f = torch.empty(len(x), dtype=torch.float64, device="cuda")
        mem.eval_points(p, comps, e, tperm, dev(x), f, charge=charge)
        torch.cuda.synchronize()
        got = f.cpu().numpy()
        assert np.all(np.isfinite(got))
        for k, xi in enumerate(x):
            want = oracle.sl_integrand(po, d["obs"][e], tperm, xi)[0]
            if want == 0.0 and got[k] == 0.0:
                continue
            r = abs(got[k] - want) / max(abs(want), 1e-300)
            assert r <= 1e-5, (e, k, got[k], want)
            n_cmp += 1
            worst = max(worst, r)
    say(f"sl grid compared {n_cmp}, worst rel {worst:.3g}")
    assert n_cmp > 100


@pytest.mark.parametrize("precision,tol", [(1, 1e-5), (0, 1e-10)])
def test_parton_weights_grid(mem, precision, tol):
    g = flavour_grid()
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=precision)
    p.set_pdf_grid(g.xf, g.bounds)
    po = oracle.with_pdf(oracle.tt_params(), g)
    d = events.ttbar_dilepton_partons(1000, 13)
    say(f"parton weights grid precision={precision}")
    comps = torch.as_tensor(np.ascontiguousarray(d["obs"].transpose(2, 1, 0)), dtype=torch.float64).cuda()
    got = mem.parton_weights(p, comps).cpu().numpy()
    want = np.array([oracle.tt_parton_weight(po, ev) for ev in d["obs"]])
    assert np.all(want > 0.0)
    rel = np.abs(got - want) / want
    say(f"  worst rel {rel.max():.3g}, 99.9 % {np.quantile(rel, 0.999):.3g}")
    if precision == 0:
        assert rel.max() <= tol
    else:
        assert np.quantile(rel, 0.999) <= tol and rel.max() <= 3 * tol


def test_grid_integration_and_reset(mem):
    """a mixed batch integrated with toy tables on a grid agrees with the toy
    densities within the tables' accuracy; removing the grid restores the
    toy results bit for bit"""
    from test_gpu_parity import sl_split
    g = oracle.pdf_tabulate_toy(320, 16, BOUNDS)
    tt = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    dt = events.ttbar_dilepton(24, 5)
    comps = mem.to_components(dt["obs"]).cuda()
    say("grid integration: toy densities")
    P0, E0, S0 = mem.integrate_events(comps, tt, 32768, 6, seed=11)
    tt.set_pdf_grid(g.xf, g.bounds)
    say("grid integration: toy tables on a grid")
    P1, E1, S1 = mem.integrate_events(comps, tt, 32768, 6, seed=11)
    tt.set_pdf_grid(None, None)
    say("grid integration: grid removed")
    P2, _, _ = mem.integrate_events(comps, tt, 32768, 6, seed=11)
    torch.cuda.synchronize()
    P0, E0, P1, E1, P2 = (t.cpu().numpy() for t in (P0, E0, P1, E1, P2))
    assert np.all(S0.cpu().numpy() == 0) and np.all(S1.cpu().numpy() == 0)
    assert np.array_equal(P0, P2)
    ok = (P0 > 0) & (E0 < 0.05 * P0)
    assert ok.sum() >= 12
    dev_ = np.abs(P1[ok] - P0[ok]) / np.sqrt(E0[ok] ** 2 + E1[ok] ** 2 + (0.006 * P0[ok]) ** 2)
    say(f"  grid vs toy: median |dP|/sigma {np.median(dev_):.3g}, max {dev_.max():.3g}")
    assert np.max(dev_) < 4.0
