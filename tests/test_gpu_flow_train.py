"""The proposal's training and persistence calls: mem_train_proposal
(VEGAS on the training events, capture of the adapted grids' samples,
minibatch training with Adam and a cosine learning rate, all inside the
library), mem_flow_save / mem_flow_load, and mem_set_proposal."""
import os
import sys
import tempfile

import numpy as np
import pytest

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


SMALL = dict(vegas_points=8192, vegas_iter=3, capture=256, batch=16384, epochs=6, lr_max=3e-3, lr_min=3e-4)


def ess_from_iter(rec, N):
    I, var = rec[..., 0], rec[..., 1]
    den = var * (N - 1) + I * I
    return np.where(den > 0, I * I / np.maximum(den, 1e-300), 0.0)


def test_train_proposal_deterministic_and_gain(mem):
    """two calls with the same inputs give the same parameters bit for bit;
    the loss falls; on held-out events the trained flow's ESS/N beats the
    untrained (uniform) proposal's"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    tr = mem.to_components(events.ttbar_dilepton(256, 0x71).get("obs")).cuda()
    say("train_proposal: 256 events, 20 epochs (twice)")
    f1, l1 = mem.train_proposal(p, tr, seed=5, losses=True, **dict(SMALL, epochs=20))
    f2 = mem.train_proposal(p, tr, seed=5, **dict(SMALL, epochs=20))
    torch.cuda.synchronize()
    a, b = f1.get_params(), f2.get_params()
    assert torch.equal(a, b)
    assert torch.any(a != 0)
    say("losses", np.round(l1, 4))
    assert l1[-1] < l1[0] - 0.3
    held = mem.to_components(events.ttbar_dilepton(16, 0x72)["obs"]).cuda()
    N = 8192
    med = {}
    for name, f in (("untrained", mem.Flow()), ("trained", f1)):
        rec = torch.zeros((2, 32, 2), dtype=torch.float64, device="cuda")
        mem.integrate_events(held, p, 2 * N, 2, seed=5, flow=f, ess_threshold=1e-12, iter_out=rec)
        torch.cuda.synchronize()
        med[name] = float(np.median(ess_from_iter(rec.cpu().numpy(), N)[0]))
    say("median ESS/N", med)
    assert med["trained"] > 2.0 * med["untrained"]


def test_flow_save_load(mem):
    """a saved and reloaded flow: same parameters, same Adam state (one more
    training step gives the same parameters), same samples"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    tr = mem.to_components(events.ttbar_dilepton(64, 0x73)["obs"]).cuda()
    say("save/load: train on 64 events, 2 epochs")
    f = mem.train_proposal(p, tr, seed=9, **dict(SMALL, epochs=2, batch=8192))
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "flow.bin")
        f.save(path)
        g = mem.Flow.load(path)
        with open(path, "r+b") as fh:
            fh.seek(0)
            fh.write(b"NOTAFLOW")
        with pytest.raises(mem.MemError):
            mem.Flow.load(path)
    assert torch.equal(f.get_params(), g.get_params())
    n = 4096
    ev_i = torch.zeros(4, dtype=torch.int32, device="cuda")
    pm_i = torch.tensor([0, 1, 0, 1], dtype=torch.int32, device="cuda")
    ev_i[2:] = 1
    ctx = torch.empty((4, 24), dtype=torch.float32, device="cuda")
    mem.flow_context(tr, ev_i, pm_i, ctx)
    outs = []
    for fl in (f, g):
        x = torch.empty((4, n, 8), dtype=torch.float32, device="cuda")
        lq = torch.empty((4, n), dtype=torch.float32, device="cuda")
        fl.sample(ctx, ev_i, pm_i, n, 3, 0, x, lq)
        outs.append((x, lq))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    # one Adam step from the saved state on the same batch
    sint = torch.arange(4, dtype=torch.int32, device="cuda").repeat_interleave(n)
    xs = outs[0][0].reshape(-1, 8).contiguous()
    ws = torch.full((4 * n,), 1.0 / n, dtype=torch.float32, device="cuda")
    f.train_step(ctx, sint, xs, ws, lr=1e-3, want_loss=False)
    g.train_step(ctx, sint, xs, ws, lr=1e-3, want_loss=False)
    torch.cuda.synchronize()
    assert torch.equal(f.get_params(), g.get_params())


def test_set_proposal(mem):
    """a process's proposal is used when the call names no flow (bit-equal
    to naming it); cleared, the call is plain VEGAS again"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    tr = mem.to_components(events.ttbar_dilepton(64, 0x74)["obs"]).cuda()
    f = mem.train_proposal(p, tr, seed=11, **dict(SMALL, epochs=2, batch=8192))
    comps = mem.to_components(events.ttbar_dilepton(6, 0x75)["obs"]).cuda()
    say("set_proposal: 6 events x 8192 x 3")
    want = mem.integrate_events(comps, p, 8192, 3, seed=2, flow=f, ess_threshold=1e-12)
    vegas = mem.integrate_events(comps, p, 8192, 3, seed=2)
    p.set_proposal(f)
    got = mem.integrate_events(comps, p, 8192, 3, seed=2, ess_threshold=1e-12)
    p.set_proposal(None)
    back = mem.integrate_events(comps, p, 8192, 3, seed=2)
    torch.cuda.synchronize()
    for x, y in zip(want, got):
        assert torch.equal(x, y)
    for x, y in zip(vegas, back):
        assert torch.equal(x, y)
    dy = mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64)
    with pytest.raises(mem.MemError):
        dy.set_proposal(f)
    with pytest.raises(mem.MemError):
        mem.train_proposal(dy, tr)
    with pytest.raises(mem.MemError):
        mem.train_proposal(p, tr[:, :, :2].contiguous(), capture=16, batch=4096)


def test_flow_seeded_grids(mem):
    """MEM_FLOW_SEED_GRID: VEGAS starting from grids seeded by the flow's
    samples, every iteration in the estimate.  The seeded first iteration
    has a smaller variance than the uniform grid's; it is importance
    sampling on a grid fixed before its points are drawn, so its estimate
    is unbiased: the mean ratio to a high-statistics VEGAS reference over
    the events is 1 within three standard errors.  (The combination over
    iterations weights them by their estimated variances, as plain VEGAS
    does; at low statistics that weighting pulls both low alike, so the
    combined estimates are held to plain VEGAS's calibration.)  The call
    is deterministic; other kinds and unknown modes are refused."""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    tr = mem.to_components(events.ttbar_dilepton(512, 0x76)["obs"]).cuda()
    say("seeded grids: train on 512 events, 16 epochs")
    f = mem.train_proposal(p, tr, seed=13, **dict(SMALL, epochs=16))
    n_ev = 64
    comps = mem.to_components(events.ttbar_dilepton(n_ev, 0x77)["obs"]).cuda()
    n_int = 2 * n_ev
    recs = {}
    for name, kw in (("uniform", {}), ("seeded", dict(flow=f, flow_mode=mem.MEM_FLOW_SEED_GRID))):
        rec = torch.zeros((4, n_int, 2), dtype=torch.float64, device="cuda")
        out = mem.integrate_events(comps, p, 16384, 4, seed=21, iter_out=rec, **kw)
        torch.cuda.synchronize()
        recs[name] = (rec.cpu().numpy(), [t.cpu().numpy() for t in out])
    rel0 = {k: np.sqrt(v[0][0, :, 1]) / np.maximum(v[0][0, :, 0], 1e-300) for k, v in recs.items()}
    say("first-iteration median relative error", {k: float(np.median(v)) for k, v in rel0.items()})
    assert np.median(rel0["seeded"]) < 0.8 * np.median(rel0["uniform"])
    again = mem.integrate_events(comps, p, 16384, 4, seed=21, flow=f, flow_mode=mem.MEM_FLOW_SEED_GRID)
    for a, b in zip(recs["seeded"][1], again):
        assert np.array_equal(a, b.cpu().numpy())
    say("seeded grids: VEGAS reference 262144 x 10")
    Pr, Er, Sr = (t.cpu().numpy() for t in mem.integrate_events(comps, p, 262144, 10, seed=22))
    assert np.all(Sr == 0) and np.median(Er / Pr) < 0.01 and np.all(Er < 0.03 * Pr)
    P0 = recs["seeded"][0][0, :, 0].reshape(n_ev, 2).mean(axis=1)     # the first iteration alone
    r = P0 / Pr
    t = (r.mean() - 1.0) / (r.std(ddof=1) / np.sqrt(n_ev))
    say(f"first-iteration ratio to the reference: mean {r.mean():.4f}, t {t:.2f}")
    assert abs(t) < 3.0
    # the combined estimates: no worse calibrated than plain VEGAS's with
    # the same points (median pull and median absolute pull)
    med = {}
    for name in ("uniform", "seeded"):
        Pc, Ec, Sc = recs[name][1]
        assert np.all(Sc == 0)
        pull = (Pc - Pr) / np.sqrt(Ec ** 2 + Er ** 2)
        med[name] = (float(np.median(pull)), float(np.median(np.abs(pull))))
    say("combined pulls (median, median |pull|)", med)
    assert abs(med["seeded"][0]) <= abs(med["uniform"][0]) + 0.5
    assert med["seeded"][1] <= med["uniform"][1] + 0.5
    dy = mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64)
    dcomps = mem.to_components(events.drell_yan(2, 3)["obs"]).cuda()
    with pytest.raises(mem.MemError):
        mem.integrate_events(dcomps, dy, 4096, 2, flow=f, flow_mode=mem.MEM_FLOW_SEED_GRID)
    with pytest.raises(mem.MemError):
        mem.integrate_events(comps, p, 4096, 2, flow=f, flow_mode=7)
