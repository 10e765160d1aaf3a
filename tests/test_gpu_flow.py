"""The learned proposal on the GPU (libmem flow kernels) vs the FP64 oracle.

Bars.  The GPU evaluates the two 128-wide layers of every coupling MLP as
BF16 products with FP32 accumulation; the tests give both sides the same
BF16-representable W2, W3 (and FP32 W1, biases), so the remaining
difference is the rounding of the hidden activations.
 * MEM_FLOW_BF16X2 (activations as hi + lo BF16 terms, relative error
   ~2^-17): pointwise bars at FP32 level, |dx| <= 1e-4 and |d log q| <=
   5e-3 over six layers of a network with outputs of order one; this is the
   check of the kernels' structure (indexing, layouts, masks, reversal).
 * MEM_FLOW_BF16 (activations rounded to BF16, relative 2^-9 each): the
   rounding propagated through six layers moves x by ~1e-4 and log q by
   ~1e-3 even for a near-identity network (weights scaled by 0.1), and more
   as the network grows; compared at that scale with median/max bars of
   5e-4/3e-3 (x) and 5e-3/5e-2 (log q).  Both variants define a valid
   density (each coupling layer stays a bijection whose Jacobian the
   kernels form exactly for their own arithmetic), which is what keeps the
   estimator unbiased.
 * gradients: cosine > 0.999 and relative L2 < 2e-2 (the backward products
   round their operands to BF16).
The estimator is checked by the ESS fallback (bit-equal to plain VEGAS),
by the gain of a trained flow over the untrained one and by a pull test
against VEGAS.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from synth import events

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PER = oracle.FLOW_PER_LAYER
# offsets inside one layer: W1, b1, W2, b2, W3, b3
OFF = [0, 128 * 28, 128 * 28 + 128, 128 * 28 + 128 + 128 * 128, 128 * 28 + 256 + 128 * 128,
       128 * 28 + 256 + 128 * 128 + 92 * 128, PER]


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


def bf16_round(a):
    """nearest-even BF16 value of each float32"""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return b.astype(np.uint32).view(np.float32)


def flow_params(seed, scale, bias=0.0):
    """oracle-initialised parameters, FP32, with W2 and W3 BF16-exact"""
    p = oracle.flow_init(seed, scale).astype(np.float32)
    rng = np.random.default_rng(seed + 1000)
    for l in range(6):
        o = l * PER
        for blk in (2, 4):
            sl = slice(o + OFF[blk], o + OFF[blk + 1])
            p[sl] = bf16_round(p[sl])
        for blk in (1, 3):      # small biases exercise those gradients
            sl = slice(o + OFF[blk], o + OFF[blk + 1])
            p[sl] = (bias * rng.standard_normal(OFF[blk + 1] - OFF[blk])).astype(np.float32)
    return p


def dilepton(n, seed):
    d = events.ttbar_dilepton(n, seed)
    return d, torch.as_tensor(np.ascontiguousarray(d["obs"].transpose(2, 1, 0)), dtype=torch.float64).cuda()


def contexts(mem, comps, ev_idx, perm_idx):
    n = len(ev_idx)
    ctx = torch.empty((n, 24), dtype=torch.float32, device="cuda")
    mem.flow_context(comps, dev(ev_idx, torch.int32), dev(perm_idx, torch.int32), ctx)
    torch.cuda.synchronize()
    return ctx


def oracle_ctx(d, e, perm):
    return oracle.flow_context(d["obs"][e], perm).astype(np.float32).astype(np.float64)


# ----------------------------------------------------------------- context --
def test_flow_context_matches_oracle(mem):
    d, comps = dilepton(7, 31)
    ev_idx = np.repeat(np.arange(7), 2)
    perm_idx = np.tile([0, 1], 7)
    say("flow context 7 events x 2 permutations")
    got = contexts(mem, comps, ev_idx, perm_idx).cpu().numpy()
    for i, (e, pm) in enumerate(zip(ev_idx, perm_idx)):
        want = oracle.flow_context(d["obs"][e], pm)
        assert np.allclose(got[i], want, rtol=3e-7, atol=1e-7), (i, got[i], want)


# ---------------------------------------------------------------- sampling --
def sample(mem, flow, ctx, ev_idx, perm_idx, n_per, seed, it):
    n = len(ev_idx)
    x = torch.empty((n, n_per, 8), dtype=torch.float32, device="cuda")
    lq = torch.empty((n, n_per), dtype=torch.float32, device="cuda")
    flow.sample(ctx, dev(ev_idx, torch.int32), dev(perm_idx, torch.int32), n_per, seed, it, x, lq)
    torch.cuda.synchronize()
    return x.cpu().numpy(), lq.cpu().numpy()


def base_point(seed, k, it, e, perm):
    u = oracle.uniforms(seed, k, it, e, perm, 8, block0=8)
    return np.minimum(u.astype(np.float32), np.float32(1.0 - 2.0**-24)).astype(np.float64)


def test_flow_identity_sampling(mem):
    """zero parameters: x is z in reversed coordinate order (the fixed
    reversal before layer 3) and log q = 0, up to FP32 rounding of the knots"""
    d, comps = dilepton(3, 5)
    ev_idx, perm_idx = np.array([0, 1, 2]), np.array([0, 1, 1])
    ctx = contexts(mem, comps, ev_idx, perm_idx)
    flow = mem.Flow()
    say("flow identity sampling 3 x 300")
    x, lq = sample(mem, flow, ctx, ev_idx, perm_idx, 300, 99, 0)
    for i in range(3):
        for k in range(0, 300, 7):
            z = base_point(99, k, 0, ev_idx[i], perm_idx[i])
            assert np.allclose(x[i, k], z[::-1], atol=2e-6), (i, k, x[i, k], z)
    assert np.max(np.abs(lq)) < 2e-5


# mode, weight scale, bias scale, bars on |dx| and |d log q|: (median, 99th
# percentile); the largest deviation may be 10 x the percentile bar.  The
# inverse direction divides by the spline slope, which can be as small as
# 1e-3, so single points amplify the FP32/BF16 rounding of theta.
SAMPLE_CASES = [
    ("x2", 0.6, 0.1, 1e-5, 1e-4, 2e-4, 5e-3),
    ("bf16", 0.1, 0.0, 5e-4, 3e-3, 5e-3, 5e-2),
]


def within(a, med, p99):
    return np.median(a) < med and np.quantile(a, 0.99) < p99 and a.max() < 10 * p99


@pytest.mark.parametrize("mode,scale,bias,mdx,xdx,mdl,xdl", SAMPLE_CASES)
def test_flow_sample_matches_oracle(mem, mode, scale, bias, mdx, xdx, mdl, xdl):
    d, comps = dilepton(4, 8)
    ev_idx, perm_idx = np.array([0, 1, 2, 3]), np.array([1, 0, 1, 0])
    ctx = contexts(mem, comps, ev_idx, perm_idx)
    p = flow_params(21, scale, bias=bias)
    flow = mem.Flow(mem.MEM_FLOW_BF16X2 if mode == "x2" else mem.MEM_FLOW_BF16)
    flow.set_params(torch.from_numpy(p))
    n_per, seed, it = 200, 0x5EED, 3       # 200 = one 128-point tile + a ragged 72
    say(f"flow sample 4 integrals x {n_per}")
    x, lq = sample(mem, flow, ctx, ev_idx, perm_idx, n_per, seed, it)
    P = p.astype(np.float64)
    dx, dl = [], []
    for i in range(4):
        c = oracle_ctx(d, ev_idx[i], perm_idx[i])
        for k in range(n_per):
            z = base_point(seed, k, it, ev_idx[i], perm_idx[i])
            xo, lqo = oracle.flow_inverse(P, c, z)
            dx.append(np.max(np.abs(x[i, k] - xo)))
            dl.append(abs(lq[i, k] - lqo))
    dx, dl = np.array(dx), np.array(dl)
    say(f"{mode}: |dx| median {np.median(dx):.2e} p99 {np.quantile(dx, 0.99):.2e} max {dx.max():.2e}; "
        f"|dlogq| median {np.median(dl):.2e} p99 {np.quantile(dl, 0.99):.2e} max {dl.max():.2e}")
    assert within(dx, mdx, xdx) and within(dl, mdl, xdl)
    # the GPU's own forward pass at its samples returns their log q
    sint = np.repeat(np.arange(4), n_per).astype(np.int32)
    lq2 = torch.empty(4 * n_per, dtype=torch.float32, device="cuda")
    flow.log_prob(ctx, dev(sint, torch.int32), dev(x.reshape(-1, 8), torch.float32), lq2)
    torch.cuda.synchronize()
    dself = np.abs(lq2.cpu().numpy() - lq.reshape(-1))
    say(f"{mode}: forward log q at the samples vs their sampling log q: median {np.median(dself):.2e} "
        f"max {dself.max():.2e}")
    # two GPU passes (inverse, then forward), each within the oracle bar
    assert np.median(dself) < 2 * mdl and np.quantile(dself, 0.9) < 2 * xdl


@pytest.mark.parametrize("mode,scale,bias,mdx,xdx,mdl,xdl", SAMPLE_CASES)
def test_flow_log_prob_matches_oracle(mem, mode, scale, bias, mdx, xdx, mdl, xdl):
    d, comps = dilepton(5, 9)
    ev_idx, perm_idx = np.arange(5), np.array([0, 1, 0, 1, 1])
    ctx = contexts(mem, comps, ev_idx, perm_idx)
    p = flow_params(22, scale, bias=bias)
    flow = mem.Flow(mem.MEM_FLOW_BF16X2 if mode == "x2" else mem.MEM_FLOW_BF16)
    flow.set_params(torch.from_numpy(p))
    rng = np.random.default_rng(4)
    n = 333                                # three tiles, the last ragged
    x = rng.random((n, 8)).astype(np.float32)
    x[:4] = [[0.0] * 8, [0.5] * 8, [1.0 - 2**-24] * 8, [1e-7] * 8]
    sint = rng.integers(0, 5, n).astype(np.int32)
    lq = torch.empty(n, dtype=torch.float32, device="cuda")
    say(f"flow log_prob {n} points")
    flow.log_prob(ctx, dev(sint, torch.int32), dev(x, torch.float32), lq)
    torch.cuda.synchronize()
    got = lq.cpu().numpy()
    P = p.astype(np.float64)
    want = np.array([oracle.flow_forward(P, oracle_ctx(d, ev_idx[s], perm_idx[s]), xi.astype(np.float64))[1]
                     for xi, s in zip(x, sint)])
    err = np.abs(got - want)
    say(f"{mode}: |dlogq| median {np.median(err):.2e} p99 {np.quantile(err, 0.99):.2e} max {err.max():.2e}")
    assert within(err, mdl, xdl)


# ---------------------------------------------------------------- training --
@pytest.mark.parametrize("mode,scale,bias,min_cos", [("x2", 0.5, 0.1, 0.999), ("bf16", 0.1, 0.0, 0.99)])
def test_flow_gradient_matches_oracle(mem, mode, scale, bias, min_cos):
    d, comps = dilepton(4, 10)
    ev_idx, perm_idx = np.array([0, 1, 2, 3]), np.array([0, 0, 1, 1])
    ctx = contexts(mem, comps, ev_idx, perm_idx)
    p = flow_params(23, scale, bias=bias)
    flow = mem.Flow(mem.MEM_FLOW_BF16X2 if mode == "x2" else mem.MEM_FLOW_BF16)
    flow.set_params(torch.from_numpy(p))
    rng = np.random.default_rng(5)
    n = 300
    x = (0.01 + 0.98 * rng.random((n, 8))).astype(np.float32)
    sint = rng.integers(0, 4, n).astype(np.int32)
    wt = rng.random(n).astype(np.float32)
    wt /= wt.sum()
    g = torch.zeros(oracle.FLOW_LAYERS * PER, dtype=torch.float32, device="cuda")
    say(f"flow gradient {n} samples")
    loss = flow.train_step(ctx, dev(sint, torch.int32), dev(x, torch.float32), dev(wt, torch.float32), lr=0.0,
                           grad_out=g)
    torch.cuda.synchronize()
    got = g.cpu().numpy().astype(np.float64)
    cx = np.array([oracle_ctx(d, ev_idx[s], perm_idx[s]) for s in sint])
    lo, want = oracle.flow_nll_grad(p.astype(np.float64), x.astype(np.float64), cx, wt.astype(np.float64))
    say(f"loss gpu {loss:.6g} oracle {lo:.6g}")
    assert loss == pytest.approx(lo, rel=1e-2, abs=1e-3)

    def compare(a, b, what):
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        rel = float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300))
        say(f"{what}: cosine {cos:.6f} rel L2 {rel:.3e}")
        return cos, rel

    cos, rel = compare(got, want, f"{mode}: all parameters")
    assert cos > min_cos and rel < 2e-2
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    for l in range(6):
        for blk in range(6):
            sl = slice(l * PER + OFF[blk], l * PER + OFF[blk + 1])
            if np.linalg.norm(want[sl]) == 0.0:
                continue
            cos, rel = compare(got[sl], want[sl], f"{mode}: layer {l} {names[blk]}")
            assert cos > 0.99 and rel < 5e-2, (l, names[blk])


def test_flow_adam_first_step(mem):
    """the first Adam step moves every parameter with |g| >> eps by -lr sign(g)"""
    d, comps = dilepton(2, 11)
    ctx = contexts(mem, comps, np.array([0, 1]), np.array([0, 1]))
    p = flow_params(24, 0.3)
    flow = mem.Flow()
    flow.set_params(torch.from_numpy(p))
    rng = np.random.default_rng(6)
    n = 256
    x = dev(rng.random((n, 8)), torch.float32)
    sint = dev(rng.integers(0, 2, n), torch.int32)
    wt = dev(np.full(n, 1.0 / n), torch.float32)
    g = torch.zeros(oracle.FLOW_LAYERS * PER, dtype=torch.float32, device="cuda")
    lr = 1e-3
    say("flow Adam step")
    flow.train_step(ctx, sint, x, wt, lr=lr, grad_out=g)
    torch.cuda.synchronize()
    gg = g.cpu().numpy()
    p1 = flow.get_params().numpy()
    big = np.abs(gg) > 1e-5
    assert big.sum() > 10000
    step = (p1 - p)[big]
    assert np.allclose(step, -lr * np.sign(gg[big]), rtol=2e-2, atol=2e-7)
    assert np.all(p1[~big & (gg == 0)] == p[~big & (gg == 0)])


def test_vegas_capture_matches_oracle(mem):
    from test_gpu_parity import ill_conditioned
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    po = oracle.tt_params()
    d, comps = dilepton(3, 12)
    ev_idx, perm_idx = np.array([0, 1, 2]), np.array([0, 1, 0])
    rng = np.random.default_rng(7)
    grids = np.empty((3, 8, 65))
    for i in range(3):
        for dd in range(8):
            grids[i, dd] = np.concatenate([[0.0], np.sort(rng.random(63)), [1.0]])
    n_per, seed, it = 700, 31, 2
    x = torch.empty((3, n_per, 8), dtype=torch.float32, device="cuda")
    w = torch.empty((3, n_per), dtype=torch.float32, device="cuda")
    say(f"capture 3 integrals x {n_per}")
    mem.vegas_capture(p, comps, dev(ev_idx, torch.int32), dev(perm_idx, torch.int32), dev(grids), n_per, seed, it,
                      x, w, normalise=0)
    torch.cuda.synchronize()
    xg, wg = x.cpu().numpy(), w.cpu().numpy()
    n_cmp = n_flag = 0
    for i in range(3):
        for k in range(n_per):
            u = oracle.uniforms(seed, k, it, ev_idx[i], perm_idx[i], 8)
            xo, _, _ = oracle.vegas_map(grids[i], u)
            assert np.array_equal(xg[i, k], xo.astype(np.float32)), (i, k)
            wo = oracle.weight_at(oracle.KIND_TT, po, d["obs"][ev_idx[i]], perm_idx[i], grids[i], u)
            if wo == 0.0 and wg[i, k] == 0.0:
                continue
            # FP32 integrand bar (1e-5) plus the rounding of w to FP32
            if abs(wg[i, k] - wo) > 2e-5 * abs(wo):
                f = wo / oracle.vegas_map(grids[i], u)[1]
                assert ill_conditioned(po, d["obs"][ev_idx[i]], perm_idx[i], xo, f), (i, k, wg[i, k], wo)
                n_flag += 1
                continue
            n_cmp += 1
    say(f"compared {n_cmp} nonzero weights, {n_flag} flagged ill-conditioned")
    assert n_cmp > 20 and n_flag <= 0.01 * n_cmp + 2
    # normalised per integral
    mem.vegas_capture(p, comps, dev(ev_idx, torch.int32), dev(perm_idx, torch.int32), dev(grids), n_per, seed, it,
                      x, w, normalise=1)
    torch.cuda.synchronize()
    s = w.cpu().numpy().astype(np.float64).sum(axis=1)
    assert np.allclose(s, 1.0, rtol=1e-5)


@pytest.mark.parametrize("kind", ["dy", "sl", "tth"])
def test_vegas_capture_every_process(mem, kind):
    """capture of the other process kinds on adapted grids: x bit-equal to
    the oracle's VEGAS map, w = f J within the FP32 integrand bar (points
    whose oracle value moves by more than a tenth of the bar under 1-ulp
    changes of x are counted and excluded).  t tbar H weights lie near the
    bottom of the FP32 range (~1e-40): they are compared after rounding the
    oracle's weight to FP32, with an absolute slack of two subnormal steps."""
    n_obj, D, npm = {"dy": (2, 2, 1), "sl": (5, 7, 12), "tth": (7, 9, 24)}[kind]
    if kind == "dy":
        p = mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64)
        po, okind, obs, bar = oracle.dy_params(), oracle.KIND_DY, events.drell_yan(2, 81)["obs"], 1e-6
        f_or = lambda ev, perm, x: oracle.dy_integrand(po, ev, x)
    else:
        p = mem.Process(mem.MEM_TT_SEMILEPTON if kind == "sl" else mem.MEM_TTH_SEMILEPTON, precision=mem.MEM_FP32)
        po, bar = oracle.tt_params(), 2e-5
        okind = oracle.KIND_TT_SL if kind == "sl" else oracle.KIND_TTH
        obs = (events.ttbar_semileptonic(2, 82) if kind == "sl" else events.ttbar_higgs(2, 83))["obs"]
        fn = oracle.sl_integrand if kind == "sl" else oracle.tth_integrand
        f_or = lambda ev, perm, x: fn(po, ev, perm, x)[0]
    comps = torch.as_tensor(np.ascontiguousarray(obs[:, :n_obj, :].transpose(2, 1, 0))).cuda()
    charge = torch.as_tensor(obs[:, n_obj, 0].astype(np.int32) if kind != "dy" else np.ones(2, np.int32)).cuda()
    grids = torch.empty((2 * npm, D, 65), dtype=torch.float64, device="cuda")
    mem.integrate_events(comps, p, 2048 * npm, 3, seed=41, grid_out=grids, charge=charge)
    # integrals (event 0, perm 0) and (event 1, last perm)
    sel = [0, 2 * npm - 1]
    ev_idx, perm_idx = np.array([0, 1]), np.array([0, npm - 1])
    g = grids[sel].contiguous()
    n_per, seed, it = 600, 43, 3
    x = torch.empty((2, n_per, D), dtype=torch.float32, device="cuda")
    w = torch.empty((2, n_per), dtype=torch.float32, device="cuda")
    say(f"capture {kind}: 2 integrals x {n_per}")
    mem.vegas_capture(p, comps, dev(ev_idx, torch.int32), dev(perm_idx, torch.int32), g, n_per, seed, it, x, w,
                      normalise=0, charge=charge)
    torch.cuda.synchronize()
    xg, wg, gh = x.cpu().numpy(), w.cpu().numpy(), g.cpu().numpy()
    n_cmp = n_flag = 0
    for i in range(2):
        ev = obs[ev_idx[i]]
        for k in range(n_per):
            u = oracle.uniforms(seed, k, it, ev_idx[i], perm_idx[i], D)
            xo, jac, _ = oracle.vegas_map(gh[i], u)
            assert np.array_equal(xg[i, k], xo.astype(np.float32)), (i, k)
            wo = oracle.weight_at(okind, po, ev, perm_idx[i], gh[i], u)
            assert np.isfinite(wg[i, k]), (i, k)
            if wo == 0.0 and wg[i, k] == 0.0:
                continue
            if abs(float(wg[i, k]) - float(np.float32(wo))) <= bar * abs(wo) + 2 * 2.0 ** -149:
                n_cmp += 1
                continue
            if abs(wg[i, k] - wo) > bar * abs(wo):
                f0 = wo / jac
                moved = False
                for xp in (np.nextafter(xo, 1.0), np.nextafter(xo, 0.0), xo * (1 + 2e-16)):
                    f1 = f_or(ev, perm_idx[i], np.clip(xp, 0.0, 1.0 - 2 ** -53))
                    moved |= abs(f1 - f0) > 0.1 * bar * max(abs(f0), 1e-300)
                assert moved, (kind, i, k, wg[i, k], wo)
                n_flag += 1
                continue
            n_cmp += 1
    say(f"{kind}: compared {n_cmp} nonzero weights, {n_flag} flagged ill-conditioned")
    assert n_cmp > 20 and n_flag <= 0.02 * n_cmp + 2


# --------------------------------------------------------------- estimator --
def test_flow_fallback_is_vegas(mem):
    """an ESS threshold no proposal can meet sends every event to VEGAS:
    results bit-equal to a plain VEGAS call, status FLOW_FALLBACK"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    d, comps = dilepton(5, 13)
    flow = mem.Flow()
    say("flow fallback: 5 events x 3000 x 3")
    P0, E0, S0 = mem.integrate_events(comps, p, 3000, 3, seed=17)
    P1, E1, S1 = mem.integrate_events(comps, p, 3000, 3, seed=17, flow=flow, ess_threshold=2.0)
    torch.cuda.synchronize()
    assert torch.equal(P0, P1) and torch.equal(E0, E1)
    s0, s1 = S0.cpu().numpy(), S1.cpu().numpy()
    assert np.all(s1[s0 == 0] == mem.MEM_EV_FLOW_FALLBACK) and np.all(s1[s0 != 0] == s0[s0 != 0])


def ess_from_iter(rec, N):
    I, var = rec[..., 0], rec[..., 1]
    den = var * (N - 1) + I * I
    return np.where(den > 0, I * I / np.maximum(den, 1e-300), 0.0)


def test_flow_trained_gain_and_pull(mem):
    """Train on VEGAS samples of 8 events, then: ESS/N of the trained flow
    well above the untrained (uniform) proposal's, and its estimates agree
    with VEGAS within the combined MC error"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    n_ev = 8
    d, comps = dilepton(n_ev, 14)
    n_int = 2 * n_ev
    say(f"flow training data: VEGAS {n_ev} events x 16384 x 5, capture 4096 per integral")
    grids = torch.zeros((n_int, 8, 65), dtype=torch.float64, device="cuda")
    Pv, Ev, Sv = mem.integrate_events(comps, p, 16384, 5, seed=3, grid_out=grids)
    ev_idx = np.repeat(np.arange(n_ev), 2)
    perm_idx = np.tile([0, 1], n_ev)
    n_per = 4096
    x = torch.empty((n_int, n_per, 8), dtype=torch.float32, device="cuda")
    w = torch.empty((n_int, n_per), dtype=torch.float32, device="cuda")
    e_t, p_t = dev(ev_idx, torch.int32), dev(perm_idx, torch.int32)
    mem.vegas_capture(p, comps, e_t, p_t, grids, n_per, 7, 0, x, w, normalise=1)
    ctx = contexts(mem, comps, ev_idx, perm_idx)
    sint = dev(np.repeat(np.arange(n_int), n_per), torch.int32)
    xs, ws = x.reshape(-1, 8).contiguous(), w.reshape(-1).contiguous()
    flow = mem.Flow()
    losses = []
    say("flow training: 300 Adam steps on 65536 samples")
    for step in range(300):
        loss = flow.train_step(ctx, sint, xs, ws, lr=2e-3, want_loss=(step % 50 == 0 or step == 299))
        if loss is not None:
            losses.append(loss)
            say(f"step {step} loss {loss:.5f}")
    assert losses[-1] < losses[0] - 0.5
    # ESS/N of a batch: trained vs untrained (threshold off)
    N = 8192
    it_rec = {}
    for name, f in (("untrained", mem.Flow()), ("trained", flow)):
        rec = torch.zeros((2, n_int, 2), dtype=torch.float64, device="cuda")
        say(f"flow integrate ({name}) {n_ev} events x {2 * N} x 2")
        mem.integrate_events(comps, p, 2 * N, 2, seed=5, flow=f, ess_threshold=1e-12, iter_out=rec)
        torch.cuda.synchronize()
        it_rec[name] = ess_from_iter(rec.cpu().numpy(), N)
        say(f"{name} ESS/N per integral", np.round(it_rec[name][0], 4))
    gain = np.median(it_rec["trained"][0]) / max(np.median(it_rec["untrained"][0]), 1e-12)
    say(f"median ESS/N gain {gain:.1f}")
    assert gain > 3.0
    # pull test against VEGAS at a comparable error
    Pf, Ef, Sf = mem.integrate_events(comps, p, 2 * N, 6, seed=8, flow=flow, ess_threshold=1e-12)
    Pv, Ev, Sv = mem.integrate_events(comps, p, 32768, 8, seed=9)
    torch.cuda.synchronize()
    Pf, Ef, Pv, Ev = (t.cpu().numpy() for t in (Pf, Ef, Pv, Ev))
    pl = (Pf - Pv) / np.sqrt(Ef ** 2 + Ev ** 2)
    Sf = Sf.cpu().numpy()
    say("flow rel err", np.round(Ef / Pf, 4), "pulls", np.round(pl, 2), "status", Sf)
    assert np.all(np.abs(pl) < 3.5)
    # a first batch with only zero weights (ESS 0) hands the event to VEGAS
    assert np.all((Sf == 0) | (Sf == mem.MEM_EV_FLOW_FALLBACK))
