"""ctypes binding of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, double-precision
implementation of the matrix element method integration written from the
paper (Schouten, DeAbreu, Stelzer, CPC 2014) and from the published
methods it relies on (VEGAS, Philox).  It shares no code with the HIP
library.  Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline
leg may import it.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

KIND_DY = 1
KIND_TT = 2
KIND_GENZ = 3
KIND_TT_SL = 4
KIND_TTH = 5
KIND_TTH_LL = 6
KIND_TTBB_LL = 7
# direct parametrisations of the t tbar, semileptonic and t tbar H dilepton
# integrals (closure checks of the mapped ones)
KIND_TT_DIRECT = 8
KIND_TT_SL_DIRECT = 9
KIND_TTH_LL_DIRECT = 10
# a lattice step function on [0,1]^2 (stratification check)
KIND_STEP = 11
NBINS = 64


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "sqrt_s", "m_t", "w_t", "m_w", "w_w", "alpha", "alpha_s", "g_fermi",
        "sigma_k", "tf_sigma", "r_lo", "r_hi", "m_lo", "m_hi",
        "lj_core", "lj_tail", "lj_ftail", "lj_r_lo", "lj_r_hi", "m_h", "w_h", "m_b")] + [
        ("pdf", ctypes.c_void_p)]


class _PdfGridC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("nq", ctypes.c_int), ("lx_min", ctypes.c_double),
                ("lx_max", ctypes.c_double), ("lq_min", ctypes.c_double), ("lq_max", ctypes.c_double),
                ("xf", ctypes.c_void_p)]


class PdfGrid:
    """x f(x, Q) of the flavours -5..5 on a uniform (ln x, ln Q) grid,
    values float32 [nq][nx][11]; bounds (lx_min, lx_max, lq_min, lq_max)."""

    def __init__(self, xf, bounds):
        self.xf = np.ascontiguousarray(xf, dtype=np.float32)
        nq, nx, nf = self.xf.shape
        assert nf == 11 and nx >= 2 and nq >= 2
        self.bounds = tuple(float(b) for b in bounds)
        self.c = _PdfGridC(nx, nq, *self.bounds, self.xf.ctypes.data)

    def ptr(self):
        return ctypes.cast(ctypes.pointer(self.c), ctypes.c_void_p)


def with_pdf(params, grid):
    """a copy of params whose integrands take their densities from grid
    (None: the toy densities)"""
    q = Params()
    ctypes.pointer(q)[0] = params
    q.pdf = grid.ptr().value if grid is not None else None
    q._grid = grid          # keep the table alive
    return q


def pdf_interp(grid, fl, x, Q):
    return lib().or_pdf_interp(ctypes.byref(grid.c), int(fl), float(x), float(Q))


def pdf_tabulate_toy(nx, nq, bounds):
    xf = np.zeros((nq, nx, 11), dtype=np.float32)
    g = PdfGrid(xf, bounds)
    lib().or_pdf_tabulate_toy(ctypes.byref(g.c), xf.ctypes.data)
    return g


class Result(ctypes.Structure):
    _fields_ = [("I", ctypes.c_double), ("sigma", ctypes.c_double),
                ("chi2dof", ctypes.c_double), ("n_iter_used", ctypes.c_int)]


def dy_params(**kw):
    """Drell-Yan configuration: sqrt(S) = 13 TeV, alpha = 1/137, 5% TF,
    r window [1 - 5 sigma, 1 + 5 sigma], truth window 60-120 GeV."""
    p = dict(sqrt_s=13000.0, m_t=172.5, w_t=1.4, m_w=80.4, w_w=2.1,
             alpha=1.0 / 137.0, alpha_s=0.118, g_fermi=1.1663787e-5,
             sigma_k=20.0, tf_sigma=0.05, r_lo=0.75, r_hi=1.25,
             m_lo=60.0, m_hi=120.0, lj_core=0.10, lj_tail=0.25, lj_ftail=0.2, lj_r_lo=0.1, lj_r_hi=2.25,
             m_h=125.0, w_h=0.00407, m_b=4.18)
    p.update(kw)
    return Params(**p)


def tt_params(**kw):
    """ttbar dilepton configuration: t (172.5, 1.4), W (80.4, 2.1), b-jet
    Gaussian TF 15 %, r window [0.25, 1.75], recoil sigma 20 GeV."""
    p = dict(sqrt_s=13000.0, m_t=172.5, w_t=1.4, m_w=80.4, w_w=2.1,
             alpha=1.0 / 137.0, alpha_s=0.118, g_fermi=1.1663787e-5,
             sigma_k=20.0, tf_sigma=0.15, r_lo=0.25, r_hi=1.75,
             m_lo=0.0, m_hi=0.0, lj_core=0.10, lj_tail=0.25, lj_ftail=0.2, lj_r_lo=0.1, lj_r_hi=2.25,
             m_h=125.0, w_h=0.00407, m_b=4.18)
    p.update(kw)
    return Params(**p)


def sl_params(**kw):
    """ttbar semileptonic: b-jets Gaussian 15 % (r in [0.25, 1.75]), light
    jets double Gaussian (10 %, 25 %, tail fraction 0.2; r in [0.1, 2.25])"""
    return tt_params(**kw)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        _LIB = ctypes.CDLL(path)
        _declare(_LIB)
    return _LIB


def _declare(L):
    D, I, U32, U64, I64, P = (ctypes.c_double, ctypes.c_int, ctypes.c_uint32,
                              ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p)
    sig = {
        "or_philox4x32_10": (None, [P, P, P]),
        "or_uniforms": (None, [U64, U32, U32, U32, U32, I, P]),
        "or_uniforms_block": (None, [U64, U32, U32, U32, U32, U32, I, P]),
        "or_vegas_map": (D, [P, I, P, P, P]),
        "or_vegas_uniform_grid": (None, [P, I]),
        "or_vegas_refine_dim": (None, [P, D, P]),
        "or_xf_u": (D, [D]), "or_xf_d": (D, [D]), "or_xf_qbar": (D, [D]), "or_xf_g": (D, [D]),
        "or_dy_integrand": (D, [P, P, P]),
        "or_qq_mumu_me2": (D, [P, P, P, P, D, D]),
        "or_dy_sigma_2d": (D, [P, I]),
        "or_dy_sigma_tau": (D, [P, I]),
        "or_tt_integrand": (D, [P, P, I, P, P]),
        "or_tt_parton_weight": (D, [P, P]),
        "or_pdf_interp": (D, [P, ctypes.c_int, D, D]),
        "or_pdf_tabulate_toy": (None, [P, P]),
        "or_decay_w_factor": (D, [P, D]),
        "or_ps_volume": (D, [I, D, U64, I64, P]),
        "or_top_width": (D, [P, U64, I64, P]),
        "or_tt_decayed_sigma": (D, [P, I, D, U64, I64, P]),
        "or_solve_dilepton": (I, [P, P, P, P, D, D, D, D, D, D, P, P, P]),
        "or_dilepton_residual": (None, [P, P, P, P, P, P, P]),
        "or_tt_me2_gg": (D, [P, P, P, P]),
        "or_tt_me2_qq": (D, [P, P, P, P]),
        "or_gg_ttbar_prod": (D, [D, P, P, P, P]),
        "or_qq_ttbar_prod": (D, [D, P, P, P, P]),
        "or_gg_ttbar_ward": (D, [D, P, P, P, P]),
        "or_top_decay_spinsum": (D, [D, P, P, P, P]),
        "or_integrate_one": (None, [I, P, P, I, U64, U32, I64, I, D, P, P, P, P]),
        "or_combine_iterations": (None, [P, P, I, I, I, P, P]),
        "or_strat_ns": (I, [I, I64]),
        "or_strat_allocate": (None, [I64, I64, P, I, P]),
        "or_strat_iteration": (None, [I, P, P, I, U64, U32, U32, I64, P, I, P, P, P, P, P, P]),
        "or_integrate_one_strat": (None, [I, P, P, I, U64, U32, I64, I, D, P, P, P]),
        "or_vegas_iteration": (None, [I, P, P, I, U64, U32, U32, I64, P, P, P, P]),
        "or_weight_at": (D, [I, P, P, I, P, P]),
        "or_integrate_events": (None, [I, P, P, I, I, U64, I64, I, D, D, P, P, P]),
        "or_integrate_events_iters": (None, [I, P, P, I, I, U64, I64, I, P, D, D, P, P, P]),
        "or_set_threads": (None, [I]), "or_max_threads": (I, []),
        "or_dims": (I, [I]), "or_nperm": (I, [I]),
        "or_bw_map": (D, [D, D, D, D, D, P]),
        "or_gauss_tf": (D, [D, D, D]),
        "or_genz_integrand": (D, [P]),
        "or_genz_exact": (D, []),
        "or_tt_semilep_integrand": (D, [P, P, I, I, P, P]),
        "or_semilep_perm": (None, [I, P, P, P, P]),
        "or_semilep_map": (D, [P, P, I, P, P]),
        "or_semilep_nu_z": (I, [P, D, D, D, P]),
        "or_dgauss_tf": (D, [D, D, D, D, D]),
        "or_flow_nparams": (I, []),
        "or_gg_tth_prod": (D, [D, P, P, P, P, P]),
        "or_gg_tth_ward": (D, [D, P, P, P, P, P]),
        "or_tth_soft_check": (D, [D, P, D]),
        "or_tth_me2_gg": (D, [P, P, P, P, P, P]),
        "or_tth_perm": (None, [I, P, P, P, P, P]),
        "or_tth_map": (D, [P, P, I, P, P]),
        "or_tth_integrand": (D, [P, P, I, I, P, P]),
        "or_gg_ttbb_prod": (D, [D, P, P, P, P, P, P]),
        "or_gg_ttbb_ward": (D, [D, P, P, P, P, P, P, I]),
        "or_gg_ttbb_prod_explicit": (D, [D, P, P, P, P, P, P]),
        "or_ttbb_me2_gg": (D, [P, P, P, P, P, P]),
        "or_colour_matrix_ttbb": (D, [I, I]),
        "or_colour_fabc": (D, [I, I, I]),
        "or_f2_perm": (None, [I, I, P]),
        "or_tthll_integrand": (D, [P, P, I, P, P]),
        "or_tt_direct_integrand": (D, [P, P, I, P]),
        "or_tt_semilep_direct_integrand": (D, [P, P, I, I, P, I]),
        "or_tthll_direct_integrand": (D, [P, P, I, P]),
        "or_ttbbll_integrand": (D, [P, P, I, P, P]),
        "or_f2_parton_weight": (D, [I, P, P]),
        "or_flow_forward": (D, [P, P, P, P]),
        "or_flow_inverse": (D, [P, P, P, P]),
        "or_flow_context": (None, [P, I, P]),
        "or_flow_nll_grad": (D, [P, I, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniforms(seed, k, it, event, perm, D, block0=0):
    u = np.zeros(D)
    lib().or_uniforms_block(seed, k, it, event, perm, block0, D, _ptr(u))
    return u


def uniform_grid(D):
    g = np.zeros((D, NBINS + 1))
    lib().or_vegas_uniform_grid(_ptr(g), D)
    return g


def vegas_map(grid, u):
    grid = _f64(grid)
    u = _f64(u)
    D = grid.shape[0]
    x = np.zeros(D)
    bins = np.zeros(D, dtype=np.int32)
    jac = lib().or_vegas_map(_ptr(grid), D, _ptr(u), _ptr(x), _ptr(bins))
    return x, jac, bins


def refine_dim(d, alpha, edges):
    d = _f64(d)
    e = _f64(edges).copy()
    lib().or_vegas_refine_dim(_ptr(d), alpha, _ptr(e))
    return e


def dy_integrand(p, ev, x):
    ev = _f64(ev)
    x = _f64(x)
    return lib().or_dy_integrand(ctypes.byref(p), _ptr(ev), _ptr(x))


def tt_integrand(p, ev, perm, x):
    ev = _f64(ev)
    x = _f64(x)
    ns = ctypes.c_int(0)
    v = lib().or_tt_integrand(ctypes.byref(p), _ptr(ev), perm, _ptr(x), ctypes.byref(ns))
    return v, ns.value


def ps_volume(n, sqrt_s, seed, n_points):
    err = ctypes.c_double()
    v = lib().or_ps_volume(n, sqrt_s, seed, n_points, ctypes.byref(err))
    return v, err.value


def tt_decayed_sigma(p, channel, sqrt_shat, seed, n_points):
    """partonic sigma(g g (0) / q qbar (1) -> t tbar -> b l nu b l nu) from
    the decayed matrix element over six-body phase space; (value, error)"""
    err = ctypes.c_double()
    v = lib().or_tt_decayed_sigma(ctypes.byref(p), channel, sqrt_shat, seed, n_points, ctypes.byref(err))
    return v, err.value


def top_width(p, seed, n_points):
    err = ctypes.c_double()
    v = lib().or_top_width(ctypes.byref(p), seed, n_points, ctypes.byref(err))
    return v, err.value


def tt_parton_weight(p, ev):
    """ev: [6, 4] b, bbar, l+, l-, nu, nubar"""
    return lib().or_tt_parton_weight(ctypes.byref(p), _ptr(_f64(ev)))


def sl_integrand(p, ev, perm, x, charge=0):
    ev = _f64(ev)
    x = _f64(x)
    ns = ctypes.c_int(0)
    v = lib().or_tt_semilep_integrand(ctypes.byref(p), _ptr(ev), charge, perm, _ptr(x), ctypes.byref(ns))
    return v, ns.value


def sl_perm(perm):
    vals = [ctypes.c_int() for _ in range(4)]
    lib().or_semilep_perm(perm, *[ctypes.byref(v) for v in vals])
    return tuple(v.value for v in vals)


def sl_map(p, ev, perm, x):
    ev, x = _f64(ev), _f64(x)
    E4 = np.zeros(4)
    jac = lib().or_semilep_map(ctypes.byref(p), _ptr(ev), perm, _ptr(x), _ptr(E4))
    return jac, E4


def sl_nu_z(l, nx, ny, q2):
    l = _f64(l)
    out = np.zeros(2)
    n = lib().or_semilep_nu_z(_ptr(l), nx, ny, q2, _ptr(out))
    return out[:n]


def solve_dilepton(b, bb, lp, lm, met, q2):
    b, bb, lp, lm = (_f64(a) for a in (b, bb, lp, lm))
    nu = np.zeros(16)
    nub = np.zeros(16)
    det = np.zeros(4)
    n = lib().or_solve_dilepton(_ptr(b), _ptr(bb), _ptr(lp), _ptr(lm), met[0], met[1],
                                q2[0], q2[1], q2[2], q2[3], _ptr(nu), _ptr(nub), _ptr(det))
    return nu[:4 * n].reshape(n, 4), nub[:4 * n].reshape(n, 4), det[:n]


def dilepton_q2(b, bb, lp, lm, nu, nub):
    arrs = [_f64(a) for a in (b, bb, lp, lm, nu, nub)]
    out = np.zeros(4)
    lib().or_dilepton_residual(*[_ptr(a) for a in arrs], _ptr(out))
    return out


def integrate_one(kind, p, ev, perm, seed, event_index, n_points, n_iter,
                  alpha=1.5, grid=None):
    ev = _f64(ev)
    D = lib().or_dims(kind)
    Is = np.zeros(n_iter)
    Vs = np.zeros(n_iter)
    g = None if grid is None else _f64(grid).copy()
    r = Result()
    lib().or_integrate_one(kind, ctypes.byref(p), _ptr(ev), perm, seed, event_index,
                           n_points, n_iter, alpha, None if g is None else _ptr(g),
                           _ptr(Is), _ptr(Vs), ctypes.byref(r))
    return r, Is, Vs, g


STRAT_HMAX = 16384


def combine_iterations(Is, Vs, first_kept=1, mode=0):
    """(I, sigma) of one integral from its iterations: mode 0 inverse-variance
    weights (VEGAS), mode 1 equal weights"""
    Is, Vs = _f64(Is), _f64(Vs)
    I, sg = ctypes.c_double(), ctypes.c_double()
    lib().or_combine_iterations(_ptr(Is), _ptr(Vs), len(Is), first_kept, mode, ctypes.byref(I), ctypes.byref(sg))
    return I.value, sg.value


def strat_ns(D, N):
    """hypercubes per dimension of adaptive stratified VEGAS"""
    return lib().or_strat_ns(D, N)


def strat_allocate(H, N, sig=None, first=False):
    nh = np.zeros(H, dtype=np.int64)
    sg = _f64(np.zeros(H) if sig is None else sig)
    lib().or_strat_allocate(H, N, _ptr(sg), 1 if first else 0, nh.ctypes.data)
    return nh


def strat_iteration(kind, p, ev, perm, seed, event_index, it, N, grid, ns, nh):
    """one stratified iteration: (I, var, per-hypercube deviations, bins,
    every point's weight in iteration order)"""
    ev, grid = _f64(ev), _f64(grid)
    D = lib().or_dims(kind)
    H = len(nh)
    nh = np.ascontiguousarray(nh, dtype=np.int64)
    I, var = ctypes.c_double(), ctypes.c_double()
    sig, bins, w = np.zeros(H), np.zeros(D * 64), np.zeros(N)
    lib().or_strat_iteration(kind, ctypes.byref(p), _ptr(ev), perm, seed, event_index, it, N, _ptr(grid), ns,
                             nh.ctypes.data, ctypes.byref(I), ctypes.byref(var), _ptr(sig), _ptr(bins), _ptr(w))
    return I.value, var.value, sig, bins, w


def integrate_one_strat(kind, p, ev, perm, seed, event_index, n_points, n_iter, alpha=1.5):
    ev = _f64(ev)
    Is, Vs = np.zeros(n_iter), np.zeros(n_iter)
    r = Result()
    lib().or_integrate_one_strat(kind, ctypes.byref(p), _ptr(ev), perm, seed, event_index, n_points, n_iter,
                                 alpha, _ptr(Is), _ptr(Vs), ctypes.byref(r))
    return r, Is, Vs


def vegas_iteration(kind, p, ev, perm, seed, event_index, it, n_points, grid):
    ev = _f64(ev)
    grid = _f64(grid)
    D = grid.shape[0]
    s1 = ctypes.c_double()
    s2 = ctypes.c_double()
    bins = np.zeros((D, NBINS))
    lib().or_vegas_iteration(kind, ctypes.byref(p), _ptr(ev), perm, seed, event_index, it,
                             n_points, _ptr(grid), ctypes.byref(s1), ctypes.byref(s2),
                             _ptr(bins))
    return s1.value, s2.value, bins


def weight_at(kind, p, ev, perm, grid, u):
    ev, grid, u = _f64(ev), _f64(grid), _f64(u)
    return lib().or_weight_at(kind, ctypes.byref(p), _ptr(ev), perm, _ptr(grid), _ptr(u))


def integrate_events(kind, p, events, seed, n_points, n_iter, alpha=1.5, sigma_norm=0.0):
    """P, err, status per event; n_iter is one count for every event or an
    array with one count per event"""
    ev = _f64(events)
    n_events, n_obj = ev.shape[0], ev.shape[1]
    P = np.zeros(n_events)
    err = np.zeros(n_events)
    st = np.zeros(n_events, dtype=np.int32)
    if np.ndim(n_iter) == 0:
        lib().or_integrate_events(kind, ctypes.byref(p), _ptr(ev), n_events, n_obj, seed,
                                  n_points, int(n_iter), alpha, sigma_norm, _ptr(P), _ptr(err), _ptr(st))
    else:
        its = np.ascontiguousarray(n_iter, dtype=np.int32)
        assert its.shape == (n_events,)
        lib().or_integrate_events_iters(kind, ctypes.byref(p), _ptr(ev), n_events, n_obj, seed,
                                        n_points, 0, its.ctypes.data_as(ctypes.c_void_p), alpha, sigma_norm,
                                        _ptr(P), _ptr(err), _ptr(st))
    return P, err, st


def set_threads(n):
    """OpenMP threads of later oracle calls (n < 1: the runtime default)"""
    lib().or_set_threads(int(n))


def max_threads():
    return int(lib().or_max_threads())


def _vec(a):
    return _f64(a)


def call4(name, *args):
    """call a function taking (double, p, p, p, p) or (p, p, p, p)"""
    conv = []
    keep = []
    for a in args:
        if isinstance(a, (float, int)):
            conv.append(float(a))
        elif isinstance(a, Params):
            conv.append(ctypes.byref(a))
        else:
            arr = _f64(a)
            keep.append(arr)
            conv.append(_ptr(arr))
    return getattr(lib(), name)(*conv)


# ------------------------------------------------------------ flow ----
FLOW_LAYERS, FLOW_H, FLOW_IN, FLOW_OUT = 6, 128, 28, 92
FLOW_PER_LAYER = FLOW_H * FLOW_IN + FLOW_H + FLOW_H * FLOW_H + FLOW_H + FLOW_OUT * FLOW_H + FLOW_OUT


def flow_init(seed, last_scale=0.0):
    """parameters with the shapes of the flow: W1, W2 ~ N(0, 1/fan_in),
    biases 0, the last layer scaled by last_scale (0: identity flow)"""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(FLOW_LAYERS):
        out.append(rng.standard_normal(FLOW_H * FLOW_IN) / np.sqrt(FLOW_IN))
        out.append(np.zeros(FLOW_H))
        out.append(rng.standard_normal(FLOW_H * FLOW_H) / np.sqrt(FLOW_H))
        out.append(np.zeros(FLOW_H))
        out.append(last_scale * rng.standard_normal(FLOW_OUT * FLOW_H) / np.sqrt(FLOW_H))
        out.append(last_scale * rng.standard_normal(FLOW_OUT))
    return np.concatenate(out)


def flow_forward(params, ctx, x):
    params, ctx, x = _f64(params), _f64(ctx), _f64(x)
    z = np.zeros(8)
    lq = lib().or_flow_forward(_ptr(params), _ptr(ctx), _ptr(x), _ptr(z))
    return z, lq


def flow_inverse(params, ctx, z):
    params, ctx, z = _f64(params), _f64(ctx), _f64(z)
    x = np.zeros(8)
    lq = lib().or_flow_inverse(_ptr(params), _ptr(ctx), _ptr(z), _ptr(x))
    return x, lq


def flow_context(ev, perm):
    ev = _f64(ev)
    c = np.zeros(24)
    lib().or_flow_context(_ptr(ev), perm, _ptr(c))
    return c


def flow_nll_grad(params, x, ctx, wt):
    params, x, ctx, wt = _f64(params), _f64(x), _f64(ctx), _f64(wt)
    g = np.zeros(len(params))
    loss = lib().or_flow_nll_grad(_ptr(params), len(wt), _ptr(x), _ptr(ctx), _ptr(wt), _ptr(g))
    return loss, g


# ------------------------------------------------------------ ttbar H ----
def gg_tth_prod(mt, k1, k2, pt, ptb, ph):
    a = [_f64(v) for v in (k1, k2, pt, ptb, ph)]
    return lib().or_gg_tth_prod(mt, *[_ptr(v) for v in a])


def gg_tth_ward(mt, k1, k2, pt, ptb, ph):
    a = [_f64(v) for v in (k1, k2, pt, ptb, ph)]
    return lib().or_gg_tth_ward(mt, *[_ptr(v) for v in a])


def tth_soft_check(mt, mom, delta):
    m = _f64(mom).reshape(-1)
    return lib().or_tth_soft_check(mt, _ptr(m), delta)


# ------------------------------------------------------ ttbar b bbar ----
def gg_ttbb_prod(mt, k1, k2, p3, p4, p5, p6):
    a = [_f64(v) for v in (k1, k2, p3, p4, p5, p6)]
    return lib().or_gg_ttbb_prod(mt, *[_ptr(v) for v in a])


def gg_ttbb_prod_explicit(mt, k1, k2, p3, p4, p5, p6):
    a = [_f64(v) for v in (k1, k2, p3, p4, p5, p6)]
    return lib().or_gg_ttbb_prod_explicit(mt, *[_ptr(v) for v in a])


def gg_ttbb_ward(mt, k1, k2, p3, p4, p5, p6, g):
    a = [_f64(v) for v in (k1, k2, p3, p4, p5, p6)]
    return lib().or_gg_ttbb_ward(mt, *[_ptr(v) for v in a], g)


def ttbb_me2_gg(p, k1, k2, mom, p5, p6):
    a = [_f64(v) for v in (k1, k2)]
    m = _f64(mom).reshape(-1)
    b = [_f64(v) for v in (p5, p6)]
    return lib().or_ttbb_me2_gg(ctypes.byref(p), _ptr(a[0]), _ptr(a[1]), _ptr(m), _ptr(b[0]), _ptr(b[1]))


def colour_matrix_ttbb():
    L = lib()
    return np.array([[L.or_colour_matrix_ttbb(d, e) for e in range(38)] for d in range(38)])


def colour_fabc():
    L = lib()
    return np.array([[[L.or_colour_fabc(a, b, c) for c in range(8)] for b in range(8)] for a in range(8)])


def f2_perm(kind, perm):
    """event rows of (b, bbar, pair jet 1, pair jet 2) for an assignment"""
    rows = np.zeros(4, dtype=np.int32)
    lib().or_f2_perm(kind, perm, _ptr(rows))
    return tuple(int(r) for r in rows)


def tthll_integrand(p, ev, perm, x):
    ev, x = _f64(ev), _f64(x)
    ns = ctypes.c_int(0)
    v = lib().or_tthll_integrand(ctypes.byref(p), _ptr(ev), perm, _ptr(x), ctypes.byref(ns))
    return v, ns.value


SL_DIRECT_EB = 1
SL_DIRECT_NU = 2
SL_DIRECT_EBH = 4


def tt_direct_integrand(p, ev, perm, x):
    """t tbar dilepton integrand in (nu_x, nu_y, nu_z, nubar_z) directly"""
    ev, x = _f64(ev), _f64(x)
    return lib().or_tt_direct_integrand(ctypes.byref(p), _ptr(ev), perm, _ptr(x))


def sl_direct_integrand(p, ev, perm, x, mode, charge=0):
    """semileptonic integrand with the energy of light jet b (SL_DIRECT_EB),
    of the hadronic top's b (SL_DIRECT_EBH) and/or nu_z (SL_DIRECT_NU) as
    variables"""
    ev, x = _f64(ev), _f64(x)
    return lib().or_tt_semilep_direct_integrand(ctypes.byref(p), _ptr(ev), charge, perm, _ptr(x), mode)


def tthll_direct_integrand(p, ev, perm, x):
    """t tbar H dilepton integrand with x7 the second Higgs jet's r"""
    ev, x = _f64(ev), _f64(x)
    return lib().or_tthll_direct_integrand(ctypes.byref(p), _ptr(ev), perm, _ptr(x))


def ttbbll_integrand(p, ev, perm, x):
    ev, x = _f64(ev), _f64(x)
    ns = ctypes.c_int(0)
    v = lib().or_ttbbll_integrand(ctypes.byref(p), _ptr(ev), perm, _ptr(x), ctypes.byref(ns))
    return v, ns.value


def f2_parton_weight(kind, p, ev):
    return lib().or_f2_parton_weight(kind, ctypes.byref(p), _ptr(_f64(ev)))


def tth_perm(perm):
    v = [ctypes.c_int(0) for _ in range(5)]
    lib().or_tth_perm(perm, *[ctypes.byref(x) for x in v])
    return tuple(x.value for x in v)     # i_h1, i_h2, i_bl, i_bh, o


def tth_map(p, ev, perm, x):
    ev, x = _f64(ev), _f64(x)
    E6 = np.zeros(6)
    jac = lib().or_tth_map(ctypes.byref(p), _ptr(ev), perm, _ptr(x), _ptr(E6))
    return jac, E6


def tth_integrand(p, ev, perm, x, charge=0):
    ev, x = _f64(ev), _f64(x)
    ns = ctypes.c_int(0)
    v = lib().or_tth_integrand(ctypes.byref(p), _ptr(ev), charge, perm, _ptr(x), ctypes.byref(ns))
    return v, ns.value
