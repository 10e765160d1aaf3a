"""Python binding of libmem, the MI355X matrix element method integrator.

Argument marshalling only: every step of the integration runs in the HIP
kernels of libmem.so (see include/mem.h for the C ABI).  PyTorch supplies
device memory and streams.  The library is loaded from this directory;
importing the binding fails loudly when it has not been built.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmem.so")

MEM_OK, MEM_EINVAL, MEM_ENOMEM, MEM_EDEVICE, MEM_EUNSUPPORTED = range(5)
MEM_DY_QQ_GAMMA_MUMU, MEM_TT_DILEPTON, MEM_TT_SEMILEPTON, MEM_TTH_SEMILEPTON = 1, 2, 3, 4
MEM_TTH_DILEPTON, MEM_TTBB_DILEPTON = 5, 6
MEM_FP64, MEM_FP32 = 0, 1
MEM_TF_DELTA, MEM_TF_UNIFORM, MEM_TF_GAUSS, MEM_TF_DGAUSS = range(4)
MEM_OBJ_MUON, MEM_OBJ_LEPTON, MEM_OBJ_BJET, MEM_OBJ_LJET, MEM_OBJ_NEUTRINO = range(5)
MEM_EV_OK, MEM_EV_ZERO_INTEGRAND, MEM_EV_NOT_CONVERGED, MEM_EV_NONFINITE, MEM_EV_FLOW_FALLBACK = range(5)
FLOW_NPARAMS = 192552
MEM_ALLOC_EQUAL, MEM_ALLOC_NEYMAN = 0, 1
MEM_FLOW_BF16, MEM_FLOW_BF16X2 = 0, 1
FLOW_CONTEXT = 24

# every symbol include/mem.h declares
EXPORTS = ("mem_create_process", "mem_set_transfer_functions", "mem_destroy_process",
           "mem_process_shape", "mem_integrate_events", "mem_integrate_events_noalloc", "mem_train_proposal", "mem_set_proposal",
           "mem_flow_save", "mem_flow_load", "mem_uniforms", "mem_eval_points",
           "mem_vegas_refine", "mem_vegas_capture", "mem_flow_create", "mem_flow_destroy",
           "mem_flow_set_params", "mem_flow_get_params", "mem_flow_context", "mem_flow_sample",
           "mem_flow_log_prob", "mem_flow_train_step", "mem_autotune", "mem_tuning_load",
           "mem_process_chunk_points", "mem_process_set_launch", "mem_process_waves", "mem_parton_weights", "mem_set_pdf_grid", "mem_toy_pdf_table",
           "mem_discriminant", "mem_checkpoint_create", "mem_checkpoint_destroy", "mem_checkpoint_save",
           "mem_checkpoint_load", "mem_checkpoint_iterations", "mem_status_string", "mem_last_error")


class ProcessDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("precision", ctypes.c_int32), ("sqrt_s", ctypes.c_double),
                ("m_top", ctypes.c_double), ("w_top", ctypes.c_double), ("m_w", ctypes.c_double),
                ("w_w", ctypes.c_double), ("m_h", ctypes.c_double), ("w_h", ctypes.c_double),
                ("alpha", ctypes.c_double), ("alpha_s", ctypes.c_double), ("g_fermi", ctypes.c_double),
                ("sigma_k", ctypes.c_double), ("m_lo", ctypes.c_double), ("m_hi", ctypes.c_double),
                ("sigma_norm", ctypes.c_double), ("m_b", ctypes.c_double)]


class TFDesc(ctypes.Structure):
    _fields_ = [("obj_class", ctypes.c_int32), ("kind", ctypes.c_int32), ("sigma_core", ctypes.c_double),
                ("sigma_tail", ctypes.c_double), ("f_tail", ctypes.c_double), ("window", ctypes.c_double),
                ("r_min", ctypes.c_double)]


class Events(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int32), ("n_obj", ctypes.c_int32), ("E", ctypes.c_void_p),
                ("px", ctypes.c_void_p), ("py", ctypes.c_void_p), ("pz", ctypes.c_void_p),
                ("charge", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class FlowDesc(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("vegas_iter", ctypes.c_int32), ("vegas_points", ctypes.c_int64),
                ("capture", ctypes.c_int32), ("batch", ctypes.c_int32), ("epochs", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("lr_max", ctypes.c_double), ("lr_min", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("stream", ctypes.c_void_p), ("loss_out", ctypes.c_void_p)]


class IntegrateOpts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("alpha", ctypes.c_double), ("target_rel_err", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("stream", ctypes.c_void_p), ("outputs_on_device", ctypes.c_int32),
                ("iter_out", ctypes.c_void_p), ("grid_out", ctypes.c_void_p), ("n_iter_out", ctypes.c_void_p),
                ("timing_out", ctypes.c_void_p), ("chunk_points", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("flow", ctypes.c_void_p), ("ess_threshold", ctypes.c_double), ("allocation", ctypes.c_int32),
                ("weights_out", ctypes.c_void_p), ("weights_stride", ctypes.c_int64),
                ("weights_integral", ctypes.c_int32), ("weights_rows", ctypes.c_int32), ("hooks", ctypes.c_uint32), ("hook_event", ctypes.c_int32),
                ("checkpoint", ctypes.c_void_p), ("alloc_fn", ctypes.c_void_p), ("free_fn", ctypes.c_void_p),
                ("alloc_user", ctypes.c_void_p), ("flow_mode", ctypes.c_int32), ("stratify", ctypes.c_int32),
                ("combine", ctypes.c_int32), ("tail_chunk_points", ctypes.c_int32), ("tail_iter", ctypes.c_int32)]


MEM_HOOK_NONFINITE = 1

# how a flow is used (mem_integrate_opts.flow_mode)
MEM_FLOW_SAMPLE = 0
MEM_FLOW_SEED_GRID = 1

# mem_integrate_opts.stratify
MEM_STRATIFY_OFF = 0
MEM_STRATIFY_ADAPTIVE = 1

# mem_integrate_opts.combine
MEM_COMBINE_WEIGHTED = 0
MEM_COMBINE_MEAN = 1

# bytes of the per-device scratch of mem_integrate_events_noalloc
MEM_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

# allocator hook signatures (mem_alloc_fn, mem_free_fn)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


def _torch_alloc(nbytes, stream, user):
    import torch
    return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))


def _torch_free(ptr, nbytes, stream, user):
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


# the library's work buffers from PyTorch's caching allocator
TORCH_ALLOCATOR = (ALLOC_FN(_torch_alloc), FREE_FN(_torch_free))


_lib = None


def lib():
    """Load libmem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_1407_7595_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, U32, U64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                    ctypes.c_uint32, ctypes.c_uint64)
        sigs = {
            "mem_create_process": (I32, [P, P]),
            "mem_set_transfer_functions": (I32, [P, P, I32]),
            "mem_set_pdf_grid": (I32, [P, P, I32, I32, P]),
            "mem_toy_pdf_table": (I32, [P, I32, I32, P]),
            "mem_destroy_process": (None, [P]),
            "mem_process_shape": (I32, [P, P, P]),
            "mem_integrate_events": (I32, [P, P, I32, P, I32, I32, P, P, P, P]),
            "mem_integrate_events_noalloc": (I32, [P, P, I32, P, I32, I32, P, P, P, P]),
            "mem_train_proposal": (I32, [P, P, P, P]),
            "mem_set_proposal": (I32, [P, P]),
            "mem_flow_save": (I32, [P, ctypes.c_char_p]),
            "mem_flow_load": (I32, [ctypes.c_char_p, P]),
            "mem_uniforms": (I32, [U64, U32, U32, U32, I32, I64, P, P]),
            "mem_eval_points": (I32, [P, P, I32, I32, P, I64, P, P, P]),
            "mem_discriminant": (I32, [P, P, I64, P, P]),
            "mem_parton_weights": (I32, [P, P, P, P]),
            "mem_vegas_refine": (I32, [P, P, I32, I32, D, P]),
            "mem_vegas_capture": (I32, [P, P, P, P, I32, P, I64, U64, U32, I32, P, P, P]),
            "mem_flow_create": (I32, [I32, P]),
            "mem_flow_destroy": (None, [P]),
            "mem_flow_set_params": (I32, [P, P, I64, I32]),
            "mem_flow_get_params": (I32, [P, P, I64, I32]),
            "mem_flow_context": (I32, [P, P, P, I32, P, P]),
            "mem_flow_sample": (I32, [P, P, P, P, I32, I64, U64, U32, P, P, P]),
            "mem_flow_log_prob": (I32, [P, P, P, P, I64, P, P]),
            "mem_flow_train_step": (I32, [P, P, P, P, P, I64, D, P, P, P]),
            "mem_autotune": (I32, [P, P, I64, I32, P, P, I32, P, I32, ctypes.c_char_p, P, P, P]),
            "mem_process_set_launch": (I32, [P, I32, I32]),
            "mem_process_waves": (I32, [P, P]),
            "mem_tuning_load": (I32, [P, ctypes.c_char_p, ctypes.c_char_p, P]),
            "mem_process_chunk_points": (I32, [P, P]),
            "mem_checkpoint_create": (I32, [P]),
            "mem_checkpoint_destroy": (None, [P]),
            "mem_checkpoint_save": (I32, [P, ctypes.c_char_p]),
            "mem_checkpoint_load": (I32, [ctypes.c_char_p, P]),
            "mem_checkpoint_iterations": (I32, [P, P]),
            "mem_status_string": (ctypes.c_char_p, [I32]),
            "mem_last_error": (I32, [ctypes.c_char_p, ctypes.c_size_t]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class MemError(RuntimeError):
    def __init__(self, status, where):
        buf = ctypes.create_string_buffer(512)
        lib().mem_last_error(buf, 512)
        super().__init__(f"{where}: {lib().mem_status_string(status).decode()} ({buf.value.decode()})")
        self.status = status


def _check(status, where):
    if status != MEM_OK:
        raise MemError(status, where)


def _stream_ptr(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def process_desc(kind, precision=MEM_FP32, sqrt_s=13000.0, m_top=172.5, w_top=1.4, m_w=80.4, w_w=2.1,
                 m_h=125.0, w_h=0.00407, alpha=1.0 / 137.0, alpha_s=0.118, g_fermi=1.1663787e-5,
                 sigma_k=20.0, m_lo=60.0, m_hi=120.0, sigma_norm=0.0, m_b=4.18):
    """mem_process_desc with the configurations' parameters as defaults"""
    return ProcessDesc(kind, precision, sqrt_s, m_top, w_top, m_w, w_w, m_h, w_h, alpha, alpha_s, g_fermi,
                       sigma_k, m_lo, m_hi, sigma_norm, m_b)


class Process:
    """A hypothesis (mem_create_process); released with the object.
    Keyword arguments as process_desc."""

    def __init__(self, kind, precision=MEM_FP32, **kw):
        d = process_desc(kind, precision, **kw)
        h = ctypes.c_void_p()
        _check(lib().mem_create_process(ctypes.byref(d), ctypes.byref(h)), "mem_create_process")
        self.handle = h
        self.kind = kind

    def set_transfer_functions(self, tfs):
        arr = (TFDesc * len(tfs))(*tfs)
        _check(lib().mem_set_transfer_functions(self.handle, arr, len(tfs)), "mem_set_transfer_functions")

    def set_pdf_grid(self, xf, bounds):
        """mem_set_pdf_grid: xf float32 [nq][nx][11] on the host (x f of the
        flavours -5..5), bounds (ln x_min, ln x_max, ln Q_min, ln Q_max);
        xf None restores the toy densities"""
        if xf is None:
            _check(lib().mem_set_pdf_grid(self.handle, None, 0, 0, None), "mem_set_pdf_grid")
            return
        import numpy as np
        a = np.ascontiguousarray(xf, dtype=np.float32)
        if a.ndim != 3 or a.shape[2] != 11:
            raise ValueError("xf must be [nq][nx][11]")
        b = (ctypes.c_double * 4)(*bounds)
        _check(lib().mem_set_pdf_grid(self.handle, a.ctypes.data, a.shape[1], a.shape[0], b), "mem_set_pdf_grid")

    def autotune(self, comps, n_points, candidates=None, waves=None, table_path=None, charge=None, n_iter=2,
                 target_rel_err=None, max_iter=64, allocation=0, stratify=0, seed=0x5EED, tail_chunk_points=0,
                 tail_iter=0):
        """mem_autotune on the given events over chunk sizes x waves-per-SIMD
        variants, timing n_iter-iteration integrations (or, with
        target_rel_err, target-mode integrations with these options);
        returns (chunk_points, waves, events/s)"""
        ev = events_struct(comps, charge)
        cand = (ctypes.c_int32 * len(candidates))(*candidates) if candidates else None
        wv = (ctypes.c_int32 * len(waves))(*waves) if waves else None
        base = None
        if target_rel_err is not None or allocation or stratify or tail_chunk_points or n_iter != 2:
            base = IntegrateOpts()
            base.seed, base.alpha, base.max_iter, base.use_graph = seed, 1.5, max_iter, 1
            base.target_rel_err = target_rel_err or 0.0
            base.allocation, base.stratify = allocation, stratify
            base.tail_chunk_points, base.tail_iter = tail_chunk_points, tail_iter
        best, bw, rate = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().mem_autotune(self.handle, ctypes.byref(ev), n_points, n_iter,
                                  ctypes.byref(base) if base is not None else None, cand,
                                  len(candidates) if candidates else 0, wv, len(waves) if waves else 0,
                                  table_path.encode() if table_path else None, ctypes.byref(best), ctypes.byref(bw),
                                  ctypes.byref(rate)), "mem_autotune")
        return best.value, bw.value, rate.value

    def set_launch(self, chunk_points=0, waves=0):
        """mem_process_set_launch (0: defaults)"""
        _check(lib().mem_process_set_launch(self.handle, chunk_points, waves), "mem_process_set_launch")

    def waves(self):
        w = ctypes.c_int32()
        _check(lib().mem_process_waves(self.handle, ctypes.byref(w)), "mem_process_waves")
        return w.value

    def load_tuning(self, table_path, arch=None):
        found = ctypes.c_int32()
        _check(lib().mem_tuning_load(self.handle, table_path.encode(), arch.encode() if arch else None,
                                     ctypes.byref(found)), "mem_tuning_load")
        return bool(found.value)

    def set_proposal(self, flow):
        """mem_set_proposal: the default proposal of integrations of this
        process (None: VEGAS); the Flow must outlive its use"""
        _check(lib().mem_set_proposal(self.handle, flow.handle if flow is not None else None), "mem_set_proposal")
        self._proposal = flow

    def chunk_points(self):
        c = ctypes.c_int32()
        _check(lib().mem_process_chunk_points(self.handle, ctypes.byref(c)), "mem_process_chunk_points")
        return c.value

    def shape(self):
        d, n = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mem_process_shape(self.handle, ctypes.byref(d), ctypes.byref(n)), "mem_process_shape")
        return d.value, n.value

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.mem_destroy_process(self.handle)
            self.handle = None


def events_struct(comps, charge=None):
    """comps: float64 tensor [4, n_obj, n_events] (E, px, py, pz planes),
    contiguous, on the GPU or on the host; charge: optional int32 tensor
    [n_events] on the same device."""
    import torch
    assert comps.dtype == torch.float64 and comps.is_contiguous() and comps.dim() == 3 and comps.shape[0] == 4
    n_obj, n_ev = comps.shape[1], comps.shape[2]
    base = comps.data_ptr()
    stride = n_obj * n_ev * 8
    cptr = None
    if charge is not None:
        assert charge.dtype == torch.int32 and charge.is_contiguous() and charge.numel() == n_ev
        assert charge.is_cuda == comps.is_cuda
        cptr = charge.data_ptr()
    return Events(n_ev, n_obj, base, base + stride, base + 2 * stride, base + 3 * stride, cptr,
                  1 if comps.is_cuda else 0)


def to_components(obs):
    """numpy/torch [n_events, n_obj, 4] -> contiguous float64 [4, n_obj, n_events]"""
    import torch
    t = torch.as_tensor(obs, dtype=torch.float64)
    return t.permute(2, 1, 0).contiguous()


def integrate_events(comps, processes, n_points, n_iter, seed=0x14077595, alpha=1.5, target_rel_err=0.0,
                     max_iter=64, stream=None, iter_out=None, grid_out=None, n_iter_out=None, outputs=None,
                     timing=None, charge=None, chunk_points=0, use_graph=1, flow=None, ess_threshold=0.0,
                     allocation=0, weights_out=None, weights_integral=0, hooks=0, hook_event=0,
                     checkpoint=None, allocator=None, flow_mode=0, stratify=0, combine=0, tail_chunk_points=0,
                     tail_iter=0, _noalloc=False):
    """mem_integrate_events.  comps: [4, n_obj, n_events] float64 (device
    or host); processes: one Process or a list (one per event); n_points:
    int or a list per event; timing: optional ctypes (c_double * 8) array;
    flow: optional Flow (importance sampling from it, VEGAS fallback; with
    flow_mode=MEM_FLOW_SEED_GRID it seeds the VEGAS grids instead);
    allocation: MEM_ALLOC_EQUAL or MEM_ALLOC_NEYMAN across permutations;
    weights_out: optional float64 device tensor [iterations, stride] for
    the weights of integral weights_integral; hooks / hook_event: test
    hooks (MEM_HOOK_*); checkpoint: optional Checkpoint; allocator:
    None (hipMalloc), TORCH_ALLOCATOR, or a pair (ALLOC_FN, FREE_FN);
    stratify: MEM_STRATIFY_ADAPTIVE for adaptive stratified sampling;
    combine: MEM_COMBINE_WEIGHTED or MEM_COMBINE_MEAN (the iterations'
    combination); tail_chunk_points / tail_iter: chunks of that many points
    from that iteration on (0: the call's chunk size throughout).
    Returns (P, err, status) as torch tensors on the device of `comps`
    (or writes into `outputs`)."""
    import torch
    if weights_out is not None and not (weights_out.is_cuda and weights_out.dtype == torch.float64
                                        and weights_out.dim() == 2 and weights_out.is_contiguous()):
        raise ValueError("weights_out must be a contiguous float64 device tensor [rows, stride]")
    ev = events_struct(comps, charge)
    procs = processes if isinstance(processes, (list, tuple)) else [processes]
    handles = (ctypes.c_void_p * len(procs))(*[p.handle.value for p in procs])
    npts = [int(n_points)] if isinstance(n_points, int) else [int(v) for v in n_points]
    npts_arr = (ctypes.c_int64 * len(npts))(*npts)
    dev = comps.device
    if outputs is None:
        P = torch.empty(ev.n_events, dtype=torch.float64, device=dev)
        err = torch.empty_like(P)
        status = torch.empty(ev.n_events, dtype=torch.int32, device=dev)
    else:
        P, err, status = outputs
    opt = IntegrateOpts(seed, alpha, target_rel_err, max_iter, _stream_ptr(stream), 1 if P.is_cuda else 0,
                        iter_out.data_ptr() if iter_out is not None else None,
                        grid_out.data_ptr() if grid_out is not None else None,
                        n_iter_out.data_ptr() if n_iter_out is not None else None,
                        ctypes.cast(timing, ctypes.c_void_p) if timing is not None else None,
                        chunk_points, use_graph, flow.handle.value if flow is not None else None, ess_threshold,
                        allocation,
                        weights_out.data_ptr() if weights_out is not None else None,
                        weights_out.shape[-1] if weights_out is not None else 0, weights_integral,
                        weights_out.shape[0] if weights_out is not None else 0, hooks, hook_event,
                        checkpoint.handle.value if checkpoint is not None else None,
                        ctypes.cast(allocator[0], ctypes.c_void_p) if allocator is not None else None,
                        ctypes.cast(allocator[1], ctypes.c_void_p) if allocator is not None else None, None,
                        flow_mode, stratify, combine, tail_chunk_points, tail_iter)
    entry = "mem_integrate_events_noalloc" if _noalloc else "mem_integrate_events"
    _check(getattr(lib(), entry)(ctypes.byref(ev), handles, len(procs), npts_arr, len(npts), n_iter,
                                 ctypes.byref(opt), ctypes.c_void_p(P.data_ptr()),
                                 ctypes.c_void_p(err.data_ptr()), ctypes.c_void_p(status.data_ptr())),
           entry)
    return P, err, status


def integrate_events_noalloc(comps, processes, n_points, n_iter, outputs=None, **kw):
    """mem_integrate_events_noalloc: integrate_events with every work buffer
    in the library's fixed per-device scratch (no device allocation by the
    library).  comps and the outputs must be device tensors; the returned
    outputs are allocated here by torch unless `outputs` = (P, err, status)
    is given.  VEGAS only; no timing, no allocator."""
    return integrate_events(comps, processes, n_points, n_iter, outputs=outputs, _noalloc=True, **kw)


class Checkpoint:
    """mem_checkpoint: the state of a VEGAS integration between calls"""

    def __init__(self, path=None):
        self.handle = ctypes.c_void_p()
        if path is None:
            _check(lib().mem_checkpoint_create(ctypes.byref(self.handle)), "mem_checkpoint_create")
        else:
            _check(lib().mem_checkpoint_load(os.fsencode(path), ctypes.byref(self.handle)), "mem_checkpoint_load")

    def save(self, path):
        _check(lib().mem_checkpoint_save(self.handle, os.fsencode(path)), "mem_checkpoint_save")

    @property
    def iterations(self):
        n = ctypes.c_int32()
        _check(lib().mem_checkpoint_iterations(self.handle, ctypes.byref(n)), "mem_checkpoint_iterations")
        return n.value

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.mem_checkpoint_destroy(self.handle)
            self.handle = ctypes.c_void_p()


def uniforms(seed, it, event, perm, D, n, out, stream=None):
    _check(lib().mem_uniforms(seed, it, event, perm, D, n, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
           "mem_uniforms")
    return out


def eval_points(process, comps, event, perm, x, f, nsol=None, stream=None, charge=None):
    ev = events_struct(comps, charge)
    _check(lib().mem_eval_points(process.handle, ctypes.byref(ev), event, perm, ctypes.c_void_p(x.data_ptr()),
                                 x.shape[0], ctypes.c_void_p(f.data_ptr()),
                                 ctypes.c_void_p(nsol.data_ptr()) if nsol is not None else None,
                                 _stream_ptr(stream)), "mem_eval_points")
    return f


def discriminant(p_sig, p_bkg, out=None, stream=None):
    """mem_discriminant: D = log10(p_sig / p_bkg) per event; float64 device
    tensors of one length; returns `out` (allocated when None)."""
    import torch
    if p_sig.shape != p_bkg.shape or p_sig.dtype != torch.float64 or p_bkg.dtype != torch.float64:
        raise ValueError("p_sig and p_bkg: float64 tensors of one shape")
    d = torch.empty_like(p_sig) if out is None else out
    _check(lib().mem_discriminant(ctypes.c_void_p(p_sig.data_ptr()), ctypes.c_void_p(p_bkg.data_ptr()),
                                  p_sig.numel(), ctypes.c_void_p(d.data_ptr()), _stream_ptr(stream)),
           "mem_discriminant")
    return d


def toy_pdf_table(nx, nq, bounds):
    """mem_toy_pdf_table: the library's toy densities at the nodes of an
    (ln x, ln Q) grid, float32 [nq][nx][11]"""
    import numpy as np
    a = np.zeros((nq, nx, 11), dtype=np.float32)
    b = (ctypes.c_double * 4)(*bounds)
    _check(lib().mem_toy_pdf_table(a.ctypes.data, nx, nq, b), "mem_toy_pdf_table")
    return a


def parton_weights(process, comps, out=None, stream=None):
    """mem_parton_weights: comps [4, 6, n_events] float64 (b, bbar, l+, l-,
    nu, nubar) for ttbar dilepton, [4, 8, n_events] (four b quarks, l+, l-,
    nu, nubar) for the four-b dilepton kinds, on the device or the host;
    returns the weights [n_events] float64 on the same device (or writes
    into `out`)."""
    import torch
    ev = events_struct(comps, None)
    w = torch.empty(ev.n_events, dtype=torch.float64, device=comps.device) if out is None else out
    _check(lib().mem_parton_weights(process.handle, ctypes.byref(ev), ctypes.c_void_p(w.data_ptr()),
                                    _stream_ptr(stream)), "mem_parton_weights")
    return w


def vegas_refine(bins, grids, alpha=1.5, stream=None):
    n_int, D = bins.shape[0], bins.shape[1]
    _check(lib().mem_vegas_refine(ctypes.c_void_p(bins.data_ptr()), ctypes.c_void_p(grids.data_ptr()), n_int, D,
                                  alpha, _stream_ptr(stream)), "mem_vegas_refine")
    return grids


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def vegas_capture(process, comps, event, perm, grids, n_per, seed, it, x_out, w_out, normalise=1, stream=None,
                  charge=None):
    """mem_vegas_capture: points of adapted VEGAS grids and their weights.
    event, perm: int32 device tensors [n_int]; grids: float64 device
    [n_int, D, 65]; x_out: float32 [n_int, n_per, D]; w_out: float32
    [n_int, n_per]."""
    ev = events_struct(comps, charge)
    _check(lib().mem_vegas_capture(process.handle, ctypes.byref(ev), _p(event), _p(perm), event.numel(), _p(grids),
                                   n_per, seed, it, normalise, _p(x_out), _p(w_out), _stream_ptr(stream)),
           "mem_vegas_capture")
    return x_out, w_out


class Flow:
    """The learned proposal (mem_flow_*); released with the object."""

    def __init__(self, mode=MEM_FLOW_BF16, handle=None):
        if handle is None:
            handle = ctypes.c_void_p()
            _check(lib().mem_flow_create(mode, ctypes.byref(handle)), "mem_flow_create")
        self.handle = handle
        self.mode = mode

    def save(self, path):
        """mem_flow_save: parameters, Adam moments and step to a file"""
        _check(lib().mem_flow_save(self.handle, os.fsencode(path)), "mem_flow_save")

    @classmethod
    def load(cls, path):
        """mem_flow_load: a new flow from a file written by save"""
        h = ctypes.c_void_p()
        _check(lib().mem_flow_load(os.fsencode(path), ctypes.byref(h)), "mem_flow_load")
        return cls(handle=h)

    def set_params(self, params):
        """params: float32 tensor [192552] (host or device)"""
        import torch
        assert params.dtype == torch.float32 and params.is_contiguous() and params.numel() == FLOW_NPARAMS
        _check(lib().mem_flow_set_params(self.handle, _p(params), FLOW_NPARAMS, 1 if params.is_cuda else 0),
               "mem_flow_set_params")

    def get_params(self, out=None):
        import torch
        if out is None:
            out = torch.empty(FLOW_NPARAMS, dtype=torch.float32)
        _check(lib().mem_flow_get_params(self.handle, _p(out), FLOW_NPARAMS, 1 if out.is_cuda else 0),
               "mem_flow_get_params")
        return out

    def sample(self, ctx, event, perm, n_per, seed, it, x_out, logq_out, stream=None):
        _check(lib().mem_flow_sample(self.handle, _p(ctx), _p(event), _p(perm), event.numel(), n_per, seed, it,
                                     _p(x_out), _p(logq_out), _stream_ptr(stream)), "mem_flow_sample")
        return x_out, logq_out

    def log_prob(self, ctx, sint, x, logq_out, stream=None):
        _check(lib().mem_flow_log_prob(self.handle, _p(ctx), _p(sint), _p(x), sint.numel(), _p(logq_out),
                                       _stream_ptr(stream)), "mem_flow_log_prob")
        return logq_out

    def train_step(self, ctx, sint, x, wt, lr=0.0, grad_out=None, want_loss=True, stream=None):
        """one step on L = -sum wt log q; returns L (or None)"""
        loss = ctypes.c_double(0.0)
        _check(lib().mem_flow_train_step(self.handle, _p(ctx), _p(sint), _p(x), _p(wt), sint.numel(), lr,
                                         ctypes.byref(loss) if want_loss else None,
                                         _p(grad_out) if grad_out is not None else None, _stream_ptr(stream)),
               "mem_flow_train_step")
        return loss.value if want_loss else None

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.mem_flow_destroy(self.handle)
            self.handle = None


def train_proposal(process, comps, mode=MEM_FLOW_BF16, vegas_points=0, vegas_iter=0, capture=0, batch=0,
                   epochs=0, lr_max=0.0, lr_min=0.0, seed=0x14077595, stream=None, losses=False):
    """mem_train_proposal: a Flow trained on the events `comps` (VEGAS
    samples of every (event, assignment) integral); zero arguments take the
    library's defaults.  With losses=True returns (flow, per-epoch losses)."""
    ev = events_struct(comps)
    n_ep = epochs if epochs > 0 else 24
    loss = (ctypes.c_double * n_ep)() if losses else None
    d = FlowDesc(mode, vegas_iter, vegas_points, capture, batch, epochs, 0, lr_max, lr_min, seed,
                 _stream_ptr(stream), ctypes.cast(loss, ctypes.c_void_p) if losses else None)
    h = ctypes.c_void_p()
    _check(lib().mem_train_proposal(process.handle, ctypes.byref(ev), ctypes.byref(d), ctypes.byref(h)),
           "mem_train_proposal")
    f = Flow(mode, handle=h)
    return (f, list(loss)) if losses else f


def flow_context(comps, event, perm, ctx_out, stream=None):
    """mem_flow_context: ctx_out float32 device [n, 24]"""
    ev = events_struct(comps)
    _check(lib().mem_flow_context(ctypes.byref(ev), _p(event), _p(perm), event.numel(), _p(ctx_out),
                                  _stream_ptr(stream)), "mem_flow_context")
    return ctx_out
