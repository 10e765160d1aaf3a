"""Host-forced failure handling and state management of mem_integrate_events:
the non-finite-weight hook, checkpoint / resume (bit for bit against an
uninterrupted call, through memory and through a file), mismatched
checkpoints, and work buffers from the caller's allocator."""
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


def host(*ts):
    return [t.cpu().numpy() for t in ts]


def test_nonfinite_hook(mem):
    """NaN weights forced for one event: that event ends MEM_EV_NONFINITE,
    every other event is bit-equal to a call without the hook"""
    for kind, prec, gen, n_obj in ((mem.MEM_DY_QQ_GAMMA_MUMU, mem.MEM_FP64, events.drell_yan, 2),
                                   (mem.MEM_TT_DILEPTON, mem.MEM_FP32, events.ttbar_dilepton, 4)):
        p = mem.Process(kind, precision=prec)
        d = gen(4, 31)
        comps = mem.to_components(d["obs"][:, :n_obj]).cuda()
        say(f"nonfinite hook: kind {kind}, 4 events x 8192 x 4, hook on event 2")
        ref = host(*mem.integrate_events(comps, p, 8192, 4, seed=2, allocation=mem.MEM_ALLOC_NEYMAN))
        got = host(*mem.integrate_events(comps, p, 8192, 4, seed=2, allocation=mem.MEM_ALLOC_NEYMAN,
                                         hooks=mem.MEM_HOOK_NONFINITE, hook_event=2))
        assert got[2][2] == mem.MEM_EV_NONFINITE
        others = [0, 1, 3]
        assert np.all(ref[2][others] == 0)
        for a, b in zip(ref, got):
            assert np.array_equal(a[others], b[others])
        with pytest.raises(mem.MemError):
            mem.integrate_events(comps, p, 8192, 4, hooks=mem.MEM_HOOK_NONFINITE, hook_event=4)


@pytest.mark.parametrize("allocation", [0, 1])
def test_checkpoint_resume_fixed(mem, allocation):
    """3 + 3 iterations through a checkpoint (saved to a file and loaded in
    between) equal 6 uninterrupted iterations bit for bit"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    d = events.ttbar_dilepton(6, 41)
    comps = mem.to_components(d["obs"]).cuda()
    g_ref = torch.zeros((12, 8, 65), dtype=torch.float64, device="cuda")
    n_ref = torch.zeros(6, dtype=torch.int32, device="cuda")
    say(f"checkpoint fixed mode, allocation {allocation}: 6 iterations straight")
    ref = host(*mem.integrate_events(comps, p, 12000, 6, seed=4, allocation=allocation, grid_out=g_ref,
                                     n_iter_out=n_ref))
    ck = mem.Checkpoint()
    assert ck.iterations == 0
    say("  3 iterations into a checkpoint")
    mem.integrate_events(comps, p, 12000, 3, seed=4, allocation=allocation, checkpoint=ck)
    assert ck.iterations == 3
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "state.ckpt")
        ck.save(path)
        ck2 = mem.Checkpoint(path)
    assert ck2.iterations == 3
    g = torch.zeros_like(g_ref)
    n = torch.zeros_like(n_ref)
    say("  3 more from the loaded checkpoint")
    got = host(*mem.integrate_events(comps, p, 12000, 3, seed=4, allocation=allocation, checkpoint=ck2,
                                     grid_out=g, n_iter_out=n))
    assert ck2.iterations == 6
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    assert torch.equal(g, g_ref) and torch.equal(n, n_ref)
    # the in-memory handle resumes the same way
    got2 = host(*mem.integrate_events(comps, p, 12000, 3, seed=4, allocation=allocation, checkpoint=ck))
    for a, b in zip(ref, got2):
        assert np.array_equal(a, b)


def test_checkpoint_resume_target(mem):
    """target mode stopped at 4 iterations and resumed to 16 equals one
    call to 16 (retired events stay retired, the others continue)"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    d = events.ttbar_dilepton(8, 43)
    comps = mem.to_components(d["obs"]).cuda()
    kw = dict(seed=6, target_rel_err=0.02, allocation=mem.MEM_ALLOC_NEYMAN)
    n_ref = torch.zeros(8, dtype=torch.int32, device="cuda")
    say("checkpoint target mode: straight to 16 iterations")
    ref = host(*mem.integrate_events(comps, p, 8192, 0, max_iter=16, n_iter_out=n_ref, **kw))
    ck = mem.Checkpoint()
    n1 = torch.zeros_like(n_ref)
    say("  stopped at 4 iterations")
    first = host(*mem.integrate_events(comps, p, 8192, 0, max_iter=4, n_iter_out=n1, checkpoint=ck, **kw))
    assert np.any(first[2] == mem.MEM_EV_NOT_CONVERGED), "some events continue after the checkpoint"
    n2 = torch.zeros_like(n_ref)
    say("  resumed to 16")
    got = host(*mem.integrate_events(comps, p, 8192, 0, max_iter=16, n_iter_out=n2, checkpoint=ck, **kw))
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    assert torch.equal(n2, n_ref)


def test_checkpoint_mismatch(mem):
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    d = events.ttbar_dilepton(3, 45)
    comps = mem.to_components(d["obs"]).cuda()
    ck = mem.Checkpoint()
    say("checkpoint mismatch: a state of 3 events x 4096")
    mem.integrate_events(comps, p, 4096, 2, seed=1, checkpoint=ck)
    for kw in (dict(n_points=8192, seed=1), dict(n_points=4096, seed=2)):
        with pytest.raises(mem.MemError):
            mem.integrate_events(comps, p, kw["n_points"], 2, seed=kw["seed"], checkpoint=ck)
    with pytest.raises(mem.MemError):
        mem.integrate_events(comps[:, :, :2].contiguous(), p, 4096, 2, seed=1, checkpoint=ck)
    assert ck.iterations == 2     # unchanged by the refused calls


def test_torch_allocator(mem):
    """work buffers from PyTorch's caching allocator: same results, and
    every block goes back"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    d = events.ttbar_dilepton(5, 47)
    comps = mem.to_components(d["obs"]).cuda()
    say("allocator hook: 5 events x 8192 x 3, hipMalloc vs the caching allocator")
    ref = host(*mem.integrate_events(comps, p, 8192, 3, seed=8))
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    out = mem.integrate_events(comps, p, 8192, 3, seed=8, allocator=mem.TORCH_ALLOCATOR)
    got = host(*out)
    del out
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_weights_out_shape_checked(mem):
    """weights_out with fewer rows than the call's iterations, or a stride
    below the integral's points, is refused before any launch"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    d = events.ttbar_dilepton(2, 49)
    comps = mem.to_components(d["obs"]).cuda()
    say("weights_out shape checks")
    for rows, stride in ((2, 4096), (3, 4095)):
        w = torch.zeros((rows, stride), dtype=torch.float64, device="cuda")
        with pytest.raises(mem.MemError):
            mem.integrate_events(comps, p, 8192, 3, weights_out=w, weights_integral=0)
    w = torch.zeros((3, 4096), dtype=torch.float64, device="cuda")
    mem.integrate_events(comps, p, 8192, 3, weights_out=w, weights_integral=3)
    torch.cuda.synchronize()
    assert torch.any(w != 0.0), "the weights of the integral are recorded"
