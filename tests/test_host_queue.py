"""The persistent work-queue kernel's own source (vegas_queue_kernel and
everything it inlines: the chunk loop, the dilepton kernel's LDS record and
root queues with their ballots, the per-wavefront bins, the reductions)
executed on the host under sanitizers, one workgroup of 256 lanes as 256
host threads (tests/host_queue/hip_host_emu.hpp).  One iteration on the
uniform grid against the oracle's iteration on the same point stream: the
sum of the weights within the matrix-element precision's bar (FP32 1e-5,
FP64 1e-9; the host build takes exact divisions where the GPU refines the
hardware estimates, so agreement is to the bar, not to the bit), the sum of
squares to twice that, and the per-(dimension, bin) sums of w^2 to 1e-5 of
the total.  AddressSanitizer + UndefinedBehaviorSanitizer over both
dilepton variants (LDS queues at one wave per SIMD, per-lane roots at two)
and Drell-Yan; ThreadSanitizer over the LDS-queue variant, which would
report an LDS access between lanes that no barrier orders."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import paper_1407_7595_amd as mem
from synth import events

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "host_queue", "host_queue.cpp")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def build(tmp, sanitize):
    exe = os.path.join(tmp, "host_queue_" + sanitize.replace(",", "_"))
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", "-DMEM_HOST_EMU=1",
           f"-fsanitize={sanitize}", "-fno-sanitize-recover=all",
           "-I" + os.path.join(ROOT, "paper_1407_7595_amd", "csrc"), "-I" + os.path.join(HERE, "host_queue"),
           SRC, "-o", exe]
    subprocess.run(cmd, check=True)
    return exe


def write_inputs(tmp, desc, obs, charge=None):
    dpath, epath = os.path.join(tmp, "desc.bin"), os.path.join(tmp, "events.bin")
    with open(dpath, "wb") as f:
        f.write(bytes(desc))
    n_ev, n_obj = obs.shape[0], obs.shape[1]
    planes = np.ascontiguousarray(np.transpose(obs, (2, 1, 0)), dtype=np.float64)    # [4][n_obj][n_ev]
    with open(epath, "wb") as f:
        f.write(np.array([n_ev, n_obj], dtype=np.int32).tobytes())
        f.write(planes.tobytes())
        if charge is not None:
            f.write(np.ascontiguousarray(charge, dtype=np.int32).tobytes())
    return dpath, epath


def run(exe, dpath, epath, variant, n, seed, chunk, blocks, ns=0):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", TSAN_OPTIONS="halt_on_error=1")
    args = [exe, dpath, epath, variant, str(n), str(seed), str(chunk), str(blocks)] + ([str(ns)] if ns else [])
    out = subprocess.run(args, capture_output=True, text=True, env=env, timeout=900)
    assert out.returncode == 0, out.stderr[-4000:]
    rows = [list(map(float, ln.split())) for ln in out.stdout.splitlines() if ln.strip()]
    return [(int(r[0]), int(r[1]), r[2], r[3], np.array(r[4:])) for r in rows]


def compare(rows, kind, po, obs, n, seed, D, tol):
    g0 = oracle.uniform_grid(D)
    n_nz = 0
    for e, perm, s1, s2, bins in rows:
        o1, o2, obins = oracle.vegas_iteration(kind, po, obs[e], perm, seed, e, 0, n, g0)
        assert abs(s1 - o1) <= tol * abs(o1) + 1e-300, (e, perm, s1, o1)
        assert abs(s2 - o2) <= 2 * tol * abs(o2) + 1e-300, (e, perm, s2, o2)
        assert np.all(np.abs(bins - np.asarray(obins).ravel()) <= 1e-5 * max(o2, 1e-300)), (e, perm)
        n_nz += o1 > 0
    return n_nz


@pytest.mark.parametrize("variant,prec,tol", [("tt1f", mem.MEM_FP32, 1e-5), ("tt2f", mem.MEM_FP32, 1e-5),
                                              ("tt1d", mem.MEM_FP64, 1e-9)])
def test_queue_kernel_host_asan_ubsan_dilepton(tmp_path, variant, prec, tol):
    """2 events x 2 assignments x 1536 points in chunks of 512 over 2
    workgroups (chunks popped from the shared head, a ragged wave count per
    chunk would show as a hang at a barrier)"""
    tmp = str(tmp_path)
    exe = build(tmp, "address,undefined")
    obs = events.ttbar_dilepton(2, 0x81)["obs"]
    dpath, epath = write_inputs(tmp, mem.process_desc(mem.MEM_TT_DILEPTON, prec), obs)
    rows = run(exe, dpath, epath, variant, 1536, 0x5EED, 512, 2)
    assert len(rows) == 4
    assert compare(rows, oracle.KIND_TT, oracle.tt_params(), obs, 1536, 0x5EED, 8, tol) >= 2


def test_queue_kernel_host_asan_ubsan_drell_yan(tmp_path):
    tmp = str(tmp_path)
    exe = build(tmp, "address,undefined")
    obs = events.drell_yan(3, 0x82)["obs"]
    dpath, epath = write_inputs(tmp, mem.process_desc(mem.MEM_DY_QQ_GAMMA_MUMU, mem.MEM_FP64), obs)
    rows = run(exe, dpath, epath, "dy", 1000, 7, 256, 2)
    assert len(rows) == 3
    assert compare(rows, oracle.KIND_DY, oracle.dy_params(), obs, 1000, 7, 2, 1e-11) == 3


def test_queue_kernel_host_asan_ubsan_semileptonic_and_tth(tmp_path):
    """the semileptonic kernel, and t tbar H chunks in the instance that
    carries every kind (the instance whose one-wave build once returned
    wrong sums on the GPU; its source runs clean here)"""
    tmp = str(tmp_path)
    exe = build(tmp, "address,undefined")
    sl = events.ttbar_semileptonic(1, 0x84)
    obs = np.ascontiguousarray(sl["obs"][:, :5, :])
    dpath, epath = write_inputs(tmp, mem.process_desc(mem.MEM_TT_SEMILEPTON, mem.MEM_FP32), obs,
                                sl["obs"][:, 5, 0].astype(np.int32))
    rows = run(exe, dpath, epath, "sl1f", 768, 11, 256, 2)
    assert len(rows) == 12
    compare(rows, oracle.KIND_TT_SL, oracle.sl_params(), sl["obs"], 768, 11, 7, 1e-5)
    th = events.ttbar_higgs(1, 0x85)["obs"]
    dpath, epath = write_inputs(tmp, mem.process_desc(mem.MEM_TTH_SEMILEPTON, mem.MEM_FP32),
                                np.ascontiguousarray(th[:, :7, :]), th[:, 7, 0].astype(np.int32))
    rows = run(exe, dpath, epath, "tth2f", 512, 13, 256, 2)
    assert len(rows) == 24
    compare(rows, oracle.KIND_TTH, oracle.tt_params(), th, 512, 13, 9, 1e-5)


def test_queue_kernel_host_stratified(tmp_path):
    """the stratified point mapping (hypercube search in the chunk's staged
    counts, digits, shifted uniforms, weights stored per point) in the
    first iteration's equal split, under AddressSanitizer and
    UndefinedBehaviorSanitizer: every point's weight against the oracle's
    stratified iteration (FP64 dilepton, 1e-9; Drell-Yan 1e-11), with a
    ragged chunk and unequal hypercube counts"""
    tmp = str(tmp_path)
    exe = build(tmp, "address,undefined")
    for kind, ok, po, D, obs, prec, n, ns, tol in (
            ("tt1d", oracle.KIND_TT, oracle.tt_params(), 8, events.ttbar_dilepton(2, 0x86)["obs"], mem.MEM_FP64,
             1100, 2, 1e-9),
            ("dy", oracle.KIND_DY, oracle.dy_params(), 2, events.drell_yan(2, 0x87)["obs"], mem.MEM_FP64, 1000, 20,
             1e-11)):
        pk = mem.MEM_TT_DILEPTON if kind.startswith("tt") else mem.MEM_DY_QQ_GAMMA_MUMU
        dpath, epath = write_inputs(tmp, mem.process_desc(pk, prec), obs)
        rows = run(exe, dpath, epath, kind, n, 0x77, 512, 2, ns)
        H = ns ** D
        nh = oracle.strat_allocate(H, n, first=True)
        n_nz = 0
        for e, perm, s1, s2, rest in rows:
            w = rest[D * 64:]
            assert len(w) == n
            _, _, _, _, want = oracle.strat_iteration(ok, po, obs[e], perm, 0x77, e, 0, n, oracle.uniform_grid(D),
                                                      ns, nh)
            both_zero = (w == 0) & (want == 0)
            r = np.where(both_zero, 0.0, np.abs(w - want) / np.maximum(np.abs(want), 1e-300))
            assert r.max() <= tol, (kind, e, perm, r.max())
            assert abs(s1 - w.sum()) <= 1e-12 * max(abs(s1), 1e-300)
            n_nz += int(np.sum(~both_zero))
        assert n_nz > 0


def test_queue_kernel_host_tsan(tmp_path):
    """the LDS-queue dilepton variant under ThreadSanitizer: every LDS
    access between lanes is ordered by a wavefront or workgroup barrier"""
    tmp = str(tmp_path)
    exe = build(tmp, "thread")
    obs = events.ttbar_dilepton(1, 0x83)["obs"]
    dpath, epath = write_inputs(tmp, mem.process_desc(mem.MEM_TT_DILEPTON, mem.MEM_FP32), obs)
    rows = run(exe, dpath, epath, "tt1f", 512, 0x5EED, 256, 1)
    assert compare(rows, oracle.KIND_TT, oracle.tt_params(), obs, 512, 0x5EED, 8, 1e-5) >= 1
