"""The C-ABI library loads and exports what include/mem.h declares; host
side validation (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mem.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mem_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def mem():
    import paper_1407_7595_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("libmem.so is not built (run __graft_entry__.build())")
    m.lib()
    return m


def test_exports_every_declared_symbol(mem):
    names = declared_functions()
    assert len(names) >= 10
    assert set(names) == set(mem.EXPORTS)
    L = ctypes.CDLL(mem.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(mem):
    L = mem.lib()
    assert L.mem_status_string(0) == b"ok"
    assert L.mem_status_string(1) == b"invalid argument"


def test_create_process_validation(mem):
    good = mem.Process(mem.MEM_TT_DILEPTON)
    assert good.shape() == (8, 2)
    dy = mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64)
    assert dy.shape() == (2, 1)
    with pytest.raises(mem.MemError) as e:
        mem.Process(99)
    assert e.value.status == mem.MEM_EINVAL
    with pytest.raises(mem.MemError) as e:
        mem.Process(mem.MEM_TT_DILEPTON, w_top=0.0)
    assert e.value.status == mem.MEM_EINVAL
    with pytest.raises(mem.MemError) as e:
        mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64, m_lo=120.0, m_hi=60.0)
    assert e.value.status == mem.MEM_EINVAL
    tth = mem.Process(mem.MEM_TTH_SEMILEPTON)
    assert tth.shape() == (9, 24)
    with pytest.raises(mem.MemError) as e:
        mem.Process(mem.MEM_TTH_SEMILEPTON, w_h=0.0)
    assert e.value.status == mem.MEM_EINVAL
    with pytest.raises(mem.MemError) as e:
        mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP32)
    assert e.value.status == mem.MEM_EUNSUPPORTED
    L = mem.lib()
    assert L.mem_create_process(None, None) == mem.MEM_EINVAL
    # Sec. 4's four-b dilepton kinds: 8 dimensions, 12 and 24 assignments
    assert mem.Process(mem.MEM_TTH_DILEPTON).shape() == (8, 12)
    assert mem.Process(mem.MEM_TTBB_DILEPTON, precision=mem.MEM_FP64).shape() == (8, 24)
    with pytest.raises(mem.MemError) as e:
        mem.Process(mem.MEM_TTH_DILEPTON, m_h=0.0)
    assert e.value.status == mem.MEM_EINVAL


def test_discriminant_argument_checks(mem):
    """mem_discriminant validates before touching the device: nothing to do
    for n = 0, MEM_EINVAL for n < 0 and for null arrays"""
    L = mem.lib()
    assert L.mem_discriminant(None, None, 0, None, None) == mem.MEM_OK
    assert L.mem_discriminant(None, None, -1, None, None) == mem.MEM_EINVAL
    assert L.mem_discriminant(None, None, 4, None, None) == mem.MEM_EINVAL


def test_transfer_function_validation(mem):
    p = mem.Process(mem.MEM_TT_DILEPTON)
    ok = mem.TFDesc(mem.MEM_OBJ_BJET, mem.MEM_TF_DGAUSS, 0.1, 0.25, 0.2, 5.0, 0.1)
    p.set_transfer_functions([ok])
    for bad in (mem.TFDesc(7, mem.MEM_TF_GAUSS, 0.1, 0.1, 0.0, 5.0, 0.1),
                mem.TFDesc(mem.MEM_OBJ_BJET, mem.MEM_TF_GAUSS, 0.0, 0.1, 0.0, 5.0, 0.1),
                mem.TFDesc(mem.MEM_OBJ_BJET, mem.MEM_TF_DGAUSS, 0.1, 0.25, 1.5, 5.0, 0.1),
                mem.TFDesc(mem.MEM_OBJ_BJET, mem.MEM_TF_DELTA, 0.1, 0.1, 0.0, 5.0, 0.1),
                mem.TFDesc(mem.MEM_OBJ_BJET, mem.MEM_TF_GAUSS, 0.1, 0.1, 0.0, -1.0, 0.1)):
        with pytest.raises(mem.MemError) as e:
            p.set_transfer_functions([bad])
        assert e.value.status == mem.MEM_EINVAL


def test_integrate_rejects_bad_host_events_before_any_launch(mem):
    import numpy as np
    import torch
    p = mem.Process(mem.MEM_TT_DILEPTON)
    obs = np.ones((3, 4, 4))
    obs[1, 2, 0] = np.nan
    comps = mem.to_components(obs)
    with pytest.raises(mem.MemError) as e:
        mem.integrate_events(comps, p, 1000, 3)
    assert e.value.status == mem.MEM_EINVAL
    obs[1, 2, 0] = -5.0
    with pytest.raises(mem.MemError) as e:
        mem.integrate_events(mem.to_components(obs), p, 1000, 3)
    assert e.value.status == mem.MEM_EINVAL
    good = mem.to_components(np.ones((3, 4, 4)))
    with pytest.raises(mem.MemError) as e:          # one iteration is not enough
        mem.integrate_events(good, p, 1000, 1)
    assert e.value.status == mem.MEM_EINVAL
    with pytest.raises(mem.MemError) as e:          # too few objects for tt
        mem.integrate_events(mem.to_components(np.ones((3, 2, 4))), p, 1000, 3)
    assert e.value.status == mem.MEM_EINVAL
    with pytest.raises(mem.MemError) as e:          # two hypotheses for three events
        mem.integrate_events(good, [p, p], 1000, 3)
    assert e.value.status == mem.MEM_EINVAL
    with pytest.raises(mem.MemError) as e:          # unknown point allocation
        mem.integrate_events(good, p, 1000, 3, allocation=7)
    assert e.value.status == mem.MEM_EINVAL


def test_tuning_table_lookup(mem, tmp_path):
    """mem_tuning_load reads the tuner's table (no GPU needed with an
    explicit architecture)"""
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    assert p.chunk_points() == 4096
    t = tmp_path / "tune.txt"
    t.write_text("# arch kind precision chunk_points evals_per_s\n"
                 "gfx942 2 1 2048 1e9\n"
                 "gfx950 2 0 1024 5e8\n"
                 "gfx950 2 1 8192 1.5e9\n")
    assert p.load_tuning(str(t), arch="gfx950")
    assert p.chunk_points() == 8192
    q = mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64)
    assert not q.load_tuning(str(t), arch="gfx950")
    assert q.chunk_points() == 4096
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 2 1 1000 1e9\n")
    with pytest.raises(mem.MemError) as e:
        p.load_tuning(str(bad), arch="gfx950")
    assert e.value.status == mem.MEM_EINVAL
    with pytest.raises(mem.MemError):
        p.load_tuning(str(tmp_path / "missing.txt"), arch="gfx950")


def test_toy_pdf_table_matches_oracle(mem):
    """the library's toy densities at grid nodes against the oracle's own
    tabulation (two implementations of the same densities), to FP32
    rounding"""
    import math
    import numpy as np
    import oracle
    b = (math.log(1e-5), 0.0, math.log(10.0), math.log(13000.0))
    got = mem.toy_pdf_table(320, 4, b)
    want = oracle.pdf_tabulate_toy(320, 4, b).xf
    assert got.shape == want.shape == (4, 320, 11)
    np.testing.assert_allclose(got, want, rtol=2.0 ** -23, atol=0.0)
    assert np.all(got[..., [0, 1, 2, 8, 9, 10]] == 0.0)
    assert np.all(got[:, -1, :] == 0.0)          # x = 1


def test_pdf_grid_validation(mem):
    import math
    import numpy as np
    p = mem.Process(mem.MEM_TT_DILEPTON)
    good_b = (math.log(1e-5), 0.0, math.log(10.0), math.log(13000.0))
    xf = np.ones((4, 8, 11), dtype=np.float32)
    nan = xf.copy()
    nan[1, 2, 3] = np.nan
    for a, b in ((xf, (0.0, -1.0, 1.0, 2.0)), (xf, (0.0, 1.0, 2.0, 2.0)), (xf[:, :1], good_b), (xf[:1], good_b),
                 (nan, good_b), (xf, (0.0, float("inf"), 1.0, 2.0))):
        with pytest.raises(mem.MemError) as e:
            p.set_pdf_grid(a, b)
        assert e.value.status == mem.MEM_EINVAL
    p.set_pdf_grid(None, None)                   # back to the toy densities: no device work
    tth = mem.Process(mem.MEM_TTH_SEMILEPTON)
    with pytest.raises(mem.MemError) as e:
        tth.set_pdf_grid(xf, good_b)
    assert e.value.status == mem.MEM_EUNSUPPORTED
    L = mem.lib()
    assert L.mem_set_pdf_grid(None, None, 0, 0, None) == mem.MEM_EINVAL
    assert L.mem_toy_pdf_table(None, 8, 4, None) == mem.MEM_EINVAL
