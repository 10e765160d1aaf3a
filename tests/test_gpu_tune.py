"""Autotuner on the GPU: it picks one of the candidates, records it in the
table, a new process loads it, and integrations with the tuned chunk size
agree with the default within the MC error."""
import sys

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


def test_autotune_table_and_use(mem, tmp_path):
    d = events.ttbar_dilepton(24, 61)
    comps = mem.to_components(d["obs"]).cuda()
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    table = tmp_path / "tune.txt"
    say("autotune 24 tt events x 16384, candidates 1024, 4096, 16384")
    best, rate = p.autotune(comps, 16384, candidates=[1024, 4096, 16384], table_path=str(table))
    say(f"best chunk {best} at {rate:.3g} evals/s")
    assert best in (1024, 4096, 16384) and rate > 0
    assert p.chunk_points() == best
    rows = [ln.split() for ln in table.read_text().splitlines() if not ln.startswith("#")]
    assert len(rows) == 1 and rows[0][0].startswith("gfx") and rows[0][1:4] == ["2", "1", str(best)]
    q = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    assert q.load_tuning(str(table)) and q.chunk_points() == best
    # tuned vs fixed 4096: same estimates within the MC error
    P1, E1, S1 = mem.integrate_events(comps, q, 8192, 4, seed=3)
    P2, E2, S2 = mem.integrate_events(comps, q, 8192, 4, seed=3, chunk_points=4096)
    torch.cuda.synchronize()
    P1, E1, P2, E2 = (t.cpu().numpy() for t in (P1, E1, P2, E2))
    assert np.all(S1.cpu().numpy() == 0) and np.all(S2.cpu().numpy() == 0)
    if best == 4096:
        assert np.array_equal(P1, P2)
    else:
        # other chunk sums reorder FP64 additions, so the refined grids and
        # the points differ in the last bits: far inside the MC error
        assert np.all(np.abs(P1 - P2) <= 1e-3 * np.sqrt(E1 ** 2 + E2 ** 2))
