"""The device-resident probe and diagnostic rings through the C ABI: reads in
parts continue where the last one stopped, and a ring that wrapped returns
its newest rows in order (65,536 probe rows, 4,096 diagnostic records)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")


def test_reads_in_parts_continue():
    s = wc.Solver(dict(workloads.tiny(), diag_every=1), "cuda:0")
    s.step(100)
    t1, dt1, p1 = s.read_probes()
    d1 = s.read_diagnostics()
    s.step(50)
    t2, dt2, p2 = s.read_probes()
    d2 = s.read_diagnostics()
    assert t1.size == 100 and t2.size == 50 and p2.shape == (50, 4)
    assert np.allclose(t2[0], t1[-1] + dt1[-1], rtol=1e-14, atol=0)
    assert np.all(np.diff(np.concatenate([t1, t2])) > 0)
    assert d1["step"].size == 101 and d2["step"].size == 50
    assert np.array_equal(np.concatenate([d1["step"], d2["step"]]), np.arange(151))
    s.close()


def test_rings_wrap_and_keep_the_newest_rows():
    # no disk: a long run of the channel at rest under gravity
    cfg = dict(workloads.tiny(), diag_every=1, disk_R=0.0, n_disk_ghosts=0)
    s = wc.Solver(cfg, "cuda:0")
    n = 65_536 + 300
    print(f"[gpu] rings: {n} steps of the small channel", flush=True)
    s.step(n)
    t, dt, p = s.read_probes(max_rows=1 << 17)
    d = s.read_diagnostics(max_rows=8192)
    t_end = s.fluid()[0]
    s.close()
    assert t.size == 65_536 and p.shape == (65_536, 4)
    assert np.all(np.diff(t) > 0)
    assert np.allclose(t[1:], t[:-1] + dt[:-1], rtol=1e-12, atol=0)
    assert abs(t[-1] + dt[-1] - t_end) <= 1e-12 * t_end
    assert d["step"].size == 4096
    assert np.array_equal(d["step"], np.arange(n - 4095, n + 1))
    assert "unstable" not in d
