"""Batched coefficient sweep: many uneven instances advanced by the same
launches. Each instance must equal the same problem run alone through the
plain solver (bitwise: the per-instance sorted order, summation order and
arithmetic are the same), and a small instance must match the oracle."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")


def _mixed_batch():
    return [
        workloads.tiny(),
        dict(workloads.tiny(L=0.031, W=0.019, R=0.0035, v0=500.0), alpha=0.3, delta=0.05),
        dict(workloads.C1(), alpha=0.02, delta=0.15, kin_v0=750.0,
             kin_coef=workloads.K_DRAG * 750.0 ** 2),
        dict(workloads.tiny(L=0.020, W=0.014), disk_R=0.0, n_disk_ghosts=0, probes=[(0.01, 0.0)]),
    ]


def _run_single(cfg, n):
    s = wc.Solver(cfg, "cuda:0")
    s.step(n)
    out = s.fluid(), s.read_probes(), s.read_diagnostics()
    s.close()
    return out


def test_batch_instances_equal_single_runs_bitwise():
    cfgs = _mixed_batch()
    n = 60
    print(f"[gpu] batch of {len(cfgs)} instances, {n} steps", flush=True)
    b = wc.Solver(cfgs, "cuda:0")
    assert b.n_inst == len(cfgs)
    b.step(n)
    for k, cfg in enumerate(cfgs):
        (tb, fb), (t1, dt1, p1), d1 = b.fluid(k), b.read_probes(k), b.read_diagnostics(k)
        (ts, fs), (t2, dt2, p2), d2 = _run_single(cfg, n)
        assert tb == ts
        for u, v in zip(fb, fs):
            assert np.array_equal(u, v), k
        assert np.array_equal(dt1, dt2) and np.array_equal(p1, p2)
        for key in ("mass", "ke", "e_el", "w_boundary"):
            assert np.array_equal(d1[key], d2[key]), (k, key)
    b.close()


def test_batch_instance_matches_oracle():
    cfgs = _mixed_batch()
    n = 200
    b = wc.Solver(cfgs, "cuda:0")
    b.step(n)
    k = 2  # the 80x40 mm channel at 750 m/s
    _, _, pg = b.read_probes(k)
    o = oracle.Oracle(cfgs[k])
    o.step(n)
    _, _, po = o.probes()
    for j in range(po.shape[1]):
        err = np.abs(pg[:, j] - po[:, j]).max() / np.abs(po[:, j]).max()
        print(f"batched instance {k} probe {j}: max rel err {err:.3e}")
        assert err <= 1e-3
    b.close()


def test_full_C4_sweep_sampled_instances():
    """The 64-instance sweep (seeded draws) in the launch configuration the
    benchmark times: sampled instances equal their single runs, and every
    instance conserves mass."""
    cfgs = workloads.C4()
    n = 20
    b = wc.Solver(cfgs, "cuda:0")
    print(f"[gpu] C4: {b.n_inst} instances, {b.n_fluid_total} fluid, {b.n_slots} slots", flush=True)
    assert b.n_inst == 64 and 64 * 19948 <= b.n_fluid_total <= 64 * 39948
    b.step(n)
    for k in range(64):
        d = b.read_diagnostics(k)
        assert "unstable" not in d
        assert np.abs(d["mass"] - d["mass"][0]).max() <= 1e-12 * d["mass"][0]
    for k in (0, 17, 63):
        (tb, fb), (_, _, pb) = b.fluid(k), b.read_probes(k)
        (ts, fs), (_, _, ps), _ = _run_single(cfgs[k], n)
        assert tb == ts
        for u, v in zip(fb, fs):
            assert np.array_equal(u, v), k
        assert np.array_equal(pb, ps)
    b.close()


def test_batch_beyond_one_wave_of_instances():
    """More instances than one wave has lanes: the sort's clock block commits
    the clocks 64 instances per round, so instances past the 64th take the
    second round. Those and the first ones equal their single runs bitwise,
    and every instance conserves mass."""
    cfgs = [dict(workloads.tiny(v0=300.0 + 5.0 * k), alpha=0.05 + 0.002 * k) for k in range(70)]
    n = 20
    b = wc.Solver(cfgs, "cuda:0")
    print(f"[gpu] batch of {b.n_inst} small instances, {n} steps", flush=True)
    assert b.n_inst == 70
    b.step(n)
    for k in range(70):
        d = b.read_diagnostics(k)
        assert "unstable" not in d
        assert np.abs(d["mass"] - d["mass"][0]).max() <= 1e-12 * d["mass"][0]
    for k in (0, 63, 64, 69):
        (tb, fb), (_, dtb, pb) = b.fluid(k), b.read_probes(k)
        (ts, fs), (_, dts, ps), _ = _run_single(cfgs[k], n)
        assert tb == ts, k
        for u, v in zip(fb, fs):
            assert np.array_equal(u, v), k
        assert np.array_equal(dtb, dts) and np.array_equal(pb, ps), k
    b.close()


def test_batch_step_needs_a_batched_context():
    s = wc.Solver(workloads.tiny(), "cuda:0")
    assert wc.lib().wcsph_batch_step(s.handle, 1) == wc.E_INVALID
    s.step(1)  # the plain entry point serves it, and the context is still usable
    s.close()
