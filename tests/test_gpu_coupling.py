"""Two-way disk coupling (kin_mode 2) on the HIP path against the FP64 oracle.

The disk follows the ramp, then takes the reaction of the ring's x force on
the fluid at each step's midpoint (the extension named with the energy audit
and in the Conclusions). Bars: the disk's velocity change and travel since the
ramp within 2e-3 of the oracle's over 200 steps of the 80x40 mm channel, probe
histories within 1e-3 of each probe's peak, and the GPU's own energy identity
e_disk + w_boundary = const to FP64 rounding (the midpoint force and the step's
mean velocity make it exact in exact arithmetic).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")

N_STEPS = 200


def _solver(cfg):
    print(f"[gpu] solver L={cfg['L']} W={cfg['W']} dx={cfg['dx']} kin_mode={cfg['kin_mode']}", flush=True)
    return wc.Solver(cfg, "cuda:0")


def test_two_way_C1_matches_oracle():
    cfg = workloads.two_way(workloads.C1())
    s = _solver(cfg)
    s.step(N_STEPS)
    xg, vg, ag = s.disk_state()
    tg, dtg, pg = s.read_probes()
    dg = s.read_diagnostics()
    o = oracle.Oracle(cfg)
    o.step(N_STEPS)
    xo, vo, ao = o.disk_state()
    to, dto, po = o.probes()
    do = o.diags()
    v0, tr = cfg["kin_v0"], cfg["kin_t_ramp"]
    x_r = cfg["disk_x0"] + 0.5 * v0 * tr
    print(f"disk v: gpu {vg:.6f} oracle {vo:.6f}; x: gpu {xg:.9f} oracle {xo:.9f}")
    assert vo < 0.9 * v0  # the fluid has taken a tenth of the disk's speed
    assert abs((vg - v0) - (vo - v0)) <= 2e-3 * abs(vo - v0)
    assert abs(xg - xo) <= 2e-3 * (xo - x_r)
    assert np.abs(dtg / dto - 1).max() < 1e-4
    for k in range(po.shape[1]):
        err = np.abs(pg[:, k] - po[:, k]).max() / np.abs(po[:, k]).max()
        print(f"probe {k}: max rel err {err:.3e}")
        assert err <= 1e-3
    for key in ("e_disk", "w_boundary"):
        assert abs(dg[key][-1] - do[key][-1]) <= 2e-3 * abs(do[key][-1]), key
    s.close()


def test_two_way_energy_identity():
    """The disk loses exactly the work its ring does on the fluid."""
    cfg = workloads.two_way(workloads.C1())
    s = _solver(cfg)
    s.step(N_STEPS)
    d = s.read_diagnostics()
    k = np.nonzero(d["t"] > cfg["kin_t_ramp"] + 2 * d["dt"].max())[0]
    assert k.size >= 10
    tot = d["e_disk"][k] + d["w_boundary"][k]
    dw = abs(d["w_boundary"][k[-1]] - d["w_boundary"][k[0]])
    assert dw > 0.01 * d["e_disk"][k[0]]
    assert np.abs(tot - tot[0]).max() <= 1e-9 * d["e_disk"][k[0]]
    s.close()


def test_set_kinematics_switches_to_two_way():
    """Switching a prescribed disk to mode 2 before the first step (the step
    graph is captured again with the disk update) gives the run of a context
    created in mode 2, bitwise; switching back releases the disk."""
    base = workloads.C1()
    cfg = workloads.two_way(base)
    a = _solver(cfg)
    b = _solver(dict(base, disk_mass=cfg["disk_mass"]))
    b.set_kinematics(2, cfg["kin_v0"], cfg["kin_t_ramp"], 0.0)
    a.step(60)
    b.step(60)
    assert a.disk_state() == b.disk_state()
    for u, v in zip(a.fluid()[1], b.fluid()[1]):
        assert np.array_equal(u, v)
    # back to the prescribed law: the disk state is the law's at t_next
    t = b.fluid()[0]
    b.set_kinematics(0, cfg["kin_v0"], cfg["kin_t_ramp"], base["kin_coef"])
    x, v, acc = b.disk_state()
    tau = t - cfg["kin_t_ramp"]
    ad = base["kin_coef"]
    assert abs(v - (cfg["kin_v0"] - ad * tau)) <= 1e-12 * cfg["kin_v0"]
    b.step(5)
    a.close()
    b.close()


def test_immovable_disk_equals_prescribed_constant_velocity():
    """A coupled disk of (almost) infinite mass keeps v0 after the ramp, as
    the prescribed law with no deceleration does."""
    cfg0 = dict(workloads.C1(), kin_coef=0.0, disk_mass=1.0e30)
    cfg2 = dict(workloads.two_way(cfg0), disk_mass=1.0e30)
    s0, s2 = _solver(cfg0), _solver(cfg2)
    s0.step(120)
    s2.step(120)
    x0, v0, _ = s0.disk_state()
    x2, v2, a2 = s2.disk_state()
    assert v2 == cfg0["kin_v0"] and abs(a2) < 1e-20
    assert abs(x2 - x0) <= 1e-12 * x0
    _, (xa, ya, vxa, vya, ra) = s0.fluid()
    _, (xb, yb, vxb, vyb, rb) = s2.fluid()
    assert np.abs(ra / rb - 1).max() <= 1e-5
    assert np.abs(xa - xb).max() <= 1e-5 * cfg0["dx"]
    s0.close()
    s2.close()


def test_batch_with_a_coupled_instance_equals_single_runs():
    cfgs = [workloads.two_way(workloads.C1()), workloads.tiny(), workloads.two_way(workloads.tiny())]
    n = 80
    b = wc.Solver(cfgs, "cuda:0")
    b.step(n)
    for k, cfg in enumerate(cfgs):
        s = wc.Solver(cfg, "cuda:0")
        s.step(n)
        assert b.disk_state(k) == s.disk_state()
        for u, v in zip(b.fluid(k)[1], s.fluid()[1]):
            assert np.array_equal(u, v), k
        d1, d2 = b.read_diagnostics(k), s.read_diagnostics()
        for key in ("e_disk", "w_boundary"):
            assert np.array_equal(d1[key], d2[key]), (k, key)
        s.close()
    b.close()


def test_two_way_rejections():
    cfg = workloads.two_way(workloads.C1())
    with pytest.raises(wc.WcsphError):
        wc.Solver(dict(cfg, disk_mass=0.0), "cuda:0")
    s = _solver(cfg)
    s.set_dt_table(np.full(4, 1e-8))
    with pytest.raises(wc.WcsphError):
        s.adj_forward(4, 2)
    s.close()
