"""The axisymmetric r-z form (axisym = 1) on the HIP path against the FP64
oracle: the extension the Conclusions rank first, where each particle is a
ring about the tank axis, continuity gains the hoop term -rho v_r / r, the
ghost layers below the axis mirror the fluid and the sums of mass, momentum,
energy and the sphere's force are 3D.

Bars, as for the planar form: one evaluation from a shared state (density
rate, acceleration, XSPH velocity, ghost pressure and velocity, axis ghosts
included) within 1e-4 of each field's maximum; probe histories over 200
steps within 1e-3 of each probe's own peak and dt within 1e-5; 3D mass
conserved to 1e-12; energies and the sphere's work within 1e-3. A batch of
axisymmetric instances equals its single runs bitwise.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests import shared_state

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")


def _rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def _relvec(ax, ay, bx, by):
    d = np.hypot(np.asarray(ax, np.float64) - bx, np.asarray(ay, np.float64) - by)
    return float(d.max() / max(np.hypot(bx, by).max(), 1e-300))


def _one_evaluation(cfg, steps):
    print(f"[gpu] axisymmetric L={cfg['L']} R_t={cfg['W']} dx={cfg['dx']}, shared state after {steps} steps",
          flush=True)
    s, o = shared_state.shared(cfg, steps, wc, oracle)
    g = s.export_rates()
    r = o.eval_rates()
    s.close()
    e = dict(drho=_rel(g["drho"], r["drho"]), acc=_relvec(g["ax"], g["ay"], r["ax"], r["ay"]),
             xsph=_relvec(g["Vx"], g["Vy"], r["Vx"], r["Vy"]), ghost_p=_rel(g["gp"], r["gp"]),
             ghost_v=_relvec(g["gvx"], g["gvy"], r["gvx"], r["gvy"]))
    print("axisymmetric one evaluation, max error / max value:", e)
    return e


@pytest.mark.parametrize("steps", [0, 60])
def test_one_evaluation_C1(steps):
    e = _one_evaluation(workloads.axisymmetric(workloads.C1()), steps)
    assert max(e.values()) <= 1e-4


def test_one_evaluation_full_size_C2():
    """The 300 mm x 75 mm tank at dx 0.5 mm (89,776 fluid rings): many
    pair-kernel tiles and a ragged last block."""
    e = _one_evaluation(workloads.axisymmetric(workloads.C2()), 20)
    assert max(e.values()) <= 1e-4


def test_probe_histories_C1_200_steps():
    cfg = workloads.axisymmetric(workloads.C1())
    n = 200
    print("[gpu] axisymmetric C1, 200 steps", flush=True)
    s = wc.Solver(cfg, "cuda:0")
    s.step(n)
    _, dtg, pg = s.read_probes()
    dg = s.read_diagnostics()
    s.close()
    o = oracle.Oracle(cfg)
    o.step(n)
    _, dto, po = o.probes()
    do = o.diags()
    assert np.abs(dtg / dto - 1).max() < 1e-5
    for k in range(po.shape[1]):
        peak = np.abs(po[:, k]).max()
        assert peak > 1e5, k  # the pulse has reached every probe
        err = np.abs(pg[:, k] - po[:, k]).max() / peak
        print(f"probe {k} at {cfg['probes'][k]}: max err / own peak {err:.3e}")
        assert err <= 1e-3
    assert np.abs(dg["mass"] / dg["mass"][0] - 1).max() <= 1e-12
    assert abs(dg["mass"][0] / do["mass"][0] - 1) <= 1e-12
    for key in ("ke", "e_el", "momx", "w_boundary"):
        assert abs(dg[key][-1] - do[key][-1]) <= 1e-3 * abs(do[key][-1]), key


def test_spherical_pulse_matches_oracle():
    """The acoustic pulse of the oracle's 3D linear-acoustics pin (a Gaussian
    about a point on the axis, no sphere) on both sides from the same rounded
    start, at an amplitude of 2 % of rho0 with the cutoff lifted: at the pin's
    own amplitude (5e-5 rho0) the density change of a step is a few float32
    ulps of rho0, so the FP32 state cannot carry the wave (the oracle with its
    state rounded to FP32 every step is off by about 50 %). The bar is three
    times that storage floor measured here on the oracle at this amplitude
    (about 2e-3 of each probe's peak): per axial probe, the GPU's largest
    history difference over the probe's own peak."""
    s_, xc, eps = 4e-3, 25e-3, 2e-2
    cfg = workloads.axisymmetric(workloads.base(0.06, 0.05, 0.5e-3, 0.0, 0.0, alpha=0.0, delta=0.1))
    cfg.update(disk_R=0.0, n_disk_ghosts=0, p_cav=-1e12, probes=[(xc + d, 0.0) for d in (10e-3, 15e-3, 20e-3)])
    o = oracle.Oracle(cfg)
    t0, (x, y, vx, vy, _) = o.fluid()
    rho = 1000.0 * (1.0 + eps * np.exp(-((x - xc) ** 2 + y ** 2) / s_ ** 2))
    r = shared_state.round_state(cfg, x, y, vx, vy, rho)
    o.set_fluid(t0, *r)
    print("[gpu] axisymmetric spherical pulse", flush=True)
    s = wc.Solver(cfg, "cuda:0")
    s.set_fluid(t0, *r)
    n = 250
    s.step(n)
    o.step(n)
    _, dtg, pg = s.read_probes()
    s.close()
    _, dto, po = o.probes()
    assert np.abs(dtg / dto - 1).max() < 1e-5
    # the storage floor: the oracle with its state rounded to FP32 every step
    b = oracle.Oracle(cfg)
    b.set_fluid(t0, *r)
    b.set_dt_table(dto)
    for _ in range(n):
        b.step(1)
        tb, f = b.fluid()
        b.set_fluid(tb, *shared_state.round_state(cfg, *f))
    _, _, pb = b.probes()
    for k in range(3):
        peak = np.abs(po[:, k]).max()
        err = np.abs(pg[:, k] - po[:, k]).max() / peak
        floor = np.abs(pb[:, k] - po[:, k]).max() / peak
        print(f"pulse probe {k}: max err / own peak {err:.3e} (FP32 storage floor {floor:.3e})")
        assert err <= 3.0 * floor and err <= 1e-2


def test_two_way_sphere_C1():
    """The coupled sphere (kin_mode 2) of the projectile's density: the 3D
    ring force decelerates it on both sides alike."""
    base = workloads.axisymmetric(workloads.C1())
    R = base["disk_R"]
    rho_p = workloads.PROJ_MASS / (4.0 / 3.0 * math.pi * workloads.PROJ_RADIUS ** 3)
    cfg = dict(base, kin_mode=2, disk_mass=rho_p * 4.0 / 3.0 * math.pi * R ** 3)
    n = 200
    print("[gpu] axisymmetric two-way sphere", flush=True)
    s = wc.Solver(cfg, "cuda:0")
    s.step(n)
    xg, vg, _ = s.disk_state()
    dg = s.read_diagnostics()
    s.close()
    o = oracle.Oracle(cfg)
    o.step(n)
    xo, vo, _ = o.disk_state()
    do = o.diags()
    v0 = cfg["kin_v0"]
    print(f"sphere v: gpu {vg:.6f} oracle {vo:.6f}")
    assert vo < v0  # the fluid has taken some of its speed
    assert abs(vg - vo) <= 2e-3 * abs(v0 - vo)
    for key in ("e_disk", "w_boundary"):
        assert abs(dg[key][-1] - do[key][-1]) <= 2e-3 * abs(do[key][-1]), key


def test_batch_equals_single_runs():
    cfgs = [workloads.axisymmetric(workloads.tiny()),
            dict(workloads.axisymmetric(workloads.C1()), alpha=0.05)]
    n = 40
    b = wc.Solver(cfgs, "cuda:0")
    b.step(n)
    for k, cfg in enumerate(cfgs):
        s = wc.Solver(cfg, "cuda:0")
        s.step(n)
        for u, v in zip(b.fluid(k)[1], s.fluid()[1]):
            assert np.array_equal(u, v), k
        assert np.array_equal(b.read_diagnostics(k)["mass"], s.read_diagnostics()["mass"])
        s.close()
    b.close()


def test_axisymmetric_rejections():
    base = workloads.axisymmetric(workloads.tiny())
    for bad in (dict(scheme=1), dict(gravity_y=-9.81), dict(audit=1), dict(disk_y0=1e-3), dict(axisym=2)):
        with pytest.raises(wc.WcsphError):
            wc.Solver(dict(base, **bad), "cuda:0")
    s = wc.Solver(base, "cuda:0")
    s.set_dt_table(np.full(10, 1e-8))
    with pytest.raises(wc.WcsphError):
        s.adj_forward(10, 5)
    s.close()
