"""Beyond the paper's envelope and its verification closures, on the HIP path.

* Quadratic artificial viscosity (beta mu^2 / rho_bar, which the paper
  leaves out): the 80x40 mm channel with beta > 0 against the FP64 oracle,
  probe histories within 1e-3 of each probe's peak; an impact at 1,500 m/s
  (above the paper's 600-900 m/s) with the quadratic term against the oracle
  and stable on the GPU for as long as the disk stays in the channel.
* The verification closures of the paper's Verification Protocols run
  through the GPU: the hydrostatic column at a reduced sound speed (wall and
  interior pressure within 3 % of rho0 |g| (H - y)) and the impulsively
  accelerated disk with the cavitation cutoff lifted (force of the added
  mass pi R^2 rho0 dU/dt within [0.8, 1.8] of the potential-flow value, the
  surface pressure shaped as rho0 R dU/dt cos(theta) + rho0 U^2 (1/2 - 2
  sin^2(theta))); both bars are the oracle's own (coarse lattice); and a
  planar pressure pulse reflected at the rigid ghost wall (R = 1 and twice
  the incident pressure on the wall, within 3 %).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests.test_oracle_physics import _pulse_case, pulse_reflection

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")


def _solver(cfg):
    print(f"[gpu] solver L={cfg['L']} W={cfg['W']} dx={cfg['dx']} v0={cfg['kin_v0']} "
          f"alpha={cfg['alpha']} beta={cfg.get('beta', 0.0)}", flush=True)
    return wc.Solver(cfg, "cuda:0")


def _probe_errors(pg, po):
    return [np.abs(pg[:, k] - po[:, k]).max() / np.abs(po[:, k]).max() for k in range(po.shape[1])]


def test_quadratic_av_C1_matches_oracle():
    cfg = dict(workloads.C1(), alpha=0.05, beta=1.0)
    s = _solver(cfg)
    s.step(200)
    _, dtg, pg = s.read_probes()
    dg = s.read_diagnostics()
    s.close()
    o = oracle.Oracle(cfg)
    o.step(200)
    _, dto, po = o.probes()
    do = o.diags()
    err = _probe_errors(pg, po)
    print("probe errors", [f"{e:.2e}" for e in err])
    assert max(err) <= 1e-3
    assert np.abs(dtg / dto - 1).max() < 1e-5
    for k in ("ke", "e_el", "w_boundary"):
        assert abs(dg[k][-1] - do[k][-1]) <= 1e-3 * abs(do[k][-1]), k


def test_impact_at_1500_m_s_with_quadratic_av():
    v0 = 1500.0
    cfg = dict(workloads.C1(), kin_v0=v0, kin_coef=workloads.K_DRAG * v0 * v0, alpha=0.05, beta=1.0)
    o = oracle.Oracle(cfg)
    o.step(200)
    _, _, po = o.probes()
    s = _solver(cfg)
    s.step(200)
    _, _, pg = s.read_probes()
    err = _probe_errors(pg, po)
    print("1500 m/s probe errors", [f"{e:.2e}" for e in err])
    assert max(err) <= 1e-3
    # keep going while the disk stays well inside the channel (checked on the
    # host from the prescribed law before the steps are launched)
    n_more = 200
    t_end = s.fluid()[0] + n_more * 1.2e-7
    x_end, _, _ = o.kinematics(t_end)
    assert x_end + cfg["disk_R"] < cfg["L"] - 4 * cfg["dx"]
    s.step(n_more)
    d = s.read_diagnostics()
    assert "unstable" not in d
    assert np.abs(d["mass"] - d["mass"][0]).max() <= 1e-12 * d["mass"][0]
    assert s.fluid()[0] < t_end
    s.close()


def test_hydrostatic_column_reduced_c0():
    H = 0.04
    c0 = 10 * math.sqrt(2 * 9.81 * H)
    cfg = workloads.base(0.04, H, 1e-3, 0.0, 0.0, c0=c0)
    cfg.update(disk_R=0.0, n_disk_ghosts=0, init_mode=1,
               probes=[(0.0, 0.01), (0.0, 0.02), (0.0, 0.03), (0.04, 0.02)])
    s = _solver(cfg)
    s.step(3000)
    _, _, p = s.read_probes()
    head = 1000 * 9.81 * H
    for k, (_, y) in enumerate(cfg["probes"]):
        exact = 1000 * 9.81 * (H - y)
        print(f"probe y={y}: {p[-500:, k].mean():.2f} Pa (exact {exact:.2f})")
        assert abs(p[-500:, k].mean() - exact) < 0.03 * head
    _, (x, y, vx, vy, rho) = s.fluid()
    s.close()
    B = 1000 * c0 ** 2 / 7
    pp = B * ((rho / 1000) ** 7 - 1)
    inner = (x > 0.008) & (x < 0.032) & (y > 0.005) & (y < 0.035)
    assert np.abs(pp[inner] - 1000 * 9.81 * (H - y[inner])).max() < 0.03 * head
    assert np.hypot(vx, vy).max() < 1e-2


def test_accelerated_disk_added_mass():
    R, U, tr = 4e-3, 5.0, 50e-6
    Ld = 20 * R
    cfg = workloads.base(Ld, Ld, 1e-3, R, U, alpha=0.0)
    cfg.update(disk_x0=0.5 * Ld, disk_y0=0.5 * Ld, gravity_y=0.0, p_cav=-1e12,
               kin_t_ramp=tr, kin_coef=0.0, probes=[], diag_every=1)
    s = _solver(cfg)
    Ud = U / tr
    while s.fluid()[0] < 0.9 * tr:
        s.step(10)
    d = s.read_diagnostics()
    W, t = d["w_boundary"], d["t"]
    sel = t > 0.5 * tr
    F = np.gradient(W, t)[sel] / (Ud * t[sel])
    Fam = math.pi * R * R * 1000 * Ud
    print(f"force / added-mass force: {(F / Fam).min():.3f} .. {(F / Fam).max():.3f}")
    assert np.all(F / Fam > 0.8) and np.all(F / Fam < 1.8)
    r = s.export_rates()
    gp = r["gp"][-cfg["n_disk_ghosts"]:].astype(np.float64)
    th = 2 * np.pi * np.arange(cfg["n_disk_ghosts"]) / cfg["n_disk_ghosts"]
    v = Ud * s.fluid()[0]
    s.close()
    ref = 1000 * R * Ud * np.cos(th) + 1000 * v * v * (0.5 - 2 * np.sin(th) ** 2)
    corr = np.corrcoef(gp, ref)[0, 1]
    ratio = (gp @ ref) / (ref @ ref)
    print(f"surface pressure: correlation {corr:.3f}, projection {ratio:.3f}")
    assert corr > 0.9
    assert 0.8 < ratio < 1.5


def test_rigid_wall_reflects_a_pressure_pulse():
    cfg, init, n, t_wall = _pulse_case()
    s = _solver(cfg)
    x, y, vx, vy, rho = init.T
    s.set_fluid(0.0, x, y, vx, vy, rho)
    s.step(n)
    t, _, p = s.read_probes()
    s.close()
    R, wall = pulse_reflection(t, p.astype(np.float64), t_wall)
    print(f"R = {R:.4f}, wall / (2 incident) = {wall:.4f}")
    assert abs(R - 1.0) <= 0.03 and abs(wall - 1.0) <= 0.03
