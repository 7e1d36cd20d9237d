"""The Mie-Grueneisen EOS of eq. eos in the FP64 oracle (eos_type 1), with
the specific internal energy held at zero (no energy equation is evolved).

Pins, each from something other than the oracle's own formula:
* With gamma0 = 0 the law is the linear Us-Up Hugoniot itself: for a piston
  speed Up, the shock speed Us = C + S1 Up, the mass jump
  rho0 Us = rho (Us - Up) and the momentum jump p = rho0 Us Up, solved here
  for Up at each density.
* With gamma0 > 0 and e = 0 it is the Grueneisen relation taken off that
  Hugoniot at constant Gamma rho = gamma0 rho0: p = p_H - gamma0 rho0 e_H,
  with the Hugoniot energy e_H = p_H (1/rho0 - 1/rho) / 2 of the energy jump.
* Tension is the acoustic line rho0 C^2 mu down to the cavitation cutoff,
  compression is capped at mu = 0.25, and the two branches meet at rho0 with
  slope C^2.
* The sound speed is sqrt(dp/drho) (central differences); the inverse
  returns the density; the elastic energy is the integral of p / rho^2
  (adaptive quadrature).
* The hydrostatic start holds rho0 |g| (W - y), and over a whole C1 run the
  energy ledger closes as it does for Tait, which ties e_el to the pressure
  the dynamics uses.
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import oracle
import workloads


def _cfg(**kw):
    return dict(workloads.mie_grueneisen(workloads.C1()), **kw)


def _hugoniot_pressure(cfg, rho):
    """p of the linear Us-Up Hugoniot through (rho0, p = 0) at density rho,
    from the jump conditions: find Up with rho0 Us = rho (Us - Up)."""
    r0, C, S1 = cfg["rho0"], cfg["c0"], cfg["mg_s1"]

    def mass_jump(up):
        us = C + S1 * up
        return r0 * us - rho * (us - up)

    up = optimize.brentq(mass_jump, 0.0, 5.0 * C, xtol=1e-14, rtol=1e-15)
    return r0 * (C + S1 * up) * up


RHO_COMP = [1000.5, 1010.0, 1050.0, 1100.0, 1180.0, 1249.0]


@pytest.mark.parametrize("rho", RHO_COMP)
def test_gamma0_zero_is_the_linear_us_up_hugoniot(rho):
    cfg = _cfg(mg_gamma0=0.0)
    p, _ = oracle.eos(cfg, rho)
    ph = _hugoniot_pressure(cfg, rho)
    assert abs(p - ph) <= 1e-12 * ph, (p, ph)


@pytest.mark.parametrize("rho", RHO_COMP)
def test_zero_energy_is_the_grueneisen_offset_from_the_hugoniot(rho):
    cfg = _cfg()
    p, _ = oracle.eos(cfg, rho)
    ph = _hugoniot_pressure(cfg, rho)
    eh = 0.5 * ph * (1.0 / cfg["rho0"] - 1.0 / rho)
    expect = ph - cfg["mg_gamma0"] * cfg["rho0"] * eh
    assert abs(p - expect) <= 1e-12 * ph, (p, expect)
    # and it sits below the Hugoniot, by the gamma0 share of its energy
    assert p < ph


def test_tension_branch_cutoff_and_cap():
    cfg = _cfg()
    r0, C = cfg["rho0"], cfg["c0"]
    K = r0 * C * C
    for mu in (-1e-8, -1e-6, -2e-5, -4.5e-5):
        p, c = oracle.eos(cfg, r0 * (1.0 + mu))
        # (rho0 (1 + mu) / rho0 - 1 carries an absolute rounding of about 1e-16)
        assert abs(p - K * mu) <= 1e-15 * K and c == pytest.approx(C, rel=1e-15)
    mu_cav = cfg["p_cav"] / K
    for mu in (1.01 * mu_cav, -1e-3, -0.2):
        assert oracle.eos(cfg, r0 * (1.0 + mu))[0] == cfg["p_cav"]
    p_cap, c_cap = oracle.eos(cfg, r0 * 1.25)
    for rho in (1260.0, 1400.0, 1490.0):
        p, c = oracle.eos(cfg, rho)
        assert p == p_cap and c == c_cap
    # below the cap p keeps rising
    assert oracle.eos(cfg, 1249.0)[0] < p_cap


def test_branches_meet_at_rho0_with_slope_c_squared():
    cfg = _cfg()
    r0, C = cfg["rho0"], cfg["c0"]
    assert oracle.eos(cfg, r0) == (0.0, C)
    eps = 1e-6 * r0
    right = oracle.eos(cfg, r0 + eps)[0] / eps
    left = -oracle.eos(cfg, r0 - eps)[0] / eps
    assert right == pytest.approx(C * C, rel=1e-5)
    assert left == pytest.approx(C * C, rel=1e-9)  # the rounding of rho0 - eps in mu


@pytest.mark.parametrize("rho", [999.97, 1000.2, 1020.0, 1100.0, 1200.0, 1240.0])
def test_sound_speed_is_the_slope_of_the_law(rho):
    cfg = _cfg()
    h = 1e-4
    dp = (oracle.eos(cfg, rho + h)[0] - oracle.eos(cfg, rho - h)[0]) / (2 * h)
    c = oracle.eos(cfg, rho)[1]
    assert c * c == pytest.approx(dp, rel=1e-7)


@pytest.mark.parametrize("rho", [999.96, 999.999, 1000.0, 1003.0, 1080.0, 1200.0, 1250.0])
def test_inverse(rho):
    cfg = _cfg()
    p, _ = oracle.eos(cfg, rho)
    assert oracle.eos_rho(cfg, p) == pytest.approx(rho, rel=1e-13, abs=1e-12)
    # beyond the cap the inverse returns the cap
    p_hi = oracle.eos(cfg, 1300.0)[0]
    assert oracle.eos_rho(cfg, p_hi) == pytest.approx(1250.0, rel=1e-13)


@pytest.mark.parametrize("rho", [900.0, 999.9, 999.97, 1000.0, 1000.3, 1050.0, 1200.0, 1250.0, 1400.0])
def test_elastic_energy_is_the_integral_of_p_over_rho_squared(rho):
    cfg = _cfg()
    r0 = cfg["rho0"]
    K = r0 * cfg["c0"] ** 2
    rho_cav = r0 * (1.0 + cfg["p_cav"] / K)
    f = lambda r: oracle.eos(cfg, r)[0] / (r * r)
    pts = [q for q in (rho_cav, 1250.0) if min(r0, rho) < q < max(r0, rho)]
    ref, _ = integrate.quad(f, r0, rho, points=pts or None, epsabs=0.0, epsrel=1e-13, limit=200)
    e = oracle.elastic_energy(cfg, rho)
    assert abs(e - ref) <= 1e-11 * max(abs(ref), 1e-9), (e, ref)


def test_hydrostatic_start_holds_the_column_pressure():
    H = 0.04
    cfg = workloads.mie_grueneisen(workloads.base(0.04, H, 1e-3, 0.0, 0.0))
    cfg.update(disk_R=0.0, n_disk_ghosts=0, init_mode=1, probes=[])
    o = oracle.Oracle(cfg)
    _, (x, y, _, _, rho) = o.fluid()
    p = np.array([oracle.eos(cfg, r)[0] for r in rho])
    exact = cfg["rho0"] * abs(cfg["gravity_y"]) * (H - y)
    assert np.abs(p - exact).max() <= 1e-9 * exact.max()


def test_run_conserves_mass_and_closes_the_energy_ledger():
    cfg = _cfg()
    o = oracle.Oracle(cfg)
    o.step(200)
    d = o.diags()
    assert np.abs(d["mass"] - d["mass"][0]).max() <= 1e-12 * d["mass"][0]
    e = d["ke"] + d["e_el"] + d["e_pot"]
    terms = {k: d[k][-1] for k in ("w_ghost", "d_av", "d_visc", "w_delta", "w_enforce", "w_clamp")}
    ledger = (terms["w_ghost"] - terms["d_av"] - terms["d_visc"] + terms["w_delta"] + terms["w_enforce"]
              + terms["w_clamp"])
    resid = (e[-1] - e[0]) - ledger
    print({k: round(v, 3) for k, v in terms.items()}, "residual", resid)
    assert abs(resid) <= 0.02 * abs(terms["w_ghost"])
    # the pulse is the same acoustic event as with Tait: the probe peaks agree to O(Ma^2)
    _, _, p_mg = o.probes()
    t = dict(cfg, eos_type=0)
    ot = oracle.Oracle(t)
    ot.step(200)
    _, _, p_t = ot.probes()
    ratio = np.abs(p_mg).max(0) / np.abs(p_t).max(0)
    print("MG / Tait probe peaks", ratio)
    assert np.all(ratio > 0.8) and np.all(ratio < 1.25)
    assert math.isfinite(d["e_el"][-1])
