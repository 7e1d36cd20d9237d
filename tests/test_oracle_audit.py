"""Energy audit of eq. energy-audit in the FP64 oracle, term by term.

The oracle integrates, from the midpoint rates of every step, the
irreversible dissipation of the artificial and laminar viscosity between
fluid particles (d_av, d_visc), the elastic energy rate of the delta
diffusion (w_delta) and the fluid energy rate of every fluid-ghost pair term
(w_ghost), and it adds the energy the corrector's enforcement and density
clamp change (w_enforce, w_clamp).

Pins:
* For any state, the energy rate of the fluid computed from the per-particle
  rates (sum_i m_i (v_i.a_i + P_i drho_i - v_i.g)) equals the audit rates
  w_ghost' - d_av' - d_visc' + w_delta'. Between fluid particles the pressure
  work cancels the elastic energy rate pair by pair, so this holds to
  rounding; it fixes the signs, the halves of the pair terms and the masses.
* With the fluid at rest near every wall and the disk, each dissipation rate
  equals minus the power of its own force (the rates with the coefficient
  minus the rates without it), and the delta rate equals the elastic energy
  rate of its density change.
* The dissipations never decrease and vanish with their coefficient.
* Over whole runs the ledger closes: the change of ke + e_el + e_pot equals
  w_ghost - d_av - d_visc + w_delta + w_enforce + w_clamp to 2 % of w_ghost
  (what is left is the midpoint rule across enforcement and cutoff events;
  dropping any single term leaves 6 % or more).
"""
import numpy as np
import pytest

import oracle
import workloads


def _pressure_term(cfg, rho):
    """P = p / rho^2 of the Tait law with its cutoff."""
    return np.array([oracle.eos(cfg, r)[0] for r in rho]) / rho ** 2


def _state(cfg, seed, quiet=0.0):
    """The lattice of cfg with seeded velocities (50 m/s scale) and density
    (+-1 %), at rest within `quiet` of the walls and the disk."""
    o = oracle.Oracle(cfg)
    _, (x, y, _, _, _) = o.fluid()
    rng = np.random.default_rng(seed)
    vx = rng.normal(0.0, 50.0, x.size)
    vy = rng.normal(0.0, 50.0, x.size)
    rho = cfg["rho0"] * (1.0 + rng.uniform(-0.01, 0.01, x.size))
    if quiet > 0.0:
        dwall = np.minimum.reduce([x, cfg["L"] - x, y, cfg["W"] - y])
        ddisk = np.hypot(x - cfg["disk_x0"], y - cfg["disk_y0"]) - cfg["disk_R"]
        calm = np.minimum(dwall, ddisk) < quiet
        vx[calm] = 0.0
        vy[calm] = 0.0
    return np.stack([x, y, vx, vy, rho], 1)


def _rates(cfg, init):
    o = oracle.Oracle(cfg, init=init)
    r = o.eval_rates()
    return r, o.audit_rates()


def test_energy_rate_identity_on_any_state():
    cfg = dict(workloads.tiny(), mu_dyn=5.0, alpha=0.2)
    init = _state(cfg, 11)
    r, a = _rates(cfg, init)
    _, _, vx, vy, rho = init.T
    m = cfg["rho0"] * cfg["dx"] ** 2
    g = cfg["gravity_y"]
    P = _pressure_term(cfg, rho)
    ke_rate = m * (vx * r["ax"] + vy * (r["ay"] - g))
    el_rate = m * P * r["drho"]
    lhs = ke_rate.sum() + el_rate.sum()
    rhs = a["w_ghost"] - a["d_av"] - a["d_visc"] + a["w_delta"]
    scale = np.abs(ke_rate).sum() + np.abs(el_rate).sum()
    assert a["d_av"] > 0 and a["d_visc"] > 0 and a["w_ghost"] != 0 and a["w_delta"] != 0
    assert abs(lhs - rhs) <= 1e-11 * scale, (lhs, rhs, scale)


@pytest.mark.parametrize("coef", ["alpha", "mu_dyn", "delta"])
def test_each_term_equals_the_power_of_its_own_force(coef):
    base = dict(workloads.tiny(), alpha=0.2, mu_dyn=5.0, delta=0.1)
    h = base["h_over_dx"] * base["dx"]
    init = _state(base, 5, quiet=3.0 * h)
    r_on, a_on = _rates(base, init)
    r_off, a_off = _rates(dict(base, **{coef: 0.0}), init)
    _, _, vx, vy, rho = init.T
    m = base["rho0"] * base["dx"] ** 2
    # no fluid moves near a ghost, so no ghost pair term does work
    assert a_on["w_ghost"] == 0.0 and a_off["w_ghost"] == 0.0
    power = m * (vx * (r_on["ax"] - r_off["ax"]) + vy * (r_on["ay"] - r_off["ay"]))
    if coef == "alpha":
        assert a_off["d_av"] == 0.0 and a_on["d_av"] > 0.0
        assert abs(power.sum() + a_on["d_av"]) <= 1e-11 * np.abs(power).sum()
    elif coef == "mu_dyn":
        assert a_off["d_visc"] == 0.0 and a_on["d_visc"] > 0.0
        assert abs(power.sum() + a_on["d_visc"]) <= 1e-11 * np.abs(power).sum()
    else:
        el = m * _pressure_term(base, rho) * (r_on["drho"] - r_off["drho"])
        assert a_off["w_delta"] == 0.0 and a_on["w_delta"] != 0.0
        assert abs(el.sum() - a_on["w_delta"]) <= 1e-11 * np.abs(el).sum()


def test_dissipation_never_decreases_and_vanishes_without_its_coefficient():
    cfg = workloads.C1()
    o = oracle.Oracle(cfg)
    o.step(100)
    d = o.diags()
    assert d["d_av"][-1] > 0 and d["d_visc"][-1] > 0
    assert np.all(np.diff(d["d_av"]) >= 0) and np.all(np.diff(d["d_visc"]) >= 0)
    o = oracle.Oracle(dict(cfg, alpha=0.0, mu_dyn=0.0, delta=0.0))
    o.step(60)
    d = o.diags()
    assert np.all(d["d_av"] == 0) and np.all(d["d_visc"] == 0) and np.all(d["w_delta"] == 0)


@pytest.mark.parametrize("mode", ["two_way", "prescribed"])
def test_ledger_closes_over_a_run(mode):
    cfg = workloads.C1()
    if mode == "two_way":
        cfg = workloads.two_way(cfg)
    o = oracle.Oracle(cfg)
    o.step(200)
    d = o.diags()
    e = d["ke"] + d["e_el"] + d["e_pot"]
    terms = {k: d[k][-1] for k in ("w_ghost", "d_av", "d_visc", "w_delta", "w_enforce", "w_clamp")}
    ledger = (terms["w_ghost"] - terms["d_av"] - terms["d_visc"] + terms["w_delta"] + terms["w_enforce"]
              + terms["w_clamp"])
    resid = (e[-1] - e[0]) - ledger
    print(mode, {k: round(v, 3) for k, v in terms.items()}, "residual", resid)
    assert abs(resid) <= 0.02 * abs(terms["w_ghost"])
    # the terms the pins above cannot see matter here: each is over 3x the residual
    for k in ("d_av", "w_delta", "w_enforce"):
        assert abs(terms[k]) >= 3.0 * abs(resid), k
