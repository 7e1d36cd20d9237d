"""Quadratic artificial viscosity (beta mu^2 / rho_bar) in the FP64 oracle.

The paper keeps only the linear term of the Monaghan form
(eq. artificial-viscosity) and names the quadratic one for impacts beyond its
envelope. Pins:
* two fluid particles closing head on at the speed where |mu_ij| = c_bar:
  the quadratic term with beta = a equals the linear term with alpha = a;
  doubling the speed doubles the linear term and quadruples the quadratic
  one; separating particles feel neither;
* with beta > 0 the audit's dissipation still equals the power of the
  artificial-viscosity force (the term is dissipative and enters the
  momentum and the audit the same way);
* momentum is conserved pairwise with beta > 0.
"""
import numpy as np
import pytest

import oracle
import workloads


def _pair_ax(cfg, u, r):
    """x acceleration of particle 0 of a pair on the x axis, 0 at the
    origin moving at +u/2, 1 at x = r moving at -u/2; no pressure."""
    rho0 = cfg["rho0"]
    m = rho0 * cfg["dx"] ** 2
    out = oracle.pair_rates(cfg, [0.0, r], [0.0, 0.0], [0.5 * u, -0.5 * u], [0.0, 0.0],
                            [rho0, rho0], [0.0, 0.0], [m, m], [0, 0])
    return out["ax"][0]


def _clean(cfg, **kw):
    return dict(cfg, delta=0.0, mu_dyn=0.0, eps_xsph=0.0, gravity_y=0.0, **kw)


def test_quadratic_term_equals_linear_term_where_mu_equals_c_bar():
    base = workloads.tiny()
    h = base["h_over_dx"] * base["dx"]
    r = 1.1 * h
    c = base["c0"]  # both particles at rho0
    u = c * (r * r + base["eta2"] * h * h) / (h * r)  # |mu| = h u r / (r^2 + eta^2 h^2) = c_bar
    lin = _pair_ax(_clean(base, alpha=0.3, beta=0.0), u, r)
    quad = _pair_ax(_clean(base, alpha=0.0, beta=0.3), u, r)
    assert lin < 0.0  # particle 0 moves toward +x and is pushed back
    assert abs(quad - lin) <= 1e-12 * abs(lin)
    # orders in the closing speed
    lin2 = _pair_ax(_clean(base, alpha=0.3, beta=0.0), 2 * u, r)
    quad2 = _pair_ax(_clean(base, alpha=0.0, beta=0.3), 2 * u, r)
    assert abs(lin2 / lin - 2.0) <= 1e-12 and abs(quad2 / quad - 4.0) <= 1e-12
    # separating: no artificial viscosity at all
    assert _pair_ax(_clean(base, alpha=0.3, beta=0.3), -u, r) == 0.0


def _state(cfg, seed, quiet):
    o = oracle.Oracle(cfg)
    _, (x, y, _, _, _) = o.fluid()
    rng = np.random.default_rng(seed)
    vx = rng.normal(0.0, 200.0, x.size)
    vy = rng.normal(0.0, 200.0, x.size)
    rho = cfg["rho0"] * (1.0 + rng.uniform(-0.01, 0.01, x.size))
    dwall = np.minimum.reduce([x, cfg["L"] - x, y, cfg["W"] - y])
    ddisk = np.hypot(x - cfg["disk_x0"], y - cfg["disk_y0"]) - cfg["disk_R"]
    calm = np.minimum(dwall, ddisk) < quiet
    vx[calm] = 0.0
    vy[calm] = 0.0
    return np.stack([x, y, vx, vy, rho], 1)


def test_quadratic_term_dissipates_as_its_force_works():
    base = dict(workloads.tiny(), alpha=0.1)
    h = base["h_over_dx"] * base["dx"]
    init = _state(base, 3, 3.0 * h)
    rates = {}
    for beta in (0.0, 2.0):
        o = oracle.Oracle(dict(base, beta=beta), init=init)
        rates[beta] = (o.eval_rates(), o.audit_rates())
    _, _, vx, vy, _ = init.T
    m = base["rho0"] * base["dx"] ** 2
    (r0, a0), (r1, a1) = rates[0.0], rates[2.0]
    power = m * (vx * (r1["ax"] - r0["ax"]) + vy * (r1["ay"] - r0["ay"]))
    extra = a1["d_av"] - a0["d_av"]
    assert extra > 0.0
    assert abs(power.sum() + extra) <= 1e-11 * np.abs(power).sum()


def test_momentum_conserved_pairwise_with_quadratic_term():
    cfg = _clean(workloads.tiny(), alpha=0.1, beta=2.0)
    rng = np.random.default_rng(9)
    n = 40
    x = rng.uniform(0.0, 4e-3, n)
    y = rng.uniform(0.0, 4e-3, n)
    vx = rng.normal(0.0, 300.0, n)
    vy = rng.normal(0.0, 300.0, n)
    rho = cfg["rho0"] * (1.0 + rng.uniform(-0.02, 0.02, n))
    pres = np.array([oracle.eos(cfg, r)[0] for r in rho])
    m = np.full(n, cfg["rho0"] * cfg["dx"] ** 2)
    out = oracle.pair_rates(cfg, x, y, vx, vy, rho, pres, m, np.zeros(n, np.int32))
    fx, fy = (m * out["ax"]).sum(), (m * out["ay"]).sum()
    scale = (m * np.abs(out["ax"])).sum() + (m * np.abs(out["ay"])).sum()
    assert abs(fx) <= 1e-12 * scale and abs(fy) <= 1e-12 * scale
