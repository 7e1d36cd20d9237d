"""Pins of the oracle's scheme 1, the paper's scheme as published: summation
density (eq. density-sum) over fluid and ghosts with the [0.5, 1.5] rho0
clamp (Density Summation), the leapfrog update (Time Integration), and the
specific internal energy of eq. eos heated by the artificial viscosity.

Each test checks the oracle against something other than its own formulas:
* the undisturbed lattice sums to rho0 with the lattice-normalised mass, in
  the bulk and next to the walls (which the ghost layers complete), and the
  mass tends to rho0 dx^2 as the kernel's support widens (partition of unity);
* a compressed block is clamped to exactly 1.5 rho0 and counted;
* free fall of an isolated block with every pair term switched off is the
  closed form y = y0 + g t^2 / 2, v(t + dt/2) = g (t + dt/2) at every step of
  a varying time-step table (the merged kick and the half kick at the start);
* with only pressure acting, the leapfrog keeps momentum exactly and the
  energy ke + sum m e_el(rho) to second order in dt (error ratio ~4 when dt
  halves) with no drift;
* the artificial-viscosity heating equals the kinetic energy the same pairs
  remove: sum m v.a + sum m de/dt = 0, and it is linear in alpha;
* without the artificial viscosity the internal energy stays zero;
* the energy term of eq. eos at mu = 0 is gamma0 rho0 e, and the law is
  continuous across mu = 0 for e > 0.
"""
import numpy as np
import pytest

import oracle
import workloads


def _scheme1(cfg, **kw):
    c = workloads.paper_scheme(cfg)
    c.update(kw)
    return c


@pytest.mark.parametrize("kernel_type", [0, 1])
def test_undisturbed_lattice_sums_to_rho0(kernel_type):
    """No disk, three ghost layers: every fluid particle, the ones next to the
    walls included, sums to rho0 (the ghosts complete the support)."""
    cfg = _scheme1(workloads.C1(), kernel_type=kernel_type, disk_R=0.0, n_disk_ghosts=0)
    o = oracle.Oracle(cfg)
    rho, p = o.eval_density()
    assert np.abs(rho / cfg["rho0"] - 1).max() < 1e-12
    # with one ghost layer the rows next to the walls lack part of their support
    o1 = oracle.Oracle(dict(cfg, ghost_layers=1))
    r1, _ = o1.eval_density()
    assert r1.min() < 0.999 * cfg["rho0"]
    assert np.median(r1) == pytest.approx(cfg["rho0"], rel=1e-12)


@pytest.mark.parametrize("kernel_type,h_over_dx,tol", [(0, 2.0, 2e-3), (1, 2.0, 2e-3), (0, 1.3, 1.1e-2),
                                                     (1, 1.3, 1e-4)])
def test_lattice_mass_tends_to_rho0_dx2(kernel_type, h_over_dx, tol):
    """The kernel sum of a square lattice approximates int W = 1 / dx^2, so
    the normalised mass approaches rho0 dx^2."""
    cfg = dict(workloads.C1(), kernel_type=kernel_type, h_over_dx=h_over_dx)
    m = oracle.lattice_mass(cfg)
    assert abs(m / (cfg["rho0"] * cfg["dx"] ** 2) - 1) < tol


def _block(cfg, nx, ny, x0, y0, spacing):
    gx, gy = np.meshgrid(x0 + spacing * np.arange(nx), y0 + spacing * np.arange(ny))
    n = gx.size
    return np.column_stack([gx.ravel(), gy.ravel(), np.zeros(n), np.zeros(n), np.full(n, cfg["rho0"])])


def test_compressed_block_is_clamped():
    cfg = _scheme1(workloads.C1(), disk_R=0.0, n_disk_ghosts=0, gravity_y=0.0, eos_type=0, c0=1480.0)
    dx = cfg["dx"]
    init = _block(cfg, 12, 12, 0.03, 0.012, 0.6 * dx)
    o = oracle.Oracle(cfg, init)
    rho, _ = o.eval_density()
    assert rho.max() == 1.5 * cfg["rho0"]
    n_hi = int((rho == 1.5 * cfg["rho0"]).sum())
    assert n_hi > 50
    o.step(cfg["diag_every"])  # one diagnostic record
    assert o.diags()["n_clamp"][-1] >= n_hi


def _isolated(cfg, nx=10, ny=10):
    """A block of fluid in the middle of a large box, more than 2h from every
    wall, with no disk."""
    dx = cfg["dx"]
    return _block(cfg, nx, ny, 0.030 + 0.5 * dx, 0.020 + 0.5 * dx, dx)


def test_free_fall_is_exact_with_a_varying_step():
    cfg = _scheme1(workloads.C1(), disk_R=0.0, n_disk_ghosts=0, alpha=0.0, mu_dyn=0.0, eps_xsph=0.0,
                   eos_type=0, c0=1480.0, p_cav=0.0, gravity_y=-9.81e6)
    init = _isolated(cfg)
    o = oracle.Oracle(cfg, init)
    rng = np.random.default_rng(5)
    dts = 1e-7 * (1.0 + rng.random(40))
    o.set_dt_table(dts)
    g = cfg["gravity_y"]
    t = 0.0
    for n in range(40):
        o.step(1)
        t_half = t + 0.5 * dts[n]
        t += dts[n]
        _, (x, y, vx, vy, _) = o.fluid()
        assert np.abs(vy - g * t_half).max() <= 1e-12 * abs(g * t_half)
        # (the bulk pressure is zero up to the rounding of the density sum)
        assert np.abs(vx).max() <= 1e-12 * abs(g * t_half)
        dy = y - init[:, 1]
        assert np.abs(dy - 0.5 * g * t * t).max() <= 1e-9 * abs(0.5 * g * t * t)
        assert np.abs(x - init[:, 0]).max() <= 1e-12 * cfg["dx"]
    assert np.all(o.energy() == 0.0)


def _energy_run(cfg, init, dt, n):
    """ke at whole steps (the mean of the two half-step velocities) plus the
    elastic energy of the summed density at the same positions."""
    o = oracle.Oracle(cfg, init)
    o.set_dt_table(np.full(n, dt))
    m = oracle.lattice_mass(cfg)
    E, P = [], []
    rho, _ = o.eval_density()
    v_prev = None
    for k in range(n):
        _, (x, y, vx, vy, _) = o.fluid()
        eel = sum(oracle.elastic_energy(cfg, r) for r in rho)
        if v_prev is not None:
            ux, uy = 0.5 * (v_prev[0] + vx), 0.5 * (v_prev[1] + vy)
            E.append(0.5 * m * (ux * ux + uy * uy).sum() + m * eel_prev)
        P.append((m * vx.sum(), m * vy.sum()))
        o.step(1)
        v_prev = (vx, vy)
        eel_prev = eel
        rho, _ = o.eval_density()
    _, (x, y, vx, vy, _) = o.fluid()
    ux, uy = 0.5 * (v_prev[0] + vx), 0.5 * (v_prev[1] + vy)
    E.append(0.5 * m * (ux * ux + uy * uy).sum() + m * eel_prev)
    return np.array(E), np.array(P)


def test_leapfrog_conserves_momentum_and_energy_to_second_order():
    """An isolated block under its own pressure only (tension at its edges,
    held at the cutoff), from rest: momentum stays zero, and the energy error
    at dt/2 is about a quarter of that at dt."""
    cfg = _scheme1(workloads.C1(), disk_R=0.0, n_disk_ghosts=0, alpha=0.0, mu_dyn=0.0, eps_xsph=0.0,
                   eos_type=0, c0=1480.0, gravity_y=0.0, rho_lo=0.05)
    init = _isolated(cfg, 8, 8)
    # a compressed centre: density above rho0 in the middle, so pressure drives the motion
    cx, cy = init[:, 0].mean(), init[:, 1].mean()
    init[:, 0] = cx + (init[:, 0] - cx) * 0.97
    init[:, 1] = cy + (init[:, 1] - cy) * 0.97
    dt = 2.0e-8
    E1, P1 = _energy_run(cfg, init, dt, 60)
    E2, P2 = _energy_run(cfg, init, dt / 2, 120)
    scale = np.abs(E1).max()
    assert np.abs(P1).max() <= 1e-12 * scale ** 0.5 + 1e-15
    assert np.abs(P2).max() <= 1e-12 * scale ** 0.5 + 1e-15
    err1 = np.abs(E1 - E1[0]).max() / scale
    err2 = np.abs(E2 - E2[0]).max() / scale
    print(f"energy error dt {err1:.3e}, dt/2 {err2:.3e}, ratio {err1 / err2:.2f}")
    assert err1 < 1e-3
    assert 3.0 < err1 / err2 < 5.0


def _random_velocity_block(cfg, seed=7):
    init = _isolated(cfg, 12, 12)
    rng = np.random.default_rng(seed)
    init[:, 2] = 50.0 * rng.standard_normal(init.shape[0])
    init[:, 3] = 50.0 * rng.standard_normal(init.shape[0])
    return init


def test_av_heating_balances_the_kinetic_energy_it_removes():
    """Pressure held at zero (p_cav = 0 with every summed density <= rho0),
    no gravity, laminar or XSPH: a_i is the artificial viscosity alone and
    sum_i m v_i.a_i = -sum_i m de_i/dt exactly, pair by pair."""
    cfg = _scheme1(workloads.C1(), disk_R=0.0, n_disk_ghosts=0, mu_dyn=0.0, eps_xsph=0.0, eos_type=0,
                   c0=1480.0, p_cav=0.0, gravity_y=0.0, alpha=0.1)
    init = _random_velocity_block(cfg)
    o = oracle.Oracle(cfg, init)
    r = o.eval_rates()
    rho, p = o.eval_density()
    assert np.abs(p).max() < 1e-3  # zero up to the rounding of the density sum
    m = oracle.lattice_mass(cfg)
    work = m * (init[:, 2] * r["ax"] + init[:, 3] * r["ay"]).sum()
    heat = m * r["drho"].sum()
    assert heat > 0.0
    assert abs(work + heat) <= 1e-10 * heat
    assert np.all(r["drho"] >= 0.0)
    r2 = oracle.Oracle(dict(cfg, alpha=0.3), init).eval_rates()
    assert np.abs(r2["drho"] - 3.0 * r["drho"]).max() <= 1e-12 * np.abs(r["drho"]).max()


def test_no_artificial_viscosity_no_heating():
    cfg = _scheme1(workloads.C1(), disk_R=0.0, n_disk_ghosts=0, alpha=0.0, gravity_y=0.0)
    o = oracle.Oracle(cfg, _random_velocity_block(cfg))
    o.step(20)
    assert np.all(o.energy() == 0.0)
    assert o.diags()["e_th"][-1] == 0.0


def test_energy_term_of_the_eos():
    cfg = _scheme1(workloads.C1())
    r0, e = cfg["rho0"], 2.0e4
    assert oracle.eos_pe(cfg, r0, e) == pytest.approx(cfg["mg_gamma0"] * r0 * e, rel=1e-12)
    lo, hi = oracle.eos_pe(cfg, r0 * (1 - 1e-9), e), oracle.eos_pe(cfg, r0 * (1 + 1e-9), e)
    # no jump at mu = 0: the change over |d mu| = 2e-9 is the slope's
    slope = cfg["rho0"] * cfg["c0"] ** 2 + (cfg["mg_gamma0"] + cfg["mg_a"]) * r0 * e
    assert abs(hi - lo) <= 1.1 * slope * 2e-9
    # at e = 0 the law is the one the other scheme uses
    for rho in (0.9 * r0, r0, 1.1 * r0, 1.3 * r0):
        assert oracle.eos_pe(cfg, rho, 0.0) == oracle.eos(cfg, rho)[0]
    # e raises the pressure at fixed density (gamma0 + a mu > 0)
    assert oracle.eos_pe(cfg, 1.1 * r0, e) > oracle.eos(cfg, 1.1 * r0)[0]


def test_scheme1_run_records_internal_energy():
    """C1 with the paper's scheme: the disk heats the fluid through the
    artificial viscosity; e >= 0 everywhere and the record's e_th is its sum."""
    cfg = _scheme1(workloads.C1())
    o = oracle.Oracle(cfg)
    o.step(40)
    e = o.energy()
    assert e.min() >= 0.0 and e.max() > 0.0
    d = o.diags()
    m = oracle.lattice_mass(cfg)
    assert d["e_th"][-1] == pytest.approx(m * e.sum(), rel=1e-12)
    assert d["mass"][-1] == pytest.approx(m * o.nf, rel=1e-12)


def test_coupled_disk_not_built_for_scheme1():
    with pytest.raises(ValueError):
        oracle.Oracle(workloads.two_way(_scheme1(workloads.C1())))


def test_internal_energy_advances_by_the_step_times_its_rate():
    """e^(n+1) = e^n + dt^n de/dt^n over two steps of unequal dt, with the
    rate of each step's own evaluation (a second oracle taken to the same
    state evaluates it)."""
    cfg = _scheme1(workloads.C1(), disk_R=0.0, n_disk_ghosts=0, mu_dyn=0.0, gravity_y=0.0, alpha=0.1)
    init = _random_velocity_block(cfg)
    dts = np.array([1.0e-8, 1.7e-8])
    o = oracle.Oracle(cfg, init)
    o.set_dt_table(dts)
    ref = oracle.Oracle(cfg, init)
    ref.set_dt_table(dts)
    e_prev = np.zeros(o.nf)
    for n in range(2):
        rate = ref.eval_rates()["drho"]
        ref.step(1)
        o.step(1)
        e = o.energy()
        assert np.abs(e - (e_prev + dts[n] * rate)).max() <= 1e-12 * np.abs(e).max()
        e_prev = e
