"""The tabulated prescribed disk motion (kin_mode 3) of the oracle: rows
(t, x, v, a) interpolated linearly per column, extrapolated at the end rows'
velocity. Pins: the rows themselves, midpoints and extrapolation against the
definition written out by hand; and a table sampled from the closed-form ramp
and constant deceleration (eq. velocity-ramp, eq. drag at v0) reproducing that
law's run (the velocity is piecewise linear in both, so only the position
carries the interpolation error a dt^2 / 8)."""
import numpy as np

import oracle
import workloads


def test_table_rows_midpoints_and_extrapolation():
    cfg = dict(workloads.tiny(), kin_mode=3)
    o = oracle.Oracle(cfg)
    rows = np.array([[0.0, 3e-3, 0.0, 4e7],
                     [2e-6, 3.05e-3, 80.0, 4e7],
                     [5e-6, 3.4e-3, 200.0, -1e6]])
    o.set_kin_table(rows)
    for t, x, v, a in rows:
        assert o.kinematics(t) == (x, v, a)
    x, v, a = o.kinematics(3.5e-6)  # halfway through the second interval
    assert abs(x - 0.5 * (3.05e-3 + 3.4e-3)) < 1e-18 and abs(v - 140.0) < 1e-12
    assert abs(a - 0.5 * (4e7 - 1e6)) < 1e-6
    x, v, a = o.kinematics(7e-6)  # past the last row: on at its velocity
    assert abs(x - (3.4e-3 + 200.0 * 2e-6)) < 1e-18 and v == 200.0 and a == 0.0
    x, v, a = o.kinematics(-1e-6)
    assert x == 3e-3 and v == 0.0 and a == 0.0


def ramp_decel_table(cfg, t_end, dt_row):
    """Rows of the closed-form ramp then constant deceleration, with a row at
    the end of the ramp."""
    v0, tr, ad, x0 = cfg["kin_v0"], cfg["kin_t_ramp"], cfg["kin_coef"], cfg["disk_x0"]
    ts = np.unique(np.concatenate([np.arange(0.0, t_end, dt_row), [tr, t_end]]))
    rows = []
    for t in ts:
        if t < tr:
            rows.append((t, x0 + 0.5 * v0 * t * t / tr, v0 * t / tr, v0 / tr))
        else:
            tau = t - tr
            rows.append((t, x0 + 0.5 * v0 * tr + v0 * tau - 0.5 * ad * tau * tau, v0 - ad * tau, -ad))
    return np.array(rows)


def test_sampled_closed_form_reproduces_its_run():
    cfg = workloads.C1()
    n = 60  # past the end of the ramp
    ref = oracle.Oracle(cfg)
    ref.step(n)
    _, dt_ref, p_ref = ref.probes()
    t_end = float(np.sum(dt_ref)) * 1.5
    tab = oracle.Oracle(dict(cfg, kin_mode=3))
    tab.set_kin_table(ramp_decel_table(cfg, t_end, 5e-9))
    tab.step(n)
    _, dt_tab, p_tab = tab.probes()
    # the ring's centre differs by the interpolation error (~1e-9 m), which
    # moves the ghost velocities (and so the CFL step) at the 1e-8 level
    assert np.abs(dt_tab / dt_ref - 1).max() < 1e-7
    scale = np.abs(p_ref).max()
    assert np.abs(p_tab - p_ref).max() <= 1e-6 * scale
    xr, vr, _ = ref.disk_state()
    xt, vt, _ = tab.disk_state()
    assert abs(vt - vr) <= 1e-9 * vr and abs(xt - xr) <= 1e-9  # 1e-6 dx
