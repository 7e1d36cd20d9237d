"""Two-way disk coupling in the FP64 oracle (kin_mode 2, the extension the
paper names in its energy-audit discussion and Conclusions).

Pins: the ramp is the prescribed one; with an immovable disk the coupled
motion is the prescribed constant-velocity law; the disk loses exactly the
kinetic energy that the boundary work of eq. energy-audit gives the fluid
(the midpoint force and the step's mean velocity make this exact up to
rounding); and the fluid's reaction slows the disk down.
"""
import numpy as np

import oracle
import workloads


def _run(cfg, n):
    o = oracle.Oracle(cfg)
    o.step(n)
    return o


def test_ramp_steps_equal_the_prescribed_ramp():
    """Every step that ends within the ramp is the same as with the
    prescribed law (mode 0)."""
    cfg0 = workloads.C1()
    cfg2 = workloads.two_way(cfg0)
    o0, o2 = oracle.Oracle(cfg0), oracle.Oracle(cfg2)
    n = 0
    while True:
        o0.step(1)
        o2.step(1)
        t, _ = o0.fluid()
        if t > cfg0["kin_t_ramp"]:
            break
        n += 1
        for a, b in zip(o0.fluid()[1], o2.fluid()[1]):
            assert np.array_equal(a, b)
        assert o0.disk_state() == o2.disk_state()
    assert n > 20


def test_immovable_disk_moves_at_constant_velocity():
    """With an (almost) infinite disk mass the coupled disk keeps v0 after
    the ramp, as the prescribed law with zero deceleration does."""
    cfg0 = dict(workloads.C1(), kin_coef=0.0, disk_mass=1.0e30)
    cfg2 = dict(workloads.two_way(cfg0), disk_mass=1.0e30)
    o0, o2 = _run(cfg0, 120), _run(cfg2, 120)
    x0, v0, _ = o0.disk_state()
    x2, v2, a2 = o2.disk_state()
    assert v2 == cfg0["kin_v0"] and abs(a2) < 1e-20
    assert abs(x2 - x0) <= 1e-12 * x0
    for a, b in zip(o0.fluid()[1], o2.fluid()[1]):
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max())
    d0, d2 = o0.diags(), o2.diags()
    assert abs(d2["w_boundary"][-1] - d0["w_boundary"][-1]) <= 1e-9 * abs(d0["w_boundary"][-1])


def test_disk_energy_loss_equals_boundary_work():
    """After the coupling starts, e_disk + w_boundary is constant."""
    cfg = workloads.two_way(workloads.C1())
    o = _run(cfg, cfg["steps"])
    d = o.diags()
    coupled = d["t"] >= cfg["kin_t_ramp"] + 2.0 * d["dt"].max()
    k = np.nonzero(coupled)[0]
    assert k.size >= 10
    s = d["e_disk"][k] + d["w_boundary"][k]
    dw = abs(d["w_boundary"][k[-1]] - d["w_boundary"][k[0]])
    assert dw > 1e-6 * d["e_disk"][k[0]]  # the fluid does take work
    assert np.abs(s - s[0]).max() <= 1e-9 * dw


def test_fluid_reaction_slows_the_disk():
    cfg = workloads.two_way(workloads.C1())
    o = _run(cfg, cfg["steps"])
    x, v, a = o.disk_state()
    assert a < 0.0 and 0.0 < v < cfg["kin_v0"]
    # the prescribed constant-velocity law would be ahead of the coupled disk
    x_free, _, _ = o.kinematics(o.fluid()[0])
    assert x < x_free
