"""Seeded synthetic workload definitions for the planar WCSPH hot path.

This module only names the inputs: channel sizes, lattice spacing, material
and scheme coefficients, disk kinematics, probe stations and the seeded draws
of the batched coefficient sweep. It holds none of the method's arithmetic;
the GPU library and the FP64 oracle each turn a workload dict into their own
geometry and state.

Constants follow the paper (Numerical Methodology section): h = 1.3 dx
(eq. cubic-kernel text), eta^2 = 0.01 (eq. artificial-viscosity),
eps_XSPH = 0.02 (eq. xsph), mu_d = 8.9e-4 Pa s, density band [0.5, 1.5] rho0
(Density Summation), cavitation cutoff -0.1 MPa (eq. eos), 5 us velocity ramp
(eq. velocity-ramp), N_g = 100 disk ghosts (Projectile section), wall
pull-back 1e-6 m (Channel Walls section). The scheme choices that the hot path
fixes are Tait gamma = 7, c0 = 1480 m/s, CFL 0.2, Wendland C2 kernel,
continuity with a delta-diffusion term and a predictor-corrector update.

The prescribed deceleration a_d = k v0^2 uses the drag constant
k = C_d rho_f pi R_p^2 / (2 M_p) of eq. drag with M_p = 8.01 g,
R_p = 6.25 mm, C_d = 0.05, rho_f = 1000 kg/m^3 (Projectile Dynamics).
"""
from __future__ import annotations

import math

import numpy as np

# drag-law constants of the real projectile (Projectile Dynamics, eq. drag)
PROJ_MASS = 8.01e-3
PROJ_RADIUS = 6.25e-3
PROJ_CD = 0.05
RHO_F = 1000.0
K_DRAG = 0.5 * PROJ_CD * RHO_F * math.pi * PROJ_RADIUS ** 2 / PROJ_MASS

C4_SEED = 2609

# Mie-Grueneisen water (eq. eos and its parameter table): bulk sound speed C,
# Hugoniot slope S1, gamma0, compression cap of mu = rho/rho0 - 1
MG_C = 1448.0
MG_S1 = 1.979
MG_GAMMA0 = 0.11
MG_MU_MAX = 0.25
MG_A = 3.0


def _cell_size(dx: float, h_over_dx: float) -> float:
    """Smallest float32 that is >= 2h: the cell edge both sides use.

    A float32 edge lets the GPU keep cell-relative offsets exact under
    renormalisation; rounding up keeps every pair with r < 2h inside the
    3x3 block of cells.
    """
    two_h = 2.0 * h_over_dx * dx
    c = np.float32(two_h)
    if float(c) < two_h:
        c = np.nextafter(c, np.float32(np.inf))
    return float(c)


def base(L: float, W: float, dx: float, R: float, v0: float, *,
         alpha: float = 0.1, delta: float = 0.1, c0: float = 1480.0,
         probes_x=(0.010, 0.030), steps: int = 200) -> dict:
    """One workload: a channel [0,L]x[0,W] (metres) with a disk of radius R
    starting at (R, W/2) and moving along +x from rest, ramped to v0 over
    5 us and then decelerating at k v0^2."""
    h_over_dx = 1.3
    probes = []
    for x in probes_x:
        probes.append((x, 0.0))
        probes.append((x, W))
    return dict(
        L=L, W=W, dx=dx, h_over_dx=h_over_dx, cell_size=_cell_size(dx, h_over_dx),
        rho0=1000.0, c0=c0, gamma=7.0, p_cav=-1.0e5,
        alpha=alpha, delta=delta, eps_xsph=0.02, mu_dyn=8.9e-4, eta2=0.01,
        cfl=0.2, gravity_y=-9.81,
        rho_lo=0.5, rho_hi=1.5, eps_wall=1.0e-6,
        ghost_layers=3, n_disk_ghosts=100, ghost_rho_mode=0, init_mode=0,
        disk_R=R, disk_x0=R, disk_y0=0.5 * W, disk_mass=PROJ_MASS,
        probes=probes, diag_every=10,
        kin_mode=0, kin_v0=v0, kin_t_ramp=5.0e-6, kin_coef=K_DRAG * v0 * v0,
        eos_type=0, mg_s1=MG_S1, mg_gamma0=MG_GAMMA0, mg_mu_max=MG_MU_MAX,
        scheme=0, mg_a=MG_A,
        steps=steps,
    )


def C1() -> dict:
    """80x40 mm, dx = 1 mm (3,148 fluid), R = 4 mm, 600 m/s, 200 steps."""
    return base(0.080, 0.040, 1.0e-3, 4.0e-3, 600.0, steps=200)


def two_way(cfg: dict) -> dict:
    """The same workload with two-way disk coupling (kin_mode 2): the ramp,
    then the disk moves with the reaction of the ring's force on the fluid.
    In the plane the disk is the cross-section of a cylinder of the
    projectile's density (M_p over the volume of a sphere of radius R_p),
    so its mass per unit depth is that density times pi R^2."""
    rho_p = PROJ_MASS / (4.0 / 3.0 * math.pi * PROJ_RADIUS ** 3)
    return dict(cfg, kin_mode=2, disk_mass=rho_p * math.pi * cfg["disk_R"] ** 2)


def paper_geometry(v0: float = 900.0) -> dict:
    """The paper's own channel (Validation Problem Setup): 750x150 mm at
    dx = 1.5 mm, a disk of the projectile's radius 6.25 mm, probes at the PTn
    and PTf stations x = 30 and 105 mm on both walls, with the paper's cubic
    B-spline kernel, alpha = 0.03 and single-line wall ghosts. Density
    (continuity with delta), EOS (Tait) and the update (predictor-corrector)
    stay those of the hot path."""
    cfg = base(0.750, 0.150, 1.5e-3, PROJ_RADIUS, v0, alpha=0.03, probes_x=(0.030, 0.105), steps=2000)
    return dict(cfg, kernel_type=1, ghost_layers=1)


def mie_grueneisen(cfg: dict) -> dict:
    """The same workload with the paper's Mie-Grueneisen EOS (eos_type 1) at
    zero specific internal energy in place of Tait, and the reference
    celerity c0 = C = 1448 m/s that the paper ties to it."""
    return dict(cfg, eos_type=1, c0=MG_C)


def paper_scheme(cfg: dict) -> dict:
    """The same workload with the paper's scheme as published (scheme 1):
    summation density over fluid and ghosts with the [0.5, 1.5] rho0 clamp
    (Density Summation), no delta term, the Mie-Grueneisen EOS of eq. eos with
    an evolving specific internal energy, c0 = C = 1448 m/s, the cubic
    B-spline kernel, and the leapfrog update at CFL 0.25 (eq. cfl)."""
    return dict(cfg, scheme=1, eos_type=1, c0=MG_C, kernel_type=1, cfl=0.25, delta=0.0)


def axisymmetric(cfg: dict) -> dict:
    """The same workload in the axisymmetric r-z form (axisym = 1), the
    extension the Conclusions rank first: the plane is the meridian
    half-plane through the tank axis, x the axial coordinate and y >= 0 the
    radius, so the box is [0, L] x [0, W/2] (the planar channel's half-width
    is the tank radius) with the axis at y = 0 and the disk's centre, now a
    sphere's, on it. Gravity is off (across the axis it would break the
    symmetry). The probes keep their axial stations, on the axis (the
    paper's centreline gauges) and on the tank wall. disk_mass stays the
    projectile's 3D mass."""
    Rt = 0.5 * cfg["W"]
    xs = sorted({x for x, _ in cfg["probes"]})
    probes = [pt for x in xs for pt in ((x, 0.0), (x, Rt))]
    return dict(cfg, W=Rt, disk_y0=0.0, gravity_y=0.0, axisym=1, probes=probes)


def C2() -> dict:
    """300x150 mm, dx = 0.5 mm (179,552 fluid), R = 6 mm, 900 m/s, 2,000 steps,
    four wall probes at the PTn / PTf stations x = 30 and 105 mm."""
    return base(0.300, 0.150, 0.5e-3, 6.0e-3, 900.0,
                probes_x=(0.030, 0.105), steps=2000)


def C3() -> dict:
    """600x300 mm, dx = 0.5 mm (719,552 fluid), otherwise as C2; 1,000 steps."""
    return base(0.600, 0.300, 0.5e-3, 6.0e-3, 900.0,
                probes_x=(0.030, 0.105), steps=1000)


def C4(n_inst: int = 64, seed: int = C4_SEED) -> list:
    """Batched coefficient sweep: per instance four uniforms drawn in the
    order (L, alpha, delta, v0); L = round(200 + 200u) mm x 100 mm at
    dx = 1 mm, alpha in [0.01, 0.5], delta in [0, 0.2], v0 in [600, 900] m/s,
    R = 4 mm, 1,000 steps each."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        u = rng.random(4)
        L = round(200.0 + 200.0 * u[0]) * 1e-3
        alpha = 0.01 + 0.49 * u[1]
        delta = 0.2 * u[2]
        v0 = 600.0 + 300.0 * u[3]
        out.append(base(L, 0.100, 1.0e-3, 4.0e-3, v0, alpha=alpha, delta=delta,
                        probes_x=(0.030, 0.105), steps=1000))
    return out


def C5() -> dict:
    """Adjoint form: 120x60 mm, dx = 0.5 mm (28,352 fluid), R = 6 mm, 900 m/s,
    500 steps, checkpoint every 50, probes at x = 10 and 30 mm."""
    d = base(0.120, 0.060, 0.5e-3, 6.0e-3, 900.0, steps=500)
    d["ckpt_every"] = 50
    return d


def tiny(L: float = 0.024, W: float = 0.016, dx: float = 1.0e-3, R: float = 3.0e-3,
         v0: float = 300.0, **kw) -> dict:
    """A small channel (a few hundred particles) for brute-force and
    finite-difference checks."""
    d = base(L, W, dx, R, v0, probes_x=(0.006, 0.012), **kw)
    return d


CONFIGS = {"C1": C1, "C2": C2, "C3": C3, "C5": C5}
