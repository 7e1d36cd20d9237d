"""ctypes wrapper of the FP64 CPU oracle (oracle/wcsph_oracle.cpp).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to check the GPU path. The product path never imports
this package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "wcsph_oracle.cpp")
MAX_PROBES = 16
NDIAG = 22
DIAG_FIELDS = ("t", "dt", "vmax", "mass", "momx", "momy", "ke", "e_el", "e_pot", "e_disk",
               "w_boundary", "step", "n_clamp", "n_cav", "n_enforce",
               "d_av", "d_visc", "w_delta", "w_ghost", "w_enforce", "w_clamp", "e_th")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (C++17, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", LIB, SRC]
        subprocess.run(cmd, check=True, cwd=HERE)
    return LIB


class Params(C.Structure):
    _fields_ = [
        ("L", C.c_double), ("W", C.c_double), ("dx", C.c_double), ("h_over_dx", C.c_double),
        ("cell_size", C.c_double),
        ("rho0", C.c_double), ("c0", C.c_double), ("gamma", C.c_double), ("p_cav", C.c_double),
        ("alpha", C.c_double), ("delta", C.c_double), ("eps_xsph", C.c_double),
        ("mu_dyn", C.c_double), ("eta2", C.c_double),
        ("cfl", C.c_double), ("gravity_y", C.c_double),
        ("rho_lo", C.c_double), ("rho_hi", C.c_double), ("eps_wall", C.c_double),
        ("ghost_layers", C.c_int), ("n_disk_ghosts", C.c_int), ("ghost_rho_mode", C.c_int),
        ("init_mode", C.c_int),
        ("disk_R", C.c_double), ("disk_x0", C.c_double), ("disk_y0", C.c_double),
        ("disk_mass", C.c_double),
        ("n_probes", C.c_int), ("probe_xy", C.c_double * (2 * MAX_PROBES)),
        ("diag_every", C.c_int),
        ("kin_mode", C.c_int), ("kin_v0", C.c_double), ("kin_t_ramp", C.c_double),
        ("kin_coef", C.c_double), ("beta", C.c_double), ("kernel_type", C.c_int),
        ("eos_type", C.c_int), ("mg_s1", C.c_double), ("mg_gamma0", C.c_double),
        ("mg_mu_max", C.c_double), ("scheme", C.c_int), ("mg_a", C.c_double),
        ("axisym", C.c_int),
    ]


def params(cfg: dict) -> Params:
    p = Params()
    for name, _ in Params._fields_:
        if name in ("n_probes", "probe_xy"):
            continue
        if name in cfg:
            setattr(p, name, cfg[name])
    probes = cfg.get("probes", [])
    p.n_probes = len(probes)
    for k, (x, y) in enumerate(probes):
        p.probe_xy[2 * k] = x
        p.probe_xy[2 * k + 1] = y
    return p


_lib = None
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.POINTER(Params)
        sig = {
            "orc_create": (C.c_void_p, [P, C.c_int, _D]),
            "orc_destroy": (None, [C.c_void_p]),
            "orc_num_fluid": (C.c_int, [C.c_void_p]),
            "orc_num_ghost": (C.c_int, [C.c_void_p]),
            "orc_num_cells": (C.c_int, [C.c_void_p]),
            "orc_set_dt_table": (None, [C.c_void_p, C.c_int, _D]),
            "orc_set_kin_table": (None, [C.c_void_p, C.c_int, _D]),
            "orc_step": (C.c_int, [C.c_void_p, C.c_int]),
            "orc_get_fluid": (None, [C.c_void_p, _D, _D, _D, _D, _D, _D]),
            "orc_set_fluid": (None, [C.c_void_p, C.c_double, _D, _D, _D, _D, _D]),
            "orc_probe_rows": (C.c_int, [C.c_void_p]),
            "orc_get_probes": (None, [C.c_void_p, _D, _D, _D]),
            "orc_diag_rows": (C.c_int, [C.c_void_p]),
            "orc_get_diags": (None, [C.c_void_p, _D]),
            "orc_impulse": (C.c_double, [C.c_void_p]),
            "orc_eval_rates": (None, [C.c_void_p] + [_D] * 10),
            "orc_audit_rates": (None, [C.c_void_p, _D]),
            "orc_get_ghosts": (None, [C.c_void_p, _D, _D, _D]),
            "orc_get_order": (None, [C.c_void_p, _I, _I]),
            "orc_kinematics": (None, [C.c_void_p, C.c_double, _D, _D, _D]),
            "orc_disk_state": (None, [C.c_void_p, _D, _D, _D]),
            "orc_kernel": (None, [C.c_double, C.c_double, _D, _D]),
            "orc_kernel_type": (None, [C.c_int, C.c_double, C.c_double, _D, _D]),
            "orc_eos": (None, [P, C.c_double, _D, _D]),
            "orc_elastic_energy": (C.c_double, [P, C.c_double]),
            "orc_eos_rho": (C.c_double, [P, C.c_double]),
            "orc_cfl_dt": (C.c_double, [C.c_double] * 4),
            "orc_cell_list": (C.c_int, [P, C.c_int, _D, _D, _I, _I, _I]),
            "orc_brute_pairs": (C.c_long, [P, C.c_int, _D, _D, _I, C.c_long]),
            "orc_cell_pairs": (C.c_long, [P, C.c_int, _D, _D, _I, C.c_long]),
            "orc_neighbour_stats": (None, [P, C.c_int, _D, _D, _I, C.c_double, _I,
                                           C.POINTER(C.c_longlong), _I]),
            "orc_ghost_point": (None, [P, C.c_double, C.c_double, _D, _D, C.c_int] + [_D] * 6
                                + [_D, _D, _D]),
            "orc_pair_rates": (None, [P, C.c_int] + [_D] * 7 + [_I] + [_D] * 5),
            "orc_tangent_J": (None, [P, C.c_int, _D, _D, _D]),
            "orc_tangent_J_f32": (None, [P, C.c_int, _D, _D, _D]),
            "orc_eval_density": (None, [C.c_void_p, _D, _D]),
            "orc_get_energy": (None, [C.c_void_p, _D]),
            "orc_eos_pe": (C.c_double, [P, C.c_double, C.c_double]),
            "orc_lattice_mass": (C.c_double, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def iptr(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I)


def f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """The whole FP64 solver on the host."""

    def __init__(self, cfg: dict, init: np.ndarray | None = None):
        self.cfg = cfg
        self.p = params(cfg)
        L = lib()
        if init is None:
            self.h = L.orc_create(C.byref(self.p), 0, None)
        else:
            init = f64(init).reshape(-1, 5)
            self.h = L.orc_create(C.byref(self.p), init.shape[0], dptr(init))
        if not self.h:
            raise ValueError("not built: scheme 1 with the coupled disk (kin_mode 2), or the "
                             "axisymmetric form with scheme 1 or with gravity")
        self.nf = L.orc_num_fluid(self.h)
        self.ng = L.orc_num_ghost(self.h)
        self.ncells = L.orc_num_cells(self.h)
        self.n_probes = self.p.n_probes

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def set_dt_table(self, dt):
        dt = f64(dt)
        lib().orc_set_dt_table(self.h, dt.size, dptr(dt))

    def set_kin_table(self, rows):
        """kin_mode 3: rows (t, x, v, a) of the prescribed disk motion."""
        rows = np.ascontiguousarray(rows, dtype=np.float64).reshape(-1, 4)
        lib().orc_set_kin_table(self.h, rows.shape[0], dptr(rows))

    def step(self, n: int = 1):
        lib().orc_step(self.h, n)

    def fluid(self):
        t = C.c_double()
        a = [np.empty(self.nf) for _ in range(5)]
        lib().orc_get_fluid(self.h, C.byref(t), *[dptr(x) for x in a])
        return t.value, a

    def set_fluid(self, t, x, y, vx, vy, rho):
        arrs = [f64(v) for v in (x, y, vx, vy, rho)]
        lib().orc_set_fluid(self.h, t, *[dptr(v) for v in arrs])

    def probes(self):
        n = lib().orc_probe_rows(self.h)
        t = np.empty(n); dt = np.empty(n); p = np.empty((n, self.n_probes))
        lib().orc_get_probes(self.h, dptr(t), dptr(dt), dptr(p))
        return t, dt, p

    def diags(self):
        n = lib().orc_diag_rows(self.h)
        rows = np.empty((n, NDIAG))
        lib().orc_get_diags(self.h, dptr(rows))
        return {k: rows[:, i] for i, k in enumerate(DIAG_FIELDS)}

    def impulse(self) -> float:
        return lib().orc_impulse(self.h)

    def eval_rates(self):
        nf, ng = self.nf, self.ng
        out = [np.empty(nf) for _ in range(5)] + [np.empty(ng) for _ in range(4)]
        vmax = np.empty(1)
        lib().orc_eval_rates(self.h, *[dptr(x) for x in out], dptr(vmax))
        keys = ("drho", "ax", "ay", "Vx", "Vy", "gp", "grho", "gvx", "gvy")
        d = dict(zip(keys, out))
        d["vmax"] = float(vmax[0])
        return d

    def eval_density(self):
        """Fluid density and pressure by id (scheme 1: the clamped summation at
        the current positions, which the oracle then stores)."""
        rho = np.empty(self.nf); p = np.empty(self.nf)
        lib().orc_eval_density(self.h, dptr(rho), dptr(p))
        return rho, p

    def energy(self):
        """Specific internal energy by fluid id (scheme 1)."""
        e = np.empty(self.nf)
        lib().orc_get_energy(self.h, dptr(e))
        return e

    def ghosts(self):
        g = [np.empty(self.ng) for _ in range(3)]
        lib().orc_get_ghosts(self.h, *[dptr(x) for x in g])
        return g

    def order(self):
        o = np.empty(self.nf + self.ng, dtype=np.int32)
        cs = np.empty(self.ncells + 1, dtype=np.int32)
        lib().orc_get_order(self.h, iptr(o), iptr(cs))
        return o, cs

    def kinematics(self, t):
        x, v, a = C.c_double(), C.c_double(), C.c_double()
        lib().orc_kinematics(self.h, t, C.byref(x), C.byref(v), C.byref(a))
        return x.value, v.value, a.value

    def audit_rates(self):
        """Energy audit rates of the last rate evaluation (eval_rates or the
        midpoint of the last step): d_av, d_visc, w_delta, w_ghost."""
        out = np.empty(4)
        lib().orc_audit_rates(self.h, dptr(out))
        return dict(zip(("d_av", "d_visc", "w_delta", "w_ghost"), out))

    def disk_state(self):
        """Disk centre x, velocity and acceleration at the current time
        (kin_mode 2: the coupled state once it has started)."""
        x, v, a = C.c_double(), C.c_double(), C.c_double()
        lib().orc_disk_state(self.h, C.byref(x), C.byref(v), C.byref(a))
        return x.value, v.value, a.value


def kernel(q: float, h: float, kernel_type: int = 0):
    W, F = C.c_double(), C.c_double()
    lib().orc_kernel_type(kernel_type, q, h, C.byref(W), C.byref(F))
    return W.value, F.value


def eos(cfg: dict, rho: float):
    p, c = C.c_double(), C.c_double()
    lib().orc_eos(C.byref(params(cfg)), rho, C.byref(p), C.byref(c))
    return p.value, c.value


def elastic_energy(cfg: dict, rho: float) -> float:
    return lib().orc_elastic_energy(C.byref(params(cfg)), rho)


def eos_rho(cfg: dict, pres: float) -> float:
    """Density at pressure pres (>= p_cav) on the workload's EOS."""
    return lib().orc_eos_rho(C.byref(params(cfg)), pres)


def cfl_dt(cfl, h, c0, vmax) -> float:
    return lib().orc_cfl_dt(cfl, h, c0, vmax)


def cell_list(cfg: dict, x, y):
    x, y = f64(x), f64(y)
    n = x.size
    p = params(cfg)
    keys = np.empty(n, dtype=np.int32)
    perm = np.empty(n, dtype=np.int32)
    # ncells from a dry call with n = 0
    nc = lib().orc_cell_list(C.byref(p), 0, dptr(x), dptr(y), None, None, None)
    cs = np.empty(nc + 1, dtype=np.int32)
    lib().orc_cell_list(C.byref(p), n, dptr(x), dptr(y), iptr(keys), iptr(perm), iptr(cs))
    return keys, perm, cs


def brute_pairs(cfg: dict, x, y):
    x, y = f64(x), f64(y)
    p = params(cfg)
    m = lib().orc_brute_pairs(C.byref(p), x.size, dptr(x), dptr(y), None, 0)
    out = np.empty(2 * max(m, 1), dtype=np.int32)
    lib().orc_brute_pairs(C.byref(p), x.size, dptr(x), dptr(y), iptr(out), m)
    return out[: 2 * m].reshape(-1, 2)


def cell_pairs(cfg: dict, x, y):
    x, y = f64(x), f64(y)
    p = params(cfg)
    m = lib().orc_cell_pairs(C.byref(p), x.size, dptr(x), dptr(y), None, 0)
    out = np.empty(2 * max(m, 1), dtype=np.int32)
    lib().orc_cell_pairs(C.byref(p), x.size, dptr(x), dptr(y), iptr(out), m)
    return out[: 2 * m].reshape(-1, 2)


def neighbour_stats(cfg: dict, x, y, ids, tol=1e-5):
    x, y = f64(x), f64(y)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    n = x.size
    cnt = np.empty(n, dtype=np.int32)
    sm = np.empty(n, dtype=np.int64)
    bd = np.empty(n, dtype=np.int32)
    lib().orc_neighbour_stats(C.byref(params(cfg)), n, dptr(x), dptr(y), iptr(ids), tol,
                              iptr(cnt), sm.ctypes.data_as(C.POINTER(C.c_longlong)), iptr(bd))
    return cnt, sm, bd


def ghost_point(cfg: dict, g, vw, aw, x, y, vx, vy, rho, pres):
    arrs = [f64(a) for a in (x, y, vx, vy, rho, pres)]
    vw, aw = f64(vw), f64(aw)
    pg, rg = C.c_double(), C.c_double()
    vg = np.empty(2)
    lib().orc_ghost_point(C.byref(params(cfg)), g[0], g[1], dptr(vw), dptr(aw), arrs[0].size,
                          *[dptr(a) for a in arrs], C.byref(pg), C.byref(rg), dptr(vg))
    return pg.value, rg.value, vg


def pair_rates(cfg: dict, x, y, vx, vy, rho, pres, m, kind):
    arrs = [f64(a) for a in (x, y, vx, vy, rho, pres, m)]
    kind = np.ascontiguousarray(kind, dtype=np.int32)
    n = arrs[0].size
    out = [np.zeros(n) for _ in range(5)]
    lib().orc_pair_rates(C.byref(params(cfg)), n, *[dptr(a) for a in arrs], iptr(kind),
                         *[dptr(o) for o in out])
    return dict(zip(("drho", "ax", "ay", "Vx", "Vy"), out))


def tangent_J(cfg: dict, dt, round_f32: bool = False):
    """J and dJ/d(alpha, delta, c0) by the FP64 forward-mode tangent on a
    fixed dt table; round_f32: the state's values rounded to the hot path's
    FP32 representation after every step (tangents kept)."""
    dt = f64(dt)
    J = C.c_double()
    dJ = np.empty(3)
    fn = lib().orc_tangent_J_f32 if round_f32 else lib().orc_tangent_J
    fn(C.byref(params(cfg)), dt.size, dptr(dt), C.byref(J), dptr(dJ))
    return J.value, dJ


def eos_pe(cfg: dict, rho: float, e: float) -> float:
    """Pressure of eq. eos with the cutoff at density rho and specific
    internal energy e."""
    return lib().orc_eos_pe(C.byref(params(cfg)), rho, e)


def lattice_mass(cfg: dict) -> float:
    """The particle mass of scheme 1: rho0 over the kernel sum of the square
    lattice of spacing dx."""
    return lib().orc_lattice_mass(C.byref(params(cfg)))
