"""MI355X planar WCSPH hot path: Python binding of libwcsph.so.

Argument marshalling only: every step of the particle pipeline runs in the
HIP kernels of libwcsph.so. PyTorch supplies device memory (its caching
allocator, through the library's allocator hook) and the HIP stream the
library queues its work and graph on.

The binding fails loudly when the shared library is missing or no GPU is
present; there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# the library built in-tree; WCSPH_LIB names another build of it (e.g. a tuner variant)
LIB_PATH = os.environ.get("WCSPH_LIB", os.path.join(PKG, "libwcsph.so"))
MAX_PROBES = 16

OK, E_INVALID, E_OOM, E_HIP, E_STATE, E_UNSTABLE, E_RANGE = range(7)
_STATUS = {0: "OK", 1: "E_INVALID", 2: "E_OOM", 3: "E_HIP", 4: "E_STATE", 5: "E_UNSTABLE", 6: "E_RANGE"}
SYMBOLS = (
    "wcsph_create", "wcsph_batch_create", "wcsph_destroy", "wcsph_last_error", "wcsph_get_info",
    "wcsph_instance_info", "wcsph_set_disk_kinematics", "wcsph_set_dt_table", "wcsph_step", "wcsph_batch_step",
    "wcsph_synchronize", "wcsph_read_probes", "wcsph_read_diagnostics", "wcsph_get_fluid", "wcsph_get_disk",
    "wcsph_set_fluid", "wcsph_save_state", "wcsph_load_state", "wcsph_export_cells",
    "wcsph_export_rates", "wcsph_export_neighbours", "wcsph_export_neighbour_lists",
    "wcsph_export_neighbour_lists_noalloc", "wcsph_time_pair_kernel",
    "wcsph_set_coefficients", "wcsph_adj_forward", "wcsph_adj_backward",
    "wcsph_get_internal_energy", "wcsph_export_density",
)


class WcsphError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class WcsphUnstable(WcsphError):
    """E_UNSTABLE: the device state carries a validity flag. `result` holds
    what the call read (kept for inspection)."""

    def __init__(self, msg: str, result=None):
        super().__init__(E_UNSTABLE, msg)
        self.result = result


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
        ("kin_coef", C.c_double), ("audit", C.c_int), ("beta", C.c_double),
        ("kernel_type", C.c_int), ("eos_type", C.c_int), ("mg_s1", C.c_double),
        ("mg_gamma0", C.c_double), ("mg_mu_max", C.c_double), ("scheme", C.c_int), ("mg_a", C.c_double),
        ("axisym", C.c_int),
    ]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("vmax", C.c_double), ("mass", C.c_double),
                ("mom", C.c_double * 2), ("ke", C.c_double), ("e_el", C.c_double),
                ("e_pot", C.c_double), ("e_disk", C.c_double), ("w_boundary", C.c_double),
                ("step", C.c_longlong), ("n_clamp", C.c_longlong), ("n_cav", C.c_longlong),
                ("n_enforce", C.c_longlong), ("d_av", C.c_double), ("d_visc", C.c_double),
                ("w_delta", C.c_double), ("w_ghost", C.c_double), ("w_enforce", C.c_double),
                ("w_clamp", C.c_double), ("e_th", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n_inst", C.c_int), ("n_fluid", C.c_longlong), ("n_ghost", C.c_longlong),
                ("n_slots", C.c_longlong), ("n_cells", C.c_longlong), ("steps", C.c_longlong)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


def params(cfg: dict) -> Params:
    p = Params()
    for name, _ in Params._fields_:
        if name in ("n_probes", "probe_xy"):
            continue
        if name in cfg:
            setattr(p, name, cfg[name])
    probes = cfg.get("probes", [])
    if len(probes) > MAX_PROBES:
        raise ValueError("at most 16 probes")
    p.n_probes = len(probes)
    for k, (x, y) in enumerate(probes):
        p.probe_xy[2 * k] = x
        p.probe_xy[2 * k + 1] = y
    return p


_lib = None
_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)
_U = C.POINTER(C.c_uint)
_I = C.POINTER(C.c_int)
_LL = C.POINTER(C.c_longlong)
_V = C.c_void_p


def lib():
    """Load libwcsph.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built: run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950)")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(Params)
        sig = {
            "wcsph_create": [P, C.POINTER(Allocator), _V, C.POINTER(_V)],
            "wcsph_batch_create": [P, C.c_int, C.POINTER(Allocator), _V, C.POINTER(_V)],
            "wcsph_destroy": [_V],
            "wcsph_get_info": [_V, C.POINTER(Info)],
            "wcsph_instance_info": [_V, C.c_int, _I, _I, _I],
            "wcsph_set_disk_kinematics": [_V, C.c_int, C.c_int, _D, C.c_int],
            "wcsph_set_dt_table": [_V, _D, C.c_int],
            "wcsph_step": [_V, C.c_int],
            "wcsph_batch_step": [_V, C.c_int],
            "wcsph_synchronize": [_V],
            "wcsph_read_probes": [_V, C.c_int, _D, _D, _F, C.c_int, _I],
            "wcsph_read_diagnostics": [_V, C.c_int, C.POINTER(Diag), C.c_int, _I],
            "wcsph_get_fluid": [_V, C.c_int, _D, _D, _D, _D, _D, _D, C.c_int],
            "wcsph_get_disk": [_V, C.c_int, _D, _D, _D],
            "wcsph_get_internal_energy": [_V, C.c_int, _D, C.c_int],
            "wcsph_export_density": [_V, _F, _F, C.c_int],
            "wcsph_set_fluid": [_V, C.c_double, _D, _D, _D, _D, _D, C.c_int],
            "wcsph_save_state": [_V, _V, C.c_size_t, C.POINTER(C.c_size_t)],
            "wcsph_load_state": [_V, _V, C.c_size_t],
            "wcsph_export_cells": [_V, _U, _U, _D, _D, _U, _U, _U, C.c_size_t, C.c_size_t],
            "wcsph_export_rates": [_V, _F, _F, _F, _F, _F, _F, _F, _F, _F, C.c_int, C.c_int],
            "wcsph_export_neighbours": [_V, _U, _I, _LL, _D, _D, C.c_size_t],
            "wcsph_export_neighbour_lists": [_V, _I, _U, C.c_int, C.c_int],
            "wcsph_export_neighbour_lists_noalloc": [_V, _I, _U, C.c_int, C.c_int],
            "wcsph_time_pair_kernel": [_V, C.c_int, _F],
            "wcsph_set_coefficients": [_V, C.c_int, C.c_double, C.c_double, C.c_double],
            "wcsph_adj_forward": [_V, C.c_int, C.c_int, _D],
            "wcsph_adj_backward": [_V, C.c_double, _D],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.wcsph_last_error.argtypes = [_V]
        L.wcsph_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


class _TorchMemory:
    """Device memory and stream from PyTorch for one context."""

    def __init__(self, device):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the WCSPH hot path runs only on the GPU")
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)  # default priority
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = Allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, stream, user):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device.index or 0,
                                                           self.stream)
        except Exception:  # out of memory -> the library reports E_OOM
            return None

    def _do_free(self, ptr, stream, user):
        cuda = getattr(self.torch, "cuda", None)
        if cuda is not None and getattr(cuda, "caching_allocator_delete", None) is not None:
            cuda.caching_allocator_delete(ptr)
        # else: interpreter shutdown, the process releases the memory


_live = weakref.WeakSet()


@atexit.register
def _close_all():
    """Destroy open contexts while PyTorch is still alive."""
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass


class Solver:
    """One planar WCSPH problem (or a batch of them) on one GPU."""

    def __init__(self, cfg, device: str = "cuda:0"):
        self.mem = _TorchMemory(device)
        self.handle = _V()
        L = lib()
        self.batched = isinstance(cfg, (list, tuple))
        if self.batched:
            self.cfgs = list(cfg)
            arr = (Params * len(cfg))(*[params(c) for c in cfg])
            st = L.wcsph_batch_create(arr, len(cfg), C.byref(self.mem.struct),
                                      _V(self.mem.stream.cuda_stream), C.byref(self.handle))
        else:
            self.cfgs = [cfg]
            st = L.wcsph_create(C.byref(params(cfg)), C.byref(self.mem.struct),
                                _V(self.mem.stream.cuda_stream), C.byref(self.handle))
        if st != OK:
            raise WcsphError(st, L.wcsph_last_error(None).decode())
        info = Info()
        self._check(L.wcsph_get_info(self.handle, C.byref(info)))
        self.n_inst = info.n_inst
        self.n_fluid_total = info.n_fluid
        self.n_slots = info.n_slots
        self.n_cells = info.n_cells
        self.sizes = []
        for i in range(self.n_inst):
            nf, ng, nc = C.c_int(), C.c_int(), C.c_int()
            self._check(L.wcsph_instance_info(self.handle, i, C.byref(nf), C.byref(ng), C.byref(nc)))
            self.sizes.append((nf.value, ng.value, nc.value))
        self.nf, self.ng, self.ncells = self.sizes[0]
        self.n_probes = [len(c.get("probes", [])) for c in self.cfgs]
        _live.add(self)

    def _check(self, st, result=None):
        if st != OK:
            msg = lib().wcsph_last_error(self.handle).decode() if self.handle else ""
            if st == E_UNSTABLE:
                raise WcsphUnstable(msg, result)
            raise WcsphError(st, msg)

    def close(self):
        if self.handle:
            lib().wcsph_destroy(self.handle)
            self.handle = _V()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- driving ------------------------------------------------------------
    def set_kinematics(self, mode: int, v0: float, t_ramp: float, coef: float, inst: int = 0):
        c = np.array([v0, t_ramp, coef], dtype=np.float64)
        self._check(lib().wcsph_set_disk_kinematics(self.handle, inst, mode, _p(c, C.c_double), 3))

    def set_kinematics_table(self, rows, inst: int = 0):
        """kin_mode 3: the disk motion as rows (t, x, v, a)."""
        r = np.ascontiguousarray(rows, dtype=np.float64).reshape(-1, 4)
        self._check(lib().wcsph_set_disk_kinematics(self.handle, inst, 3, _p(r, C.c_double), r.shape[0]))

    def set_dt_table(self, dt):
        dt = np.ascontiguousarray(dt, dtype=np.float64)
        self._check(lib().wcsph_set_dt_table(self.handle, _p(dt, C.c_double), dt.size))

    def step(self, n: int = 1):
        fn = lib().wcsph_batch_step if self.batched else lib().wcsph_step
        self._check(fn(self.handle, n))

    def synchronize(self):
        self._check(lib().wcsph_synchronize(self.handle))

    # -- results --------------------------------------------------------------
    def read_probes(self, inst: int = 0, max_rows: int = 1 << 20):
        np_ = self.n_probes[inst]
        rows = C.c_int()
        t = np.empty(max_rows)
        dt = np.empty(max_rows)
        p = np.empty((max_rows, max(np_, 1)), dtype=np.float32)
        st = lib().wcsph_read_probes(self.handle, inst, _p(t, C.c_double), _p(dt, C.c_double),
                                     _p(p, C.c_float), max_rows, C.byref(rows))
        n = rows.value
        out = (t[:n].copy(), dt[:n].copy(), p[:n, :np_].copy())
        self._check(st, out)
        return out

    def read_diagnostics(self, inst: int = 0, max_rows: int = 4096, check: bool = True):
        """Diagnostic records since the last read. A flagged state raises
        WcsphUnstable (with the records as .result), or with check=False
        returns them with out["unstable"] = True."""
        buf = (Diag * max_rows)()
        n = C.c_int()
        st = lib().wcsph_read_diagnostics(self.handle, inst, buf, max_rows, C.byref(n))
        rows = [buf[k] for k in range(n.value)]
        out = {k: np.array([getattr(r, k) for r in rows]) for k, _ in Diag._fields_ if k != "mom"}
        out["momx"] = np.array([r.mom[0] for r in rows])
        out["momy"] = np.array([r.mom[1] for r in rows])
        if st == E_UNSTABLE and not check:
            out["unstable"] = True
            return out
        self._check(st, out)
        return out

    def fluid(self, inst: int = 0):
        nf = self.sizes[inst][0]
        t = C.c_double()
        a = [np.empty(nf) for _ in range(5)]
        st = lib().wcsph_get_fluid(self.handle, inst, C.byref(t), *[_p(x, C.c_double) for x in a], nf)
        self._check(st, (t.value, a))
        return t.value, a

    def internal_energy(self, inst: int = 0):
        """Specific internal energy per fluid id (scheme 1; zeros otherwise)."""
        nf = self.sizes[inst][0]
        e = np.empty(nf)
        st = lib().wcsph_get_internal_energy(self.handle, inst, _p(e, C.c_double), nf)
        self._check(st, e)
        return e

    def export_density(self):
        """Density and pressure per fluid id at the current state (scheme 1:
        the clamped summation at the current positions)."""
        nf = self.nf
        rho = np.empty(nf, np.float32)
        p = np.empty(nf, np.float32)
        self._check(lib().wcsph_export_density(self.handle, _p(rho, C.c_float), _p(p, C.c_float), nf))
        return rho, p

    def disk_state(self, inst: int = 0):
        """(x, v, a) of the disk at the newest state's time."""
        o = [C.c_double() for _ in range(3)]
        st = lib().wcsph_get_disk(self.handle, inst, *[C.byref(x) for x in o])
        out = tuple(x.value for x in o)
        self._check(st, out)
        return out

    def set_fluid(self, t, x, y, vx, vy, rho):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, vx, vy, rho)]
        self._check(lib().wcsph_set_fluid(self.handle, float(t), *[_p(v, C.c_double) for v in arrs],
                                          arrs[0].size))

    def save_state(self) -> bytes:
        need = C.c_size_t()
        self._check(lib().wcsph_save_state(self.handle, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        self._check(lib().wcsph_save_state(self.handle, buf, need.value, C.byref(need)))
        return buf.raw

    def load_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(lib().wcsph_load_state(self.handle, buf, len(blob)))

    # -- test hooks -----------------------------------------------------------
    def export_cells(self):
        n, nc = self.n_slots, self.n_cells
        keys = np.empty(n, np.uint32); ids_pre = np.empty(n, np.uint32)
        x = np.empty(n); y = np.empty(n)
        perm = np.empty(n, np.uint32); ids_post = np.empty(n, np.uint32)
        cs = np.empty(nc + 1, np.uint32)
        self._check(lib().wcsph_export_cells(self.handle, _p(keys, C.c_uint), _p(ids_pre, C.c_uint),
                                             _p(x, C.c_double), _p(y, C.c_double), _p(perm, C.c_uint),
                                             _p(ids_post, C.c_uint), _p(cs, C.c_uint), n, nc + 1))
        return dict(keys=keys, ids_pre=ids_pre, x=x, y=y, perm=perm, ids_post=ids_post, cell_start=cs)

    def export_rates(self):
        nf, ng = self.nf, self.ng
        f = [np.empty(nf, np.float32) for _ in range(5)]
        g = [np.empty(ng, np.float32) for _ in range(4)]
        self._check(lib().wcsph_export_rates(self.handle, *[_p(a, C.c_float) for a in f + g], nf, ng))
        return dict(zip(("drho", "ax", "ay", "Vx", "Vy", "gp", "grho", "gvx", "gvy"), f + g))

    def export_neighbours(self):
        n = self.n_slots
        ids = np.empty(n, np.uint32); cnt = np.empty(n, np.int32); sm = np.empty(n, np.int64)
        x = np.empty(n); y = np.empty(n)
        self._check(lib().wcsph_export_neighbours(self.handle, _p(ids, C.c_uint), _p(cnt, C.c_int),
                                                  _p(sm, C.c_longlong), _p(x, C.c_double),
                                                  _p(y, C.c_double), n))
        return dict(ids=ids, count=cnt, idsum=sm, x=x, y=y)

    def export_neighbour_lists(self, max_per: int = 64, noalloc: bool = False):
        """Per fluid id, the ids of the neighbours the pair kernel sums
        (unordered); noalloc: through the entry point that allocates nothing."""
        nf = self.nf
        cnt = np.zeros(nf, np.int32)
        nbr = np.zeros((nf, max_per), np.uint32)
        fn = lib().wcsph_export_neighbour_lists_noalloc if noalloc else lib().wcsph_export_neighbour_lists
        self._check(fn(self.handle, _p(cnt, C.c_int), _p(nbr, C.c_uint), max_per, nf))
        return [nbr[k, :cnt[k]].copy() for k in range(nf)]

    # -- coefficients and reverse sweep ----------------------------------------
    def set_coefficients(self, alpha: float, delta: float, c0: float, inst: int = 0):
        self._check(lib().wcsph_set_coefficients(self.handle, inst, float(alpha), float(delta), float(c0)))

    def adj_forward(self, n_steps: int, ckpt_every: int = 50) -> float:
        J = C.c_double()
        self._check(lib().wcsph_adj_forward(self.handle, n_steps, ckpt_every, C.byref(J)))
        return J.value

    def adj_backward(self, dJ: float = 1.0) -> np.ndarray:
        g = np.zeros(3)
        self._check(lib().wcsph_adj_backward(self.handle, float(dJ), _p(g, C.c_double)))
        return g

    def time_pair_kernel(self, reps: int = 20) -> float:
        ms = C.c_float()
        self._check(lib().wcsph_time_pair_kernel(self.handle, reps, C.byref(ms)))
        return ms.value


def impulse_fn():
    """torch.autograd.Function computing the summed wall-probe pressure
    impulse J(alpha, delta, c0) of a solver run from a saved state, with the
    library's reverse sweep as its backward."""
    import torch

    class ImpulseFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, alpha, delta, c0, solver, state0, n_steps, ckpt_every):
            solver.load_state(state0)
            solver.set_coefficients(float(alpha), float(delta), float(c0))
            J = solver.adj_forward(n_steps, ckpt_every)
            ctx.solver = solver
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            g = ctx.solver.adj_backward(float(gJ))
            t = [torch.tensor(x, dtype=torch.float64) for x in g]
            return t[0], t[1], t[2], None, None, None, None

    return ImpulseFn
