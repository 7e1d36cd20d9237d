"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every function include/wcsph.h declares, and rejects invalid parameters
before touching the device."""
import ctypes as C
import os
import re

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "wcsph.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^(?:wcsph_status|const char\*)\s+(wcsph_\w+)\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("wcsph_create", "wcsph_set_disk_kinematics", "wcsph_step", "wcsph_read_probes",
              "wcsph_read_diagnostics", "wcsph_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    wc = pytest.importorskip("paper_2609_05494_amd")
    L = wc.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(_declared()) == set(wc.SYMBOLS)


def test_invalid_parameters_rejected_before_allocation():
    wc = pytest.importorskip("paper_2609_05494_amd")
    L = wc.lib()
    fake_stream = C.c_void_p(0x1)  # never used: validation fails first
    out = C.c_void_p()
    for bad in (dict(dx=0.0), dict(h_over_dx=0.5), dict(disk_x0=1.0), dict(cell_size=1e-4),
                dict(probes=[(5.0, 5.0)]), dict(cfl=0.0), dict(n_disk_ghosts=500), dict(eos_type=2),
                dict(eos_type=1, mg_s1=0.5), dict(eos_type=1, mg_mu_max=2.0), dict(eos_type=1, mg_gamma0=-1.0)):
        cfg = dict(workloads.C1(), **bad)
        st = L.wcsph_create(C.byref(wc.params(cfg)), None, fake_stream, C.byref(out))
        assert st == wc.E_INVALID, bad
        assert out.value is None
        assert L.wcsph_last_error(None)
    # the axisymmetric form: scheme 0, no gravity, no audit, the sphere on the axis
    rz = workloads.axisymmetric(workloads.C1())
    for bad in (dict(axisym=2), dict(scheme=1), dict(gravity_y=-9.81), dict(audit=1), dict(disk_y0=1e-3)):
        st = L.wcsph_create(C.byref(wc.params(dict(rz, **bad))), None, fake_stream, C.byref(out))
        assert st == wc.E_INVALID, bad
    st = L.wcsph_create(C.byref(wc.params(workloads.C1())), None, None, C.byref(out))
    assert st == wc.E_INVALID  # NULL stream refused
    assert L.wcsph_step(None, 1) == wc.E_STATE
    assert L.wcsph_destroy(None) == wc.E_STATE
