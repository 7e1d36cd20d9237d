"""Failure handling through the C ABI, each condition forced from the host so
that every kernel still exits normally.

* A non-finite velocity planted in a saved state: the particle is left out
  of every neighbour's sums (its distance test is false), the step goes on,
  and the next diagnostic record reports the state as unstable.
* Non-finite input to wcsph_set_fluid is rejected before anything runs.
* An allocator that fails on its k-th call: creation returns E_OOM and every
  block it did get is given back.
"""
import ctypes as C
import struct

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")


def _plant_nan_velocity(s, blob: bytes) -> bytes:
    """The blob with vx = NaN in the first fluid slot. Layout: a 64-byte
    header, the clocks, then cell[N] u32, id[N] u32, pv[N] float4 (offset x,
    offset y, vx, vy), aux[N] float4, inst[N] u16, ghost slots u32."""
    N, ng = s.n_slots, s.ng
    clk_bytes = len(blob) - 64 - N * 42 - ng * 4
    assert clk_bytes > 0 and clk_bytes % s.n_inst == 0
    ids = np.frombuffer(blob, np.uint32, N, 64 + clk_bytes + 4 * N)
    slot = int(np.nonzero(ids < s.nf)[0][0])
    off = 64 + clk_bytes + 8 * N + 16 * slot + 8
    b = bytearray(blob)
    b[off:off + 4] = struct.pack("<f", float("nan"))
    return bytes(b)


def test_non_finite_state_is_reported_at_the_next_record():
    cfg = workloads.tiny()
    s = wc.Solver(cfg, "cuda:0")
    s.step(10)
    d0 = s.read_diagnostics()
    assert "unstable" not in d0
    s.load_state(_plant_nan_velocity(s, s.save_state()))
    print("[gpu] stepping a state with one non-finite velocity", flush=True)
    s.step(cfg["diag_every"])
    with pytest.raises(wc.WcsphUnstable) as e:
        s.read_diagnostics()
    assert e.value.status == wc.E_UNSTABLE and "non-finite" in str(e.value)
    assert e.value.result["mass"].size >= 1  # the records are still returned
    assert s.read_diagnostics(check=False)["unstable"]
    # every reader of the flagged state says so, and still returns what it read
    with pytest.raises(wc.WcsphUnstable) as e:
        s.read_probes()
    assert e.value.result[2].shape[0] == cfg["diag_every"]
    with pytest.raises(wc.WcsphUnstable):
        s.disk_state()
    with pytest.raises(wc.WcsphUnstable) as e:
        s.fluid()
    # the other particles are untouched by the planted value
    _, (x, y, vx, vy, rho) = e.value.result
    assert np.isfinite(rho).sum() >= rho.size - 1
    s.close()


def test_non_finite_input_rejected():
    cfg = workloads.tiny()
    s = wc.Solver(cfg, "cuda:0")
    t, (x, y, vx, vy, rho) = s.fluid()
    vx = vx.copy()
    vx[3] = np.inf
    with pytest.raises(wc.WcsphError) as e:
        s.set_fluid(t, x, y, vx, vy, rho)
    assert e.value.status == wc.E_INVALID
    s.step(5)  # the context is unchanged and still usable
    assert "unstable" not in s.read_diagnostics()
    s.close()


@pytest.mark.parametrize("fail_at", [1, 5, 12])
def test_failing_allocator_gives_e_oom_and_returns_every_block(fail_at):
    mem = wc._TorchMemory("cuda:0")
    calls, live = [0], {}

    def alloc(nbytes, stream, user):
        calls[0] += 1
        if calls[0] == fail_at:
            return None
        p = mem._do_alloc(nbytes, stream, user)
        live[p] = nbytes
        return p

    def free(ptr, stream, user):
        live.pop(ptr, None)
        mem._do_free(ptr, stream, user)

    a_fn, f_fn = wc.ALLOC_FN(alloc), wc.FREE_FN(free)
    al = wc.Allocator(a_fn, f_fn, None)
    h = C.c_void_p()
    L = wc.lib()
    st = L.wcsph_create(C.byref(wc.params(workloads.tiny())), C.byref(al), C.c_void_p(mem.stream.cuda_stream),
                        C.byref(h))
    assert st == wc.E_OOM, st
    assert not h.value
    assert calls[0] >= fail_at and not live


def test_cell_overflow_is_flagged_and_kernels_finish():
    """More than 64 particles in one cell (bucket capacity), forced from the
    host through set_fluid: the fill flags it, the sort fills the slots the
    dropped entries leave with inert entries, every kernel finishes, and every
    reader reports E_UNSTABLE with the cause."""
    cfg = workloads.tiny()
    s = wc.Solver(cfg, "cuda:0")
    t, (x, y, vx, vy, rho) = s.fluid()
    x, y = x.copy(), y.copy()
    dc = cfg["cell_size"]
    lo = -cfg["ghost_layers"] * cfg["dx"]
    # 72 fluid particles on a 9 x 8 grid inside the cell whose corner is (4 dc, 3 dc) + lo
    cx0, cy0 = lo + 4 * dc, lo + 3 * dc
    gx, gy = np.meshgrid(cx0 + (np.arange(9) + 0.5) * dc / 9, cy0 + (np.arange(8) + 0.5) * dc / 8)
    far = np.argsort(-np.hypot(x - cfg["disk_x0"], y - cfg["disk_y0"]))[:72]
    x[far], y[far] = gx.ravel(), gy.ravel()
    assert x.max() < cfg["L"] and y.max() < cfg["W"]
    s.set_fluid(t, x, y, vx, vy, rho)
    print("[gpu] 72 particles in one cell, stepping", flush=True)
    s.step(cfg["diag_every"])
    s.synchronize()
    with pytest.raises(wc.WcsphUnstable) as e:
        s.read_diagnostics()
    assert "more than 64 particles in one cell" in str(e.value)
    with pytest.raises(wc.WcsphUnstable):
        s.fluid()
    s.close()
    # the GPU is still fine: a fresh context runs normally
    s2 = wc.Solver(cfg, "cuda:0")
    s2.step(5)
    assert "unstable" not in s2.read_diagnostics()
    s2.close()
