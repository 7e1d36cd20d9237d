"""Precision form: the FP32 GPU path (pair sums on cell-relative offsets,
FP64 time, kinematics and diagnostics) against the FP64 oracle at full
size, with the error of every result printed.

* 600x300 mm channel at dx 0.5 mm (719,552 fluid): one evaluation from a
  shared state, 100 steps from t = 0 (fields and FP64 diagnostics), and
  the configured 1,000 steps against the stored oracle run.
* 300x150 mm channel (179,552 fluid): the whole 2,000-step run on the
  oracle's time-step table, wall-probe histories (the entry pulse reaches
  the near probes after about 1,100 steps and the far ones near the end).
"""
import numpy as np
import pytest

import oracle
import workloads
from tests import shared_state

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")


def _rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300))


def _relvec(ax, ay, bx, by):
    d = np.hypot(np.asarray(ax, np.float64) - bx, np.asarray(ay, np.float64) - by)
    return float(d.max() / max(np.hypot(bx, by).max(), 1e-300))


def test_C3_one_evaluation_and_100_steps():
    cfg = workloads.C3()
    print(f"[gpu] C3 solver", flush=True)
    # one evaluation from the oracle's state after 20 steps, rounded to the
    # FP32 representation and loaded into both sides
    s, o = shared_state.shared(cfg, 20, wc, oracle)
    assert s.nf == 719552
    g = s.export_rates()
    r = o.eval_rates()
    e1 = dict(drho=_rel(g["drho"], r["drho"]), acc=_relvec(g["ax"], g["ay"], r["ax"], r["ay"]),
              xsph=_relvec(g["Vx"], g["Vy"], r["Vx"], r["Vy"]), ghost_p=_rel(g["gp"], r["gp"]))
    print("C3 one evaluation, max error / max value:", e1)
    assert max(e1.values()) <= 1e-4
    s.close()
    # 100 steps from t = 0 on both sides
    n = 100
    s = wc.Solver(cfg, "cuda:0")
    s.step(n)
    tg, (xg, yg, vxg, vyg, rg) = s.fluid()
    dg = s.read_diagnostics()
    o = oracle.Oracle(cfg)
    o.step(n)
    to, (xo, yo, vxo, vyo, ro) = o.fluid()
    do = o.diags()
    dx = cfg["dx"]
    e2 = dict(time=abs(tg - to) / to,
              density=float(np.abs(rg / ro - 1).max()),
              position_over_dx=float(max(np.abs(xg - xo).max(), np.abs(yg - yo).max()) / dx),
              velocity=_relvec(vxg, vyg, vxo, vyo))
    for k in ("mass", "momx", "ke", "e_el", "w_boundary"):
        e2[k] = abs(dg[k][-1] - do[k][-1]) / abs(do[k][-1])
    print("C3 100 steps, errors vs the FP64 oracle:", e2)
    # the FP64 mass sum of 719,552 equal terms: both sides carry rounding of
    # at most n u (u = 2^-53) in different summation orders
    assert e2["time"] <= 1e-6 and e2["mass"] <= 2 * s.nf * 2.0 ** -53
    assert e2["density"] <= 1e-4 and e2["position_over_dx"] <= 1e-3 and e2["velocity"] <= 1e-3
    for k in ("momx", "ke", "e_el", "w_boundary"):
        assert e2[k] <= 1e-3, k
    s.close()


def test_C3_1000_steps_against_the_stored_oracle_run():
    """The precision form's whole configured run (600x300 mm, dx 0.5 mm,
    719,552 fluid, 1,000 steps) on the oracle's time-step table, against the
    oracle's run stored by tests/golden/c3_reference.py (too long to repeat
    here): mass to the FP64 sum's rounding at every record (every 10
    steps); momx, ke, e_el and w_boundary, each as the largest difference
    over the records relative to the largest record, within twice the
    oracle's own FP32 floor at this workload (the FP64 oracle against itself
    with its state rounded to the FP32 representation every step, with and
    without FP32-sized noise on each step's change: tests/golden/
    chaos_floor.py, case c3_diag; floors momx 1.6e-3, ke 6.8e-3, e_el
    2.9e-3, w_boundary 4.2e-3); e_disk (the prescribed disk's kinetic
    energy) to 1e-12. Within 1,000 steps the entry pulse has not reached the
    wall probes (75 mm and more from the path): they read the hydrostatic
    compression of a few hundred Pa, below what a float32 density resolves
    (one ulp of rho0 is about 130 Pa), so they are bounded as an absolute
    difference of twice the oracle's peak."""
    import os
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "c3_1000.npz"))
    cfg = workloads.C3()
    n = cfg["steps"]
    assert int(ref["steps"]) == n
    print(f"[gpu] C3 {n} steps on the stored oracle dt table", flush=True)
    s = wc.Solver(cfg, "cuda:0")
    assert s.nf == int(ref["n_fluid"])
    s.set_dt_table(ref["dt"])
    s.step(n)
    _, dtg, pg = s.read_probes()
    dg = s.read_diagnostics()
    s.close()
    assert np.array_equal(dtg, ref["dt"])
    # records of the same steps on both sides (every 10 steps, the last at step 1,000)
    steps_g = np.asarray(dg["step"], np.int64)
    steps_o = np.asarray(ref["diag_step"], np.int64)
    common = np.intersect1d(steps_g[steps_g > 0], steps_o[steps_o > 0])
    assert common.size >= 99 and common.max() == n
    ig = np.searchsorted(steps_g, common)
    io = np.searchsorted(steps_o, common)
    e = {}
    e["mass"] = float(np.abs(dg["mass"][ig] / ref["diag_mass"][io] - 1).max())
    for k in ("momx", "ke", "e_el", "w_boundary", "e_disk"):
        o = ref["diag_" + k][io]
        e[k] = float(np.abs(dg[k][ig] - o).max() / np.abs(o).max())
    peaks = np.abs(ref["p"]).max(0)
    e["probe_abs_over_peak"] = (np.abs(pg - ref["p"]).max(0) / peaks).tolist()
    fl = _floor_c3()
    print("C3 1,000 steps, errors vs the stored FP64 run:", e)
    print("C3 bars (2x the FP32 floor):", fl)
    assert e["mass"] <= 2 * s.nf * 2.0 ** -53
    for k in ("momx", "ke", "e_el", "w_boundary"):
        assert e[k] <= fl[k], k
    assert e["e_disk"] <= 1e-12
    assert peaks.max() < 1e4  # the pulse has not arrived: hydrostatic only
    assert max(e["probe_abs_over_peak"]) <= 2.0


def _floor_c3():
    """Twice the larger of the two floor runs per C3 diagnostic."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "chaos_floor.json")) as f:
        fl = json.load(f)["c3_diag"]
    return {k: 2.0 * max(fl["rounded"][k], fl["rounded_noise"][k]) for k in ("momx", "ke", "e_el", "w_boundary")}


def _floor(case):
    """Bars from the committed oracle-only measurement (tests/golden/
    chaos_floor.py): per metric, twice the largest per-probe difference of
    the FP64 oracle from itself with its state rounded to the FP32
    representation every step, with and without FP32-sized noise on each
    step's change."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "chaos_floor.json")) as f:
        fl = json.load(f)[case]
    runs = [fl["rounded"], fl["rounded_noise"]]
    return fl, {k: 2.0 * max(max(r[k]) if isinstance(r[k], list) else r[k] for r in runs)
                for k in ("history_over_peak", "peak_rel", "impulse_rel", "dt_rel")}


def test_C2_full_run_probe_histories():
    """The whole 2,000-step C2 run on the oracle's time-step table (both sides
    on one time grid; v_max -> dt is an extreme statistic that FP32 moves by
    a few per cent once the disk front has formed).

    The flow at the disk front is sensitive to the last bits, and the
    wall-probe histories integrate over that region. The bars come from
    the FP64 oracle against itself at this same workload with its state
    rounded to FP32 every step (with and without noise the size of FP32
    rounding on each step's change): twice the largest per-probe
    difference it shows, for the history (over each probe's own peak), the
    peak pressure and the impulse sum p dt. Measured floors: history 0.015,
    peak 7.6e-3, impulse 1.4e-3; bars 0.029, 0.015, 2.8e-3."""
    cfg = workloads.C2()
    n = cfg["steps"]
    fl, bar = _floor("c2")
    assert fl["steps"] == n and fl["replay_dt"]
    o = oracle.Oracle(cfg)
    o.step(n)
    to, dto, po = o.probes()
    do = o.diags()
    print(f"[gpu] C2 {n} steps on the oracle's dt table", flush=True)
    s = wc.Solver(cfg, "cuda:0")
    s.set_dt_table(dto)
    s.step(n)
    tg, dtg, pg = s.read_probes()
    dg = s.read_diagnostics()
    s.close()
    assert pg.shape == po.shape == (n, 4)
    assert np.array_equal(dtg, dto)
    peaks = np.abs(po).max(0)
    errs = np.abs(pg - po).max(0) / peaks
    peak_err = np.abs(np.abs(pg).max(0) / peaks - 1)
    imp_o = (po * dto[:, None]).sum(0)
    imp_err = np.abs((pg * dto[:, None]).sum(0) / imp_o - 1)
    print(f"C2 {n} steps: probe peaks {peaks.tolist()} Pa; max error / own peak {errs.tolist()} "
          f"(bar {bar['history_over_peak']:.3g}); peak error {peak_err.tolist()} (bar {bar['peak_rel']:.3g}); "
          f"impulse error {imp_err.tolist()} (bar {bar['impulse_rel']:.3g}); "
          f"ke {abs(dg['ke'][-1] / do['ke'][-1] - 1):.2e} e_el {abs(dg['e_el'][-1] / do['e_el'][-1] - 1):.2e} "
          f"w_b {abs(dg['w_boundary'][-1] / do['w_boundary'][-1] - 1):.2e}")
    assert peaks.min() > 1e8  # the pulse has reached every probe
    assert errs.max() <= bar["history_over_peak"]
    assert peak_err.max() <= bar["peak_rel"]
    assert imp_err.max() <= bar["impulse_rel"]
    assert abs(dg["mass"][-1] - dg["mass"][0]) <= 1e-12 * dg["mass"][0]
