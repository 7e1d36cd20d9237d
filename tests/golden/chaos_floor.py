"""Write chaos_floor.json: how far the FP64 oracle moves from itself when its
fluid state is stored in the FP32 representation the GPU path keeps (cell
index + float32 offset, float32 velocity and density), at the full-run
workloads whose GPU parity bars are set from this measurement.

Run A is the oracle as it is. Run B is the same oracle whose fluid state is
rounded to that representation after every step (the GPU rounds its stored
state at every evaluation), on run A's time-step table where the GPU test
replays that table, else on its own CFL step. Run C adds to run B, every
step, the size of the FP32 arithmetic's own error in the rates: each
particle's change over the step (position, velocity and density, each
component) is scaled by 1 + u, u uniform in [-n 2^-24, n 2^-24] with n = 20
(the worst-case relative rounding of a float32 sum of the twenty in-support
neighbour terms), from a seeded generator, before the rounding. All runs
are the oracle's arithmetic only; nothing here comes from the GPU path. Per wall probe the file records, for B and C against A,
the largest history difference over the probe's own peak, the peak
difference and the impulse (sum p dt) difference, and the largest relative
difference of dt where the run keeps its own step.

For the adjoint form the file records the same comparison for the FP64
forward-mode tangent of the summed probe impulse: J and dJ/d(alpha, delta,
c0) on the oracle's dt table with and without the per-step rounding. For
the precision form (C3, 1,000 steps) it records runs B and C's FP64
diagnostics (x momentum, ke, e_el, w_boundary) against run A's, stored by
tests/golden/c3_reference.py.

python -m tests.golden.chaos_floor [c2|paper|c5_adjoint|c3_diag|all]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from tests.shared_state import round_state  # noqa: E402

OUT = os.path.join(HERE, "chaos_floor.json")


NOISE = 20 * 2.0 ** -24
SEED = 2609


def perturbed(cfg: dict, steps: int, dta, noise: float) -> tuple:
    """Run B (noise = 0) or C: the state rounded every step, C with the
    arithmetic-sized relative noise on v and rho."""
    rng = np.random.default_rng(SEED)
    b = oracle.Oracle(cfg)
    if dta is not None:
        b.set_dt_table(dta)

    def store(prev):
        t_, f = b.fluid()
        if noise > 0.0 and prev is not None:
            f = [p + (c - p) * (1.0 + noise * rng.uniform(-1.0, 1.0, c.size)) for c, p in zip(f, prev)]
        r = round_state(cfg, *f)
        b.set_fluid(t_, *r)
        return r

    prev = store(None)
    for n in range(steps):
        b.step(1)
        prev = store(prev)
        if n % 200 == 199:
            print(f"  step {n + 1}/{steps}", flush=True)
    _, dtb, pb = b.probes()
    return dtb, pb


def compare(pa, dta, pb, dtb) -> dict:
    peaks = np.abs(pa).max(0)
    hist = np.abs(pb - pa).max(0) / peaks
    peak = np.abs(np.abs(pb).max(0) / peaks - 1)
    imp = np.abs((pb * dtb[:, None]).sum(0) / (pa * dta[:, None]).sum(0) - 1)
    return dict(history_over_peak=hist.tolist(), peak_rel=peak.tolist(), impulse_rel=imp.tolist(),
                dt_rel=float(np.abs(dtb / dta - 1).max()))


def floor(cfg: dict, steps: int, replay_dt: bool) -> dict:
    a = oracle.Oracle(cfg)
    t0 = time.perf_counter()
    a.step(steps)
    _, dta, pa = a.probes()
    out = dict(steps=steps, replay_dt=replay_dt, probe_peaks_pa=np.abs(pa).max(0).tolist(), noise=NOISE)
    for name, noise in (("rounded", 0.0), ("rounded_noise", NOISE)):
        dtb, pb = perturbed(cfg, steps, dta if replay_dt else None, noise)
        out[name] = compare(pa, dta, pb, dtb)
    out["wall_s"] = round(time.perf_counter() - t0, 1)
    return out


def tangent_floor(cfg: dict, steps: int) -> dict:
    """The FP64 forward-mode tangent of the summed probe impulse J on the
    oracle's own dt table, with and without the state rounded to the FP32
    representation after every step (tangents kept): how far FP32 storage
    alone moves J and dJ/d(alpha, delta, c0)."""
    t0 = time.perf_counter()
    a = oracle.Oracle(cfg)
    a.step(steps)
    _, dt, _ = a.probes()
    J, g = oracle.tangent_J(cfg, dt)
    Jr, gr = oracle.tangent_J(cfg, dt, round_f32=True)
    return dict(steps=steps, J=J, grad=g.tolist(), J_rounded=Jr, grad_rounded=gr.tolist(),
                J_rel=abs(Jr / J - 1), grad_rel=(np.abs(gr / g - 1)).tolist(),
                wall_s=round(time.perf_counter() - t0, 1))


DIAG_KEYS = ("momx", "ke", "e_el", "w_boundary")


def diag_floor(cfg: dict, ref_file: str) -> dict:
    """The FP64 diagnostics (records every 10 steps) of runs B and C against
    the oracle's own run A stored in ref_file (by tests/golden/c3_reference.py),
    on A's dt table: per quantity, the largest difference over the records
    divided by the largest value."""
    t0 = time.perf_counter()
    ref = np.load(os.path.join(HERE, ref_file))
    steps = int(ref["steps"])
    out = dict(steps=steps, replay_dt=True, ref=ref_file, noise=NOISE)
    for name, noise in (("rounded", 0.0), ("rounded_noise", NOISE)):
        rng = np.random.default_rng(SEED)
        b = oracle.Oracle(cfg)
        b.set_dt_table(ref["dt"])

        def store(prev):
            t_, f = b.fluid()
            if noise > 0.0 and prev is not None:
                f = [p + (c - p) * (1.0 + noise * rng.uniform(-1.0, 1.0, c.size)) for c, p in zip(f, prev)]
            r = round_state(cfg, *f)
            b.set_fluid(t_, *r)
            return r

        prev = store(None)
        for n in range(steps):
            b.step(1)
            prev = store(prev)
            if n % 100 == 99:
                print(f"  {name} step {n + 1}/{steps}", flush=True)
        d = b.diags()
        out[name] = {k: float(np.abs(d[k][1:] - ref["diag_" + k][1:]).max() / np.abs(ref["diag_" + k][1:]).max())
                     for k in DIAG_KEYS}
    out["wall_s"] = round(time.perf_counter() - t0, 1)
    return out


CASES = {
    # the whole 300x150 mm run on one time-step table
    "c2": lambda: floor(workloads.C2(), workloads.C2()["steps"], True),
    # the paper's 750x150 mm channel at dx 1.5 mm, each run on its own CFL step
    "paper": lambda: floor(workloads.paper_geometry(), 300, False),
    # the adjoint form (120x60 mm, 500 steps): the gradient's FP32-storage floor
    "c5_adjoint": lambda: tangent_floor(workloads.C5(), workloads.C5()["steps"]),
    # the precision form's 1,000 steps (600x300 mm): its FP64 diagnostics
    "c3_diag": lambda: diag_floor(workloads.C3(), "c3_1000.npz"),
}


def main(which: str = "all") -> None:
    try:
        with open(OUT) as f:
            res = json.load(f)
    except (OSError, ValueError):
        res = {}
    if which != "all" and which not in CASES:
        raise SystemExit(f"unknown case {which}; one of {sorted(CASES)} or all")
    for k, fn in CASES.items():
        if which in ("all", k):
            print(f"[floor] {k}", flush=True)
            res[k] = fn()
            print(json.dumps(res[k]), flush=True)
    res["method"] = ("FP64 oracle against itself with the fluid state rounded every step to the "
                     "FP32 representation (cell + float32 offset, float32 v and rho); rounded_noise "
                     "scales every particle's change over each step by 1 + u, |u| <= 20 * 2^-24 (seed 2609)")
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "all")
