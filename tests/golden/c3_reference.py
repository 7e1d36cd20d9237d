"""Write c3_1000.npz: the FP64 oracle's whole 1,000-step run of the
precision workload (600 x 300 mm channel, dx 0.5 mm, 719,552 fluid, disk
R 6 mm at 900 m/s), too long to repeat inside a GPU test: its time-step
table, wall-probe histories and diagnostic records (every 10 steps). Only
the oracle runs here; nothing comes from the GPU path.

python -m tests.golden.c3_reference
"""
from __future__ import annotations

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

OUT = os.path.join(HERE, "c3_1000.npz")


def main() -> None:
    cfg = workloads.C3()
    n = cfg["steps"]
    o = oracle.Oracle(cfg)
    t0 = time.perf_counter()
    for k in range(0, n, 50):
        o.step(50)
        print(f"  step {k + 50}/{n} ({time.perf_counter() - t0:.0f} s)", flush=True)
    t, dt, p = o.probes()
    d = o.diags()
    np.savez_compressed(OUT, t=t, dt=dt, p=p, **{"diag_" + k: v for k, v in d.items()},
                        steps=n, n_fluid=o.nf)
    print(f"wrote {OUT}: {n} steps, {o.nf} fluid, {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
