"""Throughput of the FP64 CPU oracle (test infrastructure: the reported
CPU baseline, never part of the product path).

    python -m oracle.timing CASE STEPS THREADS [CASE STEPS THREADS ...]

CASE is a workload name (C1, C2, C3). Each run is a fresh process with
OMP_NUM_THREADS set, so that the thread count is fixed when the OpenMP
runtime starts. It prints one line per run: fluid particles, steps, threads,
wall seconds of the stepping alone, and fluid particle-steps/s.
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import time


def _one(case: str, steps: int) -> dict:
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import oracle
    import workloads
    cfg = getattr(workloads, case)()
    o = oracle.Oracle(cfg)
    t0 = time.perf_counter()
    o.step(steps)
    wall = time.perf_counter() - t0
    return {"case": case, "n_fluid": int(o.nf), "steps": steps,
            "threads": int(os.environ.get("OMP_NUM_THREADS", "0")), "wall_s": round(wall, 3),
            "value": o.nf * steps / wall}


def main(argv) -> None:
    if argv and argv[0] == "--one":
        print(json.dumps(_one(argv[1], int(argv[2]))), flush=True)
        return
    if len(argv) % 3:
        raise SystemExit(__doc__)
    for i in range(0, len(argv), 3):
        case, steps, threads = argv[i], argv[i + 1], argv[i + 2]
        env = dict(os.environ, OMP_NUM_THREADS=threads)
        r = subprocess.run([sys.executable, "-m", "oracle.timing", "--one", case, steps], env=env,
                           capture_output=True, text=True, check=True,
                           cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        print(r.stdout.strip(), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
