"""Benchmark of the planar WCSPH hot path on one MI355X.

Workload: the 300x150 mm channel at dx = 0.5 mm (179,552 fluid particles,
5,536 ghosts), disk R = 6 mm at 900 m/s decelerating, four wall probes
recorded every step, 2,000 predictor-corrector steps from t = 0.

value = fluid particle-steps per second over the timed steps, with the
state already resident in HBM. The roofline block prices the pair-sum
kernel (the dominant kernel) with its algorithmic flops against the FP32
vector peak, timed with HIP events on the library's stream; its traffic
is the HBM bytes per launch from the committed hardware-counter summary
(null once the kernel source differs from the one measured).
step_roofline prices the whole step with its algorithmic HBM bytes per
fluid particle-step against the HBM peak. cpu_baseline times the FP64
oracle on the host cores on a bounded sample of the same workload (its
first steps).

python bench.py [--gpus 1] [--steps 2000] [--warmup 50]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic work of one pair-kernel launch: per fluid particle, every
# candidate of its 3x3 cells costs the distance test and every in-support
# neighbour the pair law (FMA = 2 flops; sqrt and reciprocals not counted)
FLOP_PER_CANDIDATE = 5     # the two coordinate differences and |r|^2 as a multiply and an FMA
FLOP_PER_PAIR = 53         # kernel, continuity + delta, pressure + AV, laminar, XSPH
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (published; packed FP32)
PEAK_FP32_SCALAR_TFLOPS = 78.6  # the same without packed FP32: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E peak (published)
# algorithmic HBM bytes of one fluid particle-step (two evaluations): the
# state read and written by each evaluation plus the cell-list rebuild
# (keys, counting sort, permuted state), neighbour data counted once
ALG_BYTES_PER_PARTICLE_STEP = 292
KERNELS_SRC = os.path.join(ROOT, "paper_2609_05494_amd", "csrc", "wcsph_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pair_traffic.json")


def kernels_sha256() -> str:
    """Digest of the kernel source, and of the autotuned scan shapes when
    there are any (a different shape is a different binary)."""
    import hashlib
    h = hashlib.sha256()
    with open(KERNELS_SRC, "rb") as f:
        h.update(f.read())
    tuned = os.path.join(os.path.dirname(KERNELS_SRC), "wcsph_tuned.h")
    if os.path.exists(tuned):
        with open(tuned, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pair_traffic():
    """HBM bytes per pair-kernel launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or
    None when the kernel source has changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernels_sha256") != kernels_sha256():
        return None
    return float(t["bytes_per_launch"])


def pair_flops(s) -> float:
    """Algorithmic flops of one pair-kernel launch on the solver's current
    state: per fluid particle, the candidates in its 3x3 cells and the
    in-support neighbours."""
    nb = s.export_neighbours()
    ex = s.export_cells()
    cs = ex["cell_start"].astype(np.int64)
    occ = np.diff(cs)
    nf = s.nf
    fluid = nb["ids"] < nf
    cfg = s.cfgs[0]
    ncx = int(np.ceil((cfg["L"] + 6 * cfg["dx"]) / cfg["cell_size"]))
    ncy = occ.size // ncx
    grid = occ.reshape(ncy, ncx)
    pad = np.pad(grid, 1)
    cand = sum(pad[1 + dy:1 + dy + ncy, 1 + dx:1 + dx + ncx] for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    cand_per_cell = cand.ravel()
    # candidates of each fluid particle = occupancy of its 3x3 block (minus itself)
    keys = np.repeat(np.arange(occ.size), occ)  # key of each sorted slot
    n_cand = (cand_per_cell[keys] - 1)[fluid]
    n_pair = nb["count"][fluid]
    return float(n_cand.sum() * FLOP_PER_CANDIDATE + n_pair.sum() * FLOP_PER_PAIR), \
        float(n_cand.mean()), float(n_pair.mean())


def host_cpu():
    """CPU model, physical cores and logical CPUs of the host (/proc/cpuinfo),
    and the CPUs this process may run on."""
    model, cores, logical = "unknown", set(), 0
    try:
        phys = core = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name":
                    model = v
                    logical += 1
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return model, len(cores) or logical, logical, avail


def cpu_baseline(steps_1: int = 12, steps_n: int = 240):
    """The FP64 oracle on the host cores (test infrastructure, as it stands):
    the first steps of the same 300x150 mm workload, once on one thread and
    once on every thread the process may use, each run a fresh process."""
    import subprocess
    model, phys, logical, avail = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", avail))
    threads = max(1, min(threads, avail))
    runs = {}
    for n_thr, steps in ((1, steps_1), (threads, steps_n)):
        r = subprocess.run([sys.executable, "-m", "oracle.timing", "C2", str(steps), str(n_thr)],
                           capture_output=True, text=True, check=True, cwd=ROOT, timeout=600)
        runs[n_thr] = json.loads(r.stdout.strip().splitlines()[-1])
    one, alln = runs[1], runs[threads]
    return dict(value=alln["value"], unit="fluid particle-steps/s", cores=threads, kind="oracle",
                value_1thread=one["value"], cpu_model=model, physical_cores=phys, logical_cpus=logical,
                sample=f"FP64 oracle (C++17, OpenMP) on the same 300x150 mm / dx 0.5 mm workload from "
                       f"t = 0: first {alln['steps']} steps on {threads} threads ({alln['wall_s']} s) and "
                       f"first {one['steps']} steps on 1 thread ({one['wall_s']} s), stepping only")


def batched_vs_plain(wc, workloads, steps: int):
    """The 64-instance coefficient sweep (seeded draws) in one batched
    context vs the same 64 problems run one after another through the plain
    solver, both for `steps` steps from t = 0 on the same GPU."""
    import torch
    cfgs = workloads.C4()
    b = wc.Solver(cfgs, "cuda:0")
    blob = b.save_state()
    b.step(5)
    b.synchronize()
    b.load_state(blob)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.synchronize()
    tb = time.perf_counter() - t0
    nf = b.n_fluid_total
    unstable = any("unstable" in b.read_diagnostics(k, check=False) for k in range(b.n_inst))
    b.close()
    tp = 0.0
    for cfg in cfgs:
        s = wc.Solver(cfg, "cuda:0")
        s.step(2)
        s.synchronize()
        blob = s.save_state()
        s.load_state(blob)
        t0 = time.perf_counter()
        s.step(steps)
        s.synchronize()
        tp += time.perf_counter() - t0
        s.close()
    return dict(workload="64 instances, L in 200-400 mm x 100 mm, dx 1 mm, alpha in [0.01, 0.5], "
                         "delta in [0, 0.2], v0 in [600, 900] m/s, seed 2609",
                n_fluid=int(nf), steps=steps,
                batched_s=round(tb, 4), plain_sequential_s=round(tp, 4),
                batched_value=nf * steps / tb, plain_value=nf * steps / tp,
                speedup=round(tp / tb, 3), unit="fluid particle-steps/s", unstable=unstable)


def adjoint_vs_fd(wc, workloads, steps: int, ckpt: int):
    """Gradient of the summed wall-probe impulse w.r.t. (alpha, delta, c0) on
    the 120x60 mm / dx 0.5 mm channel: one forward + reverse sweep vs the
    plain solver's forward + six runs a central finite difference needs, on
    the same GPU and fixed time-step table. ckpt >= steps: the forward tapes
    the whole run (about 2.2 GB at 500 steps) and nothing is replayed. One
    untimed call first allocates the tape (the plain runs' graphs are
    likewise built before their timing)."""
    cfg = workloads.C5()
    s = wc.Solver(cfg, "cuda:0")
    blob = s.save_state()
    s.step(steps)
    _, dt, _ = s.read_probes()
    s.load_state(blob)
    s.set_dt_table(dt)
    s.adj_forward(steps, ckpt)
    s.adj_backward(1.0)
    s.load_state(blob)
    s.synchronize()
    t0 = time.perf_counter()
    J = s.adj_forward(steps, ckpt)
    g = s.adj_backward(1.0)
    t_adj = time.perf_counter() - t0
    # plain runs: forward + 6 perturbed runs of the same length
    t_plain = 0.0
    for k in range(7):
        s.load_state(blob)
        s.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        s.synchronize()
        t_plain += time.perf_counter() - t0
    nf = s.nf
    s.close()
    return dict(workload="120x60 mm channel, dx 0.5 mm, 28,352 fluid, 900 m/s, " + f"{steps} steps, " +
                         ("the whole run taped by the forward" if ckpt >= steps else f"checkpoint every {ckpt}"),
                n_fluid=int(nf), steps=steps, J=J, grad_alpha_delta_c0=[float(x) for x in g],
                adjoint_s=round(t_adj, 4), forward_plus_6_fd_s=round(t_plain, 4),
                ratio_fd_over_adjoint=round(t_plain / t_adj, 3))


def two_way_run(wc, workloads, steps: int, prescribed_value: float):
    """The headline workload with the two-way coupled disk (the extra disk
    update launch per step), `steps` steps from t = 0, with the disk's final
    velocity and the drift of e_disk + w_boundary since the coupling began."""
    import torch
    cfg = workloads.two_way(workloads.C2())
    s = wc.Solver(cfg, "cuda:0")
    blob = s.save_state()
    s.step(20)
    s.synchronize()
    s.load_state(blob)
    s.read_diagnostics()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.synchronize()
    el = time.perf_counter() - t0
    d = s.read_diagnostics(check=False)
    x, v, _ = s.disk_state()
    k = np.nonzero(d["t"] > cfg["kin_t_ramp"] + 2 * d["dt"].max())[0]
    drift = None
    if k.size:
        tot = d["e_disk"][k] + d["w_boundary"][k]
        drift = float(np.abs(tot - tot[0]).max() / d["e_disk"][k[0]])
    nf = s.nf
    s.close()
    value = nf * steps / el
    return dict(workload="300x150 mm channel, dx 0.5 mm, disk of steel density per unit depth "
                         f"({cfg['disk_mass']:.4g} kg/m) released at 900 m/s after the ramp",
                steps=steps, value=value, unit="fluid particle-steps/s",
                ms_per_step=round(el / steps * 1e3, 5), vs_prescribed=round(value / prescribed_value, 4),
                disk_v_end=v, disk_x_end=x, energy_drift_rel=drift,
                unstable=bool(d.get("unstable", False)))


def audit_run(wc, workloads, steps: int, prescribed_value: float):
    """The headline workload with the energy audit on (the second pair pass
    carries the audit sums), `steps` steps from t = 0: its cost and the
    ledger of eq. energy-audit at the end."""
    import torch
    cfg = dict(workloads.C2(), audit=1)
    s = wc.Solver(cfg, "cuda:0")
    blob = s.save_state()
    s.step(20)
    s.synchronize()
    s.load_state(blob)
    s.read_diagnostics()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.synchronize()
    el = time.perf_counter() - t0
    d = s.read_diagnostics(check=False)
    nf = s.nf
    s.close()
    e = d["ke"] + d["e_el"] + d["e_pot"]
    keys = ("w_boundary", "w_ghost", "d_av", "d_visc", "w_delta", "w_enforce", "w_clamp")
    terms = {k: float(d[k][-1]) for k in keys}
    ledger = (terms["w_ghost"] - terms["d_av"] - terms["d_visc"] + terms["w_delta"] + terms["w_enforce"]
              + terms["w_clamp"])
    value = nf * steps / el
    return dict(workload="300x150 mm channel, dx 0.5 mm, prescribed disk, energy audit on",
                steps=steps, value=value, unit="fluid particle-steps/s",
                ms_per_step=round(el / steps * 1e3, 5), vs_plain=round(value / prescribed_value, 4),
                delta_e_fluid=float(e[-1] - e[0]), **terms,
                residual_rel=float(((e[-1] - e[0]) - ledger) / abs(terms["w_ghost"])),
                unstable=bool(d.get("unstable", False)))


def qav_run(wc, workloads, steps: int, prescribed_value: float, beta: float = 1.0):
    """The headline workload with the quadratic artificial viscosity term
    (beta mu^2 / rho_bar on top of the linear term), `steps` steps from t = 0."""
    import torch
    cfg = dict(workloads.C2(), beta=beta)
    s = wc.Solver(cfg, "cuda:0")
    blob = s.save_state()
    s.step(20)
    s.synchronize()
    s.load_state(blob)
    s.read_probes()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.synchronize()
    el = time.perf_counter() - t0
    _, _, p = s.read_probes()
    unstable = bool(s.read_diagnostics(check=False).get("unstable", False))
    nf = s.nf
    s.close()
    value = nf * steps / el
    return dict(workload=f"300x150 mm channel, dx 0.5 mm, 900 m/s, alpha 0.1 and beta {beta}",
                steps=steps, value=value, unit="fluid particle-steps/s",
                ms_per_step=round(el / steps * 1e3, 5), vs_linear=round(value / prescribed_value, 4),
                probe_peak_pa=float(np.abs(p).max()), unstable=unstable)


def mg_run(wc, workloads, steps: int, tait_value: float):
    """The headline workload with the paper's Mie-Grueneisen EOS at zero
    specific internal energy (C = c0 = 1448 m/s) in place of Tait, `steps`
    steps from t = 0."""
    import torch
    cfg = workloads.mie_grueneisen(workloads.C2())
    s = wc.Solver(cfg, "cuda:0")
    blob = s.save_state()
    s.step(20)
    s.synchronize()
    s.load_state(blob)
    s.read_probes()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.synchronize()
    el = time.perf_counter() - t0
    _, _, p = s.read_probes()
    unstable = bool(s.read_diagnostics(check=False).get("unstable", False))
    nf = s.nf
    s.close()
    value = nf * steps / el
    return dict(workload="300x150 mm channel, dx 0.5 mm, 900 m/s, Mie-Grueneisen EOS (e = 0), C = 1448 m/s",
                steps=steps, value=value, unit="fluid particle-steps/s",
                ms_per_step=round(el / steps * 1e3, 5), vs_tait=round(value / tait_value, 4),
                probe_peak_pa=float(np.abs(p).max()), unstable=unstable)


def axisymmetric_run(wc, workloads, steps: int, planar_peaks):
    """The headline workload in the axisymmetric r-z form (a 300 mm tank of
    radius 75 mm, 89,776 fluid rings, the sphere on the axis), `steps` steps
    from t = 0: its rate, and its wall-probe peaks against the planar run's
    at the same stations (75 mm from the projectile's path): the
    out-of-plane relief the planar section discards."""
    import torch
    cfg = workloads.axisymmetric(workloads.C2())
    s = wc.Solver(cfg, "cuda:0")
    blob = s.save_state()
    s.step(20)
    s.synchronize()
    s.load_state(blob)
    s.read_probes()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.synchronize()
    el = time.perf_counter() - t0
    _, _, p = s.read_probes()
    d = s.read_diagnostics(check=False)
    nf = s.nf
    s.close()
    peaks = np.abs(p).max(0)  # probes: (30 mm, axis), (30 mm, wall), (105 mm, axis), (105 mm, wall)
    wall = [float(peaks[1]), float(peaks[3])]
    out = dict(workload="300 mm tank of radius 75 mm (r-z), dx 0.5 mm, 89,776 fluid rings, sphere R 6 mm "
                        "on the axis at 900 m/s",
               steps=steps, value=nf * steps / el, unit="fluid ring-steps/s",
               ms_per_step=round(el / steps * 1e3, 5),
               probe_peaks_pa={"axis_30mm": float(peaks[0]), "wall_30mm": wall[0],
                               "axis_105mm": float(peaks[2]), "wall_105mm": wall[1]},
               mass_3d_kg=float(d["mass"][-1]), unstable=bool(d.get("unstable", False)))
    if planar_peaks is not None:
        out["planar_over_rz_wall_peak"] = [round(planar_peaks[k] / wall[k], 3) for k in range(2)]
    return out


def paper_production_run(wc, workloads, t_end: float = 150e-6):
    """The paper's production case in its own geometry (750x150 mm channel,
    dx = 1.5 mm, 49,947 fluid, 900 m/s) with the paper's kernel, alpha and
    single-line walls, simulated to 150 us as the paper's run was; the
    paper's wall clock for that run (0.23 min on a TITAN RTX with its own
    scheme: summation density, Mie-Grueneisen EOS, leapfrog) is context."""
    import torch
    cfg = workloads.paper_geometry()
    s = wc.Solver(cfg, "cuda:0")
    blob = s.save_state()
    s.step(20)
    s.synchronize()
    s.load_state(blob)
    s.read_probes()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, t_sim, peak = 0, 0.0, 0.0
    while t_sim < t_end:
        s.step(100)
        steps += 100
        t, dt, p = s.read_probes()  # the rows of these steps only
        t_sim = float(t[-1] + dt[-1])
        peak = max(peak, float(np.abs(p).max()))
    el = time.perf_counter() - t0
    nf = s.nf
    unstable = bool(s.read_diagnostics(check=False).get("unstable", False))
    s.close()
    return dict(workload="750x150 mm channel, dx 1.5 mm, 49,947 fluid, 900 m/s, cubic spline kernel, "
                         "alpha 0.03, single-line walls, to 150 us",
                steps=steps, simulated_us=round(t_sim * 1e6, 3), wall_s=round(el, 4),
                value=nf * steps / el, unit="fluid particle-steps/s", ms_per_step=round(el / steps * 1e3, 5),
                paper_wall_s=13.8, paper_hardware="NVIDIA TITAN RTX, Numba-CUDA, the paper's own scheme",
                probe_peak_pa=peak, unstable=unstable)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--reps", type=int, default=50, help="pair-kernel timing launches")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--batch-steps", type=int, default=1000,
                    help="steps of the batched-sweep comparison (0 skips it)")
    ap.add_argument("--adj-steps", type=int, default=500,
                    help="steps of the adjoint comparison (0 skips it)")
    ap.add_argument("--two-way-steps", type=int, default=2000,
                    help="steps of the two-way coupled run (0 skips it)")
    ap.add_argument("--audit-steps", type=int, default=2000,
                    help="steps of the energy-audit run (0 skips it)")
    ap.add_argument("--qav-steps", type=int, default=2000,
                    help="steps of the quadratic-viscosity run (0 skips it)")
    ap.add_argument("--mg-steps", type=int, default=2000,
                    help="steps of the Mie-Grueneisen run (0 skips it)")
    ap.add_argument("--axisym-steps", type=int, default=2000,
                    help="steps of the axisymmetric r-z run (0 skips it)")
    ap.add_argument("--paper-run", type=int, default=1,
                    help="1: time the paper's production case to 150 us (0 skips it)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference kernel "
                         "of known traffic for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_2609_05494_amd as wc

    if args.copy_calibration > 0:
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cfg = workloads.C2()
    s = wc.Solver(cfg, "cuda:0")
    blob0 = s.save_state()
    s.step(args.warmup)
    s.synchronize()
    s.load_state(blob0)
    s.read_probes()
    s.read_diagnostics()
    print(f"[bench] C2 nf={s.nf} slots={s.n_slots} cells={s.n_cells}: timing {args.steps} steps",
          file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    s.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = s.nf * args.steps / elapsed
    d = s.read_diagnostics(check=False)
    unstable = bool(d.get("unstable", False))
    _, _, p = s.read_probes()

    # roofline of the pair kernel, timed on the final state of the timed run
    flops, mean_cand, mean_pair = pair_flops(s)
    pair_ms = s.time_pair_kernel(args.reps)
    achieved = flops / (pair_ms * 1e-3) / 1e12
    roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(achieved / PEAK_FP32_TFLOPS, 4), traffic=pair_traffic(),
                peak_scalar=PEAK_FP32_SCALAR_TFLOPS,
                frac_scalar=round(achieved / PEAK_FP32_SCALAR_TFLOPS, 4),
                kernel="k_pair<EV_A>", kernel_ms=round(pair_ms, 5),
                flop_per_launch=flops, flop_per_candidate=FLOP_PER_CANDIDATE, flop_per_pair=FLOP_PER_PAIR,
                mean_candidates=round(mean_cand, 2), mean_pairs=round(mean_pair, 2))
    step_gbs = ALG_BYTES_PER_PARTICLE_STEP * value / 1e9
    step_roof = dict(bound="hbm", alg_bytes_per_particle_step=ALG_BYTES_PER_PARTICLE_STEP,
                     achieved=round(step_gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                     frac=round(step_gbs / PEAK_HBM_GBS, 4))
    nf = s.nf
    s.close()

    batched = batched_vs_plain(wc, workloads, args.batch_steps) if args.batch_steps > 0 else None
    adjoint = adjoint_vs_fd(wc, workloads, args.adj_steps, args.adj_steps) if args.adj_steps > 0 else None
    two_way = two_way_run(wc, workloads, args.two_way_steps, value) if args.two_way_steps > 0 else None
    audit = audit_run(wc, workloads, args.audit_steps, value) if args.audit_steps > 0 else None
    qav = qav_run(wc, workloads, args.qav_steps, value) if args.qav_steps > 0 else None
    mg = mg_run(wc, workloads, args.mg_steps, value) if args.mg_steps > 0 else None
    # planar wall-probe peaks at the 30 and 105 mm stations (probes on y = 0)
    planar_wall = [float(np.abs(p[:, 0]).max()), float(np.abs(p[:, 2]).max())] if p.size else None
    axisym = axisymmetric_run(wc, workloads, args.axisym_steps, planar_wall) if args.axisym_steps > 0 else None
    paper = paper_production_run(wc, workloads) if args.paper_run else None
    cpu = None if args.no_cpu else cpu_baseline()
    out = {
        "metric": "WCSPH fluid particle-steps/s at 180k particles",
        "value": value,
        "unit": "fluid particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "300x150 mm channel, dx 0.5 mm, 179,552 fluid + 5,536 ghosts, "
                               "disk R 6 mm at 900 m/s, 4 wall probes, predictor-corrector",
                   "n_fluid": nf, "steps": args.steps, "parallelism": "single GPU"},
        "roofline": roof,
        "step_roofline": step_roof,
        "cpu_baseline": cpu,
        "batched_sweep": batched,
        "adjoint": adjoint,
        "two_way": two_way,
        "energy_audit": audit,
        "quadratic_av": qav,
        "mie_grueneisen": mg,
        "axisymmetric": axisym,
        "paper_production_run": paper,
        "unstable": unstable,
        "probe_peak_pa": float(np.abs(p).max()) if p.size else None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
