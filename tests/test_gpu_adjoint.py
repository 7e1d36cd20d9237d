"""Reverse sweep on the GPU: dJ/d(alpha, delta, c0) of the summed wall-probe
pressure impulse against the oracle's FP64 forward-mode tangent, at a fixed
time-step table taken from an oracle run (so dt does not depend on c0).
The GPU adjoint runs in FP32 on the FP32 trajectory; the tolerance is
stated per test and the measured error printed."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")


def _table(cfg, n):
    o = oracle.Oracle(cfg)
    o.step(n)
    return o.probes()[1]


def _gpu_grad(cfg, dt, ckpt):
    s = wc.Solver(cfg, "cuda:0")
    s.set_dt_table(dt)
    J = s.adj_forward(dt.size, ckpt)
    g = s.adj_backward(1.0)
    s.close()
    return J, g


def _report(name, J, g, Jo, go):
    rel = np.abs(g - go) / np.abs(go)
    print(f"{name}: J gpu {J:.8e} oracle {Jo:.8e} (rel {abs(J - Jo) / abs(Jo):.2e}); "
          f"grad gpu {g} oracle {go}; rel err {rel}")
    return rel


def test_adjoint_small_case_vs_oracle_tangent():
    cfg = workloads.tiny(v0=600.0)
    n = 40
    dt = _table(cfg, n)
    print(f"[gpu] adjoint tiny case, {n} steps", flush=True)
    J, g = _gpu_grad(cfg, dt, 10)
    Jo, go = oracle.tangent_J(cfg, dt)
    rel = _report("tiny", J, g, Jo, go)
    assert abs(J - Jo) <= 1e-4 * abs(Jo)
    assert np.all(rel <= 2e-3)


def test_adjoint_checkpointing_does_not_change_the_gradient():
    """The forward that tapes the whole run itself (ckpt_every >= n_steps:
    nothing replayed), a ckpt_every far beyond the run (taken as the run),
    and 7-step checkpoint segments with replays give the same J and gradient
    bit for bit; a second forward and backward on the same context reuses
    its tape and gives them again."""
    cfg = workloads.tiny(v0=600.0)
    n = 30
    dt = _table(cfg, n)
    print(f"[gpu] adjoint tape forms, {n} steps", flush=True)
    J1, g1 = _gpu_grad(cfg, dt, n)
    J2, g2 = _gpu_grad(cfg, dt, 7)
    J3, g3 = _gpu_grad(cfg, dt, 1 << 30)
    assert J1 == J2 == J3
    assert np.array_equal(g1, g2) and np.array_equal(g1, g3)
    s = wc.Solver(cfg, "cuda:0")
    s.set_dt_table(dt)
    blob = s.save_state()
    for _ in range(2):
        s.load_state(blob)
        assert s.adj_forward(n, n) == J1
        assert np.array_equal(s.adj_backward(1.0), g1)
    s.close()


def test_autograd_function_matches_reverse_sweep():
    import torch
    cfg = workloads.tiny(v0=600.0)
    n = 20
    dt = _table(cfg, n)
    s = wc.Solver(cfg, "cuda:0")
    s.set_dt_table(dt)
    blob = s.save_state()
    Fn = wc.impulse_fn()
    th = [torch.tensor(cfg[k], dtype=torch.float64, requires_grad=True) for k in ("alpha", "delta", "c0")]
    J = Fn.apply(th[0], th[1], th[2], s, blob, n, 5)
    J.backward()
    s.load_state(blob)
    s.set_coefficients(cfg["alpha"], cfg["delta"], cfg["c0"])
    J2 = s.adj_forward(n, 5)
    g2 = s.adj_backward(1.0)
    assert float(J.detach()) == J2
    assert np.array_equal(np.array([t.grad.item() for t in th]), g2)
    s.close()


def test_adjoint_C5_full_size():
    """120x60 mm at dx 0.5 mm (28,352 fluid), 900 m/s, 500 steps,
    checkpoint every 50 steps, and the same with the whole run taped by the
    forward (bitwise equal). Bars per component: twice the oracle's own
    FP32 floor at this workload, the FP64 tangent run with its state rounded
    to the FP32 representation after every step against the plain FP64
    tangent (tests/golden/chaos_floor.py, case c5_adjoint: relative
    differences 1.5e-2, 1.2e-3 and 2.0e-4 for alpha, delta and c0)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "chaos_floor.json")) as f:
        floor = np.array(json.load(f)["c5_adjoint"]["grad_rel"])
    cfg = workloads.C5()
    n = cfg["steps"]
    dt = _table(cfg, n)
    print(f"[gpu] adjoint C5, {n} steps, checkpoint 50", flush=True)
    J, g = _gpu_grad(cfg, dt, 50)
    # the whole run taped by the forward (about 2.2 GB, nothing replayed):
    # bitwise the checkpointed sweep's J and gradient
    Jt, gt = _gpu_grad(cfg, dt, n)
    assert Jt == J and np.array_equal(gt, g)
    Jo, go = oracle.tangent_J(cfg, dt)
    rel = _report("C5", J, g, Jo, go)
    print(f"C5 bars (2x the FP32 floor): {2.0 * floor}")
    assert abs(J - Jo) <= 1e-3 * abs(Jo)
    assert np.all(rel <= 2.0 * floor)


def test_adjoint_matches_central_differences_of_the_gpu_forward():
    """The reverse sweep against central differences of the GPU's own forward
    run (same kernels, same dt table), tiny case, 40 steps. Steps: 3 % of
    alpha and delta, 1 % of c0; at these steps the FP64 oracle's central
    differences match its tangent to 6e-5, 3e-4 and 5e-6 (truncation), and
    they move J by 0.3 %, 0.2 % and 8 %, far above FP32 run-to-run rounding
    of J (about 1e-6 relative)."""
    cfg = workloads.tiny(v0=600.0)
    n = 40
    dt = _table(cfg, n)
    print(f"[gpu] adjoint vs central differences, tiny, {n} steps", flush=True)
    J, g = _gpu_grad(cfg, dt, 10)
    fd = np.zeros(3)
    for k, (key, eps) in enumerate((("alpha", 0.03), ("delta", 0.03), ("c0", 0.01))):
        h = eps * cfg[key]
        Jp, _ = _gpu_grad(dict(cfg, **{key: cfg[key] + h}), dt, 10)
        Jm, _ = _gpu_grad(dict(cfg, **{key: cfg[key] - h}), dt, 10)
        fd[k] = (Jp - Jm) / (2.0 * h)
    rel = np.abs(fd / g - 1.0)
    # the same differences of the FP64 oracle's forward run
    fdo = np.zeros(3)
    for k, (key, eps) in enumerate((("alpha", 0.03), ("delta", 0.03), ("c0", 0.01))):
        h = eps * cfg[key]
        Jo = []
        for sgn in (1.0, -1.0):
            o = oracle.Oracle(dict(cfg, **{key: cfg[key] + sgn * h}))
            o.set_dt_table(dt)
            o.step(n)
            Jo.append(o.impulse())
        fdo[k] = (Jo[0] - Jo[1]) / (2.0 * h)
    rel_o = np.abs(fd / fdo - 1.0)
    print(f"adjoint {g} GPU central differences {fd} (rel {rel}) oracle central differences {fdo} "
          f"(GPU vs oracle {rel_o})")
    assert np.all(rel <= 2e-3)
    assert np.all(rel_o <= 2e-3)
