"""Energy audit (audit = 1) on the HIP path against the FP64 oracle.

Bars: over 200 steps of the 80x40 mm channel (prescribed and two-way disk),
each audit integral (d_av, w_delta, w_ghost, w_enforce, w_clamp) within 2e-3
of the oracle's w_ghost and d_visc within 1e-2 of its own value; the GPU's
ledger closes as the oracle's does (2 % of w_ghost); the audit leaves the
state bitwise unchanged; a checkpoint restores the running sums.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")

TERMS = ("d_av", "d_visc", "w_delta", "w_ghost", "w_enforce", "w_clamp")


def _solver(cfg):
    print(f"[gpu] solver L={cfg['L']} W={cfg['W']} dx={cfg['dx']} audit={cfg.get('audit', 0)}", flush=True)
    return wc.Solver(cfg, "cuda:0")


def _ledger(d):
    e = d["ke"] + d["e_el"] + d["e_pot"]
    led = d["w_ghost"] - d["d_av"] - d["d_visc"] + d["w_delta"] + d["w_enforce"] + d["w_clamp"]
    return (e - e[0]) - led


@pytest.mark.parametrize("mode", ["prescribed", "two_way"])
def test_audit_C1_matches_oracle(mode):
    cfg = workloads.C1()
    if mode == "two_way":
        cfg = workloads.two_way(cfg)
    s = _solver(dict(cfg, audit=1))
    s.step(200)
    dg = s.read_diagnostics()
    s.close()
    o = oracle.Oracle(cfg)
    o.step(200)
    do = o.diags()
    scale = abs(do["w_ghost"][-1])
    for k in TERMS:
        print(f"{mode} {k}: gpu {dg[k][-1]:.6f} oracle {do[k][-1]:.6f}")
    for k in ("d_av", "w_delta", "w_ghost", "w_enforce", "w_clamp"):
        assert np.abs(dg[k] - do[k]).max() <= 2e-3 * scale, k
    assert abs(dg["d_visc"][-1] - do["d_visc"][-1]) <= 1e-2 * do["d_visc"][-1]
    rg, ro = _ledger(dg), _ledger(do)
    print(f"{mode} ledger residual: gpu {rg[-1]:.3f} oracle {ro[-1]:.3f} (w_ghost {scale:.1f})")
    assert abs(rg[-1]) <= 0.02 * scale
    assert np.all(np.diff(dg["d_av"]) >= 0) and np.all(np.diff(dg["d_visc"]) >= 0)


def test_audit_leaves_the_state_unchanged():
    cfg = workloads.two_way(workloads.C1())
    a, b = _solver(cfg), _solver(dict(cfg, audit=1))
    a.step(60)
    b.step(60)
    for u, v in zip(a.fluid()[1], b.fluid()[1]):
        assert np.array_equal(u, v)
    da, db = a.read_diagnostics(), b.read_diagnostics()
    for k in TERMS:
        assert np.all(da[k] == 0.0), k
    assert db["d_av"][-1] > 0 and db["w_ghost"][-1] > 0
    for k in ("ke", "e_el", "w_boundary", "e_disk"):
        assert np.array_equal(da[k], db[k]), k
    a.close()
    b.close()


def test_audit_checkpoint_restores_the_sums():
    cfg = dict(workloads.C1(), audit=1)
    s = _solver(cfg)
    s.step(20)
    blob = s.save_state()
    s.step(30)
    d1 = s.read_diagnostics()
    s.load_state(blob)
    s.step(30)
    d2 = s.read_diagnostics()
    for k in TERMS:
        assert d1[k][-1] == d2[k][-1], k
    s.close()


def test_audit_needs_a_single_instance_context():
    with pytest.raises(wc.WcsphError):
        wc.Solver([dict(workloads.tiny(), audit=1), workloads.tiny()], "cuda:0")
