"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (FP32 GPU vs FP64 oracle): cell keys, stable permutation, cell ranges
and in-support neighbour sets bit-exact; one evaluation's density rate,
acceleration, XSPH velocity and ghost pressure within 1e-4 of the field's
maximum; wall-probe histories over 200 steps within 1e-3 of each probe's
peak; mass conserved to 1e-12.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests import shared_state

pytestmark = pytest.mark.gpu

wc = pytest.importorskip("paper_2609_05494_amd")


def _solver(cfg):
    print(f"[gpu] solver L={cfg['L']} W={cfg['W']} dx={cfg['dx']} R={cfg['disk_R']}", flush=True)
    return wc.Solver(cfg, "cuda:0")


def _rel(a, b):
    """max_i |a_i - b_i| / max_i |b_i|"""
    return np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300)


def _relvec(ax, ay, bx, by):
    """max_i |a_i - b_i| / max_i |b_i| for 2-vectors"""
    d = np.hypot(np.asarray(ax, np.float64) - bx, np.asarray(ay, np.float64) - by)
    return d.max() / max(np.hypot(bx, by).max(), 1e-300)


def p_quantum(cfg):
    """Pressure step of one FP32 ulp of rho near rho0: gamma B ulp(rho0) / rho0.
    Pressures below a few of these are not resolved by an FP32 density."""
    B = cfg["rho0"] * cfg["c0"] ** 2 / cfg["gamma"]
    return cfg["gamma"] * B * float(np.spacing(np.float32(cfg["rho0"]))) / cfg["rho0"]


def _shared_state(cfg, steps):
    """Oracle state after `steps` steps rounded to the FP32 representation
    (in the test) and loaded into both sides."""
    print(f"[gpu] shared state after {steps} oracle steps", flush=True)
    s, o = shared_state.shared(cfg, steps, wc, oracle)
    t, f = s.fluid()
    to, fo = o.fluid()
    assert t == to
    for a, b in zip(f, fo):  # the GPU holds exactly the rounded values
        assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max())
    return s, o


# ---------------------------------------------------------------- cell list

def _all_positions(o, f):
    """Fluid positions (rounded state) followed by the oracle's own ghost
    positions, in particle-id order (the storage order after a load)."""
    gx, gy, _ = o.ghosts()
    return np.concatenate([f[0], gx]), np.concatenate([f[1], gy])


def _sort_inputs(cfg, steps):
    s, o = _shared_state(cfg, steps)
    o.eval_rates()  # places the disk ring at the state's time
    _, f = o.fluid()
    x, y = _all_positions(o, f)
    return s, o, x, y


@pytest.mark.parametrize("steps", [0, 30])
def test_cell_list_bit_exact(steps):
    """Keys, stable permutation and cell ranges of one cell-list build from
    the same state (the oracle's state after `steps` steps, rounded)."""
    cfg = workloads.C1()
    s, o, x, y = _sort_inputs(cfg, steps)
    ex = s.export_cells()
    assert np.array_equal(ex["ids_pre"], np.arange(s.n_slots))  # load order = id order
    keys, perm, cs = oracle.cell_list(cfg, x, y)
    assert np.array_equal(keys, ex["keys"].astype(np.int32))
    assert np.array_equal(perm, ex["perm"].astype(np.int32))
    assert np.array_equal(cs, ex["cell_start"].astype(np.int32))
    assert np.array_equal(ex["ids_post"], ex["ids_pre"][ex["perm"]])
    assert np.array_equal(np.sort(ex["ids_post"]), np.arange(s.n_slots))
    s.close()


def _oracle_neighbour_lists(cfg, x, y, nf, tol=1e-5):
    """In-support neighbour sets of the nf fluid particles by O(N^2) search
    over all particles (x, y: fluid then ghosts, index = particle id), and the
    pairs within tol of the support radius (|r^2 - 4h^2| < tol 4h^2), where
    the FP32 test of the encoded state may fall either side."""
    h = cfg["h_over_dx"] * cfg["dx"]
    s2 = 4.0 * h * h
    wide = dict(cfg, h_over_dx=cfg["h_over_dx"] * np.sqrt(1.0 + 2.0 * tol))
    pr = oracle.brute_pairs(wide, x, y)
    r2 = (x[pr[:, 0]] - x[pr[:, 1]]) ** 2 + (y[pr[:, 0]] - y[pr[:, 1]]) ** 2
    border = np.abs(r2 - s2) < tol * s2
    inside = (r2 < s2) & ~border
    sets = [set() for _ in range(nf)]
    near = [set() for _ in range(nf)]
    for (i, j), a, b in zip(pr, inside, border):
        for u, v in ((i, j), (j, i)):
            if u < nf:
                if a:
                    sets[u].add(int(v))
                elif b:
                    near[u].add(int(v))
    return sets, near


@pytest.mark.parametrize("case,steps", [("tiny", 15), ("C1", 40)])
def test_neighbour_lists_bit_exact(case, steps):
    """The in-support neighbour list of every fluid particle, element by
    element, as the pair kernel finds and sums it, against the oracle's
    O(N^2) search from the same state. Only single pairs within 1e-5 of the
    support radius (W ~ 1e-20 there) are left out, and they are counted."""
    cfg = workloads.tiny() if case == "tiny" else workloads.C1()
    s, o, x, y = _sort_inputs(cfg, steps)
    gl = s.export_neighbour_lists()
    want, near = _oracle_neighbour_lists(cfg, x, y, s.nf)
    n_near = sum(len(b) for b in near)
    n_pairs = sum(len(a) for a in want)
    print(f"[gpu] {case}: {n_pairs} in-support pair entries, {n_near} within 1e-5 of 2h")
    assert n_near <= 1e-3 * n_pairs + 4
    for k in range(s.nf):
        got = gl[k].astype(np.int64)
        assert np.unique(got).size == got.size, k  # no neighbour twice
        assert set(got.tolist()) - near[k] == want[k], k
    s.close()


def test_neighbour_sets_bit_exact():
    """In-support neighbour count and neighbour-id sum of every particle from
    the same state (the test hook's own walk of the 3x3 cells); pairs within
    1e-5 of the support radius (W ~ 0) may fall either side in FP32 and are
    excluded."""
    cfg = workloads.C1()
    s, o, x, y = _sort_inputs(cfg, 40)
    nb = s.export_neighbours()
    cnt, idsum, border = oracle.neighbour_stats(cfg, x, y, np.arange(x.size, dtype=np.int32), tol=1e-5)
    ids = nb["ids"].astype(np.int64)
    clean = border[ids] == 0
    assert clean.mean() > 0.99
    assert np.array_equal(cnt[ids][clean], nb["count"][clean])
    assert np.array_equal(idsum[ids][clean], nb["idsum"][clean])
    s.close()


# ---------------------------------------------------------------- one evaluation

@pytest.mark.parametrize("steps", [0, 100])
def test_one_evaluation_rates_C1(steps):
    cfg = workloads.C1()
    s, o = _shared_state(cfg, steps)
    g = s.export_rates()
    r = o.eval_rates()
    assert _rel(g["drho"], r["drho"]) <= 1e-4
    assert _relvec(g["ax"], g["ay"], r["ax"], r["ay"]) <= 1e-4
    assert _rel(g["Vx"], r["Vx"]) <= 1e-4 and _rel(g["Vy"], r["Vy"]) <= 1e-4
    assert _rel(g["gp"], r["gp"]) <= 1e-4
    assert _rel(g["gvx"], r["gvx"]) <= 1e-4
    s.close()


def test_one_step_state_C1():
    """One full predictor-corrector step from a shared state: density within
    1e-4 relative per particle, positions within 1e-4 dx."""
    cfg = workloads.C1()
    s, o = _shared_state(cfg, 100)
    s.step(1)
    o.step(1)
    _, (xg, yg, vxg, vyg, rg) = s.fluid()
    _, (xo, yo, vxo, vyo, ro) = o.fluid()
    assert np.abs(rg / ro - 1).max() <= 1e-4
    assert np.abs(xg - xo).max() <= 1e-4 * cfg["dx"] and np.abs(yg - yo).max() <= 1e-4 * cfg["dx"]
    assert _relvec(vxg, vyg, vxo, vyo) <= 1e-4
    s.close()


# ---------------------------------------------------------------- whole runs

def test_probe_history_C1_200_steps():
    cfg = workloads.C1()
    s = _solver(cfg)
    s.step(200)
    tg, dtg, pg = s.read_probes()
    o = oracle.Oracle(cfg)
    o.step(200)
    to, dto, po = o.probes()
    assert pg.shape == po.shape == (200, 4)
    assert np.abs(dtg / dto - 1).max() < 1e-5
    assert np.abs(tg - to).max() < 1e-5 * to[-1]
    for k in range(4):
        err = np.abs(pg[:, k] - po[:, k]).max() / np.abs(po[:, k]).max()
        print(f"probe {k}: max rel err {err:.3e} (peak {np.abs(po[:, k]).max():.4g} Pa)")
        assert err <= 1e-3
    d = s.read_diagnostics()
    do = o.diags()
    assert d["mass"].size == do["mass"].size == 21
    assert np.abs(d["mass"] - d["mass"][0]).max() <= 1e-12 * d["mass"][0]
    assert abs(d["mass"][0] - do["mass"][0]) <= 1e-12 * do["mass"][0]
    for k in ("ke", "e_el", "w_boundary"):
        assert abs(d[k][-1] - do[k][-1]) <= 1e-3 * abs(do[k][-1]), k
    assert abs(d["momx"][-1] - do["momx"][-1]) <= 1e-3 * abs(do["momx"][-1])
    s.close()


def test_deterministic_and_checkpoint_roundtrip():
    cfg = workloads.C1()
    s = _solver(cfg)
    s.step(20)
    blob = s.save_state()
    s.step(30)
    a = s.fluid()[1]
    s.load_state(blob)
    s.step(30)
    b = s.fluid()[1]
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    s2 = _solver(cfg)
    s2.step(50)
    c = s2.fluid()[1]
    for u, v in zip(a, c):
        assert np.array_equal(u, v)
    s.close()
    s2.close()


# ---------------------------------------------------------------- full size

def test_full_size_C2_evaluation():
    """C2 (179,552 fluid, 185,088 particles) in the launch configuration the
    benchmark times: one evaluation from a shared state after 20 oracle steps
    (density rate, acceleration, XSPH velocity, ghost pressure and velocity),
    the cell keys, permutation and ranges, and 20 GPU steps' mass."""
    cfg = workloads.C2()
    s, o = _shared_state(cfg, 20)
    g = s.export_rates()
    r = o.eval_rates()
    assert _rel(g["drho"], r["drho"]) <= 1e-4
    assert _relvec(g["ax"], g["ay"], r["ax"], r["ay"]) <= 1e-4
    assert _rel(g["Vx"], r["Vx"]) <= 1e-4 and _rel(g["Vy"], r["Vy"]) <= 1e-4
    assert _rel(g["gp"], r["gp"]) <= 1e-4
    assert _rel(g["gvx"], r["gvx"]) <= 1e-4
    ex = s.export_cells()
    o.eval_rates()
    _, f = o.fluid()
    x, y = _all_positions(o, f)
    keys, perm, cs = oracle.cell_list(cfg, x, y)
    assert np.array_equal(keys, ex["keys"].astype(np.int32))
    assert np.array_equal(perm, ex["perm"].astype(np.int32))
    assert np.array_equal(cs, ex["cell_start"].astype(np.int32))
    s.step(20)
    d = s.read_diagnostics()
    assert np.abs(d["mass"] - d["mass"][0]).max() <= 1e-12 * d["mass"][0]
    s.close()


# ---------------------------------------------------------------- edge cases

def test_edge_cases_small_ragged_and_diskless():
    cases = [
        workloads.tiny(),                                             # a few hundred particles
        dict(workloads.tiny(L=0.0173, W=0.0091), probes=[]),         # ragged grid, no probes
        dict(workloads.tiny(), disk_R=0.0, n_disk_ghosts=0),          # no disk
        dict(workloads.tiny(L=0.006, W=0.006, R=0.0029), probes=[(0.003, 0.0)]),  # disk fills most of the box
    ]
    for cfg in cases:
        s = _solver(cfg)
        s.step(15)
        o = oracle.Oracle(cfg)
        o.step(15)
        _, fg = s.fluid()
        _, fo = o.fluid()
        assert fg[0].size == fo[0].size
        assert np.abs(fg[4] / fo[4] - 1).max() <= 1e-4
        assert np.abs(fg[0] - fo[0]).max() <= 1e-3 * cfg["dx"]
        if cfg["probes"]:
            _, _, pg = s.read_probes()
            _, _, po = o.probes()
            assert np.abs(pg - po).max() <= 1e-3 * np.abs(po).max() + 2 * p_quantum(cfg)
        s.close()


def test_invalid_params_rejected():
    bad = [dict(workloads.C1(), dx=-1.0), dict(workloads.C1(), h_over_dx=2.5),
           dict(workloads.C1(), disk_x0=0.079), dict(workloads.C1(), cell_size=1e-3)]
    for cfg in bad:
        with pytest.raises(wc.WcsphError) as e:
            wc.Solver(cfg, "cuda:0")
        assert e.value.status == wc.E_INVALID


def test_pair_timing_hook_restores_the_state():
    """The measurement hook runs real steps and puts the state back: the run
    continues bit for bit as if the hook had not been called."""
    cfg = workloads.C1()
    s = _solver(cfg)
    s.step(30)
    ms = s.time_pair_kernel(5)
    assert ms > 0.0
    s.step(20)
    a = s.fluid()[1]
    _, _, pa = s.read_probes()
    s2 = _solver(cfg)
    s2.step(50)
    b = s2.fluid()[1]
    _, _, pb = s2.read_probes()
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert np.array_equal(pa, pb)
    s.close()
    s2.close()
