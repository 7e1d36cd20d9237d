"""Round an FP64 fluid state to the representation the FP32 path stores
(cell index + float32 offset inside a cell of edge cell_size, float32
velocity and density), written out here so that both the oracle and the GPU
can start from the same values without either taking the other's output."""
import numpy as np


def round_state(cfg, x, y, vx, vy, rho):
    dc = float(cfg["cell_size"])
    lo = -cfg["ghost_layers"] * cfg["dx"]

    def axis(v):
        c = np.floor((v - lo) / dc)
        o = (v - lo - c * dc).astype(np.float32).astype(np.float64)
        up = o >= np.float32(dc)
        c = np.where(up, c + 1, c)
        o = np.where(up, 0.0, o)
        return lo + c * dc + o

    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    return axis(np.asarray(x)), axis(np.asarray(y)), f32(vx), f32(vy), f32(rho)


def shared(cfg, steps, wc, oracle, device="cuda:0"):
    """Oracle state after `steps` steps, rounded, loaded into a GPU solver and
    a fresh oracle."""
    o = oracle.Oracle(cfg)
    o.step(steps)
    t, f = o.fluid()
    r = round_state(cfg, *f)
    s = wc.Solver(cfg, device)
    s.set_fluid(t, *r)
    o2 = oracle.Oracle(cfg)
    o2.set_fluid(t, *r)
    return s, o2
