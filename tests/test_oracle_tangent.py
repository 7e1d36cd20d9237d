"""Forward-mode tangent of the oracle (dual numbers in alpha, delta, c0)
against FP64 central finite differences of J = sum_k sum_n p_k^n dt_n at a
fixed time-step table (relative step 1e-4). The table comes from an oracle
run with the CFL gate, so dt does not depend on c0."""
import numpy as np
import pytest

import oracle
import workloads


def _J(cfg, dt):
    o = oracle.Oracle(cfg)
    o.set_dt_table(dt)
    o.step(dt.size)
    return o.impulse()


@pytest.mark.parametrize("n", [40])
def test_tangent_matches_central_differences(n):
    cfg = workloads.tiny(v0=600.0)
    o = oracle.Oracle(cfg)
    o.step(n)
    _, dt, _ = o.probes()
    J, dJ = oracle.tangent_J(cfg, dt)
    assert abs(J - _J(cfg, dt)) <= 1e-12 * abs(J)
    assert abs(J) > 0
    for k, name in enumerate(("alpha", "delta", "c0")):
        h = 1e-4 * cfg[name]
        Jp = _J(dict(cfg, **{name: cfg[name] + h}), dt)
        Jm = _J(dict(cfg, **{name: cfg[name] - h}), dt)
        fd = (Jp - Jm) / (2 * h)
        print(f"{name}: tangent {dJ[k]:.10e} fd {fd:.10e}")
        assert abs(fd - dJ[k]) <= 1e-5 * abs(dJ[k]) + 1e-12 * abs(J) / cfg[name]
