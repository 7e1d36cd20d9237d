"""The paper's cubic B-spline kernel (eq. cubic-kernel) in the FP64 oracle
(kernel_type 1), and the whole solver with it.

Pins: the 2D normalisation sigma_d = 10 / (7 pi h^2) integrates W to one; F
is (1/r) dW/dr; W and dW/dq are continuous at q = 1 and vanish at q = 2; the
lattice moment sum_j V_j r_ij (x) grad W_ij is -I; a whole run with the cubic
kernel conserves mass and momentum along the channel's free direction as
the Wendland run does.
"""
import math

import numpy as np
from scipy import integrate

import oracle
import workloads


def test_cubic_normalised_and_paper_constant():
    h = 1.3e-3
    val, _ = integrate.quad(lambda r: 2 * math.pi * r * oracle.kernel(r / h, h, 1)[0], 0, 2 * h,
                            points=[h], epsabs=1e-12, limit=200)
    assert abs(val - 1.0) < 1e-10
    assert abs(oracle.kernel(0.0, h, 1)[0] - 10.0 / (7.0 * math.pi * h * h)) < 1e-9 / (h * h)


def test_cubic_gradient_is_the_derivative():
    h = 1.0
    for q in (0.1, 0.5, 0.9, 1.1, 1.5, 1.9):
        e = 1e-6
        dW = (oracle.kernel(q + e, h, 1)[0] - oracle.kernel(q - e, h, 1)[0]) / (2 * e)  # dW/dq
        F = oracle.kernel(q, h, 1)[1]
        assert abs(F - dW / (h * q * h)) <= 1e-7 * max(1.0, abs(F)), q


def test_cubic_smooth_at_one_and_zero_at_two():
    h = 1.0
    e = 1e-9
    a, b = oracle.kernel(1.0 - e, h, 1), oracle.kernel(1.0 + e, h, 1)
    assert abs(a[0] - b[0]) < 1e-8 and abs(a[1] - b[1]) < 1e-8
    assert oracle.kernel(2.0, h, 1) == (0.0, 0.0)
    assert abs(oracle.kernel(2.0 - 1e-6, h, 1)[0]) < 1e-17


def test_cubic_gradient_moment_is_minus_identity():
    dx = 1.0
    h = 3.0 * dx
    n = int(math.ceil(2 * h / dx)) + 1
    M = np.zeros((2, 2))
    for i in range(-n, n + 1):
        for j in range(-n, n + 1):
            if i == 0 and j == 0:
                continue
            r = np.array([-i * dx, -j * dx])
            F = oracle.kernel(np.hypot(*r) / h, h, 1)[1]
            M += dx * dx * np.outer(r, F * r)
    assert np.allclose(M, -np.eye(2), atol=5e-3)


def test_cubic_run_conserves_mass_and_differs_from_wendland():
    cfg = workloads.tiny()
    ow, oc = oracle.Oracle(cfg), oracle.Oracle(dict(cfg, kernel_type=1))
    ow.step(40)
    oc.step(40)
    dw, dc = ow.diags(), oc.diags()
    assert np.abs(dc["mass"] - dc["mass"][0]).max() <= 1e-12 * dc["mass"][0]
    _, _, pw = ow.probes()
    _, _, pc = oc.probes()
    # the same flow seen through another kernel: close, not equal
    assert np.abs(pc).max() > 0 and not np.array_equal(pw, pc)
    assert np.abs(pc - pw).max() <= 0.5 * np.abs(pw).max()
