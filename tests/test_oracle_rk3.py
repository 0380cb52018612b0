"""Pins of the oracle's three-stage TVD Runge-Kutta step (Sec. 4.3): its
stability polynomial and third-order convergence."""
import math

import numpy as np
import torch

from oracle import snap_oracle as O


def test_amplification_polynomial_real():
    for z in (-2.5, -1.0, -0.1, 0.3, 1.0):
        y = O.rk3(lambda y: z * y, torch.tensor([1.0], dtype=torch.float64), 1.0)
        assert abs(float(y) - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-14


def test_amplification_polynomial_imaginary():
    """y' = A y with A = [[0, -w], [w, 0]] has eigenvalues +-iw: growth |R(iw)|."""
    for w in (0.5, 1.0, 1.5, math.sqrt(3.0)):
        A = torch.tensor([[0.0, -w], [w, 0.0]], dtype=torch.float64)
        y = O.rk3(lambda y: A @ y, torch.tensor([1.0, 0.0], dtype=torch.float64), 1.0)
        R = 1 + 1j * w + (1j * w) ** 2 / 2 + (1j * w) ** 3 / 6
        assert abs(float(y[0]) - R.real) < 1e-14 and abs(float(y[1]) - R.imag) < 1e-14


def test_third_order_convergence():
    # y' = -y^2, y(0) = 1: y(t) = 1 / (1 + t)
    errs = []
    for n in (20, 40, 80, 160):
        dt = 2.0 / n
        y = torch.tensor([1.0], dtype=torch.float64)
        for _ in range(n):
            y = O.rk3(lambda v: -v * v, y, dt)
        errs.append(abs(float(y) - 1.0 / 3.0))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert min(orders) > 2.85 and max(orders) < 3.2, orders
