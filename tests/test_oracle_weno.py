"""Pins of the oracle's WENO5 reconstruction (Sec. 4.2) against what the paper
and the mathematics fix: the printed I_poly and sub-stencil coefficients,
polynomial exactness, the Jiang-Shu smoothness integrals, fifth-order
convergence, the non-oscillatory property and exact symmetries."""
import math
import os
from fractions import Fraction

import numpy as np
import numpy.polynomial.polynomial as P
import pytest
import torch

from oracle import snap_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_fracs(name):
    rows = {}
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if "/" in parts[0] or parts[0].lstrip("-").isdigit():
                rows.setdefault("_", []).append([Fraction(p) for p in parts])
            else:
                rows[parts[0]] = [Fraction(p) for p in parts[1:]]
    return rows


def _unit_args(j):
    return [torch.tensor([1.0 if m == j else 0.0], dtype=torch.float64) for m in range(5)]


def test_ipoly_coefficients_equal_paper():
    gold = _read_fracs("weno5_ipoly.txt")["_"][0]
    assert sum(gold) == 1
    got = [float(O.weno5(*_unit_args(j), linear=True)) for j in range(5)]
    for g_, c in zip(gold, got):
        assert abs(c - float(g_)) < 2e-16


def test_substencils_and_linear_weights_equal_paper():
    gold = _read_fracs("weno5_substencils.txt")
    for k in range(3):
        got = [float(O.weno5_substencils(*_unit_args(j))[k]) for j in range(5)]
        for g_, c in zip(gold["stencil%d" % k], got):
            assert abs(c - float(g_)) < 4e-16
    assert [Fraction(w).limit_denominator(100) for w in O.LINEAR_WEIGHTS] == gold["linear_weights"]


def _poly_cell_averages(coefs, edges):
    """Exact cell averages of sum_k coefs[k] x^k over [edges[i], edges[i+1]]."""
    out = []
    for a, b in zip(edges[:-1], edges[1:]):
        s = Fraction(0)
        for k, c in enumerate(coefs):
            s += c * (b ** (k + 1) - a ** (k + 1)) / (k + 1)
        out.append(s / (b - a))
    return out


def _poly_value(coefs, x):
    return sum(c * x ** k for k, c in enumerate(coefs))


def _face_errors(deg, linear, seed=0, h=Fraction(1, 7)):
    """Left/right reconstruction errors at the face x = 0 for a random degree-``deg`` polynomial."""
    rng = np.random.default_rng(seed)
    coefs = [Fraction(int(c)) / 7 for c in rng.integers(-20, 20, size=deg + 1)]
    if coefs[-1] == 0:
        coefs[-1] = Fraction(3, 7)
    edges = [h * m for m in range(-3, 4)]            # cells -3..2 around the face x = 0
    avg = [torch.tensor([float(v)], dtype=torch.float64) for v in _poly_cell_averages(coefs, edges)]
    exact = float(_poly_value(coefs, Fraction(0)))
    # cells: avg[0] = Q_{-3}, ..., avg[5] = Q_{2}; the face is i-1/2 with i = 0
    left = float(O.weno5(avg[0], avg[1], avg[2], avg[3], avg[4], linear=linear))
    right = float(O.weno5(avg[5], avg[4], avg[3], avg[2], avg[1], linear=linear))
    scale = max(abs(float(c)) for c in coefs)
    return abs(left - exact) / scale, abs(right - exact) / scale


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_linear_weno_exact_up_to_degree_4(deg):
    for seed in range(4):
        el, er = _face_errors(deg, linear=True, seed=seed)
        assert el < 1e-13 and er < 1e-13


def test_linear_weno_not_exact_at_degree_5():
    el, er = _face_errors(5, linear=True, seed=1, h=Fraction(1))
    assert el > 1e-6 and er > 1e-6


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_nonlinear_weno_exact_up_to_degree_2(deg):
    for seed in range(4):
        el, er = _face_errors(deg, linear=False, seed=seed)
        assert el < 1e-12 and er < 1e-12


def _quadratic_from_averages(avgs, cells):
    """Coefficients (c0, c1, c2) of the quadratic whose cell averages over ``cells`` equal ``avgs``."""
    A = np.zeros((3, 3))
    for r, (a, b) in enumerate(cells):
        for k in range(3):
            A[r, k] = (b ** (k + 1) - a ** (k + 1)) / (k + 1) / (b - a)
    return np.linalg.solve(A, np.asarray(avgs, dtype=np.float64))


def test_smoothness_indicators_equal_jiang_shu_integrals():
    """beta_k = sum_{l=1,2} int_cell h^(2l-1) (p_k^(l))^2 dx with h = 1, target cell [-1, 0]."""
    rng = np.random.default_rng(7)
    cells = [(-3.0, -2.0), (-2.0, -1.0), (-1.0, 0.0), (0.0, 1.0), (1.0, 2.0)]
    for _ in range(20):
        v = rng.standard_normal(5)
        betas = O.weno5_smoothness(*[torch.tensor([x], dtype=torch.float64) for x in v])
        subs = O.weno5_substencils(*[torch.tensor([x], dtype=torch.float64) for x in v])
        for k in range(3):
            c = _quadratic_from_averages(v[k:k + 3], cells[k:k + 3])
            beta = 0.0
            for l in (1, 2):
                d = P.polyder(c, l)
                integ = P.polyint(P.polymul(d, d))
                beta += P.polyval(0.0, integ) - P.polyval(-1.0, integ)
            assert abs(float(betas[k]) - beta) <= 1e-12 * max(1.0, abs(beta))
            # the candidate value is that quadratic at the face x = 0
            assert abs(float(subs[k]) - P.polyval(0.0, c)) < 1e-12


def _sine_face_error(n):
    h = 1.0 / n
    edges = np.arange(-3, n + 4) * h
    avg = (np.cos(2 * np.pi * edges[:-1]) - np.cos(2 * np.pi * edges[1:])) / (2 * np.pi * h)
    v = torch.tensor(avg, dtype=torch.float64)         # padded by 3 on both sides
    left, right = O.reconstruct_faces(v, 0, n, 1e-6, False)
    exact = torch.tensor(np.sin(2 * np.pi * np.arange(n + 1) * h), dtype=torch.float64)
    return float(torch.max(torch.abs(left - exact))), float(torch.max(torch.abs(right - exact)))


def test_weno5_fifth_order_on_smooth_data():
    ns = [32, 64, 128, 256]
    errs = [_sine_face_error(n) for n in ns]
    for side in (0, 1):
        orders = [math.log2(errs[i][side] / errs[i + 1][side]) for i in range(len(ns) - 1)]
        assert min(orders[1:]) >= 4.7, orders


def test_weno5_non_oscillatory_at_a_step():
    v = torch.tensor([0.0] * 8 + [1.0] * 8, dtype=torch.float64)
    left, right = O.reconstruct_faces(v, 0, 10, 1e-6, False)
    for s in (left, right):
        assert float(s.min()) > -1e-6 and float(s.max()) < 1.0 + 1e-6
    lin_l, _ = O.reconstruct_faces(v, 0, 10, 1e-6, True)
    assert float(lin_l.max()) > 1.0 + 1e-3 or float(lin_l.min()) < -1e-3   # linear scheme overshoots


def test_weno5_odd_symmetry_is_exact():
    rng = np.random.default_rng(3)
    v = torch.tensor(rng.standard_normal((5, 1000)), dtype=torch.float64)
    a = O.weno5(*v)
    b = O.weno5(*(-v))
    assert torch.equal(a, -b)


def test_weno5_translation_invariance():
    rng = np.random.default_rng(4)
    v = torch.tensor(rng.standard_normal((5, 1000)), dtype=torch.float64)
    a = O.weno5(*v)
    b = O.weno5(*(v + 3.0))
    assert float(torch.max(torch.abs(b - 3.0 - a))) < 1e-13


def test_weno5_uniform_data_gives_linear_weights():
    v = torch.full((5,), 2.5, dtype=torch.float64)
    w = O.weno5_weights(*v, eps=1e-6)
    assert all(abs(float(a) - b) < 1e-15 for a, b in zip(w, O.LINEAR_WEIGHTS))
