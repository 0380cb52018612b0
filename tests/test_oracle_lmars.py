"""Pins of the oracle's LMARS flux (Sec. 4.1, eqs. rp and ru): consistency with
the physical Euler flux, contact and wall behaviour, mirror symmetry, and
agreement to second order in jump size with an exact Riemann solver."""
import math

import numpy as np
import pytest
import torch

from oracle import snap_oracle as O

GAMMA = 1.4
T = lambda x: torch.tensor(np.atleast_1d(np.asarray(x, dtype=np.float64)))  # noqa: E731


def state(rho, u, v, w, p, pbar=0.0, q=()):
    return {"rho": T(rho), "u": T(u), "v": T(v), "w": T(w), "p": T(p), "pp": T(p - pbar),
            "q": [T(x) for x in q]}


def physical_flux(S, normal, gamma):
    """Euler flux of Sec. 2 along ``normal`` with pressure replaced by the perturbation pressure."""
    vel = [S["u"], S["v"], S["w"]]
    un = vel[normal]
    E = S["p"] / (gamma - 1.0) + 0.5 * S["rho"] * (S["u"] ** 2 + S["v"] ** 2 + S["w"] ** 2)
    f = [S["rho"] * un]
    for m in range(3):
        f.append(S["rho"] * vel[m] * un + (S["pp"] if m == normal else 0.0))
    f.append((E + S["p"]) * un)
    f += [S["rho"] * qt * un for qt in S["q"]]
    return f


@pytest.mark.parametrize("normal", [0, 1, 2])
def test_identical_states_give_physical_flux(normal):
    S = state(1.1, 3.0, -2.0, 1.5, 9.5e4, pbar=9.4e4, q=(0.01, 0.002))
    flux, pstar, ustar = O.lmars_flux(S, S, normal, GAMMA, 2)
    ref = physical_flux(S, normal, GAMMA)
    for a, b in zip(flux, ref):
        assert abs(float(a) - float(b)) <= 1e-12 * max(1.0, abs(float(b)))


def test_contact_is_pure_upwind():
    for u in (2.0, -2.0):
        L = state(1.3, u, 5.0, 0.0, 1e5, q=(0.1,))
        R = state(0.9, u, -4.0, 0.0, 1e5, q=(0.3,))
        flux, pstar, ustar = O.lmars_flux(L, R, 0, GAMMA, 1)
        up = L if u > 0 else R
        assert float(ustar) == u and float(pstar) == 1e5
        assert abs(float(flux[0]) - float(up["rho"]) * u) < 1e-12
        assert abs(float(flux[2]) - float(up["rho"] * up["v"]) * u) < 1e-12
        assert abs(float(flux[5]) - float(up["rho"] * up["q"][0]) * u) < 1e-12


def test_wall_mirror_gives_zero_mass_energy_and_tracer_flux():
    R = state(1.2, -3.0, 2.0, 1.0, 1.01e5, pbar=1.0e5, q=(0.05,))
    L = dict(R)
    L["u"] = -R["u"]
    flux, pstar, ustar = O.lmars_flux(L, R, 0, GAMMA, 1)
    assert float(ustar) == 0.0
    for m in (0, 2, 3, 4, 5):
        assert float(flux[m]) == 0.0
    c = math.sqrt(GAMMA * 1.01e5 / 1.2)
    assert abs(float(flux[1]) - (1e3 - 1.2 * c * (-3.0))) < 1e-9


def test_mirror_swap_flips_ustar():
    rng = np.random.default_rng(1)
    for _ in range(10):
        a = state(1 + rng.random(), rng.normal(), rng.normal(), rng.normal(), 1e5 + 100 * rng.normal())
        b = state(1 + rng.random(), rng.normal(), rng.normal(), rng.normal(), 1e5 + 100 * rng.normal())
        f1, p1, u1 = O.lmars_flux(a, b, 0, GAMMA, 0)
        am, bm = dict(a), dict(b)
        am["u"], bm["u"] = -a["u"], -b["u"]
        f2, p2, u2 = O.lmars_flux(bm, am, 0, GAMMA, 0)
        assert abs(float(u1) + float(u2)) < 1e-14 and abs(float(p1) - float(p2)) < 1e-9
        assert abs(float(f1[0]) + float(f2[0])) < 1e-12


def test_zero_ustar_takes_mean_of_sides():
    L = state(1.0, 0.0, 1.0, 0.0, 1e5)
    R = state(2.0, 0.0, 3.0, 0.0, 1e5)
    flux, _, ustar = O.lmars_flux(L, R, 0, GAMMA, 0)
    assert float(ustar) == 0.0 and float(flux[0]) == 0.0


# --- exact Riemann solver (pressure-function method for the ideal-gas Euler equations) ---

def _f_side(p, rho, pk, gamma):
    c = math.sqrt(gamma * pk / rho)
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def exact_star(rl, ul, pl, rr, ur, pr, gamma):
    f = lambda p: _f_side(p, rl, pl, gamma) + _f_side(p, rr, pr, gamma) + (ur - ul)  # noqa: E731
    lo, hi = 1e-8 * min(pl, pr), 10.0 * max(pl, pr)
    for _ in range(200):                      # bisection: f is increasing in p
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    u = 0.5 * (ul + ur) + 0.5 * (_f_side(p, rr, pr, gamma) - _f_side(p, rl, pl, gamma))
    return p, u


def test_lmars_star_state_matches_exact_riemann_to_second_order():
    rng = np.random.default_rng(11)
    r0, u0, p0 = 1.2, 4.0, 1.0e5
    c0 = math.sqrt(GAMMA * p0 / r0)
    dirs = rng.standard_normal((8, 6))
    for d in dirs:
        errs = []
        for amp in (1e-2, 5e-3, 2.5e-3):
            rl, rr = r0 * (1 + amp * d[0]), r0 * (1 + amp * d[1])
            ul, ur = u0 + amp * c0 * d[2], u0 + amp * c0 * d[3]
            pl, pr = p0 * (1 + amp * d[4]), p0 * (1 + amp * d[5])
            pe, ue = exact_star(rl, ul, pl, rr, ur, pr, GAMMA)
            _, ps, us = O.lmars_flux(state(rl, ul, 0, 0, pl), state(rr, ur, 0, 0, pr), 0, GAMMA, 0)
            errs.append((abs(float(ps) - pe) / p0, abs(float(us) - ue) / c0))
            # first-order agreement: error well below the jump itself
            assert errs[-1][0] < 0.05 * amp and errs[-1][1] < 0.05 * amp
        for k in (0, 1):
            ratio = errs[0][k] / errs[1][k], errs[1][k] / errs[2][k]
            # second order or better; a wrong sign or factor leaves a first-order error (ratio 2)
            assert all(r > 3.0 for r in ratio), (k, ratio, errs)
