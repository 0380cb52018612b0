"""Pins of the oracle's HLLC flux (the Riemann solver the paper compares LMARS
with): consistency with the physical Euler flux, exact resolution of an
isolated contact and of a shear wave, upwinding of supersonic states, the
integral conservation identity of its star states, second-order agreement of
its star state with an exact Riemann solver for weak jumps, and a right-hand
side that keeps a free stream and conserves."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import snap_oracle as O
from tests.test_oracle_lmars import GAMMA, exact_star, physical_flux, state


def close(a, b, tol=1e-12):
    return abs(float(a) - float(b)) <= tol * max(1.0, abs(float(b)))


@pytest.mark.parametrize("normal", [0, 1, 2])
def test_identical_states_give_physical_flux(normal):
    S = state(1.1, 3.0, -2.0, 1.5, 9.5e4, pbar=9.4e4, q=(0.01, 0.002))
    flux, _, _ = O.hllc_flux(S, S, normal, GAMMA, 2)
    for a, b in zip(flux, physical_flux(S, normal, GAMMA)):
        assert close(a, b)


@pytest.mark.parametrize("u", [35.0, -35.0, 0.0])
def test_isolated_contact_is_resolved_exactly(u):
    """Equal pressure and normal velocity, different density, tangential
    velocity and tracer: the flux is the upwind side's physical flux (for
    u = 0: pressure only)."""
    L = state(1.3, u, 5.0, -1.0, 1e5, pbar=0.99e5, q=(0.1,))
    R = state(0.9, u, -4.0, 2.0, 1e5, pbar=0.99e5, q=(0.3,))
    flux, _, ss = O.hllc_flux(L, R, 0, GAMMA, 1)
    assert close(ss, u, 1e-13)
    ref = physical_flux(L if u >= 0 else R, 0, GAMMA)
    for m, (a, b) in enumerate(zip(flux, ref)):
        assert close(a, b, 1e-11), (m, float(a), float(b))


def test_supersonic_states_are_upwinded():
    for u, side in ((900.0, "L"), (-900.0, "R")):
        L = state(1.2, u, 1.0, 0.0, 1.0e5, q=(0.2,))
        R = state(0.8, u * 1.1, -2.0, 3.0, 0.7e5, q=(0.4,))
        flux, _, _ = O.hllc_flux(L, R, 0, GAMMA, 1)
        ref = physical_flux(L if side == "L" else R, 0, GAMMA)
        for a, b in zip(flux, ref):
            assert close(a, b)


def test_star_states_conserve_across_the_fan():
    """(S_R - S*) U*_R + (S* - S_L) U*_L = S_R U_R - S_L U_L - (F_R - F_L):
    the star states hold exactly what the Riemann fan takes in."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        L = state(1 + rng.random(), 30 * rng.normal(), 10 * rng.normal(), 10 * rng.normal(),
                  1e5 * (1 + 0.2 * rng.random()), q=(rng.random(),))
        R = state(1 + rng.random(), 30 * rng.normal(), 10 * rng.normal(), 10 * rng.normal(),
                  1e5 * (1 + 0.2 * rng.random()), q=(rng.random(),))
        for normal in (0, 1, 2):
            SL, SR, Ss = O.hllc_wave_speeds(L, R, normal, GAMMA)
            sL = O.hllc_star(L, SL, Ss, normal, GAMMA)
            sR = O.hllc_star(R, SR, Ss, normal, GAMMA)
            UL, FL = O._conserved_and_flux(L, normal, GAMMA)
            UR, FR = O._conserved_and_flux(R, normal, GAMMA)
            for m in range(len(UL)):
                lhs = (SR - Ss) * sR[m] + (Ss - SL) * sL[m]
                rhs = SR * UR[m] - SL * UL[m] - (FR[m] - FL[m])
                assert close(lhs, rhs, 1e-10), (normal, m, float(lhs), float(rhs))


def test_star_state_matches_exact_riemann_to_second_order():
    rng = np.random.default_rng(11)
    r0, u0, p0 = 1.2, 4.0, 1.0e5
    c0 = math.sqrt(GAMMA * p0 / r0)
    for d in rng.standard_normal((8, 6)):
        errs = []
        for amp in (1e-2, 5e-3, 2.5e-3):
            rl, rr = r0 * (1 + amp * d[0]), r0 * (1 + amp * d[1])
            ul, ur = u0 + amp * c0 * d[2], u0 + amp * c0 * d[3]
            pl, pr = p0 * (1 + amp * d[4]), p0 * (1 + amp * d[5])
            pe, ue = exact_star(rl, ul, pl, rr, ur, pr, GAMMA)
            _, ps, us = O.hllc_flux(state(rl, ul, 0, 0, pl), state(rr, ur, 0, 0, pr), 0, GAMMA, 0)
            errs.append((abs(float(ps) - pe) / p0, abs(float(us) - ue) / c0))
            assert errs[-1][0] < 0.05 * amp and errs[-1][1] < 0.05 * amp
        for k in (0, 1):
            ratio = errs[0][k] / errs[1][k], errs[1][k] / errs[2][k]
            assert all(r > 3.0 for r in ratio), (k, ratio, errs)


def test_wall_mirror_gives_zero_mass_flux():
    R = state(1.2, -3.0, 2.0, 1.0, 1.01e5, pbar=1.0e5, q=(0.05,))
    L = dict(R)
    L["u"] = -R["u"]
    flux, _, ss = O.hllc_flux(L, R, 0, GAMMA, 1)
    assert float(ss) == 0.0
    SL, _, _ = O.hllc_wave_speeds(L, R, 0, GAMMA)
    U, _ = O._conserved_and_flux(L, 0, GAMMA)
    for m in (0, 2, 3, 4, 5):
        # star-region flux F_L + S_L (U*_L - U_L): rounding of terms of size |S_L U|
        assert abs(float(flux[m])) <= 1e-14 * abs(float(SL) * float(U[m])) + 1e-300, m


def test_hllc_rhs_keeps_free_stream_and_conserves():
    g = W.Grid(nx=12, ny=8, nz=10, dx=10.0, dy=12.0, dz=9.0, grav=0.0, bc=(0, 0, 0), ntracer=2,
               riemann=W.RIEMANN_HLLC)
    g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.uniform_references(10, 1.1, 1.0e5)
    shp = (g.nz, g.ny, g.nx)
    q = W.state_from_primitives(g, np.full(shp, 1.2), 3.0, -2.0, 1.5, 0.9e5,
                                [np.full(shp, 0.01), np.full(shp, 0.02)])
    assert float(O.rhs(q, g).abs().max()) == 0.0
    q = W.random_smooth_state(g, seed=5)
    s0 = O.conservation_sums(q, g)
    qn = O.run(q, g, O.cfl_dt(q, g, 0.9), 5)
    s1 = O.conservation_sums(qn, g)
    scale = np.abs(g.interior(q)).reshape(g.nvar, -1).sum(axis=1)
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s1 - s0) / scale
    # and it is a different solver: the right-hand sides differ
    r_h = O.rhs(q, g).numpy()
    r_l = O.rhs(q, g.copy(riemann=W.RIEMANN_LMARS)).numpy()
    assert np.max(np.abs(r_h[0] - r_l[0])) > 1e-3 * np.max(np.abs(r_l[0]))
