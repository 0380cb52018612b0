"""Pins of the oracle's thermodynamics (App. B) and of its discrete adjoint.

* The passive-tracer cons -> prim equals the general mixture formula of
  App. B (eq. p2) in its stated special case (no clouds, sigma_v,i = 1/eps_i).
* prim -> cons -> prim round trip.
* The autograd adjoint satisfies the dot-product identity against central
  finite differences of the forward oracle.
"""
import numpy as np
import torch

import workloads as W
from oracle import snap_oracle as O


def general_mixture_pressure(E, K, A, q_vap, q_cld, sigma_v, sigma_c, eps, gamma_d):
    """Pressure from internal energy for a mixture (App. B, eq. p2)."""
    num = 1.0 + sum(qi * (1.0 / ei - 1.0) for qi, ei in zip(q_vap, eps)) - sum(q_cld)
    den = (1.0 + sum(qi * (si - 1.0) for qi, si in zip(q_vap, sigma_v))
           + sum(qc * (sc - 1.0) for qc, sc in zip(q_cld, sigma_c)))
    return (gamma_d - 1.0) * num / den * (E - K - A)


def test_passive_reduction_equals_general_mixture_formula():
    g, q = W.jovian_3d(nx=6, ny=5, nz=12, dxy=5.5e3, lz=400e3)
    prim = O.cons_to_prim(torch.as_tensor(q), g)
    qi = g.interior(q)
    isl = (slice(3, 3 + g.nz), slice(3, 3 + g.ny), slice(3, 3 + g.nx))
    rho = qi[0]
    u, v, w = qi[1] / rho, qi[2] / rho, qi[3] / rho
    K = 0.5 * rho * (u * u + v * v + w * w)
    eps = [18.0 / 2.3, 17.0 / 2.3]                    # molecular weight ratios of the vapours
    qv = [qi[5] / rho, qi[6] / rho]
    qc = [qi[7] / rho, qi[8] / rho]
    p_gen = general_mixture_pressure(qi[4], K, 0.0, qv, qc, [1 / e for e in eps], [1.0, 1.0], eps, g.gamma)
    p_or = prim["p"][isl].numpy()
    assert np.max(np.abs(p_or - p_gen) / p_gen) < 1e-13
    assert np.max(qv[0]) > 1e-4                       # tracers are present


def test_prim_cons_round_trip():
    g = W.Grid(nx=8, ny=6, nz=5, dx=1.0, dy=1.0, dz=1.0, grav=0.0, ntracer=2, bc=(0, 0, 0))
    g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.uniform_references(5, 1.0, 1.0e5)
    rng = np.random.default_rng(2)
    shp = (5, 6, 8)
    rho = 1.0 + 0.1 * rng.random(shp)
    u, v, w = rng.normal(size=shp), rng.normal(size=shp), rng.normal(size=shp)
    p = 1e5 * (1 + 0.01 * rng.random(shp))
    tr = [0.01 * rng.random(shp), 0.02 * rng.random(shp)]
    q = W.state_from_primitives(g, rho, u, v, w, p, tr)
    prim = O.cons_to_prim(torch.as_tensor(q), g)
    isl = (slice(3, 8), slice(3, 9), slice(3, 11))
    for name, ref in (("rho", rho), ("u", u), ("v", v), ("w", w), ("p", p)):
        got = prim[name][isl].numpy()
        assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    for t in range(2):
        assert np.max(np.abs(prim["q"][t][isl].numpy() - tr[t])) < 1e-16


def _scaled_direction(g, q, seed):
    qi = g.interior(q)
    scale = np.array([np.max(np.abs(qi[m])) for m in range(g.nvar)])
    d = W.seeded_normal(g.interior_shape, seed)
    return d * scale[:, None, None, None]


def _dot_product_check(g, q, fwd, adj, seed, h=1e-7):
    """<J v, w> by Richardson-extrapolated central differences against <v, J^T w>.

    The Jiang-Shu weights are strongly curved wherever a stencil's pressure
    differences are small compared with the perturbation, so a plain central
    difference needs h^2 extrapolated away to reach 1e-6 relative agreement.
    """
    v = _scaled_direction(g, q, seed)
    wv = W.seeded_normal(g.interior_shape, seed + 100)

    def shifted(s):
        qq = q.copy()
        g.interior(qq)[...] += s * v
        return qq

    def central(hh):
        return (fwd(shifted(hh)) - fwd(shifted(-hh))) / (2 * hh)

    jv = (4.0 * central(0.5 * h) - central(h)) / 3.0
    lhs = float(np.sum(jv * wv))
    rhs = float(np.sum(v * adj(q, wv)))
    return lhs, rhs


def test_rhs_adjoint_dot_product_against_finite_differences():
    g = W.Grid(nx=10, ny=8, nz=9, dx=100.0, dy=90.0, dz=80.0, ntracer=1)
    base = W.DryIsentropic()
    g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.reference_profiles(base, 9, 80.0, 9.81)
    q = W.random_smooth_state(g, seed=3)
    fwd = lambda qq: O.rhs(qq, g).numpy()                              # noqa: E731
    adj = lambda qq, r: O.rhs_adjoint(qq, g, r).numpy()                # noqa: E731
    for seed in (1, 2, 3):
        lhs, rhs = _dot_product_check(g, q, fwd, adj, seed)
        assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)


def test_rk3_adjoint_dot_product_against_finite_differences():
    # a developed flow: a bubble state right after launch has p' at round-off,
    # where any finite step in E crosses the sqrt(eps) scale of the weights
    g, _ = W.bubble_2d(nx=16, nz=16)
    q = W.random_smooth_state(g, seed=9)
    dt = 0.5 * O.cfl_dt(q, g, 0.9)
    fwd = lambda qq: g.interior(O.rk3_step(qq, g, dt).numpy())          # noqa: E731
    adj = lambda qq, r: O.rk3_step_adjoint(qq, g, dt, r).numpy()        # noqa: E731
    for seed in (4, 5):
        lhs, rhs = _dot_product_check(g, q, fwd, adj, seed)
        assert abs(lhs - rhs) <= 1e-6 * abs(rhs), (lhs, rhs)
