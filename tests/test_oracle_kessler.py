"""Pins of the oracle's Kessler microphysics (Sec. 3) and saturation vapour
pressure (App. D).

* each process alone has a closed-form backward-Euler step (condensation and
  autoconversion: linear; accretion and evaporation: the smaller root of a
  quadratic), which the oracle's Newton iteration must reproduce;
* with every process on, the step conserves each species' total mixing ratio
  and satisfies its defining equation X = X^n + dt Phi(X);
* the saturation vapour pressure solves the Clausius-Clapeyron relation
  d ln p* / dT = L(T) / (R T^2) with the Kirchhoff latent heat;
* moving mass from vapour to cloud at constant total density and energy
  changes the mixture's temperature by the paper's constant-volume jump
  dT = d_rho (L(T) - R T) / (heat capacity after) (Sec. 2, eq. phase);
* the derivative of the step that autograd takes through the oracle (the
  reference of the GPU adjoint) agrees with central differences of the step.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import snap_oracle as O

F64 = torch.float64
RV = W.RGAS / 18.015e-3                     # water vapour gas constant
LREF, TREF, PREF = 2.501e6, 273.16, 611.7
CPV, CL = 1847.0, 4184.0
BETA, DELTA = W.clausius_clapeyron(LREF, CL - CPV, RV, TREF)


def species(k1=0.0, k2=0.0, k3=0.0, k4=0.0):
    return W.KesslerSpecies(vapour=0, cloud=1, precip=2, k1=k1, k2=k2, k3=k3, k4=k4,
                            p_ref=PREF, t_ref=TREF, beta=BETA, delta=DELTA, eps=18.015 / 28.96)


def mix(n, seed):
    rng = np.random.default_rng(seed)
    qv = torch.as_tensor(10.0 ** rng.uniform(-4, -2, n), dtype=F64)
    qc = torch.as_tensor(10.0 ** rng.uniform(-5, -3, n), dtype=F64)
    qp = torch.as_tensor(10.0 ** rng.uniform(-5, -3, n), dtype=F64)
    qs = torch.as_tensor(10.0 ** rng.uniform(-4, -2, n), dtype=F64)
    return qv, qc, qp, qs


DT = 5.0


def test_condensation_alone_is_linear():
    qv, qc, qp, qs = mix(200, 1)
    sp = species(k1=0.3)
    v, c, p = O.kessler_solve(qv, qc, qp, qs, sp, DT)
    sat = qv > qs
    expect_v = torch.where(sat, (qv + DT * sp.k1 * qs) / (1.0 + DT * sp.k1), qv)
    assert torch.allclose(v, expect_v, rtol=1e-14, atol=0)
    assert torch.allclose(c, qc + (qv - expect_v), rtol=1e-13, atol=1e-20)
    assert torch.equal(p, qp)
    assert bool((v[sat] > qs[sat]).all())          # stays saturated


def test_autoconversion_alone_is_linear():
    qv, qc, qp, qs = mix(200, 2)
    sp = species(k2=1e-3)
    v, c, p = O.kessler_solve(qv, qc, qp, qs, sp, DT)
    assert torch.allclose(c, qc / (1.0 + DT * sp.k2), rtol=1e-14, atol=0)
    assert torch.allclose(p, qp + qc - qc / (1.0 + DT * sp.k2), rtol=1e-14, atol=0)
    assert torch.equal(v, qv)


def test_accretion_alone_is_the_smaller_quadratic_root():
    qv, qc, qp, qs = mix(200, 3)
    # strong enough that the quadratic term matters (dt k3 (q_c + q_p) up to 0.5),
    # below dt k3 (q_c - q_p) = 1, past which the iteration started at X^n
    # heads for the other, unphysical root of the quadratic
    sp = species(k3=50.0)
    v, c, p = O.kessler_solve(qv, qc, qp, qs, sp, DT)
    a = DT * sp.k3
    B = 1.0 + a * (qc + qp)
    x = 2.0 * qc / (B + torch.sqrt(B * B - 4.0 * a * qc))     # smaller root, cancellation-free
    assert torch.allclose(c, x, rtol=1e-13, atol=0)
    assert torch.allclose(p, qp + qc - x, rtol=1e-13, atol=1e-20)


def test_evaporation_alone_is_the_smaller_quadratic_root():
    qv, qc, qp, qs = mix(200, 4)
    sp = species(k4=5e2)
    v, c, p = O.kessler_solve(qv, qc, qp, qs, sp, DT)
    unsat = qv <= qs
    a = DT * sp.k4
    T2 = qv + qp
    B = 1.0 + a * (T2 + qs)
    C = qv + a * T2 * qs
    y = 2.0 * C / (B + torch.sqrt(B * B - 4.0 * a * C))
    assert torch.allclose(v[unsat], y[unsat], rtol=1e-13, atol=0)
    # q_p = (q_v + q_p) - q_v' cancels when most rain evaporates: bound it by the total
    assert float(((p - (T2 - y)).abs() / T2)[unsat].max()) < 1e-14
    assert torch.equal(v[~unsat], qv[~unsat])
    assert bool((v[unsat] <= qs[unsat]).all())       # stays unsaturated


def test_all_processes_conserve_and_satisfy_backward_euler():
    qv, qc, qp, qs = mix(500, 5)
    sp = species(k1=0.3, k2=1e-3, k3=2.2, k4=5e-1)
    v, c, p = O.kessler_solve(qv, qc, qp, qs, sp, DT)
    S0 = qv + qc + qp
    assert torch.max(torch.abs(v + c + p - S0) / S0) < 1e-14
    sat = qv > qs
    X = torch.stack([v, c, p], dim=-1)
    res = X - torch.stack([qv, qc, qp], dim=-1) - DT * O.kessler_rates(v, c, p, qs, sp, sat)
    assert float((res.abs().amax(dim=-1) / S0).max()) < 1e-14
    assert bool((X >= 0).all())


def test_saturation_vapour_pressure_solves_clausius_clapeyron():
    sp = species()
    T = torch.linspace(200.0, 330.0, 27, dtype=F64)
    assert abs(float(O.saturation_vapour_pressure(torch.tensor([TREF], dtype=F64), sp)[0]) - PREF) < 1e-12 * PREF
    h = 1e-3
    dlnp = (torch.log(O.saturation_vapour_pressure(T + h, sp))
            - torch.log(O.saturation_vapour_pressure(T - h, sp))) / (2 * h)
    latent = LREF - (CL - CPV) * (T - TREF)              # Kirchhoff (Sec. 2, eq. latent)
    assert torch.allclose(dlnp, latent / (RV * T * T), rtol=1e-8, atol=0)


def test_constant_volume_phase_change_heats_as_the_paper_states():
    """Condensing d_rho of vapour into cloud at fixed rho and E raises T by
    d_rho (L(T) - R_v T) / C_after, C_after = sum of rho_s c_v,s after."""
    rd, gd = 287.0, 1.4
    cvd = rd / (gd - 1.0)
    eps = 18.015e-3 / (W.RGAS / rd)
    mu_c = -(LREF + (CL - CPV) * TREF)
    g = W.Grid(nx=1, ny=1, nz=1, dx=1.0, dy=1.0, dz=1.0, gamma=gd, grav=0.0, ntracer=2,
               eos=W.EOS_MIXTURE, tracer_kind=(W.TRACER_VAPOUR, W.TRACER_CONDENSATE),
               tracer_eps=(eps, 1.0), tracer_sigma=((CPV - RV) / cvd, CL / cvd), tracer_mu=(0.0, mu_c))
    g.rhobar_cell, g.pbar_cell, g.rhobar_face, g.pbar_face = W.uniform_references(1, 1.0, 1e5)
    rho_d, rho_v, rho_c, T = 1.1, 0.012, 0.0004, 290.0
    E = (rho_d * cvd + rho_v * (CPV - RV) + rho_c * CL) * T + mu_c * rho_c

    def state(rv, rc):
        q = np.zeros(g.shape)
        qi = g.interior(q)
        qi[0], qi[4], qi[5], qi[6] = rho_d + rho_v + rho_c, E, rv, rc
        return q

    t0 = float(g.interior(O.temperature(state(rho_v, rho_c), g, rd).unsqueeze(0).numpy())[0].item())
    assert abs(t0 - T) < 1e-11 * T
    for d in (1e-4, 1e-3, 5e-3):
        t1 = float(g.interior(O.temperature(state(rho_v - d, rho_c + d), g, rd).unsqueeze(0).numpy())[0].item())
        c_after = rho_d * cvd + (rho_v - d) * (CPV - RV) + (rho_c + d) * CL
        latent = LREF - (CL - CPV) * (T - TREF)
        expect = d * (latent - RV * T) / c_after
        assert abs((t1 - t0) - expect) < 1e-9 * abs(expect), (d, t1 - t0, expect)


def test_kessler_step_keeps_density_momentum_and_energy():
    rd = 3614.98
    base = W.jovian_base()
    table = W.condensable_species(base.cp - base.rd, W.JOVIAN_MU)
    g, _ = W.dry_grid(6, 5, 8, 6e3, 5e3, 8e3)
    g = W.with_mixture(g, [table[0], table[2], table[2]])
    q = W.random_smooth_state(g, seed=9, amp_q=3e-3)
    sp = W.KesslerSpecies(vapour=0, cloud=1, precip=2, k1=0.3, k2=1e-3, k3=2.2, k4=0.5,
                          p_ref=PREF, t_ref=TREF, beta=BETA, delta=DELTA, eps=g.tracer_eps[0])
    out = O.kessler_step(q, g, 5.0, W.Kessler(species=(sp,), rd=rd)).numpy()
    a, b = g.interior(q), g.interior(out)
    assert np.array_equal(a[:5], b[:5])
    tot0 = a[5] + a[6] + a[7]
    assert np.max(np.abs(b[5] + b[6] + b[7] - tot0) / tot0) < 1e-14
    assert not np.array_equal(a[5:], b[5:])


def test_kessler_step_autograd_matches_central_differences():
    """<J^T w, v> by autograd through the oracle's step against <w, J v> by
    Richardson-extrapolated central differences, on the small microphysics
    case of the GPU tests (every field perturbed, scaled to its magnitude)."""
    from tests import cases as C
    c, kes = C.build_kessler_case("kessler_3d_ragged_9x7x5", dict(C.KESSLER_SPECS)["kessler_3d_ragged_9x7x5"])
    g = c.grid
    q0 = torch.as_tensor(c.q)
    rng = np.random.default_rng(77)
    qi = g.interior(c.q)
    scale = np.abs(qi).reshape(g.nvar, -1).max(axis=1)[:, None, None, None]
    v = rng.standard_normal(qi.shape) * scale
    w = rng.standard_normal(qi.shape)

    def step(q):
        return g.interior(O.kessler_step(q, g, c.dt, kes))

    qg = q0.clone().requires_grad_(True)
    (step(qg) * torch.as_tensor(w)).sum().backward()
    lhs = float((g.interior(qg.grad).numpy() * v).sum())

    def shifted(h):
        qq = c.q.copy()
        g.interior(qq)[...] += h * v
        return step(torch.as_tensor(qq)).numpy()

    def central(h):
        return (shifted(h) - shifted(-h)) / (2.0 * h)

    h = 1e-7
    jv = (4.0 * central(0.5 * h) - central(h)) / 3.0
    rhs = float((w * jv).sum())
    assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), abs(rhs)), (lhs, rhs)
