"""Pins of the oracle's saturation adjustment (App. D: phase equilibrium of
each vapour with its cloud at constant volume and total energy).

* the paper's own iteration, written here in molar mixing ratios (the
  projected transfer of eq. dxf with the isochoric alpha, limited to keep
  every substance non-negative, then temperature and pressure updated),
  reaches the same state as the oracle's bisection on the equilibrium
  condition;
* the result is in equilibrium: where cloud remains, the vapour's partial
  pressure rho_v (R_d / eps) T equals p*(T); where none remains it is below
  p*(T) (T computed here from the conserved energy and the species' heat
  capacities);
* density, momentum and total energy are untouched; each pair's total is
  conserved; condensation warms and evaporation cools; adjusting twice
  changes nothing; a state unsaturated without cloud is left as it is;
* its derivative (the implicit-function form of saturation_adjust_diff)
  matches central differences of the bisection, returns the cotangent of a
  pair's total unchanged, and matches the closed form of a pair whose
  transfer leaves the temperature alone.
"""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as W
from oracle import snap_oracle as O

BASE = W.jovian_base()
RD, GD = BASE.rd, BASE.cp / (BASE.cp - BASE.rd)
CVD = BASE.cp - BASE.rd


def column(nz=48, seed=5):
    """Water and ammonia vapour and cloud over a Jovian-like column: vapour
    supersaturated in some cells and below saturation in others, clouds from
    none to abundant."""
    g, q, adj = W.jovian_satadj_3d(nx=5, ny=4, nz=nz, seed_q=seed)
    return g, q, adj


def temperature_from_energy(g, qi):
    """T = (E - K - sum mu rho) / (c_vd (rho_d + sum sigma rho)), from the
    species' heat capacities and chemical potentials (Sec. 2, eq. energy)."""
    rho = qi[0]
    kin = 0.5 * (qi[1] ** 2 + qi[2] ** 2 + qi[3] ** 2) / rho
    chem = sum(g.tracer_mu[t] * qi[5 + t] for t in range(g.ntracer))
    heat = CVD * (rho - sum(qi[5 + t] for t in range(g.ntracer))
                  + sum(g.tracer_sigma[t] * qi[5 + t] for t in range(g.ntracer)))
    return (qi[4] - kin - chem) / heat


def psat(T, sp):
    t = T / sp.t_ref
    return sp.p_ref * np.exp(sp.beta * (1.0 - 1.0 / t) - sp.delta * np.log(t))


def paper_iteration(g, q, adj, sweeps=60):
    """App. D in molar mixing ratios, isochoric: for each pair in turn, the
    projected transfer dq = (x_i - s/(1-s) g) / (1 + s/(1-s)^2 (beta/t - delta)
    alpha g) with s = p*(T)/p, g the molar ratio of the other gases and
    alpha = (gamma_d - 1)(beta/t - delta - 1) / (1 + sum (x_i + x_ij)(sigma_i - 1)),
    limited to -x_cloud <= dq <= x_vapour; then T from the conserved energy and
    p = R_d T (rho_d + sum rho_v / eps_v). Where p* >= p (s >= 1, which the
    printed formula does not cover: the vapour could only match p* above the
    total pressure) no cloud can remain and all of it evaporates."""
    qi = g.interior(np.array(q, dtype=np.float64))
    eps = np.array(g.tracer_eps)
    vap = [t for t in range(g.ntracer) if g.tracer_kind[t] == W.TRACER_VAPOUR]
    cloud_of = {sp.cloud: sp.vapour for sp in adj.species}
    molar = [eps[t] if g.tracer_kind[t] == W.TRACER_VAPOUR else eps[cloud_of[t]]
             for t in range(g.ntracer)]
    for _ in range(sweeps):
        for sp in adj.species:
            rho = qi[0]
            rho_d = rho - sum(qi[5 + t] for t in range(g.ntracer))
            n = [qi[5 + t] / molar[t] for t in range(g.ntracer)]      # moles x M_d per volume
            ntot = rho_d + sum(n)
            x = [nt / ntot for nt in n]
            xd = rho_d / ntot
            T = temperature_from_energy(g, qi)
            p = RD * T * (rho_d + sum(qi[5 + t] / eps[t] for t in vap))
            s = psat(T, sp) / p
            others = xd + sum(x[t] for t in vap if t != sp.vapour)
            tt = T / sp.t_ref
            lam = sp.beta / tt - sp.delta
            sig = sum((x[sp2.vapour] + x[sp2.cloud]) * (g.tracer_sigma[sp2.vapour] * eps[sp2.vapour] - 1.0)
                      for sp2 in adj.species)
            alpha = (GD - 1.0) * (lam - 1.0) / (1.0 + sig)
            with np.errstate(divide="ignore", invalid="ignore"):
                dq = (x[sp.vapour] - s / (1.0 - s) * others) / (1.0 + s / (1.0 - s) ** 2 * lam * alpha * others)
            dq = np.where(s >= 1.0, -x[sp.cloud], dq)
            dq = np.clip(dq, -x[sp.cloud], x[sp.vapour])
            dm = dq * ntot * molar[sp.vapour]      # mass moved from vapour to cloud
            qi[5 + sp.vapour] = np.maximum(qi[5 + sp.vapour] - dm, 0.0)
            qi[5 + sp.cloud] = np.maximum(qi[5 + sp.cloud] + dm, 0.0)
    return qi


def test_paper_iteration_reaches_the_oracles_equilibrium():
    """Compared where the iteration is defined: its derivative factor
    beta/t - delta - 1 = (L(T) - R_v T) / (R_v T), the latent heat at constant
    volume, must be positive. Deep in the column (ammonia above ~640 K) the
    linear Kirchhoff law drives L(T) below R_v T and the projected transfer
    changes sign; the vapour there is far below saturation and the oracle
    evaporates all cloud, which the equilibrium pin checks."""
    g, q, adj = column()
    a = g.interior(q)
    out = g.interior(O.saturation_adjust(q, g, adj).numpy())
    ref = paper_iteration(g, q, adj)
    T = temperature_from_energy(g, a)
    valid = np.all([sp.beta / (T / sp.t_ref) - sp.delta > 1.0 for sp in adj.species], axis=0)
    assert valid.mean() > 0.5
    for sp in adj.species:
        tot = a[5 + sp.vapour] + a[5 + sp.cloud]
        for t in (sp.vapour, sp.cloud):
            err = np.max(np.abs(out[5 + t] - ref[5 + t])[valid] / tot[valid])
            assert err < 1e-12, (t, err)
    # and the compared cells hold both regimes
    for sp in adj.species:
        cl = out[5 + sp.cloud][valid]
        assert (cl > 0).any() and (cl == 0).any()


def test_result_is_in_phase_equilibrium():
    g, q, adj = column(seed=7)
    out = g.interior(O.saturation_adjust(q, g, adj).numpy())
    T = temperature_from_energy(g, out)
    for sp in adj.species:
        pv = out[5 + sp.vapour] * (RD / g.tracer_eps[sp.vapour]) * T
        ps = psat(T, sp)
        cloudy = out[5 + sp.cloud] > 0
        assert np.max(np.abs(pv[cloudy] - ps[cloudy]) / ps[cloudy]) < 1e-12
        assert np.all(pv[~cloudy] <= ps[~cloudy] * (1 + 1e-12))


def test_conserves_and_heats_by_the_sign_of_the_transfer():
    g, q, adj = column(seed=9)
    a = g.interior(q)
    b = g.interior(O.saturation_adjust(q, g, adj).numpy())
    assert np.array_equal(a[:5], b[:5])
    for sp in adj.species:
        t0 = a[5 + sp.vapour] + a[5 + sp.cloud]
        t1 = b[5 + sp.vapour] + b[5 + sp.cloud]
        assert np.max(np.abs(t1 - t0) / np.where(t0 > 0, t0, 1.0)) < 1e-15
        assert np.all(b[5 + sp.vapour] >= 0) and np.all(b[5 + sp.cloud] >= 0)
    # one species at a time (the other pair removed): condensing warms,
    # evaporating cools, where the latent heat at constant volume
    # L(T) - R_v T is positive (beta/t - delta > 1; the linear Kirchhoff law
    # takes ammonia's below zero above ~600 K, deep in the column)
    for sp in adj.species:
        q1 = np.array(q)
        for other in adj.species:
            if other is not sp:
                g.interior(q1)[5 + other.vapour] = 0.0
                g.interior(q1)[5 + other.cloud] = 0.0
        a1 = g.interior(q1)
        b1 = g.interior(O.saturation_adjust(q1, g, adj).numpy())
        T0 = temperature_from_energy(g, a1)
        dT = temperature_from_energy(g, b1) - T0
        grow = b1[5 + sp.cloud] - a1[5 + sp.cloud]
        ok = sp.beta / (T0 / sp.t_ref) - sp.delta > 1.0
        assert (grow[ok] > 0).any() and (grow[ok] < 0).any()
        assert np.all(dT[ok & (grow > 0)] > 0) and np.all(dT[ok & (grow < 0)] < 0)


def test_adjusting_twice_changes_nothing():
    g, q, adj = column(seed=11)
    once = O.saturation_adjust(q, g, adj)
    twice = O.saturation_adjust(once, g, adj)
    a, b = g.interior(once.numpy()), g.interior(twice.numpy())
    for sp in adj.species:
        tot = a[5 + sp.vapour] + a[5 + sp.cloud]
        assert np.max(np.abs(b[5 + sp.cloud] - a[5 + sp.cloud]) / np.where(tot > 0, tot, 1.0)) < 1e-14


def test_unsaturated_without_cloud_is_unchanged():
    g, q, adj = column(seed=13)
    qi = g.interior(q)
    for sp in adj.species:
        qi[5 + sp.vapour] *= 1e-4          # far below saturation everywhere
        qi[5 + sp.cloud] = 0.0
    out = O.saturation_adjust(q, g, adj).numpy()
    assert np.array_equal(g.interior(out), g.interior(q))


# ---------------------------------------------------------------------------
# The derivative of the adjustment (saturation_adjust_diff / _adjoint): pinned
# by central differences of the bisection itself, by the conservation of each
# pair's total and by the closed form of a pair whose transfer leaves T alone.
# ---------------------------------------------------------------------------

def _tracer_cotangent(g, seed):
    """A seeded cotangent on the tracers only: the five dynamic fields pass
    through the adjustment unchanged, and E (~5e7) would drown the transfer's
    part of a finite difference in rounding."""
    qb = W.seeded_normal(g.interior_shape, seed)
    qb[:5] = 0.0
    return qb


@pytest.mark.parametrize("seed", [5, 8])
def test_adjoint_matches_central_differences(seed):
    g, q, adj = column(nz=32, seed=seed)
    qi = g.interior(q)
    qb = _tracer_cotangent(g, seed + 40)
    gb = O.saturation_adjust_adjoint(q, g, adj, qb).numpy()
    rng = np.random.default_rng(seed)
    h = 1e-6
    for _ in range(3):
        d = rng.normal(size=qi.shape) * np.abs(qi)     # relative perturbation of every field
        qp, qm = q.copy(), q.copy()
        g.interior(qp)[...] += h * d
        g.interior(qm)[...] -= h * d
        sp = g.interior(O.saturation_adjust(qp, g, adj).numpy())
        sm = g.interior(O.saturation_adjust(qm, g, adj).numpy())
        # the transfer's part: (S(q + h d) - S(q - h d)) / 2h minus d itself
        fd = float(np.sum(qb * ((sp - sm) / (2 * h) - d)))
        ad = float(np.sum(gb * d) - np.sum(qb * d))
        print(f"seed {seed}: fd {fd:.10e} ad {ad:.10e}")
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


def test_adjoint_keeps_each_pairs_total():
    """rho_v + rho_c of every pair leaves the adjustment unchanged, so a
    cotangent of 1 on both members of a pair comes back as itself."""
    g, q, adj = column(nz=24, seed=11)
    qb = np.zeros(g.interior_shape)
    for sp in adj.species[:1]:
        qb[5 + sp.vapour] = 1.0
        qb[5 + sp.cloud] = 1.0
    gb = O.saturation_adjust_adjoint(q, g, adj, qb).numpy()
    np.testing.assert_allclose(gb, qb, rtol=0, atol=1e-12)


def test_adjoint_closed_form_when_the_transfer_leaves_T_alone():
    """With cloud and vapour of equal heat capacity and chemical potential the
    transfer does not change T, so where cloud remains X = rho_v - p*(T) /
    (R_v T) with T(q) from the energy alone. The cotangent of the cloud is
    then d(rho_c + X)/dq: 1 on rho_c, 1 on rho_v, and -d/dT[p*/(R_v T)] dT/dq
    on the fields T depends on, with d/dT[p*/(R_v T)] = p* (lam - 1) / (R_v T^2),
    lam = beta t_ref / T - delta (the logarithmic slope of p*). The oracle
    evaluates dG/dT at the remaining vapour rho_v - X*, which carries the
    rounding of that difference where most of the vapour condensed (up to
    ~2e-7 of it here); the closed form uses p*(T) / (R_v T) instead, hence
    the 1e-6 bar."""
    g, q, adj = column(nz=32, seed=7)
    sp = adj.species[0]
    sig, mu = list(g.tracer_sigma), list(g.tracer_mu)
    sig[sp.cloud], mu[sp.cloud] = sig[sp.vapour], mu[sp.vapour]
    g = g.copy(tracer_sigma=tuple(sig), tracer_mu=tuple(mu))
    adj1 = dataclasses.replace(adj, species=(sp,))
    qb = np.zeros(g.interior_shape)
    qb[5 + sp.cloud] = 1.0
    gb = O.saturation_adjust_adjoint(q, g, adj1, qb).numpy()
    qi = g.interior(q)
    out = g.interior(O.saturation_adjust(q, g, adj1).numpy())
    T = temperature_from_energy(g, qi)
    rv = RD / g.tracer_eps[sp.vapour]
    lam = sp.beta * sp.t_ref / T - sp.delta
    dxdt = -psat(T, sp) * (lam - 1.0) / (rv * T * T)     # dX/dT
    rho = qi[0]
    heat = CVD * (rho - sum(qi[5 + t] for t in range(g.ntracer))
                  + sum(sig[t] * qi[5 + t] for t in range(g.ntracer)))
    wet = out[5 + sp.cloud] > 0.0
    assert wet.sum() > 20 and (~wet).sum() > 20
    # dT/dE = 1 / heat, dT/d(rho u) = -u / heat
    np.testing.assert_allclose(gb[4][wet], (dxdt / heat)[wet], rtol=1e-6)
    np.testing.assert_allclose(gb[1][wet], (-dxdt * qi[1] / rho / heat)[wet], rtol=1e-6)
    # where the cloud evaporated entirely the output cloud is 0 whatever q is
    assert np.all(gb[:, ~wet] == 0.0)
