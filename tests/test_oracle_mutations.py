"""Planted mistakes: each test plants one plausible error in the oracle (on the
CPU, via monkeypatch) and checks that a pin of the oracle catches it."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import snap_oracle as O
from tests import test_oracle_lmars as TL
from tests import test_oracle_weno as TW


def test_swapped_linear_weights_break_polynomial_exactness(monkeypatch):
    assert max(TW._face_errors(4, linear=True)) < 1e-13
    monkeypatch.setattr(O, "LINEAR_WEIGHTS", (0.3, 0.6, 0.1))
    assert max(TW._face_errors(3, linear=True)) > 1e-6


def test_wrong_smoothness_coefficient_breaks_jiang_shu_pin(monkeypatch):
    orig = O.weno5_smoothness

    def bad(a, b, c, d, e):
        b0, b1, b2 = orig(a, b, c, d, e)
        return b0 - (1.0 / 12.0) * (a - 2.0 * b + c) ** 2, b1, b2   # 13/12 -> 1
    monkeypatch.setattr(O, "weno5_smoothness", bad)
    with pytest.raises(AssertionError):
        TW.test_smoothness_indicators_equal_jiang_shu_integrals()


def test_wrong_substencil_breaks_fifth_order(monkeypatch):
    orig = O.weno5_substencils

    def bad(a, b, c, d, e):
        q0, q1, q2 = orig(a, b, c, d, e)
        return q0, q1, q2 + 1e-3 * (c - d)          # a small wrong term in one candidate
    monkeypatch.setattr(O, "weno5_substencils", bad)
    with pytest.raises(AssertionError):
        TW.test_weno5_fifth_order_on_smooth_data()


def test_flipped_pressure_term_in_ustar_breaks_riemann_pin(monkeypatch):
    orig = O.lmars_flux

    def bad(L, R, normal, gamma, ntracer):
        L2, R2 = dict(L), dict(R)
        # exchanging only the perturbation pressures flips the sign of the
        # pressure-difference term of u*
        L2["pp"], R2["pp"] = R["pp"], L["pp"]
        return orig(L2, R2, normal, gamma, ntracer)
    monkeypatch.setattr(O, "lmars_flux", bad)
    with pytest.raises(AssertionError):
        TL.test_lmars_star_state_matches_exact_riemann_to_second_order()


def test_swapped_rk3_weights_break_amplification_pin(monkeypatch):
    def bad(rhs_fn, y0, dt):
        y1 = y0 + dt * rhs_fn(y0)
        y2 = 0.25 * y0 + 0.75 * (y1 + dt * rhs_fn(y1))
        return (1.0 / 3.0) * y0 + (2.0 / 3.0) * (y2 + dt * rhs_fn(y2))
    monkeypatch.setattr(O, "rk3", bad)
    from tests import test_oracle_rk3 as TR
    with pytest.raises(AssertionError):
        TR.test_amplification_polynomial_real()


def test_unsigned_wall_mirror_breaks_mass_conservation(monkeypatch):
    orig = O.fill_ghosts

    def bad(q, grid):
        qf = orig(q, grid).clone()
        G, nz = O.G, grid.nz
        for k in list(range(G)) + list(range(G + nz, 2 * G + nz)):
            qf[3, k] = -qf[3, k]            # undo the sign flip of the wall-normal momentum
        return qf
    g, q = W.bubble_2d(nx=16, nz=16)
    g.interior(q)[3] += 0.3 * g.interior(q)[0]        # flow towards the walls
    s0 = O.conservation_sums(q, g)[0]
    good = abs(O.conservation_sums(O.rk3_step(q, g, 0.3), g)[0] - s0) / s0
    monkeypatch.setattr(O, "fill_ghosts", bad)
    planted = abs(O.conservation_sums(O.rk3_step(q, g, 0.3), g)[0] - s0) / s0
    assert good < 1e-14 and planted > 1e-6, (good, planted)


def test_dropped_kinetic_energy_breaks_round_trip(monkeypatch):
    orig = O.cons_to_prim

    def bad(q, grid):
        prim = orig(q, grid)
        prim["p"] = (grid.gamma - 1.0) * q[4]
        prim["pp"] = prim["p"] - O._t(grid.pbar_cell).reshape(-1, 1, 1)
        return prim
    monkeypatch.setattr(O, "cons_to_prim", bad)
    from tests import test_oracle_eos_adjoint as TE
    with pytest.raises(AssertionError):
        TE.test_prim_cons_round_trip()


# --- mixture equation of state ----------------------------------------------

def _moist_pins():
    from tests import test_oracle_moist as TM
    return TM


def test_inverted_mixture_ratio_breaks_dalton_pin(monkeypatch):
    TM = _moist_pins()
    orig = O.mixture_ratio
    monkeypatch.setattr(O, "mixture_ratio", lambda qs, coef: 1.0 / orig(qs, coef))
    with pytest.raises(AssertionError):
        TM.test_mixture_pressure_is_daltons_law()


def test_molar_mass_ratio_not_inverted_breaks_dalton_pin(monkeypatch):
    TM = _moist_pins()
    orig = O.mixture_coefficients

    def bad(grid):
        coef = orig(grid)
        if coef is None:
            return None
        return [((grid.tracer_eps[t] - 1.0) if grid.tracer_kind[t] == 0 else a, b, mu)
                for t, (a, b, mu) in enumerate(coef)]          # eps - 1 instead of 1/eps - 1
    monkeypatch.setattr(O, "mixture_coefficients", bad)
    with pytest.raises(AssertionError):
        TM.test_mixture_pressure_is_daltons_law()


def test_condensate_counted_as_gas_breaks_dalton_pin(monkeypatch):
    TM = _moist_pins()
    orig = O.mixture_coefficients

    def bad(grid):
        coef = orig(grid)
        if coef is None:
            return None
        return [(0.0 if grid.tracer_kind[t] == 1 else a, b, mu) for t, (a, b, mu) in enumerate(coef)]
    monkeypatch.setattr(O, "mixture_coefficients", bad)
    with pytest.raises(AssertionError):
        TM.test_mixture_pressure_is_daltons_law()


def test_dry_gamma_at_faces_breaks_one_gas_pin(monkeypatch):
    TM = _moist_pins()
    orig = O.lmars_flux
    monkeypatch.setattr(O, "lmars_flux",
                        lambda L, R, normal, gamma, ntracer, thermo=None: orig(L, R, normal, gamma, ntracer))
    with pytest.raises(AssertionError):
        TM.test_uniform_mixture_is_one_ideal_gas()


def test_chemical_energy_dropped_at_faces_breaks_advection_pin(monkeypatch):
    TM = _moist_pins()
    orig = O.lmars_flux

    def bad(L, R, normal, gamma, ntracer, thermo=None):
        if thermo is not None:
            thermo = [(a, b, 0.0) for a, b, _ in thermo]
        return orig(L, R, normal, gamma, ntracer, thermo)
    monkeypatch.setattr(O, "lmars_flux", bad)
    with pytest.raises(AssertionError):
        TM.test_chemical_energy_is_advected_with_its_tracer()


# --- Kessler microphysics ---------------------------------------------------

def _kessler_pins():
    from tests import test_oracle_kessler as TK
    return TK


def test_evaporation_sign_breaks_closed_form_pin(monkeypatch):
    TK = _kessler_pins()
    orig = O.kessler_rates

    def bad(qv, qc, qp, qs, sp, saturated):
        r = orig(qv, qc, qp, qs, sp, saturated)
        evap = torch.where(saturated, torch.zeros_like(qv), sp.k4 * qp * (qs - qv))
        return r + torch.stack([-2 * evap, torch.zeros_like(qv), 2 * evap], dim=-1)   # evaporation reversed
    monkeypatch.setattr(O, "kessler_rates", bad)
    with pytest.raises(AssertionError):
        TK.test_evaporation_alone_is_the_smaller_quadratic_root()


def test_accretion_lost_from_precipitation_breaks_conservation(monkeypatch):
    TK = _kessler_pins()
    orig = O.kessler_rates

    def bad(qv, qc, qp, qs, sp, saturated):
        r = orig(qv, qc, qp, qs, sp, saturated)
        acc = sp.k3 * qc * qp
        return r - torch.stack([torch.zeros_like(qv), torch.zeros_like(qv), acc], dim=-1)
    monkeypatch.setattr(O, "kessler_rates", bad)
    with pytest.raises(AssertionError):
        TK.test_all_processes_conserve_and_satisfy_backward_euler()


def test_wrong_kirchhoff_term_breaks_clausius_clapeyron_pin(monkeypatch):
    TK = _kessler_pins()

    def bad(T, sp):
        t = T / sp.t_ref
        return sp.p_ref * torch.exp(sp.beta * (1.0 - 1.0 / t) + sp.delta * torch.log(t))
    monkeypatch.setattr(O, "saturation_vapour_pressure", bad)
    with pytest.raises(AssertionError):
        TK.test_saturation_vapour_pressure_solves_clausius_clapeyron()


def test_vapour_molar_mass_ignored_breaks_latent_heating_pin(monkeypatch):
    TK = _kessler_pins()

    def bad(q, grid, rd):
        q = O._t(q)
        p = O.cons_to_prim(q, grid.copy(rhobar_cell=np.zeros(1), pbar_cell=np.zeros(1)))["p"]
        rho_d = q[0] - sum(q[5 + t] for t in range(grid.ntracer))
        gas = rho_d + sum(q[5 + t] for t in range(grid.ntracer) if grid.tracer_kind[t] == 0)
        return p / (rd * gas)                   # R_v taken equal to R_d
    monkeypatch.setattr(O, "temperature", bad)
    with pytest.raises(AssertionError):
        TK.test_constant_volume_phase_change_heats_as_the_paper_states()


# --- sedimentation ------------------------------------------------------------

def _sediment_pins():
    from tests import test_oracle_sediment as TS
    return TS


def test_open_lid_breaks_ground_budget(monkeypatch):
    TS = _sediment_pins()

    def bad(qf, grid, prim, R, isl):   # the lid lets condensate in from the mirrored ghost
        return orig(qf, grid.copy(bc=(grid.bc[0], grid.bc[1], 0)), prim, R, isl)
    orig = O._add_sedimentation
    monkeypatch.setattr(O, "_add_sedimentation", bad)
    with pytest.raises(AssertionError):
        TS.test_wall_column_loses_rain_only_through_the_ground()


def test_heating_sign_breaks_uniform_pin(monkeypatch):
    TS = _sediment_pins()
    orig = O._add_sedimentation

    def bad(qf, grid, prim, R, isl):
        orig(qf, grid, prim, R, isl)
        for t, wt in enumerate(grid.tracer_wt):
            R[4] = R[4] + 2.0 * grid.grav * wt * qf[5 + t][isl]
    monkeypatch.setattr(O, "_add_sedimentation", bad)
    with pytest.raises(AssertionError):
        TS.test_uniform_state_only_heats()


def test_chemical_energy_not_carried_breaks_ground_budget(monkeypatch):
    TS = _sediment_pins()
    orig = O._add_sedimentation
    monkeypatch.setattr(O, "_add_sedimentation",
                        lambda qf, grid, prim, R, isl: orig(qf, grid.copy(tracer_mu=(0.0,) * grid.ntracer),
                                                            prim, R, isl))
    with pytest.raises(AssertionError):
        TS.test_wall_column_loses_rain_only_through_the_ground()


def test_downwind_flux_breaks_falling_pin(monkeypatch):
    TS = _sediment_pins()
    orig = O._add_sedimentation

    def bad(qf, grid, prim, R, isl):   # flip the upwind side by flipping the velocity sign twice
        g2 = grid.copy(tracer_wt=tuple(-w for w in grid.tracer_wt))
        R2 = [r.clone() for r in R]
        orig(qf, g2, prim, R2, isl)
        for m in range(len(R)):
            R[m] = R[m] - (R2[m] - R[m])    # = sedimentation with the opposite upwind side, same sign
    monkeypatch.setattr(O, "_add_sedimentation", bad)
    with pytest.raises(AssertionError):
        TS.test_rain_falls_into_the_cell_below()


# --- HLLC ----------------------------------------------------------------------

def _hllc_pins():
    from tests import test_oracle_hllc as TH
    return TH


def test_contact_speed_pressure_sign_breaks_exact_star_pin(monkeypatch):
    TH = _hllc_pins()
    orig = O.hllc_wave_speeds

    def bad(L, R, normal, gamma):
        SL, SR, Ss = orig(L, R, normal, gamma)
        den = L["rho"] * (SL - L["u"]) - R["rho"] * (SR - R["u"])
        return SL, SR, Ss - 2.0 * (R["p"] - L["p"]) / den          # p_L - p_R in the numerator
    monkeypatch.setattr(O, "hllc_wave_speeds", bad)
    with pytest.raises(AssertionError):
        TH.test_star_state_matches_exact_riemann_to_second_order()


def test_star_energy_without_pressure_work_breaks_fan_conservation(monkeypatch):
    TH = _hllc_pins()
    orig = O.hllc_star

    def bad(S, Sk, Ss, normal, gamma):
        U = orig(S, Sk, Ss, normal, gamma)
        vel = [S["u"], S["v"], S["w"]]
        fac = S["rho"] * (Sk - vel[normal]) / (Sk - Ss)
        U[4] = U[4] - fac * (Ss - vel[normal]) * S["p"] / (S["rho"] * (Sk - vel[normal]))
        return U
    monkeypatch.setattr(O, "hllc_star", bad)
    with pytest.raises(AssertionError):
        TH.test_star_states_conserve_across_the_fan()


def test_star_momentum_with_side_velocity_breaks_fan_conservation(monkeypatch):
    TH = _hllc_pins()
    orig = O.hllc_star

    def bad(S, Sk, Ss, normal, gamma):
        U = orig(S, Sk, Ss, normal, gamma)
        vel = [S["u"], S["v"], S["w"]]
        U[1 + normal] = U[0] * vel[normal]          # normal momentum of the side, not S*
        return U
    monkeypatch.setattr(O, "hllc_star", bad)
    with pytest.raises(AssertionError):
        TH.test_star_states_conserve_across_the_fan()


# --- saturation adjustment ---------------------------------------------------

def _satadj_pins():
    from tests import test_oracle_satadj as TS
    return TS


def test_vapour_with_the_dry_gas_constant_breaks_equilibrium_pin(monkeypatch):
    TS = _satadj_pins()
    monkeypatch.setattr(O, "vapour_gas_constant", lambda grid, sp, rd: rd)
    with pytest.raises(AssertionError):
        TS.test_result_is_in_phase_equilibrium()


def test_temperature_without_latent_heat_breaks_paper_iteration_pin(monkeypatch):
    TS = _satadj_pins()
    orig = O.temperature_from_energy
    frozen = {}

    def held(qi, grid, rd, ek):
        key = id(ek)
        if key not in frozen:
            frozen[key] = orig(qi, grid, rd, ek)   # the temperature before any transfer
        return frozen[key]
    monkeypatch.setattr(O, "temperature_from_energy", held)
    with pytest.raises(AssertionError):
        TS.test_paper_iteration_reaches_the_oracles_equilibrium()


def test_cloud_that_cannot_evaporate_breaks_equilibrium_pin(monkeypatch):
    TS = _satadj_pins()
    monkeypatch.setattr(O, "transfer_bounds", lambda rv, rc: (torch.zeros_like(rc), rv.clone()))
    with pytest.raises(AssertionError):
        TS.test_result_is_in_phase_equilibrium()

