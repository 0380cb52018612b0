"""Seeded parity cases shared by the GPU tests (inputs only; no arithmetic of the method).

Each case is a (grid, padded state, dt) triple built from the ``workloads``
generators. Sizes are chosen so that the oracle finishes in seconds while the
GPU kernels still see several tiles and ragged edges along every axis.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import workloads as wl

# (name, nx, ny, nz, ntracer, bc, lx, ly, lz, linear, seed)
SPECS = [
    ("2d_bubble_64x64", None),
    ("2d_smooth_37x29_nt3", dict(nx=37, ny=1, nz=29, nt=3, bc=(0, 0, 1), seed=11)),
    ("2d_reflect_21x19", dict(nx=21, ny=1, nz=19, nt=0, bc=(1, 0, 1), seed=12)),
    ("2d_narrow_1x8", dict(nx=1, ny=1, nz=8, nt=0, bc=(0, 0, 1), seed=13)),
    ("2d_thin_19x2", dict(nx=19, ny=1, nz=2, nt=1, bc=(1, 0, 1), seed=14)),
    ("3d_smooth_35x21x19", dict(nx=35, ny=21, nz=19, nt=0, bc=(0, 0, 1), seed=21)),
    ("3d_tracers_20x18x24_nt4", dict(nx=20, ny=18, nz=24, nt=4, bc=(1, 0, 1), seed=22)),
    ("3d_linear_17x9x11", dict(nx=17, ny=9, nz=11, nt=1, bc=(0, 1, 1), seed=23, linear=True)),
    ("3d_nt8_10x12x9", dict(nx=10, ny=12, nz=9, nt=8, bc=(0, 0, 1), seed=24)),
    ("3d_periodic_z_12x10x14", dict(nx=12, ny=10, nz=14, nt=2, bc=(0, 0, 0), seed=25, grav=0.0)),
    ("3d_small_2x3x4", dict(nx=2, ny=3, nz=4, nt=0, bc=(1, 1, 1), seed=26)),
    # no tracers: the stage kernel reads ghost cells in place (periodic z, an x
    # wall with periodic y, and a periodic domain narrower than the ghost width)
    ("3d_periodic_all_13x11x10", dict(nx=13, ny=11, nz=10, nt=0, bc=(0, 0, 0), seed=27, grav=0.0)),
    ("3d_xwall_19x17x12", dict(nx=19, ny=17, nz=12, nt=0, bc=(1, 0, 1), seed=28)),
    ("3d_tiny_periodic_2x2x5", dict(nx=2, ny=2, nz=5, nt=0, bc=(0, 0, 0), seed=29, grav=0.0)),
]

# Cases with the mixture equation of state: ``species`` picks tracers of
# workloads.condensable_species (0, 1 = vapours; 2, 3 = their clouds).
MIX_SPECS = [
    ("mix_3d_25x19x22_nt4", dict(nx=25, ny=19, nz=22, nt=4, bc=(0, 0, 1), seed=31, species=(0, 1, 2, 3))),
    ("mix_2d_33x27_nt2", dict(nx=33, ny=1, nz=27, nt=2, bc=(0, 0, 1), seed=32, species=(0, 2))),
    ("mix_3d_walls_14x11x13_nt1", dict(nx=14, ny=11, nz=13, nt=1, bc=(1, 1, 1), seed=33, species=(1,))),
    ("mix_3d_periodic_12x10x14_nt3", dict(nx=12, ny=10, nz=14, nt=3, bc=(0, 0, 0), seed=34, grav=0.0,
                                          species=(2, 0, 3))),
]


@dataclasses.dataclass
class Case:
    name: str
    grid: wl.Grid
    q: np.ndarray
    dt: float


def build_case(name: str, spec) -> Case:
    if spec is None:
        grid, q = wl.bubble_2d()
        return Case(name, grid, q, 0.25)
    nx, ny, nz = spec["nx"], spec["ny"], spec["nz"]
    lx, ly, lz = 200.0 * nx, 200.0 * ny, 150.0 * nz
    grav = spec.get("grav", 9.81)
    if grav == 0.0:
        base = wl.DryIsentropic(grav=0.0)
        grid, _ = wl.dry_grid(nx, ny, nz, lx, ly, lz, bc=spec["bc"], base=base)
        rc, pc, rf, pf = wl.uniform_references(nz, 1.1, 9.5e4)
        grid.rhobar_cell, grid.pbar_cell, grid.rhobar_face, grid.pbar_face = rc, pc, rf, pf
        grid.grav = 0.0
    else:
        grid, _ = wl.dry_grid(nx, ny, nz, lx, ly, lz, bc=spec["bc"])
    if ny == 1:
        grid.dy = 1.0
    grid.ntracer = spec["nt"]
    grid.weno_linear = bool(spec.get("linear", False))
    if "species" in spec:
        base = wl.DryIsentropic()
        table = wl.condensable_species(base.cp - base.rd, wl.RGAS / base.rd)
        grid = wl.with_mixture(grid, [table[i] for i in spec["species"]])
    q = wl.random_smooth_state(grid, spec["seed"])
    return Case(name, grid, q, 0.2)


def all_cases():
    return [build_case(n, s) for n, s in SPECS]


CASE_NAMES = [n for n, _ in SPECS]
MIX_NAMES = [n for n, _ in MIX_SPECS]


# Cases of the Kessler microphysics: water and ammonia (vapour, cloud,
# precipitation; workloads.kessler_tracers) on an isentropic 300 K base,
# 10 km deep, so that water is saturated aloft and not below.
KESSLER_SPECS = [
    ("kessler_3d_21x13x16", dict(nx=21, ny=13, nz=16, seed=41)),
    ("kessler_2d_37x24", dict(nx=37, ny=1, nz=24, seed=42)),
    ("kessler_3d_ragged_9x7x5", dict(nx=9, ny=7, nz=5, seed=43)),
]
KESSLER_NAMES = [n for n, _ in KESSLER_SPECS]


def build_kessler_case(name: str, spec):
    """(grid, padded state, Kessler parameters, dt) of a microphysics case."""
    nx, ny, nz = spec["nx"], spec["ny"], spec["nz"]
    base = wl.DryIsentropic()
    grid, _ = wl.dry_grid(nx, ny, nz, 250.0 * nx, 250.0 * ny, 10e3, bc=(0, 0, 1))
    if ny == 1:
        grid.dy = 1.0
    table, kes = wl.kessler_tracers(base.cp - base.rd, wl.RGAS / base.rd, base.rd)
    grid = wl.with_mixture(grid, table)
    rng = np.random.default_rng(spec["seed"])
    shp = (nz, ny, nx)
    rho, p = wl.rest_fields(grid)
    rho = rho * (1.0 + 0.01 * rng.standard_normal(shp))
    u, v, w = (2.0 * rng.standard_normal(shp) for _ in range(3))
    if ny == 1:
        v = np.zeros(shp)
    vap = [10.0 ** rng.uniform(-3.5, -1.5, shp) for _ in range(2)]
    cond = [10.0 ** rng.uniform(-5.0, -3.0, shp) for _ in range(4)]
    q = wl.state_from_primitives(grid, rho, u, v, w, p, vap + cond)
    return Case(name, grid, q, 2.0), kes


# Cases with falling precipitation (sedimentation): the Kessler cases with the
# water and ammonia rain falling at 6 and 4 m/s, with walls or periodic in z.
SED_SPECS = [
    ("sed_3d_walls_21x13x16", dict(nx=21, ny=13, nz=16, seed=51, bc=(0, 0, 1))),
    ("sed_3d_periodic_z_12x9x14", dict(nx=12, ny=9, nz=14, seed=52, bc=(0, 0, 0))),
    ("sed_2d_walls_29x20", dict(nx=29, ny=1, nz=20, seed=53, bc=(1, 0, 1))),
]
SED_NAMES = [n for n, _ in SED_SPECS]


def build_sediment_case(name: str, spec) -> Case:
    c, _ = build_kessler_case(name, spec)
    base = wl.DryIsentropic()
    g = c.grid
    if tuple(spec["bc"]) != tuple(g.bc):
        g2, _ = wl.dry_grid(g.nx, g.ny, g.nz, g.dx * g.nx, g.dy * g.ny, g.dz * g.nz, bc=spec["bc"])
        g = g.copy(bc=tuple(spec["bc"]), rhobar_cell=g2.rhobar_cell, pbar_cell=g2.pbar_cell,
                   rhobar_face=g2.rhobar_face, pbar_face=g2.pbar_face)
    g = g.copy(tracer_wt=(0.0, 0.0, 0.0, 0.0, -6.0, -4.0), rd=base.rd)
    return Case(name, g, c.q, 0.2)
