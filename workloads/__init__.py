"""Seeded synthetic inputs shared by the solver's tests, its benchmark and the oracle.

This module only *generates* inputs: grid shapes, boundary descriptors, charged
spheres and loss weights. It holds none of the solver's arithmetic (no stencil,
no deposition rule, no multigrid step), so both the HIP path and the CPU oracle
can draw from it without sharing any part of the method.

The workloads mirror the paper's setups: a Poisson problem for the electric
potential on the lattice-Boltzmann cell grid (Sec. 2.4), with charged spheres as
the only sources and Dirichlet potentials on two opposite faces with homogeneous
Neumann conditions on the other four (the showcase and scaling setups of Sec. 7
and Sec. 8.1). Lattice units are used for the sphere cases: spacing h = 1 and
permittivity eps = 1 (Sec. 2.1 normalises the lattice spacing to one).

Sphere recipe: numpy ``default_rng(seed)``; radii R ~ U[R_lo, R_hi]
(continuous), then each centre coordinate ~ U[R, N_axis - R] in cell units (the
sphere lies entirely inside the domain), then charges +1 or -1 with probability
1/2. Draw order: radii (n), centres (n x 3, row-major), sign bits (n).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

DIRICHLET = 0
NEUMANN = 1

# face order used everywhere: x-, x+, y-, y+, z-, z+
FACE_NAMES = ("x-", "x+", "y-", "y+", "z-", "z+")


@dataclass(frozen=True)
class Spheres:
    centers: np.ndarray  # [n, 3] float64, physical units (x, y, z)
    radii: np.ndarray    # [n] float64, physical units
    charges: np.ndarray  # [n] float64

    @property
    def n(self) -> int:
        return int(self.radii.shape[0])


@dataclass(frozen=True)
class Workload:
    name: str
    shape: Tuple[int, int, int]          # (nx, ny, nz); arrays are [nz][ny][nx]
    h: float
    kinds: Tuple[int, ...]               # 6 face kinds, DIRICHLET or NEUMANN
    values: Tuple[float, ...]            # 6 face values (Dirichlet potential / outward dphi/dn)
    levels: int
    nu1: int = 2
    nu2: int = 2
    omega: float = 1.95                  # coarse-correction factor "about 2" (Sec. 3); 1.95 takes one
                                         # cycle fewer than 2 on every workload here
    eps: float = 1.0
    rtol: float = 1e-10
    n_spheres: int = 0
    r_lo: float = 0.0
    r_hi: float = 0.0
    seed: int = 0
    precision: str = "fp64"              # "fp64" or "fp32-ir"
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def scaled(self, shape: Tuple[int, int, int], levels: int, n_spheres: Optional[int] = None,
               name: Optional[str] = None) -> "Workload":
        """Same boundary setup and sphere recipe on a smaller grid (for parity tests)."""
        return replace(self, shape=shape, levels=levels,
                       n_spheres=self.n_spheres if n_spheres is None else n_spheres,
                       name=name or f"{self.name}@{shape[0]}x{shape[1]}x{shape[2]}")


def _dirichlet_pair_axis(axis: int, lo: float, hi: float):
    kinds = [NEUMANN] * 6
    values = [0.0] * 6
    kinds[2 * axis] = DIRICHLET
    kinds[2 * axis + 1] = DIRICHLET
    values[2 * axis] = lo
    values[2 * axis + 1] = hi
    return tuple(kinds), tuple(values)


_ALL_D = (DIRICHLET,) * 6
_ZERO6 = (0.0,) * 6
_ZK, _ZV = _dirichlet_pair_axis(2, 0.0, 1.0)   # phi=0 at z=0, phi=1 at z=L, Neumann sides
_XK, _XV = _dirichlet_pair_axis(0, 0.0, 1.0)   # phi=0 at x=0, phi=1 at x=L, Neumann elsewhere

# The five workloads. C1: manufactured sine solution on the unit cube.
C1 = Workload("c1_sine_32", (32, 32, 32), 1.0 / 32, _ALL_D, _ZERO6, levels=4)
# C2: 256^3, 200 spheres of radius 4, plain FP64 multigrid down to 8^3.
C2 = Workload("c2_spheres_256", (256, 256, 256), 1.0, _ZK, _ZV, levels=6,
              n_spheres=200, r_lo=4.0, r_hi=4.0, seed=1002)
# C3: 512^3, 2000 spheres of radius U[3,6], FP32 cycles inside FP64 refinement.
C3 = Workload("c3_spheres_512", (512, 512, 512), 1.0, _ZK, _ZV, levels=7,
              n_spheres=2000, r_lo=3.0, r_hi=6.0, seed=1003, precision="fp32-ir")
# C4: 128^3, all-Dirichlet zero, 100 spheres of radius 4; loss sum_i w_i phi_i.
C4 = Workload("c4_adjoint_128", (128, 128, 128), 1.0, _ALL_D, _ZERO6, levels=5,
              n_spheres=100, r_lo=4.0, r_hi=4.0, seed=1004,
              extra={"weight_seed": 2004, "fd_seed": 3004, "fd_count": 16, "fd_step": 1e-6})
# C5: microchannel 1024 x 256 x 256, 10,000 spheres of radius U[3,5], 7 levels.
C5 = Workload("c5_channel_1024x256x256", (1024, 256, 256), 1.0, _XK, _XV, levels=7,
              n_spheres=10000, r_lo=3.0, r_hi=5.0, seed=1005, precision="fp32-ir")

ALL = {w.name: w for w in (C1, C2, C3, C4, C5)}

# SI constants for the per-node scene
EPS0 = 8.8541878128e-12        # vacuum permittivity, F/m
E_CHARGE = 1.602176634e-19     # elementary charge, C

# The paper's per-node time-step scene (parameters of the agglomeration
# showcase, Sec. 7; single-node set-up of the scaling runs, Sec. 8.1):
# 256 x 512 x 256 cells of 10 um (2 x 4 x 2 blocks of 128^3), in each block one
# set of 6^3 spheres of radius 6 cells at 12-cell centre spacing, centred in the
# block (3456 spheres); 8000 e per sphere, eps = 78.5 eps0; phi = -100 V at the
# bottom plane (z = 0) and 0 V at the top plane, insulating (zero-Neumann)
# sides; V(3,3) on 7 levels (coarsest 4 x 8 x 4), sub-sampling factor 2;
# 5 cycles at the first time step, then 1 per step, 240 steps.  The spheres
# drift by a seeded velocity per step (a common 0.004 cells/step towards the
# bottom plus a uniform jitter of up to 0.004 cells/step per axis).
_SK, _SV = _dirichlet_pair_axis(2, -100.0, 0.0)
SCENE = Workload("scene_256x512x256", (256, 512, 256), 1e-5, _SK, _SV, levels=7, nu1=3, nu2=3,
                 eps=78.5 * EPS0, n_spheres=3456, r_lo=6.0, r_hi=6.0, seed=1006,
                 extra={"block": 128, "set": 6, "spacing": 12.0, "charge": 8000 * E_CHARGE, "subsample": 2,
                        "steps": 240, "first_cycles": 5, "cycles": 1, "drift": 0.004})


def scene_spheres(w: Workload) -> Spheres:
    """Initial spheres of a time-step scene: one set^3 lattice per block, centred."""
    b, m, d = w.extra["block"], w.extra["set"], w.extra["spacing"]
    first = b / 2.0 - d * (m - 1) / 2.0
    offs = first + d * np.arange(m)
    nbx, nby, nbz = (n // b for n in w.shape)
    cs = []
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                for z in offs:
                    for y in offs:
                        for x in offs:
                            cs.append((bx * b + x, by * b + y, bz * b + z))
    c = np.asarray(cs, dtype=np.float64) * w.h
    n = c.shape[0]
    return Spheres(np.ascontiguousarray(c), np.full(n, w.r_lo * w.h), np.full(n, float(w.extra["charge"])))


def scene_trajectory(w: Workload, steps: int) -> np.ndarray:
    """Sphere centres for time steps 0..steps-1, [steps, n, 3], physical units."""
    s0 = scene_spheres(w)
    rng = np.random.default_rng(w.seed)
    d = w.extra["drift"]
    v = rng.uniform(-d, d, size=(s0.n, 3))
    v[:, 2] -= d
    t = np.arange(steps, dtype=np.float64)[:, None, None]
    return np.ascontiguousarray(s0.centers[None] + t * v[None] * w.h)


def cell_centers_1d(n: int, h: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def sine_rhs(shape: Tuple[int, int, int], h: float) -> np.ndarray:
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) sampled at cell centres, array [nz][ny][nx].

    Its continuum solution with phi = 0 on the unit-cube boundary is
    sin(pi x) sin(pi y) sin(pi z)."""
    nx, ny, nz = shape
    sx = np.sin(math.pi * cell_centers_1d(nx, h))
    sy = np.sin(math.pi * cell_centers_1d(ny, h))
    sz = np.sin(math.pi * cell_centers_1d(nz, h))
    return (3.0 * math.pi ** 2) * (sz[:, None, None] * sy[None, :, None] * sx[None, None, :])


def sine_exact(shape: Tuple[int, int, int], h: float) -> np.ndarray:
    nx, ny, nz = shape
    sx = np.sin(math.pi * cell_centers_1d(nx, h))
    sy = np.sin(math.pi * cell_centers_1d(ny, h))
    sz = np.sin(math.pi * cell_centers_1d(nz, h))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def make_spheres(n: int, shape: Tuple[int, int, int], h: float, r_lo: float, r_hi: float,
                 seed: int) -> Spheres:
    """Seeded charged spheres, fully inside the domain (recipe in the module docstring).

    Radii and centres are drawn in cell units and returned in physical units (x h)."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(r_lo, r_hi, size=n)   # r_lo == r_hi gives exactly r_lo
    u = rng.uniform(0.0, 1.0, size=(n, 3))
    ext = np.asarray(shape, dtype=np.float64)[None, :]
    centers = radii[:, None] + (ext - 2.0 * radii[:, None]) * u
    bits = rng.integers(0, 2, size=n)
    charges = np.where(bits == 1, 1.0, -1.0)
    return Spheres(np.ascontiguousarray(centers * h), np.ascontiguousarray(radii * h),
                   np.ascontiguousarray(charges))


def workload_spheres(w: Workload) -> Spheres:
    return make_spheres(w.n_spheres, w.shape, w.h, w.r_lo, w.r_hi, w.seed)


def loss_weights(w: Workload) -> np.ndarray:
    """w ~ N(0,1) per cell, [nz][ny][nx], for the loss L = sum_i w_i phi_i."""
    rng = np.random.default_rng(w.extra.get("weight_seed", 2004))
    nx, ny, nz = w.shape
    return rng.standard_normal((nz, ny, nx))


def fd_sphere_indices(w: Workload, n_spheres: Optional[int] = None) -> np.ndarray:
    rng = np.random.default_rng(w.extra.get("fd_seed", 3004))
    n = w.n_spheres if n_spheres is None else n_spheres
    return np.sort(rng.choice(n, size=min(w.extra.get("fd_count", 16), n), replace=False))


def random_field(shape: Tuple[int, int, int], seed: int, dtype=np.float64) -> np.ndarray:
    nx, ny, nz = shape
    return np.random.default_rng(seed).standard_normal((nz, ny, nx)).astype(dtype)
