"""GPU parity of the sub-sampled deposition, its charge gradient and per-cell
boundary values (Sec. 2.4, "Subsampling" and "Boundary conditions"), and the
charged-sphere validation of Sec. 6.3 against the analytic potential.

Bars: summed overlap ratios W_s bit-identical to the oracle (both are an
integer count divided by s_f^3); deposited fields within a rounding step (the
atomic adds of overlapping spheres run in another order); gradients within
1e-12 of their magnitude (another summation order); solves with per-cell
boundary values as the other FP64 solves (same cycles, 1e-12).  The analytic
comparison is loose (the paper's error norms are reproduced to about 25 % in
the maximum norm; exact values are parity-unpinned).
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1410_6609_amd as pkg
import workloads as W
from workloads import DIRICHLET as D, NEUMANN as N

from test_gpu_parity import DEV, log_case, rhs, to_dev

pytestmark = pytest.mark.gpu

MODES = [pkg.SPREAD, pkg.VOLUME]


def sphere_set(shape=(96, 64, 80), n=120, seed=1002, r=(2.5, 5.5)):
    """Seeded spheres, some cut by the domain boundary, plus one covering no
    sub-cell centre (radius far below a sub-cell) and one far outside."""
    w = W.Workload("sub", shape, 1.0, (N, N, N, N, D, D), (0, 0, 0, 0, 0.0, 1.0), levels=4, n_spheres=n,
                   r_lo=r[0], r_hi=r[1], seed=seed)
    s = W.workload_spheres(w)
    rng = np.random.default_rng(seed + 1)
    edge = np.column_stack([rng.uniform(-2, 2, 6), rng.uniform(0, shape[1], 6), rng.uniform(0, shape[2], 6)])
    c = np.vstack([s.centers, edge, [[10.013, 10.017, 10.019]], [[-40.0, 5.0, 5.0]]])
    rad = np.concatenate([s.radii, rng.uniform(2, 5, 6), [1e-6], [3.0]])
    q = np.concatenate([s.charges, rng.choice([-1.0, 1.0], 6), [1.0], [1.0]])
    return w, c, rad, q


def make_solver(w, **opt):
    return pkg.Solver(w.shape, w.h, list(zip(w.kinds, w.values)), pkg.Options(levels=w.levels, **opt), device=DEV)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("sf", [1, 2, 3, 4, 5, 8])
def test_deposit_sub_parity(sf, mode):
    log_case("deposit_sub", sf, mode)
    w, c, r, q = sphere_set()
    s = make_solver(w)
    eps = 0.7
    f, wsum = s.deposit(to_dev(c), to_dev(r), to_dev(q), eps, counts=True, subsample=sf, mode=mode)
    f_ref, w_ref = oracle.deposit_sub(w.shape, w.h, c, r, q, eps, subsample=sf, mode=mode)
    assert np.array_equal(wsum.cpu().numpy(), w_ref)
    assert w_ref[-2] == 0.0 and w_ref[-1] == 0.0
    got = f.cpu().numpy()
    assert np.array_equal(got != 0, f_ref != 0)
    assert np.abs(got - f_ref).max() <= 4e-16 * np.abs(f_ref).max()


def test_deposit_sub_sf1_spread_is_the_naive_deposition():
    """Disjoint spheres (no atomic-order effects): bit-identical fields."""
    w = W.C2.scaled((64, 64, 64), levels=3, n_spheres=8)
    c = np.array([[12.5 + 14 * (i % 4), 14.2 + 30 * (i // 4), 31.7] for i in range(8)])
    r = np.full(8, 5.5)
    q = np.linspace(-1, 1, 8)
    s = make_solver(w)
    f0, cnt = s.deposit(to_dev(c), to_dev(r), to_dev(q), 0.9, counts=True)
    f1, wsum = s.deposit(to_dev(c), to_dev(r), to_dev(q), 0.9, counts=True, subsample=1, mode=pkg.SPREAD)
    assert torch.equal(f0, f1)
    assert torch.equal(cnt.to(torch.float64), wsum)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("sf", [1, 3, 4])
def test_charge_gradient_parity(sf, mode):
    log_case("charge_gradient", sf, mode)
    w, c, r, q = sphere_set(seed=77)
    s = make_solver(w)
    lam = rhs(w.shape, 31)
    dq = s.charge_gradient(to_dev(lam), to_dev(c), to_dev(r), 1.3, subsample=sf, mode=mode)
    ref = oracle.dq_sub(lam, w.h, c, r, 1.3, subsample=sf, mode=mode)
    assert np.abs(dq.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    assert ref[-2] == 0.0 and ref[-1] == 0.0


@pytest.mark.parametrize("mode", MODES)
def test_autograd_with_subsampling(mode):
    w = W.C4.scaled((64, 64, 64), levels=4, n_spheres=24)
    sph = W.workload_spheres(w)
    s = make_solver(w)
    wts = W.random_field(w.shape, 41)
    c, r, q = (to_dev(a) for a in (sph.centers, sph.radii, sph.charges))
    qg = q.clone().requires_grad_(True)
    phi = pkg.PoissonFn.apply(qg, c, r, s, 0.8, 1e-11, 100, 3, mode)
    (phi * to_dev(wts)).sum().backward()
    lam, _, _ = oracle.adjoint(wts, w.h, w.kinds, w.levels, rtol=1e-11)
    ref = oracle.dq_sub(lam, w.h, sph.centers, sph.radii, 0.8, subsample=3, mode=mode)
    assert np.abs(qg.grad.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
    # forward against the oracle's sub-sampled deposition and solve
    f_ref, _ = oracle.deposit_sub(w.shape, w.h, sph.centers, sph.radii, sph.charges, 0.8, subsample=3, mode=mode)
    phi_ref, _, _ = oracle.solve_problem(f_ref, w.h, w.kinds, w.values, w.levels, rtol=1e-11)
    assert np.abs(phi.detach().cpu().numpy() - phi_ref).max() <= 1e-12 * np.abs(phi_ref).max()


# ---- per-cell boundary values ------------------------------------------------
FACE_SHAPES = lambda nx, ny, nz: [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2  # noqa: E731


@pytest.mark.parametrize("shape,levels,kinds", [
    ((64, 48, 40), 3, (N, N, D, N, D, D)),
    ((96, 80, 72), 4, (N, D, D, N, D, N)),
    ((16, 8, 32), 3, (D, D, D, D, D, D)),
])
def test_face_values_solve_parity(shape, levels, kinds):
    log_case("face values", shape)
    nx, ny, nz = shape
    h = 1.0 / nx
    values = (0.2, -0.1, 0.3, 0.05, 0.0, 1.0)
    s = pkg.Solver(shape, h, list(zip(kinds, values)), pkg.Options(levels=levels), device=DEV)
    rng = np.random.default_rng(9)
    faces = [rng.standard_normal(fs) if fc % 3 != 1 else None for fc, fs in enumerate(FACE_SHAPES(*shape))]
    for fc, a in enumerate(faces):
        if a is not None:
            s.set_face_values(fc, to_dev(a))
    f = rhs(shape, 21)
    phi, st = s.solve(to_dev(f), rtol=1e-10)
    b = oracle.fold_field(f, h, kinds, values, faces)
    ref, hist, _ = oracle.solve(b, h, kinds, levels, rtol=1e-10)
    assert st.cycles == len(hist) - 1
    assert np.abs(phi.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    # the adjoint keeps homogeneous boundary values
    lam, _, _, _ = s.adjoint(to_dev(f), rtol=1e-10)
    lref, _, _ = oracle.adjoint(f, h, kinds, levels, rtol=1e-10)
    assert np.abs(lam.cpu().numpy() - lref).max() <= 1e-12 * np.abs(lref).max()
    # None restores the constant values
    for fc in range(6):
        s.set_face_values(fc, None)
    phi2, _ = s.solve(to_dev(f), rtol=1e-10)
    ref2, _, _ = oracle.solve_problem(f, h, kinds, values, levels, rtol=1e-10)
    assert np.abs(phi2.cpu().numpy() - ref2).max() <= 1e-12 * np.abs(ref2).max()


def test_face_values_argument_errors():
    s = pkg.Solver((32, 32, 32), 1 / 32, [(D, 0.0)] * 6, pkg.Options(levels=3), device=DEV)
    L = pkg.lib()
    assert L.ccmg_set_face_values(s._h, 6, None) == pkg.E_ARG
    host = np.zeros(32 * 32)
    import ctypes
    assert L.ccmg_set_face_values(s._h, 0, ctypes.c_void_p(host.ctypes.data)) == pkg.E_ARG
    assert L.ccmg_deposit_charges_sub(s._h, 0, None, None, None, 1.0, 9, 0, None, None) == pkg.E_ARG


# ---- charged-sphere validation (Sec. 6.3, Tab. ValidPotSubs) ---------------
GOLDEN_SUB = os.path.join(os.path.dirname(__file__), "golden", "volume_mapping_subsampled.txt")
# ||e_rPhi||_inf and ||e_rPhi||_L2 in percent as printed (Tab. ValidPotSubs), keyed by (R, s_f)
PAPER_PHI = {(4, 2): (3.37, 0.622), (4, 3): (-2.06, 0.568), (4, 4): (1.13, 0.192),
             (6, 2): (-2.19, 0.568), (6, 3): (-0.80, 0.290), (6, 4): (-0.61, 0.273),
             (9, 2): (-0.82, 0.290), (9, 3): (0.44, 0.185), (9, 4): (-0.39, 0.244)}


def analytic_potential(x, y, z, c, R, Q, eps):
    """Potential of a homogeneously charged sphere in free space (Sec. 6.3)."""
    r = torch.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    k = Q / (4 * math.pi * eps)
    return torch.where(r >= R, k / torch.clamp(r, min=1e-300), k / (2 * R) * (3 - (r / R) ** 2))


def golden_shift(R, sf):
    with open(GOLDEN_SUB) as fh:
        for line in fh:
            p = line.split()
            if p and not line.startswith("#") and int(p[0]) == R and int(p[1]) == sf:
                return np.array([float(p[4]), float(p[5]), float(p[6])])
    raise KeyError((R, sf))


@pytest.mark.parametrize("R,sf", sorted(PAPER_PHI))
def test_charged_sphere_against_analytic_potential(R, sf):
    """256^3 domain, sphere near the centre at the shift of maximal volume-mapping
    error, the paper's charge density q / V times the overlap ratio, Dirichlet
    values from the analytic potential on all faces.  The maximum relative
    potential error has the printed sign and is within 25 % of the printed
    value; the domain RMS of the relative error stays below 1.25x the printed
    L2 value (parity-unpinned: the paper's exact norms are not reproduced)."""
    n, h, Q, eps = 256, 1.0, 1.0, 1.0
    log_case("charged sphere", R, sf)
    c = n / 2 + (0.5 + golden_shift(R, sf)) / sf
    s = pkg.Solver((n, n, n), h, [(D, 0.0)] * 6, pkg.Options(levels=7), device=DEV)
    ax = (torch.arange(n, device=DEV, dtype=torch.float64) + 0.5) * h
    v, u = torch.meshgrid(ax, ax, indexing="ij")
    lo, hi = torch.zeros_like(u), torch.full_like(u, n * h)
    faces = [analytic_potential(lo, u, v, c, R, Q, eps), analytic_potential(hi, u, v, c, R, Q, eps),
             analytic_potential(u, lo, v, c, R, Q, eps), analytic_potential(u, hi, v, c, R, Q, eps),
             analytic_potential(u, v, lo, c, R, Q, eps), analytic_potential(u, v, hi, c, R, Q, eps)]
    for fc, a in enumerate(faces):
        s.set_face_values(fc, a.contiguous())
    f, wsum = s.deposit(to_dev(c[None]), to_dev([float(R)]), to_dev([Q]), eps, counts=True, subsample=sf,
                        mode=pkg.VOLUME)
    phi, st = s.solve(f, rtol=1e-10)
    z, y, x = torch.meshgrid(ax, ax, ax, indexing="ij")
    ex = analytic_potential(x, y, z, c, R, Q, eps)
    e = (phi - ex) / ex
    del x, y, z, ex
    emax = float(e.flatten()[torch.argmax(e.abs())]) * 100
    rms = float(torch.sqrt((e ** 2).mean())) * 100
    want_max, want_l2 = PAPER_PHI[(R, sf)]
    print(f"R={R} sf={sf}: e_rV={(float(wsum[0]) - 4 / 3 * math.pi * R ** 3) / (4 / 3 * math.pi * R ** 3) * 100:.3f}% "
          f"max e_rPhi {emax:.3f}% (paper {want_max}%), rms {rms:.3f}% (paper L2 {want_l2}%)", flush=True)
    assert np.sign(emax) == np.sign(want_max)
    assert abs(emax - want_max) <= 0.25 * abs(want_max)
    assert rms <= 1.25 * want_l2
