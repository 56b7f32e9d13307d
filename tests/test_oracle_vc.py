"""Pins of the oracle's variable-permittivity operator and multigrid
(-div(eps grad phi) = rho; Galerkin coarsening with the cell-centred
transfers, Sec. 3; stored per-unknown stencils, Sec. 5.3).

References: constant permittivity reduces to the (independently pinned)
constant-coefficient operator; the coarse operators equal the explicit
Galerkin product R A P; symmetry and definiteness; a layered medium whose
exact solution is piecewise linear; dense solves; convergence with jumping
coefficients."""
import numpy as np
import pytest

import workloads as W
from workloads import DIRICHLET as D, NEUMANN as N

from test_oracle_operator import dense_matrix, prolongation_matrix

KINDS = [(D,) * 6, (N, N, N, N, D, D), (D, N, N, D, N, D), (N, D, D, N, D, N)]


def vc_dense(orc, shape, h, kinds, k, level=0):
    nx, ny, nz = shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    e = np.zeros((nz, ny, nx))
    for c in range(n):
        e.flat[c] = 1.0
        A[:, c] = orc.vc_apply(e, h, kinds, k, level).ravel()
        e.flat[c] = 0.0
    return A


def random_eps(shape, seed, lo=0.5, hi=4.0):
    nx, ny, nz = shape
    return np.random.default_rng(seed).uniform(lo, hi, (nz, ny, nx))


@pytest.mark.parametrize("kinds", KINDS)
def test_constant_permittivity_is_the_constant_operator(orc, kinds):
    shape, h, c = (6, 4, 8), 0.3, 2.5
    k = orc.vc_faces(np.full((8, 4, 6), c))
    kc = orc.vc_coarsen(k)
    phi = W.random_field(shape, 3)
    assert np.allclose(orc.vc_apply(phi, h, kinds, k, 0), c * orc.apply(phi, h, kinds, 0), rtol=1e-14, atol=1e-12)
    phic = W.random_field((3, 2, 4), 4)
    assert np.allclose(orc.vc_apply(phic, h, kinds, kc, 1), c * orc.apply(phic, h, kinds, 1), rtol=1e-14,
                       atol=1e-12)


def test_harmonic_face_coefficients(orc):
    eps = random_eps((4, 3, 5), 1)
    kx, ky, kz = orc.vc_faces(eps)
    a, b = eps[2, 1, 1], eps[2, 1, 2]
    assert kx[2, 1, 2] == pytest.approx(2 * a * b / (a + b), rel=1e-15)
    assert kx[2, 1, 0] == eps[2, 1, 0] and kx[2, 1, 4] == eps[2, 1, 3]
    assert ky[0, 3, 1] == eps[0, 2, 1] and kz[5, 0, 2] == eps[4, 0, 2]


@pytest.mark.parametrize("kinds", KINDS)
def test_galerkin_coarse_operator_is_r_a_p(orc, kinds):
    """A_{l+1} = R A_l P for a random permittivity, R = P^T / 8: the coarse
    operator the oracle builds from averaged face coefficients is the exact
    Galerkin product (a plain matrix identity, independent of the formula)."""
    fine, h = (4, 6, 4), 0.5
    eps = random_eps(fine, 7)
    k0 = orc.vc_faces(eps)
    k1 = orc.vc_coarsen(k0)
    A0 = vc_dense(orc, fine, h, kinds, k0, 0)
    A1 = vc_dense(orc, (2, 3, 2), h, kinds, k1, 1)
    P = prolongation_matrix(fine)
    assert np.allclose(P.T @ A0 @ P / 8.0, A1, rtol=1e-13, atol=1e-12 * np.abs(A1).max())
    # and one level further
    k2 = orc.vc_coarsen(orc.vc_coarsen(orc.vc_faces(random_eps((8, 8, 4), 8))))
    assert k2[0].shape == (1, 2, 3)


@pytest.mark.parametrize("kinds", KINDS)
def test_symmetric_positive_definite(orc, kinds):
    shape = (4, 4, 6)
    A = vc_dense(orc, shape, 0.5, kinds, orc.vc_faces(random_eps(shape, 11, 0.1, 50.0)))
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0.0
    assert (np.count_nonzero(A, axis=1) <= 7).all()


@pytest.mark.parametrize("kinds", [(D, D, N, N, N, N), (D, D, D, D, D, D)])
def test_layered_medium_exact_solution(orc, kinds):
    """-(eps phi')' = 0 between phi = 0 at x = 0 and phi = 1 at x = L with eps = 1
    for x < L/2 and 10 beyond (the jump on a cell face): the flux is constant,
    phi is piecewise linear, and the harmonic-mean finite volumes reproduce it
    exactly at the cell centres (with Dirichlet data on the y/z faces taken from
    the same profile when they are Dirichlet)."""
    nx, ny, nz, h = 16, 4, 4, 1.0 / 16
    e1, e2 = 1.0, 10.0
    eps = np.where(np.arange(nx)[None, None, :] < nx // 2, e1, e2) * np.ones((nz, ny, nx))
    J = 1.0 / (0.5 / e1 + 0.5 / e2)
    x = (np.arange(nx) + 0.5) * h
    prof = np.where(x <= 0.5, J * x / e1, J * 0.5 / e1 + J * (x - 0.5) / e2)
    exact = np.broadcast_to(prof, (nz, ny, nx)).copy()
    k = orc.vc_faces(eps)
    faces = [None, None, None, None, None, None]
    if kinds[2] == D:
        faces = [None, None, np.broadcast_to(prof, (nz, nx)).copy(), np.broadcast_to(prof, (nz, nx)).copy(),
                 np.broadcast_to(prof, (ny, nx)).copy(), np.broadcast_to(prof, (ny, nx)).copy()]
    b = orc.vc_fold(np.zeros((nz, ny, nx)), h, kinds, (0.0, 1.0, 0, 0, 0, 0), k, faces)
    phi, hist, st = orc.vc_solve(b, h, kinds, 2, eps, rtol=1e-14, max_cycles=200)
    assert st == 0
    assert np.abs(phi - exact).max() <= 1e-12


@pytest.mark.parametrize("kinds", KINDS[:3])
def test_multigrid_matches_dense_solve(orc, kinds):
    shape, h = (8, 8, 8), 1.0 / 8
    eps = random_eps(shape, 21, 0.2, 20.0)
    k = orc.vc_faces(eps)
    f = W.random_field(shape, 22)
    b = orc.vc_fold(f, h, kinds, (0.3, -0.2, 0.1, 0.0, 1.0, -1.0), k)
    A = vc_dense(orc, shape, h, kinds, k)
    ref = np.linalg.solve(A, b.ravel()).reshape(b.shape)
    phi, hist, st = orc.vc_solve(b, h, kinds, 3, eps, rtol=1e-13)
    assert st == 0
    assert np.abs(phi - ref).max() <= 1e-10 * np.abs(ref).max()


def test_fold_with_unit_permittivity_is_the_constant_fold(orc):
    shape, h = (6, 5, 4), 0.2
    kinds, values = (D, N, D, N, N, D), (0.4, -0.3, 1.0, 0.2, 0.0, -0.6)
    f = W.random_field(shape, 5)
    k = orc.vc_faces(np.ones((4, 5, 6)))
    assert np.allclose(orc.vc_fold(f, h, kinds, values, k), orc.fold(f, h, kinds, values), rtol=1e-15, atol=1e-13)


def test_jumping_permittivity_converges(orc):
    """Low-permittivity spheres (eps 2.5) in a high-permittivity fluid (eps 78.5),
    a jump of 31x: Galerkin multigrid still contracts the residual by a
    size-independent factor per cycle."""
    rates = []
    for n, levels in ((32, 3), (64, 4)):
        w = W.C2.scaled((n, n, n), levels=levels, n_spheres=n // 4)
        w = W.Workload(**{**w.__dict__, "r_lo": 3.0, "r_hi": 5.0})
        s = W.workload_spheres(w)
        ax = np.arange(n) + 0.5
        Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
        eps = np.full((n, n, n), 78.5)
        for c, r in zip(s.centers, s.radii):
            eps[(X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2 <= r * r] = 2.5
        k = orc.vc_faces(eps)
        f, _ = orc.deposit(w.shape, 1.0, s.centers, s.radii, s.charges)
        b = orc.vc_fold(f, 1.0, w.kinds, w.values, k)
        phi, hist, st = orc.vc_solve(b, 1.0, w.kinds, levels, eps, rtol=1e-10)
        assert st == 0
        rates.append((hist[-1] / hist[1]) ** (1.0 / (len(hist) - 2)))
    assert max(rates) < 0.3, rates
    assert rates[1] < 1.5 * rates[0] + 0.02, rates
