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


# ---- periodic faces (Sec. 2.4: they cyclically extend the domain) -------------
P = 2   # periodic face kind
PERIODIC_KINDS = [(P, P, P, P, D, D), (P, P, N, D, P, P), (D, N, P, P, N, D)]


@pytest.mark.parametrize("kinds", PERIODIC_KINDS[:1])
def test_periodic_eigenmodes(orc, kinds):
    """cos(2 pi m (i+1/2)/nx) cos(2 pi m'(j+1/2)/ny) sin(pi p (k+1/2)/nz) is an
    eigenvector with eigenvalue s (2-2cos(2 pi m/nx) + 2-2cos(2 pi m'/ny) + 2-2cos(pi p/nz))."""
    nx, ny, nz, h = 8, 6, 10, 0.4
    k = orc.vc_faces(np.ones((nz, ny, nx)), kinds)
    i, j, kk = np.arange(nx) + 0.5, np.arange(ny) + 0.5, np.arange(nz) + 0.5
    for m, m2, p in ((1, 2, 1), (3, 1, 4), (4, 3, 7)):
        v = (np.sin(np.pi * p * kk / nz)[:, None, None] * np.cos(2 * np.pi * m2 * j / ny)[None, :, None] *
             np.cos(2 * np.pi * m * i / nx)[None, None, :])
        lam = (2 - 2 * np.cos(2 * np.pi * m / nx) + 2 - 2 * np.cos(2 * np.pi * m2 / ny) +
               2 - 2 * np.cos(np.pi * p / nz)) / (h * h)
        assert np.allclose(orc.vc_apply(v, h, kinds, k), lam * v, rtol=0, atol=1e-12 * lam)


@pytest.mark.parametrize("kinds", PERIODIC_KINDS)
def test_periodic_galerkin_and_definiteness(orc, kinds):
    fine, h = (4, 6, 4), 0.5
    eps = random_eps(fine, 17)
    k0 = orc.vc_faces(eps, kinds)
    A0 = vc_dense(orc, fine, h, kinds, k0, 0)
    A1 = vc_dense(orc, (2, 3, 2), h, kinds, orc.vc_coarsen(k0), 1)
    Pm = prolongation_matrix(fine)
    assert np.allclose(Pm.T @ A0 @ Pm / 8.0, A1, rtol=1e-13, atol=1e-12 * np.abs(A1).max())
    assert np.abs(A0 - A0.T).max() <= 1e-13 * np.abs(A0).max()
    assert np.linalg.eigvalsh(A0).min() > 0.0


def test_periodic_translation_invariance(orc):
    """Shifting eps and f cyclically along periodic x and y shifts the solution."""
    kinds, values = (P, P, P, P, D, D), (0, 0, 0, 0, 0.5, -0.3)
    shape, h = (16, 8, 16), 1.0 / 16
    eps, f = random_eps(shape, 31, 0.5, 5.0), W.random_field(shape, 32)
    def solve(e, ff):
        b = orc.vc_fold(ff, h, kinds, values, orc.vc_faces(e, kinds))
        phi, _, st = orc.vc_solve(b, h, kinds, 3, e, rtol=1e-13)
        assert st == 0
        return phi
    base = solve(eps, f)
    sh = solve(np.roll(eps, (3, 5), axis=(1, 2)), np.roll(f, (3, 5), axis=(1, 2)))
    assert np.abs(sh - np.roll(base, (3, 5), axis=(1, 2))).max() <= 1e-10 * np.abs(base).max()


@pytest.mark.parametrize("kinds", PERIODIC_KINDS)
def test_periodic_multigrid_matches_dense_solve(orc, kinds):
    shape, h = (8, 8, 8), 1.0 / 8
    eps = random_eps(shape, 41, 0.2, 20.0)
    k = orc.vc_faces(eps, kinds)
    b = orc.vc_fold(W.random_field(shape, 42), h, kinds, (0.3, -0.2, 0.1, 0.0, 1.0, -1.0), k)
    ref = np.linalg.solve(vc_dense(orc, shape, h, kinds, k), b.ravel()).reshape(b.shape)
    phi, _, st = orc.vc_solve(b, h, kinds, 3, eps, rtol=1e-13)
    assert st == 0 and np.abs(phi - ref).max() <= 1e-10 * np.abs(ref).max()


def test_periodic_gradient_of_a_sine(orc):
    """phi = sin(2 pi x / L) on a periodic x axis: every D3Q19 pair with an x
    step carries the same central difference, so grad_x = cos(x') sin(h')/h
    (x' = 2 pi x / L, h' = 2 pi h / L) exactly, on the wrapped cells too."""
    nx, ny, nz, L = 16, 6, 8, 2.0
    h = L / nx
    kinds = (P, P, N, N, D, D)
    x = (np.arange(nx) + 0.5) * h
    phi = np.broadcast_to(np.sin(2 * np.pi * x / L), (nz, ny, nx)).copy()
    g = orc.gradient(phi, h, kinds, (0.0,) * 6)
    want = np.cos(2 * np.pi * x / L) * np.sin(2 * np.pi * h / L) / h
    inner = (slice(1, -1), slice(1, -1), slice(None))   # away from the non-periodic y/z layers
    assert np.allclose(g[0][inner], np.broadcast_to(want, (nz, ny, nx))[inner], rtol=0, atol=1e-13)
    # the boundary layers of y/z use D3Q7 in x, also exact: (phi(x+h) - phi(x-h)) / 2h
    assert np.allclose(g[0][0], np.broadcast_to(want, (ny, nx)), rtol=0, atol=1e-13)


@pytest.mark.parametrize("kinds", KINDS + PERIODIC_KINDS)
@pytest.mark.parametrize("level", [0, 1])
def test_vc_rbgs_equals_dense_gauss_seidel(orc, kinds, level):
    """One variable-permittivity red-black sweep is one Gauss-Seidel sweep over
    the unknowns ordered red first, then black (Sec. 5.3), on the operator whose
    columns vc_apply gives (itself pinned above); two sweeps are two of them."""
    shape, h = (4, 6, 4), 0.4
    nx, ny, nz = shape
    fine = (2 * nx, 2 * ny, 2 * nz) if level else shape
    k = orc.vc_faces(random_eps(fine, 31), kinds)
    if level:
        k = orc.vc_coarsen(k)
    A = vc_dense(orc, shape, h, kinds, k, level)
    rng = np.random.default_rng(32)
    n = A.shape[0]
    b = rng.standard_normal(n)
    phi0 = rng.standard_normal(n)
    col = ((np.arange(n) % nx) + (np.arange(n) // nx) % ny + np.arange(n) // (nx * ny)) % 2
    order = list(np.flatnonzero(col == 0)) + list(np.flatnonzero(col == 1))
    x = phi0.copy()
    for sweep in range(2):
        for c in order:
            x[c] = (b[c] - (A[c] @ x - A[c, c] * x[c])) / A[c, c]
        got = orc.vc_rbgs_sweep(phi0.reshape(nz, ny, nx), b.reshape(nz, ny, nx), h, kinds, k, level, sweeps=sweep + 1)
        assert np.abs(got.ravel() - x).max() <= 1e-13 * max(1.0, np.abs(x).max()), sweep
