"""Pins of the oracle's Poisson-Boltzmann extension (the paper's outlook names
the equation, Sec. 9, without writing it out; the reading taken, and the
coarse operators and iteration used, are stated in the oracle's source).

Linear (Debye-Hueckel) operator -Lap + kappa^2: closed-form eigenpairs,
Galerkin and rediscretisation identities, the smoother against dense
Gauss-Seidel, CG and multigrid against dense solves, and the exact discrete
solution of a planar double layer (a combination of discrete exponentials),
which also converges to the continuous one at second order.  Nonlinear
operator -Lap + kappa^2 sinh: the planar Gouy-Chapman double layer (second
order), a manufactured discrete solution, the small-potential limit (the
linear solution), and kappa = 0 (Poisson's equation)."""
import math

import numpy as np
import pytest

from test_oracle_multigrid import colours
from test_oracle_operator import AXIS_PAIRS, axis_modes, dense_matrix, prolongation_matrix
from workloads import DIRICHLET as D, NEUMANN as N

BC_SETS = [(D,) * 6, (N, N, N, N, D, D), (D, N, N, D, N, D), (N, D, D, N, D, N)]


def dense_pb(orc, shape, h, kinds, k2, level=0):
    nx, ny, nz = shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    e = np.zeros((nz, ny, nx))
    for c in range(n):
        e.flat[c] = 1.0
        A[:, c] = orc.pb_apply(e, h, kinds, k2, level).ravel()
        e.flat[c] = 0.0
    return A


@pytest.mark.parametrize("px,py,pz", [
    (AXIS_PAIRS[0], AXIS_PAIRS[0], AXIS_PAIRS[0]),
    (AXIS_PAIRS[1], AXIS_PAIRS[1], AXIS_PAIRS[0]),
    (AXIS_PAIRS[2], AXIS_PAIRS[3], AXIS_PAIRS[1]),
])
@pytest.mark.parametrize("level", [0, 1])
def test_eigenmodes_shifted_by_kappa_squared(orc, px, py, pz, level):
    """The eigenvectors of the Poisson operator, eigenvalues shifted by k2."""
    shape = (8, 6, 10)
    h, k2 = 0.37, 3.7
    kinds = px + py + pz
    s = 1.0 / (2 ** level * h * h)
    rng = np.random.default_rng(17)
    for _ in range(6):
        ks = [int(rng.integers(0, n)) for n in shape]
        vx, tx = axis_modes(*px, shape[0], ks[0])
        vy, ty = axis_modes(*py, shape[1], ks[1])
        vz, tz = axis_modes(*pz, shape[2], ks[2])
        v = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
        mu = s * 4 * (math.sin(tx / 2) ** 2 + math.sin(ty / 2) ** 2 + math.sin(tz / 2) ** 2) + k2
        Av = orc.pb_apply(v, h, kinds, k2, level)
        assert np.linalg.norm(Av - mu * v) <= 1e-13 * mu * np.linalg.norm(v)


@pytest.mark.parametrize("kinds", BC_SETS)
def test_galerkin_product_and_coarse_operator(orc, kinds):
    """R (A + k2 I) P = A_coarse + k2 I (Galerkin: R P = I), and the coarse
    operator the cycle uses, A_1 + 2 k2 I, is exactly twice the operator
    rediscretised at spacing 2h."""
    fine = (8, 4, 8)
    h, k2 = 0.3, 5.0
    P = prolongation_matrix(fine)
    R = P.T / 8
    coarse = tuple(n // 2 for n in fine)
    Af = dense_pb(orc, fine, h, kinds, k2, 0)
    Ac = dense_pb(orc, coarse, h, kinds, k2, 1)
    assert np.abs(R @ Af @ P - Ac).max() <= 1e-12 * np.abs(Ac).max()
    A_cycle = dense_pb(orc, coarse, h, kinds, 2 * k2, 1)
    A_2h = dense_pb(orc, coarse, 2 * h, kinds, k2, 0)
    assert np.abs(A_cycle - 2.0 * A_2h).max() <= 1e-12 * np.abs(A_2h).max()
    # symmetric positive definite, also with Neumann faces only on the sides
    assert np.abs(Af - Af.T).max() == 0.0 and np.linalg.eigvalsh(Af).min() > 0.0


@pytest.mark.parametrize("kinds", BC_SETS)
def test_pb_smoother_equals_dense_gauss_seidel(orc, kinds):
    shape = (4, 6, 4)
    h, k2 = 0.5, 2.5
    A = dense_pb(orc, shape, h, kinds, k2, level=1)
    rng = np.random.default_rng(5)
    n = A.shape[0]
    b = rng.standard_normal(n)
    phi0 = rng.standard_normal(n)
    col = colours(shape)
    x = phi0.copy()
    for c in list(np.flatnonzero(col == 0)) + list(np.flatnonzero(col == 1)):
        x[c] = (b[c] - (A[c] @ x - A[c, c] * x[c])) / A[c, c]
    nx, ny, nz = shape
    got = orc.pb_rbgs_sweep(phi0.reshape(nz, ny, nx), b.reshape(nz, ny, nx), h, kinds, k2, level=1)
    assert np.abs(got.ravel() - x).max() <= 1e-14 * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("kinds", BC_SETS)
def test_pb_cg_matches_dense_solve(orc, kinds):
    shape = (4, 4, 8)
    h, k2 = 1.0, 0.3
    A = dense_pb(orc, shape, h, kinds, k2, level=3)
    b = np.random.default_rng(13).standard_normal(A.shape[0])
    x_ref = np.linalg.solve(A, b)
    nx, ny, nz = shape
    x, it = orc.pb_cg(b.reshape(nz, ny, nx), h, kinds, k2, level=3, rtol=1e-13)
    assert 0 < it <= 2 * A.shape[0]
    assert np.abs(x.ravel() - x_ref).max() <= 1e-11 * np.abs(x_ref).max()


@pytest.mark.parametrize("shape,levels", [((8, 8, 8), 3), ((4, 4, 8), 2)])
@pytest.mark.parametrize("kinds", BC_SETS)
@pytest.mark.parametrize("k2", [0.5, 40.0, 4000.0])
def test_pb_multigrid_matches_dense(orc, shape, levels, kinds, k2):
    h = 1.0 / shape[0]
    A = dense_pb(orc, shape, h, kinds, k2)
    nx, ny, nz = shape
    b = np.random.default_rng(21).standard_normal((nz, ny, nx))
    ref = np.linalg.solve(A, b.ravel()).reshape(nz, ny, nx)
    phi, hist, st = orc.pb_solve(b, h, kinds, levels, k2, rtol=1e-13)
    assert st == 0
    assert all(hist[i + 1] < hist[i] for i in range(len(hist) - 1))
    assert np.abs(phi - ref).max() <= 1e-12 * np.abs(ref).max()


def debye_hueckel_discrete(n, h, k2, g0, gL):
    """Exact solution of the folded 1-D problem (2 psi_k - psi_{k-1} - psi_{k+1}) / h^2
    + k2 psi_k = 0 with Dirichlet values on the two end faces: psi_k = A l^k + B l^-k,
    l + 1/l = 2 + k2 h^2, and the folding's ghost relations psi_{-1} + psi_0 = 2 g0,
    psi_{n-1} + psi_n = 2 gL."""
    a = 1.0 + 0.5 * k2 * h * h
    lam = a + math.sqrt(a * a - 1.0)
    M = np.array([[lam ** -1 + 1.0, lam + 1.0],
                  [lam ** (n - 1) + lam ** n, lam ** -(n - 1) + lam ** -n]])
    A, B = np.linalg.solve(M, [2 * g0, 2 * gL])
    k = np.arange(n)
    return A * lam ** k + B * lam ** -k.astype(float)


def test_planar_debye_hueckel_layer_exact_and_second_order(orc):
    """Dirichlet psi0 at z = 0, 0 at z = L, zero-Neumann sides, no charge: the
    multigrid solution is the discrete closed form, and it converges at second
    order to psi0 sinh(kappa (L - z)) / sinh(kappa L)."""
    kappa, L, psi0 = 6.0, 1.0, 0.8
    kinds = (N, N, N, N, D, D)
    errs = []
    for nz in (16, 32, 64, 128):
        h = L / nz
        b = orc.fold(np.zeros((nz, 4, 4)), h, kinds, (0, 0, 0, 0, psi0, 0.0))
        psi, hist, st = orc.pb_solve(b, h, kinds, 3, kappa ** 2, rtol=1e-13)
        assert st == 0
        exact_d = debye_hueckel_discrete(nz, h, kappa ** 2, psi0, 0.0)
        assert np.abs(psi - exact_d[:, None, None]).max() <= 1e-12 * psi0
        z = (np.arange(nz) + 0.5) * h
        errs.append(np.abs(psi[:, 0, 0] - psi0 * np.sinh(kappa * (L - z)) / math.sinh(kappa * L)).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    # second order: the ratio of successive errors approaches 4 from below
    assert all(3.3 < r < 4.2 for r in ratios) and ratios[-1] > 3.8 and ratios == sorted(ratios), ratios


def gouy_chapman(z, psi0, kappa):
    """The planar double layer of the nonlinear equation psi'' = kappa^2 sinh(psi)
    decaying into the electrolyte: 4 artanh(tanh(psi0 / 4) exp(-kappa z))."""
    return 4.0 * np.arctanh(np.tanh(psi0 / 4.0) * np.exp(-kappa * z))


@pytest.mark.parametrize("psi0", [1.0, 3.0])
def test_gouy_chapman_layer_second_order(orc, psi0):
    """Its restriction to [0, L] solves the problem with Dirichlet values psi0 and
    GC(L) (uniqueness of the monotone problem); the discrete nonlinear solutions
    converge to it at second order."""
    kappa, L = 6.0, 1.0
    kinds = (N, N, N, N, D, D)
    errs = []
    for nz in (32, 64, 128, 256):
        h = L / nz
        b = orc.fold(np.zeros((nz, 4, 4)), h, kinds, (0, 0, 0, 0, psi0, float(gouy_chapman(L, psi0, kappa))))
        psi, hist, st = orc.pb_nl_solve(b, h, kinds, 3, kappa ** 2, inner=2, rtol=1e-12, max_outer=400)
        assert st == 0 and hist[-1] < 1e-12
        z = (np.arange(nz) + 0.5) * h
        errs.append(np.abs(psi[:, 0, 0] - gouy_chapman(z, psi0, kappa)).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.5 < r < 4.3 for r in ratios[1:]), (errs, ratios)


@pytest.mark.parametrize("kinds", BC_SETS[:3])
def test_nonlinear_manufactured_discrete_solution(orc, kinds):
    """b = A psi* + k2 sinh(psi*) for a smooth field psi* with |psi*| up to 2: the
    iteration returns psi*."""
    shape = (16, 16, 16)
    h, k2 = 1.0 / 16, 30.0
    nx, ny, nz = shape
    z, y, x = np.meshgrid(*[(np.arange(n) + 0.5) * h for n in (nz, ny, nx)], indexing="ij")
    psi_star = 2.0 * np.sin(2.1 * x + 0.3) * np.cos(1.3 * y) * np.exp(-0.7 * z) + 0.4 * x * y
    b = orc.apply(psi_star, h, kinds) + k2 * np.sinh(psi_star)
    psi, hist, st = orc.pb_nl_solve(b, h, kinds, 4, k2, inner=2, rtol=1e-13, max_outer=300)
    assert st == 0
    assert np.abs(psi - psi_star).max() <= 1e-10 * np.abs(psi_star).max()


def test_small_potentials_give_the_linear_solution(orc):
    """For psi ~ 1e-3 the nonlinear solution differs from the linear one by the
    cubic term of sinh, about psi^3 / 6 relative to kappa^2 psi."""
    shape = (16, 16, 16)
    h, k2 = 1.0 / 16, 50.0
    kinds = BC_SETS[1]
    f = 1e-3 * k2 * np.random.default_rng(9).standard_normal((16, 16, 16))
    b = orc.fold(f, h, kinds, (0, 0, 0, 0, 1e-3, -1e-3))
    lin, _, st0 = orc.pb_solve(b, h, kinds, 4, k2, rtol=1e-13)
    nl, _, st1 = orc.pb_nl_solve(b, h, kinds, 4, k2, inner=2, rtol=1e-13)
    assert st0 == 0 and st1 == 0
    scale = np.abs(lin).max()
    assert 0 < np.abs(nl - lin).max() <= scale ** 3


def test_kappa_zero_is_poisson(orc):
    shape = (16, 16, 16)
    h = 1.0 / 16
    kinds = BC_SETS[2]
    b = np.random.default_rng(4).standard_normal((16, 16, 16))
    p0, h0, _ = orc.solve(b, h, kinds, 4, rtol=1e-12)
    p1, h1, _ = orc.pb_solve(b, h, kinds, 4, 0.0, rtol=1e-12)
    assert np.array_equal(p0, p1) and np.array_equal(h0, h1)
    # the nonlinear iteration with k2 = 0 is defect correction by V-cycles
    p2, h2, st = orc.pb_nl_solve(b, h, kinds, 4, 0.0, inner=1, rtol=1e-12)
    assert st == 0 and np.abs(p2 - p0).max() <= 1e-11 * np.abs(p0).max()


@pytest.mark.parametrize("kinds", BC_SETS[:3])
def test_nonlinear_residual(orc, kinds):
    """The nonlinear residual b - A psi - kappa^2 sinh(psi): zero (to rounding)
    at a manufactured solution, and at a random potential equal to the
    residual formed with the assembled linear operator (its columns from the
    pinned operator) and the library sinh."""
    shape, h, k2 = (6, 4, 8), 1.0 / 8, 30.0
    nx, ny, nz = shape
    z, y, x = np.meshgrid(*[(np.arange(n) + 0.5) * h for n in (nz, ny, nx)], indexing="ij")
    psi_star = 2.0 * np.sin(2.1 * x + 0.3) * np.cos(1.3 * y) * np.exp(-0.7 * z)
    b = orc.apply(psi_star, h, kinds) + k2 * np.sinh(psi_star)
    r = orc.pb_nl_residual(psi_star, b, h, kinds, k2)
    assert np.abs(r).max() <= 1e-12 * np.abs(b).max()
    A = dense_pb(orc, shape, h, kinds, 0.0)
    psi = 1.5 * np.random.default_rng(41).standard_normal((nz, ny, nx))
    ref = b.ravel() - A @ psi.ravel() - k2 * np.sinh(psi.ravel())
    got = orc.pb_nl_residual(psi, b, h, kinds, k2).ravel()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
