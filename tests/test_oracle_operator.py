"""Pins of the oracle's operator, boundary folding and grid transfers.

None of these checks re-types the oracle's formulas: they test it against
closed-form eigenpairs, exact solutions of the continuous problem, algebraic
identities (symmetry, definiteness, Galerkin products) and lattice geometry.
"""
import itertools
import math

import numpy as np
import pytest

from workloads import DIRICHLET as D, NEUMANN as N

AXIS_PAIRS = [(D, D), (N, N), (D, N), (N, D)]


def axis_modes(kind_lo, kind_hi, n, k):
    """1-D eigenvector of the folded second difference and its angle theta.

    Dirichlet at a face makes the mode odd about that face, Neumann even; the
    eigenvalue of (1/h^2)[-1 2 -1] with folding is (4/h^2) sin^2(theta/2)."""
    x = np.arange(n) + 0.5
    if (kind_lo, kind_hi) == (D, D):
        th = (k + 1) * math.pi / n
        return np.sin(th * x), th
    if (kind_lo, kind_hi) == (N, N):
        th = k * math.pi / n
        return np.cos(th * x), th
    if (kind_lo, kind_hi) == (D, N):
        th = (k + 0.5) * math.pi / n
        return np.sin(th * x), th
    th = (k + 0.5) * math.pi / n
    return np.cos(th * x), th


@pytest.mark.parametrize("px,py,pz", [
    (AXIS_PAIRS[0], AXIS_PAIRS[0], AXIS_PAIRS[0]),
    (AXIS_PAIRS[1], AXIS_PAIRS[1], AXIS_PAIRS[0]),
    (AXIS_PAIRS[2], AXIS_PAIRS[3], AXIS_PAIRS[1]),
    (AXIS_PAIRS[3], AXIS_PAIRS[0], AXIS_PAIRS[2]),
    (AXIS_PAIRS[1], AXIS_PAIRS[2], AXIS_PAIRS[3]),
])
@pytest.mark.parametrize("level", [0, 2])
def test_eigenmodes_closed_form(orc, px, py, pz, level):
    shape = (8, 6, 10)   # nx, ny, nz
    h = 0.37
    kinds = px + py + pz
    s = 1.0 / (2 ** level * h * h)
    rng = np.random.default_rng(7)
    for _ in range(6):
        ks = [int(rng.integers(0, n)) for n in shape]
        vx, tx = axis_modes(*px, shape[0], ks[0])
        vy, ty = axis_modes(*py, shape[1], ks[1])
        vz, tz = axis_modes(*pz, shape[2], ks[2])
        v = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
        mu = s * 4 * (math.sin(tx / 2) ** 2 + math.sin(ty / 2) ** 2 + math.sin(tz / 2) ** 2)
        if mu == 0.0:
            continue
        Av = orc.apply(v, h, kinds, level)
        assert np.linalg.norm(Av - mu * v) <= 1e-13 * mu * np.linalg.norm(v)


def dense_matrix(orc, shape, h, kinds, level=0):
    nx, ny, nz = shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    e = np.zeros((nz, ny, nx))
    for c in range(n):
        e.flat[c] = 1.0
        A[:, c] = orc.apply(e, h, kinds, level).ravel()
        e.flat[c] = 0.0
    return A


@pytest.mark.parametrize("kinds", [
    (D,) * 6, (N, N, N, N, D, D), (D, N, N, D, N, D), (N, D, D, N, D, N), (N, N, N, N, N, D)])
def test_symmetric_positive_definite(orc, kinds):
    shape = (4, 4, 6)
    A = dense_matrix(orc, shape, 0.5, kinds)
    assert np.abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0.0
    # 7-point structure: at most 7 non-zeros per row
    assert (np.count_nonzero(A, axis=1) <= 7).all()


def test_all_neumann_is_singular(orc):
    A = dense_matrix(orc, (4, 4, 4), 1.0, (N,) * 6)
    assert abs(np.linalg.eigvalsh(A).min()) < 1e-12
    assert np.abs(A @ np.ones(64)).max() < 1e-14


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_profile_dirichlet_pair_exact(orc, axis):
    """phi = g_lo + (g_hi - g_lo) t is harmonic; with Dirichlet values on the
    two faces normal to `axis` and zero-Neumann elsewhere it is the exact
    solution, and the finite-volume scheme with folded BCs reproduces it at
    the cell centres."""
    shape = (12, 8, 10)
    h = 0.25
    g_lo, g_hi = -0.7, 1.3
    kinds = [N] * 6
    values = [0.0] * 6
    kinds[2 * axis], kinds[2 * axis + 1] = D, D
    values[2 * axis], values[2 * axis + 1] = g_lo, g_hi
    n_ax = shape[axis]
    t = (np.arange(n_ax) + 0.5) / n_ax
    prof = g_lo + (g_hi - g_lo) * t
    nx, ny, nz = shape
    phi = np.broadcast_to(
        prof[None, None, :] if axis == 0 else prof[None, :, None] if axis == 1 else prof[:, None, None],
        (nz, ny, nx)).copy()
    b = orc.fold(np.zeros((nz, ny, nx)), h, kinds, values)
    r = orc.residual(phi, b, h, kinds)
    assert np.abs(r).max() <= 1e-12 * np.abs(b).max()
    sol, hist, st = orc.solve(b, h, kinds, levels=2, rtol=1e-13)
    assert st == 0
    assert np.abs(sol - phi).max() <= 1e-12


@pytest.mark.parametrize("lo_kind", [D, N])
def test_linear_profile_neumann_sign(orc, lo_kind):
    """phi = a x with an outward normal derivative prescribed on a Neumann face:
    the outward derivative is -a at x = 0 and +a at x = L."""
    shape = (16, 4, 4)
    h = 0.5
    a = 0.8
    L = shape[0] * h
    x = (np.arange(shape[0]) + 0.5) * h
    phi = np.broadcast_to(a * x[None, None, :], (4, 4, 16)).copy()
    kinds = [N] * 6
    values = [0.0] * 6
    if lo_kind == D:      # phi(0) = 0, outward derivative at x = L is +a
        kinds[0], values[0] = D, 0.0
        kinds[1], values[1] = N, a
    else:                 # outward derivative at x = 0 is -a, phi(L) = a L
        kinds[0], values[0] = N, -a
        kinds[1], values[1] = D, a * L
    b = orc.fold(np.zeros_like(phi), h, kinds, values)
    r = orc.residual(phi, b, h, kinds)
    assert np.abs(r).max() <= 1e-12 * np.abs(b).max()


def prolongation_matrix(fine_shape):
    nx, ny, nz = fine_shape
    cnx, cny, cnz = nx // 2, ny // 2, nz // 2
    P = np.zeros((nx * ny * nz, cnx * cny * cnz))
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        P[(k * ny + j) * nx + i, ((k // 2) * cny + j // 2) * cnx + i // 2] = 1.0
    return P


def test_transfers(orc):
    fine = (8, 4, 6)
    nx, ny, nz = fine
    P = prolongation_matrix(fine)
    nf, nc = P.shape
    # the oracle's prolongation (omega = 1 on a zero fine field) is P
    Pm = np.zeros_like(P)
    for c in range(nc):
        e = np.zeros((nz // 2, ny // 2, nx // 2))
        e.flat[c] = 1.0
        Pm[:, c] = orc.prolong_add(np.zeros((nz, ny, nx)), e, 1.0).ravel()
    assert np.array_equal(Pm, P)
    # the oracle's restriction is the averaging R = P^T / 8
    Rm = np.zeros((nc, nf))
    for c in range(nf):
        e = np.zeros((nz, ny, nx))
        e.flat[c] = 1.0
        Rm[:, c] = orc.restrict(e).ravel()
    assert np.array_equal(Rm, P.T / 8)
    assert np.array_equal(Rm @ P, np.eye(nc))
    assert np.allclose(Rm @ np.ones(nf), 1.0) and np.allclose(P @ np.ones(nc), 1.0)


@pytest.mark.parametrize("kinds", [(D,) * 6, (N, N, N, N, D, D), (D, N, N, D, N, D), (N, D, D, N, D, N)])
def test_galerkin_coarse_operator_closed_form(orc, kinds):
    """R A_l P equals the oracle's level-(l+1) operator, s_{l+1} times the
    integer stencil with the same per-face centre entries (Sec. 3: Galerkin
    coarsening keeps the seven-point stencil)."""
    fine = (8, 4, 8)
    h = 0.3
    P = prolongation_matrix(fine)
    R = P.T / 8
    for level in (0, 1):
        Af = dense_matrix(orc, fine, h, kinds, level)
        coarse = tuple(n // 2 for n in fine)
        Ac = dense_matrix(orc, coarse, h, kinds, level + 1)
        Ag = R @ Af @ P
        assert np.abs(Ag - Ac).max() <= 1e-12 * np.abs(Ac).max()
    # Galerkin coarsening of the operator discretised at spacing h gives exactly
    # twice the operator discretised at 2h (why Sec. 3 magnifies the correction
    # by about 2)
    A_h = dense_matrix(orc, fine, h, kinds, 0)
    A_2h = dense_matrix(orc, tuple(n // 2 for n in fine), 2 * h, kinds, 0)
    assert np.abs(R @ A_h @ P - 2.0 * A_2h).max() <= 1e-12 * np.abs(A_2h).max()


def test_fold_terms(orc):
    """Right-hand side adaptation: with phi = constant g in a cube whose six faces
    are all Dirichlet g, A phi = b holds exactly for f = 0 (one cell checks every
    corner, edge and face contribution at once)."""
    g = 2.5
    h = 0.125
    shape = (5, 4, 3)
    nx, ny, nz = shape
    phi = np.full((nz, ny, nx), g)
    b = orc.fold(np.zeros((nz, ny, nx)), h, (D,) * 6, (g,) * 6)
    assert np.allclose(orc.apply(phi, h, (D,) * 6), b, rtol=1e-14, atol=0)


def multilinear(coef, x, y, z):
    """phi = c0 + c1 x + c2 y + c3 z + c4 xy + c5 yz + c6 xz + c7 xyz and its
    three partial derivatives.  phi is linear along every axis, so every second
    difference of the seven-point stencil vanishes and a boundary ghost value
    extrapolated linearly through the face (Sec. 2.4) is exact."""
    c = coef
    phi = c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z + c[6] * x * z + c[7] * x * y * z
    dx = c[1] + c[4] * y + c[6] * z + c[7] * y * z
    dy = c[2] + c[4] * x + c[5] * z + c[7] * x * z
    dz = c[3] + c[5] * y + c[6] * x + c[7] * x * y
    return phi, dx, dy, dz


def face_data(coef, shape, h, kinds):
    """Per-cell boundary values of a multilinear potential at the face centres
    of the boundary cells: phi there on Dirichlet faces, the outward normal
    derivative on Neumann faces.  Arrays x faces (nz, ny), y faces (nz, nx),
    z faces (ny, nx), first index slowest."""
    nx, ny, nz = shape
    L = [nx * h, ny * h, nz * h]
    cx, cy, cz = ((np.arange(n) + 0.5) * h for n in shape)
    out = []
    for fc in range(6):
        ax, hi = fc // 2, fc % 2
        pos = L[ax] if hi else 0.0
        if ax == 0:
            Z, Y = np.meshgrid(cz, cy, indexing="ij")
            phi, *d = multilinear(coef, np.full_like(Z, pos), Y, Z)
        elif ax == 1:
            Z, X = np.meshgrid(cz, cx, indexing="ij")
            phi, *d = multilinear(coef, X, np.full_like(Z, pos), Z)
        else:
            Y, X = np.meshgrid(cy, cx, indexing="ij")
            phi, *d = multilinear(coef, X, Y, np.full_like(Y, pos))
        outward = d[ax] if hi else -d[ax]
        out.append(phi if kinds[fc] == D else outward)
    return out


@pytest.mark.parametrize("kinds", [(D,) * 6, (D, N, N, D, D, N), (N, D, D, N, N, D), (N, N, N, N, D, D),
                                   (D, D, N, N, N, N)])
def test_fold_field_reproduces_multilinear_potential(orc, kinds):
    """Per-cell boundary values (Sec. 2.4 "Boundary conditions"; the validation
    of Sec. 6.3 sets them per boundary cell): a multilinear potential with its
    face-centre values on Dirichlet faces and its face-centre outward
    derivatives on Neumann faces (non-constant on every face) satisfies the
    folded finite-volume system exactly.  The faces are non-square, so a swap
    of the two in-face indices, a wrong face or a wrong Neumann sign leaves a
    residual of the order of the boundary terms."""
    shape = (6, 10, 8)
    nx, ny, nz = shape
    h = 0.3
    coef = np.random.default_rng(401).uniform(-1.0, 1.0, 8)
    cx, cy, cz = ((np.arange(n) + 0.5) * h for n in shape)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    phi, _, _, _ = multilinear(coef, X, Y, Z)
    faces = face_data(coef, shape, h, kinds)
    for a in faces:   # every face array varies over the face
        assert np.ptp(a) > 0.1
    b = orc.fold_field(np.zeros((nz, ny, nx)), h, kinds, [0.0] * 6, faces)
    r = orc.residual(phi, b, h, kinds)
    assert np.abs(r).max() <= 1e-12 * np.abs(b).max()
    # the transposed arrays (u and v swapped) must not satisfy it
    tr = [a.T.copy().reshape(a.shape) for a in faces]
    r_bad = orc.residual(phi, orc.fold_field(np.zeros((nz, ny, nx)), h, kinds, [0.0] * 6, tr), h, kinds)
    assert np.abs(r_bad).max() > 1e-3 * np.abs(b).max()
    # and the multigrid solve of the folded system returns the potential itself
    sol, hist, st = orc.solve(b, h, kinds, levels=2, rtol=1e-13)
    assert st == 0
    assert np.abs(sol - phi).max() <= 1e-11 * np.abs(phi).max()


@pytest.mark.parametrize("kinds", [(D,) * 6, (N, D, D, N, D, N)])
def test_fold_field_constant_arrays_equal_constant_fold(orc, kinds):
    """Arrays holding each face's constant value give the constant fold bit for
    bit (same terms, added in the same face order)."""
    shape = (6, 10, 8)
    nx, ny, nz = shape
    h = 0.7
    values = [0.3, -1.1, 2.5, 0.0, -0.4, 1.7]
    f = np.random.default_rng(402).standard_normal((nz, ny, nx))
    shapes = [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2
    faces = [np.full(sh, v) for sh, v in zip(shapes, values)]
    b_const = orc.fold(f, h, kinds, values)
    b_field = orc.fold_field(f, h, kinds, [99.0] * 6, faces)   # the constants must not be used
    assert np.array_equal(b_const, b_field)
    # a face without an array falls back to its constant value
    mixed = [None, faces[1], None, faces[3], faces[4], None]
    assert np.array_equal(orc.fold_field(f, h, kinds, values, mixed), b_const)


def test_diagonal_matches_the_paper_centres_and_the_operator(orc):
    """d_c at boundary cells (Sec. 5.3, the stencil's boundary adaptation):
    one Dirichlet face gives the centre 7, one Neumann face 5, interior 6, and
    every face adds its own +1 / -1 (corners of three faces: 9 or 3).  The
    diagonal also equals h^2 times the operator's dense diagonal, read off by
    applying the operator to unit vectors."""
    shape = (4, 6, 4)
    h = 0.5
    dd = [D] * 6
    nn = [N] * 6
    assert orc.diag_at(shape, dd, 1, 2, 1) == 6
    assert orc.diag_at(shape, dd, 0, 2, 1) == 7
    assert orc.diag_at(shape, nn, 0, 2, 1) == 5
    assert orc.diag_at(shape, dd, 0, 0, 0) == 9
    assert orc.diag_at(shape, nn, 3, 5, 3) == 3
    mixed = [D, N, N, D, D, N]
    nx, ny, nz = shape
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        e = np.zeros((nz, ny, nx))
        e[k, j, i] = 1.0
        col = orc.apply(e, h, mixed, 0)
        assert orc.diag_at(shape, mixed, i, j, k) == round(col[k, j, i] * h * h)
        assert col[k, j, i] * h * h == float(orc.diag_at(shape, mixed, i, j, k))


def test_norm2_against_numpy(orc):
    """The Euclidean norm: numpy's on random vectors, exact on a Pythagorean
    triple, zero on the zero vector."""
    rng = np.random.default_rng(3)
    for n in (1, 7, 4096, 100_000):
        v = rng.standard_normal(n) * 10.0 ** rng.integers(-3, 4)
        assert abs(orc.norm2(v) - np.linalg.norm(v)) <= 1e-14 * np.linalg.norm(v)
    assert orc.norm2(np.array([3.0, 4.0, 12.0])) == 13.0
    assert orc.norm2(np.zeros(9)) == 0.0
