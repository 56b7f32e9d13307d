"""Pins of the oracle's potential gradient and electrostatic force
(Sec. 2.4, "Coulomb force", Eq. ElectrostatForce; validation of Sec. 6.3).

References: exactness of the second-order D3Q19 gradient for quadratic
potentials, of the boundary-layer D3Q7 differences for linear potentials with
consistent boundary data, the force on a sphere in a uniform field (q E for
the charge-conserving density, q (1 + e_rV) E for the paper's q/V density),
and the paper's printed force errors (Tab. ValidClmbForceSubs_PotMaxErr).
"""
import math
import os

import numpy as np
import pytest

from workloads import DIRICHLET as D, NEUMANN as N

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "coulomb_force_diagonal.txt")


def centres(shape, h):
    nx, ny, nz = shape
    ax = [(np.arange(n) + 0.5) * h for n in (nx, ny, nz)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def test_d3q19_gradient_exact_for_quadratics(orc):
    shape, h = (12, 10, 14), 0.37
    X, Y, Z = centres(shape, h)
    phi = 0.3 * X ** 2 - 1.1 * X * Y + 0.7 * Z * Z + 0.2 * Y * Z - 0.45 * X * Z + 2 * X - Y + 0.5
    g = orc.gradient(phi, h, (D,) * 6, (0.0,) * 6)
    ex = np.stack([0.6 * X - 1.1 * Y - 0.45 * Z + 2, -1.1 * X + 0.2 * Z - 1, 1.4 * Z + 0.2 * Y - 0.45 * X])
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.abs(g[inner] - ex[inner]).max() <= 1e-12 * np.abs(ex).max()


def test_d3q19_weights_are_isotropic_and_second_order(orc):
    """A cubic x^3: the D3Q19 x-derivative is 3x^2 + h^2 (every direction
    pair carries the same central difference), and rotating the field by axis
    permutation permutes the gradient."""
    shape, h = (9, 9, 9), 0.5
    X, Y, Z = centres(shape, h)
    g = orc.gradient(X ** 3, h, (D,) * 6, (0.0,) * 6)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.allclose(g[0][inner], (3 * X ** 2 + h * h)[inner], rtol=1e-13, atol=1e-13)
    assert np.abs(g[1][inner]).max() < 1e-12 and np.abs(g[2][inner]).max() < 1e-12
    gz = orc.gradient(Z ** 3, h, (D,) * 6, (0.0,) * 6)
    assert np.allclose(gz[2][inner], np.transpose(g[0], (2, 1, 0))[inner], rtol=1e-13, atol=1e-13)


def linear_case(shape, h, a, kinds):
    """phi = a . x + c with boundary data consistent with it: Dirichlet values
    at the face centres, Neumann outward normal derivatives."""
    X, Y, Z = centres(shape, h)
    c0 = 0.3
    phi = a[0] * X + a[1] * Y + a[2] * Z + c0
    nx, ny, nz = shape
    L = (nx * h, ny * h, nz * h)
    axes = [(np.arange(n) + 0.5) * h for n in shape]
    faces = []
    for fc in range(6):
        ax, hi = fc // 2, fc % 2
        u_ax, v_ax = [(1, 2), (0, 2), (0, 1)][ax]
        V, U = np.meshgrid(axes[v_ax], axes[u_ax], indexing="ij")
        pos = [None, None, None]
        pos[ax] = L[ax] if hi else 0.0
        pos[u_ax], pos[v_ax] = U, V
        if kinds[fc] == D:
            faces.append(a[0] * pos[0] + a[1] * pos[1] + a[2] * pos[2] + c0 + 0 * U)
        else:
            faces.append(np.full(U.shape, a[ax] if hi else -a[ax]))
    return phi, faces


@pytest.mark.parametrize("kinds", [(D, D, N, N, N, N), (N, D, D, N, N, D), (D,) * 6])
def test_gradient_exact_for_linear_fields_with_consistent_boundaries(orc, kinds):
    shape, h, a = (8, 6, 10), 0.25, (1.5, -0.7, 0.35)
    phi, faces = linear_case(shape, h, a, kinds)
    g = orc.gradient(phi, h, kinds, (0.0,) * 6, faces)
    for d in range(3):
        assert np.abs(g[d] - a[d]).max() <= 1e-12, d


@pytest.mark.parametrize("sf", [1, 2, 3])
def test_force_in_a_uniform_field(orc, sf):
    """F = -grad(phi) * (charge carried): q E for the charge-conserving density,
    q (1 + e_rV) E for the paper's q/V density."""
    shape, h = (24, 24, 24), 1.0
    a = (0.4, -0.2, 0.1)
    kinds = (D, D, N, N, D, N)
    phi, faces = linear_case(shape, h, a, kinds)
    c = np.array([[11.3, 12.1, 10.7], [2.0, 12.0, 12.0], [40.0, 5.0, 5.0]])   # inside, cut by x-, outside
    r = np.array([4.5, 3.0, 2.0])
    q = np.array([1.3, -0.8, 1.0])
    F0 = orc.coulomb(phi, h, kinds, (0.0,) * 6, c, r, q, subsample=sf, mode=0, faces=faces)
    E = -np.asarray(a)
    assert np.allclose(F0[:2], q[:2, None] * E[None], rtol=1e-12, atol=0)
    assert not F0[2].any()
    F1 = orc.coulomb(phi, h, kinds, (0.0,) * 6, c, r, q, subsample=sf, mode=1, faces=faces)
    _, wsum = orc.deposit_sub(shape, h, c, r, q, subsample=sf)
    carried = q * wsum * h ** 3 / (4.0 / 3.0 * math.pi * r ** 3)
    assert np.allclose(F1[:2], carried[:2, None] * E[None], rtol=1e-12, atol=0)


def read_golden():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                p = line.split()
                rows.append((int(p[0]), int(p[1]), float(p[2]), p[3], np.array([float(v) for v in p[4:7]]),
                             float(p[7]), float(p[8])))
    return rows


def test_golden_coulomb_force_errors(orc):
    """Homogeneous field (phi = 0 at x = 0, -10 at x = L), sphere at the position
    of maximal volume-mapping error, equal subsampling for potential and
    force: the printed e_rFC is reproduced for the pinned rows, and the force
    error equals the volume-mapping error (the self-field exerts no net force)."""
    rows = read_golden()
    assert len(rows) == 15 and sum(r[3] == "pinned" for r in rows) == 11
    n, kinds, values = 64, (D, D, N, N, N, N), (0.0, -10.0, 0, 0, 0, 0)
    for R, sf, e_paper, status, shift, ev_or, ef_or in rows:
        c = (32 + (0.5 + shift) / sf)[None]
        r, q = np.array([float(R)]), np.array([1.0])
        f, wsum = orc.deposit_sub((n, n, n), 1.0, c, r, q, subsample=sf, mode=1)
        phi, _, st = orc.solve_problem(f, 1.0, kinds, values, 5, rtol=1e-12)
        F = orc.coulomb(phi, 1.0, kinds, values, c, r, q, subsample=sf, mode=1)
        FC = 10.0 / n
        ef = (F[0, 0] - FC) / FC * 100
        ev = (wsum[0] - 4 / 3 * math.pi * R ** 3) / (4 / 3 * math.pi * R ** 3) * 100
        assert abs(ef - ef_or) < 1e-5 and abs(ev - ev_or) < 1e-5
        assert abs(ef - ev) < 0.004, (R, sf, ef, ev)
        assert np.abs(F[0, 1:]).max() < 1e-4 * FC
        if status == "pinned":
            assert abs(ef - e_paper) < 0.006, (R, sf, ef, e_paper)
        else:
            assert abs(ef) < abs(e_paper)


def test_force_of_a_sphere_in_its_own_field_vanishes_by_symmetry(orc):
    """A sphere at the centre of a cube with equal boundaries (a cell vertex:
    the grid, the sub-cells and the sphere share the cube's mirror symmetries):
    the self-force cancels to rounding."""
    n = 32
    c = np.array([[16.0, 16.0, 16.0]])
    r, q = np.array([5.0]), np.array([2.0])
    f, _ = orc.deposit_sub((n, n, n), 1.0, c, r, q, subsample=2)
    phi, _, _ = orc.solve_problem(f, 1.0, (D,) * 6, (0.0,) * 6, 4, rtol=1e-12)
    F = orc.coulomb(phi, 1.0, (D,) * 6, (0.0,) * 6, c, r, q, subsample=2)
    g = orc.gradient(phi, 1.0, (D,) * 6, (0.0,) * 6)
    assert np.abs(F).max() <= 1e-12 * q[0] * np.abs(g).max()


# ---- adjoint of the force ------------------------------------------------------
def spheres_near_walls():
    c = np.array([[6.3, 7.1, 5.2], [1.2, 8.0, 9.5], [14.6, 3.3, 14.4], [8.0, 8.0, 1.0]])
    r = np.array([3.4, 2.6, 2.9, 2.2])
    q = np.array([1.3, -0.7, 0.9, 2.0])
    return c, r, q


@pytest.mark.parametrize("kinds", [(D, D, N, N, N, N), (N, D, D, N, D, N)])
def test_force_adjoint_is_the_transpose(orc, kinds):
    """<mu, psi> equals sum_s gF_s . (F_s(psi) - F_s(0)) for random psi: the
    scatter is the exact transpose of the (linear part of the) force map,
    boundary-layer cells included."""
    shape, h = (16, 12, 16), 0.8
    values = (0.3, -0.2, 0.1, 0.4, -0.5, 0.2)
    c, r, q = spheres_near_walls()
    c, r = c * h, r * h
    rng = np.random.default_rng(1)
    gF = rng.standard_normal((4, 3))
    psi = rng.standard_normal((16, 12, 16))
    for sf, mode in ((1, 0), (2, 1), (3, 0)):
        mu, direct = orc.coulomb_adjoint(np.zeros_like(psi), h, kinds, values, c, r, q, gF, sf, mode)
        F1 = orc.coulomb(psi, h, kinds, values, c, r, q, sf, mode)
        F0 = orc.coulomb(np.zeros_like(psi), h, kinds, values, c, r, q, sf, mode)
        lhs = float(np.vdot(mu, psi))
        rhs_ = float(np.sum(gF * (F1 - F0)))
        assert abs(lhs - rhs_) <= 1e-12 * max(1.0, abs(rhs_))
        # direct term at fixed phi: gF_s . F_s / q_s
        Fp = orc.coulomb(psi, h, kinds, values, c, r, q, sf, mode)
        _, d2 = orc.coulomb_adjoint(psi, h, kinds, values, c, r, q, gF, sf, mode)
        assert np.allclose(d2, np.sum(gF * Fp, axis=1) / q, rtol=1e-12, atol=1e-14)


def test_force_charge_gradient_by_finite_differences(orc):
    """dL/dq for L = sum_s gF_s . F_s(q) through deposition, solve and force:
    direct term + charge gradient of lambda = A^-1 mu, against central
    differences of the full forward map (affine in every q_t... quadratic in q
    overall, so central differences are exact up to solver tolerance)."""
    shape, h, eps = (16, 16, 16), 1.0, 0.7
    kinds, values = (D, D, N, N, N, N), (0.0, -2.0, 0, 0, 0, 0)
    c, r, q = spheres_near_walls()
    gF = np.random.default_rng(2).standard_normal((4, 3))
    sf_d, sf_f, mode = 2, 3, 1

    def forces(qv):
        f, _ = orc.deposit_sub(shape, h, c, r, qv, eps, subsample=sf_d, mode=mode)
        phi, _, _ = orc.solve_problem(f, h, kinds, values, 3, rtol=1e-14, max_cycles=80)
        return orc.coulomb(phi, h, kinds, values, c, r, qv, sf_f, mode), phi

    F, phi = forces(q)
    mu, direct = orc.coulomb_adjoint(phi, h, kinds, values, c, r, q, gF, sf_f, mode)
    lam, _, _ = orc.adjoint(mu, h, kinds, 3, rtol=1e-14, max_cycles=80)
    grad = direct + orc.dq_sub(lam, h, c, r, eps, subsample=sf_d, mode=mode)
    step = 1e-3
    for t in range(4):
        qp, qm = q.copy(), q.copy()
        qp[t] += step
        qm[t] -= step
        fd = (np.sum(gF * forces(qp)[0]) - np.sum(gF * forces(qm)[0])) / (2 * step)
        assert abs(fd - grad[t]) <= 1e-8 * max(1.0, abs(grad[t])), (t, fd, grad[t])
