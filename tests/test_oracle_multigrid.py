"""Pins of the oracle's smoother, coarsest-grid CG, V-cycle and solve.

Independent references: dense linear algebra (numpy), an explicit sparse
Galerkin multigrid cycle written here with scipy (its own transfer matrices,
Galerkin products R A P and colour-block Gauss-Seidel), closed-form discrete
solutions and the second-order accuracy of the scheme.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from workloads import DIRICHLET as D, NEUMANN as N

from test_oracle_operator import dense_matrix, prolongation_matrix

BC_SETS = [(D,) * 6, (N, N, N, N, D, D), (D, N, N, D, N, D), (N, D, D, N, D, N)]


def colours(shape):
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i + j + k) % 2).ravel()


@pytest.mark.parametrize("kinds", BC_SETS)
def test_rbgs_equals_dense_gauss_seidel(orc, kinds):
    """One red-black sweep = one Gauss-Seidel sweep over the unknowns ordered
    red first, then black (Sec. 5.3: checker-board reordering)."""
    shape = (4, 6, 4)
    h = 0.5
    A = dense_matrix(orc, shape, h, kinds, level=1)
    rng = np.random.default_rng(3)
    n = A.shape[0]
    b = rng.standard_normal(n)
    phi0 = rng.standard_normal(n)
    col = colours(shape)
    order = list(np.flatnonzero(col == 0)) + list(np.flatnonzero(col == 1))
    x = phi0.copy()
    for c in order:
        x[c] = (b[c] - (A[c] @ x - A[c, c] * x[c])) / A[c, c]
    nx, ny, nz = shape
    got = orc.rbgs_sweep(phi0.reshape(nz, ny, nx), b.reshape(nz, ny, nx), h, kinds, level=1)
    assert np.abs(got.ravel() - x).max() <= 1e-14 * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("kinds", BC_SETS)
def test_cg_matches_dense_solve(orc, kinds):
    shape = (4, 4, 8)
    h = 1.0
    A = dense_matrix(orc, shape, h, kinds, level=3)
    b = np.random.default_rng(11).standard_normal(A.shape[0])
    x_ref = np.linalg.solve(A, b)
    nx, ny, nz = shape
    x, it = orc.cg(b.reshape(nz, ny, nx), h, kinds, level=3, rtol=1e-13)
    assert 0 < it <= 2 * A.shape[0]
    assert np.abs(x.ravel() - x_ref).max() <= 1e-11 * np.abs(x_ref).max()


class SparseGalerkinMG:
    """Explicit-matrix multigrid: A_{l+1} = R A_l P with R = P^T/8, P = piecewise
    constant; colour-block Gauss-Seidel (red cells couple only to black ones, so
    each colour is one diagonal solve); dense solve on the coarsest level."""

    def __init__(self, A0, shape, levels, nu1=2, nu2=2, omega=2.0):
        self.A, self.P, self.col, self.shapes = [A0.tocsr()], [], [], [shape]
        for l in range(levels - 1):
            P = sp.csr_matrix(prolongation_matrix(self.shapes[-1]))
            self.P.append(P)
            self.A.append((P.T / 8 @ self.A[-1] @ P).tocsr())
            self.shapes.append(tuple(n // 2 for n in self.shapes[-1]))
        self.col = [colours(s) for s in self.shapes]
        self.dense_coarse = self.A[-1].toarray()
        self.nu1, self.nu2, self.omega, self.L = nu1, nu2, omega, levels

    def smooth(self, l, x, b):
        A = self.A[l]
        d = A.diagonal()
        for c in (0, 1):
            m = self.col[l] == c
            r = b - A @ x + d * x
            x[m] = r[m] / d[m]
        return x

    def cycle(self, l, x, b):
        if l == self.L - 1:
            return x + np.linalg.solve(self.dense_coarse, b - self.A[l] @ x)
        for _ in range(self.nu1):
            x = self.smooth(l, x, b)
        r = b - self.A[l] @ x
        bc = self.P[l].T @ r / 8
        e = self.cycle(l + 1, np.zeros(bc.shape[0]), bc)
        x = x + self.omega * (self.P[l] @ e)
        for _ in range(self.nu2):
            x = self.smooth(l, x, b)
        return x


@pytest.mark.parametrize("kinds", BC_SETS)
def test_vcycle_matches_explicit_sparse_galerkin(orc, kinds):
    shape = (16, 8, 16)
    h = 1.0 / 16
    levels = 3
    nx, ny, nz = shape
    A0 = sp.csr_matrix(dense_matrix(orc, shape, h, kinds))
    mg = SparseGalerkinMG(A0, shape, levels)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(A0.shape[0])
    x = np.zeros_like(b)
    phi = np.zeros((nz, ny, nx))
    for cyc in range(1, 5):
        x = mg.cycle(0, x, b)
        phi, hist, st = orc.solve(b.reshape(nz, ny, nx), h, kinds, levels, rtol=0.0,
                                  max_cycles=1, phi0=phi, cg_rtol=1e-15, cg_maxit=10000)
        assert np.abs(phi.ravel() - x).max() <= 1e-11 * np.abs(x).max(), cyc


@pytest.mark.parametrize("shape,kinds", [((8, 8, 8), (D, N, N, D, N, D)),
                                         ((4, 4, 8), (N, N, D, N, N, N)),
                                         ((8, 8, 8), (D,) * 6)])
def test_solve_matches_dense(orc, shape, kinds):
    h = 0.1
    nx, ny, nz = shape
    rng = np.random.default_rng(17)
    f = rng.standard_normal((nz, ny, nx))
    values = tuple(rng.standard_normal(6))
    b = orc.fold(f, h, kinds, values)
    A = dense_matrix(orc, shape, h, kinds)
    x_ref = np.linalg.solve(A, b.ravel())
    phi, hist, st = orc.solve(b, h, kinds, levels=2, rtol=1e-13)
    assert st == 0
    assert np.abs(phi.ravel() - x_ref).max() <= 1e-11 * np.abs(x_ref).max()


def c_of_h(h):
    """Discrete amplitude: f = 3 pi^2 prod sin(pi x_d) is the (1,1,1) eigenvector
    of the folded all-Dirichlet operator with eigenvalue 12 sin^2(pi h/2)/h^2,
    so the discrete solution is (pi^2 h^2 / (4 sin^2(pi h / 2))) prod sin."""
    return (math.pi * h) ** 2 / (4.0 * math.sin(math.pi * h / 2) ** 2)


def test_sine_problem_closed_form_and_second_order(orc):
    errs = {}
    for n in (16, 32, 64):
        h = 1.0 / n
        shape = (n, n, n)
        f = W.sine_rhs(shape, h)
        b = orc.fold(f, h, (D,) * 6, (0.0,) * 6)
        phi, hist, st = orc.solve(b, h, (D,) * 6, levels=int(math.log2(n)) - 1, rtol=1e-13)
        assert st == 0
        ex = W.sine_exact(shape, h)
        assert np.abs(phi - c_of_h(h) * ex).max() <= 1e-12
        errs[n] = np.abs(phi - ex).max()
    assert abs(errs[32] - 8.0067e-4) < 1e-7
    # O(h^2): halving h divides the error by 4 (Sec. 2.4)
    assert 3.9 < errs[16] / errs[32] < 4.05
    assert 3.95 < errs[32] / errs[64] < 4.02


def test_c1_workload_cycles_and_rate(orc):
    w = W.C1
    f = W.sine_rhs(w.shape, w.h)
    phi, hist, st = orc.solve_problem(f, w.h, w.kinds, w.values, w.levels)
    assert st == 0 and hist[-1] < 1e-10 <= hist[-2]
    rates = hist[1:] / hist[:-1]
    assert (rates < 1).all()                   # every cycle contracts
    assert 0.08 < rates[-4:].mean() < 0.16     # V(2,2), omega = 2
    assert len(hist) - 1 <= 14


def test_correction_factor_two_and_vcycle_11(orc):
    """Sec. 3: without magnifying the correction the cycle converges slowly;
    V(1,1) is much weaker than V(2,2)."""
    w = W.C1
    b = orc.fold(W.sine_rhs(w.shape, w.h), w.h, w.kinds, w.values)
    def rate(**kw):
        _, hist, _ = orc.solve(b, w.h, w.kinds, w.levels, rtol=0.0, max_cycles=10, **kw)
        return (hist[-1] / hist[-4]) ** (1 / 3)
    r2 = rate()
    r1 = rate(omega=1.0)
    r11 = rate(nu1=1, nu2=1)
    assert r2 < 0.16 and r1 > 0.5 and r11 > 0.5


def test_status_codes(orc):
    w = W.C1
    b = orc.fold(W.sine_rhs(w.shape, w.h), w.h, w.kinds, w.values)
    phi, hist, st = orc.solve(b, w.h, w.kinds, w.levels, max_cycles=2)
    assert st == orc.E_NOCONV and len(hist) == 3
    bad = b.copy()
    bad[3, 4, 5] = np.nan
    phi, hist, st = orc.solve(bad, w.h, w.kinds, w.levels)
    assert st == orc.E_NONFINITE
    phi, hist, st = orc.solve(np.zeros_like(b), w.h, w.kinds, w.levels, phi0=np.ones_like(b))
    assert st == 0 and len(hist) == 1 and not phi.any()


def test_initial_guess_is_used(orc):
    w = W.C1
    b = orc.fold(W.sine_rhs(w.shape, w.h), w.h, w.kinds, w.values)
    phi, hist, st = orc.solve(b, w.h, w.kinds, w.levels, rtol=1e-12)
    phi2, hist2, st2 = orc.solve(b, w.h, w.kinds, w.levels, rtol=1e-10, phi0=phi)
    assert st2 == 0 and len(hist2) == 1


def test_fp32_refinement_reaches_fp64_solution(orc):
    w = W.C2.scaled((32, 32, 32), levels=3, n_spheres=6)
    s = W.workload_spheres(w)
    f, _ = orc.deposit(w.shape, w.h, s.centers, s.radii, s.charges)
    b = orc.fold(f, w.h, w.kinds, w.values)
    phi64, h64, st = orc.solve(b, w.h, w.kinds, w.levels, rtol=1e-12)
    phi32, h32, st32 = orc.solve_ir(b, w.h, w.kinds, w.levels, inner=2, rtol=1e-10)
    assert st32 == 0 and h32[-1] < 1e-10
    assert (h32[1:] < h32[:-1]).all()
    assert np.abs(phi32 - phi64).max() <= 1e-8 * np.abs(phi64).max()
    # two FP32 cycles per outer step contract at least as much as one FP64 cycle
    assert len(h32) <= len(h64)


def test_adjoint_dot_product_identity(orc):
    """<w, A^{-1} b> = <A^{-1} w, b>: the adjoint solve of the symmetric operator."""
    shape = (16, 16, 16)
    kinds = (N, N, D, N, D, D)
    rng = np.random.default_rng(23)
    b = rng.standard_normal((16, 16, 16))
    wv = rng.standard_normal((16, 16, 16))
    x, _, _ = orc.solve(b, 1.0, kinds, 3, rtol=1e-13)
    lam, _, _ = orc.adjoint(wv, 1.0, kinds, 3, rtol=1e-13)
    lhs, rhs = np.vdot(wv, x), np.vdot(lam, b)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
