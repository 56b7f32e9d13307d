"""GPU parity of the Poisson-Boltzmann extension (the equation the paper's
outlook names, Sec. 9; the reading and iteration are those of the oracle's
Poisson-Boltzmann section).

Linear (Debye-Hueckel) operator -Lap + kappa^2: per-cycle iterates and solves
against the oracle at the FP64 bar (1e-12 of the field), FP32 refinement to
the FP64 solution, the adjoint solve.  Nonlinear -Lap + kappa^2 sinh: the
shifted chord iteration against the oracle's (same outer steps, same
solution), and the planar Gouy-Chapman double layer.  kappa ranges from
kappa h = 0.03 (Poisson-like) to kappa h = 2 (reaction-dominated)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1410_6609_amd as pkg
from test_gpu_parity import CASES, DEV, ids, log_case, rhs, to_dev
from workloads import DIRICHLET as D, NEUMANN as N

pytestmark = pytest.mark.gpu

KAPPA_H = [0.03, 0.4, 2.0]


def pb_solver(shape, levels, kinds, values, k2, h=None, **opt):
    h = 1.0 / shape[0] if h is None else h
    return pkg.Solver(shape, h, list(zip(kinds, values)), pkg.Options(levels=levels, kappa2=k2, **opt), device=DEV)


@pytest.mark.parametrize("kh", KAPPA_H)
@pytest.mark.parametrize("case", CASES, ids=ids)
def test_linear_pb_cycles_and_solve_match_oracle(case, kh):
    shape, levels, kinds, values = case
    h = 1.0 / shape[0]
    k2 = (kh / h) ** 2
    log_case("linear pb", shape, kh)
    s = pb_solver(shape, levels, kinds, values, k2)
    f = rhs(shape, 31)
    b = oracle.fold(f, h, kinds, values)
    # three cycles from zero, compared cycle by cycle through the history and at the end
    phi, st = s.solve(to_dev(f), rtol=0.0, max_cycles=3, check=False)
    ref, hist, _ = oracle.pb_solve(b, h, kinds, levels, k2, rtol=0.0, max_cycles=3)
    assert st.cycles == 3
    assert np.abs(phi.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.allclose(np.array(s.history()), hist, rtol=1e-8, atol=1e-14)
    # solve to 1e-10: same cycle count
    phi, st = s.solve(to_dev(f), rtol=1e-10)
    ref, hist, ost = oracle.pb_solve(b, h, kinds, levels, k2, rtol=1e-10)
    assert ost == 0 and st.rel_res < 1e-10 and st.cycles == len(hist) - 1
    assert np.abs(phi.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("kh", KAPPA_H[1:])
@pytest.mark.parametrize("case", CASES[1::2], ids=ids)
def test_linear_pb_fp32_refinement_and_adjoint(case, kh):
    shape, levels, kinds, values = case
    h = 1.0 / shape[0]
    k2 = (kh / h) ** 2
    log_case("linear pb ir/adjoint", shape, kh)
    f = to_dev(rhs(shape, 32))
    s64 = pb_solver(shape, levels, kinds, values, k2)
    s32 = pb_solver(shape, levels, kinds, values, k2, precision=pkg.FP32_IR)
    p64, st64 = s64.solve(f, rtol=1e-10)
    p32, st32 = s32.solve(f, rtol=1e-10)
    assert st64.rel_res < 1e-10 and st32.rel_res < 1e-10
    _, rel = s64.residual(p32, f, want_field=False)
    assert rel < 1e-10
    assert (p32 - p64).abs().max().item() <= 1e-9 * p64.abs().max().item()
    # adjoint: the operator is symmetric, lambda = A^-1 g with homogeneous faces
    g = rhs(shape, 33)
    lam, _, _, ast = s64.adjoint(to_dev(g), None, None, rtol=1e-10)
    ref, hist, _ = oracle.pb_solve(g, h, kinds, levels, k2, rtol=0.0, max_cycles=ast.cycles)
    assert np.abs(lam.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("amp", [0.5, 2.5])
@pytest.mark.parametrize("case", CASES[:3], ids=ids)
def test_nonlinear_pb_matches_oracle(case, amp):
    shape, levels, kinds, values = case
    h = 1.0 / shape[0]
    k2 = (0.5 / h) ** 2
    log_case("nonlinear pb", shape, amp)
    s = pb_solver(shape, levels, kinds, [amp * v for v in values], k2)
    f = amp * k2 * rhs(shape, 34)
    b = oracle.fold(f, h, kinds, [amp * v for v in values])
    psi, st = s.solve_pb(to_dev(f), rtol=1e-10, max_outer=300, inner=2)
    ref, hist, ost = oracle.pb_nl_solve(b, h, kinds, levels, k2, inner=2, rtol=1e-10, max_outer=300)
    print(f"outer steps {st.cycles} (oracle {len(hist) - 1}), max|psi| {np.abs(ref).max():.2f}", flush=True)
    assert ost == 0 and st.rel_res < 1e-10
    assert abs(st.cycles - (len(hist) - 1)) <= 1
    assert np.abs(psi.cpu().numpy() - ref).max() <= 1e-11 * np.abs(ref).max()
    # the same number of steps as the oracle from the same start: the iterates agree
    psi2, st2 = s.solve_pb(to_dev(f), rtol=0.0, max_outer=4, inner=2, check=False)
    ref2, _, _ = oracle.pb_nl_solve(b, h, kinds, levels, k2, inner=2, rtol=0.0, max_outer=4)
    assert st2.cycles == 4
    assert np.abs(psi2.cpu().numpy() - ref2).max() <= 1e-11 * np.abs(ref2).max()


def test_gouy_chapman_double_layer_on_the_gpu():
    """Planar double layer of the nonlinear equation: 4 artanh(tanh(psi0/4) e^(-kappa z))
    with Dirichlet psi0 at the wall and the layer's value at z = L, zero-Neumann sides;
    the GPU solution at 256 cells across is within its second-order discretisation error."""
    kappa, L, psi0 = 6.0, 1.0, 2.0
    nz = 256
    h = L / nz
    gc = lambda z: 4.0 * np.arctanh(np.tanh(psi0 / 4.0) * np.exp(-kappa * z))
    kinds = (N, N, N, N, D, D)
    values = (0, 0, 0, 0, psi0, float(gc(L)))
    s = pkg.Solver((8, 8, nz), h, list(zip(kinds, values)), pkg.Options(levels=3, kappa2=kappa ** 2), device=DEV)
    psi, st = s.solve_pb(s.zeros(), rtol=1e-12, max_outer=400, inner=2)
    z = (np.arange(nz) + 0.5) * h
    p = psi.cpu().numpy()
    assert np.abs(p - p[:, :1, :1]).max() <= 1e-12 * psi0   # uniform across the sides
    err = np.abs(p[:, 0, 0] - gc(z)).max()
    print(f"Gouy-Chapman: {st.cycles} outer steps, max error {err:.2e}", flush=True)
    assert err < 2e-3
