"""The allocation-free solve (ccmg_solve_zero_static): the library's static
device scratch stands in for the caller's workspace.  Checked through the C
ABI against ccmg_solve_zero on an attached workspace, bit for bit, on three
calls in a row (the second on a smaller grid, in FP32 refinement; the third
with the linearised Poisson-Boltzmann shift), then the first case again (the
scratch keeps the previous call's contents, which must not leak into a
solve)."""
import numpy as np
import pytest
import torch

import paper_1410_6609_amd as pkg
import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")

# (workload, levels, spheres, precision, kappa^2): 128^3 FP64 needs 40 MiB of
# the 64 MiB scratch; the second case is smaller, the third the linearised
# Poisson-Boltzmann operator (a diagonal shift on every level)
CASES = [((128, 128, 128), 5, 100, pkg.FP64, 0.0), ((64, 64, 32), 4, 24, pkg.FP32_IR, 0.0),
         ((96, 64, 64), 4, 40, pkg.FP64, 0.0625)]


def problem(shape, levels, n_spheres, precision, workspace, kappa2=0.0):
    w = W.C2.scaled(shape, levels=levels, n_spheres=n_spheres)
    opt = pkg.Options(levels=w.levels, omega=w.omega, precision=precision, kappa2=kappa2)
    s = pkg.Solver(w.shape, w.h, list(zip(w.kinds, w.values)), opt, device=DEV, workspace=workspace)
    return w, s


def rhs(w):
    sph = W.workload_spheres(w)
    _, s = problem(w.shape, w.levels, len(sph.radii), pkg.FP64, True)
    c, r, q = (torch.tensor(a, device=DEV) for a in (sph.centers, sph.radii, sph.charges))
    return s.deposit(c, r, q)


def reference(shape, levels, n, precision, f, kappa2=0.0):
    _, s = problem(shape, levels, n, precision, True, kappa2)
    phi, st = s.solve(f, rtol=1e-10, zero_guess=True)
    torch.cuda.synchronize()
    return phi, st


def test_static_scratch_solve_matches_workspace_solve():
    results = []
    # one right-hand side per case, reused by the repeated case: cells covered
    # by three spheres take their charges by atomics in no fixed order, so two
    # depositions can differ in the last bit
    rhs_of = {}
    for shape, levels, n, precision, k2 in CASES + CASES[:1]:
        print(f"static-scratch solve {shape} levels={levels} precision={precision} kappa2={k2}", flush=True)
        w, s = problem(shape, levels, n, precision, False, k2)
        assert s.workspace is None
        if shape not in rhs_of:
            rhs_of[shape] = rhs(w)
        f = rhs_of[shape]
        phi_ref, st_ref = reference(shape, levels, n, precision, f, k2)
        nx, ny, nz = shape
        phi = torch.full((nz, ny, nx), float("nan"), dtype=torch.float64, device=DEV)
        _, st = s.solve_static(f, phi, rtol=1e-10)
        torch.cuda.synchronize()
        assert torch.equal(phi, phi_ref), float((phi - phi_ref).abs().max())
        assert (st.cycles, st.inner_cycles, st.rel_res0, st.rel_res) == \
            (st_ref.cycles, st_ref.inner_cycles, st_ref.rel_res0, st_ref.rel_res)
        assert st.rel_res < 1e-10
        results.append(phi.cpu().numpy())
    assert np.array_equal(results[0], results[3])


def test_static_scratch_leaves_an_attached_workspace_in_use():
    shape, levels, n, precision, _ = CASES[1]
    print(f"static-scratch solve beside a workspace {shape}", flush=True)
    w, s = problem(shape, levels, n, precision, True)
    f = rhs(w)
    phi_a, st_a = s.solve(f, rtol=1e-10, zero_guess=True)
    nx, ny, nz = shape
    phi_b = torch.empty((nz, ny, nx), dtype=torch.float64, device=DEV)
    s.solve_static(f, phi_b, rtol=1e-10)
    phi_c, st_c = s.solve(f, rtol=1e-10, zero_guess=True)
    torch.cuda.synchronize()
    assert torch.equal(phi_a, phi_b) and torch.equal(phi_a, phi_c) and st_a.cycles == st_c.cycles
