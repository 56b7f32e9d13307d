"""GPU parity of the two extensions: FP32 cycles inside FP64 iterative
refinement, and the adjoint solve with gradients (dL/df, dL/drho, dL/dq,
autograd), plus the error paths of the C ABI forced from the host."""
import numpy as np
import pytest
import torch

import oracle
import paper_1410_6609_amd as pkg
import workloads as W
from workloads import DIRICHLET as D, NEUMANN as N

from test_gpu_parity import CASES, DEV, ids, log_case, rhs, to_dev

pytestmark = pytest.mark.gpu


def solver(shape, levels, kinds, values, h=None, **opt):
    h = 1.0 / shape[0] if h is None else h
    return pkg.Solver(shape, h, list(zip(kinds, values)), pkg.Options(levels=levels, **opt), device=DEV)


@pytest.mark.parametrize("inner", [1, 2, 3, 4])
@pytest.mark.parametrize("case", CASES, ids=ids)
def test_fp32_ir_reaches_fp64_accuracy(case, inner):
    shape, levels, kinds, values = case
    log_case("ir", shape, inner)
    h = 1.0 / shape[0]
    s = solver(shape, levels, kinds, values, precision=pkg.FP32_IR, ir_inner_cycles=inner)
    f = rhs(shape, 11)
    phi, st = s.solve(to_dev(f), rtol=1e-10)
    assert st.rel_res < 1e-10 and st.inner_cycles == inner * st.cycles
    got = phi.cpu().numpy()
    b = oracle.fold(f, h, kinds, values)
    # the oracle's own FP64 residual of the GPU result
    rel = oracle.norm2(oracle.residual(got, b, h, kinds)) / oracle.norm2(b)
    assert rel < 1.0001e-10
    ref, _, _ = oracle.solve(b, h, kinds, levels, rtol=1e-13)
    # stopping at a relative residual of 1e-10 leaves up to about 1.5e-10 of
    # max|phi| on these cases (the oracle's own refinement measures the same)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    # same refinement algorithm in the oracle (float arithmetic on the CPU)
    _, ohist, ost = oracle.solve_ir(b, h, kinds, levels, inner=inner, rtol=1e-10)
    assert ost == 0 and abs((len(ohist) - 1) - st.cycles) <= 1


@pytest.mark.parametrize("case", CASES[:4], ids=ids)
def test_adjoint_parity(case):
    shape, levels, kinds, values = case
    log_case("adjoint", shape)
    h = 1.0 / shape[0]
    s = solver(shape, levels, kinds, values)
    g = rhs(shape, 12)
    lam, _, drho, st = s.adjoint(to_dev(g), eps=0.5, want_drho=True, rtol=1e-10)
    ref, hist, _ = oracle.adjoint(g, h, kinds, levels, rtol=1e-10)
    assert st.cycles == len(hist) - 1
    got = lam.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert torch.equal(drho, lam * 2.0)   # dL/drho = lambda / eps with eps = 1/2 (exact)


def spheres_case(shape=(64, 64, 64), levels=4, n=24, seed=77, r=(2.5, 4.0)):
    w = W.Workload("adj", shape, 1.0, (D,) * 6, (0.0,) * 6, levels=levels, n_spheres=n, r_lo=r[0],
                   r_hi=r[1], seed=seed)
    return w, W.workload_spheres(w)


def test_dq_parity_and_autograd():
    w, sph = spheres_case()
    s = solver(w.shape, w.levels, w.kinds, w.values, h=w.h)
    wts = W.random_field(w.shape, 13)
    c, r, q = (to_dev(a) for a in (sph.centers, sph.radii, sph.charges))
    lam, dq, _, st = s.adjoint(to_dev(wts), c, r, eps=1.0, rtol=1e-10)
    lam_ref, hist, _ = oracle.adjoint(wts, w.h, w.kinds, w.levels, rtol=1e-10)
    dq_ref = oracle.dq(lam_ref, w.h, sph.centers, sph.radii)
    assert np.abs(dq.cpu().numpy() - dq_ref).max() <= 1e-11 * np.abs(dq_ref).max()
    # the same gradient through torch.autograd
    qg = q.clone().requires_grad_(True)
    phi = pkg.PoissonFn.apply(qg, c, r, s, 1.0, 1e-10, 100)
    loss = (phi * to_dev(wts)).sum()
    loss.backward()
    assert np.abs(qg.grad.cpu().numpy() - dq_ref).max() <= 1e-11 * np.abs(dq_ref).max()
    # RhsSolveFn: dL/df = lambda
    fr = s.deposit(c, r, q).requires_grad_(True)
    phi2 = pkg.RhsSolveFn.apply(fr, s, 1e-10, 100)
    (phi2 * to_dev(wts)).sum().backward()
    assert np.abs(fr.grad.cpu().numpy() - lam_ref).max() <= 1e-12 * np.abs(lam_ref).max()


@pytest.mark.parametrize("shape,levels", [((64, 64, 64), 4), ((128, 128, 128), 5)])
def test_dq_matches_finite_differences_fixed_cycles(shape, levels):
    """Central differences (step 1e-6) of L = sum w phi over 16 seeded sphere
    charges, with the forward solves run for a fixed cycle count so that the
    discrete map q -> phi is linear (its contraction makes the remainder
    negligible); the 128^3 case is the full gradient workload."""
    w = W.C4 if shape == W.C4.shape else W.C4.scaled(shape, levels=levels, n_spheres=40)
    log_case("fd", shape)
    sph = W.workload_spheres(w)
    s = solver(w.shape, w.levels, w.kinds, w.values, h=w.h)
    wts = to_dev(W.loss_weights(w))
    c, r = to_dev(sph.centers), to_dev(sph.radii)
    idx = W.fd_sphere_indices(w)
    _, dq, _, _ = s.adjoint(wts, c, r, rtol=1e-13, max_cycles=60)
    k = 24
    def loss(qv):
        f = s.deposit(c, r, to_dev(qv))
        phi, _ = s.solve(f, rtol=0.0, max_cycles=k, check=False)
        return float((phi * wts).sum())
    step = w.extra["fd_step"]
    dq = dq.cpu().numpy()
    assert len(idx) == 16
    for i in idx:
        qp, qm = sph.charges.copy(), sph.charges.copy()
        qp[i] += step
        qm[i] -= step
        fd = (loss(qp) - loss(qm)) / (2 * step)
        assert abs(fd - dq[i]) <= 1e-6 * max(abs(dq[i]), 1e-3 * np.abs(dq).max()), (i, fd, dq[i])


def test_fp32_ir_gradient_matches_fp64():
    w = W.C4.scaled((128, 128, 128), levels=5, n_spheres=100)
    sph = W.workload_spheres(w)
    c, r = to_dev(sph.centers), to_dev(sph.radii)
    wts = to_dev(W.loss_weights(w))
    out = {}
    for prec in (pkg.FP64, pkg.FP32_IR):
        s = solver(w.shape, w.levels, w.kinds, w.values, h=w.h, precision=prec)
        _, dq, _, st = s.adjoint(wts, c, r, rtol=1e-10)
        out[prec] = dq.cpu().numpy()
    rel = np.abs(out[pkg.FP32_IR] - out[pkg.FP64]).max() / np.abs(out[pkg.FP64]).max()
    assert rel <= 1e-6


def test_channel_forward_and_adjoint_fp32_ir_vs_fp64():
    """Full 1024x256x256 channel: FP32-IR forward and adjoint solves agree with
    the FP64 solver (both to 1e-10), and the charge gradient agrees to 1e-6."""
    w = W.C5
    log_case("channel fwd+adj")
    sph = W.workload_spheres(w)
    c, r, q = (to_dev(a) for a in (sph.centers, sph.radii, sph.charges))
    wts = torch.tensor(np.random.default_rng(5005).standard_normal((256, 256, 1024)), device=DEV)
    out = {}
    for prec in (pkg.FP64, pkg.FP32_IR):
        s = solver(w.shape, w.levels, w.kinds, w.values, h=w.h, precision=prec)
        f = s.deposit(c, r, q)
        phi, st = s.solve(f, rtol=1e-10)
        lam, dq, _, ast = s.adjoint(wts, c, r, rtol=1e-10)
        assert st.rel_res < 1e-10 and ast.rel_res < 1e-10
        out[prec] = (phi.cpu().numpy(), dq.cpu().numpy())
        del s, phi, lam, f
        torch.cuda.empty_cache()
    p64, g64 = out[pkg.FP64]
    p32, g32 = out[pkg.FP32_IR]
    assert np.abs(p32 - p64).max() <= 1e-6 * np.abs(p64).max()
    assert np.abs(g32 - g64).max() <= 1e-6 * np.abs(g64).max()


# ---- error paths, forced from the host ------------------------------------
def test_nonfinite_rhs_reports_error():
    shape, levels, kinds, values = CASES[1]
    s = solver(shape, levels, kinds, values)
    f = rhs(shape, 14)
    f[3, 4, 5] = np.nan
    phi, st = s.solve(to_dev(f), check=False)
    assert st.status == pkg.E_NONFINITE


def test_max_cycles_reports_noconv():
    shape, levels, kinds, values = CASES[1]
    s = solver(shape, levels, kinds, values)
    phi, st = s.solve(to_dev(rhs(shape, 15)), rtol=1e-10, max_cycles=1, check=False)
    assert st.status == pkg.E_NOCONV and st.cycles == 1 and st.rel_res > 1e-10
    with pytest.raises(pkg.CcmgError):
        s.solve(to_dev(rhs(shape, 15)), rtol=1e-10, max_cycles=1)


def test_zero_rhs_gives_zero_solution():
    shape, levels, kinds, _ = CASES[1]
    s = solver(shape, levels, kinds, (0.0,) * 6)
    phi = torch.ones((shape[2], shape[1], shape[0]), dtype=torch.float64, device=DEV)
    phi, st = s.solve(s.zeros(), phi)
    assert st.cycles == 0 and not phi.any()


def test_host_pointer_rejected():
    import ctypes
    shape, levels, kinds, values = CASES[0]
    s = solver(shape, levels, kinds, values)
    host = np.zeros((shape[2], shape[1], shape[0]))
    hp = ctypes.c_void_p(host.ctypes.data)
    rc = pkg.lib().ccmg_solve(s._h, hp, hp, 1e-10, 10, None)
    assert rc == pkg.E_ARG
    assert b"device memory" in pkg.lib().ccmg_last_error(s._h)


def test_initial_guess_warm_start():
    shape, levels, kinds, values = CASES[3]
    s = solver(shape, levels, kinds, values)
    f = to_dev(rhs(shape, 16))
    phi, st = s.solve(f, rtol=1e-11)
    phi2, st2 = s.solve(f, phi.clone(), rtol=1e-10)
    assert st2.cycles == 0 and torch.equal(phi2, phi)


def test_fp32_ir_with_face_values():
    """Per-cell boundary values enter the FP64 fold that the refinement steps
    use: the FP32-IR solution meets the oracle's FP64 residual bar."""
    shape, levels, kinds, values = CASES[3]
    h = 1.0 / shape[0]
    s = solver(shape, levels, kinds, values, precision=pkg.FP32_IR)
    rng = np.random.default_rng(61)
    nx, ny, nz = shape
    shapes = [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2
    faces = [rng.standard_normal(sh) if fc in (0, 3, 4) else None for fc, sh in enumerate(shapes)]
    for fc, a in enumerate(faces):
        if a is not None:
            s.set_face_values(fc, to_dev(a))
    f = rhs(shape, 62)
    phi, st = s.solve(to_dev(f), rtol=1e-10)
    b = oracle.fold_field(f, h, kinds, values, faces)
    rel = oracle.norm2(oracle.residual(phi.cpu().numpy(), b, h, kinds)) / oracle.norm2(b)
    assert st.rel_res < 1e-10 and rel < 1.0001e-10


def test_vcycles_refinement_steps():
    """ccmg_vcycles in FP32-IR mode: k refinement steps without host waits,
    the residual after the last one on the device, equal to the synchronising
    single-step path run k times."""
    shape, levels, kinds, values = CASES[1]
    s = solver(shape, levels, kinds, values, precision=pkg.FP32_IR)
    f = to_dev(rhs(shape, 63))
    a = s.zeros()
    rel_dev = torch.zeros(1, dtype=torch.float64, device=DEV)
    s.vcycles(a, f, 4, rel_dev)
    b = s.zeros()
    for _ in range(4):
        rel = s.vcycle(b, f)
    assert torch.equal(a, b)
    assert float(rel_dev[0]) == rel


@pytest.mark.parametrize("inner", [1, 3])
def test_fp32_ir_vcycle_matches_oracle_refinement_step(inner):
    """One FP32-IR cycle call (ccmg_vcycle) is one refinement step: the FP64
    residual of phi scaled by a power of two, `inner` FP32 V-cycles from zero,
    the FP64 update.  The oracle's refinement (float arithmetic on the CPU)
    from the same phi agrees to FP32 rounding of the correction."""
    shape, levels, kinds, values = CASES[3]
    log_case("ir vcycle", shape, inner)
    h = 1.0 / shape[0]
    s = solver(shape, levels, kinds, values, precision=pkg.FP32_IR, ir_inner_cycles=inner)
    f = rhs(shape, 64)
    phi0 = rhs(shape, 65)
    phi = to_dev(phi0)
    rel = s.vcycle(phi, to_dev(f))
    b = oracle.fold(f, h, kinds, values)
    ref, hist, st = oracle.solve_ir(b, h, kinds, levels, inner=inner, rtol=0.0, max_outer=1, phi0=phi0)
    assert st in (oracle.OK, oracle.E_NOCONV) and len(hist) == 2   # rtol = 0: one step, never "converged"
    got = phi.cpu().numpy()
    step = np.abs(ref - phi0).max()
    assert step > 1e-2 * np.abs(phi0).max()
    err = np.abs(got - ref).max()
    print(f"ir vcycle inner={inner}: max|dphi| vs oracle {err:.2e} of a step {step:.2e}", flush=True)
    assert err <= 1e-5 * step
    assert abs(rel - hist[1]) <= 1e-3 * hist[1]


def test_fp32_ir_vcycle_on_zero_rhs_corrects_phi():
    """f = 0 with homogeneous boundary values: b vanishes but phi != 0 still has
    a residual, so the refinement step must update phi (one FP32 cycle gives
    the FP64 cycle's correction to FP32 accuracy) and never copy stale
    workspace data into it (an earlier solve leaves its last iterate there)."""
    shape, levels, kinds, _ = CASES[1]
    values = (0.0,) * 6
    log_case("ir vcycle zero rhs", shape)
    s32 = solver(shape, levels, kinds, values, precision=pkg.FP32_IR, ir_inner_cycles=1)
    s64 = solver(shape, levels, kinds, values)
    s32.solve(to_dev(rhs(shape, 67)), rtol=1e-10)       # leaves data in the workspace
    phi0 = rhs(shape, 68)
    zero = s64.zeros()
    a = to_dev(phi0)
    s64.vcycle(a, zero, norm=False)
    b_ = to_dev(phi0)
    rel = s32.vcycle(b_, zero)
    assert np.isfinite(rel)
    corr = (a - to_dev(phi0)).abs().max().item()
    assert corr > 0.1 * np.abs(phi0).max()
    assert (b_ - a).abs().max().item() <= 1e-4 * corr
    # vcycles (no host wait) takes the same path
    c_ = to_dev(phi0)
    s32.vcycles(c_, zero, 1)
    assert torch.equal(c_, b_)
