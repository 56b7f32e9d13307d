"""Full-size checks at the benchmark's shapes and launch configuration.

256^3 (FP64): element-wise parity with the oracle after the same cycle count.
512^3 and 1024x256x256 (FP64 and FP32-IR): the oracle recomputes the FP64
residual of the GPU solution over the whole grid (a property that holds at any
size), deposition counts are compared exactly, and the two precisions agree.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1410_6609_amd as pkg
import workloads as W

from test_gpu_parity import DEV, log_case, to_dev

pytestmark = pytest.mark.gpu


def make(w, precision=pkg.FP64):
    return pkg.Solver(w.shape, w.h, list(zip(w.kinds, w.values)),
                      pkg.Options(levels=w.levels, precision=precision), device=DEV)


def test_c2_full_parity():
    w = W.C2
    log_case("c2 full")
    sph = W.workload_spheres(w)
    s = make(w)
    f, cnt = s.deposit(*(to_dev(a) for a in (sph.centers, sph.radii, sph.charges)), counts=True)
    phi, st = s.solve(f, rtol=w.rtol)
    assert st.rel_res < 1e-10
    f_ref, cnt_ref = oracle.deposit(w.shape, w.h, sph.centers, sph.radii, sph.charges)
    assert np.array_equal(cnt.cpu().numpy(), cnt_ref)
    ref, hist, _ = oracle.solve_problem(f_ref, w.h, w.kinds, w.values, w.levels, rtol=0.0,
                                        max_cycles=st.cycles)
    assert hist[-1] < 1e-10
    assert np.abs(phi.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["c3_spheres_512", "c5_channel_1024x256x256"])
def test_large_workloads_residual_and_precisions(name):
    w = W.ALL[name]
    log_case("full", name)
    sph = W.workload_spheres(w)
    c, r, q = (to_dev(a) for a in (sph.centers, sph.radii, sph.charges))
    res = {}
    for prec in (pkg.FP64, pkg.FP32_IR):
        s = make(w, prec)
        f, cnt = s.deposit(c, r, q, counts=True)
        phi, st = s.solve(f, rtol=w.rtol)
        assert st.rel_res < 1e-10
        res[prec] = phi.cpu().numpy()
        del s, phi
        torch.cuda.empty_cache()
    f_ref, cnt_ref = oracle.deposit(w.shape, w.h, sph.centers, sph.radii, sph.charges)
    assert np.array_equal(cnt.cpu().numpy(), cnt_ref)
    b = oracle.fold(f_ref, w.h, w.kinds, w.values)
    bn = oracle.norm2(b)
    for prec, phi in res.items():
        rel = oracle.norm2(oracle.residual(phi, b, w.h, w.kinds)) / bn
        assert rel < 1.0001e-10, (prec, rel)
    scale = np.abs(res[pkg.FP64]).max()
    assert np.abs(res[pkg.FP32_IR] - res[pkg.FP64]).max() <= 1e-6 * scale
