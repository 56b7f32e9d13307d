"""GPU parity of the warm-started time-step use of the solver (Sec. 8.1: five
V(3,3)-cycles at the first time step, then one per step from the previous
potential), on a reduced per-node scene: 128 x 256 x 128 cells (two blocks of
the scene, same 4 x 8 x 4 coarsest grid), moving spheres deposited with
sub-sampling factor 2 and the volume normalisation, SI units."""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
import paper_1410_6609_amd as pkg
import workloads as W

from test_gpu_parity import DEV, log_case, to_dev

pytestmark = pytest.mark.gpu


def test_time_steps_match_the_oracle():
    w = replace(W.SCENE, shape=(128, 256, 128), levels=6, name="scene@128x256x128")
    steps = 6
    traj = W.scene_trajectory(w, steps)
    sph = W.scene_spheres(w)
    sf = w.extra["subsample"]
    log_case("time steps", w.shape, sph.n)
    s = pkg.Solver(w.shape, w.h, list(zip(w.kinds, w.values)),
                   pkg.Options(levels=w.levels, nu1=w.nu1, nu2=w.nu2), device=DEV)
    assert s.level_dims(w.levels - 1) == (4, 8, 4)
    r, q = to_dev(sph.radii), to_dev(sph.charges)
    phi = s.zeros()
    f = s.zeros()
    ref = np.zeros((128, 256, 128))
    rels = torch.full((steps,), -1.0, dtype=torch.float64, device=DEV)
    for t in range(steps):
        k = w.extra["first_cycles"] if t == 0 else w.extra["cycles"]
        s.deposit(to_dev(traj[t]), r, q, w.eps, out=f, subsample=sf, mode=pkg.VOLUME)
        if t % 2 == 0:   # the asynchronous entry point (residual written on the device) ...
            s.vcycles(phi, f, k, rels[t:t + 1])
            torch.cuda.synchronize()
            rel = float(rels[t])
        else:            # ... and single synchronising cycles
            for m in range(k):
                rel = s.vcycle(phi, f, norm=(m == k - 1))
        fr, _ = oracle.deposit_sub(w.shape, w.h, traj[t], sph.radii, sph.charges, w.eps, subsample=sf,
                                   mode=pkg.VOLUME)
        b = oracle.fold(fr, w.h, w.kinds, w.values)
        ref, hist, _ = oracle.solve(b, w.h, w.kinds, w.levels, nu1=w.nu1, nu2=w.nu2, rtol=0.0, max_cycles=k,
                                    phi0=ref)
        got = phi.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), t
        # relative residuals near 1e-9 of a boundary-dominated ||b||: allow the
        # rounding floor of the residual itself (1e-15 of ||b||) besides 1e-8 relative
        assert abs(rel - hist[-1]) <= 1e-8 * hist[-1] + 1e-15, (t, rel, hist[-1])
        # one warm-started cycle per step (contraction about 0.06) keeps the
        # residual below the change the moving spheres bring per step
        if t > 0:
            assert rel < 1e-7, (t, rel)
