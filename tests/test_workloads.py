"""The seeded input generators: determinism, ranges and draw order."""
import numpy as np

import workloads as W


def test_spheres_deterministic_and_inside():
    for w in (W.C2, W.C3, W.C4, W.C5):
        a = W.workload_spheres(w)
        b = W.workload_spheres(w)
        assert np.array_equal(a.centers, b.centers) and np.array_equal(a.charges, b.charges)
        assert a.n == w.n_spheres
        assert (a.radii >= w.r_lo).all() and (a.radii <= w.r_hi).all()
        ext = np.asarray(w.shape, float)[None, :] * w.h
        assert (a.centers - a.radii[:, None] >= 0).all()
        assert (a.centers + a.radii[:, None] <= ext).all()
        assert set(np.unique(a.charges)) <= {-1.0, 1.0}
        assert abs(a.charges.mean()) < 0.2


def test_sine_rhs_shape_and_peak():
    f = W.sine_rhs((32, 16, 8), 1 / 32)
    assert f.shape == (8, 16, 32)
    assert f.max() <= 3 * np.pi ** 2


def test_config_levels_divide():
    for w in W.ALL.values():
        d = 1 << (w.levels - 1)
        assert all(n % d == 0 for n in w.shape)
