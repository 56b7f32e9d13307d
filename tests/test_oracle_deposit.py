"""Pins of the oracle's charge deposition and charge gradient.

References: exact integer lattice-point counts, charge conservation, the
symmetry of a ball centred on a cell centre, the paper's printed
volume-mapping errors (Tab. ValidPotSubs, s_f = 1), and finite differences of
the full solve for dL/dq.
"""
import itertools
import math
import os

import numpy as np
import pytest

import workloads as W
from workloads import DIRICHLET as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "volume_mapping_sf1.txt")


def integer_ball_count(R2_num, den=1):
    """#{(a,b,c) in Z^3 : a^2 + b^2 + c^2 <= R2_num / den}, in integers."""
    r = int(math.isqrt(R2_num // den)) + 1
    a = np.arange(-r, r + 1)
    s = (a[:, None, None] ** 2 + a[None, :, None] ** 2 + a[None, None, :] ** 2) * den
    return int((s <= R2_num).sum())


@pytest.mark.parametrize("R", [1, 2, 3, 4, 5, 6, 7.5])
def test_count_cell_centred_ball(orc, R):
    n = 24
    c = np.array([[12.5, 12.5, 12.5]])
    f, cnt = orc.deposit((n, n, n), 1.0, c, np.array([float(R)]), np.array([1.0]))
    want = integer_ball_count(int(round(4 * R * R)), 4)
    assert cnt[0] == want
    # charge spread evenly: every covered cell holds q / n_s
    assert np.count_nonzero(f) == want
    assert np.allclose(f[f != 0], 1.0 / want, rtol=0, atol=1e-17)


def test_vertex_centred_ball_count(orc):
    """Centre on a cell corner: offsets are half-integers, count (2a+1)^2+... <= 4R^2."""
    n = 20
    R = 4.0
    f, cnt = orc.deposit((n, n, n), 1.0, np.array([[10.0, 10.0, 10.0]]), np.array([R]), np.array([1.0]))
    r = 6
    a = np.arange(-r, r)
    s = (2 * a + 1)[:, None, None] ** 2 + (2 * a + 1)[None, :, None] ** 2 + (2 * a + 1)[None, None, :] ** 2
    assert cnt[0] == int((s <= 4 * 16).sum())


def test_cell_centred_sphere_has_cube_symmetry(orc):
    n = 16
    f, _ = orc.deposit((n, n, n), 0.5, np.array([[4.25, 4.25, 4.25]]), np.array([2.1]), np.array([3.0]))
    core = f[2:15, 2:15, 2:15]   # centred on cell 8 in each axis
    for perm in itertools.permutations(range(3)):
        assert np.array_equal(core, np.transpose(core, perm))
    for ax in range(3):
        assert np.array_equal(core, np.flip(core, ax))


def test_charge_conservation_and_overlaps(orc):
    w = W.C2.scaled((48, 40, 56), levels=3, n_spheres=60)
    s = W.workload_spheres(w)
    eps, h = 0.7, 0.25
    f, cnt = orc.deposit(w.shape, h, s.centers * h, s.radii * h, s.charges, eps)
    assert (cnt > 0).all()
    total = f.sum() * h ** 3 * eps
    assert abs(total - s.charges.sum()) <= 1e-12 * np.abs(s.charges).sum()


def test_golden_volume_mapping_errors(orc):
    """Max relative volume-mapping error over shifted sphere positions
    (Tab. ValidPotSubs, s_f = 1).  The count is even in each shift component
    and symmetric under axis permutations, so sorted shifts in [0, 1/2] cover
    the +-0.51 cell range of the paper's protocol."""
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                R, e, status = line.split()
                rows.append((float(R), float(e), status))
    g = np.round(np.arange(0, 26) * 0.02, 10)
    shifts = np.array([s for s in itertools.product(g, g, g) if s[0] <= s[1] <= s[2]])
    n = 32
    for R, e_paper, status in rows:
        centers = 16.5 + shifts
        _, cnt = orc.deposit((n, n, n), 1.0, centers, np.full(len(shifts), R), np.ones(len(shifts)))
        V = 4.0 / 3.0 * math.pi * R ** 3
        e = (cnt - V) / V * 100.0
        e_max = e[np.argmax(np.abs(e))]
        if status == "pinned":
            assert abs(e_max - e_paper) < 0.006, (R, e_max, e_paper)
        else:
            # documented gap: the printed value needs one more cell than any shift gives
            assert abs(e_max) < abs(e_paper)


def test_dq_matches_finite_differences(orc):
    """dL/dq for L = sum w phi from the adjoint solve vs central differences of
    the full forward map q -> phi (linear in q, so differences are exact up to
    solver tolerance)."""
    w = W.C4.scaled((16, 16, 16), levels=3, n_spheres=5)
    w = W.Workload(**{**w.__dict__, "r_lo": 2.0, "r_hi": 3.0})
    s = W.workload_spheres(w)
    wts = np.random.default_rng(2).standard_normal((16, 16, 16))
    def loss(q):
        f, _ = orc.deposit(w.shape, w.h, s.centers, s.radii, q)
        phi, _, _ = orc.solve_problem(f, w.h, w.kinds, w.values, w.levels, rtol=1e-14, max_cycles=60)
        return float(np.vdot(wts, phi))
    lam, _, _ = orc.adjoint(wts, w.h, w.kinds, w.levels, rtol=1e-14, max_cycles=60)
    g = orc.dq(lam, w.h, s.centers, s.radii)
    step = 1e-3
    for i in range(s.n):
        qp, qm = s.charges.copy(), s.charges.copy()
        qp[i] += step
        qm[i] -= step
        fd = (loss(qp) - loss(qm)) / (2 * step)
        assert abs(fd - g[i]) <= 1e-8 * max(1.0, abs(g[i]))
