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


# ---- sub-sampled deposition (Sec. 2.4, "Subsampling"; Sec. 6.3) -------------
GOLDEN_SUB = os.path.join(os.path.dirname(__file__), "golden", "volume_mapping_subsampled.txt")


def test_sub_sf1_is_the_naive_deposition(orc):
    w = W.C2.scaled((40, 36, 44), levels=3, n_spheres=30)
    s = W.workload_spheres(w)
    f0, cnt = orc.deposit(w.shape, 0.5, s.centers * 0.5, s.radii * 0.5, s.charges, 0.8)
    f1, wsum = orc.deposit_sub(w.shape, 0.5, s.centers * 0.5, s.radii * 0.5, s.charges, 0.8, subsample=1)
    assert np.array_equal(wsum, cnt.astype(float))
    assert np.allclose(f1, f0, rtol=1e-15, atol=0)


@pytest.mark.parametrize("sf", [2, 3, 4, 5])
@pytest.mark.parametrize("R", [1.37, 2.71, 3.43])
def test_sub_weights_count_sub_cell_lattice_points(orc, sf, R):
    """A sphere centred on a cell centre: in sub-cell units the sub-cell centres
    sit at integer offsets (s_f odd) or odd half-integer offsets (s_f even), so
    s_f^3 W_s is an exact lattice-point count (radii keep (2 s_f R)^2 well away
    from integers, so rounding cannot move a point across the sphere)."""
    n = 12
    _, wsum = orc.deposit_sub((n, n, n), 1.0, np.array([[6.5, 6.5, 6.5]]), np.array([R]), np.array([1.0]),
                              subsample=sf)
    rr = (2 * sf * R) ** 2
    m = int(2 * sf * R) + 2
    a = np.arange(-m, m + 1)
    a = a[a % 2 == 1 - sf % 2]   # 2 x offset in sub-cell widths: odd for even s_f, even for odd s_f
    s2 = a[:, None, None] ** 2 + a[None, :, None] ** 2 + a[None, None, :] ** 2
    assert abs(rr - round(rr)) > 1e-3
    m_ = wsum[0] * sf ** 3   # sum of ratios k / s_f^3: integer up to rounding
    assert abs(m_ - round(m_)) < 1e-9 and round(m_) == int((s2 <= rr).sum())


@pytest.mark.parametrize("mode", [0, 1])
def test_sub_charge_totals(orc, mode):
    """Mode 0 (spread) conserves every sphere's charge; mode 1 (volume) carries
    q W_s h^3 / V_s, i.e. the charge times (1 + e_rV)."""
    w = W.C2.scaled((48, 40, 56), levels=3, n_spheres=40)
    s = W.workload_spheres(w)
    eps, h, sf = 0.7, 0.25, 3
    f, wsum = orc.deposit_sub(w.shape, h, s.centers * h, s.radii * h, s.charges, eps, subsample=sf, mode=mode)
    total = f.sum() * h ** 3 * eps
    V = 4.0 / 3.0 * math.pi * (s.radii * h) ** 3
    want = s.charges.sum() if mode == 0 else float((s.charges * wsum * h ** 3 / V).sum())
    assert abs(total - want) <= 1e-12 * np.abs(s.charges).sum()
    # every overlap ratio is a multiple of 1/s_f^3
    ff = orc.deposit_sub(w.shape, h, s.centers[:1] * h, s.radii[:1] * h, np.ones(1), 1.0, subsample=sf)[0]
    m = ff[ff != 0] * wsum[0] * h ** 3 * sf ** 3
    assert np.allclose(m, np.round(m), atol=1e-9) and m.max() == pytest.approx(sf ** 3)


def test_golden_subsampled_volume_mapping_errors(orc):
    """Tab. ValidPotSubs, e_rV,max for s_f = 2, 3, 4: the error at the stored
    argmax shift reproduces the printed value for the pinned rows, and no
    sampled shift of the same grid exceeds it."""
    rows = []
    with open(GOLDEN_SUB) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                R, sf, e_paper, status, sx, sy, sz, e_or = line.split()
                rows.append((int(R), int(sf), float(e_paper), status, np.array([float(sx), float(sy), float(sz)]),
                             float(e_or)))
    assert len(rows) == 15 and sum(r[3] == "pinned" for r in rows) == 12
    g = np.round(np.arange(0, 26) * 0.02, 10)
    grid = np.array([s for s in itertools.product(g, g, g) if s[0] <= s[1] <= s[2]])
    rng = np.random.default_rng(5)
    for R, sf, e_paper, status, shift, e_or in rows:
        shifts = np.vstack([shift, grid[rng.choice(len(grid), 24, replace=False)]])
        c = 32.0 + (0.5 + shifts) / sf
        _, wsum = orc.deposit_sub((64, 64, 64), 1.0, c, np.full(len(c), float(R)), np.ones(len(c)), subsample=sf)
        V = 4.0 / 3.0 * math.pi * R ** 3
        e = (wsum - V) / V * 100.0
        assert abs(e[0] - e_or) < 1e-6   # stored with six decimals
        assert np.abs(e[1:]).max() <= abs(e[0]) + 1e-12
        if status == "pinned":
            assert abs(e[0] - e_paper) < 0.006, (R, sf, e[0], e_paper)
        else:
            assert abs(e[0]) < abs(e_paper)


def test_sub_mean_volume_error_tracks_the_paper(orc):
    """Mean |e_rV| over uniformly random positions against the printed means
    (Tab. ValidPotSubs, row mean |e_rV|): within 20 % (sampling noise), and
    roughly halved per increment of s_f (Sec. 6.3)."""
    paper = {4: [1.14, 0.284, 0.145, 0.081], 6: [0.638, 0.140, 0.065, 0.039]}
    rng = np.random.default_rng(7)
    for R, want in paper.items():
        got = []
        for sf in (1, 2, 3, 4):
            c = 32.0 + rng.random((300, 3))
            _, wsum = orc.deposit_sub((64, 64, 64), 1.0, c, np.full(300, float(R)), np.ones(300), subsample=sf)
            V = 4.0 / 3.0 * math.pi * R ** 3
            got.append(float(np.mean(np.abs(wsum - V) / V * 100.0)))
        for g_, w_ in zip(got, want):
            assert abs(g_ - w_) <= 0.2 * w_, (R, got, want)
        assert all(got[i + 1] < got[i] for i in range(3))


@pytest.mark.parametrize("mode", [0, 1])
def test_sub_dq_matches_finite_differences(orc, mode):
    w = W.C4.scaled((16, 16, 16), levels=3, n_spheres=5)
    w = W.Workload(**{**w.__dict__, "r_lo": 2.0, "r_hi": 3.0})
    s = W.workload_spheres(w)
    wts = np.random.default_rng(3).standard_normal((16, 16, 16))
    def loss(q):
        f, _ = orc.deposit_sub(w.shape, w.h, s.centers, s.radii, q, subsample=3, mode=mode)
        phi, _, _ = orc.solve_problem(f, w.h, w.kinds, w.values, w.levels, rtol=1e-14, max_cycles=60)
        return float(np.vdot(wts, phi))
    lam, _, _ = orc.adjoint(wts, w.h, w.kinds, w.levels, rtol=1e-14, max_cycles=60)
    g = orc.dq_sub(lam, w.h, s.centers, s.radii, subsample=3, mode=mode)
    step = 1e-3
    for i in range(s.n):
        qp, qm = s.charges.copy(), s.charges.copy()
        qp[i] += step
        qm[i] -= step
        fd = (loss(qp) - loss(qm)) / (2 * step)
        assert abs(fd - g[i]) <= 1e-8 * max(1.0, abs(g[i]))
