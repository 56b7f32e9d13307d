"""Writes coulomb_force_diagonal.txt: the relative Coulomb-force error of a
charged sphere in a homogeneous field (Sec. 6.3, Tab.
ValidClmbForceSubs_PotMaxErr, entries with equal potential and force
subsampling factors s_f = 1, 2, 3) as computed by the oracle: sub-sampled
deposition with the paper's q/V density, multigrid solve with phi = 0 at x = 0
and -10 at x = L, zero-Neumann elsewhere, force by Eq. ElectrostatForce, at the
sphere position of maximal volume-mapping error.  Calls only the oracle.

Domain 64^3, h = 1, q = 1, eps = 1; the sphere centre is the first sub-cell
centre of cell 32 shifted by the argmax shift (sub-cell widths).

    python tests/golden/make_coulomb_force.py
"""
import itertools
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "coulomb_force_diagonal.txt")

# e_rFC in percent as printed, keyed by (R, s_f) with s_f(potential) = s_f(force)
PAPER = {(4, 1): 7.06, (4, 2): 2.58, (4, 3): -1.43,
         (6, 1): -2.74, (6, 2): -1.43, (6, 3): -0.33,
         (8, 1): 2.58, (8, 2): 0.72, (8, 3): -0.25,
         (9, 1): 1.91, (9, 2): -0.33, (9, 3): 0.32,
         (12, 1): -1.43, (12, 2): -0.25, (12, 3): -0.11}
N, BASE, LEVELS = 64, 32, 5
KINDS = (0, 0, 1, 1, 1, 1)
VALUES = (0.0, -10.0, 0.0, 0.0, 0.0, 0.0)


def shift_grid():
    g = np.round(np.arange(0, 26) * 0.02, 10)
    return np.array([s for s in itertools.product(g, g, g) if s[0] <= s[1] <= s[2]])


def argmax_shift(R, sf, shifts):
    c = BASE + (0.5 + shifts) / sf
    _, wsum = oracle.deposit_sub((N, N, N), 1.0, c, np.full(len(shifts), float(R)), np.ones(len(shifts)),
                                 subsample=sf)
    V = 4.0 / 3.0 * math.pi * R ** 3
    e = (wsum - V) / V * 100.0
    k = int(np.argmax(np.abs(e)))
    return shifts[k], e[k]


def force_error(R, sf, shift):
    c = (BASE + (0.5 + shift) / sf)[None]
    r, q = np.array([float(R)]), np.array([1.0])
    f, _ = oracle.deposit_sub((N, N, N), 1.0, c, r, q, subsample=sf, mode=1)
    phi, _, st = oracle.solve_problem(f, 1.0, KINDS, VALUES, LEVELS, rtol=1e-12)
    assert st == 0
    F = oracle.coulomb(phi, 1.0, KINDS, VALUES, c, r, q, subsample=sf, mode=1)
    FC = 10.0 / N
    return (F[0, 0] - FC) / FC * 100.0


def main():
    shifts = shift_grid()
    lines = [
        "# Relative Coulomb-force error e_rFC of a charged sphere in a homogeneous field,",
        "# at the sphere position of maximal volume-mapping error, equal potential and force",
        "# subsampling factors.  Source: Table \"Coulomb force validation\" (Tab.",
        "# ValidClmbForceSubs_PotMaxErr), diagonal entries, Sec. 6.3 of Bartuschat & Ruede",
        "# (arXiv:1410.6609); the paper notes that these equal e_rV,max.",
        "# Columns 1-3 and 'status' restate the paper; the argmax shift (sub-cell widths from",
        "# the first sub-cell centre of cell 32, 64^3 domain), e_rV and e_rFC of the oracle were",
        "# written by make_coulomb_force.py (oracle only).  'pinned': e_rFC equals the printed",
        "# value to its two decimals; 'unreached': the printed volume-mapping extreme is not",
        "# reached (the s_f*R = 4, 8 and 36 balls, as in the volume-mapping tables).",
        "# R  s_f  e_paper  status     sx    sy    sz   e_rV_oracle  e_rF_oracle",
    ]
    for (R, sf), e_paper in sorted(PAPER.items()):
        sh, ev = argmax_shift(R, sf, shifts)
        ef = force_error(R, sf, sh)
        status = "pinned" if abs(ef - e_paper) < 0.006 else "unreached"
        lines.append(f"{R:<3d} {sf:<4d} {e_paper:7.2f}  {status:<9s} {sh[0]:5.2f} {sh[1]:5.2f} {sh[2]:5.2f}  "
                     f"{ev:11.6f}  {ef:11.6f}")
        print(lines[-1], flush=True)
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
