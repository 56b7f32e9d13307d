"""Writes volume_mapping_subsampled.txt: for each (radius, subsampling factor)
entry of the paper's table of volume-mapping errors (Tab. ValidPotSubs, row
e_rV,max, columns s_f = 2, 3, 4; Sec. 6.3), the sphere shift with the largest
relative volume-mapping error found by the oracle's sub-sampled deposition,
and that error.  Calls only the oracle.

Shifts are measured in sub-cell widths h/s_f from a sub-cell centre; the
overlap count depends on the centre only modulo the sub-cell lattice and is
even in each shift component and symmetric under axis permutations, so sorted
shifts in [0, 1/2]^3 on a 0.02 grid cover the paper's protocol (shifts up to
+-0.51 h/s_f from the domain centre).

    python tests/golden/make_volume_mapping_sub.py
"""
import itertools
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "volume_mapping_subsampled.txt")

# e_rV,max in percent as printed (Tab. ValidPotSubs), keyed by (R, s_f)
PAPER = {(4, 2): 2.58, (4, 3): -1.43, (4, 4): 0.72,
         (6, 2): -1.43, (6, 3): -0.33, (6, 4): -0.25,
         (8, 2): 0.72, (8, 3): -0.25, (8, 4): -0.14,
         (9, 2): -0.33, (9, 3): 0.32, (9, 4): -0.11,
         (12, 2): -0.25, (12, 3): -0.11, (12, 4): -0.10}

N = 64          # grid cells per axis, h = 1
BASE_CELL = 32  # sphere centres start at the first sub-cell centre of this cell


def shift_grid():
    g = np.round(np.arange(0, 26) * 0.02, 10)
    return np.array([s for s in itertools.product(g, g, g) if s[0] <= s[1] <= s[2]])


def centres(sf, shifts):
    return BASE_CELL + (0.5 + shifts) / sf


def errors(R, sf, shifts):
    c = centres(sf, shifts)
    _, wsum = oracle.deposit_sub((N, N, N), 1.0, c, np.full(len(shifts), float(R)), np.ones(len(shifts)),
                                 subsample=sf)
    V = 4.0 / 3.0 * math.pi * R ** 3
    return (wsum - V) / V * 100.0


def main():
    shifts = shift_grid()
    lines = [
        "# Relative volume-mapping error of the sub-sampled deposition, maximal over",
        "# sphere positions shifted by up to half a sub-cell width per axis.",
        "# Source: Table \"Electric potential validation for homogeneously charged sphere\"",
        "# (Tab. ValidPotSubs), row e_rV,max, columns s_f = 2, 3, 4, Sec. 6.3 of Bartuschat &",
        "# Ruede (arXiv:1410.6609).  e_rV = (W_s h^3 - 4/3 pi R^3) / (4/3 pi R^3), W_s = summed",
        "# overlap ratios (fraction of the s_f^3 sub-cell centres of a cell inside the ball).",
        "# columns 1-3 and 'status' restate the paper; argmax shift (in sub-cell widths from a",
        "# sub-cell centre) and e_oracle were written by make_volume_mapping_sub.py (oracle only).",
        "# status 'pinned': the oracle's maximum equals the printed value to its two decimals;",
        "# 'unreached': no shift gives the printed value (the same s_f*R = 8 and 36 balls that",
        "# also miss in the s_f = 1 column, so the paper's inclusion test differs there).",
        "# R  s_f  e_paper  status     sx    sy    sz   e_oracle",
    ]
    for (R, sf), e_paper in sorted(PAPER.items()):
        e = errors(R, sf, shifts)
        k = int(np.argmax(np.abs(e)))
        status = "pinned" if abs(e[k] - e_paper) < 0.006 else "unreached"
        sx, sy, sz = shifts[k]
        lines.append(f"{R:<3d} {sf:<4d} {e_paper:7.2f}  {status:<9s} {sx:5.2f} {sy:5.2f} {sz:5.2f}  {e[k]:.6f}")
        print(lines[-1], flush=True)
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
