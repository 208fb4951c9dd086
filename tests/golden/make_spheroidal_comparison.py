"""Writes spheroidal_comparison.txt: the least-misfit gridding functions against the alpha = 1 prolate
spheroidal function at the same support W (x0 = 1/4, optimal correction of Eq. 12 for both): the largest map
error over |x| <= x0 and its mean (E, Eq. 16, on 101 points), W = 6 .. 10; the spheroidal W = 10 function over
|x| <= 0.2; and the alias of a unit point source outside the image at x = 1/2 + d in the retained field of the
2,000-visibility dirty image at W = 7 (largest departure from the direct DFT, in units of the source's dirty
peak). Context for the paper's comparison (Secs. 2.2 and 4), not a target.

Calls only the oracle and the seeded input generator. Run from the repository root:
python tests/golden/make_spheroidal_comparison.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import imaging as im  # noqa: E402
from oracle import lmtable as lt  # noqa: E402
from oracle import spheroidal as sp  # noqa: E402


def main():
    x = np.linspace(0.0, 0.25, 101)
    lines = ["# W  lm_max_ell  lm_mean_ell  sph_max_ell  sph_mean_ell  ratio_of_max  smallest_ratio_over_x"]
    for W in range(6, 11):
        ll, _, _, _ = lt.map_error(lambda d: lt.kernel(lt.optimal_h(W, 0.25), W, 0.25, d), W, x)
        ls, _, _, _ = sp.map_error(W, x)
        lines.append(f"{W} {ll.max():.3e} {ll.mean():.3e} {ls.max():.3e} {ls.mean():.3e} "
                     f"{ls.max() / ll.max():.3e} {np.min(ls / ll):.3e}")
        print(lines[-1], flush=True)
    x2 = np.linspace(0.0, 0.2, 81)
    ls10, _, _, _ = sp.map_error(10, x2)
    lines.append(f"# spheroidal W = 10 over |x| <= 0.2: max {ls10.max():.3e}, median {np.median(ls10):.3e}")
    c = synth.small_case()
    N, x0 = c.N, 0.25
    otab, h = lt.make_table(7, x0, 300, 3)
    hp = lt.correction(h, 7, x0, N)
    stab = sp.table(7, 2000, 3)
    hs = sp.correction(7, N)
    lines.append("# alias at W = 7 (x = 1/2 + d): d  least_misfit  spheroidal")
    for d in (0.25, 0.375, 0.5):
        vis = np.exp(-2j * np.pi * (c.uv[:, 0] * (0.5 + d) + c.uv[:, 1] * 0.1))
        dft = im.dft_dirty_image(c.uv, vis, None, N, x0)
        a = np.abs(im.make_dirty_image(c.uv, vis, None, N, x0, otab, hp) - dft).max() / len(vis)
        b = np.abs(im.make_dirty_image(c.uv, vis, None, N, x0, stab, hs) - dft).max() / len(vis)
        lines.append(f"{d} {a:.3e} {b:.3e}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "spheroidal_comparison.txt"), "w") as f:
        f.write("# Least-misfit vs alpha = 1 prolate spheroidal gridding functions, x0 = 1/4 (context, Secs. 2.2, 4).\n")
        f.write("# Written by tests/golden/make_spheroidal_comparison.py (oracle only).\n")
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
