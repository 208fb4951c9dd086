"""Writes precision_reference_16m_4096.txt: for W = 3, 5, 7 (300-entry cubic
tables, x0 = 1/4), the relative RMS difference between the oracle's FP64 dirty
image (grid, FFT, correct, crop) of the 16,777,152-visibility array workload
on a 4096^2 grid (the same uv, scaled for W = 7, at every W) and the direct DFT, over the 256 x 256 pixel lattice
of dft_samples_16m_4096.npy (every 8th pixel of the retained field). This is the method's own error (Eqs. 7-8, 11) with
no rounding beyond FP64, against which the library's FP32, compensated FP32
and FP64 modes are compared.

Calls only the oracle and the seeded input generator. Run from the repository
root:  python tests/golden/make_precision_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import imaging as im  # noqa: E402
from oracle import lmtable as lt  # noqa: E402


def load_dft():
    return np.load(os.path.join(HERE, "dft_samples_16m_4096.npy"))


def main():
    t0 = time.time()
    dft = load_dft()
    c = synth.array_16m_case(with_vis=True, device="cpu")
    vis = c.vis.astype(np.complex64).astype(np.complex128)
    M = im.crop_size(c.N, c.x0)
    sel = -1024 + 8 * np.arange(256) + M // 2
    lines = []
    for W in (3, 5, 7):
        tab, h = lt.make_table(W, c.x0, 300, 3)
        hp = lt.correction(h, W, c.x0, c.N)
        img = im.make_dirty_image(c.uv, vis, None, c.N, c.x0, tab, hp)
        s = img[np.ix_(sel, sel)]
        err = np.linalg.norm(s - dft) / np.linalg.norm(dft)
        lines.append(f"{W} {err:.6e}")
        print(f"W={W} rel_rms={err:.3e} ({time.time() - t0:.0f} s)", flush=True)
    out = os.path.join(HERE, "precision_reference_16m_4096.txt")
    with open(out, "w") as f:
        f.write("# Relative RMS error of the FP64 oracle dirty image against the direct DFT over the 256 x 256\n")
        f.write("# lattice of dft_samples_16m_4096.npy; 300-entry cubic tables, x0 = 1/4.\n")
        f.write("# Written by tests/golden/make_precision_reference.py (oracle only). Columns: W, rel_rms.\n")
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
