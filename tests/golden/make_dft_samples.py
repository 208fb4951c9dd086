"""Writes dft_samples_16m_4096.npy: the direct-DFT dirty image (Eq. 3) of the
16,777,152-visibility array workload on a 4096^2 grid, sampled on the
256 x 256 lattice of pixels p, q = -1024 + 8 a (a = 0..255), every 8th pixel
of the retained field |x|, |y| < x0 = 1/4, as a complex128 array [q index,
p index] (numpy's .npy format, no pickled objects).

Calls only the oracle and the seeded input generator. The visibilities are
rounded to complex64 first, as the FP32 library paths receive them (the FP64
path receives the same values widened), with unit weights. Run from the
repository root:  python tests/golden/make_dft_samples.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import imaging as im  # noqa: E402

PIXELS = -1024 + 8 * np.arange(256)


def main():
    t0 = time.time()
    c = synth.array_16m_case(with_vis=True, device="cpu")
    vis = c.vis.astype(np.complex64).astype(np.complex128)
    img = im.dft_dirty_image(c.uv, vis, None, c.N, c.x0, pixels_x=PIXELS, pixels_y=PIXELS, chunk=1 << 15)
    out = os.path.join(HERE, "dft_samples_16m_4096.npy")
    np.save(out, img)
    print(f"wrote {out} in {time.time() - t0:.1f} s; sum |V|^2 = {np.sum(np.abs(vis) ** 2):.17e}")


if __name__ == "__main__":
    main()
