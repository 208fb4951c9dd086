"""Writes dft_multichannel.npz: for four channels (0, 85, 170, 255) of the 256-channel workload (1024^2 grids,
log-uniform visibility counts, complex64 N(0, 1) visibilities of seed 55, unit weights), the direct-DFT dirty
image (Eq. 3) on the 64 x 64 lattice p, q = -256 + 8 a (every 8th pixel of the retained 512^2 field, x0 = 1/4),
as complex128 arrays 'chan_<c>' [q index, p index] (numpy's .npz, no pickled objects).

Calls only the oracle and the seeded input generators. Run from the repository root:
python tests/golden/make_multichannel_dft.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import imaging as im  # noqa: E402

CHANNELS = (0, 85, 170, 255)
PIXELS = -256 + 8 * np.arange(64)


def main():
    uv, off, _ = synth.multichannel_case()
    vis = synth.multichannel_vis(len(uv)).astype(np.complex128)
    out = {}
    for c in CHANNELS:
        a, b = int(off[c]), int(off[c + 1])
        out[f"chan_{c}"] = im.dft_dirty_image(uv[a:b], vis[a:b], None, 1024, 0.25, PIXELS, PIXELS)
        print(f"channel {c}: {b - a} visibilities", flush=True)
    np.savez(os.path.join(HERE, "dft_multichannel.npz"), **out)


if __name__ == "__main__":
    main()
