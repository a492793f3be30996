"""Writes the FP64 oracle's headline image to tests/golden/c2_headline.npz.

The headline workload: 200 x 200 px at 0.05"/px, supersampling 3, SIE +
external shear + 10,000 NFW subhalos, one lens-light and two source Sersic
components, 41 x 41 PSF (workloads.config2_scene(), seed 1002).  The file
holds `unconvolved` (the supersample-averaged image before the PSF) and
`convolved` (after it), both float64 (200, 200); c2_headline.sha256 holds the
SHA-256 of each array's bytes.

Only the oracle and the seeded input generators are called.  The 3.6e9
(sub-pixel, subhalo) pairs are split by pixel row over a process pool; every
pixel is computed exactly as oracle.simulate_unconvolved computes it (each
worker ray-shoots its own rows of the full sub-pixel grid).

Usage:  python tests/golden/make_c2.py [processes]
"""
import hashlib
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O          # noqa: E402
import workloads as W       # noqa: E402

OUT = os.path.join(HERE, "c2_headline.npz")
SUM = os.path.join(HERE, "c2_headline.sha256")


def _rows(args):
    r0, r1 = args
    sc = W.config2_scene()
    g = sc.grid
    tx, ty = O.subpixel_coords(g.nx, g.ny, g.pixel_scale, g.x0, g.y0, g.supersample)
    tx, ty = tx[r0:r1], ty[r0:r1]
    bx, by = O.ray_shoot(tx, ty, sc.lens)
    sb = O.surface_brightness(tx, ty, bx, by, sc.source, sc.lens_light, sc.bn_exact)
    return r0, O.supersample_reduce(sb, g.pixel_scale)


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else len(os.sched_getaffinity(0))
    sc = W.config2_scene()
    ny = sc.grid.ny
    bands = [(r, min(r + 2, ny)) for r in range(0, ny, 2)]
    un = np.empty((ny, sc.grid.nx))
    t0 = time.time()
    with get_context("fork").Pool(procs) as pool:
        for r0, part in pool.imap_unordered(_rows, bands):
            un[r0:r0 + part.shape[0]] = part
    conv = O.convolve_same(un, sc.psf)
    np.savez_compressed(OUT, unconvolved=un, convolved=conv)
    with open(SUM, "w") as f:
        f.write(f"unconvolved {digest(un)}\nconvolved {digest(conv)}\n")
    print(f"wrote {OUT} in {time.time() - t0:.1f} s on {procs} processes; "
          f"max {un.max():.6e} (unconvolved), {conv.max():.6e} (convolved)")


if __name__ == "__main__":
    main()
