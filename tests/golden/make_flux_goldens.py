"""Writes the full-pixel flux goldens of the two FP32 forward workloads from the
FP64 oracle (Sec. 2.1 Eqs. 1-9; the plain windowed sum, Gauss-3 in mu):

  flux_1500_1700nm_golden.npz   every pixel of the 1500-1700 nm workload
                                (37,550 pixels, 2e5 lines, 72 depths):
                                F, Fc float64 [N]
  flux_300_1000nm_slices_golden.npz  three exact 2-nm slices of the 300-1000 nm
                                workload (361,193 pixels, 5e6 lines): the blue
                                end from 300 nm, the middle from 650 nm and the
                                red end up to 1000 nm.  pix int64 [n], F, Fc
                                float64 [n].  A pixel's flux depends only on the
                                lines within W of it, so a slice of the oracle is
                                exactly that part of the whole spectrum.
  flux_batch_stars_golden.npz   every pixel of three stars of the 256-star
                                batch (stars 0, 101 and 255: their own
                                atmospheres, windows and catalogues):
                                F_<b>, Fc_<b> float64 [N_b]

Calls only oracle/ and workloads/ (seeded generators).

Usage: python tests/golden/make_flux_goldens.py [--procs 8]   (a few minutes on 8 cores)
"""
import argparse
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import synth as O  # noqa: E402

WL = None
BATCH_STARS = (0, 101, 255)
SLICE_STARTS_NM = (300.0, 650.0, None)   # None: the slice that ends at the last pixel
SLICE_NM = 2.0


def _init(name):
    global WL
    if name == "1500_1700":
        WL = W.giant_1500_1700nm()
    elif name == "300_1000":
        WL = W.solar_300_1000nm()
    else:
        WL = W.batch_star(int(name.split("_")[1]))


def _fwd(pix):
    return O.synthesize(WL, pix=pix)


def slice_pixels(grid):
    """The pixel indices of the three 2-nm slices of the 300-1000 nm grid."""
    lam = O.wavelengths_nm(grid)
    out = []
    for lo in SLICE_STARTS_NM:
        if lo is None:
            i1 = grid.N
            i0 = int(np.searchsorted(lam, lam[-1] - SLICE_NM, side="left"))
        else:
            i0 = int(np.searchsorted(lam, lo, side="left"))
            i1 = int(np.searchsorted(lam, lo + SLICE_NM, side="left"))
        out.append(np.arange(i0, i1, dtype=np.int64))
    return out


def run(name, pix, procs, chunk):
    parts = [pix[a:a + chunk] for a in range(0, pix.size, chunk)]
    with get_context("fork").Pool(procs, initializer=_init, initargs=(name,)) as pool:
        res = pool.map(_fwd, parts, chunksize=1)
    return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--only", choices=["1500_1700", "300_1000", "batch"], default=None)
    args = ap.parse_args()
    if args.only in (None, "1500_1700"):
        t0 = time.time()
        wl = W.giant_1500_1700nm()
        F, Fc = run("1500_1700", np.arange(wl.grid.N, dtype=np.int64), args.procs, 256)
        np.savez_compressed(os.path.join(HERE, "flux_1500_1700nm_golden.npz"), F=F, Fc=Fc,
                            workload=wl.name)
        print("1500-1700 nm: %d pixels, %.0f s" % (F.size, time.time() - t0), flush=True)
    if args.only in (None, "300_1000"):
        t0 = time.time()
        wl = W.solar_300_1000nm()
        pix = np.concatenate(slice_pixels(wl.grid))
        F, Fc = run("300_1000", pix, args.procs, 64)
        np.savez_compressed(os.path.join(HERE, "flux_300_1000nm_slices_golden.npz"), pix=pix, F=F, Fc=Fc,
                            workload=wl.name)
        print("300-1000 nm slices: %d pixels, %.0f s" % (F.size, time.time() - t0), flush=True)
    if args.only in (None, "batch"):
        t0 = time.time()
        out = {}
        for b in BATCH_STARS:
            wl = W.batch_star(b)
            F, Fc = run("star_%d" % b, np.arange(wl.grid.N, dtype=np.int64), args.procs, 256)
            out["F_%d" % b], out["Fc_%d" % b] = F, Fc
        np.savez_compressed(os.path.join(HERE, "flux_batch_stars_golden.npz"), stars=np.array(BATCH_STARS), **out)
        print("batch stars %s: %.0f s" % (BATCH_STARS, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
