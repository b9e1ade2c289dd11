"""Writes fit_1500_1700nm_golden.npz: FP64 oracle reference for differentiating the
1500-1700 nm workload (37,550 pixels, 2e5 lines, 20 species) through a chi^2
loss at S/N = 100 (Sec. 5 objective, Eq. 9 ratio, Eq. 30 corrections).

Calls only oracle/ and workloads/.  Contents:
  y        float32 [N]  target: f(truth corrections) + N(0, 0.01^2) noise
  seed     float32 [N]  dL/dF of L = sum((F/Fc - y)/sigma)^2 at the base corrections
  loss     float64      L at the base corrections
  lines    int          sampled line indices (caller order)
  g_loggf, g_damp, abs_loggf, abs_damp   oracle adjoint (and sum|terms|) at those lines
  g_abund, abs_abund [20], g_xi, abs_xi  species and microturbulence
  fd_kind, fd_index, fd_value, fd_value_half   FP64 central differences of L for
           50 parameters (20 log gf, 20 damping, 9 abundances, xi) with steps h and h/2,
           the loss change summed per pixel (no cancellation against the whole loss)
The adjoint is evaluated with the float32 seed (as a float64 copy), exactly the
input the GPU test passes to synth_backward.

Usage: python tests/golden/make_fit_1500_1700nm_golden.py [--procs 8]   (about 15 min on 8 cores)
"""
import argparse
import copy
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


def _init():
    global WL
    WL = W.giant_1500_1700nm_fit()


def _fwd(args):
    params, pix = args
    return O.synthesize(WL, params, pix=pix)


def _adj(args):
    params, pix, seed = args
    r = O.adjoint(WL, params, seed, pix=pix, conditions=True)
    return r["g_loggf"], r["g_damp"], r["g_xi"], r["abs_loggf"], r["abs_damp"], r["abs_xi"]


def _chunks(N, n):
    return [np.arange(a, min(N, a + n)) for a in range(0, N, n)]


def forward_all(pool, params, N):
    parts = pool.map(_fwd, [(params, c) for c in _chunks(N, 512)])
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def loss_of(F, Fc, y, sigma):
    return float(np.sum(((F / Fc - y) / sigma) ** 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--out", default=os.path.join(HERE, "fit_1500_1700nm_golden.npz"))
    args = ap.parse_args()
    t0 = time.time()
    _init()
    wl = WL
    N, L, S = wl.grid.N, wl.lines.L, wl.atm.S
    sigma = wl.extra["sigma"]
    base = wl.params
    with get_context("fork").Pool(args.procs, initializer=_init) as pool:
        Ft, Fct = forward_all(pool, wl.extra["truth"], N)
        y = (Ft / Fct + wl.extra["noise"]).astype(np.float32)
        print("truth forward %.0f s" % (time.time() - t0), flush=True)
        F, Fc = forward_all(pool, base, N)
        yd = y.astype(np.float64)
        loss = loss_of(F, Fc, yd, sigma)
        dF, _ = O.chi2_seed(F, Fc, yd, sigma)
        seed = dF.astype(np.float32)
        s64 = seed.astype(np.float64)
        print("base forward %.0f s, loss %.6e" % (time.time() - t0, loss), flush=True)
        parts = pool.map(_adj, [(base, c, s64[c]) for c in _chunks(N, 512)])
        Ggf = sum(p[0] for p in parts)
        Gd = sum(p[1] for p in parts)
        Gxi = sum(p[2] for p in parts)
        Agf = sum(p[3] for p in parts)
        Ad = sum(p[4] for p in parts)
        Axi = sum(p[5] for p in parts)
        GA = np.zeros(S)
        AA = np.zeros(S)
        np.add.at(GA, wl.lines.species, Ggf)
        np.add.at(AA, wl.lines.species, Agf)
        print("adjoint %.0f s" % (time.time() - t0), flush=True)

        rng = np.random.default_rng(424242)
        lines = np.unique(np.concatenate([rng.choice(L, 256, replace=False),
                                          np.argsort(-np.abs(Ggf))[:32]]))
        # finite differences: 20 log gf and 20 damping (half random, half among the
        # 200 largest |gradient|), 9 abundances, xi.  The loss change is summed per
        # pixel as (f+ - f-)(f+ + f- - 2y)/sigma^2, which has no cancellation against
        # the whole loss; pixels outside a line's window do not change.
        top = np.argsort(-np.abs(Ggf))[:200]
        fd_lines_gf = np.concatenate([rng.choice(L, 10, replace=False), rng.choice(top, 10, replace=False)])
        topd = np.argsort(-np.abs(Gd))[:200]
        fd_lines_d = np.concatenate([rng.choice(L, 10, replace=False), rng.choice(topd, 10, replace=False)])
        fd_species = rng.choice(S, 9, replace=False)
        kinds, idx, val, val_half = [], [], [], []

        def _local(params, pix):
            parts = pool.map(_fwd, [(params, c) for c in np.array_split(pix, args.procs)])
            return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])

        def loss_change(p1, p2, pix):
            if pix is None:
                F1, Fc1 = forward_all(pool, p1, N)
                F2, Fc2 = forward_all(pool, p2, N)
                yy = yd
            else:
                F1, Fc1 = _local(p1, pix)
                F2, Fc2 = _local(p2, pix)
                yy = yd[pix]
            f1, f2 = F1 / Fc1, F2 / Fc2
            return float(np.sum((f1 - f2) * (f1 + f2 - 2.0 * yy)) / sigma ** 2)

        def central(setter, h, pix):
            p1, p2 = copy.deepcopy(base), copy.deepcopy(base)
            setter(p1, h)
            setter(p2, -h)
            return loss_change(p1, p2, pix) / (2 * h)

        for kind, arr in (("loggf", fd_lines_gf), ("damp", fd_lines_d)):
            for l in arr:
                pix = O.window_pixels(wl, [l])
                if kind == "loggf":
                    def st(p, h, l=l):
                        p.dgf[l] += h
                else:
                    def st(p, h, l=l):
                        p.ddamp[l] += h
                kinds.append(kind)
                idx.append(int(l))
                val.append(central(st, 1e-3, pix))
                val_half.append(central(st, 5e-4, pix))
        print("line FD %.0f s" % (time.time() - t0), flush=True)
        for sp in fd_species:
            def st(p, h, sp=sp):
                p.dA[sp] += h
            kinds.append("abund")
            idx.append(int(sp))
            val.append(central(st, 1e-3, None))
            val_half.append(central(st, 5e-4, None))
            print("abundance %d FD %.0f s" % (sp, time.time() - t0), flush=True)

        def stx(p, h):
            p.xi_kms += h
        kinds.append("xi")
        idx.append(0)
        val.append(central(stx, 1e-3, None))
        val_half.append(central(stx, 5e-4, None))
    np.savez_compressed(
        args.out, y=y, seed=seed, loss=loss, lines=lines,
        g_loggf=Ggf[lines], g_damp=Gd[lines], abs_loggf=Agf[lines], abs_damp=Ad[lines],
        g_abund=GA, abs_abund=AA, g_xi=float(np.sum(Gxi)), abs_xi=float(np.sum(Axi)),
        fd_kind=np.array(kinds), fd_index=np.array(idx), fd_value=np.array(val), fd_value_half=np.array(val_half),
        fd_adjoint=np.array([Ggf[i] if k == "loggf" else Gd[i] if k == "damp" else GA[i] if k == "abund"
                             else float(np.sum(Gxi)) for k, i in zip(kinds, idx)]),
        fd_abs=np.array([Agf[i] if k == "loggf" else Ad[i] if k == "damp" else AA[i] if k == "abund"
                         else float(np.sum(Axi)) for k, i in zip(kinds, idx)]))
    print("wrote %s in %.0f s" % (args.out, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
