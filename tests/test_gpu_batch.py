"""Batched synthesis (persistent work-queue launches over many stars) through
the C ABI: bitwise equal to per-star calls, replayable from a hipGraph, and
matching the FP64 oracle on stars of the batched workload."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import synth as O

pytestmark = pytest.mark.gpu


class Star:
    """Device buffers and descriptor of one star."""

    def __init__(self, pz, wl, tile_px=0, target=False, seed=0, fam=False):
        self.wl = wl
        self.plan = pz.plan_for(wl, tile_px=tile_px, flags=pz.PZ_FLAG_DAMPING_FAMILIES if fam else 0)
        self.atm = pz.Atmos(wl.atm)
        self.par = pz.Params.from_host(wl.params)
        p = self.plan
        rng = np.random.default_rng(seed)
        d = "cuda"
        self.F = torch.full((p.N,), np.nan, device=d)
        self.Fc = torch.full((p.N,), np.nan, device=d)
        self.seed = torch.as_tensor(rng.normal(size=p.N).astype(np.float32) * 1e-6, device=d)
        self.y = torch.as_tensor(rng.uniform(0.3, 1.0, p.N).astype(np.float32), device=d) if target else None
        self.sigma = 0.01
        self.loss = torch.full((1,), np.nan, device=d)
        self.g = [torch.full((p.L,), np.nan, device=d), torch.full(((3 if fam else 1) * p.L,), np.nan, device=d),
                  torch.full((p.S,), np.nan, device=d), torch.full((1,), np.nan, device=d)]

    def descr(self, pz):
        ptr = lambda t: None if t is None else t.data_ptr()
        return pz.pz_star(self.plan.handle.value, self.atm.c, self.par.c, ptr(self.F), ptr(self.Fc),
                          ptr(self.seed), ptr(self.y), self.sigma, ptr(self.loss), *[ptr(x) for x in self.g])

    def outputs(self):
        out = [self.F, self.Fc] + self.g + ([self.loss] if self.y is not None else [])
        return [x.detach().cpu().numpy().copy() for x in out]

    def sequential(self, pz, mode):
        pz.synth_forward(self.plan, self.atm, self.par, self.F, self.Fc)
        seed = self.seed
        if self.y is not None:
            seed = torch.empty_like(self.F)
            pz.pz_chi2_seed(self.F, self.Fc, self.y, self.sigma, seed, None, self.loss)
        if mode == pz.PZ_MODE_FWD_BWD:
            pz.synth_backward(self.plan, self.atm, self.par, seed, *self.g)


def _stars(pz):
    specs = [dict(seed=41, L=30, N=700, D=72, tile=32), dict(seed=42, L=80, N=1500, D=72, tile=64),
             dict(seed=43, L=10, N=257, D=8, tile=128), dict(seed=44, L=0, N=300, D=72, tile=64),
             dict(seed=45, L=120, N=2500, D=40, tile=64), dict(seed=46, L=55, N=999, D=72, tile=128),
             dict(seed=47, L=40, N=600, D=72, tile=32, quad="e2"), dict(seed=48, L=70, N=1100, D=72, tile=32, eta=1e-3),
             dict(seed=49, L=50, N=800, D=72, tile=32, fam=True)]
    out = []
    for k, sp in enumerate(specs):
        wl = W.tiny(seed=sp["seed"], L=sp["L"], N=sp["N"], D=sp["D"], S=4, n_molecular=1)
        wl.quadrature = sp.get("quad", "gauss3")
        wl.center_eta = sp.get("eta", 0.0)
        wl.params = W.random_params(np.random.default_rng(k), wl.lines.L, wl.atm.S, 1.1 + 0.2 * k)
        if sp.get("fam"):
            wl.params.ddamp_family = np.random.default_rng(k + 100).normal(0.0, 0.2, (3, wl.lines.L))
        out.append(Star(pz, wl, sp["tile"], target=(k % 2 == 0), seed=k, fam=sp.get("fam", False)))
    return out


@pytest.mark.parametrize("mode", [1, 2])
def test_batch_bitwise_equals_per_star(gpu_lib, mode):
    pz = gpu_lib
    stars = _stars(pz)
    batch = pz.Batch([s.descr(pz) for s in stars])
    print("synth_batch mode", mode, flush=True)
    pz.synth_batch(batch, mode)
    torch.cuda.synchronize()
    got = [s.outputs() for s in stars]
    for s in stars:
        s.sequential(pz, mode)
    torch.cuda.synchronize()
    for k, s in enumerate(stars):
        ref = s.outputs()
        n = 2 if mode == 1 else len(ref)
        for a, b in zip(got[k][:n], ref[:n]):
            np.testing.assert_array_equal(a, b)
        if s.y is not None:
            np.testing.assert_array_equal(got[k][-1], ref[-1])
    batch.destroy()


def _scatter_stars(pz):
    """Two stars with continuum scattering (Eq. 6; one with a target and its
    chi^2 seed) beside a plain one."""
    import copy
    stars = []
    for k, (L, N, D, sig) in enumerate([(30, 600, 72, 0.7), (25, 500, 72, 0.0), (40, 700, 40, 2.0)]):
        wl = W.tiny(seed=91 + k, L=L, N=N, D=D, S=4, n_molecular=1)
        wl.params = W.random_params(np.random.default_rng(91 + k), L, 4, 1.3)
        if sig:
            wl.atm = copy.deepcopy(wl.atm)
            wl.atm.sigma_c = sig * (1.0 + 0.5 * np.sin(0.7 * np.arange(D)))
            wl.atm.sigma_alpha = 0.0
        stars.append(Star(pz, wl, 32, target=(k == 0), seed=k))
    return stars


@pytest.mark.parametrize("mode", [1, 2])
def test_batch_with_scattering_stars_bitwise(gpu_lib, mode):
    """Stars with continuum scattering in a batch: their transfer and reverse
    transfer run in launches of their own, bitwise equal to per-star calls."""
    pz = gpu_lib
    stars = _scatter_stars(pz)
    batch = pz.Batch([s.descr(pz) for s in stars])
    print("synth_batch with scattering stars, mode", mode, flush=True)
    pz.synth_batch(batch, mode)
    torch.cuda.synchronize()
    got = [s.outputs() for s in stars]
    for s in stars:
        s.sequential(pz, mode)
    torch.cuda.synchronize()
    for k, s in enumerate(stars):
        ref = s.outputs()
        n = 2 if mode == 1 else len(ref)
        for a, b in zip(got[k][:n], ref[:n]):
            np.testing.assert_array_equal(a, b)
        if s.y is not None:
            np.testing.assert_array_equal(got[k][-1], ref[-1])
    batch.destroy()


@pytest.mark.parametrize("chunk", [1, 3, 5])
def test_batch_small_lds_chunks_bitwise(gpu_lib, chunk):
    """The batch kernels' chunk loop (one body, the LDS buffer chosen at run
    time) against the single-star kernels' paired loop, with chunks of 1 to 5
    lines (tiles of 4 to 59 lines: chunk counts from 1 to 59): the same sums
    in the same order, so bitwise equal outputs."""
    pz = gpu_lib
    stars = []
    for k, (L, D, tile) in enumerate([(61, 72, 32), (20, 72, 64), (9, 40, 32)]):
        wl = W.tiny(seed=76 + k, L=L, N=400, D=D, S=4, n_molecular=1)
        wl.params = W.random_params(np.random.default_rng(76 + k), L, 4, 1.2)
        st = Star(pz, wl, tile, target=(k == 0), seed=k)
        st.plan = pz.plan_for(wl, tile_px=tile, lines_per_chunk=chunk)
        stars.append(st)
    batch = pz.Batch([s.descr(pz) for s in stars])
    print("synth_batch chunk", chunk, flush=True)
    pz.synth_batch(batch, pz.PZ_MODE_FWD_BWD)
    torch.cuda.synchronize()
    got = [s.outputs() for s in stars]
    for s in stars:
        s.sequential(pz, pz.PZ_MODE_FWD_BWD)
    torch.cuda.synchronize()
    for k, s in enumerate(stars):
        for a, b in zip(got[k], s.outputs()):
            np.testing.assert_array_equal(a, b)
    batch.destroy()


@pytest.mark.parametrize("which", ["plain", "scattering"])
def test_batch_graph_replay(gpu_lib, which):
    """The whole forward+backward batch captured in one graph; every replay
    (with eager work and synchronisations in between) equals the eager run."""
    pz = gpu_lib
    stars = _stars(pz) if which == "plain" else _scatter_stars(pz)
    batch = pz.Batch([s.descr(pz) for s in stars])
    pz.synth_batch(batch, pz.PZ_MODE_FWD_BWD)
    torch.cuda.synchronize()
    eager = [s.outputs() for s in stars]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pz.synth_batch(batch, pz.PZ_MODE_FWD_BWD)   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        pz.synth_batch(batch, pz.PZ_MODE_FWD_BWD)
    for rep in range(3):
        for s in stars:                              # eager work between replays
            s.F.fill_(np.nan)
            for x in s.g:
                x.fill_(np.nan)
        torch.cuda.synchronize()
        print("graph replay", rep, flush=True)
        g.replay()
        torch.cuda.synchronize()
        for k, s in enumerate(stars):
            for a, b in zip(s.outputs(), eager[k]):
                np.testing.assert_array_equal(a, b)
    del g
    batch.destroy()


from test_gpu_adjoint import grad_close_cond


def test_batch_stars_vs_oracle(gpu_lib):
    """Eight stars of the batched 1500-1700 nm workload (own atmosphere, window
    length and line count each): sampled pixels against the oracle at 1e-4;
    three of them also sampled-line gradients against the oracle adjoint."""
    pz = gpu_lib
    stars = [Star(pz, W.batch_star(b), seed=b) for b in (0, 1, 2, 3, 100, 101, 200, 255)]
    batch = pz.Batch([s.descr(pz) for s in stars])
    print("synth_batch 8 stars", [s.plan.N for s in stars], [s.plan.L for s in stars], flush=True)
    pz.synth_batch(batch, pz.PZ_MODE_FWD_BWD)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    for k, s in enumerate(stars):
        F, Fc = s.F.cpu().numpy().astype(np.float64), s.Fc.cpu().numpy().astype(np.float64)
        pix = np.unique(np.concatenate([[0, s.plan.N - 1], rng.integers(0, s.plan.N, 24)]))
        Fo, Fco = O.synthesize(s.wl, pix=pix)
        for got, ref in ((F[pix], Fo), (Fc[pix], Fco), (F[pix] / Fc[pix], Fo / Fco)):
            assert np.max(np.abs(got - ref) / ref) <= 1e-4
        if k < 3:
            L = s.plan.L
            lines = rng.choice(L, 6, replace=False)
            wpix = O.window_pixels(s.wl, lines)
            seed = s.seed.cpu().numpy().astype(np.float64)
            ref = O.adjoint(s.wl, s.wl.params, seed[wpix], pix=wpix, line_subset=lines, conditions=True)
            grad_close_cond(s.g[0].cpu().numpy()[lines], ref["g_loggf"][lines], ref["abs_loggf"][lines], name="gf")
            grad_close_cond(s.g[1].cpu().numpy()[lines], ref["g_damp"][lines], ref["abs_damp"][lines], name="damp")
    batch.destroy()


def test_autotune_returns_supported_config(gpu_lib):
    pz = gpu_lib
    wl = W.tiny(seed=9, L=300, N=3000, D=72)
    tile, chunk, ms = pz.pz_autotune(wl.grid, wl.lines, wl.atm.S, wl.atm.D, pz.Atmos(wl.atm),
                                     pz.Params.from_host(wl.params), reps=2)
    assert tile in (32, 64, 128) and chunk in (8, 16) and ms > 0


def test_batch_stars_every_pixel_vs_golden(gpu_lib):
    """Three stars of the batch (stars 0, 101 and 255) in one synth_batch
    call: every pixel of F, F_c and f against the oracle's full spectra
    (tests/golden/flux_batch_stars_golden.npz) at 1e-4."""
    import os
    pz = gpu_lib
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", "flux_batch_stars_golden.npz"))
    ids = [int(b) for b in z["stars"]]
    stars = [Star(pz, W.batch_star(b), seed=b) for b in ids]
    batch = pz.Batch([s.descr(pz) for s in stars])
    print("synth_batch stars", ids, [s.plan.N for s in stars], flush=True)
    pz.synth_batch(batch, pz.PZ_MODE_FWD)
    torch.cuda.synchronize()
    for b, s in zip(ids, stars):
        F, Fc = s.F.cpu().numpy().astype(np.float64), s.Fc.cpu().numpy().astype(np.float64)
        Fo, Fco = z["F_%d" % b], z["Fc_%d" % b]
        errs = [np.max(np.abs(got - ref) / ref) for got, ref in ((F, Fo), (Fc, Fco), (F / Fc, Fo / Fco))]
        print("star", b, "max rel err F, Fc, f", errs, flush=True)
        assert max(errs) <= 1e-4
    batch.destroy()
