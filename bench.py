"""Benchmark of the MI355X synthesis path (one JSON line on stdout).

value: forward spectra/s on the 1500-1700 nm, R = 300,000 workload (37,550
pixels x 72 depths, 2e5 lines, 30 % in molecular-band-like sequences), inputs
resident in HBM, K timed steps between device synchronisations.  A step is
one whole forward synthesis (populations, line parameters, windowed Voigt
opacity, depth scan and Gauss-3 flux for both branches).  Extra fields: the
forward+backward step (chi^2 loss seed and the adjoint for all 4e5 + 20 + 1
corrections), the centre test, continuum scattering (the source function
iterated to its fixed point, forward and forward+backward), the exact E2
angle integral instead of Gauss-3, the line-selection keep test (and the
forward of its kept subset), the instrument operator, the line calibration
(objective evaluation and L-BFGS updates over 25,147 correction groups of a
two-star, three-spectrum fit) and the batched launch over 256 stars, the roofline of the
dominant kernel (opacity) and the FP64 CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                      [--modes fwd,fwdbwd,center,select,scatter,e2,instrument,calibration,batch] [--cal-updates 40] [--no-cpu]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spectra/s, Voigt evals/s: fwd, fwd+bwd, batched vs plain fwd at 1e-4 rel"
# Algorithmic float32 operations of one Voigt evaluation (one line, one depth,
# one in-window pixel) in the wing formula, FMA = 2: detuning scale and u = v^2
# (2), a^2, u - a^2, 4 u a^2, u + a^2 (5), three node pairs x (sub, FMA, add, mul,
# rcp, FMA = 8), a * sum (1), kappa += K H (2).
FLOPS_PER_EVAL = 34
PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector peak
# sources of the opacity kernel: a committed HBM-traffic measurement is used only if they are unchanged
# The opacity kernel's code: its tile body and the Voigt evaluator, plus the
# kernel's own definition in pz_kernels.hip (other code in that file is not
# part of it).
KERNEL_SOURCES = ("paper_2607_24141_amd/csrc/pz_opacity.h", "paper_2607_24141_amd/csrc/pz_voigt.h",
                  "paper_2607_24141_amd/csrc/voigt_consts.h")
KERNEL_DEF = ("paper_2607_24141_amd/csrc/pz_kernels.hip", "void k_opacity(")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, KERNEL_DEF[0])) as fh:
        txt = fh.read()
    i = txt.index(KERNEL_DEF[1])
    i = txt.rindex("\n", 0, txt.rindex("\n", 0, i)) + 1      # from the template line above
    h.update(txt[i:txt.index("\n}\n", i) + 3].encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(kind="opacity"):
    """HBM bytes per launch from the committed counter summary, if it was taken on these sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kind)
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def cpu_baseline(wl, target_s=12.0):
    """The FP64 oracle on a bounded pixel sample of the same workload, scaled to spectra/s."""
    import numpy as np
    from oracle import synth as O
    rng = np.random.default_rng(0)
    done, t = 0, 0.0
    while t < target_s and done < wl.grid.N:
        pix = np.sort(rng.choice(wl.grid.N, 32, replace=False))
        t0 = time.perf_counter()
        O.synthesize(wl, pix=pix)
        t += time.perf_counter() - t0
        done += pix.size
    per_spectrum = t / done * wl.grid.N
    return {"value": 1.0 / per_spectrum, "unit": "spectra/s", "cores": 1, "kind": "oracle",
            "sample": "%d random pixels of the %d-pixel spectrum (all lines within W of each), "
                      "%.1f s of single-threaded numpy/scipy FP64, scaled to the full spectrum"
                      % (done, wl.grid.N, t),
            "voigt_evals_per_s": None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--modes", default="fwd,fwdbwd,center,select,scatter,e2,instrument,calibration,batch")
    ap.add_argument("--cal-updates", type=int, default=40, help="L-BFGS updates of the calibration block")
    ap.add_argument("--batch-stars", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run a plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    modes = set(args.modes.split(","))

    import numpy as np
    import torch

    import paper_2607_24141_amd as pz
    import workloads as W

    torch.cuda.set_device(0)
    dev = "cuda"
    log("generating 1500-1700 nm workload")
    wl = W.giant_1500_1700nm_fit()
    atm = pz.Atmos(wl.atm)
    par = pz.Params.from_host(wl.params)
    plan = pz.plan_tuned(wl, atm, par)
    N, L, S = plan.N, plan.L, plan.S
    F = torch.empty(N, dtype=torch.float32, device=dev)
    Fc = torch.empty_like(F)

    # ---- forward (the headline)
    log("forward: N=%d L=%d evals=%.3e" % (N, L, plan.voigt_evals))
    fwd = lambda: pz.synth_forward(plan, atm, par, F, Fc)
    fwd()
    torch.cuda.synchronize()
    plan.profile(True)
    ms_fwd, wall_fwd = timed(fwd, args.steps, args.warmup, torch)
    prof = plan.profile_read()
    plan.profile(False)
    op_ms, op_n = prof["opacity"]
    op_avg_ms = op_ms / max(op_n, 1)
    achieved_tflops = plan.voigt_evals * FLOPS_PER_EVAL / (op_avg_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": 1000.0 / ms_fwd,
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_fwd,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name.replace("_fwdbwd", ""), "lambda_nm": [1500, 1700], "R": 3.0e5,
                   "N": N, "D": plan.D, "L": L, "S": S, "window_nm": wl.window_nm, "quadrature": "gauss3",
                   "mode": "fwd", "tile_px": plan.tile_px, "autotune_key": pz.tune_key(wl)},
        "voigt_evals_per_s": plan.voigt_evals / (ms_fwd * 1e-3),
        "stage_ms": {k: (v[0] / max(v[1], 1)) for k, v in prof.items() if v[1]},
        "roofline": {"bound": "alu", "kernel": "k_opacity", "achieved": achieved_tflops,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP32_TFLOPS,
                     "traffic": traffic_from_profiles("opacity"), "kernel_avg_ms": op_avg_ms,
                     "flops_per_eval": FLOPS_PER_EVAL, "evals_per_launch": plan.voigt_evals},
        "wall_s_timed": wall_fwd,
    }

    # ---- forward + backward with the chi^2 loss (S/N = 100)
    if "fwdbwd" in modes:
        sigma = wl.extra["sigma"]
        y = torch.as_tensor(np.ones(N, np.float32), device=dev)
        # target: synthesis at the perturbed (truth) corrections plus noise
        tpar = pz.Params.from_host(wl.extra["truth"])
        Ft, Fct = torch.empty_like(F), torch.empty_like(F)
        pz.synth_forward(plan, atm, tpar, Ft, Fct)
        y = (Ft / Fct + torch.as_tensor(wl.extra["noise"].astype(np.float32), device=dev)).contiguous()
        gF = torch.empty_like(F)
        gFc = torch.empty_like(F)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        g = [torch.empty(L, device=dev), torch.empty(L, device=dev), torch.empty(S, device=dev),
             torch.empty(1, device=dev)]

        def fb():
            pz.synth_forward(plan, atm, par, F, Fc)
            pz.pz_chi2_seed(F, Fc, y, sigma, gF, gFc, loss)
            pz.synth_backward(plan, atm, par, gF, *g)

        log("forward+backward")
        plan.profile(True)
        ms_fb, _ = timed(fb, args.steps, args.warmup, torch)
        prof_fb = plan.profile_read()
        plan.profile(False)
        out["fwd_bwd"] = {"spectra_per_s": 1000.0 / ms_fb, "ms_per_step": ms_fb, "ratio_to_fwd": ms_fb / ms_fwd,
                          "voigt_evals_per_s": 2 * plan.voigt_evals / (ms_fb * 1e-3),
                          "stage_ms": {k: (v[0] / max(v[1], 1)) for k, v in prof_fb.items() if v[1]}}

    # ---- the continuum-referenced centre test (a different result by design)
    if "center" in modes:
        eta = 1.0e-3
        log("centre test, eta = %g" % eta)
        f_plain = (F / Fc).clone()
        cplan = pz.plan_for(wl, tile_px=plan.tile_px, lines_per_chunk=16, center_eta=eta)
        cf = lambda: pz.synth_forward(cplan, atm, par, F, Fc)
        cf()
        torch.cuda.synchronize()
        dmax = float(torch.max(torch.abs(F / Fc - f_plain)).item())
        ms_cf, _ = timed(cf, args.steps, args.warmup, torch)
        out["center_test"] = {"eta": eta, "fwd_spectra_per_s": 1000.0 / ms_cf, "fwd_ms": ms_cf,
                              "speedup_vs_plain_fwd": ms_fwd / ms_cf, "max_abs_dflux_vs_plain": dmax}
        if "fwdbwd" in modes:
            gFc_ = torch.empty_like(F)

            def cfb():
                pz.synth_forward(cplan, atm, par, F, Fc)
                pz.pz_chi2_seed(F, Fc, y, sigma, gF, gFc_, loss)
                pz.synth_backward(cplan, atm, par, gF, *g)

            ms_cfb, _ = timed(cfb, args.steps, args.warmup, torch)
            out["center_test"].update({"fwd_bwd_spectra_per_s": 1000.0 / ms_cfb, "fwd_bwd_ms": ms_cfb,
                                       "speedup_vs_plain_fwd_bwd": out["fwd_bwd"]["ms_per_step"] / ms_cfb})
        cplan.destroy()

    # ---- the line-selection keep test of Eqs. 17-19, then synthesis of the kept subset
    if "select" in modes:
        eta_sel, bin_ln = 1.0e-3, 1.0e-3
        keep_t = torch.empty(L, dtype=torch.uint8, device=dev)
        nk = torch.empty(1, dtype=torch.int32, device=dev)
        ms_sel, _ = timed(lambda: pz.pz_select_lines(plan, atm, par, eta_sel, bin_ln, keep=keep_t, n_keep=nk),
                          args.steps, args.warmup, torch)
        keep = keep_t.cpu().numpy().astype(bool)
        idx = np.flatnonzero(keep)
        sub = W.Workload(wl.name + "_selected", wl.grid, wl.atm, wl.lines.take(idx),
                         W.Params(wl.params.dgf[idx], wl.params.ddamp[idx], wl.params.dA, wl.params.xi_kms),
                         window_nm=wl.window_nm)
        splan = pz.plan_for(sub, tile_px=plan.tile_px)
        spar = pz.Params.from_host(sub.params)
        pz.synth_forward(plan, atm, par, F, Fc)
        f_full, F_full = (F / Fc).clone(), F.clone()
        sf = lambda: pz.synth_forward(splan, atm, spar, F, Fc)
        sf()
        torch.cuda.synchronize()
        dmax = float(torch.max(torch.abs(F / Fc - f_full)).item())
        dF_rel = float(torch.max(torch.abs(F - F_full) / F_full).item())
        n_diff = int((F != F_full).sum().item())
        ms_sf, _ = timed(sf, args.steps, args.warmup, torch)
        out["selection"] = {"eta_sel": eta_sel, "bin_ln": bin_ln, "select_ms": ms_sel, "kept": int(idx.size),
                            "kept_fraction": idx.size / L, "fwd_ms_selected": ms_sf,
                            "speedup_vs_full_fwd": ms_fwd / ms_sf, "max_abs_dflux_vs_full": dmax,
                            "max_rel_dF_vs_full": dF_rel, "pixels_changed": n_diff}
        splan.destroy()

    # ---- transfer with continuum scattering (Eq. 6 iterated to its fixed point), same lines
    if "scatter" in modes:
        import copy
        swl = copy.deepcopy(wl)
        swl.atm.sigma_c = np.full(wl.atm.D, 0.5 * wl.atm.kappa0)     # grey scattering, half the continuum
        swl.atm.sigma_alpha = 0.0
        splan = pz.plan_for(swl, tile_px=plan.tile_px)
        satm = pz.Atmos(swl.atm)
        sfwd = lambda: pz.synth_forward(splan, satm, par, F, Fc)
        splan.profile(True)
        ms_sf, _ = timed(sfwd, args.steps, args.warmup, torch)
        sprof = splan.profile_read()
        splan.profile(False)
        it_f = splan.scatter_iterations()
        gS = torch.empty_like(F)
        gl = [torch.empty(L, device=dev), torch.empty(L, device=dev), torch.empty(S, device=dev),
              torch.empty(1, device=dev)]
        ys = torch.ones_like(F)

        def sfb():
            pz.synth_forward(splan, satm, par, F, Fc)
            pz.pz_chi2_seed(F, Fc, ys, 0.01, gS, None, None)
            pz.synth_backward(splan, satm, par, gS, *gl)

        splan.profile(True)
        ms_sfb, _ = timed(sfb, args.steps, args.warmup, torch)
        sprof_b = splan.profile_read()
        splan.profile(False)
        it_b = splan.scatter_iterations()
        out["scattering"] = {"sigma_c_over_kappa_c": 0.5, "fwd_spectra_per_s": 1000.0 / ms_sf, "fwd_ms": ms_sf,
                             "fwd_bwd_spectra_per_s": 1000.0 / ms_sfb, "fwd_bwd_ms": ms_sfb,
                             "flux_stage_ms": sprof["flux"][0] / max(sprof["flux"][1], 1),
                             "max_iterations_fwd": [int(it_f[0]), int(it_f[1])],
                             "max_iterations_adjoint": int(it_b[2]),
                             "stage_ms_fwd_bwd": {k: (v[0] / max(v[1], 1)) for k, v in sprof_b.items() if v[1]}}
        splan.destroy()

    # ---- the same workload with the exact E2 angle integral (float64 transfer)
    if "e2" in modes:
        import copy
        ewl = copy.copy(wl)
        ewl.quadrature = "e2"
        eplan = pz.plan_for(ewl, tile_px=plan.tile_px)
        efwd = lambda: pz.synth_forward(eplan, atm, par, F, Fc)
        eplan.profile(True)
        ms_ef, _ = timed(efwd, args.steps, args.warmup, torch)
        eprof = eplan.profile_read()
        eplan.profile(False)
        egF = torch.empty_like(F)
        eg = [torch.empty(L, device=dev), torch.empty(L, device=dev), torch.empty(S, device=dev),
              torch.empty(1, device=dev)]
        eys = torch.ones_like(F)

        def efb():
            pz.synth_forward(eplan, atm, par, F, Fc)
            pz.pz_chi2_seed(F, Fc, eys, 0.01, egF, None, None)
            pz.synth_backward(eplan, atm, par, egF, *eg)

        eplan.profile(True)
        ms_efb, _ = timed(efb, args.steps, args.warmup, torch)
        eprof_b = eplan.profile_read()
        eplan.profile(False)
        out["e2"] = {"fwd_spectra_per_s": 1000.0 / ms_ef, "fwd_ms": ms_ef,
                     "fwd_bwd_spectra_per_s": 1000.0 / ms_efb, "fwd_bwd_ms": ms_efb,
                     "stage_ms_fwd": {k: (v[0] / max(v[1], 1)) for k, v in eprof.items() if v[1]},
                     "stage_ms_fwd_bwd": {k: (v[0] / max(v[1], 1)) for k, v in eprof_b.items() if v[1]}}
        eplan.destroy()

    # ---- the instrument operator of Eq. 31 on APOGEE-like pixels (one flux pair)
    if "instrument" in modes:
        lam_obs, sig, vbmax = W.apogee_instrument(wl.grid)
        inst = pz.Instrument(wl.grid, lam_obs, sig, vbmax)
        vel = torch.tensor([12.0, 6.0], dtype=torch.float32, device=dev)
        fobs = torch.empty(inst.P, dtype=torch.float32, device=dev)
        dFi, dFci = torch.empty_like(F), torch.empty_like(F)
        gv = torch.empty(2, dtype=torch.float32, device=dev)
        iseed = torch.randn(inst.P, dtype=torch.float32, device=dev)
        ms_if, _ = timed(lambda: pz.pz_inst_forward(inst, F, Fc, vel, None, None, fobs), args.steps, args.warmup, torch)
        ms_ib, _ = timed(lambda: pz.pz_inst_backward(inst, F, Fc, vel, iseed, dFi, dFci, gv), args.steps,
                         args.warmup, torch)
        out["instrument"] = {"observed_pixels": inst.P, "native_pixels": int(F.numel()),
                             "fwd_us_per_flux_pair": ms_if * 1e3, "bwd_us_per_flux_pair": ms_ib * 1e3}
        inst.destroy()

    # ---- line calibration (Sec. 6): two stars, three spectra, shared group corrections, L-BFGS
    if "calibration" in modes:
        from paper_2607_24141_amd import calibrate as CAL
        log("calibration workload")
        cw = W.calibration()
        t0 = time.perf_counter()
        q, G = pz.correction_groups(cw.lines, W.CAL_DE_CM, W.CAL_DLAM_NM, active=cw.active)
        t_group = time.perf_counter() - t0
        gc = CAL.Calibration(cw, groups=(q, G))
        truth = W.calibration_truth(np.random.default_rng(11), G)
        cal_sigma = 2e-3
        gc.set_observed(CAL.mock_observed(gc, truth, cal_sigma, seed=12))
        theta0 = torch.zeros(4, G, device=dev)
        ms_eval, _ = timed(lambda: gc.evaluate(theta0), args.steps, args.warmup, torch)
        log("calibration: %d groups, %.2f ms per evaluation; L-BFGS" % (G, ms_eval))
        r = CAL.fit(gc, max_iter=args.cal_updates)
        out["calibration"] = {
            "workload": cw.name, "records": int(cw.active.sum()), "lines": int(cw.lines.L), "groups": int(G),
            "corrections": 4 * int(G), "spectra": len(gc.epochs), "syntheses_per_eval": len(gc.stars),
            "grouping_ms": t_group * 1e3, "ms_per_eval": ms_eval,
            "lbfgs": {"updates": r["iters"], "evals": r["evals"], "seconds": r["seconds"],
                      "ms_per_update": r["seconds"] * 1e3 / max(r["iters"], 1), "loss0": r["loss0"],
                      "loss": r["loss"], "noise_floor": cal_sigma ** 2,
                      "excess_loss_ratio": (r["loss"] - cal_sigma ** 2) / (r["loss0"] - cal_sigma ** 2)}}
        del gc

    # ---- batched forward + backward over many stars (one captured graph)
    if "batch" in modes:
        nb = args.batch_stars
        log("generating %d-star batch" % nb)
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(16) as ex:
            stars_wl = list(ex.map(W.batch_star, range(nb)))
        opts = {}
        for w in stars_wl:                      # one autotune per size bucket
            k = pz.tune_key(w)
            if k not in opts:
                opts[k] = pz.tuned_options(w)
        with ThreadPoolExecutor(16) as ex:
            plans = list(ex.map(lambda w: pz.plan_for(w, tile_px=opts[pz.tune_key(w)][0],
                                                      lines_per_chunk=opts[pz.tune_key(w)][1]), stars_wl))
        keep, descr, total_evals = [], [], 0
        rng = np.random.default_rng(5)
        for w, p in zip(stars_wl, plans):
            a = pz.Atmos(w.atm)
            q = pz.Params.from_host(w.params)
            bufs = dict(F=torch.empty(p.N, device=dev), Fc=torch.empty(p.N, device=dev),
                        y=torch.as_tensor(rng.uniform(0.5, 1.0, p.N).astype(np.float32), device=dev),
                        loss=torch.empty(1, device=dev),
                        gl=torch.empty(p.L, device=dev), gd=torch.empty(p.L, device=dev),
                        ga=torch.empty(p.S, device=dev), gx=torch.empty(1, device=dev))
            keep.append((a, q, bufs))
            descr.append(pz.pz_star(p.handle.value, a.c, q.c, bufs["F"].data_ptr(), bufs["Fc"].data_ptr(), None,
                                    bufs["y"].data_ptr(), 0.01, bufs["loss"].data_ptr(), bufs["gl"].data_ptr(),
                                    bufs["gd"].data_ptr(), bufs["ga"].data_ptr(), bufs["gx"].data_ptr()))
            total_evals += p.voigt_evals
        batch = pz.Batch(descr)
        log("batch: %d stars, %.3e evals per forward" % (nb, total_evals))
        graphs = {}
        for mode in (pz.PZ_MODE_FWD, pz.PZ_MODE_FWD_BWD):
            pz.synth_batch(batch, mode)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                pz.synth_batch(batch, mode)
            graphs[mode] = g
        bsteps = max(2, args.steps // 4)
        ms_bf, _ = timed(graphs[pz.PZ_MODE_FWD].replay, bsteps, 1, torch)
        ms_bb, _ = timed(graphs[pz.PZ_MODE_FWD_BWD].replay, bsteps, 1, torch)
        out["batched"] = {"stars": nb, "hipgraph": True, "fwd_spectra_per_s": nb * 1000.0 / ms_bf, "fwd_ms": ms_bf,
                          "fwd_bwd_spectra_per_s": nb * 1000.0 / ms_bb, "fwd_bwd_ms": ms_bb,
                          "fwd_voigt_evals_per_s": total_evals / (ms_bf * 1e-3),
                          "fwd_bwd_over_fwd": ms_bb / ms_bf,
                          "evals_per_fwd": total_evals, "tile_px_used": sorted(set(p.tile_px for p in plans)),
                          "pixels": int(sum(p.N for p in plans)), "lines": int(sum(p.L for p in plans))}
        del graphs
        batch.destroy()
        for p in plans:
            p.destroy()

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cb = cpu_baseline(W.giant_1500_1700nm())
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
