"""Benchmark of the MI355X synthesis path (one JSON line on stdout).

value: forward spectra/s on the 1500-1700 nm, R = 300,000 workload (37,550
pixels x 72 depths, 2e5 lines, 30 % in molecular-band-like sequences), inputs
resident in HBM, K timed steps between device synchronisations.  A step is
one whole forward synthesis (populations, line parameters, windowed Voigt
opacity, depth scan and Gauss-3 flux for both branches).  Extra fields: the
forward+backward step (chi^2 loss seed and the adjoint for all 4e5 + 20 + 1
corrections), the widest workload (300-1000 nm, 361,193 pixels, 5e6 lines,
forward), the centre test, continuum scattering (the source function
iterated to its fixed point, forward and forward+backward), the exact E2
angle integral instead of Gauss-3, the line-selection keep test (and the
forward of its kept subset), the instrument operator, the line calibration
(objective evaluation and L-BFGS updates over 25,147 correction groups of a
two-star, three-spectrum fit) and the batched launch over 256 stars (median of
per-replay times of the captured graph), the roofline of the dominant kernel
(opacity; float32 operations per evaluation from the committed SQ VALU
counters) and of the depth scans, and the FP64 CPU oracle on the host cores
(the whole 1500-1700 nm spectrum over a pool of worker processes, and one
thread alone on a sample).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                      [--modes fwd,fwdbwd,wide,center,select,scatter,e2,instrument,calibration,batch]
                      [--cal-updates 40] [--batch-replays 20] [--wide-steps 5] [--no-cpu]
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
# Nominal float32 operations of one Voigt evaluation (one line, one depth, one
# in-window pixel) in the four-node wing formula, FMA = 2: detuning scale and
# u = v^2 (2), a^2, u - a^2, 4 u a^2, u + a^2 (5), two node pairs x (sub, FMA,
# add, mul, rcp, FMA = 8), a * sum (1), kappa += K H (2).  Used only when no
# counter measurement of the current kernel sources is committed.
FLOPS_PER_EVAL_NOMINAL = 34
PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0      # MI355X published HBM3E bandwidth
# sources of the opacity kernel: a committed counter measurement (HBM bytes,
# VALU instruction counts) is used only if they are unchanged.  The opacity
# kernel's code: its tile body and the Voigt evaluator, plus the kernel's own
# definition in pz_kernels.hip (other code in that file is not part of it).
KERNEL_SOURCES = ("paper_2607_24141_amd/csrc/pz_opacity.h", "paper_2607_24141_amd/csrc/pz_voigt.h",
                  "paper_2607_24141_amd/csrc/voigt_consts.h")
KERNEL_DEF = ("paper_2607_24141_amd/csrc/pz_kernels.hip", "void k_opacity(")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# The gather kernel's code: its stage bodies, the Voigt evaluator and its
# definition in pz_kernels.hip.
GATHER_SOURCES = ("paper_2607_24141_amd/csrc/pz_stages.h", "paper_2607_24141_amd/csrc/pz_voigt.h",
                  "paper_2607_24141_amd/csrc/voigt_consts.h")
GATHER_DEF = ("paper_2607_24141_amd/csrc/pz_kernels.hip", "void k_gather(")


def kernel_hash(sources=KERNEL_SOURCES, definition=KERNEL_DEF):
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, definition[0])) as fh:
        txt = fh.read()
    i = txt.index(definition[1])
    i = txt.rindex("\n", 0, txt.rindex("\n", 0, i)) + 1      # from the template line above
    h.update(txt[i:txt.index("\n}\n", i) + 3].encode())
    return h.hexdigest()[:16]


def gather_hash():
    return kernel_hash(GATHER_SOURCES, GATHER_DEF)


def _profile_json(name, hash_fn=kernel_hash):
    """A committed counter summary under profiles/, if it was taken on these kernel sources."""
    try:
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    return d if d.get("kernel_hash") == hash_fn() else None


def traffic_from_profiles(kind="opacity"):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE) from the committed counter summary."""
    d = _profile_json("traffic_%s.json" % kind)
    return None if d is None else d.get("bytes_per_launch")


def flops_per_eval_from_profiles():
    """Float32 operations per Voigt evaluation from the SQ VALU instruction counters of the
    opacity kernel (64 lanes x (ADD + MUL + TRANS + 2 FMA) per launch / evaluations per launch)."""
    d = _profile_json("valu_opacity.json")
    return (None, None) if d is None else (d.get("flops_per_eval"), d)


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


def timed_each(fn, steps, warmup, torch):
    """Median and spread of per-step hipEvent times (each step bracketed on its own)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return {"median_ms": ms[len(ms) // 2], "min_ms": ms[0], "max_ms": ms[-1], "replays": steps}


# ------------------------------------------------------------------ CPU oracle
_CPU_WL = None


def _cpu_chunk(pix):
    """One pool task: the oracle forward at the pixels pix (a fresh single-threaded process)."""
    global _CPU_WL
    import workloads as W
    from oracle import synth as O
    if _CPU_WL is None:
        _CPU_WL = W.giant_1500_1700nm()
    t0 = time.perf_counter()
    O.synthesize(_CPU_WL, pix=pix)
    return time.perf_counter() - t0, len(pix)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(N, voigt_evals, budget_s=45.0, one_thread_s=8.0):
    """The FP64 oracle, as it stands, on the host cores: the whole 1500-1700 nm
    spectrum split into 256-pixel pieces over a pool of single-threaded worker
    processes (all cores of the box's share, at most 16), stopped at budget_s
    and extrapolated if unfinished; plus one worker alone on a random sample."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor, as_completed
    from multiprocessing import get_context
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"            # each worker single-threaded
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    P = max(1, min(16, avail))
    ctx = get_context("spawn")         # the parent holds a GPU context: no fork
    order = np.random.default_rng(0).permutation(N)
    pieces = [np.sort(order[a:a + 256]) for a in range(0, N, 256)]
    with ProcessPoolExecutor(P, mp_context=ctx) as ex:
        list(ex.map(_cpu_chunk, [np.arange(2)] * P))          # start and warm every worker
        t0 = time.perf_counter()
        futs = [ex.submit(_cpu_chunk, p) for p in pieces]
        done_px = 0
        for f in as_completed(futs):
            done_px += f.result()[1]
            if time.perf_counter() - t0 > budget_s:
                break
        for f in futs:
            f.cancel()
        wall = time.perf_counter() - t0
    frac = done_px / N
    per_spec = wall / frac
    with ProcessPoolExecutor(1, mp_context=ctx) as ex:
        ex.submit(_cpu_chunk, np.arange(2)).result()
        t1, n1 = 0.0, 0
        k = 0
        while t1 < one_thread_s and k < len(pieces):
            dt, n = ex.submit(_cpu_chunk, pieces[k][:64]).result()
            t1 += dt
            n1 += n
            k += 1
    one = (t1 / n1) * N
    return {"value": 1.0 / per_spec, "unit": "spectra/s", "cores": P, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus_available": avail,
            "voigt_evals_per_s": voigt_evals / per_spec,
            "sample": ("%s of the %d-pixel 1500-1700 nm spectrum (%d pixels, all lines within W of each) in %.1f s "
                       "wall on %d single-threaded worker processes of the FP64 numpy/scipy oracle%s"
                       % ("all" if done_px >= N else "%.1f %%" % (100 * frac), N, done_px, wall, P,
                          "" if done_px >= N else ", scaled to the full spectrum")),
            "one_thread": {"value": 1.0 / one, "unit": "spectra/s", "pixels": n1, "seconds": t1,
                           "voigt_evals_per_s": voigt_evals / one}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--modes", default="fwd,fwdbwd,wide,center,select,scatter,e2,instrument,calibration,batch")
    ap.add_argument("--cal-updates", type=int, default=40, help="L-BFGS updates of the calibration block")
    ap.add_argument("--batch-stars", type=int, default=256)
    ap.add_argument("--batch-replays", type=int, default=20, help="timed graph replays per batch mode")
    ap.add_argument("--wide-steps", type=int, default=5, help="timed forwards of the 300-1000 nm workload")
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
    fpe, valu = flops_per_eval_from_profiles()
    flops_source = "SQ VALU counters (profiles/valu_opacity.json)" if fpe else "nominal (no counters of these sources)"
    fpe = fpe or FLOPS_PER_EVAL_NOMINAL
    achieved_tflops = plan.voigt_evals * fpe / (op_avg_ms * 1e-3) / 1e12
    stage = {k: (v[0] / max(v[1], 1)) for k, v in prof.items() if v[1]}
    roof = {"bound": "alu", "kernel": "k_opacity", "achieved": achieved_tflops, "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP32_TFLOPS,
            "traffic": traffic_from_profiles("opacity"), "kernel_avg_ms": op_avg_ms,
            "flops_per_eval": fpe, "flops_source": flops_source, "evals_per_launch": plan.voigt_evals}
    if valu:
        # issue rate of all VALU instructions against the measured ceiling of the part
        # (0.84 wave64 instructions per SIMD per ns with independent FMA chains)
        per_ns = valu["valu_insts_per_launch"] / (1024 * op_avg_ms * 1e6)
        roof["valu_issue"] = {"wave64_insts_per_simd_per_ns": per_ns, "ceiling": 0.84, "frac": per_ns / 0.84}
    # the depth scans: algorithmic HBM bytes (kappa_line read once, F and F_c written) per launch
    scan = {}
    if "flux" in stage:
        b = 4.0 * plan.D * N + 8.0 * N
        scan["k_flux"] = {"bytes": b, "ms": stage["flux"], "GB_s": b / (stage["flux"] * 1e6),
                          "frac_hbm": b / (stage["flux"] * 1e6) / PEAK_HBM_GBS}
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
        "stage_ms": stage,
        "roofline": roof,
        "scan_roofline": scan,
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
        st_fb = {k: (v[0] / max(v[1], 1)) for k, v in prof_fb.items() if v[1]}
        if "reverse_scan" in st_fb:
            b = 8.0 * plan.D * N + 4.0 * N          # kappa_line read, dL/dkappa written, seed read
            out["scan_roofline"]["k_reverse_scan"] = {"bytes": b, "ms": st_fb["reverse_scan"],
                                                      "GB_s": b / (st_fb["reverse_scan"] * 1e6),
                                                      "frac_hbm": b / (st_fb["reverse_scan"] * 1e6) / PEAK_HBM_GBS}
        vg = _profile_json("valu_gather.json", gather_hash)
        if vg and "gather" in st_fb:
            tg = vg["flops_per_eval"] * plan.voigt_evals / (st_fb["gather"] * 1e-3) / 1e12
            out["roofline_gather"] = {"bound": "alu", "kernel": "k_gather", "achieved": tg, "peak": PEAK_FP32_TFLOPS,
                                      "unit": "TFLOP/s", "frac": tg / PEAK_FP32_TFLOPS,
                                      "flops_per_eval": vg["flops_per_eval"], "kernel_avg_ms": st_fb["gather"],
                                      "flops_source": "SQ VALU counters (profiles/valu_gather.json)"}
        out["fwd_bwd"] = {"spectra_per_s": 1000.0 / ms_fb, "ms_per_step": ms_fb, "ratio_to_fwd": ms_fb / ms_fwd,
                          "voigt_evals_per_s": 2 * plan.voigt_evals / (ms_fb * 1e-3),
                          "stage_ms": {k: (v[0] / max(v[1], 1)) for k, v in prof_fb.items() if v[1]}}

    # ---- the widest workload: 300-1000 nm (361,193 pixels, 5e6 lines), forward only
    if "wide" in modes:
        log("generating 300-1000 nm workload")
        t0 = time.perf_counter()
        wwl = W.solar_300_1000nm()
        t_gen = time.perf_counter() - t0
        t0 = time.perf_counter()
        wplan = pz.plan_for(wwl, tile_px=32, lines_per_chunk=16)
        t_plan = time.perf_counter() - t0
        watm, wpar = pz.Atmos(wwl.atm), pz.Params.from_host(wwl.params)
        WF = torch.empty(wplan.N, dtype=torch.float32, device=dev)
        WFc = torch.empty_like(WF)
        log("300-1000 nm forward: N=%d L=%d evals=%.3e (plan %.1f s)" % (wplan.N, wplan.L, wplan.voigt_evals, t_plan))
        wfwd = lambda: pz.synth_forward(wplan, watm, wpar, WF, WFc)
        wplan.profile(True)
        tw = timed_each(wfwd, args.wide_steps, 1, torch)
        wprof = wplan.profile_read()
        wplan.profile(False)
        wst = {k: (v[0] / max(v[1], 1)) for k, v in wprof.items() if v[1]}
        w_tflops = wplan.voigt_evals * fpe / (wst["opacity"] * 1e-3) / 1e12
        bw = 4.0 * wplan.D * wplan.N + 8.0 * wplan.N
        out["wide_300_1000nm"] = {
            "workload": wwl.name, "N": wplan.N, "L": wplan.L, "D": wplan.D, "S": wwl.atm.S,
            "tile_px": wplan.tile_px, "fwd_ms": tw["median_ms"], "fwd_ms_min": tw["min_ms"],
            "fwd_ms_max": tw["max_ms"], "steps": tw["replays"], "spectra_per_s": 1000.0 / tw["median_ms"],
            "voigt_evals": wplan.voigt_evals, "voigt_evals_per_s": wplan.voigt_evals / (tw["median_ms"] * 1e-3),
            "stage_ms": wst, "line_params_bytes": 16 * wplan.L * wplan.D,
            "opacity_roofline": {"achieved": w_tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                 "frac": w_tflops / PEAK_FP32_TFLOPS, "flops_per_eval": fpe},
            "flux_GB_s": bw / (wst["flux"] * 1e6),
            "host_generate_s": t_gen, "host_plan_s": t_plan}
        wplan.destroy()
        del WF, WFc, watm, wpar

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
        inst.destroy()
        # the same with the rotation stage (v sin i up to 40 km/s, limb darkening 0.6)
        rinst = pz.Instrument(wl.grid, lam_obs, sig, vbmax, vrot_max_kms=40.0, limb_eps=0.6)
        rvel = torch.tensor([12.0, 6.0, 25.0], dtype=torch.float32, device=dev)
        rgv = torch.empty(3, dtype=torch.float32, device=dev)
        ms_rf, _ = timed(lambda: pz.pz_inst_forward(rinst, F, Fc, rvel, None, None, fobs), args.steps, args.warmup,
                         torch)
        ms_rb, _ = timed(lambda: pz.pz_inst_backward(rinst, F, Fc, rvel, iseed, dFi, dFci, rgv), args.steps,
                         args.warmup, torch)
        rinst.destroy()
        out["instrument"] = {"observed_pixels": inst.P, "native_pixels": int(F.numel()),
                             "fwd_us_per_flux_pair": ms_if * 1e3, "bwd_us_per_flux_pair": ms_ib * 1e3,
                             "with_rotation": {"vsini_kms": 25.0, "vrot_max_kms": 40.0,
                                               "fwd_us_per_flux_pair": ms_rf * 1e3,
                                               "bwd_us_per_flux_pair": ms_rb * 1e3}}

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
        CAL.fit(gc, max_iter=3)                 # warm-up: one-time library set-up (BLAS handles, kernels)
        r = CAL.fit(gc, max_iter=args.cal_updates)
        out["calibration"] = {
            "workload": cw.name, "records": int(cw.active.sum()), "lines": int(cw.lines.L), "groups": int(G),
            "corrections": 4 * int(G), "spectra": len(gc.epochs), "syntheses_per_eval": len(gc.stars),
            "grouping_ms": t_group * 1e3, "ms_per_eval": ms_eval,
            "lbfgs": {"updates": r["iters"], "evals": r["evals"], "seconds": r["seconds"],
                      "ms_per_update": r["seconds"] * 1e3 / max(r["iters"], 1),
                      "update_over_eval_time": (r["seconds"] * 1e3 / max(r["iters"], 1)) /
                                               (ms_eval * r["evals"] / max(r["iters"], 1)),
                      "loss0": r["loss0"],
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
        bsteps = max(2, args.batch_replays)
        tf = timed_each(graphs[pz.PZ_MODE_FWD].replay, bsteps, 2, torch)
        tb = timed_each(graphs[pz.PZ_MODE_FWD_BWD].replay, bsteps, 2, torch)
        ms_bf, ms_bb = tf["median_ms"], tb["median_ms"]
        out["batched"] = {"stars": nb, "hipgraph": True, "timing": "median of per-replay hipEvents",
                          "fwd_replays": tf, "fwd_bwd_replays": tb, "fwd_spectra_per_s": nb * 1000.0 / ms_bf, "fwd_ms": ms_bf,
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
        cb = cpu_baseline(N, plan.voigt_evals)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
