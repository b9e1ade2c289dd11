"""Line-list calibration on the GPU (Sec. 6, Eq. 30).

Four logarithmic corrections per correction group (log gf and the radiative,
Stark and van der Waals damping constants, theta [4][G]) are fitted jointly
to several standard spectra that share one line list.  One evaluation of the
objective runs entirely in the library's kernels:

    theta --pz_groups_expand--> per-line dgf, ddamp_family  (one [4][L] array)
    per star:   synth_forward --> F, Fc                      (shared by its epochs)
      per epoch: pz_inst_forward --> f;  pz_wmse_seed --> loss, dL/df;
                 pz_inst_backward --> dL/dF
    per star:   synth_backward (damping-family gradients) --> [4][L]
                pz_groups_reduce (accumulating over stars) --> dL/dtheta [4][G]

The objective is sum_s c_s sum_p w_sp (f_sp - y_sp)^2 over the standards s
(each star's epochs share its synthesis).  The optimiser is PyTorch's L-BFGS
with a strong-Wolfe line search over unconstrained u, with the smooth bound
transform theta = b tanh(u / b) per correction kind.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import (PZ_FLAG_DAMPING_FAMILIES, Atmos, Groups, Instrument, Params, plan_for, pz_inst_backward,
               pz_inst_forward, pz_wmse_seed, synth_backward, synth_forward)
from . import correction_groups  # noqa: F401  (re-exported for callers)

KINDS = ("loggf", "radiative", "stark", "vdw")
DEFAULT_BOUNDS = (1.0, 1.5, 1.5, 1.5)    # dex, per correction kind


class _Epoch:
    def __init__(self, std, y, device):
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)
        self.name = std.name
        self.inst = Instrument(std.wl.grid, std.lam_obs_nm, std.lsf_sigma_ln, std.vb_max_kms)
        self.vel = f32(std.vel)
        self.y = f32(y) if y is not None else torch.zeros(self.inst.P, device=device)
        self.w = f32(std.w)
        self.c = float(std.c)
        self.f = torch.empty(self.inst.P, device=device)
        self.df = torch.empty(self.inst.P, device=device)


class _Star:
    def __init__(self, wl, X, device):
        self.wl = wl
        self.plan = plan_for(wl, flags=PZ_FLAG_DAMPING_FAMILIES)
        self.atm = Atmos(wl.atm, device=device)
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)
        # line corrections come from the shared [4][L] array: row 0 = dgf, rows 1-3 = families
        self.par = Params(X[0], None, f32(wl.params.dA), f32([wl.params.xi_kms]), X[1:])
        N = wl.grid.N
        self.F = torch.empty(N, device=device)
        self.Fc = torch.empty(N, device=device)
        self.dF = torch.empty(N, device=device)
        self.dFe = torch.empty(N, device=device)
        self.epochs = []


class Calibration:
    """The calibration objective of a CalWorkload-like description on the GPU.

    cal: .lines, .active and .standards (each with .wl, .lam_obs_nm,
    .lsf_sigma_ln, .vb_max_kms, .vel, .w, .c; standards with the same .wl
    object are epochs of one star).  y: one observed spectrum per standard
    (numpy or device arrays), or None to set later with set_observed.
    groups: (group_of_line, G) or None to build them with the paper's
    tolerances (2.0 cm^-1, 0.035 nm)."""

    def __init__(self, cal, y=None, groups=None, dE_cm=2.0, dlam_nm=0.035, device="cuda"):
        self.device = device
        if groups is None:
            groups = correction_groups(cal.lines, dE_cm, dlam_nm, active=cal.active)
        self.q, self.G = groups
        self.L = int(cal.lines.L)
        self.groups = Groups(self.q, self.G)
        self.X = torch.zeros(4, self.L, device=device)        # expanded line corrections
        self.GL = torch.zeros(4, self.L, device=device)       # line gradients
        self.loss = torch.zeros(1, device=device)
        self.grad = torch.zeros(4, self.G, device=device)
        self.stars = []
        by_wl = {}
        for k, std in enumerate(cal.standards):
            if id(std.wl) not in by_wl:
                by_wl[id(std.wl)] = _Star(std.wl, self.X, device)
                self.stars.append(by_wl[id(std.wl)])
            by_wl[id(std.wl)].epochs.append(_Epoch(std, None if y is None else y[k], device))
        self.n_evals = 0

    @property
    def epochs(self):
        return [e for s in self.stars for e in s.epochs]

    def set_observed(self, ys):
        for e, y in zip(self.epochs, ys):
            e.y.copy_(torch.as_tensor(y, dtype=torch.float32, device=self.device))

    def model(self, theta):
        """Observed-pixel models f of every standard at theta [4][G] (device)."""
        self.groups.expand(theta.contiguous(), self.X)
        out = []
        for s in self.stars:
            synth_forward(s.plan, s.atm, s.par, s.F, s.Fc)
            for e in s.epochs:
                pz_inst_forward(e.inst, s.F, s.Fc, e.vel, None, None, e.f)
                out.append(e.f.clone())
        return out

    def evaluate(self, theta):
        """(loss [1], dL/dtheta [4][G]) at theta [4][G] (device float32).
        The returned tensors are reused by the next call."""
        self.groups.expand(theta.contiguous(), self.X)
        first = True
        for k, s in enumerate(self.stars):
            synth_forward(s.plan, s.atm, s.par, s.F, s.Fc)
            for i, e in enumerate(s.epochs):
                pz_inst_forward(e.inst, s.F, s.Fc, e.vel, None, None, e.f)
                pz_wmse_seed(e.f, e.y, e.w, e.c, e.df, self.loss, accumulate=not first)
                first = False
                pz_inst_backward(e.inst, s.F, s.Fc, e.vel, e.df, s.dF if i == 0 else s.dFe, None, None)
                if i > 0:
                    s.dF.add_(s.dFe)
            synth_backward(s.plan, s.atm, s.par, s.dF, self.GL[0], self.GL[1:], None, None)
            self.groups.reduce(self.GL, self.grad, accumulate=k > 0)
        self.n_evals += 1
        return self.loss, self.grad


class _LossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, cal):
        loss, grad = cal.evaluate(theta.detach())
        ctx.save_for_backward(grad.clone())
        return loss.clone()[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None


def loss_fn(cal, theta):
    """The objective as a differentiable function of theta [4][G] (autograd)."""
    return _LossFn.apply(theta, cal)


def bound(u, b):
    """Smooth bound transform theta = b tanh(u / b) (b: [4, 1])."""
    return b * torch.tanh(u / b)


def fit(cal, theta0=None, bounds=DEFAULT_BOUNDS, max_iter=40, history_size=10, max_eval=None, log=None):
    """L-BFGS (strong Wolfe) over the group corrections.  Returns dict(theta,
    loss0, loss, iters, evals, seconds)."""
    dev = cal.device
    b = torch.tensor(bounds, dtype=torch.float32, device=dev)[:, None]
    if theta0 is None:
        u = torch.zeros(4, cal.G, device=dev)
    else:
        t = torch.as_tensor(theta0, dtype=torch.float32, device=dev)
        u = b * torch.atanh(torch.clamp(t / b, -0.999999, 0.999999))
    u.requires_grad_(True)
    opt = torch.optim.LBFGS([u], lr=1.0, max_iter=max_iter, max_eval=max_eval or 4 * max_iter,
                            history_size=history_size, line_search_fn="strong_wolfe",
                            tolerance_grad=0.0, tolerance_change=0.0)
    e0 = cal.n_evals
    hist = []

    def closure():
        with torch.no_grad():
            t = torch.tanh(u / b)
            loss, g = cal.evaluate((b * t).contiguous())
            u.grad = (g * (1.0 - t * t)).contiguous()
            val = loss[0].clone()
        hist.append(float(val))
        if log:
            log(len(hist), hist[-1])
        return val

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    opt.step(closure)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = opt.state[u]
    with torch.no_grad():
        theta = bound(u, b).detach()
        loss = float(cal.evaluate(theta.contiguous())[0][0])
    return dict(theta=theta, loss0=hist[0], loss=loss, iters=int(st.get("n_iter", 0)),
                evals=cal.n_evals - e0 - 1, seconds=secs, history=hist)


def mock_observed(cal, theta_true, sigma, seed):
    """Observed spectra: the model at theta_true plus Gaussian noise sigma
    (device, seeded per standard)."""
    fs = cal.model(torch.as_tensor(theta_true, dtype=torch.float32, device=cal.device))
    out = []
    for k, f in enumerate(fs):
        rng = np.random.Generator(np.random.PCG64(seed + k))
        n = torch.as_tensor(rng.normal(0.0, sigma, f.numel()).astype(np.float32), device=cal.device)
        out.append(f + n)
    return out


def correlation(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    a, b = a - a.mean(), b - b.mean()
    return float(a @ b / math.sqrt((a @ a) * (b @ b)))
