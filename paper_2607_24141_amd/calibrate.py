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
(each star's epochs share its synthesis).  The optimiser is L-BFGS with a
strong-Wolfe line search over unconstrained u, with the smooth bound
transform theta = b tanh(u / b) per correction kind; its vectors stay on the
device, each evaluation costs one host transfer of two scalars and each
iteration one more of the inner products with the stored pairs.
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


def _cubic_min(t0, f0, d0, t1, f1, d1, lo, hi):
    """Minimiser of the cubic through (t0, f0, f0') and (t1, f1, f1'), clamped to
    [lo, hi]; the midpoint of [lo, hi] if the cubic has no real minimiser."""
    d1s = d0 + d1 - 3.0 * (f0 - f1) / (t0 - t1)
    disc = d1s * d1s - d0 * d1
    if disc < 0.0:
        return 0.5 * (lo + hi)
    d2 = math.copysign(math.sqrt(disc), t1 - t0)
    den = d1 - d0 + 2.0 * d2
    if den == 0.0:
        return 0.5 * (lo + hi)
    t = t1 - (t1 - t0) * (d1 + d2 - d1s) / den
    return min(max(t, lo), hi)


def _strong_wolfe(phi, f0, d0, t, c1=1e-4, c2=0.9, max_ls=25):
    """Step length satisfying the strong Wolfe conditions along a descent
    direction (bracketing, then zoom by safeguarded cubic interpolation;
    Nocedal and Wright, Numerical Optimization, Algorithms 3.5 and 3.6).
    phi(t) -> (f, f', state) evaluates the objective; returns (t, f, state) of
    the accepted point (the best one seen if max_ls evaluations do not
    settle it)."""
    best = None
    t_prev, f_prev, d_prev = 0.0, f0, d0
    lo = hi = None
    for i in range(max_ls):
        f, d, st = phi(t)
        if best is None or f < best[1]:
            best = (t, f, st)
        if lo is None:
            if f > f0 + c1 * t * d0 or (i > 0 and f >= f_prev):
                lo, hi = (t_prev, f_prev, d_prev), (t, f, d)
            elif abs(d) <= -c2 * d0:
                return t, f, st
            elif d >= 0.0:
                lo, hi = (t, f, d), (t_prev, f_prev, d_prev)
            else:
                t_new = _cubic_min(t_prev, f_prev, d_prev, t, f, d, t + 0.01 * (t - t_prev), 10.0 * t)
                t_prev, f_prev, d_prev = t, f, d
                t = t_new
                continue
        else:
            if f > f0 + c1 * t * d0 or f >= lo[1]:
                hi = (t, f, d)
            else:
                if abs(d) <= -c2 * d0:
                    return t, f, st
                if d * (hi[0] - lo[0]) >= 0.0:
                    hi = lo
                lo = (t, f, d)
        a, b = sorted((lo[0], hi[0]))
        if b - a < 1e-12 * max(1.0, b):
            break
        t = _cubic_min(lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], a + 0.1 * (b - a), b - 0.1 * (b - a))
    return best


class _Pairs:
    """Curvature pairs (s_i, y_i) of L-BFGS in one device buffer B of 2 (m+1) + 1
    rows of n: rows [0, m] hold s, rows [m+1, 2m+1] the matching y (slot k: rows k and
    m+1+k), and the last
    row the current gradient (m+1 slots, so a new pair never evicts an old one
    before it is accepted).  The inner products that the compact form needs are
    kept on the host in float64: R[i][j] = s_i.y_j and YY[i][j] = y_i.y_j by slot."""

    def __init__(self, m, n, like):
        self.m, self.M = m, m + 1
        self.B = torch.zeros(2 * self.M + 1, n, dtype=like.dtype, device=like.device)
        self.SY = np.zeros((self.M, self.M))
        self.YY = np.zeros((self.M, self.M))
        self.order = []                              # accepted slots, oldest first
        self.gamma = 1.0

    def free_slot(self):
        return next(k for k in range(self.M) if k not in self.order)

    def reset(self):
        self.order = []
        self.gamma = 1.0


def _compact_direction(P, a, b, gg):
    """d = -H g from the compact representation of the L-BFGS inverse Hessian
    (Byrd, Nocedal and Schnabel 1994; Nocedal and Wright eq. 7.24),
        H = gamma I + [S  gamma Y] [[R^-T (D + gamma Y^T Y) R^-1, -R^-T], [-R^-1, 0]] [S  gamma Y]^T,
    R the upper triangle of S^T Y (pairs oldest first), D its diagonal: the
    same H g as the two-loop recursion with H_0 = gamma I.  a = S^T g, b =
    Y^T g by slot.  Returns the coefficients c of d = B^T c and g.d."""
    o = P.order
    c = np.zeros(2 * P.M + 1)
    c[2 * P.M] = -P.gamma
    if not o:
        return c, -gg
    idx = np.array(o)
    R = np.triu(P.SY[np.ix_(idx, idx)])
    Dg = np.diag(np.diag(R))
    av, bv = a[idx], b[idx]
    u = np.linalg.solve(R, av)                                      # R^-1 S^T g
    q = -u
    pv = np.linalg.solve(R.T, (Dg + P.gamma * P.YY[np.ix_(idx, idx)]) @ u - P.gamma * bv)
    c[idx] = -pv
    c[P.M + idx] = -P.gamma * q
    gd = -P.gamma * gg - av @ pv - P.gamma * (bv @ q)
    return c, gd


def lbfgs(fg, x0, max_iter=40, history_size=10, max_eval=None):
    """Limited-memory BFGS with a strong-Wolfe line search.  fg(x) -> (f [1], g)
    on the device.  The direction comes from the compact representation of the
    inverse Hessian (equal to the two-loop recursion of Nocedal and Wright,
    Algorithm 7.4): two matrix-vector products give every inner product with
    the stored pairs, a host solve of at most m x m, and one more product forms
    the direction.  Each iteration costs one host transfer for those inner
    products and one per evaluation (f and the slope along the direction, read
    together).  Returns dict(x, f, iters, evals, history)."""
    max_eval = max_eval or 4 * max_iter
    x = x0.detach().clone()
    shape = x.shape
    f_t, g = fg(x)
    f = float(f_t[0])
    evals, hist = 1, [f]
    n = x.numel()
    P = _Pairs(history_size, n, x)
    M = P.M
    B = P.B
    prods = torch.empty(2, 2 * M + 1, dtype=x.dtype, device=x.device)
    new_slot = None                                  # pair written by the last iteration, not yet tested
    it = 0
    while it < max_iter and evals < max_eval:
        B[2 * M].copy_(g.reshape(-1))
        torch.mv(B, g.reshape(-1), out=prods[0])
        if new_slot is not None:
            torch.mv(B, B[M + new_slot], out=prods[1])
        v = prods.cpu().double().numpy()
        a, b, gg = v[0, :M], v[0, M:2 * M], float(v[0, 2 * M])
        if new_slot is not None:
            k = new_slot
            sy, yy = v[1, :M], v[1, M:2 * M]               # s_i.y_k and y_i.y_k by slot
            ys = float(sy[k])
            if ys > 1e-10:
                P.SY[:, k] = sy
                P.YY[:, k] = yy
                P.YY[k, :] = yy
                P.order.append(k)
                if len(P.order) > P.m:
                    P.order.pop(0)
                P.gamma = ys / float(yy[k])
            new_slot = None
        c, gd = _compact_direction(P, a, b, gg)
        d = torch.mv(B.t(), torch.as_tensor(c, dtype=x.dtype).to(x.device, non_blocking=False)).reshape(shape)
        if not gd < 0.0:                          # not a descent direction: restart from -g
            P.reset()
            d = -g
            gd = -gg
            if gd == 0.0:
                break
        t0 = min(1.0, 1.0 / float(g.abs().sum())) if it == 0 else 1.0

        def phi(t):
            nonlocal evals
            xt = torch.add(x, d, alpha=t)
            ft, gt = fg(xt)
            evals += 1
            w = torch.stack([ft.reshape(-1)[0], torch.dot(gt.flatten(), d.flatten())]).tolist()
            return w[0], w[1], (xt, gt)

        t, f_new, (x_new, g_new) = _strong_wolfe(phi, f, gd, t0, max_ls=max(1, min(25, max_eval - evals)))
        k = P.free_slot()
        torch.sub(x_new.reshape(-1), x.reshape(-1), out=B[k])
        torch.sub(g_new.reshape(-1), g.reshape(-1), out=B[M + k])
        new_slot = k
        x, g, f = x_new, g_new, f_new
        hist.append(f)
        it += 1
    return dict(x=x, f=f, iters=it, evals=evals, history=hist)


def fit(cal, theta0=None, bounds=DEFAULT_BOUNDS, max_iter=40, history_size=10, max_eval=None, log=None):
    """L-BFGS (strong Wolfe) over the group corrections in the unconstrained
    u of theta = b tanh(u / b).  Returns dict(theta, loss0, loss, iters, evals,
    seconds, history)."""
    dev = cal.device
    b = torch.tensor(bounds, dtype=torch.float32, device=dev)[:, None]
    if theta0 is None:
        u0 = torch.zeros(4, cal.G, device=dev)
    else:
        t = torch.as_tensor(theta0, dtype=torch.float32, device=dev)
        u0 = b * torch.atanh(torch.clamp(t / b, -0.999999, 0.999999))
    e0 = cal.n_evals

    def fg(u):
        with torch.no_grad():
            t = torch.tanh(u / b)
            loss, g = cal.evaluate((b * t).contiguous())
            return loss.clone(), g * (1.0 - t * t)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = lbfgs(fg, u0, max_iter=max_iter, history_size=history_size, max_eval=max_eval)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    if log:
        for k, v in enumerate(r["history"]):
            log(k + 1, v)
    with torch.no_grad():
        theta = bound(r["x"], b).detach()
        loss = float(cal.evaluate(theta.contiguous())[0][0])
    return dict(theta=theta, loss0=r["history"][0], loss=loss, iters=r["iters"],
                evals=cal.n_evals - e0 - 1, seconds=secs, history=r["history"])


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
