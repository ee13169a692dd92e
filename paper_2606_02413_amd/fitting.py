"""Fitting a parameterised corona to its own maps through the library's
reverse mode (the iterative tuning of a coronal model against maps that the
paper names as the use of a differentiable forward model, Sec. 4).

The maps and their gradient with respect to ln n_e and ln T of every vertex come
from the HIP library (rtsun.rtsun_function: rt_trace_maps forward,
rt_trace_adjoint backward); torch chains that vertex gradient to the few
parameters of the corona.
"""
from __future__ import annotations

import math

import numpy as np


class ParamCorona:
    """A structured corona as a differentiable function of a few parameters: its
    density scale s, background temperature T_bg and active-region density
    factors A_k,
        ln n_e = s + ln n_BA + 0.3 g + sum_k ln(1 + (A_k - 1) G_k),
        T = T_bg + max(0, max_k (T_k - T_bg) G_k),
    with the seeded random field g, active-region profiles G_k and peak
    temperatures T_k of corona.structured_parts.  theta = (s, ln T_bg,
    ln(A_k - 1)); s = 0 and the drawn T_bg, A_k give corona.structured()."""

    def __init__(self, parts, device="cuda", amp=0.3):
        import torch
        self.base = torch.from_numpy(np.log(parts["ba"]) + amp * parts["g"]).to(device)
        self.G = torch.from_numpy(parts["G"]).to(device)
        self.T = torch.from_numpy(parts["T"]).to(device)
        self.A = parts["A"]

    def truth(self, t_bg=1.2e6):
        return np.concatenate([[0.0, math.log(t_bg)], np.log(self.A - 1.0)])

    def __call__(self, theta, shape):
        import torch
        s, ln_tbg, a = theta[0], theta[1], theta[2:]
        ln_ne = s + self.base + torch.log1p(torch.exp(a)[:, None] * self.G).sum(0)
        tbg = torch.exp(ln_tbg)
        dte = torch.clamp(((self.T[:, None] - tbg) * self.G).max(0).values, min=0.0)
        ln_te = torch.log(tbg + dte)
        return ln_ne.reshape(shape).float(), ln_te.reshape(shape).float()


def fit_params(cor_kw, n_pix, half, freqs, iters, lr, start, log=None, log_every=10, decay=1.0, polish=0):
    """Fit theta of ParamCorona to the maps of the truth (the same
    parameterisation at its drawn values) through rtsun_function(): forward
    rt_trace_maps, backward rt_trace_adjoint, chained to theta by torch.  Loss =
    mean squared T_b difference / mean squared data.  `iters` Adam steps with
    learning rate lr * decay^step, then `polish` L-BFGS iterations (strong Wolfe
    line search).  Returns the truth, the history and the final theta."""
    import torch
    from . import corona, rtsun as R
    parts = corona.structured_parts(device="cuda", **cor_kw)
    pc = ParamCorona(parts)
    shape = (cor_kw["nr"], cor_kw["nt"], cor_kw["nph"])
    truth = pc.truth(cor_kw.get("t_bg", 1.2e6))
    th_true = torch.tensor(truth, dtype=torch.float64, device="cuda")
    ln_ne, ln_te = pc(th_true, shape)
    cor = corona.Corona(*shape, cor_kw["r_in"], cor_kw["r_max"], torch.exp(ln_ne).cpu().numpy(),
                        torch.exp(ln_te).cpu().numpy(), "param-truth")
    model = R.Model.from_corona(cor)
    try:
        theta, hist = _fit(pc, model, shape, n_pix, half, freqs, iters, lr, start, log, log_every, decay, polish,
                           ln_ne, ln_te)
    finally:
        model.close()
    return truth, hist, theta


def _fit(pc, model, shape, n_pix, half, freqs, iters, lr, start, log, log_every, decay, polish, ln_ne, ln_te):
    import torch
    from . import rtsun as R
    im = R.image_desc(n_pix, half)
    prm = R.params(ds_max=0.01, n_floor=0.1)
    F = R.rtsun_function()
    with torch.no_grad():
        data = F.apply(ln_ne, ln_te, model, freqs, im, prm).clone()
    norm = float((data.double() ** 2).mean())
    theta = torch.tensor(start, dtype=torch.float64, device="cuda", requires_grad=True)
    hist = []

    def objective():
        ne_t, te_t = pc(theta, shape)
        tb = F.apply(ne_t, te_t, model, freqs, im, prm)
        return ((tb.double() - data.double()) ** 2).mean() / norm

    def record(step, loss, kind):
        th = theta.detach().cpu().numpy()
        hist.append({"step": step, "kind": kind, "loss": float(loss), "s": float(th[0]),
                     "T_bg": float(math.exp(th[1])), "A": (1.0 + np.exp(th[2:])).tolist()})
        if log is not None and (step % log_every == 0 or kind == "lbfgs"):
            log(f"fit-params {kind} step {step}: loss {float(loss):.3e} s {th[0]:+.4f} T_bg {math.exp(th[1]):.4e}")

    opt = torch.optim.Adam([theta], lr=lr)
    sched = torch.optim.lr_scheduler.ExponentialLR(opt, gamma=decay)
    for it in range(iters):
        opt.zero_grad()
        loss = objective()
        loss.backward()
        record(it, loss, "adam")
        opt.step()
        sched.step()
    if polish > 0:
        lb = torch.optim.LBFGS([theta], lr=1.0, max_iter=8, history_size=10, line_search_fn="strong_wolfe")

        def closure():
            lb.zero_grad()
            loss = objective()
            loss.backward()
            return loss

        for k in range(polish):
            lb.step(closure)
            with torch.no_grad():
                record(iters + k, objective(), "lbfgs")
    with torch.no_grad():
        record(iters + polish, objective(), "final")
    return theta.detach().cpu().numpy(), hist
