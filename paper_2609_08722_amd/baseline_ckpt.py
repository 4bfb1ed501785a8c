"""Checkpointed-autograd baseline: the soft render written with PyTorch ops
(FP32, on the GPU) and differentiated by autograd, with activation
checkpoints every `every` strokes (torch.utils.checkpoint). This is the
conventional alternative to the replay adjoint (the paper's Table adjoint
compares against autograd with checkpoints); it is only used to report time
and peak memory beside the HIP path, never by it.

Same definitions as the HIP kernels: Sec. 4 chart and Eq. back with the floor
C >= (eps r)^2, Eq. relax clamped at 1 - 1e-7, Eq. chain / Eq. render,
c = softmax(z / tau_c) P, background P[0].
"""

from __future__ import annotations

import math

import torch
from torch.utils.checkpoint import checkpoint

PI = math.pi


def _psi_alpha(x, y, mx, my, phi, L, r, tau, tau_min, eps):
    ce, se = torch.cos(phi), torch.sin(phi)
    dx, dy = x - mx, y - my
    s = dx * ce + dy * se
    h = dy * ce - dx * se
    ss = torch.where(s < 0, -1.0, 1.0)
    sh = torch.where(h < 0, -1.0, 1.0)
    S, H = s * ss, h * sh
    ell = L * torch.where(L < 0, -1.0, 1.0)  # |L| with d|L|/dL = +1 at L = 0
    hl = 0.5 * ell
    E = torch.clamp(S - hl, min=0.0)
    sig = torch.sqrt(H * H + E * E)
    th = torch.atan2(E, H)
    t = torch.minimum(S, hl) + sig * th
    per = 2 * ell + 2 * PI * sig
    w = t / per
    wd = torch.clamp(tau * r, min=tau_min)
    alpha = torch.clamp(torch.sigmoid((r - sig) / wd), max=1.0 - 1e-7)
    C = (sig - r) * (2 * ell + PI * (sig + r))
    C = torch.maximum(C, (eps * r) ** 2)
    rho = C / (ell + torch.sqrt(ell * ell + PI * C))
    tp = w * (2 * ell + 2 * PI * rho)
    thp = torch.clamp(tp - hl, min=0.0) / rho
    Sp = torch.minimum(tp, hl) + rho * torch.sin(thp)
    Hp = rho * torch.cos(thp)
    a, b = ss * Sp, sh * Hp
    return mx + a * ce - b * se, my + a * se + b * ce, alpha


def _chunk(x, y, C, T, cx, cy, ang, ln, hw, col, tau, tau_min, eps):
    for j in range(cx.shape[0] - 1, -1, -1):  # strokes of this chunk, last to first
        nx, ny, a = _psi_alpha(x, y, cx[j], cy[j], ang[j], ln[j], hw[j], tau, tau_min, eps)
        C = C + (T * a)[:, None] * col[j][None, :]
        T = T * (1.0 - a)
        x, y = nx, ny
    return x, y, C, T


def soft_render(prog: dict, width: int, height: int, tau=1e-3, tau_min=None, tau_c=1.0,
                eps=1e-3, every=50):
    """R [H*W, 3] with autograd through every program tensor."""
    tau_min = 0.7 / width if tau_min is None else tau_min
    dev = prog["cx"].device
    jj = torch.arange(width, device=dev, dtype=torch.float32)
    ii = torch.arange(height, device=dev, dtype=torch.float32)
    yy, xx = torch.meshgrid((ii + 0.5) / height, (jj + 0.5) / width, indexing="ij")
    x, y = xx.reshape(-1), yy.reshape(-1)
    n = prog["cx"].shape[0]
    if tau_c > 0:
        s = torch.softmax(prog["logits"] / tau_c, dim=1)
    else:
        s = torch.nn.functional.one_hot(prog["logits"].argmax(1), prog["palette"].shape[0]).float()
    col = s @ prog["palette"]
    C = torch.zeros(x.shape[0], 3, device=dev)
    T = torch.ones(x.shape[0], device=dev)
    hi = n
    while hi > 0:
        lo = max(0, hi - every)
        args = (prog["cx"][lo:hi], prog["cy"][lo:hi], prog["angle"][lo:hi],
                prog["length"][lo:hi], prog["half_width"][lo:hi], col[lo:hi])
        x, y, C, T = checkpoint(_chunk, x, y, C, T, *args, tau, tau_min, eps,
                                use_reentrant=False)
        hi = lo
    return C + T[:, None] * prog["palette"][0][None, :]


class CkptFit:
    """One fit step (L2 loss, torch.optim.Adam) on the checkpointed baseline."""

    def __init__(self, prog: dict, width: int, height: int, tau=1e-3, tau_c=1.0, every=50,
                 lr=0.012):
        self.params = {k: v.detach().clone().requires_grad_(True) for k, v in prog.items()}
        self.w, self.h, self.tau, self.tau_c, self.every = width, height, tau, tau_c, every
        self.opt = torch.optim.Adam(self.params.values(), lr=lr)

    def step(self, target: torch.Tensor) -> torch.Tensor:
        self.opt.zero_grad(set_to_none=True)
        R = soft_render(self.params, self.w, self.h, tau=self.tau, tau_c=self.tau_c,
                        every=self.every)
        loss = torch.mean((R - target.reshape(-1, 3)) ** 2)
        loss.backward()
        self.opt.step()
        return loss.detach()
