"""FP64 oracle of the fitting loop around the fit step -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the GPU library never loads it and shares no code with it.

What it states, from the paper (TBR, arxiv 2609.08722):
  * the parameterisation of Sec. 5.1 ("Parameterisation and relaxation"):
    half-width r = r_lo + (r_hi - r_lo) sigmoid(theta_r) inside a per-stroke
    window [0.6 r0, 1.7 r0] with r0 geometric from 0.120 to 0.005 over the
    program (Table hyper); offset d = l_max tanh(theta_d); anchor
    a = a_lo + (a_hi - a_lo) sigmoid(theta_a); palette P = sigmoid(theta_P);
    colour logits z = theta_c. The stroke is the segment from a to a + d
    (Sec. 3), so its centre is m = a + d / 2, its length l = |d| and its
    angle phi = atan2(d_y, d_x);
  * the regularisers: lambda sum_i l_i (Table hyper) and the area budget
    lambda_A sum_i A_l(r_i), A_l(r) = 2 l r + pi r^2 (Eq. steiner; the
    penalty and its gradient d A / d r = P_l(r) in Sec. 8 "Area budget");
  * the schedule: tau annealed geometrically from 0.35 to 0.02, the colour
    temperature from 1.0 to 0.05, and Adam step sizes with cosine decay
    (Table hyper);
  * Adam with bias correction (beta 0.9 / 0.999, eps 1e-8).

Readings where the paper is silent (listed with the project design): tanh and
sigmoid act componentwise on the 2-vectors d and a; the anchor window is the
canvas [0, 1]^2; the colour temperature is annealed geometrically like tau;
cosine decay is lr_s = lr_0 (1 + cos(pi s / T)) / 2 for s = 0 .. T - 1;
at l = 0 the angle is 0 and the gradients through d / |d| are taken as 0.

Parity status: every function is pinned by tests/test_oracle_fitloop.py
(finite differences of the window map and of the regularisers, schedule end
points and ratios, closed forms of the first Adam step).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class WindowCfg:
    a_lo: float = 0.0
    a_hi: float = 1.0
    l_max: float = 0.30
    r0_first: float = 0.120
    r0_last: float = 0.005
    r_lo_frac: float = 0.6
    r_hi_frac: float = 1.7
    lambda_length: float = 3e-4
    lambda_area: float = 0.0


@dataclass(frozen=True)
class ScheduleCfg:
    total_steps: int = 240
    tau_first: float = 0.35
    tau_last: float = 0.02
    tau_c_first: float = 1.0
    tau_c_last: float = 0.05


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def r0(n: int, cfg: WindowCfg) -> np.ndarray:
    """Window centre r0_i, geometric from r0_first (i = 0) to r0_last (i = n-1)."""
    if n <= 1:
        return np.full(n, cfg.r0_first)
    t = np.arange(n) / (n - 1)
    return cfg.r0_first * (cfg.r0_last / cfg.r0_first) ** t


def split(vec: np.ndarray, n: int, k: int):
    """Packed [5 blocks of n | n*k | 3k] -> the seven arrays (views)."""
    o = 0
    blocks = []
    for _ in range(5):
        blocks.append(vec[o:o + n])
        o += n
    blocks.append(vec[o:o + n * k].reshape(n, k))
    o += n * k
    blocks.append(vec[o:o + 3 * k].reshape(k, 3))
    return blocks


def window_map(theta: np.ndarray, n: int, k: int, cfg: WindowCfg) -> np.ndarray:
    """Free parameters [th_ax|th_ay|th_dx|th_dy|th_r|th_c|th_P] -> natural
    parameters [cx|cy|angle|length|half_width|logits|palette]."""
    tax, tay, tdx, tdy, tr, tc, tp = split(np.asarray(theta, np.float64), n, k)
    ax = cfg.a_lo + (cfg.a_hi - cfg.a_lo) * sigmoid(tax)
    ay = cfg.a_lo + (cfg.a_hi - cfg.a_lo) * sigmoid(tay)
    dx = cfg.l_max * np.tanh(tdx)
    dy = cfg.l_max * np.tanh(tdy)
    c0 = r0(n, cfg)
    r = cfg.r_lo_frac * c0 + (cfg.r_hi_frac - cfg.r_lo_frac) * c0 * sigmoid(tr)
    length = np.hypot(dx, dy)
    angle = np.where(length > 0, np.arctan2(dy, dx), 0.0)
    out = np.concatenate([ax + 0.5 * dx, ay + 0.5 * dy, angle, length, r,
                          tc.reshape(-1), sigmoid(tp).reshape(-1)])
    return out


def window_vjp(theta: np.ndarray, g_nat: np.ndarray, n: int, k: int,
               cfg: WindowCfg) -> np.ndarray:
    """Vector-Jacobian product of window_map: dL/dtheta from dL/dnatural,
    written out from the derivatives of sigmoid, tanh, hypot and atan2."""
    tax, tay, tdx, tdy, tr, tc, tp = split(np.asarray(theta, np.float64), n, k)
    gmx, gmy, gphi, gl, gr, gz, gP = split(np.asarray(g_nat, np.float64), n, k)
    sax, say = sigmoid(tax), sigmoid(tay)
    dx, dy = cfg.l_max * np.tanh(tdx), cfg.l_max * np.tanh(tdy)
    length = np.hypot(dx, dy)
    safe = np.where(length > 0, length, 1.0)
    on = length > 0
    # m = a + d / 2, l = |d|, phi = atan2(d_y, d_x)
    gdx = 0.5 * gmx + np.where(on, gl * dx / safe - gphi * dy / safe ** 2, 0.0)
    gdy = 0.5 * gmy + np.where(on, gl * dy / safe + gphi * dx / safe ** 2, 0.0)
    span = cfg.a_hi - cfg.a_lo
    c0 = r0(n, cfg)
    sr = sigmoid(tr)
    sP = sigmoid(tp)
    return np.concatenate([
        gmx * span * sax * (1 - sax),
        gmy * span * say * (1 - say),
        gdx * cfg.l_max * (1 - np.tanh(tdx) ** 2),
        gdy * cfg.l_max * (1 - np.tanh(tdy) ** 2),
        gr * (cfg.r_hi_frac - cfg.r_lo_frac) * c0 * sr * (1 - sr),
        gz.reshape(-1),
        (gP * sP * (1 - sP)).reshape(-1),
    ])


def regularisers(natural: np.ndarray, n: int, k: int, cfg: WindowCfg):
    """lambda sum l + lambda_A sum A_l(r) and its gradient w.r.t. the natural
    parameters (nonzero only in the length and half-width blocks)."""
    _, _, _, length, r, _, _ = split(np.asarray(natural, np.float64), n, k)
    ell = np.abs(length)
    value = cfg.lambda_length * ell.sum() + cfg.lambda_area * (2 * ell * r + math.pi * r * r).sum()
    g = np.zeros_like(np.asarray(natural, np.float64))
    sgn = np.where(length < 0, -1.0, 1.0)
    g[3 * n:4 * n] = sgn * (cfg.lambda_length + cfg.lambda_area * 2 * r)
    g[4 * n:5 * n] = cfg.lambda_area * (2 * ell + 2 * math.pi * r)  # P_l(r)
    return value, g


def schedule(step: int, cfg: ScheduleCfg):
    """(tau, tau_c, lr factor) at step s in [0, T): geometric annealing of the
    two temperatures, cosine decay of the step sizes."""
    T = cfg.total_steps
    f = step / (T - 1) if T > 1 else 0.0
    tau = cfg.tau_first * (cfg.tau_last / cfg.tau_first) ** f
    tau_c = cfg.tau_c_first * (cfg.tau_c_last / cfg.tau_c_first) ** f
    lr = 0.5 * (1.0 + math.cos(math.pi * step / T))
    return tau, tau_c, lr


def group_lrs(n: int, k: int, lr_anchor, lr_offset, lr_width, lr_colour, lr_palette):
    """Per-entry step sizes of the packed free parameters (Table hyper groups)."""
    return np.concatenate([np.full(2 * n, lr_anchor), np.full(2 * n, lr_offset),
                           np.full(n, lr_width), np.full(n * k, lr_colour),
                           np.full(3 * k, lr_palette)])


def adam_step(theta, g, m, v, step: int, lrs, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lrs * mh / (np.sqrt(vh) + eps), m, v


def window_inverse(natural: np.ndarray, n: int, k: int, cfg: WindowCfg, margin=1e-4):
    """Free parameters of a natural program (values pulled inside the windows
    by `margin` of their span); used to start a fit from a given program."""
    cx, cy, angle, length, r, z, P = split(np.asarray(natural, np.float64), n, k)
    dx, dy = length * np.cos(angle), length * np.sin(angle)
    ax, ay = cx - 0.5 * dx, cy - 0.5 * dy

    def logit(u):
        u = np.clip(u, margin, 1 - margin)
        return np.log(u / (1 - u))

    span = cfg.a_hi - cfg.a_lo
    c0 = r0(n, cfg)
    return np.concatenate([
        logit((ax - cfg.a_lo) / span), logit((ay - cfg.a_lo) / span),
        np.arctanh(np.clip(dx / cfg.l_max, -1 + margin, 1 - margin)),
        np.arctanh(np.clip(dy / cfg.l_max, -1 + margin, 1 - margin)),
        logit((r - cfg.r_lo_frac * c0) / ((cfg.r_hi_frac - cfg.r_lo_frac) * c0)),
        z.reshape(-1), logit(P).reshape(-1),
    ])
