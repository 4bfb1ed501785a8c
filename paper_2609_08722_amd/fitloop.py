"""The fitting loop around the fit step (Sec. 5.1, Table hyper, Sec. 8):
free parameters behind windows, annealed relaxation and colour temperature,
cosine step decay, length and area regularisers, export with palette
snapping, prefix replay and program edits.

Every step runs in the library (tbr_window_map, tbr_fit_loop_step,
tbr_schedule_at); this module only marshals arguments and edits program
arrays.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L
from .api import Adam, Opts, _ptr, _stream, unpack


@dataclass
class Window:
    """tbr_window_opts; defaults are Table hyper's (anchor kept on the canvas)."""
    a_lo: float = 0.0
    a_hi: float = 1.0
    l_max: float = 0.30
    r0_first: float = 0.120
    r0_last: float = 0.005
    r_lo_frac: float = 0.6
    r_hi_frac: float = 1.7
    lambda_length: float = 3e-4
    lambda_area: float = 0.0

    def c(self) -> L.WindowOpts:
        return L.WindowOpts(self.a_lo, self.a_hi, self.l_max, self.r0_first, self.r0_last,
                            self.r_lo_frac, self.r_hi_frac, self.lambda_length, self.lambda_area)


@dataclass
class Schedule:
    """Table hyper: tau 0.35 -> 0.02 and tau_c 1.0 -> 0.05 geometric, cosine
    decay of the group steps (anchor, width, offset, colour, palette)."""
    total_steps: int = 240
    tau_first: float = 0.35
    tau_last: float = 0.02
    tau_c_first: float = 1.0
    tau_c_last: float = 0.05
    lr_anchor: float = 0.012
    lr_width: float = 0.018
    lr_offset: float = 0.015
    lr_colour: float = 0.030
    lr_palette: float = 0.010

    def at(self, step: int):
        lib = L.load()
        tau, tau_c, lr = C.c_float(), C.c_float(), C.c_float()
        lib.tbr_schedule_at(step, self.total_steps, self.tau_first, self.tau_last,
                            self.tau_c_first, self.tau_c_last, C.byref(tau), C.byref(tau_c),
                            C.byref(lr))
        return tau.value, tau_c.value, lr.value


def window_map(theta: torch.Tensor, n: int, k: int, window: Window) -> torch.Tensor:
    """The program (packed) of free parameters theta."""
    lib = L.load()
    out = torch.empty_like(theta)
    w = window.c()
    L.check(lib.tbr_window_map(n, k, _ptr(theta), _ptr(out), C.byref(w), _stream()))
    return out


class FitLoop:
    """Device state of a fit: free parameters theta, Adam moments, and the
    program, gradient and loss of the last step. coupling: [N, 3] profile
    coefficients of the calibrated transport, or None (capsule)."""

    def __init__(self, theta: torch.Tensor, n: int, k: int, width: int, height: int,
                 window: Window | None = None, schedule: Schedule | None = None,
                 ckpt: int = 256, side_slots: int = 16, coupling: torch.Tensor | None = None):
        self.theta = theta.to(torch.float32).contiguous().clone()
        self.n, self.k = n, k
        self.window = window or Window()
        self.schedule = schedule or Schedule()
        self.opts = Opts(width, height, ckpt=ckpt, side_slots=side_slots, coupling=coupling)
        self.params = torch.empty_like(self.theta)
        self.grads = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.theta.device)
        self.step_index = 0
        self._alloc()

    def _alloc(self):
        lib = L.load()
        self.nbytes = lib.tbr_fit_workspace_bytes(C.byref(self.opts.c(self.n)), self.n, self.k)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.theta.device)

    def step(self, target: torch.Tensor) -> torch.Tensor:
        """One loop step at the schedule's current point; returns the device
        loss (data + regularisers) of the program before the update."""
        lib = L.load()
        s = self.schedule
        tau, tau_c, lr = s.at(self.step_index)
        self.opts.tau, self.opts.tau_c = tau, tau_c
        a = Adam()
        ao = L.AdamOpts(s.lr_anchor * lr, 0.0, s.lr_offset * lr, s.lr_width * lr,
                        s.lr_colour * lr, s.lr_palette * lr, a.beta1, a.beta2, a.eps,
                        a.r_lo, a.r_hi, a.l_max, self.step_index + 1)
        w = self.window.c()
        t = target.to(torch.float32).contiguous()
        L.check(lib.tbr_fit_loop_step(self.n, self.k, _ptr(self.theta), _ptr(self.params),
                                      _ptr(self.grads), _ptr(self.m), _ptr(self.v), C.byref(w),
                                      C.byref(ao), C.byref(self.opts.c(self.n)), _ptr(t),
                                      _ptr(self.loss), _ptr(self.ws), self.nbytes, _stream()))
        self.step_index += 1  # counted only once the library has taken the step
        return self.loss

    def _records(self):
        lib = L.load()
        mr = C.c_int32(0)
        st = lib.tbr_tape_records(_ptr(self.ws), self.nbytes, C.byref(self.opts.c(self.n)), self.n,
                                  C.byref(mr), _stream())
        return st, mr.value

    def step_checked(self, target: torch.Tensor, headroom: int = 4) -> torch.Tensor:
        """step(), repeated with a larger side table when it overflowed (the
        update was then skipped, so the repeat is exact). Synchronises."""
        while True:
            loss = self.step(target)
            st, need = self._records()
            if st != L.TBR_E_OVERFLOW:
                L.check(st)
                return loss
            self.step_index -= 1
            self.opts.side_slots = need + headroom
            self._alloc()

    def program(self) -> dict:
        """The current program (window map of theta), as views of one buffer."""
        return unpack(window_map(self.theta, self.n, self.k, self.window), self.n, self.k)


def export(prog: dict) -> dict:
    """Program with palette colours snapped (Sec. 7 export): each stroke's
    colour becomes the palette entry of its largest logit, i.e. one-hot
    logits, which renders the same at any colour temperature."""
    out = {f: v.clone() for f, v in prog.items()}
    z = out["logits"]
    out["logits"] = torch.nn.functional.one_hot(z.argmax(1), z.shape[1]).to(z.dtype)
    return out


def prefix(prog: dict, k: int) -> dict:
    """The first k strokes (Sec. 8, prefix replay): views, palette shared."""
    return {f: (v if f == "palette" else v[:k]) for f, v in prog.items()}


def insert_drop(prog: dict, at: int, centre, radius: float, logits_row) -> dict:
    """Insert a drop (L = 0) of the given radius and colour logits before
    stroke `at` (Sec. 8 edits)."""
    dev = prog["cx"].device

    def ins(v, x):
        return torch.cat([v[:at], torch.as_tensor(x, dtype=v.dtype, device=dev).reshape(1, *v.shape[1:]), v[at:]])

    return {"cx": ins(prog["cx"], centre[0]), "cy": ins(prog["cy"], centre[1]),
            "angle": ins(prog["angle"], 0.0), "length": ins(prog["length"], 0.0),
            "half_width": ins(prog["half_width"], radius),
            "logits": ins(prog["logits"], logits_row), "palette": prog["palette"].clone()}


def recolour_swap(prog: dict, first: int, a: int, b: int) -> dict:
    """Swap palette entries a and b in the colour choice of strokes >= first."""
    out = {f: v.clone() for f, v in prog.items()}
    z = out["logits"][first:]
    za, zb = z[:, a].clone(), z[:, b].clone()
    z[:, a], z[:, b] = zb, za
    return out


def translate(prog: dict, first: int, dx: float, dy: float = 0.0) -> dict:
    """Translate strokes >= first by (dx, dy)."""
    out = {f: v.clone() for f, v in prog.items()}
    out["cx"][first:] += dx
    out["cy"][first:] += dy
    return out
