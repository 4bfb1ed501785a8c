"""Python surface of the HIP renderer: marshalling of torch CUDA tensors into
the C ABI of include/tbr.h. Every step of the computation runs in the HIP
kernels of libtbr.so; there is no CPU or PyTorch fallback.

Functions
  render(prog, opts, mode, tape)       soft / hard forward (Sec. 3, Eq. render)
  render_backward(prog, opts, tape, g) replay adjoint (Sec. 5.2)
  TBRRender                            torch.autograd.Function around both
  FitState.step(target)                one L2 fit step with Adam (Sec. 5.1)
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L

GEOM = ("cx", "cy", "angle", "length", "half_width")
FIELDS = GEOM + ("logits", "palette")


@dataclass
class Opts:
    """Render options (tbr_render_opts)."""
    width: int
    height: int
    tau: float = 1e-3
    tau_min: float | None = None      # default 0.7 pixel: 0.7 / width
    tau_c: float = 0.0
    eps: float = 1e-3
    ckpt: int = 256
    side_slots: int = 16
    # calibrated coupling (Eq. coupling, Eq. profile): a contiguous float32
    # CUDA tensor [N, 3] of (c_1, c_2, c_3) per stroke, or None (capsule map)
    coupling: "torch.Tensor | None" = None
    # "inert" (R_U, psi = id) or "drops16" (R_D, sixteen drops); None: the
    # capsule map, or its coupling when coupling is given
    transport: str | None = None

    def c(self, n_strokes: int | None = None) -> L.RenderOpts:
        """The C options; with n_strokes, also checks the coupling's size
        (the library reads 3 coefficients per stroke)."""
        tm = 0.7 / self.width if self.tau_min is None else self.tau_min
        cp = self.coupling
        if cp is not None and not (cp.is_cuda and cp.dtype == torch.float32 and cp.is_contiguous()):
            raise ValueError("coupling must be a contiguous float32 CUDA tensor [N, 3]")
        if cp is not None and n_strokes is not None and cp.numel() != 3 * n_strokes:
            raise ValueError(f"coupling has {cp.numel()} values, expected 3 x {n_strokes}")
        if self.transport is not None and cp is not None:
            raise ValueError("coupling applies to the capsule map only")
        tr = {None: L.TBR_TRANSPORT_CAPSULE if cp is None else L.TBR_TRANSPORT_COUPLED,
              "inert": L.TBR_TRANSPORT_INERT, "drops16": L.TBR_TRANSPORT_DROPS16}[self.transport]
        return L.RenderOpts(int(self.width), int(self.height), float(self.tau), float(tm),
                            float(self.tau_c), float(self.eps), int(self.ckpt),
                            int(self.side_slots), tr, None if cp is None else cp.data_ptr())

    @property
    def pixels(self) -> int:
        return self.width * self.height


def check_coupling(coupling) -> float:
    """Exact positivity check of per-stroke profile coefficients [N, 3]
    (tbr_coupling_check, on a host copy); returns the smallest g and raises
    TbrError when a profile is not positive."""
    c = np.ascontiguousarray(torch.as_tensor(coupling).detach().cpu().numpy(), dtype=np.float32)
    c = c.reshape(-1, 3)
    m = C.c_float(0.0)
    L.check(L.load().tbr_coupling_check(c.ctypes.data_as(C.c_void_p), len(c), C.byref(m)))
    return m.value


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def to_device(arrs: dict, device="cuda") -> dict:
    """Program dict (numpy or torch) -> contiguous float32 CUDA tensors."""
    out = {}
    for k in FIELDS:
        v = arrs[k]
        t = v if isinstance(v, torch.Tensor) else torch.from_numpy(np.asarray(v))
        out[k] = t.to(device=device, dtype=torch.float32).contiguous()
    return out


def _check_prog(prog: dict):
    n = prog["cx"].numel()
    k = prog["palette"].numel() // 3
    for f in FIELDS:
        t = prog[f]
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"{f} must be a contiguous float32 CUDA tensor")
    for f in GEOM:
        if prog[f].numel() != n:
            raise ValueError(f"{f} has {prog[f].numel()} entries, expected {n}")
    if prog["logits"].numel() != n * k or prog["palette"].numel() != 3 * k:
        raise ValueError("logits must be [N, K] and palette [K, 3]")
    return n, k


def validate_program(prog: dict) -> None:
    """Value checks the library leaves to its caller (it does not read
    device arrays on the host): every array finite, half-widths > 0,
    palette in [0, 1]. Synchronises; raises ValueError."""
    _check_prog(prog)
    for f in FIELDS:
        if prog[f].numel() and not bool(torch.isfinite(prog[f]).all()):
            raise ValueError(f"{f} holds a NaN or an infinity")
    if prog["half_width"].numel() and float(prog["half_width"].min()) <= 0.0:
        raise ValueError("half_width must be > 0")
    pal = prog["palette"]
    if float(pal.min()) < 0.0 or float(pal.max()) > 1.0:
        raise ValueError("palette values must lie in [0, 1]")


def c_program(prog: dict) -> L.Program:
    n, k = _check_prog(prog)
    return L.Program(n, k, *[_ptr(prog[f]) for f in FIELDS])


@dataclass
class Tape:
    """Workspace holding the replay tape of one soft render."""
    ws: torch.Tensor
    opts: Opts
    n_strokes: int
    max_records: int = -1
    keep: list = field(default_factory=list)


def render(prog: dict, opts: Opts, mode: str = "soft", tape: bool = False,
           check_overflow: bool = True) -> dict:
    """Forward render. mode: 'soft', 'hard' or 'both'. Returns rgb [H,W,3]
    (soft if requested), label / owner [H,W] int32 for hard, and the tape."""
    lib = L.load()
    cp = c_program(prog)
    flags = {"soft": L.TBR_SOFT, "hard": L.TBR_HARD, "both": L.TBR_SOFT | L.TBR_HARD}[mode]
    dev = prog["cx"].device
    H, W = opts.height, opts.width
    while True:
        co = opts.c(cp.n_strokes)
        nbytes = lib.tbr_render_workspace_bytes(C.byref(co), cp.n_strokes, flags, int(tape))
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        rgb = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
        label = owner = None
        if flags & L.TBR_HARD:
            label = torch.empty((H, W), dtype=torch.int32, device=dev)
            owner = torch.empty((H, W), dtype=torch.int32, device=dev)
        L.check(lib.tbr_render(C.byref(cp), C.byref(co), flags, _ptr(rgb), _ptr(label),
                               _ptr(owner), _ptr(ws), nbytes, int(tape), _stream()))
        out = {"rgb": rgb, "label": label, "owner": owner}
        if not tape:
            return out
        t = Tape(ws, opts, cp.n_strokes)
        if check_overflow:
            mr = C.c_int32(0)
            st = lib.tbr_tape_records(_ptr(ws), nbytes, C.byref(co), cp.n_strokes,
                                      C.byref(mr), _stream())
            t.max_records = mr.value
            if st == L.TBR_E_OVERFLOW:
                opts = Opts(**{**opts.__dict__, "side_slots": max(mr.value, 1)})
                continue
            L.check(st)
        out["tape"] = t
        return out


def render_static(prog: dict, opts: Opts, mode: str = "soft") -> dict:
    """Forward render through tbr_render_static, which allocates nothing: no
    tape, no workspace (the library's per-device scratch holds the stroke
    records). Same outputs as render(prog, opts, mode)."""
    lib = L.load()
    cp = c_program(prog)
    flags = {"soft": L.TBR_SOFT, "hard": L.TBR_HARD, "both": L.TBR_SOFT | L.TBR_HARD}[mode]
    dev = prog["cx"].device
    H, W = opts.height, opts.width
    co = opts.c(cp.n_strokes)
    rgb = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    label = owner = None
    if flags & L.TBR_HARD:
        label = torch.empty((H, W), dtype=torch.int32, device=dev)
        owner = torch.empty((H, W), dtype=torch.int32, device=dev)
    L.check(lib.tbr_render_static(C.byref(cp), C.byref(co), flags, _ptr(rgb), _ptr(label),
                                  _ptr(owner), _stream()))
    return {"rgb": rgb, "label": label, "owner": owner}


def render_backward(prog: dict, tape: Tape, grad_rgb: torch.Tensor) -> dict:
    """Replay adjoint: gradients of sum(grad_rgb * R) w.r.t. every program
    array (same shapes as the program)."""
    lib = L.load()
    cp = c_program(prog)
    co = tape.opts.c(cp.n_strokes)
    g = grad_rgb.to(torch.float32).contiguous()
    if g.numel() != 3 * tape.opts.pixels or not g.is_cuda:
        raise ValueError("grad_rgb must be a CUDA tensor of H*W*3 values")
    grads = {f: torch.empty_like(prog[f]) for f in FIELDS}
    cg = L.ProgramGrad(*[_ptr(grads[f]) for f in FIELDS])
    nbytes = lib.tbr_backward_workspace_bytes(C.byref(co), cp.n_strokes, cp.n_palette)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=g.device)
    L.check(lib.tbr_render_backward(C.byref(cp), C.byref(co), _ptr(tape.ws), tape.ws.numel(),
                                    _ptr(g), C.byref(cg), _ptr(ws), nbytes, _stream()))
    return grads


def compensate(prog: dict, endpoint: bool = False, skip_blocked: bool = False,
               eps: float = 1e-3):
    """Closed-form compensation of an inert-mark program (tbr_compensate):
    returns the compensated program and each stroke's blocked-step count."""
    lib = L.load()
    cp = c_program(prog)
    n = cp.n_strokes
    dev = prog["cx"].device
    out = {f: prog[f].clone() for f in FIELDS}
    blocked = torch.zeros(n, dtype=torch.int32, device=dev)
    nbytes = lib.tbr_compensate_workspace_bytes(n, int(endpoint))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    L.check(lib.tbr_compensate(C.byref(cp), float(eps), int(endpoint), int(skip_blocked),
                               _ptr(out["cx"]), _ptr(out["cy"]), _ptr(out["angle"]),
                               _ptr(out["length"]), _ptr(blocked), _ptr(ws), nbytes, _stream()))
    return out, blocked



class TBRRender(torch.autograd.Function):
    """rgb = R(program) (soft render) with the replay adjoint as backward."""

    @staticmethod
    def forward(ctx, cx, cy, angle, length, half_width, logits, palette, opts: Opts):
        prog = {"cx": cx.contiguous(), "cy": cy.contiguous(), "angle": angle.contiguous(),
                "length": length.contiguous(), "half_width": half_width.contiguous(),
                "logits": logits.contiguous(), "palette": palette.contiguous()}
        out = render(prog, opts, "soft", tape=True)
        ctx.prog = prog
        ctx.tape = out["tape"]
        return out["rgb"]

    @staticmethod
    def backward(ctx, grad_rgb):
        g = render_backward(ctx.prog, ctx.tape, grad_rgb)
        return (g["cx"], g["cy"], g["angle"], g["length"], g["half_width"],
                g["logits"].view_as(ctx.prog["logits"]), g["palette"].view_as(ctx.prog["palette"]),
                None)


def render_soft_autograd(prog: dict, opts: Opts) -> torch.Tensor:
    return TBRRender.apply(*[prog[f] for f in FIELDS], opts)


@dataclass
class Adam:
    """Per-group Adam settings (paper Table hyper step sizes)."""
    lr_centre: float = 0.012
    lr_angle: float = 0.015
    lr_length: float = 0.015
    lr_width: float = 0.018
    lr_logits: float = 0.030
    lr_palette: float = 0.010
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    r_lo: float = 0.002
    r_hi: float = 0.2
    l_max: float = 0.3


def pack(prog: dict) -> torch.Tensor:
    return torch.cat([prog[f].reshape(-1) for f in FIELDS]).contiguous()


def unpack(vec: torch.Tensor, n: int, k: int) -> dict:
    out, o = {}, 0
    for f in GEOM:
        out[f] = vec[o:o + n]
        o += n
    out["logits"] = vec[o:o + n * k].view(n, k)
    o += n * k
    out["palette"] = vec[o:o + 3 * k].view(k, 3)
    return out


class FitState:
    """Device-resident state of the fused fit step (tbr_fit_step)."""

    def __init__(self, prog: dict, opts: Opts, adam: Adam | None = None):
        prog = to_device(prog) if not isinstance(prog["cx"], torch.Tensor) or not prog["cx"].is_cuda else prog
        self.n, self.k = _check_prog(prog)
        validate_program(prog)
        self.opts = opts
        self.adam = adam or Adam()
        self.params = pack(prog)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.params.device)
        self.step_index = 0
        self._alloc()

    def _alloc(self):
        lib = L.load()
        co = self.opts.c(self.n)
        self.nbytes = lib.tbr_fit_workspace_bytes(C.byref(co), self.n, self.k)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.params.device)

    def program(self) -> dict:
        return unpack(self.params, self.n, self.k)

    def step(self, target: torch.Tensor) -> torch.Tensor:
        """One fit step; returns the device loss (before the update)."""
        lib = L.load()
        a = self.adam
        ao = L.AdamOpts(a.lr_centre, a.lr_angle, a.lr_length, a.lr_width, a.lr_logits,
                        a.lr_palette, a.beta1, a.beta2, a.eps, a.r_lo, a.r_hi, a.l_max,
                        self.step_index + 1)
        co = self.opts.c(self.n)
        t = target.to(torch.float32).contiguous()
        L.check(lib.tbr_fit_step(self.n, self.k, _ptr(self.params), _ptr(self.grads),
                                 _ptr(self.m), _ptr(self.v), C.byref(ao), C.byref(co), _ptr(t),
                                 _ptr(self.loss), _ptr(self.ws), self.nbytes, _stream()))
        self.step_index += 1  # counted only once the library has taken the step
        return self.loss

    def _records(self):
        lib = L.load()
        co = self.opts.c(self.n)
        mr = C.c_int32(0)
        st = lib.tbr_tape_records(_ptr(self.ws), self.nbytes, C.byref(co), self.n, C.byref(mr),
                                  _stream())
        return st, mr.value

    def tape_records(self) -> int:
        """Max side-table records of the last step (synchronises); raises
        TbrError(TBR_E_OVERFLOW) if the capacity was exceeded."""
        st, n = self._records()
        L.check(st)
        return n

    def grow_side_table(self, slots: int):
        self.opts = Opts(**{**self.opts.__dict__, "side_slots": int(slots)})
        self._alloc()

    def step_checked(self, target: torch.Tensor, headroom: int = 4) -> torch.Tensor:
        """One fit step that is repeated with a larger side table when the
        table overflowed (the library then skipped the update, so the repeat
        is exact). Synchronises the stream."""
        while True:
            loss = self.step(target)
            st, need = self._records()
            if st != L.TBR_E_OVERFLOW:
                L.check(st)
                return loss
            self.step_index -= 1  # the update did not happen
            self.grow_side_table(need + headroom)


class MultiFit:
    """Several FitStates stepped together by tbr_fit_multi_step: their soft
    forwards and replay adjoints share one fused persistent launch."""

    def __init__(self, states: list):
        self.states = states
        self._alloc()

    def _jobs(self):
        arr = (L.FitJob * len(self.states))()
        for j, f in enumerate(self.states):
            a = f.adam
            arr[j] = L.FitJob(f.n, f.k, _ptr(f.params), _ptr(f.grads), _ptr(f.m), _ptr(f.v),
                              _ptr(f._target), _ptr(f.loss), f.opts.c(f.n),
                              L.AdamOpts(a.lr_centre, a.lr_angle, a.lr_length, a.lr_width,
                                         a.lr_logits, a.lr_palette, a.beta1, a.beta2, a.eps,
                                         a.r_lo, a.r_hi, a.l_max, max(f.step_index, 1)))
        return arr

    def _alloc(self):
        for f in self.states:
            f._target = getattr(f, "_target", None)
        lib = L.load()
        jobs = self._jobs()
        self.nbytes = lib.tbr_fit_multi_workspace_bytes(jobs, len(self.states))
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.states[0].params.device)

    def step(self, targets: list) -> list:
        lib = L.load()
        for f, t in zip(self.states, targets):
            f._target = t.to(torch.float32).contiguous()
            f.step_index += 1
        jobs = self._jobs()
        try:
            L.check(lib.tbr_fit_multi_step(jobs, len(self.states), _ptr(self.ws), self.nbytes,
                                           _stream()))
        except L.TbrError:
            for f in self.states:  # the library rejected the step: nothing was updated
                f.step_index -= 1
            raise
        return [f.loss for f in self.states]

    def tape_records(self) -> list:
        lib = L.load()
        jobs = self._jobs()
        out = (C.c_int32 * len(self.states))()
        L.check(lib.tbr_fit_multi_records(jobs, len(self.states), _ptr(self.ws), self.nbytes,
                                          out, _stream()))
        return list(out)


class Server:
    """Continuous-batching server of replay requests (tbr_serve_*).

    The device arena is a torch uint8 tensor owned by this object; programs
    are copied into it once. submit() returns a ticket at once; poll() says
    when the request's outputs are complete on the device."""

    OUTS = {"rgb": L.TBR_OUT_RGB, "label": L.TBR_OUT_LABEL, "owner": L.TBR_OUT_OWNER}

    def __init__(self, arena_bytes: int = 256 << 20, max_slots: int = 64, max_queue: int = 4096,
                 max_tick_items: int = 1 << 17, streams: int = 3, fake_device: bool = False,
                 fake_ns_per_pixel_stroke: float = 0.0, fake_fail_launch: int = 0,
                 solo_tiles: int = 1024, device="cuda"):
        lib = L.load()
        self.arena = None if fake_device else torch.empty(arena_bytes, dtype=torch.uint8,
                                                          device=device)
        self.opts = L.ServeOpts(_ptr(self.arena), int(arena_bytes), int(max_slots),
                                int(max_queue), int(max_tick_items), int(streams),
                                int(fake_device), float(fake_ns_per_pixel_stroke),
                                int(fake_fail_launch), int(solo_tiles))
        h = C.c_void_p()
        L.check(lib.tbr_serve_create(C.byref(self.opts), C.byref(h)))
        self.h = h
        self.fake = fake_device
        self._keep = {}
        self._shape = {}  # ticket -> (width, height, arena_outputs mask)

    def register(self, prog: dict) -> int:
        lib = L.load()
        if self.fake:
            n = len(prog["cx"])
            k = np.asarray(prog["palette"]).reshape(-1, 3).shape[0]
            cp = L.Program(n, k, *([None] * 7))
        else:
            validate_program(prog)
            cp = c_program(prog)
        pid = C.c_uint64()
        L.check(lib.tbr_serve_register_program(self.h, C.byref(cp), C.byref(pid)))
        return pid.value

    def submit(self, program_id: int, mode: str, width: int, height: int, rgb=None, label=None,
               owner=None, tau=1e-3, tau_min=0.0, tau_c=0.0, eps=1e-3,
               arena_outputs=()) -> int:
        """Queue a request. arena_outputs: names among 'rgb', 'label', 'owner'
        that the server holds in its arena (counted in the request's
        footprint; see poll and release)."""
        lib = L.load()
        mask = 0
        for name in arena_outputs:
            mask |= self.OUTS[name]
        r = L.Request(int(program_id), L.TBR_SOFT if mode == "soft" else L.TBR_HARD, int(width),
                      int(height), float(tau), float(tau_min), float(tau_c), float(eps),
                      _ptr(rgb), _ptr(label), _ptr(owner), mask)
        t = C.c_uint64()
        L.check(lib.tbr_serve_submit(self.h, C.byref(r), C.byref(t)))
        if mask:
            self._shape[t.value] = (int(width), int(height), mask)
        return t.value

    def _view(self, ptr, nbytes, dtype, shape):
        off = int(ptr) - self.arena.data_ptr()
        return self.arena[off:off + nbytes].view(dtype).view(shape)

    def poll(self, ticket: int):
        """None while pending; else a dict with status and timestamps, and
        for arena outputs views of them into the arena ('rgb' [H,W,3],
        'label', 'owner' [H,W]), valid until release(ticket)."""
        lib = L.load()
        res = L.Result()
        st = lib.tbr_serve_poll(self.h, C.c_uint64(ticket), C.byref(res))
        if st == L.TBR_PENDING:
            return None
        if st not in (L.TBR_OK, L.TBR_E_CANCELLED):
            self._shape.pop(ticket, None)
            L.check(st)
        out = {"status": st, "t_submit": res.t_submit, "t_admit": res.t_admit,
               "t_start": res.t_start, "t_done": res.t_done,
               "pixel_strokes": res.pixel_strokes}
        shp = self._shape.get(ticket)
        if st == L.TBR_OK and shp and not self.fake:
            W, H, mask = shp
            if mask & L.TBR_OUT_RGB:
                out["rgb"] = self._view(res.rgb, H * W * 12, torch.float32, (H, W, 3))
            if mask & L.TBR_OUT_LABEL:
                out["label"] = self._view(res.label, H * W * 4, torch.int32, (H, W))
            if mask & L.TBR_OUT_OWNER:
                out["owner"] = self._view(res.owner, H * W * 4, torch.int32, (H, W))
        return out

    def release(self, ticket: int) -> int:
        """Give back a finished request's arena outputs; the caller's reads
        of them must be complete (synchronise first)."""
        st = L.load().tbr_serve_release(self.h, C.c_uint64(ticket))
        if st not in (L.TBR_OK, L.TBR_PENDING):
            L.check(st)
        if st == L.TBR_OK:
            self._shape.pop(ticket, None)
        return st

    def cancel(self, ticket: int) -> int:
        return L.load().tbr_serve_cancel(self.h, C.c_uint64(ticket))

    def stats(self) -> dict:
        s = L.ServeStats()
        L.check(L.load().tbr_serve_get_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in L.ServeStats._fields_}

    @staticmethod
    def now() -> float:
        return L.load().tbr_serve_now()

    def close(self):
        if self.h:
            L.load().tbr_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
