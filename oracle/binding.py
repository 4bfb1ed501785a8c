"""ctypes binding of the FP64 oracle (test infrastructure, see package doc)."""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tbr_oracle.cpp")
_LIB = os.path.join(_HERE, "libtbr_oracle.so")
_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain IEEE FP64: no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrcProgram(C.Structure):
    _fields_ = [("n", C.c_int32), ("k", C.c_int32),
                ("cx", C.c_void_p), ("cy", C.c_void_p), ("angle", C.c_void_p),
                ("length", C.c_void_p), ("half_width", C.c_void_p),
                ("logits", C.c_void_p), ("palette", C.c_void_p)]


class OrcOpts(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("tau", C.c_double), ("tau_min", C.c_double),
                ("tau_c", C.c_double), ("eps", C.c_double),
                ("transport", C.c_int32), ("coupling", C.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = C.CDLL(_LIB)
        vp, i64, dbl, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int
        _lib.orc_psi.argtypes = [vp, dbl, i64, vp, vp, vp, vp]
        _lib.orc_phi.argtypes = [vp, i64, vp, vp, vp]
        _lib.orc_chart.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        _lib.orc_map_jacobian.argtypes = [i32, vp, dbl, i64, vp, vp, vp]
        _lib.orc_psi_drops.argtypes = [vp, dbl, i64, vp, vp, vp]
        _lib.orc_compensate.argtypes = [vp, dbl, i32, i32, vp, vp, vp, vp, vp, vp, vp,
                                        vp, vp, vp, vp, vp]
        _lib.orc_phi_drops.argtypes = [vp, i64, vp, vp]
        _lib.orc_render.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
        _lib.orc_render.restype = i32
        _lib.orc_backward.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
        _lib.orc_backward.restype = i32
        _lib.orc_hard_points.argtypes = [vp, vp, i64, vp, vp]
        _lib.orc_num_threads.restype = i32
        _lib.orc_set_num_threads.argtypes = [i32]
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    _load().orc_set_num_threads(int(n))


def _stroke(stroke):
    s = _f64(stroke).reshape(5)
    return s


def _coup(coupling):
    return None if coupling is None else _f64(coupling).reshape(3)


def psi(stroke, pts, eps=1e-3, coupling=None):
    """Backward map of one stroke (m_x, m_y, phi, L, r) at points [n,2];
    coupling = (c_1, c_2, c_3) of the calibrated variant, or None."""
    s = _stroke(stroke)
    p = _f64(pts).reshape(-1, 2)
    c = _coup(coupling)
    out = np.empty_like(p)
    rec = np.empty(len(p), dtype=np.int32)
    _load().orc_psi(_ptr(s), float(eps), len(p), _ptr(p), _ptr(out), _ptr(rec), _ptr(c))
    return out, rec.astype(bool)


def phi(stroke, pts, coupling=None):
    """Exterior forward map of one stroke at points [n,2]."""
    s = _stroke(stroke)
    p = _f64(pts).reshape(-1, 2)
    c = _coup(coupling)
    out = np.empty_like(p)
    _load().orc_phi(_ptr(s), len(p), _ptr(p), _ptr(out), _ptr(c))
    return out


def chart(stroke, pts, coupling=None, edge=False):
    """(sigma, w): distance to the segment and centred arclength fraction;
    with edge=True also the deposit's edge on each point's leaf."""
    s = _stroke(stroke)
    p = _f64(pts).reshape(-1, 2)
    c = _coup(coupling)
    sig = np.empty(len(p))
    w = np.empty(len(p))
    e = np.empty(len(p)) if edge else None
    _load().orc_chart(_ptr(s), len(p), _ptr(p), _ptr(sig), _ptr(w), _ptr(e), _ptr(c))
    return (sig, w, e) if edge else (sig, w)


def psi_drops(stroke, pts, eps=1e-3):
    """R_D's backward displacement of one stroke (16 drops) at points [n,2]."""
    s = _stroke(stroke)
    p = _f64(pts).reshape(-1, 2)
    out = np.empty_like(p)
    rec = np.empty(len(p), dtype=np.int32)
    _load().orc_psi_drops(_ptr(s), float(eps), len(p), _ptr(p), _ptr(out), _ptr(rec))
    return out, rec.astype(bool)


def phi_drops(stroke, pts):
    """R_D's forward displacement of one stroke at points [n,2]."""
    s = _stroke(stroke)
    p = _f64(pts).reshape(-1, 2)
    out = np.empty_like(p)
    _load().orc_phi_drops(_ptr(s), len(p), _ptr(p), _ptr(out))
    return out


def map_jacobian(which, stroke, pts, eps=1e-3, coupling=None):
    """Exact Jacobian [n,2,7] w.r.t. (x, y, m_x, m_y, phi, L, r) of psi
    ('psi'), Phi ('phi') or R_D's displacements ('psi_drops', 'phi_drops')."""
    s = _stroke(stroke)
    p = _f64(pts).reshape(-1, 2)
    c = _coup(coupling)
    jac = np.empty((len(p), 2, 7))
    code = {"psi": 0, "phi": 1, "psi_drops": 2, "phi_drops": 3}[which]
    _load().orc_map_jacobian(code, _ptr(s), float(eps), len(p), _ptr(p), _ptr(jac), _ptr(c))
    return jac


class _Prog:
    """Holds FP64 copies alive for the duration of a call."""

    def __init__(self, prog):
        self.arrs = {k: _f64(prog[k]) for k in
                     ("cx", "cy", "angle", "length", "half_width", "logits", "palette")}
        n = len(self.arrs["cx"])
        k = self.arrs["palette"].reshape(-1, 3).shape[0]
        assert self.arrs["logits"].size == n * k
        self.s = OrcProgram(n, k, *[_ptr(self.arrs[f]) for f in
                                    ("cx", "cy", "angle", "length", "half_width",
                                     "logits", "palette")])
        self.n, self.k = n, k


class _Coupling:
    """Holds the FP64 [N][3] coefficient copy alive for the duration of a call."""

    def __init__(self, coupling, n):
        self.arr = None if coupling is None else _f64(coupling).reshape(n, 3)

    def ptr(self):
        return _ptr(self.arr)


def _opts(width, height, tau, tau_min, tau_c, eps, transport, coup=None):
    return OrcOpts(int(width), int(height), float(tau), float(tau_min), float(tau_c),
                   float(eps), int(transport), None if coup is None else coup.ptr())


def render(prog, width, height, *, tau=1e-3, tau_min=None, tau_c=0.0, eps=1e-3,
           transport=True, pixels=None, soft=True, hard=True, coupling=None):
    # transport: True / 1 = the capsule renderer R_A, False / 0 = the
    # inert-mark model R_U, 2 = R_D (sixteen drops per stroke)
    """Render a program (dict of arrays, see the synthetic generator) at pixel
    centres. Returns a dict with 'soft' [n,3], 'hard' [n,3], 'label', 'owner',
    'dmin', 'n_rec' (flat pixel order, or the order of ``pixels``).
    coupling: [N,3] c_1..c_3 per stroke of the calibrated variant, or None."""
    if tau_min is None:
        tau_min = 0.7 / width
    pr = _Prog(prog)
    cp = _Coupling(coupling, pr.n)
    o = _opts(width, height, tau, tau_min, tau_c, eps, transport, cp)
    pix = None if pixels is None else np.ascontiguousarray(np.asarray(pixels, dtype=np.int64))
    n = width * height if pix is None else len(pix)
    out = {}
    if soft:
        out["soft"] = np.empty((n, 3))
        out["n_rec"] = np.empty(n, dtype=np.int32)
    if hard:
        out["hard"] = np.empty((n, 3))
        out["label"] = np.empty(n, dtype=np.int32)
        out["owner"] = np.empty(n, dtype=np.int32)
        out["dmin"] = np.empty(n)
    _load().orc_render(C.byref(pr.s), C.byref(o), n, _ptr(pix), _ptr(out.get("soft")),
                       _ptr(out.get("hard")), _ptr(out.get("label")), _ptr(out.get("owner")),
                       _ptr(out.get("dmin")), _ptr(out.get("n_rec")))
    return out


def backward(prog, width, height, grad_rgb, *, tau=1e-3, tau_min=None, tau_c=0.0, eps=1e-3,
             transport=True, pixels=None, coupling=None):
    """Vector-Jacobian product of the soft render with grad_rgb [n,3].
    Returns dict: 'geom' [5,N] (m_x, m_y, phi, L, r), 'colour' [N,3],
    'logits' [N,K], 'palette' [K,3]. The coupling coefficients are
    constants (no gradient)."""
    if tau_min is None:
        tau_min = 0.7 / width
    pr = _Prog(prog)
    cp = _Coupling(coupling, pr.n)
    o = _opts(width, height, tau, tau_min, tau_c, eps, transport, cp)
    pix = None if pixels is None else np.ascontiguousarray(np.asarray(pixels, dtype=np.int64))
    n = width * height if pix is None else len(pix)
    g = _f64(grad_rgb).reshape(n, 3)
    geom = np.empty((5, pr.n))
    colour = np.empty((pr.n, 3))
    logits = np.empty((pr.n, pr.k))
    palette = np.empty((pr.k, 3))
    _load().orc_backward(C.byref(pr.s), C.byref(o), n, _ptr(pix), _ptr(g), _ptr(geom),
                         _ptr(colour), _ptr(logits), _ptr(palette))
    return {"geom": geom, "colour": colour, "logits": logits, "palette": palette}


def hard_points(prog, pts, *, eps=1e-3, transport=True, coupling=None):
    """Owner (0-based stroke index or -1) of arbitrary final-plane points."""
    pr = _Prog(prog)
    cp = _Coupling(coupling, pr.n)
    o = _opts(1, 1, 1e-3, 1e-3, 0.0, eps, transport, cp)
    p = _f64(pts).reshape(-1, 2)
    own = np.empty(len(p), dtype=np.int32)
    _load().orc_hard_points(C.byref(pr.s), C.byref(o), len(p), _ptr(p), _ptr(own))
    return own


def compensate(prog, *, eps=1e-3, endpoint=False, skip=False, with_dmin=False, later=None,
               with_amp=False):
    """Closed-form compensation of an inert-mark program: returns the
    compensated program (dict) and the blocked-step count of each stroke.
    with_dmin: also each stroke's closest approach |sigma' - r_j| to a later
    footprint's edge and smallest sigma' at a blocked step. later: a dict of
    cx, cy, angle, length [N] to pre-image through instead (each stroke is
    then the compensation step alone, given that later geometry). with_amp:
    also each stroke's largest error growth from any step to its chain's end
    (Frobenius norm of the Jacobian product)."""
    pr = _Prog(prog)
    n = pr.n
    out = {k: np.empty(n) for k in ("cx", "cy", "angle", "length")}
    blocked = np.empty(n, dtype=np.int32)
    dmin = np.empty(n)
    smin = np.empty(n)
    lat = None if later is None else {k: _f64(later[k]).reshape(n) for k in
                                      ("cx", "cy", "angle", "length")}
    lp = [None] * 4 if lat is None else [_ptr(lat[k]) for k in ("cx", "cy", "angle", "length")]
    amp = np.empty(n) if with_amp else None
    _load().orc_compensate(C.byref(pr.s), float(eps), int(bool(endpoint)), int(bool(skip)),
                           _ptr(out["cx"]), _ptr(out["cy"]), _ptr(out["angle"]),
                           _ptr(out["length"]), _ptr(blocked), _ptr(dmin), _ptr(smin), *lp,
                           _ptr(amp))
    res = {k: _f64(prog[k]).copy() for k in ("half_width", "logits", "palette")}
    res.update(out)
    extra = ((dmin, smin) if with_dmin else ()) + ((amp,) if with_amp else ())
    return (res, blocked) + extra
