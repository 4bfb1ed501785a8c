"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/tbr.h declares, and rejects invalid scalar arguments on the host
(no GPU work is launched by any call here)."""

import ctypes as C
import os
import re

import pytest

from paper_2609_08722_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "tbr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tbr_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2609_08722_amd import build
        build.build()
    return L.load()


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert "tbr_render" in syms and "tbr_render_backward" in syms and "tbr_fit_step" in syms
    for s in syms:
        assert hasattr(lib, s), s
    # the binding declares a signature for every symbol too
    assert set(syms) <= set(L.SIGNATURES)


def test_version(lib):
    assert b"gfx950" in lib.tbr_version()


def opts(**kw):
    base = dict(width=64, height=64, tau=1e-3, tau_min=0.7 / 64, tau_c=0.0, eps_floor=1e-3,
                ckpt_interval=16, side_slots=4)
    base.update(kw)
    return L.RenderOpts(*[base[f] for f, _ in L.RenderOpts._fields_])


def test_workspace_sizes_grow_with_tape(lib):
    o = opts()
    a = lib.tbr_render_workspace_bytes(C.byref(o), 50, L.TBR_SOFT, 0)
    b = lib.tbr_render_workspace_bytes(C.byref(o), 50, L.TBR_SOFT, 1)
    P = 64 * 64
    # tape: nrec + ckpt (1 + 49 // 16 = 4 states of 16 B) + side (4 slots x 12 B)
    assert b - a >= P * (4 + 4 * 16 + 4 * 12)
    assert lib.tbr_render_workspace_bytes(None, 50, L.TBR_SOFT, 0) == 0
    assert lib.tbr_backward_workspace_bytes(C.byref(o), 50, 8) >= 16 * (51 * 8 * 4)
    assert lib.tbr_fit_workspace_bytes(C.byref(o), 50, 8) > b


@pytest.mark.parametrize("bad", [dict(width=0), dict(height=20000), dict(tau=-1.0),
                                 dict(tau_min=0.0), dict(tau_c=-0.5), dict(eps_floor=0.0),
                                 dict(ckpt_interval=-1)])
def test_invalid_options_rejected(lib, bad):
    o = opts(**bad)
    prog = L.Program(0, 1, None, None, None, None, None, None, C.c_void_p(16))
    buf = C.create_string_buffer(1 << 16)
    st = lib.tbr_render(C.byref(prog), C.byref(o), L.TBR_SOFT, None, None, None,
                        C.cast(buf, C.c_void_p), 1 << 16, 0, None)
    assert st == L.TBR_E_INVALID
    assert lib.tbr_last_error()


def test_invalid_program_rejected(lib):
    o = opts()
    buf = C.create_string_buffer(1 << 16)
    for prog in (L.Program(-1, 8, *([None] * 7)), L.Program(5, 0, *([None] * 7)),
                 L.Program(5, 8, *([None] * 6), C.c_void_p(16))):
        st = lib.tbr_render(C.byref(prog), C.byref(o), L.TBR_SOFT, None, None, None,
                            C.cast(buf, C.c_void_p), 1 << 16, 0, None)
        assert st == L.TBR_E_INVALID
    assert lib.tbr_render(None, C.byref(o), L.TBR_SOFT, None, None, None,
                          C.cast(buf, C.c_void_p), 1 << 16, 0, None) == L.TBR_E_INVALID


def test_mode_and_workspace_checks(lib):
    o = opts()
    prog = L.Program(0, 1, None, None, None, None, None, None, C.c_void_p(16))
    buf = C.create_string_buffer(64)
    args = (None, None, None, C.cast(buf, C.c_void_p))
    assert lib.tbr_render(C.byref(prog), C.byref(o), 0, *args, 64, 0, None) == L.TBR_E_INVALID
    assert lib.tbr_render(C.byref(prog), C.byref(o), L.TBR_HARD, *args, 64, 1, None) == L.TBR_E_INVALID
    # workspace too small
    assert lib.tbr_render(C.byref(prog), C.byref(o), L.TBR_SOFT, *args, 8, 0, None) == L.TBR_E_INVALID
    assert b"workspace" in lib.tbr_last_error()


def test_fit_step_rejects_bad_adam(lib):
    o = opts()
    a = L.AdamOpts(0.01, 0.01, 0.01, 0.01, 0.01, 0.01, 0.9, 0.999, 1e-8, 0.002, 0.2, 0.3, 0)
    buf = C.create_string_buffer(64)
    p = C.cast(buf, C.c_void_p)
    st = lib.tbr_fit_step(10, 4, p, None, p, p, C.byref(a), C.byref(o), p, p, p, 64, None)
    assert st == L.TBR_E_INVALID
