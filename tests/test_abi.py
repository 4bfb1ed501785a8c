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
                ckpt_interval=16, side_slots=4, transport=0, coupling=None)
    base.update(kw)
    return L.RenderOpts(*[base[f] for f, _ in L.RenderOpts._fields_])


def test_workspace_sizes_grow_with_tape(lib):
    o = opts()
    a = lib.tbr_render_workspace_bytes(C.byref(o), 50, L.TBR_SOFT, 0)
    b = lib.tbr_render_workspace_bytes(C.byref(o), 50, L.TBR_SOFT, 1)
    P = 64 * 64
    # tape: nrec (4 B) + checkpoints (1 + 49 // 16 = 4 states of 16 B position
    # + 8 B transmittance) + side table (4 slots x (4 B index + 16 B position))
    assert b - a >= P * (4 + 4 * 24 + 4 * 20)
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


def test_schedule_matches_the_loop_oracle(lib):
    """tbr_schedule_at (host) against the FP64 oracle of Table hyper's
    schedule: geometric temperatures and cosine step factor."""
    from oracle import fitloop as fl
    cfg = fl.ScheduleCfg(total_steps=240)
    tau, tau_c, lr = C.c_float(), C.c_float(), C.c_float()
    for s in (0, 1, 17, 119, 120, 238, 239):
        lib.tbr_schedule_at(s, 240, 0.35, 0.02, 1.0, 0.05, C.byref(tau), C.byref(tau_c),
                            C.byref(lr))
        want = fl.schedule(s, cfg)
        assert tau.value == pytest.approx(want[0], rel=2e-7)
        assert tau_c.value == pytest.approx(want[1], rel=2e-7)
        assert lr.value == pytest.approx(want[2], rel=2e-7, abs=1e-7)
    # a one-step schedule stays at the first values with the full step
    lib.tbr_schedule_at(0, 1, 0.35, 0.02, 1.0, 0.05, C.byref(tau), C.byref(tau_c), C.byref(lr))
    assert (tau.value, tau_c.value, lr.value) == (pytest.approx(0.35), 1.0, 1.0)


def window(**kw):
    base = dict(a_lo=0.0, a_hi=1.0, l_max=0.3, r0_first=0.12, r0_last=0.005, r_lo_frac=0.6,
                r_hi_frac=1.7, lambda_length=3e-4, lambda_area=0.0)
    base.update(kw)
    return L.WindowOpts(*[base[f] for f, _ in L.WindowOpts._fields_])


@pytest.mark.parametrize("bad", [dict(a_hi=0.0), dict(l_max=0.0), dict(r0_first=0.0),
                                 dict(r0_last=-1.0), dict(r_lo_frac=0.0),
                                 dict(r_hi_frac=0.5), dict(lambda_length=-1.0),
                                 dict(lambda_area=float("nan"))])
def test_loop_entries_reject_bad_windows(lib, bad):
    w = window(**bad)
    buf = C.create_string_buffer(64)
    p = C.cast(buf, C.c_void_p)
    assert lib.tbr_window_map(10, 4, p, p, C.byref(w), None) == L.TBR_E_INVALID
    assert b"window" in lib.tbr_last_error()
    a = L.AdamOpts(0.01, 0.01, 0.01, 0.01, 0.01, 0.01, 0.9, 0.999, 1e-8, 0.002, 0.2, 0.3, 1)
    st = lib.tbr_fit_loop_step(10, 4, p, p, None, p, p, C.byref(w), C.byref(a), C.byref(opts()),
                               p, p, p, 64, None)
    assert st == L.TBR_E_INVALID


def test_loop_entries_reject_null_and_sizes(lib):
    w = window()
    buf = C.create_string_buffer(64)
    p = C.cast(buf, C.c_void_p)
    assert lib.tbr_window_map(-1, 4, p, p, C.byref(w), None) == L.TBR_E_INVALID
    assert lib.tbr_window_map(10, 0, p, p, C.byref(w), None) == L.TBR_E_INVALID
    assert lib.tbr_window_map(10, 4, None, p, C.byref(w), None) == L.TBR_E_INVALID
    assert lib.tbr_window_map(10, 4, p, p, None, None) == L.TBR_E_INVALID
    a = L.AdamOpts(0.01, 0.01, 0.01, 0.01, 0.01, 0.01, 0.9, 0.999, 1e-8, 0.002, 0.2, 0.3, 0)
    st = lib.tbr_fit_loop_step(10, 4, p, p, None, p, p, C.byref(w), C.byref(a), C.byref(opts()),
                               p, p, p, 64, None)
    assert st == L.TBR_E_INVALID  # Adam step counts from 1


def test_loop_step_checks_workspace_before_launching(lib):
    """A workspace too small is rejected before the window map runs (this
    process has no GPU: any launch would fail with a device error)."""
    w = window()
    buf = C.create_string_buffer(64)
    p = C.cast(buf, C.c_void_p)
    a = L.AdamOpts(0.01, 0.01, 0.01, 0.01, 0.01, 0.01, 0.9, 0.999, 1e-8, 0.002, 0.2, 0.3, 1)
    st = lib.tbr_fit_loop_step(10, 4, p, p, None, p, p, C.byref(w), C.byref(a), C.byref(opts()),
                               p, p, p, 64, None)
    assert st == L.TBR_E_INVALID and b"workspace" in lib.tbr_last_error()


@pytest.mark.parametrize("seed", range(6))
def test_coupling_check_is_exact(lib, seed):
    """tbr_coupling_check's minimum of g = 1 + sum_k c_k cos(4 pi k v)
    against dense sampling of the definition; a profile that dips below 0
    is rejected."""
    import numpy as np
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.6, 0.6, size=(200, 3)).astype(np.float32)
    v = np.linspace(0.0, 0.25, 200001)
    g = 1.0 + sum(c[:, k:k + 1].astype(np.float64) * np.cos(4 * np.pi * (k + 1) * v)[None]
                  for k in range(3))
    want = g.min()
    got = C.c_float()
    st = lib.tbr_coupling_check(c.ctypes.data_as(C.c_void_p), len(c), C.byref(got))
    assert got.value == pytest.approx(want, abs=1e-6)
    assert (st == L.TBR_OK) == (want > 0)
    ok = c[g.min(1) > 0]
    st = lib.tbr_coupling_check(ok.ctypes.data_as(C.c_void_p), len(ok), C.byref(got))
    assert st == L.TBR_OK and got.value > 0


def test_coupled_options_need_coefficients(lib):
    o = opts(transport=L.TBR_TRANSPORT_COUPLED, coupling=None)
    prog = L.Program(0, 1, None, None, None, None, None, None, C.c_void_p(16))
    buf = C.create_string_buffer(1 << 16)
    st = lib.tbr_render(C.byref(prog), C.byref(o), L.TBR_SOFT, None, None, None,
                        C.cast(buf, C.c_void_p), 1 << 16, 0, None)
    assert st == L.TBR_E_INVALID and b"coupling" in lib.tbr_last_error()
    o = opts(transport=5)
    st = lib.tbr_render(C.byref(prog), C.byref(o), L.TBR_SOFT, None, None, None,
                        C.cast(buf, C.c_void_p), 1 << 16, 0, None)
    assert st == L.TBR_E_INVALID and b"transport" in lib.tbr_last_error()


def test_compensate_validation(lib):
    """Host-side checks of tbr_compensate (nothing is launched)."""
    buf = C.create_string_buffer(64)
    p = C.cast(buf, C.c_void_p)
    empty = L.Program(0, 1, None, None, None, None, None, None, C.c_void_p(16))
    assert lib.tbr_compensate(C.byref(empty), 1e-3, 1, 0, None, None, None, None, None, None, 0,
                              None) == L.TBR_OK
    prog = L.Program(10, 2, p, p, p, p, p, p, p)
    assert lib.tbr_compensate(C.byref(prog), 0.0, 0, 0, p, p, p, p, p, p, 1 << 20,
                              None) == L.TBR_E_INVALID
    assert lib.tbr_compensate(C.byref(prog), 1e-3, 1, 0, p, p, p, p, p, p, 64,
                              None) == L.TBR_E_INVALID
    assert b"workspace" in lib.tbr_last_error()
    assert lib.tbr_compensate_workspace_bytes(10, 1) >= 10 * 2 * 16
