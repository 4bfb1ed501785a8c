"""Pins of the fitting-loop oracle (Sec. 5.1 parameterisation, Table hyper
schedule and regulariser, Sec. 8 area budget): finite differences, the
values printed in Table hyper, closed forms of the schedule and of Adam."""

import math

import numpy as np
import pytest

from oracle import fitloop as fl

N, K = 7, 3


def rand_theta(seed, n=N, k=K, scale=1.5):
    rng = np.random.default_rng(seed)
    return rng.normal(size=5 * n + n * k + 3 * k) * scale


def test_table_hyper_window_range_and_parameter_count():
    # "r in [0.003, 0.204]" and "2000 / 26,024 (13 per stroke, palette 8x3)"
    cfg = fl.WindowCfg()
    c0 = fl.r0(2000, cfg)
    assert c0[0] == pytest.approx(0.120) and c0[-1] == pytest.approx(0.005)
    lo, hi = cfg.r_lo_frac * c0.min(), cfg.r_hi_frac * c0.max()
    assert lo == pytest.approx(0.003) and hi == pytest.approx(0.204)
    n, k = 2000, 8
    assert 5 * n + n * k + 3 * k == 26024


def test_r0_is_geometric():
    c0 = fl.r0(50, fl.WindowCfg())
    ratios = c0[1:] / c0[:-1]
    assert np.allclose(ratios, ratios[0], rtol=1e-13, atol=0)


def test_window_map_respects_windows_and_segment_geometry():
    cfg = fl.WindowCfg()
    th = rand_theta(1, scale=4.0)
    nat = fl.window_map(th, N, K, cfg)
    cx, cy, angle, length, r, z, P = fl.split(nat, N, K)
    tax, tay, tdx, tdy, tr, tc, tp = fl.split(th, N, K)
    c0 = fl.r0(N, cfg)
    assert np.all(r >= 0.6 * c0) and np.all(r <= 1.7 * c0)
    assert np.all((P > 0) & (P < 1))
    assert np.array_equal(z, tc)
    dx, dy = length * np.cos(angle), length * np.sin(angle)
    assert np.allclose(dx, cfg.l_max * np.tanh(tdx), atol=1e-15)
    assert np.allclose(dy, cfg.l_max * np.tanh(tdy), atol=1e-15)
    # the anchor (segment start) is back inside the window
    ax, ay = cx - dx / 2, cy - dy / 2
    assert np.all((ax >= 0) & (ax <= 1) & (ay >= 0) & (ay <= 1))
    assert np.allclose(ax, 1 / (1 + np.exp(-tax)), atol=1e-15)


@pytest.mark.parametrize("seed", [2, 3, 4])
def test_window_vjp_matches_central_differences(seed):
    cfg = fl.WindowCfg(a_lo=-0.2, a_hi=1.3)
    th = rand_theta(seed)
    rng = np.random.default_rng(100 + seed)
    g_nat = rng.normal(size=th.size)
    got = fl.window_vjp(th, g_nat, N, K, cfg)
    h = 1e-6
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        fd = (fl.window_map(th + e, N, K, cfg) - fl.window_map(th - e, N, K, cfg)) @ g_nat / (2 * h)
        assert got[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_drop_offset_has_zero_angle_and_no_direction_gradient():
    cfg = fl.WindowCfg()
    th = rand_theta(5)
    th[2 * N:4 * N] = 0.0  # d = 0: a drop
    nat = fl.window_map(th, N, K, cfg)
    _, _, angle, length, _, _, _ = fl.split(nat, N, K)
    assert np.all(angle == 0) and np.all(length == 0)
    g_nat = np.zeros_like(th)
    g_nat[0:N] = 1.0          # dL/dm_x
    g_nat[2 * N:3 * N] = 7.0  # dL/dphi: no effect at a drop
    g_nat[3 * N:4 * N] = 5.0  # dL/dl: no direction at a drop
    g = fl.window_vjp(th, g_nat, N, K, cfg)
    # d m_x / d d_x = 1/2 and d d_x / d th_dx = l_max at th = 0
    assert np.allclose(g[2 * N:3 * N], 0.5 * cfg.l_max)
    assert np.allclose(g[3 * N:4 * N], 0.0)


def test_regulariser_gradient_and_area_derivative():
    cfg = fl.WindowCfg(lambda_length=3e-4, lambda_area=0.7)
    nat = fl.window_map(rand_theta(6), N, K, cfg)
    value, g = fl.regularisers(nat, N, K, cfg)
    h = 1e-7
    for i in range(3 * N, 5 * N):
        e = np.zeros_like(nat)
        e[i] = h
        fd = (fl.regularisers(nat + e, N, K, cfg)[0] - fl.regularisers(nat - e, N, K, cfg)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6), i
    # d A_l(r) / d r is the Steiner perimeter P_l(r) = 2 l + 2 pi r
    _, _, _, length, r, _, _ = fl.split(nat, N, K)
    assert np.allclose(g[4 * N:5 * N], 0.7 * (2 * length + 2 * math.pi * r), rtol=1e-14)
    assert value == pytest.approx(3e-4 * length.sum() + 0.7 * (2 * length * r + math.pi * r * r).sum())


def test_schedule_end_points_and_ratios():
    cfg = fl.ScheduleCfg(total_steps=240)
    t0, c0, l0 = fl.schedule(0, cfg)
    t1, c1, l1 = fl.schedule(239, cfg)
    assert (t0, c0, l0) == (pytest.approx(0.35), pytest.approx(1.0), pytest.approx(1.0))
    assert t1 == pytest.approx(0.02) and c1 == pytest.approx(0.05)
    taus = np.array([fl.schedule(s, cfg)[0] for s in range(240)])
    assert np.allclose(taus[1:] / taus[:-1], (0.02 / 0.35) ** (1 / 239), rtol=1e-12)
    lrs = np.array([fl.schedule(s, cfg)[2] for s in range(240)])
    assert np.all(np.diff(lrs) < 0) and lrs[-1] == pytest.approx(0.5 * (1 + math.cos(math.pi * 239 / 240)))
    assert fl.schedule(120, cfg)[2] == pytest.approx(0.5)


def test_first_adam_steps_move_by_the_step_size():
    rng = np.random.default_rng(7)
    th = rng.normal(size=20)
    g = rng.normal(size=20)
    lrs = np.full(20, 0.015)
    m = v = np.zeros(20)
    t1, m, v = fl.adam_step(th, g, m, v, 1, lrs)
    # bias-corrected m / sqrt(v) = g / |g| at step 1
    assert np.allclose(t1, th - 0.015 * np.sign(g), atol=1e-9)
    t2, m, v = fl.adam_step(t1, g, m, v, 2, lrs)  # the same gradient again
    assert np.allclose(t2, t1 - 0.015 * np.sign(g), atol=1e-9)


def test_window_inverse_round_trip():
    cfg = fl.WindowCfg()
    th = rand_theta(8, scale=1.0)
    nat = fl.window_map(th, N, K, cfg)
    back = fl.window_inverse(nat, N, K, cfg)
    assert np.allclose(fl.window_map(back, N, K, cfg), nat, atol=1e-12)
