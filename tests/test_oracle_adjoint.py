"""Pins of the oracle's gradient (Sec. 5.2 Eq. adjstep / Eq. adjparam are
what the GPU implements; the oracle instead uses the generic chain rule with
dual-number Jacobians) against FP64 central differences of the oracle's own
forward render, which the render and operator pins fix independently."""

import numpy as np
import pytest

from paper_2609_08722_amd import synth

GEOM = ("cx", "cy", "angle", "length", "half_width")


def loss_and_seed(orc, prog, W, H, target, **kw):
    R = orc.render(prog, W, H, hard=False, **kw)["soft"]
    diff = R - target
    return float(np.mean(diff ** 2)), 2.0 * diff / diff.size


def close(a, b, rtol, group, atol=0.0):
    """|a - b| <= rtol (|b| + 0.01 RMS(b over the group)) + atol."""
    rms = np.sqrt(np.mean(np.asarray(group) ** 2))
    return np.abs(a - b) <= rtol * (np.abs(b) + 0.01 * rms) + atol


# The fourth case has a floor width so small that far pixels reach
# (r - sigma) / w_d < -709, where exp(-z) overflows in FP64: the coverage
# and its derivative must still come out as the limits 0, not NaN. The last
# is the sixteen-drop renderer R_D.
@pytest.mark.parametrize("tau,tau_c,transport,tau_min", [(1e-3, 1.0, True, None),
                                                          (0.35, 0.5, True, None),
                                                          (1e-3, 1.0, False, None),
                                                          (1e-3, 1.0, True, 1e-4),
                                                          (1e-3, 1.0, 2, None)])
def test_gradient_matches_central_differences(orc, tau, tau_c, transport, tau_min):
    W = H = 24
    prog = synth.make_program(12, 4, 21, synth.DIST_SMALL, beta=2.0, dtype=np.float64)
    prog["half_width"] = prog["half_width"] * 3  # larger strokes: more interaction
    target_prog = synth.make_program(12, 4, 22, synth.DIST_SMALL, dtype=np.float64)
    kw = dict(tau=tau, tau_min=0.7 / W if tau_min is None else tau_min, tau_c=tau_c,
              transport=transport)
    target = orc.render(target_prog, W, H, hard=False, **kw)["soft"]
    loss, seed = loss_and_seed(orc, prog, W, H, target, **kw)
    g = orc.backward(prog, W, H, seed, **kw)
    # The map is only C1 at the flank/cap seams, which sit within l/2 of
    # each end: a small central step is needed (rounding ~ 1e-16 L / h).
    h = 1e-7
    drops = prog["length"] == 0

    def central(name, idx, step):
        pp = {k: v.copy() for k, v in prog.items()}
        pp[name].flat[idx] += step
        lp, _ = loss_and_seed(orc, pp, W, H, target, **kw)
        pp[name].flat[idx] -= 2 * step
        lm, _ = loss_and_seed(orc, pp, W, H, target, **kw)
        return (lp - lm) / (2 * step)

    def fd(name, idx):
        return central(name, idx, h)

    noise = 50 * np.finfo(float).eps * loss / h  # rounding of the FD quotient

    n = len(prog["cx"])
    for q, name in enumerate(GEOM):
        for i in range(n):
            if drops[i] and name in ("angle", "length"):
                continue  # |L| kink at a drop: analytic is the right derivative
            f = fd(name, i)
            assert close(g["geom"][q, i], f, 1e-4, g["geom"][q], noise), (name, i, g["geom"][q, i], f)
    for idx in range(prog["logits"].size):
        f = fd("logits", idx)
        assert close(g["logits"].flat[idx], f, 1e-4, g["logits"], noise), ("logits", idx)
    for idx in range(prog["palette"].size):
        f = fd("palette", idx)
        assert close(g["palette"].flat[idx], f, 1e-4, g["palette"], noise), ("palette", idx)


def test_drop_angle_gradient_is_zero(orc):
    W = H = 24
    prog = synth.make_program(20, 4, 23, synth.StrokeDist(p_drop=1.0), beta=2.0,
                              dtype=np.float64)
    seed = np.random.default_rng(0).normal(size=(W * H, 3))
    g = orc.backward(prog, W, H, seed, tau_c=1.0)
    assert np.max(np.abs(g["geom"][2])) <= 1e-12 * np.max(np.abs(g["geom"]))


def test_colour_gradient_is_soft_owned_area(orc):
    """Upstream gradient 1 everywhere, c_0 = 0, c_i = 1: dL/dc_i is the soft
    area v_i = sum_x T_i alpha_i, and sum_i v_i = sum_x (1 - T_0) = sum_x R."""
    W = H = 32
    n = 40
    prog = synth.make_program(n, 2, 24, synth.DIST_SMALL, dtype=np.float64)
    prog["palette"] = np.array([[0.0, 0, 0], [1.0, 1, 1]])
    prog["logits"] = np.tile([0.0, 1.0], (n, 1))
    R = orc.render(prog, W, H, tau=0.35, hard=False)["soft"]
    g = orc.backward(prog, W, H, np.ones((W * H, 3)), tau=0.35)
    v = g["colour"]
    assert np.all(v >= 0)
    assert np.allclose(v[:, 0], v[:, 1], rtol=0, atol=0)
    assert abs(v[:, 0].sum() - R[:, 0].sum()) <= 1e-12 * R[:, 0].sum()


def test_masked_upstream_equals_pixel_subset(orc):
    W = H = 32
    prog = synth.make_program(25, 4, 25, synth.DIST_SMALL, beta=2.0, dtype=np.float64)
    pix = synth.sample_pixels(W * H, 64, 7)
    rng = np.random.default_rng(1)
    gsub = rng.normal(size=(len(pix), 3))
    full = np.zeros((W * H, 3))
    full[pix] = gsub
    a = orc.backward(prog, W, H, full, tau_c=1.0)
    b = orc.backward(prog, W, H, gsub, tau_c=1.0, pixels=pix)
    for k in a:
        assert np.allclose(a[k], b[k], rtol=1e-13, atol=1e-15), k
