"""Pins of the oracle's R_D displacement (Sec. "Transfer across transport
constructions": K = 16 drop maps of Lu 2012 of radius s, K pi s^2 =
A_l(r), laid along the segment) against the textbook drop map and its
composition, and of how the renderer uses R_D beside R_A and R_U."""

import math

import numpy as np
import pytest

import textbook as tb
from paper_2609_08722_amd import synth

K = 16
SHAPES = [(0.10, 0.03), (0.05, 0.01), (0.30, 0.005), (0.08, 0.04)]


def stroke_for(ell, r, phi=0.7, m=(0.43, 0.57)):
    return np.array([m[0], m[1], phi, ell, r])


def box_points(stroke, n, seed, half=0.4):
    rng = np.random.default_rng(seed)
    return stroke[:2] + (rng.random((n, 2)) * 2 - 1) * half


def textbook_forward(g, pts, order=1):
    """K classical drop insertions of radius s at the centres of K equal
    pieces of the segment, laid from its -e end (order=1) or the other way."""
    a, b = tb.segment_ends(g)
    s = math.sqrt(tb.steiner_area(abs(g[3]), g[4]) / (K * math.pi))
    js = range(K) if order == 1 else range(K - 1, -1, -1)
    p = np.asarray(pts, dtype=np.float64)
    for j in js:
        p = tb.drop_forward(a + (j + 0.5) / K * (b - a), s, p)
    return p


@pytest.mark.parametrize("r", [0.03, 0.005])
def test_at_a_drop_sixteen_drops_are_one_drop(orc, r):
    """l = 0: sixteen concentric drops of area pi r^2 / 16 are the drop map
    of radius r (Lu 2012), both ways."""
    g = stroke_for(0.0, r)
    p = box_points(g, 20000, 1)
    ext = np.linalg.norm(p - g[:2], axis=1) > r * (1 + 1e-6)
    got, rec = orc.psi_drops(g, p[ext])
    assert not rec.any()
    assert np.max(np.abs(got - tb.drop_backward(g[:2], r, p[ext]))) <= 1e-13
    assert np.max(np.abs(orc.phi_drops(g, p) - tb.drop_forward(g[:2], r, p))) <= 1e-13


@pytest.mark.parametrize("eps", [1e-3, 1e-2])
def test_floor_inside_a_drop(orc, eps):
    """Inside the deposit each drop's map is floored like the capsule's
    C >= (eps r)^2, for the drop's own radius s: pi (rho^2 - s^2) >=
    (eps s)^2. At l = 0 the sixteen drops are concentric with s = r / 4, so
    a point inside ends on the ray it started on, at pi rho'^2 = (eps s)^2."""
    r = 0.03
    g = stroke_for(0.0, r)
    rng = np.random.default_rng(11)
    ang = rng.random(500) * 2 * np.pi
    rad = r * np.sqrt(rng.random(500)) * 0.9 + 1e-4
    p = g[:2] + rad[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    out, rec = orc.psi_drops(g, p, eps=eps)
    assert rec.all()
    s = r / 4
    d = out - g[:2]
    assert np.allclose(np.linalg.norm(d, axis=1), eps * s / math.sqrt(math.pi), rtol=1e-12)
    assert np.allclose(np.arctan2(d[:, 1], d[:, 0]), np.arctan2(p[:, 1] - g[1], p[:, 0] - g[0]),
                       atol=1e-12)


@pytest.mark.parametrize("ell,r", SHAPES)
def test_backward_inverts_the_textbook_sweep(orc, ell, r):
    """psi_D undoes the K textbook insertions laid from the -e end, and not
    the reverse sweep: the drops do not commute."""
    g = stroke_for(ell, r)
    q = box_points(g, 50000, 2)
    y = textbook_forward(g, q)
    back, rec = orc.psi_drops(g, y)
    assert not rec.any()
    assert np.max(np.abs(back - q)) <= 1e-12
    assert np.max(np.abs(orc.phi_drops(g, q) - y)) <= 1e-13
    rev = textbook_forward(g, q, order=-1)
    assert np.max(np.abs(orc.psi_drops(g, rev)[0] - q)) > 1e-6


@pytest.mark.parametrize("ell,r", SHAPES)
def test_jacobian_determinant_is_one(orc, ell, r):
    """Each drop map preserves area outside its disc."""
    g = stroke_for(ell, r)
    p = box_points(g, 20000, 3)
    _, rec = orc.psi_drops(g, p, eps=0.0)
    p = p[~rec]
    for which in ("psi_drops", "phi_drops"):
        J = orc.map_jacobian(which, g, p)[:, :, :2]
        det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
        assert np.max(np.abs(det - 1.0)) <= 1e-11, which


@pytest.mark.parametrize("ell,r", [(0.10, 0.03), (0.30, 0.02)])
def test_inserted_area_monte_carlo(orc, ell, r):
    """The points whose backward path enters a drop's disc (the sixteen
    drops' deposit) cover the stroke's area A_l(r)."""
    g = stroke_for(ell, r, m=(0.0, 0.0))
    rng = np.random.default_rng(4)
    half = ell / 2 + 3 * r
    n = 2_000_000
    pts = (rng.random((n, 2)) * 2 - 1) * half
    _, rec = orc.psi_drops(g, pts, eps=0.0)
    box = (2 * half) ** 2
    frac = rec.mean()
    sd = box * math.sqrt(frac * (1 - frac) / n)
    assert abs(frac * box - tb.steiner_area(ell, r)) <= 4 * sd


def test_renderer_transports(orc):
    """R_D keeps capsule coverage: on a program of drops only it renders as
    R_A; on any program the topmost stroke's footprint (met before any
    displacement) is the same under R_A, R_D and R_U; and with strokes of
    length the three differ."""
    W = H = 40
    drops = synth.make_program(30, 4, 5, synth.StrokeDist(p_drop=1.0), beta=2.0,
                               dtype=np.float64)
    # inside a deposit the floors differ (the capsule's (eps r)^2 against
    # each drop's (eps s)^2), so the two agree as eps -> 0
    a = orc.render(drops, W, H, tau=0.35, tau_c=1.0, transport=1, eps=1e-10)
    d = orc.render(drops, W, H, tau=0.35, tau_c=1.0, transport=2, eps=1e-10)
    assert np.max(np.abs(a["soft"] - d["soft"])) <= 1e-9
    far = a["dmin"] > 1e-9
    assert np.array_equal(a["owner"][far], d["owner"][far])
    prog = synth.make_program(30, 4, 6, synth.DIST_SMALL, beta=2.0, dtype=np.float64)
    prog["half_width"] = prog["half_width"] * 2
    prog["length"] = prog["length"] * 3  # long strokes: the displacements differ most
    outs = [orc.render(prog, W, H, transport=t) for t in (1, 2, 0)]
    top = [o["owner"] == 29 for o in outs]
    assert np.array_equal(top[0], top[1]) and np.array_equal(top[0], top[2]) and top[0].any()
    assert np.mean(outs[0]["owner"] != outs[1]["owner"]) > 0.01
    assert np.mean(outs[0]["owner"] != outs[2]["owner"]) > 0.01
