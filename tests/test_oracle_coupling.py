"""Pins of the oracle's calibrated coupling Phi_g (Sec. 4, "A variant closer
to line-source potential flow": Eq. coupling, Eq. profile) against closed
forms, invariants and brute force. The variant adds the area A_l(r) g(v)
along the leaf of centred fraction v, with g(v) = 1 + sum_k c_k cos(4 pi k v),
so its deposit is {u <= A_l(r) g(v)}."""

import math

import numpy as np
import pytest

import textbook as tb
from paper_2609_08722_amd import synth

GEOM = ("cx", "cy", "angle", "length", "half_width")

# profiles with g > 0 everywhere (min over v: 0.8, 0.7, 0.77)
COEFFS = [(0.2, 0.0, 0.0), (0.15, -0.1, 0.05), (-0.25, 0.1, 0.08)]
SHAPES = [(0.10, 0.03), (0.0, 0.03), (0.05, 0.01), (0.30, 0.005)]


def stroke_for(ell, r, phi=0.7, m=(0.43, 0.57)):
    return np.array([m[0], m[1], phi, ell, r])


def box_points(stroke, n, seed, half=0.4):
    rng = np.random.default_rng(seed)
    return stroke[:2] + (rng.random((n, 2)) * 2 - 1) * half


def g_of(theta_n, c):
    """Eq. profile at a drop, where the centred fraction is the polar angle
    from the normal over 2 pi: g = 1 + sum_k c_k cos(2 k theta_n)."""
    return 1.0 + sum(ck * np.cos(2.0 * (k + 1) * theta_n) for k, ck in enumerate(c))


def exterior_coupled(orc, g, c, pts, factor):
    sig, _, edge = orc.chart(g, pts, coupling=c, edge=True)
    return pts[sig >= factor * edge]


def test_zero_coefficients_give_the_uniform_map(orc):
    for ell, r in SHAPES:
        g = stroke_for(ell, r)
        p = box_points(g, 20000, 1)
        a, ra = orc.psi(g, p)
        b, rb = orc.psi(g, p, coupling=(0.0, 0.0, 0.0))
        assert np.max(np.abs(a - b)) <= 1e-13 and np.array_equal(ra, rb)
        assert np.max(np.abs(orc.phi(g, p) - orc.phi(g, p, coupling=(0, 0, 0)))) <= 1e-13
    prog = synth.make_program(30, 4, 3, synth.DIST_SMALL, beta=2.0, dtype=np.float64)
    u = orc.render(prog, 32, 32, tau=0.35, tau_c=1.0)
    z = orc.render(prog, 32, 32, tau=0.35, tau_c=1.0, coupling=np.zeros((30, 3)))
    assert np.max(np.abs(u["soft"] - z["soft"])) <= 1e-12
    assert np.array_equal(u["owner"], z["owner"])


@pytest.mark.parametrize("c", COEFFS)
@pytest.mark.parametrize("ell,r", SHAPES)
def test_round_trips_outside_deposit(orc, ell, r, c):
    g = stroke_for(ell, r)
    p = exterior_coupled(orc, g, c, box_points(g, 100000, 4), 1.0 + 1e-5)
    back, rec = orc.psi(g, p, coupling=c)
    assert not rec.any()
    assert np.max(np.abs(orc.phi(g, back, coupling=c) - p)) <= 1e-12
    q = box_points(g, 100000, 5)
    fwd = orc.phi(g, q, coupling=c)
    # Phi_g maps the plane minus the segment outside its deposit
    sig, _, edge = orc.chart(g, fwd, coupling=c, edge=True)
    assert np.all(sig > edge)
    again, rec2 = orc.psi(g, fwd, coupling=c)
    ok = ~rec2
    assert ok.mean() > 0.999
    assert np.max(np.abs(again[ok] - q[ok])) <= 1e-12


@pytest.mark.parametrize("c", COEFFS)
@pytest.mark.parametrize("ell,r", SHAPES)
def test_jacobian_determinant_is_one(orc, ell, r, c):
    """Eq. coupling is unit triangular in the area chart: det J = 1, by the
    dual-number Jacobian and by a 5-point stencil away from the C1 seams."""
    g = stroke_for(ell, r)
    p = exterior_coupled(orc, g, c, box_points(g, 20000, 6), 1.1)
    for which in ("psi", "phi"):
        J = orc.map_jacobian(which, g, p, coupling=c)[:, :, :2]
        det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
        assert np.max(np.abs(det - 1.0)) <= 1e-12, which
    p = p[:3000]
    out, _ = orc.psi(g, p, coupling=c)
    s_in, _ = tb.local(g, p)
    s_out, _ = tb.local(g, out)
    seam = (np.minimum(np.abs(np.abs(s_in) - ell / 2), np.abs(np.abs(s_out) - ell / 2))
            if ell > 0 else np.full(len(p), np.inf))
    keep = seam > 1e-3
    p, sig_out, seam = p[keep], tb.seg_distance(g, out[keep]), seam[keep]
    h = np.maximum(1e-3 * np.minimum(sig_out, seam), 1e-6)[:, None]
    cols = []
    for k in range(2):
        e = np.zeros(2)
        e[k] = 1.0
        f = [orc.psi(g, p + s * h * e, coupling=c)[0] for s in (2, 1, -1, -2)]
        cols.append((-f[0] + 8 * f[1] - 8 * f[2] + f[3]) / (12 * h))
    det = cols[0][:, 0] * cols[1][:, 1] - cols[1][:, 0] * cols[0][:, 1]
    assert len(det) > 1000
    assert np.max(np.abs(det - 1.0)) <= 1e-9


@pytest.mark.parametrize("c", COEFFS)
def test_drop_closed_form(orc, c):
    """At l = 0 the leaf fraction is the polar angle from the normal over
    2 pi, so Phi_g moves a point radially from sigma to
    sqrt(sigma^2 + r^2 g) and psi_g back to sqrt(sigma'^2 - r^2 g)."""
    r = 0.03
    g = stroke_for(0.0, r)
    p = box_points(g, 50000, 7)
    s_, h_ = tb.local(g, p)
    th = np.arctan2(s_, h_)  # angle from the normal n toward e
    d = np.hypot(s_, h_)
    gv = g_of(th, c)
    ext = d * d > r * r * gv * (1 + 1e-6)
    want_b = g[:2] + (p - g[:2]) * (np.sqrt(np.maximum(d * d - r * r * gv, 0)) / d)[:, None]
    got_b, _ = orc.psi(g, p, coupling=c)
    assert np.max(np.abs(got_b[ext] - want_b[ext])) <= 1e-13
    want_f = g[:2] + (p - g[:2]) * (np.sqrt(d * d + r * r * gv) / d)[:, None]
    assert np.max(np.abs(orc.phi(g, p, coupling=c) - want_f)) <= 1e-13


def test_first_mode_widens_the_flank_and_shortens_the_tips(orc):
    """Sec. 4, Eq. profile: with c_1 > 0 the profile g is above 1 across the
    middle of the segment and below 1 beyond its ends, so the deposit reaches
    past r beside the segment and stops short of r past its ends."""
    ell, r, c1 = 0.10, 0.03, 0.3
    g = stroke_for(ell, r)
    prog = {"cx": g[:1], "cy": g[1:2], "angle": g[2:3], "length": g[3:4],
            "half_width": g[4:5], "logits": np.zeros((1, 1)), "palette": np.zeros((1, 3))}
    A = tb.steiner_area(ell, r)
    wide = tb.inverse_area(ell, A * (1 + c1))   # flank midpoint, g = 1 + c_1
    short = tb.inverse_area(ell, A * (1 - c1))  # tip, g = 1 - c_1
    assert wide > r > short
    d_in = np.linspace(r, wide, 7)[1:-1]
    d_out = np.linspace(short, r, 7)[1:-1]
    for sgn in (1, -1):
        on_normal = tb.from_local(g, np.zeros_like(d_in), sgn * d_in)
        past_end = tb.from_local(g, sgn * (ell / 2 + d_out), np.zeros_like(d_out))
        cp = np.array([[c1, 0.0, 0.0]])
        assert np.all(orc.hard_points(prog, on_normal, coupling=cp) == 0)
        assert np.all(orc.hard_points(prog, past_end, coupling=cp) == -1)
        assert np.all(orc.hard_points(prog, past_end) == 0)  # inside under g = 1


@pytest.mark.parametrize("c", COEFFS)
@pytest.mark.parametrize("ell,r", [(0.10, 0.03), (0.05, 0.01)])
def test_reflection_commutation(orc, ell, r, c):
    """The modes cos(4 pi k v) respect both reflections of Prop. centred
    arclength, so psi_g commutes with them."""
    g = stroke_for(ell, r)
    p = exterior_coupled(orc, g, c, box_points(g, 50000, 9), 1.0 + 1e-5)
    s_, h_ = tb.local(g, p)
    base, _ = orc.psi(g, p, coupling=c)
    bs, bh = tb.local(g, base)
    for fs, fh in ((-1, 1), (1, -1)):
        refl, _ = orc.psi(g, tb.from_local(g, fs * s_, fh * h_), coupling=c)
        want = tb.from_local(g, fs * bs, fh * bh)
        assert np.max(np.abs(refl - want)) <= 1e-13


def test_owner_area_law_monte_carlo(orc):
    """g has unit mean, so each stroke still inserts A_l(r): in the final
    plane the set a stroke owns has area A_l(r) whatever later strokes do."""
    rng = np.random.default_rng(19)
    n = 6
    prog = {
        "cx": 0.3 + 0.4 * rng.random(n), "cy": 0.3 + 0.4 * rng.random(n),
        "angle": rng.random(n) * 2 * np.pi,
        "length": np.where(rng.random(n) < 0.3, 0.0, 0.3 * rng.random(n)),
        "half_width": 0.05 + 0.07 * rng.random(n),
        "logits": np.zeros((n, 2)), "palette": np.zeros((2, 3)),
    }
    coup = np.array([COEFFS[i % 3] for i in range(n)])
    box_lo, box_hi = -0.5, 1.5
    m = 4_000_000
    pts = box_lo + (box_hi - box_lo) * rng.random((m, 2))
    own = orc.hard_points(prog, pts, coupling=coup)
    area_box = (box_hi - box_lo) ** 2
    for i in range(n):
        frac = np.mean(own == i)
        est = frac * area_box
        sd = area_box * math.sqrt(frac * (1 - frac) / m)
        want = tb.steiner_area(abs(prog["length"][i]), prog["half_width"][i])
        assert abs(est - want) <= 4 * sd, (i, est, want, sd)


def test_gradient_matches_central_differences(orc):
    """The oracle's gradient under the coupling (dual numbers through g(v))
    against FP64 central differences of its own render. A drop's angle now
    matters: g is taken in the stroke's frame."""
    W = H = 24
    prog = synth.make_program(12, 4, 21, synth.DIST_SMALL, beta=2.0, dtype=np.float64)
    prog["half_width"] = prog["half_width"] * 3
    coup = np.array([COEFFS[i % 3] for i in range(12)])
    target_prog = synth.make_program(12, 4, 22, synth.DIST_SMALL, dtype=np.float64)
    kw = dict(tau=0.35, tau_min=0.7 / W, tau_c=1.0, coupling=coup)
    target = orc.render(target_prog, W, H, hard=False, tau=0.35, tau_c=1.0)["soft"]

    def loss(pp):
        R = orc.render(pp, W, H, hard=False, **kw)["soft"]
        return float(np.mean((R - target) ** 2)), R

    l0, R = loss(prog)
    g = orc.backward(prog, W, H, 2.0 * (R - target) / R.size, **kw)
    h = 1e-7
    noise = 50 * np.finfo(float).eps * l0 / h
    drops = prog["length"] == 0
    assert drops.any()
    for q, name in enumerate(GEOM):
        rms = np.sqrt(np.mean(g["geom"][q] ** 2))
        for i in range(12):
            if drops[i] and name == "length":
                continue  # |L| kink at a drop
            pp = {k: v.copy() for k, v in prog.items()}
            pp[name][i] += h
            lp, _ = loss(pp)
            pp[name][i] -= 2 * h
            lm, _ = loss(pp)
            f = (lp - lm) / (2 * h)
            assert abs(g["geom"][q, i] - f) <= 1e-4 * (abs(f) + 0.01 * rms) + noise, (name, i)
    # a drop's angle gradient is not zero under a non-trivial profile
    assert np.any(np.abs(g["geom"][2][drops]) > 1e-6 * np.abs(g["geom"][2]).max())


def test_soft_tends_to_hard(orc):
    """tau, tau_min -> 0: the soft composite under the coupling becomes its
    hard render (deposit {u <= A_l(r) g(v)}) away from the deposits' edges,
    and differs from the uniform hard render."""
    W = H = 48
    prog = synth.make_program(40, 4, 13, synth.DIST_SMALL, beta=2.0, dtype=np.float64)
    prog["half_width"] = prog["half_width"] * 2
    coup = np.array([COEFFS[i % 3] for i in range(40)]) * 2.0  # min g 0.4
    hard = orc.render(prog, W, H, coupling=coup)
    for tm in (1e-4, 1e-6):
        soft = orc.render(prog, W, H, tau=0.0, tau_min=tm, hard=False, coupling=coup)["soft"]
        far = hard["dmin"] > 25 * tm
        assert far.mean() > 0.9
        assert np.max(np.abs(soft[far] - hard["hard"][far])) <= 1e-6
    uni = orc.render(prog, W, H)
    assert np.mean(uni["owner"] != hard["owner"]) > 0.01
