"""Pins of the oracle's renderer (Sec. 3 Eq. chain / Eq. render, Sec. 5.1
Eq. relax, Sec. 5.2 alpha clamp) against independent yardsticks."""

import math

import numpy as np
import pytest

import textbook as tb
from paper_2609_08722_amd import synth

ALPHA_MAX = 1.0 - 1e-7


def small_program(n=30, k=8, seed=5, beta=1.0, dist=synth.DIST_SMALL):
    return synth.make_program(n, k, seed, dist, beta, dtype=np.float64)


def colours(prog, tau_c):
    z = prog["logits"]
    P = prog["palette"]
    if tau_c > 0:
        e = np.exp((z - z.max(1, keepdims=True)) / tau_c)
        s = e / e.sum(1, keepdims=True)
    else:
        s = np.zeros_like(z)
        s[np.arange(len(z)), np.argmax(z, 1)] = 1.0
    return s @ P


def textbook_alpha(prog, pts, tau, tau_min):
    n = len(prog["cx"])
    out = np.empty((n, len(pts)))
    for i in range(n):
        g = [prog[k][i] for k in ("cx", "cy", "angle", "length", "half_width")]
        d = tb.seg_distance(g, pts)
        r = g[4]
        wdt = max(tau * r, tau_min)
        out[i] = np.minimum(tb.sigmoid((r - d) / wdt), ALPHA_MAX)
    return out


@pytest.mark.parametrize("tau,tau_c", [(1e-3, 0.0), (0.35, 1.0)])
def test_inert_soft_is_porter_duff(orc, tau, tau_c):
    W = H = 32
    prog = small_program(beta=2.0)
    tau_min = 0.7 / W
    out = orc.render(prog, W, H, tau=tau, tau_min=tau_min, tau_c=tau_c, transport=False)
    pts = tb.pixel_centres(W, H)
    a = textbook_alpha(prog, pts, tau, tau_min)
    want = tb.porter_duff(colours(prog, tau_c), a, prog["palette"][0])
    assert np.max(np.abs(out["soft"] - want)) <= 1e-14


def test_inert_hard_is_topmost_footprint(orc):
    W = H = 48
    prog = small_program(n=40)
    out = orc.render(prog, W, H, transport=False)
    pts = tb.pixel_centres(W, H)
    owner = np.full(len(pts), -1)
    for i in range(len(prog["cx"])):
        g = [prog[k][i] for k in ("cx", "cy", "angle", "length", "half_width")]
        inside = tb.seg_distance(g, pts) <= g[4]
        owner[inside] = i  # later strokes overwrite
    assert np.array_equal(out["owner"], owner)
    lab = np.where(owner >= 0, np.argmax(prog["logits"][np.maximum(owner, 0)], 1), 0)
    assert np.array_equal(out["label"], lab)
    assert np.array_equal(out["hard"], prog["palette"][lab])


def drops_renderer(prog, W, H, tau, tau_min, eps):
    """Ten-line independent renderer for drops-only programs: the chain is a
    composition of classical drop maps (with the implemented floor)."""
    pts = tb.pixel_centres(W, H)
    cols = colours(prog, 0.0)
    C = np.zeros((len(pts), 3))
    T = np.ones(len(pts))
    owner = np.full(len(pts), -1)
    for i in range(len(prog["cx"]) - 1, -1, -1):
        c = np.array([prog["cx"][i], prog["cy"][i]])
        r = prog["half_width"][i]
        d = np.linalg.norm(pts - c, axis=1)
        a = np.minimum(tb.sigmoid((r - d) / max(tau * r, tau_min)), ALPHA_MAX)
        C += (T * a)[:, None] * cols[i]
        T *= 1 - a
        owner = np.where((owner == -1) & (d <= r), -2 - i, owner)  # first hit only
        pts = tb.drop_backward(c, r, pts, floor_c=(eps * r) ** 2)
    return C + T[:, None] * prog["palette"][0], np.where(owner <= -2, -2 - owner, -1)


def test_drops_only_chain(orc):
    W = H = 40
    dist = synth.StrokeDist(p_drop=1.0, r_lo=0.02, r_hi=0.06)
    prog = small_program(n=60, dist=dist, seed=9)
    out = orc.render(prog, W, H, tau=1e-3, tau_min=0.7 / W)
    soft, owner = drops_renderer(prog, W, H, 1e-3, 0.7 / W, 1e-3)
    assert np.max(np.abs(out["soft"] - soft)) <= 1e-13
    assert np.array_equal(out["owner"], owner)


def test_unit_colour_identity(orc):
    """c_i = 1, c_0 = 0: R = 1 - T_0 per channel, a value in [0, 1) that
    grows with every stroke (the compositing identity of the paper's
    non-visible-pigment penalty)."""
    W = H = 32
    prog = small_program(n=50)
    prog["palette"] = np.array([[0.0, 0, 0], [1.0, 1, 1]])
    prog["logits"] = np.tile([0.0, 1.0], (50, 1))
    out = orc.render(prog, W, H, tau=0.35, tau_min=0.7 / W)
    R = out["soft"]
    assert np.allclose(R[:, 0], R[:, 1], rtol=0, atol=0) and np.allclose(R[:, 0], R[:, 2], atol=0)
    pts = tb.pixel_centres(W, H)
    # with transport off, T_0 = prod(1 - alpha_i) directly
    inert = orc.render(prog, W, H, tau=0.35, tau_min=0.7 / W, transport=False)
    a = textbook_alpha(prog, pts, 0.35, 0.7 / W)
    assert np.max(np.abs(inert["soft"][:, 0] - (1 - np.prod(1 - a, axis=0)))) <= 1e-14
    assert R.min() >= 0 and R.max() < 1


def test_recolour_changes_only_owned_pixels(orc):
    W = H = 48
    prog = small_program(n=40)
    base = orc.render(prog, W, H)
    pal = prog["palette"].copy()
    pal[3] = [0.123, 0.456, 0.789]
    prog2 = dict(prog, palette=pal)
    new = orc.render(prog2, W, H)
    assert np.array_equal(base["owner"], new["owner"])
    changed = np.any(base["hard"] != new["hard"], axis=1)
    assert np.array_equal(changed, base["label"] == 3)
    # soft colours move only where stroke colours 3 (or background) appear
    assert np.array_equal(base["n_rec"], new["n_rec"])


def test_rotation_metamorphic(orc):
    """Rotating every stroke by 90 degrees about the canvas centre permutes
    the pixel-centre grid (a symmetry of the canvas and of the operator)."""
    W = H = 40
    prog = small_program(n=40, seed=12)
    rot = dict(prog)
    rot["cx"] = 1.0 - prog["cy"]
    rot["cy"] = prog["cx"].copy()
    rot["angle"] = prog["angle"] + math.pi / 2
    a = orc.render(prog, W, H)
    b = orc.render(rot, W, H)
    # (x, y) -> (1 - y, x): pixel (row i, col j) -> (row j, col W-1-i)
    ii, jj = np.divmod(np.arange(W * H), W)
    dest = jj * W + (W - 1 - ii)
    assert np.array_equal(b["owner"][dest], a["owner"])
    assert np.array_equal(b["label"][dest], a["label"])
    assert np.max(np.abs(b["soft"][dest] - a["soft"])) <= 1e-12


def test_soft_tends_to_hard(orc):
    """tau, tau_min -> 0: the soft composite becomes the hard render away
    from footprint boundaries."""
    W = H = 48
    prog = small_program(n=40, seed=13)
    hard = orc.render(prog, W, H)
    errs = []
    for tm in (1e-3, 1e-4, 1e-6):
        soft = orc.render(prog, W, H, tau=0.0, tau_min=tm, hard=False)["soft"]
        far = hard["dmin"] > 25 * tm
        errs.append(np.max(np.abs(soft[far] - hard["hard"][far])))
    assert far.mean() > 0.9
    assert max(errs) <= 1e-6
    # near boundaries the relaxation really is different
    soft = orc.render(prog, W, H, tau=0.0, tau_min=1e-3, hard=False)["soft"]
    assert np.max(np.abs(soft - hard["hard"])) > 1e-2


def test_inert_record_count_is_footprint_count(orc):
    """With transport off, the floor binds exactly inside footprints (plus a
    sliver thinner than eps^2 r / (2 pi), which pixel centres avoid here)."""
    W = H = 40
    prog = small_program(n=40, seed=14)
    out = orc.render(prog, W, H, transport=False, hard=False)
    pts = tb.pixel_centres(W, H)
    cnt = np.zeros(len(pts), dtype=np.int32)
    for i in range(len(prog["cx"])):
        g = [prog[k][i] for k in ("cx", "cy", "angle", "length", "half_width")]
        cnt += (tb.seg_distance(g, pts) <= g[4]).astype(np.int32)
    assert np.array_equal(out["n_rec"], cnt)


def test_pixel_subset_matches_full(orc):
    W = H = 32
    prog = small_program(n=30, seed=15)
    full = orc.render(prog, W, H)
    pix = synth.sample_pixels(W * H, 100, 3)
    sub = orc.render(prog, W, H, pixels=pix)
    for k in ("soft", "hard", "label", "owner", "dmin", "n_rec"):
        assert np.array_equal(sub[k], full[k][pix]), k


def test_inert_dmin_is_textbook_minimum_over_visited_strokes(orc):
    """The hard trace's boundary distance (the quantity that exempts a pixel
    from hard-label parity, a pixel within 1e-5 of a closed footprint's edge,
    Sec. 3): with transport off the point stays put, so it is the minimum of
    |dist(x, segment_i) - r_i| over the strokes the trace visits, N-1 down to
    the owner (all of them when no stroke owns the pixel)."""
    W = H = 40
    prog = small_program(n=45, seed=17)
    out = orc.render(prog, W, H, transport=False)
    pts = tb.pixel_centres(W, H)
    want = np.full(len(pts), np.inf)
    done = np.zeros(len(pts), bool)
    for i in range(len(prog["cx"]) - 1, -1, -1):
        g = [prog[k][i] for k in ("cx", "cy", "angle", "length", "half_width")]
        d = tb.seg_distance(g, pts)
        want = np.where(done, want, np.minimum(want, np.abs(d - g[4])))
        done |= d <= g[4]
    assert np.max(np.abs(out["dmin"] - want)) <= 1e-14
    # an owner-step-only minimum, or one over every stroke, would differ
    assert np.any(out["owner"] == -1) and np.any(out["owner"] >= 0)


def test_drops_dmin_follows_the_textbook_chain(orc):
    """With transport on, a drops-only program's boundary distance is the
    minimum of ||x_i - c_i| - r_i| along the chain of classical drop maps,
    up to the first hit."""
    W = H = 40
    dist = synth.StrokeDist(p_drop=1.0, r_lo=0.02, r_hi=0.06)
    prog = small_program(n=60, dist=dist, seed=9)
    out = orc.render(prog, W, H)
    pts = tb.pixel_centres(W, H)
    want = np.full(len(pts), np.inf)
    done = np.zeros(len(pts), bool)
    for i in range(len(prog["cx"]) - 1, -1, -1):
        c = np.array([prog["cx"][i], prog["cy"][i]])
        r = prog["half_width"][i]
        d = np.linalg.norm(pts - c, axis=1)
        want = np.where(done, want, np.minimum(want, np.abs(d - r)))
        done |= d <= r
        pts = tb.drop_backward(c, r, pts, floor_c=(1e-3 * r) ** 2)
    assert np.max(np.abs(out["dmin"] - want)) <= 1e-12
