"""GPU parity of the closed-form compensation pass (tbr_compensate) with the
FP64 oracle, anchor and endpoint variants, blocked steps clamped or skipped,
up to 2000 strokes.

Blocked chains are chaotic: a clamp into a later footprint can land points
of different strokes on top of one another, and a later clamp of a point
lying on a segment has no defined side (or, at a drop, direction). On a
sparse program (test_sparse_2000_end_to_end) the parity is end to end: the
oracle compensates the inert program alone, and every stroke whose chain
is clean in the oracle's own pass must match. On the dense programs it is
step-wise: each stroke, pre-imaged by the oracle through the GPU's own
compensated later strokes, must match the GPU's stroke; strokes whose chain passed within 1e-5 of a footprint edge,
clamped a point within 1e-6 of a segment, or grows an error more than
100-fold from some step to its end (the oracle's Jacobian products), are
exempt (their counts are logged), as are hard labels near an edge. Unblocked strokes must also
round-trip: pushed forward through the later strokes by the oracle's FP64
map, they land on the inert program's points."""

import numpy as np
import pytest

from gpu_util import log, require_gpu
from paper_2609_08722_amd import api, synth

pytestmark = pytest.mark.gpu
FIELDS = ("cx", "cy", "angle", "length")


def dense_program(n, seed, widen=3.0, lengthen=2.0):
    prog = synth.make_program(n, 4, seed, synth.DIST_SMALL, beta=2.0)
    prog["length"] = (prog["length"] * lengthen).astype(np.float32)
    prog["half_width"] = (prog["half_width"] * widen).astype(np.float32)
    return prog


def ends(prog, i, endpoint):
    e = np.stack([np.cos(prog["angle"][i]), np.sin(prog["angle"][i])], -1)
    m = np.stack([prog["cx"][i], prog["cy"][i]], -1)
    h = 0.5 * prog["length"][i][..., None] * e
    return [m - h, m + h] if endpoint else [m - h]


def check(orc, prog, endpoint, skip, name, min_clean=0.9, tol=1e-5):
    require_gpu()
    out, blocked = api.compensate(api.to_device(prog), endpoint=endpoint, skip_blocked=skip)
    got = {f: out[f].cpu().numpy().astype(np.float64) for f in FIELDS}
    gb = blocked.cpu().numpy()
    ref, rb, dmin, smin, amp = orc.compensate(prog, endpoint=endpoint, skip=skip,
                                              with_dmin=True, later=got, with_amp=True)
    # a chain that keeps 1e-5 from every footprint edge, clamps no point
    # lying on a segment and grows an error at most 100-fold is
    # well-conditioned: FP32 maps then stay within about 1e-5 of FP64
    clean = (dmin >= 1e-5) & (smin >= 1e-6) & (amp <= 100)
    dpos = np.maximum(np.abs(got["cx"] - ref["cx"]), np.abs(got["cy"] - ref["cy"]))
    dang = np.abs(np.angle(np.exp(1j * (got["angle"] - ref["angle"]))))
    dlen = np.abs(got["length"] - ref["length"])
    n = len(gb)
    # round trip of the unblocked strokes through the GPU's later strokes
    g64 = {**got, "half_width": np.asarray(prog["half_width"], np.float64)}
    inert = {f: np.asarray(prog[f], np.float64) for f in ("cx", "cy", "angle", "length")}
    pts = ends(g64, np.arange(n), endpoint)
    for j in range(1, n):
        stroke = np.array([g64[f][j] for f in ("cx", "cy", "angle", "length", "half_width")])
        for q in range(len(pts)):
            pts[q][:j] = orc.phi(stroke, pts[q][:j])
    want = ends(inert, np.arange(n), endpoint)
    rt = np.max([np.abs(a - b).max(1) for a, b in zip(pts, want)], axis=0)
    unb = gb == 0
    log(f"[compensate {name}] N={n}: blocked {int((gb > 0).sum())}; exempt {int((~clean).sum())}; "
        f"clean max |d centre| {dpos[clean].max(initial=0):.2e}, "
        f"|d length| {dlen[clean].max(initial=0):.2e}; unblocked round trip max "
        f"{rt[unb].max(initial=0):.2e}")
    assert clean.mean() >= min_clean
    assert np.array_equal(gb[clean], rb[clean])
    assert dpos[clean].max(initial=0) <= tol and dlen[clean].max(initial=0) <= tol
    long_ = clean & (ref["length"] > 1e-3)
    assert dang[long_].max(initial=0) <= 1e3 * tol
    assert rt[unb].max(initial=0) <= tol
    return gb


@pytest.mark.parametrize("endpoint", [False, True])
def test_small_dense_clamp(orc, endpoint):
    gb = check(orc, dense_program(60, 5), endpoint, False, f"60 endpoint={endpoint}")
    assert (gb > 0).sum() >= 10


@pytest.mark.parametrize("endpoint", [False, True])
def test_skip_blocked(orc, endpoint):
    check(orc, dense_program(60, 5), endpoint, True, f"60 skip endpoint={endpoint}")


# Least clean fractions, from the oracle's own chains with margin: clamping
# collapses blocked points onto later segments; skipping does not, but
# leaves them where later maps stretch the most.
@pytest.mark.parametrize("skip,min_clean", [(False, 0.7), (True, 0.85)])
def test_500_strokes(orc, skip, min_clean):
    w = synth.WORKLOADS["adj256x256_n500"]
    check(orc, synth.workload_program(w), True, skip, f"500 endpoint skip={skip}", min_clean)


@pytest.mark.parametrize("endpoint", [False, True])
@pytest.mark.parametrize("skip,min_clean", [(False, 0.3), (True, 0.45)])
def test_2000_strokes(orc, endpoint, skip, min_clean):
    """The benchmark program: 1,999,000 anchor maps, 3,998,000 endpoint maps."""
    w = synth.WORKLOADS["fit1024x1024_n2000"]
    check(orc, synth.workload_program(w), endpoint, skip,
          f"2000 endpoint={endpoint} skip={skip}", min_clean)


def test_edge_cases(orc):
    require_gpu()
    empty = {f: np.zeros(0, np.float32) for f in ("cx", "cy", "angle", "length", "half_width")}
    empty["logits"] = np.zeros((0, 2), np.float32)
    empty["palette"] = np.zeros((2, 3), np.float32)
    out, blocked = api.compensate(api.to_device(empty))
    assert blocked.numel() == 0
    one = dense_program(1, 3)
    out, blocked = api.compensate(api.to_device(one), endpoint=True)
    assert int(blocked[0]) == 0
    assert abs(float(out["cx"][0]) - float(one["cx"][0])) <= 1e-7
    # drops only: the endpoint variant keeps a drop a drop
    drops = synth.make_program(40, 4, 7, synth.StrokeDist(p_drop=1.0))
    drops["half_width"] = drops["half_width"] * 3
    check(orc, drops, True, False, "drops")
    out, _ = api.compensate(api.to_device(drops), endpoint=True)
    assert float(out["length"].abs().max()) <= 1e-7


SPARSE = synth.StrokeDist(p_drop=0.3, len_lo=0.0, len_hi=0.04, r_lo=0.001, r_hi=0.008)


@pytest.mark.parametrize("endpoint", [False, True])
@pytest.mark.parametrize("skip", [False, True])
def test_sparse_2000_end_to_end(orc, endpoint, skip):
    """2000 strokes small enough that most chains stay clear of later
    footprints (about a fifth still has a blocked step): the oracle's
    compensation of the inert program alone, its clean mask from its own
    chains, and every clean stroke's two ends within 1e-5 of the GPU's."""
    require_gpu()
    prog = synth.make_program(2000, 4, 50, SPARSE, beta=2.0)
    out, blocked = api.compensate(api.to_device(prog), endpoint=endpoint, skip_blocked=skip)
    got = {f: out[f].cpu().numpy().astype(np.float64) for f in FIELDS}
    gb = blocked.cpu().numpy()
    ref, rb, dmin, smin, amp = orc.compensate(prog, endpoint=endpoint, skip=skip,
                                              with_dmin=True, with_amp=True)
    clean = (dmin >= 1e-5) & (smin >= 1e-6) & (amp <= 100)
    n = len(gb)
    ge = ends({**got, "length": got["length"]}, np.arange(n), True)
    re_ = ends({f: np.asarray(ref[f], np.float64) for f in FIELDS}, np.arange(n), True)
    dend = np.max([np.abs(a - b).max(1) for a, b in zip(ge, re_)], axis=0)
    log(f"[compensate sparse 2000 endpoint={endpoint} skip={skip}] blocked "
        f"{int((rb > 0).sum())}; clean {clean.mean():.4f}; clean ends max |d| "
        f"{dend[clean].max(initial=0):.2e}, median {np.median(dend[clean]):.2e}; "
        f"blocked counts equal on clean {np.array_equal(gb[clean], rb[clean])}")
    assert (rb > 0).sum() >= 200
    assert clean.mean() >= 0.9
    assert np.array_equal(gb[clean], rb[clean])
    assert dend[clean].max(initial=0) <= 1e-5
