"""Pins of the oracle's closed-form compensation (Sec. "Closed-form
compensation baseline", Lemma obstruction): each stroke of an inert-mark
program is pre-imaged through every later, already compensated stroke,
from the last stroke to the first."""

import numpy as np
import pytest

import textbook as tb
from paper_2609_08722_amd import synth


def ends(prog, i):
    e = np.array([np.cos(prog["angle"][i]), np.sin(prog["angle"][i])])
    m = np.array([prog["cx"][i], prog["cy"][i]])
    return m - 0.5 * prog["length"][i] * e, m + 0.5 * prog["length"][i] * e


def stroke_of(prog, j):
    return np.array([prog["cx"][j], prog["cy"][j], prog["angle"][j], prog["length"][j],
                     prog["half_width"][j]])


def inert_program(n=60, seed=5):
    """Dense enough that many strokes lie in later footprints."""
    prog = synth.make_program(n, 4, seed, synth.DIST_SMALL, beta=2.0, dtype=np.float64)
    prog["length"] = prog["length"] * 2
    prog["half_width"] = prog["half_width"] * 3
    return prog


def test_one_stroke_is_unchanged(orc):
    prog = inert_program(1)
    for endpoint in (False, True):
        out, blocked = orc.compensate(prog, endpoint=endpoint)
        assert blocked[0] == 0
        for f in ("cx", "cy", "length"):
            assert out[f][0] == pytest.approx(prog[f][0], abs=1e-15)


@pytest.mark.parametrize("endpoint", [False, True])
def test_unblocked_points_round_trip(orc, endpoint):
    """Pushing an unblocked stroke's compensated anchor (and end) forward
    through the later compensated strokes, Phi_{i+1} first, lands on the
    inert program's point."""
    prog = inert_program()
    out, blocked = orc.compensate(prog, endpoint=endpoint)
    n = len(prog["cx"])
    assert (blocked == 0).sum() >= 10 and (blocked > 0).sum() >= 3
    for i in np.flatnonzero(blocked == 0):
        pts = np.array(ends(out, i) if endpoint else ends(out, i)[:1])
        want = np.array(ends(prog, i) if endpoint else ends(prog, i)[:1])
        for j in range(i + 1, n):
            pts = orc.phi(stroke_of(out, j), pts)
        assert np.max(np.abs(pts - want)) <= 1e-12, i
    if not endpoint:  # the anchor variant keeps the offset
        assert np.array_equal(out["angle"], prog["angle"])
        assert np.array_equal(out["length"], prog["length"])


def test_compensated_program_draws_unblocked_strokes_in_place(orc):
    """Under R_A the compensated program owns each unblocked stroke's inert
    anchor point with that stroke; a blocked anchor is owned by a later
    stroke (the first footprint the backward path met)."""
    prog = inert_program()
    out, blocked = orc.compensate(prog)
    n = len(prog["cx"])
    anchors = np.array([ends(prog, i)[0] for i in range(n)])
    own = orc.hard_points(out, anchors)
    ok = blocked == 0
    assert np.array_equal(own[ok], np.flatnonzero(ok))
    assert np.all(own[~ok] > np.flatnonzero(~ok))
    # the uncompensated program misplaces strokes that later strokes moved
    own_raw = orc.hard_points(prog, anchors)
    assert np.sum(own_raw[ok] != np.flatnonzero(ok)) >= 3


def two_strokes(anchor_inside):
    """Stroke 0's anchor placed inside (or outside) stroke 1's footprint."""
    y0 = 0.5 if anchor_inside else 0.58
    return {"cx": np.array([0.45, 0.5]), "cy": np.array([y0, 0.5]),
            "angle": np.array([0.0, 0.0]), "length": np.array([0.1, 0.2]),
            "half_width": np.array([0.01, 0.05]), "logits": np.zeros((2, 2)),
            "palette": np.zeros((2, 3))}


@pytest.mark.parametrize("inside", [False, True])
def test_blocked_step_clamp_or_skip(orc, inside):
    prog = two_strokes(inside)
    a0 = ends(prog, 0)[0]
    g1 = stroke_of(prog, 1)
    for skip in (False, True):
        out, blocked = orc.compensate(prog, skip=skip, eps=1e-3)
        assert list(blocked) == [1 if inside else 0, 0]
        a0c = ends(out, 0)[0]
        if inside and skip:  # left where it was
            assert np.allclose(a0c, a0, atol=1e-15)
        elif inside:  # clamped onto stroke 1's segment by the extended psi (floor eps r)
            assert tb.seg_distance(g1, a0c[None])[0] <= 1e-3 * g1[4]
        else:  # a true pre-image, outside the segment
            assert np.allclose(orc.phi(g1, a0c[None])[0], a0, atol=1e-13)


def test_endpoint_variant_moves_both_ends(orc):
    prog = inert_program()
    anc, _ = orc.compensate(prog)
    end, blocked = orc.compensate(prog, endpoint=True)
    # the endpoint variant changes lengths, so the later geometry that each
    # anchor is pre-imaged through, and with it the anchors, differ
    a_anc = np.array([ends(anc, i)[0] for i in range(len(prog["cx"]))])
    a_end = np.array([ends(end, i)[0] for i in range(len(prog["cx"]))])
    assert np.mean(np.abs(end["length"] - prog["length"]) > 1e-9) > 0.2
    assert np.any(np.abs(a_anc - a_end).max(1) > 1e-9)  # later geometry differs


@pytest.mark.parametrize("endpoint", [False, True])
def test_stepwise_mode_reproduces_the_pass(orc, endpoint):
    """Pre-imaging each stroke through given later geometry, when that
    geometry is the pass's own result, is the pass itself."""
    prog = inert_program()
    out, blocked, dmin, smin = orc.compensate(prog, endpoint=endpoint, with_dmin=True)
    again, b2, d2, s2 = orc.compensate(prog, endpoint=endpoint, with_dmin=True, later=out)
    for f in ("cx", "cy", "angle", "length"):
        assert np.array_equal(again[f], out[f])
    assert np.array_equal(blocked, b2) and np.array_equal(dmin, d2) and np.array_equal(smin, s2)
    assert np.all(np.isinf(smin[blocked == 0])) and np.all(smin[blocked > 0] <= out["half_width"].max())
