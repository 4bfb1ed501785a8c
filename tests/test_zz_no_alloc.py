"""The allocation-free render entry point (tbr_render_static) against
tbr_render with a workspace: two calls in a row, the second on a smaller
input, for every mode and the coupled transport; and its stroke limit."""

import numpy as np
import pytest
import torch

from gpu_util import log, require_gpu
from paper_2609_08722_amd import _lib as L
from paper_2609_08722_amd import api, synth

pytestmark = pytest.mark.gpu


def both(prog, opts, mode):
    dp = api.to_device(prog)
    want = api.render(dp, opts, mode)
    torch.cuda.synchronize()
    got = api.render_static(dp, opts, mode)
    torch.cuda.synchronize()
    return got, want


def same(got, want, mode, name):
    keys = ["rgb"] + (["label", "owner"] if mode != "soft" else [])
    for k in keys:
        assert torch.equal(got[k], want[k]), (name, k)
    log(f"[static {name}] {mode}: bitwise equal to tbr_render")


def test_static_render_matches_workspace_render_twice():
    require_gpu()
    big = synth.make_program(3000, 8, 31, beta=2.0)
    small = synth.make_program(200, 5, 32, beta=2.0)
    for mode in ("soft", "hard", "both"):
        o1 = api.Opts(512, 384, tau_c=1.0)
        got, want = both(big, o1, mode)
        same(got, want, mode, "3000 strokes 512x384")
        o2 = api.Opts(97, 61, tau_c=0.0)  # smaller program, ragged canvas
        got, want = both(small, o2, mode)
        same(got, want, mode, "200 strokes 97x61")


def test_static_render_coupled_and_empty():
    require_gpu()
    prog = synth.make_program(500, 8, 33, beta=2.0)
    coup = torch.from_numpy(synth.coupling_coeffs(500, 34)).cuda()
    o = api.Opts(256, 256, tau_c=1.0, coupling=coup)
    got, want = both(prog, o, "both")
    same(got, want, "both", "coupled 500 strokes 256x256")
    for tr in ("inert", "drops16"):
        got, want = both(prog, api.Opts(128, 96, tau_c=1.0, transport=tr), "both")
        same(got, want, "both", f"{tr} 500 strokes 128x96")
    empty = synth.make_program(0, 4, 35, beta=2.0)
    got, want = both(empty, api.Opts(40, 24), "both")
    same(got, want, "both", "empty program 40x24")


def test_static_render_rejects_more_strokes_than_its_scratch():
    require_gpu()
    n = L.TBR_STATIC_MAX_STROKES + 1
    prog = api.to_device(synth.make_program(n, 4, 36))
    with pytest.raises(L.TbrError) as e:
        api.render_static(prog, api.Opts(16, 16), "soft")
    assert e.value.status == L.TBR_E_CAPACITY
    log(f"[static] {n} strokes rejected: {e.value}")
