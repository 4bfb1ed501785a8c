"""GPU parity of the forward trace (soft composite and hard labels) with the
FP64 oracle on identical seeded programs."""

import numpy as np
import pytest
import torch

from gpu_util import hard_parity, log, require_gpu
from paper_2609_08722_amd import api, synth

pytestmark = pytest.mark.gpu


def run_both(orc, prog, W, H, tau=1e-3, tau_c=0.0):
    require_gpu()
    opts = api.Opts(W, H, tau=tau, tau_c=tau_c)
    dp = api.to_device(prog)
    soft = api.render(dp, opts, "soft")["rgb"].cpu().numpy().reshape(-1, 3)
    hard = api.render(dp, opts, "hard")
    ref = orc.render(prog, W, H, tau=tau, tau_min=0.7 / W, tau_c=tau_c)
    return soft, hard, ref


def check(orc, prog, W, H, name, tau=1e-3, tau_c=0.0, soft_tol=1e-4):
    soft, hard, ref = run_both(orc, prog, W, H, tau, tau_c)
    err = np.abs(soft - ref["soft"])
    exempt, bad = hard_parity(hard["owner"].cpu().numpy(), hard["label"].cpu().numpy(), ref)
    log(f"[{name}] {W}x{H} N={len(prog['cx'])}: soft max err {err.max():.3e} "
        f"(p99.9 {np.quantile(err, 0.999):.3e}); hard exempt {exempt}, mismatches {bad}")
    assert err.max() <= soft_tol
    assert bad == 0
    rgb_hard = api.render(api.to_device(prog), api.Opts(W, H), "hard")["rgb"].cpu().numpy()
    assert np.array_equal(rgb_hard.reshape(-1, 3)[ref["dmin"] >= 1e-5],
                          ref["hard"][ref["dmin"] >= 1e-5].astype(np.float32))


def test_forward_64x64_n50(orc):
    w = synth.WORKLOADS["fwd64x64_n50"]
    check(orc, synth.workload_program(w), 64, 64, w.name)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_forward_more_seeds(orc, seed):
    check(orc, synth.make_program(50, 8, seed), 64, 64, f"seed{seed}")


def test_forward_relative_width_branch(orc):
    """tau = 0.35: the relaxation width is tau r (the other side of the max)."""
    prog = synth.make_program(60, 8, 7, beta=2.0)
    check(orc, prog, 64, 64, "tau0.35", tau=0.35, tau_c=1.0)


def test_forward_ragged_canvas(orc):
    """Canvas not a multiple of the 16x16 block tile (partial waves)."""
    check(orc, synth.make_program(80, 8, 8), 70, 45, "ragged")


def test_forward_256_n500(orc):
    w = synth.WORKLOADS["adj256x256_n500"]
    check(orc, synth.workload_program(w), 256, 256, w.name, tau_c=w.tau_c)


def test_forward_degenerate_programs(orc):
    # no strokes: background everywhere, no owner
    prog = synth.make_program(0, 4, 0)
    soft, hard, ref = run_both(orc, prog, 32, 16)
    assert np.allclose(soft, prog["palette"][0][None, :], atol=0)
    assert (hard["owner"].cpu().numpy() == -1).all()
    # one stroke, all drops, and a single pixel canvas
    for p, W, H in ((synth.make_program(1, 3, 5), 40, 40),
                    (synth.make_program(40, 4, 6, synth.StrokeDist(p_drop=1.0)), 48, 48),
                    (synth.make_program(30, 4, 9), 1, 1)):
        check(orc, p, W, H, f"degenerate N={len(p['cx'])} {W}x{H}")


def test_forward_deterministic():
    require_gpu()
    w = synth.WORKLOADS["adj256x256_n500"]
    dp = api.to_device(synth.workload_program(w))
    opts = api.Opts(256, 256, tau_c=1.0)
    a = api.render(dp, opts, "both")
    b = api.render(dp, opts, "both")
    assert torch.equal(a["rgb"], b["rgb"]) and torch.equal(a["owner"], b["owner"])


def test_program_value_checks():
    """The Python layer checks the values the library does not read on the
    host: finite arrays, positive half-widths, palette in [0, 1]."""
    require_gpu()
    good = api.to_device(synth.make_program(20, 4, 5))
    api.validate_program(good)
    for field, value in (("half_width", 0.0), ("cx", float("nan")), ("palette", 1.5)):
        bad = {k: v.clone() for k, v in good.items()}
        bad[field].view(-1)[0] = value
        with pytest.raises(ValueError):
            api.validate_program(bad)
        with pytest.raises(ValueError):
            api.FitState(bad, api.Opts(32, 32))
