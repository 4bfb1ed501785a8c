"""GPU checks of tbr_fit_step: its gradient is the replay adjoint of its own
soft render under the L2 seed, its loss is the pixel MSE, its update is Adam
per parameter group (Sec. 5.1), and the loss goes down."""

import numpy as np
import pytest
import torch

from gpu_util import require_gpu
from paper_2609_08722_amd import api, synth

pytestmark = pytest.mark.gpu


def setup(W=64, H=48, n=60, k=6, seed=31):
    require_gpu()
    prog = synth.make_program(n, k, seed, beta=2.0)
    tprog = synth.make_program(n, k, seed + 1)
    opts = api.Opts(W, H, tau_c=1.0, ckpt=16, side_slots=16)
    target = api.render(api.to_device(tprog), api.Opts(W, H), "hard")["rgb"]
    return prog, opts, target


def test_fit_step_gradient_and_loss_match_decomposed_path():
    prog, opts, target = setup()
    W, H = opts.width, opts.height
    dp = api.to_device(prog)
    out = api.render(dp, opts, "soft", tape=True)
    R = out["rgb"]
    sc = torch.tensor(2.0 / (3.0 * W * H), dtype=torch.float32, device=R.device)
    seed = (R - target) * sc
    g = api.render_backward(dp, out["tape"], seed)
    fit = api.FitState(dp, opts, api.Adam(lr_centre=0, lr_angle=0, lr_length=0, lr_width=0,
                                           lr_logits=0, lr_palette=0))
    loss = fit.step(target)
    mse = torch.mean((R.double() - target.double()) ** 2).item()
    assert abs(loss.item() - mse) <= 1e-6 * mse
    got = api.unpack(fit.grads, fit.n, fit.k)
    for f in api.FIELDS:
        assert torch.equal(got[f].reshape(-1), g[f].reshape(-1)), f


def test_adam_update_matches_torch():
    prog, opts, target = setup(seed=33)
    dp = api.to_device(prog)
    adam = api.Adam(r_lo=1e-4, r_hi=1.0, l_max=10.0)
    fit = api.FitState(dp, opts, adam)
    p0 = fit.params.clone()
    # reference: torch.optim.Adam per group, fed the gradients the fit step used
    n, k = fit.n, fit.k
    lrs = [adam.lr_centre] * 2 * n + [adam.lr_angle] * n + [adam.lr_length] * n + \
          [adam.lr_width] * n + [adam.lr_logits] * n * k + [adam.lr_palette] * 3 * k
    ref = [torch.nn.Parameter(p0[j:j + 1].detach().clone()) for j in range(len(lrs))]
    groups = {}
    for j, lr in enumerate(lrs):
        groups.setdefault(lr, []).append(ref[j])
    opt = torch.optim.Adam([{"params": v, "lr": lr} for lr, v in groups.items()],
                           betas=(adam.beta1, adam.beta2), eps=adam.eps)
    for _ in range(3):
        fit.step(target)
        torch.cuda.synchronize()
        gr = fit.grads.clone()
        for j in range(len(lrs)):
            ref[j].grad = gr[j:j + 1].clone()
        opt.step()
        with torch.no_grad():  # the fit step's projections after each update
            for r in ref[4 * n:5 * n]:
                r.clamp_(adam.r_lo, adam.r_hi)
            for r in ref[3 * n:4 * n]:
                r.clamp_(-adam.l_max, adam.l_max)
            for r in ref[len(lrs) - 3 * k:]:
                r.clamp_(0.0, 1.0)
        want = torch.cat([r.detach() for r in ref])
        # compare the accumulated updates; Adam's first steps move every
        # parameter by about lr whatever |g| is, so rounding of g / |g| near
        # eps shows up at the 1e-6 level
        d_got, d_want = fit.params - p0, want - p0
        err = (d_got - d_want).abs().max().item()
        assert err <= 1e-4 * d_want.abs().max().item() + 2e-6, err


def test_loss_decreases():
    prog, opts, target = setup(W=64, H=64, n=80, seed=35)
    fit = api.FitState(api.to_device(prog), opts, api.Adam(r_lo=0.003, r_hi=0.05, l_max=0.12))
    losses = [fit.step(target).item() for _ in range(30)]
    assert losses[-1] < 0.8 * losses[0]
    assert fit.tape_records() >= 0
