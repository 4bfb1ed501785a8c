"""GPU checks of tbr_fit_step: its gradient is the replay adjoint of its own
soft render under the L2 seed, its loss is the pixel MSE, its update is Adam
per parameter group (Sec. 5.1), and the loss goes down."""

import numpy as np
import pytest
import torch

from gpu_util import assert_grads, hard_parity, log, require_gpu, rounding_envelope
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


def test_benchmark_workload_fit_step_matches_oracle_on_samples(orc):
    """The benchmarked step at its full size (1024^2 x 2000, checkpoints
    every 256 strokes, the same options and entry point): soft colours, hard
    labels and the fit step's own gradient on 4096 sampled pixels (seed 3)
    against the FP64 oracle. The target equals the step's own soft render
    outside the samples, so the L2 seed vanishes there and the oracle can
    take the gradient over the samples alone."""
    require_gpu()
    w = synth.WORKLOADS["fit1024x1024_n2000"]
    W, H, P = w.width, w.height, w.pixels
    prog = synth.workload_program(w)
    dp = api.to_device(prog)
    opts = api.Opts(W, H, tau=w.tau, tau_c=w.tau_c, eps=w.eps, ckpt=w.ckpt, side_slots=16)
    out = api.render(dp, opts, "soft", tape=True)
    R = out["rgb"].reshape(-1, 3)
    hard = api.render(dp, api.Opts(W, H), "hard")
    pix = synth.sample_pixels(P, 4096, 3)
    ipix = torch.from_numpy(pix).cuda()
    ref = orc.render(prog, W, H, tau=w.tau, tau_c=w.tau_c, eps=w.eps, pixels=pix)

    ferr = np.abs(R[ipix].cpu().numpy() - ref["soft"])
    exempt, bad = hard_parity(hard["owner"].reshape(-1)[ipix].cpu().numpy(),
                              hard["label"].reshape(-1)[ipix].cpu().numpy(), ref)

    # target: the step's render, replaced on the samples by another program's hard colours
    tprog = synth.workload_program(w, seed=w.target_seed)
    tref = orc.render(tprog, W, H, pixels=pix, soft=False)["hard"]
    target = R.clone()
    target[ipix] = torch.from_numpy(tref.astype(np.float32)).cuda()
    opts.side_slots = out["tape"].max_records + 4
    fit = api.FitState(dp, opts, api.Adam(lr_centre=0, lr_angle=0, lr_length=0, lr_width=0,
                                           lr_logits=0, lr_palette=0))
    loss = fit.step(target.reshape(H, W, 3)).item()
    got = {k: v.cpu().numpy() for k, v in api.unpack(fit.grads, fit.n, fit.k).items()}
    diff = R[ipix].cpu().numpy().astype(np.float64) - target[ipix].cpu().numpy()
    seed = 2.0 * diff / (3.0 * P)
    assert abs(loss - float(np.sum(diff ** 2)) / (3.0 * P)) <= 1e-5 * loss
    def grads_of(p):
        r = orc.backward(p, W, H, seed, tau=w.tau, tau_c=w.tau_c, eps=w.eps, pixels=pix)
        out = {f: r["geom"][q] for q, f in enumerate(api.GEOM)}
        out["logits"], out["palette"] = r["logits"], r["palette"]
        return out

    refg = grads_of(prog)
    # on 4096 sampled pixels a component is a few pixels' sum: where one FP32
    # rounding of the program moves the oracle's own component by more than
    # 1e-3 relative, that change is the allowance
    env = rounding_envelope(prog, grads_of, refg)
    log(f"[{w.name}] soft max err {ferr.max():.2e}; hard exempt {exempt} of {len(pix)}, "
        f"mismatches {bad}")
    assert ferr.max() <= 1e-4
    assert bad == 0
    assert_grads(got, refg, 1e-3, w.name, envelope=env)


def test_side_table_overflow_skips_the_update_and_retry_is_exact():
    """A step whose side table overflows leaves parameters and Adam moments
    unchanged and reports the needed capacity; step_checked then repeats it
    with a larger table, bitwise equal to a step that had room from the
    start."""
    prog, opts, target = setup(seed=35)
    prog["half_width"] = prog["half_width"] * 4  # overlapping deposits: several records per pixel
    dp = api.to_device(prog)
    roomy = api.FitState(dp, api.Opts(**{**opts.__dict__, "side_slots": 32}))
    roomy.step(target)
    need = roomy.tape_records()
    assert need >= 2
    tight = api.FitState(dp, api.Opts(**{**opts.__dict__, "side_slots": 1}))
    p0 = tight.params.clone()
    tight.step(target)
    with pytest.raises(api.L.TbrError):
        tight.tape_records()
    assert torch.equal(tight.params, p0)
    assert not torch.any(tight.m) and not torch.any(tight.v)
    tight.step_index -= 1
    tight.grow_side_table(32)
    tight.step(target)
    assert tight.tape_records() == need
    assert torch.equal(tight.params, roomy.params)
    again = api.FitState(dp, api.Opts(**{**opts.__dict__, "side_slots": 1}))
    again.step_checked(target)
    assert again.opts.side_slots >= need
    assert torch.equal(again.params, roomy.params) and torch.equal(again.m, roomy.m)
