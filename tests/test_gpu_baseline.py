"""The checkpointed-autograd baseline computes the same soft render and
gradient as the HIP path (it is only used for time / memory comparisons)."""

import numpy as np
import pytest
import torch

from gpu_util import group_errors, log, require_gpu
from paper_2609_08722_amd import api, synth
from paper_2609_08722_amd.baseline_ckpt import soft_render

pytestmark = pytest.mark.gpu


def test_ckpt_baseline_matches_hip_path():
    require_gpu()
    W, H = 48, 48
    prog = synth.make_program(60, 4, 41, beta=2.0)
    dp = api.to_device(prog)
    leaves = {k: v.clone().requires_grad_(True) for k, v in dp.items()}
    R = soft_render(leaves, W, H, tau_c=1.0, every=7)
    w = torch.randn_like(R)
    (R * w).sum().backward()
    out = api.render(dp, api.Opts(W, H, tau_c=1.0, ckpt=16), "soft", tape=True)
    assert torch.max(torch.abs(out["rgb"].reshape(-1, 3) - R.detach())).item() < 1e-4
    g = api.render_backward(dp, out["tape"], w.reshape(H, W, 3))
    for f in api.FIELDS:
        rel, cos = group_errors(leaves[f].grad.cpu().numpy(), g[f].cpu().numpy())
        log(f"[ckpt baseline] {f}: rel {rel:.2e} cos {cos:.6f}")
        assert cos > 0.999, f
