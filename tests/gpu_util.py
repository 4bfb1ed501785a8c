"""Helpers shared by the GPU parity tests (comparison rules only)."""

from __future__ import annotations

import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def log(*a):
    print(*a, flush=True)


# Exempt pixels are a geometric band (trajectories passing within 1e-5 of a
# footprint edge): the oracle's own fraction is 0.02-0.34% on the parity
# workloads (0.12% at 1024^2 x 2000), so more than 0.5% (+2 pixels on tiny
# canvases) means the exemption itself is wrong.
MAX_EXEMPT_FRAC = 0.005


def hard_parity(gpu_owner, gpu_label, ref, tol=1e-5):
    """Owners and labels must agree except where the oracle's FP64 trajectory
    passed within tol of a footprint boundary, and the exempt set must stay a
    thin band. Returns (exempt, mismatches)."""
    go = np.asarray(gpu_owner).reshape(-1)
    gl = np.asarray(gpu_label).reshape(-1)
    exempt = ref["dmin"] < tol
    bad = ((go != ref["owner"]) | (gl != ref["label"])) & ~exempt
    n_ex = int(exempt.sum())
    assert n_ex <= MAX_EXEMPT_FRAC * exempt.size + 2, (n_ex, exempt.size)
    return n_ex, int(bad.sum())


def group_errors(gpu: np.ndarray, ref: np.ndarray):
    """Norm-wise relative error and cosine of one parameter group."""
    g, r = np.asarray(gpu, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    nr = np.linalg.norm(r)
    rel = np.linalg.norm(g - r) / nr if nr > 0 else np.linalg.norm(g)
    cos = float(g @ r / (np.linalg.norm(g) * nr)) if nr > 0 and np.linalg.norm(g) > 0 else 1.0
    return float(rel), cos


def componentwise_ok(gpu, ref, rtol):
    """|gpu - ref| <= rtol (|ref| + 0.01 RMS(ref over the group)), elementwise;
    returns the fraction of components that fail and the worst ratio."""
    g, r = np.asarray(gpu, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    rms = np.sqrt(np.mean(r * r)) if r.size else 0.0
    lim = rtol * (np.abs(r) + 0.01 * rms) + 1e-30
    ratio = np.abs(g - r) / lim
    return float(np.mean(ratio > 1)), float(ratio.max() if ratio.size else 0.0)


GEOM_FIELDS = ("cx", "cy", "angle", "length", "half_width")


def rounding_envelope(prog: dict, grads_of, ref: dict, trials: int = 4, seed: int = 1000,
                      factor: float = 2.0):
    """The oracle's own sensitivity to FP32 rounding: ``factor`` times the
    largest change of each gradient component over ``trials`` FP64 oracle
    runs whose geometric parameters are scaled by (1 + u 2^-24), u ~ U(-1, 1)
    (one rounding, at most half an FP32 ulp). The FP32 kernels round at
    every step, not once, hence the factor. ``grads_of(prog) -> dict`` runs
    the oracle."""
    env = {f: np.zeros_like(np.asarray(ref[f], np.float64)) for f in ref}
    for t in range(trials):
        rng = np.random.default_rng(seed + t)
        q = {k: np.asarray(v, np.float64).copy() for k, v in prog.items() if k != "index"}
        for k in GEOM_FIELDS:
            q[k] = q[k] * (1.0 + 2.0 ** -24 * rng.uniform(-1.0, 1.0, q[k].shape))
        g = grads_of(q)
        for f in env:
            env[f] = np.maximum(env[f], np.abs(np.asarray(g[f], np.float64).reshape(env[f].shape)
                                               - np.asarray(ref[f], np.float64)))
    return {f: factor * e for f, e in env.items()}


def assert_grads(gpu: dict, ref: dict, rtol: float, name: str, groups=None, envelope=None):
    """The gradient parity rule for every group: the norm-wise relative error
    is at most rtol, and every component satisfies
    |gpu - ref| <= rtol (|ref| + 0.01 RMS(ref over the group)), or, where
    ``envelope`` is given, is no larger than the oracle's own change under
    FP32 rounding of the program (rounding_envelope), if that is larger.
    Logs every group before asserting."""
    groups = list(ref) if groups is None else list(groups)
    fails = []
    for f in groups:
        rel, cos = group_errors(gpu[f], ref[f])
        frac, ratio = componentwise_ok(gpu[f], ref[f], rtol)
        msg = f"[{name}] {f:10s} rel {rel:.2e} cos {cos:.9f} fail {frac:.4f} worst {ratio:.2f}"
        bad = frac
        if envelope is not None and f in envelope:
            g = np.asarray(gpu[f], np.float64).ravel()
            r = np.asarray(ref[f], np.float64).ravel()
            e = np.asarray(envelope[f], np.float64).ravel()
            rms = np.sqrt(np.mean(r * r)) if r.size else 0.0
            lim = np.maximum(rtol * (np.abs(r) + 0.01 * rms), e) + 1e-30
            over = np.abs(g - r) / lim
            bad = float(np.mean(over > 1))
            msg += f"; with the rounding envelope fail {bad:.4f} worst {over.max():.2f}"
        log(msg)
        if rel > rtol or bad > 0:
            fails.append((f, rel, bad, ratio))
    assert not fails, f"{name}: {fails}"
