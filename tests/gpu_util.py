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


def hard_parity(gpu_owner, gpu_label, ref, tol=1e-5):
    """Owners and labels must agree except where the oracle's FP64 trajectory
    passed within tol of a footprint boundary. Returns (exempt, mismatches)."""
    go = np.asarray(gpu_owner).reshape(-1)
    gl = np.asarray(gpu_label).reshape(-1)
    exempt = ref["dmin"] < tol
    bad = ((go != ref["owner"]) | (gl != ref["label"])) & ~exempt
    return int(exempt.sum()), int(bad.sum())


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
