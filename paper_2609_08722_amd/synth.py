"""Seeded synthetic workloads (stroke programs, targets' programs, arrivals).

This module only draws random numbers: it holds none of the renderer's
arithmetic, so both the FP64 oracle tests and the GPU path consume the very
same arrays. The paper fits photographs of marbled sheets that are not
available here; these seeded programs stand in for them, with the stroke
distributions stated per workload below.

Draw order per program (numpy PCG64, ``default_rng(seed)``): centres [N,2],
angles [N], drop mask [N], lengths [N], half-widths [N], palette [K,3],
palette indices [N]. Logits are ``beta * onehot(index)``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class StrokeDist:
    p_drop: float = 0.3          # probability that L is exactly 0
    len_lo: float = 0.0          # L ~ U(len_lo, len_hi) otherwise
    len_hi: float = 0.1
    r_lo: float = 0.005          # half-width ~ U[r_lo, r_hi]
    r_hi: float = 0.03


DIST_SMALL = StrokeDist()                                        # 50/500-stroke programs
DIST_LARGE = StrokeDist(p_drop=0.0, len_lo=0.0, len_hi=0.08,      # 2000-stroke programs
                        r_lo=0.002, r_hi=0.02)


@dataclass(frozen=True)
class Workload:
    name: str
    width: int
    height: int
    n_strokes: int
    n_palette: int
    dist: StrokeDist
    beta: float                  # logit scale of the one-hot palette choice
    tau: float = 1e-3            # relative relaxation width (Eq. relax)
    tau_c: float = 0.0           # colour temperature; 0 = argmax colours
    eps: float = 1e-3            # floor constant of the implemented map
    ckpt: int = 256              # position checkpoint interval of the adjoint
    seed: int = 0
    target_seed: int | None = None

    @property
    def tau_min(self) -> float:  # floor of the relaxation width: 0.7 pixel
        return 0.7 / self.width

    @property
    def pixels(self) -> int:
        return self.width * self.height


# The workloads this project measures and tests (names state their sizes).
WORKLOADS = {
    "fwd64x64_n50": Workload("fwd64x64_n50", 64, 64, 50, 8, DIST_SMALL, beta=1.0, tau_c=0.0),
    "adj256x256_n500": Workload("adj256x256_n500", 256, 256, 500, 8, DIST_SMALL, beta=2.0,
                                tau_c=1.0, target_seed=1),
    "fit1024x1024_n2000": Workload("fit1024x1024_n2000", 1024, 1024, 2000, 16, DIST_LARGE,
                                   beta=2.0, tau_c=1.0, target_seed=1),
}


# Batched fitting: 8 uneven jobs, two each of these (canvas side, strokes);
# job j draws its initial program from seed 10 + 2j and its target program
# from seed 11 + 2j, with the 2000-stroke distributions and 16 colours.
BATCH_JOBS = ((512, 1000), (512, 1000), (1024, 2000), (1024, 2000), (1536, 3000), (1536, 3000),
              (2048, 4000), (2048, 4000))


def batch_job(j: int):
    side, n = BATCH_JOBS[j]
    w = Workload(f"batch{j}_{side}x{side}_n{n}", side, side, n, 16, DIST_LARGE, beta=2.0,
                 tau_c=1.0, seed=10 + 2 * j, target_seed=11 + 2 * j)
    return w


# Fitting loop (Table hyper: 2000 strokes, 8 colours, 240 steps at 1024^2).
# A program is drawn in free parameters: anchors th_a ~ N(0, 1.2^2), offsets
# th_d ~ N(0, 0.3^2), half-widths th_r ~ N(0, 0.5^2) inside the windows, a
# uniform palette index with logit 2, palette th_P ~ N(0, 1.5^2). The initial
# program uses seed 20, the target program seed 21 (its hard render is the
# target image).
LOOP_FIT = {"width": 1024, "height": 1024, "n": 2000, "k": 8, "steps": 240, "seed": 20,
            "target_seed": 21}


def loop_theta(n: int, k: int, seed: int) -> np.ndarray:
    """Free parameters [th_ax|th_ay|th_dx|th_dy|th_r|th_c|th_P] of a program."""
    rng = np.random.default_rng(seed)
    ta = rng.normal(0.0, 1.2, size=2 * n)
    td = rng.normal(0.0, 0.3, size=2 * n)
    tr = rng.normal(0.0, 0.5, size=n)
    idx = rng.integers(0, k, size=n)
    tc = np.zeros((n, k))
    tc[np.arange(n), idx] = 2.0
    tp = rng.normal(0.0, 1.5, size=3 * k)
    return np.concatenate([ta, td, tr, tc.reshape(-1), tp]).astype(np.float32)


def coupling_coeffs(n: int, seed: int, amp: float = 0.15) -> np.ndarray:
    """Per-stroke coefficients (c_1, c_2, c_3) of the calibrated coupling,
    each U(-amp, amp): every profile stays above 1 - 3 amp (the fitted
    coefficients of the paper are not available)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(n, 3)).astype(np.float32)


def make_program(n: int, k: int, seed: int, dist: StrokeDist = DIST_SMALL,
                 beta: float = 1.0, dtype=np.float32) -> dict:
    """Draw one program of ``n`` capsule strokes over a ``k``-colour palette."""
    rng = np.random.default_rng(seed)
    centres = rng.random((n, 2))
    angles = rng.random(n) * (2.0 * math.pi)
    drop = rng.random(n) < dist.p_drop
    lengths = dist.len_lo + (dist.len_hi - dist.len_lo) * rng.random(n)
    lengths = np.where(drop, 0.0, lengths)
    widths = dist.r_lo + (dist.r_hi - dist.r_lo) * rng.random(n)
    palette = rng.random((k, 3))
    index = rng.integers(0, k, size=n)
    logits = np.zeros((n, k))
    logits[np.arange(n), index] = beta
    return {
        "cx": centres[:, 0].astype(dtype), "cy": centres[:, 1].astype(dtype),
        "angle": angles.astype(dtype), "length": lengths.astype(dtype),
        "half_width": widths.astype(dtype),
        "logits": logits.astype(dtype), "palette": palette.astype(dtype),
        "index": index.astype(np.int32),
    }


def workload_program(w: Workload, seed: int | None = None) -> dict:
    return make_program(w.n_strokes, w.n_palette, w.seed if seed is None else seed,
                        w.dist, w.beta)


def sample_pixels(n_total: int, n: int, seed: int) -> np.ndarray:
    """Distinct flat pixel indices, sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=min(n, n_total), replace=False)).astype(np.int64)


def random_points(n: int, seed: int, lo: float, hi: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.random((n, 2))


@dataclass
class Request:
    t_arrival: float
    program: int
    soft: bool
    width: int
    n_strokes: int


@dataclass
class ServeMix:
    """Replay requests: Poisson arrivals, log-uniform program length,
    hard/soft 50/50, resolution uniform over a set."""
    rate: float = 200.0
    n_lo: int = 200
    n_hi: int = 4000
    resolutions: tuple = (256, 512, 1024, 2048)
    n_programs: int = 256
    program_seed0: int = 1000
    seed: int = 4
    programs: list = field(default_factory=list)

    def program_lengths(self) -> np.ndarray:
        rng = np.random.default_rng(self.program_seed0 - 1)
        u = rng.random(self.n_programs)
        return np.round(np.exp(math.log(self.n_lo) + u * (math.log(self.n_hi) - math.log(self.n_lo)))
                        ).astype(np.int64)

    def trace(self, duration: float) -> list:
        rng = np.random.default_rng(self.seed)
        lens = self.program_lengths()
        out, t = [], 0.0
        while True:
            t += rng.exponential(1.0 / self.rate)
            if t >= duration:
                break
            j = int(rng.integers(0, self.n_programs))
            out.append(Request(t, j, bool(rng.random() < 0.5),
                               int(self.resolutions[int(rng.integers(0, len(self.resolutions)))]),
                               int(lens[j])))
        return out
