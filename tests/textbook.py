"""Independent textbook geometry used to pin the oracle (numpy, FP64).

Nothing here is shared with the oracle or the GPU path: distances use the
clamped-projection formula, drops use the classical drop map, compositing uses
the Porter-Duff sum of products, and arclength is measured by brute-force
polylines. These are the yardsticks the oracle is checked against.
"""

from __future__ import annotations

import math

import numpy as np


def segment_ends(stroke):
    mx, my, phi, L, r = [float(v) for v in stroke]
    ell = abs(L)
    e = np.array([math.cos(phi), math.sin(phi)])
    m = np.array([mx, my])
    return m - 0.5 * ell * e, m + 0.5 * ell * e


def seg_distance(stroke, pts):
    """Distance from points [n,2] to the stroke's segment (clamped projection)."""
    a, b = segment_ends(stroke)
    p = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    d = b - a
    dd = float(d @ d)
    if dd == 0.0:
        return np.linalg.norm(p - a, axis=1)
    t = np.clip(((p - a) @ d) / dd, 0.0, 1.0)
    return np.linalg.norm(p - (a + t[:, None] * d), axis=1)


def local(stroke, pts):
    """Coordinates (s, h) along / across the stroke direction about its centre."""
    mx, my, phi, L, r = [float(v) for v in stroke]
    p = np.asarray(pts, dtype=np.float64).reshape(-1, 2) - np.array([mx, my])
    c, s = math.cos(phi), math.sin(phi)
    return p[:, 0] * c + p[:, 1] * s, -p[:, 0] * s + p[:, 1] * c


def from_local(stroke, s_, h_):
    mx, my, phi, L, r = [float(v) for v in stroke]
    c, s = math.cos(phi), math.sin(phi)
    return np.stack([mx + s_ * c - h_ * s, my + s_ * s + h_ * c], axis=1)


def drop_backward(centre, r, pts, floor_c=0.0):
    """Classical drop map (Lu 2012): a point at distance d from the centre
    came from distance sqrt(d^2 - r^2); with an optional floor on the area
    difference pi (d^2 - r^2) >= floor_c (the implemented regularisation)."""
    p = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    v = p - np.asarray(centre)
    d = np.linalg.norm(v, axis=1)
    area = math.pi * (d * d - r * r)
    area = np.maximum(area, floor_c)
    new = np.sqrt(area / math.pi)
    return np.asarray(centre) + v * (new / d)[:, None]


def drop_forward(centre, r, pts):
    """Classical drop insertion: c + (p - c) sqrt(1 + r^2 / |p - c|^2)."""
    p = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    v = p - np.asarray(centre)
    d2 = np.sum(v * v, axis=1)
    return np.asarray(centre) + v * np.sqrt(1.0 + r * r / d2)[:, None]


def steiner_area(ell, sig):
    """Area of the parallel set of a segment (textbook: rectangle + disc)."""
    return 2.0 * ell * sig + math.pi * sig * sig


def inverse_area(ell, area):
    """Distance whose parallel set has the given area (quadratic formula)."""
    return (-2.0 * ell + math.sqrt(4.0 * ell * ell + 4.0 * math.pi * area)) / (2.0 * math.pi)


def level_curve_quarter(stroke, sig, n=200001):
    """Brute-force polyline of the first-quadrant quarter of {dist = sig}:
    rays from the centre at polar angles in [0, pi/2] (measured from the
    normal n), each radius found by bisection on the textbook distance."""
    mx, my, phi, L, r = [float(v) for v in stroke]
    beta = np.linspace(0.0, math.pi / 2, n)
    dirs_s, dirs_h = np.sin(beta), np.cos(beta)  # beta = 0 -> along +n
    lo = np.zeros(n)
    hi = np.full(n, abs(L) + sig + 1.0)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        pts = from_local(stroke, mid * dirs_s, mid * dirs_h)
        inside = seg_distance(stroke, pts) < sig
        lo = np.where(inside, mid, lo)
        hi = np.where(inside, hi, mid)
    R = 0.5 * (lo + hi)
    return R * dirs_s, R * dirs_h  # local (s, h) along the quarter


def centred_fraction_bruteforce(stroke, pts, n=200001):
    """Centred arclength fraction of each point on its own level curve,
    folded into the first quadrant, by polyline length."""
    sig = seg_distance(stroke, pts)
    s_, h_ = local(stroke, pts)
    out = []
    for j in range(len(sig)):
        qs, qh = level_curve_quarter(stroke, sig[j], n)
        seg = np.hypot(np.diff(qs), np.diff(qh))
        cum = np.concatenate([[0.0], np.cumsum(seg)])
        total = cum[-1]
        beta_p = math.atan2(abs(s_[j]), abs(h_[j]))
        beta = np.linspace(0.0, math.pi / 2, n)
        arc = np.interp(beta_p, beta, cum)
        out.append((arc / (4.0 * total), 4.0 * total))
    return np.array(out)  # columns: fraction in [0, 1/4], full perimeter


def point_at_fraction_bruteforce(stroke, signs, frac, sig, n=200001):
    """Point of {dist = sig} at centred fraction ``frac`` in the quadrant
    given by signs (sgn s, sgn h), by polyline length."""
    qs, qh = level_curve_quarter(stroke, sig, n)
    seg = np.hypot(np.diff(qs), np.diff(qh))
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    target = frac * 4.0 * cum[-1]
    s_ = np.interp(target, cum, qs)
    h_ = np.interp(target, cum, qh)
    return from_local(stroke, np.array([signs[0] * s_]), np.array([signs[1] * h_]))[0]


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def porter_duff(colours, alphas, background):
    """Eq. (render) written as a sum of products: sum_i c_i a_i prod_{j>i}
    (1 - a_j) + c_0 prod_j (1 - a_j). colours [N,3], alphas [N,P]."""
    N, P = alphas.shape
    out = np.zeros((P, 3))
    trans_above = np.ones(P)
    for i in range(N - 1, -1, -1):
        out += (colours[i][None, :] * (alphas[i] * trans_above)[:, None])
        trans_above = trans_above * (1.0 - alphas[i])
    return out + background[None, :] * trans_above[:, None]


def pixel_centres(width, height):
    jj, ii = np.meshgrid(np.arange(width), np.arange(height))
    return np.stack([(jj.ravel() + 0.5) / width, (ii.ravel() + 0.5) / height], axis=1)
