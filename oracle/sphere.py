"""FP64 reference of the batched sphere-fit detector (Sec. "Geometric fruit perception",
Eq. spherefit).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU baseline, never
by the product path.

Each patch of back-projected depth points p_i is fitted by linear least squares on
2 p_i . c + b = |p_i|^2 with b = R^2 - |c|^2, which gives the centre c and the radius
R = sqrt(b + |c|^2); the fit residual is the RMS of the geometric distances |p_i - c| - R.
A candidate is accepted when it has at least min_points points, its system is not
degenerate, its radius lies in [r_min, r_max] and its residual is at most rms_max.
Status codes: 0 accepted, 1 too few points, 2 degenerate, 3 radius out of range,
4 residual too large.
"""
from __future__ import annotations

import numpy as np


def fit_patch(p: np.ndarray):
    """(centre, radius, rms) of one patch [n, 3] in FP64 (numpy least squares), or None if
    the system is rank-deficient."""
    p = np.asarray(p, np.float64)
    A = np.hstack([2.0 * p, np.ones((len(p), 1))])
    y = np.sum(p * p, axis=1)
    sol, _, rank, _ = np.linalg.lstsq(A, y, rcond=None)
    if rank < 4:
        return None
    c, b = sol[:3], sol[3]
    R = np.sqrt(max(b + c @ c, 0.0))
    rms = np.sqrt(np.mean((np.linalg.norm(p - c, axis=1) - R) ** 2))
    return c, R, rms


def fit_patches(points, offsets, gate: dict, patches=None):
    """Rows (cx, cy, cz, R, rms, n, status) for the listed patches (all by default)."""
    points = np.asarray(points)
    offsets = np.asarray(offsets)
    idx = range(len(offsets) - 1) if patches is None else patches
    out = []
    for k in idx:
        p = points[offsets[k]:offsets[k + 1]]
        n = len(p)
        if n < max(gate["min_points"], 4):
            out.append([0, 0, 0, 0, 0, n, 1])
            continue
        f = fit_patch(p)
        if f is None:
            out.append([0, 0, 0, 0, 0, n, 2])
            continue
        c, R, rms = f
        st = 0 if gate["r_min"] <= R <= gate["r_max"] else 3
        if st == 0 and rms > gate["rms_max"]:
            st = 4
        out.append([*c, R, rms, n, st])
    return np.array(out, np.float64).reshape(-1, 7)
