"""Pins of the FP64 sphere-fit reference (Eq. spherefit).

* Points exactly on a sphere give its centre and radius (any cap, any position) with a
  zero residual.
* The fit is the least-squares solution: the normal equations hold at it, and any
  perturbation of (c, b) raises the algebraic residual.
* Translating the points translates the centre and leaves radius and residual alone.
* Points on a plane are rejected as degenerate or out of range; a cylinder section
  fits with a residual far above the gate; noisy fruit caps of the synthetic workload
  are accepted with centres within a few noise levels of the truth.
CPU only.
"""
import numpy as np

from orchard_inputs.patches import GATE, make_patches
from oracle.sphere import fit_patch, fit_patches


def _cap(rng, c, R, n, half):
    cosv = rng.uniform(np.cos(half), 1, n)
    phi = rng.uniform(0, 2 * np.pi, n)
    s = np.sqrt(1 - cosv ** 2)
    return c + R * np.stack([s * np.cos(phi), s * np.sin(phi), cosv], axis=1)


def test_exact_sphere_points():
    rng = np.random.default_rng(1)
    for _ in range(20):
        c, R = rng.uniform(-2, 2, 3), rng.uniform(0.01, 0.1)
        p = _cap(rng, c, R, int(rng.integers(4, 300)), rng.uniform(0.3, np.pi))
        cc, RR, rms = fit_patch(p)
        assert np.max(np.abs(cc - c)) < 1e-9 * max(1, np.abs(c).max()) / R
        assert abs(RR - R) < 1e-9 * max(1, np.abs(c).max())
        assert rms < 1e-9


def test_least_squares_optimality():
    rng = np.random.default_rng(2)
    p = _cap(rng, np.array([0.3, -0.1, 1.2]), 0.03, 200, 1.0) + rng.normal(0, 1e-3, (200, 3))
    c, R, _ = fit_patch(p)
    A = np.hstack([2 * p, np.ones((200, 1))])
    y = np.sum(p * p, axis=1)
    x = np.concatenate([c, [R * R - c @ c]])
    g = A.T @ (A @ x - y)
    assert np.max(np.abs(g)) < 1e-9 * np.max(np.abs(A.T @ y))
    base = np.sum((A @ x - y) ** 2)
    for _ in range(10):
        d = rng.normal(size=4) * 1e-4
        assert np.sum((A @ (x + d) - y) ** 2) > base


def test_translation_equivariance():
    rng = np.random.default_rng(3)
    p = _cap(rng, np.array([0.0, 0.0, 1.0]), 0.03, 150, 1.2) + rng.normal(0, 5e-4, (150, 3))
    c0, R0, r0 = fit_patch(p)
    t = np.array([0.7, -1.1, 0.4])
    c1, R1, r1 = fit_patch(p + t)
    assert np.max(np.abs(c1 - c0 - t)) < 1e-10 and abs(R1 - R0) < 1e-10 and abs(r1 - r0) < 1e-10


def test_plane_and_cylinder_are_rejected():
    rng = np.random.default_rng(4)
    plane = np.stack([rng.uniform(-0.04, 0.04, 100), rng.uniform(-0.04, 0.04, 100), np.full(100, 1.5)], axis=1)
    row = fit_patches(plane, np.array([0, 100]), GATE)[0]
    assert row[6] in (2, 3)
    ang = rng.uniform(-np.pi / 2, np.pi / 2, 300)
    cyl = np.stack([rng.uniform(-0.05, 0.05, 300), 0.012 * np.sin(ang), 1.0 + 0.012 * np.cos(ang)], axis=1)
    row = fit_patches(cyl, np.array([0, 300]), GATE)[0]
    assert row[6] != 0 and (row[6] == 3 or row[4] > GATE["rms_max"])


def test_synthetic_fruit_is_found():
    pts, off, kind, truth = make_patches(400, seed=7)
    rows = fit_patches(pts, off, GATE)
    fruit = kind == 0
    acc = rows[:, 6] == 0
    assert np.mean(acc[fruit]) > 0.9 and np.mean(acc[~fruit]) < 0.2
    err = np.linalg.norm(rows[fruit & acc, :3] - truth[fruit & acc, :3], axis=1)
    assert np.median(err) < 2e-3
