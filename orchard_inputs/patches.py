"""Synthetic depth patches for the sphere-fit detector (seeded).

A patch is the set of back-projected depth points of one depth-continuous region in a
camera frame (the segmentation itself needs rendering, which is not part of this
repository).  Three kinds, with the shapes of an orchard canopy seen by a wrist camera:

* fruit: the visible cap of a sphere, radius U(2.4, 3.5) cm (4.8-7 cm diameter), facing
  the camera, cap half-angle U(45, 80) degrees;
* branch: the camera-facing half of a cylinder of radius U(0.75, 3) cm and length
  U(3, 12) cm in a random direction;
* leaf: a flat ellipse of 8.5 x 5 cm scaled by U(0.5, 1), slightly bent.

Range z ~ U(0.3, 3) m; the number of points follows the pixel footprint of a 75-degree,
640-pixel camera (f = 417 px): about pi (s f / z)^2 / 2 for a patch of size s, clipped
to [8, 4096]; every point gets isotropic N(0, sigma) noise (sigma 0.5 mm by default).
Points are float32 [n_points][3] (camera frame, metres); patches are CSR offsets int32
[n_patch + 1].  Kind codes: 0 fruit, 1 branch, 2 leaf.
"""
from __future__ import annotations

import numpy as np

F_PX = 417.0

# gate of the detector: radius 2-5.8 cm (Sec. "Geometric fruit perception"), RMS fit
# residual at most 2 mm ("millimetric"), at least 8 points
GATE = dict(r_min=0.02, r_max=0.058, rms_max=0.002, min_points=8)


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def make_patches(n_patch: int, seed: int = 6_000_000, mix=(0.6, 0.25, 0.15), noise: float = 5e-4,
                 max_points: int = 4096):
    """Returns (points float32 [N, 3], offsets int32 [n_patch + 1], kind int8 [n_patch],
    truth float64 [n_patch, 4]: centre and radius of the fruit, zeros for other kinds)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kind = rng.choice(3, size=n_patch, p=np.asarray(mix, float) / np.sum(mix)).astype(np.int8)
    z = rng.uniform(0.3, 3.0, n_patch)
    centre = np.stack([rng.uniform(-0.6, 0.6, n_patch) * z, rng.uniform(-0.45, 0.45, n_patch) * z, z], axis=1)
    size = np.where(kind == 0, rng.uniform(0.024, 0.035, n_patch),
                    np.where(kind == 1, rng.uniform(0.0075, 0.03, n_patch), rng.uniform(0.5, 1.0, n_patch)))
    foot = np.where(kind == 0, size, np.where(kind == 1, 0.05, 0.05 * size))
    count = np.clip(np.round(0.5 * np.pi * (foot * F_PX / z) ** 2), 8, max_points).astype(np.int64)
    off = np.zeros(n_patch + 1, np.int64)
    off[1:] = np.cumsum(count)
    N = int(off[-1])
    pid = np.repeat(np.arange(n_patch), count)
    # per-patch frame: third axis toward the camera (fruit), or random (branch, leaf)
    view = -_unit(centre)
    rnd = _unit(rng.normal(size=(n_patch, 3)))
    zax = np.where((kind == 0)[:, None], view, rnd)
    xax = _unit(np.cross(zax, _unit(rng.normal(size=(n_patch, 3)))))
    yax = np.cross(zax, xax)
    u1, u2 = rng.uniform(size=N), rng.uniform(size=N)
    k = kind[pid]
    loc = np.zeros((N, 3))
    # fruit: uniform on the cap around +z
    half = np.deg2rad(rng.uniform(45.0, 80.0, n_patch))[pid]
    cosv = np.cos(half) + (1 - np.cos(half)) * u1
    sinv = np.sqrt(np.maximum(0.0, 1 - cosv ** 2))
    phi = 2 * np.pi * u2
    fr = np.stack([sinv * np.cos(phi), sinv * np.sin(phi), cosv], axis=1) * size[pid, None]
    # branch: half cylinder along x, facing +z
    L = rng.uniform(0.03, 0.12, n_patch)[pid]
    ang = np.pi * (u1 - 0.5)
    r = size[pid] / 2
    br = np.stack([L * (u2 - 0.5), r * np.sin(ang), r * np.cos(ang)], axis=1)
    # leaf: bent ellipse in the xy plane
    rr = np.sqrt(u1)
    lx, ly = 0.0425 * size[pid] * rr * np.cos(phi), 0.025 * size[pid] * rr * np.sin(phi)
    bend = rng.uniform(-3.0, 3.0, n_patch)[pid]
    lf = np.stack([lx, ly, bend * (lx * lx + ly * ly)], axis=1)
    loc = np.where((k == 0)[:, None], fr, np.where((k == 1)[:, None], br, lf))
    pts = centre[pid] + loc[:, 0:1] * xax[pid] + loc[:, 1:2] * yax[pid] + loc[:, 2:3] * zax[pid]
    pts += rng.normal(0.0, noise, pts.shape)
    truth = np.zeros((n_patch, 4))
    truth[kind == 0, :3] = centre[kind == 0]
    truth[kind == 0, 3] = size[kind == 0]
    return pts.astype(np.float32), off.astype(np.int32), kind, truth
