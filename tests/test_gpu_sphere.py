"""GPU parity of the batched sphere-fit detector (orchard_sphere_fit, through the C ABI)
against the FP64 reference on the same FP32 points.

Bars: the kernel reads the same FP32 points and fits in FP64 (only the summation order
differs), so what remains is the FP32 rounding of its outputs: centre within 5e-7 m (an
ulp of a coordinate of up to 4 m is 4.8e-7 m), radius within two ulps (2.4e-7 relative),
RMS residual within 1e-9 m + 1e-6 relative.  Both sides take the gate decision in FP64; status codes must
agree except where the reference's radius or residual lies within 1e-9 (relative) of a
threshold.
"""
import numpy as np
import pytest

from orchard_inputs.patches import GATE, make_patches
from oracle.sphere import fit_patches

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

TOL_CENTRE, TOL_R_REL, TOL_RMS_ABS, TOL_RMS_REL, BAND = 5e-7, 2.4e-7, 1e-9, 1e-6, 1e-9


def _gpu(points, offsets, gate=GATE):
    from paper_2607_06337_amd import sphere_fit
    p = torch.tensor(points, device="cuda").contiguous()
    o = torch.tensor(offsets, device="cuda").contiguous()
    out = sphere_fit(p, o, gate)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def _compare(name, g, r, gate=GATE):
    assert np.array_equal(g[:, 5], r[:, 5])                    # point counts
    fit = (r[:, 6] != 1) & (r[:, 6] != 2) & (g[:, 6] != 2)
    dpos = np.max(np.abs(g[fit, :3] - r[fit, :3]), initial=0.0)
    dR = np.max(np.abs(g[fit, 3] - r[fit, 3]) / np.maximum(r[fit, 3], 1e-3), initial=0.0)
    drms = np.abs(g[fit, 4] - r[fit, 4])
    near = (np.abs(r[:, 3] / gate["r_min"] - 1) < BAND) | (np.abs(r[:, 3] / gate["r_max"] - 1) < BAND) | \
           (np.abs(r[:, 4] / gate["rms_max"] - 1) < BAND)
    same = (g[:, 6] == r[:, 6]) | near
    print(f"[{name}] patches {len(g)} fitted {fit.sum()} max |d centre| {dpos:.2e} m, |d R| / R {dR:.2e}, max |d rms| "
          f"{np.max(drms, initial=0.0):.2e} m, status equal {np.mean(g[:, 6] == r[:, 6]):.5f} "
          f"(in band {near.sum()}), accepted {np.sum(g[:, 6] == 0)}", flush=True)
    assert dpos < TOL_CENTRE and dR < TOL_R_REL
    assert np.all(drms <= TOL_RMS_ABS + TOL_RMS_REL * r[fit, 4])
    assert np.all(same), np.flatnonzero(~same)[:10]


def test_synthetic_patches_all_compared():
    pts, off, kind, truth = make_patches(4096, seed=11)
    g = _gpu(pts, off)
    r = fit_patches(pts, off, GATE)
    _compare("synthetic4096", g, r)
    fruit = kind == 0
    assert np.mean(g[fruit, 6] == 0) > 0.9


def test_edge_cases():
    rng = np.random.default_rng(5)
    patches = [np.zeros((0, 3)), rng.normal(size=(3, 3)), rng.normal(size=(7, 3))]  # empty, < 4, < 8 points
    # exactly four and exactly eight points of a sphere
    for n in (4, 8, 4096):
        d = rng.normal(size=(n, 3))
        patches.append(np.array([0.1, -0.2, 1.5]) + 0.03 * d / np.linalg.norm(d, axis=1, keepdims=True))
    # a plane (no volume), a line
    patches.append(np.stack([rng.uniform(-0.04, 0.04, 50), rng.uniform(-0.04, 0.04, 50), np.full(50, 2.0)], axis=1))
    patches.append(np.stack([np.linspace(0, 0.1, 30), np.zeros(30), np.full(30, 1.0)], axis=1))
    off = np.concatenate([[0], np.cumsum([len(p) for p in patches])]).astype(np.int32)
    pts = np.concatenate(patches).astype(np.float32)
    g = _gpu(pts, off)
    gate8 = dict(GATE)
    r = fit_patches(pts, off, gate8)
    assert list(g[:3, 6]) == [1, 1, 1] and list(r[:3, 6]) == [1, 1, 1]
    assert g[-2, 6] == 2 and g[-1, 6] == 2
    # four points: the gate's minimum count rejects them; the fits of 8 and 4096 points
    assert g[3, 6] == 1
    for k in (4, 5):
        assert g[k, 6] == 0 and abs(g[k, 3] - 0.03) < 1e-5
        assert np.max(np.abs(g[k, :3] - [0.1, -0.2, 1.5])) < 1e-5
    # with a minimum of four points, four exact sphere points determine it
    g4 = _gpu(pts, off, dict(GATE, min_points=4))
    assert g4[3, 6] == 0 and abs(g4[3, 3] - 0.03) < 1e-4
    # no patches at all
    from paper_2607_06337_amd import sphere_fit
    out = sphere_fit(torch.zeros(0, 3, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda"), GATE)
    assert out.shape == (0, 8)


def test_full_workload_sampled():
    # the benchmark's workload size: 65536 patches (about 26 M points); 1500 patches,
    # spread over the batch, against the reference
    pts, off, kind, truth = make_patches(65536)
    g = _gpu(pts, off)
    pick = np.unique(np.linspace(0, len(off) - 2, 1500).round().astype(int))
    r = fit_patches(pts, off, GATE, patches=pick)
    _compare("workload65536-sample", g[pick], r)
    # properties over the whole batch: counts, and every accepted candidate within the gate
    assert np.array_equal(g[:, 5], np.diff(off))
    acc = g[:, 6] == 0
    assert np.all((g[acc, 3] >= GATE["r_min"]) & (g[acc, 3] <= GATE["r_max"]) & (g[acc, 4] <= GATE["rms_max"]))
    assert np.mean(acc[kind == 0]) > 0.9
