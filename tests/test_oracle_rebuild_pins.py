"""Pins of the oracle's per-world geometry perturbation (the definition the on-device
rebuild is checked against).

* The bent rest orientation is the rest rotation followed by rotations about the
  segment's own x then y axis (checked against scipy's rotation composition).
* Factors (1, 1, 0, 0) leave the batch as it is.
* Lengths alone scale a straight chain's tip and every fruit's rest position with the
  chain; radius and length factors scale Kp by f_r^4 / f_l (Eq. beam) and M_max by
  f_r^3 (Eq. break).
CPU only.
"""
import numpy as np
from scipy.spatial.transform import Rotation

from orchard_inputs import assemble, chain_tree, gen_tree, geometry_perturbation, make_batch, step_constants
from oracle.oracle import Oracle, perturbed_batch


def _R(q):
    return Rotation.from_quat(np.concatenate([q[..., 1:], q[..., :1]], axis=-1)).as_matrix()


def test_bend_is_rotation_about_own_axes():
    b = make_batch("pull1024", env_ids=range(3))
    f = geometry_perturbation(b, strength=3.0)
    p = perturbed_batch(b, f)
    ref = _R(b.seg_rest_quat) @ Rotation.from_euler("x", f[:, 2]).as_matrix() @ Rotation.from_euler("y", f[:, 3]).as_matrix()
    assert np.max(np.abs(_R(p.seg_rest_quat) - ref)) < 1e-14
    assert np.max(np.abs(np.linalg.norm(p.seg_rest_quat, axis=1) - 1)) < 1e-15


def test_zero_strength_is_identity():
    b = make_batch("pull1024", env_ids=range(3))
    p = perturbed_batch(b, geometry_perturbation(b, strength=0.0))
    for k in ("seg_length", "seg_radius", "seg_rest_quat", "apple_hang"):
        assert np.array_equal(getattr(p, k), getattr(b, k)), k


def test_length_and_radius_scaling_laws():
    N, l = 6, 0.2
    t = chain_tree(N, length=l, radius=0.01)
    t.apple_seg = np.array([N - 1], np.int32)
    t.apple_hang = np.array([[0.0, 0.0, l]])
    t.apple_mass, t.apple_radius, t.apple_detach = np.array([0.2]), np.array([0.035]), np.array([20.0])
    b = assemble([t])
    fl, fr = 1.3, 0.8
    f = np.tile([fl, fr, 0.0, 0.0], (N, 1))
    p = perturbed_batch(b, f)
    c = step_constants()
    o, op = Oracle(b, c), Oracle(p, c)
    R, pj = o.fk(0, np.zeros(2 * N))
    Rp, pjp = op.fk(0, np.zeros(2 * N))
    tip = pj[-1] + R[-1] @ [0, 0, l]
    tipp = pjp[-1] + Rp[-1] @ [0, 0, l * fl]
    assert np.max(np.abs(tipp - fl * tip)) < 1e-14
    hang = pjp[-1] + Rp[-1] @ p.apple_hang[0]
    assert np.max(np.abs(hang - fl * tip)) < 1e-14       # the fruit moved with its tip
    d, dp = o.derived(), op.derived()
    assert np.allclose(dp["kp"], d["kp"] * fr ** 4 / fl, rtol=1e-14, atol=0)
    assert np.allclose(dp["mmax"], d["mmax"] * fr ** 3, rtol=1e-14, atol=0)
