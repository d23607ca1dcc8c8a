"""The on-device rebuild (orchard_model_rebuild, one thread per world) against the FP64
oracle on the perturbed descriptor, and against create itself.

* Factors (1, 1, 0, 0) reproduce the created model: gains and fruit rest points equal
  create's (FP64 derivation with the same operations on host and device, rounded to
  FP32), and rollouts of the two models are bitwise equal.
* A perturbed rebuild equals a model created from the perturbed descriptor, and its
  gains, fruit rest points and rollouts match the oracle on that descriptor.
* A world with an invalid factor is left as it is and counted.
"""
import time

import numpy as np
import pytest

from orchard_inputs import EXTRAS_ON, geometry_perturbation, make_batch, pull_forces, step_constants
from oracle.oracle import Oracle, perturbed_batch
from tests.parity import TOL, run_parity
from tests.test_gpu_parity import _report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def _params(m):
    return tuple(m.seg_to_desc(t.cpu().numpy()) for t in m.default_params())


def _rollout(m, F, n=150):
    st = m.rest_state()
    kp, kd = m.default_params()
    Ft = torch.tensor(m.apple_from_desc(F.astype(np.float32), axis=0), device="cuda")
    m.step(st, kp, kd, n, aforce=Ft)
    return m.seg_to_desc(st.q.cpu().numpy()), m.apple_to_desc(st.apple[0:6].cpu().numpy(), axis=1), sorted(m.events(st))


CONSTS = dict(rng_seed=3_000_000, wrench_fraction=0.05, **EXTRAS_ON)


def test_zero_perturbation_reproduces_create():
    from paper_2607_06337_amd import Model
    b = make_batch("pull1024", env_ids=range(40))
    c = step_constants(**CONSTS)
    F = pull_forces(b, fraction=0.3)
    ref = Model(b, c)
    m = Model(b, c)
    kp0, kd0 = _params(m)
    rest0 = m.apple_hang_rest.copy()
    m.rebuild(geometry_perturbation(b, strength=0.0))
    kp1, kd1 = _params(m)
    print(f"zero perturbation: kp equal {np.mean(kp0 == kp1):.6f}, kd equal {np.mean(kd0 == kd1):.6f}, "
          f"fruit rest max diff {np.max(np.abs(m.apple_hang_rest - rest0)):.2e}", flush=True)
    assert np.array_equal(kp0, kp1) and np.array_equal(kd0, kd1)
    assert np.array_equal(m.apple_hang_rest, rest0)
    a, bb = _rollout(ref, F), _rollout(m, F)
    assert np.array_equal(a[0], bb[0]) and np.array_equal(a[1], bb[1]) and a[2] == bb[2]


def test_perturbed_rebuild_equals_create_and_matches_the_oracle():
    from paper_2607_06337_amd import Model
    b = make_batch("pull1024", env_ids=range(48))
    c = step_constants(**CONSTS)
    f = geometry_perturbation(b, strength=1.0)
    bp = perturbed_batch(b, f)
    m = Model(b, c)
    t0 = time.perf_counter()
    m.rebuild(f)
    torch.cuda.synchronize()
    print(f"rebuild of {b.n_env} worlds ({b.n_seg} segments): {1e3 * (time.perf_counter() - t0):.2f} ms", flush=True)
    direct = Model(bp, c)
    kp, kd = _params(m)
    kpd, kdd = _params(direct)
    ulp = lambda x, y: np.max(np.abs(x.astype(np.float64) / y - 1))
    print(f"rebuilt vs created: kp {ulp(kp, kpd):.2e} kd {ulp(kd, kdd):.2e} (relative)", flush=True)
    assert ulp(kp, kpd) <= 2.4e-7 and ulp(kd, kdd) <= 2.4e-7
    assert np.max(np.abs(m.apple_hang_rest - direct.apple_hang_rest)) < 1e-12
    d = Oracle(bp, c).derived()
    assert np.max(np.abs(kp / d["kp"] - 1)) < 1e-6 and np.max(np.abs(kd / d["kd"] - 1)) < 1e-6
    assert np.max(np.abs(kp / _params(Model(b, c))[0] - 1)) > 0.1   # the geometry really changed
    # rollouts of the rebuilt model against the oracle on the perturbed descriptor
    F = pull_forces(b, fraction=0.3)
    errs, bad, n_band, *_ = run_parity(bp, c, 300, 30, aforce_desc=F, aforce_from=50, model=m)
    wq, wqd = _report("rebuild", errs, bad, n_band)
    assert wq < TOL and wqd < TOL
    assert not bad


def test_invalid_factors_leave_the_world_unchanged():
    from paper_2607_06337_amd import Model
    b = make_batch("pull1024", env_ids=range(6))
    c = step_constants()
    m = Model(b, c)
    kp0, kd0 = _params(m)
    f = geometry_perturbation(b, strength=1.0)
    s0, s1 = b.seg_offset[3], b.seg_offset[4]
    f[s0 + 2, 0] = 0.0
    rej = torch.zeros(1, dtype=torch.int32, device="cuda")
    m.rebuild(f, rejected=rej)
    assert int(rej.item()) == 1
    kp1, kd1 = _params(m)
    assert np.array_equal(kp1[s0:s1], kp0[s0:s1])
    assert not np.array_equal(np.delete(kp1, np.arange(s0, s1)), np.delete(kp0, np.arange(s0, s1)))
