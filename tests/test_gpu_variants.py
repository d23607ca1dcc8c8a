"""GPU parity of the model variants and extras against the FP64 oracle (through the C ABI).

* per-level exponential stiffness (derived gains and a pulled-fruit rollout);
* translational (3-DoF) fruit: bitwise equal in position, velocity, joints and events to
  the rigid-body fruit on the GPU, and within the bar of the oracle;
* drag, post-break friction ramp, power fade and speed brake on the weak-wood workload
  with random body forces and pulled fruit; each extra moves the oracle's result far
  beyond the bar, so the comparison exercises all of them;
* every mapping gives the same bits with the extras on; the adjoint refuses them.
"""
import numpy as np
import pytest

from orchard_inputs import EXP_STIFFNESS, EXTRAS_ON, make_batch, pull_forces, step_constants
from oracle.oracle import Oracle
from tests.parity import TOL, run_parity
from tests.test_gpu_parity import _report, weak_wood_batch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def test_exponential_stiffness():
    from paper_2607_06337_amd import Model
    b = make_batch("pull1024", env_ids=range(16))
    c = step_constants(**EXP_STIFFNESS)
    m = Model(b, c)
    kp, kd = (m.seg_to_desc(t.cpu().numpy().astype(np.float64)) for t in m.default_params())
    d = Oracle(b, c).derived()
    assert np.max(np.abs(kp / d["kp"] - 1)) < 1e-6 and np.max(np.abs(kd / d["kd"] - 1)) < 1e-6
    assert np.max(d["kp"]) / np.min(d["kp"]) > 1e3   # the stiffness falls level by level
    del m
    F = pull_forces(b, fraction=0.3)
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, c, 500, 50, aforce_desc=F, aforce_from=100)
    wq, wqd = _report("exp-stiffness", errs, bad, n_band, oev)
    assert wq < TOL and wqd < TOL
    assert not bad and len(oev) >= 20


def test_translational_fruit():
    from paper_2607_06337_amd import Model
    b = make_batch("pull1024", env_ids=range(12))
    F = pull_forces(b, fraction=0.3)
    out = []
    for dof in (6, 3):
        c = step_constants(fruit_dof=dof, rng_seed=3_000_000, wrench_fraction=0.05)
        m = Model(b, c)
        st = m.rest_state()
        assert st.apple.shape[0] == (13 if dof == 6 else 6)
        kp, kd = m.default_params()
        Ft = torch.tensor(m.apple_from_desc(F.astype(np.float32), axis=0), device="cuda")
        m.step(st, kp, kd, 300, aforce=Ft)
        out.append((st.q.cpu(), st.qd.cpu(), st.apple[0:6].cpu(), sorted(m.events(st)), m.ckpt_words))
    for a, b_ in zip(out[0][:3], out[1][:3]):
        assert torch.equal(a, b_)
    assert out[0][3] == out[1][3] and len(out[0][3]) > 0
    assert out[0][4] - out[1][4] == 7 * b.n_apple     # seven fewer state floats per fruit
    c3 = step_constants(fruit_dof=3)
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, c3, 400, 40, aforce_desc=F, aforce_from=100)
    wq, wqd = _report("fruit-3dof", errs, bad, n_band, oev)
    assert wq < TOL and wqd < TOL
    assert not bad and len(oev) > 0


def _extras_consts(**over):
    c = dict(EXTRAS_ON, rng_seed=3_000_000, wrench_fraction=0.05, wrench_sigma=5.0)
    c.update(over)
    return step_constants(**c)


def test_extras_on_breaking_limbs():
    # weak wood, random body forces, 30 % of the fruit pulled from step 100: breaks start
    # the friction ramps, snapped limbs get the reduced drag, fast twigs meet the fade and
    # the brake.  First: each extra on its own moves the oracle's joint state by far more
    # than the bar (so the parity below tests all of them)
    b = weak_wood_batch(n_env=48)
    F = pull_forces(b, fraction=0.3)
    envs = list(range(0, 48, 6))

    def oracle_q(c):
        o = Oracle(b, c)
        st = o.rest_state()
        o.rollout(st, 100, envs=envs)
        o.rollout(st, 300, envs=envs, aforce=F)
        return st.q

    base = oracle_q(_extras_consts(**{k: 0.0 for k in EXTRAS_ON}))
    scale = np.max(np.abs(base))
    for name, part in (("drag", dict(drag_lin=1.0, drag_ang=1.0, drag_snapped=0.1)),
                       ("friction", dict(friction_base=0.25, friction_growth=5.0, friction_ramp_time=1.5,
                                         friction_speed=0.05)),
                       ("fade", dict(fade_speed=0.5)), ("brake", dict(brake_rate=50.0))):
        off = {k: 0.0 for k in EXTRAS_ON}
        off.update(part)
        moved = np.max(np.abs(oracle_q(_extras_consts(**off)) - base)) / scale
        print(f"[extras] {name} alone moves the oracle's joint state by {moved:.2e} (relative)", flush=True)
        assert moved > 10 * TOL, name
    c = _extras_consts()
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, c, 400, 20, aforce_desc=F, aforce_from=100)
    wq, wqd = _report("extras", errs, bad, n_band, oev)
    assert wq < TOL and wqd < TOL
    assert not bad, bad[:5]
    assert sum(1 for k in oev if k[1] == 1) >= 50


@pytest.mark.parametrize("tuning", [dict(threads=256, pack_fill=1.0, lds_width=240, steps_per_launch=10),
                                    dict(threads=64, pack_fill=1.0, lds_width=64, persistent=1)])
def test_extras_mappings_are_bitwise_identical(tuning):
    from paper_2607_06337_amd import Model
    b = weak_wood_batch(n_env=30)
    c = _extras_consts(fruit_dof=3, **EXP_STIFFNESS)
    F = pull_forces(b, fraction=0.3)
    res = []
    for t in (dict(threads=128, pack_fill=0.0, lds_width=0), tuning):
        m = Model(b, c, t)
        st = m.rest_state()
        kp, kd = m.default_params()
        Ft = torch.tensor(m.apple_from_desc(F.astype(np.float32), axis=0), device="cuda")
        m.step(st, kp, kd, 250, aforce=Ft)
        res.append((m.seg_to_desc(st.q.cpu().numpy()), m.apple_to_desc(st.apple.cpu().numpy(), axis=1),
                    sorted(m.events(st))))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2] and len(res[0][2]) > 0


def test_adjoint_refuses_the_extras():
    from paper_2607_06337_amd import Model, OrchardError
    b = make_batch("pull1024", env_ids=range(2))
    m = Model(b, _extras_consts(), dict(threads=64, adjoint_ckpt_max=4))
    kp, kd = m.default_params()
    ck = torch.zeros(m.ckpt_words, device="cuda")
    st = m.rest_state()
    m.step(st, kp, kd, 4, ckpt=ck, ckpt_every=4)
    adj = dict(q=torch.zeros(m.n_seg, 2, device="cuda"), qd=torch.zeros(m.n_seg, 2, device="cuda"),
               ax=torch.zeros(3, m.n_apple, device="cuda"), av=torch.zeros(3, m.n_apple, device="cuda"))
    with pytest.raises(OrchardError) as e:
        m.step_backward(ck, 4, 4, kp, kd, adj, torch.zeros_like(kp), torch.zeros_like(kd))
    assert e.value.code == 1 and "does not cover" in str(e.value)
