"""GPU parity of the HIP step against the FP64 oracle (through the C ABI).

Inputs are the seeded synthetic workloads of ``orchard_inputs``; expected values
come only from ``oracle/``.
"""
import numpy as np
import pytest

from orchard_inputs import assemble, chain_tree, gen_tree, make_batch, pull_forces, step_constants
from tests.parity import TOL, run_parity, stratified_envs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def _report(name, errs, bad, n_band):
    worst_q = max(v[0] for v in errs.values())
    worst_qd = max(v[1] for v in errs.values())
    eq = max(errs, key=lambda e: errs[e][0])
    eqd = max(errs, key=lambda e: errs[e][1])
    print(f"[{name}] envs={len(errs)} worst rel q={worst_q:.3e} (env {eq}) qd={worst_qd:.3e} (env {eqd}, "
          f"{errs[eqd][2]} compared steps) event mismatches={len(bad)} in-band ids={n_band}", flush=True)
    return worst_q, worst_qd


def test_single_tree_1000_steps():
    # one 64-segment tree with 8 apples, gravity only, 1000 steps, compared every 10
    b = assemble([gen_tree(0, 64, 8)])
    errs, bad, n_band, *_ = run_parity(b, step_constants(), 1000, 10)
    wq, wqd = _report("single64", errs, bad, n_band)
    assert wq < TOL and wqd < TOL
    assert not bad


def test_stiffness_proportional_damping():
    # the paper's solver damping Kd = c_d Kp with c_d = 0.1 s instead of the damping-ratio
    # reading; each side derives Kd itself.  Two trees and a chain, 500 steps
    b = assemble([gen_tree(5, 64, 8), gen_tree(6, 150, 20), chain_tree(10, length=0.2, radius=0.02)])
    errs, bad, n_band, m, *_ = run_parity(b, step_constants(damping_cd=0.1), 500, 50)
    wq, wqd = _report("damping_cd", errs, bad, n_band)
    assert wq < TOL and wqd < TOL
    assert not bad
    kp, kd = (t.cpu().numpy().astype(np.float64) for t in m.default_params())
    assert np.allclose(kd, 0.1 * kp, rtol=1e-6, atol=0)


def test_pull_workload_full_batch_sampled():
    # all 1024 trees on the GPU; pulls on 10 % of apples from step 200; 40 envs
    # (stratified by size) against the oracle over 1000 steps
    b = make_batch("pull1024")
    F = pull_forces(b)
    envs = stratified_envs(b, 40)
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, step_constants(), 1000, 100, envs=envs, aforce_desc=F,
                                                         aforce_from=200)
    wq, wqd = _report("pull1024", errs, bad, n_band)
    assert wq < TOL and wqd < TOL
    assert not bad, bad[:5]
    assert len(oev) > 0  # the pulls detach fruit


def test_uneven_workload_full_batch_random_wrenches():
    # the full 8192-tree uneven batch in the benchmark's launch configuration, with the
    # in-step random body forces; 24 stratified envs against the oracle for 200 steps
    from bench import BENCH_TUNING
    b = make_batch("uneven8192")
    envs = stratified_envs(b, 24)
    errs, bad, n_band, *_ = run_parity(b, step_constants("uneven8192"), 200, 50, envs=envs, tuning=BENCH_TUNING)
    wq, wqd = _report("uneven8192", errs, bad, n_band)
    assert wq < TOL and wqd < TOL
    assert not bad


def test_row_scale_batch_one_launch():
    # the orchard-row batch in one launch: 64 trees of 5000 segments next to 16384 of 80
    # (wide levels that take the global exchange next to LDS packs); the oracle follows
    # 4 large and 28 small trees over 300 steps with breakage enabled
    from bench import BENCH_TUNING
    b = make_batch("row64x16k")
    rng = np.random.default_rng(11)
    envs = [0, 21, 42, 63] + sorted(int(e) for e in rng.choice(np.arange(64, b.n_env), 28, replace=False))
    errs, bad, n_band, *_ = run_parity(b, step_constants(), 300, 50, envs=envs, tuning=BENCH_TUNING, threads=8)
    wq, wqd = _report("row-scale", errs, bad, n_band)
    assert wq < TOL and wqd < TOL
    assert not bad


@pytest.mark.parametrize("tuning", [
    dict(threads=64, pack_fill=0.0), dict(threads=128, pack_fill=1.0), dict(threads=256, pack_fill=2.0),
    dict(threads=512, pack_fill=1.0, persistent=1), dict(threads=128, pack_fill=1.0, steps_per_launch=7),
    dict(threads=256, pack_fill=1.0, persistent=1, steps_per_launch=10),
    dict(threads=64, pack_fill=1.0, lds_width=64), dict(threads=256, pack_fill=2.0, lds_width=256),
    dict(threads=128, pack_fill=1.0, lds_width=0), dict(threads=128, pack_fill=1.0, lds_width=48),
    dict(threads=256, pack_fill=1.0, lds_width=0, steps_per_launch=5),
    dict(threads=256, pack_fill=1.0, lds_width=240, steps_per_launch=50),
    dict(threads=128, pack_fill=1.0, lds_width=128, pack_skew=1), dict(threads=64, pack_fill=2.0, lds_width=64, pack_skew=1)])
def test_mappings_are_bitwise_identical(tuning):
    # the mapping (workgroup per tree, exchange through LDS or global scratch) changes
    # which workgroup walks a tree and where levels hand data over, never the
    # arithmetic of a node
    from paper_2607_06337_amd import Model
    b = make_batch("uneven8192", env_ids=range(40))
    c = step_constants("uneven8192")
    ref = Model(b, c, dict(threads=128, pack_fill=0.0, lds_width=0))
    alt = Model(b, c, tuning)
    out = []
    for m in (ref, alt):
        st = m.rest_state()
        kp, kd = m.default_params()
        m.step(st, kp, kd, 60)
        out.append((m.seg_to_desc(st.q.cpu().numpy()), m.seg_to_desc(st.qd.cpu().numpy()),
                    m.apple_to_desc(st.apple.cpu().numpy(), axis=1), sorted(m.events(st))))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])
    assert out[0][3] == out[1][3]


def test_batch_independence_bitwise():
    from paper_2607_06337_amd import Model
    from orchard_inputs import make_trees
    trees = make_trees("uneven8192", env_ids=range(30))
    c = step_constants()
    alone = Model(assemble([trees[7]]), c)
    batch = Model(assemble(trees), c)
    res = []
    for m in (alone, batch):
        st = m.rest_state()
        kp, kd = m.default_params()
        m.step(st, kp, kd, 50)
        res.append(m.seg_to_desc(st.q.cpu().numpy()))
    s0 = batch.batch.seg_offset[7]
    assert np.array_equal(res[0], res[1][s0:s0 + trees[7].n_seg])


def test_degenerate_trees():
    # single segment, a straight chain, a tree without apples in an apple-less batch
    b = assemble([chain_tree(1, length=0.2, radius=0.01), chain_tree(12, length=0.1, radius=0.01),
                  gen_tree(3, 40, 0)])
    errs, bad, n_band, *_ = run_parity(b, step_constants(), 300, 30)
    wq, wqd = _report("degenerate", errs, bad, n_band)
    assert wq < TOL and wqd < TOL


def test_deep_horizontal_chain():
    # 300 levels of width one (a 6 m horizontal cantilever of 2 cm segments) next to a
    # small tree: the deepest level chain a pack can have, in the benchmark mapping
    from bench import BENCH_TUNING
    side = (np.cos(np.pi / 4), np.sin(np.pi / 4), 0.0, 0.0)
    b = assemble([chain_tree(300, length=0.02, radius=0.05, root_quat=side), gen_tree(2, 60, 6)])
    errs, bad, n_band, *_ = run_parity(b, step_constants(), 200, 20, tuning=BENCH_TUNING)
    wq, wqd = _report("chain300", errs, bad, n_band)
    assert wq < TOL and wqd < TOL
    assert not bad


def test_nonfinite_env_is_flagged_and_frozen():
    from paper_2607_06337_amd import Model
    b = make_batch("uneven8192", env_ids=range(6))
    m = Model(b, step_constants())
    st = m.rest_state()
    kp, kd = m.default_params()
    m.step(st, kp, kd, 5)
    bad_env = 2
    nodes = np.flatnonzero(m.seg_map == b.seg_offset[bad_env])  # the root of env 2
    q = st.q.clone()
    q[int(nodes[0]), 0] = float("nan")
    st.q.copy_(q)
    m.step(st, kp, kd, 3)
    status = m.status(st)
    assert status[bad_env] & 1 and np.all(np.delete(status, bad_env) == 0)
    frozen = st.q.cpu().numpy()
    m.step(st, kp, kd, 4)
    mine = np.flatnonzero(np.isin(m.seg_map, np.arange(b.seg_offset[bad_env], b.seg_offset[bad_env + 1])))
    assert np.array_equal(st.q.cpu().numpy()[mine], frozen[mine], equal_nan=True)
    others = np.flatnonzero(~np.isin(np.arange(m.n_seg), mine))
    assert np.all(np.isfinite(st.q.cpu().numpy()[others]))


def test_checkpoint_roundtrip_bitwise():
    from paper_2607_06337_amd import Model
    b = make_batch("pull1024", env_ids=range(8))
    m = Model(b, step_constants())
    st = m.rest_state()
    kp, kd = m.default_params()
    F = torch.tensor(m.apple_from_desc(pull_forces(b, fraction=0.5).astype(np.float32), axis=0), device="cuda")
    ck = torch.zeros(3 * m.ckpt_words, dtype=torch.float32, device="cuda")
    m.step(st, kp, kd, 30, aforce=F, ckpt=ck, ckpt_every=10)
    final = st.clone()
    st2 = m.new_state()
    m.ckpt_load(st2, ck[m.ckpt_words:2 * m.ckpt_words])
    assert int(st2.step.item()) == 10
    m.step(st2, kp, kd, 20, aforce=F)
    for f in ("q", "qd", "apple", "seg_evt", "apple_evt", "evt_step", "env_status", "step"):
        assert torch.equal(getattr(final, f), getattr(st2, f)), f
