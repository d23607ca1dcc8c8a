"""GPU parity of the HIP step against the FP64 oracle (through the C ABI).

Inputs are the seeded synthetic workloads of ``orchard_inputs``; expected values
come only from ``oracle/``.
"""
import numpy as np
import pytest

from orchard_inputs import assemble, chain_tree, gen_tree, make_batch, pull_forces, step_constants
from tests.parity import APPLE_TOL, EPS, TOL, event_ratio_errors, run_parity, stratified_envs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def _report(name, errs, bad, n_band, oev=None):
    worst_q = max(v[0] for v in errs.values())
    worst_qd = max(v[1] for v in errs.values())
    worst_ax = max(v[3] for v in errs.values())
    worst_av = max(v[4] for v in errs.values())
    eq = max(errs, key=lambda e: errs[e][0])
    eqd = max(errs, key=lambda e: errs[e][1])
    kinds = "" if oev is None else " oracle events (break/pull/tension)=%d/%d/%d" % tuple(
        sum(1 for k in oev if k[1] == j) for j in (1, 2, 3))
    print(f"[{name}] envs={len(errs)} worst rel q={worst_q:.3e} (env {eq}) qd={worst_qd:.3e} (env {eqd}, "
          f"{errs[eqd][2]} compared steps) fruit x={worst_ax:.3e} v={worst_av:.3e} event mismatches={len(bad)} "
          f"in-band ids={n_band}{kinds}", flush=True)
    # fruit position state and velocity are gated with the joint state
    assert worst_ax < APPLE_TOL and worst_av < APPLE_TOL, (worst_ax, worst_av)
    return worst_q, worst_qd


def _no_events(gev, oev):
    """A workload below every threshold: the check is that neither side invents an event."""
    assert len(oev) == 0 and len(gev) == 0, (list(oev.items())[:5], list(gev.items())[:5])


def _check_event_ratios(tag, m, st, b, ost, envs, n_gev):
    # the threshold ratio each event records (mu, pi or tau on its step) against the
    # oracle's, within the band width: an event outside the band is decided identically
    # only while both sides' ratios stay that close
    n, worst, flag_bad = event_ratio_errors(m, st, b, ost, envs)
    print(f"[{tag}] event ratios: {n} compared, largest difference {worst:.2e}", flush=True)
    assert n >= 0.9 * n_gev and n > 0
    assert worst < EPS
    assert not flag_bad, flag_bad[:5]


def test_single_tree_1000_steps():
    # one 64-segment tree with 8 apples, gravity only, 1000 steps, compared every 10
    b = assemble([gen_tree(0, 64, 8)])
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, step_constants(), 1000, 10)
    wq, wqd = _report("single64", errs, bad, n_band, oev)
    assert wq < TOL and wqd < TOL
    _no_events(gev, oev)


def test_stiffness_proportional_damping():
    # the paper's solver damping Kd = c_d Kp with c_d = 0.1 s instead of the damping-ratio
    # reading; each side derives Kd itself.  Two trees and a chain, 500 steps
    b = assemble([gen_tree(5, 64, 8), gen_tree(6, 150, 20), chain_tree(10, length=0.2, radius=0.02)])
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, step_constants(damping_cd=0.1), 500, 50)
    wq, wqd = _report("damping_cd", errs, bad, n_band, oev)
    assert wq < TOL and wqd < TOL
    _no_events(gev, oev)
    kp, kd = (t.cpu().numpy().astype(np.float64) for t in m.default_params())
    assert np.allclose(kd, 0.1 * kp, rtol=1e-6, atol=0)


def test_pull_workload_all_envs():
    # all 1024 trees on the GPU and on the oracle; pulls on 10 % of apples from step 200,
    # 1000 steps, every env compared every 100 steps
    b = make_batch("pull1024")
    F = pull_forces(b)
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, step_constants(), 1000, 100, aforce_desc=F,
                                                         aforce_from=200)
    wq, wqd = _report("pull1024", errs, bad, n_band, oev)
    assert len(errs) == 1024
    assert wq < TOL and wqd < TOL
    assert not bad, bad[:5]
    # the pulls detach fruit (by pull, and some by stem tension)
    assert sum(1 for k in oev if k[1] == 2) >= 100
    assert len(gev) >= 100
    _check_event_ratios("pull1024", m, st, b, ost, range(b.n_env), len(gev))


def test_uneven_workload_2000_steps_stratified():
    # the full 8192-tree uneven batch in the benchmark's launch configuration, with the
    # in-step random body forces, for the benchmark's 2000 steps; 256 envs stratified by
    # size against the oracle, compared every 250 steps.  The break fraction of the whole
    # batch is reported (the random forces stay below the rupture moments: none breaks)
    from bench import BENCH_TUNING
    b = make_batch("uneven8192")
    envs = stratified_envs(b, 256)
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, step_constants("uneven8192"), 2000, 250, envs=envs,
                                                         tuning=BENCH_TUNING)
    wq, wqd = _report("uneven8192", errs, bad, n_band, oev)
    n_break_all = int((st.evt_step[:m.n_seg] >= 0).sum().item())
    print(f"[uneven8192] break fraction over 2000 steps: {n_break_all} of {m.n_seg} joints "
          f"({n_break_all / m.n_seg:.2e}), sample {sum(1 for k in oev if k[1] == 1)} of "
          f"{sum(b.seg_offset[e + 1] - b.seg_offset[e] for e in envs)}", flush=True)
    assert len(errs) == 256
    assert wq < TOL and wqd < TOL
    _no_events(gev, oev)


def weak_wood_batch(n_env=64, mor_scale=0.2):
    """Trees of the pull workload with the modulus of rupture scaled down, so that their
    own weight, the pulled fruit and the in-step random forces break limbs."""
    b = make_batch("pull1024", env_ids=range(n_env))
    b.seg_mor = b.seg_mor * mor_scale
    return b


def test_breaking_limbs_and_free_hinges():
    # rupture (Eq. break) with the hinge left free and applied forces switched off on the
    # snapped sub-tree: weak wood, random body forces on 5 % of segments per step and 30 %
    # of the fruit pulled from step 100; 400 steps, every env compared every 20 steps
    b = weak_wood_batch()
    c = step_constants(rng_seed=3_000_000, wrench_fraction=0.05, wrench_sigma=5.0)
    F = pull_forces(b, fraction=0.3)
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, c, 400, 20, aforce_desc=F, aforce_from=100)
    wq, wqd = _report("weak-wood", errs, bad, n_band, oev)
    assert wq < TOL and wqd < TOL
    assert not bad, bad[:5]
    breaks = [k for k in oev if k[1] == 1]
    assert len(breaks) >= 50 and sum(1 for k in gev if k[1] == 1) >= 50
    assert sum(1 for k in oev if k[1] in (2, 3)) >= 20
    # broken joints whose sub-tree carries fruit (the reaction stays on a snapped limb)
    # and breaks of limbs below an earlier break (a snapped sub-tree breaking again)
    with_fruit, nested = 0, 0
    for (e, _, j) in breaks:
        s0, s1 = b.seg_offset[e], b.seg_offset[e + 1]
        par = b.seg_parent[s0:s1]
        sub = np.zeros(s1 - s0, bool)
        sub[j] = True
        for i in range(j + 1, s1 - s0):
            sub[i] = sub[i] or (par[i] >= 0 and sub[par[i]])
        a0, a1 = b.apple_offset[e], b.apple_offset[e + 1]
        with_fruit += bool(np.any(sub[b.apple_seg[a0:a1]]))
        i = par[j]
        while i >= 0:
            if (e, 1, int(i)) in oev and oev[(e, 1, int(i))] <= oev[(e, 1, j)]:
                nested += 1
                break
            i = par[i]
    print(f"[weak-wood] breaks {len(breaks)}, with fruit below {with_fruit}, below an earlier break {nested}",
          flush=True)
    assert with_fruit >= 10
    _check_event_ratios("weak-wood", m, st, b, ost, range(b.n_env), len(gev))


def test_row_scale_batch_one_launch():
    # the orchard-row batch in one launch: 64 trees of 5000 segments next to 16384 of 80
    # (the large trees, 310-420 nodes on their widest levels, in the wide-tree bucket beside
    # the small trees' LDS packs); the oracle follows
    # 8 large and 64 small trees over the workload's 1000 steps with breakage enabled
    from bench import BENCH_TUNING
    b = make_batch("row64x16k")
    rng = np.random.default_rng(11)
    envs = list(range(0, 64, 8)) + sorted(int(e) for e in rng.choice(np.arange(64, b.n_env), 64, replace=False))
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, step_constants(), 1000, 100, envs=envs,
                                                         tuning=BENCH_TUNING, threads=8)
    wq, wqd = _report("row-scale", errs, bad, n_band, oev)
    assert wq < TOL and wqd < TOL
    # gravity alone breaks a few joints of the large trees late in the run (two, near steps
    # 770 and 800): identical events outside the band
    assert not bad, bad[:5]
    assert len(oev) >= 1 and sum(1 for k in gev if k[1] == 1) >= 1


def test_renumbered_descriptor_is_bitwise_identical():
    # a depth-first (not breadth-first) parent-before-child numbering of every tree and a
    # reversed env order describe the same batch: the library's own renumbering makes the
    # GPU results bitwise equal, and the oracle agrees with itself to rounding.  (The
    # in-step random forces are keyed by env and segment number, so they stay off here;
    # the pulls are permuted with the fruit.)
    from paper_2607_06337_amd import Model
    from orchard_inputs import make_trees
    from oracle.oracle import Oracle
    from tests.test_oracle_structure_pins import permute_tree
    trees = make_trees("pull1024", env_ids=range(12))
    rng = np.random.default_rng(17)
    perm = [permute_tree(t, rng, keep_sibling_order=True) for t in trees]
    for tp, order, _ in perm:
        depth = np.zeros(tp.n_seg, int)
        for i in range(1, tp.n_seg):
            depth[i] = depth[tp.parent[i]] + 1
        assert np.any(np.diff(depth) < 0)
    b0 = assemble(trees)
    b1 = assemble([p[0] for p in perm][::-1])
    c = step_constants()
    F0 = pull_forces(b0, fraction=0.5)
    F1 = np.concatenate([F0[b0.apple_offset[e]:b0.apple_offset[e + 1]][perm[e][2]] for e in range(12)][::-1])
    out = []
    for b, F in ((b0, F0), (b1, F1)):
        m = Model(b, c)
        st = m.rest_state()
        kp, kd = m.default_params()
        Ft = torch.tensor(m.apple_from_desc(F.astype(np.float32), axis=0), device="cuda")
        m.step(st, kp, kd, 300, aforce=Ft)
        q = m.seg_to_desc(st.q.cpu().numpy())
        ap = m.apple_to_desc(st.apple[0:6].cpu().numpy(), axis=1)
        out.append((b, q, ap, sorted(m.events(st))))
    (_, q0, a0, ev0), (_, q1, a1, ev1) = out
    n_ev = 0
    for e in range(12):
        e1 = 11 - e
        tp, order, aperm = perm[e]
        s0, s1 = b0.seg_offset[e], b0.seg_offset[e + 1]
        r0 = b1.seg_offset[e1]
        assert np.array_equal(q1[r0:r0 + tp.n_seg], q0[s0:s1][order])
        A0, A1 = b0.apple_offset[e], b0.apple_offset[e + 1]
        R0 = b1.apple_offset[e1]
        assert np.array_equal(a1[:, R0:R0 + tp.n_apple], a0[:, A0:A1][:, aperm])
        new_of = np.empty(tp.n_seg, np.int64)
        new_of[order] = np.arange(tp.n_seg)
        inv_a = np.empty(tp.n_apple, np.int64)
        inv_a[aperm] = np.arange(tp.n_apple)
        mine0 = sorted((k, int(new_of[i]) if k == 1 else int(inv_a[i]), s) for (ee, k, i, s) in ev0 if ee == e)
        mine1 = sorted((k, i, s) for (ee, k, i, s) in ev1 if ee == e1)
        assert mine0 == mine1
        n_ev += len(mine0)
    assert n_ev > 0
    # the oracle on both numberings, two trees
    o0, o1 = Oracle(b0, c), Oracle(b1, c)
    s0_, s1_ = o0.rest_state(), o1.rest_state()
    o0.rollout(s0_, 200, envs=[0, 1], aforce=F0)
    o1.rollout(s1_, 200, envs=[10, 11], aforce=F1)
    for e in (0, 1):
        tp, order, aperm = perm[e]
        x0 = s0_.q[b0.seg_offset[e]:b0.seg_offset[e + 1]][order]
        r0 = b1.seg_offset[11 - e]
        x1 = s1_.q[r0:r0 + tp.n_seg]
        assert np.max(np.abs(x1 - x0)) <= 1e-12 * np.max(np.abs(x0))


@pytest.mark.parametrize("tuning", [
    dict(threads=64, pack_fill=0.0), dict(threads=128, pack_fill=1.0), dict(threads=256, pack_fill=2.0),
    dict(threads=512, pack_fill=1.0, persistent=1), dict(threads=128, pack_fill=1.0, steps_per_launch=7),
    dict(threads=256, pack_fill=1.0, persistent=1, steps_per_launch=10),
    dict(threads=64, pack_fill=1.0, lds_width=64), dict(threads=256, pack_fill=2.0, lds_width=256),
    dict(threads=128, pack_fill=1.0, lds_width=0), dict(threads=128, pack_fill=1.0, lds_width=48),
    dict(threads=256, pack_fill=1.0, lds_width=0, steps_per_launch=5),
    dict(threads=256, pack_fill=1.0, lds_width=240, steps_per_launch=50),
    dict(threads=128, pack_fill=1.0, lds_width=128, pack_skew=1), dict(threads=64, pack_fill=2.0, lds_width=64, pack_skew=1),
    # size buckets: wave packs for trees whose widest level fits a wavefront, the wide-tree
    # bucket (packs of big_threads work-items on a second stream) for trees wider than lds_width
    dict(threads=256, pack_fill=1.0, lds_width=240, steps_per_launch=50, wave_width=64),
    dict(threads=128, pack_fill=1.0, lds_width=64, wave_width=32, big_threads=256, steps_per_launch=7),
    dict(threads=64, pack_fill=1.0, lds_width=48, wave_width=24, big_threads=512),
    dict(threads=256, pack_fill=1.0, lds_width=96, big_threads=512, pack_skew=1),
    # 512-wide LDS packs for every tree
    dict(threads=512, pack_fill=1.0, lds_width=480, steps_per_launch=50)])
def test_mappings_are_bitwise_identical(tuning):
    # the mapping (workgroup per tree, exchange through LDS or global scratch) changes
    # which workgroup walks a tree and where levels hand data over, never the
    # arithmetic of a node
    from paper_2607_06337_amd import Model
    b = make_batch("uneven8192", env_ids=range(40))
    c = step_constants("uneven8192")
    ref = Model(b, c, dict(threads=128, pack_fill=0.0, lds_width=0))
    alt = Model(b, c, tuning)
    # a bucket that is asked for is used by some trees of this batch
    assert (alt.n_wave_packs > 0) == (tuning.get("wave_width", 0) > 0)
    assert (alt.n_big_packs > 0) == (tuning.get("big_threads", 0) > tuning.get("lds_width", 128))
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


def test_row_batch_mappings_are_bitwise_identical():
    # the orchard-row batch's two benchmark mappings (large trees in the wide-tree bucket
    # beside 240-wide packs, or every tree in 512-wide packs) on 8 large and 64 small trees
    from bench import ROW_CANDIDATES
    from paper_2607_06337_amd import Model
    b = make_batch("row64x16k", env_ids=list(range(0, 64, 8)) + list(range(64, 128)))
    c = step_constants()
    out = []
    for t in ROW_CANDIDATES:
        m = Model(b, c, t)
        assert (m.n_big_packs > 0) == (t["lds_width"] < 460)
        st = m.rest_state()
        kp, kd = m.default_params()
        m.step(st, kp, kd, 120)
        out.append((m.seg_to_desc(st.q.cpu().numpy()), m.seg_to_desc(st.qd.cpu().numpy()),
                    m.apple_to_desc(st.apple.cpu().numpy(), axis=1), sorted(m.events(st, ratios=True))))
    for a, b_ in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b_)
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
    errs, bad, n_band, m, st, ost, gev, oev = run_parity(b, step_constants(), 200, 20, tuning=BENCH_TUNING)
    wq, wqd = _report("chain300", errs, bad, n_band, oev)
    assert wq < TOL and wqd < TOL
    _no_events(gev, oev)


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
