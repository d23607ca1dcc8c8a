"""Runtime pieces around the step: K-step HIP graphs and the autotuner (through the C ABI)."""
import json

import numpy as np
import pytest

from orchard_inputs import make_batch, step_constants

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def _snapshot(m, st):
    return (st.q.cpu().numpy().copy(), st.qd.cpu().numpy().copy(), st.apple.cpu().numpy().copy(),
            st.evt_step.cpu().numpy().copy(), int(st.step.item()))


@pytest.mark.parametrize("tuning", [dict(threads=128, pack_fill=1.0, lds_width=128),
                                    dict(threads=256, pack_fill=1.0, persistent=1, steps_per_launch=4),
                                    dict(threads=256, pack_fill=1.0, lds_width=240, steps_per_launch=50),
                                    # wave packs beside workgroup packs, and the wide-tree bucket on
                                    # its own stream joined inside the captured graph
                                    dict(threads=128, pack_fill=1.0, lds_width=64, wave_width=32, big_threads=256,
                                         steps_per_launch=10)])
def test_graph_replays_equal_eager_steps(tuning):
    from paper_2607_06337_amd import Model
    b = make_batch("uneven8192", env_ids=range(48))
    c = step_constants("uneven8192")
    m = Model(b, c, tuning)
    K = 25
    g = torch.Generator().manual_seed(7)
    af = (torch.randn(K, m.n_apple, 3, generator=g) * 4.0).cuda().contiguous()
    eager = m.rest_state()
    graphed = m.rest_state()
    kp, kd = m.default_params()
    gr = m.graph(graphed, kp, kd, K, aforce=af)
    for r in range(4):
        m.step(eager, kp, kd, K, aforce=af)
        gr.launch()
        torch.cuda.synchronize()
        # eager work between replays
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        a, bb = _snapshot(m, eager), _snapshot(m, graphed)
        for u, v in zip(a[:4], bb[:4]):
            assert np.array_equal(u, v), f"replay {r}"
        assert a[4] == bb[4] == K * (r + 1)
        del x


def test_autotune_returns_the_fastest_candidate(tmp_path):
    from paper_2607_06337_amd import autotune
    b = make_batch("uneven8192", env_ids=range(64))
    c = step_constants("uneven8192")
    cands = [dict(threads=64, pack_fill=1.0, lds_width=0), dict(threads=128, pack_fill=1.0, lds_width=128),
             dict(threads=256, pack_fill=0.0, lds_width=256)]
    cache = str(tmp_path / "tune.json")
    best, timings = autotune(b, c, cands, n_warm=2, n_steps=5, cache=cache)
    ms = [t[1] for t in timings]
    assert all(x > 0 for x in ms)
    k = int(np.argmin(ms))
    for key, v in cands[k].items():
        assert best[key] == v
    # cached: same answer without timing
    best2, timings2 = autotune(b, c, cands, n_warm=2, n_steps=5, cache=cache)
    assert best2 == best and [t[1] for t in timings2] == ms
    assert len(json.load(open(cache))) == 1


@pytest.mark.parametrize("tuning", [dict(threads=256, pack_fill=1.0, lds_width=240, steps_per_launch=50),
                                    dict(threads=128, pack_fill=1.0, lds_width=0),
                                    dict(threads=64, pack_fill=2.0, lds_width=64, pack_skew=1)])
def test_internal_order_is_a_parent_first_permutation(tuning):
    # the passes rely on the internal order: every segment and apple exactly once, each
    # segment after its parent, and the reported depth the deepest tree's
    from paper_2607_06337_amd import Model
    b = make_batch("uneven8192", env_ids=range(200))
    m = Model(b, step_constants("uneven8192"), tuning)
    assert np.array_equal(np.sort(m.seg_map), np.arange(b.n_seg))
    assert np.array_equal(np.sort(m.apple_map), np.arange(b.n_apple))
    inv = np.empty(b.n_seg, np.int64)
    inv[m.seg_map] = np.arange(b.n_seg)
    env = np.repeat(np.arange(b.n_env), np.diff(b.seg_offset))
    par = b.seg_parent.astype(np.int64)
    has = par >= 0
    g = np.flatnonzero(has)
    assert np.all(inv[b.seg_offset[env[g]] + par[g]] < inv[g])
    depth = np.zeros(b.n_seg, np.int64)
    for k in range(b.n_seg):
        if par[k] >= 0:
            depth[k] = depth[b.seg_offset[env[k]] + par[k]] + 1
    assert m.max_depth == depth.max() + 1
    assert 1 <= m.n_pack <= b.n_env


def test_tips_need_a_model_with_adjoint_support():
    # the tip kernels keep their fields among the adjoint's scratch fields: on a model
    # created without adjoint support both entry points refuse before any device work
    from paper_2607_06337_amd import Model, OrchardError
    b = make_batch("grad512", env_ids=range(2))
    m = Model(b, step_constants())
    st = m.rest_state()
    node = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(OrchardError) as ei:
        m.tips(st.q, node)
    assert ei.value.code == 1
    gq = torch.zeros_like(st.q)
    with pytest.raises(OrchardError) as ei:
        m.tips_backward(st.q, node, torch.ones(4, 3, device="cuda"), gq)
    assert ei.value.code == 1
    assert torch.count_nonzero(gq) == 0


def test_state_without_a_ratio_buffer_steps_identically():
    # evt_ratio is nullable: the same steps with and without it give the same state and
    # events, the events then carrying ratio 0 (and no in-band flag)
    import ctypes as C

    from orchard_inputs import pull_forces
    from paper_2607_06337_amd import Model
    from paper_2607_06337_amd.orchard import Event, load_library
    b = make_batch("pull1024", env_ids=range(16))
    m = Model(b, step_constants())
    kp, kd = m.default_params()
    F = torch.tensor(m.apple_from_desc(pull_forces(b, fraction=0.5).astype(np.float32), axis=0), device="cuda")
    ref = m.rest_state()
    m.step(ref, kp, kd, 300, aforce=F)
    st = m.rest_state()
    st.evt_ratio = None          # the binding passes a null pointer for it
    m.step(st, kp, kd, 300, aforce=F)
    torch.cuda.synchronize()
    for f in ("q", "qd", "apple", "seg_evt", "apple_evt", "evt_step", "env_status", "step"):
        assert torch.equal(getattr(st, f), getattr(ref, f)), f
    with_r = m.events(ref, ratios=True)
    without = m.events(st, ratios=True)
    assert len(with_r) > 0 and [e[:4] for e in with_r] == [e[:4] for e in without]
    assert all(e[4] > 1.0 for e in with_r) and all(e[4] == 0.0 and e[5] == 0 for e in without)
    # the raw record through the C ABI
    cs = st.c()
    assert cs.evt_ratio is None
    buf = (Event * len(without))()
    n = C.c_int32(0)
    assert load_library().orchard_events(m.h, C.byref(cs), buf, len(without), C.byref(n), None) == 0
    assert n.value == len(without) and all(e.ratio == 0.0 for e in buf)
