"""The step on the library's fixed scratch array (orchard_step_static_scratch, for callers
that cannot allocate) against orchard_step through the C ABI: bitwise equal results on two
calls in a row, the second on a smaller batch, and a clear error for a model whose scratch
does not fit the array."""
import numpy as np
import pytest

from orchard_inputs import make_batch, pull_forces, step_constants

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def _run(batch, consts, tuning, n_steps, static):
    from paper_2607_06337_amd import Model
    m = Model(batch, consts, tuning)
    st = m.rest_state()
    kp, kd = m.default_params()
    F = torch.tensor(m.apple_from_desc(pull_forces(batch, fraction=0.5).astype(np.float32), axis=0), device="cuda")
    m.step(st, kp, kd, n_steps, aforce=F, static_scratch=static)
    torch.cuda.synchronize()
    return [getattr(st, f).cpu().clone() for f in ("q", "qd", "apple", "seg_evt", "apple_evt", "evt_step",
                                                       "env_status", "step", "evt_ratio")], sorted(m.events(st, ratios=True))


@pytest.mark.parametrize("tuning", [dict(threads=256, pack_fill=1.0, lds_width=240, steps_per_launch=25),
                                    dict(threads=128, pack_fill=1.0, lds_width=0, persistent=1, steps_per_launch=7),
                                    # size buckets: wave packs and the wide-tree bucket's launch
                                    dict(threads=128, pack_fill=1.0, lds_width=64, wave_width=32, big_threads=256,
                                         steps_per_launch=10)])
def test_static_scratch_step_equals_step(tuning):
    c = step_constants(rng_seed=3_000_000, wrench_fraction=0.05)
    big = make_batch("uneven8192", env_ids=range(200))      # ~85 K segments
    small = make_batch("pull1024", env_ids=range(9))         # ~2 K segments
    for batch, steps in ((big, 60), (small, 45)):
        ref, ev_ref = _run(batch, c, tuning, steps, static=False)
        out, ev_out = _run(batch, c, tuning, steps, static=True)
        for a, b in zip(ref, out):
            assert torch.equal(a, b)
        assert ev_ref == ev_out and len(ev_ref) > 0


def test_static_scratch_rejects_a_model_that_does_not_fit():
    from paper_2607_06337_amd import Model, OrchardError
    b = make_batch("pull1024", env_ids=range(600))           # ~150 K segments
    m = Model(b, step_constants())
    st = m.rest_state()
    kp, kd = m.default_params()
    q0 = st.q.clone()
    with pytest.raises(OrchardError) as e:
        m.step(st, kp, kd, 5, static_scratch=True)
    assert e.value.code == 6 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(st.q, q0)  # rejected before any device work
