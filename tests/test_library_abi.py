"""CPU checks of the C ABI: the built library loads and exports every entry point
declared in include/orchard.h; descriptor validation errors are reported before any
device work (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from orchard_inputs import assemble, gen_tree, step_constants

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "orchard.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(orchard_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2607_06337_amd.orchard import EXPORTS, LIB_PATH
    assert os.path.exists(LIB_PATH), "liborchard.so not built"
    lib = C.CDLL(LIB_PATH)
    declared = header_functions()
    assert set(declared) == set(EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def _bad(batch_mut, code_expected, **consts):
    from paper_2607_06337_amd import Model, OrchardError
    b = assemble([gen_tree(1, 20, 3)])
    batch_mut(b)
    with pytest.raises(OrchardError) as ei:
        Model(b, step_constants(**consts))
    assert ei.value.code == code_expected, str(ei.value)


def test_create_rejects_invalid_descriptions():
    def parent_after(b): b.seg_parent[5] = 7
    def neg_length(b): b.seg_length[3] = -0.1
    def zero_radius(b): b.seg_radius[0] = 0.0
    def bad_quat(b): b.seg_rest_quat[2] = [1.0, 0.1, 0.0, 0.0]
    def apple_seg(b): b.apple_seg[0] = 99
    _bad(parent_after, 2)
    _bad(neg_length, 2)
    _bad(zero_radius, 2)
    _bad(bad_quat, 2)
    _bad(apple_seg, 2)
    _bad(lambda b: None, 1, dt=0.0)
    _bad(lambda b: None, 1, wrench_fraction=1.5)
    _bad(lambda b: None, 1, event_band=-1e-3)
    _bad(lambda b: None, 1, event_band=float("nan"))


def test_create_rejects_batches_beyond_32_bit_record_offsets():
    # 2^27 + 1 segments or 2^26 + 1 apples: rejected from the offsets alone, before any
    # per-segment array is read (the small arrays passed here are never touched)
    from paper_2607_06337_amd.orchard import Desc, OrchardError, _check, load_library
    L = load_library()
    small_i = np.zeros(16, np.int32)
    small_d = np.zeros(64, np.float64)
    for ns, na in ((2 ** 27 + 1, 0), (10, 2 ** 26 + 1)):
        d = Desc()
        d.n_env = 1
        so = np.array([0, ns], np.int32)
        ao = np.array([0, na], np.int32)
        d.seg_offset, d.apple_offset = so.ctypes.data, ao.ctypes.data
        for name in ("seg_parent", "apple_seg"):
            setattr(d, name, small_i.ctypes.data)
        for name in ("seg_rest_quat", "seg_length", "seg_radius", "seg_density", "seg_youngs", "seg_mor",
                     "apple_hang", "apple_mass", "apple_radius", "apple_detach"):
            setattr(d, name, small_d.ctypes.data)
        d.dt, d.tether_k, d.tension_factor, d.v_cap, d.react_max_factor = 1e-3, 2e3, 1.1, 5.0, 2.0
        d.n_break = d.n_pull = d.n_tension = 5
        d.stiffness_gamma, d.fruit_dof, d.drag_snapped, d.friction_growth = 1.0, 6, 1.0, 1.0
        h = C.c_void_p()
        with pytest.raises(OrchardError) as e:
            _check(L.orchard_model_create(C.byref(d), None, C.byref(h)))
        assert e.value.code == 1 and "too large" in str(e.value) and not h.value


def test_event_record_layout():
    # orchard_event_t: env, kind, id, step, ratio, in_band (24 bytes, ratio at offset 16)
    from paper_2607_06337_amd.orchard import CState, Event
    assert C.sizeof(Event) == 24 and Event.ratio.offset == 16 and Event.in_band.offset == 20
    # orchard_state_t ends with the nullable evt_ratio pointer
    assert CState._fields_[-1][0] == "evt_ratio" and C.sizeof(CState) == 9 * C.sizeof(C.c_void_p)


def test_create_rejects_invalid_mappings():
    from paper_2607_06337_amd import Model, OrchardError
    b = assemble([gen_tree(1, 20, 3)])
    for tun in (dict(threads=96), dict(lds_width=-1), dict(threads=64, lds_width=65), dict(adjoint_ckpt_max=-2),
                dict(wave_width=65), dict(wave_width=-1), dict(big_threads=300), dict(big_threads=1024)):
        with pytest.raises(OrchardError) as ei:
            Model(b, step_constants(), tun)
        assert ei.value.code == 1, (tun, str(ei.value))


def test_autotune_and_graph_reject_bad_arguments():
    from paper_2607_06337_amd import load_library
    from paper_2607_06337_amd.orchard import Tuning
    L = load_library()
    best = Tuning()
    assert L.orchard_autotune(None, None, 0, 0, 1, C.byref(best), None, None) == 1
    assert L.orchard_graph_launch(None, None) == 1
    assert L.orchard_graph_create(None, None, None, None, 5, None) == 1
    L.orchard_graph_destroy(None)


def test_create_rejects_empty_and_null_descriptions():
    # an empty batch and a missing descriptor are argument errors, reported before any
    # device work
    from paper_2607_06337_amd import load_library
    from paper_2607_06337_amd.orchard import _desc
    L = load_library()
    keep = []
    d = _desc(assemble([gen_tree(1, 20, 3)]), step_constants(), keep)
    out = C.c_void_p()
    d.n_env = 0
    assert L.orchard_model_create(C.byref(d), None, C.byref(out)) == 1
    assert not out.value
    assert L.orchard_model_create(None, None, C.byref(out)) == 1
    d.n_env = 1
    assert L.orchard_model_create(C.byref(d), None, None) == 1
    assert L.orchard_last_error()


def test_sphere_fit_rejects_bad_arguments_before_device_work():
    import ctypes as C
    from paper_2607_06337_amd import load_library
    from paper_2607_06337_amd.orchard import SphereGate
    L = load_library()
    good = SphereGate(0.02, 0.058, 0.002, 8)
    bad = SphereGate(0.06, 0.02, 0.002, 8)
    assert L.orchard_sphere_fit(None, None, -1, C.byref(good), None, None) == 1
    assert L.orchard_sphere_fit(None, None, 5, C.byref(good), None, None) == 1
    assert L.orchard_sphere_fit(None, None, 0, C.byref(bad), None, None) == 1
    assert b"gate" in L.orchard_last_error()
    assert L.orchard_sphere_fit(None, None, 0, C.byref(good), None, None) == 0
