"""ctypes binding of liborchard.so (the C ABI in include/orchard.h).

Argument marshalling only: every step of the dynamics runs in the HIP kernels of
the library.  PyTorch supplies device memory and the current stream.  There is
no fallback: without the built library (or a GPU) the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborchard.so")

OK, ERR_INVALID_ARG, ERR_INVALID_TOPOLOGY, ERR_OOM, ERR_HIP, ERR_NONFINITE, ERR_CAPACITY = range(7)
EVENT_BREAK, EVENT_DETACH_PULL, EVENT_DETACH_TENSION = 1, 2, 3

_P = C.c_void_p


class Desc(C.Structure):
    _fields_ = [("n_env", C.c_int32)] + [(n, _P) for n in (
        "seg_offset", "seg_parent", "seg_rest_quat", "seg_length", "seg_radius", "seg_density",
        "seg_youngs", "seg_mor", "apple_offset", "apple_seg", "apple_hang", "apple_mass",
        "apple_radius", "apple_detach")] + [
        ("dt", C.c_double), ("gravity", C.c_double * 3), ("tether_k", C.c_double),
        ("tether_zeta", C.c_double), ("damping_zeta", C.c_double), ("damping_cd", C.c_double),
        ("tension_factor", C.c_double), ("v_cap", C.c_double), ("react_max_factor", C.c_double),
        ("n_break", C.c_int32), ("n_pull", C.c_int32), ("n_tension", C.c_int32), ("pad0", C.c_int32),
        ("rng_seed", C.c_uint64), ("wrench_fraction", C.c_double), ("wrench_sigma", C.c_double),
        ("stiffness_k0", C.c_double), ("stiffness_gamma", C.c_double), ("fruit_dof", C.c_int32), ("pad1", C.c_int32)] + [
        (k, C.c_double) for k in ("drag_lin", "drag_ang", "drag_snapped", "friction_base", "friction_growth",
                                  "friction_ramp_time", "friction_speed", "fade_speed", "brake_rate",
                                  "event_band")]

# descriptor fields a constants dict may leave out (their "off" values)
_DESC_DEFAULTS = dict(stiffness_k0=0.0, stiffness_gamma=1.0, fruit_dof=6, drag_lin=0.0, drag_ang=0.0, drag_snapped=1.0,
                      friction_base=0.0, friction_growth=1.0, friction_ramp_time=0.0, friction_speed=0.0,
                      fade_speed=0.0, brake_rate=0.0, event_band=0.0)


# the library's defaults (orchard_model_create with a null tuning)
DEFAULT_TUNING = dict(threads=128, pack_fill=1.0, steps_per_launch=1, persistent=0, adjoint_ckpt_max=0, lds_width=128,
                      pack_skew=0, wave_width=0, big_threads=0)


class Tuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("pack_fill", C.c_float), ("steps_per_launch", C.c_int32),
                ("persistent", C.c_int32), ("adjoint_ckpt_max", C.c_int32), ("lds_width", C.c_int32),
                ("pack_skew", C.c_int32), ("wave_width", C.c_int32), ("big_threads", C.c_int32)]


class CAdjoint(C.Structure):
    _fields_ = [("q", _P), ("qd", _P), ("apple_x", _P), ("apple_v", _P)]


class Layout(C.Structure):
    _fields_ = [("n_env", C.c_int64), ("n_seg", C.c_int64), ("n_apple", C.c_int64), ("n_pack", C.c_int32),
                ("max_depth", C.c_int32), ("scratch_bytes", C.c_int64), ("apple_planes", C.c_int32),
                ("n_wave_packs", C.c_int32), ("n_big_packs", C.c_int32), ("pad", C.c_int32)]


class CState(C.Structure):
    _fields_ = [(n, _P) for n in ("q", "qd", "apple", "seg_evt", "apple_evt", "evt_step", "env_status", "step",
                                  "evt_ratio")]


class CParams(C.Structure):
    _fields_ = [("kp", _P), ("kd", _P)]


class CInputs(C.Structure):
    _fields_ = [("body_wrench", _P), ("body_wrench_stride", C.c_int64), ("apple_force", _P),
                ("apple_force_stride", C.c_int64)]


class SphereGate(C.Structure):
    _fields_ = [("r_min", C.c_float), ("r_max", C.c_float), ("rms_max", C.c_float), ("min_points", C.c_int32)]


class Event(C.Structure):
    _fields_ = [("env", C.c_int32), ("kind", C.c_int32), ("id", C.c_int32), ("step", C.c_int32),
                ("ratio", C.c_float), ("in_band", C.c_int32)]


# every exported entry point of include/orchard.h
EXPORTS = ("orchard_model_create", "orchard_model_destroy", "orchard_model_layout", "orchard_model_maps",
           "orchard_model_apple_rest", "orchard_model_rebuild",
           "orchard_default_params", "orchard_state_rest", "orchard_step", "orchard_step_static_scratch",
           "orchard_ckpt_words",
           "orchard_ckpt_load", "orchard_events", "orchard_status", "orchard_last_error", "orchard_step_backward",
           "orchard_tips", "orchard_tips_backward", "orchard_graph_create", "orchard_graph_launch",
           "orchard_graph_destroy", "orchard_autotune", "orchard_sphere_fit")

_lib = None


class OrchardError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"orchard error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH):
    """Load liborchard.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(python paper_2607_06337_amd/build.py)")
    L = C.CDLL(path)
    st = C.c_int
    L.orchard_model_create.argtypes = [C.POINTER(Desc), C.POINTER(Tuning), C.POINTER(_P)]
    L.orchard_model_create.restype = st
    L.orchard_model_destroy.argtypes = [_P]
    L.orchard_model_destroy.restype = None
    L.orchard_model_layout.argtypes = [_P, C.POINTER(Layout)]
    L.orchard_model_layout.restype = st
    L.orchard_model_maps.argtypes = [_P, _P, _P]
    L.orchard_model_maps.restype = st
    L.orchard_model_apple_rest.argtypes = [_P, _P]
    L.orchard_model_apple_rest.restype = st
    L.orchard_model_rebuild.argtypes = [_P, _P, _P, _P]
    L.orchard_model_rebuild.restype = st
    L.orchard_default_params.argtypes = [_P, _P, _P, _P]
    L.orchard_default_params.restype = st
    L.orchard_state_rest.argtypes = [_P, C.POINTER(CState), _P]
    L.orchard_state_rest.restype = st
    L.orchard_step.argtypes = [_P, C.POINTER(CState), C.POINTER(CParams), C.POINTER(CInputs), C.c_int32, _P,
                               C.c_int32, _P]
    L.orchard_step.restype = st
    L.orchard_step_static_scratch.argtypes = L.orchard_step.argtypes
    L.orchard_step_static_scratch.restype = st
    L.orchard_ckpt_words.argtypes = [_P]
    L.orchard_ckpt_words.restype = C.c_int64
    L.orchard_ckpt_load.argtypes = [_P, C.POINTER(CState), _P, _P]
    L.orchard_ckpt_load.restype = st
    L.orchard_events.argtypes = [_P, C.POINTER(CState), C.POINTER(Event), C.c_int32, C.POINTER(C.c_int32), _P]
    L.orchard_events.restype = st
    L.orchard_status.argtypes = [_P, C.POINTER(CState), _P, _P]
    L.orchard_status.restype = st
    L.orchard_step_backward.argtypes = [_P, _P, C.c_int32, C.c_int32, C.POINTER(CParams), C.POINTER(CInputs),
                                        C.POINTER(CAdjoint), _P, _P, _P, _P]
    L.orchard_step_backward.restype = st
    L.orchard_tips.argtypes = [_P, _P, C.c_int32, _P, _P, _P]
    L.orchard_tips.restype = st
    L.orchard_tips_backward.argtypes = [_P, _P, C.c_int32, _P, _P, _P, _P]
    L.orchard_tips_backward.restype = st
    L.orchard_graph_create.argtypes = [_P, C.POINTER(CState), C.POINTER(CParams), C.POINTER(CInputs), C.c_int32,
                                       C.POINTER(_P)]
    L.orchard_graph_create.restype = st
    L.orchard_graph_launch.argtypes = [_P, _P]
    L.orchard_graph_launch.restype = st
    L.orchard_graph_destroy.argtypes = [_P]
    L.orchard_graph_destroy.restype = None
    L.orchard_autotune.argtypes = [C.POINTER(Desc), C.POINTER(Tuning), C.c_int32, C.c_int32, C.c_int32,
                                   C.POINTER(Tuning), _P, _P]
    L.orchard_autotune.restype = st
    L.orchard_sphere_fit.argtypes = [_P, _P, C.c_int32, C.POINTER(SphereGate), _P, _P]
    L.orchard_sphere_fit.restype = st
    L.orchard_last_error.argtypes = []
    L.orchard_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(code: int):
    if code != OK:
        msg = load_library().orchard_last_error().decode()
        raise OrchardError(code, msg)


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def _tptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


@dataclass
class State:
    """Device state of a batch (torch tensors, the model's internal order)."""
    q: "torch.Tensor"          # float32 [n_seg, 2]
    qd: "torch.Tensor"         # float32 [n_seg, 2]
    apple: "torch.Tensor"      # float32 [apple_planes, n_apple] (13, or 6 for a translational fruit)
    seg_evt: "torch.Tensor"    # uint8 [2, n_seg]
    apple_evt: "torch.Tensor"  # uint8 [4, n_apple]
    evt_step: "torch.Tensor"   # int32 [n_seg + n_apple]
    env_status: "torch.Tensor" # int32 [n_env] (bit pattern of the uint32 status words)
    step: "torch.Tensor"       # int64 [1]
    evt_ratio: "torch.Tensor"  # float32 [n_seg + n_apple]: threshold ratio on the event's step

    def c(self) -> CState:
        cs = CState()
        for f in CState._fields_:
            setattr(cs, f[0], _tptr(getattr(self, f[0])))
        # apple arrays may be empty; the library accepts NULL then
        return cs

    def clone(self) -> "State":
        return State(*[getattr(self, f).clone() for f in self.__dataclass_fields__])


def _desc(batch, consts: dict, keep: list) -> Desc:
    """Model descriptor over the batch's host arrays (kept alive in `keep`)."""
    d = Desc()
    d.n_env = batch.n_env
    for name in ("seg_offset", "seg_parent", "apple_offset", "apple_seg"):
        a = np.ascontiguousarray(getattr(batch, name), dtype=np.int32)
        keep.append(a)
        setattr(d, name, _np_ptr(a) if a.size else C.c_void_p(a.ctypes.data))
    for name in ("seg_rest_quat", "seg_length", "seg_radius", "seg_density", "seg_youngs", "seg_mor",
                 "apple_hang", "apple_mass", "apple_radius", "apple_detach"):
        a = np.ascontiguousarray(getattr(batch, name), dtype=np.float64)
        keep.append(a)
        setattr(d, name, C.c_void_p(a.ctypes.data))
    d.dt = consts["dt"]
    for i in range(3):
        d.gravity[i] = consts["gravity"][i]
    for k in ("tether_k", "tether_zeta", "damping_zeta", "damping_cd", "tension_factor", "v_cap",
              "react_max_factor", "wrench_fraction", "wrench_sigma"):
        setattr(d, k, float(consts[k]))
    for k in ("n_break", "n_pull", "n_tension"):
        setattr(d, k, int(consts[k]))
    d.rng_seed = int(consts["rng_seed"])
    for k, v in _DESC_DEFAULTS.items():
        setattr(d, k, type(v)(consts.get(k, v)))
    return d


def _tuning(t: dict) -> Tuning:
    u = dict(DEFAULT_TUNING)
    u.update(t)
    if "lds_width" not in t:
        u["lds_width"] = min(int(u["lds_width"]), int(u["threads"]))
    return Tuning(int(u["threads"]), float(u["pack_fill"]), int(u["steps_per_launch"]), int(u["persistent"]),
                  int(u["adjoint_ckpt_max"]), int(u["lds_width"]), int(u["pack_skew"]), int(u["wave_width"]),
                  int(u["big_threads"]))


def _tuning_dict(t: Tuning) -> dict:
    return {f: (float if f == "pack_fill" else int)(getattr(t, f)) for f, _ in Tuning._fields_}


class Graph:
    """n_steps of Model.step captured once into a HIP graph; launch() replays it."""

    def __init__(self, model: "Model", state: "State", kp, kd, n_steps: int, wrench=None, aforce=None):
        self.model = model  # the graph uses the model's device buffers
        self._keep = (state, kp, kd, wrench, aforce)
        inp = model._inputs(n_steps, wrench, None, aforce, None)
        cs = state.c()
        pr = CParams(_tptr(kp), _tptr(kd))
        h = C.c_void_p()
        _check(load_library().orchard_graph_create(model.h, C.byref(cs), C.byref(pr), C.byref(inp), int(n_steps),
                                                    C.byref(h)))
        self.h = h
        self.n_steps = int(n_steps)

    def launch(self, stream=None):
        _check(load_library().orchard_graph_launch(self.h, _stream(stream)))

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.orchard_graph_destroy(self.h)
            self.h = None


def autotune(batch, consts: dict, candidates: list | None = None, n_warm: int = 5, n_steps: int = 20,
             cache: str | None = None, stream=None):
    """Time candidate kernel mappings on this batch with the library's autotuner and
    return (best tuning dict, [(candidate, ms per step)]).  With `cache` (a JSON file),
    a result stored for the same batch signature and device is returned without timing."""
    import hashlib
    import json
    import torch
    if candidates is None:
        candidates = [dict(threads=t, pack_fill=f, lds_width=w)
                      for t in (64, 128, 256) for f in (1.0, 2.0) for w in (0, t)]
    sig = hashlib.sha256()
    for name in ("seg_offset", "seg_parent", "apple_offset"):
        sig.update(np.ascontiguousarray(getattr(batch, name), dtype=np.int32).tobytes())
    sig.update(json.dumps([candidates, n_warm, n_steps, sorted((k, str(v)) for k, v in consts.items()),
                           torch.cuda.get_device_name()], sort_keys=True).encode())
    key = sig.hexdigest()
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            store = json.load(f)
        if key in store:
            return store[key]["best"], [tuple(x) for x in store[key]["timings"]]
    keep = []
    d = _desc(batch, consts, keep)
    arr = (Tuning * len(candidates))(*[_tuning(c) for c in candidates])
    best = Tuning()
    ms = (C.c_float * len(candidates))()
    _check(load_library().orchard_autotune(C.byref(d), arr, len(candidates), int(n_warm), int(n_steps),
                                           C.byref(best), ms, _stream(stream)))
    best_d = _tuning_dict(best)
    timings = [(dict(c), float(m)) for c, m in zip(candidates, ms)]
    if cache:
        store[key] = {"best": best_d, "timings": timings}
        with open(cache, "w") as f:
            json.dump(store, f, indent=1)
    return best_d, timings


class Model:
    """A batch of trees on the current HIP device."""

    def __init__(self, batch, consts: dict, tuning: dict | None = None):
        L = load_library()
        self.batch = batch
        self._keep = []
        d = _desc(batch, consts, self._keep)
        self.consts = dict(consts)
        tun = None if tuning is None else _tuning(tuning)
        self.tuning = tun
        h = C.c_void_p()
        _check(L.orchard_model_create(C.byref(d), C.byref(tun) if tun is not None else None, C.byref(h)))
        self.h = h
        lay = Layout()
        _check(L.orchard_model_layout(self.h, C.byref(lay)))
        self.n_env, self.n_seg, self.n_apple = int(lay.n_env), int(lay.n_seg), int(lay.n_apple)
        self.apple_planes = int(lay.apple_planes)
        self.n_pack, self.max_depth, self.scratch_bytes = int(lay.n_pack), int(lay.max_depth), int(lay.scratch_bytes)
        self.n_wave_packs, self.n_big_packs = int(lay.n_wave_packs), int(lay.n_big_packs)
        self.seg_map = np.zeros(self.n_seg, np.int32)
        self.apple_map = np.zeros(self.n_apple, np.int32)
        _check(L.orchard_model_maps(self.h, _np_ptr(self.seg_map), _np_ptr(self.apple_map)))
        self.ckpt_words = int(L.orchard_ckpt_words(self.h))
        self.apple_hang_rest = np.zeros((self.n_apple, 3))
        _check(L.orchard_model_apple_rest(self.h, _np_ptr(self.apple_hang_rest)))

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.orchard_model_destroy(self.h)
            self.h = None

    # ---- state -------------------------------------------------------------------------
    def new_state(self) -> State:
        import torch
        dev = torch.device("cuda")
        return State(q=torch.zeros(self.n_seg, 2, device=dev), qd=torch.zeros(self.n_seg, 2, device=dev),
                     apple=torch.zeros(self.apple_planes, self.n_apple, device=dev),
                     seg_evt=torch.zeros(2, self.n_seg, dtype=torch.uint8, device=dev),
                     apple_evt=torch.zeros(4, self.n_apple, dtype=torch.uint8, device=dev),
                     evt_step=torch.full((self.n_seg + self.n_apple,), -1, dtype=torch.int32, device=dev),
                     env_status=torch.zeros(self.n_env, dtype=torch.int32, device=dev),
                     step=torch.zeros(1, dtype=torch.int64, device=dev),
                     evt_ratio=torch.zeros(self.n_seg + self.n_apple, device=dev))

    def rest(self, state: State, stream=None) -> State:
        cs = state.c()
        _check(load_library().orchard_state_rest(self.h, C.byref(cs), _stream(stream)))
        return state

    def rest_state(self) -> State:
        return self.rest(self.new_state())

    def rebuild(self, seg_perturb, rejected=None, stream=None):
        """On-device rebuild of every world's geometry (orchard_model_rebuild).
        seg_perturb: float64 [n_seg, 4] in DESCRIPTOR order (length factor, radius factor,
        bend about x, bend about y), numpy or a device tensor; rejected: optional device
        int32 tensor [1] receiving the number of worlds left unchanged."""
        import torch
        f = torch.as_tensor(seg_perturb, dtype=torch.float64, device="cuda").contiguous()
        assert f.shape == (self.n_seg, 4)
        self._rebuild_factors = f  # kept alive until the stream has used it
        _check(load_library().orchard_model_rebuild(self.h, _tptr(f), _tptr(rejected), _stream(stream)))
        _check(load_library().orchard_model_apple_rest(self.h, _np_ptr(self.apple_hang_rest)))

    def default_params(self, stream=None):
        import torch
        kp = torch.empty(self.n_seg, device="cuda")
        kd = torch.empty(self.n_seg, device="cuda")
        _check(load_library().orchard_default_params(self.h, _tptr(kp), _tptr(kd), _stream(stream)))
        return kp, kd

    # ---- stepping -------------------------------------------------------------------------
    def step(self, state: State, kp, kd, n_steps: int, wrench=None, wrench_stride: int | None = None,
             aforce=None, aforce_stride: int | None = None, ckpt=None, ckpt_every: int = 0, stream=None,
             static_scratch: bool = False):
        """Advance all envs by n_steps.  wrench: float32 [n_seg, 6] (constant) or
        [T, n_seg, 6]; aforce: [n_apple, 3] or [T, n_apple, 3] (internal order).
        static_scratch: run on the library's fixed scratch array (orchard_step_static_scratch)
        instead of the model's own scratch."""
        assert kp.dtype == kd.dtype and kp.numel() == self.n_seg and kd.numel() == self.n_seg
        assert kp.is_contiguous() and kd.is_contiguous()
        inp = CInputs()
        if wrench is not None:
            assert wrench.is_contiguous() and wrench.shape[-2:] == (self.n_seg, 6)
            assert wrench.dim() == 2 or wrench.shape[0] >= n_steps
            inp.body_wrench = _tptr(wrench)
            inp.body_wrench_stride = (0 if wrench.dim() == 2 else self.n_seg * 6) if wrench_stride is None else wrench_stride
        if aforce is not None and self.n_apple:
            assert aforce.is_contiguous() and aforce.shape[-2:] == (self.n_apple, 3)
            assert aforce.dim() == 2 or aforce.shape[0] >= n_steps
            inp.apple_force = _tptr(aforce)
            inp.apple_force_stride = (0 if aforce.dim() == 2 else self.n_apple * 3) if aforce_stride is None else aforce_stride
        if ckpt is not None:
            need = -(-n_steps // ckpt_every) * self.ckpt_words
            assert ckpt.is_contiguous() and ckpt.numel() >= need and ckpt.element_size() == 4
        cs = state.c()
        pr = CParams(_tptr(kp), _tptr(kd))
        fn = load_library().orchard_step_static_scratch if static_scratch else load_library().orchard_step
        _check(fn(self.h, C.byref(cs), C.byref(pr), C.byref(inp), int(n_steps), _tptr(ckpt), int(ckpt_every),
                  _stream(stream)))
        return state

    def graph(self, state: State, kp, kd, n_steps: int, wrench=None, aforce=None) -> Graph:
        """Capture n_steps of step(state, kp, kd, ...) into a replayable HIP graph."""
        return Graph(self, state, kp, kd, n_steps, wrench, aforce)

    def _inputs(self, n_steps, wrench, wrench_stride, aforce, aforce_stride):
        inp = CInputs()
        if wrench is not None:
            assert wrench.is_contiguous() and wrench.shape[-2:] == (self.n_seg, 6)
            assert wrench.dim() == 2 or wrench.shape[0] >= n_steps
            inp.body_wrench = _tptr(wrench)
            inp.body_wrench_stride = (0 if wrench.dim() == 2 else self.n_seg * 6) if wrench_stride is None else wrench_stride
        if aforce is not None and self.n_apple:
            assert aforce.is_contiguous() and aforce.shape[-2:] == (self.n_apple, 3)
            assert aforce.dim() == 2 or aforce.shape[0] >= n_steps
            inp.apple_force = _tptr(aforce)
            inp.apple_force_stride = (0 if aforce.dim() == 2 else self.n_apple * 3) if aforce_stride is None else aforce_stride
        return inp

    def step_backward(self, ckpt, ckpt_every: int, n_steps: int, kp, kd, adj: dict, grad_kp, grad_kd,
                      grad_aforce=None, wrench=None, wrench_stride=None, aforce=None, aforce_stride=None, stream=None):
        """adj: dict of device tensors q, qd [n_seg, 2], ax, av [3, n_apple] holding dL/dS_T;
        overwritten with dL/dS_0.  Gradients accumulate into grad_kp, grad_kd, grad_aforce."""
        inp = self._inputs(n_steps, wrench, wrench_stride, aforce, aforce_stride)
        ca = CAdjoint(_tptr(adj["q"]), _tptr(adj["qd"]), _tptr(adj["ax"]), _tptr(adj["av"]))
        pr = CParams(_tptr(kp), _tptr(kd))
        if grad_aforce is not None:
            assert grad_aforce.is_contiguous() and grad_aforce.numel() >= n_steps * self.n_apple * 3
        _check(load_library().orchard_step_backward(self.h, _tptr(ckpt), int(ckpt_every), int(n_steps), C.byref(pr),
                                                    C.byref(inp), C.byref(ca), _tptr(grad_kp), _tptr(grad_kd),
                                                    _tptr(grad_aforce), _stream(stream)))

    def tips(self, q, node, stream=None):
        import torch
        out = torch.empty(node.numel(), 3, device=q.device)
        _check(load_library().orchard_tips(self.h, _tptr(q), int(node.numel()), _tptr(node), _tptr(out), _stream(stream)))
        return out

    def tips_backward(self, q, node, grad_out, grad_q, stream=None):
        _check(load_library().orchard_tips_backward(self.h, _tptr(q), int(node.numel()), _tptr(node),
                                                    _tptr(grad_out.contiguous()), _tptr(grad_q), _stream(stream)))
        return grad_q

    def ckpt_load(self, state: State, record, stream=None):
        cs = state.c()
        _check(load_library().orchard_ckpt_load(self.h, C.byref(cs), _tptr(record), _stream(stream)))
        return state

    # ---- host queries -------------------------------------------------------------------
    def events(self, state: State, capacity: int = 1 << 16, stream=None, ratios: bool = False):
        """Events as (env, kind, id, step) in descriptor ids; with ratios=True also the
        threshold ratio on the event's step and the in-band flag."""
        L = load_library()
        cs = state.c()
        buf = (Event * max(capacity, 1))()
        n = C.c_int32(0)
        code = L.orchard_events(self.h, C.byref(cs), buf, int(capacity), C.byref(n), _stream(stream))
        if code == ERR_CAPACITY:
            return self.events(state, int(n.value), stream, ratios)
        _check(code)
        if ratios:
            return [(e.env, e.kind, e.id, e.step, e.ratio, e.in_band) for e in buf[: n.value]]
        return [(e.env, e.kind, e.id, e.step) for e in buf[: n.value]]

    def status(self, state: State, stream=None) -> np.ndarray:
        L = load_library()
        cs = state.c()
        out = np.zeros(self.n_env, np.uint32)
        code = L.orchard_status(self.h, C.byref(cs), _np_ptr(out), _stream(stream))
        if code not in (OK, ERR_NONFINITE):
            _check(code)
        return out

    # ---- order conversion (descriptor order <-> internal order) --------------------------
    def seg_to_desc(self, x_internal: np.ndarray) -> np.ndarray:
        out = np.empty_like(x_internal)
        out[self.seg_map] = x_internal
        return out

    def seg_from_desc(self, x_desc: np.ndarray) -> np.ndarray:
        return x_desc[self.seg_map]

    def apple_to_desc(self, x_internal: np.ndarray, axis: int = 0) -> np.ndarray:
        out = np.empty_like(x_internal)
        idx = [slice(None)] * x_internal.ndim
        idx[axis] = self.apple_map
        out[tuple(idx)] = x_internal
        return out

    def apple_from_desc(self, x_desc: np.ndarray, axis: int = 0) -> np.ndarray:
        return np.take(x_desc, self.apple_map, axis=axis)


def sphere_fit(points, offsets, gate: dict, out=None, stream=None):
    """Batched sphere fit (orchard_sphere_fit).  points: device float32 [N, 3]; offsets:
    device int32 [n_patch + 1]; gate: r_min, r_max, rms_max, min_points.  Returns (and
    fills) out: device float32 [n_patch, 8] = centre, radius, rms, count, status, 0."""
    import torch
    assert points.dtype == torch.float32 and points.is_contiguous() and points.shape[-1] == 3
    assert offsets.dtype == torch.int32 and offsets.is_contiguous()
    n_patch = offsets.numel() - 1
    if out is None:
        out = torch.empty(n_patch, 8, dtype=torch.float32, device=points.device)
    g = SphereGate(float(gate["r_min"]), float(gate["r_max"]), float(gate["rms_max"]), int(gate["min_points"]))
    _check(load_library().orchard_sphere_fit(_tptr(points), _tptr(offsets), int(n_patch), C.byref(g), _tptr(out),
                                             _stream(stream)))
    return out
