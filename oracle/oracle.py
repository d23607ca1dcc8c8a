"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the CPU
baseline of the benchmark, never by the product path.  The oracle and the HIP
path share no code; the only common module is the seeded input generator
``orchard_inputs``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of the same sources (the sanitizer test's)
LIB = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, f) for f in ("oracle.cpp", "oracle_math.hpp", "tape.hpp", "dual.hpp", "adjoint.cpp")]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (host code only)."""
    srcs = [os.path.join(HERE, "oracle.cpp")]
    if os.path.exists(os.path.join(HERE, "adjoint.cpp")):
        srcs.append(os.path.join(HERE, "adjoint.cpp"))
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", LIB + ".tmp", *srcs, "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


# the extras of the step, in the order of the C struct
EXTRAS = ("drag_lin", "drag_ang", "drag_snapped", "friction_base", "friction_growth", "friction_ramp_time",
          "friction_speed", "fade_speed", "brake_rate")


class Globals(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_double * 3), ("tether_k", C.c_double),
                ("tether_zeta", C.c_double), ("damping_zeta", C.c_double), ("damping_cd", C.c_double),
                ("tension_factor", C.c_double), ("v_cap", C.c_double), ("react_max_factor", C.c_double),
                ("event_band", C.c_double), ("n_break", C.c_int32), ("n_pull", C.c_int32),
                ("n_tension", C.c_int32), ("pad", C.c_int32), ("rng_seed", C.c_uint64),
                ("wrench_fraction", C.c_double), ("wrench_sigma", C.c_double),
                ("stiffness_k0", C.c_double), ("stiffness_gamma", C.c_double), ("fruit_dof", C.c_int32),
                ("pad1", C.c_int32)] + [(k, C.c_double) for k in EXTRAS]


_P = C.c_void_p


class Desc(C.Structure):
    _fields_ = [("n_env", C.c_int32)] + [(n, _P) for n in (
        "seg_offset", "seg_parent", "seg_rest_quat", "seg_length", "seg_radius", "seg_density",
        "seg_youngs", "seg_mor", "apple_offset", "apple_seg", "apple_hang", "apple_mass",
        "apple_radius", "apple_detach")]


class IO(C.Structure):
    _fields_ = [(n, _P) for n in ("q", "qd", "ax", "av", "aq", "aw", "broken", "cnt", "det", "cntp",
                                  "cntt", "det_path", "break_step", "det_step", "status", "kp", "kd",
                                  "wrench")] + [("wrench_stride", C.c_int64), ("aforce", _P),
                                                ("aforce_stride", C.c_int64)] + \
        [(n, _P) for n in ("band_jmin", "band_amin", "band_jfirst", "band_afirst", "break_ratio", "det_ratio")]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or any(os.path.exists(s) and os.path.getmtime(s) > os.path.getmtime(LIB) for s in SRC):
            build()
        L = C.CDLL(LIB)
        L.oracle_create.restype = C.c_void_p
        L.oracle_create.argtypes = [C.POINTER(Desc), C.POINTER(Globals)]
        L.oracle_destroy.argtypes = [C.c_void_p]
        L.oracle_derived.argtypes = [C.c_void_p] + [_P] * 7
        L.oracle_fk.argtypes = [C.c_void_p, C.c_int, _P, _P, _P]
        L.oracle_mass_matrix.argtypes = [C.c_void_p, C.c_int, _P, _P]
        L.oracle_inverse_dynamics.argtypes = [C.c_void_p, C.c_int, _P, _P, _P, _P, C.c_int, _P]
        L.oracle_ltdl_solve.argtypes = [C.c_void_p, C.c_int, _P, _P, _P, _P]
        L.oracle_rest_state.argtypes = [C.c_void_p, C.POINTER(IO)]
        L.oracle_rollout.argtypes = [C.c_void_p, C.POINTER(IO), C.c_int, _P, C.c_int64, C.c_int, C.c_int]
        L.oracle_rng_u24.restype = C.c_uint32
        L.oracle_rng_u24.argtypes = [C.c_uint64] * 5
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_splitmix64.argtypes = [C.c_uint64]
        L.oracle_rng_normals.argtypes = [C.c_uint64, C.c_int, C.c_int64, C.c_int, _P]
        L.oracle_ltdl_pivots.argtypes = [C.c_void_p, C.c_int, _P, _P, _P]
        L.oracle_step_dot.argtypes = [C.c_void_p, C.c_int, C.c_int64] + [_P] * 12
        _lib = L
    return _lib


@dataclass
class State:
    """Batch state in descriptor order (float64)."""
    q: np.ndarray
    qd: np.ndarray
    ax: np.ndarray
    av: np.ndarray
    aq: np.ndarray
    aw: np.ndarray
    broken: np.ndarray
    cnt: np.ndarray
    det: np.ndarray
    cntp: np.ndarray
    cntt: np.ndarray
    det_path: np.ndarray
    break_step: np.ndarray
    det_step: np.ndarray
    status: np.ndarray
    break_ratio: np.ndarray  # mu on the step the joint broke (0 before)
    det_ratio: np.ndarray    # pi (pull) or tau (tension) on the step the apple detached
    step: int = 0

    def copy(self) -> "State":
        return State(*[getattr(self, f).copy() for f in self.__dataclass_fields__ if f != "step"], step=self.step)


class Band:
    """Band-rule log: min |ratio - 1| and first in-band step per joint / apple."""

    def __init__(self, n_seg: int, n_apple: int):
        self.jmin = np.full(n_seg, np.inf)
        self.amin = np.full(n_apple, np.inf)
        self.jfirst = np.full(n_seg, -1, np.int32)
        self.afirst = np.full(n_apple, -1, np.int32)


def make_globals(consts: dict) -> Globals:
    g = Globals()
    g.dt = consts["dt"]
    for i in range(3):
        g.gravity[i] = consts["gravity"][i]
    for k in ("tether_k", "tether_zeta", "damping_zeta", "damping_cd", "tension_factor", "v_cap",
              "react_max_factor", "event_band", "wrench_fraction", "wrench_sigma"):
        setattr(g, k, float(consts[k]))
    for k in ("n_break", "n_pull", "n_tension"):
        setattr(g, k, int(consts[k]))
    g.rng_seed = int(consts["rng_seed"])
    g.stiffness_k0 = float(consts.get("stiffness_k0", 0.0))
    g.stiffness_gamma = float(consts.get("stiffness_gamma", 1.0))
    g.fruit_dof = int(consts.get("fruit_dof", 6))
    for k in EXTRAS:
        setattr(g, k, float(consts.get(k, 0.0)))
    return g


class Oracle:
    def __init__(self, batch, consts: dict):
        self.batch = batch
        self.consts = dict(consts)
        self._keep = {}
        d = Desc()
        d.n_env = batch.n_env
        for name in ("seg_offset", "seg_parent", "apple_offset", "apple_seg"):
            a = np.ascontiguousarray(getattr(batch, name), dtype=np.int32)
            self._keep[name] = a
            setattr(d, name, _ptr(a))
        for name in ("seg_rest_quat", "seg_length", "seg_radius", "seg_density", "seg_youngs", "seg_mor",
                     "apple_hang", "apple_mass", "apple_radius", "apple_detach"):
            a = np.ascontiguousarray(getattr(batch, name), dtype=np.float64)
            self._keep[name] = a
            setattr(d, name, _ptr(a))
        self.g = make_globals(consts)
        h = lib().oracle_create(C.byref(d), C.byref(self.g))
        if not h:
            raise ValueError("oracle_create rejected the tree description")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.oracle_destroy(self.h)
            self.h = None

    # ---- derived parameters -------------------------------------------------------------
    def derived(self) -> dict:
        S, A = self.batch.n_seg, self.batch.n_apple
        out = {k: np.zeros(S) for k in ("mass", "It", "Ia", "kp", "kd", "mmax")}
        out["apple_cs"] = np.zeros(A)
        lib().oracle_derived(self.h, *[_ptr(out[k]) for k in ("mass", "It", "Ia", "kp", "kd", "mmax", "apple_cs")])
        return out

    def _S(self, env):
        return int(self.batch.seg_offset[env + 1] - self.batch.seg_offset[env])

    # ---- single-tree kernels (tests) ------------------------------------------------------
    def fk(self, env: int, q):
        S = self._S(env)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(2 * S)
        R = np.zeros((S, 3, 3))
        p = np.zeros((S, 3))
        lib().oracle_fk(self.h, env, _ptr(q), _ptr(R), _ptr(p))
        return R, p

    def mass_matrix(self, env: int, q):
        S = self._S(env)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(2 * S)
        H = np.zeros((2 * S, 2 * S))
        lib().oracle_mass_matrix(self.h, env, _ptr(q), _ptr(H))
        return H

    def inverse_dynamics(self, env, q, qd, qdd, wrench=None, gravity=True):
        S = self._S(env)
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        q, qd, qdd = f(q), f(qd), f(qdd)
        w = None if wrench is None else f(wrench)
        tau = np.zeros(2 * S)
        lib().oracle_inverse_dynamics(self.h, env, _ptr(q), _ptr(qd), _ptr(qdd), _ptr(w), int(gravity), _ptr(tau))
        return tau

    def ltdl_solve(self, env, q, diag, b):
        S = self._S(env)
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64).reshape(2 * S)
        q, diag, b = f(q), f(diag), f(b)
        x = np.zeros(2 * S)
        lib().oracle_ltdl_solve(self.h, env, _ptr(q), _ptr(diag), _ptr(b), _ptr(x))
        return x

    def ltdl_pivots(self, env, q, diag):
        """Pivots D [2S] of the leaf-first L^T D L factorisation of H(q) + diag."""
        S = self._S(env)
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64).reshape(2 * S)
        q, diag = f(q), f(diag)
        D = np.zeros(2 * S)
        lib().oracle_ltdl_pivots(self.h, env, _ptr(q), _ptr(diag), _ptr(D))
        return D

    def step_dot(self, env, n, x, kp, kd, F, vx, vkp, vkd, vF, w, broken0=None, det0=None):
        """Dot-product test of one step (switches frozen): (<J v, w>, <v, J^T w>).
        The numbers of switches the step used are left in ``last_switch_counts``.

        x, vx, w: [4S + 6A] (q, qd, apple position state, apple velocity); kp, kd, vkp,
        vkd: [S]; F, vF: [A, 3] or None; broken0 [S], det0 [A]: entry flags or None."""
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        u8 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.uint8)
        args = [f(x), f(kp), f(kd), f(F), u8(broken0), u8(det0), f(vx), f(vkp), f(vkd), f(vF), f(w)]
        out = np.zeros(6)
        lib().oracle_step_dot(self.h, env, int(n), *[_ptr(a) for a in args], _ptr(out))
        self.last_switch_counts = dict(broken=int(out[2]), detached=int(out[3]), clamped=int(out[4]), capped=int(out[5]))
        return float(out[0]), float(out[1])

    # ---- state and rollout ----------------------------------------------------------------
    def empty_state(self) -> State:
        S, A, B = self.batch.n_seg, self.batch.n_apple, self.batch.n_env
        return State(q=np.zeros((S, 2)), qd=np.zeros((S, 2)), ax=np.zeros((A, 3)), av=np.zeros((A, 3)),
                     aq=np.zeros((A, 4)), aw=np.zeros((A, 3)), broken=np.zeros(S, np.uint8),
                     cnt=np.zeros(S, np.uint8), det=np.zeros(A, np.uint8), cntp=np.zeros(A, np.uint8),
                     cntt=np.zeros(A, np.uint8), det_path=np.zeros(A, np.uint8),
                     break_step=np.full(S, -1, np.int32), det_step=np.full(A, -1, np.int32),
                     status=np.zeros(B, np.uint32), break_ratio=np.zeros(S), det_ratio=np.zeros(A))

    def _io(self, st: State, kp=None, kd=None, wrench=None, wrench_stride=0, aforce=None, aforce_stride=0,
            band: Band | None = None):
        io = IO()
        for f in ("q", "qd", "ax", "av", "aq", "aw", "broken", "cnt", "det", "cntp", "cntt", "det_path",
                  "break_step", "det_step", "status", "break_ratio", "det_ratio"):
            setattr(io, f, _ptr(getattr(st, f)))
        io.kp = _ptr(kp)
        io.kd = _ptr(kd)
        io.wrench = _ptr(wrench)
        io.wrench_stride = int(wrench_stride)
        io.aforce = _ptr(aforce)
        io.aforce_stride = int(aforce_stride)
        if band is not None:
            io.band_jmin, io.band_amin = _ptr(band.jmin), _ptr(band.amin)
            io.band_jfirst, io.band_afirst = _ptr(band.jfirst), _ptr(band.afirst)
        return io

    def rest_state(self) -> State:
        st = self.empty_state()
        io = self._io(st)
        lib().oracle_rest_state(self.h, C.byref(io))
        return st

    def rollout(self, st: State, n_steps: int, kp=None, kd=None, envs=None, wrench=None, wrench_stride=None,
                aforce=None, aforce_stride=None, band: Band | None = None, threads: int | None = None) -> State:
        """Advance ``st`` in place by n_steps (envs: subset of env indices).

        wrench: [S_tot, 6] constant or [n_steps, S_tot, 6]; aforce: [A_tot, 3] constant or
        [n_steps, A_tot, 3] (descriptor order, world frame)."""
        d = self.derived() if (kp is None or kd is None) else None
        kp = np.ascontiguousarray(d["kp"] if kp is None else kp, dtype=np.float64)
        kd = np.ascontiguousarray(d["kd"] if kd is None else kd, dtype=np.float64)
        if wrench is not None:
            wrench = np.ascontiguousarray(wrench, dtype=np.float64)
            if wrench_stride is None:
                wrench_stride = 0 if wrench.ndim == 2 else wrench.shape[1] * 6
        if aforce is not None:
            aforce = np.ascontiguousarray(aforce, dtype=np.float64)
            if aforce_stride is None:
                aforce_stride = 0 if aforce.ndim == 2 else aforce.shape[1] * 3
        io = self._io(st, kp, kd, wrench, wrench_stride or 0, aforce, aforce_stride or 0, band)
        envs = np.arange(self.batch.n_env, dtype=np.int32) if envs is None else np.asarray(envs, np.int32)
        if threads is None:
            threads = min(len(envs), os.cpu_count() or 1, 16)
        lib().oracle_rollout(self.h, C.byref(io), int(len(envs)), _ptr(envs), int(st.step), int(n_steps), int(threads))
        st.step += n_steps
        return st


def rng_u24(seed, env, step, seg, k) -> int:
    return int(lib().oracle_rng_u24(seed, env, step, seg, k))


def splitmix64(x: int) -> int:
    return int(lib().oracle_splitmix64(x))


def rng_normals(seed, env, step, seg) -> np.ndarray:
    """The three standard normals of the in-step random force of (env, step, segment)."""
    z = np.zeros(3)
    lib().oracle_rng_normals(seed, env, step, seg, _ptr(z))
    return z


# ---- adjoint (FP64, taped step, switches frozen) ------------------------------------------
def _setup_adjoint(L):
    if getattr(L, "_adj_ready", False):
        return
    L.oracle_record_new.restype = C.c_void_p
    L.oracle_record_free.argtypes = [C.c_void_p]
    L.oracle_loss.restype = C.c_double
    L.oracle_loss.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_int] + [_P] * 7 + [C.c_int, _P, _P, _P, C.c_void_p,
                                                                                   C.c_void_p, _P]
    L.oracle_adjoint.restype = C.c_double
    L.oracle_adjoint.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_int] + [_P] * 7 + [C.c_int, _P, _P, _P] + [_P] * 4
    L._adj_ready = True


class Record:
    """Switch schedule of a forward run (replayed by finite differences)."""

    def __init__(self):
        L = lib()
        _setup_adjoint(L)
        self.h = L.oracle_record_new()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.oracle_record_free(self.h)
            self.h = None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _adj_args(o, env, x0, kp, kd, F, tips, target):
    b = o.batch
    S = int(b.seg_offset[env + 1] - b.seg_offset[env])
    A = int(b.apple_offset[env + 1] - b.apple_offset[env])
    q0, qd0, ax0, av0 = (_f64(x0[k]) for k in ("q", "qd", "ax", "av"))
    assert q0.size == 2 * S and ax0.size == 3 * A
    tips = np.ascontiguousarray(tips, dtype=np.int32)
    target = _f64(target).reshape(-1, 3)
    return S, A, q0, qd0, ax0, av0, _f64(kp), _f64(kd), _f64(F), tips, target


def env_state0(o, st, env):
    """Initial-state dict of one env from a batch State (descriptor order)."""
    b = o.batch
    s0, s1 = b.seg_offset[env], b.seg_offset[env + 1]
    a0, a1 = b.apple_offset[env], b.apple_offset[env + 1]
    return dict(q=st.q[s0:s1], qd=st.qd[s0:s1], ax=st.ax[a0:a1], av=st.av[a0:a1])


def _w_state(w_state, S, A):
    if w_state is None:
        return None
    if isinstance(w_state, dict):
        z = lambda k, n: np.zeros(n) if w_state.get(k) is None else np.asarray(w_state[k], np.float64).reshape(-1)
        w_state = np.concatenate([z("q", 2 * S), z("qd", 2 * S), z("ax", 3 * A), z("av", 3 * A)])
    w = np.ascontiguousarray(w_state, dtype=np.float64)
    assert w.size == 4 * S + 6 * A
    return w


def loss(o, env, x0, kp, kd, F, n_steps, tips, target, step0=0, record_in=None, record_out=None, return_q=False,
         w_state=None):
    """Tip loss after n_steps, plus w_state . S_T if given (dict of q, qd, ax, av weights)."""
    L = lib()
    _setup_adjoint(L)
    S, A, q0, qd0, ax0, av0, kp, kd, F, tips, target = _adj_args(o, env, x0, kp, kd, F, tips, target)
    ws = _w_state(w_state, S, A)
    qf = np.zeros(4 * S) if return_q else None
    v = L.oracle_loss(o.h, env, step0, n_steps, _ptr(q0), _ptr(qd0), _ptr(ax0), _ptr(av0), _ptr(kp), _ptr(kd), _ptr(F),
                      len(tips), _ptr(tips), _ptr(target), _ptr(ws), record_in.h if record_in else None,
                      record_out.h if record_out else None, _ptr(qf))
    return (v, qf) if return_q else v


def adjoint(o, env, x0, kp, kd, F, n_steps, tips, target, step0=0, w_state=None):
    """Returns (L, dL/dkp, dL/dkd, dL/dF [n_steps, A, 3] or None, dL/dx0 dict)."""
    L = lib()
    _setup_adjoint(L)
    S, A, q0, qd0, ax0, av0, kp, kd, F, tips, target = _adj_args(o, env, x0, kp, kd, F, tips, target)
    ws = _w_state(w_state, S, A)
    gkp, gkd = np.zeros(S), np.zeros(S)
    gF = np.zeros((n_steps, A, 3)) if F is not None else None
    gx = np.zeros(4 * S + 6 * A)
    v = L.oracle_adjoint(o.h, env, step0, n_steps, _ptr(q0), _ptr(qd0), _ptr(ax0), _ptr(av0), _ptr(kp), _ptr(kd),
                         _ptr(F), len(tips), _ptr(tips), _ptr(target), _ptr(ws), _ptr(gkp), _ptr(gkd), _ptr(gF),
                         _ptr(gx))
    g0 = dict(q=gx[:2 * S].reshape(S, 2), qd=gx[2 * S:4 * S].reshape(S, 2), ax=gx[4 * S:4 * S + 3 * A].reshape(A, 3),
              av=gx[4 * S + 3 * A:].reshape(A, 3))
    return v, gkp, gkd, gF, g0


# ---- per-world geometry perturbation (the on-device rebuild's definition) --------------
def _qmul(a, b):
    """Hamilton product of quaternions (w, x, y, z), row-wise."""
    w1, x1, y1, z1 = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    w2, x2, y2, z2 = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def perturbed_batch(batch, factors):
    """The batch with every segment's length and radius scaled by factors[:, 0] and [:, 1]
    and its rest orientation bent by factors[:, 2] about its own x axis, then by
    factors[:, 3] about its y axis; a fruit's hang point keeps its place in its segment's
    frame, scaled with the segment's length.  factors: [S_tot, 4] descriptor order."""
    from dataclasses import replace
    f = np.asarray(factors, np.float64)
    zero = np.zeros(len(f))
    qx = np.stack([np.cos(f[:, 2] / 2), np.sin(f[:, 2] / 2), zero, zero], axis=1)
    qy = np.stack([np.cos(f[:, 3] / 2), zero, np.sin(f[:, 3] / 2), zero], axis=1)
    quat = _qmul(_qmul(batch.seg_rest_quat, qx), qy)
    env_of_apple = np.repeat(np.arange(batch.n_env), np.diff(batch.apple_offset))
    gseg = batch.seg_offset[env_of_apple] + batch.apple_seg
    return replace(batch, seg_length=batch.seg_length * f[:, 0], seg_radius=batch.seg_radius * f[:, 1],
                   seg_rest_quat=quat, apple_hang=batch.apple_hang * f[gseg, 0:1])
