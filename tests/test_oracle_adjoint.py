"""Pins of the FP64 oracle adjoint: central finite differences of the loss with the
forward's event schedule replayed (switches frozen), coordinate-wise and along random
directions.  CPU only."""
import numpy as np
import pytest

from orchard_inputs import assemble, gen_tree, step_constants
from oracle.oracle import Oracle, Record, adjoint, env_state0, loss


def _setup(seed=4, S=25, A=5, T=40, pre=50):
    t = gen_tree(seed, S, A)
    b = assemble([t])
    o = Oracle(b, step_constants())
    d = o.derived()
    st = o.rest_state()
    o.rollout(st, pre)
    x0 = env_state0(o, st, 0)
    rng = np.random.default_rng(seed)
    F = rng.normal(0, 2, (T, b.n_apple, 3))
    leaves = np.flatnonzero(np.bincount(t.parent[1:], minlength=t.n_seg) == 0)
    tips = leaves[:4]
    R, p = o.fk(0, st.q.reshape(-1))
    target = p[tips] + R[tips][:, :, 2] * t.length[tips][:, None] + rng.normal(0, 0.05, (len(tips), 3))
    return o, d, x0, F, tips, target, T, pre


def test_oracle_adjoint_matches_replayed_central_differences():
    o, d, x0, F, tips, target, T, pre = _setup()
    Lv, gkp, gkd, gF, g0 = adjoint(o, 0, x0, d["kp"], d["kd"], F, T, tips, target, step0=pre)
    rec = Record()
    L0 = loss(o, 0, x0, d["kp"], d["kd"], F, T, tips, target, step0=pre, record_out=rec)
    assert abs(Lv - L0) <= 1e-14 * abs(L0)

    def fd(f, x, i, h):
        xp, xm = x.copy(), x.copy()
        xp.flat[i] += h
        xm.flat[i] -= h
        return (f(xp) - f(xm)) / (2 * h)

    fl = lambda kp, kd, FF, x: loss(o, 0, x, kp, kd, FF, T, tips, target, step0=pre, record_in=rec)
    for i in (0, 3, 10, 20):
        g = fd(lambda v: fl(v, d["kd"], F, x0), d["kp"], i, 1e-4 * d["kp"][i])
        assert abs(g - gkp[i]) <= 1e-5 * np.abs(gkp).max()
        g = fd(lambda v: fl(d["kp"], v, F, x0), d["kd"], i, 1e-4 * d["kd"][i])
        assert abs(g - gkd[i]) <= 1e-5 * np.abs(gkd).max()
    for i in (0, 7, 50, 200, gF.size - 1):
        g = fd(lambda v: fl(d["kp"], d["kd"], v, x0), F, i, 1e-4)
        assert abs(g - gF.flat[i]) <= 1e-5 * np.abs(gF).max()
    for key in ("q", "qd", "ax", "av"):
        for i in (0, 3):
            def f(v, key=key):
                xx = dict(x0)
                xx[key] = v
                return fl(d["kp"], d["kd"], F, xx)
            g = fd(f, x0[key], i, 1e-6)
            assert abs(g - g0[key].flat[i]) <= 1e-5 * np.abs(g0[key]).max() + 1e-12


def test_oracle_adjoint_directional_derivatives():
    o, d, x0, F, tips, target, T, pre = _setup(seed=7, S=18, A=4, T=30, pre=20)
    Lv, gkp, gkd, gF, g0 = adjoint(o, 0, x0, d["kp"], d["kd"], F, T, tips, target, step0=pre)
    rec = Record()
    loss(o, 0, x0, d["kp"], d["kd"], F, T, tips, target, step0=pre, record_out=rec)
    rng = np.random.default_rng(1)
    for _ in range(4):
        dkp = rng.normal(size=gkp.size) * d["kp"]
        dkd = rng.normal(size=gkd.size) * d["kd"]
        dF = rng.normal(size=F.shape)
        e = 1e-5
        Lp = loss(o, 0, x0, d["kp"] + e * dkp, d["kd"] + e * dkd, F + e * dF, T, tips, target, step0=pre, record_in=rec)
        Lm = loss(o, 0, x0, d["kp"] - e * dkp, d["kd"] - e * dkd, F - e * dF, T, tips, target, step0=pre, record_in=rec)
        fd = (Lp - Lm) / (2 * e)
        an = gkp @ dkp + gkd @ dkd + np.sum(gF * dF)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12)


def switch_window(seed=12, S=30, A=6, T=40, pre=20):
    """A differentiated window that contains every discrete switch of the step:
    a joint that breaks at window step 4 (a leaf segment with a tiny modulus of rupture),
    a fruit pulled off at window step 4 (1.5 f_det from the window's start), a fruit
    whose spur reaction is clamped (0.9 f_det against a clamp of 0.4 f_det) until its
    stem tension tears it off late in the window, and in-step
    random body forces of 100 N on 30 % of the segments, capped on the light ones.  The
    loss adds the pulled fruit's final position and velocity to the tip loss, so the
    ballistic flight after the detach (which leaves from the hang point) is
    differentiated too."""
    t = gen_tree(seed, S, A)
    leaves = np.flatnonzero(np.bincount(t.parent[1:], minlength=S) == 0)
    jb = int(leaves[-1])
    t.mor = t.mor.copy()
    t.mor[jb] = 1e3
    c = step_constants(react_max_factor=0.4, rng_seed=99, wrench_fraction=0.3, wrench_sigma=100.0)
    o = Oracle(assemble([t]), c)
    d = o.derived()
    st = o.rest_state()
    o.rollout(st, pre)
    x0 = env_state0(o, st, 0)
    rng = np.random.default_rng(seed)
    F = rng.normal(0, 1, (T, A, 3))
    F[:, 0] = 1.5 * t.apple_detach[0] * np.array([0.6, 0.0, 0.8])
    F[:, 1] = 0.9 * t.apple_detach[1] * np.array([0.0, 1.0, 0.0])
    tips = leaves[:4]
    R, p = o.fk(0, st.q.reshape(-1))
    target = p[tips] + R[tips][:, :, 2] * t.length[tips][:, None] + rng.normal(0, 0.05, (len(tips), 3))
    w = dict(ax=np.zeros((A, 3)), av=np.zeros((A, 3)))
    w["ax"][0] = [0.7, -0.2, 0.5]
    w["av"][0] = [0.01, 0.03, -0.02]
    return o, d, t, x0, F, tips, target, T, pre, jb, w


def test_oracle_adjoint_through_every_switch():
    o, d, t, x0, F, tips, target, T, pre, jb, w = switch_window()
    rec = Record()
    L0 = loss(o, 0, x0, d["kp"], d["kd"], F, T, tips, target, step0=pre, record_out=rec, w_state=w)
    # the window's switches, from a plain rollout of the same window
    st = o.rest_state()
    st.q[:], st.qd[:], st.ax[:], st.av[:] = x0["q"], x0["qd"], x0["ax"], x0["av"]
    st.step = pre
    o.rollout(st, T, aforce=F)
    assert st.break_step[jb] == pre + 4 and st.broken.sum() == 1
    assert st.det_step[0] == pre + 4 and st.det_path[0] == 1
    # the clamped fruit's stem tension overshoots and tears it off by the tension path
    assert st.det_path[1] == 2 and pre + 20 <= st.det_step[1] < pre + T and st.det.sum() == 2
    sw = o.step_dot(0, pre + 10, np.concatenate([x0["q"].reshape(-1), x0["qd"].reshape(-1), x0["ax"].reshape(-1),
                                                 x0["av"].reshape(-1)]), d["kp"], d["kd"], F[10],
                    *[np.zeros(n) for n in (4 * t.n_seg + 6 * t.n_apple, t.n_seg, t.n_seg)], np.zeros_like(F[10]),
                    np.zeros(4 * t.n_seg + 6 * t.n_apple))
    counts = o.last_switch_counts
    assert counts["clamped"] >= 1 and counts["capped"] >= 1, counts
    Lv, gkp, gkd, gF, g0 = adjoint(o, 0, x0, d["kp"], d["kd"], F, T, tips, target, step0=pre, w_state=w)
    assert abs(Lv - L0) <= 1e-13 * abs(L0)
    fl = lambda kp, kd, FF, x: loss(o, 0, x, kp, kd, FF, T, tips, target, step0=pre, record_in=rec, w_state=w)

    def fd(f, x, i, h):
        xp, xm = x.copy(), x.copy()
        xp.flat[i] += h
        xm.flat[i] -= h
        return (f(xp) - f(xm)) / (2 * h)

    # the broken joint's gains act only in the four steps before the break
    for i in (jb, 0, 5, int(t.apple_seg[1])):
        g = fd(lambda v: fl(v, d["kd"], F, x0), d["kp"], i, 1e-4 * d["kp"][i])
        assert abs(g - gkp[i]) <= 1e-6 * np.abs(gkp).max(), (i, g, gkp[i])
        g = fd(lambda v: fl(d["kp"], v, F, x0), d["kd"], i, 1e-4 * d["kd"][i])
        assert abs(g - gkd[i]) <= 1e-6 * np.abs(gkd).max(), (i, g, gkd[i])
    assert gkp[jb] != 0.0
    # forces on the pulled fruit before, at and after the detach step; on the clamped fruit
    for s, a in ((0, 0), (4, 0), (20, 0), (T - 1, 0), (3, 1), (30, 1), (12, 4)):
        for c in range(3):
            i = np.ravel_multi_index((s, a, c), F.shape)
            g = fd(lambda v: fl(d["kp"], d["kd"], v, x0), F, i, 1e-4)
            assert abs(g - gF.flat[i]) <= 1e-6 * np.abs(gF).max(), (s, a, c, g, gF.flat[i])
    for key in ("q", "qd", "ax", "av"):
        for i in (0, 3, x0[key].size - 1):
            def f(v, key=key):
                xx = dict(x0)
                xx[key] = v
                return fl(d["kp"], d["kd"], F, xx)
            g = fd(f, x0[key], i, 1e-6)
            assert abs(g - g0[key].flat[i]) <= 1e-6 * np.abs(g0[key]).max() + 1e-12, (key, i)
    # and along random directions in all parameters at once
    rng = np.random.default_rng(2)
    for _ in range(3):
        dkp, dkd, dF = rng.normal(size=gkp.size) * d["kp"], rng.normal(size=gkd.size) * d["kd"], rng.normal(size=F.shape)
        e = 1e-5
        fdv = (fl(d["kp"] + e * dkp, d["kd"] + e * dkd, F + e * dF, x0) -
               fl(d["kp"] - e * dkp, d["kd"] - e * dkd, F - e * dF, x0)) / (2 * e)
        an = gkp @ dkp + gkd @ dkd + np.sum(gF * dF)
        assert abs(fdv - an) <= 1e-6 * abs(an)
