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
