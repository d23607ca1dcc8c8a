"""Pins of the oracle's apple path (Sec. "Fruit") against closed forms.

* a fruit on a rigid spur is a damped spring-mass: the oracle's apple converges at
  first order in h to the analytic damped oscillator;
* a constant pull F on a fruit loads its spur exactly like the force F applied at the
  hang point: the settled tree equals the static equilibrium under that point force
  (Newton on the oracle's inverse dynamics, no apple code involved);
* a detached fruit is a ballistic body: the discrete sequence of the semi-implicit
  update in closed form, within h a t / 2 of the parabola;
* the coupled tree + fruit step converges at first order in h to an RK4 solution of
  the continuous equations (tree: H q'' = -Kp q - Kd q' - c(q, q', f_react at the hang
  point); fruit: m x'' = m g - k_s (x - x_hang) - c_s x'), which pins the position
  state kept as the stretch from the hang point;
* the in-step normal draws have the moments and distribution of N(0, 1).
CPU only.
"""
import math

import numpy as np
import pytest
import scipy.stats

from orchard_inputs import assemble, chain_tree, random_small_tree, step_constants
from oracle.oracle import Oracle, rng_normals

G = 9.81
K_S = 2e3


def qrot(axis, ang):
    s = math.sin(ang / 2)
    return (math.cos(ang / 2), axis[0] * s, axis[1] * s, axis[2] * s)


def with_apples(t, segs, mass, fdet, hang=None):
    """Tree t with apples on the listed segments, hanging at the segment tips."""
    segs = np.asarray(segs, np.int32)
    A = segs.size
    t.apple_seg = segs
    t.apple_hang = np.zeros((A, 3)) if hang is None else np.asarray(hang, float).reshape(A, 3)
    if hang is None:
        t.apple_hang[:, 2] = t.length[segs]
    t.apple_mass = np.full(A, float(mass)) if np.isscalar(mass) else np.asarray(mass, float)
    t.apple_radius = np.full(A, 0.035)
    t.apple_detach = np.full(A, float(fdet)) if np.isscalar(fdet) else np.asarray(fdet, float)
    return t


# ------------------------------------------------------------------------------------------
# a fruit on a rigid spur: damped spring-mass (tether of Sec. "Fruit")
# ------------------------------------------------------------------------------------------
def _damped_oscillator(y0, v0, w0, zeta, t):
    wd = w0 * math.sqrt(1 - zeta * zeta)
    e = math.exp(-zeta * w0 * t)
    B = (v0 + zeta * w0 * y0) / wd
    y = e * (y0 * math.cos(wd * t) + B * math.sin(wd * t))
    v = e * (-zeta * w0 * (y0 * math.cos(wd * t) + B * math.sin(wd * t)) + wd * (-y0 * math.sin(wd * t) + B * math.cos(wd * t)))
    return y, v


def test_fruit_on_rigid_spur_converges_to_damped_oscillator():
    m, zeta = 0.2, 0.05
    y0 = np.array([0.01, -0.02, 0.015])
    v0 = np.array([0.1, 0.0, -0.2])
    T = 0.1
    errs = []
    for h in (1e-3, 5e-4, 2.5e-4):
        # a stubby spur of absurd stiffness does not move: the hang point is fixed
        t = with_apples(chain_tree(1, length=0.1, radius=0.05, youngs=1e24), [0], m, 1e6)
        o = Oracle(assemble([t]), step_constants(dt=h, tether_zeta=zeta))
        st = o.rest_state()
        s_eq = st.ax[0].copy()
        assert np.allclose(s_eq, [0, 0, -m * G / K_S], rtol=0, atol=1e-15)
        st.ax[0] = s_eq + y0     # stretch (the hang point is at rest)
        st.av[0] = v0
        o.rollout(st, int(round(T / h)))
        assert np.max(np.abs(st.q)) < 1e-15
        w0 = math.sqrt(K_S / m)
        e = 0.0
        for c in range(3):
            y, v = _damped_oscillator(y0[c], v0[c], w0, zeta, T)
            e = max(e, abs(st.ax[0, c] - s_eq[c] - y) / np.max(np.abs(y0)), abs(st.av[0, c] - v) / (w0 * np.max(np.abs(y0))))
        errs.append(e)
    # first order in h, and small
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2, errs
    assert errs[-1] < 0.01


# ------------------------------------------------------------------------------------------
# a pull on the fruit loads the spur like the same force at the hang point
# ------------------------------------------------------------------------------------------
def _hang_points(o, q, t):
    R, p = o.fk(0, q)
    return p[t.apple_seg] + np.einsum("aij,aj->ai", R[t.apple_seg], t.apple_hang), R, p


def _static_with_point_force(o, t, kp, a, F, q0):
    """Newton solve of Kp q + ID(q, 0, 0; gravity, F at the hang point of apple a) = 0."""
    S, n = t.n_seg, 2 * t.n_seg
    b = int(t.apple_seg[a])

    def residual(q):
        xh, R, p = _hang_points(o, q, t)
        com = p[b] + R[b][:, 2] * t.length[b] / 2
        W = np.zeros((S, 6))
        W[b, :3] = F
        W[b, 3:] = np.cross(xh[a] - com, F)
        return kp * q + o.inverse_dynamics(0, q, np.zeros(n), np.zeros(n), wrench=W)

    q = q0.copy()
    for _ in range(12):
        r = residual(q)
        J = np.zeros((n, n))
        for k in range(n):
            e = np.zeros(n); e[k] = 1e-7
            J[:, k] = (residual(q + e) - residual(q - e)) / 2e-7
        q = q - np.linalg.solve(J, r)
    return q, np.max(np.abs(residual(q)))


def test_pull_on_fruit_equals_force_at_hang_point():
    t = with_apples(random_small_tree(41, 6), [3, 5], 0.2, 25.0)
    t.youngs[:] = 3e8        # compliant enough that the pull visibly bends the tree
    o = Oracle(assemble([t]), step_constants(tether_zeta=1.0))
    d = o.derived()
    J = np.array([np.diag(o.mass_matrix(0, np.zeros(12)))[2 * i] for i in range(6)])
    kd = 2.0 * np.sqrt(d["kp"] * J)     # about critical damping: settles in a few thousand steps
    F = np.array([4.0, -3.0, 2.5])       # below the detach and clamp thresholds
    Fa = np.zeros((2, 3)); Fa[1] = F
    st = o.rest_state()
    o.rollout(st, 6000, kp=d["kp"], kd=kd, aforce=Fa)
    assert np.max(np.abs(st.qd)) < 1e-12 and st.det.sum() == 0
    kp2 = np.repeat(d["kp"], 2)
    q_ref, res = _static_with_point_force(o, t, kp2, 1, F, st.q.reshape(-1))
    assert res < 1e-12
    q_rest, _ = _static_with_point_force(o, t, kp2, 1, np.zeros(3), np.zeros(12))
    # the pull moves the equilibrium well beyond the tolerance, the step lands on it
    assert np.max(np.abs(q_ref - q_rest)) > 1e-3 * np.max(np.abs(q_ref))
    assert np.max(np.abs(st.q.reshape(-1) - q_ref)) < 1e-9 * np.max(np.abs(q_ref))
    # the fruit hangs where its tether balances weight and pull: k_s s = m g + F
    s_expect = (0.2 * np.array([0, 0, -G]) + F) / K_S
    assert np.max(np.abs(st.ax[1] - s_expect)) < 1e-12


# ------------------------------------------------------------------------------------------
# a detached fruit is a ballistic body
# ------------------------------------------------------------------------------------------
def test_detached_fruit_is_ballistic():
    t = with_apples(chain_tree(2, length=0.2, radius=0.02, root_quat=qrot((0, 1, 0), 0.6)), [1, 1], 0.2, 15.0)
    o = Oracle(assemble([t]), step_constants())
    m, h = 0.2, 1e-3
    F = np.array([[20.0, 10.0, 5.0], [0.0, 0.0, 0.0]])   # 23 N > 15 N on apple 0 from step 0
    st = o.rest_state()
    o.rollout(st, 6, aforce=F)
    assert st.det[0] == 1 and st.det_step[0] == 4 and st.det_path[0] == 1 and st.det[1] == 0
    x0, v0 = st.ax[0].copy(), st.av[0].copy()
    a = np.array([0, 0, -G]) + F[0] / m
    N = 400
    o.rollout(st, N, aforce=F)
    n = N
    x_disc = x0 + n * h * v0 + a * h * h * n * (n + 1) / 2
    v_disc = v0 + n * h * a
    assert np.max(np.abs(st.av[0] - v_disc)) < 1e-12 * np.max(np.abs(v_disc))
    assert np.max(np.abs(st.ax[0] - x_disc)) < 1e-12 * np.max(np.abs(x_disc))
    # within h a t / 2 of the continuous parabola
    tt = n * h
    x_cont = x0 + v0 * tt + a * tt * tt / 2
    assert np.all(np.abs(st.ax[0] - x_cont) <= np.abs(a) * h * tt / 2 * (1 + 1e-9) + 1e-15)


def test_detach_hands_over_the_absolute_position():
    # at the detach step the fruit leaves from where the tether held it: hang point plus
    # stretch, then one ballistic update
    t = with_apples(chain_tree(2, length=0.2, radius=0.02, root_quat=qrot((0, 1, 0), 0.6)), [1], 0.2, 15.0)
    o = Oracle(assemble([t]), step_constants())
    h = 1e-3
    F = np.array([[20.0, 10.0, 5.0]])
    st = o.rest_state()
    o.rollout(st, 4, aforce=F)           # steps 0..3: attached
    q, qd = st.q.reshape(-1).copy(), st.qd.reshape(-1).copy()
    xh, _, _ = _hang_points(o, q, t)
    eps = 1e-7
    vh = (_hang_points(o, q + eps * qd, t)[0] - _hang_points(o, q - eps * qd, t)[0]) / (2 * eps)
    s = st.ax[0] - h * vh[0]             # stretch at the start of the detach step
    o.rollout(st, 1, aforce=F)           # step 4: detach
    assert st.det[0] == 1 and st.det_step[0] == 4
    x_expect = xh[0] + s + h * st.av[0]
    assert np.max(np.abs(st.ax[0] - x_expect)) < 1e-9


def test_tension_detach_records_the_stem_tension_ratio():
    # a downward pull just below f_det plus the weight loads the stem above alpha f_det:
    # the detach goes by tension, and its ratio is tau = k_s |s| / (alpha f_det) of the
    # stretch s at the start of the detach step (s = position state - h v_hang)
    t = with_apples(chain_tree(2, length=0.2, radius=0.02, root_quat=qrot((0, 1, 0), 0.6)), [1], 0.2, 15.0)
    c = step_constants()
    o = Oracle(assemble([t]), c)
    h = c["dt"]
    F = np.array([[0.0, 0.0, -0.99 * 15.0]])
    st = o.rest_state()
    o.rollout(st, 400, aforce=F)
    assert st.det[0] == 1 and st.det_path[0] == 2
    nd = int(st.det_step[0])
    st2 = o.rest_state()
    o.rollout(st2, nd, aforce=F)
    q, qd = st2.q.reshape(-1).copy(), st2.qd.reshape(-1).copy()
    eps = 1e-7
    vh = (_hang_points(o, q + eps * qd, t)[0] - _hang_points(o, q - eps * qd, t)[0]) / (2 * eps)
    s = st2.ax[0] - h * vh[0]
    tau = K_S * np.linalg.norm(s) / (c["tension_factor"] * 15.0)
    o.rollout(st2, 1, aforce=F)
    assert st2.det[0] == 1 and st2.det_step[0] == nd
    assert st2.det_ratio[0] == st.det_ratio[0]
    assert 1.0 < tau and abs(st.det_ratio[0] - tau) < 1e-8 * tau


# ------------------------------------------------------------------------------------------
# coupled tree + fruit: first-order convergence to the continuous model
# ------------------------------------------------------------------------------------------
def _continuous_rhs(o, t, kp, kd, ks, cs, g):
    S, n = t.n_seg, 2 * t.n_seg
    A = t.n_apple

    def f(y):
        q, qd = y[:n], y[n:2 * n]
        x, v = y[2 * n:2 * n + 3 * A].reshape(A, 3), y[2 * n + 3 * A:].reshape(A, 3)
        xh, R, p = _hang_points(o, q, t)
        W = np.zeros((S, 6))
        for a in range(A):
            b = int(t.apple_seg[a])
            fr = ks * (x[a] - xh[a]) - t.apple_mass[a] * g   # elastic part minus weight
            com = p[b] + R[b][:, 2] * t.length[b] / 2
            W[b, :3] += fr
            W[b, 3:] += np.cross(xh[a] - com, fr)
        c = o.inverse_dynamics(0, q, qd, np.zeros(n), wrench=W)
        qdd = np.linalg.solve(o.mass_matrix(0, q), -kp * q - kd * qd - c)
        acc = g[None, :] + (-ks * (x - xh) - cs[:, None] * v) / t.apple_mass[:, None]
        return np.concatenate([qd, qdd, v.reshape(-1), acc.reshape(-1)])
    return f


@pytest.mark.parametrize("apples", [False, True])
def test_step_converges_first_order_to_continuous_model(apples):
    t = chain_tree(3, length=0.2, radius=0.02, youngs=3e7, root_quat=qrot((1, 0, 0), 0.8))
    if apples:
        t = with_apples(t, [2], 0.2, 1e3)
    S, n, A = t.n_seg, 6, t.n_apple
    g = np.array([0, 0, -G])
    rng = np.random.default_rng(3)
    q0 = rng.uniform(-0.02, 0.02, n)
    T = 0.05
    o_ref = Oracle(assemble([t]), step_constants())
    d = o_ref.derived()
    kp, kd = np.repeat(d["kp"], 2), np.repeat(d["kd"], 2)
    cs = d["apple_cs"]
    xh0, _, _ = _hang_points(o_ref, q0, t)
    s0 = np.array([[0.004, -0.003, 0.005]]) + np.array([[0, 0, -0.2 * G / K_S]]) if apples else np.zeros((0, 3))
    y = np.concatenate([q0, np.zeros(n), (xh0 + s0).reshape(-1), np.zeros(3 * A)])
    f = _continuous_rhs(o_ref, t, kp, kd, K_S, cs, g)
    hr = 2e-5
    for _ in range(int(round(T / hr))):
        k1 = f(y); k2 = f(y + 0.5 * hr * k1); k3 = f(y + 0.5 * hr * k2); k4 = f(y + hr * k3)
        y = y + hr / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    q_ref, qd_ref = y[:n], y[n:2 * n]
    x_ref, v_ref = y[2 * n:2 * n + 3 * A].reshape(A, 3), y[2 * n + 3 * A:].reshape(A, 3)
    errs = []
    for h in (1e-3, 5e-4, 2.5e-4, 1.25e-4):
        o = Oracle(assemble([t]), step_constants(dt=h))
        st = o.rest_state()
        st.q[:] = q0.reshape(S, 2)
        if apples:
            st.ax[:] = s0              # the tree starts at rest, so the stretch state is s0
        o.rollout(st, int(round(T / h)), kp=d["kp"], kd=d["kd"])
        q, qd = st.q.reshape(-1), st.qd.reshape(-1)
        e = [np.max(np.abs(q - q_ref)) / np.max(np.abs(q_ref)), np.max(np.abs(qd - qd_ref)) / np.max(np.abs(qd_ref))]
        if apples:
            # absolute position = hang point + (stretch state - h v_hang)
            xh, _, _ = _hang_points(o, q, t)
            eps = 1e-7
            vh = (_hang_points(o, q + eps * qd, t)[0] - _hang_points(o, q - eps * qd, t)[0]) / (2 * eps)
            x = xh + st.ax - h * vh
            e += [np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref - xh0)), np.max(np.abs(st.av - v_ref)) / np.max(np.abs(v_ref))]
        errs.append(np.array(e))
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    print("errors", errs, "ratios", ratios)
    # the error halves with h (first order), approaching the asymptotic ratio 2
    assert all(np.all((r > 1.6) & (r < 2.4)) for r in ratios), ratios
    assert np.all((ratios[-1] > 1.85) & (ratios[-1] < 2.15)), ratios
    assert np.all(errs[-1] < 0.1)


# ------------------------------------------------------------------------------------------
# the in-step normal draws
# ------------------------------------------------------------------------------------------
def test_box_muller_normals_are_standard_normal():
    z = np.array([rng_normals(11, e, s, i) for e in range(4) for s in range(250) for i in range(200)]).reshape(-1)
    assert z.size == 600_000
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert abs(np.mean(z ** 4) - 3.0) < 0.03
    assert abs(np.mean(z ** 3)) < 0.02
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # the three components of one draw are uncorrelated
    Z = z.reshape(-1, 3)
    C = np.corrcoef(Z.T)
    assert np.max(np.abs(C - np.eye(3))) < 0.01
