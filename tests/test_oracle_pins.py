"""Pins of the FP64 oracle against closed forms, brute force and library routines.

Each test checks the oracle against something other than itself: textbook
formulas, finite differences of independent quantities, numpy's dense solver,
Monte-Carlo integrals or exact discrete recurrences.  CPU only.
"""
import math

import numpy as np
import pytest
import scipy.special

from orchard_inputs import (assemble, chain_tree, gen_tree, random_small_tree, step_constants,
                            ternary_lsystem_count)
from oracle.oracle import Band, Oracle, rng_u24, splitmix64

G = 9.81


def one(tree, **over):
    return Oracle(assemble([tree]), step_constants(**over))


def qrot(axis, ang):
    s = math.sin(ang / 2)
    return (math.cos(ang / 2), axis[0] * s, axis[1] * s, axis[2] * s)


# ------------------------------------------------------------------------------------------
# generator pins (Eq. lsystem, Eq. pipe)
# ------------------------------------------------------------------------------------------
def test_ternary_lsystem_body_count():
    # body count 1 + 2 (3^n - 1) printed with Eq. lsystem
    assert [ternary_lsystem_count(n) for n in range(1, 8)] == [5, 17, 53, 161, 485, 1457, 4373]
    assert all(ternary_lsystem_count(n) == 1 + 2 * (3 ** n - 1) for n in range(0, 8))


@pytest.mark.parametrize("S,A", [(50, 10), (300, 40), (1200, 120)])
def test_generator_structure_and_pipe_rule(S, A):
    t = gen_tree(12345 + S, S, A)
    assert t.n_seg == S and t.n_apple == A
    par = t.parent
    assert par[0] == -1 and np.all(par[1:] < np.arange(1, S)) and np.all(par[1:] >= 0)
    # breadth-first: depth non-decreasing, children contiguous
    depth = np.zeros(S, int)
    for i in range(1, S):
        depth[i] = depth[par[i]] + 1
    assert np.all(np.diff(depth) >= 0)
    assert np.all(np.diff(par[1:]) >= 0)
    # pipe model at every fork: r_p^beta = sum r_c^beta (beta = 2.25), chains keep r
    beta = 2.25
    for p in range(S):
        kids = np.flatnonzero(par == p)
        if kids.size:
            assert abs(t.radius[p] ** beta - np.sum(t.radius[kids] ** beta)) < 1e-12 * t.radius[p] ** beta
    assert abs(t.radius[0] - 0.04) < 1e-15
    assert np.allclose(np.linalg.norm(t.rest_quat, axis=1), 1.0, atol=1e-12)
    assert np.all((t.length >= 0.05) & (t.length <= 0.3))
    leaves = set(np.flatnonzero(np.bincount(par[1:], minlength=S) == 0))
    assert set(t.apple_seg.tolist()) <= leaves


# ------------------------------------------------------------------------------------------
# mass properties and derived gains (Eq. beam, Eq. break, capsule geometry)
# ------------------------------------------------------------------------------------------
def test_capsule_mass_properties_monte_carlo():
    r, l, rho = 0.03, 0.12, 800.0
    o = one(chain_tree(1, length=l, radius=r))
    d = o.derived()
    rng = np.random.default_rng(7)
    n = 4_000_000
    # sample the bounding box of the capsule centred on its COM
    P = rng.uniform([-r, -r, -(l / 2 + r)], [r, r, l / 2 + r], size=(n, 3))
    rho2 = P[:, 0] ** 2 + P[:, 1] ** 2
    zc = np.clip(P[:, 2], -l / 2, l / 2)
    inside = rho2 + (P[:, 2] - zc) ** 2 <= r * r
    vol_box = (2 * r) ** 2 * (l + 2 * r)
    w = inside * rho * vol_box / n
    m = w.sum()
    Izz = np.sum(w * rho2)
    Ixx = np.sum(w * (P[:, 1] ** 2 + P[:, 2] ** 2))
    assert abs(m - d["mass"][0]) < 3e-3 * m
    assert abs(Izz - d["Ia"][0]) < 5e-3 * Izz
    assert abs(Ixx - d["It"][0]) < 5e-3 * Ixx


def test_beam_stiffness_rupture_moment_and_damping():
    r, l, E, sig = 0.01, 0.2, 9e9, 75e6
    o = one(chain_tree(1, length=l, radius=r, youngs=E, mor=sig))
    d = o.derived()
    I_sec = math.pi * r ** 4 / 4
    assert abs(d["kp"][0] - E * I_sec / l) < 1e-12 * d["kp"][0]          # Eq. beam: EI / l
    assert abs(d["mmax"][0] - sig * math.pi * r ** 3 / 4) < 1e-12 * d["mmax"][0]  # Eq. break
    Jp = d["It"][0] + d["mass"][0] * (l / 2) ** 2                          # about the joint
    assert abs(d["kd"][0] - 2 * 0.05 * math.sqrt(d["kp"][0] * Jp)) < 1e-12 * d["kd"][0]
    # stiffness-proportional mode of the paper: Kd = c_d Kp
    d2 = one(chain_tree(1, length=l, radius=r, youngs=E), damping_cd=0.1).derived()
    assert abs(d2["kd"][0] - 0.1 * d2["kp"][0]) < 1e-12 * d2["kd"][0]


# ------------------------------------------------------------------------------------------
# kinematics
# ------------------------------------------------------------------------------------------
def _world_quats_from_generator(t):
    """World rest orientation by composing rest quaternions (quaternion algebra,
    independent of the oracle's matrix kinematics)."""
    def qmul(a, b):
        aw, ax, ay, az = a
        bw, bx, by, bz = b
        return np.array([aw * bw - ax * bx - ay * by - az * bz, aw * bx + ax * bw + ay * bz - az * by,
                         aw * by - ax * bz + ay * bw + az * bx, aw * bz + ax * by - ay * bx + az * bw])
    Q = np.zeros((t.n_seg, 4))
    for i in range(t.n_seg):
        Q[i] = t.rest_quat[i] if t.parent[i] < 0 else qmul(Q[t.parent[i]], t.rest_quat[i])
    return Q


def test_fk_rest_pose_matches_quaternion_composition():
    t = gen_tree(3, 80, 0)
    o = one(t)
    R, p = o.fk(0, np.zeros(2 * t.n_seg))
    Q = _world_quats_from_generator(t)
    for i in range(t.n_seg):
        w, x, y, z = Q[i]
        # rotate e_z by the quaternion: rest heading
        hz = np.array([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)])
        assert np.allclose(R[i][:, 2], hz, atol=1e-12)
        if t.parent[i] >= 0:
            assert abs(np.linalg.norm(p[i] - p[t.parent[i]]) - t.length[t.parent[i]]) < 1e-12


def test_fk_planar_two_link_closed_form():
    l1, l2 = 0.3, 0.2
    t = chain_tree(2, length=l1, radius=0.01)
    t.length[1] = l2
    o = one(t)
    for th1, th2 in [(0.3, -0.7), (1.1, 0.4), (-0.2, 2.0)]:
        q = np.array([th1, 0.0, th2, 0.0])
        R, p = o.fk(0, q)
        tip = p[1] + R[1] @ np.array([0, 0, l2])
        # planar 2R arm rotating about x: (y, z) = -l sin, l cos
        exp = np.array([0.0, -l1 * math.sin(th1) - l2 * math.sin(th1 + th2), l1 * math.cos(th1) + l2 * math.cos(th1 + th2)])
        assert np.allclose(tip, exp, atol=1e-14)


# ------------------------------------------------------------------------------------------
# CRBA vs brute-force J^T M J from finite-difference Jacobians
# ------------------------------------------------------------------------------------------
def _brute_mass_matrix(o, env, q, d, s0, eps=1e-6):
    n = q.size
    S = n // 2
    R0, p0 = o.fk(env, q)
    L = o.batch.seg_length[s0:s0 + S]
    com = lambda R, p: p + np.einsum("sij,j->si", R, np.stack([np.zeros(S), np.zeros(S), L / 2], 1)) \
        if False else p + R[:, :, 2] * (L[:, None] / 2)
    Jv = np.zeros((S, 3, n))
    Jw = np.zeros((S, 3, n))
    for k in range(n):
        e = np.zeros(n); e[k] = eps
        Rp, pp = o.fk(env, q + e)
        Rm, pm = o.fk(env, q - e)
        Jv[:, :, k] = (com(Rp, pp) - com(Rm, pm)) / (2 * eps)
        dR = (Rp - Rm) / (2 * eps)
        W = np.einsum("sij,skj->sik", dR, R0)  # dR R^T = [w]x
        Jw[:, :, k] = np.stack([W[:, 2, 1], W[:, 0, 2], W[:, 1, 0]], 1)
    H = np.zeros((n, n))
    for b in range(S):
        Ic = R0[b] @ np.diag([d["It"][s0 + b], d["It"][s0 + b], d["Ia"][s0 + b]]) @ R0[b].T
        H += d["mass"][s0 + b] * Jv[b].T @ Jv[b] + Jw[b].T @ Ic @ Jw[b]
    return H


@pytest.mark.parametrize("seed,S", [(1, 1), (2, 3), (3, 7), (4, 12)])
def test_crba_matches_brute_force_jtmj(seed, S):
    t = random_small_tree(seed, S)
    o = one(t)
    rng = np.random.default_rng(seed)
    q = rng.uniform(-1, 1, 2 * S)
    H = o.mass_matrix(0, q)
    Hb = _brute_mass_matrix(o, 0, q, o.derived(), 0)
    assert np.allclose(H, H.T, atol=0)
    assert np.max(np.abs(H - Hb)) < 1e-7 * np.max(np.abs(H))
    assert np.all(np.linalg.eigvalsh(H) > 0)


# ------------------------------------------------------------------------------------------
# RNEA pins
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed,S", [(5, 2), (6, 6), (7, 10)])
def test_rnea_against_mass_matrix_lagrangian_and_potential(seed, S):
    t = random_small_tree(seed, S)
    o = one(t)
    d = o.derived()
    n = 2 * S
    rng = np.random.default_rng(seed)
    q, qd, qdd = rng.uniform(-1, 1, n), rng.uniform(-2, 2, n), rng.uniform(-3, 3, n)
    H = o.mass_matrix(0, q)
    # ID(q, qd, qdd) - ID(q, qd, 0) = H qdd
    diff = o.inverse_dynamics(0, q, qd, qdd) - o.inverse_dynamics(0, q, qd, np.zeros(n))
    assert np.max(np.abs(diff - H @ qdd)) < 1e-12 * np.max(np.abs(H @ qdd))
    # gravity term = dV/dq, V = sum m g z_com (central differences of the potential)
    L = t.length

    def V(qq):
        R, p = o.fk(0, qq)
        zc = p[:, 2] + R[:, 2, 2] * L / 2
        return np.sum(d["mass"] * G * zc)
    eps = 1e-6
    dV = np.array([(V(q + eps * np.eye(n)[k]) - V(q - eps * np.eye(n)[k])) / (2 * eps) for k in range(n)])
    gq = o.inverse_dynamics(0, q, np.zeros(n), np.zeros(n))
    assert np.max(np.abs(gq - dV)) < 1e-7 * np.max(np.abs(gq))
    # velocity product terms = Christoffel symbols of H (central differences of H)
    dH = np.zeros((n, n, n))
    for k in range(n):
        e = np.zeros(n); e[k] = 1e-5
        dH[:, :, k] = (o.mass_matrix(0, q + e) - o.mass_matrix(0, q - e)) / 2e-5
    cor = np.einsum("ijk,j,k->i", dH, qd, qd) - 0.5 * np.einsum("jki,j,k->i", dH, qd, qd)
    cq = o.inverse_dynamics(0, q, qd, np.zeros(n)) - gq
    assert np.max(np.abs(cq - cor)) < 1e-6 * np.max(np.abs(cq))


def test_rnea_external_wrench_is_jacobian_transpose():
    S = 5
    t = random_small_tree(11, S)
    o = one(t)
    rng = np.random.default_rng(3)
    n = 2 * S
    q = rng.uniform(-1, 1, n)
    W = rng.normal(size=(S, 6))
    tau0 = o.inverse_dynamics(0, q, np.zeros(n), np.zeros(n), gravity=False)
    tauW = o.inverse_dynamics(0, q, np.zeros(n), np.zeros(n), wrench=W, gravity=False)
    # virtual work: tau_ext = -sum_b Jv_b^T F_b - Jw_b^T T_b (finite-difference Jacobians)
    R0, _ = o.fk(0, q)
    exp = np.zeros(n)
    eps = 1e-6
    for k in range(n):
        e = np.zeros(n); e[k] = eps
        Rp, pp = o.fk(0, q + e)
        Rm, pm = o.fk(0, q - e)
        cp = pp + Rp[:, :, 2] * (t.length[:, None] / 2)
        cm = pm + Rm[:, :, 2] * (t.length[:, None] / 2)
        Jv = (cp - cm) / (2 * eps)
        Wm = np.einsum("sij,skj->sik", (Rp - Rm) / (2 * eps), R0)
        Jw = np.stack([Wm[:, 2, 1], Wm[:, 0, 2], Wm[:, 1, 0]], 1)
        exp[k] = -np.sum(Jv * W[:, :3]) - np.sum(Jw * W[:, 3:])
    assert np.max(np.abs((tauW - tau0) - exp)) < 1e-7 * np.max(np.abs(exp))


@pytest.mark.parametrize("seed,S", [(21, 4), (22, 15), (23, 40)])
def test_ltdl_solve_matches_dense_solve(seed, S):
    t = random_small_tree(seed, S)
    o = one(t)
    rng = np.random.default_rng(seed)
    n = 2 * S
    q = rng.uniform(-1, 1, n)
    dg = rng.uniform(0, 1e-3, n)
    b = rng.normal(size=n)
    x = o.ltdl_solve(0, q, dg, b)
    xr = np.linalg.solve(o.mass_matrix(0, q) + np.diag(dg), b)
    assert np.max(np.abs(x - xr)) < 1e-9 * np.max(np.abs(xr))


# ------------------------------------------------------------------------------------------
# single-link pendulum and damping: exact discrete map of the implicit step
# ------------------------------------------------------------------------------------------
def _discrete_map(J, kp, kd, G_lin, h):
    den = J + h * kd + h * h * kp
    a = -(kp + G_lin) / den
    b = -(h * kp + kd) / den
    return np.array([[1 + h * h * a, h * (1 + h * b)], [h * a, 1 + h * b]])


@pytest.mark.parametrize("mode", ["nograv", "hanging", "upright", "damped"])
def test_single_link_pendulum_exact_discrete_map(mode):
    l, r = 0.25, 0.01
    root = (1.0, 0.0, 0.0, 0.0)
    grav = (0.0, 0.0, 0.0) if mode in ("nograv", "damped") else (0.0, 0.0, -G)
    if mode == "hanging":
        root = qrot((1, 0, 0), math.pi)
    t = chain_tree(1, length=l, radius=r, root_quat=root)
    o = one(t, gravity=grav)
    d = o.derived()
    m, kp = d["mass"][0], d["kp"][0]
    Jp = d["It"][0] + m * (l / 2) ** 2
    kd = d["kd"][0] if mode == "damped" else 0.0
    s = {"nograv": 0, "damped": 0, "hanging": 1, "upright": -1}[mode]
    Glin = s * m * G * l / 2
    h = 1e-3
    amp = 1e-4
    st = o.rest_state()
    st.q[0, 0] = amp
    n = 400
    traj = np.zeros(n)
    kpv, kdv = np.array([kp]), np.array([kd])
    for i in range(n):
        o.rollout(st, 1, kp=kpv, kd=kdv)
        traj[i] = st.q[0, 0]
    M = _discrete_map(Jp, kp, kd, Glin, h)
    x = np.array([amp, 0.0])
    ref = np.zeros(n)
    for i in range(n):
        x = M @ x
        ref[i] = x[0]
    tol = 1e-11 if s == 0 else 1e-7   # gravity: sin(theta) vs theta at 1e-4 rad
    assert np.max(np.abs(traj - ref)) < tol * amp
    if mode == "nograv":
        # |lambda| = (1 + h^2 w^2)^(-1/2), arg lambda = atan(h w): the implicit step's
        # damping and frequency warp of an undamped spring
        w = math.sqrt(kp / Jp)
        lam = np.linalg.eigvals(M)
        assert abs(abs(lam[0]) - (1 + h * h * w * w) ** -0.5) < 1e-12
        assert abs(abs(np.angle(lam[0])) / h - math.atan(h * w) / h) < 1e-6 * w
        # continuous small-angle frequency is the h -> 0 limit
        assert abs(math.atan(h * w) / h - w) < (h * w) ** 2 / 3 * w


# ------------------------------------------------------------------------------------------
# cantilever tip deflection PL^3/3EI of the discrete chain
# ------------------------------------------------------------------------------------------
def _static_solve(o, kp, W, n, iters=20):
    q = np.zeros(n)
    for _ in range(iters):
        res = kp * q + o.inverse_dynamics(0, q, np.zeros(n), np.zeros(n), wrench=W, gravity=False)
        J = np.diag(kp).astype(float)
        for k in range(n):
            e = np.zeros(n); e[k] = 1e-7
            J[:, k] += (o.inverse_dynamics(0, q + e, np.zeros(n), np.zeros(n), wrench=W, gravity=False)
                        - o.inverse_dynamics(0, q - e, np.zeros(n), np.zeros(n), wrench=W, gravity=False)) / 2e-7
        q = q - np.linalg.solve(J, res)
    return q


@pytest.mark.parametrize("N", [1, 2, 8])
def test_cantilever_tip_deflection(N):
    L, r, E = 1.0, 0.01, 9e9
    l = L / N
    t = chain_tree(N, length=l, radius=r, youngs=E, root_quat=qrot((0, 1, 0), math.pi / 2))
    o = one(t, gravity=(0.0, 0.0, 0.0))
    d = o.derived()
    EI = E * math.pi * r ** 4 / 4
    delta_c = 1e-4 * L
    P = delta_c * 3 * EI / L ** 3
    W = np.zeros((N, 6))
    W[-1, 2] = P                      # tip force P z at the last tip, moved to the COM
    W[-1, 3:] = np.cross([l / 2, 0, 0], [0, 0, P])
    exact = P * L ** 3 / (3 * EI) * (N + 1) * (2 * N + 1) / (2 * N * N)
    # settle the implicit step (large damping) and read the tip
    st = o.rest_state()
    kd = np.full(N, 0.02) * d["kp"]
    o.rollout(st, 3000, kp=d["kp"], kd=kd, wrench=W)
    R, p = o.fk(0, st.q.reshape(-1))
    tip = p[-1] + R[-1] @ np.array([0, 0, l])
    assert np.max(np.abs(st.qd)) < 1e-9
    assert abs(tip[2] - exact) < 1e-6 * exact + 1e-5 * delta_c
    # the settled state is the static equilibrium Kp q + g_ext(q) = 0 (Newton on ID)
    qs = _static_solve(o, np.repeat(d["kp"], 2), W, 2 * N)
    assert np.max(np.abs(st.q.reshape(-1) - qs)) < 1e-9 * np.max(np.abs(qs)) + 1e-15


def test_cantilever_converges_to_euler_bernoulli():
    # (N+1)(2N+1)/(2N^2) -> 1: the discrete chain converges to PL^3/3EI
    f = lambda N: (N + 1) * (2 * N + 1) / (2 * N * N)
    assert [round(f(N), 4) for N in (1, 2, 8, 32, 128, 512)] == [3.0, 1.875, 1.1953, 1.0474, 1.0117, 1.0029]


# ------------------------------------------------------------------------------------------
# energy of the continuous model (RK4 on H^-1(tau - c)), zero damping
# ------------------------------------------------------------------------------------------
@pytest.mark.slow
def test_energy_conservation_continuous_model():
    S = 5
    t = random_small_tree(31, S)
    t.radius[:] = np.linspace(0.03, 0.015, S)
    o = one(t)
    d = o.derived()
    n = 2 * S
    kp = np.repeat(d["kp"], 2)
    rng = np.random.default_rng(2)
    q = rng.uniform(-0.05, 0.05, n)
    qd = rng.uniform(-0.5, 0.5, n)

    def acc(q, qd):
        return np.linalg.solve(o.mass_matrix(0, q), -kp * q - o.inverse_dynamics(0, q, qd, np.zeros(n)))

    def energy(q, qd):
        R, p = o.fk(0, q)
        zc = p[:, 2] + R[:, 2, 2] * t.length / 2
        return 0.5 * qd @ o.mass_matrix(0, q) @ qd + 0.5 * np.sum(kp * q * q) + np.sum(d["mass"] * G * zc)

    h = 2e-5
    E0 = energy(q, qd)
    scale = 0.5 * qd @ o.mass_matrix(0, q) @ qd + 0.5 * np.sum(kp * q * q)
    for _ in range(2500):
        k1q, k1v = qd, acc(q, qd)
        k2q, k2v = qd + 0.5 * h * k1v, acc(q + 0.5 * h * k1q, qd + 0.5 * h * k1v)
        k3q, k3v = qd + 0.5 * h * k2v, acc(q + 0.5 * h * k2q, qd + 0.5 * h * k2v)
        k4q, k4v = qd + h * k3v, acc(q + h * k3q, qd + h * k3v)
        q = q + h / 6 * (k1q + 2 * k2q + 2 * k3q + k4q)
        qd = qd + h / 6 * (k1v + 2 * k2v + 2 * k3v + k4v)
    assert abs(energy(q, qd) - E0) < 1e-8 * scale


# ------------------------------------------------------------------------------------------
# rest invariants: static equilibrium and the apple reaction (Sec. "Fruit")
# ------------------------------------------------------------------------------------------
def test_static_equilibrium_is_fixed_point_and_apples_do_not_load_it():
    t = gen_tree(5, 30, 6)
    o_fruit = one(t)
    d = o_fruit.derived()
    S = t.n_seg
    n = 2 * S
    kp = np.repeat(d["kp"], 2)
    # static equilibrium of the fruitless tree: Kp q + g(q) = 0, Newton on the oracle's ID
    q = np.zeros(n)
    for _ in range(8):
        res = kp * q + o_fruit.inverse_dynamics(0, q, np.zeros(n), np.zeros(n))
        J = np.diag(kp).astype(float)
        for k in range(n):
            e = np.zeros(n); e[k] = 1e-7
            J[:, k] += (o_fruit.inverse_dynamics(0, q + e, np.zeros(n), np.zeros(n))
                        - o_fruit.inverse_dynamics(0, q - e, np.zeros(n), np.zeros(n))) / 2e-7
        q = q - np.linalg.solve(J, res)
    gnorm = np.max(np.abs(o_fruit.inverse_dynamics(0, np.zeros(n), np.zeros(n), np.zeros(n))))
    assert np.max(np.abs(kp * q + o_fruit.inverse_dynamics(0, q, np.zeros(n), np.zeros(n)))) < 1e-9 * gnorm
    # put the fruited tree there with every apple hanging m g / k_s below its hang point
    st = o_fruit.rest_state()
    st.q[:] = q.reshape(S, 2)
    for a in range(t.n_apple):  # apple state = stretch from the hang point while attached
        st.ax[a] = np.array([0, 0, -t.apple_mass[a] * G / 2e3])
    x0 = st.ax.copy()
    o_fruit.rollout(st, 5)
    # the step leaves it in place: zero reaction at rest, rest pose unaffected by fruit
    assert np.max(np.abs(st.q.reshape(-1) - q)) < 1e-9 * np.max(np.abs(q))
    assert np.max(np.abs(st.qd)) < 1e-9
    assert np.max(np.abs(st.ax - x0)) < 1e-12


# ------------------------------------------------------------------------------------------
# events: break threshold (Eq. break), detach timing (Sec. "Fruit"), free hinge
# ------------------------------------------------------------------------------------------
def test_break_threshold_ramp():
    # stubby link: the breaking angle sigma l / (E r) stays small (~0.02 rad)
    l, r = 0.05, 0.02
    t = chain_tree(1, length=l, radius=r, root_quat=qrot((0, 1, 0), math.pi / 2))
    # the impulse cap (m v_cap / h) would clip the load: lift it
    o = one(t, gravity=(0.0, 0.0, 0.0), v_cap=1e6)
    d = o.derived()
    kp, mmax = d["kp"][0], d["mmax"][0]
    th_b = mmax / kp
    Pb = mmax / (l * math.cos(th_b))   # quasi-static tip load at which kp |theta| = M_max
    n = 4000
    ramp = np.linspace(0.5, 1.5, n) * Pb
    W = np.zeros((n, 1, 6))
    W[:, 0, 2] = ramp
    W[:, 0, 3:] = np.cross([l / 2, 0, 0], np.stack([0 * ramp, 0 * ramp, ramp], 1))
    st = o.rest_state()
    o.rollout(st, n, kp=d["kp"], kd=np.array([1e-5 * kp]), wrench=W)
    # the test at step n sees the state after the load of step n-1
    n_cross = int(np.argmax(ramp > Pb)) + 1
    assert st.broken[0] == 1
    # first exceeding step + (N_break - 1)
    assert abs(int(st.break_step[0]) - (n_cross + 4)) <= 1
    # the event's ratio is mu = kp |theta| / M_max of the state at the start of the break
    # step: roll to that step again, form mu from its state, take the break step
    nb = int(st.break_step[0])
    st2 = o.rest_state()
    o.rollout(st2, nb, kp=d["kp"], kd=np.array([1e-5 * kp]), wrench=W[:nb])
    assert st2.broken[0] == 0 and st2.break_ratio[0] == 0.0
    mu = kp * math.hypot(st2.q[0, 0], st2.q[0, 1]) / mmax
    o.rollout(st2, 1, kp=d["kp"], kd=np.array([1e-5 * kp]), wrench=W[nb:nb + 1])
    assert st2.broken[0] == 1 and st2.break_step[0] == nb
    assert abs(st2.break_ratio[0] - mu) <= 1e-14 * mu
    assert st.break_ratio[0] == st2.break_ratio[0]
    # a quasi-static ramp of 1/4000 of the load per step, five steps in a row above 1
    assert 1.0 < mu < 1.0 + 6.0 / n * 1.5


def test_detach_pull_timing_and_tension_path():
    t = gen_tree(9, 20, 3)
    o = one(t)
    A = t.n_apple
    n0 = 37
    # constant pull 1.2 f_det on apple 0 from step n0: detach at n0 + N_pull - 1 exactly
    F = np.zeros((120, A, 3))
    F[n0:, 0, 0] = 1.2 * t.apple_detach[0]
    F[:, 1, 2] = -0.5 * t.apple_detach[1]    # below both thresholds: never
    st = o.rest_state()
    o.rollout(st, 120, aforce=F)
    assert st.det[0] == 1 and st.det_step[0] == n0 + 5 - 1 and st.det_path[0] == 1
    assert st.det[1] == 0 and st.det_step[1] == -1
    # pull ratio pi = |F| / f_det at the detach step; none for the apple that stays
    assert abs(st.det_ratio[0] - 1.2) <= 1e-15 * 1.2 and st.det_ratio[1] == 0.0
    # tension path: downward pull just below f_det, weight pushes the stem above 1.1 f_det
    F2 = np.zeros((A, 3))
    F2[2, 2] = -0.99 * t.apple_detach[2]
    st2 = o.rest_state()
    o.rollout(st2, 400, aforce=F2)
    assert st2.det[2] == 1 and st2.det_path[2] == 2
    assert st2.det[0] == 0 and st2.det[1] == 0
    # the tension detach records tau = k_s |s| / (alpha f_det) (above 1), not the pull's 0.99
    assert st2.det_ratio[2] > 1.0 and st2.det_ratio[0] == 0.0


def test_free_hinge_swings_at_gravity_rate():
    # a broken joint is a rigid pendulum: period 4 sqrt(Jp / (m g l/2)) K(sin(theta0/2))
    l, r = 0.2, 0.005
    t = chain_tree(1, length=l, radius=r, root_quat=qrot((1, 0, 0), math.pi))
    o = one(t)
    d = o.derived()
    m = d["mass"][0]
    Jp = d["It"][0] + m * (l / 2) ** 2
    th0 = 1.0
    st = o.rest_state()
    st.q[0, 0] = th0
    st.broken[0] = 1
    h = 1e-3
    n = 3000
    tr = np.zeros(n)
    for i in range(n):
        o.rollout(st, 1)
        tr[i] = st.q[0, 0]
    # downward zero crossings -> period
    idx = np.flatnonzero((tr[:-1] > 0) & (tr[1:] <= 0))
    tc = [(i + tr[i] / (tr[i] - tr[i + 1])) * h for i in idx]
    T = np.mean(np.diff(tc))
    T_exact = 4 * math.sqrt(Jp / (m * G * l / 2)) * scipy.special.ellipk(math.sin(th0 / 2) ** 2)
    assert abs(T - T_exact) < 2e-3 * T_exact
    assert abs(np.max(tr[-800:]) - th0) < 2e-2   # no spring, no damper: amplitude kept


def test_impulse_cap_and_snapped_mask():
    t = chain_tree(2, length=0.15, radius=0.01)
    o = one(t, gravity=(0.0, 0.0, 0.0))
    d = o.derived()
    cap = d["mass"][1] * 1.0 / 1e-3
    W1 = np.zeros((2, 6)); W1[1, 0] = 1e6
    W2 = np.zeros((2, 6)); W2[1, 0] = cap
    a, b = o.rest_state(), o.rest_state()
    o.rollout(a, 3, wrench=W1)
    o.rollout(b, 3, wrench=W2)
    assert np.array_equal(a.q, b.q)
    # forces on a snapped sub-tree are disabled: root broken -> wrench has no effect
    c, e = o.rest_state(), o.rest_state()
    c.broken[0] = 1; e.broken[0] = 1
    o.rollout(c, 3, wrench=W2)
    o.rollout(e, 3)
    assert np.array_equal(c.q, e.q)


# ------------------------------------------------------------------------------------------
# invariances
# ------------------------------------------------------------------------------------------
def test_frame_invariance_gravity_and_root_rotation():
    t = gen_tree(17, 40, 5)
    Rq = qrot(np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8]), 0.9)

    def qmul(a, b):
        aw, ax, ay, az = a
        bw, bx, by, bz = b
        return np.array([aw * bw - ax * bx - ay * by - az * bz, aw * bx + ax * bw + ay * bz - az * by,
                         aw * by - ax * bz + ay * bw + az * bx, aw * bz + ax * by - ay * bx + az * bw])
    w, x, y, z = Rq
    Rm = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                   [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                   [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    t2 = gen_tree(17, 40, 5)
    t2.rest_quat = t2.rest_quat.copy()
    t2.rest_quat[0] = qmul(Rq, t.rest_quat[0])
    o1 = one(t)
    o2 = one(t2, gravity=tuple(Rm @ np.array([0, 0, -G])))
    s1, s2 = o1.rest_state(), o2.rest_state()
    o1.rollout(s1, 300)
    o2.rollout(s2, 300)
    assert np.max(np.abs(s1.q - s2.q)) < 1e-12 * np.max(np.abs(s1.q))


def test_env_order_invariance_and_batch_independence():
    trees = [gen_tree(100 + i, 20 + 7 * i, 3) for i in range(4)]
    ob = Oracle(assemble(trees), step_constants())
    orv = Oracle(assemble(trees[::-1]), step_constants())
    sb, sr = ob.rest_state(), orv.rest_state()
    ob.rollout(sb, 200)
    orv.rollout(sr, 200)
    bo = ob.batch.seg_offset
    ro = orv.batch.seg_offset
    for e in range(4):
        a = sb.q[bo[e]:bo[e + 1]]
        er = 3 - e
        b = sr.q[ro[er]:ro[er + 1]]
        assert np.array_equal(a, b)


# ------------------------------------------------------------------------------------------
# counter-based generator (SplitMix64)
# ------------------------------------------------------------------------------------------
def test_splitmix64_published_value_and_u24_statistics():
    # first output of SplitMix64 from state 0 (Steele-Lea-Flood / Vigna reference code)
    assert splitmix64(0) == 0xE220A8397B1DCDAF
    u = np.array([rng_u24(7, e, s, i, 0) for e in range(4) for s in range(50) for i in range(100)])
    assert u.max() < 2 ** 24 and u.min() >= 0
    frac = np.mean(u < int(0.05 * 2 ** 24))
    assert abs(frac - 0.05) < 0.01
    assert abs(u.mean() / 2 ** 24 - 0.5) < 0.01
