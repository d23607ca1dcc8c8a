"""Pins of the oracle's factorisation, forward dynamics, energy decay, ordering and
tangent/adjoint consistency against independent computations.

* An articulated-body recursion (Featherstone's ABA, written here in numpy on
  world-frame spatial vectors) gives the 2x2 joint pivots D_i = S_i^T I^A_i S_i and the
  joint accelerations of the implicit system; the oracle's explicit mass matrix,
  inverse dynamics and scalar leaf-first L^T D L must agree with both.
* In the linear regime without damping the implicit step removes a fixed fraction of
  each mode's energy per step: E_n = sum_k E_k(0) (1 + h^2 w_k^2)^-n, with w_k, v_k
  from the generalised eigenproblem K v = w^2 H(0) v.
* Renumbering the segments (any parent-before-child order) and the apples changes
  nothing but rounding.
* The tangent-linear and the reverse mode of one step agree: <J v, w> = <v, J^T w>,
  with every discrete switch (broken joints, detached and clamped fruit, capped body
  forces) frozen.
CPU only.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from orchard_inputs import assemble, chain_tree, gen_tree, random_small_tree, step_constants
from orchard_inputs.treegen import TreeDesc
from oracle.oracle import Oracle

G = 9.81


def skew(c):
    return np.array([[0, -c[2], c[1]], [c[2], 0, -c[0]], [-c[1], c[0], 0]])


def crm(v):
    """Motion cross product matrix of a spatial motion vector (angular, linear)."""
    X = np.zeros((6, 6))
    X[:3, :3] = skew(v[:3]); X[3:, 3:] = skew(v[:3]); X[3:, :3] = skew(v[3:])
    return X


def crf(v):
    return -crm(v).T


class ABA:
    """Articulated-body forward dynamics on world-frame spatial vectors (6-vectors at the
    world origin, angular first).  Each joint is two revolutes at the parent's tip:
    first about a0 = (R_parent Q_rest) e_x, then about a1 = R e_y."""

    def __init__(self, o, t, q, qd):
        self.t = t
        S = t.n_seg
        d = o.derived()
        R, p = o.fk(0, q)
        self.S = S
        self.I = np.zeros((S, 6, 6))
        self.s = np.zeros((S, 6, 2))
        self.v = np.zeros((S, 6))
        self.c = np.zeros((S, 6))
        qq = q.reshape(S, 2)
        qdd = qd.reshape(S, 2)
        for i in range(S):
            m = d["mass"][i]
            com = p[i] + R[i][:, 2] * t.length[i] / 2
            Ic = R[i] @ np.diag([d["It"][i], d["It"][i], d["Ia"][i]]) @ R[i].T
            C = skew(com)
            self.I[i] = np.block([[Ic + m * C @ C.T, m * C], [m * C.T, m * np.eye(3)]])
            cy, sy = math.cos(qq[i, 1]), math.sin(qq[i, 1])
            a0 = R[i] @ np.array([cy, 0.0, sy])
            a1 = R[i][:, 1]
            self.s[i, :, 0] = np.concatenate([a0, np.cross(p[i], a0)])
            self.s[i, :, 1] = np.concatenate([a1, np.cross(p[i], a1)])
            vp = np.zeros(6) if t.parent[i] < 0 else self.v[t.parent[i]]
            v_mid = vp + self.s[i, :, 0] * qdd[i, 0]
            self.v[i] = v_mid + self.s[i, :, 1] * qdd[i, 1]
            self.c[i] = qdd[i, 0] * crm(vp) @ self.s[i, :, 0] + qdd[i, 1] * crm(v_mid) @ self.s[i, :, 1]

    def solve(self, tau, dg, fext=None, gravity=(0.0, 0.0, -G)):
        """Joint accelerations of (H + diag(dg)) qdd = tau - c; also the 2x2 pivots."""
        S, t = self.S, self.t
        tau = tau.reshape(S, 2)
        dg = dg.reshape(S, 2)
        IA = self.I.copy()
        pA = np.array([crf(self.v[i]) @ self.I[i] @ self.v[i] for i in range(S)])
        if fext is not None:
            pA -= fext
        U = np.zeros((S, 6, 2)); D = np.zeros((S, 2, 2)); u = np.zeros((S, 2))
        for i in range(S - 1, -1, -1):
            U[i] = IA[i] @ self.s[i]
            D[i] = self.s[i].T @ U[i] + np.diag(dg[i])
            u[i] = tau[i] - self.s[i].T @ pA[i]
            par = t.parent[i]
            if par >= 0:
                Di = np.linalg.inv(D[i])
                Ia = IA[i] - U[i] @ Di @ U[i].T
                IA[par] += Ia
                pA[par] += pA[i] + Ia @ self.c[i] + U[i] @ Di @ u[i]
        a = np.zeros((S, 6))
        qdd = np.zeros((S, 2))
        a_base = np.concatenate([np.zeros(3), -np.asarray(gravity)])
        for i in range(S):
            ap = a_base if t.parent[i] < 0 else a[t.parent[i]]
            a1 = ap + self.c[i]
            qdd[i] = np.linalg.solve(D[i], u[i] - U[i].T @ a1)
            a[i] = a1 + self.s[i] @ qdd[i]
        return qdd.reshape(-1), D


@pytest.mark.parametrize("seed,S", [(51, 1), (52, 5), (53, 14), (54, 30)])
def test_articulated_pivots_equal_ltdl_pivots(seed, S):
    t = random_small_tree(seed, S)
    o = Oracle(assemble([t]), step_constants())
    rng = np.random.default_rng(seed)
    q = rng.uniform(-0.4, 0.4, 2 * S)
    dg = rng.uniform(0.0, 0.5, 2 * S)
    _, D2 = ABA(o, t, q, np.zeros(2 * S)).solve(np.zeros(2 * S), dg)
    Dl = o.ltdl_pivots(0, q, dg)
    # leaf-first: the second DoF of a joint is eliminated first, so its pivot is the
    # (1, 1) entry of the joint's 2x2 pivot and the first DoF's is the Schur complement
    ref = np.zeros(2 * S)
    ref[1::2] = D2[:, 1, 1]
    ref[0::2] = D2[:, 0, 0] - D2[:, 0, 1] ** 2 / D2[:, 1, 1]
    assert np.max(np.abs(Dl - ref) / np.abs(ref)) < 1e-12


@pytest.mark.parametrize("seed,S", [(61, 3), (62, 12), (63, 40)])
def test_articulated_body_forward_dynamics_equals_mass_matrix_solve(seed, S):
    t = random_small_tree(seed, S)
    o = Oracle(assemble([t]), step_constants())
    rng = np.random.default_rng(seed)
    n = 2 * S
    q, qd, tau = rng.uniform(-0.4, 0.4, n), rng.uniform(-2, 2, n), rng.normal(0, 1, n)
    dg = rng.uniform(0.0, 0.1, n)
    W = np.zeros((S, 6))
    W[:, :3] = rng.normal(0, 2, (S, 3))
    W[:, 3:] = rng.normal(0, 0.2, (S, 3))
    aba = ABA(o, t, q, qd)
    R, p = o.fk(0, q)
    fext = np.zeros((S, 6))
    for i in range(S):  # wrench at the COM as a spatial force at the origin
        com = p[i] + R[i][:, 2] * t.length[i] / 2
        fext[i, :3] = W[i, 3:] + np.cross(com, W[i, :3])
        fext[i, 3:] = W[i, :3]
    qdd_aba, _ = aba.solve(tau, dg, fext)
    H = o.mass_matrix(0, q) + np.diag(dg)
    c = o.inverse_dynamics(0, q, qd, np.zeros(n), wrench=W)
    qdd_ref = np.linalg.solve(H, tau - c)
    assert np.max(np.abs(qdd_aba - qdd_ref)) < 1e-11 * np.max(np.abs(qdd_ref))


def test_articulated_body_forward_dynamics_equals_the_step():
    # the step's joint accelerations (q' after one step) against ABA with the implicit
    # spring/damper terms: tau = -Kp (q + h q') - Kd q', dg = h Kd + h^2 Kp
    t = random_small_tree(71, 20)
    S, n, h = 20, 40, 1e-3
    o = Oracle(assemble([t]), step_constants())
    d = o.derived()
    rng = np.random.default_rng(71)
    st = o.rest_state()
    st.q[:] = rng.uniform(-0.05, 0.05, (S, 2))
    st.qd[:] = rng.uniform(-1, 1, (S, 2))
    q, qd = st.q.reshape(-1).copy(), st.qd.reshape(-1).copy()
    o.rollout(st, 1)
    qdd_step = (st.qd.reshape(-1) - qd) / h
    kp, kd = np.repeat(d["kp"], 2), np.repeat(d["kd"], 2)
    qdd_aba, _ = ABA(o, t, q, qd).solve(-kp * (q + h * qd) - kd * qd, h * kd + h * h * kp)
    assert np.max(np.abs(qdd_step - qdd_aba)) < 1e-9 * np.max(np.abs(qdd_aba))


# ------------------------------------------------------------------------------------------
# energy decay of the implicit step in the linear regime
# ------------------------------------------------------------------------------------------
def test_linear_regime_energy_decay_per_mode():
    t = random_small_tree(81, 6)
    t.youngs[:] = 2e8
    o = Oracle(assemble([t]), step_constants(gravity=(0.0, 0.0, 0.0)))
    d = o.derived()
    S, n, h = 6, 12, 1e-3
    kp = np.repeat(d["kp"], 2)
    H0 = o.mass_matrix(0, np.zeros(n))
    w2, V = scipy.linalg.eigh(np.diag(kp), H0)      # V^T H0 V = I
    rng = np.random.default_rng(8)
    amp = 1e-5
    q0 = amp * rng.uniform(-1, 1, n)
    qd0 = amp * 30 * rng.uniform(-1, 1, n)
    a, b = V.T @ H0 @ q0, V.T @ H0 @ qd0           # modal coordinates
    Ek0 = 0.5 * (b ** 2 + w2 * a ** 2)
    st = o.rest_state()
    st.q[:] = q0.reshape(S, 2)
    st.qd[:] = qd0.reshape(S, 2)
    E0 = Ek0.sum()
    for nstep in (1, 10, 100, 400):
        while o.batch and st.step < nstep:
            o.rollout(st, 1, kp=d["kp"], kd=np.zeros(S))
        q, qd = st.q.reshape(-1), st.qd.reshape(-1)
        E = 0.5 * qd @ o.mass_matrix(0, q) @ qd + 0.5 * np.sum(kp * q * q)
        E_pred = np.sum(Ek0 * (1 + h * h * w2) ** (-nstep))
        assert abs(E - E_pred) < 1e-6 * E0, (nstep, E, E_pred)
    # the decay is real: the stiffest mode lost a measurable fraction
    assert E_pred < 0.999 * E0


# ------------------------------------------------------------------------------------------
# renumbering invariance
# ------------------------------------------------------------------------------------------
def permute_tree(t: TreeDesc, rng, keep_sibling_order=False):
    """A random parent-before-child renumbering of t (and a shuffle of its apples).
    keep_sibling_order: children of a node and apples of a segment keep their relative
    order (so a breadth-first renumbering of the result reproduces t's order)."""
    S = t.n_seg
    kids = [[] for _ in range(S)]
    for i in range(1, S):
        kids[t.parent[i]].append(i)
    ready, order = [0], []
    while ready:
        k = int(rng.integers(len(ready)))
        i = ready.pop(k)
        order.append(i)
        if keep_sibling_order:
            if kids[i]:
                # only the first unvisited child becomes ready; each child frees its sibling
                ready.append(kids[i][0])
        else:
            ready.extend(kids[i])
        if keep_sibling_order and t.parent[i] >= 0:
            sib = kids[t.parent[i]]
            j = sib.index(i)
            if j + 1 < len(sib):
                ready.append(sib[j + 1])
    order = np.asarray(order)
    assert sorted(order.tolist()) == list(range(S))
    new_of = np.empty(S, np.int64)
    new_of[order] = np.arange(S)
    parent = np.array([-1 if t.parent[o] < 0 else new_of[t.parent[o]] for o in order], np.int32)
    assert np.all(parent < np.arange(S))
    A = t.n_apple
    if keep_sibling_order:
        aperm = np.argsort(new_of[t.apple_seg], kind="stable")
    else:
        aperm = rng.permutation(A)
    tp = TreeDesc(parent=parent, rest_quat=t.rest_quat[order], length=t.length[order], radius=t.radius[order],
                  density=t.density[order], youngs=t.youngs[order], mor=t.mor[order],
                  apple_seg=new_of[t.apple_seg[aperm]].astype(np.int32), apple_hang=t.apple_hang[aperm],
                  apple_mass=t.apple_mass[aperm], apple_radius=t.apple_radius[aperm],
                  apple_detach=t.apple_detach[aperm], seed=t.seed)
    return tp, order, aperm


def test_segment_renumbering_changes_nothing_but_rounding():
    t = gen_tree(91, 120, 14)
    rng = np.random.default_rng(9)
    tp, order, aperm = permute_tree(t, rng)
    depth = np.zeros(tp.n_seg, int)
    for i in range(1, tp.n_seg):
        depth[i] = depth[tp.parent[i]] + 1
    assert np.any(np.diff(depth) < 0)       # not breadth-first
    F = np.zeros((t.n_apple, 3))
    F[:4] = [[30, 0, 0], [0, 0, -20], [5, 5, 5], [0, -26, 3]]
    c = step_constants(rng_seed=5, wrench_fraction=0.0)
    o1, o2 = Oracle(assemble([t]), c), Oracle(assemble([tp]), c)
    s1, s2 = o1.rest_state(), o2.rest_state()
    o1.rollout(s1, 400, aforce=F)
    o2.rollout(s2, 400, aforce=F[aperm])
    assert np.max(np.abs(s2.q - s1.q[order])) < 1e-12 * np.max(np.abs(s1.q))
    assert np.max(np.abs(s2.qd - s1.qd[order])) < 1e-11 * np.max(np.abs(s1.qd))
    assert np.max(np.abs(s2.ax - s1.ax[aperm])) < 1e-12 * np.max(np.abs(s1.ax))
    assert np.max(np.abs(s2.av - s1.av[aperm])) < 1e-11 * np.max(np.abs(s1.av))
    assert np.array_equal(s2.det_step, s1.det_step[aperm]) and (s1.det_step >= 0).sum() >= 2
    assert np.array_equal(s2.break_step, s1.break_step[order])


# ------------------------------------------------------------------------------------------
# tangent-linear vs reverse mode of one step (switches frozen)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["plain", "switches"])
def test_step_tangent_and_adjoint_dot_product(case):
    t = gen_tree(95, 40, 8)
    S, A = t.n_seg, t.n_apple
    over = {}
    if case == "switches":
        # random body forces on every segment, large enough to hit the impulse cap;
        # a lowered reaction clamp
        over = dict(rng_seed=17, wrench_fraction=1.0, wrench_sigma=400.0, react_max_factor=0.3)
    o = Oracle(assemble([t]), step_constants(**over))
    d = o.derived()
    rng = np.random.default_rng(3)
    st = o.rest_state()
    F = rng.normal(0, 3, (A, 3))
    o.rollout(st, 30, aforce=F)
    broken0 = det0 = None
    if case == "switches":
        broken0 = np.zeros(S, np.uint8); broken0[[7, 20]] = 1      # two free hinges (one sub-tree snapped)
        det0 = np.zeros(A, np.uint8); det0[2] = 1                  # one detached fruit (absolute position)
        st.ax[2] = st.ax[2] + np.array([0.3, -0.1, 1.5])
        F[0] = [0.0, 0.0, -14.0]                                   # stretches apple 0's stem past the clamp
    x = np.concatenate([st.q.reshape(-1), st.qd.reshape(-1), st.ax.reshape(-1), st.av.reshape(-1)])
    vx = rng.normal(0, 1, x.size) * np.concatenate([np.full(4 * S, 1e-2), np.full(6 * A, 1e-3)])
    vkp, vkd = rng.normal(0, 1, S) * d["kp"] * 1e-2, rng.normal(0, 1, S) * d["kd"] * 1e-2
    vF = rng.normal(0, 1, (A, 3))
    w = rng.normal(0, 1, x.size)
    a, b = o.step_dot(0, st.step, x, d["kp"], d["kd"], F, vx, vkp, vkd, vF, w, broken0, det0)
    assert abs(a - b) < 1e-12 * max(abs(a), abs(b)), (a, b)
    assert abs(a) > 0
    sw = o.last_switch_counts
    if case == "switches":
        assert sw["broken"] == 2 and sw["detached"] == 1 and sw["clamped"] >= 1 and sw["capped"] >= 10, sw
    else:
        assert sum(sw.values()) == 0, sw
