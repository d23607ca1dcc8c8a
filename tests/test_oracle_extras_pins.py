"""Pins of the oracle's model variants and extras against independent computations.

* Per-level exponential stiffness (Sec. "Compliant branch dynamics"): the settled tip
  deflection of an N-link cantilever with joint stiffnesses k0 gamma^j equals the sum
  over joints of P (L - x_j)^2 / Kp_j, the discrete chain's small-load closed form.
* Translational fruit (Sec. "Fruit"): the fruit's position and velocity do not depend on
  its orientation state (bitwise equal to the full rigid body); a full body spinning at
  a constant rate turns its quaternion by exp(w t / 2) exactly.
* Drag, post-break friction, power fade and speed brake (Sec. "Compliant branch
  dynamics", Sec. "Branch breaking", Sec. "Numerical Stability"): a single link swinging
  about one joint axis is a one-degree-of-freedom system; the implicit step of the tree
  reduces to a scalar recursion that the tests write out independently
  ((J + h kd + h^2 kp) a = -kp (th + h w) - kd w + tau, w+ = w + h a, th+ = th + h w+)
  and the oracle must follow it to rounding.  Physical checks on top: the broken limb
  falls, swings and is then held (it creeps no faster than the friction's damper
  regime allows); the faded force never drives a body beyond twice the fade speed; the
  brake holds it near the speed limit.
CPU only.
"""
import math

import numpy as np

from orchard_inputs import EXTRAS_ON, assemble, chain_tree, gen_tree, pull_forces, step_constants
from oracle.oracle import Oracle

G = 9.81


def one(tree, **over):
    return Oracle(assemble([tree]), step_constants(**over))


def qrot(axis, ang):
    s = math.sin(ang / 2)
    return (math.cos(ang / 2), axis[0] * s, axis[1] * s, axis[2] * s)


# ------------------------------------------------------------------------------------------
# per-level exponential stiffness
# ------------------------------------------------------------------------------------------
def test_exponential_stiffness_cantilever():
    N, L, r = 12, 1.2, 0.012
    l = L / N
    k0, gam = 2.0e3, 0.8
    t = chain_tree(N, length=l, radius=r, root_quat=qrot((0, 1, 0), math.pi / 2))
    o = one(t, gravity=(0.0, 0.0, 0.0), stiffness_k0=k0, stiffness_gamma=gam)
    d = o.derived()
    kp_expect = k0 * gam ** np.arange(N)          # the chain's joint j sits j levels down
    assert np.allclose(d["kp"], kp_expect, rtol=1e-14, atol=0)
    x = l * np.arange(N)                          # joint positions along the chain
    P = 1e-4 * np.min(kp_expect) / L              # small load: deflection ~1e-4 L
    W = np.zeros((N, 6))
    W[-1, 2] = P
    W[-1, 3:] = np.cross([l / 2, 0, 0], [0, 0, P])
    exact = np.sum(P * (L - x) ** 2 / kp_expect)
    st = o.rest_state()
    o.rollout(st, 4000, kp=d["kp"], kd=0.05 * d["kp"], wrench=W)
    R, p = o.fk(0, st.q.reshape(-1))
    tip = p[-1] + R[-1] @ np.array([0, 0, l])
    assert np.max(np.abs(st.qd)) < 1e-9
    assert abs(tip[2] - exact) < 1e-4 * exact     # small-angle closed form; nonlinearity ~1e-4
    # the Eq.-beam chain of the same geometry is far stiffer at the tip joints: the variant
    # really changes the model
    assert abs(tip[2] - exact) < 0.1 * abs(exact - np.sum(P * (L - x) ** 2 / (math.pi / 4 * 9e9 * r ** 4 / l)))


# ------------------------------------------------------------------------------------------
# translational fruit
# ------------------------------------------------------------------------------------------
def test_translational_fruit_equals_full_body_in_position():
    t = gen_tree(44, 70, 9)
    b = assemble([t])
    F = pull_forces(b, fraction=0.6, seed=5)
    out = []
    for dof in (6, 3):
        o = Oracle(b, step_constants(fruit_dof=dof))
        st = o.rest_state()
        o.rollout(st, 300, aforce=F)
        out.append(st)
    s6, s3 = out
    for f in ("q", "qd", "ax", "av", "det_step"):
        assert np.array_equal(getattr(s6, f), getattr(s3, f)), f
    assert (s6.det_step >= 0).sum() >= 1


def test_full_body_fruit_turns_at_constant_rate():
    t = gen_tree(45, 40, 5)
    b = assemble([t])
    h, n = 1e-3, 700
    w = np.array([[3.0, -1.0, 2.0], [0.0, 0.0, 5.0], [0.3, 0.2, -0.1], [0, 0, 0], [10.0, 0, 0]])
    res = {}
    for dof in (6, 3):
        o = Oracle(b, step_constants(fruit_dof=dof))
        st = o.rest_state()
        st.aw[:] = w
        o.rollout(st, n)
        res[dof] = st
    o0 = Oracle(b, step_constants())
    st0 = o0.rest_state()
    o0.rollout(st0, n)
    # the spin does not couple into the fruit's position or velocity
    assert np.array_equal(res[6].ax, st0.ax) and np.array_equal(res[6].av, st0.av)
    # constant angular velocity: q(t) = exp(w t / 2) q(0), q(0) = 1
    for a in range(5):
        th = np.linalg.norm(w[a]) * n * h / 2
        axis = w[a] / np.linalg.norm(w[a]) if np.linalg.norm(w[a]) > 0 else np.zeros(3)
        q = np.concatenate([[math.cos(th)], math.sin(th) * axis])
        assert np.max(np.abs(res[6].aq[a] - q)) < 1e-12, (a, res[6].aq[a], q)
        assert np.array_equal(res[6].aw[a], w[a])
    # the translational fruit has no orientation state to advance
    assert np.array_equal(res[3].aq, np.tile([1.0, 0, 0, 0], (5, 1))) and np.array_equal(res[3].aw, w)


# ------------------------------------------------------------------------------------------
# single link about one joint axis: the scalar recursion of the implicit step
# ------------------------------------------------------------------------------------------
def scalar_run(J, n, th, w, h, kp_of, kd_of, tau_of):
    """n steps of (J + h kd + h^2 kp) a = -kp (th + h w) - kd w + tau(th, w, k)."""
    ths, ws = [], []
    for k in range(n):
        kp, kd, tau = kp_of(k, th, w), kd_of(k, th, w), tau_of(k, th, w)
        a = (-kp * (th + h * w) - kd * w + tau) / (J + h * kd + h * h * kp)
        w = w + h * a
        th = th + h * w
        ths.append(th)
        ws.append(w)
    return np.array(ths), np.array(ws)


def oracle_run(o, n, th0, w0, kp, kd, wrench=None, every=1):
    st = o.rest_state()
    st.q[0, 0], st.qd[0, 0] = th0, w0
    ths, ws, ys = [], [], []
    for _ in range(n // every):
        o.rollout(st, every, kp=kp, kd=kd, wrench=wrench)
        ths.append(st.q[0, 0])
        ws.append(st.qd[0, 0])
        ys.append(abs(st.q[0, 1]) + abs(st.qd[0, 1]))
    return np.array(ths), np.array(ws), max(ys), st


def link(l=0.25, r=0.008, hanging=True, mor=75e6):
    # hanging: the rest frame turns z to -z about x, so the link hangs below its joint
    return chain_tree(1, length=l, radius=r, mor=mor, root_quat=qrot((1, 0, 0), math.pi) if hanging else (1, 0, 0, 0))


def test_drag_on_a_swinging_link():
    l, h = 0.25, 1e-3
    t = link(l)
    c = dict(drag_lin=2.0, drag_ang=3.0)
    o = one(t, **c)
    d = o.derived()
    m, It = d["mass"][0], d["It"][0]
    J = It + m * (l / 2) ** 2
    D = c["drag_lin"] * m * (l / 2) ** 2 + c["drag_ang"] * It
    zero = np.zeros(1)
    th, w, y, _ = oracle_run(o, 1500, 0.4, 0.0, zero, zero)
    sth, sw = scalar_run(J, 1500, 0.4, 0.0, h, lambda *a: 0.0, lambda *a: 0.0,
                         lambda k, th, w: -m * G * l / 2 * math.sin(th) - D * w)
    assert y < 1e-12                              # the motion stays about the one axis
    assert np.max(np.abs(th - sth)) < 1e-12 and np.max(np.abs(w - sw)) < 1e-11
    # gravity off: the exact geometric decay of the swing rate
    o2 = one(t, gravity=(0.0, 0.0, 0.0), **c)
    _, w2, _, _ = oracle_run(o2, 200, 0.0, 1.5, zero, zero)
    assert np.max(np.abs(w2 - 1.5 * (1 - h * D / J) ** np.arange(1, 201))) < 1e-13


def test_broken_limb_falls_swings_and_is_held():
    # a limb held at 1.2 rad from the vertical by a feeble spring loaded past its (tiny)
    # rupture moment from the first step breaks at step N_break - 1 = 4; then its hinge is
    # free (no spring, no damper), its drag is reduced to a tenth and the friction of the
    # torn fibres grows from a quarter of its weight moment to five quarters over 1.5 s
    l, h = 0.25, 1e-3
    t = link(l, mor=1e-6)
    c = dict(EXTRAS_ON, friction_speed=1e-3)
    o = one(t, **c)
    d = o.derived()
    m, It = d["mass"][0], d["It"][0]
    J = It + m * (l / 2) ** 2
    D = c["drag_lin"] * m * (l / 2) ** 2 + c["drag_ang"] * It
    Gm = G * m * l / 2                            # the limb's weight moment about its hinge
    nb = 4
    n = 3000

    def tc(k):
        return c["friction_base"] * Gm * (1 + (c["friction_growth"] - 1) * min(1.0, (k - nb) * h / c["friction_ramp_time"]))

    kp, kd = np.full(1, 1e-6), np.zeros(1)
    kp_of = lambda k, th, w: kp[0] if k < nb else 0.0
    kd_of = lambda k, th, w: 0.0 if k < nb else tc(k) / max(abs(w), c["friction_speed"])
    tau_of = lambda k, th, w: -Gm * math.sin(th) - (1.0 if k < nb else c["drag_snapped"]) * D * w
    th, w, y, st = oracle_run(o, n, 1.2, 0.0, kp, kd)
    sth, sw = scalar_run(J, n, 1.2, 0.0, h, kp_of, kd_of, tau_of)
    assert st.break_step[0] == nb
    assert y < 1e-12
    assert np.max(np.abs(th - sth)) < 1e-11 and np.max(np.abs(w - sw)) < 1e-10
    # it swings through the bottom once ...
    assert np.min(th[:1000]) < 0.0 < th[0]
    # ... and after the ramp it creeps no faster than the damper regime of the friction
    # allows against at most its full weight moment: |w| <= (Gm / tc) friction_speed
    late = np.abs(w[int(2.5 / h):])
    assert np.max(late) <= Gm / tc(n) * c["friction_speed"] * (1 + 1e-9)


def test_power_fade_and_speed_brake():
    l, h = 0.2, 1e-3
    t = link(l, r=0.01, hanging=False)
    F0 = 0.5
    W = np.zeros((1, 6))
    W[0, 1] = -F0                                  # world force at the centre of mass
    zero = np.zeros(1)
    for c, bound in ((dict(fade_speed=0.5), None), (dict(brake_rate=50.0, v_cap=0.6), "brake")):
        o = one(t, gravity=(0.0, 0.0, 0.0), **c)
        d = o.derived()
        m, It = d["mass"][0], d["It"][0]
        J = It + m * (l / 2) ** 2
        vf, vcap, beta = c.get("fade_speed", 0.0), c.get("v_cap", 1.0), c.get("brake_rate", 0.0)

        def tau(k, th, w):
            dvec = np.array([0.0, -math.sin(th), math.cos(th)])      # link axis
            tang = np.array([0.0, -math.cos(th), -math.sin(th)])     # d(dvec)/d(th)
            F = np.array([0.0, -F0, 0.0])
            sp = abs(w) * l / 2
            if sp > 0:
                u = math.copysign(1.0, w) * tang
                fu = F @ u
                if vf > 0 and fu > 0 and sp > vf:
                    phi = max(0.0, 1 - (sp - vf) / vf)
                    F = F - (1 - phi) * fu * u
                if beta > 0 and sp > vcap:
                    F = F - beta * m * (sp - vcap) * u
            nF = np.linalg.norm(F)
            cap = m * vcap / h
            if nF > cap:
                F = F * cap / nF
            return np.cross(l / 2 * dvec, F)[0]

        th, w, y, _ = oracle_run(o, 2000, 0.0, 0.0, zero, zero, wrench=W)
        sth, sw = scalar_run(J, 2000, 0.0, 0.0, h, lambda *a: 0.0, lambda *a: 0.0, tau)
        assert y < 1e-12
        assert np.max(np.abs(th - sth)) < 1e-10 and np.max(np.abs(w - sw)) < 1e-10
        sp = np.abs(w) * l / 2
        if bound is None:
            # the push fades out: never beyond twice the fade speed (plus one step of it)
            assert 1.5 * vf < np.max(sp) <= 2 * vf + h * F0 / m * (l / 2) ** 2 * m / J
        else:
            # the brake balances the push a little above the limit
            assert vcap < np.max(sp) <= vcap + F0 / (beta * m) * 1.05
