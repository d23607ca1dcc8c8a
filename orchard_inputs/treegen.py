"""Seeded synthetic apple-tree descriptions.

This module is the ONLY code shared by the FP64 oracle and the HIP path.  It
draws inputs -- topology, rest frames, segment dimensions, wood properties and
fruit placement -- and contains none of the arithmetic of the dynamics step
(no masses, stiffnesses, inertias, kinematics or forces).

The tree grammar follows the paper's description of its default stochastic
apple-tree generator (Sec. "Tree Generation", paragraph "Grammar"): a vertical
central leader emits a phyllotactic spiral of 3-6 scaffold limbs at crotch
angles of 42-65 degrees from vertical, every other axis forks into a small
number of laterals, laterals droop, buds abort with some probability.  The
paper does not publish its grammar's parameters or seeds, so the numbers below
are this project's own budgeted version (exactly ``n_seg`` internodes):

* axes are chains of U{3..6} internodes, grown breadth-first over buds;
* the leader ends in 3-6 scaffold buds (crotch U(42, 65) deg, divergence
  137.5 +- 10 deg) plus a vertical continuation bud;
* other axes fork at their end into 2 or 3 buds (p = 1/2) at U(20, 45) deg,
  divergence 137.5 deg (golden angle, Sec. "Tree Generation");
* each bud aborts with p = 0.15 unless that would stop growth early;
* lateral internodes droop by U(0, 6) deg toward -z;
* segment lengths U(0.05, 0.3) m; radii from the pipe model (Eq. pipe)
  r_i = r_trunk * (n_tips(i) / n_tips(root))^(1/beta), beta = 2.25, which
  meets r_parent^beta = sum r_child^beta at every fork exactly;
* wood: density 800 kg/m^3, E ~ U(7, 11) GPa and modulus of rupture
  ~ U(60, 90) MPa drawn once per tree;
* apples on leaf segments, drawn without replacement with weight
  proportional to rest height (outer-canopy bias, Sec. "Fruit"), mass
  U(0.15, 0.25) kg, detach force U(15, 25) N, radius 0.035 m, hung at the
  segment tip (0, 0, l) in the segment frame.

Segments are returned in breadth-first (level) order: parent < child, every
level is a contiguous index range and the children of a segment are
contiguous.  Rest frames are quaternions (w, x, y, z); ``rest_quat[i]`` is
q_rel = conj(Q_parent) * Q_child, the joint rest rotation of the paper's
joint-frame equation (Sec. "Physical Model"); for a root it is the world
orientation.
"""
from __future__ import annotations

import math
from collections import deque
from dataclasses import dataclass, field

import numpy as np

DEG = math.pi / 180.0
GOLDEN_DEG = 137.5


# --- small quaternion helpers (input geometry only) -------------------------
def _qmul(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return (aw * bw - ax * bx - ay * by - az * bz,
            aw * bx + ax * bw + ay * bz - az * by,
            aw * by - ax * bz + ay * bw + az * bx,
            aw * bz + ax * by - ay * bx + az * bw)


def _qaxis(axis, ang):
    s = math.sin(0.5 * ang)
    return (math.cos(0.5 * ang), axis[0] * s, axis[1] * s, axis[2] * s)


def _qrot(q, v):
    w, x, y, z = q
    # v' = v + 2w (u x v) + 2 u x (u x v), u = (x, y, z)
    cx = y * v[2] - z * v[1]
    cy = z * v[0] - x * v[2]
    cz = x * v[1] - y * v[0]
    ccx = y * cz - z * cy
    ccy = z * cx - x * cz
    ccz = x * cy - y * cx
    return (v[0] + 2 * (w * cx + ccx), v[1] + 2 * (w * cy + ccy), v[2] + 2 * (w * cz + ccz))


def _qconj(q):
    return (q[0], -q[1], -q[2], -q[3])


def _qnormalize(q):
    n = math.sqrt(sum(c * c for c in q))
    return tuple(c / n for c in q)


@dataclass
class TreeDesc:
    """One tree: arrays in breadth-first segment order (see module docstring)."""
    parent: np.ndarray          # int32 [S], -1 = attached to the world origin
    rest_quat: np.ndarray       # float64 [S, 4]
    length: np.ndarray          # float64 [S]  (m)
    radius: np.ndarray          # float64 [S]  (m)
    density: np.ndarray         # float64 [S]  (kg/m^3)
    youngs: np.ndarray          # float64 [S]  (Pa)
    mor: np.ndarray             # float64 [S]  (Pa)
    apple_seg: np.ndarray       # int32 [A]   tree-local segment index
    apple_hang: np.ndarray      # float64 [A, 3] hang point in the segment frame
    apple_mass: np.ndarray      # float64 [A]
    apple_radius: np.ndarray    # float64 [A]
    apple_detach: np.ndarray    # float64 [A]  detach force threshold (N)
    seed: int = 0
    stats: dict = field(default_factory=dict)

    @property
    def n_seg(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_apple(self) -> int:
        return int(self.apple_seg.shape[0])


def depth_stats(parent: np.ndarray) -> dict:
    """Level statistics of a parent array in parent<child order."""
    S = parent.shape[0]
    depth = np.zeros(S, dtype=np.int64)
    for i in range(S):
        p = parent[i]
        depth[i] = 0 if p < 0 else depth[p] + 1
    widths = np.bincount(depth)
    n_child = np.bincount(parent[parent >= 0], minlength=S)
    return dict(max_depth=int(depth.max()) + 1 if S else 0,
                mean_depth=float(depth.mean() + 1) if S else 0.0,
                widest_level=int(widths.max()) if S else 0,
                n_tips=int((n_child == 0).sum()))


def gen_tree(seed: int, n_seg: int, n_apple: int, *, trunk_radius: float = 0.04,
             beta: float = 2.25, density: float = 800.0,
             youngs_range=(7e9, 11e9), mor_range=(60e6, 90e6),
             length_range=(0.05, 0.3), apple_mass_range=(0.15, 0.25),
             apple_detach_range=(15.0, 25.0), apple_radius: float = 0.035) -> TreeDesc:
    """Draw one tree with exactly ``n_seg`` segments and ``n_apple`` apples."""
    if n_seg < 1:
        raise ValueError("n_seg must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    youngs = float(rng.uniform(*youngs_range))
    mor = float(rng.uniform(*mor_range))
    droop_all = rng.uniform(0.0, 6.0 * DEG, size=n_seg)

    # creation-order arrays
    par: list[int] = []
    quat: list[tuple] = []
    kind_leader, kind_scaffold, kind_lateral = 0, 1, 2
    ident = (1.0, 0.0, 0.0, 0.0)
    queue = deque([(-1, ident, kind_leader)])
    ez = (0.0, 0.0, 1.0)
    while len(par) < n_seg:
        if not queue:  # cannot happen (abortion never empties the queue) but stay safe
            queue.append((len(par) - 1, quat[-1], kind_lateral))
        parent, Q, kind = queue.popleft()
        k = int(rng.integers(3, 7))
        for j in range(k):
            if len(par) == n_seg:
                break
            if kind != kind_leader and j > 0:
                h = _qrot(Q, ez)
                ax = (h[1] * -1.0 - h[2] * 0.0, h[2] * 0.0 - h[0] * -1.0, 0.0)  # h x (-z)
                n = math.hypot(ax[0], ax[1])
                if n > 1e-9:
                    Q = _qnormalize(_qmul(_qaxis((ax[0] / n, ax[1] / n, 0.0),
                                                 float(droop_all[len(par)])), Q))
            par.append(parent)
            quat.append(Q)
            parent = len(par) - 1
        if len(par) == n_seg:
            break
        children = []
        phi0 = float(rng.uniform(0.0, 2 * math.pi))
        if kind == kind_leader:
            n_sc = int(rng.integers(3, 7))
            az = phi0
            for _ in range(n_sc):
                crotch = float(rng.uniform(42.0, 65.0)) * DEG
                Qc = _qmul(Q, _qmul(_qaxis(ez, az), _qaxis((1.0, 0.0, 0.0), crotch)))
                children.append((parent, _qnormalize(Qc), kind_scaffold))
                az += (GOLDEN_DEG + float(rng.uniform(-10.0, 10.0))) * DEG
            children.append((parent, Q, kind_leader))
        else:
            nf = 2 if rng.random() < 0.5 else 3
            for f in range(nf):
                ang = float(rng.uniform(20.0, 45.0)) * DEG
                az = phi0 + f * GOLDEN_DEG * DEG
                Qc = _qmul(Q, _qmul(_qaxis(ez, az), _qaxis((1.0, 0.0, 0.0), ang)))
                children.append((parent, _qnormalize(Qc), kind_lateral))
        kept = [c for c in children if rng.random() >= 0.15]
        if not kept and not queue:
            kept = [children[0]]
        queue.extend(kept)

    S = n_seg
    # breadth-first renumbering (children visited in creation order)
    kids: list[list[int]] = [[] for _ in range(S)]
    roots = []
    for i, p in enumerate(par):
        (kids[p] if p >= 0 else roots).append(i)
    order = []
    dq = deque(roots)
    while dq:
        i = dq.popleft()
        order.append(i)
        dq.extend(kids[i])
    new_of = np.empty(S, dtype=np.int64)
    new_of[np.asarray(order)] = np.arange(S)
    parent = np.array([-1 if par[o] < 0 else new_of[par[o]] for o in order], dtype=np.int32)
    Qw = [quat[o] for o in order]

    length = rng.uniform(length_range[0], length_range[1], size=S)
    rest = np.empty((S, 4))
    for i in range(S):
        p = parent[i]
        rest[i] = Qw[i] if p < 0 else _qnormalize(_qmul(_qconj(Qw[p]), Qw[i]))

    # pipe-model radii from tip counts
    n_child = np.bincount(parent[parent >= 0], minlength=S)
    tips = (n_child == 0).astype(np.float64)
    for i in range(S - 1, 0, -1):
        if parent[i] >= 0:
            tips[parent[i]] += tips[i]
    root_tips = tips[0]
    radius = trunk_radius * (tips / root_tips) ** (1.0 / beta)

    # rest tip heights for the fruit-placement weight
    base = np.zeros((S, 3))
    tip_z = np.zeros(S)
    for i in range(S):
        p = parent[i]
        if p >= 0:
            base[i] = base[p] + np.asarray(_qrot(Qw[p], (0.0, 0.0, length[p])))
        tip_z[i] = base[i][2] + _qrot(Qw[i], (0.0, 0.0, length[i]))[2]
    leaves = np.flatnonzero(n_child == 0)
    w = np.maximum(tip_z[leaves], 0.01)
    w = w / w.sum()
    if n_apple <= leaves.size:
        aseg = rng.choice(leaves, size=n_apple, replace=False, p=w)
    else:
        first = rng.permutation(leaves)
        extra = rng.choice(leaves, size=n_apple - leaves.size, replace=True, p=w)
        aseg = np.concatenate([first, extra])
    aseg = np.sort(aseg).astype(np.int32)
    A = aseg.size
    hang = np.zeros((A, 3))
    hang[:, 2] = length[aseg]
    desc = TreeDesc(parent=parent, rest_quat=rest, length=length, radius=radius,
                    density=np.full(S, density), youngs=np.full(S, youngs),
                    mor=np.full(S, mor), apple_seg=aseg, apple_hang=hang,
                    apple_mass=rng.uniform(*apple_mass_range, size=A),
                    apple_radius=np.full(A, apple_radius),
                    apple_detach=rng.uniform(*apple_detach_range, size=A), seed=seed)
    desc.stats = depth_stats(parent)
    desc.stats.update(n_seg=S, n_apple=A, r_tip=float(radius.min()))
    return desc


def ternary_lsystem_count(n: int) -> int:
    """Body count of the deterministic ternary L-system of Eq. lsystem after n
    derivations, obtained by literally rewriting the bracketed string.

    Axiom: the trunk internode followed by the apex ``A``.  One derivation
    rewrites every ``A`` into ``F [F A] [F A] [F A]`` (the width and angle
    modules carry no bodies, so they are left out).  Each ``F`` is one body.
    """
    s = "FA"
    for _ in range(n):
        s = s.replace("A", "F[FA][FA][FA]")
    return s.count("F")


def chain_tree(n_seg: int, *, length: float, radius: float, youngs: float = 9e9,
               mor: float = 75e6, density: float = 800.0,
               root_quat=(1.0, 0.0, 0.0, 0.0)) -> TreeDesc:
    """Straight chain of identical segments (cantilever / pendulum fixtures)."""
    parent = np.arange(-1, n_seg - 1, dtype=np.int32)
    rest = np.zeros((n_seg, 4))
    rest[:, 0] = 1.0
    rest[0] = root_quat
    z = np.zeros(0)
    return TreeDesc(parent=parent, rest_quat=rest, length=np.full(n_seg, length),
                    radius=np.full(n_seg, radius), density=np.full(n_seg, density),
                    youngs=np.full(n_seg, youngs), mor=np.full(n_seg, mor),
                    apple_seg=np.zeros(0, np.int32), apple_hang=np.zeros((0, 3)),
                    apple_mass=z, apple_radius=z, apple_detach=z)


def random_small_tree(seed: int, n_seg: int, n_apple: int = 0) -> TreeDesc:
    """Tiny random tree (random parents, random rest rotations) for brute-force pins."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parent = np.empty(n_seg, dtype=np.int32)
    parent[0] = -1
    for i in range(1, n_seg):
        parent[i] = rng.integers(0, i)
    # keep breadth-first order: sort by depth, stable
    d = np.zeros(n_seg, dtype=np.int64)
    for i in range(1, n_seg):
        d[i] = d[parent[i]] + 1
    kids = [[] for _ in range(n_seg)]
    for i in range(1, n_seg):
        kids[parent[i]].append(i)
    order, dq = [], deque([0])
    while dq:
        i = dq.popleft()
        order.append(i)
        dq.extend(kids[i])
    new_of = np.empty(n_seg, dtype=np.int64)
    new_of[np.asarray(order)] = np.arange(n_seg)
    parent = np.array([-1 if parent[o] < 0 else new_of[parent[o]] for o in order], np.int32)
    rest = rng.normal(size=(n_seg, 4))
    rest /= np.linalg.norm(rest, axis=1, keepdims=True)
    length = rng.uniform(0.05, 0.3, n_seg)
    radius = rng.uniform(0.004, 0.03, n_seg)
    aseg = np.sort(rng.integers(0, n_seg, n_apple)).astype(np.int32)
    hang = np.zeros((n_apple, 3))
    hang[:, 2] = length[aseg]
    return TreeDesc(parent=parent, rest_quat=rest, length=length, radius=radius,
                    density=np.full(n_seg, 800.0), youngs=rng.uniform(7e9, 11e9, n_seg),
                    mor=rng.uniform(60e6, 90e6, n_seg), apple_seg=aseg, apple_hang=hang,
                    apple_mass=rng.uniform(0.15, 0.25, n_apple),
                    apple_radius=np.full(n_apple, 0.035),
                    apple_detach=rng.uniform(15.0, 25.0, n_apple), seed=seed)
