"""Workload presets and batch assembly for the synthetic orchard inputs.

The five workloads (named by what they are):

* ``single64``  - one tree, seed 0, 64 segments, 8 apples, gravity only, 1000 steps.
* ``pull1024``  - 1024 trees, S ~ U{100..400}, A ~ U{20..80}; 10 % of apples are
  pulled by a constant 0-30 N force in a random direction from step 200.
* ``uneven8192``- 8192 trees, S = round(exp(U(ln 50, ln 1500))), A ~ U{10..120};
  random body wrenches drawn inside the step (see the step's RNG spec).
* ``grad512``   - 512 trees of 300 segments and 40 apples (differentiable rollout).
* ``row64x16k`` - 64 trees of 5000 segments / 400 apples plus 16384 trees of
  80 segments / 8 apples.

Tree ``e`` of workload number ``c`` (1..5 in the order above) uses seed
``10**6 * c + e``; the single-tree workload uses seed 0.  Sizes are drawn from
the tree's own seed so any tree can be regenerated alone.

Per-step force inputs (pulls, per-step apple forces) are generated here too, as
plain seeded arrays; random numbers drawn *inside* the step (body wrenches of
``uneven8192``) are not: each side implements the counter-based generator.
"""
from __future__ import annotations

import math
import multiprocessing
import os
import sys
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass

import numpy as np

from .treegen import TreeDesc, gen_tree

WORKLOADS = ("single64", "pull1024", "uneven8192", "grad512", "row64x16k")


def _sizes(name: str, e: int):
    c = WORKLOADS.index(name) + 1
    if name == "single64":
        return 0, 64, 8
    seed = 10**6 * c + e
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5EED))
    if name == "pull1024":
        return seed, int(rng.integers(100, 401)), int(rng.integers(20, 81))
    if name == "uneven8192":
        S = int(round(math.exp(rng.uniform(math.log(50), math.log(1500)))))
        return seed, S, int(rng.integers(10, 121))
    if name == "grad512":
        return seed, 300, 40
    if name == "row64x16k":
        return (seed, 5000, 400) if e < 64 else (seed, 80, 8)
    raise KeyError(name)


def n_trees(name: str) -> int:
    return {"single64": 1, "pull1024": 1024, "uneven8192": 8192, "grad512": 512,
            "row64x16k": 64 + 16384}[name]


def _gen_one(args):
    seed, S, A = args
    return gen_tree(seed, S, A)


def make_trees(name: str, env_ids=None, workers: int | None = None) -> list[TreeDesc]:
    """Generate the trees of a workload (all, or the listed env indices)."""
    if env_ids is None:
        env_ids = range(n_trees(name))
    jobs = [_sizes(name, int(e)) for e in env_ids]
    if workers is None:
        # ORCHARD_GEN_WORKERS=1 generates in this process (e.g. under a profiler whose
        # signal handlers a fork server's workers cannot inherit)
        workers = int(os.environ.get("ORCHARD_GEN_WORKERS", min(8, os.cpu_count() or 1)))
    # the fork server re-imports the main script in its workers: without one (an
    # interactive session, a script on stdin) the trees are generated here
    main_file = getattr(sys.modules.get("__main__"), "__file__", None)
    if len(jobs) < 64 or workers <= 1 or not main_file or not os.path.exists(main_file):
        return [_gen_one(j) for j in jobs]
    # workers come from a fork server (a fresh interpreter), never forked from a caller
    # that may already hold a GPU context
    ctx = multiprocessing.get_context("forkserver")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        return list(ex.map(_gen_one, jobs, chunksize=max(1, len(jobs) // (8 * workers))))


@dataclass
class Batch:
    """Flat CSR batch of trees (the layout of the C descriptor)."""
    seg_offset: np.ndarray      # int32 [B+1]
    seg_parent: np.ndarray      # int32 [S_tot] env-local
    seg_rest_quat: np.ndarray   # float64 [S_tot, 4]
    seg_length: np.ndarray
    seg_radius: np.ndarray
    seg_density: np.ndarray
    seg_youngs: np.ndarray
    seg_mor: np.ndarray
    apple_offset: np.ndarray    # int32 [B+1]
    apple_seg: np.ndarray       # int32 [A_tot] env-local
    apple_hang: np.ndarray      # float64 [A_tot, 3]
    apple_mass: np.ndarray
    apple_radius: np.ndarray
    apple_detach: np.ndarray

    @property
    def n_env(self) -> int:
        return int(self.seg_offset.shape[0] - 1)

    @property
    def n_seg(self) -> int:
        return int(self.seg_offset[-1])

    @property
    def n_apple(self) -> int:
        return int(self.apple_offset[-1])

    def tree(self, e: int) -> TreeDesc:
        s0, s1 = self.seg_offset[e], self.seg_offset[e + 1]
        a0, a1 = self.apple_offset[e], self.apple_offset[e + 1]
        return TreeDesc(parent=self.seg_parent[s0:s1], rest_quat=self.seg_rest_quat[s0:s1],
                        length=self.seg_length[s0:s1], radius=self.seg_radius[s0:s1],
                        density=self.seg_density[s0:s1], youngs=self.seg_youngs[s0:s1],
                        mor=self.seg_mor[s0:s1], apple_seg=self.apple_seg[a0:a1],
                        apple_hang=self.apple_hang[a0:a1], apple_mass=self.apple_mass[a0:a1],
                        apple_radius=self.apple_radius[a0:a1],
                        apple_detach=self.apple_detach[a0:a1])


def assemble(trees: list[TreeDesc]) -> Batch:
    so = np.zeros(len(trees) + 1, dtype=np.int32)
    ao = np.zeros(len(trees) + 1, dtype=np.int32)
    so[1:] = np.cumsum([t.n_seg for t in trees])
    ao[1:] = np.cumsum([t.n_apple for t in trees])
    cat = lambda f: np.ascontiguousarray(np.concatenate([getattr(t, f) for t in trees]))
    return Batch(seg_offset=so, seg_parent=cat("parent").astype(np.int32),
                 seg_rest_quat=cat("rest_quat").reshape(-1, 4), seg_length=cat("length"),
                 seg_radius=cat("radius"), seg_density=cat("density"), seg_youngs=cat("youngs"),
                 seg_mor=cat("mor"), apple_offset=ao, apple_seg=cat("apple_seg").astype(np.int32),
                 apple_hang=cat("apple_hang").reshape(-1, 3), apple_mass=cat("apple_mass"),
                 apple_radius=cat("apple_radius"), apple_detach=cat("apple_detach"))


def make_batch(name: str, env_ids=None, workers: int | None = None) -> Batch:
    return assemble(make_trees(name, env_ids, workers))


# --- per-step force inputs ----------------------------------------------------
def pull_forces(batch: Batch, seed: int = 2_000_000, fraction: float = 0.10,
                fmax: float = 30.0) -> np.ndarray:
    """Constant apple pulls of the pull1024 workload: a fraction of apples get a
    force of magnitude U(0, fmax) N in a direction uniform on the sphere.
    Returns float64 [A_tot, 3] in descriptor apple order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = batch.n_apple
    sel = rng.random(A) < fraction
    d = rng.normal(size=(A, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    mag = rng.uniform(0.0, fmax, size=A)
    return np.where(sel[:, None], d * mag[:, None], 0.0)


def geometry_perturbation(batch: Batch, seed: int = 5_000_000, strength: float = 1.0) -> np.ndarray:
    """Per-world geometry perturbation for the on-device rebuild: [S_tot, 4] float64 in
    descriptor order — length factor 1 + 0.25 s U(-1, 1), radius factor 1 + 0.15 s U(-1, 1),
    bends about the segment's x and y axes s N(0, 4 deg) each.  s = 0 gives (1, 1, 0, 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S = batch.n_seg
    f = np.empty((S, 4))
    f[:, 0] = 1.0 + 0.25 * strength * rng.uniform(-1.0, 1.0, S)
    f[:, 1] = 1.0 + 0.15 * strength * rng.uniform(-1.0, 1.0, S)
    f[:, 2:] = strength * np.deg2rad(4.0) * rng.normal(size=(S, 2))
    return f


def grad_apple_forces(batch: Batch, n_steps: int, seed: int = 4_000_000,
                      sigma: float = 2.0) -> np.ndarray:
    """Per-step apple forces of the grad512 workload, N(0, sigma) per component.
    Returns float64 [n_steps, A_tot, 3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, sigma, size=(n_steps, batch.n_apple, 3))


def grad_targets(batch: Batch, rest_tips: np.ndarray, n_tips: int = 16,
                 seed: int = 4_100_000, sigma: float = 0.05):
    """Tip indices (env-local leaf segments, 16 per tree) and targets for the
    grad512 loss.  ``rest_tips`` [S_tot, 3] are the rest tip positions, which the
    caller computes with its own kinematics.  Returns (idx int32 [B, n_tips],
    target float64 [B, n_tips, 3])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = batch.n_env
    idx = np.zeros((B, n_tips), dtype=np.int32)
    tgt = np.zeros((B, n_tips, 3))
    for e in range(B):
        s0, s1 = batch.seg_offset[e], batch.seg_offset[e + 1]
        par = batch.seg_parent[s0:s1]
        nc = np.bincount(par[par >= 0], minlength=s1 - s0)
        leaves = np.flatnonzero(nc == 0)
        pick = rng.choice(leaves, size=n_tips, replace=leaves.size < n_tips)
        idx[e] = pick
        tgt[e] = rest_tips[s0 + pick] + rng.normal(0.0, sigma, size=(n_tips, 3))
    return idx, tgt


# --- constants of the step shared by all workloads (the paper's values where it gives
# them, chosen readings where it does not): time step, gravity, tether, damping and event
# parameters ---------------------------------------------------------------------------
STEP_CONSTANTS = dict(
    dt=1e-3,
    gravity=(0.0, 0.0, -9.81),
    tether_k=2e3,            # N/m
    tether_zeta=0.05,        # c_s = 2 zeta sqrt(k_s m)
    damping_zeta=0.05,       # Kd = 2 zeta sqrt(Kp J)
    damping_cd=0.0,          # > 0 selects the stiffness-proportional Kd = c_d Kp instead
    tension_factor=1.1,      # tension threshold = 1.1 f_detach
    v_cap=1.0,               # impulse cap speed (m/s)
    react_max_factor=1.0,    # reaction clamp = f_detach
    event_band=1e-3,         # band of the event comparison
    n_break=5, n_pull=5, n_tension=20,
    rng_seed=0, wrench_fraction=0.0, wrench_sigma=5.0,
    # variants: per-level exponential stiffness (off at k0 = 0), fruit degrees of freedom
    stiffness_k0=0.0, stiffness_gamma=1.0, fruit_dof=6,
    # extras, off at 0: drag, post-break friction ramp, power fade and speed brake
    drag_lin=0.0, drag_ang=0.0, drag_snapped=1.0,
    friction_base=0.0, friction_growth=1.0, friction_ramp_time=0.0, friction_speed=0.0,
    fade_speed=0.0, brake_rate=0.0,
)

# the extras as a workload turns them on (readings of constants the paper does not
# give): drag 1/s on segments (a tenth of it on a snapped sub-tree), friction from a
# quarter of the limb's weight moment growing five-fold over 1.5 s, damper below
# 0.05 rad/s, power fade from 0.5 m/s, speed brake 50/s above the impulse-cap speed
EXTRAS_ON = dict(drag_lin=1.0, drag_ang=1.0, drag_snapped=0.1, friction_base=0.25, friction_growth=5.0,
                 friction_ramp_time=1.5, friction_speed=0.05, fade_speed=0.5, brake_rate=50.0)
# the per-level exponential stiffness as a workload uses it: about the trunk's Eq.-beam
# stiffness at the root, falling to twig stiffness twenty levels down
EXP_STIFFNESS = dict(stiffness_k0=1.0e5, stiffness_gamma=0.65)


def step_constants(name: str | None = None, **over) -> dict:
    """Constants for a workload; the uneven workload turns on the in-step wrenches
    (5 % of bodies, N(0, 5 N) per component)."""
    c = dict(STEP_CONSTANTS)
    if name == "uneven8192":
        c.update(rng_seed=3_000_000, wrench_fraction=0.05, wrench_sigma=5.0)
    c.update(over)
    return c
