"""Helpers shared by the GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded inputs and compare them element by element.

Tolerances (joint state): per env and per class, the largest deviation over all
compared steps and DoF divided by max(largest oracle magnitude in that env, floor),
floors 1e-3 rad (angles) and 1e-2 rad/s (rates); bar 1e-4.  Fruit state (position
state and velocity) is compared the same way, with floors 1e-3 m and 1e-2 m/s and bar
APPLE_TOL.  Events: every (env,
joint) and (env, apple) whose oracle ratio |mu - 1| (or |pi - 1|, |tau - 1|) stayed
at least EPS away from 1 over the compared steps must have the identical event (kind
and step) or none on both sides; ids that came within EPS ("in band") are excluded,
and if such an id's event differs, the env's state comparison stops at the first
in-band step.
"""
from __future__ import annotations

import numpy as np

from oracle.oracle import Band, Oracle

TOL = 1e-4
APPLE_TOL = 1e-4
FLOOR_Q, FLOOR_QD = 1e-3, 1e-2
FLOOR_AX, FLOOR_AV = 1e-3, 1e-2
EPS = 1e-3


def gpu_events_desc(model, state):
    """GPU events as {(env, kind, id): step} with descriptor-local ids."""
    return {(e, k, i): s for (e, k, i, s) in model.events(state)}


def oracle_events(batch, st, envs):
    ev = {}
    for e in envs:
        s0, s1 = batch.seg_offset[e], batch.seg_offset[e + 1]
        a0, a1 = batch.apple_offset[e], batch.apple_offset[e + 1]
        for i in np.flatnonzero(st.break_step[s0:s1] >= 0):
            ev[(int(e), 1, int(i))] = int(st.break_step[s0 + i])
        for a in np.flatnonzero(st.det_step[a0:a1] >= 0):
            ev[(int(e), 1 + int(st.det_path[a0 + a]), int(a))] = int(st.det_step[a0 + a])
    return ev


def event_ratio_errors(model, state, batch, ost, envs, band_eps=EPS):
    """Threshold ratio of every event that the GPU and the oracle record for the same id,
    kind and step: returns (number compared, largest |GPU - oracle|, events whose in-band
    flag disagrees with |ratio - 1| < band_eps)."""
    envs = set(envs)
    n, worst, flag_bad = 0, 0.0, []
    for (e, k, i, s, r, ib) in model.events(state, ratios=True):
        if e not in envs:
            continue
        if bool(ib) != (abs(float(r) - 1.0) < band_eps):
            flag_bad.append((e, k, i, s, r, ib))
        if k == 1:
            j = batch.seg_offset[e] + i
            if ost.break_step[j] != s:
                continue
            ro = ost.break_ratio[j]
        else:
            a = batch.apple_offset[e] + i
            if ost.det_step[a] != s or 1 + int(ost.det_path[a]) != k:
                continue
            ro = ost.det_ratio[a]
        n += 1
        worst = max(worst, abs(float(r) - float(ro)))
    return n, worst, flag_bad


def _rel(g, o, floor):
    if g.size == 0:
        return 0.0
    return float(np.max(np.abs(g - o)) / max(np.max(np.abs(o)), floor))


class Recorder:
    """Collects GPU and oracle joint and fruit states at the compared steps (fruit:
    position state and velocity, descriptor order [A_tot, 3])."""

    def __init__(self, batch, envs):
        self.batch = batch
        self.envs = list(envs)
        self.steps = []
        self.g = {k: [] for k in ("q", "qd", "ax", "av")}
        self.o = {k: [] for k in ("q", "qd", "ax", "av")}

    def add(self, step, gq_desc, gqd_desc, ost, gax_desc=None, gav_desc=None):
        self.steps.append(step)
        for k, v in (("q", gq_desc), ("qd", gqd_desc), ("ax", gax_desc), ("av", gav_desc)):
            self.g[k].append(None if v is None else v.copy())
            self.o[k].append(getattr(ost, k).copy())

    def errors(self, cut=None):
        """Per env: (rel q, rel qd, n compared steps, rel fruit position, rel fruit velocity)."""
        out = {}
        steps = np.array(self.steps)
        have_apples = all(x is not None for x in self.g["ax"])
        for e in self.envs:
            s0, s1 = self.batch.seg_offset[e], self.batch.seg_offset[e + 1]
            a0, a1 = self.batch.apple_offset[e], self.batch.apple_offset[e + 1]
            use = np.ones(len(steps), bool) if cut is None or cut.get(e) is None else steps <= cut[e]
            if not use.any():
                out[e] = (0.0, 0.0, 0, 0.0, 0.0)
                continue
            st = lambda d, k, lo, hi: np.stack([x[lo:hi] for x in d[k]])[use]
            rq = _rel(st(self.g, "q", s0, s1), st(self.o, "q", s0, s1), FLOOR_Q)
            rqd = _rel(st(self.g, "qd", s0, s1), st(self.o, "qd", s0, s1), FLOOR_QD)
            rax = rav = 0.0
            if have_apples and a1 > a0:
                rax = _rel(st(self.g, "ax", a0, a1), st(self.o, "ax", a0, a1), FLOOR_AX)
                rav = _rel(st(self.g, "av", a0, a1), st(self.o, "av", a0, a1), FLOOR_AV)
            out[e] = (rq, rqd, int(use.sum()), rax, rav)
        return out


def compare_events(batch, gpu_ev, ora_ev, band: Band, envs):
    """Returns (mismatches outside the band, per-env cut step for in-band differences,
    number of in-band ids)."""
    bad, cut, n_band = [], {}, 0
    for e in envs:
        s0, s1 = batch.seg_offset[e], batch.seg_offset[e + 1]
        a0, a1 = batch.apple_offset[e], batch.apple_offset[e + 1]
        ids = [(1, i, band.jmin[s0 + i], band.jfirst[s0 + i]) for i in range(s1 - s0)]
        ids += [(None, a, band.amin[a0 + a], band.afirst[a0 + a]) for a in range(a1 - a0)]
        for kind, i, m, first in ids:
            keys = [(e, 1, i)] if kind == 1 else [(e, 2, i), (e, 3, i)]
            g = {k: gpu_ev.get(k) for k in keys if k in gpu_ev}
            o = {k: ora_ev.get(k) for k in keys if k in ora_ev}
            if m < EPS:
                n_band += 1
                if g != o:
                    cut[e] = min(cut.get(e, 1 << 30), int(first))
                continue
            if g != o:
                bad.append((e, keys, g, o))
    return bad, cut, n_band


def run_parity(batch, consts, n_steps, every, *, envs=None, tuning=None, aforce_desc=None, aforce_from=0,
               wrench_desc=None, threads=None, model=None):
    """Run the whole batch on the GPU and the listed envs on the oracle.

    aforce_desc: constant apple force [A_tot, 3] (descriptor order) applied from step
    aforce_from on.  model: an existing GPU model of this batch (else one is created).
    Returns (errors per env, event mismatches, in-band count, model, gpu state, oracle
    state)."""
    import torch

    from paper_2607_06337_amd import Model

    envs = list(range(batch.n_env)) if envs is None else list(envs)
    m = Model(batch, consts, tuning) if model is None else model
    st = m.rest_state()
    kp, kd = m.default_params()
    o = Oracle(batch, consts)
    d = o.derived()
    ost = o.rest_state()
    band = Band(batch.n_seg, batch.n_apple)
    af_int = None
    if aforce_desc is not None:
        af_int = torch.tensor(m.apple_from_desc(np.asarray(aforce_desc, np.float32), axis=0), device="cuda").contiguous()
    w_int = None
    if wrench_desc is not None:
        w_int = torch.tensor(m.seg_from_desc(np.asarray(wrench_desc, np.float32)), device="cuda").contiguous()
    rec = Recorder(batch, envs)
    rest_desc = m.apple_to_desc(m.apple_hang_rest, axis=0)
    marks = sorted(set(list(range(every, n_steps + 1, every)) + ([aforce_from] if 0 < aforce_from < n_steps else [])))
    done = 0
    for mk in marks:
        k = mk - done
        use_f = aforce_desc is not None and done >= aforce_from
        m.step(st, kp, kd, k, aforce=af_int if use_f else None, wrench=w_int)
        o.rollout(ost, k, kp=d["kp"], kd=d["kd"], envs=envs, aforce=aforce_desc if use_f else None,
                  wrench=wrench_desc, band=band, threads=threads)
        done = mk
        torch.cuda.synchronize()
        gq = m.seg_to_desc(st.q.cpu().numpy().astype(np.float64))
        gqd = m.seg_to_desc(st.qd.cpu().numpy().astype(np.float64))
        ga = m.apple_to_desc(st.apple[0:6].cpu().numpy().astype(np.float64), axis=1)
        # a detached fruit's position state is kept relative to its rest hang point on the
        # GPU, absolute in the oracle
        det = m.apple_to_desc(st.apple_evt[0].cpu().numpy(), axis=0) != 0
        gax = ga[0:3].T + np.where(det[:, None], rest_desc, 0.0)
        rec.add(done, gq, gqd, ost, gax, ga[3:6].T)
    gev = gpu_events_desc(m, st)
    gev = {k: v for k, v in gev.items() if k[0] in set(envs)}
    oev = oracle_events(batch, ost, envs)
    bad, cut, n_band = compare_events(batch, gev, oev, band, envs)
    errs = rec.errors(cut)
    return errs, bad, n_band, m, st, ost, gev, oev


def stratified_envs(batch, n, seed=0):
    """n env indices spread over the size distribution (sorted by segment count)."""
    sizes = np.diff(batch.seg_offset)
    order = np.argsort(sizes, kind="stable")
    pick = np.unique(np.linspace(0, len(order) - 1, n).round().astype(int))
    return sorted(int(order[i]) for i in pick)
