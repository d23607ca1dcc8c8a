"""Benchmark: batched forward-dynamics step of 8192 uneven apple trees on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one pass of the whole hot path (events, kinematics, forces, apples, bias,
factorisation, solve, integration) over all 8192 trees.  The workload is the uneven
batch: 8192 seeded trees with round(exp(U(ln 50, ln 1500))) segments and U{10..120}
apples, random body forces (5 % of bodies per step, N(0, 5 N) per component) drawn
inside the step.  Inputs live in HBM before the timed region starts.

Prints ONE JSON line with the metric, the roofline of the step kernel (algorithmic
bytes per launch over its measured average duration, HIP events on the launch
stream) and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# kernel mapping used by the full-size parity test and the adjoint ratio, and the first of
# the candidates the autotuner times for the benchmark
# (trees wider than lds_width but not than 512 nodes per level go to the wide-tree bucket,
# packs of 512 work-items launched on a second stream; no tree of the uneven batch is that
# wide, the 5000-segment trees of the orchard-row batch are)
BENCH_TUNING = dict(threads=256, pack_fill=1.0, steps_per_launch=50, persistent=0, lds_width=240, big_threads=512)
# candidates of the autotuner: workgroup size, LDS width, steps per launch (a multi-step
# launch fuses the second down pass of a step with the first of the next), persistent
# queue, wave packs for trees whose widest level fits a wavefront
AUTOTUNE_CANDIDATES = [BENCH_TUNING, dict(BENCH_TUNING, steps_per_launch=10), dict(BENCH_TUNING, steps_per_launch=1),
                       dict(BENCH_TUNING, lds_width=256), dict(BENCH_TUNING, lds_width=224),
                       dict(BENCH_TUNING, lds_width=192), dict(BENCH_TUNING, threads=128, lds_width=128),
                       dict(BENCH_TUNING, lds_width=0), dict(BENCH_TUNING, threads=128, lds_width=0),
                       dict(BENCH_TUNING, wave_width=64), dict(BENCH_TUNING, wave_width=32),
                       dict(BENCH_TUNING, threads=64, lds_width=64),
                       dict(BENCH_TUNING, persistent=1)]
TUNING_KEYS = ("threads", "pack_fill", "steps_per_launch", "persistent", "lds_width", "pack_skew", "wave_width",
               "big_threads")
GRAPH_STEPS = 100  # steps per captured HIP graph in the timed rollout
# the plain per-step kernel: one 256-thread workgroup per tree, one launch per step,
# levels exchange through global scratch
PLAIN_TUNING = dict(threads=256, pack_fill=0.0, steps_per_launch=1, persistent=0, lds_width=0)

HBM_PEAK_GBS = 8000.0
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4   # wave64 VALU instructions per second, whole chip
FP32_PEAK = 78.6e12                  # FP32 vector FLOP/s without packed math
SEG_BYTES, APPLE_BYTES = 84, 146   # algorithmic bytes per segment-step / apple-step
WORKLOAD = "uneven8192"


def algorithmic_bytes(batch) -> int:
    """Bytes a streaming step must move per batch step: FP32 SoA joint state read and
    written, event bytes, static segment data; apple state, flags and static data."""
    return SEG_BYTES * batch.n_seg + APPLE_BYTES * batch.n_apple


def code_without_comments(text: str) -> str:
    """C++ source with comments and trailing blanks removed: two sources that differ only in
    their comments compile to the same kernel."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


STEP_SOURCES = ("paper_2607_06337_amd/csrc/orchard_step.hip", "paper_2607_06337_amd/csrc/orchard_dev.h")
SPHERE_SOURCES = ("paper_2607_06337_amd/csrc/orchard_sphere.hip",)


def kernel_source_hash(files=STEP_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(code_without_comments(open(os.path.join(ROOT, f)).read()).encode())
    return h.hexdigest()[:16]


def profiled_counters(kernel: str, tuning, files=STEP_SOURCES):
    """Counter figures of the committed rocprofv3 summaries of this kernel (HBM bytes per
    launch, VALU instructions and FP32 operations), merged over the summaries taken on the
    current source of `files` and mapping `tuning`; None if there is none."""
    cur = kernel_source_hash(files)
    out = {}
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if line.startswith("machine-readable: "):
                rec = json.loads(line[len("machine-readable: "):])
                if rec.get("kernel") == kernel and rec.get("src_hash") == cur and rec.get("tuning") == tuning:
                    out.update(rec)
    return out or None


def time_gpu(model, n_steps, warmup, graph_steps=0, repeats=1):
    """Time n_steps after warmup eager steps.  With graph_steps > 0 the rollout is a HIP
    graph of min(graph_steps, n_steps) steps replayed (capture and one replay happen
    before the timed region; a remainder runs eagerly inside it).  Returns (ms, wall s,
    non-finite envs, state, description of what was timed, kernel launches timed, [ms of
    each of `repeats` timed rollouts of n_steps, the first being the returned one])."""
    import torch
    st = model.rest_state()
    kp, kd = model.default_params()
    model.step(st, kp, kd, warmup)
    g = None
    gs = min(graph_steps, n_steps)
    if gs > 0:
        g = model.graph(st, kp, kd, gs)
        g.launch()  # the first replay is not timed
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    spl = max(1, int(model.tuning.steps_per_launch))
    launches = lambda k: -(-k // spl)
    runs = []
    for r in range(max(1, repeats)):
        t0 = time.perf_counter()
        ev0.record(stream)
        if g is not None:
            reps, rem = n_steps // gs, n_steps % gs
            for _ in range(reps):
                g.launch(stream)
            if rem:
                model.step(st, kp, kd, rem)
            what = f"HIP graph of {gs} steps replayed {reps} times" + (f" + {rem} eager steps" if rem else "")
            n_launch = reps * launches(gs) + launches(rem)
        else:
            model.step(st, kp, kd, n_steps)
            what = f"one eager call of {n_steps} steps"
            n_launch = launches(n_steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        if r == 0:
            wall = time.perf_counter() - t0
        runs.append(ev0.elapsed_time(ev1))
    ms = runs[0]
    status = model.status(st)
    what += f" ({n_launch} launches of up to {spl} steps)"
    return ms, wall, int((status != 0).sum()), st, what, n_launch, runs


def event_counts(model, st):
    """Breaks and detachments recorded in a state (event kinds 1: break, 2: pull detach,
    3: tension detach), with the fraction of joints broken."""
    ev = model.events(st)
    kinds = np.bincount(np.array([k for (_, k, _, _) in ev], dtype=np.int64), minlength=4) if ev else np.zeros(4, int)
    return dict(breaks=int(kinds[1]), break_fraction=round(int(kinds[1]) / model.n_seg, 6),
                pull_detachments=int(kinds[2]), tension_detachments=int(kinds[3]))


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, consts, n_envs=512, n_steps=200, n_envs_1=64, n_steps_1=100, pull_steps=100):
    """FP64 oracle on size-stratified samples of the same workload: all cores of the
    process's CPU share on n_envs trees x n_steps steps, and one core on n_envs_1 trees x
    n_steps_1 steps; beside them, all 1024 trees of the pull workload (100-400 segments)
    x pull_steps steps on all cores."""
    from oracle.oracle import Oracle
    from orchard_inputs import assemble

    def sample(n):
        sizes = np.diff(batch.seg_offset)
        order = np.argsort(sizes, kind="stable")
        pick = sorted(int(order[i]) for i in np.unique(np.linspace(0, len(order) - 1, n).round().astype(int)))
        return pick, int(sizes[pick].sum())

    def run(n, steps, threads):
        pick, segs = sample(n)
        o = Oracle(assemble([batch.tree(e) for e in pick]), consts)
        st = o.rest_state()
        t0 = time.perf_counter()
        o.rollout(st, steps, threads=threads)
        dt = time.perf_counter() - t0
        return len(pick) * steps / dt, dt, len(pick), segs

    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    threads = max(1, avail)
    v_all, dt_all, n_all, seg_all = run(n_envs, n_steps, threads)
    v_one, dt_one, n_one, seg_one = run(n_envs_1, n_steps_1, 1)
    from orchard_inputs import make_batch, step_constants
    pb = make_batch("pull1024")
    o = Oracle(pb, step_constants("pull1024"))
    st = o.rest_state()
    t0 = time.perf_counter()
    o.rollout(st, pull_steps, threads=threads)
    dt_pull = time.perf_counter() - t0
    return dict(value=v_all, unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"{n_all} size-stratified trees of the workload ({seg_all} segments) x {n_steps} steps, FP64, "
                       f"{dt_all:.1f} s on {threads} threads",
                single_core=dict(value=v_one, sample=f"{n_one} size-stratified trees ({seg_one} segments) x "
                                                     f"{n_steps_1} steps, {dt_one:.1f} s on 1 thread"),
                pull1024=dict(value=pb.n_env * pull_steps / dt_pull,
                              sample=f"all {pb.n_env} trees of the pull workload ({pb.n_seg} segments) x {pull_steps} "
                                     f"steps, {dt_pull:.1f} s on {threads} threads"),
                nproc=os.cpu_count(), affinity=avail, cpu_model=_cpu_model())


def cpu_adjoint_baseline(n_trees: int = 8, n_steps: int = 200):
    """FP64 oracle adjoint on the first n_trees trees of the differentiable workload (300
    segments, 40 apples, per-step apple forces): the loss rollout alone and the adjoint
    (taped forward plus reverse sweep) of a random state loss, one tree per thread."""
    from concurrent.futures import ThreadPoolExecutor

    from orchard_inputs import grad_apple_forces, make_batch, step_constants
    from oracle.oracle import Oracle, adjoint, env_state0, loss
    b = make_batch("grad512", env_ids=range(n_trees))
    F = grad_apple_forces(b, n_steps)
    o = Oracle(b, step_constants())
    d = o.derived()
    st = o.rest_state()
    rng = np.random.default_rng(0)
    jobs = []
    for e in range(n_trees):
        s0, s1 = b.seg_offset[e], b.seg_offset[e + 1]
        a0, a1 = b.apple_offset[e], b.apple_offset[e + 1]
        jobs.append((e, env_state0(o, st, e), d["kp"][s0:s1], d["kd"][s0:s1], F[:, a0:a1],
                     dict(q=rng.normal(size=(s1 - s0, 2)))))
    no_tip, no_target = np.zeros(0, np.int32), np.zeros((0, 3))
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    threads = max(1, min(n_trees, avail))
    with ThreadPoolExecutor(threads) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda j: loss(o, j[0], j[1], j[2], j[3], j[4], n_steps, no_tip, no_target, w_state=j[5]), jobs))
        t1 = time.perf_counter()
        list(ex.map(lambda j: adjoint(o, j[0], j[1], j[2], j[3], j[4], n_steps, no_tip, no_target, w_state=j[5]), jobs))
        t2 = time.perf_counter()
    return dict(value=round(n_trees * n_steps / (t2 - t1), 1), unit="env-steps/s", cores=threads, kind="oracle",
                forward_env_steps_per_s=round(n_trees * n_steps / (t1 - t0), 1), ratio=round((t2 - t1) / (t1 - t0), 2),
                sample=f"{n_trees} trees of the differentiable workload x {n_steps} steps, FP64 adjoint of a state "
                       f"loss: forward {t1 - t0:.1f} s, adjoint {t2 - t1:.1f} s on {threads} threads, one tree each")


def workload_stats(batch) -> dict:
    """Shape of a batch: depth in levels (max, mean over trees), widest level of any tree,
    tip (leaf) count and mean tip radius."""
    sizes = np.diff(batch.seg_offset)
    env = np.repeat(np.arange(batch.n_env), sizes)
    par = np.asarray(batch.seg_parent, np.int64)
    gpar = np.where(par >= 0, par + batch.seg_offset[:-1][env], -1)
    depth = np.zeros(batch.n_seg, np.int64)
    while True:  # parents precede children: a fixed point after max-depth sweeps
        nd = np.where(gpar >= 0, depth[np.maximum(gpar, 0)] + 1, 0)
        if np.array_equal(nd, depth):
            break
        depth = nd
    tree_depth = np.zeros(batch.n_env, np.int64)
    np.maximum.at(tree_depth, env, depth + 1)
    _, width = np.unique(env * (int(depth.max()) + 1) + depth, return_counts=True)
    tip = np.bincount(gpar[gpar >= 0], minlength=batch.n_seg) == 0
    return dict(max_depth=int(tree_depth.max()), mean_depth=round(float(tree_depth.mean()), 2),
                widest_level=int(width.max()), tips=int(tip.sum()),
                r_tip_mm=round(float(np.mean(batch.seg_radius[tip])) * 1e3, 3))


ADJOINT_CANDIDATES = [BENCH_TUNING, dict(BENCH_TUNING, threads=128, lds_width=128),
                      dict(BENCH_TUNING, threads=128, lds_width=64)]


def adjoint_ratio(reps: int = 5, candidates=None):
    """Adjoint/forward cost ratio on the differentiable-rollout workload: 512 trees of 300
    segments and 40 apples, 200 steps with checkpoints every 20, per-step apple forces;
    backward = recompute of every checkpoint segment + adjoint kernels.  The mapping is the
    candidate with the least forward + backward time (one untimed and `reps` timed
    repetitions each, medians); the ratio reported is that mapping's."""
    import torch
    from orchard_inputs import grad_apple_forces, make_batch, step_constants
    from paper_2607_06337_amd import Model
    T, K = 200, 20
    batch = make_batch("grad512")
    Fh = grad_apple_forces(batch, T).astype(np.float32)
    tried = []
    for tun in (candidates or ADJOINT_CANDIDATES):
        m = Model(batch, step_constants(), dict(tun, adjoint_ckpt_max=K))
        kp, kd = m.default_params()
        F = torch.tensor(m.apple_from_desc(Fh, axis=1), device="cuda").contiguous()
        ck = torch.empty(-(-T // K) * m.ckpt_words, device="cuda")
        fw, bw = [], []
        for _ in range(reps + 1):
            st = m.rest_state()
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            adj = dict(q=torch.randn(m.n_seg, 2, device="cuda"), qd=torch.zeros(m.n_seg, 2, device="cuda"),
                       ax=torch.zeros(3, m.n_apple, device="cuda"), av=torch.zeros(3, m.n_apple, device="cuda"))
            gkp, gkd, gF = torch.zeros_like(kp), torch.zeros_like(kd), torch.zeros_like(F)
            torch.cuda.synchronize()
            e0.record()
            m.step(st, kp, kd, T, aforce=F, ckpt=ck, ckpt_every=K)
            e1.record()
            m.step_backward(ck, K, T, kp, kd, adj, gkp, gkd, gF, aforce=F)
            e2.record()
            torch.cuda.synchronize()
            fw.append(e0.elapsed_time(e1))
            bw.append(e1.elapsed_time(e2))
        tried.append(dict(tuning={k: tun[k] for k in ("threads", "lds_width")}, forward_ms=round(float(np.median(fw[1:])), 2),
                          backward_ms=round(float(np.median(bw[1:])), 2)))
        del m
    best = min(tried, key=lambda r: r["forward_ms"] + r["backward_ms"])
    return dict(ratio=round(best["backward_ms"] / best["forward_ms"], 3), forward_ms=best["forward_ms"],
                backward_ms=best["backward_ms"], tuning=best["tuning"], candidates=tried, shape=workload_stats(batch),
                workload="grad512: 512 trees x 300 segments x 40 apples, 200 steps, checkpoints every 20")


# the orchard-row batch's mappings: the forward workload's (small trees in 240-wide packs, the
# 5000-segment trees in the wide-tree bucket beside them) and 512-wide packs for all trees
ROW_CANDIDATES = [BENCH_TUNING, dict(BENCH_TUNING, threads=512, lds_width=480)]


def row_scale(fwd_steps: int = 200, warm: int = 10, lead: int = 900, tail: int = 100, K: int = 20, reps: int = 5):
    """Orchard-row batch (64 trees of 5000 segments + 16384 of 80) in one launch: forward
    throughput in the faster of the ROW_CANDIDATES mappings (both listed), then in that
    mapping the 64 large trees alone: forward to step lead + tail with checkpoints
    over the final tail steps, and the adjoint over those steps (recompute included), both
    from the same state after lead steps, one untimed and `reps` timed repetitions, medians.
    Algorithmic-byte rates use the same per-segment / per-apple bytes as the main figure."""
    import torch
    from orchard_inputs import make_batch, step_constants
    from paper_2607_06337_amd import Model
    batch = make_batch("row64x16k")
    consts = step_constants()
    tried = []
    for tun in ROW_CANDIDATES:
        m = Model(batch, consts, tun)
        ms, _, n_bad, _, _, _, _ = time_gpu(m, fwd_steps, warm, GRAPH_STEPS)
        tried.append((ms, n_bad, tun))
        del m
    ms, n_bad, tun = min(tried, key=lambda r: r[0])
    fwd = dict(ms_per_step=round(ms / fwd_steps, 4), env_steps_per_s=round(batch.n_env * fwd_steps / (ms / 1e3), 1),
               alg_GBps=round(algorithmic_bytes(batch) * fwd_steps / (ms / 1e3) / 1e9, 1), nonfinite_envs=n_bad,
               tuning={k: tun[k] for k in ("threads", "lds_width", "big_threads")},
               candidates=[dict(tuning={k: t[k] for k in ("threads", "lds_width", "big_threads")},
                                ms_per_step=round(x / fwd_steps, 4)) for x, _, t in tried])
    large = make_batch("row64x16k", env_ids=range(64))
    ml = Model(large, consts, dict(tun, adjoint_ckpt_max=K))
    st = ml.rest_state()
    kp, kd = ml.default_params()
    ml.step(st, kp, kd, lead)
    st_lead = st.clone()
    ck = torch.empty(-(-tail // K) * ml.ckpt_words, device="cuda")
    adj = dict(q=torch.randn(ml.n_seg, 2, device="cuda"), qd=torch.zeros(ml.n_seg, 2, device="cuda"),
               ax=torch.zeros(3, ml.n_apple, device="cuda"), av=torch.zeros(3, ml.n_apple, device="cuda"))
    fws, bws = [], []
    for _ in range(reps + 1):   # from the same state each time; the first is untimed
        for f in st.__dataclass_fields__:
            getattr(st, f).copy_(getattr(st_lead, f))
        gkp, gkd = torch.zeros_like(kp), torch.zeros_like(kd)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record()
        ml.step(st, kp, kd, tail, ckpt=ck, ckpt_every=K)
        e1.record()
        ml.step_backward(ck, K, tail, kp, kd, adj, gkp, gkd)
        e2.record()
        torch.cuda.synchronize()
        fws.append(e0.elapsed_time(e1))
        bws.append(e1.elapsed_time(e2))
    fw, bw = float(np.median(fws[1:])), float(np.median(bws[1:]))
    lb = algorithmic_bytes(large) * tail
    return dict(workload="row64x16k: 64 trees x 5000 segments x 400 apples + 16384 trees x 80 segments x 8 apples, "
                         "one launch, gravity and breakage",
                shape=workload_stats(batch), forward=fwd,
                adjoint_large=dict(steps=f"{lead}..{lead + tail}", forward_ms=round(fw, 2), backward_ms=round(bw, 2),
                                   ratio=round(bw / fw, 3), forward_alg_GBps=round(lb / (fw / 1e3) / 1e9, 1),
                                   backward_alg_GBps=round(lb / (bw / 1e3) / 1e9, 1)))


def sphere_fit_leg(n_patch: int = 65536, reps: int = 20, cpu_patches: int = 2000):
    """Batched sphere-fit detector on synthetic depth patches (fruit caps, branch sections,
    leaves; about 400 points per patch): one launch per batch, HIP events over `reps`
    launches.  Algorithmic bytes: 12 per point read, 4 per patch offset, 32 per patch
    written.  CPU baseline: the FP64 reference on a sample of patches, one thread."""
    import torch
    from orchard_inputs.patches import GATE, make_patches
    from oracle.sphere import fit_patches
    from paper_2607_06337_amd import sphere_fit
    pts, off, kind, _ = make_patches(n_patch)
    P = torch.tensor(pts, device="cuda")
    O = torch.tensor(off, device="cuda")
    out = torch.empty(n_patch, 8, device="cuda")
    sphere_fit(P, O, GATE, out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        sphere_fit(P, O, GATE, out)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    n_pts = int(off[-1])
    alg = 12 * n_pts + 4 * (n_patch + 1) + 32 * n_patch
    acc = out[:, 6].cpu().numpy() == 0
    pick = np.unique(np.linspace(0, n_patch - 1, cpu_patches).round().astype(int))
    t0 = time.perf_counter()
    fit_patches(pts, off, GATE, patches=pick)
    cpu_s = time.perf_counter() - t0
    roof = dict(bound="hbm", achieved=round(alg / (us * 1e-6) / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4), bytes_per_launch=alg)
    prof = profiled_counters("k_sphere_fit", None, SPHERE_SOURCES)
    if prof and prof.get("hbm_bytes_per_launch"):
        roof["traffic"] = int(prof["hbm_bytes_per_launch"])
    if prof and prof.get("valu_insts_per_launch"):
        # VALU issue against 1024 SIMDs x one wave64 instruction per 4 cycles at 2.4 GHz:
        # the busier resource of this kernel
        vi = prof["valu_insts_per_launch"]
        roof["valu"] = dict(insts_per_launch=vi, frac=round(vi / (us * 1e-6) / VALU_ISSUE_PEAK, 4),
                            peak_insts_per_s=VALU_ISSUE_PEAK)
    return dict(workload=f"{n_patch} synthetic depth patches ({n_pts} points; fruit caps, branch sections, leaves)",
                us_per_launch=round(us, 2), patches_per_s=round(n_patch / (us * 1e-6), 1),
                points_per_s=round(n_pts / (us * 1e-6), 1), accepted=int(acc.sum()),
                fruit_recall=round(float(acc[kind == 0].mean()), 4), roofline=roof,
                cpu_baseline=dict(value=round(len(pick) / cpu_s, 1), unit="patches/s", cores=1, kind="oracle",
                                  sample=f"{len(pick)} patches of the workload, FP64 least squares, {cpu_s:.1f} s"))


def copy_bandwidth(n_bytes: int = 1 << 30, reps: int = 5) -> float:
    """Measured device-to-device copy rate (GB/s, bytes read plus written) of a plain
    tensor copy: the practical HBM ceiling beside the 8 TB/s datasheet figure."""
    import torch
    x = torch.empty(n_bytes // 4, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n_bytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del x, y
    return gbs


def _copy_probe():
    """Three launches of one plain elementwise kernel (256 MiB read, 256 MiB written): the
    reference that scales the HBM counters."""
    import torch
    x = torch.ones(64 << 20, device="cuda")
    for _ in range(3):
        y = x * 1.0001
    torch.cuda.synchronize()
    del x, y


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-row-scale", action="store_true")
    ap.add_argument("--no-sphere", action="store_true")
    ap.add_argument("--batch-cache", type=str, default=None,
                    help="npz file holding the generated batch (written if missing): profiler runs load it instead "
                         "of generating the trees in worker processes")
    ap.add_argument("--cache-only", action="store_true", help="write --batch-cache and exit (no GPU)")
    ap.add_argument("--sphere-only", action="store_true", help="run only the sphere-fit leg (for its profile)")
    ap.add_argument("--tuning", type=str, default=None,
                    help="kernel mapping as JSON (skips the autotuner), e.g. the one a profile was taken with")
    ap.add_argument("--row-scale-only", action="store_true",
                    help="run only the orchard-row phases and print their figures (for per-phase counters)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint/forward leg (differentiable-rollout batch) and print it (for its profile); "
                         "with --tuning, in that mapping only")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB read + 256 MiB write kernel (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (trees are independent, "
              "a multi-GPU run would give each GPU a share of the envs balanced by segment count and depth)", file=sys.stderr)
        sys.exit(2)

    if args.sphere_only:
        import torch
        torch.cuda.init()
        if args.copy_probe:
            _copy_probe()
        print(json.dumps(dict(sphere_fit=sphere_fit_leg())), flush=True)
        return

    if args.adjoint_only:
        import torch
        torch.cuda.init()
        cands = [dict(BENCH_TUNING, **json.loads(args.tuning))] if args.tuning else None
        print(json.dumps(dict(adjoint=adjoint_ratio(candidates=cands))), flush=True)
        return

    if args.row_scale_only:
        import torch
        torch.cuda.init()
        if args.copy_probe:
            _copy_probe()
        print(json.dumps(dict(row_scale=row_scale())), flush=True)
        return

    from orchard_inputs import make_batch, step_constants
    t_gen = time.perf_counter()
    if args.batch_cache and os.path.exists(args.batch_cache):
        import dataclasses

        from orchard_inputs import Batch
        with np.load(args.batch_cache) as z:
            batch = Batch(**{f.name: z[f.name] for f in dataclasses.fields(Batch)})
    else:
        batch = make_batch(WORKLOAD)
        if args.batch_cache:
            import dataclasses
            np.savez(args.batch_cache, **dataclasses.asdict(batch))
    if args.cache_only:
        return
    consts = step_constants(WORKLOAD)
    t_gen = time.perf_counter() - t_gen
    print(f"# generated {batch.n_env} trees, {batch.n_seg} segments, {batch.n_apple} apples in {t_gen:.1f} s",
          file=sys.stderr, flush=True)

    import torch
    from paper_2607_06337_amd import DEFAULT_TUNING, Model, autotune
    torch.cuda.init()
    if args.tuning:
        tuning, tune_log = dict(DEFAULT_TUNING, **json.loads(args.tuning)), None
    else:
        t_tune = time.perf_counter()
        tuning, timings = autotune(batch, consts, AUTOTUNE_CANDIDATES, n_warm=3, n_steps=100)
        tune_log = [dict(c, ms_per_step=round(ms, 4)) for c, ms in timings]
        print(f"# autotune {time.perf_counter() - t_tune:.1f} s: {tuning}", file=sys.stderr, flush=True)
    tuning = {k: tuning[k] for k in TUNING_KEYS}
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    model = Model(batch, consts, tuning)
    st_mem = model.rest_state()
    torch.cuda.synchronize()
    # device memory of the model (static records, scratch) and of one batch state
    memory = dict(model_bytes=int(model.scratch_bytes),
                  state_bytes=int(sum(getattr(st_mem, f).numel() * getattr(st_mem, f).element_size()
                                      for f in st_mem.__dataclass_fields__)),
                  device_bytes_used=int(free0 - torch.cuda.mem_get_info()[0]))
    del st_mem
    # the first timed rollout is the reported one; four more of the same length (continuing
    # from its state) give the median beside it
    ms, wall, n_bad, st_end, what, n_launch, runs = time_gpu(model, args.steps, args.warmup, GRAPH_STEPS, repeats=5)
    # events of the whole rollout (warmup plus the five timed rollouts)
    events = dict(event_counts(model, st_end), steps=args.warmup + 5 * args.steps)
    del st_end
    print(f"# optimized: {args.steps} steps in {ms:.1f} ms ({wall:.2f} s wall), packs={model.n_pack}", file=sys.stderr,
          flush=True)
    plain = None
    if not args.no_plain:
        pm = Model(batch, consts, PLAIN_TUNING)
        pms, _, _, _, _, _, _ = time_gpu(pm, max(1, args.steps // 4), args.warmup)
        plain = dict(value=batch.n_env * max(1, args.steps // 4) / (pms / 1e3), ms_per_step=pms / max(1, args.steps // 4),
                     tuning=PLAIN_TUNING)
        del pm
        print(f"# plain per-step kernel: {plain['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    if args.copy_probe:
        _copy_probe()
    ms_step = ms / args.steps
    value = batch.n_env * args.steps / (ms / 1e3)
    # the step kernel's launches in the timed region: average duration and the algorithmic
    # bytes of the steps one launch runs
    steps_per_launch = args.steps / n_launch
    per_launch_bytes = algorithmic_bytes(batch) * steps_per_launch
    launch_ms = ms / n_launch
    achieved = per_launch_bytes / (launch_ms / 1e3) / 1e9
    prof = profiled_counters("k_step_packs", tuning)
    # measured HBM bytes per step of the profiled launches, times the steps of these launches
    traffic = None
    if prof and prof.get("hbm_bytes_per_launch"):
        traffic = int(prof["hbm_bytes_per_launch"] / prof["tuning"]["steps_per_launch"] * steps_per_launch)
    copy_gbs = copy_bandwidth()
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                copy_peak_GBps=round(copy_gbs, 1), frac_of_copy_peak=round(achieved / copy_gbs, 4),
                kernel="k_step_packs", bytes_per_launch=int(per_launch_bytes),
                launch_us=round(launch_ms * 1e3, 2), launches_timed=n_launch)
    if traffic:
        # measured HBM bytes of the profiled launches over this run's launch time
        roof["traffic_GBps"] = round(traffic / (launch_ms / 1e3) / 1e9, 1)
    if prof and prof.get("valu_insts_per_step"):
        # issue-rate ceiling of the vector ALUs: 1024 SIMDs, one wave64 VALU instruction
        # per 4 cycles at 2.4 GHz; FP32 lane operations (FMA = 2) against 78.6 TFLOP/s
        vi = prof["valu_insts_per_step"]
        roof["valu"] = dict(insts_per_step=vi, frac=round(vi / (ms_step / 1e3) / VALU_ISSUE_PEAK, 4),
                            peak_insts_per_s=VALU_ISSUE_PEAK)
        if prof.get("fp32_flops_per_step"):
            fl = prof["fp32_flops_per_step"]
            roof["valu"].update(fp32_flops_per_step=fl, fp32_frac=round(fl / (ms_step / 1e3) / FP32_PEAK, 4),
                                fp32_peak_flops=FP32_PEAK)
    adj = None
    if not args.no_adjoint:
        adj = adjoint_ratio()
        print(f"# adjoint/forward: {adj}", file=sys.stderr, flush=True)
    rows = None
    if not args.no_row_scale:
        rows = row_scale()
        print(f"# row scale: {rows}", file=sys.stderr, flush=True)
    sph = None
    if not args.no_sphere:
        sph = sphere_fit_leg()
        print(f"# sphere fit: {sph}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batch, consts)
        print(f"# cpu baseline: {cpu['value']:.1f} env-steps/s on {cpu['cores']} threads", file=sys.stderr, flush=True)
        if not args.no_adjoint:
            cpu["adjoint8"] = cpu_adjoint_baseline()
            print(f"# cpu adjoint: {cpu['adjoint8']}", file=sys.stderr, flush=True)
    out = dict(metric="tree-env steps/sec (FP32, 8192 uneven trees) + adjoint/forward cost ratio",
               value=round(value, 1), unit="env-steps/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=round(ms_step, 5), higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32", data="synthetic",
               config=dict(workload=f"{WORKLOAD}: 8192 seeded L-system trees, log-uniform 50-1500 segments, "
                                    f"10-120 apples, in-step random body forces 5% N(0,5N), dt 1 ms",
                           n_env=batch.n_env, segments=batch.n_seg, apples=batch.n_apple,
                           shape=workload_stats(batch), tuning=tuning, rollout=what, autotune=tune_log),
               repeat_ms=[round(x, 3) for x in runs], median_ms_per_step=round(float(np.median(runs)) / args.steps, 5),
               events=events, adjoint_forward_ratio=adj["ratio"] if adj else None, adjoint=adj, nonfinite_envs=n_bad,
               memory=memory, plain_per_step_kernel=plain,
               roofline=roof, cpu_baseline=cpu, row_scale=rows, sphere_fit=sph)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
