/* orchard.h -- C ABI of liborchard.so: a batched forward-dynamics step of many
 * independent, differently shaped articulated apple trees on one MI355X (gfx950).
 *
 * The physical model follows OrchardBench (arXiv 2607.06337):
 *   - every internode is a rigid capsule link joined to its parent's tip by a
 *     compliant two-DoF bending joint whose rest rotation is q_rel
 *     (Sec. "Physical Model", joint-frame equation; Sec. "Compliant branch
 *     dynamics": two bending DoF, twist and translation locked);
 *   - joint stiffness Kp = (pi/4) E r^4 / l (Eq. beam), torque -Kp theta - Kd omega,
 *     integrated implicitly;
 *   - rupture when Kp |theta| > sigma_r pi r^3 / 4 (Eq. break) for N consecutive
 *     steps; the broken joint loses spring and damper in place and becomes a free
 *     hinge (Sec. "Branch breaking");
 *   - apples are free bodies on a tether f = -k_s (x - x_hang) - c_s v whose elastic
 *     part minus the static weight loads the spur, clamped; they detach by a
 *     sustained pull or stem tension (Sec. "Fruit");
 *   - applied forces pass an impulse cap and are disabled on snapped sub-trees
 *     (Sec. "Numerical Stability").
 *
 * Conventions.
 *   - All device pointers are raw HIP device pointers (e.g. torch data_ptr()).
 *   - Segment and apple arrays on the device are in the model's INTERNAL order
 *     (trees grouped into packs, level-major inside a pack).  orchard_model_maps()
 *     gives, for every internal slot, the descriptor's global index.
 *   - Units SI; world frame z up; quaternions (w, x, y, z).
 *   - Functions return orchard_status_t; no C++ exception crosses the ABI.  A
 *     message for the last failure on the calling thread: orchard_last_error().
 *   - Stream-ordered calls are asynchronous and allocate nothing after create.
 *     A model is used by one stream at a time (not thread-safe).
 */
#ifndef ORCHARD_H
#define ORCHARD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orchard_model_s* orchard_model_t;
typedef void* orchard_stream_t; /* a hipStream_t; NULL = the null stream */

typedef enum {
  ORCHARD_OK = 0,
  ORCHARD_ERR_INVALID_ARG = 1,      /* bad pointer, size or parameter            */
  ORCHARD_ERR_INVALID_TOPOLOGY = 2, /* parent >= child, non-positive size, ...   */
  ORCHARD_ERR_OUT_OF_MEMORY = 3,
  ORCHARD_ERR_HIP = 4,              /* a HIP runtime call failed                  */
  ORCHARD_ERR_NONFINITE = 5,        /* an env produced a non-finite state         */
  ORCHARD_ERR_CAPACITY = 6          /* caller's event buffer was too small        */
} orchard_status_t;

/* Tree batch description.  HOST memory, read during orchard_model_create; the
 * caller keeps ownership.  Arrays are concatenated over envs (CSR offsets). */
typedef struct {
  int32_t n_env;
  const int32_t* seg_offset;    /* [n_env+1]                                         */
  const int32_t* seg_parent;    /* [n_seg] env-local parent, -1 = world, parent < i  */
  const double* seg_rest_quat;  /* [n_seg][4] q_rel = conj(Q_parent) Q_child, unit   */
  const double* seg_length;     /* [n_seg] l > 0                                     */
  const double* seg_radius;     /* [n_seg] r > 0                                     */
  const double* seg_density;    /* [n_seg] rho > 0                                   */
  const double* seg_youngs;     /* [n_seg] E > 0                                     */
  const double* seg_mor;        /* [n_seg] modulus of rupture sigma_r > 0            */
  const int32_t* apple_offset;  /* [n_env+1]                                         */
  const int32_t* apple_seg;     /* [n_apple] env-local segment the apple hangs from  */
  const double* apple_hang;     /* [n_apple][3] hang point in that segment's frame   */
  const double* apple_mass;     /* [n_apple] > 0                                     */
  const double* apple_radius;   /* [n_apple] (solid sphere inertia 2/5 m R^2)        */
  const double* apple_detach;   /* [n_apple] detach force threshold f_det > 0        */
  /* step constants */
  double dt;                    /* time step h                                        */
  double gravity[3];
  double tether_k;              /* k_s                                                */
  double tether_zeta;           /* c_s = 2 zeta sqrt(k_s m)                           */
  double damping_zeta;          /* Kd = 2 zeta sqrt(Kp J), J = mean rest mass-matrix  */
  double damping_cd;            /*   diagonal of the joint; if > 0: Kd = c_d Kp       */
  double tension_factor;        /* tension threshold = factor * f_det                 */
  double v_cap;                 /* impulse cap: |F| <= m_body v_cap / h               */
  double react_max_factor;      /* spur reaction clamp = factor * f_det               */
  int32_t n_break, n_pull, n_tension; /* consecutive steps before an event           */
  int32_t pad0;
  uint64_t rng_seed;            /* in-step random body forces (see orchard_step)      */
  double wrench_fraction;       /* fraction of bodies pushed per step (0 = off)       */
  double wrench_sigma;          /* N(0, sigma) per force component                    */
  /* model variants (Sec. "Compliant branch dynamics", Sec. "Fruit") */
  double stiffness_k0;          /* > 0: per-level exponential stiffness instead of    */
  double stiffness_gamma;       /*   Eq. beam: Kp = k0 gamma^depth, depth of the      */
                                /*   joint below the root (root 0), 0 < gamma        */
  int32_t fruit_dof;            /* 3: translational fruit (state: position and        */
                                /*   velocity only); 6 or 0: rigid body (also the    */
                                /*   quaternion and angular velocity)                */
  int32_t pad1;
  /* extras, each off at 0 (Sec. "Compliant branch dynamics", Sec. "Branch breaking",
   * Sec. "Numerical Stability"); orchard_step_backward rejects a model that uses any */
  double drag_lin;              /* c_v: drag force -c_v m v at the centre of mass (1/s) */
  double drag_ang;              /* c_w: drag torque -c_w I w (1/s)                    */
  double drag_snapped;          /* factor on both drags on a snapped sub-tree         */
  double friction_base;         /* Coulomb torque at a broken joint right after the   */
                                /*   break, as a fraction of the limb's largest      */
                                /*   weight moment |g| sum_b m_b |c_b - p_joint|     */
  double friction_growth;       /* factor the torque reaches at the end of the ramp   */
  double friction_ramp_time;    /* length of the linear ramp (s)                      */
  double friction_speed;        /* joint speed (rad/s) below which the friction acts  */
                                /*   as a damper tau_c / friction_speed              */
  double fade_speed;            /* power fade: the part of an applied force along the */
                                /*   body's velocity that pushes it on falls from    */
                                /*   full at this speed to none at twice it          */
  double brake_rate;            /* speed brake: -rate m (|v| - v_cap) v/|v| on a body */
                                /*   with an applied force above v_cap (1/s)         */
  double event_band;            /* >= 0: orchard_events marks an event whose ratio    */
                                /*   lies within event_band of 1 (its threshold) as  */
                                /*   in band: FP32 rounding of the state can move    */
                                /*   such an event by a step (Eq. break, Sec. "Fruit"); */
                                /*   0 = none marked                                  */
} orchard_model_desc_t;

/* Kernel mapping choices (nullable in create: defaults {128, 1.0, 1, 0, 0, 128, 0, 0, 0}).
 * threads: workgroup size for the pack kernel (64, 128, 256 or 512).  pack_fill: a
 * pack collects trees of similar depth until it holds about pack_fill * threads *
 * depth nodes (0 = one tree per pack).  lds_width (0 .. threads): capacity, in nodes
 * per level, of the LDS buffer through which neighbouring levels of a pack exchange
 * their data (2 x 28 x lds_width floats of LDS per workgroup); packs are then also
 * closed before a level would exceed it, and a tree wider than it exchanges through
 * global scratch.  0 = global scratch for every pack.  pack_skew (LDS exchange only):
 * 1 = place trees at level offsets inside a strip of pack_fill x (deepest tree) levels
 * so that their widest levels do not coincide.  wave_width (0 .. 64, ignored with
 * persistent = 1): size buckets; a tree whose widest level has at most wave_width nodes
 * goes to a wave pack that one wavefront walks alone, with no workgroup barrier, its
 * levels exchanging through 28 x 64 floats of LDS of its own (threads / 64 wave packs per
 * workgroup, launched after the workgroup-wide packs); 0 = every pack takes a whole
 * workgroup.  big_threads (0, 256 or 512; used when it exceeds lds_width, ignored with
 * persistent = 1): the wide-tree bucket; a tree whose widest level exceeds lds_width but
 * not big_threads goes to a pack of big_threads work-items with an LDS exchange of
 * big_threads slots instead of exchanging through global scratch; its launch goes on the
 * caller's stream and the other packs' launch on a second stream of the model's (default
 * priority), concurrently, both joined to the caller's stream before orchard_step's work
 * there ends.  The adjoint's recompute and reverse pass run these packs in the wide-tree
 * mapping when every pack of the model is in the bucket, otherwise every pack in the main
 * mapping.  No mapping choice changes any result bit. */
typedef struct {
  int32_t threads;
  float pack_fill;
  int32_t steps_per_launch;     /* steps fused in one launch by orchard_step (>= 1)   */
  int32_t persistent;           /* 1: persistent grid pulling packs from a queue      */
  int32_t adjoint_ckpt_max;     /* > 0: allocate recompute buffers for                */
                                /*   orchard_step_backward with ckpt_every up to this */
                                /*   (two sets of K scratch copies and K + 1 state    */
                                /*   records, a second stream and five events)        */
  int32_t lds_width;
  int32_t pack_skew;
  int32_t wave_width;
  int32_t big_threads;
} orchard_tuning_t;

typedef struct {
  int64_t n_env, n_seg, n_apple;
  int32_t n_pack, max_depth;
  int64_t scratch_bytes;        /* device memory the model owns                       */
  int32_t apple_planes;         /* float planes of the apple state: 13 (rigid body) or */
                                /*   6 (translational fruit)                          */
  int32_t n_wave_packs;         /* packs walked by one wavefront (tuning.wave_width)   */
  int32_t n_big_packs;          /* packs of the wide-tree bucket (tuning.big_threads)  */
  int32_t pad;
} orchard_layout_t;

/* Caller-owned device state (internal order). */
typedef struct {
  float* q;            /* [n_seg][2]   bending angles (theta_x, theta_y)               */
  float* qd;           /* [n_seg][2]   their rates                                      */
  float* apple;        /* [P][n_apple] planes, P = layout.apple_planes: x(3) v(3) and  */
                       /*   for a rigid-body fruit quat(4, w first) omega(3);          */
                       /*   v is the absolute velocity.  x: while attached, the stretch */
                       /*   x_abs - x_hang plus h v (the stretch advanced by the apple  */
                       /*   but not yet by the hang point); once detached, x_abs minus  */
                       /*   the rest hang point (orchard_model_apple_rest)              */
  uint8_t* seg_evt;    /* [2][n_seg]   broken flag, consecutive-exceed counter          */
  uint8_t* apple_evt;  /* [4][n_apple] detached flag, pull counter, tension counter,   */
                       /*              detach path (1 pull, 2 tension)                  */
  int32_t* evt_step;   /* [n_seg + n_apple] step of break / detach, -1 = none          */
  uint32_t* env_status;/* [n_env] bit 0: non-finite state produced; env frozen from   */
                       /*   the next step on; bit 1: an apple state was among the    */
                       /*   non-finite values (with bit 0)          */
  int64_t* step;       /* device scalar: index of the next step (event stamps, RNG)    */
  float* evt_ratio;    /* [n_seg + n_apple] threshold ratio on the step of the event:  */
                       /*   mu = Kp |theta| / M_max for a break (Eq. break), pi =     */
                       /*   |F| / f_det for a pull detach, tau = k_s |s| / (alpha     */
                       /*   f_det) for a tension detach (Sec. "Fruit"); written only  */
                       /*   on that step (orchard_state_rest zeroes it); not part of  */
                       /*   checkpoint records.  Nullable: no ratios recorded         */
} orchard_state_t;

typedef struct {
  const float* kp;     /* [n_seg] joint stiffness (both DoF), device                    */
  const float* kd;     /* [n_seg] joint damping                                         */
} orchard_params_t;

typedef struct {
  const float* body_wrench;  /* [n_seg][6] force(3), torque(3) about the COM, world; or NULL */
  int64_t body_wrench_stride;/* floats between consecutive steps' arrays; 0 = constant      */
  const float* apple_force;  /* [n_apple][3] world force on the apple; or NULL              */
  int64_t apple_force_stride;/* floats between steps; 0 = constant                         */
} orchard_inputs_t;

typedef struct {
  int32_t env;     /* descriptor env index                                  */
  int32_t kind;    /* 1 break, 2 detach by pull, 3 detach by stem tension   */
  int32_t id;      /* env-local descriptor segment / apple index            */
  int32_t step;
  float ratio;     /* state.evt_ratio of the event (0 if the state has none) */
  int32_t in_band; /* 1 if |ratio - 1| < the model's event_band            */
} orchard_event_t;

/* Build a model: validates the description (synchronously), derives masses,
 * inertias, Kp (Eq. beam), M_max (Eq. break) and Kd on the host in FP64, groups
 * trees into packs, and copies everything to the current HIP device.
 * Limits: at most 2^27 segments and 2^26 apples per model (the kernels address
 * per-segment and per-apple records with 32-bit byte offsets); larger batches are
 * INVALID_ARG.
 * Errors: INVALID_ARG, INVALID_TOPOLOGY (parent >= child, sizes <= 0, quaternion
 * not unit within 1e-6, apple_seg out of range), OUT_OF_MEMORY, HIP; on error
 * nothing stays allocated and *out is NULL.  Test hook: with ORCHARD_FAIL_ALLOC=k in
 * the environment, the k-th device allocation of the call (k = 1, 2, ...) fails as
 * if the device were out of memory. */
orchard_status_t orchard_model_create(const orchard_model_desc_t* desc, const orchard_tuning_t* tuning,
                                      orchard_model_t* out);
void orchard_model_destroy(orchard_model_t model);
orchard_status_t orchard_model_layout(orchard_model_t model, orchard_layout_t* out);

/* Host arrays: seg_map[n_seg] = descriptor global segment index of each internal
 * slot; apple_map[n_apple] likewise.  Either may be NULL. */
orchard_status_t orchard_model_maps(orchard_model_t model, int32_t* seg_map, int32_t* apple_map);

/* Rest hang points of the apples, host double [n_apple][3], internal order (the
 * origin of a detached apple's position state).  Attached apples keep their stretch
 * relative to the current hang point as state, so the stiff tether never sees
 * absolute-position round-off in FP32.  Synchronises the device (the points follow
 * orchard_model_rebuild). */
orchard_status_t orchard_model_apple_rest(orchard_model_t model, double* host_out);

/* Derived Kp, Kd (device arrays [n_seg], internal order) -- the defaults of the
 * differentiable parameters. */
orchard_status_t orchard_default_params(orchard_model_t model, float* kp, float* kd, orchard_stream_t stream);

/* On-device rebuild of every world's geometry (Sec. "Parallelism and cost": the
 * per-world geometry build as one kernel, one thread per world).  seg_perturb: device
 * double [n_seg][4] in DESCRIPTOR order — length factor, radius factor, and a bend of the
 * segment's rest orientation about its own x axis then its y axis (radians).  The
 * factors apply to the descriptor values given at create; every parameter that depends
 * on them is derived again on the device in FP64 with the operations create uses (mass
 * properties, Kp by Eq. beam or the per-level model, M_max by Eq. break, Kd from the rest
 * mass-matrix diagonal, the friction scale, the rest pose and the fruit's rest hang
 * points; a hang point keeps its place in its segment's frame, scaled with the length).
 * Factors (1, 1, 0, 0) reproduce the created model.  Topology, packing, fruit masses and
 * detach forces are unchanged; the default gains change, so call orchard_default_params
 * again.  A world with a non-positive or non-finite factor is left as it is and counted
 * in *rejected (device int32, nullable, zeroed by the call).  Stream-ordered, no
 * allocation; it uses the model's step scratch as workspace, so it must not overlap a
 * step of the same model. */
orchard_status_t orchard_model_rebuild(orchard_model_t model, const double* seg_perturb, int32_t* rejected,
                                       orchard_stream_t stream);

/* Rest state: q = qd = 0 (the generated skeleton pose), apples hanging
 * m |g| / k_s below their hang point at rest, counters and flags zero, event steps
 * -1, event ratios 0 (if the state has them), status 0, step counter 0. */
orchard_status_t orchard_state_rest(orchard_model_t model, const orchard_state_t* state, orchard_stream_t stream);

/* Advance every env by n_steps (stream-ordered, asynchronous, no allocation).
 * Per step: event tests on the current state (rupture, detachment; an event stamps
 * its step and, if the state has the array, its threshold ratio), snapped mask,
 * applied forces (inputs plus, if wrench_fraction > 0, the counter-based random
 * forces), apple reactions, bias forces, factorisation of the implicit mass
 * matrix, solve, integration.  If ckpt is non-NULL, the full state is written to
 * ckpt every ckpt_every steps (ckpt[k] = state before step k*ckpt_every of this
 * call), orchard_ckpt_words() 32-bit words per checkpoint; ckpt needs room for
 * ceil(n_steps / ckpt_every) records. */
orchard_status_t orchard_step(orchard_model_t model, const orchard_state_t* state, const orchard_params_t* params,
                              const orchard_inputs_t* inputs, int32_t n_steps, float* ckpt, int32_t ckpt_every,
                              orchard_stream_t stream);

/* ---- batched sphere-fit detector (Sec. "Geometric fruit perception", Eq. spherefit) ---- */

/* Gate of a sphere candidate: radius in [r_min, r_max] (m), RMS geometric residual at
 * most rms_max (m), at least min_points points (and at least 4). */
typedef struct {
  float r_min, r_max, rms_max;
  int32_t min_points;
} orchard_sphere_gate_t;

/* Fit a sphere to every patch of back-projected depth points: the least-squares solution
 * of 2 p.c + b = |p|^2 with b = R^2 - |c|^2 over the patch's points, its radius
 * R = sqrt(b + |c|^2), the RMS of the geometric residuals |p - c| - R, and the gate.
 * points: device float [n_points][3]; patch_offset: device int32 [n_patch + 1],
 * non-decreasing, patch k = points[patch_offset[k] .. patch_offset[k+1]); gate: host.
 * out: device float [n_patch][8] = centre x, y, z, radius, rms residual, point count,
 * status (0 accepted, 1 too few points, 2 degenerate (no volume spanned), 3 radius out
 * of range, 4 residual too large), 0.  Stream-ordered, no allocation.  Errors:
 * INVALID_ARG (null pointer with n_patch > 0, n_patch < 0, a gate with r_max < r_min or
 * negative bounds), HIP. */
orchard_status_t orchard_sphere_fit(const float* points, const int32_t* patch_offset, int32_t n_patch,
                                    const orchard_sphere_gate_t* gate, float* out, orchard_stream_t stream);

/* Bytes of the library's fixed step scratch (one array per GPU, held until the process
 * ends). */
#define ORCHARD_STATIC_SCRATCH_BYTES ((uint64_t)64 << 20)

/* orchard_step for callers that cannot allocate device memory at step time (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * identical arguments, kernels and results, but the step's scratch (the per-node
 * scratch blocks, the dense apple-node arrays and the persistent queue counter) lives
 * in the library's fixed device array of ORCHARD_STATIC_SCRATCH_BYTES instead of the
 * model's own scratch.  Calls no hipMalloc, hipFree or allocating routine.  A model
 * whose step scratch (reported by the error message) exceeds the array is rejected
 * with ORCHARD_ERR_CAPACITY before any device work; about 120 K segments fit a model
 * without adjoint support.  The model's device must be current.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (two streams, two
 * threads) race and must be serialised by the caller.  The queue counter is cleared by
 * a kernel at the start of each call; nothing else in the array has to start at any
 * value (every field a step reads was written earlier in the same step). */
orchard_status_t orchard_step_static_scratch(orchard_model_t model, const orchard_state_t* state,
                                             const orchard_params_t* params, const orchard_inputs_t* inputs,
                                             int32_t n_steps, float* ckpt, int32_t ckpt_every,
                                             orchard_stream_t stream);

/* Adjoint state (caller-owned device arrays, internal order): dL/dq, dL/dqd
 * [n_seg][2] and dL/d(apple position state), dL/d(apple velocity) [3][n_apple]. */
typedef struct {
  float* q;
  float* qd;
  float* apple_x;
  float* apple_v;
} orchard_adjoint_t;

/* Reverse-mode gradient of a rollout (growth direction "differentiation"):
 * given the checkpoints a forward orchard_step call wrote (ckpt, ckpt_every <=
 * tuning.adjoint_ckpt_max) and, in adj, dL/dS_T of the state after its n_steps
 * steps, recompute each checkpoint segment once (every step keeps what its reverse
 * pass reads in a scratch copy of its own) and walk the steps backwards: per step
 * lambda = Mt^-1 (h dL/dqd+) with the step's own factorisation (Mt is symmetric),
 * then the reverse of the inverse dynamics, kinematics, apple tether and reaction
 * and of the implicit-Euler update, with every discrete switch of the forward
 * (breaks, detachments, clamp branch, impulse cap, snapped mask) frozen.
 * On return adj holds dL/dS_0 (in place).  Accumulates (+=) into grad_kp, grad_kd
 * [n_seg] and, if non-NULL, grad_apple_force [n_steps][n_apple][3].  Params and
 * inputs must be those of the forward call.  The quaternion and angular velocity of
 * the apples are not differentiated (no torque acts on an apple); a fruit that
 * detaches inside the window carries the dependence of its launch point (hang point
 * plus stretch) on the tree pose into the tree's gradient.  Stream-ordered with respect to stream; the recompute
 * of each checkpoint segment runs on the model's second stream, overlapping the
 * reverse sweep of the segment after it (two sets of recompute buffers), and is joined
 * back before the call's last work on stream.  No allocation. */
orchard_status_t orchard_step_backward(orchard_model_t model, const float* ckpt, int32_t ckpt_every, int32_t n_steps,
                                       const orchard_params_t* params, const orchard_inputs_t* inputs,
                                       const orchard_adjoint_t* adj, float* grad_kp, float* grad_kd,
                                       float* grad_apple_force, orchard_stream_t stream);

/* Tip positions p_b + R_b (0, 0, l_b) (world frame, tree base at the origin) of the
 * segments node[k] (internal indices, device int32 [n_tips]) at joint angles q
 * (device [n_seg][2]) into out (device float [n_tips][3]).  Stream-ordered.
 * Precondition: the model was created with adjoint support (tuning.adjoint_ckpt_max
 * >= 1), whose scratch holds the tip kernels' fields; otherwise ORCHARD_ERR_INVALID_ARG
 * is returned before any device work.  The same holds for orchard_tips_backward. */
orchard_status_t orchard_tips(orchard_model_t model, const float* q, int32_t n_tips, const int32_t* node, float* out,
                              orchard_stream_t stream);

/* Accumulates (+=) into grad_q ([n_seg][2]) the gradient of sum_k grad_out[k] . tip_k(q). */
orchard_status_t orchard_tips_backward(orchard_model_t model, const float* q, int32_t n_tips, const int32_t* node,
                                       const float* grad_out, float* grad_q, orchard_stream_t stream);

/* Size in 32-bit words of one checkpoint record written by orchard_step. */
int64_t orchard_ckpt_words(orchard_model_t model);

/* Restore a state from one checkpoint record (stream-ordered). */
orchard_status_t orchard_ckpt_load(orchard_model_t model, const orchard_state_t* state, const float* record,
                                   orchard_stream_t stream);

/* Events so far (synchronises the stream).  Writes up to capacity events to
 * host_out in (env, step, kind, id) order and their total count to *n_out;
 * returns ORCHARD_ERR_CAPACITY if there were more. */
orchard_status_t orchard_events(orchard_model_t model, const orchard_state_t* state, orchard_event_t* host_out,
                                int32_t capacity, int32_t* n_out, orchard_stream_t stream);

/* Per-env status words (synchronises).  Returns ORCHARD_ERR_NONFINITE if any env
 * is flagged. */
orchard_status_t orchard_status(orchard_model_t model, const orchard_state_t* state, uint32_t* host_env_status,
                                orchard_stream_t stream);

/* Message of the last error on this thread ("" if none). */
const char* orchard_last_error(void);

/* ---- K-step rollouts as one HIP graph (uneven batching: launch-bound inner loops) ----
 * orchard_graph_create captures n_steps of orchard_step (no checkpoints) on a private
 * stream into a HIP graph of kernel nodes only (no allocation, copy or memset nodes)
 * and instantiates it.  The state, params and inputs pointers are baked in: each
 * orchard_graph_launch advances that same state by n_steps on `stream`, reading input
 * rows 0 .. n_steps-1 again (stride semantics as in orchard_step).  The step counter
 * lives in device memory, so event stamps and the random wrench keys keep counting
 * across replays and a replay equals the eager call bit for bit.  The graph holds no
 * reference to the model's host object but uses its device buffers: destroy it first.
 * Errors: ORCHARD_ERR_INVALID_ARG as orchard_step, ORCHARD_ERR_HIP if capture or
 * instantiation fails (the message names the HIP error). */
typedef struct orchard_graph_s* orchard_graph_t;
orchard_status_t orchard_graph_create(orchard_model_t model, const orchard_state_t* state, const orchard_params_t* params,
                                      const orchard_inputs_t* inputs, int32_t n_steps, orchard_graph_t* out);
orchard_status_t orchard_graph_launch(orchard_graph_t graph, orchard_stream_t stream);
void orchard_graph_destroy(orchard_graph_t graph);

/* ---- autotuner: pick the kernel mapping for a batch by measurement ----
 * Builds a model for each of the n_candidates mappings (adjoint_ckpt_max ignored),
 * runs n_warm steps from rest, then times n_steps steps with HIP events on `stream`
 * (default params, the descriptor's own random wrenches, no other inputs), and writes
 * the fastest mapping to *best and every candidate's milliseconds per step to
 * ms_out[n_candidates] (nullable; a candidate that fails to build gets -1).  Allocates
 * and frees its own state; synchronises the stream.  Errors: ORCHARD_ERR_INVALID_ARG
 * for null pointers, n_candidates < 1 or n_steps < 1; the descriptor's own errors if
 * no candidate builds. */
orchard_status_t orchard_autotune(const orchard_model_desc_t* desc, const orchard_tuning_t* candidates,
                                  int32_t n_candidates, int32_t n_warm, int32_t n_steps, orchard_tuning_t* best,
                                  float* ms_out, orchard_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* ORCHARD_H */
