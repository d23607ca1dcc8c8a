// Device-side model description and small vector helpers for the orchard kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace orchard {

// ---- scratch fields: one float per node per field, field f at scr + f * n_seg -----------
// A node's "publication" is what its neighbours on the next level read: children in the
// down passes, the parent in the up pass.  Packs whose levels fit the workgroup keep
// publications in LDS (double-buffered by level parity); wide packs keep them in these
// global fields.
enum : int {
  // Publication of the two down passes (values at the node's tip point), one slot of 28
  // floats; an LDS slot uses the same offsets.  Down 1 writes F_R .. F_SNAP, down 2
  // F_SNAP .. F_AT + 5, a fused pass (down 2 of one step, down 1 of the next) all of it.
  F_R = 0,          // 6: body rotation, columns 1 and 2 (column 0 is their cross product)
  F_PT = 6,         // 3: tip point (absolute; only detached apples use positions)
  F_W = 9,          // 3: angular velocity
  F_VT = 12,        // 3: linear velocity of the tip point
  F_AVA = 15,       // 3: velocity-product (+ base) acceleration at the tip, angular
  F_AVL = 18,       // 3:   linear
  F_SNAP = 21,      // 1: flags: snapped (down 1 part) + 2 x the env's frozen flag (down 2 part)
  N_PUB1 = 22,
  F_AT = 22,        // 6: acceleration at the tip (ang, lin)
  N_PUBD = 28,
  // node-private data kept from the down pass for the up and second down passes; the
  // own-body inertia, l z and the spring terms are formed again from static data, z and
  // the state instead of being stored
  F_A0 = 28,        // 3: joint axis x (world)
  F_A1 = 31,        // 3: joint axis y (world)
  F_WV = 34,        // 6: angular velocity and joint-point velocity (the velocity-product
                    //    acceleration and the bias are formed from them again)
  F_FLG = 40,       // 1: flags of the step (broken, snapped, broken at the start, rupture count)
  // up-pass publication (27): articulated inertia and bias at the node's joint point
  F_IA = 60,        // 6: A (rotational block, sym)
  F_IB = 66,        // 9: B (coupling block, row major)
  F_IM = 75,        // 6: M (linear block, sym)
  F_PA = 81,        // 6: bias (ang, lin)
  N_PUBU = 27,
  // node-private factor data for the second down pass: qdd = D^-1 u - W^T (A_parent + c)
  F_WM = 87,        // 12: W = U D^-1, U = I^A S (col 0: ang 3 lin 3, col 1: ang 3 lin 3)
  F_DU = 99,        // 2: D^-1 u, u = tau - S^T p^A
  F_DI = 101,       // 3: D^-1 (00 01 11), stored only in save mode (the adjoint's solves)
  // node-private outputs of the down 1 and up passes, each a contiguous range of fields
  N_OUT1 = 13,      // F_A0 .. F_FLG
  N_OUTU = 14,      // F_WM .. F_DU + 1
  F_SFRZ = 104,     // 1: the env's frozen flag at the start of the step, stored in save mode
  F_SSNP = 105,     // 1: the snapped flag, stored in save mode
  F_Z = 106,        // 3: body axis z (world), stored in save mode only: the step's later
                    //    passes rebuild it from F_A0, F_A1 and theta_y
  N_FIELDS = 128,
  // Nodes that carry apples (a minority) keep their apple data in two dense arrays
  // indexed by the node's apple-node index, so it moves in whole sectors:
  // the kinematics down 1 keeps for the apple phase, [n_anode][K_N] floats
  K_R = 0,          // 9: body rotation, row major
  K_W = 9,          // 3: angular velocity
  K_V = 12,         // 3: velocity of the joint point
  K_AA = 15,        // 3: velocity-product (+ base) acceleration at the joint point, angular
  K_AL = 18,        // 3:   linear
  K_PJ = 21,        // 3: joint point (absolute)
  K_N = 24,
  // the apples' sums the apple phase hands to the up pass, [n_anode][E_N] floats
  E_MO = 0,         // 1: virtual mass
  E_HO = 1,         // 3: its first moment about the joint point
  E_JO = 4,         // 6: its rotational inertia about the joint (xx yy zz xy xz yz)
  E_P = 10,         // 6: reaction bias (ang, lin)
  E_N = 16,
  N_PUB_MAX = 28,
  X_STRIDE = 28,     // LDS exchange floats per node slot (N_PUB_MAX, a multiple of 16 B)
  // ---- fields of the adjoint ----
  // saved by the forward step in save mode (the body frame is rebuilt from F_A1 and F_Z)
  F_SR = 128,       // 9: body rotation, row major (scratch of the tip-position kernels only)
  F_SAVP = 137,     // 6: velocity-product (+ base) acceleration at the joint point
  F_SIA = 143,      // 21: articulated inertia before the pivot update (A 6, B 9, M 6)
  F_SPA = 164,      // 6: articulated bias before the pivot update
  F_SA = 170,       // 6: total acceleration at the joint point
  F_SQDD = 176,     // 2: joint accelerations
  // adjoint passes
  F_LU = 178,       // 2: D^-1 u of the solve M lambda = qdd_bar
  F_LPA = 180,      // 6: bias of that solve passed to the parent
  F_LA = 186,       // 6: acceleration of that solve at the tip
  F_NU = 192,       // 6: virtual velocity nu at the joint point
  F_LAM = 198,      // 2: lambda
  F_RB = 200,       // 27: reverse-pass publication: tau_bar 3, omega_bar 3, vt_bar 3, At_bar 6, Avt_bar 6, f_lin 3,
                    //     joint-point position adjoint of the sub-tree 3
  N_FIELDS_ADJ = 228
};

// Static records read by the forward step: one 32-byte record per node for the first down
// pass and one 64-byte record per apple (a few wide loads instead of one load per array).
struct NodeRec {
  float4 rq;    // rest quaternion (w, x, y, z)
  float l;      // length
  float inv_mmax;  // 1 / M_max (rupture moment)
  int par;      // parent (-1 for a root)
  int anode;    // apple-node index, -1 if the segment carries no apple
};
static_assert(sizeof(NodeRec) == 32, "the first down pass reads one 32-byte record per segment");
struct AppleRec {
  float4 hang;  // hang point in the segment frame, mass
  float4 par;   // (1 / f_det, c_s, F_max, 1 / (alpha f_det))
  float4 rest;  // rest hang point (origin of a detached apple's position), h / m
  int4 link;    // (node, env, 1 if the first apple of its node, the node's apple-node index)
};

enum : int32_t { X_DRAG = 1, X_RAILS = 2, X_FRIC = 4 };
struct ExtraConsts {
  float drag_lin, drag_ang, drag_snp;
  float fric_base, fric_growth, fric_inv_ramp, fric_speed;  // fric_inv_ramp < 0: no ramp
  float fade, brake;
  const float* wmom;         // per node: the limb's largest weight moment (friction scale)
};

struct DevModel {
  int32_t n_env, n_seg, n_apple, n_pack;
  // packs: nodes [pack_node[p], pack_node[p+1]); levels lvl_off[pack_lvl[p] .. pack_lvl[p+1]-1]
  // (the last entry of a pack is its end)
  const int32_t* pack_node;
  const int32_t* pack_lvl;
  const int32_t* lvl_off;
  const int32_t* pack_wmax;  // nodes on the pack's widest level: its levels exchange through
                             // LDS when that fits the launch's exchange buffer (<= lds_cap)
  const int32_t* pack_apl;   // [n_pack+1] apples of pack p: pack_apl[p] .. pack_apl[p+1]-1
  const NodeRec* nrec;       // per node (internal order)
  const int4* ntopo;         // per node: (env, first child, children | apples << 16, apple-node index)
  const AppleRec* arec;      // per apple (internal order)
  // per node (internal order)
  const int32_t* par;        // parent node, -1 = world
  const int32_t* child;      // first child node
  const int32_t* nchild;     // number of children (contiguous)
  const int32_t* env;        // descriptor env index
  const int32_t* orig;       // env-local descriptor segment index
  const uint64_t* hkey;      // random-wrench key of the node (rng_node_key)
  const int32_t* apple_beg;  // [n_seg+1] apples of node i: apple_beg[i] .. apple_beg[i+1]-1
  const float4* rq;          // rest quaternion (w, x, y, z)
  const float4* geo;         // (l, m, Jt about the joint, Ia)
  const float* len;          // l alone, for the passes that need only the length
  const float* mmax;         // rupture moment
  // per apple (internal order)
  const float4* ahang;       // (hang x, y, z in the segment frame, mass)
  const float4* apar;        // (f_det, c_s, F_max, unused)
  const float4* ahrest;      // rest hang point (x, y, z, unused): origin of a detached apple's position
  // constants
  float h, gx, gy, gz, ks, alpha, vcap, pad;
  int32_t n_break, n_pull, n_tension, use_rng;
  uint64_t seed;
  uint32_t rng_thr;
  float wsig;
  int32_t apl;               // float planes of the apple state: 13 (rigid body) or 6 (translational)
  // extras (drag, post-break friction ramp, power fade, speed brake): which are on, and
  // their constants in device memory, read only where an extra is on (so they hold no
  // scalar registers through the step's loops)
  int32_t xflags;            // X_DRAG | X_RAILS | X_FRIC
  const struct ExtraConsts* xc;
  float* scr;                // blocks of 64 nodes, each [scr_nf][64] floats (see scr_idx)
  float* asnap;              // [n_anode][K_N] kinematics of the nodes that carry apples
  float* aext;               // [n_anode][E_N] apple sums per node that carries apples
  int32_t* queue;            // persistent-kernel pack counter(s)
  int32_t save_adj;          // forward step also writes the fields the adjoint reads back
  int32_t scr_nf;            // fields per node: N_FIELDS, or N_FIELDS_ADJ with adjoint support
  int32_t lds_cap;           // LDS exchange capacity in nodes per level (0: global exchange)
  int32_t n_wide;            // packs [0, n_wide) take a whole workgroup; packs [n_wide, n_pack)
                             // are walked by one wavefront each, threads / 64 per workgroup
  int32_t pack_base;         // pack of the launch's first workgroup
};

// Scratch layout: nodes in blocks of 64 (one wavefront), each block [scr_nf][64].  A node's
// fields then sit in one ~26-50 KB window instead of scr_nf streams n_seg apart, which keeps
// DRAM rows and TLB entries shared across the fields a wavefront touches.
__device__ __forceinline__ size_t scr_idx(const DevModel& M, int f, int i) {
  return ((size_t)(i >> 6) * (size_t)M.scr_nf + (size_t)f) * 64u + (size_t)(i & 63);
}

// Static per-pack tables that no kernel writes are read through the constant address
// space, so a uniform index becomes a scalar load.
#ifndef ORCHARD_CONST_AS
#define ORCHARD_CONST_AS __attribute__((address_space(4)))
#endif
template <class T>
__device__ __forceinline__ T ldc(const T* p, int64_t i) {
  return ((const ORCHARD_CONST_AS T*)p)[i];
}

// element idx of p with the byte offset formed in 32 bits (arrays stay below 4 GiB), so
// the address is a uniform base plus one 32-bit lane offset
template <class T>
__device__ __forceinline__ T& at(T* p, uint32_t idx) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + idx * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ const T& at(const T* p, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + idx * (uint32_t)sizeof(T));
}

struct DevState {
  float2* q;
  float2* qd;
  float* apple;       // [13][n_apple]
  uint8_t* seg_evt;   // [2][n_seg]
  uint8_t* apple_evt; // [4][n_apple]
  int32_t* evt_step;  // [n_seg + n_apple]
  uint32_t* status;   // [n_env]
  int64_t* step;
  float* evt_ratio;   // [n_seg + n_apple] threshold ratio on an event's step, or null
};

struct DevInputs {
  const float* kp;
  const float* kd;
  const float* wrench;
  int64_t wrench_stride;
  const float* aforce;
  int64_t aforce_stride;
};

// ---- small vector helpers ---------------------------------------------------------------
struct V3 { float x, y, z; };
__device__ __forceinline__ V3 v3(float a, float b, float c) { return V3{a, b, c}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return V3{fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z), fmaf(a.x, b.y, -a.y * b.x)};
}
__device__ __forceinline__ V3 fma3(float s, V3 a, V3 b) { return V3{fmaf(s, a.x, b.x), fmaf(s, a.y, b.y), fmaf(s, a.z, b.z)}; }

static_assert(F_A1 == F_A0 + 3 && F_WV == F_A1 + 3 && F_FLG == F_WV + 6 && F_FLG + 1 - F_A0 == N_OUT1,
              "down 1 outputs are one field range");
static_assert(F_Z > F_SSNP && F_Z + 3 <= N_FIELDS, "the saved body axis sits among the save-mode fields");
static_assert(F_DU == F_WM + 12 && F_DU + 2 - F_WM == N_OUTU, "up outputs are one field range");
static_assert(F_AT == F_SNAP + 1 && N_PUB1 == F_SNAP + 1 && N_PUBD == F_AT + 6 && N_PUBD <= X_STRIDE &&
              N_PUBD <= F_A0 && F_FLG < F_IA, "down-pass publication slot, then node-private fields");

// symmetric 3x3 stored (xx yy zz xy xz yz)
struct Sym3 { float xx, yy, zz, xy, xz, yz; };
__device__ __forceinline__ V3 mul(const Sym3& A, V3 v) {
  return V3{fmaf(A.xx, v.x, fmaf(A.xy, v.y, A.xz * v.z)), fmaf(A.xy, v.x, fmaf(A.yy, v.y, A.yz * v.z)),
            fmaf(A.xz, v.x, fmaf(A.yz, v.y, A.zz * v.z))};
}
// general 3x3 row major
struct Mat3 { float m[9]; };
__device__ __forceinline__ V3 mul(const Mat3& A, V3 v) {
  return V3{fmaf(A.m[0], v.x, fmaf(A.m[1], v.y, A.m[2] * v.z)), fmaf(A.m[3], v.x, fmaf(A.m[4], v.y, A.m[5] * v.z)),
            fmaf(A.m[6], v.x, fmaf(A.m[7], v.y, A.m[8] * v.z))};
}
__device__ __forceinline__ V3 mulT(const Mat3& A, V3 v) {
  return V3{fmaf(A.m[0], v.x, fmaf(A.m[3], v.y, A.m[6] * v.z)), fmaf(A.m[1], v.x, fmaf(A.m[4], v.y, A.m[7] * v.z)),
            fmaf(A.m[2], v.x, fmaf(A.m[5], v.y, A.m[8] * v.z))};
}

// ---- SplitMix64 (Steele, Lea & Flood 2014): output mix of x + golden gamma ------------------
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Random-wrench draws: static key of (env, env-local segment) and the per-step draw
// x = splitmix64(key ^ splitmix64(step)); the top 24 bits select, a selected segment's
// uniforms are bits 63..40 and 39..16 of y1 = splitmix64(x) and y2 = splitmix64(y1).
__host__ __device__ __forceinline__ uint64_t rng_node_key(uint64_t seed, uint64_t env, uint64_t seg) {
  return splitmix64(splitmix64(seed ^ splitmix64(env)) ^ splitmix64(seg));
}

// Applied force on segment i at the step whose key is kstep = splitmix64(step): the input
// wrench plus the counter-based random force (node key hkey), disabled on a snapped
// sub-tree; then, with the rails on, the power fade and the speed brake on the body's
// centre-of-mass velocity vc; last the impulse cap |F| <= m v_cap / h.  Returns false if
// there is none.
__device__ __forceinline__ bool applied_force(const DevModel& M, const DevInputs& I, int i, uint64_t kstep, int s_call,
                                              float m, bool snp, uint64_t hkey, V3 vc, V3& F, V3& T) {
  F = v3(0, 0, 0);
  T = v3(0, 0, 0);
  if (snp) return false;
  bool any = false;
  if (I.wrench) {
    const float* wp = I.wrench + (int64_t)s_call * I.wrench_stride;
    const uint32_t o = 6u * (uint32_t)i;
    F = v3(at(wp, o), at(wp, o + 1), at(wp, o + 2));
    T = v3(at(wp, o + 3), at(wp, o + 4), at(wp, o + 5));
    any = true;
  }
  if (M.use_rng) {
    const uint64_t x = splitmix64(hkey ^ kstep);
    if ((uint32_t)(x >> 40) < M.rng_thr) {
      const uint64_t y1 = splitmix64(x), y2 = splitmix64(y1);
      const float sc = 1.f / 16777216.f;
      const float u0 = ((float)(uint32_t)(y1 >> 40) + 0.5f) * sc;
      const float u1 = ((float)(uint32_t)((y1 >> 16) & 0xFFFFFFu) + 0.5f) * sc;
      const float u2 = ((float)(uint32_t)(y2 >> 40) + 0.5f) * sc;
      const float u3 = ((float)(uint32_t)((y2 >> 16) & 0xFFFFFFu) + 0.5f) * sc;
      // Box-Muller
      const float r0 = sqrtf(-2.f * logf(u0)), r1 = sqrtf(-2.f * logf(u2));
      float s1, c1v, s3, c3;
      sincosf(6.283185307179586f * u1, &s1, &c1v);
      sincosf(6.283185307179586f * u3, &s3, &c3);
      F = F + M.wsig * v3(r0 * c1v, r0 * s1, r1 * c3);
      any = true;
    }
  }
  if (any && (M.xflags & X_RAILS)) {
    const float sp = sqrtf(dot(vc, vc));
    if (sp > 0.f) {
      const float fade = M.xc->fade, brake = M.xc->brake;
      const V3 u = (1.f / sp) * vc;
      const float fu = dot(F, u);
      // power fade: the push along the motion falls from full at the fade speed to
      // nothing at twice it
      if (fade > 0.f && fu > 0.f && sp > fade) {
        const float phi = fmaxf(0.f, 1.f - (sp - fade) / fade);
        F = F - ((1.f - phi) * fu) * u;
      }
      // soft speed brake above the speed limit
      if (brake > 0.f && sp > M.vcap) F = F - (brake * m * (sp - M.vcap)) * u;
    }
  }
  if (any) {
    const float nF = sqrtf(dot(F, F));
    const float cap = m * M.vcap / M.h;
    if (nF > cap) F = (cap / nF) * F;
  }
  return any;
}

// ---- per-pack scratch and the level exchange, shared by the step and adjoint kernels ----
// Scratch of one pack: P points at the pack's first 64-node block and li = node - i0
// (i0 = that block's first node), so offsets stay 32-bit; the layout is the global one.
// A node's fields share one address (base + its 32-bit lane offset); field f adds the
// constant f*64, which the loads and stores carry as an immediate offset.
__device__ __forceinline__ uint32_t slane(int nf, int li) {
  return (uint32_t)(li >> 6) * (uint32_t)nf * 64u + (uint32_t)(li & 63);
}
__device__ __forceinline__ float pld(const float* P, int nf, int f, int li) { return (&at(P, slane(nf, li)))[f * 64]; }
__device__ __forceinline__ void pst(float* P, int nf, int f, int li, float v) { (&at(P, slane(nf, li)))[f * 64] = v; }
__device__ __forceinline__ V3 pld3(const float* P, int nf, int f, int li) {
  return v3(pld(P, nf, f, li), pld(P, nf, f + 1, li), pld(P, nf, f + 2, li));
}
__device__ __forceinline__ void pst3(float* P, int nf, int f, int li, V3 v) {
  pst(P, nf, f, li, v.x); pst(P, nf, f + 1, li, v.y); pst(P, nf, f + 2, li, v.z);
}

// Level-local node index that work-item t takes on the LDS path: the level's first 64
// nodes go to wave (level mod waves), so narrow levels, which fill one wave, rotate over
// the SIMDs instead of all landing on the first wave.
template <int NT>
__device__ __forceinline__ int lvl_lane(int t, int lv) {
  return (t + NT - 64 * (lv & (NT / 64 - 1))) & (NT - 1);
}

// Where a pass stands: the pack's scratch, its exchange buffer and the current level.
struct Lvl {
  float* P;    // pack scratch
  float* X;    // LDS exchange buffer (LDS path)
  int nf;      // scratch fields per node
  int cap;     // exchange slots per level
  int i0;      // first node of the pack's first scratch block
  int a;       // first node of this level
  int nbr;     // first node of the neighbouring level that is read (parent or child level)
  int b;       // this level's exchange buffer (level parity)
};

// a whole publication: NF fields from f0 of node j on the neighbouring level (load) or of
// node i on this level (store); in an LDS slot the fields start at offset OFF.  Aligned
// publications move as 128-bit LDS accesses (the last one also covers slot padding,
// which nobody reads).
template <bool XL, int NF, int OFF = 0>
__device__ __forceinline__ void xload(const Lvl& L, int f0, int j, float (&v)[NF]) {
  if constexpr (XL) {
    const float* sl = L.X + (uint32_t)(((L.b ^ 1) * L.cap + (j - L.nbr)) * X_STRIDE);
    if constexpr (OFF % 4 == 0 && OFF + 4 * ((NF + 3) / 4) <= X_STRIDE) {
      const float4* s = reinterpret_cast<const float4*>(sl + OFF);
#pragma unroll
      for (int k = 0; k < (NF + 3) / 4; ++k) {
        const float4 t = s[k];
        v[4 * k] = t.x;
        if (4 * k + 1 < NF) v[4 * k + 1] = t.y;
        if (4 * k + 2 < NF) v[4 * k + 2] = t.z;
        if (4 * k + 3 < NF) v[4 * k + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < NF; ++k) v[k] = sl[OFF + k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < NF; ++k) v[k] = pld(L.P, L.nf, f0 + k, j - L.i0);
  }
}
template <bool XL, int NF, int OFF = 0>
__device__ __forceinline__ void xstore(const Lvl& L, int f0, int i, const float (&v)[NF]) {
  if constexpr (XL) {
    float* sl = L.X + (uint32_t)((L.b * L.cap + (i - L.a)) * X_STRIDE);
    if constexpr (OFF % 4 == 0 && OFF + 4 * ((NF + 3) / 4) <= X_STRIDE) {
      float4* d = reinterpret_cast<float4*>(sl + OFF);
#pragma unroll
      for (int k = 0; k < (NF + 3) / 4; ++k)
        d[k] = make_float4(v[4 * k], 4 * k + 1 < NF ? v[4 * k + 1] : 0.f, 4 * k + 2 < NF ? v[4 * k + 2] : 0.f,
                           4 * k + 3 < NF ? v[4 * k + 3] : 0.f);
    } else {
#pragma unroll
      for (int k = 0; k < NF; ++k) sl[OFF + k] = v[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < NF; ++k) pst(L.P, L.nf, f0 + k, i - L.i0, v[k]);
  }
}

// Between levels the LDS path needs only the LDS exchange to be complete (node-private
// scratch is written and read back by the same thread); pass ends are full barriers.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The same two synchronisations for a pack that one wavefront walks alone: its lanes
// execute in lockstep and a wave's LDS and memory operations complete in issue order once
// waited for, so the fences (which wait for the wave's outstanding operations and keep the
// compiler from moving accesses across them) are all it needs; no workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void sync_lds() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  } else {
    lds_barrier();
  }
}
template <bool WAVE>
__device__ __forceinline__ void sync_all() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __syncthreads();
  }
}

}  // namespace orchard
