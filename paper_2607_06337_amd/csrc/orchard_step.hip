// Forward step kernels: one workgroup walks one pack (a small forest of trees of
// similar depth) level by level.  Three passes per step:
//   down 1 (root -> leaf): events, snapped mask, kinematics, velocities, applied
//          forces, apples, bias forces, spring/damper torques
//   up     (leaf -> root): articulated inertia and bias, i.e. the leaf-first
//          L^T D L factorisation of the implicit mass matrix (2x2 pivots per joint)
//          together with the forward substitution of the right-hand side
//   down 2 (root -> leaf): back substitution for the joint accelerations, then the
//          implicit-Euler update of the joint state.
// Spatial quantities of a node live at its joint point with world-aligned axes, so
// moving them between parent and child is a pure translation by l z.
//
// What a node hands to the next level (its "publication") goes through LDS when every
// level of the pack fits the workgroup's exchange buffer, double-buffered by level
// parity; a node's publication is one contiguous 16-byte aligned slot (indexed by the
// node's position within its level), so it moves with 128-bit LDS accesses.  Otherwise
// (very wide packs) it goes through global scratch.  For the adjoint's recompute the step also stores the values
// the reverse pass reads back.
#include "orchard_dev.h"

namespace orchard {

__device__ __forceinline__ bool finite3(V3 a) { return isfinite(a.x) && isfinite(a.y) && isfinite(a.z); }

// Status word of an env: bit 0 = frozen (a non-finite state was produced), set at the end
// of a step; bit 1 = an apple went non-finite during this step, promoted to bit 0 by the
// tree's root at the end of the step.  A step's frozen test reads bit 0 only, so it never
// depends on what other nodes of the same step have done.
enum : uint32_t { ST_FROZEN = 1u, ST_APPLE_BAD = 2u };

// First moment and rotational inertia about the joint point of an axisymmetric capsule
// of length l, mass m, transverse / axial inertia Jt / Ia about the joint (geo = l, m, Jt,
// Ia) whose axis is z.  Down 1 and up both form them, bit for bit the same.
__device__ __forceinline__ void own_inertia(float4 geo, V3 z, V3& ho, Sym3& Jo) {
  const float l = geo.x, m = geo.y, Jt = geo.z, Ia = geo.w;
  ho = (0.5f * m * l) * z;
  const float dJ = Ia - Jt;
  Jo = Sym3{fmaf(dJ, z.x * z.x, Jt), fmaf(dJ, z.y * z.y, Jt), fmaf(dJ, z.z * z.z, Jt), dJ * z.x * z.y, dJ * z.x * z.z,
            dJ * z.y * z.z};
}

// Body axis z = R e_z from the joint axes a0 = J e_x and a1 = R e_y and the angle theta_y:
// R = [a0, a1, a0 x a1] R_y(theta_y), so z = sin(theta_y) a0 + cos(theta_y) (a0 x a1), with
// sin and cos formed from the half angle as down 1 forms them.  The up and second down
// passes rebuild z this way instead of loading it.
__device__ __forceinline__ V3 body_z(V3 a0, V3 a1, float qy) {
  float sh, ch;
  sincosf(0.5f * qy, &sh, &ch);
  const float sy = 2.f * sh * ch, cy = 1.f - 2.f * sh * sh;
  return fma3(sy, a0, cy * cross(a0, a1));
}

// Velocity-product acceleration (ang, lin) at the joint point of a body with angular
// velocity wi and joint-point velocity v, whose joint turns at rates qd about a0, a1.
__device__ __forceinline__ void vel_product(V3 a0, V3 a1, float2 qd, V3 wi, V3 v, V3& cang, V3& clin) {
  const V3 u = fma3(qd.x, a0, qd.y * a1);
  cang = fma3(qd.x * qd.y, cross(a0, a1), cross(wi, u));
  clin = cross(v, u);
}

// Bias wrench (ang, lin) of a segment's own body about its joint point: v x* (I v) minus
// the applied body force (input and counter-based random, through the rails and the
// impulse cap, none on a snapped sub-tree) and, with drag on, minus the drag wrench, both
// acting at the segment's midpoint.  Down 1 needs none of it; the up pass forms it from
// the stored velocities.
__device__ __forceinline__ void body_bias(const DevModel& M, const DevInputs& I, int i, uint64_t kstep, int s_call,
                                          float4 geo, V3 z, V3 wi, V3 v, bool snp, uint64_t hkey, V3& pang, V3& plin) {
  const float l = geo.x, m = geo.y;
  V3 ho;
  Sym3 Jo;
  own_inertia(geo, z, ho, Jo);
  const V3 K = mul(Jo, wi) + cross(ho, v);
  const V3 Lm = m * v - cross(ho, wi);
  pang = cross(wi, K) + cross(v, Lm);
  plin = cross(wi, Lm);
  const V3 rc = (0.5f * l) * z;          // joint point -> centre of mass
  const V3 vc = v + cross(wi, rc);       // centre-of-mass velocity
  V3 F, T;
  if (applied_force(M, I, i, kstep, s_call, m, snp, hkey, vc, F, T)) {
    pang = pang - (T + cross(rc, F));
    plin = plin - F;
  }
  if (M.xflags & X_DRAG) {
    // velocity-proportional drag F = -c_v m v_c, tau = -c_w I_c w (inertia about the
    // centre of mass), reduced on a snapped sub-tree
    const ExtraConsts& X = *M.xc;
    const float f = snp ? X.drag_snp : 1.f;
    const float Itc = geo.z - 0.25f * m * l * l, Ia = geo.w;
    const V3 Iw = fma3((Ia - Itc) * dot(z, wi), z, Itc * wi);
    const V3 Fd = (-f * X.drag_lin * m) * vc;
    const V3 Td = (-f * X.drag_ang) * Iw;
    pang = pang - (Td + cross(rc, Fd));
    plin = plin - Fd;
  }
}

// ------------------------------------------------------------------------------------------
// down pass 1
// ------------------------------------------------------------------------------------------
// Frozen envs run the arithmetic on whatever their state holds but write no state, event
// or status; their scratch and publications are read only by nodes of the same env.
//
// Each pass is split into a load stage (the node's own inputs, independent of other
// nodes) and a compute stage, so the LDS path can issue the next level's loads before
// the current level's arithmetic.

// Node flags of a step (F_FLG), an integer below 2^11 held exactly in a float: broken
// after the rupture test, snapped, broken at the start of the step, rupture counter.
__device__ __forceinline__ float flg_pack(bool brk, bool snp, bool brk0, int cnt) {
  return (float)((brk ? 1 : 0) | (snp ? 2 : 0) | (brk0 ? 4 : 0) | (cnt << 3));
}
struct Flags {
  bool brk, snp, brk0;
  int cnt;
};
__device__ __forceinline__ Flags flg_unpack(float f) {
  const int v = (int)f;
  return Flags{(v & 1) != 0, (v & 2) != 0, (v & 4) != 0, v >> 3};
}

// Rupture ratio mu = Kp |theta| / M_max of Eq. break; the up pass forms it again, in the
// same operations, for the event record of a joint that breaks.
__device__ __forceinline__ float rupture_ratio(float kp, float2 q, float inv_mmax) {
  const float th = sqrtf(fmaf(q.x, q.x, q.y * q.y));
  return kp * th * inv_mmax;
}

// down 1 inputs that do not depend on other nodes
struct In1 {
  NodeRec nr;
  float2 q, qd;
  float kp;
  uint8_t brk, cnt;
};
// STATE: also the joint state (a fused pass takes it from the second down pass instead)
template <bool STATE = true>
__device__ __forceinline__ In1 load1(const DevModel& M, const DevState& S, const DevInputs& I, int i) {
  In1 r;
  r.nr = at(M.nrec, (uint32_t)i);
  if constexpr (STATE) {
    r.q = at(S.q, (uint32_t)i);
    r.qd = at(S.qd, (uint32_t)i);
  } else {
    r.q = r.qd = make_float2(0.f, 0.f);
  }
  r.kp = at(I.kp, (uint32_t)i);
  r.brk = at(S.seg_evt, (uint32_t)i);
  r.cnt = at(S.seg_evt, (uint32_t)(M.n_seg + i));
  return r;
}

// pv: the parent's publication (not read for a root); q, qd: the joint state at the start
// of the step; pub: this node's publication, o: its node-private outputs (both stored by
// the caller).
template <bool XL>
__device__ __forceinline__ void node_down1(const DevModel& M, const DevState& S, const Lvl& L, int i, const In1& in,
                                           float2 q, float2 qd, const float (&pv)[N_PUB1], float (&pub)[N_PUB1],
                                           float (&o)[N_OUT1]) {
  const int nf = M.scr_nf, li = i - L.i0;
  const NodeRec& nr = in.nr;
  const float kp = in.kp;
  uint8_t brk = in.brk;
  const uint8_t cnt0 = in.cnt;
  const int par = nr.par;
  const float l = nr.l;

  // ---- parent publication ----
  // Down 1 writes nothing that depends on the env's frozen flag: its event writes are left
  // to the up pass, and the frozen test of the state writes is made in down 2.
  Mat3 Rp;
  V3 pj, w, vt, Aa, Al;
  bool snp;
  if (par < 0) {
    for (int k = 0; k < 9; ++k) Rp.m[k] = (k % 4 == 0) ? 1.f : 0.f;
    pj = v3(0, 0, 0); w = pj; vt = pj; Aa = pj;
    Al = v3(-M.gx, -M.gy, -M.gz);  // gravity as a base acceleration
    snp = false;
  } else {
    const V3 r1 = v3(pv[F_R], pv[F_R + 1], pv[F_R + 2]), r2 = v3(pv[F_R + 3], pv[F_R + 4], pv[F_R + 5]);
    const V3 r0 = cross(r1, r2);
    Rp.m[0] = r0.x; Rp.m[1] = r1.x; Rp.m[2] = r2.x;
    Rp.m[3] = r0.y; Rp.m[4] = r1.y; Rp.m[5] = r2.y;
    Rp.m[6] = r0.z; Rp.m[7] = r1.z; Rp.m[8] = r2.z;
    pj = v3(pv[F_PT], pv[F_PT + 1], pv[F_PT + 2]);
    w = v3(pv[F_W], pv[F_W + 1], pv[F_W + 2]);
    vt = v3(pv[F_VT], pv[F_VT + 1], pv[F_VT + 2]);
    Aa = v3(pv[F_AVA], pv[F_AVA + 1], pv[F_AVA + 2]);
    Al = v3(pv[F_AVL], pv[F_AVL + 1], pv[F_AVL + 2]);
    snp = (((int)pv[F_SNAP]) & 1) != 0;
  }

  // ---- rupture test on the state at the start of the step (Eq. break) ----
  const bool brk0 = brk != 0;
  int cnt1 = 0;
  if (!brk0) {
    const float mu = rupture_ratio(kp, q, nr.inv_mmax);
    cnt1 = mu > 1.f ? (int)cnt0 + 1 : 0;
    cnt1 = cnt1 > 255 ? 255 : cnt1;
    if (cnt1 >= M.n_break) brk = 1;
  }
  snp = snp || brk;

  // ---- kinematics: R = R_parent Q_rest R_x(theta_x) R_y(theta_y) ----
  // the joint rotations are formed from half-angle sines (1 - cos = 2 sin^2(theta/2))
  Mat3 Q;
  {
    const float ww = nr.rq.x, xx = nr.rq.y, yy = nr.rq.z, zz = nr.rq.w;
    Q.m[0] = 1.f - 2.f * (yy * yy + zz * zz); Q.m[1] = 2.f * (xx * yy - ww * zz); Q.m[2] = 2.f * (xx * zz + ww * yy);
    Q.m[3] = 2.f * (xx * yy + ww * zz); Q.m[4] = 1.f - 2.f * (xx * xx + zz * zz); Q.m[5] = 2.f * (yy * zz - ww * xx);
    Q.m[6] = 2.f * (xx * zz - ww * yy); Q.m[7] = 2.f * (yy * zz + ww * xx); Q.m[8] = 1.f - 2.f * (xx * xx + yy * yy);
  }
  // columns of J = R_parent Q
  const V3 J0 = mul(Rp, v3(Q.m[0], Q.m[3], Q.m[6]));
  const V3 J1 = mul(Rp, v3(Q.m[1], Q.m[4], Q.m[7]));
  const V3 J2 = mul(Rp, v3(Q.m[2], Q.m[5], Q.m[8]));
  float shx, chx, shy, chy;
  sincosf(0.5f * q.x, &shx, &chx);
  sincosf(0.5f * q.y, &shy, &chy);
  const float sx = 2.f * shx * chx, cx = 1.f - 2.f * shx * shx;
  const float sy = 2.f * shy * chy, cy = 1.f - 2.f * shy * shy;
  const V3 c0 = fma3(cy, J0, fma3(sx * sy, J1, (-cx * sy) * J2));
  const V3 c1 = fma3(cx, J1, sx * J2);
  const V3 c2 = fma3(sy, J0, fma3(-sx * cy, J1, (cx * cy) * J2));
  const V3 a0 = J0, a1 = c1, z = c2;

  // ---- velocities and velocity-product acceleration (at the joint point) ----
  const V3 wi = w + fma3(qd.x, a0, qd.y * a1);  // plus the relative angular velocity
  const V3 v = vt;                               // joint point moves with the parent
  V3 cang, clin;
  vel_product(a0, a1, qd, wi, v, cang, clin);
  const V3 Ava = Aa + cang, Avl = Al + clin;

  // ---- publish for children (values at the tip point) ----
  const V3 lz = l * z;
  {
    const V3 pt = pj + lz, vtp = v + cross(wi, lz), alt = Avl + cross(Ava, lz);
    const float ov[N_PUB1] = {c1.x, c1.y, c1.z, c2.x, c2.y, c2.z,
                              pt.x, pt.y, pt.z, wi.x, wi.y, wi.z, vtp.x, vtp.y, vtp.z,
                              Ava.x, Ava.y, Ava.z, alt.x, alt.y, alt.z, snp ? 1.f : 0.f};
    for (int k = 0; k < N_PUB1; ++k) pub[k] = ov[k];
  }
  if (M.save_adj) {
    // the adjoint reads these from global scratch whichever way levels exchange
    float* P = L.P;
    if constexpr (XL) {
      pst3(P, nf, F_W, li, wi);
      pst3(P, nf, F_VT, li, v + cross(wi, lz));
    }
    pst(P, nf, F_SSNP, li, snp ? 1.f : 0.f);
    pst3(P, nf, F_Z, li, z);
    pst3(P, nf, F_SAVP, li, Ava); pst3(P, nf, F_SAVP + 3, li, Avl);
  }

  // apples are handled by the apple phase after this pass; keep what it needs
  if (nr.anode >= 0) {
    static_assert(K_R == 0 && K_W == 9 && K_V == 12 && K_AA == 15 && K_AL == 18 && K_PJ == 21 && K_N == 24,
                  "snapshot layout");
    float4* ks = reinterpret_cast<float4*>(M.asnap + (size_t)nr.anode * K_N);
    ks[0] = make_float4(c0.x, c1.x, c2.x, c0.y);
    ks[1] = make_float4(c1.y, c2.y, c0.z, c1.z);
    ks[2] = make_float4(c2.z, wi.x, wi.y, wi.z);
    ks[3] = make_float4(v.x, v.y, v.z, Ava.x);
    ks[4] = make_float4(Ava.y, Ava.z, Avl.x, Avl.y);
    ks[5] = make_float4(Avl.z, pj.x, pj.y, pj.z);
  }

  // node-private outputs (fields F_A0 .. F_FLG), stored by the caller; the flags carry the
  // rupture test's result for the up pass, which forms the spring terms and writes the events
  const float out[N_OUT1] = {a0.x, a0.y, a0.z, a1.x, a1.y, a1.z, wi.x, wi.y, wi.z, v.x, v.y, v.z,
                             flg_pack(brk != 0, snp, brk0, cnt1)};
  for (int k = 0; k < N_OUT1; ++k) o[k] = out[k];
}

// a pass's node-private outputs, fields F0 .. F0 + K - 1, at a node's scratch address
template <int F0, int K>
__device__ __forceinline__ void put_fields(float* base, const float (&o)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) base[(F0 + k) * 64] = o[k];
}

// ------------------------------------------------------------------------------------------
// apple phase (between down 1 and up): every apple of the pack at once
// ------------------------------------------------------------------------------------------
// Thread per apple over chunks of NT apples: events, the reaction on the spur and the
// virtual point mass at the hang point (from the node's kinematics kept by down 1), and
// the apple's own update.  A node's apples are contiguous; the thread holding a node's
// first apple of the chunk adds the chunk's contributions to the node's bias and own
// inertia in apple order, so the sums do not depend on the mapping.
struct AppleCon { float mv; V3 d, pang, plin; };

template <int NT, bool WAVE = false>
__device__ __forceinline__ void apple_phase(const DevModel& M, const DevState& S, const DevInputs& I, const Lvl& L,
                                            float* C, int pk, int64_t n, int s_call, int t) {
  const int A0 = ldc(M.pack_apl, pk), A1 = ldc(M.pack_apl, pk + 1);
  const int NS = M.n_seg;
  const uint32_t NA = (uint32_t)M.n_apple;
  const float h = M.h;
  const V3 gv = v3(M.gx, M.gy, M.gz);
  // C: [11][NT] LDS, the chunk's contributions and node ids
  for (int c0 = A0; c0 < A1; c0 += NT) {
    const int a = c0 + t;
    const bool has = a < A1;
    AppleCon con{0.f, v3(0, 0, 0), v3(0, 0, 0), v3(0, 0, 0)};
    int node = -1;
    bool first = false;  // the node's first apple
    int an = 0;          // the node's apple-node index
    if (has) {
      const uint32_t ua = (uint32_t)a;
      const AppleRec ar = at(M.arec, ua);
      node = ar.link.x;
      first = ar.link.z != 0;
      an = ar.link.w;
      // the env's frozen flag (status bit 0) changes only in down 2, so here it still holds
      // its value at the start of the step
      const bool live = (at(S.status, (uint32_t)ar.link.y) & ST_FROZEN) == 0u;
      const float4* ks = reinterpret_cast<const float4*>(M.asnap + (size_t)ar.link.w * K_N);
      const float4 k0 = ks[0], k1 = ks[1], k2 = ks[2], k3 = ks[3], k4 = ks[4], k5 = ks[5];
      Mat3 R;
      R.m[0] = k0.x; R.m[1] = k0.y; R.m[2] = k0.z; R.m[3] = k0.w; R.m[4] = k1.x; R.m[5] = k1.y;
      R.m[6] = k1.z; R.m[7] = k1.w; R.m[8] = k2.x;
      const V3 wi = v3(k2.y, k2.z, k2.w), v = v3(k3.x, k3.y, k3.z);
      const V3 Ava = v3(k3.w, k4.x, k4.y), Avl = v3(k4.z, k4.w, k5.x), pj = v3(k5.y, k5.z, k5.w);
      float* Pa = S.apple;
      // position state: while attached sigma = (x - x_hang) + h v from the previous
      // update, so the stretch now is s = sigma - h v_hang; once detached, x minus the
      // rest hang point.  The stretch never passes through absolute positions.
      const V3 sig = v3(at(Pa, ua), at(Pa, NA + ua), at(Pa, 2 * NA + ua));
      V3 va = v3(at(Pa, 3 * NA + ua), at(Pa, 4 * NA + ua), at(Pa, 5 * NA + ua));
      const uint8_t det0 = at(S.apple_evt, ua), cp0 = at(S.apple_evt, NA + ua), ct0 = at(S.apple_evt, 2 * NA + ua);
      V3 Fa = v3(0, 0, 0);
      if (I.aforce) {
        const float* fp = I.aforce + (int64_t)s_call * I.aforce_stride;
        Fa = v3(at(fp, 3 * ua), at(fp, 3 * ua + 1), at(fp, 3 * ua + 2));
      }
      const float ma = ar.hang.w, cs = ar.par.y, fmax = ar.par.z;
      // hang point offset from the joint point: R (hx, hy, hz) by columns of R
      const V3 d = fma3(ar.hang.x, v3(R.m[0], R.m[3], R.m[6]),
                        fma3(ar.hang.y, v3(R.m[1], R.m[4], R.m[7]), ar.hang.z * v3(R.m[2], R.m[5], R.m[8])));
      const V3 vh = v + cross(wi, d);
      const V3 sa = det0 ? v3(0, 0, 0) : fma3(-h, vh, sig);
      uint8_t det = det0;
      if (!det) {
        const float pi = sqrtf(dot(Fa, Fa)) * ar.par.x;
        const float tau = M.ks * sqrtf(dot(sa, sa)) * ar.par.w;
        int cp = pi > 1.f ? (int)cp0 + 1 : 0;
        int ct = tau > 1.f ? (int)ct0 + 1 : 0;
        cp = cp > 255 ? 255 : cp;
        ct = ct > 255 ? 255 : ct;
        const int path = cp >= M.n_pull ? 1 : (ct >= M.n_tension ? 2 : 0);
        if (live) {
          at(S.apple_evt, NA + ua) = (uint8_t)cp;
          at(S.apple_evt, 2 * NA + ua) = (uint8_t)ct;
          if (path) {
            at(S.apple_evt, ua) = 1;
            at(S.apple_evt, 3 * NA + ua) = (uint8_t)path;
            at(S.evt_step, (uint32_t)NS + ua) = (int32_t)n;
            if (S.evt_ratio) at(S.evt_ratio, (uint32_t)NS + ua) = path == 1 ? pi : tau;
          }
        }
        if (path) det = 1;
      }
      if (!det) {
        // reaction on the spur: elastic tether force minus static weight, hang point
        // taken at the end of the step to first order (linearly implicit); the clamp
        // scales explicit part and implicit term alike by s = min(1, F_max / |f|)
        V3 fh = M.ks * fma3(-h, vh, sa) - ma * gv;
        const float nfh = sqrtf(dot(fh, fh));
        const float sc = nfh > fmax ? fmax / nfh : 1.f;
        fh = sc * fh;
        // virtual point mass s h^2 k_s at the hang point (only its q-acceleration part)
        const float mv = sc * h * h * M.ks;
        const V3 wvp = Avl + cross(Ava, d);
        con.mv = mv;
        con.d = d;
        con.pang = (-1.f) * (cross(d, fh) + mv * cross(d, wvp));
        con.plin = (-1.f) * (fh + mv * wvp);
      }
      // apple update: explicit symplectic Euler
      V3 fa = fma3(ma, gv, Fa);
      if (!det) fa = fa - M.ks * sa - cs * va;
      va = fma3(ar.rest.w, fa, va);
      // attached: sigma+ = s + h v+;  detached: (x - x_hang,rest)+ = x - x_hang,rest + h v+
      V3 base = sa;
      if (det) base = det0 ? sig : (pj + d - v3(ar.rest.x, ar.rest.y, ar.rest.z)) + sa;
      const V3 x = fma3(h, va, base);
      if (live) {
        at(Pa, ua) = x.x; at(Pa, NA + ua) = x.y; at(Pa, 2 * NA + ua) = x.z;
        at(Pa, 3 * NA + ua) = va.x; at(Pa, 4 * NA + ua) = va.y; at(Pa, 5 * NA + ua) = va.z;
        // orientation (rigid-body fruit only): no torque acts on an apple, so omega is
        // carried and the quaternion only turns while omega is non-zero
        const V3 om = M.apl == 13 ? v3(at(Pa, 10 * NA + ua), at(Pa, 11 * NA + ua), at(Pa, 12 * NA + ua)) : v3(0, 0, 0);
        const V3 hw = (0.5f * h) * om;
        const float th = sqrtf(dot(hw, hw));
        if (th > 0.f) {
          float sn, cn;
          sincosf(th, &sn, &cn);
          const float scq = sn / th;
          const float ew = cn, ex = scq * hw.x, ey = scq * hw.y, ez = scq * hw.z;
          const float q0 = at(Pa, 6 * NA + ua), q1 = at(Pa, 7 * NA + ua), q2 = at(Pa, 8 * NA + ua), q3 = at(Pa, 9 * NA + ua);
          float nw = ew * q0 - ex * q1 - ey * q2 - ez * q3;
          float nx = ew * q1 + ex * q0 + ey * q3 - ez * q2;
          float ny = ew * q2 - ex * q3 + ey * q0 + ez * q1;
          float nz = ew * q3 + ex * q2 - ey * q1 + ez * q0;
          const float inv = 1.f / sqrtf(nw * nw + nx * nx + ny * ny + nz * nz);
          at(Pa, 6 * NA + ua) = nw * inv; at(Pa, 7 * NA + ua) = nx * inv; at(Pa, 8 * NA + ua) = ny * inv;
          at(Pa, 9 * NA + ua) = nz * inv;
        }
        if (!finite3(x) || !finite3(va)) atomicOr(&at(S.status, (uint32_t)ar.link.y), ST_APPLE_BAD);
      }
    }
    C[0 * NT + t] = con.mv;
    C[1 * NT + t] = con.d.x; C[2 * NT + t] = con.d.y; C[3 * NT + t] = con.d.z;
    C[4 * NT + t] = con.pang.x; C[5 * NT + t] = con.pang.y; C[6 * NT + t] = con.pang.z;
    C[7 * NT + t] = con.plin.x; C[8 * NT + t] = con.plin.y; C[9 * NT + t] = con.plin.z;
    C[10 * NT + t] = __int_as_float(node);
    sync_lds<WAVE>();
    // the thread with a node's first apple in this chunk adds the chunk's contributions;
    // the virtual inertia starts from zero at the node's first apple
    if (has && (t == 0 || __float_as_int(C[10 * NT + t - 1]) != node)) {
      static_assert(E_MO == 0 && E_HO == 1 && E_JO == 4 && E_P == 10 && E_N == 16, "apple sums layout");
      float4* es = reinterpret_cast<float4*>(M.aext + (size_t)an * E_N);
      float4 e0 = make_float4(0.f, 0.f, 0.f, 0.f), e1 = e0, e2 = e0, e3 = e0;
      if (!first) { e0 = es[0]; e1 = es[1]; e2 = es[2]; e3 = es[3]; }
      float mo = e0.x;
      V3 ho = v3(e0.y, e0.z, e0.w);
      Sym3 Jo{e1.x, e1.y, e1.z, e1.w, e2.x, e2.y};
      V3 pang = v3(e2.z, e2.w, e3.x), plin = v3(e3.y, e3.z, e3.w);
      for (int k = t; k < NT && c0 + k < A1 && __float_as_int(C[10 * NT + k]) == node; ++k) {
        const float mv = C[0 * NT + k];
        const V3 d = v3(C[1 * NT + k], C[2 * NT + k], C[3 * NT + k]);
        mo += mv;
        ho = fma3(mv, d, ho);
        const float dd = dot(d, d);
        Jo.xx = fmaf(mv, dd - d.x * d.x, Jo.xx); Jo.yy = fmaf(mv, dd - d.y * d.y, Jo.yy);
        Jo.zz = fmaf(mv, dd - d.z * d.z, Jo.zz); Jo.xy = fmaf(-mv, d.x * d.y, Jo.xy);
        Jo.xz = fmaf(-mv, d.x * d.z, Jo.xz); Jo.yz = fmaf(-mv, d.y * d.z, Jo.yz);
        pang = pang + v3(C[4 * NT + k], C[5 * NT + k], C[6 * NT + k]);
        plin = plin + v3(C[7 * NT + k], C[8 * NT + k], C[9 * NT + k]);
      }
      es[0] = make_float4(mo, ho.x, ho.y, ho.z);
      es[1] = make_float4(Jo.xx, Jo.yy, Jo.zz, Jo.xy);
      es[2] = make_float4(Jo.xz, Jo.yz, pang.x, pang.y);
      es[3] = make_float4(pang.z, plin.x, plin.y, plin.z);
    }
    // node sums of this chunk are visible to the next chunk's threads; the LDS can be reused
    sync_all<WAVE>();
  }
}

// ------------------------------------------------------------------------------------------
// up pass: gather children's articulated inertia / bias, factor the 2x2 pivot
// ------------------------------------------------------------------------------------------
// the part of a node's topology word the up pass reads
struct TopoU {
  int env, child, cnt, an;  // env, first child, children | apples << 16, apple-node index
};
__device__ __forceinline__ TopoU topo_up(const DevModel& M, int i) {
  const int4 w = at(M.ntopo, (uint32_t)i);
  return TopoU{w.x, w.y, w.z, w.w};
}
// up-pass inputs: the node's own data from down 1, its static record and state
struct InU {
  TopoU topo;
  float4 geo;
  V3 a0, a1, wi, v;
  float2 q, qd;
  float kp, kd, flg;
  uint32_t hk0, hk1;  // random-wrench key
};
__device__ __forceinline__ InU loadU(const DevModel& M, const DevState& S, const DevInputs& I, const Lvl& L, int i) {
  const int nf = M.scr_nf, li = i - L.i0;
  const float* P = L.P;
  InU u;
  u.topo = topo_up(M, i);
  u.geo = at(M.geo, (uint32_t)i);
  u.q = at(S.q, (uint32_t)i);
  u.qd = at(S.qd, (uint32_t)i);
  u.kp = at(I.kp, (uint32_t)i);
  u.kd = at(I.kd, (uint32_t)i);
  u.flg = pld(P, nf, F_FLG, li);
  u.a0 = pld3(P, nf, F_A0, li);
  u.a1 = pld3(P, nf, F_A1, li);
  u.wi = pld3(P, nf, F_WV, li);
  u.v = pld3(P, nf, F_WV + 3, li);
  const uint64_t hk = at(M.hkey, (uint32_t)i);
  u.hk0 = (uint32_t)hk;
  u.hk1 = (uint32_t)(hk >> 32);
  return u;
}

template <bool XL>
__device__ __forceinline__ void node_up(const DevModel& M, const DevState& S, const DevInputs& I, const Lvl& L, int i,
                                        const InU& in, int64_t n, uint64_t kstep, int s_call, float (&o)[N_OUTU]) {
  const int nf = M.scr_nf, li = i - L.i0;
  const TopoU topo = in.topo;
  // the env's frozen flag at the start of the step (bit 0 changes only in down 2) decides the
  // event writes at the end
  const uint32_t stat = at(S.status, (uint32_t)in.topo.env);
  const Flags fl = flg_unpack(in.flg);
  const V3 a0 = in.a0, a1 = in.a1, z = body_z(a0, a1, in.q.y);
  const V3 r = in.geo.x * z;  // l z, joint point -> tip
  // the apple sums of a node that carries apples are loaded here rather than a level
  // ahead (they would double in the prefetch registers); their first use comes after the
  // bias and the children's gather
  float4 e0 = make_float4(0.f, 0.f, 0.f, 0.f), e1 = e0, e2 = e0, e3 = e0;
  if (topo.cnt >> 16) {
    const float4* es = reinterpret_cast<const float4*>(M.aext + (size_t)topo.an * E_N);
    e0 = es[0]; e1 = es[1]; e2 = es[2]; e3 = es[3];
  }
  // velocity-product acceleration and the own body's bias, formed from the velocities
  V3 ca, cl, pang, plin;
  vel_product(a0, a1, in.qd, in.wi, in.v, ca, cl);
  const bool snp = fl.snp;
  body_bias(M, I, i, kstep, s_call, in.geo, z, in.wi, in.v, snp, (uint64_t)in.hk0 | ((uint64_t)in.hk1 << 32), pang,
            plin);
  // own body plus the apples' virtual masses and reactions (zero without apples)
  V3 ho;
  Sym3 Jo;
  own_inertia(in.geo, z, ho, Jo);
  const float mo = in.geo.y + e0.x;
  ho = ho + v3(e0.y, e0.z, e0.w);
  Jo.xx += e1.x; Jo.yy += e1.y; Jo.zz += e1.z; Jo.xy += e1.w; Jo.xz += e2.x; Jo.yz += e2.y;
  const V3 pon = pang + v3(e2.z, e2.w, e3.x), pof = plin + v3(e3.y, e3.z, e3.w);
  // spring / damper with the implicit diagonal; a broken joint has none
  const float h = M.h;
  const bool brk = fl.brk;
  const float2 q = in.q, qd = in.qd;
  const float kpe = brk ? 0.f : in.kp;
  float kde = brk ? 0.f : in.kd;
  if (brk && (M.xflags & X_FRIC)) {
    // Coulomb friction of the torn fibres: tau_c ramps linearly from friction_base to
    // friction_growth x friction_base of the limb's weight moment, acting as the linearly
    // implicit damper tau_c / max(|qd|, friction_speed)
    const ExtraConsts& X = *M.xc;
    const int64_t nb = fl.brk0 ? (int64_t)at(S.evt_step, (uint32_t)i) : n;  // step of the break
    const float ramp = X.fric_inv_ramp < 0.f ? 1.f : fminf(1.f, (float)(n - nb) * h * X.fric_inv_ramp);
    const float tc = X.fric_base * at(X.wmom, (uint32_t)i) * fmaf(X.fric_growth - 1.f, ramp, 1.f);
    kde = tc / fmaxf(sqrtf(fmaf(qd.x, qd.x, qd.y * qd.y)), X.fric_speed);
  }
  const float tau0 = -kpe * fmaf(h, qd.x, q.x) - kde * qd.x;
  const float tau1 = -kpe * fmaf(h, qd.y, q.y) - kde * qd.y;
  const float dg = fmaf(h, kde, h * h * kpe);

  Sym3 A{0, 0, 0, 0, 0, 0}, Mm{0, 0, 0, 0, 0, 0};
  Mat3 B;
  for (int k = 0; k < 9; ++k) B.m[k] = 0.f;
  V3 pn = v3(0, 0, 0), pf = v3(0, 0, 0);
  const int cb = topo.child, ce = cb + (topo.cnt & 0xFFFF);
  for (int c = cb; c < ce; ++c) {
    float cv[N_PUBU];
    xload<XL>(L, F_IA, c, cv);
#define XG(f) cv[(f) - F_IA]
    A.xx += XG(F_IA + 0); A.yy += XG(F_IA + 1); A.zz += XG(F_IA + 2);
    A.xy += XG(F_IA + 3); A.xz += XG(F_IA + 4); A.yz += XG(F_IA + 5);
    for (int k = 0; k < 9; ++k) B.m[k] += XG(F_IB + k);
    Mm.xx += XG(F_IM + 0); Mm.yy += XG(F_IM + 1); Mm.zz += XG(F_IM + 2);
    Mm.xy += XG(F_IM + 3); Mm.xz += XG(F_IM + 4); Mm.yz += XG(F_IM + 5);
    pn = pn + v3(XG(F_PA + 0), XG(F_PA + 1), XG(F_PA + 2));
    pf = pf + v3(XG(F_PA + 3), XG(F_PA + 4), XG(F_PA + 5));
#undef XG
  }
  if (ce > cb) {
    // move the children's sum from the tip to the joint point (translation by r):
    // A' = A - B[r] - (B[r])^T - [r]M[r],  B' = B + [r]M,  M' = M,  n' = n + r x f
    V3 b0 = v3(B.m[0], B.m[1], B.m[2]), b1 = v3(B.m[3], B.m[4], B.m[5]), b2 = v3(B.m[6], B.m[7], B.m[8]);
    const V3 x0 = cross(b0, r), x1 = cross(b1, r), x2 = cross(b2, r);  // rows of B[r]
    // Y = [r] M: columns r x m_k
    const V3 m0 = v3(Mm.xx, Mm.xy, Mm.xz), m1 = v3(Mm.xy, Mm.yy, Mm.yz), m2 = v3(Mm.xz, Mm.yz, Mm.zz);
    const V3 y0 = cross(r, m0), y1 = cross(r, m1), y2 = cross(r, m2);  // columns of Y
    // rows of Y
    const V3 yr0 = v3(y0.x, y1.x, y2.x), yr1 = v3(y0.y, y1.y, y2.y), yr2 = v3(y0.z, y1.z, y2.z);
    const V3 z0 = cross(yr0, r), z1 = cross(yr1, r), z2 = cross(yr2, r);  // rows of Y[r]
    A.xx -= 2.f * x0.x + z0.x; A.yy -= 2.f * x1.y + z1.y; A.zz -= 2.f * x2.z + z2.z;
    A.xy -= x0.y + x1.x + z0.y; A.xz -= x0.z + x2.x + z0.z; A.yz -= x1.z + x2.y + z1.z;
    B.m[0] += yr0.x; B.m[1] += yr0.y; B.m[2] += yr0.z;
    B.m[3] += yr1.x; B.m[4] += yr1.y; B.m[5] += yr1.z;
    B.m[6] += yr2.x; B.m[7] += yr2.y; B.m[8] += yr2.z;
    pn = pn + cross(r, pf);
  }
  // add the node's own body (+ virtual apple masses) and bias
  A.xx += Jo.xx; A.yy += Jo.yy; A.zz += Jo.zz; A.xy += Jo.xy; A.xz += Jo.xz; A.yz += Jo.yz;
  // B += [h]
  B.m[1] -= ho.z; B.m[2] += ho.y; B.m[3] += ho.z; B.m[5] -= ho.x; B.m[6] -= ho.y; B.m[7] += ho.x;
  Mm.xx += mo; Mm.yy += mo; Mm.zz += mo;
  pn = pn + pon;
  pf = pf + pof;
  if (M.save_adj) {
    float* Pw = L.P;
    pst(Pw, nf, F_SIA + 0, li, A.xx); pst(Pw, nf, F_SIA + 1, li, A.yy); pst(Pw, nf, F_SIA + 2, li, A.zz);
    pst(Pw, nf, F_SIA + 3, li, A.xy); pst(Pw, nf, F_SIA + 4, li, A.xz); pst(Pw, nf, F_SIA + 5, li, A.yz);
    for (int k = 0; k < 9; ++k) pst(Pw, nf, F_SIA + 6 + k, li, B.m[k]);
    pst(Pw, nf, F_SIA + 15, li, Mm.xx); pst(Pw, nf, F_SIA + 16, li, Mm.yy); pst(Pw, nf, F_SIA + 17, li, Mm.zz);
    pst(Pw, nf, F_SIA + 18, li, Mm.xy); pst(Pw, nf, F_SIA + 19, li, Mm.xz); pst(Pw, nf, F_SIA + 20, li, Mm.yz);
    pst3(Pw, nf, F_SPA, li, pn); pst3(Pw, nf, F_SPA + 3, li, pf);
  }
  // U = I^A S,  S = [a0 a1; 0 0]
  const V3 U0a = mul(A, a0), U1a = mul(A, a1);
  const V3 U0l = mulT(B, a0), U1l = mulT(B, a1);
  const float D00 = dot(a0, U0a) + dg, D01 = dot(a0, U1a), D11 = dot(a1, U1a) + dg;
  const float idet = 1.f / fmaf(D00, D11, -D01 * D01);
  const float Di00 = D11 * idet, Di01 = -D01 * idet, Di11 = D00 * idet;
  const float uu0 = tau0 - dot(a0, pn);
  const float uu1 = tau1 - dot(a1, pn);
  // W = U D^-1
  const V3 W0a = fma3(Di00, U0a, Di01 * U1a), W1a = fma3(Di01, U0a, Di11 * U1a);
  const V3 W0l = fma3(Di00, U0l, Di01 * U1l), W1l = fma3(Di01, U0l, Di11 * U1l);
  // articulated inertia passed to the parent: I^A - W U^T
  A.xx -= W0a.x * U0a.x + W1a.x * U1a.x; A.yy -= W0a.y * U0a.y + W1a.y * U1a.y;
  A.zz -= W0a.z * U0a.z + W1a.z * U1a.z; A.xy -= W0a.x * U0a.y + W1a.x * U1a.y;
  A.xz -= W0a.x * U0a.z + W1a.x * U1a.z; A.yz -= W0a.y * U0a.z + W1a.y * U1a.z;
  B.m[0] -= W0a.x * U0l.x + W1a.x * U1l.x; B.m[1] -= W0a.x * U0l.y + W1a.x * U1l.y; B.m[2] -= W0a.x * U0l.z + W1a.x * U1l.z;
  B.m[3] -= W0a.y * U0l.x + W1a.y * U1l.x; B.m[4] -= W0a.y * U0l.y + W1a.y * U1l.y; B.m[5] -= W0a.y * U0l.z + W1a.y * U1l.z;
  B.m[6] -= W0a.z * U0l.x + W1a.z * U1l.x; B.m[7] -= W0a.z * U0l.y + W1a.z * U1l.y; B.m[8] -= W0a.z * U0l.z + W1a.z * U1l.z;
  Mm.xx -= W0l.x * U0l.x + W1l.x * U1l.x; Mm.yy -= W0l.y * U0l.y + W1l.y * U1l.y;
  Mm.zz -= W0l.z * U0l.z + W1l.z * U1l.z; Mm.xy -= W0l.x * U0l.y + W1l.x * U1l.y;
  Mm.xz -= W0l.x * U0l.z + W1l.x * U1l.z; Mm.yz -= W0l.y * U0l.z + W1l.y * U1l.z;
  // bias passed to the parent: p^A + I^a c + W u
  pn = pn + mul(A, ca) + mul(B, cl) + fma3(uu0, W0a, uu1 * W1a);
  pf = pf + mulT(B, ca) + mul(Mm, cl) + fma3(uu0, W0l, uu1 * W1l);
  {
    const float ov[N_PUBU] = {A.xx, A.yy, A.zz, A.xy, A.xz, A.yz,
                              B.m[0], B.m[1], B.m[2], B.m[3], B.m[4], B.m[5], B.m[6], B.m[7], B.m[8],
                              Mm.xx, Mm.yy, Mm.zz, Mm.xy, Mm.xz, Mm.yz,
                              pn.x, pn.y, pn.z, pf.x, pf.y, pf.z};
    static_assert(F_IB - F_IA == 6 && F_IM - F_IA == 15 && F_PA - F_IA == 21, "publication order");
    xstore<XL>(L, F_IA, i, ov);
  }
  float* Pw = L.P;
  if (M.save_adj) { pst(Pw, nf, F_DI, li, Di00); pst(Pw, nf, F_DI + 1, li, Di01); pst(Pw, nf, F_DI + 2, li, Di11); }
  // rupture events of this step (the test ran in down 1)
  if ((stat & ST_FROZEN) == 0u && !fl.brk0) {
    at(S.seg_evt, (uint32_t)(M.n_seg + i)) = (uint8_t)fl.cnt;
    if (fl.brk) {
      at(S.seg_evt, (uint32_t)i) = 1;
      at(S.evt_step, (uint32_t)i) = (int32_t)n;
      if (S.evt_ratio) at(S.evt_ratio, (uint32_t)i) = rupture_ratio(in.kp, in.q, at(M.nrec, (uint32_t)i).inv_mmax);
    }
  }
  // node-private outputs (fields F_WM .. F_DU + 1), stored by the caller
  const float out[N_OUTU] = {W0a.x, W0a.y, W0a.z, W0l.x, W0l.y, W0l.z, W1a.x, W1a.y, W1a.z, W1l.x, W1l.y, W1l.z,
                             fmaf(Di00, uu0, Di01 * uu1), fmaf(Di01, uu0, Di11 * uu1)};
  for (int k = 0; k < N_OUTU; ++k) o[k] = out[k];
}

// ------------------------------------------------------------------------------------------
// down pass 2: accelerations and integration
// ------------------------------------------------------------------------------------------
// down 2 inputs: the node's factor data from the up pass and its state
struct In2 {
  int par;
  float du0, du1, l;
  V3 wi, v, W0a, W0l, W1a, W1l, a0, a1;
  float2 q, qd;
};
// TOPO: also the parent and the length (a fused pass takes them from the first down pass's
// record instead)
template <bool TOPO = true>
__device__ __forceinline__ In2 load2(const DevModel& M, const DevState& S, const Lvl& L, int i) {
  const int nf = M.scr_nf, li = i - L.i0;
  const float* P = L.P;
  In2 d;
  if constexpr (TOPO) {
    d.par = at(M.par, (uint32_t)i);
    d.l = at(M.len, (uint32_t)i);
  } else {
    d.par = -1;
    d.l = 0.f;
  }
  d.wi = pld3(P, nf, F_WV, li);
  d.v = pld3(P, nf, F_WV + 3, li);
  d.W0a = pld3(P, nf, F_WM, li);
  d.W0l = pld3(P, nf, F_WM + 3, li);
  d.W1a = pld3(P, nf, F_WM + 6, li);
  d.W1l = pld3(P, nf, F_WM + 9, li);
  d.du0 = pld(P, nf, F_DU, li);
  d.du1 = pld(P, nf, F_DU + 1, li);
  d.a0 = pld3(P, nf, F_A0, li);
  d.a1 = pld3(P, nf, F_A1, li);
  d.q = at(S.q, (uint32_t)i);
  d.qd = at(S.qd, (uint32_t)i);
  return d;
}

// pv: the parent's flags and acceleration at the tip (not read for a root); pub: this
// node's, stored by the caller; qn, qdn: the joint state after the step (unchanged in a
// frozen env), also written to the state here.
template <bool XL>
__device__ __forceinline__ void node_down2(const DevModel& M, const DevState& S, const Lvl& L, int i, const In2& in,
                                           const float (&pv)[7], float (&pub)[7], float2& qn, float2& qdn) {
  const int nf = M.scr_nf, li = i - L.i0;
  const int par = in.par;
  const V3 W0a = in.W0a, W0l = in.W0l, W1a = in.W1a, W1l = in.W1l;
  const V3 a0 = in.a0, a1 = in.a1, lz = in.l * body_z(a0, a1, in.q.y);
  float2 q = in.q, qd = in.qd;
  V3 ca, cl;
  vel_product(a0, a1, qd, in.wi, in.v, ca, cl);
  // The env's frozen flag at the start of the step is read by the root (nothing of this
  // step has set bit 0 yet: only down 2 does) and handed down with the acceleration.
  V3 Aa, Al;
  bool frozen;
  uint32_t rstat = 0;
  if (par < 0) {
    Aa = v3(0, 0, 0); Al = v3(-M.gx, -M.gy, -M.gz);
    rstat = at(S.status, (uint32_t)at(M.env, (uint32_t)i));
    frozen = (rstat & ST_FROZEN) != 0u;
  } else {
    frozen = (((int)pv[0]) & 2) != 0;
    Aa = v3(pv[1], pv[2], pv[3]);
    Al = v3(pv[4], pv[5], pv[6]);
  }
  Aa = Aa + ca;
  Al = Al + cl;
  const float qdd0 = in.du0 - (dot(W0a, Aa) + dot(W0l, Al));
  const float qdd1 = in.du1 - (dot(W1a, Aa) + dot(W1l, Al));
  Aa = fma3(qdd0, a0, fma3(qdd1, a1, Aa));
  if (M.save_adj) {
    float* Pw = L.P;
    pst3(Pw, nf, F_SA, li, Aa); pst3(Pw, nf, F_SA + 3, li, Al);
    pst(Pw, nf, F_SQDD, li, qdd0); pst(Pw, nf, F_SQDD + 1, li, qdd1);
    pst(Pw, nf, F_SFRZ, li, frozen ? 1.f : 0.f);
  }
  {
    const V3 alt = Al + cross(Aa, lz);
    const float ov[7] = {frozen ? 2.f : 0.f, Aa.x, Aa.y, Aa.z, alt.x, alt.y, alt.z};
    for (int k = 0; k < 7; ++k) pub[k] = ov[k];
  }
  qn = q;
  qdn = qd;
  if (frozen) return;
  const float h = M.h;
  qd.x = fmaf(h, qdd0, qd.x);
  qd.y = fmaf(h, qdd1, qd.y);
  q.x = fmaf(h, qd.x, q.x);
  q.y = fmaf(h, qd.y, q.y);
  at(S.q, (uint32_t)i) = q;
  at(S.qd, (uint32_t)i) = qd;
  qn = q;
  qdn = qd;
  // a non-finite state freezes the env; the root promotes this step's apple flag once every
  // node of the step has run down 1 (only these rare cases touch the status word)
  const bool bad = !(isfinite(q.x) && isfinite(q.y) && isfinite(qd.x) && isfinite(qd.y));
  if (bad || (par < 0 && (rstat & ST_APPLE_BAD))) atomicOr(&at(S.status, (uint32_t)at(M.env, (uint32_t)i)), ST_FROZEN);
}

// ------------------------------------------------------------------------------------------
// pack kernels
// ------------------------------------------------------------------------------------------
// One node of a down pass: the parent's publication in (nothing for a root), the node's
// own out through the exchange, its node-private outputs to scratch.
template <bool XL>
__device__ __forceinline__ void pass_down1(const DevModel& M, const DevState& S, const Lvl& L, int i, const In1& in) {
  float pv[N_PUB1], pub[N_PUB1], o[N_OUT1];
  if (in.nr.par >= 0) xload<XL>(L, F_R, in.nr.par, pv);
  node_down1<XL>(M, S, L, i, in, in.q, in.qd, pv, pub, o);
  xstore<XL>(L, F_R, i, pub);
  put_fields<F_A0>(&at(L.P, slane(L.nf, i - L.i0)), o);
}
template <bool XL>
__device__ __forceinline__ void pass_down2(const DevModel& M, const DevState& S, const Lvl& L, int i, const In2& in) {
  float pv[7], pub[7];
  float2 qn, qdn;
  if (in.par >= 0) xload<XL, 7, F_SNAP>(L, F_SNAP, in.par, pv);
  node_down2<XL>(M, S, L, i, in, pv, pub, qn, qdn);
  xstore<XL, 7, F_SNAP>(L, F_SNAP, i, pub);
}
// Fused pass of a multi-step launch: down 2 of one step and down 1 of the next walk the
// tree in the same direction, so one sweep does both.  The parent's whole slot comes in
// once; the joint state goes from one part to the other in registers; the flags float
// carries the next step's snapped flag and this step's frozen flag.
template <bool XL>
__device__ __forceinline__ void pass_fused(const DevModel& M, const DevState& S, const Lvl& L, int i, const In2& in2_,
                                           const In1& in1) {
  In2 in2 = in2_;
  in2.par = in1.nr.par;
  in2.l = in1.nr.l;
  float pv[N_PUBD], pv1[N_PUB1], pv2[7];
  if (in2.par >= 0) {
    xload<XL>(L, F_R, in2.par, pv);
    for (int k = 0; k < N_PUB1; ++k) pv1[k] = pv[k];
    for (int k = 0; k < 7; ++k) pv2[k] = pv[F_SNAP + k];
  }
  float pub2[7], pub1[N_PUB1], o[N_OUT1];
  float2 qn, qdn;
  node_down2<XL>(M, S, L, i, in2, pv2, pub2, qn, qdn);
  node_down1<XL>(M, S, L, i, in1, qn, qdn, pv1, pub1, o);
  float pub[N_PUBD];
  for (int k = 0; k < F_SNAP; ++k) pub[k] = pub1[k];
  pub[F_SNAP] = pub1[F_SNAP] + pub2[0];
  for (int k = 1; k < 7; ++k) pub[F_SNAP + k] = pub2[k];
  xstore<XL>(L, F_R, i, pub);
  put_fields<F_A0>(&at(L.P, slane(L.nf, i - L.i0)), o);
}

template <bool XL>
__device__ __forceinline__ void level_barrier() {
  if constexpr (XL) lds_barrier();
  else __syncthreads();
}

// Steps of a launch: down 1 of the first step, then per step the apple phase, the up pass
// and either the fused pass into the next step or, after the last, down 2.  Save mode (the
// adjoint's recompute) runs one step per launch, so it never fuses.

// Global exchange: any number of nodes per thread and level, loads then arithmetic.
template <int NT>
__device__ __forceinline__ void run_pack_global(const DevModel& M, const DevState& S, const DevInputs& I, Lvl& L,
                                                float* Abuf, int pk, int lb, int le, int64_t n0, int n_inner,
                                                int call_step0) {
  const int t = (int)threadIdx.x;
  for (int lv = lb; lv < le; ++lv) {
    L.a = M.lvl_off[lv];
    const int e = M.lvl_off[lv + 1];
    for (int i = L.a + t; i < e; i += NT) pass_down1<false>(M, S, L, i, load1(M, S, I, i));
    __syncthreads();
  }
  for (int st = 0; st < n_inner; ++st) {
    const int64_t n = n0 + st;
    const uint64_t kstep = splitmix64((uint64_t)n);
    apple_phase<NT>(M, S, I, L, Abuf, pk, n, call_step0 + st, t);
    for (int lv = le - 1; lv >= lb; --lv) {
      L.a = M.lvl_off[lv];
      const int e = M.lvl_off[lv + 1];
      for (int i = L.a + t; i < e; i += NT) {
        float o[N_OUTU];
        node_up<false>(M, S, I, L, i, loadU(M, S, I, L, i), n, kstep, call_step0 + st, o);
        put_fields<F_WM>(&at(L.P, slane(L.nf, i - L.i0)), o);
      }
      __syncthreads();
    }
    const bool fuse = st + 1 < n_inner;
    for (int lv = lb; lv < le; ++lv) {
      L.a = M.lvl_off[lv];
      const int e = M.lvl_off[lv + 1];
      for (int i = L.a + t; i < e; i += NT) {
        if (fuse) pass_fused<false>(M, S, L, i, load2<false>(M, S, L, i), load1<false>(M, S, I, i));
        else pass_down2<false>(M, S, L, i, load2(M, S, L, i));
      }
      __syncthreads();
    }
  }
}

// LDS exchange: at most one node per thread and level (level width <= lds_width <=
// threads).  Each pass is software-pipelined: the loads of this thread's node on the
// next level are issued before the current level's arithmetic; they read only static
// data, data this thread wrote itself, or data completed before the pass began.
// WAVE: the pack is walked by one wavefront (NT = 64, t its lane) without workgroup
// barriers; its exchange is then a single buffer (L.cap = 0): every lane reads its
// neighbours' slots before any lane of the wave writes its own.
template <int NT, bool WAVE = false>
__device__ __forceinline__ void run_pack_lds(const DevModel& M, const DevState& S, const DevInputs& I, Lvl& L,
                                             float* Abuf, int pk, int lb, int le, int64_t n0, int n_inner,
                                             int call_step0) {
  const int t = WAVE ? (int)(threadIdx.x & 63u) : (int)threadIdx.x;
  {
    int i = M.lvl_off[lb] + lvl_lane<NT>(t, lb);
    bool has = i < M.lvl_off[lb + 1];
    In1 cur{};
    if (has) cur = load1(M, S, I, i);
    for (int lv = lb; lv < le; ++lv) {
      L.a = M.lvl_off[lv];
      L.nbr = lv > lb ? M.lvl_off[lv - 1] : L.a;
      L.b = (lv - lb) & 1;
      const int in_ = M.lvl_off[lv + 1] + lvl_lane<NT>(t, lv + 1);
      const bool hn = lv + 1 < le && in_ < M.lvl_off[lv + 2];
      In1 nxt{};
      if (hn) nxt = load1(M, S, I, in_);
      if (has) pass_down1<true>(M, S, L, i, cur);
      if (lv + 1 < le) sync_lds<WAVE>();
      i = in_; has = hn; cur = nxt;
    }
  }
  sync_all<WAVE>();
  for (int st = 0; st < n_inner; ++st) {
    const int64_t n = n0 + st;
    const uint64_t kstep = splitmix64((uint64_t)n);
    apple_phase<NT, WAVE>(M, S, I, L, Abuf, pk, n, call_step0 + st, t);
    {
      int i = M.lvl_off[le - 1] + lvl_lane<NT>(t, le - 1);
      bool has = i < M.lvl_off[le];
      InU cur{};
      if (has) cur = loadU(M, S, I, L, i);
      for (int lv = le - 1; lv >= lb; --lv) {
        L.a = M.lvl_off[lv];
        L.nbr = M.lvl_off[lv + 1];
        L.b = (lv - lb) & 1;
        const int in_ = lv > lb ? M.lvl_off[lv - 1] + lvl_lane<NT>(t, lv - 1) : 0;
        const bool hn = lv > lb && in_ < M.lvl_off[lv];
        InU nxt{};
        if (hn) nxt = loadU(M, S, I, L, in_);
        if (has) {
          float o[N_OUTU];
          node_up<true>(M, S, I, L, i, cur, n, kstep, call_step0 + st, o);
          put_fields<F_WM>(&at(L.P, slane(L.nf, i - L.i0)), o);
        }
        if (lv > lb) sync_lds<WAVE>();
        i = in_; has = hn; cur = nxt;
      }
    }
    sync_all<WAVE>();
    if (st + 1 < n_inner) {
      int i = M.lvl_off[lb] + lvl_lane<NT>(t, lb);
      bool has = i < M.lvl_off[lb + 1];
      In2 c2{};
      In1 c1{};
      if (has) { c2 = load2<false>(M, S, L, i); c1 = load1<false>(M, S, I, i); }
      for (int lv = lb; lv < le; ++lv) {
        L.a = M.lvl_off[lv];
        L.nbr = lv > lb ? M.lvl_off[lv - 1] : L.a;
        L.b = (lv - lb) & 1;
        const int in_ = M.lvl_off[lv + 1] + lvl_lane<NT>(t, lv + 1);
        const bool hn = lv + 1 < le && in_ < M.lvl_off[lv + 2];
        In2 n2{};
        In1 n1{};
        if (hn) { n2 = load2<false>(M, S, L, in_); n1 = load1<false>(M, S, I, in_); }
        if (has) pass_fused<true>(M, S, L, i, c2, c1);
        if (lv + 1 < le) sync_lds<WAVE>();
        i = in_; has = hn; c2 = n2; c1 = n1;
      }
    } else {
      int i = M.lvl_off[lb] + lvl_lane<NT>(t, lb);
      bool has = i < M.lvl_off[lb + 1];
      In2 cur{};
      if (has) cur = load2(M, S, L, i);
      for (int lv = lb; lv < le; ++lv) {
        L.a = M.lvl_off[lv];
        L.nbr = lv > lb ? M.lvl_off[lv - 1] : L.a;
        L.b = (lv - lb) & 1;
        const int in_ = M.lvl_off[lv + 1] + lvl_lane<NT>(t, lv + 1);
        const bool hn = lv + 1 < le && in_ < M.lvl_off[lv + 2];
        In2 nxt{};
        if (hn) nxt = load2(M, S, L, in_);
        if (has) pass_down2<true>(M, S, L, i, cur);
        if (lv + 1 < le) sync_lds<WAVE>();
        i = in_; has = hn; cur = nxt;
      }
    }
    sync_all<WAVE>();
  }
}

template <int NT, bool XL>
__device__ __forceinline__ void run_pack(const DevModel& M, const DevState& S, const DevInputs& I, float* X,
                                         float* Abuf, int pk, int64_t n0, int n_inner, int call_step0) {
  const int lb = ldc(M.pack_lvl, pk), le = ldc(M.pack_lvl, pk + 1) - 1;
  Lvl L;
  L.i0 = ldc(M.pack_node, pk) & ~63;
  L.nf = M.scr_nf;
  L.P = M.scr + (size_t)(L.i0 >> 6) * (size_t)L.nf * 64u;
  L.X = X;
  L.cap = M.lds_cap;
  L.b = 0;
  if constexpr (XL) run_pack_lds<NT>(M, S, I, L, Abuf, pk, lb, le, n0, n_inner, call_step0);
  else run_pack_global<NT>(M, S, I, L, Abuf, pk, lb, le, n0, n_inner, call_step0);
}

template <int NT>
__device__ __forceinline__ void run_pack_any(const DevModel& M, const DevState& S, const DevInputs& I, float* X,
                                             float* Abuf, int pk, int64_t n0, int n_inner, int call_step0) {
  if (M.lds_cap > 0 && ldc(M.pack_wmax, pk) <= M.lds_cap) run_pack<NT, true>(M, S, I, X, Abuf, pk, n0, n_inner, call_step0);
  else run_pack<NT, false>(M, S, I, X, Abuf, pk, n0, n_inner, call_step0);
}

// A pack walked by one wavefront: its levels fit 64 lanes and exchange through the
// wave's own X_STRIDE x 64 floats of LDS (a single buffer), which also hold the apple
// phase's chunk buffer.
__device__ __forceinline__ void run_pack_wave(const DevModel& M, const DevState& S, const DevInputs& I, float* X,
                                              int pk, int64_t n0, int n_inner, int call_step0) {
  const int lb = ldc(M.pack_lvl, pk), le = ldc(M.pack_lvl, pk + 1) - 1;
  Lvl L;
  L.i0 = ldc(M.pack_node, pk) & ~63;
  L.nf = M.scr_nf;
  L.P = M.scr + (size_t)(L.i0 >> 6) * (size_t)L.nf * 64u;
  L.X = X;
  L.cap = 0;
  L.b = 0;
  run_pack_lds<64, true>(M, S, I, L, X, pk, lb, le, n0, n_inner, call_step0);
}

// Packs [0, n_wide): one workgroup each; dynamic LDS max(2 * X_STRIDE * lds_cap, 11 * NT)
// floats, the level exchange and, between down 1 and up, the apple phase's chunk buffer.
// Packs [n_wide, n_pack): NT / 64 per workgroup, one per wavefront, X_STRIDE * 64 floats
// of LDS each.  At least three waves per SIMD (at most 168 VGPRs): the exchange LDS of
// the widest packs also allows three workgroups of 256 work-items per CU.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_step_packs(DevModel M, DevState S, DevInputs I, int n_inner, int call_step0) {
  HIP_DYNAMIC_SHARED(float4, xlds4)
  float* xlds = reinterpret_cast<float*>(xlds4);
  const int64_t n0 = *S.step;
  const int b = (int)blockIdx.x + M.pack_base;
  if (b < M.n_wide) {
    run_pack_any<NT>(M, S, I, xlds, xlds, b, n0, n_inner, call_step0);
    return;
  }
  const int w = (int)(threadIdx.x >> 6);
  const int pk = M.n_wide + (b - M.n_wide) * (NT / 64) + w;
  if (pk < M.n_pack) run_pack_wave(M, S, I, xlds + w * (X_STRIDE * 64), pk, n0, n_inner, call_step0);
}

// persistent grid: workgroups pull packs (largest first) from a counter
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_step_persistent(DevModel M, DevState S, DevInputs I, int n_inner,
                                                        int call_step0, int32_t* counter) {
  HIP_DYNAMIC_SHARED(float4, xlds4)
  float* xlds = reinterpret_cast<float*>(xlds4);
  __shared__ int pk;
  const int64_t n0 = *S.step;
  for (;;) {
    if (threadIdx.x == 0) pk = atomicAdd(counter, 1);
    __syncthreads();
    const int p = pk;
    __syncthreads();
    if (p >= M.n_pack) break;
    run_pack_any<NT>(M, S, I, xlds, xlds, p, n0, n_inner, call_step0);
  }
}

__global__ void k_advance(int64_t* step, int32_t* counter, int n) {
  *step += n;
  if (counter) *counter = 0;
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = v;
}

// rest state: q = qd = 0, apples at rest, counters zero
__global__ void k_state_rest(DevModel M, DevState S, const float* apple_rest) {
  const int NS = M.n_seg, NA = M.n_apple;
  const int64_t tot = (int64_t)NS + NA;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
    if (k < NS) {
      const int i = (int)k;
      S.q[i] = make_float2(0.f, 0.f);
      S.qd[i] = make_float2(0.f, 0.f);
      S.seg_evt[i] = 0; S.seg_evt[NS + i] = 0;
      S.evt_step[i] = -1;
      if (S.evt_ratio) S.evt_ratio[i] = 0.f;
    } else {
      const int a = (int)(k - NS);
      for (int c = 0; c < 3; ++c) { S.apple[c * NA + a] = apple_rest[c * NA + a]; S.apple[(3 + c) * NA + a] = 0.f; }
      if (M.apl == 13) {
        for (int c = 0; c < 3; ++c) S.apple[(10 + c) * NA + a] = 0.f;
        S.apple[6 * NA + a] = 1.f; S.apple[7 * NA + a] = 0.f; S.apple[8 * NA + a] = 0.f; S.apple[9 * NA + a] = 0.f;
      }
      for (int c = 0; c < 4; ++c) S.apple_evt[c * NA + a] = 0;
      S.evt_step[NS + a] = -1;
      if (S.evt_ratio) S.evt_ratio[NS + a] = 0.f;
    }
    if (k < M.n_env) S.status[k] = 0u;
    if (k == 0) *S.step = 0;
  }
}

// checkpoint: copy the state into one contiguous 32-bit record
//   q (2S) qd (2S) apple (P A, P planes) seg_evt (S words) apple_evt (A words) evt_step (S+A) status (B) step (2)
__device__ __forceinline__ int64_t ckpt_words(const DevModel& M) {
  return 4LL * M.n_seg + (int64_t)M.apl * M.n_apple + M.n_seg + M.n_apple + M.n_seg + M.n_apple + M.n_env + 2;
}

__global__ void k_ckpt_save(DevModel M, DevState S, uint32_t* out) {
  const int NS = M.n_seg, NA = M.n_apple, NB = M.n_env;
  const int64_t PA = (int64_t)M.apl * NA;
  const int64_t tot = ckpt_words(M);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = k;
    uint32_t v;
    if (j < 2LL * NS) v = __float_as_uint(reinterpret_cast<const float*>(S.q)[j]);
    else if ((j -= 2LL * NS) < 2LL * NS) v = __float_as_uint(reinterpret_cast<const float*>(S.qd)[j]);
    else if ((j -= 2LL * NS) < PA) v = __float_as_uint(S.apple[j]);
    else if ((j -= PA) < NS) v = (uint32_t)S.seg_evt[j] | ((uint32_t)S.seg_evt[NS + j] << 8);
    else if ((j -= NS) < NA) v = (uint32_t)S.apple_evt[j] | ((uint32_t)S.apple_evt[NA + j] << 8) |
                                 ((uint32_t)S.apple_evt[2 * NA + j] << 16) | ((uint32_t)S.apple_evt[3 * NA + j] << 24);
    else if ((j -= NA) < (int64_t)NS + NA) v = (uint32_t)S.evt_step[j];
    else if ((j -= (int64_t)NS + NA) < NB) v = S.status[j];
    else { j -= NB; const uint64_t st = (uint64_t)*S.step; v = (uint32_t)(j == 0 ? (st & 0xffffffffull) : (st >> 32)); }
    out[k] = v;
  }
}

__global__ void k_ckpt_load(DevModel M, DevState S, const uint32_t* in) {
  const int NS = M.n_seg, NA = M.n_apple, NB = M.n_env;
  const int64_t PA = (int64_t)M.apl * NA;
  const int64_t tot = ckpt_words(M);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = k;
    const uint32_t v = in[k];
    if (j < 2LL * NS) reinterpret_cast<float*>(S.q)[j] = __uint_as_float(v);
    else if ((j -= 2LL * NS) < 2LL * NS) reinterpret_cast<float*>(S.qd)[j] = __uint_as_float(v);
    else if ((j -= 2LL * NS) < PA) S.apple[j] = __uint_as_float(v);
    else if ((j -= PA) < NS) { S.seg_evt[j] = v & 255u; S.seg_evt[NS + j] = (v >> 8) & 255u; }
    else if ((j -= NS) < NA) {
      S.apple_evt[j] = v & 255u; S.apple_evt[NA + j] = (v >> 8) & 255u; S.apple_evt[2 * NA + j] = (v >> 16) & 255u;
      S.apple_evt[3 * NA + j] = (v >> 24) & 255u;
    } else if ((j -= NA) < (int64_t)NS + NA) S.evt_step[j] = (int32_t)v;
    else if ((j -= (int64_t)NS + NA) < NB) S.status[j] = v;
    else if (j - NB == 1) *S.step = (int64_t)(((uint64_t)v << 32) | (uint64_t)in[k - 1]);
  }
}

template __global__ void k_step_packs<64>(DevModel, DevState, DevInputs, int, int);
template __global__ void k_step_packs<128>(DevModel, DevState, DevInputs, int, int);
template __global__ void k_step_packs<256>(DevModel, DevState, DevInputs, int, int);
template __global__ void k_step_packs<512>(DevModel, DevState, DevInputs, int, int);
template __global__ void k_step_persistent<64>(DevModel, DevState, DevInputs, int, int, int32_t*);
template __global__ void k_step_persistent<128>(DevModel, DevState, DevInputs, int, int, int32_t*);
template __global__ void k_step_persistent<256>(DevModel, DevState, DevInputs, int, int, int32_t*);
template __global__ void k_step_persistent<512>(DevModel, DevState, DevInputs, int, int, int32_t*);

}  // namespace orchard
