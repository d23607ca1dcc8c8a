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
// parity and indexed by the node's slot within its level; otherwise (very wide packs,
// and the adjoint's recompute, which reads these values back) through global scratch.
#include "orchard_dev.h"

namespace orchard {

__device__ __forceinline__ float ld(const DevModel& M, int f, int i) { return M.scr[scr_idx(M, f, i)]; }
__device__ __forceinline__ void sto(const DevModel& M, int f, int i, float v) { M.scr[scr_idx(M, f, i)] = v; }
__device__ __forceinline__ V3 ld3(const DevModel& M, int f, int i) { return v3(ld(M, f, i), ld(M, f + 1, i), ld(M, f + 2, i)); }
__device__ __forceinline__ void sto3(const DevModel& M, int f, int i, V3 v) { sto(M, f, i, v.x); sto(M, f + 1, i, v.y); sto(M, f + 2, i, v.z); }

// publication access: field f of a publication block starting at field f0, of node i
// (slot s within its level, level-parity buffer b)
template <bool XL>
__device__ __forceinline__ float xget(const DevModel& M, const float* X, int f0, int f, int i, int s, int b) {
  if constexpr (XL) return X[(b * N_PUB_MAX + (f - f0)) * M.lds_cap + s];
  else return ld(M, f, i);
}
template <bool XL>
__device__ __forceinline__ void xput(const DevModel& M, float* X, int f0, int f, int i, int s, int b, float v) {
  if constexpr (XL) X[(b * N_PUB_MAX + (f - f0)) * M.lds_cap + s] = v;
  else sto(M, f, i, v);
}
template <bool XL>
__device__ __forceinline__ V3 xget3(const DevModel& M, const float* X, int f0, int f, int i, int s, int b) {
  return v3(xget<XL>(M, X, f0, f, i, s, b), xget<XL>(M, X, f0, f + 1, i, s, b), xget<XL>(M, X, f0, f + 2, i, s, b));
}
template <bool XL>
__device__ __forceinline__ void xput3(const DevModel& M, float* X, int f0, int f, int i, int s, int b, V3 v) {
  xput<XL>(M, X, f0, f, i, s, b, v.x); xput<XL>(M, X, f0, f + 1, i, s, b, v.y); xput<XL>(M, X, f0, f + 2, i, s, b, v.z);
}

__device__ __forceinline__ bool finite3(V3 a) { return isfinite(a.x) && isfinite(a.y) && isfinite(a.z); }

// ------------------------------------------------------------------------------------------
// down pass 1
// ------------------------------------------------------------------------------------------
// i: node, s: its slot in its level, b: its level's buffer, pb: first node of the parent level
template <bool XL>
__device__ void node_down1(const DevModel& M, const DevState& S, const DevInputs& I, float* X, int i, int s, int b,
                           int pb, int64_t n, int s_call) {
  const int NS = M.n_seg;
  const int e = M.env[i];
  const bool skip = S.status[e] != 0u;
  sto(M, F_SKIP, i, skip ? 1.f : 0.f);
  if (skip) return;
  const int par = M.par[i];
  Mat3 Rp;
  V3 pj, w, vt, Aa, Al;
  bool snp;
  if (par < 0) {
    for (int k = 0; k < 9; ++k) Rp.m[k] = (k % 4 == 0) ? 1.f : 0.f;
    pj = v3(0, 0, 0); w = pj; vt = pj; Aa = pj;
    Al = v3(-M.gx, -M.gy, -M.gz);  // gravity as a base acceleration
    snp = false;
  } else {
    const int ps = par - pb, bp = b ^ 1;
    for (int k = 0; k < 9; ++k) Rp.m[k] = xget<XL>(M, X, F_R, F_R + k, par, ps, bp);
    pj = xget3<XL>(M, X, F_R, F_PT, par, ps, bp);
    w = xget3<XL>(M, X, F_R, F_W, par, ps, bp);
    vt = xget3<XL>(M, X, F_R, F_VT, par, ps, bp);
    Aa = xget3<XL>(M, X, F_R, F_AVA, par, ps, bp);
    Al = xget3<XL>(M, X, F_R, F_AVL, par, ps, bp);
    snp = xget<XL>(M, X, F_R, F_SNAP, par, ps, bp) != 0.f;
  }
  const float2 q = S.q[i], qd = S.qd[i];
  const float kp = I.kp[i], kd = I.kd[i];
  const float4 g4 = M.geo[i];
  const float l = g4.x, m = g4.y, Jt = g4.z, Ia = g4.w;
  const float h = M.h;

  // ---- rupture test on the state at the start of the step (Eq. break) ----
  uint8_t brk = S.seg_evt[i];
  if (!brk) {
    const float th = sqrtf(fmaf(q.x, q.x, q.y * q.y));
    const float mu = kp * th / M.mmax[i];
    int c = mu > 1.f ? (int)S.seg_evt[NS + i] + 1 : 0;
    c = c > 255 ? 255 : c;
    if (c >= M.n_break) { brk = 1; S.seg_evt[i] = 1; S.evt_step[i] = (int32_t)n; }
    S.seg_evt[NS + i] = (uint8_t)c;
  }
  snp = snp || brk;

  // ---- kinematics: R = R_parent Q_rest R_x(theta_x) R_y(theta_y) ----
  // the joint rotations are formed from half-angle sines (1 - cos = 2 sin^2(theta/2))
  const float4 r = M.rq[i];
  Mat3 Q;
  {
    const float ww = r.x, xx = r.y, yy = r.z, zz = r.w;
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
  const V3 u = fma3(qd.x, a0, qd.y * a1);       // relative angular velocity
  const V3 wi = w + u;
  const V3 v = vt;                              // joint point moves with the parent
  const V3 cang = fma3(qd.x * qd.y, cross(a0, a1), cross(wi, u));
  const V3 clin = cross(v, u);
  const V3 Ava = Aa + cang, Avl = Al + clin;

  // ---- publish for children (values at the tip point) ----
  const V3 lz = l * z;
  xput<XL>(M, X, F_R, F_R + 0, i, s, b, c0.x); xput<XL>(M, X, F_R, F_R + 1, i, s, b, c1.x); xput<XL>(M, X, F_R, F_R + 2, i, s, b, c2.x);
  xput<XL>(M, X, F_R, F_R + 3, i, s, b, c0.y); xput<XL>(M, X, F_R, F_R + 4, i, s, b, c1.y); xput<XL>(M, X, F_R, F_R + 5, i, s, b, c2.y);
  xput<XL>(M, X, F_R, F_R + 6, i, s, b, c0.z); xput<XL>(M, X, F_R, F_R + 7, i, s, b, c1.z); xput<XL>(M, X, F_R, F_R + 8, i, s, b, c2.z);
  xput3<XL>(M, X, F_R, F_PT, i, s, b, pj + lz);
  xput3<XL>(M, X, F_R, F_W, i, s, b, wi);
  xput3<XL>(M, X, F_R, F_VT, i, s, b, v + cross(wi, lz));
  xput3<XL>(M, X, F_R, F_AVA, i, s, b, Ava);
  xput3<XL>(M, X, F_R, F_AVL, i, s, b, Avl + cross(Ava, lz));
  xput<XL>(M, X, F_R, F_SNAP, i, s, b, snp ? 1.f : 0.f);
  if (!XL && M.save_adj) {
    sto(M, F_SR + 0, i, c0.x); sto(M, F_SR + 1, i, c1.x); sto(M, F_SR + 2, i, c2.x);
    sto(M, F_SR + 3, i, c0.y); sto(M, F_SR + 4, i, c1.y); sto(M, F_SR + 5, i, c2.y);
    sto(M, F_SR + 6, i, c0.z); sto(M, F_SR + 7, i, c1.z); sto(M, F_SR + 8, i, c2.z);
    sto3(M, F_SAVP, i, Ava); sto3(M, F_SAVP + 3, i, Avl);
  }

  // ---- rigid body inertia about the joint point: axisymmetric capsule ----
  const float ml2 = 0.5f * m * l;
  V3 ho = ml2 * z;
  const float dJ = Ia - Jt;
  Sym3 Jo{fmaf(dJ, z.x * z.x, Jt), fmaf(dJ, z.y * z.y, Jt), fmaf(dJ, z.z * z.z, Jt), dJ * z.x * z.y, dJ * z.x * z.z,
          dJ * z.y * z.z};
  float mo = m;
  // bias force p = v x* (I v)
  const V3 K = mul(Jo, wi) + cross(ho, v);
  const V3 L = m * v - cross(ho, wi);
  V3 pang = cross(wi, K) + cross(v, L);
  V3 plin = cross(wi, L);

  // ---- applied body force (input and counter-based random), impulse cap, snapped mask ----
  {
    V3 F, T;
    if (applied_force(M, I, i, e, n, s_call, m, snp, F, T)) {
      pang = pang - (T + cross(0.5f * lz, F));
      plin = plin - F;
    }
  }

  // ---- apples hanging from this segment ----
  const int ab = M.apple_beg[i], ae = M.apple_beg[i + 1];
  const int NA = M.n_apple;
  bool apple_bad = false;
  for (int a = ab; a < ae; ++a) {
    const float4 hm = M.ahang[a];
    const float4 ap = M.apar[a];
    const float ma = hm.w, fdet = ap.x, cs = ap.y, fmax = ap.z;
    const V3 d = fma3(hm.x, c0, fma3(hm.y, c1, hm.z * c2));
    const V3 vh = v + cross(wi, d);
    float* P = S.apple;
    // position state: while attached sigma = (x - x_hang) + h v from the previous
    // update, so the stretch now is s = sigma - h v_hang; once detached, x minus the
    // rest hang point.  The stretch never passes through absolute positions.
    const V3 sig = v3(P[a], P[NA + a], P[2 * NA + a]);
    V3 va = v3(P[3 * NA + a], P[4 * NA + a], P[5 * NA + a]);
    const uint8_t det0 = S.apple_evt[a];
    const V3 sa = det0 ? v3(0, 0, 0) : fma3(-h, vh, sig);
    V3 Fa = v3(0, 0, 0);
    if (I.aforce) {
      const float* fp = I.aforce + (int64_t)s_call * I.aforce_stride + 3 * (int64_t)a;
      Fa = v3(fp[0], fp[1], fp[2]);
    }
    uint8_t det = S.apple_evt[a];
    if (!det) {
      const float pi = sqrtf(dot(Fa, Fa)) / fdet;
      const float tau = M.ks * sqrtf(dot(sa, sa)) / (M.alpha * fdet);
      int cp = pi > 1.f ? (int)S.apple_evt[NA + a] + 1 : 0;
      int ct = tau > 1.f ? (int)S.apple_evt[2 * NA + a] + 1 : 0;
      cp = cp > 255 ? 255 : cp;
      ct = ct > 255 ? 255 : ct;
      S.apple_evt[NA + a] = (uint8_t)cp;
      S.apple_evt[2 * NA + a] = (uint8_t)ct;
      const int path = cp >= M.n_pull ? 1 : (ct >= M.n_tension ? 2 : 0);
      if (path) {
        det = 1;
        S.apple_evt[a] = 1;
        S.apple_evt[3 * NA + a] = (uint8_t)path;
        S.evt_step[NS + a] = (int32_t)n;
      }
    }
    const V3 gv = v3(M.gx, M.gy, M.gz);
    if (!det) {
      // reaction on the spur: elastic tether force minus static weight, hang point
      // taken at the end of the step to first order (linearly implicit); the clamp
      // scales explicit part and implicit term alike by s = min(1, F_max / |f|)
      V3 fh = M.ks * fma3(-h, vh, sa) - ma * gv;
      const float nf = sqrtf(dot(fh, fh));
      const float sc = nf > fmax ? fmax / nf : 1.f;
      fh = sc * fh;
      pang = pang - cross(d, fh);
      plin = plin - fh;
      {
        // virtual point mass s h^2 k_s at the hang point (only its q-acceleration part)
        const float mv = sc * h * h * M.ks;
        mo += mv;
        ho = fma3(mv, d, ho);
        const float dd = dot(d, d);
        Jo.xx = fmaf(mv, dd - d.x * d.x, Jo.xx); Jo.yy = fmaf(mv, dd - d.y * d.y, Jo.yy);
        Jo.zz = fmaf(mv, dd - d.z * d.z, Jo.zz); Jo.xy = fmaf(-mv, d.x * d.y, Jo.xy);
        Jo.xz = fmaf(-mv, d.x * d.z, Jo.xz); Jo.yz = fmaf(-mv, d.y * d.z, Jo.yz);
        const V3 wvp = Avl + cross(Ava, d);
        pang = pang - mv * cross(d, wvp);
        plin = plin - mv * wvp;
      }
    }
    // apple update: explicit symplectic Euler
    V3 fa = fma3(ma, gv, Fa);
    if (!det) fa = fa - M.ks * sa - cs * va;
    va = fma3(h / ma, fa, va);
    // attached: sigma+ = s + h v+;  detached: (x - x_hang,rest)+ = x - x_hang,rest + h v+
    V3 base = sa;
    if (det) {
      if (det0) base = sig;
      else {
        const float4 hr = M.ahrest[a];
        base = (pj + d - v3(hr.x, hr.y, hr.z)) + sa;
      }
    }
    const V3 x = fma3(h, va, base);
    P[a] = x.x; P[NA + a] = x.y; P[2 * NA + a] = x.z;
    P[3 * NA + a] = va.x; P[4 * NA + a] = va.y; P[5 * NA + a] = va.z;
    const V3 om = v3(P[10 * NA + a], P[11 * NA + a], P[12 * NA + a]);
    const V3 hw = (0.5f * h) * om;
    const float th = sqrtf(dot(hw, hw));
    if (th > 0.f) {
      float sn, cn;
      sincosf(th, &sn, &cn);
      const float sc = sn / th;
      const float ew = cn, ex = sc * hw.x, ey = sc * hw.y, ez = sc * hw.z;
      const float q0 = P[6 * NA + a], q1 = P[7 * NA + a], q2 = P[8 * NA + a], q3 = P[9 * NA + a];
      float nw = ew * q0 - ex * q1 - ey * q2 - ez * q3;
      float nx = ew * q1 + ex * q0 + ey * q3 - ez * q2;
      float ny = ew * q2 - ex * q3 + ey * q0 + ez * q1;
      float nz = ew * q3 + ex * q2 - ey * q1 + ez * q0;
      const float inv = 1.f / sqrtf(nw * nw + nx * nx + ny * ny + nz * nz);
      P[6 * NA + a] = nw * inv; P[7 * NA + a] = nx * inv; P[8 * NA + a] = ny * inv; P[9 * NA + a] = nz * inv;
    }
    apple_bad = apple_bad || !finite3(x) || !finite3(va);
  }
  if (apple_bad) atomicOr(&S.status[e], 1u);

  // ---- spring / damper, implicit diagonal ----
  const float kpe = brk ? 0.f : kp, kde = brk ? 0.f : kd;
  const float tau0 = -kpe * fmaf(h, qd.x, q.x) - kde * qd.x;
  const float tau1 = -kpe * fmaf(h, qd.y, q.y) - kde * qd.y;
  const float dg = fmaf(h, kde, h * h * kpe);

  sto3(M, F_A0, i, a0); sto3(M, F_A1, i, a1);
  sto3(M, F_C, i, cang); sto3(M, F_C + 3, i, clin);
  sto3(M, F_P, i, pang); sto3(M, F_P + 3, i, plin);
  sto(M, F_MO, i, mo); sto3(M, F_HO, i, ho);
  sto(M, F_JO + 0, i, Jo.xx); sto(M, F_JO + 1, i, Jo.yy); sto(M, F_JO + 2, i, Jo.zz);
  sto(M, F_JO + 3, i, Jo.xy); sto(M, F_JO + 4, i, Jo.xz); sto(M, F_JO + 5, i, Jo.yz);
  sto(M, F_TAU, i, tau0); sto(M, F_TAU + 1, i, tau1);
  sto(M, F_DG, i, dg);
  sto3(M, F_LZ, i, lz);
}

// ------------------------------------------------------------------------------------------
// up pass: gather children's articulated inertia / bias, factor the 2x2 pivot
// ------------------------------------------------------------------------------------------
// i: node, s: its slot, b: its level's buffer, nb: first node of the next level
template <bool XL>
__device__ void node_up(const DevModel& M, float* X, int i, int s, int b, int nb) {
  if (ld(M, F_SKIP, i) != 0.f) return;
  Sym3 A{0, 0, 0, 0, 0, 0}, Mm{0, 0, 0, 0, 0, 0};
  Mat3 B;
  for (int k = 0; k < 9; ++k) B.m[k] = 0.f;
  V3 pn = v3(0, 0, 0), pf = v3(0, 0, 0);
  const int cb = M.child[i], ce = cb + M.nchild[i];
  for (int c = cb; c < ce; ++c) {
    const int cs = c - nb, bc = b ^ 1;
#define XG(f) xget<XL>(M, X, F_IA, (f), c, cs, bc)
    A.xx += XG(F_IA + 0); A.yy += XG(F_IA + 1); A.zz += XG(F_IA + 2);
    A.xy += XG(F_IA + 3); A.xz += XG(F_IA + 4); A.yz += XG(F_IA + 5);
    for (int k = 0; k < 9; ++k) B.m[k] += XG(F_IB + k);
    Mm.xx += XG(F_IM + 0); Mm.yy += XG(F_IM + 1); Mm.zz += XG(F_IM + 2);
    Mm.xy += XG(F_IM + 3); Mm.xz += XG(F_IM + 4); Mm.yz += XG(F_IM + 5);
    pn = pn + v3(XG(F_PA + 0), XG(F_PA + 1), XG(F_PA + 2));
    pf = pf + v3(XG(F_PA + 3), XG(F_PA + 4), XG(F_PA + 5));
#undef XG
  }
  const V3 r = ld3(M, F_LZ, i);
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
  {
    const float mo = ld(M, F_MO, i);
    const V3 ho = ld3(M, F_HO, i);
    A.xx += ld(M, F_JO + 0, i); A.yy += ld(M, F_JO + 1, i); A.zz += ld(M, F_JO + 2, i);
    A.xy += ld(M, F_JO + 3, i); A.xz += ld(M, F_JO + 4, i); A.yz += ld(M, F_JO + 5, i);
    // B += [h]
    B.m[1] -= ho.z; B.m[2] += ho.y; B.m[3] += ho.z; B.m[5] -= ho.x; B.m[6] -= ho.y; B.m[7] += ho.x;
    Mm.xx += mo; Mm.yy += mo; Mm.zz += mo;
    pn = pn + ld3(M, F_P, i);
    pf = pf + ld3(M, F_P + 3, i);
  }
  if (!XL && M.save_adj) {
    sto(M, F_SIA + 0, i, A.xx); sto(M, F_SIA + 1, i, A.yy); sto(M, F_SIA + 2, i, A.zz);
    sto(M, F_SIA + 3, i, A.xy); sto(M, F_SIA + 4, i, A.xz); sto(M, F_SIA + 5, i, A.yz);
    for (int k = 0; k < 9; ++k) sto(M, F_SIA + 6 + k, i, B.m[k]);
    sto(M, F_SIA + 15, i, Mm.xx); sto(M, F_SIA + 16, i, Mm.yy); sto(M, F_SIA + 17, i, Mm.zz);
    sto(M, F_SIA + 18, i, Mm.xy); sto(M, F_SIA + 19, i, Mm.xz); sto(M, F_SIA + 20, i, Mm.yz);
    sto3(M, F_SPA, i, pn); sto3(M, F_SPA + 3, i, pf);
  }
  const V3 a0 = ld3(M, F_A0, i), a1 = ld3(M, F_A1, i);
  const float dg = ld(M, F_DG, i);
  // U = I^A S,  S = [a0 a1; 0 0]
  const V3 U0a = mul(A, a0), U1a = mul(A, a1);
  const V3 U0l = mulT(B, a0), U1l = mulT(B, a1);
  const float D00 = dot(a0, U0a) + dg, D01 = dot(a0, U1a), D11 = dot(a1, U1a) + dg;
  const float idet = 1.f / fmaf(D00, D11, -D01 * D01);
  const float Di00 = D11 * idet, Di01 = -D01 * idet, Di11 = D00 * idet;
  const float uu0 = ld(M, F_TAU, i) - dot(a0, pn);
  const float uu1 = ld(M, F_TAU + 1, i) - dot(a1, pn);
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
  const V3 ca = ld3(M, F_C, i), cl = ld3(M, F_C + 3, i);
  pn = pn + mul(A, ca) + mul(B, cl) + fma3(uu0, W0a, uu1 * W1a);
  pf = pf + mulT(B, ca) + mul(Mm, cl) + fma3(uu0, W0l, uu1 * W1l);
#define XP(f, v) xput<XL>(M, X, F_IA, (f), i, s, b, (v))
  XP(F_IA + 0, A.xx); XP(F_IA + 1, A.yy); XP(F_IA + 2, A.zz);
  XP(F_IA + 3, A.xy); XP(F_IA + 4, A.xz); XP(F_IA + 5, A.yz);
  for (int k = 0; k < 9; ++k) XP(F_IB + k, B.m[k]);
  XP(F_IM + 0, Mm.xx); XP(F_IM + 1, Mm.yy); XP(F_IM + 2, Mm.zz);
  XP(F_IM + 3, Mm.xy); XP(F_IM + 4, Mm.xz); XP(F_IM + 5, Mm.yz);
  XP(F_PA + 0, pn.x); XP(F_PA + 1, pn.y); XP(F_PA + 2, pn.z);
  XP(F_PA + 3, pf.x); XP(F_PA + 4, pf.y); XP(F_PA + 5, pf.z);
#undef XP
  sto3(M, F_U, i, U0a); sto3(M, F_U + 3, i, U0l); sto3(M, F_U + 6, i, U1a); sto3(M, F_U + 9, i, U1l);
  sto(M, F_DI, i, Di00); sto(M, F_DI + 1, i, Di01); sto(M, F_DI + 2, i, Di11);
  sto(M, F_UU, i, uu0); sto(M, F_UU + 1, i, uu1);
}

// ------------------------------------------------------------------------------------------
// down pass 2: accelerations and integration
// ------------------------------------------------------------------------------------------
// i: node, s: its slot, b: its level's buffer, pb: first node of the parent level
template <bool XL>
__device__ void node_down2(const DevModel& M, const DevState& S, float* X, int i, int s, int b, int pb) {
  if (ld(M, F_SKIP, i) != 0.f) return;
  const int par = M.par[i];
  V3 Aa, Al;
  if (par < 0) { Aa = v3(0, 0, 0); Al = v3(-M.gx, -M.gy, -M.gz); }
  else {
    const int ps = par - pb, bp = b ^ 1;
    Aa = xget3<XL>(M, X, F_AT, F_AT, par, ps, bp);
    Al = xget3<XL>(M, X, F_AT, F_AT + 3, par, ps, bp);
  }
  Aa = Aa + ld3(M, F_C, i);
  Al = Al + ld3(M, F_C + 3, i);
  const V3 U0a = ld3(M, F_U, i), U0l = ld3(M, F_U + 3, i), U1a = ld3(M, F_U + 6, i), U1l = ld3(M, F_U + 9, i);
  const float t0 = ld(M, F_UU, i) - (dot(U0a, Aa) + dot(U0l, Al));
  const float t1 = ld(M, F_UU + 1, i) - (dot(U1a, Aa) + dot(U1l, Al));
  const float Di00 = ld(M, F_DI, i), Di01 = ld(M, F_DI + 1, i), Di11 = ld(M, F_DI + 2, i);
  const float qdd0 = fmaf(Di00, t0, Di01 * t1);
  const float qdd1 = fmaf(Di01, t0, Di11 * t1);
  const V3 a0 = ld3(M, F_A0, i), a1 = ld3(M, F_A1, i);
  Aa = fma3(qdd0, a0, fma3(qdd1, a1, Aa));
  const V3 lz = ld3(M, F_LZ, i);
  if (!XL && M.save_adj) {
    sto3(M, F_SA, i, Aa); sto3(M, F_SA + 3, i, Al);
    sto(M, F_SQDD, i, qdd0); sto(M, F_SQDD + 1, i, qdd1);
  }
  xput3<XL>(M, X, F_AT, F_AT, i, s, b, Aa);
  xput3<XL>(M, X, F_AT, F_AT + 3, i, s, b, Al + cross(Aa, lz));
  const float h = M.h;
  float2 q = S.q[i], qd = S.qd[i];
  qd.x = fmaf(h, qdd0, qd.x);
  qd.y = fmaf(h, qdd1, qd.y);
  q.x = fmaf(h, qd.x, q.x);
  q.y = fmaf(h, qd.y, q.y);
  S.q[i] = q;
  S.qd[i] = qd;
  if (!(isfinite(q.x) && isfinite(q.y) && isfinite(qd.x) && isfinite(qd.y))) atomicOr(&S.status[M.env[i]], 1u);
}

// ------------------------------------------------------------------------------------------
// pack kernels
// ------------------------------------------------------------------------------------------
template <int NT, bool XL>
__device__ __forceinline__ void run_pack(const DevModel& M, const DevState& S, const DevInputs& I, float* X, int pk,
                                         int64_t n0, int n_inner, int call_step0) {
  const int lb = M.pack_lvl[pk], le = M.pack_lvl[pk + 1] - 1;
  for (int st = 0; st < n_inner; ++st) {
    const int64_t n = n0 + st;
    for (int lv = lb; lv < le; ++lv) {
      const int a = M.lvl_off[lv], e = M.lvl_off[lv + 1], pb = lv > lb ? M.lvl_off[lv - 1] : a, b = (lv - lb) & 1;
      for (int i = a + (int)threadIdx.x; i < e; i += NT) node_down1<XL>(M, S, I, X, i, i - a, b, pb, n, call_step0 + st);
      __syncthreads();
    }
    for (int lv = le - 1; lv >= lb; --lv) {
      const int a = M.lvl_off[lv], e = M.lvl_off[lv + 1], b = (lv - lb) & 1;
      for (int i = a + (int)threadIdx.x; i < e; i += NT) node_up<XL>(M, X, i, i - a, b, e);
      __syncthreads();
    }
    for (int lv = lb; lv < le; ++lv) {
      const int a = M.lvl_off[lv], e = M.lvl_off[lv + 1], pb = lv > lb ? M.lvl_off[lv - 1] : a, b = (lv - lb) & 1;
      for (int i = a + (int)threadIdx.x; i < e; i += NT) node_down2<XL>(M, S, X, i, i - a, b, pb);
      __syncthreads();
    }
  }
}

template <int NT>
__device__ __forceinline__ void run_pack_any(const DevModel& M, const DevState& S, const DevInputs& I, float* X, int pk,
                                             int64_t n0, int n_inner, int call_step0) {
  if (M.lds_cap > 0 && !M.save_adj && M.pack_lds[pk]) run_pack<NT, true>(M, S, I, X, pk, n0, n_inner, call_step0);
  else run_pack<NT, false>(M, S, I, X, pk, n0, n_inner, call_step0);
}

// one workgroup per pack; dynamic LDS: 2 * N_PUB_MAX * lds_cap floats
template <int NT>
__global__ __launch_bounds__(NT) void k_step_packs(DevModel M, DevState S, DevInputs I, int n_inner, int call_step0) {
  extern __shared__ float xlds[];
  const int64_t n0 = *S.step;
  run_pack_any<NT>(M, S, I, xlds, (int)blockIdx.x, n0, n_inner, call_step0);
}

// persistent grid: workgroups pull packs (largest first) from a counter
template <int NT>
__global__ __launch_bounds__(NT) void k_step_persistent(DevModel M, DevState S, DevInputs I, int n_inner,
                                                        int call_step0, int32_t* counter) {
  extern __shared__ float xlds[];
  __shared__ int pk;
  const int64_t n0 = *S.step;
  for (;;) {
    if (threadIdx.x == 0) pk = atomicAdd(counter, 1);
    __syncthreads();
    const int p = pk;
    __syncthreads();
    if (p >= M.n_pack) break;
    run_pack_any<NT>(M, S, I, xlds, p, n0, n_inner, call_step0);
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
    } else {
      const int a = (int)(k - NS);
      for (int c = 0; c < 3; ++c) { S.apple[c * NA + a] = apple_rest[c * NA + a]; S.apple[(3 + c) * NA + a] = 0.f; S.apple[(10 + c) * NA + a] = 0.f; }
      S.apple[6 * NA + a] = 1.f; S.apple[7 * NA + a] = 0.f; S.apple[8 * NA + a] = 0.f; S.apple[9 * NA + a] = 0.f;
      for (int c = 0; c < 4; ++c) S.apple_evt[c * NA + a] = 0;
      S.evt_step[NS + a] = -1;
    }
    if (k < M.n_env) S.status[k] = 0u;
    if (k == 0) *S.step = 0;
  }
}

// checkpoint: copy the state into one contiguous 32-bit record
//   q (2S) qd (2S) apple (13A) seg_evt (S words) apple_evt (A words) evt_step (S+A) status (B) step (2)
__device__ __forceinline__ int64_t ckpt_words(const DevModel& M) {
  return 4LL * M.n_seg + 13LL * M.n_apple + M.n_seg + M.n_apple + M.n_seg + M.n_apple + M.n_env + 2;
}

__global__ void k_ckpt_save(DevModel M, DevState S, uint32_t* out) {
  const int NS = M.n_seg, NA = M.n_apple, NB = M.n_env;
  const int64_t tot = ckpt_words(M);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = k;
    uint32_t v;
    if (j < 2LL * NS) v = __float_as_uint(reinterpret_cast<const float*>(S.q)[j]);
    else if ((j -= 2LL * NS) < 2LL * NS) v = __float_as_uint(reinterpret_cast<const float*>(S.qd)[j]);
    else if ((j -= 2LL * NS) < 13LL * NA) v = __float_as_uint(S.apple[j]);
    else if ((j -= 13LL * NA) < NS) v = (uint32_t)S.seg_evt[j] | ((uint32_t)S.seg_evt[NS + j] << 8);
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
  const int64_t tot = ckpt_words(M);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = k;
    const uint32_t v = in[k];
    if (j < 2LL * NS) reinterpret_cast<float*>(S.q)[j] = __uint_as_float(v);
    else if ((j -= 2LL * NS) < 2LL * NS) reinterpret_cast<float*>(S.qd)[j] = __uint_as_float(v);
    else if ((j -= 2LL * NS) < 13LL * NA) S.apple[j] = __uint_as_float(v);
    else if ((j -= 13LL * NA) < NS) { S.seg_evt[j] = v & 255u; S.seg_evt[NS + j] = (v >> 8) & 255u; }
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
