// Adjoint of one step (switches frozen) and tip positions.
//
// The step solves r(qdd; q, qd, s, kp, kd) = Mt(q) qdd + c(q, qd, s) + Kp(q + h qd) + Kd qd = 0.
// Given the adjoint of the state after the step, with qdd_bar = h (qd_bar' + h q_bar'):
//   lambda = Mt^-1 qdd_bar  (same factorisation as the forward: Mt is symmetric),
//   theta_bar -= (dr/dtheta)^T lambda  for theta in {q, qd, apple stretch, kp, kd},
// and lambda^T r is evaluated as sum_i nu_i . f_i^B + spring terms, where nu (the
// acceleration field of the lambda solve) is the virtual velocity of every body.  The
// reverse pass walks leaf -> root accumulating the adjoints of the down-pass quantities
// of the forward step; rotation adjoints travel as 3-vectors (for R = [dphi] R
// perturbations), so every DoF's derivative is its axis dotted with that vector.
#include "orchard_dev.h"

namespace orchard {

__device__ __forceinline__ float aldf(const DevModel& M, int f, int i) { return M.scr[scr_idx(M, f, i)]; }
__device__ __forceinline__ void asto(const DevModel& M, int f, int i, float v) { M.scr[scr_idx(M, f, i)] = v; }
__device__ __forceinline__ V3 ald3(const DevModel& M, int f, int i) { return v3(aldf(M, f, i), aldf(M, f + 1, i), aldf(M, f + 2, i)); }
__device__ __forceinline__ void asto3(const DevModel& M, int f, int i, V3 v) { asto(M, f, i, v.x); asto(M, f + 1, i, v.y); asto(M, f + 2, i, v.z); }

struct DevAdj {
  float2* q;        // [n_seg] adjoint of q (in: after the step, out: before)
  float2* qd;       // [n_seg]
  float* ax;        // [3][n_apple] adjoint of the apple position state
  float* av;        // [3][n_apple] adjoint of the apple velocity
  float* gkp;       // [n_seg] accumulated
  float* gkd;       // [n_seg] accumulated
  float* gF;        // [n_steps][n_apple][3] or null (this step's slice is gF + s_call * 3 * n_apple)
};

// record words: q (2S) qd (2S) apple (P A, P planes) seg_evt (S) apple_evt (A) ...
struct RecView {
  const float* w;
  int NS, NA, P;
  __device__ float2 q(int i) const { return make_float2(w[2 * i], w[2 * i + 1]); }
  __device__ float2 qd(int i) const { return make_float2(w[2 * NS + 2 * i], w[2 * NS + 2 * i + 1]); }
  __device__ float apple(int plane, int a) const { return w[4 * NS + plane * NA + a]; }
  __device__ uint32_t apple_evt(int a) const { return __float_as_uint(w[4 * NS + P * NA + NS + a]); }
};

// Each pass is split, as in the forward step, into a load stage (the node's own data:
// forward scratch of this step, adjoint state, static records) and a compute stage that
// also reads the neighbouring level's publications; on the LDS path the load stage of the
// next level is issued before the current level's arithmetic, and publications move
// through the LDS exchange (otherwise through the global fields F_LPA, F_LA, F_RB).
// Frozen envs run the arithmetic and skip only the writes that change the adjoint state or
// the gradients; their scratch and publications are read only by nodes of the same env.

// ---- lambda solve, up pass: forward substitution with the stored factor ------------------
struct InLU {
  int cb, ce;
  float l, Di00, Di01, Di11;
  V3 z, a0, a1, W0a, W0l, W1a, W1l;
  float2 qb, qdb;
};
__device__ __forceinline__ InLU load_lu(const DevModel& M, const DevAdj& X, const Lvl& L, int i) {
  const int nf = M.scr_nf, li = i - L.i0;
  const float* P = L.P;
  const int4 topo = at(M.ntopo, (uint32_t)i);
  InLU r;
  r.cb = topo.y;
  r.ce = topo.y + (topo.z & 0xFFFF);
  r.l = at(M.len, (uint32_t)i);
  r.z = pld3(P, nf, F_Z, li);
  r.qb = at(X.q, (uint32_t)i);
  r.qdb = at(X.qd, (uint32_t)i);
  r.a0 = pld3(P, nf, F_A0, li);
  r.a1 = pld3(P, nf, F_A1, li);
  r.W0a = pld3(P, nf, F_WM, li); r.W0l = pld3(P, nf, F_WM + 3, li);
  r.W1a = pld3(P, nf, F_WM + 6, li); r.W1l = pld3(P, nf, F_WM + 9, li);
  r.Di00 = pld(P, nf, F_DI, li); r.Di01 = pld(P, nf, F_DI + 1, li); r.Di11 = pld(P, nf, F_DI + 2, li);
  return r;
}
template <bool XL>
__device__ __forceinline__ void node_lam_up(const DevModel& M, const Lvl& L, int i, const InLU& in) {
  const int nf = M.scr_nf, li = i - L.i0;
  const V3 lz = in.l * in.z;
  const float2 qb = in.qb, qdb = in.qdb;
  const V3 a0 = in.a0, a1 = in.a1;
  const V3 W0a = in.W0a, W0l = in.W0l, W1a = in.W1a, W1l = in.W1l;
  const float Di00 = in.Di00, Di01 = in.Di01, Di11 = in.Di11;
  V3 pn = v3(0, 0, 0), pf = v3(0, 0, 0);
  for (int c = in.cb; c < in.ce; ++c) {
    float cv[6];
    xload<XL>(L, F_LPA, c, cv);
    pn = pn + v3(cv[0], cv[1], cv[2]);
    pf = pf + v3(cv[3], cv[4], cv[5]);
  }
  pn = pn + cross(lz, pf);
  const float h = M.h;
  const float b0 = h * fmaf(h, qb.x, qdb.x), b1 = h * fmaf(h, qb.y, qdb.y);  // qdd_bar
  const float u0 = b0 - dot(a0, pn), u1 = b1 - dot(a1, pn);
  // U D^-1 u = W u; the down pass needs D^-1 u
  pn = fma3(u0, W0a, fma3(u1, W1a, pn));
  pf = fma3(u0, W0l, fma3(u1, W1l, pf));
  pst(L.P, nf, F_LU, li, fmaf(Di00, u0, Di01 * u1)); pst(L.P, nf, F_LU + 1, li, fmaf(Di01, u0, Di11 * u1));
  const float ov[6] = {pn.x, pn.y, pn.z, pf.x, pf.y, pf.z};
  xstore<XL>(L, F_LPA, i, ov);
}

// ---- lambda solve, down pass: back substitution; the field is the virtual velocity nu --
struct InLD {
  int par;
  float l, du0, du1;
  V3 z, a0, a1, W0a, W0l, W1a, W1l;
};
__device__ __forceinline__ InLD load_ld(const DevModel& M, const Lvl& L, int i) {
  const int nf = M.scr_nf, li = i - L.i0;
  const float* P = L.P;
  InLD r;
  r.par = at(M.par, (uint32_t)i);
  r.l = at(M.len, (uint32_t)i);
  r.z = pld3(P, nf, F_Z, li);
  r.W0a = pld3(P, nf, F_WM, li); r.W0l = pld3(P, nf, F_WM + 3, li);
  r.W1a = pld3(P, nf, F_WM + 6, li); r.W1l = pld3(P, nf, F_WM + 9, li);
  r.du0 = pld(P, nf, F_LU, li); r.du1 = pld(P, nf, F_LU + 1, li);
  r.a0 = pld3(P, nf, F_A0, li);
  r.a1 = pld3(P, nf, F_A1, li);
  return r;
}
template <bool XL>
__device__ __forceinline__ void node_lam_down(const DevModel& M, const Lvl& L, int i, const InLD& in) {
  const int nf = M.scr_nf, li = i - L.i0;
  const V3 W0a = in.W0a, W0l = in.W0l, W1a = in.W1a, W1l = in.W1l;
  const float du0 = in.du0, du1 = in.du1;
  const V3 a0 = in.a0, a1 = in.a1, lz = in.l * in.z;
  V3 aa = v3(0, 0, 0), al = v3(0, 0, 0);
  if (in.par >= 0) {
    float pv[6];
    xload<XL>(L, F_LA, in.par, pv);
    aa = v3(pv[0], pv[1], pv[2]);
    al = v3(pv[3], pv[4], pv[5]);
  }
  const float l0 = du0 - (dot(W0a, aa) + dot(W0l, al));
  const float l1 = du1 - (dot(W1a, aa) + dot(W1l, al));
  aa = fma3(l0, a0, fma3(l1, a1, aa));
  float* P = L.P;
  pst3(P, nf, F_NU, li, aa); pst3(P, nf, F_NU + 3, li, al);
  pst(P, nf, F_LAM, li, l0); pst(P, nf, F_LAM + 1, li, l1);
  const V3 at_l = al + cross(aa, lz);
  const float ov[6] = {aa.x, aa.y, aa.z, at_l.x, at_l.y, at_l.z};
  xstore<XL>(L, F_LA, i, ov);
}

// ---- reverse pass (leaf -> root) ---------------------------------------------------------
struct InRV {
  int par, cb, ce, a_beg, a_end;
  uint32_t hk0, hk1;
  float flg, snp, kp, kd, qdd0, qdd1, l0, l1;
  uint8_t brk;
  float4 g4;
  Sym3 IA, IM;
  Mat3 IB;
  V3 a0, a1, z, om, v, Aa, Al, Pa, Pl, na, nl, spn, spf;
  float2 q, qd, qbn, qdbn, gk;
};
__device__ __forceinline__ InRV load_rv(const DevModel& M, const DevState& W, const RecView& R0, const DevInputs& I,
                                        const DevAdj& X, const Lvl& L, int i) {
  const int nf = M.scr_nf, li = i - L.i0;
  const float* P = L.P;
  const int4 topo = at(M.ntopo, (uint32_t)i);
  InRV r;
  r.par = at(M.par, (uint32_t)i);
  r.cb = topo.y;
  r.ce = topo.y + (topo.z & 0xFFFF);
  r.a_beg = at(M.apple_beg, (uint32_t)i);
  r.a_end = at(M.apple_beg, (uint32_t)i + 1u);
  const uint64_t hk = at(M.hkey, (uint32_t)i);
  r.hk0 = (uint32_t)hk;
  r.hk1 = (uint32_t)(hk >> 32);
  r.flg = pld(P, nf, F_SFRZ, li);
  r.snp = pld(P, nf, F_SSNP, li);
  r.a0 = pld3(P, nf, F_A0, li);
  r.a1 = pld3(P, nf, F_A1, li);
  r.z = pld3(P, nf, F_Z, li);
  r.g4 = at(M.geo, (uint32_t)i);
  r.om = pld3(P, nf, F_W, li);
  // the parent's tip velocity comes from this step's forward scratch, not from a
  // publication of this pass
  r.v = r.par >= 0 ? pld3(P, nf, F_VT, r.par - L.i0) : v3(0, 0, 0);
  r.Aa = pld3(P, nf, F_SA, li); r.Al = pld3(P, nf, F_SA + 3, li);
  r.Pa = pld3(P, nf, F_SAVP, li); r.Pl = pld3(P, nf, F_SAVP + 3, li);
  r.qdd0 = pld(P, nf, F_SQDD, li); r.qdd1 = pld(P, nf, F_SQDD + 1, li);
  r.l0 = pld(P, nf, F_LAM, li); r.l1 = pld(P, nf, F_LAM + 1, li);
  r.na = pld3(P, nf, F_NU, li); r.nl = pld3(P, nf, F_NU + 3, li);
  r.IA = Sym3{pld(P, nf, F_SIA + 0, li), pld(P, nf, F_SIA + 1, li), pld(P, nf, F_SIA + 2, li),
              pld(P, nf, F_SIA + 3, li), pld(P, nf, F_SIA + 4, li), pld(P, nf, F_SIA + 5, li)};
  for (int k = 0; k < 9; ++k) r.IB.m[k] = pld(P, nf, F_SIA + 6 + k, li);
  r.IM = Sym3{pld(P, nf, F_SIA + 15, li), pld(P, nf, F_SIA + 16, li), pld(P, nf, F_SIA + 17, li),
              pld(P, nf, F_SIA + 18, li), pld(P, nf, F_SIA + 19, li), pld(P, nf, F_SIA + 20, li)};
  r.spn = pld3(P, nf, F_SPA, li);
  r.spf = pld3(P, nf, F_SPA + 3, li);
  r.q = R0.q(i);
  r.qd = R0.qd(i);
  r.brk = at(W.seg_evt, (uint32_t)i);
  r.kp = at(I.kp, (uint32_t)i);
  r.kd = at(I.kd, (uint32_t)i);
  r.qbn = at(X.q, (uint32_t)i);
  r.qdbn = at(X.qd, (uint32_t)i);
  r.gk = make_float2(at(X.gkp, (uint32_t)i), at(X.gkd, (uint32_t)i));
  return r;
}

template <bool XL>
__device__ __forceinline__ void node_reverse(const DevModel& M, const DevState& W, const RecView& R0,
                                             const DevInputs& I, const DevAdj& X, const Lvl& L, int i,
                                             const InRV& in, int64_t n, int s_call) {
  const bool skip = in.flg != 0.f;  // frozen env: the step is the identity
  const float h = M.h;
  // forward quantities of this node; the body frame is (a1 x z, a1, z)
  const V3 a0 = in.a0, a1 = in.a1, z = in.z;
  const V3 c0 = cross(a1, z), c1 = a1, c2 = z;
  const float4 g4 = in.g4;
  const V3 lz = g4.x * z;
  const V3 om = in.om;
  const V3 v = in.v;
  const V3 Aa = in.Aa, Al = in.Al;
  const V3 Pa = in.Pa, Pl = in.Pl;
  const float qdd0 = in.qdd0, qdd1 = in.qdd1;
  const float l0 = in.l0, l1 = in.l1;
  const V3 na = in.na, nl = in.nl;
  // transmitted force f = I^A A + p^A (before the pivot update)
  const Sym3 IA = in.IA, IM = in.IM;
  const Mat3 IB = in.IB;
  const V3 fn = mul(IA, Aa) + mul(IB, Al) + in.spn;
  const V3 ff = mulT(IB, Aa) + mul(IM, Al) + in.spf;
  const float2 q = in.q, qd = in.qd;
  const V3 u = fma3(qd.x, a0, qd.y * a1);
  const float l = g4.x, m = g4.y, Jt = g4.z, Iax = g4.w, dJ = Iax - Jt;
  const V3 ho = (0.5f * m * l) * z;
  const Sym3 Jo{fmaf(dJ, z.x * z.x, Jt), fmaf(dJ, z.y * z.y, Jt), fmaf(dJ, z.z * z.z, Jt), dJ * z.x * z.y, dJ * z.x * z.z,
                dJ * z.y * z.z};
  const uint8_t brk = in.brk;
  const float kp = in.kp, kd = in.kd;
  const float kpe = brk ? 0.f : kp, kde = brk ? 0.f : kd;

  // accumulators
  V3 Aba = v3(0, 0, 0), Abl = v3(0, 0, 0), Pba = v3(0, 0, 0), Pbl = v3(0, 0, 0);
  V3 omb = v3(0, 0, 0), vb = v3(0, 0, 0), zb = v3(0, 0, 0), a0b = v3(0, 0, 0), a1b = v3(0, 0, 0), lzb = v3(0, 0, 0);
  V3 tau = v3(0, 0, 0);  // rotation adjoint of this body (R -> [dphi] R)
  float qdb0 = 0.f, qdb1 = 0.f;
  // ---- gather the children ----
  V3 vtb = v3(0, 0, 0), Atba = v3(0, 0, 0), Atbl = v3(0, 0, 0), Avtba = v3(0, 0, 0), Avtbl = v3(0, 0, 0), Fch = v3(0, 0, 0);
  V3 pch = v3(0, 0, 0);  // position adjoint of the children's joint points (= this tip)
  for (int c = in.cb; c < in.ce; ++c) {
    float cv[27];
    xload<XL>(L, F_RB, c, cv);
    tau = tau + v3(cv[0], cv[1], cv[2]);
    omb = omb + v3(cv[3], cv[4], cv[5]);
    vtb = vtb + v3(cv[6], cv[7], cv[8]);
    Atba = Atba + v3(cv[9], cv[10], cv[11]);
    Atbl = Atbl + v3(cv[12], cv[13], cv[14]);
    Avtba = Avtba + v3(cv[15], cv[16], cv[17]);
    Avtbl = Avtbl + v3(cv[18], cv[19], cv[20]);
    Fch = Fch + v3(cv[21], cv[22], cv[23]);
    pch = pch + v3(cv[24], cv[25], cv[26]);
  }
  // joint-point positions: children sit at p + lz, this joint point at the parent's tip
  lzb = lzb + pch;
  V3 pb = pch;
  // tip publications: At = (A_ang, A_lin + A_ang x lz), same for Avp; vt = v + om x lz
  Aba = Aba + Atba + cross(lz, Atbl);
  Abl = Abl + Atbl;
  lzb = lzb + cross(Atbl, Aa);
  Pba = Pba + Avtba + cross(lz, Avtbl);
  Pbl = Pbl + Avtbl;
  lzb = lzb + cross(Avtbl, Pa);
  vb = vb + vtb;
  omb = omb + cross(lz, vtb);
  lzb = lzb + cross(vtb, om);
  // children's transmitted force moved from the tip: n += lz x F_children
  lzb = lzb + cross(Fch, na);
  // joint torques tau_k = a_k . n
  a0b = fma3(l0, fn, a0b);
  a1b = fma3(l1, fn, a1b);

  // ---- body force, seed nu: rigid body part I A + V x* I V ----
  Aba = Aba + mul(Jo, na) + cross(ho, nl);
  Abl = Abl + m * nl + cross(na, ho);
  V3 hb = cross(Al, na) - cross(Aa, nl);
  zb = zb + dJ * (dot(na, z) * Aa + dot(Aa, z) * na);
  {
    const V3 K = mul(Jo, om) + cross(ho, v);
    const V3 L = m * v - cross(ho, om);
    const V3 Kb = cross(na, om);
    const V3 Lb = cross(na, v) + cross(nl, om);
    omb = omb + cross(K, na) + cross(L, nl);
    vb = vb + cross(L, na);
    omb = omb + mul(Jo, Kb);
    hb = hb + cross(v, Kb);
    vb = vb + cross(Kb, ho);
    zb = zb + dJ * (dot(Kb, z) * om + dot(om, z) * Kb);
    vb = vb + m * Lb;
    hb = hb - cross(om, Lb);
    omb = omb - cross(Lb, ho);
  }
  // applied force: moment arm (l/2) z
  {
    V3 F, T;
    const bool snp = in.snp != 0.f;
    const uint64_t hkey = (uint64_t)in.hk0 | ((uint64_t)in.hk1 << 32);
    // (models with the rails on are not differentiated, so vc only completes the call)
    const V3 vc = v + cross(om, (0.5f * l) * z);
    if (applied_force(M, I, i, splitmix64((uint64_t)n), s_call, m, snp, hkey, vc, F, T)) zb = zb - (0.5f * l) * cross(F, na);
  }
  zb = fma3(0.5f * m * l, hb, zb);

  // ---- apples on this segment ----
  const int NA = M.n_apple;
  const V3 gv = v3(M.gx, M.gy, M.gz);
  const V3 dAa = Aa - Pa, dAl = Al - Pl;
  float* gF = X.gF ? X.gF + (int64_t)s_call * 3 * NA : nullptr;
  for (int a = in.a_beg; a < in.a_end; ++a) {
    const float4 hm = M.ahang[a];
    const float4 ap = M.apar[a];
    const float ma = hm.w, cs = ap.y, fmax = ap.z;
    const V3 hl = v3(hm.x, hm.y, hm.z);
    const V3 d = fma3(hl.x, c0, fma3(hl.y, c1, hl.z * c2));
    const V3 vh = v + cross(om, d);
    const V3 sig = v3(R0.apple(0, a), R0.apple(1, a), R0.apple(2, a));
    const uint8_t det0 = (uint8_t)(R0.apple_evt(a) & 255u);
    const uint8_t det = W.apple_evt[a];
    const V3 xb = v3(X.ax[a], X.ax[NA + a], X.ax[2 * NA + a]);
    const V3 vbn = v3(X.av[a], X.av[NA + a], X.av[2 * NA + a]);
    const V3 vtot = fma3(h, xb, vbn);
    // Two flows meet here: the apple's own update (direct adjoint) and its reaction on
    // the spur, which enters the step residual r (adjoint -(dr/dx)^T lambda).  The
    // tree-side accumulators hold d(lambda^T r)/dx, so direct terms enter them negated.
    V3 sigb, vab, Fb, db = v3(0, 0, 0), vhb = v3(0, 0, 0);
    if (!det) {
      const V3 s = fma3(-h, vh, sig);
      const V3 fab = (h / ma) * vtot;
      const V3 sd = xb - M.ks * fab;  // direct adjoint of the stretch
      vab = vtot - cs * fab;
      Fb = fab;
      // residual part: lambda^T r contains (mv w - fhat) . nu_pt, nu_pt = nu_lin + nu_ang x d
      const V3 nup = nl + cross(na, d);
      const V3 fe = M.ks * fma3(-h, vh, s) - ma * gv;
      const float nf = sqrtf(dot(fe, fe));
      const bool clamped = nf > fmax;
      const float sc = clamped ? fmax / nf : 1.f;
      const V3 fhat = sc * fe;
      const float mv = sc * h * h * M.ks;
      const V3 w = dAl + cross(dAa, d);
      db = db + cross(mv * w - fhat, na);
      const V3 wb = mv * nup;
      Aba = Aba + cross(d, wb);
      Abl = Abl + wb;
      Pba = Pba - cross(d, wb);
      Pbl = Pbl - wb;
      db = db + cross(wb, dAa);
      const float scb = h * h * M.ks * dot(w, nup) - dot(nup, fe);
      V3 feb = (-sc) * nup;
      if (clamped) feb = feb - (fmax / (nf * nf * nf) * scb) * fe;
      const V3 gs = M.ks * feb;                 // d(lambda^T r)/ds
      sigb = sd - gs;                           // s = sigma - h vh
      vhb = (-2.f * h * M.ks) * feb + h * sd;   // d(lambda^T r)/dvh minus the direct part
    } else {
      // ballistic: x' = x + h v', v' = v + (h/m)(m g + F).  At the detach step the fruit
      // leaves from the hang point plus its stretch, x = p + d + sigma - h vh: the
      // position adjoint reaches the joint point, the hang offset and the hang velocity
      vab = vtot;
      Fb = (h / ma) * vtot;
      sigb = xb;
      if (!det0) {
        vhb = h * xb;
        db = db - xb;
        pb = pb - xb;
      }
    }
    vb = vb + vhb;
    omb = omb + cross(d, vhb);
    db = db + cross(vhb, om);
    tau = tau + cross(d, db);
    if (!skip) {
      X.ax[a] = sigb.x; X.ax[NA + a] = sigb.y; X.ax[2 * NA + a] = sigb.z;
      X.av[a] = vab.x; X.av[NA + a] = vab.y; X.av[2 * NA + a] = vab.z;
      if (gF) { gF[3 * a] += Fb.x; gF[3 * a + 1] += Fb.y; gF[3 * a + 2] += Fb.z; }
    }
  }

  // ---- c, A, Avp, omega, v recursions ----
  const V3 cba = Aba + Pba, cbl = Abl + Pbl;
  a0b = fma3(qdd0, Aba, a0b);
  a1b = fma3(qdd1, Aba, a1b);
  omb = omb + cross(u, cba);
  V3 ub = cross(cba, om);
  const float pq = qd.x * qd.y;
  a0b = fma3(pq, cross(a1, cba), a0b);
  a1b = fma3(pq, cross(cba, a0), a1b);
  const float ca = dot(cross(a0, a1), cba);
  qdb0 = fmaf(qd.y, ca, qdb0);
  qdb1 = fmaf(qd.x, ca, qdb1);
  vb = vb + cross(u, cbl);
  ub = ub + cross(cbl, v);
  ub = ub + omb;  // omega = omega_parent + u
  a0b = fma3(qd.x, ub, a0b);
  a1b = fma3(qd.y, ub, a1b);
  qdb0 += dot(a0, ub);
  qdb1 += dot(a1, ub);
  zb = fma3(l, lzb, zb);

  // ---- rotation: a1 = R e_y and z = R e_z are fixed in the body; a0 in the parent ----
  tau = tau + cross(a1, a1b) + cross(z, zb);
  float qb0 = dot(a0, tau), qb1 = dot(a1, tau);
  const V3 tau_par = tau + cross(a0, a0b);

  // ---- springs, dampers, implicit diagonal; parameter gradients ----
  const float h2 = h * h;
  if (!brk && !skip) {
    at(X.gkp, (uint32_t)i) = in.gk.x - (l0 * (h2 * qdd0 + q.x + h * qd.x) + l1 * (h2 * qdd1 + q.y + h * qd.y));
    at(X.gkd, (uint32_t)i) = in.gk.y - (l0 * (h * qdd0 + qd.x) + l1 * (h * qdd1 + qd.y));
  }
  qb0 = fmaf(kpe, l0, qb0);
  qb1 = fmaf(kpe, l1, qb1);
  qdb0 = fmaf(h * kpe + kde, l0, qdb0);
  qdb1 = fmaf(h * kpe + kde, l1, qdb1);

  // ---- state adjoint before the step ----
  const float2 qbn = in.qbn, qdbn = in.qdbn;
  const float qdp0 = fmaf(h, qbn.x, qdbn.x), qdp1 = fmaf(h, qbn.y, qdbn.y);
  if (!skip) {
    X.q[i] = make_float2(qbn.x - qb0, qbn.y - qb1);
    X.qd[i] = make_float2(qdp0 - qdb0, qdp1 - qdb1);
  }

  // ---- publish for the parent ----
  const float ov[27] = {tau_par.x, tau_par.y, tau_par.z, omb.x, omb.y, omb.z, vb.x, vb.y, vb.z,
                        Aba.x, Aba.y, Aba.z, Abl.x, Abl.y, Abl.z, Pba.x, Pba.y, Pba.z, Pbl.x, Pbl.y, Pbl.z,
                        ff.x, ff.y, ff.z, pb.x, pb.y, pb.z};
  xstore<XL>(L, F_RB, i, ov);
}

// Global exchange (levels wider than the workgroup's exchange buffer): loads then
// arithmetic, any number of nodes per thread and level.
template <int NT>
__device__ __forceinline__ void adjoint_pack_global(const DevModel& M, const DevState& W, const RecView& R0,
                                                    const DevInputs& I, const DevAdj& X, Lvl& L, int lb, int le,
                                                    int64_t n, int s_call) {
  const int t = (int)threadIdx.x;
  for (int lv = le - 1; lv >= lb; --lv) {
    L.a = M.lvl_off[lv];
    L.nbr = M.lvl_off[lv + 1];
    for (int i = L.a + t; i < L.nbr; i += NT) node_lam_up<false>(M, L, i, load_lu(M, X, L, i));
    __syncthreads();
  }
  for (int lv = lb; lv < le; ++lv) {
    L.a = M.lvl_off[lv];
    L.nbr = lv > lb ? M.lvl_off[lv - 1] : L.a;
    const int e = M.lvl_off[lv + 1];
    for (int i = L.a + t; i < e; i += NT) node_lam_down<false>(M, L, i, load_ld(M, L, i));
    __syncthreads();
  }
  for (int lv = le - 1; lv >= lb; --lv) {
    L.a = M.lvl_off[lv];
    L.nbr = M.lvl_off[lv + 1];
    for (int i = L.a + t; i < L.nbr; i += NT)
      node_reverse<false>(M, W, R0, I, X, L, i, load_rv(M, W, R0, I, X, L, i), n, s_call);
    __syncthreads();
  }
}

// LDS exchange: at most one node per thread and level; the next level's loads are issued
// before the current level's arithmetic (they read this step's forward scratch, the
// adjoint state and data this thread wrote in an earlier pass).
template <int NT>
__device__ __forceinline__ void adjoint_pack_lds(const DevModel& M, const DevState& W, const RecView& R0,
                                                 const DevInputs& I, const DevAdj& X, Lvl& L, int lb, int le,
                                                 int64_t n, int s_call) {
  const int t = (int)threadIdx.x;
  {
    int i = M.lvl_off[le - 1] + lvl_lane<NT>(t, le - 1);
    bool has = i < M.lvl_off[le];
    InLU cur{};
    if (has) cur = load_lu(M, X, L, i);
    for (int lv = le - 1; lv >= lb; --lv) {
      L.a = M.lvl_off[lv];
      L.nbr = M.lvl_off[lv + 1];
      L.b = (lv - lb) & 1;
      const int in_ = lv > lb ? M.lvl_off[lv - 1] + lvl_lane<NT>(t, lv - 1) : 0;
      const bool hn = lv > lb && in_ < M.lvl_off[lv];
      InLU nxt{};
      if (hn) nxt = load_lu(M, X, L, in_);
      if (has) node_lam_up<true>(M, L, i, cur);
      if (lv > lb) lds_barrier();
      i = in_; has = hn; cur = nxt;
    }
  }
  __syncthreads();
  {
    int i = M.lvl_off[lb] + lvl_lane<NT>(t, lb);
    bool has = i < M.lvl_off[lb + 1];
    InLD cur{};
    if (has) cur = load_ld(M, L, i);
    for (int lv = lb; lv < le; ++lv) {
      L.a = M.lvl_off[lv];
      L.nbr = lv > lb ? M.lvl_off[lv - 1] : L.a;
      L.b = (lv - lb) & 1;
      const int in_ = M.lvl_off[lv + 1] + lvl_lane<NT>(t, lv + 1);
      const bool hn = lv + 1 < le && in_ < M.lvl_off[lv + 2];
      InLD nxt{};
      if (hn) nxt = load_ld(M, L, in_);
      if (has) node_lam_down<true>(M, L, i, cur);
      if (lv + 1 < le) lds_barrier();
      i = in_; has = hn; cur = nxt;
    }
  }
  __syncthreads();
  {
    int i = M.lvl_off[le - 1] + lvl_lane<NT>(t, le - 1);
    bool has = i < M.lvl_off[le];
    InRV cur{};
    if (has) cur = load_rv(M, W, R0, I, X, L, i);
    for (int lv = le - 1; lv >= lb; --lv) {
      L.a = M.lvl_off[lv];
      L.nbr = M.lvl_off[lv + 1];
      L.b = (lv - lb) & 1;
      const int in_ = lv > lb ? M.lvl_off[lv - 1] + lvl_lane<NT>(t, lv - 1) : 0;
      const bool hn = lv > lb && in_ < M.lvl_off[lv];
      InRV nxt{};
      if (hn) nxt = load_rv(M, W, R0, I, X, L, in_);
      if (has) node_reverse<true>(M, W, R0, I, X, L, i, cur, n, s_call);
      if (lv > lb) lds_barrier();
      i = in_; has = hn; cur = nxt;
    }
  }
}

// one workgroup per pack; dynamic LDS: the level exchange of the step kernels
template <int NT>
__global__ __launch_bounds__(NT) void k_adjoint_packs(DevModel M, DevState W, const float* rec, DevInputs I, DevAdj X,
                                                      int s_call) {
  HIP_DYNAMIC_SHARED(float4, xlds4)
  const int pk = blockIdx.x;
  const int lb = ldc(M.pack_lvl, pk), le = ldc(M.pack_lvl, pk + 1) - 1;
  const int64_t n = *W.step - 1;  // the forward step just taken on W
  const RecView R0{rec, M.n_seg, M.n_apple, M.apl};
  Lvl L;
  L.i0 = ldc(M.pack_node, pk) & ~63;
  L.nf = M.scr_nf;
  L.P = M.scr + (size_t)(L.i0 >> 6) * (size_t)L.nf * 64u;
  L.X = reinterpret_cast<float*>(xlds4);
  L.cap = M.lds_cap;
  L.b = 0;
  if (M.lds_cap > 0 && ldc(M.pack_wmax, pk) <= M.lds_cap) adjoint_pack_lds<NT>(M, W, R0, I, X, L, lb, le, n, s_call);
  else adjoint_pack_global<NT>(M, W, R0, I, X, L, lb, le, n, s_call);
}

// ---- tip positions: p_b + R_b (0, 0, l_b) -----------------------------------------------
// down pass: absolute rotation (F_SR) and tip point (F_LA) of every node
__device__ void node_tip_fk(const DevModel& M, const float2* qs, int i) {
  const int par = M.par[i];
  Mat3 Rp;
  V3 pt = v3(0, 0, 0);
  if (par < 0) { for (int k = 0; k < 9; ++k) Rp.m[k] = (k % 4 == 0) ? 1.f : 0.f; }
  else { for (int k = 0; k < 9; ++k) Rp.m[k] = aldf(M, F_SR + k, par); pt = ald3(M, F_LA, par); }
  const float4 r = M.rq[i];
  const float ww = r.x, xx = r.y, yy = r.z, zz = r.w;
  const V3 Q0 = v3(1.f - 2.f * (yy * yy + zz * zz), 2.f * (xx * yy + ww * zz), 2.f * (xx * zz - ww * yy));
  const V3 Q1 = v3(2.f * (xx * yy - ww * zz), 1.f - 2.f * (xx * xx + zz * zz), 2.f * (yy * zz + ww * xx));
  const V3 Q2 = v3(2.f * (xx * zz + ww * yy), 2.f * (yy * zz - ww * xx), 1.f - 2.f * (xx * xx + yy * yy));
  const V3 J0 = mul(Rp, Q0), J1 = mul(Rp, Q1), J2 = mul(Rp, Q2);
  const float2 q = qs[i];
  float sx, cx, sy, cy;
  sincosf(q.x, &sx, &cx);
  sincosf(q.y, &sy, &cy);
  const V3 c0 = fma3(cy, J0, fma3(sx * sy, J1, (-cx * sy) * J2));
  const V3 c1 = fma3(cx, J1, sx * J2);
  const V3 c2 = fma3(sy, J0, fma3(-sx * cy, J1, (cx * cy) * J2));
  asto(M, F_SR + 0, i, c0.x); asto(M, F_SR + 1, i, c1.x); asto(M, F_SR + 2, i, c2.x);
  asto(M, F_SR + 3, i, c0.y); asto(M, F_SR + 4, i, c1.y); asto(M, F_SR + 5, i, c2.y);
  asto(M, F_SR + 6, i, c0.z); asto(M, F_SR + 7, i, c1.z); asto(M, F_SR + 8, i, c2.z);
  asto3(M, F_NU, i, pt);                         // joint point
  asto3(M, F_LA, i, fma3(M.geo[i].x, c2, pt));    // tip point
  asto3(M, F_A0, i, J0);                          // axis x
}

template <int NT>
__global__ __launch_bounds__(NT) void k_tip_fk(DevModel M, const float2* q) {
  const int pk = blockIdx.x;
  const int lb = ldc(M.pack_lvl, pk), le = ldc(M.pack_lvl, pk + 1) - 1;
  for (int lv = lb; lv < le; ++lv) {
    const int a = M.lvl_off[lv], b = M.lvl_off[lv + 1];
    for (int i = a + (int)threadIdx.x; i < b; i += NT) node_tip_fk(M, q, i);
    __syncthreads();
  }
}

__global__ void k_tip_gather(DevModel M, int n_tips, const int32_t* node, float* out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_tips; k += gridDim.x * blockDim.x) {
    const V3 p = ald3(M, F_LA, node[k]);
    out[3 * k] = p.x; out[3 * k + 1] = p.y; out[3 * k + 2] = p.z;
  }
}

// seeds: force-like adjoints at the tip points, summed per node by one thread in tip
// order (several tips may share a node; a serial sum keeps the result deterministic)
__global__ void k_tip_seed(DevModel M, int n_tips, const int32_t* node, const float* g) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int k = 0; k < n_tips; ++k) {
    const int i = node[k];
    M.scr[scr_idx(M, F_LPA + 0, i)] += g[3 * k];
    M.scr[scr_idx(M, F_LPA + 1, i)] += g[3 * k + 1];
    M.scr[scr_idx(M, F_LPA + 2, i)] += g[3 * k + 2];
  }
}

__global__ void k_clear_fields(DevModel M, int f0, int nf) {
  const int64_t tot = (int64_t)nf * M.n_seg;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot; k += (int64_t)gridDim.x * blockDim.x)
    M.scr[scr_idx(M, f0 + (int)(k / M.n_seg), (int)(k % M.n_seg))] = 0.f;
}

// up pass: wrench (n, f) of the position adjoints about each joint point; dq_k = a_k . n
__device__ void node_tip_bwd(const DevModel& M, float2* gq, int i) {
  V3 n = v3(0, 0, 0), f = ald3(M, F_LPA, i);  // seed at the tip
  const int cb = M.child[i], ce = cb + M.nchild[i];
  for (int c = cb; c < ce; ++c) { n = n + ald3(M, F_RB, c); f = f + ald3(M, F_RB + 3, c); }
  const V3 lz = ald3(M, F_LA, i) - ald3(M, F_NU, i);
  n = n + cross(lz, f);
  const V3 a0 = ald3(M, F_A0, i);
  const V3 a1 = v3(aldf(M, F_SR + 1, i), aldf(M, F_SR + 4, i), aldf(M, F_SR + 7, i));
  float2 g = gq[i];
  g.x += dot(a0, n);
  g.y += dot(a1, n);
  gq[i] = g;
  asto3(M, F_RB, i, n);
  asto3(M, F_RB + 3, i, f);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_tip_bwd(DevModel M, float2* gq) {
  const int pk = blockIdx.x;
  const int lb = ldc(M.pack_lvl, pk), le = ldc(M.pack_lvl, pk + 1) - 1;
  for (int lv = le - 1; lv >= lb; --lv) {
    const int a = M.lvl_off[lv], b = M.lvl_off[lv + 1];
    for (int i = a + (int)threadIdx.x; i < b; i += NT) node_tip_bwd(M, gq, i);
    __syncthreads();
  }
}

template __global__ void k_adjoint_packs<64>(DevModel, DevState, const float*, DevInputs, DevAdj, int);
template __global__ void k_adjoint_packs<128>(DevModel, DevState, const float*, DevInputs, DevAdj, int);
template __global__ void k_adjoint_packs<256>(DevModel, DevState, const float*, DevInputs, DevAdj, int);
template __global__ void k_adjoint_packs<512>(DevModel, DevState, const float*, DevInputs, DevAdj, int);
template __global__ void k_tip_fk<64>(DevModel, const float2*);
template __global__ void k_tip_fk<128>(DevModel, const float2*);
template __global__ void k_tip_fk<256>(DevModel, const float2*);
template __global__ void k_tip_fk<512>(DevModel, const float2*);
template __global__ void k_tip_bwd<64>(DevModel, float2*);
template __global__ void k_tip_bwd<128>(DevModel, float2*);
template __global__ void k_tip_bwd<256>(DevModel, float2*);
template __global__ void k_tip_bwd<512>(DevModel, float2*);

}  // namespace orchard
