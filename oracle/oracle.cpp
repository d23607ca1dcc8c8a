// FP64 CPU oracle of the batched orchard-tree dynamics step.
//
// TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's
// CPU-baseline leg may load this library.  It shares no code with the HIP path.
//
// What it computes (OrchardBench, Sec. "Physical Model"):
//  * each internode is a rigid capsule link (Sec. "Physical Model", first
//    paragraph), joined to its parent at the parent's tip by a joint whose rest
//    rotation is q_rel (joint-frame equation); the compliant joint has two
//    bending DoF (Sec. "Compliant branch dynamics"), read here as a Hooke joint
//    R_x(theta_x) R_y(theta_y) -- two revolutes sharing one point;
//  * joint stiffness Kp = (pi/4) E r^4 / l (Eq. beam), restoring torque
//    -Kp theta - Kd omega, integrated implicitly;
//  * rupture when Kp |theta| > sigma_r pi r^3 / 4 (Eq. break), with an N-step
//    hysteresis; a broken joint loses its spring and damper (free hinge);
//  * apples: tether f = -k_s (x - x_hang) - c_s v on the apple, the elastic
//    part minus the static weight reacted onto the spur (Sec. "Fruit"), and
//    detachment by pull or by stem tension;
//  * applied body forces with the impulse cap (Sec. "Numerical Stability").
//
// The step itself is the plain definition: the joint accelerations qdd are the
// unique solution of the dense linear system
//     Mt(q) qdd = -Kp (q + h qd) - Kd qd - c(q, qd, f_ext)
//     Mt = H(q) + diag(h Kd + h^2 Kp) + h^2 k_s sum_a s_a J_a^T J_a  (attached apples,
//          s_a the reaction clamp scale)
// with H the joint-space mass matrix assembled by the composite-rigid-body
// method and c the bias of recursive Newton-Euler (textbook forms, world-frame
// spatial vectors), factored by the tree-sparse L^T D L method.  Then
// qd+ = qd + h qdd, q+ = q + h qd+.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

#include "oracle_math.hpp"

namespace orc {

// Global constants of a batch (C layout shared with the Python wrapper).
struct Globals {
  double dt;
  double gravity[3];
  double tether_k, tether_zeta;
  double damping_zeta, damping_cd;  // damping_cd > 0 selects Kd = c_d Kp
  double tension_factor;            // alpha: tension threshold = alpha * f_detach
  double v_cap;                     // impulse cap speed
  double react_max_factor;          // reaction clamp = factor * f_detach
  double event_band;                // epsilon of the band rule
  int32_t n_break, n_pull, n_tension, pad;
  uint64_t rng_seed;
  double wrench_fraction, wrench_sigma;
  // variants (Sec. "Compliant branch dynamics", Sec. "Fruit"): per-level exponential
  // stiffness Kp = k0 gamma^depth when stiffness_k0 > 0; fruit with 3 (translational)
  // or 6 degrees of freedom
  double stiffness_k0, stiffness_gamma;
  int32_t fruit_dof, pad1;
  // extras (Sec. "Compliant branch dynamics", Sec. "Branch breaking", Sec. "Numerical
  // Stability"), all off at 0: velocity-proportional drag F = -c_v m v, tau = -c_w I w,
  // scaled by drag_snapped on a snapped sub-tree; Coulomb friction at a broken joint of
  // friction_base x (its limb's largest weight moment), growing linearly to
  // friction_growth times that over friction_ramp_time, acting as a damper below
  // friction_speed; power fade of applied force along the body's velocity from
  // fade_speed to twice it; speed brake -brake_rate m (|v| - v_cap) above v_cap
  double drag_lin, drag_ang, drag_snapped;
  double friction_base, friction_growth, friction_ramp_time, friction_speed;
  double fade_speed, brake_rate;
};

struct Tree {
  int S = 0, A = 0;
  int seg0 = 0, app0 = 0;  // offsets in the batch arrays
  std::vector<int> parent;
  std::vector<M3<double>> Q;
  std::vector<double> len, rad, mass, It, Ia, kp0, kd0, mmax;
  std::vector<double> wmom;  // largest weight moment of each joint's limb: |g| sum m_b |c_b - p_j| at rest
  // DoF tree (2 per segment): dof 2i = x axis, 2i+1 = y axis
  std::vector<int> dpar, ddepth, roff;
  int nnz = 0;
  std::vector<int> aseg;
  std::vector<V3<double>> ahang;
  std::vector<double> am, aR, afdet, acs, afmax;
};

struct Model {
  Globals g;
  int n_env = 0;
  std::vector<Tree> trees;
};

// --------------------------------------------------------------------------------------
// kinematics, CRBA, RNEA, LTDL
// --------------------------------------------------------------------------------------
template <class T> struct Kin {
  std::vector<M3<T>> R;   // body rotation (world)
  std::vector<V3<T>> p;   // joint point (world)
  std::vector<SV<T>> s;   // 2S joint axes as spatial motion vectors at the origin
  std::vector<RBI<T>> I;  // body inertias
};

template <class T> M3<T> lift(const M3<double>& a) { M3<T> r; for (int i = 0; i < 9; ++i) r.m[i] = T(a.m[i]); return r; }

// Forward kinematics at joint angles q (Sec. "Physical Model": T = (0,0,l_parent) q_rel,
// then the two bending rotations of the compliant joint).
template <class T> void fk(const Tree& t, const T* q, Kin<T>& K) {
  const int S = t.S;
  K.R.assign(S, M3<T>()); K.p.assign(S, V3<T>()); K.s.assign(2 * S, SV<T>()); K.I.assign(S, RBI<T>());
  for (int i = 0; i < S; ++i) {
    const int par = t.parent[i];
    M3<T> Rp = par < 0 ? M3<T>::eye() : K.R[par];
    V3<T> pp = par < 0 ? V3<T>() : K.p[par] + Rp * V3<T>(T(0), T(0), T(t.len[par]));
    M3<T> Jf = Rp * lift<T>(t.Q[i]);
    T cx = cos(q[2 * i]), sx = sin(q[2 * i]), cy = cos(q[2 * i + 1]), sy = sin(q[2 * i + 1]);
    K.R[i] = Jf * rot_x(cx, sx) * rot_y(cy, sy);
    K.p[i] = pp;
    V3<T> a0 = Jf.col(0), a1 = K.R[i].col(1);
    K.s[2 * i] = SV<T>{a0, cross(pp, a0)};
    K.s[2 * i + 1] = SV<T>{a1, cross(pp, a1)};
    RBI<T>& I = K.I[i];
    I.m = T(t.mass[i]);
    I.c = pp + K.R[i] * V3<T>(T(0), T(0), T(0.5 * t.len[i]));
    M3<T> Dg; Dg(0, 0) = T(t.It[i]); Dg(1, 1) = T(t.It[i]); Dg(2, 2) = T(t.Ia[i]);
    I.Ic = K.R[i] * Dg * transpose(K.R[i]);
  }
}

// Recursive Newton-Euler inverse dynamics in world coordinates (each segment's joint
// as two revolutes, the first carrying a massless body): tau = ID(q, qd, qdd) with
// gravity as a base acceleration and external spatial forces fext (per segment, at
// the origin).  vel_out (2S) receives the DoF-body velocities if non-null.
template <class T>
void rnea(const Tree& t, const Kin<T>& K, const T* qd, const T* qdd, const SV<T>* fext,
          const double* gravity, T* tau, SV<T>* vel_out = nullptr) {
  const int n = 2 * t.S;
  std::vector<SV<T>> v(n), a(n), f(n);
  SV<T> abase;
  abase.l = V3<T>(T(-gravity[0]), T(-gravity[1]), T(-gravity[2]));
  for (int k = 0; k < n; ++k) {
    const int kp = t.dpar[k];
    SV<T> vp = kp < 0 ? SV<T>() : v[kp];
    SV<T> ap = kp < 0 ? abase : a[kp];
    v[k] = vp + qd[k] * K.s[k];
    a[k] = ap + qd[k] * crm(v[k], K.s[k]);
    if (qdd) a[k] = a[k] + qdd[k] * K.s[k];
    if (k & 1) {
      const RBI<T>& I = K.I[k >> 1];
      f[k] = rbi_apply(I, a[k]) + crf(v[k], rbi_apply(I, v[k]));
      if (fext) f[k] = f[k] - fext[k >> 1];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    tau[k] = sdot(K.s[k], f[k]);
    if (t.dpar[k] >= 0) f[t.dpar[k]] = f[t.dpar[k]] + f[k];
  }
  if (vel_out) for (int k = 0; k < n; ++k) vel_out[k] = v[k];
}

// Joint-space mass matrix by the composite-rigid-body method, stored by ancestor rows:
// entry (k, j), j ancestor-or-self of k, at roff[k] + ddepth[k] - ddepth[j].
template <class T> void crba(const Tree& t, const Kin<T>& K, std::vector<T>& H) {
  const int S = t.S;
  H.assign(t.nnz, T(0));
  std::vector<S6<T>> Ic(S);
  for (int i = 0; i < S; ++i) Ic[i] = rbi_to_s6(K.I[i]);
  for (int i = S - 1; i >= 0; --i)
    if (t.parent[i] >= 0) Ic[t.parent[i]] = Ic[t.parent[i]] + Ic[i];
  for (int k = 0; k < 2 * S; ++k) {
    SV<T> F = s6_apply(Ic[k >> 1], K.s[k]);
    int j = k;
    while (j >= 0) {
      H[t.roff[k] + t.ddepth[k] - t.ddepth[j]] = sdot(K.s[j], F);
      j = t.dpar[j];
    }
  }
}

template <class T> inline T& hent(const Tree& t, std::vector<T>& H, int k, int j) {
  return H[t.roff[k] + t.ddepth[k] - t.ddepth[j]];
}

// In-place tree-sparse factorisation Mt = L^T D L (leaves first), then solve Mt x = b.
template <class T> void ltdl_factor(const Tree& t, std::vector<T>& H) {
  for (int k = 2 * t.S - 1; k >= 0; --k) {
    int i = t.dpar[k];
    while (i >= 0) {
      T a = hent(t, H, k, i) / hent(t, H, k, k);
      int j = i;
      while (j >= 0) {
        hent(t, H, i, j) = hent(t, H, i, j) - a * hent(t, H, k, j);
        j = t.dpar[j];
      }
      hent(t, H, k, i) = a;
      i = t.dpar[i];
    }
  }
}
template <class T> void ltdl_solve(const Tree& t, std::vector<T>& H, T* x /* in: b, out: x */) {
  const int n = 2 * t.S;
  for (int k = n - 1; k >= 0; --k) {  // L^T y = b
    int i = t.dpar[k];
    while (i >= 0) { x[i] = x[i] - hent(t, H, k, i) * x[k]; i = t.dpar[i]; }
  }
  for (int k = 0; k < n; ++k) x[k] = x[k] / hent(t, H, k, k);  // D z = y
  for (int k = 0; k < n; ++k) {  // L x = z
    int i = t.dpar[k];
    while (i >= 0) { x[k] = x[k] - hent(t, H, k, i) * x[i]; i = t.dpar[i]; }
  }
}

// --------------------------------------------------------------------------------------
// model derivation (capsule mass properties, Eq. beam, Eq. break, damping reading)
// --------------------------------------------------------------------------------------
static bool build_tree(Tree& t, const Globals& g, int S, int A, const int* parent, const double* quat,
                       const double* len, const double* rad, const double* rho, const double* E,
                       const double* mor, const int* aseg, const double* ahang, const double* am,
                       const double* aR, const double* afdet) {
  t.S = S; t.A = A;
  t.parent.assign(parent, parent + S);
  t.Q.resize(S);
  t.len.assign(len, len + S); t.rad.assign(rad, rad + S);
  t.mass.resize(S); t.It.resize(S); t.Ia.resize(S); t.kp0.resize(S); t.kd0.resize(S); t.mmax.resize(S);
  for (int i = 0; i < S; ++i) {
    if (parent[i] >= i || parent[i] < -1) return false;
    if (!(len[i] > 0) || !(rad[i] > 0) || !(rho[i] > 0) || !(E[i] > 0) || !(mor[i] > 0)) return false;
    const double* qq = quat + 4 * i;
    double nq = std::sqrt(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
    if (std::fabs(nq - 1.0) > 1e-6) return false;
    double qn[4] = {qq[0] / nq, qq[1] / nq, qq[2] / nq, qq[3] / nq};
    t.Q[i] = quat_to_mat(qn);
    const double r = rad[i], l = len[i];
    // capsule = cylinder (radius r, length l) + two hemispherical caps
    const double mc = rho[i] * M_PI * r * r * l;
    const double mh = rho[i] * 4.0 / 3.0 * M_PI * r * r * r;
    t.mass[i] = mc + mh;
    t.Ia[i] = mc * r * r / 2.0 + mh * 2.0 * r * r / 5.0;
    t.It[i] = mc * (l * l / 12.0 + r * r / 4.0) + mh * (2.0 * r * r / 5.0 + l * l / 4.0 + 3.0 * l * r / 8.0);
    t.kp0[i] = M_PI / 4.0 * E[i] * r * r * r * r / l;   // Eq. beam
    t.mmax[i] = mor[i] * M_PI * r * r * r / 4.0;        // Eq. break
  }
  if (g.stiffness_k0 > 0) {  // per-level exponential model: each level down scales Kp by gamma
    std::vector<int> depth(S, 0);
    for (int i = 0; i < S; ++i) {
      depth[i] = parent[i] < 0 ? 0 : depth[parent[i]] + 1;
      t.kp0[i] = g.stiffness_k0 * std::pow(g.stiffness_gamma, depth[i]);
    }
  }
  // DoF tree
  t.dpar.resize(2 * S); t.ddepth.resize(2 * S); t.roff.resize(2 * S + 1);
  for (int i = 0; i < S; ++i) {
    t.dpar[2 * i] = parent[i] < 0 ? -1 : 2 * parent[i] + 1;
    t.dpar[2 * i + 1] = 2 * i;
  }
  int off = 0;
  for (int k = 0; k < 2 * S; ++k) {
    t.ddepth[k] = t.dpar[k] < 0 ? 0 : t.ddepth[t.dpar[k]] + 1;
    t.roff[k] = off;
    off += t.ddepth[k] + 1;
  }
  t.roff[2 * S] = off;
  t.nnz = off;
  // damping: Kd = 2 zeta sqrt(Kp J), J = mean rest diagonal of H (no apples), or c_d Kp
  {
    std::vector<double> q0(2 * S, 0.0);
    Kin<double> K;
    fk(t, q0.data(), K);
    std::vector<double> H;
    crba(t, K, H);
    for (int i = 0; i < S; ++i) {
      if (g.damping_cd > 0) { t.kd0[i] = g.damping_cd * t.kp0[i]; continue; }
      double J = 0.5 * (H[t.roff[2 * i]] + H[t.roff[2 * i + 1]]);
      t.kd0[i] = 2.0 * g.damping_zeta * std::sqrt(t.kp0[i] * J);
    }
    // weight moment scale of each joint's limb (the friction reading): every body of
    // the sub-tree at the distance of its centre of mass from the joint point
    const double gn = std::sqrt(g.gravity[0] * g.gravity[0] + g.gravity[1] * g.gravity[1] + g.gravity[2] * g.gravity[2]);
    t.wmom.assign(S, 0.0);
    for (int b = 0; b < S; ++b)
      for (int j = b; j >= 0; j = parent[j]) t.wmom[j] += gn * t.mass[b] * norm(K.I[b].c - K.p[j]);
  }
  t.aseg.assign(aseg, aseg + A);
  t.ahang.resize(A); t.am.assign(am, am + A); t.aR.assign(aR, aR + A); t.afdet.assign(afdet, afdet + A);
  t.acs.resize(A); t.afmax.resize(A);
  for (int a = 0; a < A; ++a) {
    if (aseg[a] < 0 || aseg[a] >= S || !(am[a] > 0) || !(afdet[a] > 0)) return false;
    t.ahang[a] = V3<double>(ahang[3 * a], ahang[3 * a + 1], ahang[3 * a + 2]);
    t.acs[a] = 2.0 * g.tether_zeta * std::sqrt(g.tether_k * am[a]);
    t.afmax[a] = g.react_max_factor * afdet[a];
  }
  return true;
}

// --------------------------------------------------------------------------------------
// the step
// --------------------------------------------------------------------------------------
// Discrete switches of one step (recorded by the forward, replayed by FD / adjoint).
struct Switches {
  std::vector<uint8_t> broken, detached, clamped, capped;
};

struct EventRefs {  // per-env views of the event state arrays
  uint8_t *broken, *cnt, *det, *cntp, *cntt, *det_path;
  int32_t *break_step, *det_step;
  uint32_t* status;
  double* break_ratio = nullptr;  // mu on the step a joint breaks (nullable)
  double* det_ratio = nullptr;    // pi (pull) or tau (tension) on the step an apple detaches
};

struct BandRefs {  // min |ratio-1| and first in-band step, per joint / apple (nullable)
  double *jmin, *amin;
  int32_t *jfirst, *afirst;
};

// Box-Muller normal triple from the counter generator (k = 1..4).
static void rng_normals(uint64_t seed, int env, int64_t step, int seg, double z[3]) {
  double u[4];
  for (int k = 0; k < 4; ++k) u[k] = (rng_u24(seed, (uint64_t)env, (uint64_t)step, (uint64_t)seg, (uint64_t)(k + 1)) + 0.5) / 16777216.0;
  double r0 = std::sqrt(-2.0 * std::log(u[0])), r1 = std::sqrt(-2.0 * std::log(u[2]));
  z[0] = r0 * std::cos(2.0 * M_PI * u[1]);
  z[1] = r0 * std::sin(2.0 * M_PI * u[1]);
  z[2] = r1 * std::cos(2.0 * M_PI * u[3]);
}

// One step of one tree.  In/out state arrays are tree-local (q, qd: 2S; apple x, v: 3A,
// quat 4A, w 3A).  wrench: [S][6] (force, torque; world, at the COM) or null.  aforce:
// [A][3] or null.  When `replay` is set, the discrete switches come from it instead of
// the event tests; when `rec` is set, the switches used are stored there.
template <class T>
void step_tree(const Tree& t, const Globals& g, int env, int64_t n,
               const T* q, const T* qd, const T* ax, const T* av, const T* aq, const T* aw,
               const T* kp, const T* kd, const double* wrench, const T* aforce,
               T* qo, T* qdo, T* axo, T* avo, T* aqo, T* awo,
               EventRefs* ev, BandRefs* band, Switches* rec, const Switches* replay) {
  const int S = t.S, A = t.A, n2 = 2 * S;
  const double h = g.dt, ks = g.tether_k;
  Kin<T> K;
  fk(t, q, K);
  std::vector<SV<T>> vel(n2);
  for (int k = 0; k < n2; ++k) vel[k] = (t.dpar[k] < 0 ? SV<T>() : vel[t.dpar[k]]) + qd[k] * K.s[k];

  std::vector<uint8_t> broken(S), det(A), clamped(A, 0), capped(S, 0);
  // --- event tests on the state at the start of the step (Eq. break; Sec. "Fruit") ---
  for (int i = 0; i < S; ++i) broken[i] = ev ? ev->broken[i] : 0;
  for (int a = 0; a < A; ++a) det[a] = ev ? ev->det[a] : 0;
  const std::vector<uint8_t> det0(det);  // detached before this step
  // Apple position state: while attached, sigma = (x - x_hang) + h v after the
  // previous step's update, so the stretch at this step is s = sigma - h v_hang, with
  // v_hang the hang point's velocity now (the hang point moved by h v_hang during the
  // previous step); once detached, the absolute position.
  std::vector<V3<T>> xh(A), vh(A), sa(A);
  for (int a = 0; a < A; ++a) {
    const int b = t.aseg[a];
    V3<T> hb = K.R[b] * V3<T>(T(t.ahang[a].x), T(t.ahang[a].y), T(t.ahang[a].z));
    xh[a] = K.p[b] + hb;
    const SV<T>& vb = vel[2 * b + 1];
    vh[a] = vb.l + cross(vb.a, xh[a]);
    V3<T> sig(ax[3 * a], ax[3 * a + 1], ax[3 * a + 2]);
    sa[a] = det0[a] ? sig - xh[a] : sig - h * vh[a];
  }
  if (replay) {
    broken = replay->broken;
    det = replay->detached;
  } else if (ev) {
    for (int i = 0; i < S; ++i) {
      if (broken[i]) continue;
      double th = std::sqrt(val(q[2 * i]) * val(q[2 * i]) + val(q[2 * i + 1]) * val(q[2 * i + 1]));
      double mu = val(kp[i]) * th / t.mmax[i];
      if (band) {
        double d = std::fabs(mu - 1.0);
        band->jmin[i] = std::min(band->jmin[i], d);
        if (d < g.event_band && band->jfirst[i] < 0) band->jfirst[i] = (int32_t)n;
      }
      int c = mu > 1.0 ? ev->cnt[i] + 1 : 0;
      ev->cnt[i] = (uint8_t)std::min(c, 255);
      if (c >= g.n_break) {
        broken[i] = 1; ev->broken[i] = 1; ev->break_step[i] = (int32_t)n;
        if (ev->break_ratio) ev->break_ratio[i] = mu;
      }
    }
    for (int a = 0; a < A; ++a) {
      if (det[a]) continue;
      double F2 = 0.0, d2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        double f = aforce ? val(aforce[3 * a + c]) : 0.0;
        double d = val(sa[a][c]);
        F2 += f * f; d2 += d * d;
      }
      double pi = std::sqrt(F2) / t.afdet[a];
      double tau = ks * std::sqrt(d2) / (g.tension_factor * t.afdet[a]);
      if (band) {
        double d = std::min(std::fabs(pi - 1.0), std::fabs(tau - 1.0));
        band->amin[a] = std::min(band->amin[a], d);
        if (d < g.event_band && band->afirst[a] < 0) band->afirst[a] = (int32_t)n;
      }
      int cp = pi > 1.0 ? ev->cntp[a] + 1 : 0;
      int ct = tau > 1.0 ? ev->cntt[a] + 1 : 0;
      ev->cntp[a] = (uint8_t)std::min(cp, 255);
      ev->cntt[a] = (uint8_t)std::min(ct, 255);
      int path = cp >= g.n_pull ? 1 : (ct >= g.n_tension ? 2 : 0);  // pull wins ties
      if (path) {
        det[a] = 1; ev->det[a] = 1; ev->det_step[a] = (int32_t)n; ev->det_path[a] = (uint8_t)path;
        if (ev->det_ratio) ev->det_ratio[a] = path == 1 ? pi : tau;
      }
    }
  }
  // --- snapped mask (root to leaf) ---
  std::vector<uint8_t> snapped(S);
  for (int i = 0; i < S; ++i) snapped[i] = broken[i] || (t.parent[i] >= 0 && snapped[t.parent[i]]);

  // --- applied forces ---
  std::vector<SV<T>> fext(S);
  const bool use_rng = g.wrench_fraction > 0.0;
  const uint32_t sel_thr = (uint32_t)std::floor(g.wrench_fraction * 16777216.0);
  const bool drag = g.drag_lin > 0 || g.drag_ang > 0;
  const bool rails = g.fade_speed > 0 || g.brake_rate > 0;
  for (int i = 0; i < S; ++i) {
    // the body's centre-of-mass velocity and angular velocity at the start of the step
    const SV<T>& vb = vel[2 * i + 1];
    const V3<T> vc = vb.l + cross(vb.a, K.I[i].c);
    if (drag) {  // velocity-proportional drag, reduced (not removed) on a snapped sub-tree
      const double f = snapped[i] ? g.drag_snapped : 1.0;
      const V3<T> Fd = (-f * g.drag_lin * t.mass[i]) * vc;
      const V3<T> Td = (-f * g.drag_ang) * (K.I[i].Ic * vb.a);
      fext[i] = fext[i] + SV<T>{Td + cross(K.I[i].c, Fd), Fd};
    }
    if (snapped[i]) continue;  // applied forces disabled on a snapped sub-tree
    double F[3] = {0, 0, 0}, Tq[3] = {0, 0, 0};
    bool any = false;
    if (wrench) { for (int c = 0; c < 3; ++c) { F[c] += wrench[6 * i + c]; Tq[c] += wrench[6 * i + 3 + c]; } any = true; }
    if (use_rng && rng_u24(g.rng_seed, (uint64_t)env, (uint64_t)n, (uint64_t)i, 0) < sel_thr) {
      double z[3];
      rng_normals(g.rng_seed, env, n, i, z);
      for (int c = 0; c < 3; ++c) F[c] += g.wrench_sigma * z[c];
      any = true;
    }
    if (!any) continue;
    V3<T> Fv = V3<T>(T(F[0]), T(F[1]), T(F[2]));
    if (rails) {
      const T sp = norm(vc);
      if (val(sp) > 0) {
        const V3<T> u = (T(1) / sp) * vc;
        // power fade: the part of the force along the velocity, when it pushes the body
        // on, falls linearly from full at fade_speed to nothing at twice that speed
        const T fu = dot(Fv, u);
        if (g.fade_speed > 0 && val(fu) > 0 && val(sp) > g.fade_speed) {
          T phi = T(1) - (sp - g.fade_speed) / g.fade_speed;
          if (val(phi) < 0) phi = T(0);
          Fv = Fv - ((T(1) - phi) * fu) * u;
        }
        // soft speed brake above the speed limit
        if (g.brake_rate > 0 && val(sp) > g.v_cap) Fv = Fv - (g.brake_rate * t.mass[i] * (sp - g.v_cap)) * u;
      }
    }
    // impulse cap: one step of the force may not raise the body speed above v_cap
    const T nF = norm(Fv);
    const double cap = t.mass[i] * g.v_cap / h;
    bool cp = replay ? replay->capped[i] : (val(nF) > cap);
    if (cp) { Fv = (T(cap) / nF) * Fv; capped[i] = 1; }
    V3<T> Tv = V3<T>(T(Tq[0]), T(Tq[1]), T(Tq[2]));
    fext[i] = fext[i] + SV<T>{Tv + cross(K.I[i].c, Fv), Fv};
  }
  // --- apple reactions on the spur (Sec. "Fruit"): the elastic tether force minus the
  // static weight, with the hang point taken at the end of the step to first order
  // (linearly implicit: explicit part below, h^2 k_s J^T J in the matrix).  The clamp
  // scales the whole reaction, explicit part and implicit term alike, by
  // s = min(1, F_max / |f|), so the force stays continuous across the threshold ---
  std::vector<V3<T>> fh(A);
  std::vector<T> rs(A, T(0));
  for (int a = 0; a < A; ++a) {
    if (det[a]) continue;
    V3<T> gw(T(g.gravity[0]), T(g.gravity[1]), T(g.gravity[2]));
    V3<T> f = ks * (sa[a] - h * vh[a]) - t.am[a] * gw;
    T nf = norm(f);
    bool cl = replay ? replay->clamped[a] : (val(nf) > t.afmax[a]);
    T sc = cl ? T(t.afmax[a]) / nf : T(1);
    if (cl) clamped[a] = 1;
    rs[a] = sc;
    f = sc * f;
    fh[a] = f;
    fext[t.aseg[a]] = fext[t.aseg[a]] + SV<T>{cross(xh[a], f), f};
  }
  // --- bias, matrix, solve ---
  std::vector<T> c(n2), zero(n2, T(0));
  rnea(t, K, qd, zero.data(), fext.data(), g.gravity, c.data());
  std::vector<T> H;
  crba(t, K, H);
  std::vector<T> rhs(n2);
  for (int i = 0; i < S; ++i) {
    T kpe = broken[i] ? T(0) : kp[i];
    T kde = broken[i] ? T(0) : kd[i];
    if (broken[i] && g.friction_base > 0 && ev && ev->break_step[i] >= 0) {
      // Coulomb friction of the torn fibres, ramped from friction_base to
      // friction_growth x friction_base of the limb's weight moment over the ramp time,
      // as a linearly implicit damper tau_c / max(|theta'|, friction_speed): it brakes
      // the hinge toward rest and never reverses it within a step
      const double ts = (double)(n - ev->break_step[i]) * h;
      const double ramp = g.friction_ramp_time > 0 ? std::min(1.0, ts / g.friction_ramp_time) : 1.0;
      const double tc = g.friction_base * t.wmom[i] * (1.0 + (g.friction_growth - 1.0) * ramp);
      const T w = sqrt(qd[2 * i] * qd[2 * i] + qd[2 * i + 1] * qd[2 * i + 1]);
      kde = val(w) > g.friction_speed ? T(tc) / w : T(tc / g.friction_speed);
    }
    for (int d = 0; d < 2; ++d) {
      const int k = 2 * i + d;
      hent(t, H, k, k) = hent(t, H, k, k) + h * kde + h * h * kpe;
      rhs[k] = -kpe * (q[k] + h * qd[k]) - kde * qd[k] - c[k];
    }
  }
  for (int a = 0; a < A; ++a) {  // virtual point mass s h^2 k_s at the hang point
    if (det[a]) continue;
    const T mv = (h * h * ks) * rs[a];
    std::vector<int> anc;
    for (int j = 2 * t.aseg[a] + 1; j >= 0; j = t.dpar[j]) anc.push_back(j);
    std::vector<V3<T>> col(anc.size());
    for (size_t u = 0; u < anc.size(); ++u) col[u] = K.s[anc[u]].l + cross(K.s[anc[u]].a, xh[a]);
    for (size_t u = 0; u < anc.size(); ++u)
      for (size_t w = u; w < anc.size(); ++w)
        hent(t, H, anc[u], anc[w]) = hent(t, H, anc[u], anc[w]) + mv * dot(col[u], col[w]);
  }
  ltdl_factor(t, H);
  std::vector<T> qdd(rhs);
  ltdl_solve(t, H, qdd.data());
  bool finite = true;
  for (int k = 0; k < n2; ++k) {
    qdo[k] = qd[k] + h * qdd[k];
    qo[k] = q[k] + h * qdo[k];
    finite = finite && std::isfinite(val(qo[k])) && std::isfinite(val(qdo[k]));
  }
  // --- apples (explicit, symplectic Euler) ---
  for (int a = 0; a < A; ++a) {
    V3<T> v(av[3 * a], av[3 * a + 1], av[3 * a + 2]);
    V3<T> gw(T(g.gravity[0]), T(g.gravity[1]), T(g.gravity[2]));
    V3<T> f = t.am[a] * gw;
    if (aforce) f += V3<T>(aforce[3 * a], aforce[3 * a + 1], aforce[3 * a + 2]);
    if (!det[a]) f += -ks * sa[a] - t.acs[a] * v;
    V3<T> vn = v + (h / t.am[a]) * f;
    // attached: sigma+ = s + h v+;  detached: absolute x+ = x + h v+ (x = x_hang + s if it
    // detached at this step)
    V3<T> base = det[a] ? (det0[a] ? V3<T>(ax[3 * a], ax[3 * a + 1], ax[3 * a + 2]) : xh[a] + sa[a]) : sa[a];
    V3<T> xn = base + h * vn;
    for (int cc = 0; cc < 3; ++cc) { avo[3 * a + cc] = vn[cc]; axo[3 * a + cc] = xn[cc]; awo[3 * a + cc] = aw[3 * a + cc]; }
    if (g.fruit_dof == 3) {  // translational fruit: no orientation state to advance
      for (int cc = 0; cc < 4; ++cc) aqo[4 * a + cc] = aq[4 * a + cc];
      for (int cc = 0; cc < 3; ++cc) finite = finite && std::isfinite(val(axo[3 * a + cc])) && std::isfinite(val(avo[3 * a + cc]));
      continue;
    }
    // quat+ = normalize(exp(h w / 2) * quat)
    V3<T> hw = (0.5 * h) * V3<T>(aw[3 * a], aw[3 * a + 1], aw[3 * a + 2]);
    double th = val(norm(hw));
    T ew = T(1), ex = T(0), ey = T(0), ez = T(0);
    if (th > 0) {
      T nt = norm(hw);
      T sc = sin(nt) / nt;
      ew = cos(nt); ex = sc * hw.x; ey = sc * hw.y; ez = sc * hw.z;
    }
    const T* qq = aq + 4 * a;
    T w = ew * qq[0] - ex * qq[1] - ey * qq[2] - ez * qq[3];
    T xx = ew * qq[1] + ex * qq[0] + ey * qq[3] - ez * qq[2];
    T yy = ew * qq[2] - ex * qq[3] + ey * qq[0] + ez * qq[1];
    T zz = ew * qq[3] + ex * qq[2] - ey * qq[1] + ez * qq[0];
    T nq = sqrt(w * w + xx * xx + yy * yy + zz * zz);
    aqo[4 * a] = w / nq; aqo[4 * a + 1] = xx / nq; aqo[4 * a + 2] = yy / nq; aqo[4 * a + 3] = zz / nq;
    for (int cc = 0; cc < 3; ++cc) finite = finite && std::isfinite(val(axo[3 * a + cc])) && std::isfinite(val(avo[3 * a + cc]));
  }
  if (!finite && ev) *ev->status |= 1u;
  if (rec) { rec->broken = broken; rec->detached = det; rec->clamped = clamped; rec->capped = capped; }
}

}  // namespace orc

// ======================================================================================
// C interface (ctypes)
// ======================================================================================
using namespace orc;

extern "C" {

struct OracleDesc {
  int32_t n_env;
  const int32_t* seg_offset;
  const int32_t* seg_parent;
  const double* seg_rest_quat;
  const double *seg_length, *seg_radius, *seg_density, *seg_youngs, *seg_mor;
  const int32_t *apple_offset, *apple_seg;
  const double* apple_hang;
  const double *apple_mass, *apple_radius, *apple_detach;
};

// Batch state (flat, descriptor order) and inputs for oracle_rollout.
struct OracleIO {
  double *q, *qd;                 // [S_tot][2]
  double *ax, *av, *aq, *aw;      // [A_tot][3], [3], [4], [3]
  uint8_t *broken, *cnt, *det, *cntp, *cntt, *det_path;
  int32_t *break_step, *det_step;
  uint32_t* status;               // [n_env]
  const double *kp, *kd;          // [S_tot]
  const double* wrench;           // [S_tot][6] per step (stride below) or null
  int64_t wrench_stride;          // doubles between steps
  const double* aforce;           // [A_tot][3] per step or null
  int64_t aforce_stride;          // doubles between steps; 0 = constant
  double *band_jmin, *band_amin;  // nullable
  int32_t *band_jfirst, *band_afirst;
  double *break_ratio, *det_ratio;  // [S_tot], [A_tot]: threshold ratio at the event; nullable
};

void* oracle_create(const OracleDesc* d, const Globals* g) {
  Model* M = new Model();
  M->g = *g;
  M->n_env = d->n_env;
  M->trees.resize(d->n_env);
  for (int e = 0; e < d->n_env; ++e) {
    const int s0 = d->seg_offset[e], s1 = d->seg_offset[e + 1];
    const int a0 = d->apple_offset[e], a1 = d->apple_offset[e + 1];
    Tree& t = M->trees[e];
    t.seg0 = s0; t.app0 = a0;
    if (!build_tree(t, *g, s1 - s0, a1 - a0, d->seg_parent + s0, d->seg_rest_quat + 4 * s0,
                    d->seg_length + s0, d->seg_radius + s0, d->seg_density + s0, d->seg_youngs + s0,
                    d->seg_mor + s0, d->apple_seg + a0, d->apple_hang + 3 * a0, d->apple_mass + a0,
                    d->apple_radius + a0, d->apple_detach + a0)) {
      delete M;
      return nullptr;
    }
  }
  return M;
}

void oracle_destroy(void* m) { delete static_cast<Model*>(m); }

// derived per-segment parameters (descriptor order): mass, It, Ia, kp, kd, mmax
void oracle_derived(void* m, double* mass, double* It, double* Ia, double* kp, double* kd, double* mmax,
                    double* apple_cs) {
  Model* M = static_cast<Model*>(m);
  for (const Tree& t : M->trees) {
    for (int i = 0; i < t.S; ++i) {
      mass[t.seg0 + i] = t.mass[i]; It[t.seg0 + i] = t.It[i]; Ia[t.seg0 + i] = t.Ia[i];
      kp[t.seg0 + i] = t.kp0[i]; kd[t.seg0 + i] = t.kd0[i]; mmax[t.seg0 + i] = t.mmax[i];
    }
    for (int a = 0; a < t.A; ++a) apple_cs[t.app0 + a] = t.acs[a];
  }
}

// forward kinematics of one env: R [S][9] row major, p [S][3] joint points
void oracle_fk(void* m, int env, const double* q, double* R, double* p) {
  Model* M = static_cast<Model*>(m);
  const Tree& t = M->trees[env];
  Kin<double> K;
  fk(t, q, K);
  for (int i = 0; i < t.S; ++i) {
    for (int c = 0; c < 9; ++c) R[9 * i + c] = K.R[i].m[c];
    for (int c = 0; c < 3; ++c) p[3 * i + c] = K.p[i][c];
  }
}

// dense joint-space mass matrix H(q) [2S][2S]
void oracle_mass_matrix(void* m, int env, const double* q, double* Hd) {
  Model* M = static_cast<Model*>(m);
  const Tree& t = M->trees[env];
  Kin<double> K;
  fk(t, q, K);
  std::vector<double> H;
  crba(t, K, H);
  const int n = 2 * t.S;
  std::memset(Hd, 0, sizeof(double) * n * n);
  for (int k = 0; k < n; ++k)
    for (int j = k; j >= 0; j = t.dpar[j]) {
      double v = H[t.roff[k] + t.ddepth[k] - t.ddepth[j]];
      Hd[k * n + j] = v; Hd[j * n + k] = v;
    }
}

// inverse dynamics tau = ID(q, qd, qdd) with gravity (optionally off) and external
// wrenches [S][6] (force, torque about the COM; world) or null
void oracle_inverse_dynamics(void* m, int env, const double* q, const double* qd, const double* qdd,
                             const double* wrench, int gravity_on, double* tau) {
  Model* M = static_cast<Model*>(m);
  const Tree& t = M->trees[env];
  Kin<double> K;
  fk(t, q, K);
  std::vector<SV<double>> fext(t.S);
  if (wrench)
    for (int i = 0; i < t.S; ++i) {
      V3<double> F(wrench[6 * i], wrench[6 * i + 1], wrench[6 * i + 2]);
      V3<double> Tq(wrench[6 * i + 3], wrench[6 * i + 4], wrench[6 * i + 5]);
      fext[i] = SV<double>{Tq + cross(K.I[i].c, F), F};
    }
  const double g0[3] = {0, 0, 0};
  rnea(t, K, qd, qdd, fext.data(), gravity_on ? M->g.gravity : g0, tau);
}

// solve (H(q) + diag(dg)) x = b with the tree-sparse factorisation
void oracle_ltdl_solve(void* m, int env, const double* q, const double* dg, const double* b, double* x) {
  Model* M = static_cast<Model*>(m);
  const Tree& t = M->trees[env];
  Kin<double> K;
  fk(t, q, K);
  std::vector<double> H;
  crba(t, K, H);
  for (int k = 0; k < 2 * t.S; ++k) hent(t, H, k, k) += dg[k];
  ltdl_factor(t, H);
  for (int k = 0; k < 2 * t.S; ++k) x[k] = b[k];
  ltdl_solve(t, H, x);
}

// rest state: q = qd = 0, apples hanging m g / k_s below the hang point, at rest
// (apple position state = stretch from the hang point while attached)
void oracle_rest_state(void* m, const OracleIO* io) {
  Model* M = static_cast<Model*>(m);
  const Globals& g = M->g;
  for (const Tree& t : M->trees) {
    std::vector<double> q0(2 * t.S, 0.0);
    Kin<double> K;
    fk(t, q0.data(), K);
    for (int k = 0; k < 2 * t.S; ++k) { io->q[2 * t.seg0 + k] = 0.0; io->qd[2 * t.seg0 + k] = 0.0; }
    for (int a = 0; a < t.A; ++a) {
      const int b = t.aseg[a], ga = t.app0 + a;
      for (int c = 0; c < 3; ++c) {
        io->ax[3 * ga + c] = t.am[a] * g.gravity[c] / g.tether_k;  // stretch at rest
        io->av[3 * ga + c] = 0.0;
        io->aw[3 * ga + c] = 0.0;
      }
      io->aq[4 * ga] = 1.0; io->aq[4 * ga + 1] = io->aq[4 * ga + 2] = io->aq[4 * ga + 3] = 0.0;
    }
  }
}

uint32_t oracle_rng_u24(uint64_t seed, uint64_t env, uint64_t step, uint64_t seg, uint64_t k) {
  return rng_u24(seed, env, step, seg, k);
}
uint64_t oracle_splitmix64(uint64_t x) { return splitmix64(x); }

// Roll the listed envs forward n_steps from step index step0 (state in/out).
// Threads: one env at a time per worker.  Returns 0.
int oracle_rollout(void* m, const OracleIO* io, int n_sel, const int32_t* env_list, int64_t step0,
                   int n_steps, int n_threads) {
  Model* M = static_cast<Model*>(m);
  std::atomic<int> next(0);
  auto work = [&]() {
    for (;;) {
      int u = next.fetch_add(1);
      if (u >= n_sel) break;
      const int e = env_list[u];
      const Tree& t = M->trees[e];
      const int S = t.S, A = t.A, s0 = t.seg0, a0 = t.app0;
      std::vector<double> qn(2 * S), qdn(2 * S), axn(3 * A), avn(3 * A), aqn(4 * A), awn(3 * A);
      EventRefs ev{io->broken + s0, io->cnt + s0, io->det + a0, io->cntp + a0, io->cntt + a0,
                   io->det_path + a0, io->break_step + s0, io->det_step + a0, io->status + e,
                   io->break_ratio ? io->break_ratio + s0 : nullptr, io->det_ratio ? io->det_ratio + a0 : nullptr};
      BandRefs band{io->band_jmin ? io->band_jmin + s0 : nullptr, io->band_amin ? io->band_amin + a0 : nullptr,
                    io->band_jfirst ? io->band_jfirst + s0 : nullptr, io->band_afirst ? io->band_afirst + a0 : nullptr};
      double *q = io->q + 2 * s0, *qd = io->qd + 2 * s0, *ax = io->ax + 3 * a0, *av = io->av + 3 * a0,
             *aq = io->aq + 4 * a0, *aw = io->aw + 3 * a0;
      for (int s = 0; s < n_steps; ++s) {
        if (*ev.status) break;  // frozen after a non-finite step
        const int64_t n = step0 + s;
        const double* wr = io->wrench ? io->wrench + (int64_t)s * io->wrench_stride + 6 * s0 : nullptr;
        const double* af = io->aforce ? io->aforce + (int64_t)s * io->aforce_stride + 3 * a0 : nullptr;
        step_tree<double>(t, M->g, e, n, q, qd, ax, av, aq, aw, io->kp + s0, io->kd + s0, wr, af,
                          qn.data(), qdn.data(), axn.data(), avn.data(), aqn.data(), awn.data(), &ev,
                          io->band_jmin ? &band : nullptr, nullptr, nullptr);
        std::copy(qn.begin(), qn.end(), q); std::copy(qdn.begin(), qdn.end(), qd);
        std::copy(axn.begin(), axn.end(), ax); std::copy(avn.begin(), avn.end(), av);
        std::copy(aqn.begin(), aqn.end(), aq); std::copy(awn.begin(), awn.end(), aw);
      }
    }
  };
  if (n_threads <= 1) work();
  else {
    std::vector<std::thread> th;
    for (int i = 0; i < n_threads; ++i) th.emplace_back(work);
    for (auto& x : th) x.join();
  }
  return 0;
}

}  // extern "C"

// ======================================================================================
// Adjoint (FP64, reverse mode by taping the step itself; discrete switches frozen)
// ======================================================================================
#include "tape.hpp"

namespace orc {

// per-step record: switches used plus the detached flags at entry
struct StepRecord {
  Switches sw;
  std::vector<uint8_t> det0, broken0;
};

struct EnvRun {
  const Tree& t;
  const Globals& g;
  int env;
  int64_t step0;
  int n_steps;
};

// Tip positions p_b + R_b (0, 0, l_b) of the listed segments.
template <class T>
void tips(const Tree& t, const T* q, int n_tips, const int32_t* seg, V3<T>* out) {
  Kin<T> K;
  fk(t, q, K);
  for (int k = 0; k < n_tips; ++k) {
    const int b = seg[k];
    out[k] = K.p[b] + K.R[b] * V3<T>(T(0), T(0), T(t.len[b]));
  }
}

// Forward rollout of one tree in double, recording every state and switch.
static void forward_record(const EnvRun& r, const double* q0, const double* qd0, const double* ax0, const double* av0,
                           const double* kp, const double* kd, const double* F, std::vector<std::vector<double>>& states,
                           std::vector<StepRecord>* rec, const std::vector<StepRecord>* replay) {
  const Tree& t = r.t;
  const int S = t.S, A = t.A;
  std::vector<double> q(q0, q0 + 2 * S), qd(qd0, qd0 + 2 * S), ax(ax0, ax0 + 3 * A), av(av0, av0 + 3 * A);
  std::vector<double> aq(4 * A, 0.0), aw(3 * A, 0.0);
  for (int a = 0; a < A; ++a) aq[4 * a] = 1.0;
  std::vector<uint8_t> broken(S, 0), cnt(S, 0), det(A, 0), cntp(A, 0), cntt(A, 0), path(A, 0);
  std::vector<int32_t> bstep(S, -1), dstep(A, -1);
  uint32_t status = 0;
  std::vector<double> qn(2 * S), qdn(2 * S), axn(3 * A), avn(3 * A), aqn(4 * A), awn(3 * A);
  states.assign(r.n_steps + 1, {});
  auto pack = [&](std::vector<double>& s) {
    s.clear();
    s.insert(s.end(), q.begin(), q.end()); s.insert(s.end(), qd.begin(), qd.end());
    s.insert(s.end(), ax.begin(), ax.end()); s.insert(s.end(), av.begin(), av.end());
  };
  pack(states[0]);
  if (rec) rec->assign(r.n_steps, {});
  for (int s = 0; s < r.n_steps; ++s) {
    if (rec) { (*rec)[s].det0 = det; (*rec)[s].broken0 = broken; }
    Switches sw;
    const Switches* rp = nullptr;
    if (replay) { det = (*replay)[s].det0; broken = (*replay)[s].broken0; rp = &(*replay)[s].sw; }
    EventRefs ev{broken.data(), cnt.data(), det.data(), cntp.data(), cntt.data(), path.data(), bstep.data(), dstep.data(), &status};
    step_tree<double>(t, r.g, r.env, r.step0 + s, q.data(), qd.data(), ax.data(), av.data(), aq.data(), aw.data(), kp, kd,
                      nullptr, F ? F + (int64_t)s * 3 * A : nullptr, qn.data(), qdn.data(), axn.data(), avn.data(),
                      aqn.data(), awn.data(), &ev, nullptr, &sw, rp);
    if (replay) { broken = rp->broken; det = rp->detached; }
    if (rec) (*rec)[s].sw = sw;
    q = qn; qd = qdn; ax = axn; av = avn; aq = aqn; aw = awn;
    pack(states[s + 1]);
  }
}

static double loss_of(const Tree& t, const double* q, int n_tips, const int32_t* seg, const double* target) {
  std::vector<V3<double>> tp(n_tips);
  tips(t, q, n_tips, seg, tp.data());
  double L = 0;
  for (int k = 0; k < n_tips; ++k)
    for (int c = 0; c < 3; ++c) { const double d = tp[k][c] - target[3 * k + c]; L += d * d; }
  return L;
}

}  // namespace orc

extern "C" {

// Opaque record of a forward run's switches (for replay in finite differences).
void* oracle_record_new(void) { return new std::vector<StepRecord>(); }
void oracle_record_free(void* r) { delete static_cast<std::vector<StepRecord>*>(r); }

// Loss L = sum_k |tip_k(q_T) - target_k|^2 after n_steps from the given state (flags
// zero at start).  If rec_in is non-null the switches are replayed from it; if rec_out
// is non-null they are recorded there.  F: [n_steps][A][3] apple forces or null.
// w_state (nullable, [4S + 6A]): adds the linear term w_state . S_T of the final state
// (q, qd, apple position state, apple velocity) to the loss.
double oracle_loss(void* m, int env, int64_t step0, int n_steps, const double* q0, const double* qd0,
                   const double* ax0, const double* av0, const double* kp, const double* kd, const double* F,
                   int n_tips, const int32_t* tip_seg, const double* target, const double* w_state, void* rec_in,
                   void* rec_out, double* q_final) {
  Model* M = static_cast<Model*>(m);
  const Tree& t = M->trees[env];
  EnvRun r{t, M->g, env, step0, n_steps};
  std::vector<std::vector<double>> states;
  forward_record(r, q0, qd0, ax0, av0, kp, kd, F, states, static_cast<std::vector<StepRecord>*>(rec_out),
                 static_cast<std::vector<StepRecord>*>(rec_in));
  const std::vector<double>& last = states.back();
  if (q_final) std::copy(last.begin(), last.begin() + 4 * t.S, q_final);
  double L = loss_of(t, last.data(), n_tips, tip_seg, target);
  if (w_state)
    for (size_t k = 0; k < last.size(); ++k) L += w_state[k] * last[k];
  return L;
}

// Gradient of the loss above with the forward's switches frozen.  Outputs (accumulated
// into zero-initialised arrays): g_kp, g_kd [S], g_F [n_steps][A][3] (nullable),
// g_state0 [4S + 6A] = (q, qd, apple position state, apple velocity) (nullable).
double oracle_adjoint(void* m, int env, int64_t step0, int n_steps, const double* q0, const double* qd0,
                      const double* ax0, const double* av0, const double* kp, const double* kd, const double* F,
                      int n_tips, const int32_t* tip_seg, const double* target, const double* w_state, double* g_kp,
                      double* g_kd, double* g_F, double* g_state0) {
  Model* M = static_cast<Model*>(m);
  const Tree& t = M->trees[env];
  const int S = t.S, A = t.A, NX = 4 * S + 6 * A;
  EnvRun r{t, M->g, env, step0, n_steps};
  std::vector<std::vector<double>> states;
  std::vector<StepRecord> rec;
  forward_record(r, q0, qd0, ax0, av0, kp, kd, F, states, &rec, nullptr);
  Tape tp;
  tape() = &tp;
  // loss seed
  std::vector<double> xbar(NX, 0.0);
  double L;
  {
    std::vector<AD> q(2 * S);
    for (int k = 0; k < 2 * S; ++k) q[k] = AD::var(states.back()[k]);
    std::vector<V3<AD>> tips_ad(n_tips);
    tips(t, q.data(), n_tips, tip_seg, tips_ad.data());
    AD Ls(0.0);
    for (int k = 0; k < n_tips; ++k)
      for (int c = 0; c < 3; ++c) { AD d = tips_ad[k][c] - target[3 * k + c]; Ls = Ls + d * d; }
    L = Ls.v;
    tp.adj.assign(tp.nodes.size(), 0.0);
    if (Ls.i >= 0) tp.adj[Ls.i] = 1.0;
    tp.reverse();
    for (int k = 0; k < 2 * S; ++k) xbar[k] = tp.adj[q[k].i];
    tp.clear();
    if (w_state)
      for (int k = 0; k < NX; ++k) { xbar[k] += w_state[k]; L += w_state[k] * states.back()[k]; }
  }
  for (int s = n_steps - 1; s >= 0; --s) {
    const std::vector<double>& x = states[s];
    std::vector<AD> q(2 * S), qd(2 * S), ax(3 * A), av(3 * A), aq(4 * A), aw(3 * A, AD(0.0)), kpa(S), kda(S), Fa(F ? 3 * A : 0);
    for (int k = 0; k < 2 * S; ++k) { q[k] = AD::var(x[k]); qd[k] = AD::var(x[2 * S + k]); }
    for (int k = 0; k < 3 * A; ++k) { ax[k] = AD::var(x[4 * S + k]); av[k] = AD::var(x[4 * S + 3 * A + k]); }
    for (int a = 0; a < A; ++a) { aq[4 * a] = AD(1.0); aq[4 * a + 1] = aq[4 * a + 2] = aq[4 * a + 3] = AD(0.0); }
    for (int i = 0; i < S; ++i) { kpa[i] = AD::var(kp[i]); kda[i] = AD::var(kd[i]); }
    for (int k = 0; k < (int)Fa.size(); ++k) Fa[k] = AD::var(F[(int64_t)s * 3 * A + k]);
    std::vector<AD> qn(2 * S), qdn(2 * S), axn(3 * A), avn(3 * A), aqn(4 * A), awn(3 * A);
    std::vector<uint8_t> broken = rec[s].broken0, cnt(S, 0), det = rec[s].det0, cntp(A, 0), cntt(A, 0), path(A, 0);
    std::vector<int32_t> bstep(S, -1), dstep(A, -1);
    uint32_t status = 0;
    EventRefs ev{broken.data(), cnt.data(), det.data(), cntp.data(), cntt.data(), path.data(), bstep.data(), dstep.data(), &status};
    step_tree<AD>(t, M->g, env, step0 + s, q.data(), qd.data(), ax.data(), av.data(), aq.data(), aw.data(), kpa.data(),
                  kda.data(), nullptr, F ? Fa.data() : nullptr, qn.data(), qdn.data(), axn.data(), avn.data(), aqn.data(),
                  awn.data(), &ev, nullptr, nullptr, &rec[s].sw);
    tp.adj.assign(tp.nodes.size(), 0.0);
    auto seed = [&](const AD& o, double g) { if (o.i >= 0) tp.adj[o.i] += g; };
    for (int k = 0; k < 2 * S; ++k) { seed(qn[k], xbar[k]); seed(qdn[k], xbar[2 * S + k]); }
    for (int k = 0; k < 3 * A; ++k) { seed(axn[k], xbar[4 * S + k]); seed(avn[k], xbar[4 * S + 3 * A + k]); }
    tp.reverse();
    auto get = [&](const AD& v) { return v.i >= 0 ? tp.adj[v.i] : 0.0; };
    for (int k = 0; k < 2 * S; ++k) { xbar[k] = get(q[k]); xbar[2 * S + k] = get(qd[k]); }
    for (int k = 0; k < 3 * A; ++k) { xbar[4 * S + k] = get(ax[k]); xbar[4 * S + 3 * A + k] = get(av[k]); }
    for (int i = 0; i < S; ++i) { g_kp[i] += get(kpa[i]); g_kd[i] += get(kda[i]); }
    if (F && g_F) for (int k = 0; k < 3 * A; ++k) g_F[(int64_t)s * 3 * A + k] += get(Fa[k]);
    tp.clear();
  }
  tape() = nullptr;
  if (g_state0) for (int k = 0; k < NX; ++k) g_state0[k] += xbar[k];
  return L;
}

}  // extern "C"

// ======================================================================================
// Access points for the pins: the in-step normal draws, the pivots of the L^T D L
// factorisation, and the dot-product test of one step's tangent-linear and reverse modes
// ======================================================================================
#include "dual.hpp"

namespace orc {

// Entry-flag views for a single step of one tree (counters start at zero).
struct OneStepEvents {
  std::vector<uint8_t> broken, cnt, det, cntp, cntt, path;
  std::vector<int32_t> bstep, dstep;
  uint32_t status = 0;
  OneStepEvents(const Tree& t, const uint8_t* broken0, const uint8_t* det0)
      : broken(t.S, 0), cnt(t.S, 0), det(t.A, 0), cntp(t.A, 0), cntt(t.A, 0), path(t.A, 0), bstep(t.S, -1), dstep(t.A, -1) {
    if (broken0) std::copy(broken0, broken0 + t.S, broken.begin());
    if (det0) std::copy(det0, det0 + t.A, det.begin());
  }
  EventRefs refs() { return EventRefs{broken.data(), cnt.data(), det.data(), cntp.data(), cntt.data(), path.data(), bstep.data(), dstep.data(), &status}; }
};

}  // namespace orc

extern "C" {

// Three standard normals of the in-step random force of (env, step, segment).
void oracle_rng_normals(uint64_t seed, int env, int64_t step, int seg, double* z) {
  rng_normals(seed, env, step, seg, z);
}

// Pivots D (per DoF, [2S]) of the leaf-first L^T D L factorisation of H(q) + diag(dg).
void oracle_ltdl_pivots(void* m, int env, const double* q, const double* dg, double* D) {
  Model* M = static_cast<Model*>(m);
  const Tree& t = M->trees[env];
  Kin<double> K;
  fk(t, q, K);
  std::vector<double> H;
  crba(t, K, H);
  for (int k = 0; k < 2 * t.S; ++k) hent(t, H, k, k) += dg[k];
  ltdl_factor(t, H);
  for (int k = 0; k < 2 * t.S; ++k) D[k] = hent(t, H, k, k);
}

// Dot-product test of one step of tree env at step index n and state x = (q, qd, apple
// position state, apple velocity) [4S + 6A], with parameters kp, kd [S] and apple forces
// F [A][3] (nullable).  The switches the step takes from the entry flags broken0 [S] and
// det0 [A] (nullable: none) are recorded once and frozen in both modes.  Directions
// vx [4S + 6A], vkp, vkd [S], vF [A][3]; output weights w [4S + 6A].
// out[0] = <J v, w> (tangent-linear), out[1] = <v, J^T w> (reverse mode); out[2..5] = the
// numbers of broken joints, detached apples, clamped reactions and capped body forces the
// step used.
void oracle_step_dot(void* m, int env, int64_t n, const double* x, const double* kp, const double* kd, const double* F,
                     const uint8_t* broken0, const uint8_t* det0, const double* vx, const double* vkp,
                     const double* vkd, const double* vF, const double* w, double* out) {
  Model* M = static_cast<Model*>(m);
  const Tree& t = M->trees[env];
  const int S = t.S, A = t.A, N2 = 2 * S, N3 = 3 * A;
  Switches sw;
  {
    OneStepEvents E(t, broken0, det0);
    EventRefs ev = E.refs();
    std::vector<double> aq(4 * A, 0.0), aw(N3, 0.0), qo(N2), qdo(N2), axo(N3), avo(N3), aqo(4 * A), awo(N3);
    for (int a = 0; a < A; ++a) aq[4 * a] = 1.0;
    step_tree<double>(t, M->g, env, n, x, x + N2, x + 2 * N2, x + 2 * N2 + N3, aq.data(), aw.data(), kp, kd, nullptr,
                      F, qo.data(), qdo.data(), axo.data(), avo.data(), aqo.data(), awo.data(), &ev, nullptr, &sw,
                      nullptr);
  }
  const int NX = 2 * N2 + 2 * N3;
  auto count = [](const std::vector<uint8_t>& f) { double c = 0; for (uint8_t x : f) c += x ? 1 : 0; return c; };
  out[2] = count(sw.broken); out[3] = count(sw.detached); out[4] = count(sw.clamped); out[5] = count(sw.capped);
  // tangent-linear
  {
    OneStepEvents E(t, broken0, det0);
    EventRefs ev = E.refs();
    std::vector<DU> xs(NX), kps(S), kds(S), Fs(F ? N3 : 0), aq(4 * A, DU(0.0)), aw(N3, DU(0.0));
    for (int k = 0; k < NX; ++k) xs[k] = DU(x[k], vx[k]);
    for (int i = 0; i < S; ++i) { kps[i] = DU(kp[i], vkp[i]); kds[i] = DU(kd[i], vkd[i]); }
    for (int k = 0; k < (int)Fs.size(); ++k) Fs[k] = DU(F[k], vF ? vF[k] : 0.0);
    for (int a = 0; a < A; ++a) aq[4 * a] = DU(1.0);
    std::vector<DU> qo(N2), qdo(N2), axo(N3), avo(N3), aqo(4 * A), awo(N3);
    step_tree<DU>(t, M->g, env, n, xs.data(), xs.data() + N2, xs.data() + 2 * N2, xs.data() + 2 * N2 + N3, aq.data(),
                  aw.data(), kps.data(), kds.data(), nullptr, F ? Fs.data() : nullptr, qo.data(), qdo.data(),
                  axo.data(), avo.data(), aqo.data(), awo.data(), &ev, nullptr, nullptr, &sw);
    double s = 0.0;
    for (int k = 0; k < N2; ++k) s += w[k] * qo[k].d + w[N2 + k] * qdo[k].d;
    for (int k = 0; k < N3; ++k) s += w[2 * N2 + k] * axo[k].d + w[2 * N2 + N3 + k] * avo[k].d;
    out[0] = s;
  }
  // reverse mode
  {
    OneStepEvents E(t, broken0, det0);
    EventRefs ev = E.refs();
    Tape tp;
    tape() = &tp;
    std::vector<AD> xs(NX), kps(S), kds(S), Fs(F ? N3 : 0), aq(4 * A, AD(0.0)), aw(N3, AD(0.0));
    for (int k = 0; k < NX; ++k) xs[k] = AD::var(x[k]);
    for (int i = 0; i < S; ++i) { kps[i] = AD::var(kp[i]); kds[i] = AD::var(kd[i]); }
    for (int k = 0; k < (int)Fs.size(); ++k) Fs[k] = AD::var(F[k]);
    for (int a = 0; a < A; ++a) aq[4 * a] = AD(1.0);
    std::vector<AD> qo(N2), qdo(N2), axo(N3), avo(N3), aqo(4 * A), awo(N3);
    step_tree<AD>(t, M->g, env, n, xs.data(), xs.data() + N2, xs.data() + 2 * N2, xs.data() + 2 * N2 + N3, aq.data(),
                  aw.data(), kps.data(), kds.data(), nullptr, F ? Fs.data() : nullptr, qo.data(), qdo.data(),
                  axo.data(), avo.data(), aqo.data(), awo.data(), &ev, nullptr, nullptr, &sw);
    tp.adj.assign(tp.nodes.size(), 0.0);
    auto seed = [&](const AD& o, double g) { if (o.i >= 0) tp.adj[o.i] += g; };
    for (int k = 0; k < N2; ++k) { seed(qo[k], w[k]); seed(qdo[k], w[N2 + k]); }
    for (int k = 0; k < N3; ++k) { seed(axo[k], w[2 * N2 + k]); seed(avo[k], w[2 * N2 + N3 + k]); }
    tp.reverse();
    auto get = [&](const AD& v) { return v.i >= 0 ? tp.adj[v.i] : 0.0; };
    double s = 0.0;
    for (int k = 0; k < NX; ++k) s += vx[k] * get(xs[k]);
    for (int i = 0; i < S; ++i) s += vkp[i] * get(kps[i]) + vkd[i] * get(kds[i]);
    for (int k = 0; k < (int)Fs.size(); ++k) s += (vF ? vF[k] : 0.0) * get(Fs[k]);
    tape() = nullptr;
    out[1] = s;
  }
}

}  // extern "C"
