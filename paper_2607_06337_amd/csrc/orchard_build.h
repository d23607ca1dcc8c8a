// Model derivation of one tree in FP64, shared by the host (orchard_model_create) and the
// device (the one-thread-per-world rebuild kernel), so that both derive every parameter
// with the same operations: capsule mass properties, the joint stiffness (Eq. beam, or
// the per-level exponential model), the rupture moment (Eq. break), the rest pose, the
// damping (2 zeta sqrt(Kp J) with J the mean rest mass-matrix diagonal of the joint, or
// c_d Kp) and the friction scale of each joint.  Contraction of a*b + c into FMAs is off
// in these functions, so host and device round alike.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace orchard {
namespace build {

struct D3 { double x, y, z; };
__host__ __device__ inline D3 d3(double a, double b, double c) { return D3{a, b, c}; }
__host__ __device__ inline D3 add(D3 a, D3 b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline D3 sub(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline D3 scl(double s, D3 a) { return d3(s * a.x, s * a.y, s * a.z); }
__host__ __device__ inline double ddot(D3 a, D3 b) {
#pragma clang fp contract(off)
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
struct DM3 { double m[9]; };
__host__ __device__ inline DM3 mm(const DM3& a, const DM3& b) {
#pragma clang fp contract(off)
  DM3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[3 * i + j] = a.m[3 * i] * b.m[j] + a.m[3 * i + 1] * b.m[3 + j] + a.m[3 * i + 2] * b.m[6 + j];
  return r;
}
__host__ __device__ inline D3 mv(const DM3& a, D3 v) {
#pragma clang fp contract(off)
  return d3(a.m[0] * v.x + a.m[1] * v.y + a.m[2] * v.z, a.m[3] * v.x + a.m[4] * v.y + a.m[5] * v.z,
            a.m[6] * v.x + a.m[7] * v.y + a.m[8] * v.z);
}
// rotation matrix of a unit quaternion (w, x, y, z)
__host__ __device__ inline DM3 quatm(const double* q) {
#pragma clang fp contract(off)
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  return DM3{{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y), 2 * (x * y + w * z),
              1 - 2 * (x * x + z * z), 2 * (y * z - w * x), 2 * (x * z - w * y), 2 * (y * z + w * x),
              1 - 2 * (x * x + y * y)}};
}

// Constants of the derivation (from the model descriptor).
struct DeriveConsts {
  double stiffness_k0, stiffness_gamma;  // k0 > 0: Kp = k0 gamma^depth instead of Eq. beam
  double damping_cd, damping_zeta;
  double gnorm;                          // |g|
  int friction;                          // 1: compute the friction scale wmom
};

// One tree, segments 0..S-1 in descriptor order (parent < child).  Inputs: parent
// (env-local), rest quaternion [4S] (unit within 1e-6), length, radius, density, Young's
// modulus, modulus of rupture.  Outputs [S] (Rw [S], pw [S], qn [4S]): mass, transverse
// inertia about the joint point Jt, axial inertia Ia, Kp, M_max, Kd, friction scale wmom
// (if consts.friction), rest rotation Rw and joint point pw, normalised quaternion qn and
// depth.  tmp: 10 S doubles of workspace.
struct DeriveIO {
  int S;
  const int32_t* parent;
  const double *quat, *len, *rad, *rho, *E, *mor;
  double *mass, *Jt, *Ia, *kp, *mmax, *kd, *wmom, *qn;
  DM3* Rw;
  D3* pw;
  int32_t* depth;
  double* tmp;
};

__host__ __device__ inline void derive_tree(const DeriveConsts& c, const DeriveIO& t) {
#pragma clang fp contract(off)
  const int S = t.S;
  // root -> leaf: mass properties, gains, rest pose
  for (int i = 0; i < S; ++i) {
    const int p = t.parent[i];
    const double l = t.len[i], r = t.rad[i], rho = t.rho[i];
    const double* q = t.quat + 4 * i;
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double* qn = t.qn + 4 * i;
    qn[0] = q[0] / nq; qn[1] = q[1] / nq; qn[2] = q[2] / nq; qn[3] = q[3] / nq;
    // capsule: cylinder + two hemispheres
    const double mc = rho * M_PI * r * r * l, mh = rho * 4.0 / 3.0 * M_PI * r * r * r;
    t.mass[i] = mc + mh;
    t.Ia[i] = mc * r * r / 2.0 + mh * 2.0 * r * r / 5.0;
    const double It = mc * (l * l / 12.0 + r * r / 4.0) + mh * (2.0 * r * r / 5.0 + l * l / 4.0 + 3.0 * l * r / 8.0);
    t.Jt[i] = It + t.mass[i] * l * l / 4.0;  // transverse inertia about the joint point
    t.kp[i] = M_PI / 4.0 * t.E[i] * r * r * r * r / l;  // Eq. beam
    t.mmax[i] = t.mor[i] * M_PI * r * r * r / 4.0;      // Eq. break
    const DM3 Q = quatm(qn);
    if (p < 0) {
      t.Rw[i] = Q; t.pw[i] = d3(0, 0, 0); t.depth[i] = 0;
    } else {
      t.Rw[i] = mm(t.Rw[p], Q);
      t.pw[i] = add(t.pw[p], scl(t.len[p], d3(t.Rw[p].m[2], t.Rw[p].m[5], t.Rw[p].m[8])));
      t.depth[i] = t.depth[p] + 1;
    }
    // per-level exponential model: each level below the root scales the stiffness by gamma
    if (c.stiffness_k0 > 0) t.kp[i] = c.stiffness_k0 * pow(c.stiffness_gamma, (double)t.depth[i]);
  }
  // friction scale of each joint: its limb's largest weight moment, every body of the
  // sub-tree at the distance of its centre of mass from the joint point (rest pose)
  for (int i = 0; i < S; ++i) t.wmom[i] = 0.0;
  if (c.friction) {
    for (int b = 0; b < S; ++b) {
      const D3 cb = add(t.pw[b], scl(0.5 * t.len[b], d3(t.Rw[b].m[2], t.Rw[b].m[5], t.Rw[b].m[8])));
      for (int j = b; j >= 0; j = t.parent[j]) {
        const D3 r = sub(cb, t.pw[j]);
        t.wmom[j] += c.gnorm * t.mass[b] * sqrt(ddot(r, r));
      }
    }
  }
  // composite rotational inertia of every sub-tree about its joint point at rest:
  // accumulate mass, first moment and inertia about the world origin leaf -> root
  // (tmp per segment: JO 6, M 1, C 3)
  for (int k = 0; k < 10 * S; ++k) t.tmp[k] = 0.0;
  for (int i = S - 1; i >= 0; --i) {
    double* J = t.tmp + 10 * i;
    const D3 z = d3(t.Rw[i].m[2], t.Rw[i].m[5], t.Rw[i].m[8]);
    const D3 cm = add(t.pw[i], scl(0.5 * t.len[i], z));
    const double It = t.Jt[i] - t.mass[i] * t.len[i] * t.len[i] / 4.0, dI = t.Ia[i] - It;
    const double m = t.mass[i], cc = ddot(cm, cm);
    J[0] += It + dI * z.x * z.x + m * (cc - cm.x * cm.x);
    J[1] += It + dI * z.y * z.y + m * (cc - cm.y * cm.y);
    J[2] += It + dI * z.z * z.z + m * (cc - cm.z * cm.z);
    J[3] += dI * z.x * z.y - m * cm.x * cm.y;
    J[4] += dI * z.x * z.z - m * cm.x * cm.z;
    J[5] += dI * z.y * z.z - m * cm.y * cm.z;
    J[6] += m;
    J[7] += m * cm.x; J[8] += m * cm.y; J[9] += m * cm.z;
    const int p = t.parent[i];
    if (p >= 0) {
      double* Jp = t.tmp + 10 * p;
      for (int k = 0; k < 10; ++k) Jp[k] += J[k];
    }
  }
  for (int i = 0; i < S; ++i) {
    const double* JO = t.tmp + 10 * i;
    const int p = t.parent[i];
    const double M = JO[6];
    const D3 C = scl(1.0 / M, d3(JO[7], JO[8], JO[9])), P = t.pw[i], Cp = sub(C, P);
    // J_P = J_O - M(|C|^2 1 - C C^T) + M(|C-P|^2 1 - (C-P)(C-P)^T)
    const double cc = ddot(C, C), pp = ddot(Cp, Cp);
    double J[6];
    J[0] = JO[0] - M * (cc - C.x * C.x) + M * (pp - Cp.x * Cp.x);
    J[1] = JO[1] - M * (cc - C.y * C.y) + M * (pp - Cp.y * Cp.y);
    J[2] = JO[2] - M * (cc - C.z * C.z) + M * (pp - Cp.z * Cp.z);
    J[3] = JO[3] + M * C.x * C.y - M * Cp.x * Cp.y;
    J[4] = JO[4] + M * C.x * C.z - M * Cp.x * Cp.z;
    J[5] = JO[5] + M * C.y * C.z - M * Cp.y * Cp.z;
    const DM3 Rpar = p < 0 ? DM3{{1, 0, 0, 0, 1, 0, 0, 0, 1}} : t.Rw[p];
    const DM3 Jf = mm(Rpar, quatm(t.qn + 4 * i));
    const D3 a0 = d3(Jf.m[0], Jf.m[3], Jf.m[6]), a1 = d3(t.Rw[i].m[1], t.Rw[i].m[4], t.Rw[i].m[7]);
    const double q0 = J[0] * a0.x * a0.x + J[1] * a0.y * a0.y + J[2] * a0.z * a0.z +
                      2.0 * (J[3] * a0.x * a0.y + J[4] * a0.x * a0.z + J[5] * a0.y * a0.z);
    const double q1 = J[0] * a1.x * a1.x + J[1] * a1.y * a1.y + J[2] * a1.z * a1.z +
                      2.0 * (J[3] * a1.x * a1.y + J[4] * a1.x * a1.z + J[5] * a1.y * a1.z);
    const double Jj = 0.5 * (q0 + q1);
    t.kd[i] = c.damping_cd > 0 ? c.damping_cd * t.kp[i] : 2.0 * c.damping_zeta * sqrt(t.kp[i] * Jj);
  }
}

// Rest hang point of a fruit: joint point plus the rotated hang offset.
__host__ __device__ inline D3 hang_point(const DM3& R, D3 p, D3 hl) { return add(p, mv(R, hl)); }

// A segment's rest quaternion bent by angles ax about its x axis, then ay about its y
// axis: q (x) (cos ax/2, sin ax/2, 0, 0) (x) (cos ay/2, 0, sin ay/2, 0).
__host__ __device__ inline void bend_quat(const double* q, double ax, double ay, double* out) {
#pragma clang fp contract(off)
  const double cx = cos(0.5 * ax), sx = sin(0.5 * ax), cy = cos(0.5 * ay), sy = sin(0.5 * ay);
  // r = q (x) (cx, sx, 0, 0)
  const double r0 = q[0] * cx - q[1] * sx, r1 = q[0] * sx + q[1] * cx, r2 = q[2] * cx + q[3] * sx,
               r3 = q[3] * cx - q[2] * sx;
  // out = r (x) (cy, 0, sy, 0)
  out[0] = r0 * cy - r2 * sy;
  out[1] = r1 * cy - r3 * sy;
  out[2] = r0 * sy + r2 * cy;
  out[3] = r3 * cy + r1 * sy;
}

}  // namespace build
}  // namespace orchard
