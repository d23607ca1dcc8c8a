// FP64 oracle -- small vector / matrix helpers, templated on the scalar type so
// the same step can be evaluated in double or in the taping AD type.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
// call this code; it exists to check the HIP implementation.
#pragma once
#include <cmath>
#include <cstdint>

namespace orc {

using std::sqrt;
using std::sin;
using std::cos;

inline double val(double x) { return x; }

template <class T> struct V3 {
  T x, y, z;
  V3() : x(0), y(0), z(0) {}
  V3(T a, T b, T c) : x(a), y(b), z(c) {}
  T& operator[](int i) { return i == 0 ? x : (i == 1 ? y : z); }
  const T& operator[](int i) const { return i == 0 ? x : (i == 1 ? y : z); }
};
template <class T> V3<T> operator+(const V3<T>& a, const V3<T>& b) { return V3<T>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class T> V3<T> operator-(const V3<T>& a, const V3<T>& b) { return V3<T>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class T> V3<T> operator-(const V3<T>& a) { return V3<T>(-a.x, -a.y, -a.z); }
template <class T, class S> V3<T> operator*(const S& s, const V3<T>& a) { return V3<T>(s * a.x, s * a.y, s * a.z); }
template <class T> V3<T>& operator+=(V3<T>& a, const V3<T>& b) { a.x = a.x + b.x; a.y = a.y + b.y; a.z = a.z + b.z; return a; }
template <class T> V3<T>& operator-=(V3<T>& a, const V3<T>& b) { a.x = a.x - b.x; a.y = a.y - b.y; a.z = a.z - b.z; return a; }
template <class T> T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return V3<T>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <class T> T norm(const V3<T>& a) { return sqrt(dot(a, a)); }

// 3x3 matrix, row major
template <class T> struct M3 {
  T m[9];
  M3() { for (int i = 0; i < 9; ++i) m[i] = T(0); }
  static M3 eye() { M3 r; r.m[0] = r.m[4] = r.m[8] = T(1); return r; }
  T& operator()(int r, int c) { return m[3 * r + c]; }
  const T& operator()(int r, int c) const { return m[3 * r + c]; }
  V3<T> col(int c) const { return V3<T>(m[c], m[3 + c], m[6 + c]); }
};
template <class T> M3<T> operator*(const M3<T>& a, const M3<T>& b) {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = T(0);
      for (int k = 0; k < 3; ++k) s = s + a(i, k) * b(k, j);
      r(i, j) = s;
    }
  return r;
}
template <class T> V3<T> operator*(const M3<T>& a, const V3<T>& v) {
  return V3<T>(a(0, 0) * v.x + a(0, 1) * v.y + a(0, 2) * v.z,
               a(1, 0) * v.x + a(1, 1) * v.y + a(1, 2) * v.z,
               a(2, 0) * v.x + a(2, 1) * v.y + a(2, 2) * v.z);
}
template <class T> M3<T> operator+(const M3<T>& a, const M3<T>& b) { M3<T> r; for (int i = 0; i < 9; ++i) r.m[i] = a.m[i] + b.m[i]; return r; }
template <class T> M3<T> transpose(const M3<T>& a) {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r(i, j) = a(j, i);
  return r;
}
// rotation about x / y by angle (right hand)
template <class T> M3<T> rot_x(const T& c, const T& s) {
  M3<T> r; r(0, 0) = T(1); r(1, 1) = c; r(1, 2) = -s; r(2, 1) = s; r(2, 2) = c; return r;
}
template <class T> M3<T> rot_y(const T& c, const T& s) {
  M3<T> r; r(0, 0) = c; r(0, 2) = s; r(1, 1) = T(1); r(2, 0) = -s; r(2, 2) = c; return r;
}
// unit quaternion (w,x,y,z) -> rotation matrix
inline M3<double> quat_to_mat(const double* q) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  M3<double> r;
  r(0, 0) = 1 - 2 * (y * y + z * z); r(0, 1) = 2 * (x * y - w * z);     r(0, 2) = 2 * (x * z + w * y);
  r(1, 0) = 2 * (x * y + w * z);     r(1, 1) = 1 - 2 * (x * x + z * z); r(1, 2) = 2 * (y * z - w * x);
  r(2, 0) = 2 * (x * z - w * y);     r(2, 1) = 2 * (y * z + w * x);     r(2, 2) = 1 - 2 * (x * x + y * y);
  return r;
}

// ---- spatial vectors in world coordinates, reference point = world origin ----
// motion vector (angular w, linear v_O); force vector (moment n_O, force f)
template <class T> struct SV { V3<T> a, l; };
template <class T> SV<T> operator+(const SV<T>& p, const SV<T>& q) { return SV<T>{p.a + q.a, p.l + q.l}; }
template <class T> SV<T> operator-(const SV<T>& p, const SV<T>& q) { return SV<T>{p.a - q.a, p.l - q.l}; }
template <class T, class S> SV<T> operator*(const S& s, const SV<T>& p) { return SV<T>{s * p.a, s * p.l}; }
template <class T> T sdot(const SV<T>& m, const SV<T>& f) { return dot(m.a, f.a) + dot(m.l, f.l); }
// motion x motion
template <class T> SV<T> crm(const SV<T>& v, const SV<T>& m) {
  return SV<T>{cross(v.a, m.a), cross(v.a, m.l) + cross(v.l, m.a)};
}
// motion x* force
template <class T> SV<T> crf(const SV<T>& v, const SV<T>& f) {
  return SV<T>{cross(v.a, f.a) + cross(v.l, f.l), cross(v.a, f.l)};
}

// rigid-body spatial inertia about the world origin, kept as (mass, COM, rotational
// inertia about the COM); applying it avoids forming the 6x6.
template <class T> struct RBI {
  T m;
  V3<T> c;     // COM (world)
  M3<T> Ic;    // about COM, world axes
};
// I * v for motion v = (w, v_O): h_O = Ic w + c x (m (v_O + w x c)),  L = m (v_O + w x c)
template <class T> SV<T> rbi_apply(const RBI<T>& I, const SV<T>& v) {
  V3<T> vc = v.l + cross(v.a, I.c);
  V3<T> L = I.m * vc;
  return SV<T>{I.Ic * v.a + cross(I.c, L), L};
}

// dense symmetric 6x6 (articulated / composite inertia), row major
template <class T> struct S6 {
  T m[36];
  S6() { for (int i = 0; i < 36; ++i) m[i] = T(0); }
};
template <class T> S6<T> rbi_to_s6(const RBI<T>& I) {
  // columns = I * unit motion vectors
  S6<T> r;
  for (int k = 0; k < 6; ++k) {
    SV<T> e;
    if (k < 3) e.a[k] = T(1); else e.l[k - 3] = T(1);
    SV<T> f = rbi_apply(I, e);
    for (int i = 0; i < 3; ++i) { r.m[6 * i + k] = f.a[i]; r.m[6 * (i + 3) + k] = f.l[i]; }
  }
  return r;
}
template <class T> SV<T> s6_apply(const S6<T>& I, const SV<T>& v) {
  T x[6] = {v.a.x, v.a.y, v.a.z, v.l.x, v.l.y, v.l.z};
  T y[6];
  for (int i = 0; i < 6; ++i) {
    T s = T(0);
    for (int k = 0; k < 6; ++k) s = s + I.m[6 * i + k] * x[k];
    y[i] = s;
  }
  return SV<T>{V3<T>(y[0], y[1], y[2]), V3<T>(y[3], y[4], y[5])};
}
template <class T> S6<T> operator+(const S6<T>& a, const S6<T>& b) { S6<T> r; for (int i = 0; i < 36; ++i) r.m[i] = a.m[i] + b.m[i]; return r; }

// ---- SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the output function applied
// to x + golden gamma, used as a stateless counter hash ----
inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Counter-based draws for the in-step random wrenches.  Per (env, segment) a static key
// H = splitmix64(splitmix64(seed ^ splitmix64(env)) ^ splitmix64(seg)); per step
// x = splitmix64(H ^ splitmix64(step)).  The top 24 bits of x select the segment; the
// four 24-bit uniforms of a selected segment are bits 63..40 and 39..16 of
// y1 = splitmix64(x) and of y2 = splitmix64(y1).  k = 0 returns the selection bits,
// k = 1..4 the uniforms.
inline uint32_t rng_u24(uint64_t seed, uint64_t env, uint64_t step, uint64_t seg, uint64_t k) {
  const uint64_t H = splitmix64(splitmix64(seed ^ splitmix64(env)) ^ splitmix64(seg));
  const uint64_t x = splitmix64(H ^ splitmix64(step));
  if (k == 0) return (uint32_t)(x >> 40);
  const uint64_t y1 = splitmix64(x), y2 = splitmix64(y1);
  const uint64_t y = k <= 2 ? y1 : y2;
  return (uint32_t)((k & 1) ? (y >> 40) : ((y >> 16) & 0xFFFFFFull));
}

}  // namespace orc
