// Minimal reverse-mode automatic differentiation (operator overloading on a tape),
// used to differentiate the oracle's own step mechanically.
//
// TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).
#pragma once
#include <cmath>
#include <vector>

namespace orc {

struct Tape {
  struct Node { int a, b; double da, db; };
  std::vector<Node> nodes;
  std::vector<double> adj;
  int push(int a, double da, int b, double db) {
    nodes.push_back(Node{a, b, da, db});
    return (int)nodes.size() - 1;
  }
  int leaf() { return push(-1, 0.0, -1, 0.0); }
  void clear() { nodes.clear(); adj.clear(); }
  // propagate adjoints from the seeds already placed in adj
  void reverse() {
    for (int k = (int)nodes.size() - 1; k >= 0; --k) {
      const double g = adj[k];
      if (g == 0.0) continue;
      const Node& n = nodes[k];
      if (n.a >= 0) adj[n.a] += g * n.da;
      if (n.b >= 0) adj[n.b] += g * n.db;
    }
  }
};

inline Tape*& tape() {
  static thread_local Tape* t = nullptr;
  return t;
}

// AD scalar: value and tape index (-1 = constant)
struct AD {
  double v;
  int i;
  AD() : v(0.0), i(-1) {}
  AD(double x) : v(x), i(-1) {}
  static AD var(double x) { AD r; r.v = x; r.i = tape()->leaf(); return r; }
};

inline double val(const AD& x) { return x.v; }

inline AD mk(double v, int a, double da, int b, double db) {
  AD r;
  r.v = v;
  if (a < 0 && b < 0) { r.i = -1; return r; }
  r.i = tape()->push(a, da, b, db);
  return r;
}

inline AD operator+(const AD& x, const AD& y) { return mk(x.v + y.v, x.i, 1.0, y.i, 1.0); }
inline AD operator-(const AD& x, const AD& y) { return mk(x.v - y.v, x.i, 1.0, y.i, -1.0); }
inline AD operator*(const AD& x, const AD& y) { return mk(x.v * y.v, x.i, y.v, y.i, x.v); }
inline AD operator/(const AD& x, const AD& y) { return mk(x.v / y.v, x.i, 1.0 / y.v, y.i, -x.v / (y.v * y.v)); }
inline AD operator-(const AD& x) { return mk(-x.v, x.i, -1.0, -1, 0.0); }
inline AD operator+(const AD& x, double y) { return mk(x.v + y, x.i, 1.0, -1, 0.0); }
inline AD operator+(double x, const AD& y) { return mk(x + y.v, y.i, 1.0, -1, 0.0); }
inline AD operator-(const AD& x, double y) { return mk(x.v - y, x.i, 1.0, -1, 0.0); }
inline AD operator-(double x, const AD& y) { return mk(x - y.v, y.i, -1.0, -1, 0.0); }
inline AD operator*(const AD& x, double y) { return mk(x.v * y, x.i, y, -1, 0.0); }
inline AD operator*(double x, const AD& y) { return mk(x * y.v, y.i, x, -1, 0.0); }
inline AD operator/(const AD& x, double y) { return mk(x.v / y, x.i, 1.0 / y, -1, 0.0); }
inline AD operator/(double x, const AD& y) { return mk(x / y.v, y.i, -x / (y.v * y.v), -1, 0.0); }
inline AD sqrt(const AD& x) { const double s = std::sqrt(x.v); return mk(s, x.i, s > 0 ? 0.5 / s : 0.0, -1, 0.0); }
inline AD sin(const AD& x) { return mk(std::sin(x.v), x.i, std::cos(x.v), -1, 0.0); }
inline AD cos(const AD& x) { return mk(std::cos(x.v), x.i, -std::sin(x.v), -1, 0.0); }

}  // namespace orc
