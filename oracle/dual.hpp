// Forward-mode dual numbers (value and one tangent), used to evaluate the oracle's own
// step in tangent-linear mode for the dot-product test of its reverse mode.
//
// TEST INFRASTRUCTURE ONLY (part of the FP64 oracle).
#pragma once
#include <cmath>

namespace orc {

struct DU {
  double v, d;
  DU() : v(0.0), d(0.0) {}
  DU(double x) : v(x), d(0.0) {}
  DU(double x, double dx) : v(x), d(dx) {}
};

inline double val(const DU& x) { return x.v; }

inline DU operator+(const DU& x, const DU& y) { return DU(x.v + y.v, x.d + y.d); }
inline DU operator-(const DU& x, const DU& y) { return DU(x.v - y.v, x.d - y.d); }
inline DU operator*(const DU& x, const DU& y) { return DU(x.v * y.v, x.d * y.v + x.v * y.d); }
inline DU operator/(const DU& x, const DU& y) { return DU(x.v / y.v, (x.d * y.v - x.v * y.d) / (y.v * y.v)); }
inline DU operator-(const DU& x) { return DU(-x.v, -x.d); }
inline DU operator+(const DU& x, double y) { return DU(x.v + y, x.d); }
inline DU operator+(double x, const DU& y) { return DU(x + y.v, y.d); }
inline DU operator-(const DU& x, double y) { return DU(x.v - y, x.d); }
inline DU operator-(double x, const DU& y) { return DU(x - y.v, -y.d); }
inline DU operator*(const DU& x, double y) { return DU(x.v * y, x.d * y); }
inline DU operator*(double x, const DU& y) { return DU(x * y.v, x * y.d); }
inline DU operator/(const DU& x, double y) { return DU(x.v / y, x.d / y); }
inline DU operator/(double x, const DU& y) { return DU(x / y.v, -x * y.d / (y.v * y.v)); }
inline DU sqrt(const DU& x) { const double s = std::sqrt(x.v); return DU(s, s > 0 ? 0.5 * x.d / s : 0.0); }
inline DU sin(const DU& x) { return DU(std::sin(x.v), std::cos(x.v) * x.d); }
inline DU cos(const DU& x) { return DU(std::cos(x.v), -std::sin(x.v) * x.d); }

}  // namespace orc
