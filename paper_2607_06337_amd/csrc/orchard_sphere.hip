// Batched sphere-fit detector (Sec. "Geometric fruit perception", Eq. spherefit): each
// patch of back-projected depth points is fitted with the sphere that solves
// 2 p.c + b = |p|^2 (b = R^2 - |c|^2) in the least-squares sense, then gated on radius and
// RMS geometric residual.  One wavefront per patch; the work is a few streaming passes
// over 12 bytes per point, so the kernel is bound by memory, not by arithmetic.
//
// Numerics: the FP32 points are shifted by the patch's first point and centred on their
// mean in FP64 (the shift is exact there), and the moments, the solve and the residual
// run in FP64 as well, which costs nothing here (the vector units issue FP64 at the
// FP32 rate without packed math, and the kernel waits on memory) and removes the FP32
// error the fit of a shallow cap amplifies by 10^3..10^4.  Centring turns the 4x4 normal
// equations into a 3x3 system for the centre in the central second moments (the mean row
// decouples: b' = sum |u|^2 / n).
#include <hip/hip_runtime.h>

#include "../../include/orchard.h"

namespace orchard {
namespace {

constexpr int kWaves = 4;  // wavefronts (patches) per workgroup

// butterfly sums end with the same bits in every lane (each stage adds the same two
// operands in both partners)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__global__ __launch_bounds__(64 * kWaves) void k_sphere_fit(const float* __restrict__ pts,
                                                           const int32_t* __restrict__ off, int n_patch,
                                                           orchard_sphere_gate_t gate, float* __restrict__ out) {
  const int lane = (int)(threadIdx.x & 63);
  const int patch = (int)blockIdx.x * kWaves + (int)(threadIdx.x >> 6);
  if (patch >= n_patch) return;  // uniform per wavefront
  const int b = off[patch], e = off[patch + 1];
  const int n = e > b ? e - b : 0;
  float res[8] = {0.f, 0.f, 0.f, 0.f, 0.f, (float)n, 1.f, 0.f};
  if (n >= gate.min_points && n >= 4) {
    const double x0 = pts[3 * (int64_t)b], y0 = pts[3 * (int64_t)b + 1], z0 = pts[3 * (int64_t)b + 2];
    // pass 1: mean of the shifted points
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int k = b + lane; k < e; k += 64) {
      const float* p = pts + 3 * (int64_t)k;
      sx += (double)p[0] - x0; sy += (double)p[1] - y0; sz += (double)p[2] - z0;
    }
    const double inv_n = 1.0 / (double)n;
    const double mx = wave_sum(sx) * inv_n, my = wave_sum(sy) * inv_n, mz = wave_sum(sz) * inv_n;
    // pass 2: central second moments and sum |u|^2 u, sum |u|^2
    double cxx = 0.0, cxy = 0.0, cxz = 0.0, cyy = 0.0, cyz = 0.0, czz = 0.0, wx = 0.0, wy = 0.0, wz = 0.0, ww = 0.0;
    for (int k = b + lane; k < e; k += 64) {
      const float* p = pts + 3 * (int64_t)k;
      const double ux = ((double)p[0] - x0) - mx, uy = ((double)p[1] - y0) - my, uz = ((double)p[2] - z0) - mz;
      const double w = fma(ux, ux, fma(uy, uy, uz * uz));
      cxx = fma(ux, ux, cxx); cxy = fma(ux, uy, cxy); cxz = fma(ux, uz, cxz);
      cyy = fma(uy, uy, cyy); cyz = fma(uy, uz, cyz); czz = fma(uz, uz, czz);
      wx = fma(w, ux, wx); wy = fma(w, uy, wy); wz = fma(w, uz, wz);
      ww += w;
    }
    cxx = wave_sum(cxx); cxy = wave_sum(cxy); cxz = wave_sum(cxz);
    cyy = wave_sum(cyy); cyz = wave_sum(cyz); czz = wave_sum(czz);
    wx = wave_sum(wx); wy = wave_sum(wy); wz = wave_sum(wz); ww = wave_sum(ww);
    // centre c' (from the mean) solves C c' = (1/2) sum |u|^2 u; Cholesky of C, whose
    // pivots fall to rounding level when the points span no volume
    const double tr = cxx + cyy + czz;
    const double eps = 1e-9 * tr;
    const double l11sq = cxx;
    bool ok = l11sq > eps;
    const double l11 = sqrt(fmax(l11sq, 0.0));
    const double l21 = ok ? cxy / l11 : 0.0, l31 = ok ? cxz / l11 : 0.0;
    const double l22sq = cyy - l21 * l21;
    ok = ok && l22sq > eps;
    const double l22 = sqrt(fmax(l22sq, 0.0));
    const double l32 = ok ? (cyz - l31 * l21) / l22 : 0.0;
    const double l33sq = czz - l31 * l31 - l32 * l32;
    ok = ok && l33sq > eps;
    if (!ok) {
      res[6] = 2.f;  // degenerate: the points span no volume (a plane or a line)
    } else {
      const double l33 = sqrt(l33sq);
      const double r1 = 0.5 * wx, r2 = 0.5 * wy, r3 = 0.5 * wz;
      const double y1 = r1 / l11, y2 = (r2 - l21 * y1) / l22, y3 = (r3 - l31 * y1 - l32 * y2) / l33;
      const double cz = y3 / l33, cy = (y2 - l32 * cz) / l22, cx = (y1 - l21 * cy - l31 * cz) / l11;
      const double R = sqrt(fmax(fma(ww, inv_n, fma(cx, cx, fma(cy, cy, cz * cz))), 0.0));
      // pass 3: RMS of the geometric residual |u - c'| - R
      double rr = 0.0;
      for (int k = b + lane; k < e; k += 64) {
        const float* p = pts + 3 * (int64_t)k;
        const double dx = (((double)p[0] - x0) - mx) - cx, dy = (((double)p[1] - y0) - my) - cy,
                     dz = (((double)p[2] - z0) - mz) - cz;
        const double d = sqrt(fma(dx, dx, fma(dy, dy, dz * dz))) - R;
        rr = fma(d, d, rr);
      }
      const double rms = sqrt(wave_sum(rr) * inv_n);
      res[0] = (float)(x0 + (mx + cx)); res[1] = (float)(y0 + (my + cy)); res[2] = (float)(z0 + (mz + cz));
      res[3] = (float)R;
      res[4] = (float)rms;
      // the gate decides in FP64, as the reference does
      res[6] = (R < (double)gate.r_min || R > (double)gate.r_max) ? 3.f : (rms > (double)gate.rms_max ? 4.f : 0.f);
    }
  }
  if (lane < 2) {
    float4* o = reinterpret_cast<float4*>(out + 8 * (int64_t)patch);
    o[lane] = lane == 0 ? make_float4(res[0], res[1], res[2], res[3]) : make_float4(res[4], res[5], res[6], res[7]);
  }
}

}  // namespace
}  // namespace orchard

namespace orchard {
orchard_status_t report_error(orchard_status_t s, const char* msg);  // sets orchard_last_error()
}

extern "C" orchard_status_t orchard_sphere_fit(const float* points, const int32_t* patch_offset, int32_t n_patch,
                                               const orchard_sphere_gate_t* gate, float* out,
                                               orchard_stream_t stream) {
  using orchard::report_error;
  if (n_patch < 0 || !gate || (n_patch > 0 && (!points || !patch_offset || !out)))
    return report_error(ORCHARD_ERR_INVALID_ARG, "sphere fit: null pointer or n_patch < 0");
  if (!(gate->r_min >= 0.f) || !(gate->r_max >= gate->r_min) || !(gate->rms_max >= 0.f))
    return report_error(ORCHARD_ERR_INVALID_ARG, "sphere fit: gate bounds out of order");
  if (n_patch == 0) return ORCHARD_OK;
  const int blocks = (n_patch + orchard::kWaves - 1) / orchard::kWaves;
  hipLaunchKernelGGL(orchard::k_sphere_fit, dim3(blocks), dim3(64 * orchard::kWaves), 0, (hipStream_t)stream, points,
                     patch_offset, n_patch, *gate, out);
  const hipError_t he = hipGetLastError();
  return he == hipSuccess ? ORCHARD_OK : report_error(ORCHARD_ERR_HIP, hipGetErrorString(he));
}
