// Batched sphere-fit detector (Sec. "Geometric fruit perception", Eq. spherefit): each
// patch of back-projected depth points is fitted with the sphere that solves
// 2 p.c + b = |p|^2 (b = R^2 - |c|^2) in the least-squares sense, then gated on radius and
// RMS geometric residual.  One wavefront per patch, two streaming passes over 12 bytes per
// point; on the benchmark's patches the vector ALUs are the busier resource (the FP64
// passes plus each patch's cross-lane sums and solve), HBM runs well below its rate.
//
// Numerics: the FP32 points are shifted by the patch's first point in FP64 (exact), and
// one pass gathers the shifted sums n, sum q, sum q q^T, sum |q|^2 q and sum |q|^2 in FP64;
// the central moments follow from them in closed form (with shifts of a few centimetres
// FP64 loses nothing there), the centre from the 3x3 system C c' = (1/2) sum |u|^2 u of
// the centred coordinates u (centring decouples the mean row of the 4x4 normal equations:
// b' = sum |u|^2 / n), and a second pass sums the squared geometric residuals
// d = (|u - c'|^2 - R^2) / (|u - c'| + R), the numerator in FP64, the denominator in
// FP32 (relative error 1e-7 in d, without a FP64 square root per point).  FP64 costs
// little here: the vector units issue it at the FP32 rate without packed math.
#include <hip/hip_runtime.h>

#include "../../include/orchard.h"

namespace orchard {
namespace {

// One wavefront (one patch) per workgroup.  Patch sizes span 8 to 4096 points, and four
// patches to a workgroup ran 14 % slower on the benchmark's patches (a small patch's wave
// slot waits for the largest patch of its workgroup); sorting the patches by size first
// would gain 5 % more, not enough to pay for a sorting pass.
constexpr int kWaves = 1;

// butterfly sums end with the same bits in every lane (each stage adds the same two
// operands in both partners)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Wave sums of N values at once (reduce-scatter): at the stage of mask m a lane keeps the
// first half of its current list when lane & m is 0 and the second half otherwise, and
// receives its partner's copy of the half it keeps, so the lists halve while one shuffle
// per kept value crosses lanes; once a single value is left, the last stages are plain
// butterflies.  15 shuffles sum 13 values instead of 6 per value.  Lane l ends holding the
// sum whose index follows from its bits (sum_src gives the lane of each index); every
// lane then reads each sum from that lane, so all lanes hold the same bits.
template <int C, int M>
__device__ __forceinline__ void rs_stage(double* v, int lane) {
  if constexpr (C > 1) {
    constexpr int H = (C + 1) / 2;
    const bool up = (lane & M) != 0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const double lo = v[k], hi = H + k < C ? v[H + k] : 0.0;
      const double got = __shfl_xor(up ? lo : hi, M, 64);
      v[k] = (up ? hi : lo) + got;
    }
    rs_stage<H, M / 2>(v, lane);
  } else if constexpr (M >= 1) {
    v[0] += __shfl_xor(v[0], M, 64);
    rs_stage<1, M / 2>(v, lane);
  }
}
// lane holding the sum of index k after rs_stage<C, 32>
template <int C, int M>
__host__ __device__ constexpr int sum_src(int k) {
  if constexpr (C > 1) {
    constexpr int H = (C + 1) / 2;
    return k < H ? sum_src<H, M / 2>(k) : M + sum_src<H, M / 2>(k - H);
  } else {
    return 0;
  }
}
__device__ __forceinline__ double read_lane(double v, int src) {
  const int2 w = *reinterpret_cast<const int2*>(&v);
  const int2 r = make_int2(__builtin_amdgcn_readlane(w.x, src), __builtin_amdgcn_readlane(w.y, src));
  return *reinterpret_cast<const double*>(&r);
}
template <int N>
__device__ __forceinline__ void wave_sums(double (&v)[N], int lane) {
  double t[N];
#pragma unroll
  for (int k = 0; k < N; ++k) t[k] = v[k];
  rs_stage<N, 32>(t, lane);
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = read_lane(t[0], sum_src<N, 32>(k));
}

// Points are read in chunks of 64 x KP: each lane issues all KP loads of a chunk before it
// uses any, and a patch that fits one chunk is read from memory once, its second pass
// working from registers.
constexpr int KP = 4;

struct Chunk {
  float x[KP], y[KP], z[KP];
};
// The loads carry no branch (a lane past the patch's end re-reads its last point, which
// the passes then weigh zero), so the compiler issues all of them before the first wait.
__device__ __forceinline__ void load_chunk(const float* __restrict__ pts, int k0, int e, int lane, Chunk& c) {
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int k = min(k0 + 64 * j + lane, e - 1);
    const float* p = pts + 3 * (int64_t)k;
    c.x[j] = p[0]; c.y[j] = p[1]; c.z[j] = p[2];
  }
}

// the fit of one patch (points b .. e-1, n = e - b >= 4) by one wavefront; res as out[]
__device__ __forceinline__ void fit_patch(const float* __restrict__ pts, int b, int e, int lane,
                                          const orchard_sphere_gate_t& gate, float (&res)[8]) {
  const int n = e - b;
  const double x0 = pts[3 * (int64_t)b], y0 = pts[3 * (int64_t)b + 1], z0 = pts[3 * (int64_t)b + 2];
  const bool one = n <= 64 * KP;  // the whole patch stays in registers
  Chunk c;
  // pass 1: sums of the shifted points q = p - p0
  double sx = 0.0, sy = 0.0, sz = 0.0, qxx = 0.0, qxy = 0.0, qxz = 0.0, qyy = 0.0, qyz = 0.0, qzz = 0.0;
  double wx = 0.0, wy = 0.0, wz = 0.0, ww = 0.0;
  for (int k0 = b; k0 < e; k0 += 64 * KP) {
    load_chunk(pts, k0, e, lane, c);
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const bool v = k0 + 64 * j + lane < e;  // a point past the end contributes q = 0
      const double qx = v ? (double)c.x[j] - x0 : 0.0, qy = v ? (double)c.y[j] - y0 : 0.0,
                   qz = v ? (double)c.z[j] - z0 : 0.0;
      const double w = fma(qx, qx, fma(qy, qy, qz * qz));
      sx += qx; sy += qy; sz += qz;
      qxx = fma(qx, qx, qxx); qxy = fma(qx, qy, qxy); qxz = fma(qx, qz, qxz);
      qyy = fma(qy, qy, qyy); qyz = fma(qy, qz, qyz); qzz = fma(qz, qz, qzz);
      wx = fma(w, qx, wx); wy = fma(w, qy, wy); wz = fma(w, qz, wz);
      ww += w;
    }
  }
  {
    double v[13] = {sx, sy, sz, qxx, qxy, qxz, qyy, qyz, qzz, wx, wy, wz, ww};
    wave_sums(v, lane);
    sx = v[0]; sy = v[1]; sz = v[2]; qxx = v[3]; qxy = v[4]; qxz = v[5];
    qyy = v[6]; qyz = v[7]; qzz = v[8]; wx = v[9]; wy = v[10]; wz = v[11]; ww = v[12];
  }
  // central moments of u = q - m, m the mean: C = S_qq - n m m^T,
  // sum |u|^2 u = S_wq - m S_w - 2 S_qq m + 2 n |m|^2 m, sum |u|^2 = S_w - n |m|^2
  const double nd = (double)n, inv_n = 1.0 / nd;
  const double mx = sx * inv_n, my = sy * inv_n, mz = sz * inv_n;
  const double mm = fma(mx, mx, fma(my, my, mz * mz));
  const double cxx = qxx - nd * mx * mx, cxy = qxy - nd * mx * my, cxz = qxz - nd * mx * mz;
  const double cyy = qyy - nd * my * my, cyz = qyz - nd * my * mz, czz = qzz - nd * mz * mz;
  const double Qmx = qxx * mx + qxy * my + qxz * mz, Qmy = qxy * mx + qyy * my + qyz * mz,
               Qmz = qxz * mx + qyz * my + qzz * mz;
  const double uwx = wx - mx * ww - 2.0 * Qmx + 2.0 * nd * mm * mx;
  const double uwy = wy - my * ww - 2.0 * Qmy + 2.0 * nd * mm * my;
  const double uwz = wz - mz * ww - 2.0 * Qmz + 2.0 * nd * mm * mz;
  const double uww = ww - nd * mm;
  // centre c' (from the mean) solves C c' = (1/2) sum |u|^2 u; Cholesky of C, whose
  // pivots fall to rounding level when the points span no volume
  const double tr = cxx + cyy + czz;
  const double eps = 1e-9 * tr;
  const double l11sq = cxx;
  bool ok = l11sq > eps;
  // (the diagonal of L is inverted once; the substitutions multiply by the inverses)
  const double i11 = ok ? 1.0 / sqrt(l11sq) : 0.0;
  const double l21 = cxy * i11, l31 = cxz * i11;
  const double l22sq = cyy - l21 * l21;
  ok = ok && l22sq > eps;
  const double i22 = ok ? 1.0 / sqrt(l22sq) : 0.0;
  const double l32 = (cyz - l31 * l21) * i22;
  const double l33sq = czz - l31 * l31 - l32 * l32;
  ok = ok && l33sq > eps;
  if (!ok) {
    res[6] = 2.f;  // degenerate: the points span no volume (a plane or a line)
    return;
  }
  const double i33 = 1.0 / sqrt(l33sq);
  const double r1 = 0.5 * uwx, r2 = 0.5 * uwy, r3 = 0.5 * uwz;
  const double y1 = r1 * i11, y2 = (r2 - l21 * y1) * i22, y3 = (r3 - l31 * y1 - l32 * y2) * i33;
  const double cz = y3 * i33, cy = (y2 - l32 * cz) * i22, cx = (y1 - l21 * cy - l31 * cz) * i11;
  const double R2 = fmax(fma(uww, inv_n, fma(cx, cx, fma(cy, cy, cz * cz))), 0.0);
  const double R = sqrt(R2);
  // pass 2: RMS of the geometric residual |q - (m + c')| - R
  const double ox = mx + cx, oy = my + cy, oz = mz + cz;  // centre relative to p0
  const float Rf = (float)R;
  double rr = 0.0;
  for (int k0 = b; k0 < e; k0 += 64 * KP) {
    if (!one) load_chunk(pts, k0, e, lane, c);
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const bool v = k0 + 64 * j + lane < e;
      const double dx = ((double)c.x[j] - x0) - ox, dy = ((double)c.y[j] - y0) - oy, dz = ((double)c.z[j] - z0) - oz;
      const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
      const double d = (d2 - R2) * (double)(1.f / (sqrtf((float)d2) + Rf));
      rr = v ? fma(d, d, rr) : rr;
    }
  }
  const double rms = sqrt(wave_sum(rr) * inv_n);
  res[0] = (float)(x0 + ox); res[1] = (float)(y0 + oy); res[2] = (float)(z0 + oz);
  res[3] = (float)R;
  res[4] = (float)rms;
  // the gate decides in FP64, as the reference does
  res[6] = (R < (double)gate.r_min || R > (double)gate.r_max) ? 3.f : (rms > (double)gate.rms_max ? 4.f : 0.f);
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
  if (n >= gate.min_points && n >= 4) fit_patch(pts, b, e, lane, gate, res);
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
