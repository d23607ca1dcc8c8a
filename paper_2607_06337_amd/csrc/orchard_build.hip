// On-device rebuild of every world's geometry, one thread per world: the length, radius
// and rest orientation of each segment are perturbed by caller-given factors and every
// parameter that depends on them is derived again in FP64 with the same function the
// host uses at create (Sec. "Parallelism and cost": the per-world geometry build as one
// kernel, one thread per world).
#include <hip/hip_runtime.h>

#include "orchard_build.h"
#include "orchard_dev.h"
#include "orchard_rebuild.h"

namespace orchard {

__global__ void k_rebuild(RebuildArgs A) {
  const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (e >= A.n_env) return;
  const int s0 = A.seg_off[e], S = A.seg_off[e + 1] - s0;
  const int64_t NS = A.n_seg;
  double* W = A.work;
  double *quatp = W, *lenp = W + 4 * NS, *radp = W + 5 * NS;
  double *mass = W + 6 * NS, *Jt = W + 7 * NS, *Ia = W + 8 * NS, *kp = W + 9 * NS, *mmax = W + 10 * NS,
         *kd = W + 11 * NS, *wmom = W + 12 * NS, *qn = W + 13 * NS;
  build::DM3* Rw = reinterpret_cast<build::DM3*>(W + 17 * NS);
  build::D3* pw = reinterpret_cast<build::D3*>(W + 26 * NS);
  double* tmp = W + 29 * NS;
  int32_t* depth = reinterpret_cast<int32_t*>(W + 39 * NS);
  // perturbed inputs; a world with a non-positive or non-finite factor stays as it is
  for (int k = 0; k < S; ++k) {
    const int64_t g = s0 + k;
    const double* f = A.factors + 4 * g;
    if (!(f[0] > 0) || !(f[1] > 0) || !isfinite(f[0]) || !isfinite(f[1]) || !isfinite(f[2]) || !isfinite(f[3])) {
      if (A.rejected) atomicAdd(A.rejected, 1);
      return;
    }
    lenp[g] = A.blen[g] * f[0];
    radp[g] = A.rad[g] * f[1];
    build::bend_quat(A.quat + 4 * g, f[2], f[3], quatp + 4 * g);
  }
  const build::DeriveIO io{S, A.parent + s0, quatp + 4 * (int64_t)s0, lenp + s0, radp + s0, A.rho + s0, A.E + s0,
                           A.mor + s0, mass + s0, Jt + s0, Ia + s0, kp + s0, mmax + s0, kd + s0, wmom + s0,
                           qn + 4 * (int64_t)s0, Rw + s0, pw + s0, depth + s0, tmp + 10 * (int64_t)s0};
  build::derive_tree(A.consts, io);
  // the model's per-node arrays (internal order), as create writes them
  for (int k = 0; k < S; ++k) {
    const int64_t g = s0 + k;
    const int i = A.int_of[g];
    const float4 q4 = make_float4((float)qn[4 * g], (float)qn[4 * g + 1], (float)qn[4 * g + 2], (float)qn[4 * g + 3]);
    const float4 geo = make_float4((float)lenp[g], (float)mass[g], (float)Jt[g], (float)Ia[g]);
    const float mm = (float)mmax[g];
    A.rq[i] = q4;
    A.geo[i] = geo;
    A.lenf[i] = geo.x;
    A.mmaxf[i] = mm;
    A.nrec[i].rq = q4;
    A.nrec[i].l = geo.x;
    A.nrec[i].inv_mmax = (float)(1.0 / (double)mm);
    A.kp0[i] = (float)kp[g];
    A.kd0[i] = (float)kd[g];
    A.wmomf[i] = (float)wmom[g];
  }
  // fruit: hang points keep their place in their segment's frame, scaled with its length
  for (int a = A.apple_off[e]; a < A.apple_off[e + 1]; ++a) {
    const int k = A.int_apple_of[a];
    const int64_t gb = s0 + A.aseg[a];
    const double fl = A.factors[4 * gb];
    const build::D3 hl = build::d3(A.hang[3 * a] * fl, A.hang[3 * a + 1] * fl, A.hang[3 * a + 2] * fl);
    const build::D3 xh = build::hang_point(Rw[gb], pw[gb], hl);
    const float4 h4 = make_float4((float)hl.x, (float)hl.y, (float)hl.z, A.ahang[k].w);
    A.ahang[k] = h4;
    A.arec[k].hang = h4;
    A.arec[k].rest = make_float4((float)xh.x, (float)xh.y, (float)xh.z, A.arec[k].rest.w);
    A.ahrest[k] = make_float4((float)xh.x, (float)xh.y, (float)xh.z, 0.f);
    A.ahrest64[3 * k] = xh.x; A.ahrest64[3 * k + 1] = xh.y; A.ahrest64[3 * k + 2] = xh.z;
  }
}

}  // namespace orchard
