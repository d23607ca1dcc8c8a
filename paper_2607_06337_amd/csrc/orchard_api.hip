// Host side of liborchard: model creation (validation, FP64 derived parameters,
// packing trees into level-synchronous packs, device layout), launches, events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/orchard.h"
#include "orchard_build.h"
#include "orchard_dev.h"
#include "orchard_rebuild.h"

namespace orchard {

template <int NT> __global__ void k_step_packs(DevModel, DevState, DevInputs, int, int);
template <int NT> __global__ void k_step_persistent(DevModel, DevState, DevInputs, int, int, int32_t*);
__global__ void k_advance(int64_t*, int32_t*, int);
__global__ void k_state_rest(DevModel, DevState, const float*);
__global__ void k_ckpt_save(DevModel, DevState, uint32_t*);
__global__ void k_ckpt_load(DevModel, DevState, const uint32_t*);
struct DevAdj {
  float2* q;
  float2* qd;
  float* ax;
  float* av;
  float* gkp;
  float* gkd;
  float* gF;
};
template <int NT> __global__ void k_adjoint_packs(DevModel, DevState, const float*, DevInputs, DevAdj, int);
template <int NT> __global__ void k_tip_fk(DevModel, const float2*);
template <int NT> __global__ void k_tip_bwd(DevModel, float2*);
__global__ void k_tip_gather(DevModel, int, const int32_t*, float*);
__global__ void k_tip_seed(DevModel, int, const int32_t*, const float*);
__global__ void k_clear_fields(DevModel, int, int);

static thread_local std::string g_err;

static orchard_status_t fail(orchard_status_t s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) return fail(ORCHARD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

orchard_status_t report_error(orchard_status_t s, const char* msg) { return fail(s, msg); }

// zero n counters (a kernel, not a memset, so that callers may capture the work)
__global__ void k_zero_i32(int32_t* p, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
}

}  // namespace orchard

using namespace orchard;

struct orchard_model_s {
  DevModel dm{};
  orchard_tuning_t tun{};
  int64_t n_env = 0, n_seg = 0, n_apple = 0;
  int32_t n_pack = 0, max_depth = 0;
  int32_t n_wide = 0;                                 // packs that take a whole workgroup
  int32_t n_main = 0;                                 // packs of the main launch (the rest: wide-tree bucket)
  size_t big_lds_bytes = 0;                           // dynamic LDS of the wide-tree launch
  hipStream_t s_big = nullptr;                        // its stream (default priority)
  hipEvent_t ev_big[2] = {nullptr, nullptr};          // fork and join of the two launches
  std::vector<int32_t> seg_map, apple_map;            // internal -> descriptor global
  std::vector<int32_t> env_seg_off, env_apple_off;    // descriptor offsets
  std::vector<int32_t> node_env_h, apple_env_h;
  std::vector<double> apple_hang_rest;                // [n_apple][3] rest hang points
  double event_band = 0;                              // |ratio - 1| below which an event is in band
  void* arena = nullptr;
  float* scr = nullptr;
  size_t an_bytes = 0;                                // dense apple-node arrays after the scratch blocks
  int32_t n_anode = 0;
  int device = 0;                                     // the device the model lives on
  int32_t apl = 13;                                   // float planes of the apple state
  RebuildArgs rb{};                                   // the on-device rebuild's view of the model
  size_t lds_bytes = 0;                               // dynamic LDS of the step kernels
  float* kp0 = nullptr;
  float* kd0 = nullptr;
  float* apple_rest = nullptr;
  int64_t bytes = 0;
  int n_cu = 256;
  int persist_blocks = 0;
  // adjoint support: two sets of recompute buffers, so that the save-mode recompute of one
  // checkpoint interval (on a second stream) overlaps the reverse sweep of the next
  int32_t adj_kmax = 0;
  float* recs = nullptr;       // [2][adj_kmax + 1][ckpt words]
  float* reps = nullptr;       // [2 adj_kmax - 1] scratch replicas (the main scratch is set 0's first)
  size_t scr_bytes = 0;
  void* work = nullptr;        // work states of both sets
  DevState ws{}, ws2{};
  hipStream_t s_aux = nullptr;                   // recompute stream (default priority)
  hipEvent_t ev_in = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr};
};

constexpr int64_t kMaxSegments = int64_t(1) << 27, kMaxApples = int64_t(1) << 26;
static_assert(sizeof(NodeRec) * kMaxSegments <= (int64_t(1) << 32) && sizeof(AppleRec) * kMaxApples <= (int64_t(1) << 32),
              "32-bit byte offsets into the per-segment and per-apple records");

// Device allocations of orchard_model_create.  Failure injection for tests of the clean-up
// paths: with ORCHARD_FAIL_ALLOC=k in the environment the k-th allocation of a create call
// (k = 1, 2, ...) fails as if the device were out of memory.
static hipError_t model_alloc(void** p, size_t bytes, int& count) {
  ++count;
  const char* e = std::getenv("ORCHARD_FAIL_ALLOC");
  if (e && std::atoi(e) == count) { *p = nullptr; return hipErrorOutOfMemory; }
  return hipMalloc(p, bytes);
}

namespace {

using build::D3;
using build::DM3;
using build::add;
using build::d3;
using build::ddot;
using build::mv;

struct Arena {
  size_t off = 0;
  struct Item { size_t off; const void* src; size_t bytes; };
  std::vector<Item> items;
  size_t put(const void* src, size_t bytes) {
    off = (off + 255) & ~size_t(255);
    items.push_back({off, src, bytes});
    size_t o = off;
    off += bytes;
    return o;
  }
};

}  // namespace

// Allow a kernel `bytes` of dynamic LDS.  The limit is a property of the kernel, shared by
// every model in the process, so it only ever rises (to the largest any model asked for).
static void allow_lds(const void* k, int bytes) {
  static std::mutex mu;
  static std::vector<std::pair<const void*, int>> granted;
  if (bytes <= 65536) return;
  std::lock_guard<std::mutex> lock(mu);
  for (auto& g : granted)
    if (g.first == k) {
      if (g.second >= bytes) return;
      g.second = bytes;
      (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
      return;
    }
  granted.push_back({k, bytes});
  (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// allow the exchange buffer's dynamic LDS and return resident workgroups per CU
template <class KP, class KQ>
static int lds_setup(KP kp, KQ kq, int nt, int lds_bytes) {
  allow_lds((const void*)kp, lds_bytes);
  allow_lds((const void*)kq, lds_bytes);
  int per_cu = 1;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kq, nt, lds_bytes);
  return per_cu;
}

extern "C" {

const char* orchard_last_error(void) { return g_err.c_str(); }
int64_t orchard_ckpt_words(orchard_model_t m);

static build::DeriveConsts derive_consts(const orchard_model_desc_t* d) {
  build::DeriveConsts c;
  c.stiffness_k0 = d->stiffness_k0;
  c.stiffness_gamma = d->stiffness_gamma;
  c.damping_cd = d->damping_cd;
  c.damping_zeta = d->damping_zeta;
  c.gnorm = std::sqrt(d->gravity[0] * d->gravity[0] + d->gravity[1] * d->gravity[1] + d->gravity[2] * d->gravity[2]);
  c.friction = d->friction_base > 0 ? 1 : 0;
  return c;
}

orchard_status_t orchard_model_create(const orchard_model_desc_t* d, const orchard_tuning_t* tuning,
                                      orchard_model_t* out) {
  g_err.clear();
  if (!d || !out) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (d->n_env <= 0 || !d->seg_offset || !d->seg_parent || !d->seg_rest_quat || !d->seg_length || !d->seg_radius ||
      !d->seg_density || !d->seg_youngs || !d->seg_mor || !d->apple_offset)
    return fail(ORCHARD_ERR_INVALID_ARG, "missing descriptor array");
  if (!(d->dt > 0) || !(d->tether_k > 0) || d->n_break < 1 || d->n_pull < 1 || d->n_tension < 1 ||
      !(d->tension_factor > 0) || !(d->v_cap > 0) || !(d->react_max_factor > 0) || d->wrench_fraction < 0 ||
      d->wrench_fraction > 1)
    return fail(ORCHARD_ERR_INVALID_ARG, "step constant out of range");
  if (d->stiffness_k0 < 0 || (d->stiffness_k0 > 0 && !(d->stiffness_gamma > 0)) ||
      (d->fruit_dof != 0 && d->fruit_dof != 3 && d->fruit_dof != 6))
    return fail(ORCHARD_ERR_INVALID_ARG, "variant out of range (stiffness_k0 >= 0, stiffness_gamma > 0, fruit_dof 0, 3 or 6)");
  if (d->drag_lin < 0 || d->drag_ang < 0 || d->drag_snapped < 0 || d->friction_base < 0 || d->friction_growth < 0 ||
      d->friction_ramp_time < 0 || d->friction_speed < 0 || d->fade_speed < 0 || d->brake_rate < 0 ||
      (d->friction_base > 0 && !(d->friction_speed > 0)))
    return fail(ORCHARD_ERR_INVALID_ARG, "extra out of range (all >= 0; friction needs friction_speed > 0)");
  if (!(d->event_band >= 0) || !std::isfinite(d->event_band))
    return fail(ORCHARD_ERR_INVALID_ARG, "event_band must be finite and >= 0");
  orchard_tuning_t tun{128, 1.0f, 1, 0, 0, 128, 0, 0, 0};
  if (tuning) tun = *tuning;
  if (tun.lds_width < 0 || tun.lds_width > tun.threads)
    return fail(ORCHARD_ERR_INVALID_ARG, "tuning.lds_width must be in [0, threads]");
  if (tun.wave_width < 0 || tun.wave_width > 64)
    return fail(ORCHARD_ERR_INVALID_ARG, "tuning.wave_width must be in [0, 64]");
  if (tun.big_threads != 0 && tun.big_threads != 256 && tun.big_threads != 512)
    return fail(ORCHARD_ERR_INVALID_ARG, "tuning.big_threads must be 0, 256 or 512");
  if (tun.adjoint_ckpt_max < 0) return fail(ORCHARD_ERR_INVALID_ARG, "tuning.adjoint_ckpt_max < 0");
  if (tun.threads != 64 && tun.threads != 128 && tun.threads != 256 && tun.threads != 512)
    return fail(ORCHARD_ERR_INVALID_ARG, "tuning.threads must be 64, 128, 256 or 512");
  if (tun.steps_per_launch < 1) tun.steps_per_launch = 1;

  const int B = d->n_env;
  if (d->seg_offset[0] != 0 || d->apple_offset[0] != 0) return fail(ORCHARD_ERR_INVALID_ARG, "offsets must start at 0");
  for (int e = 0; e < B; ++e)
    if (d->seg_offset[e + 1] <= d->seg_offset[e] || d->apple_offset[e + 1] < d->apple_offset[e])
      return fail(ORCHARD_ERR_INVALID_TOPOLOGY, "env " + std::to_string(e) + ": empty tree or decreasing offsets");
  const int64_t NS = d->seg_offset[B], NA = d->apple_offset[B];
  // the kernels form byte offsets into per-node and per-apple arrays in 32 bits: the largest
  // record is 32 bytes per segment and 64 bytes per apple
  if (NS > kMaxSegments || NA > kMaxApples)
    return fail(ORCHARD_ERR_INVALID_ARG, "batch too large (at most 2^27 segments and 2^26 apples)");
  if (NA > 0 && (!d->apple_seg || !d->apple_hang || !d->apple_mass || !d->apple_radius || !d->apple_detach))
    return fail(ORCHARD_ERR_INVALID_ARG, "missing apple array");

  // ---- validation and FP64 derived parameters ----
  std::vector<double> mass(NS), Jt(NS), Iax(NS), kp(NS), mmax(NS), kd(NS), wmom(NS, 0.0), qn(4 * NS);
  std::vector<DM3> Rw(NS);
  std::vector<D3> pw(NS);
  std::vector<int32_t> depth(NS);
  const build::DeriveConsts dc = derive_consts(d);
  std::vector<double> tmp;
  for (int e = 0; e < B; ++e) {
    const int s0 = d->seg_offset[e], s1 = d->seg_offset[e + 1];
    for (int g = s0; g < s1; ++g) {
      const int i = g - s0, p = d->seg_parent[g];
      if (p >= i || p < -1)
        return fail(ORCHARD_ERR_INVALID_TOPOLOGY, "env " + std::to_string(e) + " segment " + std::to_string(i) + ": parent must be -1 or < index");
      const double l = d->seg_length[g], r = d->seg_radius[g], rho = d->seg_density[g];
      if (!(l > 0) || !(r > 0) || !(rho > 0) || !(d->seg_youngs[g] > 0) || !(d->seg_mor[g] > 0) || !std::isfinite(l) || !std::isfinite(r))
        return fail(ORCHARD_ERR_INVALID_TOPOLOGY, "env " + std::to_string(e) + " segment " + std::to_string(i) + ": non-positive size or material");
      const double* q = d->seg_rest_quat + 4 * (int64_t)g;
      const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      if (!(std::fabs(nq - 1.0) <= 1e-6)) return fail(ORCHARD_ERR_INVALID_TOPOLOGY, "rest quaternion not unit");
    }
    tmp.resize(10 * (size_t)(s1 - s0));
    const build::DeriveIO io{s1 - s0, d->seg_parent + s0, d->seg_rest_quat + 4 * (int64_t)s0, d->seg_length + s0,
                             d->seg_radius + s0, d->seg_density + s0, d->seg_youngs + s0, d->seg_mor + s0,
                             mass.data() + s0, Jt.data() + s0, Iax.data() + s0, kp.data() + s0, mmax.data() + s0,
                             kd.data() + s0, wmom.data() + s0, qn.data() + 4 * (int64_t)s0, Rw.data() + s0,
                             pw.data() + s0, depth.data() + s0, tmp.data()};
    build::derive_tree(dc, io);
  }
  std::vector<float> arest(3 * NA);
  std::vector<float4> ahang_h(NA), apar_h(NA), ahrest_h(NA);
  std::vector<int32_t> aseg_g(NA);
  for (int e = 0; e < B; ++e) {
    const int s0 = d->seg_offset[e], S = d->seg_offset[e + 1] - s0;
    for (int a = d->apple_offset[e]; a < d->apple_offset[e + 1]; ++a) {
      const int b = d->apple_seg[a];
      if (b < 0 || b >= S) return fail(ORCHARD_ERR_INVALID_TOPOLOGY, "apple_seg out of range");
      if (!(d->apple_mass[a] > 0) || !(d->apple_detach[a] > 0)) return fail(ORCHARD_ERR_INVALID_ARG, "apple mass / detach force must be > 0");
      aseg_g[a] = s0 + b;
    }
  }

  // ---- per-tree breadth-first order and level widths ----
  std::vector<std::vector<int32_t>> bfs(B);     // descriptor global indices in BFS order
  std::vector<std::vector<int32_t>> lvlw(B);    // nodes per level
  int32_t maxd = 0;
  for (int e = 0; e < B; ++e) {
    const int s0 = d->seg_offset[e], S = d->seg_offset[e + 1] - s0;
    std::vector<int32_t> cnt(S + 1, 0);
    for (int i = 0; i < S; ++i) if (d->seg_parent[s0 + i] >= 0) cnt[d->seg_parent[s0 + i] + 1]++;
    for (int i = 0; i < S; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> kids(cnt[S]), fill(cnt.begin(), cnt.end() - 1);
    for (int i = 0; i < S; ++i) { const int p = d->seg_parent[s0 + i]; if (p >= 0) kids[fill[p]++] = i; }
    std::vector<int32_t>& order = bfs[e];
    order.reserve(S);
    for (int i = 0; i < S; ++i) if (d->seg_parent[s0 + i] < 0) order.push_back(i);
    for (size_t k = 0; k < order.size(); ++k) {
      const int i = order[k];
      for (int c = cnt[i]; c < cnt[i + 1]; ++c) order.push_back(kids[c]);
    }
    int dmax = 0;
    for (int i = 0; i < S; ++i) dmax = std::max(dmax, depth[s0 + i]);
    lvlw[e].assign(dmax + 1, 0);
    for (int i = 0; i < S; ++i) lvlw[e][depth[s0 + i]]++;
    for (int& i : order) i += s0;
    maxd = std::max(maxd, dmax + 1);
  }

  // ---- packs: several trees share one workgroup ----
  // packs[p] lists (tree, level offset): tree t placed at offset o occupies the pack's
  // levels o .. o + depth_t - 1.  Levels of different trees never depend on each other,
  // so a pack may run different depths of different trees side by side.
  // Size buckets: with wave_width > 0 (and no persistent queue) a tree whose widest level
  // has at most wave_width nodes goes to a wave pack, which one wavefront walks alone
  // with no workgroup barrier; the other trees go to workgroup-wide packs.
  std::vector<std::vector<std::pair<int32_t, int32_t>>> packs;
  // With big_threads > lds_width (and no persistent queue) a tree whose widest level does
  // not fit the main launch's LDS exchange but fits big_threads nodes goes to the wide-tree
  // bucket: packs of big_threads work-items and an LDS exchange of big_threads slots, run
  // by a launch of their own on a second stream, concurrently with the main launch.
  std::vector<int32_t> tree_ids;   // trees of the workgroup-wide packs
  std::vector<int32_t> wave_trees;  // trees of the wave packs
  std::vector<int32_t> big_trees;   // trees of the wide-tree bucket
  std::vector<char> in_wave(B, 0), in_big(B, 0);
  const bool waves_on = tun.wave_width > 0 && !tun.persistent;
  const bool big_on = tun.big_threads > tun.lds_width && tun.lds_width > 0 && !tun.persistent;
  for (int e = 0; e < B; ++e) {
    const int64_t wm = *std::max_element(lvlw[e].begin(), lvlw[e].end());
    in_wave[e] = waves_on && wm <= tun.wave_width;
    in_big[e] = big_on && wm > tun.lds_width && wm <= tun.big_threads;
    (in_wave[e] ? wave_trees : in_big[e] ? big_trees : tree_ids).push_back(e);
  }
  // trees of similar depth, about fill * nt * depth nodes per pack; with w > 0 a pack also
  // closes before one of its levels would exceed w nodes (a tree wider than w gets a pack
  // of its own that exchanges through global scratch)
  auto depth_packs = [&](const std::vector<int32_t>& ids, int nt, int64_t w, float fill) {
    std::vector<int32_t> tord = ids;
    std::stable_sort(tord.begin(), tord.end(), [&](int a, int b) {
      if (lvlw[a].size() != lvlw[b].size()) return lvlw[a].size() > lvlw[b].size();
      return d->seg_offset[a + 1] - d->seg_offset[a] > d->seg_offset[b + 1] - d->seg_offset[b];
    });
    std::vector<std::pair<int32_t, int32_t>> cur;
    std::vector<int64_t> curw;
    int64_t cur_nodes = 0;
    size_t cur_depth = 0;
    for (int t : tord) {
      const int64_t St = d->seg_offset[t + 1] - d->seg_offset[t];
      const size_t dt = lvlw[t].size();
      bool wide = false;
      if (w > 0)
        for (size_t l = 0; l < dt && l < curw.size(); ++l) wide = wide || curw[l] + lvlw[t][l] > w;
      if (!cur.empty() && (fill <= 0.f || cur_nodes + St > (int64_t)(fill * nt * cur_depth) ||
                           dt * 10 < cur_depth * 7 || wide)) {
        packs.push_back(cur);
        cur.clear();
        curw.clear();
        cur_nodes = 0;
      }
      if (cur.empty()) cur_depth = dt;
      cur.push_back({t, 0});
      cur_nodes += St;
      if (curw.size() < dt) curw.resize(dt, 0);
      for (size_t l = 0; l < dt; ++l) curw[l] += lvlw[t][l];
    }
    if (!cur.empty()) packs.push_back(cur);
  };
  const int64_t W = tun.lds_width;
  if (W > 0 && tun.pack_fill > 0.f && tun.pack_skew) {
    // depth-offset first fit.  A pack is a strip of V levels of at most W
    // nodes (V = pack_fill x the deepest tree); trees, largest first, go to the first of
    // the last few open packs and the lowest offset where every level still fits, so
    // the wide middle of one tree sits beside the narrow ends of others.  A tree wider
    // than W gets a pack of its own that exchanges through global scratch.
    const int V = std::max<int>(maxd, (int)std::ceil(tun.pack_fill * maxd));
    std::vector<int32_t> sord(B);
    std::iota(sord.begin(), sord.end(), 0);
    std::stable_sort(sord.begin(), sord.end(), [&](int a, int b) {
      return d->seg_offset[a + 1] - d->seg_offset[a] > d->seg_offset[b + 1] - d->seg_offset[b];
    });
    std::vector<std::vector<int64_t>> pw;  // level widths of the open strips
    std::vector<size_t> strip_pack;        // strip -> pack index
    const int K = 16;
    for (int t : sord) {
      if (in_wave[t] || in_big[t]) continue;
      const auto& wt = lvlw[t];
      const int Dt = (int)wt.size();
      const int64_t wmax_t = *std::max_element(wt.begin(), wt.end());
      if (wmax_t > W) { packs.push_back({{t, 0}}); continue; }
      bool placed = false;
      for (int k = (int)pw.size() - 1; k >= 0 && k >= (int)pw.size() - K && !placed; --k) {
        auto& w = pw[k];
        for (int off = 0; off + Dt <= V && !placed; ++off) {
          bool ok = true;
          for (int l = 0; l < Dt && ok; ++l) ok = w[off + l] + wt[l] <= W;
          if (ok) {
            for (int l = 0; l < Dt; ++l) w[off + l] += wt[l];
            packs[strip_pack[k]].push_back({t, off});
            placed = true;
          }
        }
      }
      if (!placed) {
        pw.emplace_back(V, 0);
        for (int l = 0; l < Dt; ++l) pw.back()[l] += wt[l];
        strip_pack.push_back(packs.size());
        packs.push_back({{t, 0}});
      }
    }
  } else {
    depth_packs(tree_ids, tun.threads, W, tun.pack_fill);
  }
  const size_t n_wide = packs.size();
  depth_packs(wave_trees, 64, tun.wave_width, tun.pack_fill);
  const size_t n_main = packs.size();
  depth_packs(big_trees, tun.big_threads, tun.big_threads, tun.pack_fill);
  const int NT = tun.threads;
  // level widths of every pack
  std::vector<std::vector<int64_t>> packw(packs.size());
  for (size_t p = 0; p < packs.size(); ++p) {
    size_t L = 0;
    for (auto& to : packs[p]) L = std::max(L, (size_t)to.second + lvlw[to.first].size());
    packw[p].assign(L, 0);
    for (auto& to : packs[p])
      for (size_t l = 0; l < lvlw[to.first].size(); ++l) packw[p][to.second + l] += lvlw[to.first][l];
  }
  // longest-processing-time order.  Estimated cost of a pack step (in us, from per-pack
  // wall-clock stamps on the 8192-tree batch: a least-squares fit over 1437 packs):
  // 6.67 per level sweep of the three passes (ceil(width / NT) sweeps per level), 3.41 per
  // 256 nodes and 7.74 per 256 apples.
  std::vector<double> pcost(packs.size());
  for (size_t p = 0; p < packs.size(); ++p) {
    int64_t sweeps = 0, nodes = 0, apples = 0;
    const int nt = p < n_wide ? NT : p < n_main ? 64 : tun.big_threads;
    for (int64_t w : packw[p]) sweeps += (w + nt - 1) / nt;
    for (auto& to : packs[p]) {
      nodes += d->seg_offset[to.first + 1] - d->seg_offset[to.first];
      apples += d->apple_offset[to.first + 1] - d->apple_offset[to.first];
    }
    pcost[p] = 6.67 * (double)sweeps + 3.41 * (double)nodes / 256.0 + 7.74 * (double)apples / 256.0;
  }
  // workgroup-wide packs first, then the wave packs (threads / 64 consecutive ones share a
  // workgroup), then the wide-tree bucket, each in longest-processing-time order
  std::vector<int32_t> pord(packs.size());
  std::iota(pord.begin(), pord.end(), 0);
  auto by_cost = [&](int a, int b) { return pcost[a] > pcost[b]; };
  std::stable_sort(pord.begin(), pord.begin() + n_wide, by_cost);
  std::stable_sort(pord.begin() + n_wide, pord.begin() + n_main, by_cost);
  std::stable_sort(pord.begin() + n_main, pord.end(), by_cost);

  // ---- internal order ----
  std::vector<int32_t> seg_map;  seg_map.reserve(NS);
  std::vector<int32_t> pack_node, pack_lvl, lvl_off, pack_wmax;
  std::vector<int32_t> int_of(NS, -1);
  int n_lds_packs = 0;
  for (int pi : pord) {
    const auto& P = packs[pi];
    pack_node.push_back((int32_t)seg_map.size());
    pack_lvl.push_back((int32_t)lvl_off.size());
    const size_t L = packw[pi].size();
    const int64_t wmax = *std::max_element(packw[pi].begin(), packw[pi].end());
    const int fits = tun.lds_width > 0 && wmax <= tun.lds_width;
    pack_wmax.push_back((int32_t)wmax);
    n_lds_packs += fits;
    std::vector<size_t> pos(P.size(), 0);
    for (size_t l = 0; l < L; ++l) {
      lvl_off.push_back((int32_t)seg_map.size());
      for (size_t k = 0; k < P.size(); ++k) {
        const int t = P[k].first, dl = (int)l - P[k].second;
        const auto& ord = bfs[t];
        while (dl >= 0 && pos[k] < ord.size() && depth[ord[pos[k]]] == dl) {
          int_of[ord[pos[k]]] = (int32_t)seg_map.size();
          seg_map.push_back(ord[pos[k]]);
          pos[k]++;
        }
      }
    }
    lvl_off.push_back((int32_t)seg_map.size());
  }
  pack_node.push_back((int32_t)seg_map.size());
  pack_lvl.push_back((int32_t)lvl_off.size());

  std::vector<int32_t> par_i(NS), child_i(NS), nchild_i(NS, 0), env_i(NS), orig_i(NS);
  std::vector<float4> rq(NS), geo(NS);
  std::vector<float> seglen(NS);
  std::vector<float> mmax_f(NS), kp_f(NS), kd_f(NS), wmom_f(NS);
  std::vector<int32_t> env_of_g(NS);
  for (int e = 0; e < B; ++e)
    for (int g = d->seg_offset[e]; g < d->seg_offset[e + 1]; ++g) env_of_g[g] = e;
  for (int64_t i = 0; i < NS; ++i) {
    const int g = seg_map[i], e = env_of_g[g], s0 = d->seg_offset[e], p = d->seg_parent[g];
    par_i[i] = p < 0 ? -1 : int_of[s0 + p];
    child_i[i] = (int32_t)NS;  // no children marker, replaced below
    env_i[i] = e;
    orig_i[i] = g - s0;
    const double* q = qn.data() + 4 * (int64_t)g;
    rq[i] = make_float4((float)q[0], (float)q[1], (float)q[2], (float)q[3]);
    geo[i] = make_float4((float)d->seg_length[g], (float)mass[g], (float)Jt[g], (float)Iax[g]);
    seglen[i] = geo[i].x;
    mmax_f[i] = (float)mmax[g];
    kp_f[i] = (float)kp[g];
    kd_f[i] = (float)kd[g];
    wmom_f[i] = (float)wmom[g];
  }
  for (int64_t i = NS - 1; i >= 0; --i) {
    const int p = par_i[i];
    if (p >= 0) { child_i[p] = (int32_t)i; nchild_i[p]++; }
  }
  for (int64_t i = 0; i < NS; ++i) if (nchild_i[i] == 0) child_i[i] = 0;
  // apples sorted by internal node
  std::vector<int32_t> aord(NA);
  std::iota(aord.begin(), aord.end(), 0);
  std::stable_sort(aord.begin(), aord.end(), [&](int a, int b) { return int_of[aseg_g[a]] < int_of[aseg_g[b]]; });
  std::vector<int32_t> apple_beg(NS + 1, 0), apple_env(NA);
  std::vector<double> ahang_rest(3 * NA);
  for (int64_t k = 0; k < NA; ++k) {
    const int a = aord[k], g = aseg_g[a], e = env_of_g[g];
    apple_beg[int_of[g] + 1]++;
    const double ma = d->apple_mass[a];
    ahang_h[k] = make_float4((float)d->apple_hang[3 * a], (float)d->apple_hang[3 * a + 1], (float)d->apple_hang[3 * a + 2], (float)ma);
    apar_h[k] = make_float4((float)d->apple_detach[a], (float)(2.0 * d->tether_zeta * std::sqrt(d->tether_k * ma)),
                            (float)(d->react_max_factor * d->apple_detach[a]), 0.f);
    const D3 hl = d3(d->apple_hang[3 * a], d->apple_hang[3 * a + 1], d->apple_hang[3 * a + 2]);
    // attached apples store their stretch from the hang point (plus h v); at rest the
    // apple hangs m |g| / k_s below it
    const D3 xh0 = build::hang_point(Rw[g], pw[g], hl);
    ahang_rest[3 * k] = xh0.x; ahang_rest[3 * k + 1] = xh0.y; ahang_rest[3 * k + 2] = xh0.z;
    ahrest_h[k] = make_float4((float)xh0.x, (float)xh0.y, (float)xh0.z, 0.f);
    arest[k] = (float)(ma / d->tether_k * d->gravity[0]);
    arest[NA + k] = (float)(ma / d->tether_k * d->gravity[1]);
    arest[2 * NA + k] = (float)(ma / d->tether_k * d->gravity[2]);
    apple_env[k] = e;
  }
  for (int64_t i = 0; i < NS; ++i) apple_beg[i + 1] += apple_beg[i];

  // ---- forward-step records ----
  if (NS > (1LL << 25) || NA > (1LL << 25))
    return fail(ORCHARD_ERR_INVALID_ARG, "at most 2^25 segments and 2^25 apples per model (32-bit offsets)");
  std::vector<NodeRec> nrec(NS);
  std::vector<int4> ntopo(NS);
  std::vector<uint64_t> hkey(NS);
  std::vector<int32_t> anode(NS, -1);  // apple-node index, in node order
  int32_t n_anode = 0;
  for (int64_t i = 0; i < NS; ++i)
    if (apple_beg[i + 1] > apple_beg[i]) anode[i] = n_anode++;
  for (int64_t i = 0; i < NS; ++i) {
    const int napp = apple_beg[i + 1] - apple_beg[i];
    if (nchild_i[i] > 0xFFFF || napp > 0xFFFF)
      return fail(ORCHARD_ERR_INVALID_TOPOLOGY, "a segment with more than 65535 children or apples");
    const float inv_mmax = (float)(1.0 / (double)mmax_f[i]);
    hkey[i] = rng_node_key(d->rng_seed, (uint64_t)env_i[i], (uint64_t)orig_i[i]);
    nrec[i].rq = rq[i];
    nrec[i].l = geo[i].x;
    nrec[i].inv_mmax = inv_mmax;
    nrec[i].par = par_i[i];
    nrec[i].anode = anode[i];
    ntopo[i] = make_int4(env_i[i], child_i[i], nchild_i[i] | (napp << 16), anode[i]);
  }
  std::vector<AppleRec> arec(NA);
  for (int64_t k = 0; k < NA; ++k) {
    const int a = aord[k];
    const double fdet = d->apple_detach[a], ma = d->apple_mass[a];
    arec[k].hang = ahang_h[k];
    arec[k].par = make_float4((float)(1.0 / fdet), apar_h[k].y, apar_h[k].z, (float)(1.0 / (d->tension_factor * fdet)));
    arec[k].rest = make_float4(ahrest_h[k].x, ahrest_h[k].y, ahrest_h[k].z, (float)(d->dt / ma));
    const int node = int_of[aseg_g[a]];
    arec[k].link = make_int4(node, apple_env[k], (int)(k == apple_beg[node]), anode[node]);
  }
  std::vector<int32_t> pack_apl(pack_node.size());
  for (size_t p = 0; p + 1 < pack_node.size(); ++p) pack_apl[p] = apple_beg[pack_node[p]];
  pack_apl.back() = (int32_t)NA;

  // ---- device layout ----
  orchard_model_s* M = new orchard_model_s();
  M->tun = tun;
  M->n_env = B; M->n_seg = NS; M->n_apple = NA;
  M->n_pack = (int32_t)packs.size();
  M->n_wide = (int32_t)n_wide;
  M->n_main = (int32_t)n_main;
  M->max_depth = maxd;
  M->seg_map = seg_map;
  M->apple_map = aord;
  M->env_seg_off.assign(d->seg_offset, d->seg_offset + B + 1);
  M->env_apple_off.assign(d->apple_offset, d->apple_offset + B + 1);
  M->node_env_h = env_i;
  M->apple_env_h = apple_env;
  M->apple_hang_rest = ahang_rest;
  M->event_band = d->event_band;
  const int32_t zero = 0;
  Arena ar;
  size_t o_pn = ar.put(pack_node.data(), pack_node.size() * 4), o_pl = ar.put(pack_lvl.data(), pack_lvl.size() * 4),
         o_lo = ar.put(lvl_off.data(), lvl_off.size() * 4), o_par = ar.put(par_i.data(), NS * 4),
         o_ch = ar.put(child_i.data(), NS * 4), o_nc = ar.put(nchild_i.data(), NS * 4), o_env = ar.put(env_i.data(), NS * 4),
         o_or = ar.put(orig_i.data(), NS * 4), o_ab = ar.put(apple_beg.data(), (NS + 1) * 4),
         o_rq = ar.put(rq.data(), NS * 16), o_geo = ar.put(geo.data(), NS * 16), o_mm = ar.put(mmax_f.data(), NS * 4),
         o_ah = ar.put(ahang_h.data(), NA * 16), o_ap = ar.put(apar_h.data(), NA * 16),
         o_kp = ar.put(kp_f.data(), NS * 4), o_kd = ar.put(kd_f.data(), NS * 4), o_ar = ar.put(arest.data(), 3 * NA * 4),
         o_hr = ar.put(ahrest_h.data(), NA * 16), o_pd = ar.put(pack_wmax.data(), pack_wmax.size() * 4),
         o_nr = ar.put(nrec.data(), NS * sizeof(NodeRec)), o_ar2 = ar.put(arec.data(), NA * sizeof(AppleRec)),
         o_hk = ar.put(hkey.data(), NS * 8), o_pa = ar.put(pack_apl.data(), pack_apl.size() * 4),
         o_nt = ar.put(ntopo.data(), NS * 16), o_len = ar.put(seglen.data(), NS * 4),
         o_wm = ar.put(wmom_f.data(), NS * 4),
         o_q = ar.put(&zero, 4 * 16);
  // the extras' constants; their friction-scale pointer is set once the arena exists
  ExtraConsts xc_h{(float)d->drag_lin, (float)d->drag_ang, (float)d->drag_snapped, (float)d->friction_base,
                   (float)d->friction_growth,
                   d->friction_ramp_time > 0 ? (float)(1.0 / d->friction_ramp_time) : -1.f,  // < 0: no ramp
                   (float)d->friction_speed, (float)d->fade_speed, (float)d->brake_rate, nullptr};
  const size_t o_xc = ar.put(&xc_h, sizeof(ExtraConsts));
  // the descriptor as given (descriptor order) and the order maps, for the on-device rebuild
  std::vector<int32_t> int_apple_of(NA);
  for (int64_t k = 0; k < NA; ++k) int_apple_of[aord[k]] = (int32_t)k;
  const size_t o_bso = ar.put(d->seg_offset, (B + 1) * 4), o_bpar = ar.put(d->seg_parent, NS * 4),
               o_bq = ar.put(d->seg_rest_quat, NS * 32), o_bl = ar.put(d->seg_length, NS * 8),
               o_br = ar.put(d->seg_radius, NS * 8), o_brho = ar.put(d->seg_density, NS * 8),
               o_bE = ar.put(d->seg_youngs, NS * 8), o_bmor = ar.put(d->seg_mor, NS * 8),
               o_bao = ar.put(d->apple_offset, (B + 1) * 4), o_bas = ar.put(d->apple_seg, NA * 4),
               o_bh = ar.put(d->apple_hang, NA * 24), o_io = ar.put(int_of.data(), NS * 4),
               o_iao = ar.put(int_apple_of.data(), NA * 4), o_hr64 = ar.put(ahang_rest.data(), NA * 24);
  int n_alloc = 0;
  hipError_t he = model_alloc(&M->arena, ar.off + 256, n_alloc);
  if (he != hipSuccess) { delete M; return fail(ORCHARD_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(he)); }
  xc_h.wmom = (const float*)((char*)M->arena + o_wm);
  std::vector<char> zeros(64, 0);
  for (auto& it : ar.items) {
    const void* src = it.src == &zero ? zeros.data() : it.src;
    if (it.bytes) {
      he = hipMemcpy((char*)M->arena + it.off, src, it.bytes, hipMemcpyHostToDevice);
      if (he != hipSuccess) { (void)hipFree(M->arena); delete M; return fail(ORCHARD_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(he)); }
    }
  }
  const int scr_nf = tun.adjoint_ckpt_max > 0 ? (int)N_FIELDS_ADJ : (int)N_FIELDS;
  const size_t scr_bytes = (size_t)scr_nf * (size_t)((std::max<int64_t>(NS, 1) + 63) / 64) * 64 * 4;
  // per-step scratch, then the dense data of the nodes that carry apples
  const size_t an_bytes = (size_t)std::max<int32_t>(n_anode, 1) * (K_N + E_N) * 4;
  he = model_alloc((void**)&M->scr, scr_bytes + an_bytes, n_alloc);
  M->scr_bytes = scr_bytes;
  M->an_bytes = an_bytes;
  M->n_anode = n_anode;
  if (he != hipSuccess) { (void)hipFree(M->arena); delete M; return fail(ORCHARD_ERR_OUT_OF_MEMORY, std::string("hipMalloc scratch: ") + hipGetErrorString(he)); }
  M->bytes = (int64_t)(ar.off + scr_bytes + an_bytes);
  char* base = (char*)M->arena;
  DevModel& dm = M->dm;
  dm.n_env = B; dm.n_seg = (int32_t)NS; dm.n_apple = (int32_t)NA; dm.n_pack = M->n_pack;
  dm.pack_node = (const int32_t*)(base + o_pn); dm.pack_lvl = (const int32_t*)(base + o_pl);
  dm.lvl_off = (const int32_t*)(base + o_lo); dm.par = (const int32_t*)(base + o_par);
  dm.child = (const int32_t*)(base + o_ch); dm.nchild = (const int32_t*)(base + o_nc);
  dm.env = (const int32_t*)(base + o_env); dm.orig = (const int32_t*)(base + o_or);
  dm.apple_beg = (const int32_t*)(base + o_ab); dm.rq = (const float4*)(base + o_rq);
  dm.geo = (const float4*)(base + o_geo); dm.mmax = (const float*)(base + o_mm);
  dm.ahang = (const float4*)(base + o_ah); dm.apar = (const float4*)(base + o_ap);
  dm.ahrest = (const float4*)(base + o_hr); dm.pack_wmax = (const int32_t*)(base + o_pd);
  dm.nrec = (const NodeRec*)(base + o_nr); dm.arec = (const AppleRec*)(base + o_ar2);
  dm.hkey = (const uint64_t*)(base + o_hk);
  dm.pack_apl = (const int32_t*)(base + o_pa);
  dm.ntopo = (const int4*)(base + o_nt);
  dm.len = (const float*)(base + o_len);
  dm.scr_nf = scr_nf;
  dm.lds_cap = n_lds_packs > 0 ? tun.lds_width : 0;
  dm.n_wide = M->n_wide;
  dm.pack_base = 0;
  // dynamic LDS of the step kernels: the level exchange, reused by the apple phase; a
  // workgroup of wave packs holds X_STRIDE x 64 floats per wavefront
  M->lds_bytes = std::max((size_t)dm.lds_cap * 2 * X_STRIDE, (size_t)11 * tun.threads) * 4;
  if (M->n_wide < M->n_main) M->lds_bytes = std::max(M->lds_bytes, (size_t)(tun.threads / 64) * X_STRIDE * 64 * 4);
  if (M->n_main < M->n_pack)
    M->big_lds_bytes = std::max((size_t)tun.big_threads * 2 * X_STRIDE, (size_t)11 * tun.big_threads) * 4;
  M->kp0 = (float*)(base + o_kp); M->kd0 = (float*)(base + o_kd); M->apple_rest = (float*)(base + o_ar);
  dm.queue = (int32_t*)(base + o_q);
  dm.h = (float)d->dt;
  dm.gx = (float)d->gravity[0]; dm.gy = (float)d->gravity[1]; dm.gz = (float)d->gravity[2];
  dm.ks = (float)d->tether_k; dm.alpha = (float)d->tension_factor; dm.vcap = (float)d->v_cap;
  dm.n_break = d->n_break; dm.n_pull = d->n_pull; dm.n_tension = d->n_tension;
  dm.use_rng = d->wrench_fraction > 0 ? 1 : 0;
  dm.seed = d->rng_seed;
  dm.rng_thr = (uint32_t)std::floor(d->wrench_fraction * 16777216.0);
  dm.wsig = (float)d->wrench_sigma;
  dm.apl = d->fruit_dof == 3 ? 6 : 13;
  dm.xflags = ((d->drag_lin > 0 || d->drag_ang > 0) ? X_DRAG : 0) | ((d->fade_speed > 0 || d->brake_rate > 0) ? X_RAILS : 0) |
              (d->friction_base > 0 ? X_FRIC : 0);
  dm.xc = (const ExtraConsts*)(base + o_xc);
  {
    RebuildArgs& rb = M->rb;
    rb.n_env = B; rb.n_seg = NS; rb.consts = dc;
    rb.seg_off = (const int32_t*)(base + o_bso); rb.parent = (const int32_t*)(base + o_bpar);
    rb.quat = (const double*)(base + o_bq); rb.blen = (const double*)(base + o_bl); rb.rad = (const double*)(base + o_br);
    rb.rho = (const double*)(base + o_brho); rb.E = (const double*)(base + o_bE); rb.mor = (const double*)(base + o_bmor);
    rb.apple_off = (const int32_t*)(base + o_bao); rb.aseg = (const int32_t*)(base + o_bas);
    rb.hang = (const double*)(base + o_bh); rb.int_of = (const int32_t*)(base + o_io);
    rb.int_apple_of = (const int32_t*)(base + o_iao);
    rb.rq = (float4*)(base + o_rq); rb.nrec = (NodeRec*)(base + o_nr); rb.geo = (float4*)(base + o_geo);
    rb.lenf = (float*)(base + o_len); rb.mmaxf = (float*)(base + o_mm); rb.kp0 = (float*)(base + o_kp);
    rb.kd0 = (float*)(base + o_kd); rb.wmomf = (float*)(base + o_wm); rb.ahang = (float4*)(base + o_ah);
    rb.arec = (AppleRec*)(base + o_ar2); rb.ahrest = (float4*)(base + o_hr); rb.ahrest64 = (double*)(base + o_hr64);
  }
  M->apl = dm.apl;
  dm.scr = M->scr;
  dm.asnap = (float*)((char*)M->scr + scr_bytes);
  dm.aext = dm.asnap + (size_t)std::max<int32_t>(n_anode, 1) * K_N;
  int dev = 0;
  (void)hipGetDevice(&dev);
  M->device = dev;
  (void)hipDeviceGetAttribute(&M->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  int per_cu = 1;
  const int lb = (int)M->lds_bytes;
  switch (tun.threads) {
    case 64: per_cu = lds_setup(k_step_packs<64>, k_step_persistent<64>, 64, lb); break;
    case 128: per_cu = lds_setup(k_step_packs<128>, k_step_persistent<128>, 128, lb); break;
    case 256: per_cu = lds_setup(k_step_packs<256>, k_step_persistent<256>, 256, lb); break;
    default: per_cu = lds_setup(k_step_packs<512>, k_step_persistent<512>, 512, lb); break;
  }
  M->persist_blocks = std::max(1, std::min<int>(M->n_pack, std::max(1, per_cu) * std::max(1, M->n_cu)));
  if (tun.adjoint_ckpt_max > 0) {
    const void* ka = tun.threads == 64 ? (const void*)k_adjoint_packs<64>
                     : tun.threads == 128 ? (const void*)k_adjoint_packs<128>
                     : tun.threads == 256 ? (const void*)k_adjoint_packs<256> : (const void*)k_adjoint_packs<512>;
    allow_lds(ka, lb);
  }
  if (M->n_main < M->n_pack) {
    allow_lds(tun.big_threads == 512 ? (const void*)k_step_packs<512> : (const void*)k_step_packs<256>,
              (int)M->big_lds_bytes);
    if (tun.adjoint_ckpt_max > 0)
      allow_lds(tun.big_threads == 512 ? (const void*)k_adjoint_packs<512> : (const void*)k_adjoint_packs<256>,
                (int)M->big_lds_bytes);
    if (hipStreamCreateWithFlags(&M->s_big, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&M->ev_big[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&M->ev_big[1], hipEventDisableTiming) != hipSuccess) {
      orchard_model_destroy(M);
      return fail(ORCHARD_ERR_HIP, "wide-tree stream or events");
    }
  }
  if (tun.adjoint_ckpt_max > 0) {
    const int64_t words = orchard_ckpt_words(M);
    M->adj_kmax = tun.adjoint_ckpt_max;
    const size_t rb = 2 * (size_t)(M->adj_kmax + 1) * (size_t)words * 4;
    // one scratch per step of a checkpoint interval: the backward sweep runs each step's
    // forward once, keeping what the reverse pass reads back (two sets of them)
    const size_t pb = (size_t)(2 * M->adj_kmax - 1) * M->scr_bytes;
    // work state: q, qd (float2), apple (13A), seg_evt (2S), apple_evt (4A), evt_step (S+A), status (B),
    // step; every piece starts on a 256-byte boundary
    auto r256 = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t wb = 2 * r256(8 * (size_t)NS) + r256(4 * (size_t)M->apl * NA) + r256(2 * (size_t)NS) + r256(4 * (size_t)NA) +
                      r256(4 * (size_t)(NS + NA)) + r256(4 * (size_t)B) + r256(8);
    if (model_alloc((void**)&M->recs, rb, n_alloc) != hipSuccess || model_alloc(&M->work, 2 * wb, n_alloc) != hipSuccess ||
        (pb > 0 && model_alloc((void**)&M->reps, pb, n_alloc) != hipSuccess)) {
      orchard_model_destroy(M);
      return fail(ORCHARD_ERR_OUT_OF_MEMORY, "adjoint buffers");
    }
    if (hipStreamCreateWithFlags(&M->s_aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&M->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&M->ev_rec[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&M->ev_rec[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&M->ev_adj[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&M->ev_adj[1], hipEventDisableTiming) != hipSuccess) {
      orchard_model_destroy(M);
      return fail(ORCHARD_ERR_HIP, "adjoint stream or events");
    }
    char* w = (char*)M->work;
    auto take = [&](size_t b) { char* r = w; w += (b + 255) & ~size_t(255); return r; };
    for (DevState* ws : {&M->ws, &M->ws2}) {
      ws->q = (float2*)take(8 * NS); ws->qd = (float2*)take(8 * NS); ws->apple = (float*)take(4 * (size_t)M->apl * NA);
      ws->seg_evt = (uint8_t*)take(2 * NS); ws->apple_evt = (uint8_t*)take(4 * NA);
      ws->evt_step = (int32_t*)take(4 * (NS + NA)); ws->status = (uint32_t*)take(4 * B); ws->step = (int64_t*)take(8);
    }
    M->bytes += (int64_t)(rb + 2 * wb + pb);
  }
  *out = M;
  return ORCHARD_OK;
}

void orchard_model_destroy(orchard_model_t m) {
  if (!m) return;
  if (m->recs) (void)hipFree(m->recs);
  if (m->reps) (void)hipFree(m->reps);
  if (m->work) (void)hipFree(m->work);
  for (hipEvent_t e : {m->ev_in, m->ev_rec[0], m->ev_rec[1], m->ev_adj[0], m->ev_adj[1], m->ev_big[0], m->ev_big[1]})
    if (e) (void)hipEventDestroy(e);
  if (m->s_aux) (void)hipStreamDestroy(m->s_aux);
  if (m->s_big) (void)hipStreamDestroy(m->s_big);
  if (m->arena) (void)hipFree(m->arena);
  if (m->scr) (void)hipFree(m->scr);
  delete m;
}

orchard_status_t orchard_model_layout(orchard_model_t m, orchard_layout_t* out) {
  if (!m || !out) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  out->n_env = m->n_env; out->n_seg = m->n_seg; out->n_apple = m->n_apple;
  out->n_pack = m->n_pack; out->max_depth = m->max_depth; out->scratch_bytes = m->bytes;
  out->apple_planes = m->apl;
  out->n_wave_packs = m->n_main - m->n_wide;
  out->n_big_packs = m->n_pack - m->n_main;
  out->pad = 0;
  return ORCHARD_OK;
}

orchard_status_t orchard_model_maps(orchard_model_t m, int32_t* seg_map, int32_t* apple_map) {
  if (!m) return fail(ORCHARD_ERR_INVALID_ARG, "null model");
  if (seg_map) std::copy(m->seg_map.begin(), m->seg_map.end(), seg_map);
  if (apple_map) std::copy(m->apple_map.begin(), m->apple_map.end(), apple_map);
  return ORCHARD_OK;
}

orchard_status_t orchard_model_apple_rest(orchard_model_t m, double* host_out) {
  if (!m || (!host_out && m->n_apple)) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  // the device copy is the current one (orchard_model_rebuild rewrites it)
  if (m->n_apple) {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(host_out, m->rb.ahrest64, m->n_apple * 24, hipMemcpyDeviceToHost));
  }
  return ORCHARD_OK;
}

orchard_status_t orchard_model_rebuild(orchard_model_t m, const double* seg_perturb, int32_t* rejected,
                                       orchard_stream_t stream) {
  if (!m || !seg_perturb) return fail(ORCHARD_ERR_INVALID_ARG, "null model or perturbation");
  // workspace: the model's step scratch (40 doubles per segment; it holds at least 128 floats each)
  static_assert(N_FIELDS * 4 >= 40 * 8, "the step scratch holds the rebuild's workspace");
  RebuildArgs a = m->rb;
  a.factors = seg_perturb;
  a.work = reinterpret_cast<double*>(m->scr);
  a.rejected = rejected;
  hipStream_t hs = (hipStream_t)stream;
  if (rejected) hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, hs, rejected, 1);
  hipLaunchKernelGGL(k_rebuild, dim3((m->n_env + 63) / 64), dim3(64), 0, hs, a);
  HIPCHK(hipGetLastError());
  return ORCHARD_OK;
}

orchard_status_t orchard_default_params(orchard_model_t m, float* kp, float* kd, orchard_stream_t stream) {
  if (!m) return fail(ORCHARD_ERR_INVALID_ARG, "null model");
  if (kp) HIPCHK(hipMemcpyAsync(kp, m->kp0, m->n_seg * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  if (kd) HIPCHK(hipMemcpyAsync(kd, m->kd0, m->n_seg * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return ORCHARD_OK;
}

static orchard_status_t dev_state(orchard_model_t m, const orchard_state_t* s, DevState* ds) {
  if (!s || !s->q || !s->qd || !s->seg_evt || !s->evt_step || !s->env_status || !s->step)
    return fail(ORCHARD_ERR_INVALID_ARG, "state pointer missing");
  if (m->n_apple > 0 && (!s->apple || !s->apple_evt)) return fail(ORCHARD_ERR_INVALID_ARG, "apple state pointer missing");
  ds->q = (float2*)s->q; ds->qd = (float2*)s->qd; ds->apple = s->apple; ds->seg_evt = s->seg_evt;
  ds->apple_evt = s->apple_evt; ds->evt_step = s->evt_step; ds->status = s->env_status; ds->step = s->step;
  ds->evt_ratio = s->evt_ratio;
  return ORCHARD_OK;
}

static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

orchard_status_t orchard_state_rest(orchard_model_t m, const orchard_state_t* s, orchard_stream_t stream) {
  if (!m) return fail(ORCHARD_ERR_INVALID_ARG, "null model");
  DevState ds;
  orchard_status_t st = dev_state(m, s, &ds);
  if (st) return st;
  const int64_t n = std::max<int64_t>(m->n_seg + m->n_apple, m->n_env);
  hipLaunchKernelGGL(k_state_rest, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, m->dm, ds, m->apple_rest);
  HIPCHK(hipGetLastError());
  return ORCHARD_OK;
}

int64_t orchard_ckpt_words(orchard_model_t m) {
  return 4LL * m->n_seg + (int64_t)m->apl * m->n_apple + m->n_seg + m->n_apple + m->n_seg + m->n_apple + m->n_env + 2;
}

// The adjoint's recompute and reverse pass take the wide-tree mapping when every pack is in
// that bucket (a batch of wide trees only); with packs of both kinds they run the main one.
static bool adj_big(orchard_model_t m) { return m->n_main == 0 && m->n_pack > 0; }

static orchard_status_t launch_steps(orchard_model_t m, const DevModel& dm0, const DevState& ds, const DevInputs& di,
                                     int k, int s_call, hipStream_t stream, bool save = false, float* scr = nullptr) {
  const int NT = m->tun.threads;
  const unsigned lb = (unsigned)m->lds_bytes;
  if (save) {
    // the adjoint's recompute runs every pack on a whole workgroup: in the wide-tree
    // mapping when the batch has no other packs, otherwise in the main mapping (wide
    // trees exchanging through global scratch)
    DevModel dm = dm0;
    dm.save_adj = 1;
    dm.n_wide = dm.n_pack;
    if (scr) dm.scr = scr;
    const dim3 g(m->n_pack);
    if (adj_big(m)) {
      dm.lds_cap = m->tun.big_threads;
      const unsigned lbb = (unsigned)m->big_lds_bytes;
      if (m->tun.big_threads == 512) hipLaunchKernelGGL(k_step_packs<512>, g, dim3(512), lbb, stream, dm, ds, di, k, s_call);
      else hipLaunchKernelGGL(k_step_packs<256>, g, dim3(256), lbb, stream, dm, ds, di, k, s_call);
    } else switch (NT) {
      case 64: hipLaunchKernelGGL(k_step_packs<64>, g, dim3(64), lb, stream, dm, ds, di, k, s_call); break;
      case 128: hipLaunchKernelGGL(k_step_packs<128>, g, dim3(128), lb, stream, dm, ds, di, k, s_call); break;
      case 256: hipLaunchKernelGGL(k_step_packs<256>, g, dim3(256), lb, stream, dm, ds, di, k, s_call); break;
      default: hipLaunchKernelGGL(k_step_packs<512>, g, dim3(512), lb, stream, dm, ds, di, k, s_call); break;
    }
  } else if (m->tun.persistent) {
    const dim3 g(m->persist_blocks);
    switch (NT) {
      case 64: hipLaunchKernelGGL(k_step_persistent<64>, g, dim3(64), lb, stream, dm0, ds, di, k, s_call, dm0.queue); break;
      case 128: hipLaunchKernelGGL(k_step_persistent<128>, g, dim3(128), lb, stream, dm0, ds, di, k, s_call, dm0.queue); break;
      case 256: hipLaunchKernelGGL(k_step_persistent<256>, g, dim3(256), lb, stream, dm0, ds, di, k, s_call, dm0.queue); break;
      default: hipLaunchKernelGGL(k_step_persistent<512>, g, dim3(512), lb, stream, dm0, ds, di, k, s_call, dm0.queue); break;
    }
  } else {
    // the wide-tree bucket (packs [n_main, n_pack)) and the main packs run concurrently:
    // the wide-tree launch goes first on the caller's stream, so that its workgroups (most
    // of a CU's LDS each) find free CUs, and the main launch on the model's second stream;
    // both join before the step counter advances
    const bool big = m->n_main < m->n_pack;
    hipStream_t s_main = stream;
    if (big) {
      s_main = m->s_big;
      HIPCHK(hipEventRecord(m->ev_big[0], stream));
      DevModel db = dm0;
      db.pack_base = m->n_main;
      db.n_wide = db.n_pack;
      db.lds_cap = m->tun.big_threads;
      const dim3 gb(m->n_pack - m->n_main);
      const unsigned lbb = (unsigned)m->big_lds_bytes;
      if (m->tun.big_threads == 512)
        hipLaunchKernelGGL(k_step_packs<512>, gb, dim3(512), lbb, stream, db, ds, di, k, s_call);
      else
        hipLaunchKernelGGL(k_step_packs<256>, gb, dim3(256), lbb, stream, db, ds, di, k, s_call);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamWaitEvent(s_main, m->ev_big[0], 0));
    }
    if (m->n_main > 0) {
      DevModel dmm = dm0;
      dmm.n_pack = m->n_main;
      const dim3 g(m->n_wide + (m->n_main - m->n_wide + NT / 64 - 1) / (NT / 64));
      switch (NT) {
        case 64: hipLaunchKernelGGL(k_step_packs<64>, g, dim3(64), lb, s_main, dmm, ds, di, k, s_call); break;
        case 128: hipLaunchKernelGGL(k_step_packs<128>, g, dim3(128), lb, s_main, dmm, ds, di, k, s_call); break;
        case 256: hipLaunchKernelGGL(k_step_packs<256>, g, dim3(256), lb, s_main, dmm, ds, di, k, s_call); break;
        default: hipLaunchKernelGGL(k_step_packs<512>, g, dim3(512), lb, s_main, dmm, ds, di, k, s_call); break;
      }
    }
    if (big) HIPCHK(hipEventRecord(m->ev_big[1], s_main));
    if (big) HIPCHK(hipStreamWaitEvent(stream, m->ev_big[1], 0));
  }
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, stream, ds.step, (m->tun.persistent && !save) ? dm0.queue : nullptr, k);
  HIPCHK(hipGetLastError());
  return ORCHARD_OK;
}

static orchard_status_t step_with(orchard_model_t m, const DevModel& dm, const orchard_state_t* s,
                                  const orchard_params_t* params, const orchard_inputs_t* inputs, int32_t n_steps,
                                  float* ckpt, int32_t ckpt_every, orchard_stream_t stream) {
  if (n_steps < 0) return fail(ORCHARD_ERR_INVALID_ARG, "n_steps < 0");
  if (ckpt && ckpt_every < 1) return fail(ORCHARD_ERR_INVALID_ARG, "ckpt_every must be >= 1");
  DevState ds;
  orchard_status_t st = dev_state(m, s, &ds);
  if (st) return st;
  DevInputs di{params->kp, params->kd, nullptr, 0, nullptr, 0};
  if (inputs) {
    di.wrench = inputs->body_wrench; di.wrench_stride = inputs->body_wrench_stride;
    di.aforce = inputs->apple_force; di.aforce_stride = inputs->apple_force_stride;
    if (di.wrench_stride < 0 || di.aforce_stride < 0) return fail(ORCHARD_ERR_INVALID_ARG, "negative input stride");
  }
  hipStream_t hs = (hipStream_t)stream;
  const int spl = m->tun.steps_per_launch;
  const int64_t words = orchard_ckpt_words(m);
  int s0 = 0;
  while (s0 < n_steps) {
    int k = std::min(spl, n_steps - s0);
    if (ckpt) {
      if (s0 % ckpt_every == 0) {
        hipLaunchKernelGGL(k_ckpt_save, dim3(grid_for(words)), dim3(256), 0, hs, m->dm, ds,
                           (uint32_t*)ckpt + (int64_t)(s0 / ckpt_every) * words);
        HIPCHK(hipGetLastError());
      }
      k = std::min(k, ckpt_every - s0 % ckpt_every);
    }
    st = launch_steps(m, dm, ds, di, k, s0, hs);
    if (st) return st;
    s0 += k;
  }
  return ORCHARD_OK;
}

orchard_status_t orchard_step(orchard_model_t m, const orchard_state_t* s, const orchard_params_t* params,
                              const orchard_inputs_t* inputs, int32_t n_steps, float* ckpt, int32_t ckpt_every,
                              orchard_stream_t stream) {
  if (!m || !params || !params->kp || !params->kd) return fail(ORCHARD_ERR_INVALID_ARG, "null model or params");
  return step_with(m, m->dm, s, params, inputs, n_steps, ckpt, ckpt_every, stream);
}

// ---- the step on a fixed scratch array, for callers that cannot allocate ----------------
// One array per GPU the library runs on, held until the process ends.  In host code its
// name is only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is ever passed on.
static __device__ __align__(256) float scratch[ORCHARD_STATIC_SCRATCH_BYTES / 4];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this device's scratch array (resolved on the first call per device).
static orchard_status_t scratch_address(int dev, float** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ORCHARD_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != dev) return fail(ORCHARD_ERR_INVALID_ARG, "the model's device is not the current device");
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return ORCHARD_OK;
}


orchard_status_t orchard_step_static_scratch(orchard_model_t m, const orchard_state_t* s,
                                             const orchard_params_t* params, const orchard_inputs_t* inputs,
                                             int32_t n_steps, float* ckpt, int32_t ckpt_every,
                                             orchard_stream_t stream) {
  if (!m || !params || !params->kp || !params->kd) return fail(ORCHARD_ERR_INVALID_ARG, "null model or params");
  // layout in the array: the persistent queue counter (256 bytes), the per-node scratch
  // blocks, then the dense apple-node arrays, each as the model's own scratch lays them out
  const size_t need = 256 + m->scr_bytes + m->an_bytes;
  if (need > ORCHARD_STATIC_SCRATCH_BYTES)
    return fail(ORCHARD_ERR_CAPACITY, "model needs " + std::to_string(need) + " bytes of step scratch; the static "
                                      "scratch holds " + std::to_string((size_t)ORCHARD_STATIC_SCRATCH_BYTES));
  float* base = nullptr;
  orchard_status_t st = scratch_address(m->device, &base);
  if (st) return st;
  DevModel dm = m->dm;
  dm.queue = reinterpret_cast<int32_t*>(base);
  dm.scr = base + 64;
  dm.asnap = reinterpret_cast<float*>(reinterpret_cast<char*>(dm.scr) + m->scr_bytes);
  dm.aext = dm.asnap + (size_t)std::max<int32_t>(m->n_anode, 1) * K_N;
  // the queue counter must start at zero (a kernel, not a memset, so the call can be captured)
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, (hipStream_t)stream, dm.queue, 1);
  HIPCHK(hipGetLastError());
  return step_with(m, dm, s, params, inputs, n_steps, ckpt, ckpt_every, stream);
}

// load a checkpoint record written by orchard_step into the state
orchard_status_t orchard_ckpt_load(orchard_model_t m, const orchard_state_t* s, const float* rec, orchard_stream_t stream) {
  if (!m || !rec) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  DevState ds;
  orchard_status_t st = dev_state(m, s, &ds);
  if (st) return st;
  hipLaunchKernelGGL(k_ckpt_load, dim3(grid_for(orchard_ckpt_words(m))), dim3(256), 0, (hipStream_t)stream, m->dm, ds,
                     (const uint32_t*)rec);
  HIPCHK(hipGetLastError());
  return ORCHARD_OK;
}

orchard_status_t orchard_events(orchard_model_t m, const orchard_state_t* s, orchard_event_t* host_out,
                                int32_t capacity, int32_t* n_out, orchard_stream_t stream) {
  if (!m || !s || !n_out || (capacity > 0 && !host_out)) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  const int64_t NS = m->n_seg, NA = m->n_apple;
  std::vector<int32_t> steps(NS + NA);
  std::vector<uint8_t> path(NA);
  std::vector<float> ratio(NS + NA, 0.f);
  hipStream_t hs = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(steps.data(), s->evt_step, (NS + NA) * 4, hipMemcpyDeviceToHost, hs));
  if (NA) HIPCHK(hipMemcpyAsync(path.data(), s->apple_evt + 3 * NA, NA, hipMemcpyDeviceToHost, hs));
  if (s->evt_ratio) HIPCHK(hipMemcpyAsync(ratio.data(), s->evt_ratio, (NS + NA) * 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  std::vector<orchard_event_t> ev;
  auto in_band = [&](float r) { return (int32_t)(std::fabs((double)r - 1.0) < m->event_band); };
  for (int64_t i = 0; i < NS; ++i)
    if (steps[i] >= 0) {
      const int g = m->seg_map[i], e = m->node_env_h[i];
      ev.push_back({e, 1, g - m->env_seg_off[e], steps[i], ratio[i], in_band(ratio[i])});
    }
  for (int64_t a = 0; a < NA; ++a)
    if (steps[NS + a] >= 0) {
      const int g = m->apple_map[a], e = m->apple_env_h[a];
      const float r = ratio[NS + a];
      ev.push_back({e, path[a] == 2 ? 3 : 2, g - m->env_apple_off[e], steps[NS + a], r, in_band(r)});
    }
  std::sort(ev.begin(), ev.end(), [](const orchard_event_t& a, const orchard_event_t& b) {
    if (a.env != b.env) return a.env < b.env;
    if (a.step != b.step) return a.step < b.step;
    if (a.kind != b.kind) return a.kind < b.kind;
    return a.id < b.id;
  });
  *n_out = (int32_t)ev.size();
  const int32_t nw = std::min<int32_t>(capacity, (int32_t)ev.size());
  if (nw > 0) std::copy(ev.begin(), ev.begin() + nw, host_out);
  if ((int64_t)ev.size() > capacity) return fail(ORCHARD_ERR_CAPACITY, "event buffer too small");
  return ORCHARD_OK;
}

orchard_status_t orchard_status(orchard_model_t m, const orchard_state_t* s, uint32_t* host_env_status,
                                orchard_stream_t stream) {
  if (!m || !s || !host_env_status) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  hipStream_t hs = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(host_env_status, s->env_status, m->n_env * 4, hipMemcpyDeviceToHost, hs));
  HIPCHK(hipStreamSynchronize(hs));
  for (int64_t e = 0; e < m->n_env; ++e)
    if (host_env_status[e]) return fail(ORCHARD_ERR_NONFINITE, "env " + std::to_string(e) + " produced a non-finite state");
  return ORCHARD_OK;
}

orchard_status_t orchard_step_backward(orchard_model_t m, const float* ckpt, int32_t ckpt_every, int32_t n_steps,
                                       const orchard_params_t* params, const orchard_inputs_t* inputs,
                                       const orchard_adjoint_t* adj, float* grad_kp, float* grad_kd,
                                       float* grad_apple_force, orchard_stream_t stream) {
  if (!m || !ckpt || !params || !params->kp || !params->kd || !adj || !adj->q || !adj->qd || !grad_kp || !grad_kd)
    return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  if (m->n_apple > 0 && (!adj->apple_x || !adj->apple_v)) return fail(ORCHARD_ERR_INVALID_ARG, "apple adjoint missing");
  if (m->adj_kmax <= 0) return fail(ORCHARD_ERR_INVALID_ARG, "model created without adjoint support (tuning.adjoint_ckpt_max)");
  if (m->dm.xflags)
    return fail(ORCHARD_ERR_INVALID_ARG, "the adjoint does not cover drag, post-break friction or the power fade / speed brake");
  if (ckpt_every < 1 || ckpt_every > m->adj_kmax) return fail(ORCHARD_ERR_INVALID_ARG, "ckpt_every out of [1, adjoint_ckpt_max]");
  if (n_steps < 0) return fail(ORCHARD_ERR_INVALID_ARG, "n_steps < 0");
  DevInputs di{params->kp, params->kd, nullptr, 0, nullptr, 0};
  if (inputs) {
    di.wrench = inputs->body_wrench; di.wrench_stride = inputs->body_wrench_stride;
    di.aforce = inputs->apple_force; di.aforce_stride = inputs->apple_force_stride;
  }
  DevAdj X{(float2*)adj->q, (float2*)adj->qd, adj->apple_x, adj->apple_v, grad_kp, grad_kd, grad_apple_force};
  hipStream_t hs = (hipStream_t)stream;
  const int64_t words = orchard_ckpt_words(m);
  const int NT = m->tun.threads;
  const unsigned lb = (unsigned)m->lds_bytes;  // the adjoint kernel shares the step kernels' exchange layout
  const int nseg = (n_steps + ckpt_every - 1) / ckpt_every;
  // recompute set s (= checkpoint interval mod 2): work state, scratch copies, records
  const int K = m->adj_kmax;
  auto wstate = [&](int s) -> const DevState& { return s == 0 ? m->ws : m->ws2; };
  auto rep = [&](int s, int j) {
    const int k = s * K + j;  // copy k of the 2K; copy 0 is the main scratch
    return k == 0 ? m->scr : (float*)((char*)m->reps + (size_t)(k - 1) * m->scr_bytes);
  };
  auto rec_at = [&](int s, int j) { return (uint32_t*)m->recs + ((int64_t)s * (K + 1) + j) * words; };
  // forward sweep of interval sg: every step once, in save mode into its own scratch;
  // records hold the state before each step and after the last
  auto recompute = [&](int sg, hipStream_t st) -> orchard_status_t {
    const int s = sg & 1, n0 = sg * ckpt_every, nk = std::min(ckpt_every, n_steps - n0);
    const DevState& W = wstate(s);
    hipLaunchKernelGGL(k_ckpt_load, dim3(grid_for(words)), dim3(256), 0, st, m->dm, W, (const uint32_t*)ckpt + (int64_t)sg * words);
    hipLaunchKernelGGL(k_ckpt_save, dim3(grid_for(words)), dim3(256), 0, st, m->dm, W, rec_at(s, 0));
    for (int j = 0; j < nk; ++j) {
      orchard_status_t r = launch_steps(m, m->dm, W, di, 1, n0 + j, st, true, rep(s, j));
      if (r) return r;
      hipLaunchKernelGGL(k_ckpt_save, dim3(grid_for(words)), dim3(256), 0, st, m->dm, W, rec_at(s, j + 1));
    }
    HIPCHK(hipGetLastError());
    return ORCHARD_OK;
  };
  // reverse sweep of interval sg: W holds the state after step j (event flags, step counter)
  auto reverse = [&](int sg, hipStream_t st) -> orchard_status_t {
    const int s = sg & 1, n0 = sg * ckpt_every, nk = std::min(ckpt_every, n_steps - n0);
    const DevState& W = wstate(s);
    for (int j = nk - 1; j >= 0; --j) {
      if (j < nk - 1)
        hipLaunchKernelGGL(k_ckpt_load, dim3(grid_for(words)), dim3(256), 0, st, m->dm, W, (const uint32_t*)rec_at(s, j + 1));
      DevModel dm = m->dm;
      dm.scr = rep(s, j);
      const float* rec = (const float*)rec_at(s, j);
      const dim3 g(m->n_pack);
      if (adj_big(m)) {
        dm.lds_cap = m->tun.big_threads;
        const unsigned lbb = (unsigned)m->big_lds_bytes;
        if (m->tun.big_threads == 512)
          hipLaunchKernelGGL(k_adjoint_packs<512>, g, dim3(512), lbb, st, dm, W, rec, di, X, n0 + j);
        else
          hipLaunchKernelGGL(k_adjoint_packs<256>, g, dim3(256), lbb, st, dm, W, rec, di, X, n0 + j);
      } else switch (NT) {
        case 64: hipLaunchKernelGGL(k_adjoint_packs<64>, g, dim3(64), lb, st, dm, W, rec, di, X, n0 + j); break;
        case 128: hipLaunchKernelGGL(k_adjoint_packs<128>, g, dim3(128), lb, st, dm, W, rec, di, X, n0 + j); break;
        case 256: hipLaunchKernelGGL(k_adjoint_packs<256>, g, dim3(256), lb, st, dm, W, rec, di, X, n0 + j); break;
        default: hipLaunchKernelGGL(k_adjoint_packs<512>, g, dim3(512), lb, st, dm, W, rec, di, X, n0 + j); break;
      }
      HIPCHK(hipGetLastError());
    }
    return ORCHARD_OK;
  };
  if (nseg == 0) return ORCHARD_OK;
  // The recomputes run in order on the second stream, the reverse sweeps in order on the
  // caller's: interval sg - 1 is recomputed while interval sg is reversed.  Reverse sweep
  // sg waits for its recompute; recompute sg - 1 reuses the buffers of interval sg + 1,
  // so it waits for that reverse sweep.
  hipStream_t sa = m->s_aux;
  HIPCHK(hipEventRecord(m->ev_in, hs));
  HIPCHK(hipStreamWaitEvent(sa, m->ev_in, 0));
  orchard_status_t r = recompute(nseg - 1, sa);
  if (r) return r;
  HIPCHK(hipEventRecord(m->ev_rec[(nseg - 1) & 1], sa));
  for (int sg = nseg - 1; sg >= 0; --sg) {
    if (sg >= 1) {
      if (sg + 1 <= nseg - 1) HIPCHK(hipStreamWaitEvent(sa, m->ev_adj[(sg + 1) & 1], 0));
      r = recompute(sg - 1, sa);
      if (r) return r;
      HIPCHK(hipEventRecord(m->ev_rec[(sg - 1) & 1], sa));
    }
    HIPCHK(hipStreamWaitEvent(hs, m->ev_rec[sg & 1], 0));
    r = reverse(sg, hs);
    if (r) return r;
    HIPCHK(hipEventRecord(m->ev_adj[sg & 1], hs));
  }
  return ORCHARD_OK;
}

static orchard_status_t tip_fk(orchard_model_t m, const float* q, hipStream_t hs) {
  const dim3 g(m->n_pack);
  switch (m->tun.threads) {
    case 64: hipLaunchKernelGGL(k_tip_fk<64>, g, dim3(64), 0, hs, m->dm, (const float2*)q); break;
    case 128: hipLaunchKernelGGL(k_tip_fk<128>, g, dim3(128), 0, hs, m->dm, (const float2*)q); break;
    case 256: hipLaunchKernelGGL(k_tip_fk<256>, g, dim3(256), 0, hs, m->dm, (const float2*)q); break;
    default: hipLaunchKernelGGL(k_tip_fk<512>, g, dim3(512), 0, hs, m->dm, (const float2*)q); break;
  }
  HIPCHK(hipGetLastError());
  return ORCHARD_OK;
}

orchard_status_t orchard_tips(orchard_model_t m, const float* q, int32_t n_tips, const int32_t* node, float* out,
                              orchard_stream_t stream) {
  if (!m || !q || (n_tips > 0 && (!node || !out)) || n_tips < 0) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  // the tip kernels keep their fields among the adjoint's scratch fields
  if (m->dm.scr_nf < N_FIELDS_ADJ) return fail(ORCHARD_ERR_INVALID_ARG, "model created without adjoint support (tuning.adjoint_ckpt_max)");
  hipStream_t hs = (hipStream_t)stream;
  orchard_status_t st = tip_fk(m, q, hs);
  if (st) return st;
  if (n_tips) hipLaunchKernelGGL(k_tip_gather, dim3(grid_for(n_tips)), dim3(256), 0, hs, m->dm, n_tips, node, out);
  HIPCHK(hipGetLastError());
  return ORCHARD_OK;
}

orchard_status_t orchard_tips_backward(orchard_model_t m, const float* q, int32_t n_tips, const int32_t* node,
                                       const float* grad_out, float* grad_q, orchard_stream_t stream) {
  if (!m || !q || !grad_q || n_tips < 0 || (n_tips > 0 && (!node || !grad_out))) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  if (m->dm.scr_nf < N_FIELDS_ADJ) return fail(ORCHARD_ERR_INVALID_ARG, "model created without adjoint support (tuning.adjoint_ckpt_max)");
  hipStream_t hs = (hipStream_t)stream;
  orchard_status_t st = tip_fk(m, q, hs);
  if (st) return st;
  hipLaunchKernelGGL(k_clear_fields, dim3(grid_for(3 * m->n_seg)), dim3(256), 0, hs, m->dm, (int)F_LPA, 3);
  if (n_tips) hipLaunchKernelGGL(k_tip_seed, dim3(1), dim3(64), 0, hs, m->dm, n_tips, node, grad_out);
  const dim3 g(m->n_pack);
  switch (m->tun.threads) {
    case 64: hipLaunchKernelGGL(k_tip_bwd<64>, g, dim3(64), 0, hs, m->dm, (float2*)grad_q); break;
    case 128: hipLaunchKernelGGL(k_tip_bwd<128>, g, dim3(128), 0, hs, m->dm, (float2*)grad_q); break;
    case 256: hipLaunchKernelGGL(k_tip_bwd<256>, g, dim3(256), 0, hs, m->dm, (float2*)grad_q); break;
    default: hipLaunchKernelGGL(k_tip_bwd<512>, g, dim3(512), 0, hs, m->dm, (float2*)grad_q); break;
  }
  HIPCHK(hipGetLastError());
  return ORCHARD_OK;
}


// ---- K-step graphs ----
struct orchard_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

void orchard_graph_destroy(orchard_graph_t g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

orchard_status_t orchard_graph_create(orchard_model_t m, const orchard_state_t* s, const orchard_params_t* params,
                                      const orchard_inputs_t* inputs, int32_t n_steps, orchard_graph_t* out) {
  if (!m || !out) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  if (n_steps < 1) return fail(ORCHARD_ERR_INVALID_ARG, "n_steps must be >= 1");
  *out = nullptr;
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  orchard_graph_s* g = new orchard_graph_s();
  hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) {
    (void)hipStreamDestroy(cs); delete g;
    return fail(ORCHARD_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(he));
  }
  const orchard_status_t st = orchard_step(m, s, params, inputs, n_steps, nullptr, 0, (orchard_stream_t)cs);
  const std::string msg = st ? g_err : std::string();
  he = hipStreamEndCapture(cs, &g->graph);
  (void)hipStreamDestroy(cs);
  if (st) { orchard_graph_destroy(g); return fail(st, msg); }
  if (he != hipSuccess) { orchard_graph_destroy(g); return fail(ORCHARD_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he)); }
  he = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (he != hipSuccess) { orchard_graph_destroy(g); return fail(ORCHARD_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(he)); }
  *out = g;
  return ORCHARD_OK;
}

orchard_status_t orchard_graph_launch(orchard_graph_t g, orchard_stream_t stream) {
  if (!g || !g->exec) return fail(ORCHARD_ERR_INVALID_ARG, "null graph");
  HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return ORCHARD_OK;
}

// ---- autotuner ----
orchard_status_t orchard_autotune(const orchard_model_desc_t* d, const orchard_tuning_t* cand, int32_t n_cand,
                                  int32_t n_warm, int32_t n_steps, orchard_tuning_t* best, float* ms_out,
                                  orchard_stream_t stream) {
  if (!d || !cand || !best) return fail(ORCHARD_ERR_INVALID_ARG, "null argument");
  if (n_cand < 1 || n_steps < 1 || n_warm < 0) return fail(ORCHARD_ERR_INVALID_ARG, "need n_candidates >= 1, n_steps >= 1, n_warm >= 0");
  hipStream_t hs = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(ORCHARD_ERR_HIP, "hipEventCreate"); }
  void* buf = nullptr;
  float best_ms = -1.f;
  orchard_status_t first_err = ORCHARD_OK;
  std::string first_msg;
  for (int c = 0; c < n_cand; ++c) {
    if (ms_out) ms_out[c] = -1.f;
    orchard_tuning_t t = cand[c];
    t.adjoint_ckpt_max = 0;
    orchard_model_t m = nullptr;
    orchard_status_t st = orchard_model_create(d, &t, &m);
    if (st) { if (!first_err) { first_err = st; first_msg = g_err; } continue; }
    const int64_t NS = m->n_seg, NA = m->n_apple, B = m->n_env;
    auto al = [](int64_t b) { return (size_t)((b + 255) & ~int64_t(255)); };
    const size_t sz = 4 * al(8 * NS) + al(52 * NA) + al(2 * NS) + al(4 * NA) + al(4 * (NS + NA)) + al(4 * B) + al(8);
    if (!buf && hipMalloc(&buf, sz) != hipSuccess) {
      orchard_model_destroy(m); (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
      return fail(ORCHARD_ERR_OUT_OF_MEMORY, "autotune state");
    }
    char* w = (char*)buf;
    auto take = [&](int64_t b) { char* r = w; w += al(b); return r; };
    orchard_state_t S{};
    S.q = (float*)take(8 * NS); S.qd = (float*)take(8 * NS);
    float* kp = (float*)take(8 * NS); float* kd = (float*)take(8 * NS);
    S.apple = (float*)take(52 * NA); S.seg_evt = (uint8_t*)take(2 * NS); S.apple_evt = (uint8_t*)take(4 * NA);
    S.evt_step = (int32_t*)take(4 * (NS + NA)); S.env_status = (uint32_t*)take(4 * B); S.step = (int64_t*)take(8);
    orchard_params_t P{kp, kd};
    float ms = -1.f;
    st = orchard_default_params(m, kp, kd, stream);
    if (!st) st = orchard_state_rest(m, &S, stream);
    if (!st && n_warm > 0) st = orchard_step(m, &S, &P, nullptr, n_warm, nullptr, 0, stream);
    if (!st && hipEventRecord(e0, hs) != hipSuccess) st = fail(ORCHARD_ERR_HIP, "hipEventRecord");
    if (!st) st = orchard_step(m, &S, &P, nullptr, n_steps, nullptr, 0, stream);
    if (!st && hipEventRecord(e1, hs) != hipSuccess) st = fail(ORCHARD_ERR_HIP, "hipEventRecord");
    if (!st && hipEventSynchronize(e1) != hipSuccess) st = fail(ORCHARD_ERR_HIP, "hipEventSynchronize");
    if (!st && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = fail(ORCHARD_ERR_HIP, "hipEventElapsedTime");
    (void)hipStreamSynchronize(hs);
    orchard_model_destroy(m);
    if (st) {
      (void)hipFree(buf); (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
      return st;
    }
    ms /= (float)n_steps;
    if (ms_out) ms_out[c] = ms;
    if (best_ms < 0.f || ms < best_ms) { best_ms = ms; *best = cand[c]; }
  }
  if (buf) (void)hipFree(buf);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_ms < 0.f) return fail(first_err ? first_err : ORCHARD_ERR_INVALID_ARG, first_msg.empty() ? "no candidate built" : first_msg);
  return ORCHARD_OK;
}

}  // extern "C"
