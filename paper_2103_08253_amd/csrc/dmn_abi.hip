// C ABI of libdmn: argument validation, workspace layout and launch
// sequencing.  No allocation, no synchronisation, no device reads on the host.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "dmn_groups.hpp"

namespace {

constexpr size_t kAlign = 256;
// work counters of the Gauss-point launches: up to two per group
constexpr size_t kCounterBytes = 2 * 64 * sizeof(int32_t);
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

inline size_t elt_size(int prec) { return prec == DMN_F32 ? sizeof(float) : sizeof(double); }

// Workspace layout: [header 256 B: int32 error word at 0]
//                   then per table: [flag 256 B][rows L x 8 elements, aligned]
inline size_t table_bytes(int depth, int prec) {
  return kAlign + align_up(dmn::table_elems(depth) * elt_size(prec));
}

inline bool depth_ok(int32_t d) { return d >= 1 && d <= DMN_MAX_DEPTH; }
// depths whose kernels have run on the device: the Gauss-point update and the
// linear map, and the vector-Jacobian products (linear backward, adjoint)
inline bool depth_runs(int32_t d) { return d <= DMN_MAX_RUN_DEPTH; }
inline bool depth_runs_vjp(int32_t d) { return d <= DMN_MAX_RUN_DEPTH_VJP; }

// shape functions of an orientation interpolation, 0 for fixed normals, -1 invalid
inline int ori_count(int32_t shape) {
  switch (shape) {
    case DMN_ORI_NONE: return 0;
    case DMN_ORI_LINEAR: return 3;
    case DMN_ORI_TRILINEAR: return 4;
    case DMN_ORI_QUADRATIC: return 6;
    default: return -1;
  }
}

// a net with fixed normals (the calls other than the Gauss-point update)
inline int fixed_net_check(const dmn_net* net) {
  if (!net || !net->w) return DMN_EINVAL;
  if (net->ori_shape != DMN_ORI_NONE) return ori_count(net->ori_shape) < 0 ? DMN_EINVAL
                                                                           : DMN_EUNSUPPORTED;
  return net->n ? DMN_OK : DMN_EINVAL;
}

struct Table {
  int32_t* flag;
  void* rows;
};

inline Table table_at(void* ws, size_t offset) {
  char* p = (char*)ws + offset;
  return Table{(int32_t*)p, (void*)(p + kAlign)};
}

inline bool phase_ok(const dmn_elastic* f) {
  return f && f->E > 0.0 && f->nu > -1.0 && f->nu < 0.5;
}
inline bool j2_ok(const dmn_j2* m) {
  return m && m->E > 0.0 && m->nu > -1.0 && m->nu < 0.5 && m->sigma0 > 0.0 && m->k_inf >= 0.0 &&
         m->dsigma >= 0.0 && m->b >= 0.0;
}

// Process-wide launch tuning of the Gauss-point update per depth (0 = default).
std::atomic<int> g_tune_lanes[DMN_MAX_DEPTH + 1];
std::atomic<int> g_tune_waves[DMN_MAX_DEPTH + 1];

struct GpTune {
  int lanes;         // lanes per point
  int waves_per_cu;  // persistent waves per compute unit
};

inline GpTune gp_tuning(int depth) {
  const int l = g_tune_lanes[depth].load(std::memory_order_relaxed);
  const int w = g_tune_waves[depth].load(std::memory_order_relaxed);
  return GpTune{l ? l : dmn::gp_default_lanes_per_point(depth),
                w ? w : dmn::kDefaultWavesPerCu};
}

inline bool gp_variant_exists(int depth, int lanes) {
  int v[16];
  const int n = dmn::gp_lane_variants(depth, v, 16);
  for (int i = 0; i < n && i < 16; ++i)
    if (v[i] == lanes) return true;
  return false;
}

}  // namespace

extern "C" {

const char* dmn_version(void) { return "libdmn 0.1 gfx950"; }

// a net for the linear calls: fixed normals, or normals interpolated per
// sample from its fibre orientation lam (up to the depth of the VJP kernels)
static int linear_net_check(const dmn_net* net, int64_t B, const void* lam) {
  if (!net || !depth_ok(net->depth) || B < 0 || !net->w) return DMN_EINVAL;
  const int m = ori_count(net->ori_shape);
  if (m < 0) return DMN_EINVAL;
  if (m == 0) return net->n ? DMN_OK : DMN_EINVAL;
  if (!net->ori_p || !net->ori_q || (B > 0 && !lam)) return DMN_EINVAL;
  return depth_runs_vjp(net->depth) ? DMN_OK : DMN_EUNSUPPORTED;
}

static dmn::LinOriArgs lin_ori(const dmn_net* net, const void* lam, void* gang) {
  dmn::LinOriArgs o;
  o.m = ori_count(net->ori_shape);
  if (o.m > 0) {
    o.p = net->ori_p;
    o.q = net->ori_q;
    o.lam = lam;
    o.gang = gang;
  }
  return o;
}

size_t dmn_homogenize_linear_workspace_size(const dmn_net* net, int64_t B, int prec) {
  if (!net || !depth_ok(net->depth) || B < 0 || (prec != DMN_F64 && prec != DMN_F32)) return 0;
  if (ori_count(net->ori_shape) < 0) return 0;
  return kAlign + table_bytes(net->depth, prec);
}

int dmn_homogenize_linear(const dmn_net* net, int64_t B, int prec, const void* C1,
                          const void* C2, const void* lam, void* Cbar, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
  if (!net) return DMN_EINVAL;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (const int rc = linear_net_check(net, B, lam)) return rc;
  if (B > 0 && (!C1 || !C2 || !Cbar)) return DMN_EINVAL;
  if (!depth_runs(net->depth)) return DMN_EUNSUPPORTED;
  const size_t need = dmn_homogenize_linear_workspace_size(net, B, prec);
  if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) return DMN_EWORKSPACE;
  int32_t* err = (int32_t*)ws;
  Table tb = table_at(ws, kAlign);
  const void* nfix = net->ori_shape == DMN_ORI_NONE ? net->n : nullptr;
  if (dmn::launch_prep_tables(net->w, nfix, net->depth, prec, tb.rows, tb.flag, err, stream,
                              true))
    return DMN_EHIP;
  if (B == 0) return DMN_OK;
  if (dmn::launch_linear_forward(net->depth, prec, tb.rows, tb.flag, B, C1, C2, Cbar, err,
                                 lin_ori(net, lam, nullptr), stream))
    return DMN_EHIP;
  return DMN_OK;
}

size_t dmn_homogenize_backward_workspace_size(const dmn_net* net, int64_t B, int prec) {
  if (!net || !depth_ok(net->depth) || B < 0 || (prec != DMN_F64 && prec != DMN_F32)) return 0;
  const int m = ori_count(net->ori_shape);
  if (m < 0) return 0;
  const int depth = net->depth;
  const size_t L = ((size_t)1 << depth) - 1;
  const size_t slots = (size_t)dmn::linear_backward_partials(depth, B, prec == DMN_F32);
  const size_t gang = m > 0 ? align_up(L * 2 * (size_t)B * elt_size(prec)) : 0;
  return kAlign + table_bytes(depth, prec) + align_up(L * 4 * sizeof(double)) +
         align_up(slots * L * 4 * sizeof(double)) + gang;
}

int dmn_homogenize_backward(const dmn_net* net, int64_t B, int prec, const void* C1,
                            const void* C2, const void* lam, const void* gCbar, void* gw,
                            void* gn, void* gC1, void* gC2, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  if (!net) return DMN_EINVAL;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (const int rc = linear_net_check(net, B, lam)) return rc;
  if (!gw || !gn) return DMN_EINVAL;
  if (B > 0 && (!C1 || !C2 || !gCbar)) return DMN_EINVAL;
  if ((gC1 == nullptr) != (gC2 == nullptr)) return DMN_EINVAL;
  if (!depth_runs_vjp(net->depth)) return DMN_EUNSUPPORTED;
  const size_t need = dmn_homogenize_backward_workspace_size(net, B, prec);
  if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) return DMN_EWORKSPACE;
  const int K = net->depth;
  const size_t L = ((size_t)1 << K) - 1;
  const size_t slots = (size_t)dmn::linear_backward_partials(K, B, prec == DMN_F32);
  int32_t* err = (int32_t*)ws;
  Table tb = table_at(ws, kAlign);
  double* gsum = (double*)((char*)ws + kAlign + table_bytes(K, prec));
  double* partials = (double*)((char*)gsum + align_up(L * 4 * sizeof(double)));
  void* gang = (char*)partials + align_up(slots * L * 4 * sizeof(double));
  const void* nfix = net->ori_shape == DMN_ORI_NONE ? net->n : nullptr;
  if (dmn::launch_prep_tables(net->w, nfix, K, prec, tb.rows, tb.flag, err, stream, true))
    return DMN_EHIP;
  // B == 0 still runs the (empty) reductions so gw, gn are overwritten with zeros
  if (dmn::launch_linear_backward(K, prec, tb.rows, tb.flag, B, C1, C2, gCbar, gw, gn, gC1, gC2,
                                  partials, gsum, err, lin_ori(net, lam, gang), stream))
    return DMN_EHIP;
  return DMN_OK;
}

// sample offsets of a grouped linear call: G >= 1, offsets[0] = 0, non-decreasing
static bool group_offsets_ok(int32_t G, const int64_t* off) {
  if (G < 1 || !off || off[0] != 0) return false;
  for (int32_t k = 0; k < G; ++k)
    if (off[k + 1] < off[k]) return false;
  return true;
}

size_t dmn_homogenize_linear_groups_workspace_size(int32_t depth, int32_t G, int prec) {
  if (!depth_ok(depth) || G < 1 || (prec != DMN_F64 && prec != DMN_F32)) return 0;
  return kAlign + (size_t)G * table_bytes(depth, prec);
}

int dmn_homogenize_linear_groups(int32_t depth, int32_t G, const int64_t* offsets, int prec,
                                 const void* w, const void* n_groups, const void* C1,
                                 const void* C2, void* Cbar, void* ws, size_t ws_bytes,
                                 hipStream_t stream) {
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (!depth_ok(depth) || !group_offsets_ok(G, offsets) || !w || !n_groups) return DMN_EINVAL;
  const int64_t B = offsets[G];
  if (B > 0 && (!C1 || !C2 || !Cbar)) return DMN_EINVAL;
  if (!depth_runs(depth)) return DMN_EUNSUPPORTED;
  const size_t need = dmn_homogenize_linear_groups_workspace_size(depth, G, prec);
  if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) return DMN_EWORKSPACE;
  int32_t* err = (int32_t*)ws;
  Table tb = table_at(ws, kAlign);
  const long long tbytes = (long long)table_bytes(depth, prec);
  if (dmn::launch_prep_tables_groups(w, n_groups, depth, prec, G, tb.rows, tb.flag, tbytes, err,
                                     stream))
    return DMN_EHIP;
  if (B == 0) return DMN_OK;
  if (dmn::launch_linear_forward_groups(depth, prec, tb.rows, tb.flag, tbytes, G, offsets, C1, C2,
                                        Cbar, err, stream))
    return DMN_EHIP;
  return DMN_OK;
}

size_t dmn_homogenize_backward_groups_workspace_size(int32_t depth, int32_t G,
                                                     const int64_t* offsets, int prec) {
  if (!depth_ok(depth) || !group_offsets_ok(G, offsets) || (prec != DMN_F64 && prec != DMN_F32))
    return 0;
  const size_t L = ((size_t)1 << depth) - 1;
  const size_t slots =
      (size_t)dmn::linear_backward_group_slots(depth, G, offsets, prec == DMN_F32);
  return kAlign + (size_t)G * table_bytes(depth, prec) +
         align_up((size_t)G * L * 4 * sizeof(double)) + align_up(slots * L * 4 * sizeof(double));
}

int dmn_homogenize_backward_groups(int32_t depth, int32_t G, const int64_t* offsets, int prec,
                                   const void* w, const void* n_groups, const void* C1,
                                   const void* C2, const void* gCbar, void* gw_groups,
                                   void* gn_groups, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (!depth_ok(depth) || !group_offsets_ok(G, offsets) || !w || !n_groups) return DMN_EINVAL;
  if (!gw_groups || !gn_groups) return DMN_EINVAL;
  const int64_t B = offsets[G];
  if (B > 0 && (!C1 || !C2 || !gCbar)) return DMN_EINVAL;
  if (!depth_runs_vjp(depth)) return DMN_EUNSUPPORTED;
  const size_t need = dmn_homogenize_backward_groups_workspace_size(depth, G, offsets, prec);
  if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) return DMN_EWORKSPACE;
  const size_t L = ((size_t)1 << depth) - 1;
  int32_t* err = (int32_t*)ws;
  Table tb = table_at(ws, kAlign);
  const long long tbytes = (long long)table_bytes(depth, prec);
  double* gsum = (double*)((char*)ws + kAlign + (size_t)G * (size_t)tbytes);
  double* partials = (double*)((char*)gsum + align_up((size_t)G * L * 4 * sizeof(double)));
  if (dmn::launch_prep_tables_groups(w, n_groups, depth, prec, G, tb.rows, tb.flag, tbytes, err,
                                     stream))
    return DMN_EHIP;
  // B == 0 still runs the (empty) reductions so every group's gradients are zeroed
  if (dmn::launch_linear_backward_groups(depth, prec, tb.rows, tb.flag, tbytes, G, offsets, C1, C2,
                                         gCbar, gw_groups, gn_groups, partials, gsum, err, stream))
    return DMN_EHIP;
  return DMN_OK;
}

// FP64 copies of one group's per-point arrays for DMN_F32_STATE, in the order
// E, z_in, z_out, a_in, a_out, sigma, tangent (each 256-byte aligned)
static size_t staging_bytes(const dmn_point_group& g) {
  if (g.P <= 0) return 0;
  const size_t P = (size_t)g.P, M = (size_t)1 << (g.net.depth - 1);
  const size_t L = ((size_t)1 << g.net.depth) - 1;
  return 2 * align_up(P * 6 * 8) + 2 * align_up(P * 7 * M * 8) + 2 * align_up(P * 3 * L * 8) +
         align_up(P * 36 * 8);
}

size_t dmn_update_gauss_points_workspace_size(const dmn_point_group* groups, int32_t n_groups,
                                              int prec) {
  if (!groups || n_groups < 1 || n_groups > 64 || (prec != DMN_F64 && prec != DMN_F32_STATE))
    return 0;
  size_t total = kAlign + kCounterBytes;  // header, then the launches' work counters
  for (int i = 0; i < n_groups; ++i) {
    if (!depth_ok(groups[i].net.depth)) return 0;
    total += table_bytes(groups[i].net.depth, DMN_F64);  // DMN parameters are FP64
  }
  if (prec == DMN_F32_STATE)
    for (int i = 0; i < n_groups; ++i) total += staging_bytes(groups[i]);
  return total;
}

}  // extern "C"

// Argument validation of the Gauss-point update (host data only).
static int gp_check(const dmn_point_group* groups, int32_t n_groups, const dmn_elastic* fiber,
                    const dmn_j2* matrix, int prec, const dmn_newton_opts* opts,
                    GpTune (&tune)[DMN_MAX_DEPTH + 1]) {
  if (!groups || n_groups < 1 || n_groups > 64) return DMN_EINVAL;
  if (prec != DMN_F64 && prec != DMN_F32_STATE) return DMN_EUNSUPPORTED;
  if (!phase_ok(fiber) || !j2_ok(matrix) || !opts) return DMN_EINVAL;
  if (!(opts->tol > 0.0) || opts->max_iter < 0 || opts->max_backtrack < 0 ||
      !(opts->armijo >= 0.0 && opts->armijo < 1.0) || opts->local_max_iter < 0 ||
      opts->polish < 0)
    return DMN_EINVAL;
  for (int i = 0; i < n_groups; ++i) {
    const dmn_point_group& g = groups[i];
    if (!depth_ok(g.net.depth) || g.P < 0 || !g.net.w) return DMN_EINVAL;
    const int m = ori_count(g.net.ori_shape);
    if (m < 0) return DMN_EINVAL;
    if (m == 0 && !g.net.n) return DMN_EINVAL;
    if (m > 0 && (!g.net.ori_p || !g.net.ori_q || (g.P > 0 && !g.lam))) return DMN_EINVAL;
    if (g.P > 0 && (!g.E || !g.z_in || !g.z_out || !g.a_in || !g.a_out || !g.sigma ||
                    !g.tangent || !g.iters || !g.status))
      return DMN_EINVAL;
    if (g.P > 0 && (g.z_in == g.z_out || g.a_in == g.a_out)) return DMN_EINVAL;
    if (!depth_runs(g.net.depth) || (m > 0 && !depth_runs_vjp(g.net.depth)))
      return DMN_EUNSUPPORTED;
  }
  // one snapshot of the tuning table per call
  for (int k = 1; k <= DMN_MAX_DEPTH; ++k) tune[k] = gp_tuning(k);
  for (int i = 0; i < n_groups; ++i) {
    const dmn_point_group& g = groups[i];
    const int lanes = g.net.ori_shape != DMN_ORI_NONE
                          ? dmn::gp_default_lanes_per_point(g.net.depth)
                          : tune[g.net.depth].lanes;
    if ((g.P + 63) / 64 * lanes > (int64_t)0x7fffffff) return DMN_EINVAL;
  }
  return DMN_OK;
}

// Launches of the Gauss-point update on a validated call, with the workspace
// ws (at least dmn_update_gauss_points_workspace_size bytes, 256-byte
// aligned).  Allocates nothing, on the device or the host.
static int gp_launch(const dmn_point_group* groups, int32_t n_groups, const dmn_elastic* fiber,
                     const dmn_j2* matrix, int prec, const dmn_newton_opts* opts,
                     const GpTune (&tune)[DMN_MAX_DEPTH + 1], void* ws, hipStream_t stream) {
  // work counters (at most one launch, with up to two counters, per group),
  // then tables, one per group; the counters are cleared by a fill kernel
  // (graph-capturable, and a workspace that keeps an earlier call's contents
  // starts from zero)
  int32_t* counters = (int32_t*)((char*)ws + kAlign);
  if (dmn::launch_zero_ints(counters, 2 * n_groups, stream)) return DMN_EHIP;
  Table tabs[64];
  size_t off = kAlign + kCounterBytes;
  for (int i = 0; i < n_groups; ++i) {
    tabs[i] = table_at(ws, off);
    off += table_bytes(groups[i].net.depth, DMN_F64);
    const void* nfix = groups[i].net.ori_shape == DMN_ORI_NONE ? groups[i].net.n : nullptr;
    // dead subtrees are removed (tree compression), as in the linear map
    if (dmn::launch_prep_tables(groups[i].net.w, nfix, groups[i].net.depth, DMN_F64,
                                tabs[i].rows, tabs[i].flag, nullptr, stream, true))
      return DMN_EHIP;
  }

  dmn::GpLaunch base;
  memset(&base, 0, sizeof(base));
  base.max_iter = opts->max_iter;
  base.max_bt = opts->max_backtrack;
  base.polish = opts->polish;
  base.tol = opts->tol;
  base.armijo = opts->armijo;
  base.fib.K = fiber->E / (3.0 * (1.0 - 2.0 * fiber->nu));
  base.fib.G = fiber->E / (2.0 * (1.0 + fiber->nu));
  base.mat.K = matrix->E / (3.0 * (1.0 - 2.0 * matrix->nu));
  base.mat.G = matrix->E / (2.0 * (1.0 + matrix->nu));
  base.mat.sigma0 = matrix->sigma0;
  base.mat.k_inf = matrix->k_inf;
  base.mat.dsigma = matrix->dsigma;
  base.mat.b = matrix->b;
  base.mat.max_it = opts->local_max_iter > 0 ? opts->local_max_iter : dmn::kLocalMaxIt;

  auto is_ori = [&](int i) { return groups[i].net.ori_shape != DMN_ORI_NONE; };
  auto lanes_of = [&](int i) {
    return is_ori(i) ? dmn::gp_default_lanes_per_point(groups[i].net.depth)
                     : tune[groups[i].net.depth].lanes;
  };
  auto fill = [&](dmn::GroupArgs& a, int i, int block0) {
    const dmn_point_group& g = groups[i];
    a.E = g.E;
    a.z_in = g.z_in;
    a.z_out = g.z_out;
    a.a_in = g.a_in;
    a.a_out = g.a_out;
    a.sigma = g.sigma;
    a.tangent = g.tangent;
    a.iters = g.iters;
    a.status = g.status;
    a.tab = (const double*)tabs[i].rows;
    a.flag = tabs[i].flag;
    a.ori_p = (const double*)g.net.ori_p;
    a.ori_q = (const double*)g.net.ori_q;
    a.lam = (const double*)g.lam;
    a.ori_m = ori_count(g.net.ori_shape);
    a.depth = g.net.depth;
    a.P = g.P;
    a.block0 = block0;
    a.lanes = lanes_of(i);
  };
  // groups with points, deepest first, fixed normals before interpolated ones
  auto before = [&](int a, int b) {
    if ((int)is_ori(a) != (int)is_ori(b)) return (int)is_ori(a) < (int)is_ori(b);
    return groups[a].net.depth > groups[b].net.depth;
  };
  int order[64];
  int n_order = 0, n_fixed = 0;
  for (int i = 0; i < n_groups; ++i) {
    if (groups[i].P <= 0) continue;
    n_fixed += is_ori(i) ? 0 : 1;
    int j = n_order++;  // stable insertion
    while (j > 0 && before(i, order[j - 1])) {
      order[j] = order[j - 1];
      --j;
    }
    order[j] = i;
  }
  // order[0, n_fixed) are the fixed-normal groups, deepest first
  const bool fixed_depth9 = n_fixed > 0 && groups[order[0]].net.depth == dmn::kSplitDepth;
  const bool fixed_depths_differ =
      n_fixed > 0 && groups[order[0]].net.depth != groups[order[n_fixed - 1]].net.depth;

  int pos = 0;
  int counter = 0;
  const long long cus = dmn::device_cu_count();
  // fixed-normal groups of several depths, or of depth 9: mixed launches of
  // up to kMaxGroupsPerLaunch groups, depth-9 groups first
  if (n_fixed > 0 && (fixed_depth9 || fixed_depths_differ)) {
    while (pos < n_fixed && groups[order[pos]].net.depth >= dmn::kMixedLaneDepth) {
      dmn::GpLaunch args = base;
      long long items_split = 0, items = 0;
      int waves_per_cu = 1;
      while (pos < n_fixed && args.ng < dmn::kMaxGroupsPerLaunch &&
             groups[order[pos]].net.depth == dmn::kSplitDepth) {
        const int i = order[pos++];
        fill(args.g[args.ng++], i, (int)items_split);
        items_split += groups[i].P;
        waves_per_cu = std::max(waves_per_cu, tune[groups[i].net.depth].waves_per_cu);
      }
      args.ng_split = args.ng;
      // depths 2-8 run with lane subtrees of depth dmn::kMixedLaneDepth in a
      // mixed launch whatever the tuning table says (depth 1 runs on its own)
      while (pos < n_fixed && args.ng < dmn::kMaxGroupsPerLaunch &&
             groups[order[pos]].net.depth != dmn::kSplitDepth &&
             groups[order[pos]].net.depth >= dmn::kMixedLaneDepth) {
        const int i = order[pos++];
        const int K = groups[i].net.depth;
        const int lanes = 1 << (K - dmn::kMixedLaneDepth);
        const int ppb = dmn::gp_points_per_block(K, lanes);
        fill(args.g[args.ng], i, (int)items);
        args.g[args.ng++].lanes = lanes;
        items += (groups[i].P + ppb - 1) / ppb;
        waves_per_cu = std::max(waves_per_cu, tune[K].waves_per_cu);
      }
      if (args.ng == 0) break;  // only depth-1 groups left: the loop below
      if (items > 0x7fffffff || items_split > 0x7fffffff) return DMN_EINVAL;
      args.counter = counters + counter++;
      args.counter_split = counters + counter++;
      args.total = (int)items;
      args.total_split = (int)items_split;
      const long long persistent = std::max(1LL, cus * waves_per_cu / 2);
      const long long need = std::max(std::max(items_split, (items + 1) / 2), 1LL);
      if (dmn::launch_gp_mixed(args, (int)std::min(persistent, need), stream)) return DMN_EHIP;
    }
  }
  // the rest: one launch per depth and kind of normals, up to
  // kMaxGroupsPerLaunch groups each
  while (pos < n_order) {
    const int K = groups[order[pos]].net.depth;
    const bool ori = is_ori(order[pos]);
    const int lp = lanes_of(order[pos]);
    const long long persistent = cus * tune[K].waves_per_cu;
    const int ppb = dmn::gp_points_per_block(K, lp);
    dmn::GpLaunch args = base;
    long long blocks = 0;
    while (pos < n_order && groups[order[pos]].net.depth == K &&
           is_ori(order[pos]) == ori && args.ng < dmn::kMaxGroupsPerLaunch) {
      const int i = order[pos++];
      fill(args.g[args.ng++], i, (int)blocks);
      blocks += (groups[i].P + ppb - 1) / ppb;
    }
    if (blocks > 0x7fffffff) return DMN_EINVAL;
    args.counter = counters + counter++;
    args.total = (int)blocks;
    const long long waves = blocks < persistent ? blocks : persistent;
    if (dmn::launch_gp_update(K, lp, prec, ori, args, (int)waves, stream)) return DMN_EHIP;
  }
  return DMN_OK;
}

// Workspace of dmn_update_gauss_points_noalloc: one array per device, held
// until the process ends.  Its name is a host-side stand-in: host code uses
// only the device address taken from hipGetSymbolAddress, per device.
constexpr size_t kNoallocScratchBytes = DMN_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[64];

// Device address of this device's scratch array (taken once per device, with
// that device current), or null when the runtime call fails.
static void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
      return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

extern "C" {

int dmn_update_gauss_points(const dmn_point_group* groups, int32_t n_groups,
                            const dmn_elastic* fiber, const dmn_j2* matrix, int prec,
                            const dmn_newton_opts* opts, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  GpTune tune[DMN_MAX_DEPTH + 1];
  if (const int rc = gp_check(groups, n_groups, fiber, matrix, prec, opts, tune)) return rc;
  const size_t need = dmn_update_gauss_points_workspace_size(groups, n_groups, prec);
  if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) return DMN_EWORKSPACE;
  if (prec == DMN_F64) return gp_launch(groups, n_groups, fiber, matrix, prec, opts, tune, ws,
                                        stream);
  // FP32 state: widen the inputs into FP64 copies in the workspace, run the
  // FP64 update on them, round the results back into the caller's arrays
  dmn_point_group staged[64];
  char* p = (char*)ws + dmn_update_gauss_points_workspace_size(groups, n_groups, DMN_F64);
  for (int i = 0; i < n_groups; ++i) {
    const dmn_point_group& g = groups[i];
    staged[i] = g;
    if (g.P <= 0) continue;
    const long long P = g.P, M = 1LL << (g.net.depth - 1), L = (1LL << g.net.depth) - 1;
    auto take = [&](long long n) {
      double* q = (double*)p;
      p += align_up((size_t)n * 8);
      return q;
    };
    double* E = take(P * 6);
    double* zi = take(P * 7 * M);
    double* zo = take(P * 7 * M);
    double* ai = take(P * 3 * L);
    double* ao = take(P * 3 * L);
    double* sg = take(P * 6);
    double* tg = take(P * 36);
    if (dmn::launch_widen((const float*)g.E, E, P * 6, stream) ||
        dmn::launch_widen((const float*)g.z_in, zi, P * 7 * M, stream) ||
        dmn::launch_widen((const float*)g.a_in, ai, P * 3 * L, stream))
      return DMN_EHIP;
    staged[i].E = E;
    staged[i].z_in = zi;
    staged[i].z_out = zo;
    staged[i].a_in = ai;
    staged[i].a_out = ao;
    staged[i].sigma = sg;
    staged[i].tangent = tg;
  }
  if (const int rc = gp_launch(staged, n_groups, fiber, matrix, DMN_F64, opts, tune, ws, stream))
    return rc;
  for (int i = 0; i < n_groups; ++i) {
    const dmn_point_group& g = groups[i];
    if (g.P <= 0) continue;
    const long long P = g.P, M = 1LL << (g.net.depth - 1), L = (1LL << g.net.depth) - 1;
    if (dmn::launch_narrow((const double*)staged[i].sigma, (float*)g.sigma, P * 6, stream) ||
        dmn::launch_narrow((const double*)staged[i].tangent, (float*)g.tangent, P * 36, stream) ||
        dmn::launch_narrow((const double*)staged[i].z_out, (float*)g.z_out, P * 7 * M, stream) ||
        dmn::launch_narrow((const double*)staged[i].a_out, (float*)g.a_out, P * 3 * L, stream))
      return DMN_EHIP;
  }
  return DMN_OK;
}

int dmn_update_gauss_points_noalloc(const dmn_point_group* groups, int32_t n_groups,
                                    const dmn_elastic* fiber, const dmn_j2* matrix, int prec,
                                    const dmn_newton_opts* opts, hipStream_t stream) {
  GpTune tune[DMN_MAX_DEPTH + 1];
  if (const int rc = gp_check(groups, n_groups, fiber, matrix, prec, opts, tune)) return rc;
  if (prec != DMN_F64) return DMN_EUNSUPPORTED;  // FP32 state needs per-point staging
  const size_t need = dmn_update_gauss_points_workspace_size(groups, n_groups, prec);
  if (need > kNoallocScratchBytes) return DMN_EWORKSPACE;
  void* ws = scratch_address();
  if (ws == nullptr) return DMN_EHIP;
  return gp_launch(groups, n_groups, fiber, matrix, prec, opts, tune, ws, stream);
}

static size_t adjoint_group_bytes(const dmn_adjoint_group& g) {
  const size_t K = g.net.depth;
  const size_t rows = 4 * (((size_t)1 << K) - 1) + ((size_t)1 << K);
  const size_t slots = (size_t)dmn::adjoint_partial_slots((int)K, g.P);
  return table_bytes((int)K, DMN_F64) + align_up(rows * sizeof(double)) +
         align_up(rows * slots * sizeof(double));
}

size_t dmn_update_adjoint_workspace_size(const dmn_adjoint_group* groups, int32_t n_groups,
                                         int prec) {
  if (!groups || n_groups < 1 || n_groups > 64 || prec != DMN_F64) return 0;
  size_t total = kAlign;
  for (int i = 0; i < n_groups; ++i) {
    if (!depth_ok(groups[i].net.depth) || groups[i].P < 0) return 0;
    total += adjoint_group_bytes(groups[i]);
  }
  return total;
}

int dmn_update_adjoint(const dmn_adjoint_group* groups, int32_t n_groups,
                       const dmn_elastic* fiber, const dmn_j2* matrix, int prec, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
  if (!groups || n_groups < 1 || n_groups > 64) return DMN_EINVAL;
  if (prec != DMN_F64) return DMN_EUNSUPPORTED;
  if (!phase_ok(fiber) || !j2_ok(matrix)) return DMN_EINVAL;
  for (int i = 0; i < n_groups; ++i) {
    const dmn_adjoint_group& g = groups[i];
    if (!depth_ok(g.net.depth) || g.P < 0 || !g.gw || !g.gn) return DMN_EINVAL;
    if (const int rc = fixed_net_check(&g.net)) return rc;
    if (g.P > 0 && (!g.E || !g.z_in || !g.a_conv || !g.g_z_prev)) return DMN_EINVAL;
    if (g.P > 0 && g.g_z_next != nullptr && g.g_z_next == g.g_z_prev) return DMN_EINVAL;
    if (!depth_runs_vjp(g.net.depth)) return DMN_EUNSUPPORTED;
  }
  const size_t need = dmn_update_adjoint_workspace_size(groups, n_groups, prec);
  if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) return DMN_EWORKSPACE;
  int32_t* err = (int32_t*)ws;
  size_t off = kAlign;
  for (int i = 0; i < n_groups; ++i) {
    const dmn_adjoint_group& g = groups[i];
    const int K = g.net.depth;
    const size_t rows = 4 * (((size_t)1 << K) - 1) + ((size_t)1 << K);
    Table tb = table_at(ws, off);
    double* gsum = (double*)((char*)ws + off + table_bytes(K, DMN_F64));
    double* partials = (double*)((char*)gsum + align_up(rows * sizeof(double)));
    off += adjoint_group_bytes(g);
    // dead subtrees are removed (tree compression), as in the forward update
    if (dmn::launch_prep_tables(g.net.w, g.net.n, K, DMN_F64, tb.rows, tb.flag,
                                i == 0 ? err : nullptr, stream, true))
      return DMN_EHIP;
    if (g.P == 0) continue;
    dmn::AdjointLaunch a;
    memset(&a, 0, sizeof(a));
    a.E = (const double*)g.E;
    a.z_in = (const double*)g.z_in;
    a.a_conv = (const double*)g.a_conv;
    a.g_sigma = (const double*)g.g_sigma;
    a.g_z_next = (const double*)g.g_z_next;
    a.g_z_prev = (double*)g.g_z_prev;
    a.tab = (const double*)tb.rows;
    a.flag = tb.flag;
    a.partials = partials;
    a.gsum = gsum;
    a.gw = (double*)g.gw;
    a.gn = (double*)g.gn;
    a.err = err;
    a.P = g.P;
    a.fib.K = fiber->E / (3.0 * (1.0 - 2.0 * fiber->nu));
    a.fib.G = fiber->E / (2.0 * (1.0 + fiber->nu));
    a.mat.K = matrix->E / (3.0 * (1.0 - 2.0 * matrix->nu));
    a.mat.G = matrix->E / (2.0 * (1.0 + matrix->nu));
    a.mat.sigma0 = matrix->sigma0;
    a.mat.k_inf = matrix->k_inf;
    a.mat.dsigma = matrix->dsigma;
    a.mat.b = matrix->b;
    a.mat.max_it = dmn::kLocalMaxIt;
    if (dmn::launch_adjoint(K, a, stream)) return DMN_EHIP;
  }
  return DMN_OK;
}

int dmn_gp_set_tuning(int32_t depth, const dmn_gp_tuning* t) {
  if (!depth_ok(depth)) return DMN_EINVAL;
  const int lanes = t ? t->lanes_per_point : 0;
  const int waves = t ? t->waves_per_cu : 0;
  if (lanes < 0 || waves < 0 || waves > 64) return DMN_EINVAL;
  if (lanes != 0 && !gp_variant_exists(depth, lanes)) return DMN_EUNSUPPORTED;
  g_tune_lanes[depth].store(lanes, std::memory_order_relaxed);
  g_tune_waves[depth].store(waves, std::memory_order_relaxed);
  return DMN_OK;
}

int dmn_gp_get_tuning(int32_t depth, dmn_gp_tuning* t) {
  if (!depth_ok(depth) || !t) return DMN_EINVAL;
  const GpTune u = gp_tuning(depth);
  t->lanes_per_point = u.lanes;
  t->waves_per_cu = u.waves_per_cu;
  return DMN_OK;
}

int32_t dmn_gp_lane_variants(int32_t depth, int32_t* lanes, int32_t cap) {
  if (!depth_ok(depth) || cap < 0) return 0;
  return dmn::gp_lane_variants(depth, lanes, cap);
}

size_t dmn_training_loss_workspace_size(int64_t B) {
  if (B < 0) return 0;
  return kAlign + align_up(3 * (size_t)B * sizeof(double));
}

int dmn_training_loss(int64_t B, int prec, const void* Cbar, const void* target,
                      const dmn_loss_opts* opts, void* e, void* gCbar, double* stats, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  if (B < 0 || !opts || !stats) return DMN_EINVAL;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (!(opts->p >= 1.0 && opts->p < 1e300) || !(opts->q >= 1.0 && opts->q < 1e300))
    return DMN_EINVAL;
  if (B > 0 && (!Cbar || !target || !gCbar)) return DMN_EINVAL;
  if (!ws || ws_bytes < dmn_training_loss_workspace_size(B) || ((uintptr_t)ws % kAlign) != 0)
    return DMN_EWORKSPACE;
  double* scratch = (double*)((char*)ws + kAlign);
  if (dmn::launch_training_loss(prec, B, opts->p, opts->q, Cbar, target, e, gCbar, stats, scratch,
                                stream))
    return DMN_EHIP;
  return DMN_OK;
}

static int train_params_check(const dmn_train_params* t) {
  if (!t || !depth_ok(t->depth)) return DMN_EINVAL;
  if (!t->v || !t->alpha || !t->beta || !t->w || !t->n || !t->state || !t->step)
    return DMN_EINVAL;
  return DMN_OK;
}

static dmn::TrainUpdateArgs train_args(const dmn_train_params* t) {
  dmn::TrainUpdateArgs a = {};
  a.v = t->v;
  a.alpha = t->alpha;
  a.beta = t->beta;
  a.w = t->w;
  a.n = t->n;
  a.state = t->state;
  a.step = (long long*)t->step;
  a.half_period = 1;
  a.steps_per_epoch = 1;
  return a;
}

int dmn_training_update(const dmn_train_params* params, int prec, const void* gw, const void* gn,
                        const dmn_amsgrad_opts* opts, double* stats, hipStream_t stream) {
  if (const int rc = train_params_check(params)) return rc;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (!gw || !gn || !opts || !stats) return DMN_EINVAL;
  const dmn_amsgrad_opts& o = *opts;
  if (!(o.lr_min >= 0.0) || !(o.lr_max >= 0.0) || !(o.lr_decay > 0.0) || o.half_period < 1 ||
      o.steps_per_epoch < 1 || !(o.beta1 >= 0.0 && o.beta1 < 1.0) ||
      !(o.beta2 >= 0.0 && o.beta2 < 1.0) || !(o.eps > 0.0) || !(o.penalty >= 0.0))
    return DMN_EINVAL;
  dmn::TrainUpdateArgs a = train_args(params);
  a.gw = gw;
  a.gn = gn;
  a.stats = stats;
  a.lr_min = o.lr_min;
  a.lr_max = o.lr_max;
  a.lr_decay = o.lr_decay;
  a.beta1 = o.beta1;
  a.beta2 = o.beta2;
  a.eps = o.eps;
  a.penalty = o.penalty;
  a.half_period = o.half_period;
  a.steps_per_epoch = o.steps_per_epoch;
  a.take_step = 1;
  return dmn::launch_training_update(prec, params->depth, a, stream) ? DMN_EHIP : DMN_OK;
}

int dmn_training_refresh(const dmn_train_params* params, int prec, hipStream_t stream) {
  if (const int rc = train_params_check(params)) return rc;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  dmn::TrainUpdateArgs a = train_args(params);
  a.take_step = 0;
  return dmn::launch_training_update(prec, params->depth, a, stream) ? DMN_EHIP : DMN_OK;
}

int dmn_orientation_group_normals(int32_t depth, int32_t ori_shape, int32_t G, int prec,
                                  const void* p, const void* q, const void* lam, void* n,
                                  hipStream_t stream) {
  const int m = ori_count(ori_shape);
  if (!depth_ok(depth) || m <= 0 || G < 0) return DMN_EINVAL;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (!p || !q || (G > 0 && (!lam || !n))) return DMN_EINVAL;
  return dmn::launch_group_normals(prec, depth, m, G, p, q, lam, n, stream) ? DMN_EHIP : DMN_OK;
}

int dmn_orientation_group_chain(int32_t depth, int32_t ori_shape, int32_t G, int prec,
                                const void* p, const void* q, const void* lam,
                                const void* gw_groups, const void* gn_groups, void* gw,
                                void* gpq, hipStream_t stream) {
  const int m = ori_count(ori_shape);
  if (!depth_ok(depth) || m <= 0 || G < 0) return DMN_EINVAL;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (!p || !q || !gw || !gpq || (G > 0 && (!lam || !gw_groups || !gn_groups)))
    return DMN_EINVAL;
  return dmn::launch_group_chain(prec, depth, m, G, p, q, lam, gw_groups, gn_groups, gw, gpq,
                                 stream)
             ? DMN_EHIP
             : DMN_OK;
}

static int oriented_params_check(const dmn_train_params_oriented* t) {
  if (!t || !depth_ok(t->depth) || ori_count(t->ori_shape) <= 0) return DMN_EINVAL;
  if (!t->v || !t->p || !t->q || !t->w || !t->state || !t->step) return DMN_EINVAL;
  return DMN_OK;
}

static dmn::TrainUpdateArgs oriented_args(const dmn_train_params_oriented* t) {
  dmn::TrainUpdateArgs a = {};
  a.v = t->v;
  a.alpha = t->p;
  a.beta = t->q;
  a.w = t->w;
  a.state = t->state;
  a.step = (long long*)t->step;
  a.half_period = 1;
  a.steps_per_epoch = 1;
  return a;
}

int dmn_training_update_oriented(const dmn_train_params_oriented* params, int prec,
                                 const void* gw, const void* gpq, const dmn_amsgrad_opts* opts,
                                 double* stats, hipStream_t stream) {
  if (const int rc = oriented_params_check(params)) return rc;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (!gw || !gpq || !opts || !stats) return DMN_EINVAL;
  const dmn_amsgrad_opts& o = *opts;
  if (!(o.lr_min >= 0.0) || !(o.lr_max >= 0.0) || !(o.lr_decay > 0.0) || o.half_period < 1 ||
      o.steps_per_epoch < 1 || !(o.beta1 >= 0.0 && o.beta1 < 1.0) ||
      !(o.beta2 >= 0.0 && o.beta2 < 1.0) || !(o.eps > 0.0) || !(o.penalty >= 0.0))
    return DMN_EINVAL;
  dmn::TrainUpdateArgs a = oriented_args(params);
  a.gw = gw;
  a.gn = gpq;
  a.stats = stats;
  a.lr_min = o.lr_min;
  a.lr_max = o.lr_max;
  a.lr_decay = o.lr_decay;
  a.beta1 = o.beta1;
  a.beta2 = o.beta2;
  a.eps = o.eps;
  a.penalty = o.penalty;
  a.half_period = o.half_period;
  a.steps_per_epoch = o.steps_per_epoch;
  a.take_step = 1;
  return dmn::launch_training_update_coeff(prec, params->depth, ori_count(params->ori_shape), a,
                                           stream)
             ? DMN_EHIP
             : DMN_OK;
}

int dmn_training_refresh_oriented(const dmn_train_params_oriented* params, int prec,
                                  hipStream_t stream) {
  if (const int rc = oriented_params_check(params)) return rc;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  dmn::TrainUpdateArgs a = oriented_args(params);
  a.take_step = 0;
  return dmn::launch_training_update_coeff(prec, params->depth, ori_count(params->ori_shape), a,
                                           stream)
             ? DMN_EHIP
             : DMN_OK;
}

int dmn_sample_stiffness(int64_t B, int prec, const double* u, void* C1, void* C2,
                         hipStream_t stream) {
  if (B < 0) return DMN_EINVAL;
  if (prec != DMN_F64 && prec != DMN_F32) return DMN_EUNSUPPORTED;
  if (B > 0 && (!u || !C1 || !C2)) return DMN_EINVAL;
  return dmn::launch_sample_stiffness(prec, B, u, C1, C2, stream) ? DMN_EHIP : DMN_OK;
}

}  // extern "C"
