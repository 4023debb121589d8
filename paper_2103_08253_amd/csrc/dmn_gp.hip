// Batched online evaluation of direct DMNs at Gauss points (FE-DMN paper,
// Sec. 3.2 online evaluation, Sec. 4.6 convergence test) on gfx950.
//
// Work mapping.  One 64-lane wavefront owns 64 / LP Gauss points; the LP
// lanes of a point split its laminate tree: lane t owns the depth-D subtree
// whose root is laminate (K-D+1, t+1) together with its 2^D leaves, and keeps
// that subtree's jumps, Newton increments and top-down factors in registers.
// The K-D levels above the lane subtrees are combined with wavefront shuffles
// (lane t receives its right sibling's condensed response from lane
// t + 2^(m-1)); their factors and jumps live in LDS, written and read only by
// the lane that computes the laminate.
//
// One evaluation at jumps a:
//   localisation: leaf strains eps = E + A a: each lane sums its upper
//                 ancestors' terms for its subtree root, then localises down
//                 its subtree while condensing it (one pass);
//   leaves:       fibre sigma = C_f eps; matrix J2 radial return -> sigma, D;
//   bottom-up:    block-Cholesky condensation of A^T W D A in postorder (no
//                 fill-in): condensed C, tau, plain average, residual blocks;
//   root:         C is the algorithmic tangent, the plain average the effective
//                 stress, the summed squared blocks |A^T W sigma|^2.
// A Newton step adds the top-down pass for the increments da.  Each loop trip
// of the kernel performs exactly one evaluation, at a + s da (s = 0 for the
// initial state, s = 1, 1/2, ... for backtracking trials), followed by the
// per-point decision; all shuffles run in wave-uniform code.
#include "dmn_tree.hpp"

namespace dmn {
namespace {

using namespace tree;

// ---------------------------------------------------------------- outputs

template <int K, int D, int H, typename S>
__device__ __forceinline__ void write_lane_a(const LaneState<K, D>& st, int t,
                                             S* __restrict__ aout) {
  if constexpr (H <= Cfg<K, D>::NLAM) {
    const int pos = lane_pos<K, D, H>(t);
#pragma unroll
    for (int k = 0; k < 3; ++k) aout[(size_t)pos * 3 + k] = (S)st.a[H - 1][k];
    write_lane_a<K, D, H + 1>(st, t, aout);
  }
}

// Write the point's outputs.  ok: converged (z_out was written by the leaf
// laws of the last evaluation, which is the accepted state); otherwise the
// input state is copied through and the tangent is NaN.  No shuffles: runs
// under per-point control flow.  S is the storage type of the per-point
// arrays; results are rounded to it on store.
template <int K, int D, typename S>
__device__ __forceinline__ void finalize(const Ctx<K, D>& cx, const LaneState<K, D>& st,
                                         const UpperLds<K, D>& up, const GroupArgs& G,
                                         long long pt, const EvalOut& ev, int status, int iters) {
  using C = Cfg<K, D>;
  const bool ok = status == 0;
  const int t = cx.t;
  S* aout = (S*)G.a_out + (size_t)pt * C::L * 3;
  if (ok) {
    write_lane_a<K, D, 1, S>(st, t, aout);
#pragma unroll 1
    for (int m = 1; m <= C::UPLEV; ++m) {
      if (upper_active(t, m)) {
        const int pos = upper_pos<K, D>(m, t);
        const int u = cx.slot * C::NUPS + (pos - C::UP0);
#pragma unroll
        for (int k = 0; k < 3; ++k) aout[(size_t)pos * 3 + k] = (S)up.a[k][u];
      }
    }
  } else {
    // failure: this lane copies its share of the input state through
    const S* zi = (const S*)cx.zin + (size_t)t * (C::NLEAF / 2) * 7;
    S* zo = (S*)G.z_out + (size_t)pt * C::M * 7 + (size_t)t * (C::NLEAF / 2) * 7;
#pragma unroll
    for (int q = 0; q < C::NLEAF / 2 * 7; ++q) zo[q] = zi[q];
    const S* ain = (const S*)G.a_in + (size_t)pt * C::L * 3;
    for (int i = t; i < C::L * 3; i += C::LP) aout[i] = ain[i];
  }
  if (t == 0) {
    S* sg = (S*)G.sigma + (size_t)pt * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) sg[k] = (S)ev.sb[k];
    S* tg = (S*)G.tangent + (size_t)pt * 36;
    const double nan = __builtin_nan("");
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) tg[i * 6 + j] = (S)(ok ? ev.C[sidx(i, j)] : nan);
    G.iters[pt] = iters;
    G.status[pt] = status;
  }
}

// ---------------------------------------------------------------- kernel

// Persistent waves: each 64-lane workgroup takes batches of PPW points from an
// atomic counter until the launch's batches are exhausted, so points with
// more Newton iterations do not leave SIMDs idle; the DMN table of the
// current group is staged in the wave's LDS when the group changes.  S is the
// storage type of the per-point arrays (double, or float for FP32 state);
// arithmetic is FP64 either way.  ORI: the groups' normals follow each point's
// fibre orientation and are computed into LDS when the wave takes a batch.
template <int K, int D, typename S, bool ORI>
__global__ __launch_bounds__(64) void gp_update_kernel(const GpLaunch args) {
  using C = Cfg<K, D>;
  __shared__ UpperLds<K, D> up;
  __shared__ TableLds<K> tlds;
  __shared__ NormalLds<K, D, ORI> nlds;
  const int lane = threadIdx.x;
  int cur = -1;
  const double* tabp = nullptr;
#pragma unroll 1
  while (true) {
  int item = 0;
  if (lane == 0) item = atomicAdd(args.counter, 1);
  item = __shfl(item, 0, 64);
  if (item >= args.total) break;
  int gi = 0;
#pragma unroll 1
  for (int q = 1; q < args.ng; ++q)
    if (item >= args.g[q].block0) gi = q;
  const GroupArgs& G = args.g[gi];
  if (gi != cur) {
    __syncthreads();
    tabp = stage_table<K>(tlds, G.tab + table_soa_offset(K));
    __syncthreads();
    cur = gi;
  }
  Ctx<K, D> cx;
  cx.slot = lane / C::LP;
  cx.t = lane % C::LP;
  cx.base = cx.slot * C::LP;
  cx.tab = tabp;
  cx.nrm = tabp + 2 * C::L;
  cx.fib = args.fib;
  cx.mat = args.mat;
  const long long pt_raw = (long long)(item - G.block0) * C::PPW + cx.slot;
  const bool in_range = pt_raw < G.P;
  const long long pt = in_range ? pt_raw : G.P - 1;  // tail lanes shadow the last point
  cx.zin = (const S*)G.z_in + (size_t)pt * C::M * 7;
  cx.zout = (S*)G.z_out + (size_t)pt * C::M * 7;
  const S* ain = (const S*)G.a_in + (size_t)pt * C::L * 3;
  const S* zin = (const S*)cx.zin;

  LaneState<K, D> st;
  EvalOut ev;
  double E[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) E[k] = (double)((const S*)G.E)[(size_t)pt * 6 + k];

  // load the jumps and check the inputs of the point for non-finite values
  int bad = 0;
  if constexpr (ORI) {
    const double l1 = G.lam[(size_t)pt * 2], l2 = G.lam[(size_t)pt * 2 + 1];
    bad |= (isfinite(l1) && isfinite(l2)) ? 0 : 1;
    double* nrm = nlds.v + cx.slot * 3 * C::L;
    orientation_normals<double>(G.ori_p, G.ori_q, G.ori_m, l1, l2, cx.t, C::LP, C::L, nrm,
                                nullptr);
    cx.nrm = nrm;  // read by the point's other lanes after the next barrier
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) bad |= isfinite(E[k]) ? 0 : 1;
#pragma unroll
  for (int q = 0; q < C::NLEAF / 2 * 7; ++q)
    bad |= isfinite((double)zin[(size_t)cx.t * (C::NLEAF / 2) * 7 + q]) ? 0 : 1;
#pragma unroll
  for (int h = 1; h <= C::NLAM; ++h) {
    const int m = ilog2(h);
    const int k = K - D + 1 + m;
    const int pos = (1 << K) - (1 << k) + cx.t * (1 << m) + (h - (1 << m));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      st.a[h - 1][c] = (double)ain[(size_t)pos * 3 + c];
      st.da[h - 1][c] = 0.0;
      bad |= isfinite(st.a[h - 1][c]) ? 0 : 1;
    }
  }
#pragma unroll 1
  for (int m = 1; m <= C::UPLEV; ++m) {
    if (upper_active(cx.t, m)) {
      const int pos = upper_pos<K, D>(m, cx.t);
      const int u = cx.slot * C::NUPS + (pos - C::UP0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = (double)ain[(size_t)pos * 3 + c];
        up.a[c][u] = v;
        up.da[c][u] = 0.0;
        bad |= isfinite(v) ? 0 : 1;
      }
    }
  }
#pragma unroll
  for (int o = 1; o < C::LP; o <<= 1) bad |= __shfl_xor(bad, o, C::LP);

  if (*G.flag != 0) {  // invalid DMN parameters: every point of the group fails
#pragma unroll
    for (int k = 0; k < 6; ++k) ev.sb[k] = __builtin_nan("");
    if (in_range) finalize<K, D, S>(cx, st, up, G, pt, ev, DMN_STATUS_BADPARAM, 0);
    continue;
  }

  const double scale = args.tol * (double)C::L;
  int status = 0, iters = 0, bt = 0;
  int polish = args.polish;  // full steps still to take after the stop test
  bool polishing = false;    // the current trial is such a step
  bool done = !in_range;
  bool first = true;
  double s = 0.0, rn = 0.0;
#pragma unroll 1
  while (true) {
    cx.wz = !done;
    evaluate_at<K, D, NewtonLeafS<S>>(cx, st, up, E, done ? 0.0 : s, ev);
    bool just_done = false, need_dir = false;
    if (!done) {
      bool accepted = false;
      if (first) {
        first = false;
        accepted = true;
        if (bad) {
          status = DMN_STATUS_NONFINITE;
          just_done = true;
        }
      } else {
        const double rt = sqrt(ev.rr);
        const bool good = isfinite(rt) && isfinite(ev.sn2) && !ev.lfail;
        if (polishing || (good && rt <= (1.0 - args.armijo * s) * rn) || bt >= args.max_bt) {
#pragma unroll
          for (int h = 0; h < C::NLAM; ++h)
#pragma unroll
            for (int k = 0; k < 3; ++k) st.a[h][k] += s * st.da[h][k];
#pragma unroll 1
          for (int m = 1; m <= C::UPLEV; ++m) {
            if (upper_active(cx.t, m)) {
              const int u = cx.slot * C::NUPS + (upper_pos<K, D>(m, cx.t) - C::UP0);
#pragma unroll
              for (int k = 0; k < 3; ++k) up.a[k][u] += s * up.da[k][u];
            }
          }
          if (!polishing) ++iters;
          polishing = false;
          accepted = true;
        } else {
          s *= 0.5;
          ++bt;
        }
      }
      if (accepted && !just_done) {
        rn = sqrt(ev.rr);
        const double sn = sqrt(ev.sn2);
        int fin = -1;
        if (ev.lfail) fin = DMN_STATUS_LOCAL;
        else if (!isfinite(rn) || !isfinite(sn)) fin = DMN_STATUS_NONFINITE;
        else if (rn == 0.0 || rn <= scale * sn) {
          if (ev.spdfail) fin = DMN_STATUS_NOTSPD;
          else if (polish > 0) {
            --polish;
            polishing = true;  // one more full step, then the test again
          } else {
            fin = 0;
          }
        } else if (iters >= args.max_iter) fin = DMN_STATUS_MAXITER;
        else if (ev.spdfail) fin = DMN_STATUS_NOTSPD;
        if (fin >= 0) {
          status = fin;
          just_done = true;
        } else {
          need_dir = true;
        }
      }
    }
    if (just_done) {
      finalize<K, D, S>(cx, st, up, G, pt, ev, status, iters);
      done = true;
    }
    if (!__any(!done)) break;
    if (__any(need_dir)) {
      direction(cx, st, up, need_dir);
      if (need_dir) {
        s = 1.0;
        bt = 0;
      }
    }
  }
  }  // persistent loop
}

}  // namespace

// ---------------------------------------------------------------- dispatch

// Compiled (depth K, lane-subtree depth D) variants; a point of a depth-K DMN
// then spans 2^(K-D) lanes.  (8, 3) is left out: its first GPU run ended in a
// device fault whose cause is not yet found.
#define DMN_GP_VARIANTS(X)                                                                 \
  X(1, 1) X(2, 1) X(2, 2) X(3, 1) X(3, 2) X(4, 1) X(4, 2) X(5, 1) X(5, 2) X(6, 1) X(6, 2) \
  X(7, 1) X(7, 2) X(8, 2) X(9, 3) X(10, 4)

int gp_default_lanes_per_point(int depth) {
  int d = depth - 6;
  if (d < 1) d = 1;
  return 1 << (depth - d);
}

int gp_lane_variants(int depth, int* lanes, int cap) {
  int n = 0;
#define DMN_GP_LIST(KK, DD)                              \
  if (KK == depth) {                                     \
    if (n < cap && lanes) lanes[n] = 1 << (KK - DD);     \
    ++n;                                                 \
  }
  DMN_GP_VARIANTS(DMN_GP_LIST)
#undef DMN_GP_LIST
  return n;
}

int gp_points_per_block(int depth, int lanes_per_point) {
  (void)depth;
  return 64 / lanes_per_point;
}

// Only FP64 storage is instantiated: the FP32-storage instantiation of this
// kernel is not compiled (its first GPU run ended in a device fault whose cause
// was not found); FP32 state runs this kernel on FP64 copies of the per-point
// arrays instead (see dmn_update_gauss_points).
// Orientation-interpolated normals are compiled for the default split of
// each depth only.
template <int K, int D>
static int launch_kd(int prec, bool ori, const GpLaunch& args, int n_blocks, hipStream_t stream) {
  if (prec != DMN_F64) return (int)hipErrorInvalidValue;
  if (ori) {
    if constexpr (D == (K - 6 < 1 ? 1 : K - 6))
      hipLaunchKernelGGL((gp_update_kernel<K, D, double, true>), dim3(n_blocks), dim3(64), 0,
                         stream, args);
    else
      return (int)hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((gp_update_kernel<K, D, double, false>), dim3(n_blocks), dim3(64), 0,
                       stream, args);
  }
  return (int)hipGetLastError();
}

int launch_gp_update(int depth, int lanes_per_point, int prec, bool ori, const GpLaunch& args,
                     int n_blocks, hipStream_t stream) {
  if (lanes_per_point < 1 || lanes_per_point > 64) return (int)hipErrorInvalidValue;
  const int D = depth - ilog2(lanes_per_point);
  switch (depth * 16 + D) {
#define DMN_GP_CASE(KK, DD) \
  case KK * 16 + DD:        \
    return launch_kd<KK, DD>(prec, ori, args, n_blocks, stream);
    DMN_GP_VARIANTS(DMN_GP_CASE)
#undef DMN_GP_CASE
    default:
      return (int)hipErrorInvalidValue;
  }
}

}  // namespace dmn
