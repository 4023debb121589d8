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
#include <algorithm>

#include "dmn_tree.hpp"

namespace dmn {
namespace {

using namespace tree;

// ---------------------------------------------------------------- outputs

template <int K, int D, int H, typename S>
__device__ __forceinline__ void write_lane_a(const Ctx<K, D>& cx, const LaneState<K, D>& st,
                                             int t, S* __restrict__ aout) {
  if constexpr (H <= LaneCfg<D>::NLAM) {
    const int pos = lane_pos<D, H>(cx.g, t);
#pragma unroll
    for (int k = 0; k < 3; ++k) aout[(size_t)pos * 3 + k] = (S)st.a[H - 1][k];
    write_lane_a<K, D, H + 1>(cx, st, t, aout);
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
  using C = LaneCfg<D>;
  const bool ok = status == 0;
  const int t = cx.t;
  S* aout = (S*)G.a_out + (size_t)pt * cx.g.L * 3;
  if (ok) {
    write_lane_a<K, D, 1, S>(cx, st, t, aout);
#pragma unroll 1
    for (int m = 1; m <= cx.g.UPLEV; ++m) {
      if (upper_active(t, m)) {
        const int pos = upper_pos<D>(cx.g, m, t);
        const int u = cx.slot * cx.g.NUPS + (pos - cx.g.UP0);
#pragma unroll
        for (int k = 0; k < 3; ++k) aout[(size_t)pos * 3 + k] = (S)up.a[k][u];
      }
    }
  } else {
    // failure: this lane copies its share of the input state through
    const S* zi = (const S*)cx.zin + (size_t)t * (C::NLEAF / 2) * 7;
    S* zo = (S*)G.z_out + (size_t)pt * cx.g.M * 7 + (size_t)t * (C::NLEAF / 2) * 7;
#pragma unroll
    for (int q = 0; q < C::NLEAF / 2 * 7; ++q) zo[q] = zi[q];
    const S* ain = (const S*)G.a_in + (size_t)pt * cx.g.L * 3;
    for (int i = t; i < cx.g.L * 3; i += cx.g.LP) aout[i] = ain[i];
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

// One batch of PPW points of group G (item: the batch's index in the launch),
// processed by the 64 lanes of the calling wave.  up, tabp (the group's table,
// staged in LDS) and nrm_lds (orientation launches: per-point normals) are
// this wave's LDS.
template <int K, int D, typename S, bool ORI>
__device__ __forceinline__ void gp_batch(const GpLaunch& args, const GroupArgs& G, int item,
                                         int lane, UpperLds<K, D>& up, const double* tabp,
                                         double* nrm_lds) {
  using C = LaneCfg<D>;
  Ctx<K, D> cx;
  if constexpr (K == 0) cx.g.set(G.depth);  // the depth of this batch's group
  cx.slot = lane / cx.g.LP;
  cx.t = lane % cx.g.LP;
  cx.base = cx.slot * cx.g.LP;
  cx.tab = tabp;
  cx.nrm = tabp + 2 * cx.g.L;
  cx.fib = args.fib;
  cx.mat = args.mat;
  const long long pt_raw = (long long)(item - G.block0) * cx.g.PPW + cx.slot;
  const bool in_range = pt_raw < G.P;
  const long long pt = in_range ? pt_raw : G.P - 1;  // tail lanes shadow the last point
  cx.zin = (const S*)G.z_in + (size_t)pt * cx.g.M * 7;
  cx.zout = (S*)G.z_out + (size_t)pt * cx.g.M * 7;
  const S* ain = (const S*)G.a_in + (size_t)pt * cx.g.L * 3;
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
    double* nrm = nrm_lds + cx.slot * 3 * cx.g.L;
    orientation_normals<double>(G.ori_p, G.ori_q, G.ori_m, l1, l2, cx.t, cx.g.LP, cx.g.L, nrm,
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
    const int k = cx.g.depth - D + 1 + m;  // the point's depth (run time in the mixed kernel)
    const int pos = (1 << cx.g.depth) - (1 << k) + cx.t * (1 << m) + (h - (1 << m));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      st.a[h - 1][c] = (double)ain[(size_t)pos * 3 + c];
      st.da[h - 1][c] = 0.0;
      bad |= isfinite(st.a[h - 1][c]) ? 0 : 1;
    }
  }
#pragma unroll 1
  for (int m = 1; m <= cx.g.UPLEV; ++m) {
    if (upper_active(cx.t, m)) {
      const int pos = upper_pos<D>(cx.g, m, cx.t);
      const int u = cx.slot * cx.g.NUPS + (pos - cx.g.UP0);
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
  for (int o = 1; o < cx.g.LP; o <<= 1) bad |= __shfl_xor(bad, o, cx.g.LP);

  if (*G.flag != 0) {  // invalid DMN parameters: every point of the group fails
#pragma unroll
    for (int k = 0; k < 6; ++k) ev.sb[k] = __builtin_nan("");
    if (in_range) finalize<K, D, S>(cx, st, up, G, pt, ev, DMN_STATUS_BADPARAM, 0);
    return;
  }

  const double scale = args.tol * (double)cx.g.L;
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
          for (int m = 1; m <= cx.g.UPLEV; ++m) {
            if (upper_active(cx.t, m)) {
              const int u = cx.slot * cx.g.NUPS + (upper_pos<D>(cx.g, m, cx.t) - cx.g.UP0);
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
}

// Persistent waves: each 64-lane workgroup takes batches of PPW points from an
// atomic counter until the launch's batches are exhausted, so points with
// more Newton iterations do not leave SIMDs idle; the DMN table of the
// current group is staged in the wave's LDS when the group changes.  S is the
// storage type of the per-point arrays (double, or float for FP32 state);
// arithmetic is FP64 either way.  ORI: the groups' normals follow each point's
// fibre orientation and are computed into LDS when the wave takes a batch.
template <int K, int D, typename S, bool ORI>
__global__ __launch_bounds__(64) void gp_update_kernel(const GpLaunch args) {
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
      wave_sync();
      tabp = stage_table<K>(tlds, G.tab + table_soa_offset(K), lane, 64);
      wave_sync();
      cur = gi;
    }
    gp_batch<K, D, S, ORI>(args, G, item, lane, up, tabp, nlds.v);
  }
}

// ------------------------------------------------- depth 9: two waves per point

// A depth-9 point is split over the two waves of a workgroup: wave h owns the
// depth-8 subtree under child h of the root laminate (the mapping of a depth-8
// point, lane subtrees of depth 2), and the root laminate joins them through
// LDS.  No lane holds more than a depth-8 lane's state, so the point needs
// no more registers than a depth-8 point (the one-wave depth-9 variant spilled
// 1.6 KB per lane).

// Paper position, in the depth-9 tree, of position pos8 of the depth-8 subtree
// under child h of the root: level k' of pos8 (the root's child is k' = 1) has
// 256 - pos8 in (2^(k'-1), 2^k'], and the subtree's laminates of that level are
// the first (h = 0) or second half of the depth-9 level k' + 1.
__device__ __forceinline__ int split_pos(int pos8, int h) {
  const int kp = 32 - __clz(255 - pos8);  // ceil(log2(256 - pos8))
  return 256 + pos8 - (1 << kp) + h * (1 << (kp - 1));
}

// Root of a split point, shared by its two waves (LDS).
struct SplitRoot {
  double CR[21], tR[6], sR[6];  // right subtree's condensed response (wave 1)
  double C[21], tau[6], sb[6];  // left subtree's response (wave 0), then the root's:
                                // tangent, offset, effective stress
  double G[18], g[3];           // root factors; the Newton increment is -g
  double a[3], da[3];           // root jump and its increment
  double rr1, rr, sn2;
  int lfail1, spd1, lfail, spd, bad0, bad1;
  int item;
};

// Table of the subtree under root child h in depth-8 order, from the depth-9
// field-major table (lanes of the calling wave; the caller synchronises).
__device__ __forceinline__ const double* stage_split_table(TableLds<8>& lds, const double* soa9,
                                                          int h, int lane) {
  constexpr int L8 = 255, L9 = 511;
  for (int i = lane; i < 6 * L8; i += 64) {
    const int f = i / L8, p8 = i - f * L8;
    lds.v[i] = soa9[f * L9 + split_pos(p8, h)];
  }
  return lds.v;
}

template <typename S>
__device__ __forceinline__ void finalize_split(const Ctx<8, 2>& cx, const LaneState<8, 2>& st,
                                               const UpperLds<8, 2>& up, const GroupArgs& G,
                                               long long pt, int h, const SplitRoot& rs,
                                               int status, int iters) {
  using C = Cfg<8, 2>;
  constexpr int L9 = 511;
  const bool ok = status == 0;
  const int t = cx.t;
  S* aout = (S*)G.a_out + (size_t)pt * L9 * 3;
  if (ok) {
#pragma unroll
    for (int hh = 1; hh <= C::NLAM; ++hh) {
      const int m = ilog2(hh);
      const int k = 8 - 2 + 1 + m;
      const int pos = split_pos(256 - (1 << k) + t * (1 << m) + (hh - (1 << m)), h);
#pragma unroll
      for (int c = 0; c < 3; ++c) aout[(size_t)pos * 3 + c] = (S)st.a[hh - 1][c];
    }
#pragma unroll 1
    for (int m = 1; m <= C::UPLEV; ++m) {
      if (upper_active(t, m)) {
        const int p8 = upper_pos<2>(cx.g, m, t);
        const int pos = split_pos(p8, h);
        const int u = p8 - C::UP0;
#pragma unroll
        for (int c = 0; c < 3; ++c) aout[(size_t)pos * 3 + c] = (S)up.a[c][u];
      }
    }
    if (h == 0 && t == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) aout[(size_t)(L9 - 1) * 3 + c] = (S)rs.a[c];
    }
  } else {
    // failure: the input state is copied through (z by halves, a by both waves)
    const S* zi = (const S*)cx.zin + (size_t)t * (C::NLEAF / 2) * 7;
    S* zo = (S*)cx.zout + (size_t)t * (C::NLEAF / 2) * 7;
#pragma unroll
    for (int q = 0; q < C::NLEAF / 2 * 7; ++q) zo[q] = zi[q];
    const S* ain = (const S*)G.a_in + (size_t)pt * L9 * 3;
    for (int i = h * 64 + t; i < L9 * 3; i += 128) aout[i] = ain[i];
  }
  if (h == 0 && t == 0) {
    S* sg = (S*)G.sigma + (size_t)pt * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) sg[k] = (S)rs.sb[k];
    S* tg = (S*)G.tangent + (size_t)pt * 36;
    const double nan = __builtin_nan("");
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) tg[i * 6 + j] = (S)(ok ? rs.C[sidx(i, j)] : nan);
    G.iters[pt] = iters;
    G.status[pt] = status;
  }
}

// One depth-9 point, run by both waves of the workgroup (h = wave index) with
// identical control flow: every decision uses values both waves read from the
// SplitRoot, and the workgroup barriers below are reached by both.
template <typename S>
__device__ __forceinline__ void gp_split_point(const GpLaunch& args, const GroupArgs& G,
                                               long long pt, int h, int lane,
                                               UpperLds<8, 2>& up, const double* tabp,
                                               SplitRoot& rs, const LamRow& root) {
  using C = Cfg<8, 2>;
  constexpr int L9 = 511, M9 = 256;
  Ctx<8, 2> cx;
  cx.slot = 0;
  cx.t = lane;
  cx.base = 0;
  cx.tab = tabp;
  cx.nrm = tabp + 2 * C::L;
  cx.fib = args.fib;
  cx.mat = args.mat;
  cx.zin = (const S*)G.z_in + ((size_t)pt * M9 + (size_t)h * C::M) * 7;
  cx.zout = (S*)G.z_out + ((size_t)pt * M9 + (size_t)h * C::M) * 7;
  const S* ain = (const S*)G.a_in + (size_t)pt * L9 * 3;
  const S* zin = (const S*)cx.zin;

  LaneState<8, 2> st;
  EvalOut ev;
  double E[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) E[k] = (double)((const S*)G.E)[(size_t)pt * 6 + k];
  int bad = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) bad |= isfinite(E[k]) ? 0 : 1;
#pragma unroll
  for (int q = 0; q < C::NLEAF / 2 * 7; ++q)
    bad |= isfinite((double)zin[(size_t)cx.t * (C::NLEAF / 2) * 7 + q]) ? 0 : 1;
#pragma unroll
  for (int hh = 1; hh <= C::NLAM; ++hh) {
    const int m = ilog2(hh);
    const int k = 8 - 2 + 1 + m;
    const int pos = split_pos(256 - (1 << k) + cx.t * (1 << m) + (hh - (1 << m)), h);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      st.a[hh - 1][c] = (double)ain[(size_t)pos * 3 + c];
      st.da[hh - 1][c] = 0.0;
      bad |= isfinite(st.a[hh - 1][c]) ? 0 : 1;
    }
  }
#pragma unroll 1
  for (int m = 1; m <= C::UPLEV; ++m) {
    if (upper_active(cx.t, m)) {
      const int p8 = upper_pos<2>(cx.g, m, cx.t);
      const int pos = split_pos(p8, h);
      const int u = p8 - C::UP0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = (double)ain[(size_t)pos * 3 + c];
        up.a[c][u] = v;
        up.da[c][u] = 0.0;
        bad |= isfinite(v) ? 0 : 1;
      }
    }
  }
  if (h == 0 && lane == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rs.a[c] = (double)ain[(size_t)(L9 - 1) * 3 + c];
      rs.da[c] = 0.0;
      bad |= isfinite(rs.a[c]) ? 0 : 1;
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) bad |= __shfl_xor(bad, o, 64);
  if (lane == 0) {
    if (h == 0) rs.bad0 = bad;
    else rs.bad1 = bad;
  }
  __syncthreads();
  bad = rs.bad0 | rs.bad1;

  if (*G.flag != 0) {  // invalid DMN parameters: the point fails
    if (h == 0 && lane == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) rs.sb[k] = __builtin_nan("");
    }
    __syncthreads();
    finalize_split<S>(cx, st, up, G, pt, h, rs, DMN_STATUS_BADPARAM, 0);
    __syncthreads();  // rs is reused by the next point
    return;
  }

  const double scale = args.tol * (double)L9;
  const double fh = h == 0 ? -root.c2 : root.c1;  // the subtree's share of the root jump
  int status = 0, iters = 0, bt = 0;
  int polish = args.polish;
  bool polishing = false;
  bool first = true;
  double s = 0.0, rn = 0.0;
#pragma unroll 1
  while (true) {
    __syncthreads();  // the root jump and increment of the last step are visible
    double Eh[6];
    {
      double aj[3], Na[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) aj[c] = rs.a[c] + s * rs.da[c];
      root.nv.apply(aj, Na);
#pragma unroll
      for (int k = 0; k < 6; ++k) Eh[k] = E[k] + fh * Na[k];
    }
    cx.wz = true;
    double tauh[6];
    evaluate_at<8, 2, NewtonLeafS<S>>(cx, st, up, Eh, s, ev, NewtonLeafS<S>(), tauh);
    // the root laminate joins the two subtrees (wave 0, lane 0)
    // each subtree's root response goes to LDS (lane 0 of its wave); the root
    // laminate is then condensed in place on the LDS copies, so no lane holds
    // both responses in registers next to its lane-subtree state
    if (lane == 0) {
      double* Cd = h == 0 ? rs.C : rs.CR;
      double* td = h == 0 ? rs.tau : rs.tR;
      double* sd = h == 0 ? rs.sb : rs.sR;
#pragma unroll
      for (int k = 0; k < 21; ++k) Cd[k] = ev.C[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        td[k] = tauh[k];
        sd[k] = ev.sb[k];
      }
      if (h == 1) {
        rs.rr1 = ev.rr;
        rs.lfail1 = ev.lfail;
        rs.spd1 = ev.spdfail;
      }
    }
    __syncthreads();
    if (h == 0 && lane == 0) {
      double rr = ev.rr + rs.rr1;
      const bool ok = laminate_newton(rs.C, rs.tau, rs.sb, rs.CR, rs.tR, rs.sR, root.nv, root.c1,
                                      root.c2, root.rf, rs.G, rs.g, rr);
      double sn2 = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) sn2 += rs.sb[k] * rs.sb[k];
      rs.rr = rr;
      rs.sn2 = sn2;
      rs.lfail = ev.lfail | rs.lfail1;
      rs.spd = ev.spdfail | rs.spd1 | (ok ? 0 : 1);
    }
    __syncthreads();
    ev.rr = rs.rr;
    ev.sn2 = rs.sn2;
    ev.lfail = rs.lfail;
    ev.spdfail = rs.spd;

    bool just_done = false, need_dir = false;
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
        for (int q = 0; q < C::NLAM; ++q)
#pragma unroll
          for (int k = 0; k < 3; ++k) st.a[q][k] += s * st.da[q][k];
#pragma unroll 1
        for (int m = 1; m <= C::UPLEV; ++m) {
          if (upper_active(cx.t, m)) {
            const int u = upper_pos<2>(cx.g, m, cx.t) - C::UP0;
#pragma unroll
            for (int k = 0; k < 3; ++k) up.a[k][u] += s * up.da[k][u];
          }
        }
        if (h == 0 && lane == 0) {
#pragma unroll
          for (int k = 0; k < 3; ++k) rs.a[k] += s * rs.da[k];
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
          polishing = true;
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
    if (just_done) {
      __syncthreads();  // the root jump update is visible
      finalize_split<S>(cx, st, up, G, pt, h, rs, status, iters);
      __syncthreads();  // rs is reused by the next point
      return;
    }
    if (need_dir) {
      // root increment -g (its strain increment is zero), then each subtree
      // from the strain increment its root receives
      double dr[3], Nd[6], e0[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) dr[c] = -rs.g[c];
      root.nv.apply(dr, Nd);
#pragma unroll
      for (int k = 0; k < 6; ++k) e0[k] = fh * Nd[k];
      direction(cx, st, up, true, nullptr, e0);
      if (h == 0 && lane == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) rs.da[c] = dr[c];
      }
      s = 1.0;
      bt = 0;
    }
  }
}

// Groups of several depths in one persistent launch: workgroups of two waves.
// Phase 1: the points of depth-9 groups, one per workgroup at a time (split
// over both waves).  Phase 2: every wave takes batches of the other groups
// (depths 2 to 8, deepest first) on its own, with lane subtrees of depth 2 and
// the depth of each batch's group at run time (Geo<0, 2>: one code path for
// all depths); only wave-level synchronisation from there on.
constexpr int kMixedD = kMixedLaneDepth;
constexpr size_t kMixedWaveLds =
    (std::max(sizeof(UpperLds<0, kMixedD>), sizeof(UpperLds<8, 2>)) + sizeof(TableLds<8>) + 15) /
    16 * 16;

__global__ __launch_bounds__(128) void gp_mixed_kernel(const GpLaunch args) {
  __shared__ __align__(16) unsigned char smem[2 * kMixedWaveLds + sizeof(SplitRoot)];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned char* region = smem + wave * kMixedWaveLds;
  SplitRoot& rs = *reinterpret_cast<SplitRoot*>(smem + 2 * kMixedWaveLds);
  int cur = -1;
  const double* tabp = nullptr;
  if (args.total_split > 0) {
    UpperLds<8, 2>& up = *reinterpret_cast<UpperLds<8, 2>*>(region);
    TableLds<8>& tl = *reinterpret_cast<TableLds<8>*>(region + sizeof(UpperLds<8, 2>));
#pragma unroll 1
    while (true) {
      if (threadIdx.x == 0) rs.item = atomicAdd(args.counter_split, 1);
      __syncthreads();
      const int item = rs.item;
      __syncthreads();
      if (item >= args.total_split) break;
      int gi = 0;
#pragma unroll 1
      for (int q = 1; q < args.ng_split; ++q)
        if (item >= args.g[q].block0) gi = q;
      const GroupArgs& G = args.g[gi];
      const double* soa9 = G.tab + table_soa_offset(kSplitDepth);
      if (gi != cur) {
        wave_sync();
        tabp = stage_split_table(tl, soa9, wave, lane);
        wave_sync();
        cur = gi;
      }
      LamRow root;
      constexpr int L9 = 511;
      root.c1 = soa9[0 * L9 + L9 - 1];
      root.c2 = soa9[1 * L9 + L9 - 1];
      root.nv.n0 = soa9[2 * L9 + L9 - 1];
      root.nv.n1 = soa9[3 * L9 + L9 - 1];
      root.nv.n2 = soa9[4 * L9 + L9 - 1];
      root.rf = soa9[5 * L9 + L9 - 1];
      gp_split_point<double>(args, G, (long long)(item - G.block0), wave, lane, up, tabp, rs,
                             root);
    }
  }
  cur = -1;
  UpperLds<0, kMixedD>& upr = *reinterpret_cast<UpperLds<0, kMixedD>*>(region);
  TableLds<8>& tlr =
      *reinterpret_cast<TableLds<8>*>(region + sizeof(UpperLds<0, kMixedD>));
#pragma unroll 1
  while (true) {
    int item = 0;
    if (lane == 0) item = atomicAdd(args.counter, 1);
    item = __shfl(item, 0, 64);
    if (item >= args.total) break;
    int gi = args.ng_split;
#pragma unroll 1
    for (int q = args.ng_split + 1; q < args.ng; ++q)
      if (item >= args.g[q].block0) gi = q;
    const GroupArgs& G = args.g[gi];
    if (gi != cur) {  // the group's table, field-major [6][L], into this wave's LDS
      const double* soa = G.tab + table_soa_offset(G.depth);
      const int n = 6 * ((1 << G.depth) - 1);
      wave_sync();
      for (int i = lane; i < n; i += 64) tlr.v[i] = soa[i];
      wave_sync();
      cur = gi;
    }
    gp_batch<0, kMixedD, double, false>(args, G, item, lane, upr, tlr.v, nullptr);
  }
}

}  // namespace

// ---------------------------------------------------------------- dispatch

// Compiled (depth K, lane-subtree depth D) variants of the one-wave kernel; a
// point of a depth-K DMN then spans 2^(K-D) lanes.  Depth 9 runs split over
// two waves (kSplitLanes, the mixed kernel) instead: its one-wave variant
// (9, 3) holds about 1.5 KB of register spills per lane, as did the (8, 3)
// split, and spilling variants of that size have ended in device faults
// (see the design notes), so neither is compiled for the device.  A build
// may define the list itself (the sanitised CPU build adds (8, 3)).
#ifndef DMN_GP_VARIANTS
#define DMN_GP_VARIANTS(X)                                                                 \
  X(1, 1) X(2, 1) X(2, 2) X(3, 1) X(3, 2) X(4, 1) X(4, 2) X(5, 1) X(5, 2) X(6, 1) X(6, 2) \
  X(7, 1) X(7, 2) X(8, 2)
#endif

int gp_default_lanes_per_point(int depth) {
  if (depth == kSplitDepth) return kSplitLanes;
  int d = depth - 6;
  if (d < 1) d = 1;
  return 1 << (depth - d);
}

int gp_lane_variants(int depth, int* lanes, int cap) {
  if (depth == kSplitDepth) {
    if (cap > 0 && lanes) lanes[0] = kSplitLanes;
    return 1;
  }
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
  return lanes_per_point >= 64 ? 1 : 64 / lanes_per_point;
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

int launch_gp_mixed(const GpLaunch& args, int n_workgroups, hipStream_t stream) {
  hipLaunchKernelGGL(gp_mixed_kernel, dim3(n_workgroups), dim3(128), 0, stream, args);
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
