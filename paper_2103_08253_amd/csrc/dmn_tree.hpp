// Shared device building blocks of the Gauss-point kernels: lane mapping of
// the laminate tree, strain localisation, bottom-up condensation and top-down
// solve (FE-DMN paper, Sec. 3.2).  See dmn_gp.hip for the mapping.
#pragma once
#include <utility>

#include "dmn_internal.hpp"

namespace dmn {
namespace tree {

template <int K, int D>
struct Cfg {
  static_assert(D >= 1 && D <= K, "subtree depth");
  static constexpr int LP = 1 << (K - D);  // lanes per point
  static_assert(LP <= 64, "at most one point per wave is split over lanes");
  static constexpr int PPW = 64 / LP;      // points per wave
  static constexpr int NLEAF = 1 << D;     // leaves per lane
  static constexpr int NLAM = NLEAF - 1;   // laminates per lane
  static constexpr int NUP = LP - 1;       // laminates above the lane subtrees
  static constexpr int NUPS = NUP > 0 ? NUP : 1;
  static constexpr int L = (1 << K) - 1;
  static constexpr int M = 1 << (K - 1);   // matrix leaves per point
  static constexpr int UP0 = (1 << K) - LP;  // paper position of the first upper laminate
  static constexpr int UPLEV = K - D;
  static constexpr int SLOTS = PPW * NUPS;
};

__host__ __device__ constexpr int ilog2(int h) { return h <= 1 ? 0 : 1 + ilog2(h / 2); }

// Shape of a lane subtree of depth D (independent of the tree's depth).
template <int D>
struct LaneCfg {
  static constexpr int NLEAF = 1 << D;  // leaves per lane
  static constexpr int NLAM = NLEAF - 1;  // laminates per lane
};

// Geometry of a depth-K point on the lanes: compile-time constants for
// K > 0; Geo<0, D> holds the same quantities at run time (the depth of the
// batch being processed), for the kernel that serves several depths.  The
// functions below read them through an object (cx.g.L etc.), which works for
// both forms.
template <int K, int D>
struct Geo {
  using C = Cfg<K, D>;
  static constexpr int depth = K;
  static constexpr int LP = C::LP, PPW = C::PPW, L = C::L, M = C::M, UP0 = C::UP0,
                       UPLEV = C::UPLEV, NUPS = C::NUPS;
};
template <int D>
struct Geo<0, D> {
  int depth, LP, PPW, L, M, UP0, UPLEV, NUPS;
  __device__ __forceinline__ void set(int K) {
    depth = K;
    LP = 1 << (K - D);
    PPW = 64 / LP;
    L = (1 << K) - 1;
    M = 1 << (K - 1);
    UP0 = (1 << K) - LP;
    UPLEV = K - D;
    NUPS = LP > 1 ? LP - 1 : 1;
  }
};

// paper position of the lane subtree's heap node H (1-based heap) of lane t
template <int D, int H, class G>
__device__ __forceinline__ int lane_pos(const G& g, int t) {
  constexpr int m = ilog2(H);
  const int K = g.depth;
  const int k = K - D + 1 + m;
  return (1 << K) - (1 << k) + t * (1 << m) + (H - (1 << m));
}

// paper position of the upper laminate computed by lane t at upper step m
template <int D, class G>
__device__ __forceinline__ int upper_pos(const G& g, int m, int t) {
  const int K = g.depth;
  const int k = K - D + 1 - m;
  return (1 << K) - (1 << k) + (t >> m);
}

struct LamRow {
  Normal<double> nv;
  double c1, c2, rf;
};

template <int K>
struct TableLds {
  static constexpr int L = (1 << K) - 1;
  static constexpr bool kInLds = L <= 511;
  double v[kInLds ? 6 * L : 1];
};

// Synchronisation of the lanes of one wavefront around LDS data that other
// lanes of the same wave wrote: the wave's LDS instructions execute in
// order, so only the compiler must not move memory accesses across it.
// Every kernel using the tree functions keeps the lanes that share a point
// inside one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copy of the field-major table into LDS by the lanes first, first + stride,
// ... (the caller synchronises).
template <int K>
__device__ __forceinline__ const double* stage_table(TableLds<K>& lds, const double* soa_global,
                                                     int first, int stride) {
  if constexpr (TableLds<K>::kInLds) {
    for (int i = first; i < 6 * TableLds<K>::L; i += stride) lds.v[i] = soa_global[i];
    return lds.v;
  } else {
    return soa_global;
  }
}

// Upper laminates of all points of a wave: PPW (LP - 1) = 64 - PPW for every
// depth, at most 63 (the run-time form takes the largest)
template <int K, int D>
struct UpperSlots {
  static constexpr int value = Cfg<K, D>::SLOTS;
};
template <int D>
struct UpperSlots<0, D> {
  static constexpr int value = 63;
};

// LDS storage of the upper laminates of all points of a wave (SoA by field):
// top-down factors and jumps per upper laminate.
template <int K, int D>
struct UpperLds {
  static constexpr int S = UpperSlots<K, D>::value;
  double G[18][S];
  double g[3][S];
  double a[3][S];
  double da[3][S];
};

// Lane-resident state of one point's lane subtree.
template <int K, int D>
struct LaneState {
  using C = LaneCfg<D>;
  double a[C::NLAM][3];   // accepted jumps
  double da[C::NLAM][3];  // Newton increments
  double G[C::NLAM][18];  // top-down factors of the last evaluation
  double g[C::NLAM][3];
};

struct EvalOut {
  double C[21];  // condensed tangent (meaningful on the point's lane 0)
  double sb[6];  // plain stress average (lane 0)
  double rr;     // squared residual norm (reduced over the point's lanes)
  double sn2;    // squared norm of the effective stress (broadcast)
  int lfail;     // J2 return failed somewhere in the point
  int spdfail;   // a laminate pivot was not positive
};

template <int K, int D>
struct Ctx {
  Geo<K, D> g;  // the point's geometry on the lanes
  const double* __restrict__ tab;
  const double* nrm;     // normals [3][L] of this point (the table's or its own)
  const void* zin;       // this point's z_in (storage precision of the kernel)
  void* zout = nullptr;  // this point's z_out, written by the leaf law when wz is set
  IsoElastic fib;
  J2Law mat;
  int t;
  int slot;
  int base;  // first lane of this point in the wave
  bool wz = false;
};

// Laminate row of the point: fractions and residual scale from the table,
// normal from the point's normal array.
template <int K, int D>
__device__ __forceinline__ LamRow load_row(const Ctx<K, D>& cx, int pos) {
  const int L = cx.g.L;
  LamRow o;
  o.c1 = cx.tab[0 * L + pos];
  o.c2 = cx.tab[1 * L + pos];
  o.rf = cx.tab[5 * L + pos];
  o.nv.n0 = cx.nrm[0 * L + pos];
  o.nv.n1 = cx.nrm[1 * L + pos];
  o.nv.n2 = cx.nrm[2 * L + pos];
  return o;
}

// LDS normals of the points of a wave, [slot][3][L], for orientation launches.
template <int K, int D, bool ORI>
struct NormalLds {
  double v[1];
};
template <int K, int D>
struct NormalLds<K, D, true> {
  double v[Cfg<K, D>::PPW * 3 * Cfg<K, D>::L];
};

__device__ __forceinline__ double shfl_down_d(double v, int o, int width) {
  return __shfl_down(v, (unsigned)o, width);
}
__device__ __forceinline__ double shfl_up_d(double v, int o, int width) {
  return __shfl_up(v, (unsigned)o, width);
}

__device__ __forceinline__ bool upper_active(int t, int m) { return (t & ((1 << m) - 1)) == 0; }
__device__ __forceinline__ bool upper_right(int t, int m) {
  return (t & ((1 << m) - 1)) == (1 << (m - 1));
}

// ------------------------------------------------------- strain localisation

template <int K, int D, int H>
__device__ __forceinline__ void loc_node(const Ctx<K, D>& cx, const LaneState<K, D>& st, double s,
                                         const double (&e)[6],
                                         double (&eps)[LaneCfg<D>::NLEAF][6]) {
  using C = LaneCfg<D>;
  if constexpr (H >= C::NLEAF) {
#pragma unroll
    for (int k = 0; k < 6; ++k) eps[H - C::NLEAF][k] = e[k];
  } else {
    const LamRow row = load_row(cx, lane_pos<D, H>(cx.g, cx.t));
    double aj[3], eL[6], eR[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) aj[k] = st.a[H - 1][k] + s * st.da[H - 1][k];
    laminate_localize(aj, e, row.nv, row.c1, row.c2, eL, eR);
    loc_node<K, D, 2 * H>(cx, st, s, eL, eps);
    loc_node<K, D, 2 * H + 1>(cx, st, s, eR, eps);
  }
}

// Leaf strains at jumps a + s da.  The macro strain reaching a lane's subtree
// root is E plus one term per upper ancestor (-c2 N a on the left of it,
// +c1 N a on the right), so every lane sums its ancestors' contributions
// directly, without a chain through the levels.  Reads jumps written by other
// lanes of the wave: synchronises first.
template <int K, int D>
__device__ __forceinline__ void localize(const Ctx<K, D>& cx, const LaneState<K, D>& st,
                                         const UpperLds<K, D>& up, const double (&E)[6], double s,
                                         double (&eps)[LaneCfg<D>::NLEAF][6]) {
  using C = LaneCfg<D>;
  wave_sync();
  double e[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) e[k] = E[k];
#pragma unroll 1
  for (int m = cx.g.UPLEV; m >= 1; --m) {
    const int lead = cx.t & ~((1 << m) - 1);
    const int pos = upper_pos<D>(cx.g, m, lead);
    const int u = cx.slot * cx.g.NUPS + (pos - cx.g.UP0);
    const LamRow row = load_row(cx, pos);
    double aj[3], Na[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) aj[k] = up.a[k][u] + s * up.da[k][u];
    row.nv.apply(aj, Na);
    const double f = ((cx.t >> (m - 1)) & 1) ? row.c1 : -row.c2;
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] += f * Na[k];
  }
  loc_node<K, D, 1>(cx, st, s, e, eps);
}

// ---------------------------------------------------------------- bottom-up

// Leaf law of the Newton evaluation: stress, tangent, and tau = stress.  S is
// the storage type of the internal variables.  With cx.wz set, the updated
// internal variables of the matrix leaves go to z_out (the last evaluation of
// a converged point is its accepted state, so z_out then holds the result).
template <typename S>
struct NewtonLeafS {
  template <int K, int D, int Q>
  __device__ __forceinline__ void operator()(const Ctx<K, D>& cx, std::integral_constant<int, Q>,
                                             const double (&e)[6], double (&Cn)[21],
                                             double (&tn)[6], double (&sn)[6], int& lfail) const {
    using C = LaneCfg<D>;
    if constexpr (Q % 2 == 0) {  // fibre leaf
      iso_stress(cx.fib, e, sn);
      iso_packed(cx.fib, Cn);
    } else {                     // matrix leaf
      const int mloc = cx.t * (C::NLEAF / 2) + Q / 2;
      const S* z = (const S*)cx.zin + (size_t)mloc * 7;
      double epn[6], ep[6], p;
#pragma unroll
      for (int k = 0; k < 6; ++k) epn[k] = (double)z[k];
      const bool ok = j2_return(cx.mat, e, epn, (double)z[6], sn, Cn, ep, p);
      lfail |= ok ? 0 : 1;
      if (cx.wz) {
        S* zo = (S*)cx.zout + (size_t)mloc * 7;
#pragma unroll
        for (int k = 0; k < 6; ++k) zo[k] = (S)ep[k];
        zo[6] = (S)p;
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) tn[k] = sn[k];
  }
};
using NewtonLeaf = NewtonLeafS<double>;

template <int K, int D, int H, class Leaf>
__device__ __forceinline__ void up_node(const Ctx<K, D>& cx, LaneState<K, D>& st, const Leaf& leaf,
                                        const double (&eps)[LaneCfg<D>::NLEAF][6],
                                        double (&Cn)[21], double (&tn)[6], double (&sn)[6],
                                        double& rr, int& lfail, int& spdfail) {
  using C = LaneCfg<D>;
  if constexpr (H >= C::NLEAF) {
    constexpr int q = H - C::NLEAF;
    leaf(cx, std::integral_constant<int, q>{}, eps[q], Cn, tn, sn, lfail);
  } else {
    up_node<K, D, 2 * H>(cx, st, leaf, eps, Cn, tn, sn, rr, lfail, spdfail);
    double CR[21], tR[6], sR[6];
    up_node<K, D, 2 * H + 1>(cx, st, leaf, eps, CR, tR, sR, rr, lfail, spdfail);
    const LamRow row = load_row(cx, lane_pos<D, H>(cx.g, cx.t));
    const bool ok = laminate_newton(Cn, tn, sn, CR, tR, sR, row.nv, row.c1, row.c2, row.rf,
                                    st.G[H - 1], st.g[H - 1], rr);
    spdfail |= ok ? 0 : 1;
  }
}

// Lane subtree with the strains localised on the way down: node H receives
// its strain e, its children e -/+ c N (a + s da); leaf laws at the leaves,
// condensation on the way up.  Each laminate row is read once.
template <int K, int D, int H, class Leaf>
__device__ __forceinline__ void up_node_loc(const Ctx<K, D>& cx, LaneState<K, D>& st,
                                            const Leaf& leaf, double s, const double (&e)[6],
                                            double (&Cn)[21], double (&tn)[6], double (&sn)[6],
                                            double& rr, int& lfail, int& spdfail) {
  using C = LaneCfg<D>;
  if constexpr (H >= C::NLEAF) {
    leaf(cx, std::integral_constant<int, H - C::NLEAF>{}, e, Cn, tn, sn, lfail);
  } else {
    const LamRow row = load_row(cx, lane_pos<D, H>(cx.g, cx.t));
    double aj[3], eL[6], eR[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) aj[k] = st.a[H - 1][k] + s * st.da[H - 1][k];
    laminate_localize(aj, e, row.nv, row.c1, row.c2, eL, eR);
    up_node_loc<K, D, 2 * H>(cx, st, leaf, s, eL, Cn, tn, sn, rr, lfail, spdfail);
    double CR[21], tR[6], sR[6];
    up_node_loc<K, D, 2 * H + 1>(cx, st, leaf, s, eR, CR, tR, sR, rr, lfail, spdfail);
    const bool ok = laminate_newton(Cn, tn, sn, CR, tR, sR, row.nv, row.c1, row.c2, row.rf,
                                    st.G[H - 1], st.g[H - 1], rr);
    spdfail |= ok ? 0 : 1;
  }
}

// Upper levels of the bottom-up condensation (shuffles between lanes) and the
// per-point reductions, after the lane subtrees (wave-uniform).
template <int K, int D>
__device__ __forceinline__ void evaluate_upper(const Ctx<K, D>& cx, UpperLds<K, D>& up,
                                               EvalOut& out, double (&cT)[6], double rr,
                                               int lfail, int spdfail, double* tau_out = nullptr) {
  using C = LaneCfg<D>;
#pragma unroll 1
  for (int m = 1; m <= cx.g.UPLEV; ++m) {
    const int o = 1 << (m - 1);
    double rC[21], rT[6], rS[6];
#pragma unroll
    for (int k = 0; k < 21; ++k) rC[k] = shfl_down_d(out.C[k], o, cx.g.LP);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      rT[k] = shfl_down_d(cT[k], o, cx.g.LP);
      rS[k] = shfl_down_d(out.sb[k], o, cx.g.LP);
    }
    if (upper_active(cx.t, m)) {
      const int pos = upper_pos<D>(cx.g, m, cx.t);
      const int u = cx.slot * cx.g.NUPS + (pos - cx.g.UP0);
      const LamRow row = load_row(cx, pos);
      double Gu[18], gu[3];
      const bool ok = laminate_newton(out.C, cT, out.sb, rC, rT, rS, row.nv, row.c1, row.c2,
                                      row.rf, Gu, gu, rr);
      spdfail |= ok ? 0 : 1;
#pragma unroll
      for (int k = 0; k < 18; ++k) up.G[k][u] = Gu[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) up.g[k][u] = gu[k];
    }
  }
  // reductions over the LP lanes of each point; broadcast of the root average
#pragma unroll
  for (int o = 1; o < cx.g.LP; o <<= 1) {
    rr += __shfl_xor(rr, o, cx.g.LP);
    lfail |= __shfl_xor(lfail, o, cx.g.LP);
    spdfail |= __shfl_xor(spdfail, o, cx.g.LP);
  }
  double sn2 = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double v = __shfl(out.sb[k], cx.base, 64);
    sn2 += v * v;
  }
  out.rr = rr;
  out.sn2 = sn2;
  out.lfail = lfail;
  out.spdfail = spdfail;
  if (tau_out != nullptr) {  // the affine offset of the point's (sub)tree root, lane 0
#pragma unroll
    for (int k = 0; k < 6; ++k) tau_out[k] = cT[k];
  }
}

// Leaf laws, bottom-up condensation and per-point reductions at leaf strains
// eps (wave-uniform: contains shuffles).
template <int K, int D, class Leaf = NewtonLeaf>
__device__ __forceinline__ void evaluate_full(const Ctx<K, D>& cx, LaneState<K, D>& st,
                                              UpperLds<K, D>& up,
                                              const double (&eps)[LaneCfg<D>::NLEAF][6],
                                              EvalOut& out, const Leaf& leaf = Leaf()) {
  double rr = 0.0;
  int lfail = 0, spdfail = 0;
  double cT[6];
  up_node<K, D, 1>(cx, st, leaf, eps, out.C, cT, out.sb, rr, lfail, spdfail);
  evaluate_upper(cx, up, out, cT, rr, lfail, spdfail);
}

// One whole evaluation at jumps a + s da: strain of each lane subtree's root
// (E plus its upper ancestors' terms), then the lane subtree with
// localisation fused into the condensation, then the upper levels and
// reductions.  Reads upper jumps written by other lanes: synchronises first.
template <int K, int D, class Leaf>
__device__ __forceinline__ void evaluate_at(const Ctx<K, D>& cx, LaneState<K, D>& st,
                                            UpperLds<K, D>& up, const double (&E)[6], double s,
                                            EvalOut& out, const Leaf& leaf = Leaf(),
                                            double* tau_out = nullptr) {
  using C = LaneCfg<D>;
  wave_sync();
  double e[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) e[k] = E[k];
#pragma unroll 1
  for (int m = cx.g.UPLEV; m >= 1; --m) {
    const int lead = cx.t & ~((1 << m) - 1);
    const int pos = upper_pos<D>(cx.g, m, lead);
    const int u = cx.slot * cx.g.NUPS + (pos - cx.g.UP0);
    const LamRow row = load_row(cx, pos);
    double aj[3], Na[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) aj[k] = up.a[k][u] + s * up.da[k][u];
    row.nv.apply(aj, Na);
    const double f = ((cx.t >> (m - 1)) & 1) ? row.c1 : -row.c2;
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] += f * Na[k];
  }
  double rr = 0.0;
  int lfail = 0, spdfail = 0;
  double cT[6];
  up_node_loc<K, D, 1>(cx, st, leaf, s, e, out.C, cT, out.sb, rr, lfail, spdfail);
  evaluate_upper(cx, up, out, cT, rr, lfail, spdfail, tau_out);
}

// ---------------------------------------------------------------- top-down

template <int K, int D, int H>
__device__ __forceinline__ void down_node(const Ctx<K, D>& cx, LaneState<K, D>& st, bool commit,
                                          const double (&e)[6],
                                          double (*leaf_de)[6] /* [NLEAF][6] or null */) {
  using C = LaneCfg<D>;
  if constexpr (H < C::NLEAF) {
    const LamRow row = load_row(cx, lane_pos<D, H>(cx.g, cx.t));
    double eL[6], eR[6], dah[3];
    laminate_descend(st.G[H - 1], st.g[H - 1], e, row.nv, row.c1, row.c2, dah, eL, eR);
    if (commit) {
#pragma unroll
      for (int k = 0; k < 3; ++k) st.da[H - 1][k] = dah[k];
    }
    down_node<K, D, 2 * H>(cx, st, commit, eL, leaf_de);
    down_node<K, D, 2 * H + 1>(cx, st, commit, eR, leaf_de);
  } else {
    if (leaf_de != nullptr) {
#pragma unroll
      for (int k = 0; k < 6; ++k) leaf_de[H - C::NLEAF][k] = e[k];
    }
  }
}

// Newton increments da for all laminates of the points with commit set.
// Every lane walks its own root path through the upper levels (lanes of a
// group repeat their shared ancestors' small top-down step instead of
// exchanging it); the group leader stores the upper increments.  Reads
// factors written by other lanes: synchronises first.
template <int K, int D>
__device__ __forceinline__ void direction(const Ctx<K, D>& cx, LaneState<K, D>& st,
                                          UpperLds<K, D>& up, bool commit,
                                          double (*leaf_de)[6] = nullptr,
                                          const double* e0 = nullptr) {
  using C = LaneCfg<D>;
  wave_sync();
  // the macro strain is fixed during Newton; a tree that is the subtree of a
  // point's root laminate starts from that laminate's strain increment e0
  double e[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) e[k] = e0 != nullptr ? e0[k] : 0.0;
#pragma unroll 1
  for (int m = cx.g.UPLEV; m >= 1; --m) {
    const int lead = cx.t & ~((1 << m) - 1);
    const int pos = upper_pos<D>(cx.g, m, lead);
    const int u = cx.slot * cx.g.NUPS + (pos - cx.g.UP0);
    const LamRow row = load_row(cx, pos);
    double Gu[18], gu[3], dau[3], eL[6], eR[6];
#pragma unroll
    for (int k = 0; k < 18; ++k) Gu[k] = up.G[k][u];
#pragma unroll
    for (int k = 0; k < 3; ++k) gu[k] = up.g[k][u];
    laminate_descend(Gu, gu, e, row.nv, row.c1, row.c2, dau, eL, eR);
    if (commit && cx.t == lead) {
#pragma unroll
      for (int k = 0; k < 3; ++k) up.da[k][u] = dau[k];
    }
    const bool right = (cx.t >> (m - 1)) & 1;
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = right ? eR[k] : eL[k];
  }
  down_node<K, D, 1>(cx, st, commit, e, leaf_de);
}

}  // namespace tree
}  // namespace dmn
