// Linear DMN homogenisation DMN^L (FE-DMN paper, Sec. 3.1: stiffness
// propagation from level K to the root, one rank-one laminate per node) and
// its vector-Jacobian product with respect to the leaf weights and the
// lamination normals (the gradients offline training needs).
//
// Work mapping as in the Gauss-point kernel: LP lanes per sample, lane t owns
// the depth-D subtree rooted at laminate (K-D+1, t+1); the K-D upper levels
// are combined with shuffles.  Leaves alternate between C1 (even) and C2
// (odd).  The backward pass recomputes the forward, keeping the lane
// subtree's node stiffnesses in registers and the lane roots and upper nodes
// in LDS, then runs the laminate VJPs from the root down.  A sample's two
// phase stiffnesses are the same for all its lanes and sit in LDS (broadcast
// reads) rather than in every lane's registers.  Parameter
// cotangents are accumulated per lane over the samples a wave processes and
// reduced over waves in a fixed order (bit-reproducible).
//
// A launch may carry several DMNs of one depth (sample groups, one table
// each): workgroup ranges map to groups, each group's samples and partial
// sums are contiguous, and the plain calls are the one-group case.
#include "dmn_groups.hpp"

namespace dmn {
namespace {

template <int K, int D>
struct LCfg {
  static constexpr int LP = 1 << (K - D);
  static constexpr int PPW = 64 / LP;
  static constexpr int NLEAF = 1 << D;
  static constexpr int NLAM = NLEAF - 1;
  static constexpr int NUP = LP - 1;
  static constexpr int L = (1 << K) - 1;
  static constexpr int UP0 = (1 << K) - LP;
  static constexpr int UPLEV = K - D;
  static constexpr int NODES = 2 * LP - 1;  // lane roots + upper laminates per sample
};

__host__ __device__ constexpr int ilog2l(int h) { return h <= 1 ? 0 : 1 + ilog2l(h / 2); }

template <int K, int D, int H>
__device__ __forceinline__ int lpos(int t) {
  constexpr int m = ilog2l(H);
  constexpr int k = K - D + 1 + m;
  return (1 << K) - (1 << k) + t * (1 << m) + (H - (1 << m));
}

// group of this workgroup (a scan over at most kMaxLinGroups entries; a
// group without workgroups is never selected)
__device__ __forceinline__ int lin_group(const LinGroups& grp) {
  int g = 0;
#pragma unroll 1
  for (int q = 1; q < grp.ng; ++q)
    if ((int)blockIdx.x >= grp.block0[q]) g = q;
  return g;
}

template <int K, int D>
__device__ __forceinline__ int upos(int m, int t) {
  const int k = K - D + 1 - m;
  return (1 << K) - (1 << k) + (t >> m);
}

template <typename T>
struct LRow {
  Normal<T> nv;
  T c1, c2;
};


// Orientation inputs of a launch whose normals follow each sample's fibre
// orientation (Sec. 2.3): angle coefficients p, q [L][m], per-sample
// (l1, l2) lam [B][2]; the backward writes each sample's angle cotangents
// (d/dalpha, d/dbeta) per laminate to gang [L][2][B].
template <typename T>
struct LinOri {
  const T* p;
  const T* q;
  const T* lam;
  T* gang;
  int m;
};

// Laminate rows: fractions from the table, normals from the table (fixed
// normals) or from the sample's normal block nrm [3][L] (ORI).
template <typename T, int L, bool ORI>
struct Rows {
  const T* __restrict__ tab;
  const T* nrm;
  __device__ __forceinline__ LRow<T> operator()(int pos) const {
    const T* r = tab + (size_t)pos * kTabStride;
    LRow<T> o;
    o.c1 = r[0];
    o.c2 = r[1];
    if constexpr (ORI) {
      o.nv.n0 = nrm[pos];
      o.nv.n1 = nrm[L + pos];
      o.nv.n2 = nrm[2 * L + pos];
    } else {
      o.nv.n0 = r[2];
      o.nv.n1 = r[3];
      o.nv.n2 = r[4];
    }
    return o;
  }
};

// symmetric part of a row-major 6x6, packed
template <typename T>
__device__ __forceinline__ void load_sym(const T* __restrict__ A, T P[21]) {
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j)
      P[sidx(i, j)] = i == j ? A[i * 6 + i] : T(0.5) * (A[i * 6 + j] + A[j * 6 + i]);
}

template <typename T>
__device__ __forceinline__ void store_full(T* __restrict__ A, const T P[21]) {
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) A[i * 6 + j] = P[sidx(i, j)];
}

// bottom-up over the lane subtree; stores the laminate outputs when Store
template <typename T, int K, int D, int H, bool Store, class R>
__device__ __forceinline__ void lin_up(const R& rows, int t, const T* C1,
                                       const T* C2, T (&Cn)[21], int& fail,
                                       T (&nodes)[LCfg<K, D>::NLAM][21]) {
  using C = LCfg<K, D>;
  if constexpr (H >= C::NLEAF) {
    constexpr int q = H - C::NLEAF;
#pragma unroll
    for (int k = 0; k < 21; ++k) Cn[k] = (q % 2 == 0) ? C1[k] : C2[k];
  } else {
    T CL[21], CR[21];
    lin_up<T, K, D, 2 * H, Store>(rows, t, C1, C2, CL, fail, nodes);
    lin_up<T, K, D, 2 * H + 1, Store>(rows, t, C1, C2, CR, fail, nodes);
    const LRow<T> row = rows(lpos<K, D, H>(t));
    fail |= laminate_linear(CL, CR, row.nv, row.c1, row.c2, Cn) ? 0 : 1;
    if constexpr (Store) {
#pragma unroll
      for (int k = 0; k < 21; ++k) nodes[H - 1][k] = Cn[k];
    }
  }
}

template <typename T>
__device__ __forceinline__ T shfl_dn(T v, int o, int w) {
  return __shfl_down(v, (unsigned)o, w);
}
template <typename T>
__device__ __forceinline__ T shfl_upv(T v, int o, int w) {
  return __shfl_up(v, (unsigned)o, w);
}

template <typename T, int K, int D, bool ORI>
__global__ __launch_bounds__(64) void linear_fwd_kernel(const T* __restrict__ tab0,
                                                        const int32_t* __restrict__ flag0,
                                                        const T* __restrict__ C1,
                                                        const T* __restrict__ C2,
                                                        T* __restrict__ Cbar,
                                                        int32_t* __restrict__ err,
                                                        const LinOri<T> ori,
                                                        const LinGroups grp) {
  using C = LCfg<K, D>;
  __shared__ T leafC[C::PPW][2][21];
  __shared__ T nl[ORI ? C::PPW * 3 * C::L : 1];
  const int lane = threadIdx.x;
  const int slot = lane / C::LP, t = lane % C::LP;
  const int g = lin_group(grp);
  const T* tab = (const T*)((const char*)tab0 + g * grp.tab_stride);
  const int32_t* flag = (const int32_t*)((const char*)flag0 + g * grp.tab_stride);
  const long long s0 = grp.off[g], Bg = grp.off[g + 1] - s0;
  const long long braw = (long long)(blockIdx.x - grp.block0[g]) * C::PPW + slot;
  const bool in_range = braw < Bg;
  const long long b = s0 + (in_range ? braw : Bg - 1);
  if (t == 0) {
    load_sym(C1 + (size_t)b * 36, leafC[slot][0]);
    load_sym(C2 + (size_t)b * 36, leafC[slot][1]);
  }
  T* nrm = nl + (ORI ? slot * 3 * C::L : 0);
  if constexpr (ORI)
    orientation_normals<T>(ori.p, ori.q, ori.m, ori.lam[(size_t)b * 2], ori.lam[(size_t)b * 2 + 1],
                           t, C::LP, C::L, nrm, (T*)nullptr);
  __syncthreads();
  const Rows<T, C::L, ORI> rows{tab, nrm};
  int fail = 0;
  T cC[21];
  T dummy[C::NLAM][21];
  lin_up<T, K, D, 1, false>(rows, t, leafC[slot][0], leafC[slot][1], cC, fail, dummy);
#pragma unroll 1
  for (int m = 1; m <= C::UPLEV; ++m) {
    const int o = 1 << (m - 1);
    T rC[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) rC[k] = shfl_dn(cC[k], o, C::LP);
    if ((t & (2 * o - 1)) == 0) {
      const LRow<T> row = rows(upos<K, D>(m, t));
      T nC[21];
      fail |= laminate_linear(cC, rC, row.nv, row.c1, row.c2, nC) ? 0 : 1;
#pragma unroll
      for (int k = 0; k < 21; ++k) cC[k] = nC[k];
    }
  }
#pragma unroll
  for (int o = 1; o < C::LP; o <<= 1) fail |= __shfl_xor(fail, o, C::LP);
  const int invalid = *flag;
  if (t == 0 && in_range) {
    if (fail || invalid) {
#pragma unroll
      for (int k = 0; k < 21; ++k) cC[k] = T(__builtin_nan(""));
      atomicOr(err, (invalid ? 1 : 0) | (fail ? 2 : 0));
    }
    store_full(Cbar + (size_t)b * 36, cC);
  }
}

// Two samples per wave where the forward gives one sample all 64 lanes
// (depths 7 and up with fixed normals).  Every lane runs its lane subtree for
// sample B, parks the result in LDS, then runs it for sample A; the upper
// levels then serve both samples in the same steps.  At level m (o = 2^(m-1))
// sample A's laminate sits on the first lane of each group of 2o lanes and
// takes its right child from lane t + o, sample B's on the group's last lane,
// taking its left child from lane t - o; after level m A's partial results sit
// on multiples of 2o and B's on lanes 2o - 1 mod 2o, so the two sets never
// meet.  Each sample sees the same laminate operations in the same order as
// in linear_fwd_kernel; the compiler may still contract them into FMAs
// differently in the two kernels, so the results agree within rounding (a
// few ulps), not always bit for bit.  Two waves per SIMD: the FP64 depth-8
// instance fits the 256 registers that allows.
template <typename T, int K, int D>
__global__ __launch_bounds__(64, 2) void linear_fwd_pair_kernel(const T* __restrict__ tab0,
                                                             const int32_t* __restrict__ flag0,
                                                             const T* __restrict__ C1,
                                                             const T* __restrict__ C2,
                                                             T* __restrict__ Cbar,
                                                             int32_t* __restrict__ err,
                                                             const LinGroups grp) {
  using C = LCfg<K, D>;
  static_assert(C::LP == 64, "the pair mapping needs one sample per wave");
  __shared__ T leafC[2][2][21];
  __shared__ T rootB[21][64];
  const int t = threadIdx.x;
  const int g = lin_group(grp);
  const T* tab = (const T*)((const char*)tab0 + g * grp.tab_stride);
  const int32_t* flag = (const int32_t*)((const char*)flag0 + g * grp.tab_stride);
  const long long s0 = grp.off[g], Bg = grp.off[g + 1] - s0;
  const long long first = (long long)(blockIdx.x - grp.block0[g]) * 2;
  // samples A = first (always in range) and B = first + 1 of the group; a
  // missing B (odd group size) shadows A and is not stored
  if (t < 2) {
    const long long b = s0 + first + (t == 1 && first + 1 < Bg ? 1 : 0);
    load_sym(C1 + (size_t)b * 36, leafC[t][0]);
    load_sym(C2 + (size_t)b * 36, leafC[t][1]);
  }
  __syncthreads();
  const Rows<T, C::L, false> rows{tab, nullptr};
  int failA = 0, failB = 0;
  T dummy[C::NLAM][21];
  {
    T cB[21];
    lin_up<T, K, D, 1, false>(rows, t, leafC[1][0], leafC[1][1], cB, failB, dummy);
#pragma unroll
    for (int k = 0; k < 21; ++k) rootB[k][t] = cB[k];  // read back by this lane only
  }
  T cur[21];
  lin_up<T, K, D, 1, false>(rows, t, leafC[0][0], leafC[0][1], cur, failA, dummy);
#pragma unroll 1
  for (int m = 1; m <= C::UPLEV; ++m) {
    const int o = 1 << (m - 1);
    const int r = t & (2 * o - 1);
    const bool actA = r == 0, actB = r == 2 * o - 1;
    const int src = actA ? t + o : (actB ? t - o : t);
    T rC[21];
    if (m == 1) {
      // every lane holds both lane roots: even lanes pass B's, odd lanes A's,
      // and an odd lane's right child is its own B root
#pragma unroll
      for (int k = 0; k < 21; ++k) rC[k] = __shfl((t & 1) ? cur[k] : rootB[k][t], src, 64);
      if (t & 1) {
#pragma unroll
        for (int k = 0; k < 21; ++k) cur[k] = rootB[k][t];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 21; ++k) rC[k] = __shfl(cur[k], src, 64);
    }
    if (actB) {  // B's left child arrived from the lane before: left = cur
#pragma unroll
      for (int k = 0; k < 21; ++k) {
        const T x = cur[k];
        cur[k] = rC[k];
        rC[k] = x;
      }
    }
    if (actA || actB) {
      const LRow<T> row = rows(upos<K, D>(m, t));
      // the result overwrites the left operand: laminate_linear reads each
      // packed entry of its operands before it writes that entry of the result
      const int bad = laminate_linear(cur, rC, row.nv, row.c1, row.c2, cur) ? 0 : 1;
      if (actA) failA |= bad;
      else failB |= bad;
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    failA |= __shfl_xor(failA, o, 64);
    failB |= __shfl_xor(failB, o, 64);
  }
  const int invalid = *flag;
  // A's root is on lane 0, B's on lane 63
  if ((t == 0) || (t == 63 && first + 1 < Bg)) {
    const int fail = t == 0 ? failA : failB;
    if (fail || invalid) {
#pragma unroll
      for (int k = 0; k < 21; ++k) cur[k] = T(__builtin_nan(""));
      atomicOr(err, (invalid ? 1 : 0) | (fail ? 2 : 0));
    }
    store_full(Cbar + (size_t)(s0 + first + (t == 0 ? 0 : 1)) * 36, cur);
  }
}

// Angle cotangents of laminate pos of sample b from its normal cotangent gn:
// d/dalpha = gn . dn/dalpha, d/dbeta = gn . (-n1, n0, 0).
template <typename T, int L>
__device__ __forceinline__ void put_angles(const LinOri<T>& ori, long long B, long long b, int pos,
                                           const T* nrm, const T gn[3]) {
  const T* da = nrm + 3 * L;
  const T ga = gn[0] * da[pos] + gn[1] * da[L + pos] + gn[2] * da[2 * L + pos];
  const T gb = -gn[0] * nrm[L + pos] + gn[1] * nrm[pos];
  ori.gang[((size_t)pos * 2) * B + b] = ga;
  ori.gang[((size_t)pos * 2 + 1) * B + b] = gb;
}

// backward over the lane subtree: cotangent Gm of heap node H; the phase
// stiffness cotangents g1, g2 are accumulated only if IG; with ORI the
// sample's angle cotangents go to ori.gang
template <typename T, int K, int D, int H, bool IG, bool ORI, class R>
__device__ __forceinline__ void lin_back(const R& rows, const LinOri<T>& ori, long long B,
                                         long long b, int t, bool live,
                                         const T* C1, const T* C2,
                                         const T (&nodes)[LCfg<K, D>::NLAM][21],
                                         const T (&Gm)[21],
                                         double (&acc)[LCfg<K, D>::NLAM][4][64],
                                         T (&g1)[IG ? 21 : 1], T (&g2)[IG ? 21 : 1]) {
  using C = LCfg<K, D>;
  if constexpr (H >= C::NLEAF) {
    if constexpr (IG) {
      constexpr int q = H - C::NLEAF;
#pragma unroll
      for (int k = 0; k < 21; ++k) {
        if constexpr (q % 2 == 0) g1[k] += Gm[k];
        else g2[k] += Gm[k];
      }
    }
  } else {
    const T* CL;
    const T* CR;
    if constexpr (2 * H >= C::NLEAF) {
      CL = C1;
      CR = C2;
    } else {
      CL = nodes[2 * H - 1];
      CR = nodes[2 * H];
    }
    const int pos = lpos<K, D, H>(t);
    const LRow<T> row = rows(pos);
    T GL[21], GR[21], gc1, gn[3];
    laminate_linear_vjp(CL, CR, row.nv, row.c1, row.c2, Gm, GL, GR, gc1, gn);
    if (live) {
      const int ln = threadIdx.x;
      acc[H - 1][0][ln] += (double)gc1;
      acc[H - 1][1][ln] += (double)gn[0];
      acc[H - 1][2][ln] += (double)gn[1];
      acc[H - 1][3][ln] += (double)gn[2];
      if constexpr (ORI) put_angles<T, C::L>(ori, B, b, pos, rows.nrm, gn);
    }
    lin_back<T, K, D, 2 * H, IG, ORI>(rows, ori, B, b, t, live, C1, C2, nodes, GL, acc, g1, g2);
    lin_back<T, K, D, 2 * H + 1, IG, ORI>(rows, ori, B, b, t, live, C1, C2, nodes, GR, acc, g1,
                                          g2);
  }
}

template <typename T, int K, int D, bool IG, bool ORI>
__global__ __launch_bounds__(64) void linear_bwd_kernel(
    const T* __restrict__ tab0, const int32_t* __restrict__ flag0, long long B,
    const T* __restrict__ C1, const T* __restrict__ C2, const T* __restrict__ gCbar,
    T* __restrict__ gC1, T* __restrict__ gC2, double* __restrict__ partials,
    int32_t* __restrict__ err, const LinOri<T> ori, const LinGroups grp) {
  using C = LCfg<K, D>;
  static_assert(C::NLAM >= 1, "lane subtree needs a laminate");
  __shared__ T nodeC[21][C::PPW * C::NODES];
  __shared__ T leafC[C::PPW][2][21];
  __shared__ T nl[ORI ? C::PPW * 6 * C::L : 1];  // normals, then dn/dalpha, per sample
  __shared__ double accU[4][C::PPW * (C::NUP > 0 ? C::NUP : 1)];
  const int lane = threadIdx.x;
  const int slot = lane / C::LP, t = lane % C::LP;
  for (int u = lane; u < C::PPW * (C::NUP > 0 ? C::NUP : 1); u += 64)
    for (int c = 0; c < 4; ++c) accU[c][u] = 0.0;
  // per-lane sums of the lane-subtree laminates' cotangents, in LDS (each lane
  // its own column) rather than held in registers through the whole loop
  __shared__ double acc[C::NLAM][4][64];
#pragma unroll
  for (int h = 0; h < C::NLAM; ++h)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[h][c][lane] = 0.0;
  int fail = 0;
  // this workgroup's group: its table, samples s0 .. s0+Bg-1 and workgroups
  const int g = lin_group(grp);
  const T* tab = (const T*)((const char*)tab0 + g * grp.tab_stride);
  const int32_t* flag = (const int32_t*)((const char*)flag0 + g * grp.tab_stride);
  const long long s0 = grp.off[g], Bg = grp.off[g + 1] - s0;
  const int gb = (int)blockIdx.x - grp.block0[g];
  const int gblocks = grp.block0[g + 1] - grp.block0[g];
  __syncthreads();
  for (long long sg = gb; sg * C::PPW < Bg; sg += gblocks) {
    const long long braw = sg * C::PPW + slot;
    const bool live = braw < Bg;
    const long long b = s0 + (live ? braw : Bg - 1);
    if (t == 0) {
      load_sym(C1 + (size_t)b * 36, leafC[slot][0]);
      load_sym(C2 + (size_t)b * 36, leafC[slot][1]);
    }
    T* nrm = nl + (ORI ? slot * 6 * C::L : 0);
    if constexpr (ORI)
      orientation_normals<T>(ori.p, ori.q, ori.m, ori.lam[(size_t)b * 2],
                             ori.lam[(size_t)b * 2 + 1], t, C::LP, C::L, nrm, nrm + 3 * C::L);
    __syncthreads();
    const Rows<T, C::L, ORI> rows{tab, nrm};
    const T* A1 = leafC[slot][0];
    const T* A2 = leafC[slot][1];
    // forward, keeping node stiffnesses
    T nodes[C::NLAM][21];
    T cC[21];
    lin_up<T, K, D, 1, true>(rows, t, A1, A2, cC, fail, nodes);
    const int nbase = slot * C::NODES;
#pragma unroll
    for (int k = 0; k < 21; ++k) nodeC[k][nbase + t] = cC[k];
#pragma unroll 1
    for (int m = 1; m <= C::UPLEV; ++m) {
      const int o = 1 << (m - 1);
      T rC[21];
#pragma unroll
      for (int k = 0; k < 21; ++k) rC[k] = shfl_dn(cC[k], o, C::LP);
      if ((t & (2 * o - 1)) == 0) {
        const int pos = upos<K, D>(m, t);
        const LRow<T> row = rows(pos);
        T nC[21];
        fail |= laminate_linear(cC, rC, row.nv, row.c1, row.c2, nC) ? 0 : 1;
#pragma unroll
        for (int k = 0; k < 21; ++k) {
          cC[k] = nC[k];
          nodeC[k][nbase + C::LP + (pos - C::UP0)] = nC[k];
        }
      }
    }
    __syncthreads();
    // backward: root cotangent is the symmetric part of gCbar
    T Gm[21];
    load_sym(gCbar + (size_t)b * 36, Gm);
#pragma unroll 1
    for (int m = C::UPLEV; m >= 1; --m) {
      const int o = 1 << (m - 1);
      T GRs[21];
#pragma unroll
      for (int k = 0; k < 21; ++k) GRs[k] = T(0);
      if ((t & (2 * o - 1)) == 0) {
        const int pos = upos<K, D>(m, t);
        const LRow<T> row = rows(pos);
        const int vL = m == 1 ? t : C::LP + (upos<K, D>(m - 1, t) - C::UP0);
        const int vR = m == 1 ? t + 1 : C::LP + (upos<K, D>(m - 1, t + o) - C::UP0);
        T CL[21], CR[21];
#pragma unroll
        for (int k = 0; k < 21; ++k) {
          CL[k] = nodeC[k][nbase + vL];
          CR[k] = nodeC[k][nbase + vR];
        }
        T GL[21], gc1, gn[3];
        laminate_linear_vjp(CL, CR, row.nv, row.c1, row.c2, Gm, GL, GRs, gc1, gn);
        if (live) {
          const int u = slot * (C::NUP > 0 ? C::NUP : 1) + (pos - C::UP0);
          accU[0][u] += (double)gc1;
          accU[1][u] += (double)gn[0];
          accU[2][u] += (double)gn[1];
          accU[3][u] += (double)gn[2];
          if constexpr (ORI) put_angles<T, C::L>(ori, B, b, pos, nrm, gn);
        }
#pragma unroll
        for (int k = 0; k < 21; ++k) Gm[k] = GL[k];
      }
      T rcv[21];
#pragma unroll
      for (int k = 0; k < 21; ++k) rcv[k] = shfl_upv(GRs[k], o, C::LP);
      if ((t & (2 * o - 1)) == o) {
#pragma unroll
        for (int k = 0; k < 21; ++k) Gm[k] = rcv[k];
      }
    }
    T g1[IG ? 21 : 1], g2[IG ? 21 : 1];
#pragma unroll
    for (int k = 0; k < (IG ? 21 : 1); ++k) {
      g1[k] = T(0);
      g2[k] = T(0);
    }
    lin_back<T, K, D, 1, IG, ORI>(rows, ori, B, b, t, live, A1, A2, nodes, Gm, acc, g1, g2);
    if constexpr (IG) {
#pragma unroll
      for (int o = 1; o < C::LP; o <<= 1)
#pragma unroll
        for (int k = 0; k < 21; ++k) {
          g1[k] += __shfl_xor(g1[k], o, C::LP);
          g2[k] += __shfl_xor(g2[k], o, C::LP);
        }
      if (t == 0 && live) {
        store_full(gC1 + (size_t)b * 36, g1);
        store_full(gC2 + (size_t)b * 36, g2);
      }
    }
    __syncthreads();  // nodeC, leafC and nl are rewritten by the next sample group
  }
  // partial sums of this wave slot, stored [pos * 4 + c][slot] in the
  // group's region (its slots follow those of the groups before it)
  const size_t pslot = (size_t)gb * C::PPW + slot;
  const size_t nslots = (size_t)gblocks * C::PPW;
  double* gpart = partials + (size_t)grp.block0[g] * C::PPW * (4 * C::L);
  auto put = [&](int pos, const double* v) {
#pragma unroll
    for (int c = 0; c < 4; ++c) gpart[((size_t)pos * 4 + c) * nslots + pslot] = v[c];
  };
  [&] {
    if constexpr (C::NLAM >= 1) {
      // lane subtree laminates
#pragma unroll
      for (int h = 1; h <= C::NLAM; ++h) {
        const int m = ilog2l(h);
        const int k = K - D + 1 + m;
        const int pos = (1 << K) - (1 << k) + t * (1 << m) + (h - (1 << m));
        const double v[4] = {acc[h - 1][0][lane], acc[h - 1][1][lane], acc[h - 1][2][lane],
                             acc[h - 1][3][lane]};
        put(pos, v);
      }
    }
  }();
#pragma unroll
  for (int m = 1; m <= C::UPLEV; ++m) {
    const int o = 1 << (m - 1);
    if ((t & (2 * o - 1)) == 0) {
      const int pos = upos<K, D>(m, t);
      const int u = slot * (C::NUP > 0 ? C::NUP : 1) + (pos - C::UP0);
      double v[4] = {accU[0][u], accU[1][u], accU[2][u], accU[3][u]};
      put(pos, v);
    }
  }
#pragma unroll
  for (int o = 1; o < C::LP; o <<= 1) fail |= __shfl_xor(fail, o, C::LP);
  if (lane == 0 && (fail || *flag)) atomicOr(err, (*flag ? 1 : 0) | (fail ? 2 : 0));
}

// The backward with two samples per wave where it gives one sample all 64
// lanes and the registers allow it (FP32 at depths 7 and 8, FP64 at depth 7;
// fixed normals, no phase-stiffness cotangents).  Per pair of samples A, B:
// every lane computes both samples' lane-subtree roots, and the upper levels
// run forward for both in the same steps as in linear_fwd_pair_kernel,
// storing the upper nodes' stiffnesses in LDS; their VJPs then run top-down
// for both in the same steps down to level 2: A's laminate on the first lane
// of a group of 2o lanes keeps its left child's cotangent and sends the right
// one to lane t + o, B's on the group's last lane keeps the right one and
// sends the left one to lane t - o (the lanes acting for A, for B, receiving
// for A and receiving for B are four different residues mod 2o).  Last, for A
// and then B, the sample's lane subtree is recomputed, its level-1 laminate's
// VJP runs on one lane of each pair (the cotangent waited in the LDS the
// upper nodes used) and the lane subtree's VJPs follow.  Each sample's
// laminate operations are those of linear_bwd_kernel; the upper laminates'
// cotangent sums are kept per sample slot and added A then B at the end, a
// fixed order.
template <typename T, int K, int D>
__global__ __launch_bounds__(64) void linear_bwd_pair_kernel(
    const T* __restrict__ tab0, const int32_t* __restrict__ flag0, const T* __restrict__ C1,
    const T* __restrict__ C2, const T* __restrict__ gCbar, double* __restrict__ partials,
    int32_t* __restrict__ err, const LinGroups grp) {
  using C = LCfg<K, D>;
  static_assert(C::LP == 64, "the pair mapping needs one sample per wave");
  // upper nodes' stiffnesses per sample, [pos - UP0]; then each lane's
  // level-1 cotangent, [lane]
  __shared__ T nodeU[2][21][64];
  __shared__ T leafC[2][2][21];
  __shared__ double accU[2][4][C::NUP];
  __shared__ double acc[C::NLAM][4][64];
  const int t = threadIdx.x;
  for (int u = t; u < C::NUP; u += 64)
    for (int s = 0; s < 2; ++s)
      for (int c = 0; c < 4; ++c) accU[s][c][u] = 0.0;
#pragma unroll
  for (int h = 0; h < C::NLAM; ++h)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[h][c][t] = 0.0;
  int fail = 0;
  const int g = lin_group(grp);
  const T* tab = (const T*)((const char*)tab0 + g * grp.tab_stride);
  const int32_t* flag = (const int32_t*)((const char*)flag0 + g * grp.tab_stride);
  const long long s0 = grp.off[g], Bg = grp.off[g + 1] - s0;
  const int gb = (int)blockIdx.x - grp.block0[g];
  const int gblocks = grp.block0[g + 1] - grp.block0[g];
  const Rows<T, C::L, false> rows{tab, nullptr};
  const LinOri<T> none{};
  __syncthreads();
  for (long long sg = gb; sg * 2 < Bg; sg += gblocks) {
    const long long first = sg * 2;
    const bool liveB = first + 1 < Bg;  // a missing B shadows A and adds nothing
    if (t < 2) {
      const long long b = s0 + first + (t == 1 && liveB ? 1 : 0);
      load_sym(C1 + (size_t)b * 36, leafC[t][0]);
      load_sym(C2 + (size_t)b * 36, leafC[t][1]);
    }
    __syncthreads();
    // lane-subtree roots of both samples, then the upper levels forward for both
    {
      T rootA[21], rootB[21];
      {
        T dummy[C::NLAM][21];
        lin_up<T, K, D, 1, false>(rows, t, leafC[1][0], leafC[1][1], rootB, fail, dummy);
        lin_up<T, K, D, 1, false>(rows, t, leafC[0][0], leafC[0][1], rootA, fail, dummy);
      }
      T cur[21];
#pragma unroll 1
      for (int m = 1; m <= C::UPLEV; ++m) {
        const int o = 1 << (m - 1);
        const int r = t & (2 * o - 1);
        const bool actA = r == 0, actB = r == 2 * o - 1;
        T rC[21];
        if (m == 1) {
          // even lanes combine A_t, A_t+1; odd lanes B_t-1, B_t
#pragma unroll
          for (int k = 0; k < 21; ++k) rC[k] = __shfl((t & 1) ? rootA[k] : rootB[k], t ^ 1, 64);
#pragma unroll
          for (int k = 0; k < 21; ++k) {
            cur[k] = (t & 1) ? rC[k] : rootA[k];
            rC[k] = (t & 1) ? rootB[k] : rC[k];
          }
        } else {
          const int src = actA ? t + o : (actB ? t - o : t);
#pragma unroll
          for (int k = 0; k < 21; ++k) rC[k] = __shfl(cur[k], src, 64);
          if (actB) {
#pragma unroll
            for (int k = 0; k < 21; ++k) {
              const T x = cur[k];
              cur[k] = rC[k];
              rC[k] = x;
            }
          }
        }
        if (actA || actB) {
          const int pos = upos<K, D>(m, t);
          const LRow<T> row = rows(pos);
          // in place: laminate_linear reads each packed entry before writing it
          fail |= laminate_linear(cur, rC, row.nv, row.c1, row.c2, cur) ? 0 : 1;
#pragma unroll
          for (int k = 0; k < 21; ++k) nodeU[actA ? 0 : 1][k][pos - C::UP0] = cur[k];
        }
      }
    }
    __syncthreads();
    // upper levels backward, both samples; root cotangents: A on lane 0, B on 63
    T Gm[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) Gm[k] = T(0);
    if (t == 0 || t == 63)
      load_sym(gCbar + (size_t)(s0 + first + (t == 63 && liveB ? 1 : 0)) * 36, Gm);
#pragma unroll 1
    for (int m = C::UPLEV; m >= 2; --m) {
      const int o = 1 << (m - 1);
      const int r = t & (2 * o - 1);
      const bool actA = r == 0, actB = r == 2 * o - 1;
      T send[21];
#pragma unroll
      for (int k = 0; k < 21; ++k) send[k] = T(0);
      if (actA || actB) {
        const int s = actA ? 0 : 1;
        const int pos = upos<K, D>(m, t);
        const LRow<T> row = rows(pos);
        const int base = t - r;
        const int pL = upos<K, D>(m - 1, base) - C::UP0, pR = upos<K, D>(m - 1, base + o) - C::UP0;
        T CL[21], CR[21], GL[21], GR[21], gc1, gn[3];
#pragma unroll
        for (int k = 0; k < 21; ++k) {
          CL[k] = nodeU[s][k][pL];
          CR[k] = nodeU[s][k][pR];
        }
        laminate_linear_vjp(CL, CR, row.nv, row.c1, row.c2, Gm, GL, GR, gc1, gn);
        if (actA || liveB) {
          const int u = pos - C::UP0;
          accU[s][0][u] += (double)gc1;
          accU[s][1][u] += (double)gn[0];
          accU[s][2][u] += (double)gn[1];
          accU[s][3][u] += (double)gn[2];
        }
#pragma unroll
        for (int k = 0; k < 21; ++k) {
          Gm[k] = actA ? GL[k] : GR[k];
          send[k] = actA ? GR[k] : GL[k];
        }
      }
      const bool rcvA = r == o, rcvB = r == o - 1;
      const int src = rcvA ? t - o : (rcvB ? t + o : t);
      T rcv[21];
#pragma unroll
      for (int k = 0; k < 21; ++k) rcv[k] = __shfl(send[k], src, 64);
      if (rcvA || rcvB) {
#pragma unroll
        for (int k = 0; k < 21; ++k) Gm[k] = rcv[k];
      }
    }
    // each lane's cotangent of its level-1 laminate (A's on even lanes, B's on
    // odd ones) waits in LDS while the lane subtrees are recomputed
    __syncthreads();  // the upper nodes are read no more
#pragma unroll
    for (int k = 0; k < 21; ++k) nodeU[0][k][t] = Gm[k];
    T g1[1], g2[1];
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const bool live = s == 0 || liveB;
      T nodes[C::NLAM][21];
      T cC[21], Gr[21];
      lin_up<T, K, D, 1, true>(rows, t, leafC[s][0], leafC[s][1], cC, fail, nodes);
      // level 1 of sample s: on the even lane of each pair for A, the odd one
      // for B; the lane holding the laminate keeps the cotangent of its own
      // lane root and sends the other to its neighbour
      {
        const bool act = (t & 1) == s;
        T other[21], G1[21], GL[21], GR[21];
#pragma unroll
        for (int k = 0; k < 21; ++k) {
          other[k] = __shfl(cC[k], t ^ 1, 64);
          G1[k] = nodeU[0][k][t];
          GL[k] = GR[k] = T(0);
        }
        if (act) {
          const int pos = upos<K, D>(1, t);
          const LRow<T> row = rows(pos);
          T CL[21], CR[21], gc1, gn[3];
#pragma unroll
          for (int k = 0; k < 21; ++k) {
            CL[k] = s ? other[k] : cC[k];
            CR[k] = s ? cC[k] : other[k];
          }
          laminate_linear_vjp(CL, CR, row.nv, row.c1, row.c2, G1, GL, GR, gc1, gn);
          if (live) {
            const int u = pos - C::UP0;
            accU[s][0][u] += (double)gc1;
            accU[s][1][u] += (double)gn[0];
            accU[s][2][u] += (double)gn[1];
            accU[s][3][u] += (double)gn[2];
          }
        }
#pragma unroll
        for (int k = 0; k < 21; ++k) {
          const T rcv = __shfl(s ? GL[k] : GR[k], t ^ 1, 64);
          Gr[k] = act ? (s ? GR[k] : GL[k]) : rcv;
        }
      }
      lin_back<T, K, D, 1, false, false>(rows, none, 0, 0, t, live, leafC[s][0], leafC[s][1],
                                         nodes, Gr, acc, g1, g2);
    }
    __syncthreads();  // leafC and nodeU are rewritten by the next pair
  }
  // partial sums of this wave (one slot per wave), [pos * 4 + c][slot] in the
  // group's region
  const size_t pslot = (size_t)gb;
  const size_t nslots = (size_t)gblocks;
  double* gpart = partials + (size_t)grp.block0[g] * (4 * C::L);
#pragma unroll
  for (int h = 1; h <= C::NLAM; ++h) {
    const int m = ilog2l(h);
    const int k = K - D + 1 + m;
    const int pos = (1 << K) - (1 << k) + t * (1 << m) + (h - (1 << m));
#pragma unroll
    for (int c = 0; c < 4; ++c) gpart[((size_t)pos * 4 + c) * nslots + pslot] = acc[h - 1][c][t];
  }
  for (int u = t; u < C::NUP; u += 64)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      gpart[((size_t)(C::UP0 + u) * 4 + c) * nslots + pslot] = accU[0][c][u] + accU[1][c][u];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) fail |= __shfl_xor(fail, o, 64);
  if (t == 0 && (fail || *flag)) atomicOr(err, (*flag ? 1 : 0) | (fail ? 2 : 0));
}

// Sum the partials over wave slots in a fixed order, gsum[g][pos * 4 + c].  A
// group with at most kSeqSlots slots has one thread per row summing them in
// slot order (reduce_partials_seq_kernel); a larger one has one workgroup per
// row, each thread summing a strided subset, then a fixed-shape tree in LDS
// (reduce_partials_kernel).  The choice depends on the group's slot count
// only, so a group's sums are the same in a grouped and in a plain call.
constexpr long long kSeqSlots = 64;

__global__ __launch_bounds__(256) void reduce_partials_seq_kernel(
    const double* __restrict__ partials, int ppw, int L4, int rows, double* __restrict__ gsum,
    const LinGroups grp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= rows) return;
  const int g = i / L4;
  const int r = i % L4;
  const long long nslots = (long long)(grp.block0[g + 1] - grp.block0[g]) * ppw;
  if (nslots > kSeqSlots) return;  // a row of reduce_partials_kernel
  const double* row =
      partials + (size_t)grp.block0[g] * ppw * L4 + (size_t)r * nslots;
  // loads issued eight at a time, added in slot order
  double s = 0.0;
  long long q = 0;
  for (; q + 8 <= nslots; q += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = row[q + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; q < nslots; ++q) s += row[q];
  gsum[(size_t)g * L4 + r] = s;
}

__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ partials,
                                                              int ppw, int L4,
                                                              double* __restrict__ gsum,
                                                              const LinGroups grp) {
  __shared__ double part[256];
  const int g = blockIdx.x / L4;
  const int r = blockIdx.x % L4;
  const long long nslots = (long long)(grp.block0[g + 1] - grp.block0[g]) * ppw;
  if (nslots <= kSeqSlots) return;  // a row of reduce_partials_seq_kernel (whole workgroup)
  const double* row =
      partials + (size_t)grp.block0[g] * ppw * L4 + (size_t)r * nslots;
  double s = 0.0;
  for (long long q = threadIdx.x; q < nslots; q += blockDim.x) s += row[q];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) gsum[(size_t)g * L4 + r] = part[0];
}

// Leaf-weight and normal gradients from the per-laminate sums: a leaf
// collects dc1/dW_L (left subtree) or dc1/dW_R (right subtree) times the
// laminate's c1-cotangent over its root path.  Group g = blockIdx.y: sums
// gsum + g 4L, table tab_stride bytes apart, outputs gw + g 2^K, gn + g 3L.
template <typename T>
__global__ __launch_bounds__(256) void finish_grads_kernel(const double* __restrict__ gsum0,
                                                           const T* __restrict__ tab0,
                                                           long long tab_stride, int K,
                                                           T* __restrict__ gw0,
                                                           T* __restrict__ gn0, int write_gn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nleaf = 1 << K;
  const int L = nleaf - 1;
  const long long g = blockIdx.y;
  const double* gsum = gsum0 + g * 4 * L;
  const T* tab = (const T*)((const char*)tab0 + g * tab_stride);
  T* gw = gw0 + g * nleaf;
  T* gn = gn0 + g * 3 * L;
  if (i < nleaf) {
    double s = 0.0;
    for (int k = K; k >= 1; --k) {
      const int i0 = i >> (K - k + 1);
      const int pos = (1 << K) - (1 << k) + i0;
      const bool right = (i >> (K - k)) & 1;
      const double d = (double)tab[(size_t)pos * kTabStride + (right ? 7 : 6)];
      s += gsum[(size_t)pos * 4] * d;
    }
    gw[i] = (T)s;
  }
  if (write_gn && i < L) {
#pragma unroll
    for (int c = 0; c < 3; ++c) gn[(size_t)i * 3 + c] = (T)gsum[(size_t)i * 4 + 1 + c];
  }
}

// Cotangents of the angle coefficients: for laminate pos (one workgroup),
// dJ/dp_j = sum_b dJ/dalpha[b] s_j(l_b), dJ/dq_j likewise, summed over the
// samples in a fixed order (strided per thread, then a fixed tree).  Output
// gpq [L][2][m] (p first, then q).
template <typename T>
__global__ __launch_bounds__(256) void reduce_orientation_kernel(const T* __restrict__ gang,
                                                                 const T* __restrict__ lam,
                                                                 long long B, int m,
                                                                 T* __restrict__ gpq) {
  __shared__ double part[256];
  const int pos = blockIdx.x;
  double acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = 0.0;
  for (long long b = threadIdx.x; b < B; b += blockDim.x) {
    T s[6];
    orientation_shape<T>(lam[(size_t)b * 2], lam[(size_t)b * 2 + 1], m, s);
    const double ga = (double)gang[((size_t)pos * 2) * B + b];
    const double gb = (double)gang[((size_t)pos * 2 + 1) * B + b];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (j < m) {
        acc[j] += ga * (double)s[j];
        acc[6 + j] += gb * (double)s[j];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const int j = c % 6;
    if (j >= m) continue;  // uniform over the workgroup
    part[threadIdx.x] = acc[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) gpq[(size_t)pos * 2 * m + (c / 6) * m + j] = (T)part[0];
    __syncthreads();
  }
}

// deepest DMN whose linear map and VJP are compiled with per-sample orientation
constexpr int kMaxOriLinearDepth = 8;

}  // namespace

static int lin_default_D(int depth) {
  int d = depth - 6;
  return d < 1 ? 1 : d;
}

static int lin_ppw(int depth) { return 64 >> (depth - lin_default_D(depth)); }

// One-wave workgroups of the plain backward of depth K in T that one CU
// holds at once (its registers and LDS), from the runtime's occupancy query.
template <typename T, int K>
static int bwd_blocks_per_cu_t() {
  constexpr int D = (K - 6) < 1 ? 1 : (K - 6);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, linear_bwd_kernel<T, K, D, false, false>,
                                                   64, 0) != hipSuccess ||
      n < 1)
    n = 1;
  return n;
}

static int bwd_blocks_per_cu(int depth, bool f32) {
  static int cached[64][2][11] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (depth < 1 || depth > 10) return 1;
  int& c = cached[dev][f32 ? 1 : 0][depth];
  if (c == 0) {
    switch (depth) {
#define DMN_OCC_CASE(KK)                                                               \
  case KK:                                                                             \
    c = f32 ? bwd_blocks_per_cu_t<float, KK>() : bwd_blocks_per_cu_t<double, KK>();    \
    break;
      DMN_OCC_CASE(1)
      DMN_OCC_CASE(2)
      DMN_OCC_CASE(3)
      DMN_OCC_CASE(4)
      DMN_OCC_CASE(5)
      DMN_OCC_CASE(6)
      DMN_OCC_CASE(7)
      DMN_OCC_CASE(8)
      DMN_OCC_CASE(9)
      DMN_OCC_CASE(10)
#undef DMN_OCC_CASE
    }
  }
  return c;
}

// persistent waves of the backward for a group of B samples: at most as many
// as the device holds at once (more would only add waves that stage the
// table again and partial-sum slots that the reduction reads), and at least
// one, so that an empty group still writes zero gradients
static long long bwd_waves(int depth, long long B, bool f32) {
  const int ppw = lin_ppw(depth);
  long long waves = (B + ppw - 1) / ppw;
  const long long cap = (long long)bwd_blocks_per_cu(depth, f32) * device_cu_count();
  if (waves > cap) waves = cap;
  if (waves < 1) waves = 1;
  return waves;
}

long long linear_backward_partials(int depth, long long B, bool f32) {
  return bwd_waves(depth, B, f32) * lin_ppw(depth);
}

long long linear_backward_group_slots(int depth, int G, const int64_t* off, bool f32) {
  long long slots = 0;
  for (int g = 0; g < G; ++g)
    slots += bwd_waves(depth, off[g + 1] - off[g], f32) * lin_ppw(depth);
  return slots;
}

// Group table of the chunk of groups g0 .. g0+ng-1; blocks(B) gives the
// workgroups of a group of B samples.  Returns the workgroups of the launch,
// or -1 when they exceed the grid.
template <class F>
static long long chunk_groups(LinGroups& gr, const int64_t* off, int g0, int ng,
                              long long tab_stride, F blocks) {
  gr = LinGroups{};
  gr.ng = ng;
  gr.tab_stride = tab_stride;
  long long total = 0;
  for (int q = 0; q < ng; ++q) {
    gr.off[q] = off[g0 + q];
    gr.block0[q] = (int)total;
    total += blocks(off[g0 + q + 1] - off[g0 + q]);
    if (total > 0x7fffffffLL) return -1;
  }
  gr.off[ng] = off[g0 + ng];
  gr.block0[ng] = (int)total;
  return total;
}

template <typename T, int K>
static int fwd_k(const void* tab, const int32_t* flag, long long tab_stride, int G,
                 const int64_t* off, const void* C1, const void* C2, void* Cbar, int32_t* err,
                 const LinOriArgs& o, hipStream_t s) {
  constexpr int D = (K - 6) < 1 ? 1 : (K - 6);
  using C = LCfg<K, D>;
  const LinOri<T> ori{(const T*)o.p, (const T*)o.q, (const T*)o.lam, (T*)o.gang, o.m};
  // per-sample orientation: plain (one-group) calls only
  if (o.m > 0 && G != 1) return (int)hipErrorInvalidValue;
  // fixed normals with one sample per wave at depths 7 and 8: two samples
  // share a wave's upper levels (linear_fwd_pair_kernel; at depth 9 it would
  // spill) when the launch has more than 8 samples per CU, i.e. when one
  // sample per wave would take more than one round of resident waves (two
  // per SIMD); smaller batches are latency bound and keep one per wave
  constexpr bool kPair = C::PPW == 1 && K <= 8;
  const long long pair_min = 8LL * device_cu_count();
  for (int g0 = 0; g0 < G; g0 += kMaxLinGroups) {
    const int ng = G - g0 < kMaxLinGroups ? G - g0 : kMaxLinGroups;
    const bool pair = kPair && o.m == 0 && off[g0 + ng] - off[g0] > pair_min;
    const int per_block = pair ? 2 : C::PPW;
    LinGroups gr;
    const long long nb = chunk_groups(gr, off, g0, ng, tab_stride,
                                      [&](long long B) { return (B + per_block - 1) / per_block; });
    if (nb < 0) return (int)hipErrorInvalidValue;
    if (nb == 0) continue;
    const T* tabc = (const T*)((const char*)tab + g0 * tab_stride);
    const int32_t* flagc = (const int32_t*)((const char*)flag + g0 * tab_stride);
    if constexpr (kPair) {
      if (pair) {
        hipLaunchKernelGGL((linear_fwd_pair_kernel<T, K, D>), dim3((unsigned)nb), dim3(64), 0, s,
                           tabc, flagc, (const T*)C1, (const T*)C2, (T*)Cbar, err, gr);
        continue;
      }
    }
    if (o.m > 0) {
      // per-sample orientation is compiled up to the depth of the VJP kernels
      if constexpr (K <= kMaxOriLinearDepth)
        hipLaunchKernelGGL((linear_fwd_kernel<T, K, D, true>), dim3((unsigned)nb), dim3(64), 0,
                           s, tabc, flagc, (const T*)C1, (const T*)C2, (T*)Cbar, err, ori, gr);
      else
        return (int)hipErrorInvalidValue;
    } else
      hipLaunchKernelGGL((linear_fwd_kernel<T, K, D, false>), dim3((unsigned)nb), dim3(64), 0, s,
                         tabc, flagc, (const T*)C1, (const T*)C2, (T*)Cbar, err, ori, gr);
  }
  return (int)hipGetLastError();
}

template <typename T>
static int fwd_t(int depth, const void* tab, const int32_t* flag, long long tab_stride, int G,
                 const int64_t* off, const void* C1, const void* C2, void* Cbar, int32_t* err,
                 const LinOriArgs& o, hipStream_t s) {
  switch (depth) {
#define DMN_FWD_CASE(KK) \
  case KK:               \
    return fwd_k<T, KK>(tab, flag, tab_stride, G, off, C1, C2, Cbar, err, o, s);
    DMN_FWD_CASE(1)
    DMN_FWD_CASE(2)
    DMN_FWD_CASE(3)
    DMN_FWD_CASE(4)
    DMN_FWD_CASE(5)
    DMN_FWD_CASE(6)
    DMN_FWD_CASE(7)
    DMN_FWD_CASE(8)
    DMN_FWD_CASE(9)
    DMN_FWD_CASE(10)
#undef DMN_FWD_CASE
    default:
      return (int)hipErrorInvalidValue;
  }
}

int launch_linear_forward(int depth, int prec, const void* tab, const int32_t* flag, long long B,
                          const void* C1, const void* C2, void* Cbar, int32_t* err,
                          const LinOriArgs& ori, hipStream_t stream) {
  const int64_t off[2] = {0, B};
  if (prec == DMN_F32)
    return fwd_t<float>(depth, tab, flag, 0, 1, off, C1, C2, Cbar, err, ori, stream);
  return fwd_t<double>(depth, tab, flag, 0, 1, off, C1, C2, Cbar, err, ori, stream);
}

int launch_linear_forward_groups(int depth, int prec, const void* tab, const int32_t* flag,
                                 long long tab_stride, int G, const int64_t* off,
                                 const void* C1, const void* C2, void* Cbar, int32_t* err,
                                 hipStream_t stream) {
  const LinOriArgs none;
  if (prec == DMN_F32)
    return fwd_t<float>(depth, tab, flag, tab_stride, G, off, C1, C2, Cbar, err, none, stream);
  return fwd_t<double>(depth, tab, flag, tab_stride, G, off, C1, C2, Cbar, err, none, stream);
}

template <typename T, int K, bool IG, bool ORI>
static void bwd_launch(long long waves, const void* tab, const int32_t* flag, long long B,
                       const void* C1, const void* C2, const void* gCbar, void* gC1, void* gC2,
                       double* partials, int32_t* err, const LinOri<T>& ori, const LinGroups& gr,
                       hipStream_t s) {
  constexpr int D = (K - 6) < 1 ? 1 : (K - 6);
  if constexpr (ORI && K > kMaxOriLinearDepth) {
    return;  // not compiled; rejected by the caller
  } else {
    hipLaunchKernelGGL((linear_bwd_kernel<T, K, D, IG, ORI>), dim3((unsigned)waves), dim3(64), 0,
                       s, (const T*)tab, flag, B, (const T*)C1, (const T*)C2, (const T*)gCbar,
                       (T*)gC1, (T*)gC2, partials, err, ori, gr);
  }
}

template <typename T, int K>
static int bwd_k(const void* tab, const int32_t* flag, long long tab_stride, int G,
                 const int64_t* off, const void* C1, const void* C2, const void* gCbar,
                 void* gw, void* gn, void* gC1, void* gC2, double* partials, double* gsum,
                 int32_t* err, const LinOriArgs& o, hipStream_t s) {
  constexpr int D = (K - 6) < 1 ? 1 : (K - 6);
  using C = LCfg<K, D>;
  const LinOri<T> ori{(const T*)o.p, (const T*)o.q, (const T*)o.lam, (T*)o.gang, o.m};
  const bool oriented = o.m > 0;
  if (oriented && (G != 1 || K > kMaxOriLinearDepth)) return (int)hipErrorInvalidValue;
  const bool ig = gC1 != nullptr;
  const int L4 = C::L * 4;
  const int nleaf = 1 << K;
  double* part = partials;
  for (int g0 = 0; g0 < G; g0 += kMaxLinGroups) {
    const int ng = G - g0 < kMaxLinGroups ? G - g0 : kMaxLinGroups;
    LinGroups gr;
    const long long waves =
        chunk_groups(gr, off, g0, ng, tab_stride,
                     [](long long B) { return bwd_waves(K, B, sizeof(T) == 4); });
    if (waves < 0 || (long long)ng * L4 > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    const void* tabc = (const char*)tab + g0 * tab_stride;
    const int32_t* flagc = (const int32_t*)((const char*)flag + g0 * tab_stride);
    // fixed normals without phase-stiffness cotangents, one sample per wave:
    // two samples per wave (linear_bwd_pair_kernel, same waves and partial
    // slots) at depths 7 and 8 and, as for the forward, only above 8 samples
    // per CU: smaller batches are latency bound and pairs would idle half the
    // waves (the FP64 depth-8 instance spills a few hundred bytes per lane and
    // still issues less per sample).  Only launches of one group: a group
    // below the wave cap gets one wave per sample, so in a launch of many
    // small groups (training over orientations) pairs would leave half the
    // waves without work
    constexpr bool kPair = C::PPW == 1 && (K == 7 || K == 8);
    bool paired = false;
    if constexpr (kPair) {
      if (!ig && !oriented && ng == 1 && off[g0 + 1] - off[g0] > 8LL * device_cu_count()) {
        hipLaunchKernelGGL((linear_bwd_pair_kernel<T, K, D>), dim3((unsigned)waves), dim3(64), 0,
                           s, (const T*)tabc, flagc, (const T*)C1, (const T*)C2,
                           (const T*)gCbar, part, err, gr);
        paired = true;
      }
    }
    if (paired) {
    } else if (ig && oriented)
      bwd_launch<T, K, true, true>(waves, tabc, flagc, off[G], C1, C2, gCbar, gC1, gC2, part, err,
                                   ori, gr, s);
    else if (ig)
      bwd_launch<T, K, true, false>(waves, tabc, flagc, off[G], C1, C2, gCbar, gC1, gC2, part,
                                    err, ori, gr, s);
    else if (oriented)
      bwd_launch<T, K, false, true>(waves, tabc, flagc, off[G], C1, C2, gCbar, gC1, gC2, part,
                                    err, ori, gr, s);
    else
      bwd_launch<T, K, false, false>(waves, tabc, flagc, off[G], C1, C2, gCbar, gC1, gC2, part,
                                     err, ori, gr, s);
    double* gs = gsum + (size_t)g0 * L4;
    bool any_seq = false, any_tree = false;
    for (int q = 0; q < ng; ++q) {
      const long long nslots = (long long)(gr.block0[q + 1] - gr.block0[q]) * C::PPW;
      (nslots <= kSeqSlots ? any_seq : any_tree) = true;
    }
    if (any_seq)
      hipLaunchKernelGGL(reduce_partials_seq_kernel, dim3((unsigned)((ng * L4 + 255) / 256)),
                         dim3(256), 0, s, (const double*)part, C::PPW, L4, ng * L4, gs, gr);
    if (any_tree)
      hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)(ng * L4)), dim3(256), 0, s,
                         (const double*)part, C::PPW, L4, gs, gr);
    hipLaunchKernelGGL((finish_grads_kernel<T>), dim3((nleaf + 255) / 256, (unsigned)ng), dim3(256),
                       0, s, (const double*)gs, (const T*)tabc, tab_stride, K,
                       (T*)gw + (size_t)g0 * nleaf, (T*)gn + (size_t)g0 * 3 * C::L,
                       oriented ? 0 : 1);
    // per-sample orientation: gn is the angle-coefficient cotangent [L][2][m]
    if (oriented)
      hipLaunchKernelGGL((reduce_orientation_kernel<T>), dim3(C::L), dim3(256), 0, s,
                         (const T*)o.gang, (const T*)o.lam, off[G], o.m, (T*)gn);
    part += (size_t)waves * C::PPW * L4;
  }
  return (int)hipGetLastError();
}

template <typename T>
static int bwd_t(int depth, const void* tab, const int32_t* flag, long long tab_stride, int G,
                 const int64_t* off, const void* C1, const void* C2, const void* gCbar,
                 void* gw, void* gn, void* gC1, void* gC2, double* partials, double* gsum,
                 int32_t* err, const LinOriArgs& o, hipStream_t s) {
  switch (depth) {
#define DMN_BWD_CASE(KK)                                                                       \
  case KK:                                                                                     \
    return bwd_k<T, KK>(tab, flag, tab_stride, G, off, C1, C2, gCbar, gw, gn, gC1, gC2, partials, \
                        gsum, err, o, s);
    DMN_BWD_CASE(1)
    DMN_BWD_CASE(2)
    DMN_BWD_CASE(3)
    DMN_BWD_CASE(4)
    DMN_BWD_CASE(5)
    DMN_BWD_CASE(6)
    DMN_BWD_CASE(7)
    DMN_BWD_CASE(8)
    DMN_BWD_CASE(9)
    DMN_BWD_CASE(10)
#undef DMN_BWD_CASE
    default:
      return (int)hipErrorInvalidValue;
  }
}

int launch_linear_backward(int depth, int prec, const void* tab, const int32_t* flag,
                           long long B, const void* C1, const void* C2, const void* gCbar,
                           void* gw, void* gn, void* gC1, void* gC2, double* partials,
                           double* gsum, int32_t* err, const LinOriArgs& ori,
                           hipStream_t stream) {
  const int64_t off[2] = {0, B};
  if (prec == DMN_F32)
    return bwd_t<float>(depth, tab, flag, 0, 1, off, C1, C2, gCbar, gw, gn, gC1, gC2, partials,
                        gsum, err, ori, stream);
  return bwd_t<double>(depth, tab, flag, 0, 1, off, C1, C2, gCbar, gw, gn, gC1, gC2, partials,
                       gsum, err, ori, stream);
}

int launch_linear_backward_groups(int depth, int prec, const void* tab, const int32_t* flag,
                                  long long tab_stride, int G, const int64_t* off,
                                  const void* C1, const void* C2, const void* gCbar, void* gw,
                                  void* gn, double* partials, double* gsum, int32_t* err,
                                  hipStream_t stream) {
  const LinOriArgs none;
  if (prec == DMN_F32)
    return bwd_t<float>(depth, tab, flag, tab_stride, G, off, C1, C2, gCbar, gw, gn, nullptr,
                        nullptr, partials, gsum, err, none, stream);
  return bwd_t<double>(depth, tab, flag, tab_stride, G, off, C1, C2, gCbar, gw, gn, nullptr,
                       nullptr, partials, gsum, err, none, stream);
}

}  // namespace dmn
