// Adjoint of one Newton-converged load step of the DMN Gauss-point update:
// gradients of a functional of the effective stresses with respect to the
// DMN parameters (leaf weights, lamination normals) and to the internal
// variables carried into the step, by the implicit-function theorem applied to
// the Euler-Lagrange equation R(a) = A^T W sigma(E + A a, z^n) = 0 (FE-DMN
// paper, Sec. 3.2).
//
// For a step with converged jumps a, cotangent gbar of the effective stress
// and zeta of the new internal variables, with e_j = w~_j D_j gbar +
// (dZ_j/deps)^T zeta_j:
//   H lam = A^T e            (tree solve with leaf "prestress" e_j / w~_j; the
//                              Newton top-down gives -lam and A lam = -deps)
//   psi_j = w~_j (gbar - (A lam)_j)
//   mu_j  = psi_j-VJP of the leaf law w.r.t. eps (= e_j - w~_j D_j (A lam)_j)
//   zeta^n_j = (dS_j/dz)^T psi_j + (dZ_j/dz)^T zeta_j
//   dJ/dtheta = sum_j [ (dw~_j/dtheta) sigma_j.(gbar - (A lam)_j)
//                       + mu_j.((dA/dtheta) a)_j - w~_j sigma_j.((dA/dtheta) lam)_j ]
// The dA/dtheta terms are local to each laminate: with subtree sums of mu and
// w~ sigma over its two children, the normal gradient is
//   N(a)^T (-c2 Smu_L + c1 Smu_R) - N(lam)^T (-c2 Sws_L + c1 Sws_R)
// and the c1 gradient (N a).(Smu_L + Smu_R) - (N lam).(Sws_L + Sws_R), chained to
// the leaf weights through c1 = W_L / (W_L + W_R).
//
// Mapping as in the Gauss-point kernel (tree across lanes).  Each wave walks
// a fixed, strided set of points and accumulates the parameter cotangents per
// lane; the partial sums are reduced over waves in a fixed order.
#include "dmn_tree.hpp"

namespace dmn {
namespace {

using namespace tree;

struct AdjArgs {
  const double* E;
  const double* z_in;
  const double* a_conv;
  const double* g_sigma;   // may be null
  const double* g_z_next;  // may be null
  double* g_z_prev;
  const double* tab;
  const int32_t* flag;
  double* partials;        // [rows][nslots], rows = 4 L + 2^K
  int32_t* err;
  long long P;
  IsoElastic fib;
  J2Law mat;
};

// Leaf law of the adjoint solve: stress and tangent as in Newton, tau = e_j / w~_j.
template <int NLEAF>
struct AdjointLeaf {
  const double* gbar;      // [6]
  const double* zeta;      // this point's zeta^{n+1} or null
  const double* leafw;     // normalised leaf weights of the DMN
  template <int K, int D, int Q>
  __device__ __forceinline__ void operator()(const Ctx<K, D>& cx, std::integral_constant<int, Q>,
                                             const double (&e)[6], double (&Cn)[21],
                                             double (&tn)[6], double (&sn)[6], int& lfail) const {
    using C = Cfg<K, D>;
    if constexpr (Q % 2 == 0) {  // fibre: tau = C_f gbar
      iso_stress(cx.fib, e, sn);
      iso_packed(cx.fib, Cn);
      double gb[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) gb[k] = gbar[k];
      iso_stress(cx.fib, gb, tn);
    } else {
      const int mloc = cx.t * (C::NLEAF / 2) + Q / 2;
      const double* z = (const double*)cx.zin + (size_t)mloc * 7;
      double epn[6], ep[6], p;
#pragma unroll
      for (int k = 0; k < 6; ++k) epn[k] = z[k];
      const bool ok = j2_return(cx.mat, e, epn, z[6], sn, Cn, ep, p);
      lfail |= ok ? 0 : 1;
      const double wj = leafw[cx.t * C::NLEAF + Q];
      double ze[6], zp = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) ze[k] = 0.0;
      if (zeta != nullptr && wj > 0.0) {
        const double iw = 1.0 / wj;
#pragma unroll
        for (int k = 0; k < 6; ++k) ze[k] = zeta[(size_t)mloc * 7 + k] * iw;
        zp = zeta[(size_t)mloc * 7 + 6] * iw;
      }
      double gb[6], gz[7];
#pragma unroll
      for (int k = 0; k < 6; ++k) gb[k] = gbar[k];
      double sv[6];
      j2_vjp(cx.mat, e, epn, z[6], gb, ze, zp, tn, gz, sv);  // tn = e_j / w~_j
    }
  }
};

// Subtree sums of mu and w~ sigma, with the laminate parameter cotangents.
template <int K, int D, int H>
__device__ __forceinline__ void sum_node(const Ctx<K, D>& cx, const LaneState<K, D>& st,
                                         const double (&mu)[Cfg<K, D>::NLEAF][6],
                                         const double (&ws)[Cfg<K, D>::NLEAF][6], bool live,
                                         double (&acc)[Cfg<K, D>::NLAM][4], double (&Sm)[6],
                                         double (&Ss)[6]) {
  using C = Cfg<K, D>;
  if constexpr (H >= C::NLEAF) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      Sm[k] = mu[H - C::NLEAF][k];
      Ss[k] = ws[H - C::NLEAF][k];
    }
  } else {
    double SmR[6], SsR[6];
    sum_node<K, D, 2 * H>(cx, st, mu, ws, live, acc, Sm, Ss);
    sum_node<K, D, 2 * H + 1>(cx, st, mu, ws, live, acc, SmR, SsR);
    const LamRow row = load_row(cx, lane_pos<D, H>(cx.g, cx.t));
    double a[3], lam[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a[k] = st.a[H - 1][k];
      lam[k] = -st.da[H - 1][k];
    }
    double g4[4];
    laminate_param_grad(row.nv, row.c1, row.c2, a, lam, Sm, Ss, SmR, SsR, g4);
    if (live) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[H - 1][c] += g4[c];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      Sm[k] += SmR[k];
      Ss[k] += SsR[k];
    }
  }
}

template <int K, int D>
__global__ __launch_bounds__(64) void adjoint_kernel(const AdjArgs args) {
  using C = Cfg<K, D>;
  __shared__ UpperLds<K, D> up;
  __shared__ double accU[4][C::SLOTS];
  __shared__ TableLds<K> tlds;
  const int lane = threadIdx.x;
  Ctx<K, D> cx;
  cx.slot = lane / C::LP;
  cx.t = lane % C::LP;
  cx.base = cx.slot * C::LP;
  cx.tab = stage_table<K>(tlds, args.tab + table_soa_offset(K), threadIdx.x, 64);
  cx.nrm = cx.tab + 2 * C::L;
  cx.fib = args.fib;
  cx.mat = args.mat;
  const double* leafw = args.tab + (size_t)C::L * kTabStride;
  const double invW = leafw[1 << K];
  for (int u = lane; u < C::SLOTS; u += 64)
#pragma unroll
    for (int c = 0; c < 4; ++c) accU[c][u] = 0.0;
  double acc[C::NLAM][4];
  double accleaf[C::NLEAF];
#pragma unroll
  for (int h = 0; h < C::NLAM; ++h)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[h][c] = 0.0;
#pragma unroll
  for (int q = 0; q < C::NLEAF; ++q) accleaf[q] = 0.0;
  const bool invalid = *args.flag != 0;
  int lfail_any = 0, spd_any = 0;
  __syncthreads();

#pragma unroll 1
  for (long long pg = blockIdx.x; pg * C::PPW < args.P && !invalid; pg += gridDim.x) {
    const long long praw = pg * C::PPW + cx.slot;
    const bool live = praw < args.P;
    const long long pt = live ? praw : args.P - 1;
    cx.zin = args.z_in + (size_t)pt * C::M * 7;
    const double* ain = args.a_conv + (size_t)pt * C::L * 3;
    const double* zeta = args.g_z_next ? args.g_z_next + (size_t)pt * C::M * 7 : nullptr;
    double E[6], gbar[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      E[k] = args.E[(size_t)pt * 6 + k];
      gbar[k] = args.g_sigma ? args.g_sigma[(size_t)pt * 6 + k] : 0.0;
    }
    LaneState<K, D> st;
#pragma unroll
    for (int h = 1; h <= C::NLAM; ++h) {
      const int m = ilog2(h);
      const int k = K - D + 1 + m;
      const int pos = (1 << K) - (1 << k) + cx.t * (1 << m) + (h - (1 << m));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        st.a[h - 1][c] = ain[(size_t)pos * 3 + c];
        st.da[h - 1][c] = 0.0;
      }
    }
#pragma unroll 1
    for (int m = 1; m <= C::UPLEV; ++m) {
      if (upper_active(cx.t, m)) {
        const int pos = upper_pos<D>(cx.g, m, cx.t);
        const int u = cx.slot * C::NUPS + (pos - C::UP0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          up.a[c][u] = ain[(size_t)pos * 3 + c];
          up.da[c][u] = 0.0;
        }
      }
    }
    // leaf strains at the converged jumps; tree solve with the adjoint prestress
    double eps[C::NLEAF][6], de[C::NLEAF][6];
    localize(cx, st, up, E, 0.0, eps);
    AdjointLeaf<C::NLEAF> leaf{gbar, zeta, leafw};
    EvalOut ev;
    evaluate_full(cx, st, up, eps, ev, leaf);
    lfail_any |= ev.lfail;
    spd_any |= ev.spdfail;
    direction(cx, st, up, true, de);  // da = -lam, de = -(A lam)
    // leaf adjoints; the strains are localised again and the stresses
    // recomputed rather than held through the tree solve (registers)
    localize(cx, st, up, E, 0.0, eps);
    double mu[C::NLEAF][6], ws[C::NLEAF][6], rho[C::NLEAF];
    double srho = 0.0;
#pragma unroll
    for (int q = 0; q < C::NLEAF; ++q) {
      const double wj = leafw[cx.t * C::NLEAF + q];
      double gmd[6], psi[6], sig[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        gmd[k] = gbar[k] + de[q][k];
        psi[k] = wj * gmd[k];
      }
      if (q % 2 == 0) {
        iso_stress(cx.fib, eps[q], sig);
        iso_stress(cx.fib, psi, mu[q]);
      } else {
        const int mloc = cx.t * (C::NLEAF / 2) + q / 2;
        const double* z = (const double*)cx.zin + (size_t)mloc * 7;
        double epn[6], ze[6], zp = 0.0, gz[7];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          epn[k] = z[k];
          ze[k] = zeta ? zeta[(size_t)mloc * 7 + k] : 0.0;
        }
        if (zeta) zp = zeta[(size_t)mloc * 7 + 6];
        j2_vjp(cx.mat, eps[q], epn, z[6], psi, ze, zp, mu[q], gz, sig);
        if (live) {
          double* out = args.g_z_prev + (size_t)pt * C::M * 7 + (size_t)mloc * 7;
#pragma unroll
          for (int k = 0; k < 7; ++k) out[k] = gz[k];
        }
      }
      rho[q] = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        rho[q] += sig[k] * gmd[k];
        ws[q][k] = wj * sig[k];
      }
      srho += wj * rho[q];
    }
    // subtree sums and laminate parameter cotangents
    double Sm[6], Ss[6];
    sum_node<K, D, 1>(cx, st, mu, ws, live, acc, Sm, Ss);
#pragma unroll 1
    for (int m = 1; m <= C::UPLEV; ++m) {
      const int o = 1 << (m - 1);
      double SmR[6], SsR[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        SmR[k] = __shfl_down(Sm[k], (unsigned)o, C::LP);
        SsR[k] = __shfl_down(Ss[k], (unsigned)o, C::LP);
      }
      if (upper_active(cx.t, m)) {
        const int pos = upper_pos<D>(cx.g, m, cx.t);
        const int u = cx.slot * C::NUPS + (pos - C::UP0);
        const LamRow row = load_row(cx, pos);
        double a[3], lam[3], g4[4];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          a[k] = up.a[k][u];
          lam[k] = -up.da[k][u];
        }
        laminate_param_grad(row.nv, row.c1, row.c2, a, lam, Sm, Ss, SmR, SsR, g4);
        if (live) {
#pragma unroll
          for (int c = 0; c < 4; ++c) accU[c][u] += g4[c];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          Sm[k] += SmR[k];
          Ss[k] += SsR[k];
        }
      }
    }
    // direct dependence of the averages on the weights: (rho_k - sum w~ rho) / sum(w)
#pragma unroll
    for (int o = 1; o < C::LP; o <<= 1) srho += __shfl_xor(srho, o, C::LP);
    if (live) {
#pragma unroll
      for (int q = 0; q < C::NLEAF; ++q) accleaf[q] += (rho[q] - srho) * invW;
    }
  }

  // partial sums of this wave slot: rows [pos * 4 + c] then [4 L + leaf]
  const size_t pslot = (size_t)blockIdx.x * C::PPW + cx.slot;
  const size_t nslots = (size_t)gridDim.x * C::PPW;
  double* P = args.partials;
#pragma unroll
  for (int h = 1; h <= C::NLAM; ++h) {
    const int m = ilog2(h);
    const int k = K - D + 1 + m;
    const int pos = (1 << K) - (1 << k) + cx.t * (1 << m) + (h - (1 << m));
#pragma unroll
    for (int c = 0; c < 4; ++c) P[((size_t)pos * 4 + c) * nslots + pslot] = acc[h - 1][c];
  }
#pragma unroll 1
  for (int m = 1; m <= C::UPLEV; ++m) {
    if (upper_active(cx.t, m)) {
      const int pos = upper_pos<D>(cx.g, m, cx.t);
      const int u = cx.slot * C::NUPS + (pos - C::UP0);
#pragma unroll
      for (int c = 0; c < 4; ++c) P[((size_t)pos * 4 + c) * nslots + pslot] = accU[c][u];
    }
  }
#pragma unroll
  for (int q = 0; q < C::NLEAF; ++q)
    P[((size_t)4 * C::L + cx.t * C::NLEAF + q) * nslots + pslot] = accleaf[q];
  if (lane == 0 && (invalid || lfail_any || spd_any))
    atomicOr(args.err, (invalid ? 1 : 0) | (spd_any ? 2 : 0) | (lfail_any ? 4 : 0));
}

__global__ __launch_bounds__(256) void adjoint_reduce_kernel(const double* __restrict__ partials,
                                                             long long nslots, int rows,
                                                             double* __restrict__ gsum) {
  __shared__ double part[256];
  const int i = blockIdx.x;
  const double* row = partials + (size_t)i * nslots;
  double s = 0.0;
  for (long long q = threadIdx.x; q < nslots; q += blockDim.x) s += row[q];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && i < rows) gsum[i] = part[0];
}

// gw[k] += direct term + c1 cotangents along the root path; gn += normal cotangents.
__global__ __launch_bounds__(256) void adjoint_finish_kernel(const double* __restrict__ gsum,
                                                             const double* __restrict__ tab,
                                                             int K, double* __restrict__ gw,
                                                             double* __restrict__ gn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nleaf = 1 << K;
  const int L = nleaf - 1;
  if (i < nleaf) {
    double s = gsum[(size_t)4 * L + i];
    for (int k = K; k >= 1; --k) {
      const int pos = (1 << K) - (1 << k) + (i >> (K - k + 1));
      const bool right = (i >> (K - k)) & 1;
      s += gsum[(size_t)pos * 4] * tab[(size_t)pos * kTabStride + (right ? 7 : 6)];
    }
    gw[i] += s;
  }
  if (i < L) {
#pragma unroll
    for (int c = 0; c < 3; ++c) gn[(size_t)i * 3 + c] += gsum[(size_t)i * 4 + 1 + c];
  }
}

// lanes per point of the adjoint kernels: one wave holds a point's tree
// (lane subtrees of depth max(1, K - 6))
int adjoint_lanes_per_point(int depth) {
  int d = depth - 6;
  if (d < 1) d = 1;
  return 1 << (depth - d);
}

// One-wave workgroups of adjoint_kernel<K, D> that one CU holds at once (its
// registers and LDS), from the runtime's occupancy query.
template <int K, int D>
int adj_blocks_per_cu_t() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adjoint_kernel<K, D>, 64, 0) !=
          hipSuccess ||
      n < 1)
    n = 1;
  return n;
}

int adj_blocks_per_cu(int depth) {
  static int cached[64][11] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (depth < 1 || depth > 10) return 1;
  int& c = cached[dev][depth];
  if (c == 0) {
    switch (depth) {
      case 1: c = adj_blocks_per_cu_t<1, 1>(); break;
      case 2: c = adj_blocks_per_cu_t<2, 1>(); break;
      case 3: c = adj_blocks_per_cu_t<3, 1>(); break;
      case 4: c = adj_blocks_per_cu_t<4, 1>(); break;
      case 5: c = adj_blocks_per_cu_t<5, 1>(); break;
      case 6: c = adj_blocks_per_cu_t<6, 1>(); break;
      case 7: c = adj_blocks_per_cu_t<7, 1>(); break;
      case 8: c = adj_blocks_per_cu_t<8, 2>(); break;
      case 9: c = adj_blocks_per_cu_t<9, 3>(); break;
      default: c = adj_blocks_per_cu_t<10, 4>(); break;
    }
  }
  return c;
}

template <int K, int D>
int launch_adj(const AdjArgs& a, long long waves, hipStream_t s) {
  hipLaunchKernelGGL((adjoint_kernel<K, D>), dim3((unsigned)waves), dim3(64), 0, s, a);
  return (int)hipGetLastError();
}

}  // namespace

long long adjoint_partial_slots(int depth, long long P) {
  const int lp = adjoint_lanes_per_point(depth);
  const int ppw = 64 / lp;
  long long waves = (P + ppw - 1) / ppw;
  // persistent waves: at most as many as the device holds at once (more would
  // only add partial-sum slots for the reduction to read)
  const long long cap = (long long)adj_blocks_per_cu(depth) * device_cu_count();
  if (waves > cap) waves = cap;
  if (waves < 1) waves = 1;
  return waves * ppw;
}

int launch_adjoint(int depth, const AdjointLaunch& L, hipStream_t stream) {
  AdjArgs a;
  a.E = L.E;
  a.z_in = L.z_in;
  a.a_conv = L.a_conv;
  a.g_sigma = L.g_sigma;
  a.g_z_next = L.g_z_next;
  a.g_z_prev = L.g_z_prev;
  a.tab = L.tab;
  a.flag = L.flag;
  a.partials = L.partials;
  a.err = L.err;
  a.P = L.P;
  a.fib = L.fib;
  a.mat = L.mat;
  const int lp = adjoint_lanes_per_point(depth);
  const long long slots = adjoint_partial_slots(depth, L.P);
  const long long waves = slots / (64 / lp);
  const int D = depth - tree::ilog2(lp);
  int rc;
  switch (depth * 16 + D) {
#define DMN_ADJ_CASE(KK, DD) \
  case KK * 16 + DD:         \
    rc = launch_adj<KK, DD>(a, waves, stream); \
    break;
    DMN_ADJ_CASE(1, 1)
    DMN_ADJ_CASE(2, 1)
    DMN_ADJ_CASE(3, 1)
    DMN_ADJ_CASE(4, 1)
    DMN_ADJ_CASE(5, 1)
    DMN_ADJ_CASE(6, 1)
    DMN_ADJ_CASE(7, 1)
    DMN_ADJ_CASE(8, 2)
    DMN_ADJ_CASE(9, 3)
    DMN_ADJ_CASE(10, 4)
#undef DMN_ADJ_CASE
    default:
      return (int)hipErrorInvalidValue;
  }
  if (rc) return rc;
  const int Lm = (1 << depth) - 1;
  const int rows = 4 * Lm + (1 << depth);
  hipLaunchKernelGGL(adjoint_reduce_kernel, dim3(rows), dim3(256), 0, stream,
                     (const double*)L.partials, slots, rows, L.gsum);
  const int nleaf = 1 << depth;
  hipLaunchKernelGGL(adjoint_finish_kernel, dim3((nleaf + 255) / 256), dim3(256), 0, stream,
                     (const double*)L.gsum, L.tab, depth, L.gw, L.gn);
  return (int)hipGetLastError();
}

}  // namespace dmn
