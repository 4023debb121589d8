// Offline training of a DMN: the objective's data term and its cotangent
// (Sec. 3.1), the parameter update (Macaulay weights, normal angles, mixing
// penalty of Sec. 3.1; AMSGrad with the modulated learning rate of Sec. 4.5),
// the per-group normals and cotangent chain for training over a discrete set
// of fibre orientations (Sec. 2.3), and the stiffness sampler of Sec. 4.4.
//
// All of it is bandwidth- or latency-bound work next to the linear map and its
// VJP: per-sample kernels read and write whole 36-entry stiffness records,
// the batch reductions and the parameter update run in one workgroup with a
// fixed summation order, so results are bit-reproducible run to run.
#include "dmn_internal.hpp"

namespace dmn {
namespace {

constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kPi = 3.14159265358979323846;
constexpr int kReduceThreads = 1024;
constexpr int kUpdateThreads = 512;

// Voigt component of a Mandel stiffness entry (I, J): C_IJ / (s_I s_J) with
// s = (1, 1, 1, sqrt 2, sqrt 2, sqrt 2).
__device__ __forceinline__ double voigt_factor(int k) {
  const int shear = (k / 6 >= 3) + (k % 6 >= 3);
  return shear == 0 ? 1.0 : (shear == 1 ? kInvSqrt2 : 0.5);
}

__device__ __forceinline__ double pow_p(double x, double p, bool p1) { return p1 ? x : pow(x, p); }

// The per-sample kernels give each of the 36 entries of a stiffness record its
// own thread: a workgroup of 252 threads covers 7 consecutive samples, so a
// wave reads consecutive doubles of the [B][36] arrays.
constexpr int kEntryThreads = 252;
constexpr int kSamplesPerGroup = kEntryThreads / 36;

// Per sample: nd = ||V(target - Cbar)||_p, nt = ||V target||_p, e = nd / nt
// (the 36 terms summed in entry order by the sample's first thread).
template <typename T>
__global__ __launch_bounds__(kEntryThreads) void loss_norms_kernel(
    long long B, double p, const T* __restrict__ Cbar, const T* __restrict__ target,
    double* __restrict__ nd, double* __restrict__ nt, double* __restrict__ e, T* e_out) {
  __shared__ double td[kEntryThreads], tt[kEntryThreads];
  const int j = threadIdx.x;
  const int ls = j / 36, k = j - 36 * ls;
  const long long s = (long long)blockIdx.x * kSamplesPerGroup + ls;
  const bool p1 = p == 1.0;
  double a = 0.0, b = 0.0;
  if (s < B) {
    const double f = voigt_factor(k);
    const double tv = (double)target[(size_t)s * 36 + k];
    a = pow_p(fabs((tv - (double)Cbar[(size_t)s * 36 + k]) * f), p, p1);
    b = pow_p(fabs(tv * f), p, p1);
  }
  td[j] = a;
  tt[j] = b;
  __syncthreads();
  if (k == 0 && s < B) {
    double sd = 0.0, st = 0.0;
    for (int i = 0; i < 36; ++i) {
      sd += td[j + i];
      st += tt[j + i];
    }
    const double x = p1 ? sd : pow(sd, 1.0 / p);
    const double y = p1 ? st : pow(st, 1.0 / p);
    nd[s] = x;
    nt[s] = y;
    e[s] = x / y;
    if (e_out) e_out[s] = (T)(x / y);
  }
}

// NaN-propagating maximum
__device__ __forceinline__ double nan_max(double a, double b) {
  return (a != a || b != b) ? __builtin_nan("") : fmax(a, b);
}

// One workgroup, two passes over e: M = max e (NaN propagates), then
// S = sum (e / M)^q; each pass folds a strided slice per thread, combines a
// wave with a fixed butterfly and the waves in order, so the sums do not
// depend on scheduling.  stats[0..2] = M S^(1/q) / B, M, S (0 for an empty or
// error-free batch).
__global__ __launch_bounds__(kReduceThreads) void loss_reduce_kernel(long long B, double q,
                                                                     const double* __restrict__ e,
                                                                     double* __restrict__ stats) {
  constexpr int kWaves = kReduceThreads / 64;
  __shared__ double wmax[kWaves], wsum[kWaves];
  const int tid = threadIdx.x;
  double m = 0.0;
  for (long long s = tid; s < B; s += kReduceThreads) m = nan_max(m, e[s]);
  for (int o = 32; o > 0; o >>= 1) m = nan_max(m, __shfl_xor(m, o, 64));
  if ((tid & 63) == 0) wmax[tid >> 6] = m;
  __syncthreads();
  double M = wmax[0];
  for (int w = 1; w < kWaves; ++w) M = nan_max(M, wmax[w]);
  const bool any = M > 0.0 || M != M;
  double acc = 0.0;
  if (any)
    for (long long s = tid; s < B; s += kReduceThreads) acc += pow(e[s] / M, q);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((tid & 63) == 0) wsum[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double S = 0.0;
    for (int w = 0; w < kWaves; ++w) S += wsum[w];
    stats[0] = any ? M * pow(S, 1.0 / q) / (double)B : 0.0;
    stats[1] = M;
    stats[2] = S;
  }
}

// gCbar_s = d(data term)/d Cbar_s
//         = (1/B) S^(1/q - 1) (e_s / M)^(q - 1) * (-1 / nt_s) d||D||_p/dD * f
// with D = V(target - Cbar); zero where the batch or the sample has no error.
template <typename T>
__global__ __launch_bounds__(kEntryThreads) void loss_cotangent_kernel(
    long long B, double p, double q, const T* __restrict__ Cbar, const T* __restrict__ target,
    const double* __restrict__ nd, const double* __restrict__ nt, const double* __restrict__ e,
    const double* __restrict__ stats, T* __restrict__ gC) {
  const int j = threadIdx.x;
  const int ls = j / 36, k = j - 36 * ls;
  const long long s = (long long)blockIdx.x * kSamplesPerGroup + ls;
  if (s >= B) return;
  const double M = stats[1], S = stats[2];
  const double ds = nd[s];
  double coef = 0.0;
  if (M > 0.0 && ds > 0.0)
    coef = pow(S, 1.0 / q - 1.0) * pow(e[s] / M, q - 1.0) / ((double)B * nt[s]);
  else if (M != M || ds != ds)
    coef = M + ds;  // NaN in, NaN out
  const size_t idx = (size_t)s * 36 + k;
  const double f = voigt_factor(k);
  const double d = ((double)target[idx] - (double)Cbar[idx]) * f;
  const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
  const double dn = p == 1.0 ? sg : (ds > 0.0 ? pow(fabs(d) / ds, p - 1.0) * sg : 0.0);
  gC[idx] = (T)(-coef * dn * f);
}

struct AmsArgs {
  double lr_min, lr_max, lr_decay, beta1, beta2, eps, penalty;
  int half_period, steps_per_epoch;
};

// Learning rate of epoch m: decay^m (lr_min + (lr_max - lr_min)(1 + cos(pi m / M)) / 2).
__device__ __forceinline__ double modulated_rate(const AmsArgs& o, long long m) {
  return pow(o.lr_decay, (double)m) *
         (o.lr_min + 0.5 * (o.lr_max - o.lr_min) * (1.0 + cos(kPi * (double)m / o.half_period)));
}

// One workgroup.  Sums <v>_+ (fixed butterfly per wave, then the waves in
// order), then each thread owns one weight or both angles of one laminate
// (each angle's gradient needs the other's old value): with take_step it
// applies the chain
//   dJ/dv_i     = (gw_i + 2 lambda (sum <v>_+ - 1)) [v_i > 0]
//   dJ/dalpha_l = gn_l . dn/dalpha,   dJ/dbeta_l = gn_l . dn/dbeta
// and one AMSGrad step, and in any case writes w = <v>_+ and n(alpha, beta)
// of its (new) parameters for the next forward.
template <typename T>
__global__ __launch_bounds__(kUpdateThreads) void train_update_kernel(
    int K, T* __restrict__ v, T* __restrict__ alpha, T* __restrict__ beta, T* __restrict__ w,
    T* __restrict__ n, T* __restrict__ state, long long* __restrict__ step,
    const T* __restrict__ gw, const T* __restrict__ gn, AmsArgs o, double* __restrict__ stats,
    int take_step) {
  __shared__ double wsum[kUpdateThreads / 64];
  const int tid = threadIdx.x;
  const int NL = 1 << K, L = NL - 1, NP = NL + 2 * L;
  const long long t0 = take_step ? *step : 0;  // every read precedes the barrier below
  double acc = 0.0;
  for (int i = tid; i < NL; i += kUpdateThreads) acc += fmax((double)v[i], 0.0);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((tid & 63) == 0) wsum[tid >> 6] = acc;
  __syncthreads();
  double sw = 0.0;
  for (int q = 0; q < kUpdateThreads / 64; ++q) sw += wsum[q];
  const double pen_g = 2.0 * o.penalty * (sw - 1.0);
  const double lr = take_step ? modulated_rate(o, t0 / o.steps_per_epoch) : 0.0;
  const double tn = (double)(t0 + 1);
  const double step_size = take_step ? lr / (1.0 - pow(o.beta1, tn)) : 0.0;
  const double bc2 = take_step ? 1.0 - pow(o.beta2, tn) : 1.0;
  T* m1 = state;
  T* m2 = state + NP;
  T* mx = state + 2 * NP;
  // one AMSGrad update of parameter slot i with gradient g
  auto amsgrad = [&](int i, double th, double g) {
    const double a1 = o.beta1 * (double)m1[i] + (1.0 - o.beta1) * g;
    const double a2 = o.beta2 * (double)m2[i] + (1.0 - o.beta2) * g * g;
    const double ax = fmax((double)mx[i], a2);
    m1[i] = (T)a1;
    m2[i] = (T)a2;
    mx[i] = (T)ax;
    return th - step_size * a1 / (sqrt(ax / bc2) + o.eps);
  };
  for (int i = tid; i < NL + L; i += kUpdateThreads) {
    if (i < NL) {
      double th = (double)v[i];
      if (take_step) {
        th = (double)(T)amsgrad(i, th, th > 0.0 ? (double)gw[i] + pen_g : 0.0);
        v[i] = (T)th;
      }
      w[i] = (T)fmax(th, 0.0);
    } else {
      const int l = i - NL;
      double a = (double)alpha[l], b = (double)beta[l];
      double sa, ca, sb, cb;
      sincos(a, &sa, &ca);
      sincos(b, &sb, &cb);
      if (take_step) {
        const double g0 = (double)gn[3 * l], g1 = (double)gn[3 * l + 1];
        const double g2 = (double)gn[3 * l + 2];
        a = (double)(T)amsgrad(NL + l, a, g0 * ca * cb + g1 * ca * sb - g2 * sa);
        b = (double)(T)amsgrad(NL + L + l, b, -g0 * sa * sb + g1 * sa * cb);
        alpha[l] = (T)a;
        beta[l] = (T)b;
        sincos(a, &sa, &ca);
        sincos(b, &sb, &cb);
      }
      n[3 * l] = (T)(sa * cb);
      n[3 * l + 1] = (T)(sa * sb);
      n[3 * l + 2] = (T)ca;
    }
  }
  if (take_step && tid == 0) {
    const double pen = o.penalty * (sw - 1.0) * (sw - 1.0);
    stats[3] = stats[0] + pen;
    stats[4] = pen;
    stats[5] = lr;
    stats[6] = sw;
    *step = t0 + 1;
  }
}

// ---------------------------------------------------------------------------
// Training over a discrete set of fibre orientations (Sec. 2.3, Sec. 4.5):
// the samples of orientation k all see the normals n_k, so a step runs the
// fixed-normal linear map and its VJP once per orientation group; these
// kernels give the groups their normals and chain their cotangents back to
// the angle coefficients p, q [L][m].

// n[k][l] = n(p_l . s(lam_k), q_l . s(lam_k)), one thread per (k, l).
template <typename T>
__global__ __launch_bounds__(256) void group_normals_kernel(int G, int L, int m,
                                                            const T* __restrict__ p,
                                                            const T* __restrict__ q,
                                                            const T* __restrict__ lam,
                                                            T* __restrict__ n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)G * L) return;
  const int k = (int)(idx / L), l = (int)(idx - (long long)k * L);
  double sh[6];
  orientation_shape<double>((double)lam[2 * k], (double)lam[2 * k + 1], m, sh);
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j)
    if (j < m) {
      a += (double)p[(size_t)l * m + j] * sh[j];
      b += (double)q[(size_t)l * m + j] * sh[j];
    }
  double sa, ca, sb, cb;
  sincos(a, &sa, &ca);
  sincos(b, &sb, &cb);
  T* o = n + (size_t)idx * 3;
  o[0] = (T)(sa * cb);
  o[1] = (T)(sa * sb);
  o[2] = (T)ca;
}

// gw = sum_k gw_g[k] (workgroups 0 .. gw_blocks-1, one thread per leaf, k in
// order) and, per laminate l (one 64-lane workgroup each),
//   gpq[l][0][j] = sum_k (gn_g[k][l] . dn/dalpha) s_j(lam_k),
//   gpq[l][1][j] = sum_k (gn_g[k][l] . dn/dbeta)  s_j(lam_k):
// lane t takes the orientations k = t, t + 64, ... in order, then a fixed
// butterfly sums the lanes (the same order every run).
template <typename T>
__global__ __launch_bounds__(64) void group_chain_kernel(
    int G, int NL, int L, int m, int gw_blocks, const T* __restrict__ p,
    const T* __restrict__ q, const T* __restrict__ lam, const T* __restrict__ gw_g,
    const T* __restrict__ gn_g, T* __restrict__ gw, T* __restrict__ gpq) {
  const int lane = threadIdx.x;
  if ((int)blockIdx.x < gw_blocks) {
    const int i = blockIdx.x * 64 + lane;
    if (i < NL) {
      double acc = 0.0;
      for (int k = 0; k < G; ++k) acc += (double)gw_g[(size_t)k * NL + i];
      gw[i] = (T)acc;
    }
    return;
  }
  const int l = (int)blockIdx.x - gw_blocks;  // < L: the grid has gw_blocks + L workgroups
  double gp[6] = {0, 0, 0, 0, 0, 0}, gq[6] = {0, 0, 0, 0, 0, 0};
  for (int k = lane; k < G; k += 64) {
    double sh[6];
    orientation_shape<double>((double)lam[2 * k], (double)lam[2 * k + 1], m, sh);
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j < m) {
        a += (double)p[(size_t)l * m + j] * sh[j];
        b += (double)q[(size_t)l * m + j] * sh[j];
      }
    double sa, ca, sb, cb;
    sincos(a, &sa, &ca);
    sincos(b, &sb, &cb);
    const T* g = gn_g + ((size_t)k * L + l) * 3;
    const double g0 = (double)g[0], g1 = (double)g[1], g2 = (double)g[2];
    const double ga = g0 * ca * cb + g1 * ca * sb - g2 * sa;
    const double gb = -g0 * sa * sb + g1 * sa * cb;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      gp[j] += ga * sh[j];
      gq[j] += gb * sh[j];
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      gp[j] += __shfl_xor(gp[j], o, 64);
      gq[j] += __shfl_xor(gq[j], o, 64);
    }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j < m) {
        gpq[((size_t)l * 2) * m + j] = (T)gp[j];
        gpq[((size_t)l * 2 + 1) * m + j] = (T)gq[j];
      }
  }
}

// One workgroup: AMSGrad on the slots v [NL], p [L m], q [L m] with
//   dJ/dv_i = (gw_i + 2 lambda (sum <v>_+ - 1)) [v_i > 0],
//   dJ/dp, dJ/dq from gpq [L][2][m];
// then (or, without take_step, only) w = <v>_+.
template <typename T>
__global__ __launch_bounds__(kUpdateThreads) void train_update_coeff_kernel(
    int K, int m, T* __restrict__ v, T* __restrict__ p, T* __restrict__ q, T* __restrict__ w,
    T* __restrict__ state, long long* __restrict__ step, const T* __restrict__ gw,
    const T* __restrict__ gpq, AmsArgs o, double* __restrict__ stats, int take_step) {
  __shared__ double wsum[kUpdateThreads / 64];
  const int tid = threadIdx.x;
  const int NL = 1 << K, L = NL - 1, LM = L * m, NP = NL + 2 * LM;
  const long long t0 = take_step ? *step : 0;  // every read precedes the barrier below
  double acc = 0.0;
  for (int i = tid; i < NL; i += kUpdateThreads) acc += fmax((double)v[i], 0.0);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((tid & 63) == 0) wsum[tid >> 6] = acc;
  __syncthreads();
  double sw = 0.0;
  for (int r = 0; r < kUpdateThreads / 64; ++r) sw += wsum[r];
  if (!take_step) {
    for (int i = tid; i < NL; i += kUpdateThreads) w[i] = (T)fmax((double)v[i], 0.0);
    return;
  }
  const double pen_g = 2.0 * o.penalty * (sw - 1.0);
  const double lr = modulated_rate(o, t0 / o.steps_per_epoch);
  const double tn = (double)(t0 + 1);
  const double step_size = lr / (1.0 - pow(o.beta1, tn));
  const double bc2 = 1.0 - pow(o.beta2, tn);
  T* m1 = state;
  T* m2 = state + NP;
  T* mx = state + 2 * NP;
  for (int i = tid; i < NP; i += kUpdateThreads) {
    double th, g;
    if (i < NL) {
      th = (double)v[i];
      g = th > 0.0 ? (double)gw[i] + pen_g : 0.0;
    } else {
      const int r = i < NL + LM ? i - NL : i - NL - LM;  // l m + j
      const int l = r / m, j = r - l * m;
      const bool isq = i >= NL + LM;
      th = isq ? (double)q[r] : (double)p[r];
      g = (double)gpq[((size_t)l * 2 + (isq ? 1 : 0)) * m + j];
    }
    const double a1 = o.beta1 * (double)m1[i] + (1.0 - o.beta1) * g;
    const double a2 = o.beta2 * (double)m2[i] + (1.0 - o.beta2) * g * g;
    const double ax = fmax((double)mx[i], a2);
    m1[i] = (T)a1;
    m2[i] = (T)a2;
    mx[i] = (T)ax;
    const T nt = (T)(th - step_size * a1 / (sqrt(ax / bc2) + o.eps));
    if (i < NL) {
      v[i] = nt;
      w[i] = (T)fmax((double)nt, 0.0);
    } else if (i < NL + LM) {
      p[i - NL] = nt;
    } else {
      q[i - NL - LM] = nt;
    }
  }
  if (tid == 0) {
    const double pen = o.penalty * (sw - 1.0) * (sw - 1.0);
    stats[3] = stats[0] + pen;
    stats[4] = pen;
    stats[5] = lr;
    stats[6] = sw;
    *step = t0 + 1;
  }
}

// theta in [0, pi] with theta - sin(theta) = pi u: Newton from the small-angle
// estimate (6 pi u)^(1/3), which lies left of the root; the function is
// convex and increasing, so after the first step the iterates decrease
// monotonically onto the root.
__device__ double theta_from_unit(double u) {
  const double rhs = kPi * u;
  if (!(rhs > 0.0)) return 0.0;
  double th = fmin(cbrt(6.0 * rhs), kPi);
  for (int it = 0; it < 8; ++it) {
    const double d = 1.0 - cos(th);
    if (!(d > 0.0)) break;
    th = fmin(fmax(th - (th - sin(th) - rhs) / d, 0.0), kPi);
  }
  return th;
}

// Phase stiffnesses of Sec. 4.4 from a unit-cube point u[8]:
//   C1 = 3 K1 P1 + 2 G1 P2, C2 = 3 K2 P1 + 2 G2 (P2 - a N' (x) N'),
// K1 = 1, G1 = 10^e1, K2 = 10^e2, G2 = 10^e3, N' = Q diag(d) Q^T with the
// trace-free unit diagonal d(beta) = (c, s, -(c + s)) / sqrt(2 + 2 c s)
// (c = cos beta, s = sin beta) and Q the rotation by theta about
// (sin psi cos phi, sin psi sin phi, cos psi).
template <typename T>
__global__ __launch_bounds__(256) void sample_stiffness_kernel(long long B,
                                                               const double* __restrict__ u,
                                                               T* __restrict__ C1,
                                                               T* __restrict__ C2) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const double* x = u + (size_t)s * 8;
  const double a = x[0];
  const double G1 = exp10(-3.0 + 6.0 * x[1]);
  const double K2 = exp10(-3.0 + 6.0 * x[2]);
  const double G2 = exp10(-3.0 + 6.0 * x[3]);
  const double bt = 2.0 * kPi * x[4];
  const double th = theta_from_unit(x[5]);
  const double psi = kPi * x[6], phi = 2.0 * kPi * x[7];
  double cb, sb, ct, st, cp, sp, cf, sf;
  sincos(bt, &sb, &cb);
  sincos(th, &st, &ct);
  sincos(psi, &sp, &cp);
  sincos(phi, &sf, &cf);
  const double inv = 1.0 / sqrt(2.0 + 2.0 * cb * sb);
  const double d[3] = {cb * inv, sb * inv, -(cb + sb) * inv};
  const double ax[3] = {sp * cf, sp * sf, cp};
  // Rodrigues: R = cos(th) I + sin(th) [ax]_x + (1 - cos th) ax ax^T
  double R[3][3];
  const double oc = 1.0 - ct;
  R[0][0] = ct + oc * ax[0] * ax[0];
  R[1][1] = ct + oc * ax[1] * ax[1];
  R[2][2] = ct + oc * ax[2] * ax[2];
  R[0][1] = oc * ax[0] * ax[1] - st * ax[2];
  R[1][0] = oc * ax[0] * ax[1] + st * ax[2];
  R[0][2] = oc * ax[0] * ax[2] + st * ax[1];
  R[2][0] = oc * ax[0] * ax[2] - st * ax[1];
  R[1][2] = oc * ax[1] * ax[2] - st * ax[0];
  R[2][1] = oc * ax[1] * ax[2] + st * ax[0];
  auto Nr = [&](int i, int j) {
    return R[i][0] * d[0] * R[j][0] + R[i][1] * d[1] * R[j][1] + R[i][2] * d[2] * R[j][2];
  };
  const double nv[6] = {Nr(0, 0), Nr(1, 1), Nr(2, 2), kSqrt2 * Nr(1, 2), kSqrt2 * Nr(0, 2),
                        kSqrt2 * Nr(0, 1)};
  T* c1 = C1 + (size_t)s * 36;
  T* c2 = C2 + (size_t)s * 36;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const double p1 = (i < 3 && j < 3) ? 1.0 / 3.0 : 0.0;
      const double p2 = (i == j ? 1.0 : 0.0) - p1;
      c1[i * 6 + j] = (T)(3.0 * p1 + 2.0 * G1 * p2);
      c2[i * 6 + j] = (T)(3.0 * K2 * p1 + 2.0 * G2 * (p2 - a * nv[i] * nv[j]));
    }
}

inline unsigned blocks_for(long long B, int threads) {
  return (unsigned)((B + threads - 1) / threads);
}

template <typename T>
int loss_t(long long B, double p, double q, const void* Cbar, const void* target, void* e_out,
           void* gCbar, double* stats, double* scratch, hipStream_t s) {
  double* nd = scratch;
  double* nt = scratch + B;
  double* e = scratch + 2 * B;
  if (B > 0)
    hipLaunchKernelGGL((loss_norms_kernel<T>), dim3(blocks_for(B, kSamplesPerGroup)),
                       dim3(kEntryThreads), 0, s, B, p, (const T*)Cbar, (const T*)target, nd, nt,
                       e, (T*)e_out);
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, s, B, q,
                     (const double*)e, stats);
  if (B > 0)
    hipLaunchKernelGGL((loss_cotangent_kernel<T>), dim3(blocks_for(B, kSamplesPerGroup)),
                       dim3(kEntryThreads), 0, s, B, p, q, (const T*)Cbar, (const T*)target,
                       (const double*)nd, (const double*)nt, (const double*)e,
                       (const double*)stats, (T*)gCbar);
  return (int)hipGetLastError();
}

}  // namespace

int launch_training_loss(int prec, long long B, double p, double q, const void* Cbar,
                         const void* target, void* e_out, void* gCbar, double* stats,
                         double* scratch, hipStream_t stream) {
  if (prec == DMN_F32)
    return loss_t<float>(B, p, q, Cbar, target, e_out, gCbar, stats, scratch, stream);
  return loss_t<double>(B, p, q, Cbar, target, e_out, gCbar, stats, scratch, stream);
}

int launch_training_update(int prec, int depth, const TrainUpdateArgs& a, hipStream_t stream) {
  const AmsArgs o{a.lr_min, a.lr_max, a.lr_decay, a.beta1, a.beta2, a.eps, a.penalty,
                  a.half_period, a.steps_per_epoch};
  if (prec == DMN_F32)
    hipLaunchKernelGGL((train_update_kernel<float>), dim3(1), dim3(kUpdateThreads), 0, stream,
                       depth, (float*)a.v, (float*)a.alpha, (float*)a.beta, (float*)a.w,
                       (float*)a.n, (float*)a.state, a.step, (const float*)a.gw,
                       (const float*)a.gn, o, a.stats, a.take_step);
  else
    hipLaunchKernelGGL((train_update_kernel<double>), dim3(1), dim3(kUpdateThreads), 0, stream,
                       depth, (double*)a.v, (double*)a.alpha, (double*)a.beta, (double*)a.w,
                       (double*)a.n, (double*)a.state, a.step, (const double*)a.gw,
                       (const double*)a.gn, o, a.stats, a.take_step);
  return (int)hipGetLastError();
}

int launch_group_normals(int prec, int depth, int m, int G, const void* p, const void* q,
                         const void* lam, void* n, hipStream_t stream) {
  const int L = (1 << depth) - 1;
  const long long total = (long long)G * L;
  if (total == 0) return (int)hipSuccess;
  const unsigned nb = blocks_for(total, 256);
  if (prec == DMN_F32)
    hipLaunchKernelGGL((group_normals_kernel<float>), dim3(nb), dim3(256), 0, stream, G, L, m,
                       (const float*)p, (const float*)q, (const float*)lam, (float*)n);
  else
    hipLaunchKernelGGL((group_normals_kernel<double>), dim3(nb), dim3(256), 0, stream, G, L, m,
                       (const double*)p, (const double*)q, (const double*)lam, (double*)n);
  return (int)hipGetLastError();
}

int launch_group_chain(int prec, int depth, int m, int G, const void* p, const void* q,
                       const void* lam, const void* gw_g, const void* gn_g, void* gw, void* gpq,
                       hipStream_t stream) {
  const int NL = 1 << depth, L = NL - 1;
  const int gw_blocks = (int)blocks_for(NL, 64);
  const unsigned nb = (unsigned)(gw_blocks + L);
  if (prec == DMN_F32)
    hipLaunchKernelGGL((group_chain_kernel<float>), dim3(nb), dim3(64), 0, stream, G, NL, L, m,
                       gw_blocks, (const float*)p, (const float*)q, (const float*)lam,
                       (const float*)gw_g, (const float*)gn_g, (float*)gw, (float*)gpq);
  else
    hipLaunchKernelGGL((group_chain_kernel<double>), dim3(nb), dim3(64), 0, stream, G, NL, L, m,
                       gw_blocks, (const double*)p, (const double*)q, (const double*)lam,
                       (const double*)gw_g, (const double*)gn_g, (double*)gw, (double*)gpq);
  return (int)hipGetLastError();
}

int launch_training_update_coeff(int prec, int depth, int m, const TrainUpdateArgs& a,
                                 hipStream_t stream) {
  const AmsArgs o{a.lr_min, a.lr_max, a.lr_decay, a.beta1, a.beta2, a.eps, a.penalty,
                  a.half_period, a.steps_per_epoch};
  // alpha / beta carry the coefficient arrays p / q, gn the coefficient gradients
  if (prec == DMN_F32)
    hipLaunchKernelGGL((train_update_coeff_kernel<float>), dim3(1), dim3(kUpdateThreads), 0,
                       stream, depth, m, (float*)a.v, (float*)a.alpha, (float*)a.beta,
                       (float*)a.w, (float*)a.state, a.step, (const float*)a.gw,
                       (const float*)a.gn, o, a.stats, a.take_step);
  else
    hipLaunchKernelGGL((train_update_coeff_kernel<double>), dim3(1), dim3(kUpdateThreads), 0,
                       stream, depth, m, (double*)a.v, (double*)a.alpha, (double*)a.beta,
                       (double*)a.w, (double*)a.state, a.step, (const double*)a.gw,
                       (const double*)a.gn, o, a.stats, a.take_step);
  return (int)hipGetLastError();
}

int launch_sample_stiffness(int prec, long long B, const double* u, void* C1, void* C2,
                            hipStream_t stream) {
  if (B == 0) return (int)hipSuccess;
  if (prec == DMN_F32)
    hipLaunchKernelGGL((sample_stiffness_kernel<float>), dim3(blocks_for(B, 256)), dim3(256), 0,
                       stream, B, u, (float*)C1, (float*)C2);
  else
    hipLaunchKernelGGL((sample_stiffness_kernel<double>), dim3(blocks_for(B, 256)), dim3(256), 0,
                       stream, B, u, (double*)C1, (double*)C2);
  return (int)hipGetLastError();
}

}  // namespace dmn
