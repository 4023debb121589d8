// Device algebra of the DMN laminate tree on gfx950.
//
// Conventions
//   * Mandel 6-vectors [11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12]; the Mandel
//     dot product is the Frobenius product, so all norms are Frobenius norms.
//   * Symmetric 6x6 matrices are packed as their 21 upper-triangle entries,
//     row by row (index given by sidx).
//   * N(n) is the symmetrisation operator a -> sym(a (x) n) of the laminate
//     normal n (Sec. 3.2), a 6x3 matrix with nine non-zeros; it is never
//     stored, every product with it is written out.
//
// The laminate step below is the block-Cholesky elimination of the Newton
// Hessian A^T W D A (Sec. 3.2, Newton system) restricted to one laminate:
// given the affine responses  sigma_X(e) = tau_X + C_X e  of the two child
// subtrees (X = L, R), the interface condition of the laminate
//   N^T (sigma_R(e + c1 N da) - sigma_L(e - c2 N da)) = 0
// is solved for the jump increment da, giving the laminate's own affine
// response.  With S = c2 C_L + c1 C_R, K = N^T S N, U = (C_R - C_L) N:
//   C   = c1 C_L + c2 C_R - c1 c2 U K^-1 U^T        (condensed tangent)
//   tau = c1 tau_L + c2 tau_R - c1 c2 U K^-1 N^T (tau_R - tau_L)
//   da  = -(g + G e),  g = K^-1 N^T (tau_R - tau_L),  G = K^-1 U^T
// Applied to stiffnesses alone (no tau) this is the linear laminate of
// Sec. 3.1 in Schur-complement form; it equals Milton's projector formula.
#pragma once
#include <hip/hip_runtime.h>

namespace dmn {

constexpr double kRsqrt2 = 0.70710678118654752440;

// packed index of (i, j) in a symmetric 6x6 matrix
__host__ __device__ constexpr int sidx(int i, int j) {
  return i <= j ? i * 6 - (i * (i - 1)) / 2 + (j - i) : j * 6 - (j * (j - 1)) / 2 + (i - j);
}

template <typename T>
struct Normal {
  T n0, n1, n2;
  // N x for x in R^3
  __device__ __forceinline__ void apply(const T x[3], T y[6]) const {
    const T r = T(kRsqrt2);
    y[0] = n0 * x[0];
    y[1] = n1 * x[1];
    y[2] = n2 * x[2];
    y[3] = r * (n2 * x[1] + n1 * x[2]);
    y[4] = r * (n2 * x[0] + n0 * x[2]);
    y[5] = r * (n1 * x[0] + n0 * x[1]);
  }
  // N^T v for v in R^6
  __device__ __forceinline__ void applyT(const T v[6], T y[3]) const {
    const T r = T(kRsqrt2);
    y[0] = n0 * v[0] + r * (n2 * v[4] + n1 * v[5]);
    y[1] = n1 * v[1] + r * (n2 * v[3] + n0 * v[5]);
    y[2] = n2 * v[2] + r * (n1 * v[3] + n0 * v[4]);
  }
};

// Inverse M of a symmetric 3x3 matrix K from its cofactors and one reciprocal
// of the determinant.  Returns false unless K is positive definite by
// Sylvester's criterion (k00, k00 k11 - k01^2 and det K all positive; false
// for non-finite entries); M is then left unspecified.
template <typename T>
__device__ __forceinline__ bool spd3_inverse(T k00, T k01, T k02, T k11, T k12, T k22,
                                             T& m00, T& m01, T& m02, T& m11, T& m12,
                                             T& m22) {
  const T c00 = k11 * k22 - k12 * k12;
  const T c01 = k02 * k12 - k01 * k22;
  const T c02 = k01 * k12 - k02 * k11;
  const T c11 = k00 * k22 - k02 * k02;
  const T c12 = k01 * k02 - k00 * k12;
  const T c22 = k00 * k11 - k01 * k01;
  const T det = k00 * c00 + k01 * c01 + k02 * c02;
  const bool ok = k00 > T(0) && c22 > T(0) && det > T(0);
  const T inv = T(1) / (ok ? det : T(1));
  m00 = c00 * inv;
  m01 = c01 * inv;
  m02 = c02 * inv;
  m11 = c11 * inv;
  m12 = c12 * inv;
  m22 = c22 * inv;
  return ok;
}

// Rows of S N for symmetric packed S: (S N)[r][:] = N^T S[r][:]
template <typename T>
__device__ __forceinline__ void sym_times_N(const T S[21], const Normal<T>& nv, T SN[6][3]) {
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    T row[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) row[c] = S[sidx(r, c)];
    nv.applyT(row, SN[r]);
  }
}

// Linear laminate (Sec. 3.1) in Schur form: C = c1 CL + c2 CR - c1 c2 U K^-1 U^T.
// Optionally returns the intermediates the backward pass needs.
template <typename T>
__device__ __forceinline__ bool laminate_linear(const T CL[21], const T CR[21], const Normal<T>& nv,
                                                T c1, T c2, T C[21]) {
  T S[21], dC[21];
#pragma unroll
  for (int k = 0; k < 21; ++k) {
    S[k] = c2 * CL[k] + c1 * CR[k];
    dC[k] = CR[k] - CL[k];
  }
  T SN[6][3], U[6][3];
  sym_times_N(S, nv, SN);
  sym_times_N(dC, nv, U);
  T col[6], kc[3];
  T Km[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int r = 0; r < 6; ++r) col[r] = SN[r][c];
    nv.applyT(col, kc);
    Km[0][c] = kc[0];
    Km[1][c] = kc[1];
    Km[2][c] = kc[2];
  }
  T m00, m01, m02, m11, m12, m22;
  bool ok = spd3_inverse(Km[0][0], Km[0][1], Km[0][2], Km[1][1], Km[1][2], Km[2][2], m00, m01,
                         m02, m11, m12, m22);
  T V[6][3];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    V[r][0] = U[r][0] * m00 + U[r][1] * m01 + U[r][2] * m02;
    V[r][1] = U[r][0] * m01 + U[r][1] * m11 + U[r][2] * m12;
    V[r][2] = U[r][0] * m02 + U[r][1] * m12 + U[r][2] * m22;
  }
  const T cc = c1 * c2;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) {
      T vu = V[i][0] * U[j][0] + V[i][1] * U[j][1] + V[i][2] * U[j][2];
      C[sidx(i, j)] = c1 * CL[sidx(i, j)] + c2 * CR[sidx(i, j)] - cc * vu;
    }
  return ok;
}

// Vector-Jacobian product of laminate_linear.  Gm is the cotangent of the
// output C as a full symmetric matrix stored packed (so <Gm, dC> sums all 36
// entries).  Returns the cotangents of CL and CR (same convention), of c1
// (with c2 = 1 - c1), and of the normal components.
//   T = U K^-1 U^T,  Gt = -c1 c2 Gm,  V = U K^-1,  P = Gm V
//   G_U = 2 Gt V = -2 c1 c2 P,  G_K = -V^T Gt V = c1 c2 V^T P,
//   G_S = N G_K N^T,  G_dC = sym(G_U N^T)
//   G_CL = c1 Gm + c2 G_S - G_dC,  G_CR = c2 Gm + c1 G_S + G_dC
//   G_c1 = <Gm, CL - CR> - (1 - 2 c1) <Gm, T> + <G_S, CR - CL>,
//          <Gm, T> = sum U o P
//   G_N  = 2 S N G_K + dC G_U,  G_n_d = <G_N, dN/dn_d> (nine entries of G_N)
// Written to keep few values live: S and dC are formed one row at a time,
// G_S and G_dC one entry at a time straight into G_CL and G_CR.
template <typename T>
__device__ __forceinline__ void laminate_linear_vjp(const T CL[21], const T CR[21],
                                                    const Normal<T>& nv, T c1, T c2,
                                                    const T Gm[21], T GL[21], T GR[21], T& gc1,
                                                    T gn[3]) {
  T SN[6][3], U[6][3];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    T srow[6], drow[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int k = sidx(r, c);
      srow[c] = c2 * CL[k] + c1 * CR[k];
      drow[c] = CR[k] - CL[k];
    }
    nv.applyT(srow, SN[r]);
    nv.applyT(drow, U[r]);
  }
  T Km[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T col[6], kc[3];
#pragma unroll
    for (int r = 0; r < 6; ++r) col[r] = SN[r][c];
    nv.applyT(col, kc);
    Km[0][c] = kc[0];
    Km[1][c] = kc[1];
    Km[2][c] = kc[2];
  }
  T m00, m01, m02, m11, m12, m22;
  spd3_inverse(Km[0][0], Km[0][1], Km[0][2], Km[1][1], Km[1][2], Km[2][2], m00, m01, m02, m11,
               m12, m22);
  T V[6][3];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    V[r][0] = U[r][0] * m00 + U[r][1] * m01 + U[r][2] * m02;
    V[r][1] = U[r][0] * m01 + U[r][1] * m11 + U[r][2] * m12;
    V[r][2] = U[r][0] * m02 + U[r][1] * m12 + U[r][2] * m22;
  }
  // P = Gm V and <Gm, T> = sum U o P
  T P[6][3];
  T a2 = T(0);
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 6; ++j) acc += Gm[sidx(i, j)] * V[j][a];
      P[i][a] = acc;
      a2 += U[i][a] * acc;
    }
  const T cc = c1 * c2;
  T GK[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < 6; ++i) acc += V[i][a] * P[i][b];
      GK[a][b] = cc * acc;
      GK[b][a] = cc * acc;
    }
  // G_U, in place of P
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a) P[i][a] *= T(-2) * cc;
  // the nine entries of G_N = 2 SN G_K + dC G_U that dN/dn touches
  auto gN = [&](int i, int a) {
    T acc = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) acc += T(2) * SN[i][b] * GK[b][a];
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += (CR[sidx(i, j)] - CL[sidx(i, j)]) * P[j][a];
    return acc;
  };
  const T r = T(kRsqrt2);
  gn[0] = gN(0, 0) + r * (gN(4, 2) + gN(5, 1));
  gn[1] = gN(1, 1) + r * (gN(3, 2) + gN(5, 0));
  gn[2] = gN(2, 2) + r * (gN(3, 1) + gN(4, 0));
  // N G_K (6x3)
  T NGK[6][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T x[3] = {GK[0][c], GK[1][c], GK[2][c]}, y[6];
    nv.apply(x, y);
#pragma unroll
    for (int q = 0; q < 6; ++q) NGK[q][c] = y[q];
  }
  // entry (i, j), i <= j: G_S = (N NGK_i)_j, G_dC = ((N G_U_i)_j + (N G_U_j)_i) / 2
  T a1 = T(0);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T ys[6], yu[6];
    nv.apply(NGK[i], ys);
    nv.apply(P[i], yu);
#pragma unroll
    for (int j = i; j < 6; ++j) {
      const int k = sidx(i, j);
      T yt[6];
      nv.apply(P[j], yt);
      const T gdc = T(0.5) * (yu[j] + yt[i]);
      const T gs = ys[j];
      GL[k] = c1 * Gm[k] + c2 * gs - gdc;
      GR[k] = c2 * Gm[k] + c1 * gs + gdc;
      a1 += (i == j ? T(1) : T(2)) * (Gm[k] - gs) * (CR[k] - CL[k]);
    }
  }
  gc1 = -a1 - (T(1) - T(2) * c1) * a2;
}

// Newton laminate step, in place: on entry (C, tau, sb) hold the left
// child's condensed tangent, affine offset and plain stress average; on exit
// they hold the laminate's.  Also returns the top-down factors G (3x6,
// row-major) and g (3), accumulates the squared norm of the laminate's
// residual block rfac N^T (sb_R - sb_L) into rr (rfac = W_L W_R / (W sum(w))
// makes it the laminate's block of A^T W sigma), and returns false when the
// 3x3 pivot N^T S N is not positive definite.  Written to keep few values live:
// S and C_R - C_L are formed one row at a time.
template <typename T>
__device__ __forceinline__ bool laminate_newton(T C[21], T tau[6], T sb[6], const T CR[21],
                                                const T tR[6], const T sR[6],
                                                const Normal<T>& nv, T c1, T c2, T rfac,
                                                T G[18], T g[3], T& rr) {
  const T r = T(kRsqrt2);
  const T n0 = nv.n0, n1 = nv.n1, n2 = nv.n2;
  const T n0r = n0 * r, n1r = n1 * r, n2r = n2 * r;
  T k00 = 0, k01 = 0, k02 = 0, k11 = 0, k12 = 0, k22 = 0;
  T U[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T srow[6], drow[6], sn[3];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      srow[j] = c2 * C[sidx(i, j)] + c1 * CR[sidx(i, j)];
      drow[j] = CR[sidx(i, j)] - C[sidx(i, j)];
    }
    nv.applyT(srow, sn);  // row i of S N
    nv.applyT(drow, U[i]);
    // K[a][b] += N[i][a] (S N)[i][b], N's nine non-zeros written out
    if (i == 0) { k00 += n0 * sn[0]; k01 += n0 * sn[1]; k02 += n0 * sn[2]; }
    if (i == 1) { k11 += n1 * sn[1]; k12 += n1 * sn[2]; }
    if (i == 2) { k22 += n2 * sn[2]; }
    if (i == 3) { k11 += n2r * sn[1]; k12 += n2r * sn[2]; k22 += n1r * sn[2]; }
    if (i == 4) { k00 += n2r * sn[0]; k01 += n2r * sn[1]; k02 += n2r * sn[2]; k22 += n0r * sn[2]; }
    if (i == 5) { k00 += n1r * sn[0]; k01 += n1r * sn[1]; k02 += n1r * sn[2];
                  k11 += n0r * sn[1]; k12 += n0r * sn[2]; }
  }
  T m00, m01, m02, m11, m12, m22;
  const bool ok = spd3_inverse(k00, k01, k02, k11, k12, k22, m00, m01, m02, m11, m12, m22);
  const T cc = c1 * c2;
  // g = K^-1 N^T (tau_R - tau_L); tau = c1 tau_L + c2 tau_R - c1 c2 U g
  {
    T dt[6], q[3];
#pragma unroll
    for (int s = 0; s < 6; ++s) dt[s] = tR[s] - tau[s];
    nv.applyT(dt, q);
    g[0] = m00 * q[0] + m01 * q[1] + m02 * q[2];
    g[1] = m01 * q[0] + m11 * q[1] + m12 * q[2];
    g[2] = m02 * q[0] + m12 * q[1] + m22 * q[2];
#pragma unroll
    for (int s = 0; s < 6; ++s)
      tau[s] = c1 * tau[s] + c2 * tR[s] - cc * (U[s][0] * g[0] + U[s][1] * g[1] + U[s][2] * g[2]);
  }
  // residual block and plain average
  {
    T ds[6], rv[3];
#pragma unroll
    for (int s = 0; s < 6; ++s) ds[s] = sR[s] - sb[s];
    nv.applyT(ds, rv);
    rr += rfac * rfac * (rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
#pragma unroll
    for (int s = 0; s < 6; ++s) sb[s] = c1 * sb[s] + c2 * sR[s];
  }
  // G = K^-1 U^T (= (U K^-1)^T)
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    G[0 * 6 + s] = U[s][0] * m00 + U[s][1] * m01 + U[s][2] * m02;
    G[1 * 6 + s] = U[s][0] * m01 + U[s][1] * m11 + U[s][2] * m12;
    G[2 * 6 + s] = U[s][0] * m02 + U[s][1] * m12 + U[s][2] * m22;
  }
  // condensed tangent, in place: C = c1 C_L + c2 C_R - c1 c2 (U K^-1) U^T
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) {
      const T vu = G[i] * U[j][0] + G[6 + i] * U[j][1] + G[12 + i] * U[j][2];
      C[sidx(i, j)] = c1 * C[sidx(i, j)] + c2 * CR[sidx(i, j)] - cc * vu;
    }
  return ok;
}

// Top-down step: da = -(g + G e); children receive e -/+ c N da.
template <typename T>
__device__ __forceinline__ void laminate_descend(const T G[18], const T g[3], const T e[6],
                                                 const Normal<T>& nv, T c1, T c2, T da[3],
                                                 T eL[6], T eR[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T acc = g[a];
#pragma unroll
    for (int s = 0; s < 6; ++s) acc += G[a * 6 + s] * e[s];
    da[a] = -acc;
  }
  T Nd[6];
  nv.apply(da, Nd);
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    eL[s] = e[s] - c2 * Nd[s];
    eR[s] = e[s] + c1 * Nd[s];
  }
}

// Strain localisation through one laminate with jump a: children strains e -/+ c N a.
template <typename T>
__device__ __forceinline__ void laminate_localize(const T a[3], const T e[6], const Normal<T>& nv,
                                                  T c1, T c2, T eL[6], T eR[6]) {
  T Na[6];
  nv.apply(a, Na);
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    eL[s] = e[s] - c2 * Na[s];
    eR[s] = e[s] + c1 * Na[s];
  }
}

// ---------------------------------------------------------------- leaf laws

struct IsoElastic {
  double K, G;  // compression and shear modulus
};

// isotropic elastic leaf: sigma = K tr(e) I + 2G dev(e)
__device__ __forceinline__ void iso_stress(const IsoElastic& m, const double e[6], double s[6]) {
  const double tr = e[0] + e[1] + e[2];
  const double lam = m.K - 2.0 * m.G / 3.0;
  s[0] = lam * tr + 2.0 * m.G * e[0];
  s[1] = lam * tr + 2.0 * m.G * e[1];
  s[2] = lam * tr + 2.0 * m.G * e[2];
  s[3] = 2.0 * m.G * e[3];
  s[4] = 2.0 * m.G * e[4];
  s[5] = 2.0 * m.G * e[5];
}

__device__ __forceinline__ void iso_packed(const IsoElastic& m, double C[21]) {
  const double lam = m.K - 2.0 * m.G / 3.0;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) {
      double v = (i < 3 && j < 3) ? lam : 0.0;
      if (i == j) v += 2.0 * m.G;
      C[sidx(i, j)] = v;
    }
}

struct J2Law {
  double K, G, sigma0, k_inf, dsigma, b;
  int max_it;  // cap of the scalar Newton iterations of the return
};

constexpr double kSqrt23 = 0.81649658092772603273;  // sqrt(2/3)
constexpr double kLocalTol = 1e-14;
constexpr int kLocalMaxIt = 50;  // default cap of the scalar Newton iterations

// J2 radial return (implicit Euler) with sigma_Y(p) = s0 + k p + ds (1 - exp(-b p)).
// Outputs stress, packed consistent tangent and the new internal variables.
// Returns false when the scalar Newton iteration does not converge.
__device__ __forceinline__ bool j2_return(const J2Law& m, const double eps[6], const double epn[6],
                                          double pn, double sig[6], double Dp[21], double ep[6],
                                          double& p) {
  double e[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) e[s] = eps[s] - epn[s];
  const double tr = e[0] + e[1] + e[2];
  const double tr3 = tr * (1.0 / 3.0);
  double str[6];
  str[0] = 2.0 * m.G * (e[0] - tr3);
  str[1] = 2.0 * m.G * (e[1] - tr3);
  str[2] = 2.0 * m.G * (e[2] - tr3);
  str[3] = 2.0 * m.G * e[3];
  str[4] = 2.0 * m.G * e[4];
  str[5] = 2.0 * m.G * e[5];
  double q2 = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) q2 += str[s] * str[s];
  const double q = sqrt(q2);
  const double syn = m.sigma0 + m.k_inf * pn + m.dsigma * (1.0 - exp(-m.b * pn));
  const double f = q - kSqrt23 * syn;
  double x = 0.0, theta = 1.0, theta_bar = 0.0;
  bool ok = true;
  if (f > 0.0) {
    const double xtol = kLocalTol * q / (2.0 * m.G);
    ok = false;
    for (int it = 0; it < m.max_it; ++it) {
      const double pp = pn + kSqrt23 * x;
      const double ex = exp(-m.b * pp);
      const double sy = m.sigma0 + m.k_inf * pp + m.dsigma * (1.0 - ex);
      const double dsy = m.k_inf + m.dsigma * m.b * ex;
      const double gv = q - 2.0 * m.G * x - kSqrt23 * sy;
      const double dg = -2.0 * m.G - (2.0 / 3.0) * dsy;
      const double dx = -gv / dg;
      x += dx;
      if (fabs(dx) <= xtol) {
        ok = true;
        break;
      }
    }
    const double pp = pn + kSqrt23 * x;
    const double dsy = m.k_inf + m.dsigma * m.b * exp(-m.b * pp);
    theta = 1.0 - 2.0 * m.G * x / q;
    theta_bar = 1.0 / (1.0 + dsy / (3.0 * m.G)) - (1.0 - theta);
  }
  const double iq = f > 0.0 ? 1.0 / q : 0.0;
  double nh[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) nh[s] = str[s] * iq;
  const double Ktr = m.K * tr;
#pragma unroll
  for (int s = 0; s < 6; ++s) sig[s] = (s < 3 ? Ktr : 0.0) + theta * str[s];
#pragma unroll
  for (int s = 0; s < 6; ++s) ep[s] = epn[s] + x * nh[s];
  p = pn + kSqrt23 * x;
  // D = 3K P1 + 2G theta P2 - 2G theta_bar nh (x) nh
  const double g2 = 2.0 * m.G * theta;
  const double lam = m.K - g2 / 3.0;
  const double gb = 2.0 * m.G * theta_bar;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) {
      double v = (i < 3 && j < 3) ? lam : 0.0;
      if (i == j) v += g2;
      Dp[sidx(i, j)] = v - gb * nh[i] * nh[j];
    }
  return ok;
}


// Vector-Jacobian product of the J2 return mapping (j2_return).  Given the
// cotangents psi of the stress and zeta = (zeta_e, zeta_p) of the new internal
// variables (plastic strain, p), returns the cotangents of the strain (geps)
// and of the old internal variables (gz = (gz_e, gz_p)).  The forward state is
// recomputed, and the stress at eps comes out as j2_return gives it (sig).  With e = eps - ep_n, q = |s_tr|, nh = s_tr / q, dg the plastic
// multiplier, kappa = 1 / (2G + 2/3 H'(p)), beta = 2G / q, c = sqrt(2/3):
//   ge  = K (1.psi) 1 + 2G dev(psi)                         (elastic part)
//       + 2G kappa gbar nh + beta (dev(nu) - nh (nh.nu))    (plastic only)
//   gbar = -2G psi.nh + zeta_e.nh + c zeta_p,  nu = dg (zeta_e - 2G psi)
//   geps = ge,  gz_e = zeta_e - ge,  gz_p = zeta_p - c H' kappa gbar (plastic)
__device__ __forceinline__ void j2_vjp(const J2Law& m, const double eps[6], const double epn[6],
                                       double pn, const double psi[6], const double ze[6],
                                       double zp, double geps[6], double gz[7], double sig[6]) {
  double e[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) e[s] = eps[s] - epn[s];
  const double tr = e[0] + e[1] + e[2];
  const double tr3 = tr * (1.0 / 3.0);
  double str[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) str[s] = 2.0 * m.G * (s < 3 ? e[s] - tr3 : e[s]);
  double q2 = 0.0;
#pragma unroll
  for (int s = 0; s < 6; ++s) q2 += str[s] * str[s];
  const double q = sqrt(q2);
  const double syn = m.sigma0 + m.k_inf * pn + m.dsigma * (1.0 - exp(-m.b * pn));
  const double f = q - kSqrt23 * syn;
  const double ipsi = psi[0] + psi[1] + psi[2];
  double ge[6];
#pragma unroll
  for (int s = 0; s < 6; ++s)
    ge[s] = (s < 3 ? m.K * ipsi + 2.0 * m.G * (psi[s] - ipsi / 3.0) : 2.0 * m.G * psi[s]);
  double gpn = zp;
  double theta = 1.0;
  if (f > 0.0) {
    const double xtol = kLocalTol * q / (2.0 * m.G);
    double x = 0.0;
    for (int it = 0; it < m.max_it; ++it) {
      const double pp = pn + kSqrt23 * x;
      const double ex = exp(-m.b * pp);
      const double sy = m.sigma0 + m.k_inf * pp + m.dsigma * (1.0 - ex);
      const double dsy = m.k_inf + m.dsigma * m.b * ex;
      const double dx = (q - 2.0 * m.G * x - kSqrt23 * sy) / (2.0 * m.G + (2.0 / 3.0) * dsy);
      x += dx;
      if (fabs(dx) <= xtol) break;
    }
    const double pp = pn + kSqrt23 * x;
    const double Hp = m.k_inf + m.dsigma * m.b * exp(-m.b * pp);
    theta = 1.0 - 2.0 * m.G * x / q;
    const double kappa = 1.0 / (2.0 * m.G + (2.0 / 3.0) * Hp);
    const double beta = 2.0 * m.G / q;
    double nh[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) nh[s] = str[s] / q;
    double psin = 0.0, zen = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      psin += psi[s] * nh[s];
      zen += ze[s] * nh[s];
    }
    const double gbar = -2.0 * m.G * psin + zen + kSqrt23 * zp;
    double nu[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) nu[s] = x * (ze[s] - 2.0 * m.G * psi[s]);
    const double nu3 = (nu[0] + nu[1] + nu[2]) * (1.0 / 3.0);
    double nun = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) nun += nu[s] * nh[s];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const double dnu = s < 3 ? nu[s] - nu3 : nu[s];
      ge[s] += 2.0 * m.G * kappa * gbar * nh[s] + beta * (dnu - nh[s] * nun);
    }
    gpn = zp - kSqrt23 * Hp * kappa * gbar;
  }
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    geps[s] = ge[s];
    gz[s] = ze[s] - ge[s];
  }
  gz[6] = gpn;
  const double Ktr = m.K * tr;
#pragma unroll
  for (int s = 0; s < 6; ++s) sig[s] = (s < 3 ? Ktr : 0.0) + theta * str[s];
}

// Parameter cotangents of one laminate in the path adjoint: with subtree sums
// Sm_X of mu and Ss_X of w~ sigma over its children X = L, R, jumps a and
// adjoint jumps lam,
//   dJ/dn  = N(a)^T (-c2 Sm_L + c1 Sm_R) - N(lam)^T (-c2 Ss_L + c1 Ss_R)
//   dJ/dc1 = (N(n) a).(Sm_L + Sm_R) - (N(n) lam).(Ss_L + Ss_R)
// using N(n) x = N(x) n.  g4 = {dJ/dc1, dJ/dn}.
__device__ __forceinline__ void laminate_param_grad(const Normal<double>& nv, double c1, double c2,
                                                    const double a[3], const double lam[3],
                                                    const double SmL[6], const double SsL[6],
                                                    const double SmR[6], const double SsR[6],
                                                    double g4[4]) {
  double Mm[6], Ms[6], Tm[6], Ts[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    Mm[k] = -c2 * SmL[k] + c1 * SmR[k];
    Ms[k] = -c2 * SsL[k] + c1 * SsR[k];
    Tm[k] = SmL[k] + SmR[k];
    Ts[k] = SsL[k] + SsR[k];
  }
  const Normal<double> na{a[0], a[1], a[2]}, nl{lam[0], lam[1], lam[2]};
  double ga[3], gl[3];
  na.applyT(Mm, ga);
  nl.applyT(Ms, gl);
  double Na[6], Nl[6];
  nv.apply(a, Na);
  nv.apply(lam, Nl);
  double gc = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) gc += Na[k] * Tm[k] - Nl[k] * Ts[k];
  g4[0] = gc;
  g4[1] = ga[0] - gl[0];
  g4[2] = ga[1] - gl[1];
  g4[3] = ga[2] - gl[2];
}

// ------------------------------------------------ orientation interpolation

// Shape functions of the orientation-interpolation table (FE-DMN paper,
// Sec. 2.3) at fibre orientation (l1, l2): barycentric coordinates of the
// orientation triangle with vertices unidirectional (1, 0), isotropic
// (1/3, 1/3), planar isotropic (1/2, 1/2) (the closed-form solution of the
// paper's 3x3 system), then m = 3 linear, 4 tri-linear (linear minus/plus the
// cubic bubble) or 6 quadratic functions (vertex functions, then edges 1-2,
// 1-3, 2-3).
template <typename T>
__device__ __forceinline__ void orientation_shape(T l1, T l2, int m, T s[6]) {
  // Branch-free: every entry is written (zeros past m) and the callers read
  // s with compile-time indices, so the array lives in registers.  (With a
  // branch per family and a runtime-length loop over s, the uniform-branch
  // lowering merged the three families' last stores into one scratch store
  // whose offset register was left undefined on the quadratic path.)
  const T f1 = l1 - l2;
  const T f2 = T(3) - T(3) * l1 - T(3) * l2;
  const T f3 = T(2) * l1 + T(4) * l2 - T(2);
  const T b = f1 * f2 * f3;
  const bool quad = m == 6, tri = m == 4;
  s[0] = quad ? f1 * (T(2) * f1 - T(1)) : (tri ? f1 - T(9) * b : f1);
  s[1] = quad ? f2 * (T(2) * f2 - T(1)) : (tri ? f2 - T(9) * b : f2);
  s[2] = quad ? f3 * (T(2) * f3 - T(1)) : (tri ? f3 - T(9) * b : f3);
  s[3] = quad ? T(4) * f1 * f2 : (tri ? T(27) * b : T(0));
  s[4] = quad ? T(4) * f1 * f3 : T(0);
  s[5] = quad ? T(4) * f2 * f3 : T(0);
}

__device__ __forceinline__ void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sin_cos(float x, float* s, float* c) { sincosf(x, s, c); }

// Normals of laminates t, t + lanes, ... of one point / sample: angles
// alpha = p . s, beta = q . s (p, q: [L][m]) and n = (sin a cos b,
// sin a sin b, cos a) into nrm[c * L + pos]; with dalpha != nullptr also
// dn/dalpha = (cos a cos b, cos a sin b, -sin a) into dalpha[c * L + pos].
template <typename T>
__device__ __forceinline__ void orientation_normals(const T* __restrict__ p,
                                                    const T* __restrict__ q, int m, T l1,
                                                    T l2, int t, int lanes, int L, T* nrm,
                                                    T* dalpha) {
  T s[6];
  orientation_shape(l1, l2, m, s);
#pragma unroll 1
  for (int pos = t; pos < L; pos += lanes) {
    T a = T(0), b = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j < m) {
        a += p[(size_t)pos * m + j] * s[j];
        b += q[(size_t)pos * m + j] * s[j];
      }
    T sa, ca, sb, cb;
    sin_cos(a, &sa, &ca);
    sin_cos(b, &sb, &cb);
    nrm[0 * L + pos] = sa * cb;
    nrm[1 * L + pos] = sa * sb;
    nrm[2 * L + pos] = ca;
    if (dalpha != nullptr) {
      dalpha[0 * L + pos] = ca * cb;
      dalpha[1 * L + pos] = ca * sb;
      dalpha[2 * L + pos] = -sa;
    }
  }
}

}  // namespace dmn
