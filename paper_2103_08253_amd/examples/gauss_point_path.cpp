// Host-side use of libdmn from C++ without Python: the way an implicit FE
// code's material routine would drive dmn_update_gauss_points (Sec. 3.2, the
// online evaluation): device buffers for one batch of Gauss points, a strain
// path applied step by step from the last converged state, internal variables
// and jumps ping-ponged between steps.
//
//   gauss_point_path <in.bin> <out.bin>
//
// in.bin  (little endian): int32 K, int64 P, int32 T, then doubles
//         w [2^K], n [2^K - 1][3], E [T][P][6], fibre (E, nu),
//         matrix (E, nu, sigma0, k_inf, dsigma, b), Newton tol
// out.bin: per step sigma [P][6] and tangent [P][36] (doubles), then
//         status [P] and iters [P] (int32)
// Exit code 0 on success; a failed HIP call or library call prints its name.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "dmn.h"

#define HIP_OK(x)                                                  \
  do {                                                             \
    if ((x) != hipSuccess) {                                       \
      fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(x)); \
      return 2;                                                    \
    }                                                              \
  } while (0)

template <typename T>
static bool take(FILE* f, T* p, size_t n) {
  return fread(p, sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
    return 1;
  }
  FILE* in = fopen(argv[1], "rb");
  if (!in) return 1;
  int32_t K = 0, T = 0;
  int64_t P = 0;
  if (!take(in, &K, 1) || !take(in, &P, 1) || !take(in, &T, 1) || K < 1 || K > DMN_MAX_DEPTH ||
      P < 1 || T < 1)
    return 1;
  const size_t NL = (size_t)1 << K, L = NL - 1, M = NL / 2;
  std::vector<double> w(NL), n(3 * L), E((size_t)T * P * 6), fib(2), mat(6);
  double tol = 0.0;
  if (!take(in, w.data(), NL) || !take(in, n.data(), 3 * L) || !take(in, E.data(), E.size()) ||
      !take(in, fib.data(), 2) || !take(in, mat.data(), 6) || !take(in, &tol, 1))
    return 1;
  fclose(in);

  hipStream_t s;
  HIP_OK(hipStreamCreate(&s));
  double *dw, *dn, *dE, *z0, *z1, *a0, *a1, *sig, *tan;
  int32_t *iters, *status;
  HIP_OK(hipMalloc(&dw, NL * 8));
  HIP_OK(hipMalloc(&dn, 3 * L * 8));
  HIP_OK(hipMalloc(&dE, (size_t)P * 6 * 8));
  HIP_OK(hipMalloc(&z0, (size_t)P * M * 7 * 8));
  HIP_OK(hipMalloc(&z1, (size_t)P * M * 7 * 8));
  HIP_OK(hipMalloc(&a0, (size_t)P * L * 3 * 8));
  HIP_OK(hipMalloc(&a1, (size_t)P * L * 3 * 8));
  HIP_OK(hipMalloc(&sig, (size_t)P * 6 * 8));
  HIP_OK(hipMalloc(&tan, (size_t)P * 36 * 8));
  HIP_OK(hipMalloc(&iters, (size_t)P * 4));
  HIP_OK(hipMalloc(&status, (size_t)P * 4));
  HIP_OK(hipMemcpy(dw, w.data(), NL * 8, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dn, n.data(), 3 * L * 8, hipMemcpyHostToDevice));
  HIP_OK(hipMemset(z0, 0, (size_t)P * M * 7 * 8));  // initial state z = 0, a = 0
  HIP_OK(hipMemset(a0, 0, (size_t)P * L * 3 * 8));

  dmn_point_group g = {};
  g.net.depth = K;
  g.net.w = dw;
  g.net.n = dn;
  g.net.ori_shape = DMN_ORI_NONE;
  g.P = P;
  g.E = dE;
  g.sigma = sig;
  g.tangent = tan;
  g.iters = iters;
  g.status = status;
  const dmn_elastic fibre{fib[0], fib[1]};
  const dmn_j2 matrix{mat[0], mat[1], mat[2], mat[3], mat[4], mat[5]};
  const dmn_newton_opts opts{tol, 25, 10, 1e-4, 0, 0};

  g.z_in = z0;
  g.z_out = z1;
  g.a_in = a0;
  g.a_out = a1;
  const size_t ws_bytes = dmn_update_gauss_points_workspace_size(&g, 1, DMN_F64);
  if (ws_bytes == 0) {
    fprintf(stderr, "dmn_update_gauss_points_workspace_size rejected the group\n");
    return 3;
  }
  void* ws;
  HIP_OK(hipMalloc(&ws, ws_bytes));

  FILE* out = fopen(argv[2], "wb");
  if (!out) return 1;
  std::vector<double> hs((size_t)P * 6), ht((size_t)P * 36);
  std::vector<int32_t> hst(P), hit(P);
  for (int t = 0; t < T; ++t) {
    HIP_OK(hipMemcpyAsync(dE, E.data() + (size_t)t * P * 6, (size_t)P * 6 * 8,
                          hipMemcpyHostToDevice, s));
    const int rc = dmn_update_gauss_points(&g, 1, &fibre, &matrix, DMN_F64, &opts, ws, ws_bytes, s);
    if (rc != DMN_OK) {
      fprintf(stderr, "dmn_update_gauss_points returned %d\n", rc);
      return 3;
    }
    HIP_OK(hipMemcpyAsync(hs.data(), sig, hs.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(ht.data(), tan, ht.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(hst.data(), status, P * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(hit.data(), iters, P * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    fwrite(hs.data(), 8, hs.size(), out);
    fwrite(ht.data(), 8, ht.size(), out);
    fwrite(hst.data(), 4, P, out);
    fwrite(hit.data(), 4, P, out);
    // accept the step: the outputs become the next step's inputs
    const void* zt = g.z_in;
    g.z_in = g.z_out;
    g.z_out = (void*)zt;
    const void* at = g.a_in;
    g.a_in = g.a_out;
    g.a_out = (void*)at;
  }
  fclose(out);
  for (void* p : {(void*)dw, (void*)dn, (void*)dE, (void*)z0, (void*)z1, (void*)a0, (void*)a1,
                  (void*)sig, (void*)tan, (void*)iters, (void*)status, ws})
    HIP_OK(hipFree(p));
  HIP_OK(hipStreamDestroy(s));
  return 0;
}
