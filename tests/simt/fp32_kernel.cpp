// CPU build of the FP32-storage instantiation of the Gauss-point kernel
// (gp_update_kernel<K, D, float, false>: per-point arrays read and written in
// FP32, arithmetic in FP64), which the device build does not compile.  The
// kernel source is included as is; this file only adds a host entry point that
// builds the DMN table and the launch arguments the way the library's call
// does and launches the instantiation for one group.  Test infrastructure.
#include <stdlib.h>

#include "dmn_gp.hip"

namespace {

template <int K, int D>
void launch_f32(const dmn::GpLaunch& args, int n_blocks) {
  hipLaunchKernelGGL((dmn::gp_update_kernel<K, D, float, false>), dim3(n_blocks), dim3(64), 0,
                     nullptr, args);
}

}  // namespace

extern "C" int simt_gp_update_f32(int depth, int lanes, const double* w, const double* n,
                                  long long P, const float* E, const float* z_in, float* z_out,
                                  const float* a_in, float* a_out, float* sigma, float* tangent,
                                  int32_t* iters, int32_t* status, const double* fib,
                                  const double* mat, double tol, int max_iter, int max_bt,
                                  double armijo) {
  const size_t tab_bytes = 256 + (dmn::table_elems(depth) * sizeof(double) + 255) / 256 * 256;
  char* ws = (char*)aligned_alloc(256, 256 + tab_bytes);
  if (!ws) return -1;
  int32_t* counter = (int32_t*)ws;
  int32_t* flag = (int32_t*)(ws + 256);
  double* rows = (double*)(ws + 512);
  int rc = dmn::launch_prep_tables(w, n, depth, DMN_F64, rows, flag, nullptr, nullptr, true);
  rc = rc ? rc : dmn::launch_zero_ints(counter, 1, nullptr);
  dmn::GpLaunch a;
  memset(&a, 0, sizeof(a));
  a.max_iter = max_iter;
  a.max_bt = max_bt;
  a.tol = tol;
  a.armijo = armijo;
  a.fib.K = fib[0] / (3.0 * (1.0 - 2.0 * fib[1]));
  a.fib.G = fib[0] / (2.0 * (1.0 + fib[1]));
  a.mat.K = mat[0] / (3.0 * (1.0 - 2.0 * mat[1]));
  a.mat.G = mat[0] / (2.0 * (1.0 + mat[1]));
  a.mat.sigma0 = mat[2];
  a.mat.k_inf = mat[3];
  a.mat.dsigma = mat[4];
  a.mat.b = mat[5];
  a.mat.max_it = dmn::kLocalMaxIt;
  dmn::GroupArgs& g = a.g[0];
  g.E = E;
  g.z_in = z_in;
  g.z_out = z_out;
  g.a_in = a_in;
  g.a_out = a_out;
  g.sigma = sigma;
  g.tangent = tangent;
  g.iters = iters;
  g.status = status;
  g.tab = rows;
  g.flag = flag;
  g.P = P;
  g.depth = depth;
  g.lanes = lanes;
  a.ng = 1;
  a.counter = counter;
  const int ppw = 64 / lanes;
  a.total = (int)((P + ppw - 1) / ppw);
  const int D = depth - dmn::tree::ilog2(lanes);
  if (rc == 0) {
    switch (depth * 16 + D) {
      case 8 * 16 + 2: launch_f32<8, 2>(a, 2); break;
      case 5 * 16 + 1: launch_f32<5, 1>(a, 2); break;
      case 3 * 16 + 2: launch_f32<3, 2>(a, 2); break;
      case 1 * 16 + 1: launch_f32<1, 1>(a, 2); break;
      default: rc = -1;
    }
  }
  free(ws);
  return rc;
}
