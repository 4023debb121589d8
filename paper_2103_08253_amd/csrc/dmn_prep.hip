// Per-DMN parameter preparation (FE-DMN paper, Sec. 2.1 weight propagation
// and volume fractions; Sec. 3.2 weight matrix W).
//
// From the leaf weights w[2^K] and the normals n[2^K-1][3] (paper order) one
// workgroup builds the laminate table used by every kernel (workgroup g of a
// grouped launch: normals n + g L 3, table and flag tab_stride bytes after
// the first):
//   c1 = W_L / (W_L + W_R), c2 = 1 - c1   (W_X: summed leaf weights of a child)
//   n                                      (copied as passed; zero if n is null,
//                                           for normals interpolated per point)
//   rfac = W_L W_R / ((W_L + W_R) sum(w))  (scale of the laminate's block of A^T W sigma)
//   dc1/dW_L = W_R / W^2, dc1/dW_R = -W_L / W^2
// followed by the leaf section w / sum(w) [2^K] and 1 / sum(w), and a
// field-major copy of the first six fields; flags the DMN as invalid when a
// weight is negative or not finite, or no leaf carries weight.  A laminate
// whose children carry no weight (a dead subtree) is flagged too, unless the
// caller accepts dead subtrees (the linear map and its VJP): then its row is
// c1 = c2 = 1/2, rfac = 0, dc1/dW = 0, so the subtree stays finite while its
// live parent, whose fraction for it is exactly 0, takes the other child's
// result unchanged and passes it no cotangent, which is what removing the
// subtree from the tree (Sec. 3.1, tree compression) computes.  Subtree sums
// are formed pairwise in a fixed order, so the table is bit-identical run to
// run.
#include "dmn_groups.hpp"

namespace dmn {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void prep_kernel(const T* __restrict__ w, const T* __restrict__ n,
                                                   int K, T* __restrict__ tab0,
                                                   int32_t* __restrict__ flag0,
                                                   long long tab_stride,
                                                   int32_t* __restrict__ err, int allow_dead) {
  // node sums of the whole tree in LDS, heap order: node 1 = root, leaves at
  // 2^K ... 2^(K+1)-1; each internal node is the sum of its two children
  __shared__ T W[2 << DMN_MAX_DEPTH];
  __shared__ int bad;
  const int nleaf = 1 << K;
  const int L = nleaf - 1;
  const long long g = blockIdx.x;
  T* tab = (T*)((char*)tab0 + g * tab_stride);
  int32_t* flag = (int32_t*)((char*)flag0 + g * tab_stride);
  if (n) n += g * L * 3;
  if (threadIdx.x == 0) bad = 0;
  int mybad = 0;
  for (int j = threadIdx.x; j < nleaf; j += blockDim.x) {
    const T v = w[j];
    if (!(v >= T(0)) || !isfinite(v)) mybad = 1;
    W[nleaf + j] = v;
  }
  __syncthreads();
  for (int k = K; k >= 1; --k) {  // heap level k holds 2^(k-1) laminates
    const int first = 1 << (k - 1);
    for (int h = first + threadIdx.x; h < 2 * first; h += blockDim.x)
      W[h] = W[2 * h] + W[2 * h + 1];
    __syncthreads();
  }
  const T wtot = W[1];
  if (!(wtot > T(0))) mybad = 1;
  for (int pos = threadIdx.x; pos < L; pos += blockDim.x) {
    // level k and 0-based index i0 of the laminate at paper position pos
    int k = K, base = 0;
    while (pos >= base + (1 << (k - 1))) {
      base += 1 << (k - 1);
      --k;
    }
    const int h = (1 << (k - 1)) + (pos - base);  // heap index
    const T WL = W[2 * h], WR = W[2 * h + 1];
    const T Wn = WL + WR;
    const bool live = Wn > T(0);
    if (!live && !allow_dead) mybad = 1;
    T* r = tab + (size_t)pos * kTabStride;
    const T c1 = live ? WL / Wn : T(0.5);
    r[0] = c1;
    r[1] = T(1) - c1;
    r[2] = n ? n[(size_t)pos * 3 + 0] : T(0);  // no fixed normals: filled per point
    r[3] = n ? n[(size_t)pos * 3 + 1] : T(0);
    r[4] = n ? n[(size_t)pos * 3 + 2] : T(0);
    r[5] = live ? WL * WR / (Wn * wtot) : T(0);
    r[6] = live ? WR / (Wn * Wn) : T(0);
    r[7] = live ? -WL / (Wn * Wn) : T(0);
    T* soa = tab + table_soa_offset(K);
#pragma unroll
    for (int f = 0; f < 6; ++f) soa[(size_t)f * L + pos] = r[f];
  }
  // leaf section: normalised weights w / sum(w), then 1 / sum(w)
  T* leafw = tab + (size_t)L * kTabStride;
  for (int j = threadIdx.x; j < nleaf; j += blockDim.x) leafw[j] = W[nleaf + j] / wtot;
  if (threadIdx.x == 0) leafw[nleaf] = T(1) / wtot;
  if (mybad) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    *flag = bad;
    if (err) *err = 0;
  }
}

__global__ void zero_ints_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// dst[i] = (To)src[i], grid-stride; rounds to nearest when narrowing
template <typename From, typename To>
__global__ __launch_bounds__(256) void convert_kernel(const From* __restrict__ src,
                                                      To* __restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = (To)src[i];
}

template <typename From, typename To>
int launch_convert_t(const void* src, void* dst, long long n, hipStream_t stream) {
  if (n <= 0) return 0;
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((convert_kernel<From, To>), dim3((unsigned)blocks), dim3(256), 0, stream,
                     (const From*)src, (To*)dst, n);
  return (int)hipGetLastError();
}

}  // namespace

int launch_widen(const float* src, double* dst, long long n, hipStream_t stream) {
  return launch_convert_t<float, double>(src, dst, n, stream);
}

int launch_narrow(const double* src, float* dst, long long n, hipStream_t stream) {
  return launch_convert_t<double, float>(src, dst, n, stream);
}

int launch_zero_ints(int32_t* p, int n, hipStream_t stream) {
  hipLaunchKernelGGL(zero_ints_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
  return (int)hipGetLastError();
}

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

static int launch_prep(const void* w, const void* n, int depth, int prec, int G, void* tab,
                       int32_t* flag, long long tab_stride, int32_t* err, hipStream_t stream,
                       bool allow_dead) {
  if (G < 1) return (int)hipSuccess;
  if (prec == DMN_F32) {
    hipLaunchKernelGGL(prep_kernel<float>, dim3((unsigned)G), dim3(256), 0, stream,
                       (const float*)w, (const float*)n, depth, (float*)tab, flag, tab_stride,
                       err, allow_dead ? 1 : 0);
  } else {
    hipLaunchKernelGGL(prep_kernel<double>, dim3((unsigned)G), dim3(256), 0, stream,
                       (const double*)w, (const double*)n, depth, (double*)tab, flag, tab_stride,
                       err, allow_dead ? 1 : 0);
  }
  return (int)hipGetLastError();
}

int launch_prep_tables(const void* w, const void* n, int depth, int prec, void* tab, int32_t* flag,
                       int32_t* err, hipStream_t stream, bool allow_dead) {
  return launch_prep(w, n, depth, prec, 1, tab, flag, 0, err, stream, allow_dead);
}

int launch_prep_tables_groups(const void* w, const void* n, int depth, int prec, int G, void* tab,
                              int32_t* flag, long long tab_stride, int32_t* err,
                              hipStream_t stream) {
  return launch_prep(w, n, depth, prec, G, tab, flag, tab_stride, err, stream, true);
}

}  // namespace dmn
