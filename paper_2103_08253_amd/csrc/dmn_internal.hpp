// Internal declarations shared by the libdmn translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dmn.h"
#include "dmn_algebra.hpp"

namespace dmn {

// Per-laminate table row, in paper order, built on the device from (w, n):
//   c1, c2, n0, n1, n2, rfac, dc1/dW_L, dc1/dW_R
// rfac = W_L W_R / (W sum(w)) scales the laminate's residual block; the last
// two entries are the derivatives of c1 = W_L / (W_L + W_R).
constexpr int kTabStride = 8;
// After the L rows: normalised leaf weights [2^K], then 1 / sum(w), then a
// field-major copy [6][L] of c1, c2, n0, n1, n2, rfac (8-element aligned).
__host__ __device__ inline size_t table_soa_offset(int depth) {
  const size_t L = ((size_t)1 << depth) - 1;
  return (L * kTabStride + ((size_t)1 << depth) + 1 + 7) / 8 * 8;
}
__host__ __device__ inline size_t table_elems(int depth) {
  return table_soa_offset(depth) + 6 * (((size_t)1 << depth) - 1);
}

// Point-group description passed by value to the Gauss-point kernel.
struct GroupArgs {  // tab points at the table start (AoS rows first)
  // per-point arrays in the storage precision of the launch (FP64 or FP32)
  const void* E;
  const void* z_in;
  void* z_out;
  const void* a_in;
  void* a_out;
  void* sigma;
  void* tangent;
  int32_t* iters;
  int32_t* status;
  const double* ori_p;  // [L][ori_m] angle coefficients (orientation launches)
  const double* ori_q;
  const double* lam;    // [P][2] per-point (l1, l2)
  int ori_m;            // number of shape functions (3, 4, 6), 0 without interpolation
  int depth;            // DMN depth K
  const double* tab;   // [L][kTabStride]
  const int32_t* flag; // nonzero: invalid DMN parameters
  long long P;
  int block0;          // first work item of this group in its counter's numbering
  int lanes;           // lanes per point of the group's variant
};

constexpr int kMaxGroupsPerLaunch = 16;

struct GpLaunch {
  GroupArgs g[kMaxGroupsPerLaunch];
  int* counter;  // zeroed before the launch; batches are taken with atomicAdd
  int total;     // batches in this launch
  int ng;
  // mixed-depth launches: groups [0, ng_split) are depth-9 groups whose points
  // are split over two waves, taken one point at a time from counter_split
  int* counter_split;
  int total_split;
  int ng_split;
  int max_iter;
  int max_bt;
  int polish;  // full Newton steps after the stop test is met (not counted, no backtracking)
  double tol;
  double armijo;
  IsoElastic fib;
  J2Law mat;
};
static_assert(sizeof(GpLaunch) <= 4096, "kernel arguments are passed by value");

// Host launchers (return hipError_t as int).
// allow_dead: accept subtrees without weight (linear map and its VJP), see dmn_prep.hip
int launch_prep_tables(const void* w, const void* n, int depth, int prec, void* tab, int32_t* flag,
                       int32_t* err, hipStream_t stream, bool allow_dead = false);
int launch_gp_update(int depth, int lanes_per_point, int prec, bool ori, const GpLaunch& args,
                     int n_blocks, hipStream_t stream);
// one launch over groups of several depths (fixed normals, FP64): n_workgroups
// persistent workgroups of two waves
int launch_gp_mixed(const GpLaunch& args, int n_workgroups, hipStream_t stream);
// depth whose points are split over two waves, and its lanes per point
constexpr int kSplitDepth = 9;
constexpr int kSplitLanes = 128;
// lane-subtree depth of every depth in a mixed launch
constexpr int kMixedLaneDepth = 2;
int launch_zero_ints(int32_t* p, int n, hipStream_t stream);
// element-wise precision conversion of n values (FP32 <-> FP64)
int launch_widen(const float* src, double* dst, long long n, hipStream_t stream);
int launch_narrow(const double* src, float* dst, long long n, hipStream_t stream);
// compute units of the current device (cached per device)
int device_cu_count();
int gp_points_per_block(int depth, int lanes_per_point);
int gp_default_lanes_per_point(int depth);
// lane counts per point of the compiled variants for a depth (writes up to cap,
// returns how many exist)
int gp_lane_variants(int depth, int* lanes, int cap);
constexpr int kDefaultWavesPerCu = 8;

// Orientation-interpolated normals of a linear launch (m = 0: fixed normals):
// angle coefficients p, q [L][m], per-sample (l1, l2) lam [B][2], and for the
// backward the per-sample angle cotangents gang [L][2][B] (workspace).
struct LinOriArgs {
  const void* p = nullptr;
  const void* q = nullptr;
  const void* lam = nullptr;
  void* gang = nullptr;
  int m = 0;
};
int launch_linear_forward(int depth, int prec, const void* tab, const int32_t* flag, long long B,
                          const void* C1, const void* C2, void* Cbar, int32_t* err,
                          const LinOriArgs& ori, hipStream_t stream);
int launch_linear_backward(int depth, int prec, const void* tab, const int32_t* flag,
                           long long B, const void* C1, const void* C2, const void* gCbar,
                           void* gw, void* gn, void* gC1, void* gC2, double* partials,
                           double* gsum, int32_t* err, const LinOriArgs& ori,
                           hipStream_t stream);
// number of partial-sum slots (waves x samples per wave) the backward uses
long long linear_backward_partials(int depth, long long B, bool f32);

// One point group of the path adjoint (device pointers).
struct AdjointLaunch {
  const double* E;
  const double* z_in;
  const double* a_conv;
  const double* g_sigma;
  const double* g_z_next;
  double* g_z_prev;
  const double* tab;
  const int32_t* flag;
  double* partials;  // [4 L + 2^K][slots]
  double* gsum;      // [4 L + 2^K]
  double* gw;
  double* gn;
  int32_t* err;
  long long P;
  IsoElastic fib;
  J2Law mat;
};

long long adjoint_partial_slots(int depth, long long P);

// Training: data term and cotangent of the objective (scratch: 3 B doubles),
// optimiser step and parameter refresh, stiffness sampler.
int launch_training_loss(int prec, long long B, double p, double q, const void* Cbar,
                         const void* target, void* e_out, void* gCbar, double* stats,
                         double* scratch, hipStream_t stream);
struct TrainUpdateArgs {
  void* v;
  void* alpha;
  void* beta;
  void* w;
  void* n;
  void* state;
  long long* step;
  const void* gw;
  const void* gn;
  double* stats;
  double lr_min, lr_max, lr_decay, beta1, beta2, eps, penalty;
  int half_period, steps_per_epoch;
  int take_step;  // 0: only refresh w and n from v, alpha, beta
};
int launch_training_update(int prec, int depth, const TrainUpdateArgs& args, hipStream_t stream);
int launch_sample_stiffness(int prec, long long B, const double* u, void* C1, void* C2,
                            hipStream_t stream);
// Orientation groups: normals [G][L][3] of each group, chain of per-group
// cotangents to gw and the coefficient cotangents [L][2][m], and the update of
// (v, p, q) (p, q passed in TrainUpdateArgs::alpha / beta, their gradients in gn).
int launch_group_normals(int prec, int depth, int m, int G, const void* p, const void* q,
                         const void* lam, void* n, hipStream_t stream);
int launch_group_chain(int prec, int depth, int m, int G, const void* p, const void* q,
                       const void* lam, const void* gw_g, const void* gn_g, void* gw, void* gpq,
                       hipStream_t stream);
int launch_training_update_coeff(int prec, int depth, int m, const TrainUpdateArgs& args,
                                 hipStream_t stream);
int launch_adjoint(int depth, const AdjointLaunch& args, hipStream_t stream);

}  // namespace dmn
