// Sample groups of the linear map and its VJP: several DMNs of one depth in
// one launch, as orientation-group training needs (one DMN per fibre
// orientation of a discrete set, all sharing the leaf weights).
#pragma once
#include "dmn_internal.hpp"

namespace dmn {

// DMNs whose tables (and flags) sit tab_stride bytes apart; group g owns
// samples off[g] .. off[g+1]-1 of the batch and workgroups
// block0[g] .. block0[g+1]-1 of the launch.  The plain calls are the
// one-group case.
constexpr int kMaxLinGroups = 64;
struct LinGroups {
  long long off[kMaxLinGroups + 1];
  int block0[kMaxLinGroups + 1];
  int ng;
  long long tab_stride;
};

// G groups at once (sample offsets off[0..G], absolute, non-decreasing).  The
// backward writes gw [G][2^K] and gn [G][L][3] (every group, also an empty
// one, whose gradients are zero) and needs linear_backward_group_slots
// partial slots.  Launches are split into chunks of at most kMaxLinGroups
// groups.
int launch_linear_forward_groups(int depth, int prec, const void* tab, const int32_t* flag,
                                 long long tab_stride, int G, const int64_t* off,
                                 const void* C1, const void* C2, void* Cbar, int32_t* err,
                                 hipStream_t stream);
int launch_linear_backward_groups(int depth, int prec, const void* tab, const int32_t* flag,
                                  long long tab_stride, int G, const int64_t* off,
                                  const void* C1, const void* C2, const void* gCbar, void* gw,
                                  void* gn, double* partials, double* gsum, int32_t* err,
                                  hipStream_t stream);
long long linear_backward_group_slots(int depth, int G, const int64_t* off, bool f32);

// Tables of G DMNs sharing the leaf weights w, with normals n + g L 3 and
// tables and flags tab_stride bytes apart (one workgroup each); dead subtrees
// accepted as for the linear map.
int launch_prep_tables_groups(const void* w, const void* n, int depth, int prec, int G, void* tab,
                              int32_t* flag, long long tab_stride, int32_t* err,
                              hipStream_t stream);

}  // namespace dmn
