/*
 * libdmn — batched online evaluation and training kernels of direct deep
 * material networks (DMNs) on AMD Instinct MI355X (gfx950).
 *
 * A direct DMN of depth K is a perfect binary tree of 2^K - 1 rank-one
 * laminates over 2^K leaves (FE-DMN paper, Sec. 2.1).  Leaves alternate
 * between phase 1 (the linear elastic fibre; even 0-based leaf index) and
 * phase 2 (the J2 elasto-plastic matrix; odd index).  Laminate volume
 * fractions follow from the leaf weights by weight propagation
 * (c1 = W_left / (W_left + W_right), Sec. 2.1); every laminate has a
 * lamination normal.
 *
 * Conventions shared by all calls
 *   - Mandel notation: symmetric tensors are 6-vectors
 *     [11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12]; stiffnesses and tangents are
 *     6x6 Mandel matrices stored row-major as 36 numbers.  Mandel l2 norms are
 *     Frobenius norms.
 *   - Paper order of laminates (Sec. 3.1/3.2): deepest level K first, then
 *     K-1, ..., root last; laminate (k, i) (level k, 1-based index i) sits at
 *     position 2^K - 2^k + i - 1.  Normals and jump vectors use this order.
 *   - Per-point arrays are point-major: the record of point p is contiguous
 *     (an FE code's per-integration-point state vector).
 *   - Every pointer argument of type void* / int32_t* inside the structs and
 *     the data arguments is a DEVICE pointer owned by the caller; the structs
 *     themselves are host memory read during the call only.  Device buffers
 *     must stay alive until the stream reaches the enqueued work.
 *   - Calls enqueue kernels on `stream` and return at once.  They allocate
 *     nothing, never synchronise and never read device data on the host, so
 *     they can be captured into a HIP graph.  The return code reflects only
 *     host-side argument validation and launch errors; per-point device
 *     outcomes are written to the status arrays.
 *   - Workspace: each call needs a device workspace of at least the size its
 *     *_workspace_size() query returns (256-byte aligned base), queried with
 *     the device current that the call will run on: the sizes of the linear
 *     VJP and of the adjoint follow the number of waves that device holds at
 *     once.  A call given less than its device needs returns DMN_EWORKSPACE.
 *   - Sizes: point and sample counts are int64 and every element offset into
 *     a per-point or per-sample array is computed in 64 bits, so arrays may
 *     exceed 2^31 elements; a count of 0 is valid (no data array is read and
 *     its pointer may be NULL).  dmn_update_gauss_points returns DMN_EINVAL
 *     when one launch would take more than 2^31 - 1 work items (batches of
 *     points); the linear calls' limit, 2^31 - 1 workgroups of 1 to 64
 *     samples, lies beyond any batch that fits in device memory.
 *   - No C++ exception crosses this interface.  Calls on different streams
 *     may run concurrently as long as they use different workspaces.
 */
#ifndef DMN_H
#define DMN_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes (host-side) */
#define DMN_OK 0
#define DMN_EINVAL (-1)       /* null pointer, depth outside [1,10], bad sizes or options */
#define DMN_EWORKSPACE (-2)   /* workspace missing or smaller than the size query */
#define DMN_EHIP (-3)         /* a HIP launch failed */
#define DMN_EUNSUPPORTED (-4) /* precision / option combination not implemented, or a
                                 depth not run on the device (see DMN_MAX_DEPTH) */

/* precision of storage and arithmetic */
#define DMN_F64 0       /* FP64 storage, FP64 arithmetic */
#define DMN_F32 1       /* FP32 storage, FP32 arithmetic (linear map, its backward and
                           the training calls, which keep their sums in FP64) */
#define DMN_F32_STATE 2 /* FP32 storage of per-point arrays, FP64 arithmetic
                           (dmn_update_gauss_points) */

/* per-point status written by dmn_update_gauss_points */
#define DMN_STATUS_OK 0        /* converged */
#define DMN_STATUS_MAXITER 1   /* Newton iteration limit reached */
#define DMN_STATUS_NONFINITE 2 /* non-finite input or residual */
#define DMN_STATUS_NOTSPD 3    /* a laminate pivot of the Hessian is not positive definite */
#define DMN_STATUS_LOCAL 4     /* J2 return mapping did not converge */
#define DMN_STATUS_BADPARAM 5  /* negative or non-finite leaf weight, or no weight at all */

/* Depths 1..DMN_MAX_DEPTH pass argument validation.  Deeper than the depths
 * below, a call returns DMN_EUNSUPPORTED: its kernels compile but hold
 * several KB of register spills per lane and have not been run on the device.
 *   DMN_MAX_RUN_DEPTH:      dmn_update_gauss_points, dmn_homogenize_linear,
 *                           dmn_homogenize_linear_groups
 *   DMN_MAX_RUN_DEPTH_VJP:  dmn_homogenize_backward,
 *                           dmn_homogenize_backward_groups, dmn_update_adjoint,
 *                           and orientation-interpolated groups of
 *                           dmn_update_gauss_points
 * The training update, refresh and orientation-group calls take every depth
 * up to DMN_MAX_DEPTH. */
#define DMN_MAX_DEPTH 10
#define DMN_MAX_RUN_DEPTH 9
#define DMN_MAX_RUN_DEPTH_VJP 8

/* Fibre-orientation interpolation of the normals (Sec. 2.3): shape-function
 * family of the orientation-interpolation table and its number M of
 * functions. */
#define DMN_ORI_NONE 0      /* fixed normals n */
#define DMN_ORI_LINEAR 1    /* M = 3 */
#define DMN_ORI_TRILINEAR 2 /* M = 4 (linear plus the cubic bubble) */
#define DMN_ORI_QUADRATIC 3 /* M = 6 */

/* A direct DMN: depth K, leaf weights w[2^K] (non-negative, need not sum to
 * one: fractions are weight ratios and averages use w / sum(w)).  Leaves of
 * zero weight are allowed, also whole subtrees without weight (dead
 * subtrees, which training produces): the linear map, its backward, the
 * Gauss-point update and its adjoint remove them from the tree, which is the
 * paper's tree
 * compression (Sec. 3.1) computed in place (a laminate with a dead child
 * passes its other child through unchanged; dead leaves still run their leaf
 * law, their internal variables and the jumps of removed laminates carry no
 * meaning; the adjoint's cotangents of removed leaves' weights are finite but
 * not derivatives).  The net also has either
 *   ori_shape = DMN_ORI_NONE: normals n[2^K - 1][3] in paper order (unit
 *     length expected; used as passed); or
 *   ori_shape = DMN_ORI_LINEAR / TRILINEAR / QUADRATIC: normals that depend
 *     on each point's fibre orientation (l1, l2), the two largest eigenvalues
 *     of its second-order orientation tensor (Sec. 2.3).  (l1, l2) is mapped
 *     to barycentric coordinates of the orientation triangle with vertices
 *     unidirectional (1, 0), isotropic (1/3, 1/3), planar isotropic (1/2, 1/2);
 *     with the M shape functions s of the family, laminate i has angles
 *     alpha = ori_p[i] . s, beta = ori_q[i] . s and normal
 *     (sin alpha cos beta, sin alpha sin beta, cos alpha).  ori_p, ori_q are
 *     [2^K - 1][M] in paper order; n is not read.  Points outside the
 *     triangle extrapolate the polynomials.  Supported by
 *     dmn_update_gauss_points (per-point orientation) and, up to depth 8,
 *     by the linear map and its backward (per-sample orientation, see
 *     there; deeper nets return DMN_EUNSUPPORTED); training over a discrete
 *     set of orientations can also run the fixed-normal calls per
 *     orientation group (dmn_orientation_group_normals and the calls after
 *     it).  dmn_update_adjoint returns DMN_EUNSUPPORTED.
 * All arrays are device memory in the precision of the call. */
typedef struct dmn_net {
  int32_t depth;
  const void* w;
  const void* n;
  int32_t ori_shape;
  const void* ori_p;
  const void* ori_q;
} dmn_net;

/* Isotropic linear elastic phase 1 (the fibre): Young's modulus, Poisson ratio. */
typedef struct dmn_elastic {
  double E, nu;
} dmn_elastic;

/* J2 phase 2 (the matrix), Sec. 4.1: von Mises yield with
 * sigma_Y(p) = sigma0 + k_inf p + dsigma (1 - exp(-b p)), p the accumulated
 * equivalent plastic strain. */
typedef struct dmn_j2 {
  double E, nu, sigma0, k_inf, dsigma, b;
} dmn_j2;

/* Newton options (Sec. 3.2, Sec. 4.6): stop when
 * |A^T W sigma| <= tol (2^K - 1) |sigma_bar| (Frobenius norms); at most
 * max_iter Newton steps; backtracking halves the step while the trial residual
 * is non-finite or |r(a + s da)| > (1 - armijo s) |r(a)|, at most
 * max_backtrack times (the last trial is then taken as it is).
 * local_max_iter caps the scalar Newton iterations of the J2 return at every
 * matrix leaf (0 selects the default 50); a return that has not converged
 * within it fails the point with DMN_STATUS_LOCAL.  polish (>= 0) adds that
 * many full Newton steps once the stop test is met, taken without the
 * backtracking test and not counted in iters: with 1 the returned jumps
 * satisfy the Euler-Lagrange equation to roundoff, which a derivative of the
 * converged path (the path adjoint) assumes; 0 for the plain update. */
typedef struct dmn_newton_opts {
  double tol;
  int32_t max_iter;
  int32_t max_backtrack;
  double armijo;
  int32_t local_max_iter;
  int32_t polish;
} dmn_newton_opts;

/* One batch of Gauss points that share a DMN.  With M = 2^(K-1) matrix
 * leaves and L = 2^K - 1 laminates (all arrays FP64, point-major):
 *   E       [P][6]     macro strain of the new step
 *   z_in    [P][M][7]  internal variables of the last converged step, per
 *                      matrix leaf: plastic strain (Mandel 6) then p
 *   z_out   [P][M][7]  updated internal variables
 *   a_in    [P][L][3]  jumps of the last converged step (initial guess)
 *   a_out   [P][L][3]  converged jumps
 *   sigma   [P][6]     effective stress sum_j w~_j sigma_j
 *   tangent [P][36]    algorithmic tangent d sigma / d E
 *   iters   [P]        Newton steps taken
 *   status  [P]        DMN_STATUS_*
 *   lam     [P][2]     fibre orientation (l1, l2) of each point when
 *                      net.ori_shape is not DMN_ORI_NONE (else not read)
 * The update is functional: z_in and a_in are never written, and must not
 * alias z_out / a_out.  On a non-zero status z_out = z_in and a_out = a_in so
 * the caller can retry with a smaller increment; sigma then holds the last
 * iterate and tangent is NaN. */
typedef struct dmn_point_group {
  dmn_net net;
  int64_t P;
  const void* E;
  const void* z_in;
  void* z_out;
  const void* a_in;
  void* a_out;
  void* sigma;
  void* tangent;
  int32_t* iters;
  int32_t* status;
  const void* lam;
} dmn_point_group;

/* Version string of the library. */
const char* dmn_version(void);

/* Workspace bytes for dmn_homogenize_linear (0 for an invalid net, B or prec). */
size_t dmn_homogenize_linear_workspace_size(const dmn_net* net, int64_t B, int prec);

/* Linear DMN homogenisation DMN^L (Sec. 3.1, stiffness propagation):
 * for each of B samples, phase stiffnesses C1[b], C2[b] (6x6 Mandel,
 * row-major, [B][36]; read as their symmetric part) are homogenised bottom-up
 * through the laminate tree of `net`; the result goes to Cbar[b] ([B][36],
 * symmetric).  prec: DMN_F64 or DMN_F32 (all arrays, including w, n, the
 * orientation coefficients and lam, in that precision).  lam [B][2]: the
 * fibre orientation (l1, l2) of each sample for an orientation-interpolated
 * net (Sec. 2.3, see dmn_net), NULL for fixed normals.  Dead subtrees (all
 * leaf weights zero) are removed from the tree (Sec. 3.1 compression): a
 * laminate with one dead child returns its other child's stiffness.  An
 * invalid DMN (a negative or non-finite weight, or no weight at all) or a
 * non-SPD laminate pivot sets the
 * device error word at the start of the workspace (int32, 0 = fine; read it
 * after the stream has finished) and leaves NaN in the affected outputs. */
int dmn_homogenize_linear(const dmn_net* net, int64_t B, int prec, const void* C1,
                          const void* C2, const void* lam, void* Cbar, void* ws,
                          size_t ws_bytes, hipStream_t stream);

/* Workspace bytes for dmn_homogenize_backward (0 for an invalid net, B or prec). */
size_t dmn_homogenize_backward_workspace_size(const dmn_net* net, int64_t B, int prec);

/* Vector-Jacobian product of dmn_homogenize_linear: given the cotangent
 * gCbar[B][36] of Cbar, writes (overwrites)
 *   gw [2^K]     sum over samples of d<gCbar, Cbar>/d w
 *   gn [L][3]    sum over samples of d<gCbar, Cbar>/d n (n as passed; the
 *                map is invariant to the length of n, so gn is tangential);
 *                for an orientation-interpolated net gn is [L][2][M]: row i
 *                holds d/d ori_p[i] (M values) then d/d ori_q[i], each summed
 *                over the samples with their own orientation lam
 *   gC1, gC2 [B][36]  per-sample d<gCbar, Cbar>/d C1, C2 (symmetric), or NULL
 * With dead subtrees (see dmn_net) the laminates inside them and those with
 * a dead child get gn = 0, leaves inside them get nothing from their dead
 * laminates, and a zero-weight leaf next to a live sibling gets the one-sided
 * derivative d/dw at w = 0; entries of leaves inside a dead subtree are
 * finite but are not derivatives (training zeroes them through the Macaulay
 * bracket, see dmn_training_update).
 * The batch sums use a fixed reduction order (bit-reproducible run to run).
 * The forward is recomputed inside the call.  Same error word as the forward. */
int dmn_homogenize_backward(const dmn_net* net, int64_t B, int prec, const void* C1,
                            const void* C2, const void* lam, const void* gCbar, void* gw,
                            void* gn, void* gC1, void* gC2, void* ws, size_t ws_bytes,
                            hipStream_t stream);

/* Workspace bytes for dmn_update_gauss_points. */
size_t dmn_update_gauss_points_workspace_size(const dmn_point_group* groups, int32_t n_groups,
                                              int prec);

/* Online evaluation of DMNs at Gauss points (Sec. 3.2, Sec. 4.6): for every
 * point of every group, solve the DMN's Euler-Lagrange equation
 * A^T W sigma(E + A a, z_in) = 0 for the jumps a by Newton's method from
 * a_in, with the J2 return mapping at matrix leaves and linear elasticity at
 * fibre leaves; return the effective stress, the algorithmic tangent, the
 * updated internal variables and the converged jumps.  Groups may have
 * different depths and normal interpolations.  prec: DMN_F64, or
 * DMN_F32_STATE for per-point arrays (E, z, a, sigma, tangent) stored in
 * FP32: the call widens the inputs into FP64 copies in the workspace, runs
 * the FP64 update on them and rounds the results to nearest into the FP32
 * outputs (the DMN parameters, orientations and options stay FP64).  At most
 * 64 groups per call.  Launches: fixed-normal groups of depths 2-9 that differ
 * in depth, or include depth 9, share one persistent launch (up to 16 groups
 * each; a depth-9 point is split over the two wavefronts of a workgroup, the
 * other depths take batches with lane subtrees of depth 2 whatever the tuning
 * table's lane split, its wave count applies); otherwise groups of one depth
 * share a launch with the tuned lane split.  Groups with
 * orientation-interpolated normals, and depth-1 groups, run in launches of
 * their own; orientation-interpolated groups use the default lane split of
 * their depth whatever the tuning table says.  A non-finite (l1, l2) gives
 * DMN_STATUS_NONFINITE. */
int dmn_update_gauss_points(const dmn_point_group* groups, int32_t n_groups,
                            const dmn_elastic* fiber, const dmn_j2* matrix, int prec,
                            const dmn_newton_opts* opts, void* ws, size_t ws_bytes,
                            hipStream_t stream);

/* Size of the per-device array that dmn_update_gauss_points_noalloc uses as
 * its workspace (1 MiB: up to 16 groups of depth 9, 32 of depth 8). */
#define DMN_NOALLOC_SCRATCH_BYTES ((size_t)1 << 20)

/* dmn_update_gauss_points for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation and results, with the workspace taken
 * from a static device array of DMN_NOALLOC_SCRATCH_BYTES instead of an
 * argument.  The caller still passes every input and output array.  Calls
 * no hipMalloc, hipFree or other allocating routine; the array's device
 * address is looked up once per device, on the first call with that device
 * current, and the array is held until the process ends.  Returns
 * DMN_EWORKSPACE when the call needs more than DMN_NOALLOC_SCRATCH_BYTES
 * (dmn_update_gauss_points_workspace_size), DMN_EHIP when the address
 * lookup fails, DMN_EUNSUPPORTED for DMN_F32_STATE (its FP64 copies of the
 * per-point arrays do not fit), otherwise the codes of dmn_update_gauss_points.  Every call
 * on one device shares that device's array (it keeps the last call's tables;
 * the work counters are cleared by a kernel at the start of each call), so
 * calls that overlap on one device, on different streams or from different
 * threads, race: the caller orders them. */
int dmn_update_gauss_points_noalloc(const dmn_point_group* groups, int32_t n_groups,
                                    const dmn_elastic* fiber, const dmn_j2* matrix, int prec,
                                    const dmn_newton_opts* opts, hipStream_t stream);

/* Launch tuning of dmn_update_gauss_points for one DMN depth.  The kernels
 * split a point's laminate tree across lanes_per_point lanes of a 64-lane
 * wavefront (each lane owns a subtree of depth K - log2(lanes_per_point), the
 * levels above are combined across lanes), so 64 / lanes_per_point points
 * share a wavefront; waves_per_cu persistent wavefronts per compute unit take
 * batches of points from a work counter.  Depth 9 has one variant, 128 lanes
 * (a point over the two wavefronts of a workgroup).  In a launch shared by
 * several depths (see dmn_update_gauss_points) only waves_per_cu counts, the
 * largest of the depths present.  Tuning changes speed only: every variant
 * computes the same per-point result. */
typedef struct dmn_gp_tuning {
  int32_t lanes_per_point; /* a value listed by dmn_gp_lane_variants; 0 = default */
  int32_t waves_per_cu;    /* 1..64; 0 = default (8) */
} dmn_gp_tuning;

/* Set the process-wide tuning for depth (NULL restores the defaults).  Calls
 * read the table once when they start, so it may be changed from any thread;
 * it affects calls made afterwards.  DMN_EINVAL for a depth outside [1,10] or
 * a negative / too large value, DMN_EUNSUPPORTED if no kernel variant with
 * that lane count is compiled for the depth. */
int dmn_gp_set_tuning(int32_t depth, const dmn_gp_tuning* t);

/* The tuning in effect for depth (defaults resolved).  DMN_EINVAL for a depth
 * outside [1,10] or t == NULL. */
int dmn_gp_get_tuning(int32_t depth, dmn_gp_tuning* t);

/* Lane counts per point of the kernel variants compiled for depth: writes up
 * to cap of them to lanes (host memory) and returns how many exist (0 for a
 * depth outside [1,10]). */
int32_t dmn_gp_lane_variants(int32_t depth, int32_t* lanes, int32_t cap);

/* One batch of points for the load-step adjoint.  With M = 2^(K-1), L = 2^K - 1
 * (FP64, point-major, device memory):
 *   E        [P][6]     macro strain of the step
 *   z_in     [P][M][7]  internal variables entering the step (z^n)
 *   a_conv   [P][L][3]  converged jumps of the step (a^{n+1}, as returned by
 *                       dmn_update_gauss_points from the same inputs)
 *   g_sigma  [P][6]     cotangent of the step's effective stress, or NULL (zero)
 *   g_z_next [P][M][7]  cotangent of the step's new internal variables z^{n+1},
 *                       or NULL (zero)
 *   g_z_prev [P][M][7]  out: cotangent of z_in
 *   gw [2^K], gn [L][3] accumulated (+=): cotangents of the DMN's leaf weights
 *                       and normals (n as passed), summed over the points */
typedef struct dmn_adjoint_group {
  dmn_net net;
  int64_t P;
  const void* E;
  const void* z_in;
  const void* a_conv;
  const void* g_sigma;
  const void* g_z_next;
  void* g_z_prev;
  void* gw;
  void* gn;
} dmn_adjoint_group;

/* Workspace bytes for dmn_update_adjoint. */
size_t dmn_update_adjoint_workspace_size(const dmn_adjoint_group* groups, int32_t n_groups,
                                         int prec);

/* Reverse-mode sensitivity of one Newton-converged load step (implicit-function
 * adjoint of the Euler-Lagrange equation of Sec. 3.2): given the cotangents of
 * the step's outputs (effective stress, new internal variables), accumulate the
 * cotangents of the DMN parameters and return the cotangent of the internal
 * variables entering the step.  Chaining calls backwards over the steps of a
 * load path (with the states of the forward path, e.g. recomputed from
 * checkpoints) gives the gradient of any function of the path's stresses.
 * The leaf laws are re-evaluated at (E, z_in, a_conv); a_conv must be the
 * converged jumps for those inputs.  Batch sums use a fixed reduction order.
 * prec: DMN_F64.  An invalid DMN, a non-SPD pivot or a failed J2 return set
 * bits 1, 2, 4 of the device error word at the start of the workspace. */
int dmn_update_adjoint(const dmn_adjoint_group* groups, int32_t n_groups,
                       const dmn_elastic* fiber, const dmn_j2* matrix, int prec, void* ws,
                       size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Offline training of a DMN with fixed normals (Sec. 3.1 objective and
 * parameterisation, Sec. 4.4 stiffness sampling, Sec. 4.5 optimiser).  One
 * training step is dmn_homogenize_linear -> dmn_training_loss ->
 * dmn_homogenize_backward -> dmn_training_update; every call only enqueues
 * kernels, so the step can be captured into a HIP graph.
 * ------------------------------------------------------------------------- */

/* Exponents of the objective (Sec. 3.1): the error of sample s is
 *   e_s = ||V(target_s - Cbar_s)||_p / ||V target_s||_p,
 * the l^p norm over the 36 Voigt components V of the 6x6 stiffness (Voigt
 * components are the Mandel entries divided by s_I s_J with
 * s = (1, 1, 1, sqrt 2, sqrt 2, sqrt 2)); the batch of B samples contributes
 * the data term (1/B) (sum_s e_s^q)^(1/q).  The paper trains with p = 1 and
 * q = 10.  Requires 1 <= p, q (finite). */
typedef struct dmn_loss_opts {
  double p;
  double q;
} dmn_loss_opts;

/* The training calls share a device block of DMN_TRAIN_STATS doubles:
 *   [0] data term   [1] max_s e_s   [2] sum_s (e_s / max e)^q
 *   [3] objective = data term + penalty      [4] penalty
 *   [5] learning rate of the update          [6] sum_i <v_i>_+ before it
 *   [7] unused
 * dmn_training_loss writes [0..2], dmn_training_update writes [3..6]. */
#define DMN_TRAIN_STATS 8

/* Workspace bytes for dmn_training_loss (3 B doubles and a header). */
size_t dmn_training_loss_workspace_size(int64_t B);

/* Data term of the objective and its cotangent.  Cbar, target [B][36] are
 * Mandel stiffnesses (target: the reference effective stiffness of each
 * sample, nonzero); writes stats[0..2], the per-sample errors e [B] (NULL:
 * not stored) and gCbar [B][36] = d(data term)/d Cbar entry by entry (the
 * cotangent dmn_homogenize_backward takes).  Derivatives of |x| at 0 are
 * taken as 0; a batch with no error gets a zero cotangent.  prec: DMN_F64 or
 * DMN_F32 for Cbar, target, e, gCbar (sums in FP64); stats is FP64.  Batch
 * sums use a fixed order.  B = 0 writes zeros to stats[0..2]. */
int dmn_training_loss(int64_t B, int prec, const void* Cbar, const void* target,
                      const dmn_loss_opts* opts, void* e, void* gCbar, double* stats, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* Optimiser of Sec. 4.5: AMSGrad (Adam with the running maximum of the
 * second moment; Adam's bias corrections on the first moment and on that
 * maximum) with the learning rate of epoch m
 *   lr_decay^m (lr_min + (lr_max - lr_min) (1 + cos(pi m / half_period)) / 2),
 * m = (updates taken so far) / steps_per_epoch (integer division).  The
 * paper's values: lr_min = 1.5e-3, lr_max = 1.5e-2, lr_decay = 0.999,
 * half_period = 50, penalty (lambda of the mixing penalty
 * lambda (sum_i <v_i>_+ - 1)^2, Sec. 3.1) = 1e3; beta1 = 0.9,
 * beta2 = 0.999, eps = 1e-8 are Adam's customary values (the paper gives
 * none).  Requires 0 <= lr_min, lr_max; 0 < lr_decay; half_period,
 * steps_per_epoch >= 1; 0 <= beta1, beta2 < 1; eps > 0; penalty >= 0. */
typedef struct dmn_amsgrad_opts {
  double lr_min;
  double lr_max;
  double lr_decay;
  int32_t half_period;
  int32_t steps_per_epoch;
  double beta1;
  double beta2;
  double eps;
  double penalty;
} dmn_amsgrad_opts;

/* Trainable parameters of a depth-K DMN with fixed normals (Sec. 3.1):
 * unconstrained weights v [2^K] with leaf weights w = <v>_+ (Macaulay
 * bracket) and normal angles alpha, beta [L] with
 * n = (sin alpha cos beta, sin alpha sin beta, cos alpha) (Sec. 2.3).
 * All arrays are device memory in the precision of the call. */
typedef struct dmn_train_params {
  int32_t depth;
  void* v;         /* [2^K], updated in place */
  void* alpha;     /* [L], updated in place */
  void* beta;      /* [L], updated in place */
  void* w;         /* [2^K] out: <v>_+ of the current v */
  void* n;         /* [L][3] out: n(alpha, beta) of the current angles */
  void* state;     /* [3][2^K + 2L]: first moments, second moments, their
                      running maxima, for the slots v, alpha, beta in that
                      order; zero before the first update */
  int64_t* step;   /* device counter of updates taken (0 before the first) */
} dmn_train_params;

/* One optimiser step: with gw [2^K], gn [L][3] from dmn_homogenize_backward
 * of the current (w, n) and the cotangent of dmn_training_loss, the
 * gradients of the objective are
 *   dJ/dv_i = (gw_i + 2 lambda (sum_j <v_j>_+ - 1)) [v_i > 0],
 *   dJ/dalpha_l = gn_l . dn_l/dalpha_l,  dJ/dbeta_l = gn_l . dn_l/dbeta_l;
 * the call applies AMSGrad to v, alpha, beta, advances *step, writes
 * stats[3..6] (the objective of the parameters before the step) and
 * refreshes w, n for the next forward.  prec: DMN_F64 or DMN_F32 for every
 * array of params, gw and gn (arithmetic in FP64). */
int dmn_training_update(const dmn_train_params* params, int prec, const void* gw, const void* gn,
                        const dmn_amsgrad_opts* opts, double* stats, hipStream_t stream);

/* Writes w = <v>_+ and n(alpha, beta) of params without a step (the inputs of
 * the first forward). */
int dmn_training_refresh(const dmn_train_params* params, int prec, hipStream_t stream);

/* Training over a discrete set of G fibre orientations (Sec. 2.3, the
 * paper's identification of an orientation-interpolated DMN, Sec. 4.5):
 * samples of orientation k see the normals n_k, so a step evaluates the
 * fixed-normal linear map and its VJP for every orientation group with n_k
 * from dmn_orientation_group_normals (all groups at once with
 * dmn_homogenize_linear_groups / dmn_homogenize_backward_groups, or one
 * dmn_homogenize_linear / dmn_homogenize_backward call per group), takes the
 * objective over the whole batch with dmn_training_loss, chains the groups'
 * gw, gn to the angle coefficients with dmn_orientation_group_chain and
 * updates (v, p, q) with dmn_training_update_oriented. */

/* Workspace bytes for dmn_homogenize_linear_groups (0 for an invalid depth,
 * G or prec). */
size_t dmn_homogenize_linear_groups_workspace_size(int32_t depth, int32_t G, int prec);

/* The linear map (Sec. 3.1) of G DMNs of one depth that share the leaf
 * weights w [2^K] and differ in their normals n_groups [G][L][3] (paper
 * order; one DMN per orientation of a discrete set, Sec. 2.3), over one batch
 * whose samples offsets[k] .. offsets[k+1]-1 belong to group k.  offsets:
 * host array of G+1 int64 with offsets[0] = 0, non-decreasing (empty groups
 * allowed), offsets[G] = B, read during the call.  C1, C2, Cbar [B][36] as
 * for dmn_homogenize_linear, whose results (also for dead subtrees) the call
 * reproduces group by group: it prepares the G tables in one launch and
 * evaluates up to 64 groups per forward launch.  Invalid offsets or G < 1
 * return DMN_EINVAL.  Same device error word as dmn_homogenize_linear (set
 * when any group fails). */
int dmn_homogenize_linear_groups(int32_t depth, int32_t G, const int64_t* offsets, int prec,
                                 const void* w, const void* n_groups, const void* C1,
                                 const void* C2, void* Cbar, void* ws, size_t ws_bytes,
                                 hipStream_t stream);

/* Workspace bytes for dmn_homogenize_backward_groups (0 for an invalid depth,
 * G, offsets or prec). */
size_t dmn_homogenize_backward_groups_workspace_size(int32_t depth, int32_t G,
                                                     const int64_t* offsets, int prec);

/* VJP of dmn_homogenize_linear_groups: given gCbar [B][36], writes
 * (overwrites) gw_groups [G][2^K] and gn_groups [G][L][3], group k's rows
 * being what dmn_homogenize_backward returns for the samples of group k at
 * normals n_groups[k] (zero for an empty group), bit-identical to it (the
 * same waves per group and the same fixed reduction order) when both launches
 * run the same kernel.  At depths 7 and 8 the linear map takes two samples
 * per wave once a launch holds more than 8 samples per CU (the VJP does so in
 * plain calls only); where the grouped launch and the plain call fall on
 * different sides of that size, the two agree within rounding.  No phase
 * stiffness cotangents.  The forward is recomputed inside the call.  Same
 * error word as the forward. */
int dmn_homogenize_backward_groups(int32_t depth, int32_t G, const int64_t* offsets, int prec,
                                   const void* w, const void* n_groups, const void* C1,
                                   const void* C2, const void* gCbar, void* gw_groups,
                                   void* gn_groups, void* ws, size_t ws_bytes,
                                   hipStream_t stream);

/* n [G][L][3]: for orientation lam[k] = (l1, l2) (lam [G][2]) and angle
 * coefficients p, q [L][M] (M from ori_shape, see dmn_net), laminate l gets
 * alpha = p_l . s(lam_k), beta = q_l . s(lam_k) and
 * n = (sin alpha cos beta, sin alpha sin beta, cos alpha).  prec DMN_F64 or
 * DMN_F32 for every array. */
int dmn_orientation_group_normals(int32_t depth, int32_t ori_shape, int32_t G, int prec,
                                  const void* p, const void* q, const void* lam, void* n,
                                  hipStream_t stream);

/* From the groups' VJPs gw_groups [G][2^K] and gn_groups [G][L][3] (of
 * dmn_homogenize_backward at n_k): gw [2^K] = sum_k gw_groups[k] and
 * gpq [L][2][M]: row l holds d/dp_l (M values) then d/dq_l, through
 * n_k(p, q) and the shape functions at lam_k.  Sums over k in order. */
int dmn_orientation_group_chain(int32_t depth, int32_t ori_shape, int32_t G, int prec,
                                const void* p, const void* q, const void* lam,
                                const void* gw_groups, const void* gn_groups, void* gw,
                                void* gpq, hipStream_t stream);

/* Trainable parameters of an orientation-interpolated DMN: unconstrained
 * weights v [2^K] (w = <v>_+), angle coefficients p, q [L][M]. */
typedef struct dmn_train_params_oriented {
  int32_t depth;
  int32_t ori_shape; /* DMN_ORI_LINEAR, _TRILINEAR or _QUADRATIC */
  void* v;           /* [2^K], updated in place */
  void* p;           /* [L][M], updated in place */
  void* q;           /* [L][M], updated in place */
  void* w;           /* [2^K] out: <v>_+ of the current v */
  void* state;       /* [3][2^K + 2 L M]: first moments, second moments, their
                        running maxima, for the slots v, p, q in that order;
                        zero before the first update */
  int64_t* step;     /* device counter of updates taken */
} dmn_train_params_oriented;

/* One optimiser step as dmn_training_update, with the coefficient gradients
 * gpq [L][2][M] of dmn_orientation_group_chain in place of the angle chain;
 * writes stats[3..6] and refreshes w. */
int dmn_training_update_oriented(const dmn_train_params_oriented* params, int prec,
                                 const void* gw, const void* gpq, const dmn_amsgrad_opts* opts,
                                 double* stats, hipStream_t stream);

/* w = <v>_+ of params without a step. */
int dmn_training_refresh_oriented(const dmn_train_params_oriented* params, int prec,
                                  hipStream_t stream);

/* Stiffness sampler of Sec. 4.4: for each of B points u [B][8] (FP64) of
 * the unit cube, the eight parameters (a, e1, e2, e3, beta, theta, psi, phi)
 * are a = u0, e_i = -3 + 6 u_i, beta = 2 pi u4, theta in [0, pi] with
 * theta - sin(theta) = pi u5, psi = pi u6, phi = 2 pi u7, and
 *   C1 = 3 K1 P1 + 2 G1 P2,  C2 = 3 K2 P1 + 2 G2 (P2 - a N' (x) N'),
 * with K1 = 1, G1 = 10^e1, K2 = 10^e2, G2 = 10^e3 (GPa), P1, P2 the
 * spherical and deviatoric projectors, N' = Q N Q^T for the trace-free unit
 * diagonal N(beta) and Q the rotation by theta about the axis
 * (sin psi cos phi, sin psi sin phi, cos psi).  C1, C2 [B][36] Mandel in
 * prec (DMN_F64 or DMN_F32). */
int dmn_sample_stiffness(int64_t B, int prec, const double* u, void* C1, void* C2,
                         hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DMN_H */
