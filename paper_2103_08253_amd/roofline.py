"""Algorithmic work and traffic of the DMN kernels (for roofline reporting).

Flops are counted from the formulas the kernels evaluate (each multiply, add,
divide, square root and exponential counts as one flop; a fused multiply-add
counts as two).  Work the kernels skip is never credited, and work whose
amount varies per leaf is counted at its smallest value:

* a J2 leaf is counted at the cost of its elastic branch (trial state,
  yield check, stress and tangent assembly), i.e. the scalar Newton
  iterations of plastic leaves are not credited;
* a Gauss-point update is counted with iters + 1 evaluations (one per
  accepted Newton step plus the initial one); backtracking trials are not
  credited.

Bytes are the compulsory HBM traffic of one call: every per-point input read
once and every per-point output written once; the DMN tables (a few KB per
DMN) are excluded.
"""
from dataclasses import dataclass

# ---- per-item flop counts (see the kernels' formulas) ----------------------
# 3x3 inverse by cofactors: six cofactors (18), determinant (5), reciprocal (1),
# scaling (6)
INVERSE3 = 30
# laminate step of the Newton bottom-up: S and C_R - C_L (84), S N and U (216),
# K = N^T S N (54), 3x3 inverse, V = U K^-1 (90), condensed C (211), g and tau
# (99), plain average and residual block (50)
LAMINATE_NEWTON = 804 + INVERSE3
# top-down step: da = -(g + G e) (39), N da (15), children strains (24)
LAMINATE_DESCEND = 78
# strain localisation through a laminate from stored jumps: N a (15) + 24
LAMINATE_LOCALIZE = 39
# J2 leaf, elastic branch: trial strain and deviator (18), norm (12), yield stress
# and check (10), stress (13), normal and state (21), packed tangent (71)
J2_LEAF = 145
# fibre leaf: isotropic stress
FIBER_LEAF = 15
# linear laminate (forward of the training map): S, dC (84), S N and U (216),
# K (54), inverse, V (90), C (211)
LAMINATE_LINEAR = 655 + INVERSE3
# laminate VJP: recompute (forward - 211 + 63 for T), X = Gt V (126), G_K (36),
# N G_K and G_S (108 + 108), Y (90), G_CL / G_CR / inner products (378),
# G_N (324), g_n (18)
LAMINATE_LINEAR_VJP = (LAMINATE_LINEAR - 211 + 63) + 126 + 36 + 216 + 90 + 378 + 324 + 18

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector peak
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector peak
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E


@dataclass
class DmnSizes:
    depth: int

    @property
    def L(self):
        return 2 ** self.depth - 1

    @property
    def M(self):
        return 2 ** (self.depth - 1)


def gp_update_flops(depth: int, iters: int) -> int:
    """Algorithmic flops of one Gauss-point update that took `iters` Newton steps:
    per evaluation the localisation eps = E + A a, the leaf laws and the
    bottom-up condensation; per Newton step the top-down solve."""
    s = DmnSizes(depth)
    per_eval = (s.L * (LAMINATE_NEWTON + LAMINATE_LOCALIZE)
                + s.M * (J2_LEAF + FIBER_LEAF))
    return (iters + 1) * per_eval + iters * s.L * LAMINATE_DESCEND


def live_tree_counts(w) -> tuple:
    """(laminates, matrix leaves, fibre leaves) that tree compression (Sec. 3.1)
    keeps for leaf weights w [2^K]: a leaf stays when its weight is positive,
    a laminate when both of its subtrees carry weight (one with a dead child
    passes the other through).  Leaves alternate fibre (even index) and
    matrix (odd)."""
    n = len(w)
    W = [0.0] * (2 * n)  # heap order: node h has children 2h, 2h + 1; leaf j is n + j
    for j in range(n):
        W[n + j] = float(w[j]) if w[j] > 0 else 0.0
    for h in range(n - 1, 0, -1):
        W[h] = W[2 * h] + W[2 * h + 1]
    lams = sum(1 for h in range(1, n) if W[2 * h] > 0 and W[2 * h + 1] > 0)
    mat = sum(1 for j in range(1, n, 2) if W[n + j] > 0)
    fib = sum(1 for j in range(0, n, 2) if W[n + j] > 0)
    return lams, mat, fib


def gp_update_flops_live(laminates: int, matrix_leaves: int, fibre_leaves: int,
                         iters: int) -> int:
    """gp_update_flops credited for the live part of a compressed tree only
    (the kernel evaluates dead rows in place; that work is not credited)."""
    per_eval = (laminates * (LAMINATE_NEWTON + LAMINATE_LOCALIZE)
                + matrix_leaves * J2_LEAF + fibre_leaves * FIBER_LEAF)
    return (iters + 1) * per_eval + iters * laminates * LAMINATE_DESCEND


def gp_update_bytes(depth: int, elt: int = 8) -> int:
    """Compulsory HBM bytes of one update: E, z_in, a_in read; z_out, a_out, sigma,
    tangent written (elt bytes each), plus the 4-byte iteration count and status."""
    s = DmnSizes(depth)
    return elt * (6 + 7 * s.M + 3 * s.L + 7 * s.M + 3 * s.L + 6 + 36) + 8


def linear_forward_flops(depth: int) -> int:
    return DmnSizes(depth).L * LAMINATE_LINEAR


def linear_backward_flops(depth: int) -> int:
    """Backward recomputes the forward, then one VJP per laminate."""
    s = DmnSizes(depth)
    return s.L * (LAMINATE_LINEAR + LAMINATE_LINEAR_VJP)


def linear_sample_bytes(elt: int = 8, backward: bool = False) -> int:
    """Forward: C1, C2 read and Cbar written; backward: C1, C2, gCbar read."""
    return elt * 36 * 3
