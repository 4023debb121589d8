"""Tree compression of a direct DMN (Sec. 3.1).  Test infrastructure like the
rest of the oracle.

During training some leaf weights reach zero and stay there; the paper then
removes such subtrees from the binary tree: a leaf without weight is deleted,
a laminate left with a single child is replaced by that child, and a subtree
without any weight disappears.  The linear map of the compressed tree is
evaluated here with the same laminate formula (Milton's, Sec. 3.1) over the
laminates that remain, with volume fractions from the remaining weights.
"""
import numpy as np

from .linear import laminate_milton
from .tree import lam_pos


def compressed_tree(K, w):
    """The compressed tree as nested tuples: ("leaf", j) or
    ("laminate", pos, left, right), with pos the laminate's paper position;
    None when no leaf carries weight.  A weight counts as zero when its real
    part is zero (complex steps keep the structure)."""
    def build(k, i):
        # subtree of laminate (k, i); its children are (k+1, 2i-1), (k+1, 2i),
        # or leaves 2i-2, 2i-1 at level K
        if k > K:
            j = i - 1
            return ("leaf", j) if np.real(w[j]) != 0 else None
        left, right = build(k + 1, 2 * i - 1), build(k + 1, 2 * i)
        if left is None:
            return right
        if right is None:
            return left
        return ("laminate", lam_pos(K, k, i), left, right)
    return build(1, 1)


def subtree_weight(node, w):
    if node[0] == "leaf":
        return w[node[1]]
    return subtree_weight(node[2], w) + subtree_weight(node[3], w)


def dmn_linear_compressed(K, w, normals, C1, C2, alpha=None):
    """DMN^L of the compressed tree: leaves carry C1 (even index) or C2 (odd
    index); every remaining laminate mixes its children with fractions
    W_left / (W_left + W_right) of the remaining weights.  Complex-safe."""
    root = compressed_tree(K, w)
    if root is None:
        raise ValueError("no leaf carries weight")

    def evaluate(node):
        if node[0] == "leaf":
            return C1 if node[1] % 2 == 0 else C2
        _, pos, left, right = node
        WL, WR = subtree_weight(left, w), subtree_weight(right, w)
        return laminate_milton(evaluate(left), evaluate(right), WL / (WL + WR),
                               WR / (WL + WR), normals[pos], alpha)
    return evaluate(root)
