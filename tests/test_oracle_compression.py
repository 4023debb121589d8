"""Pins of the oracle's tree compression (Sec. 3.1): without zero weights it
is the full tree; with zero weights it is the limit of the uncompressed DMN
as those weights go to zero; a dead half reduces a depth-2 DMN to its live
laminate; a single live leaf returns its phase."""
import numpy as np

import synthetic as S
from oracle.compression import compressed_tree, dmn_linear_compressed
from oracle.linear import dmn_linear, laminate_milton
from oracle.tree import lam_pos


def case(K, B=3, seed=61):
    rs = S.streams(seed)
    net = S.random_dmn(rs["dmn"], K, 0.3)
    return net, S.random_spd(rs["stiffness"], B), S.random_spd(rs["stiffness"], B)


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_positive_weights_keep_the_full_tree():
    for K in (1, 3, 5):
        net, C1, C2 = case(K)
        tree = compressed_tree(K, net.w)
        count = lambda n: 0 if n[0] == "leaf" else 1 + count(n[2]) + count(n[3])
        assert count(tree) == 2 ** K - 1
        assert rel(dmn_linear_compressed(K, net.w, net.normals, C1, C2),
                   dmn_linear(K, net.w, net.normals, C1, C2)) < 1e-11  # rounding of the fractions


def test_compression_is_the_zero_weight_limit():
    """Leaves 3 (alone: its sibling 2 stays), 8-11 (a whole depth-2 subtree)
    and 14 go to zero; the uncompressed DMN with weights eps there approaches
    the compressed one linearly in eps."""
    K = 4
    net, C1, C2 = case(K)
    dead = [3, 8, 9, 10, 11, 14]
    w0 = net.w.copy()
    w0[dead] = 0.0
    Cc = dmn_linear_compressed(K, w0, net.normals, C1, C2)
    errs = []
    for eps in (1e-6, 1e-8):
        we = w0.copy()
        we[dead] = eps
        errs.append(rel(dmn_linear(K, we, net.normals, C1, C2), Cc))
    assert errs[1] < 1e-6 and errs[1] < 0.05 * errs[0]


def test_dead_half_reduces_to_the_live_laminate():
    K = 2
    net, C1, C2 = case(K)
    w = net.w.copy()
    w[2:] = 0.0
    p = lam_pos(K, 2, 1)    # laminate over leaves 0, 1
    ref = laminate_milton(C1, C2, w[0] / (w[0] + w[1]), w[1] / (w[0] + w[1]), net.normals[p])
    assert rel(dmn_linear_compressed(K, w, net.normals, C1, C2), ref) < 1e-14


def test_single_live_leaf_returns_its_phase():
    K = 3
    net, C1, C2 = case(K)
    for j in (0, 5):
        w = np.zeros(2 ** K)
        w[j] = 0.7
        ref = C1 if j % 2 == 0 else C2
        assert np.array_equal(dmn_linear_compressed(K, w, net.normals, C1, C2), ref)
    assert compressed_tree(K, np.zeros(2 ** K)) is None
