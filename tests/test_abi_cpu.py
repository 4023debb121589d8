"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/dmn.h declares, and rejects bad arguments on the host with
the documented codes before touching any device pointer."""
import ctypes
import os
import re

import pytest

from paper_2103_08253_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x100000)   # never dereferenced: validation fails first
ALIGNED = ctypes.c_void_p(0x200000)


def header_functions():
    text = open(os.path.join(ROOT, "include", "dmn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dmn_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = L.lib()
    names = header_functions()
    assert "dmn_update_gauss_points" in names and "dmn_homogenize_linear" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(L._SIGS), "binding must declare every exported function"
    assert lib.dmn_version().decode().startswith("libdmn")


def net(depth=3):
    return L.DmnNet(depth, FAKE.value, FAKE.value)


def test_linear_validation_codes():
    lib = L.lib()
    ws_need = lib.dmn_homogenize_linear_workspace_size(ctypes.byref(net(3)), 10, L.DMN_F64)
    assert ws_need > 0
    assert lib.dmn_homogenize_linear_workspace_size(ctypes.byref(net(0)), 10, L.DMN_F64) == 0
    assert lib.dmn_homogenize_linear_workspace_size(ctypes.byref(net(11)), 10, L.DMN_F64) == 0
    call = lambda n, B=10, prec=L.DMN_F64, ws=ALIGNED, nb=ws_need: lib.dmn_homogenize_linear(
        n, B, prec, FAKE, FAKE, None, FAKE, ws, nb, None)
    assert call(None) == L.DMN_EINVAL
    assert call(ctypes.byref(net(0))) == L.DMN_EINVAL
    assert call(ctypes.byref(net(11))) == L.DMN_EINVAL
    assert call(ctypes.byref(net(3)), B=-1) == L.DMN_EINVAL
    assert call(ctypes.byref(net(3)), prec=7) == L.DMN_EUNSUPPORTED
    assert call(ctypes.byref(net(3)), nb=ws_need - 1) == L.DMN_EWORKSPACE
    assert call(ctypes.byref(net(3)), ws=None) == L.DMN_EWORKSPACE
    assert call(ctypes.byref(net(3)), ws=ctypes.c_void_p(ALIGNED.value + 8)) == L.DMN_EWORKSPACE
    bad = L.DmnNet(3, None, FAKE.value)
    assert call(ctypes.byref(bad)) == L.DMN_EINVAL


def test_backward_validation_codes():
    lib = L.lib()
    need = lib.dmn_homogenize_backward_workspace_size(ctypes.byref(net(8)), 4096, L.DMN_F64)
    assert need > lib.dmn_homogenize_linear_workspace_size(ctypes.byref(net(8)), 4096, L.DMN_F64)
    n8 = net(8)
    call = lambda gw=FAKE, gc1=None, gc2=None, nb=need: lib.dmn_homogenize_backward(
        ctypes.byref(n8), 4096, L.DMN_F64, FAKE, FAKE, None, FAKE, gw, FAKE, gc1, gc2, ALIGNED, nb,
        None)
    assert call(gw=None) == L.DMN_EINVAL
    assert call(gc1=FAKE) == L.DMN_EINVAL          # gC1 without gC2
    assert call(nb=need - 1) == L.DMN_EWORKSPACE


def group(depth=2, P=4, **over):
    g = L.DmnPointGroup(net(depth), P, *([FAKE.value] * 9))
    g.z_out = 0x300000
    g.a_out = 0x400000
    for k, v in over.items():
        setattr(g, k, v)
    return g


def test_gauss_point_validation_codes():
    lib = L.lib()
    fib = L.DmnElastic(72000.0, 0.22)
    mat = L.DmnJ2(2800.0, 0.35, 50.0, 200.0, 30.0, 60.0)
    opts = L.DmnNewtonOpts(1e-10, 25, 10, 1e-4)
    arr = (L.DmnPointGroup * 2)(group(2), group(8))
    need = lib.dmn_update_gauss_points_workspace_size(arr, 2, L.DMN_F64)
    assert need > 0
    assert lib.dmn_update_gauss_points_workspace_size(arr, 2, L.DMN_F32) == 0
    # FP32 state: the FP64 workspace plus FP64 copies of every per-point array
    need32 = lib.dmn_update_gauss_points_workspace_size(arr, 2, L.DMN_F32_STATE)
    per_point = lambda K: 8 * (6 + 2 * 7 * 2 ** (K - 1) + 2 * 3 * (2 ** K - 1) + 6 + 36)
    assert need32 >= need + 4 * (per_point(2) + per_point(8))

    def call(a=arr, n=2, f=fib, m=mat, o=opts, prec=L.DMN_F64, nb=need):
        return lib.dmn_update_gauss_points(a, n, ctypes.byref(f) if f else None,
                                           ctypes.byref(m) if m else None, prec,
                                           ctypes.byref(o) if o else None, ALIGNED, nb, None)

    assert call(n=0) == L.DMN_EINVAL
    assert call(n=65) == L.DMN_EINVAL
    assert call(prec=L.DMN_F32) == L.DMN_EUNSUPPORTED
    assert call(prec=7) == L.DMN_EUNSUPPORTED
    assert call(prec=L.DMN_F32_STATE) == L.DMN_EWORKSPACE  # needs the staging space
    assert call(f=None) == L.DMN_EINVAL
    assert call(m=L.DmnJ2(2800.0, 0.5, 50.0, 200.0, 30.0, 60.0)) == L.DMN_EINVAL
    assert call(o=L.DmnNewtonOpts(0.0, 25, 10, 1e-4)) == L.DMN_EINVAL
    assert call(o=L.DmnNewtonOpts(1e-10, -1, 10, 1e-4)) == L.DMN_EINVAL
    assert call(o=L.DmnNewtonOpts(1e-10, 25, 10, 1.0)) == L.DMN_EINVAL
    assert call(o=L.DmnNewtonOpts(1e-10, 25, 10, 1e-4, -1)) == L.DMN_EINVAL
    assert call(o=L.DmnNewtonOpts(1e-10, 25, 10, 1e-4, 0, -1)) == L.DMN_EINVAL
    assert call(nb=need - 1) == L.DMN_EWORKSPACE
    alias = (L.DmnPointGroup * 1)(group(2, z_out=FAKE.value))
    assert call(a=alias, n=1) == L.DMN_EINVAL
    deep = (L.DmnPointGroup * 1)(group(11))
    assert call(a=deep, n=1) == L.DMN_EINVAL
    neg = (L.DmnPointGroup * 1)(group(2, P=-1))
    assert call(a=neg, n=1) == L.DMN_EINVAL
    nul = (L.DmnPointGroup * 1)(group(2, sigma=None))
    assert call(a=nul, n=1) == L.DMN_EINVAL


def test_noalloc_gauss_point_validation_and_size_limit():
    """The no-allocation entry point validates like dmn_update_gauss_points and
    rejects a call whose workspace would exceed its static array before any
    device call (17 groups of depth 9 need more than 1 MiB)."""
    lib = L.lib()
    fib = L.DmnElastic(72000.0, 0.22)
    mat = L.DmnJ2(2800.0, 0.35, 50.0, 200.0, 30.0, 60.0)
    opts = L.DmnNewtonOpts(1e-10, 25, 10, 1e-4)
    call = lambda arr, n, o=opts: lib.dmn_update_gauss_points_noalloc(
        arr, n, ctypes.byref(fib), ctypes.byref(mat), L.DMN_F64, ctypes.byref(o), None)
    big = (L.DmnPointGroup * 17)(*[group(9) for _ in range(17)])
    assert lib.dmn_update_gauss_points_workspace_size(big, 17, L.DMN_F64) > (1 << 20)
    assert call(big, 17) == L.DMN_EWORKSPACE
    fits = (L.DmnPointGroup * 16)(*[group(9) for _ in range(16)])
    assert lib.dmn_update_gauss_points_workspace_size(fits, 16, L.DMN_F64) <= (1 << 20)
    assert call(big, 0) == L.DMN_EINVAL
    assert call(big, 17, L.DmnNewtonOpts(0.0, 25, 10, 1e-4)) == L.DMN_EINVAL
    assert lib.dmn_update_gauss_points_noalloc(big, 1, ctypes.byref(fib), ctypes.byref(mat),
                                               L.DMN_F32_STATE, ctypes.byref(opts),
                                               None) == L.DMN_EUNSUPPORTED


def test_orientation_validation_codes():
    lib = L.lib()
    fib = L.DmnElastic(72000.0, 0.22)
    mat = L.DmnJ2(2800.0, 0.35, 50.0, 200.0, 30.0, 60.0)
    opts = L.DmnNewtonOpts(1e-10, 25, 10, 1e-4)

    def ori_group(shape, p=FAKE.value, q=FAKE.value, lam=FAKE.value, P=5):
        g = group(3, P=P)
        g.net = L.DmnNet(3, FAKE.value, None, shape, p, q)
        g.lam = lam
        return (L.DmnPointGroup * 1)(g)

    arr = ori_group(L.DMN_ORI["quadratic"])
    need = lib.dmn_update_gauss_points_workspace_size(arr, 1, L.DMN_F64)
    assert need > 0

    def call(a):
        return lib.dmn_update_gauss_points(a, 1, ctypes.byref(fib), ctypes.byref(mat), L.DMN_F64,
                                           ctypes.byref(opts), ALIGNED, need, None)

    assert call(ori_group(7)) == L.DMN_EINVAL
    assert call(ori_group(L.DMN_ORI["linear"], p=None)) == L.DMN_EINVAL
    assert call(ori_group(L.DMN_ORI["trilinear"], q=None)) == L.DMN_EINVAL
    assert call(ori_group(L.DMN_ORI["quadratic"], lam=None)) == L.DMN_EINVAL
    assert call(ori_group(L.DMN_ORI["none"])) == L.DMN_EINVAL  # fixed normals need n
    # interpolated normals run up to depth 8 (depth 9's kernel has not run)
    deep = ori_group(L.DMN_ORI["linear"])
    deep[0].net.depth = 9
    assert call(deep) == L.DMN_EUNSUPPORTED
    deep[0].net.depth = 8
    assert lib.dmn_update_gauss_points(deep, 1, ctypes.byref(fib), ctypes.byref(mat), L.DMN_F64,
                                       ctypes.byref(opts), None, 0, None) == L.DMN_EWORKSPACE
    # linear calls: per-sample orientation needs lam; the backward needs space for
    # the per-sample angle cotangents
    onet = L.DmnNet(3, FAKE.value, None, L.DMN_ORI["linear"], FAKE.value, FAKE.value)
    fnet = net(3)
    nb = lib.dmn_homogenize_linear_workspace_size(ctypes.byref(onet), 4, L.DMN_F64)
    assert nb == lib.dmn_homogenize_linear_workspace_size(ctypes.byref(fnet), 4, L.DMN_F64)
    assert lib.dmn_homogenize_linear(ctypes.byref(onet), 4, L.DMN_F64, FAKE, FAKE, None, FAKE,
                                     ALIGNED, nb, None) == L.DMN_EINVAL
    # per-sample orientation in the linear calls: valid up to depth 8 (the call
    # goes on to the workspace check), deeper nets are not compiled for it
    assert lib.dmn_homogenize_linear(ctypes.byref(onet), 4, L.DMN_F64, FAKE, FAKE, FAKE, FAKE,
                                     ALIGNED, nb - 1, None) == L.DMN_EWORKSPACE
    nbo = lib.dmn_homogenize_backward_workspace_size(ctypes.byref(onet), 4096, L.DMN_F64)
    nbf = lib.dmn_homogenize_backward_workspace_size(ctypes.byref(fnet), 4096, L.DMN_F64)
    assert nbo - nbf >= 7 * 2 * 4096 * 8
    assert lib.dmn_homogenize_backward(ctypes.byref(onet), 4096, L.DMN_F64, FAKE, FAKE, FAKE,
                                       FAKE, FAKE, FAKE, None, None, ALIGNED, nbo - 1,
                                       None) == L.DMN_EWORKSPACE
    onet9 = L.DmnNet(9, FAKE.value, None, L.DMN_ORI["linear"], FAKE.value, FAKE.value)
    nb9 = lib.dmn_homogenize_backward_workspace_size(ctypes.byref(onet9), 4, L.DMN_F64)
    assert lib.dmn_homogenize_linear(ctypes.byref(onet9), 4, L.DMN_F64, FAKE, FAKE, FAKE, FAKE,
                                     ALIGNED, nb9, None) == L.DMN_EUNSUPPORTED
    assert lib.dmn_homogenize_backward(ctypes.byref(onet9), 4, L.DMN_F64, FAKE, FAKE, FAKE,
                                       FAKE, FAKE, FAKE, None, None, ALIGNED, nb9,
                                       None) == L.DMN_EUNSUPPORTED
    bad = L.DmnNet(3, FAKE.value, None, 9, FAKE.value, FAKE.value)
    assert lib.dmn_homogenize_linear_workspace_size(ctypes.byref(bad), 4, L.DMN_F64) == 0
    # the adjoint takes fixed normals only
    ag = L.DmnAdjointGroup(onet, 4, *([FAKE.value] * 8))
    arr_a = (L.DmnAdjointGroup * 1)(ag)
    nba = lib.dmn_update_adjoint_workspace_size(arr_a, 1, L.DMN_F64)
    assert lib.dmn_update_adjoint(arr_a, 1, ctypes.byref(fib), ctypes.byref(mat), L.DMN_F64,
                                  ALIGNED, max(nba, 1 << 20), None) == L.DMN_EUNSUPPORTED


def test_training_validation_codes():
    lib = L.lib()
    assert lib.dmn_training_loss_workspace_size(-1) == 0
    need = lib.dmn_training_loss_workspace_size(100)
    assert need >= 3 * 100 * 8
    good = L.DmnLossOpts(1.0, 10.0)
    call = lambda B=100, prec=L.DMN_F64, o=good, C=FAKE, g=FAKE, st=FAKE, ws=ALIGNED, nb=need: \
        lib.dmn_training_loss(B, prec, C, FAKE, ctypes.byref(o) if o is not None else None,
                              None, g, st, ws, nb, None)
    assert call(B=-1) == L.DMN_EINVAL
    assert call(prec=L.DMN_F32_STATE) == L.DMN_EUNSUPPORTED
    assert call(o=None) == L.DMN_EINVAL
    assert call(o=L.DmnLossOpts(0.5, 10.0)) == L.DMN_EINVAL
    assert call(o=L.DmnLossOpts(1.0, 0.0)) == L.DMN_EINVAL
    assert call(o=L.DmnLossOpts(float("nan"), 2.0)) == L.DMN_EINVAL
    assert call(C=None) == L.DMN_EINVAL
    assert call(g=None) == L.DMN_EINVAL
    assert call(st=None) == L.DMN_EINVAL
    assert call(nb=need - 1) == L.DMN_EWORKSPACE
    assert call(ws=ctypes.c_void_p(ALIGNED.value + 8)) == L.DMN_EWORKSPACE

    params = L.DmnTrainParams(3, *([FAKE.value] * 7))
    opts = L.DmnAmsgradOpts(1.5e-3, 1.5e-2, 0.999, 50, 1, 0.9, 0.999, 1e-8, 1e3)
    upd = lambda pr=params, o=opts, prec=L.DMN_F64, gw=FAKE: lib.dmn_training_update(
        ctypes.byref(pr) if pr is not None else None, prec, gw, FAKE,
        ctypes.byref(o) if o is not None else None, FAKE, None)
    assert upd(pr=None) == L.DMN_EINVAL
    assert upd(pr=L.DmnTrainParams(0, *([FAKE.value] * 7))) == L.DMN_EINVAL
    assert upd(pr=L.DmnTrainParams(3, None, *([FAKE.value] * 6))) == L.DMN_EINVAL
    assert upd(pr=L.DmnTrainParams(3, *([FAKE.value] * 6), None)) == L.DMN_EINVAL
    assert upd(prec=L.DMN_F32_STATE) == L.DMN_EUNSUPPORTED
    assert upd(gw=None) == L.DMN_EINVAL
    assert upd(o=None) == L.DMN_EINVAL
    for field, bad in (("half_period", 0), ("steps_per_epoch", 0), ("beta1", 1.0),
                       ("beta2", -0.1), ("eps", 0.0), ("penalty", -1.0), ("lr_decay", 0.0),
                       ("lr_min", float("nan"))):
        o = L.DmnAmsgradOpts(1.5e-3, 1.5e-2, 0.999, 50, 1, 0.9, 0.999, 1e-8, 1e3)
        setattr(o, field, bad)
        assert upd(o=o) == L.DMN_EINVAL, field
    assert lib.dmn_training_refresh(None, L.DMN_F64, None) == L.DMN_EINVAL
    assert lib.dmn_training_refresh(ctypes.byref(params), 5, None) == L.DMN_EUNSUPPORTED

    assert lib.dmn_sample_stiffness(-1, L.DMN_F64, FAKE, FAKE, FAKE, None) == L.DMN_EINVAL
    assert lib.dmn_sample_stiffness(4, L.DMN_F64, None, FAKE, FAKE, None) == L.DMN_EINVAL
    assert lib.dmn_sample_stiffness(4, 9, FAKE, FAKE, FAKE, None) == L.DMN_EUNSUPPORTED


def test_orientation_group_validation_codes():
    lib = L.lib()
    lin = L.DMN_ORI["linear"]
    gn = lambda depth=3, shape=lin, G=4, prec=L.DMN_F64, p=FAKE, lam=FAKE: \
        lib.dmn_orientation_group_normals(depth, shape, G, prec, p, FAKE, lam, FAKE, None)
    assert gn(depth=0) == L.DMN_EINVAL
    assert gn(shape=L.DMN_ORI["none"]) == L.DMN_EINVAL
    assert gn(shape=9) == L.DMN_EINVAL
    assert gn(G=-1) == L.DMN_EINVAL
    assert gn(prec=L.DMN_F32_STATE) == L.DMN_EUNSUPPORTED
    assert gn(p=None) == L.DMN_EINVAL
    assert gn(lam=None) == L.DMN_EINVAL
    ch = lambda G=4, gw=FAKE, gpq=FAKE: lib.dmn_orientation_group_chain(
        3, lin, G, L.DMN_F64, FAKE, FAKE, FAKE, FAKE, FAKE, gw, gpq, None)
    assert ch(gw=None) == L.DMN_EINVAL
    assert ch(gpq=None) == L.DMN_EINVAL
    assert ch(G=-2) == L.DMN_EINVAL
    opts = L.DmnAmsgradOpts(1.5e-3, 1.5e-2, 0.999, 50, 1, 0.9, 0.999, 1e-8, 1e3)
    good = L.DmnTrainParamsOriented(3, lin, *([FAKE.value] * 6))
    up = lambda pr=good, o=opts, prec=L.DMN_F64: lib.dmn_training_update_oriented(
        ctypes.byref(pr) if pr is not None else None, prec, FAKE, FAKE,
        ctypes.byref(o) if o is not None else None, FAKE, None)
    assert up(pr=None) == L.DMN_EINVAL
    assert up(pr=L.DmnTrainParamsOriented(3, 0, *([FAKE.value] * 6))) == L.DMN_EINVAL
    assert up(pr=L.DmnTrainParamsOriented(11, lin, *([FAKE.value] * 6))) == L.DMN_EINVAL
    assert up(pr=L.DmnTrainParamsOriented(3, lin, None, *([FAKE.value] * 5))) == L.DMN_EINVAL
    assert up(o=None) == L.DMN_EINVAL
    assert up(prec=4) == L.DMN_EUNSUPPORTED
    bad = L.DmnAmsgradOpts(1.5e-3, 1.5e-2, 0.999, 0, 1, 0.9, 0.999, 1e-8, 1e3)
    assert up(o=bad) == L.DMN_EINVAL
    assert lib.dmn_training_refresh_oriented(None, L.DMN_F64, None) == L.DMN_EINVAL


def test_grouped_linear_validation_codes():
    lib = L.lib()
    off = lambda *v: (ctypes.c_int64 * len(v))(*v)
    good = off(0, 2, 2, 5)
    one = lib.dmn_homogenize_linear_groups_workspace_size(3, 1, L.DMN_F64)
    assert one > 0
    assert lib.dmn_homogenize_linear_groups_workspace_size(3, 3, L.DMN_F64) == 3 * one - 2 * 256
    assert lib.dmn_homogenize_linear_groups_workspace_size(0, 3, L.DMN_F64) == 0
    assert lib.dmn_homogenize_linear_groups_workspace_size(3, 0, L.DMN_F64) == 0
    assert lib.dmn_homogenize_linear_groups_workspace_size(3, 3, L.DMN_F32_STATE) == 0
    fw = lambda depth=3, G=3, o=good, prec=L.DMN_F64, w=FAKE, n=FAKE, c=FAKE, ws=None, nb=0: \
        lib.dmn_homogenize_linear_groups(depth, G, o, prec, w, n, c, c, c, ws, nb, None)
    assert fw(depth=0) == L.DMN_EINVAL
    assert fw(depth=11) == L.DMN_EINVAL
    assert fw(G=0) == L.DMN_EINVAL
    assert fw(o=None) == L.DMN_EINVAL
    assert fw(o=off(0, 3, 2, 5)) == L.DMN_EINVAL      # decreasing
    assert fw(o=off(1, 2, 3, 5)) == L.DMN_EINVAL      # does not start at 0
    assert fw(prec=L.DMN_F32_STATE) == L.DMN_EUNSUPPORTED
    assert fw(w=None) == L.DMN_EINVAL
    assert fw(n=None) == L.DMN_EINVAL
    assert fw(c=None) == L.DMN_EINVAL
    assert fw(o=off(0, 0, 0, 0), c=None) == L.DMN_EWORKSPACE   # empty batch needs no arrays
    assert fw() == L.DMN_EWORKSPACE
    assert fw(ws=ctypes.c_void_p(ALIGNED.value + 8), nb=1 << 20) == L.DMN_EWORKSPACE
    bsize = lambda o=good, G=3, depth=8: lib.dmn_homogenize_backward_groups_workspace_size(
        depth, G, o, L.DMN_F64)
    assert bsize() > lib.dmn_homogenize_linear_groups_workspace_size(8, 3, L.DMN_F64)
    assert bsize(o=off(0, 3, 2, 5)) == 0
    assert bsize(o=None) == 0
    assert bsize(G=0) == 0
    # more samples in a group need more partial slots, an empty group one wave
    assert bsize(o=off(0, 2, 2, 500)) > bsize()
    assert bsize(o=off(0, 0, 0, 0)) > 0
    bw = lambda G=3, o=good, gw=FAKE, gn=FAKE, c=FAKE, ws=None: \
        lib.dmn_homogenize_backward_groups(3, G, o, L.DMN_F64, FAKE, FAKE, c, c, c, gw, gn, ws,
                                           0, None)
    assert bw(gw=None) == L.DMN_EINVAL
    assert bw(gn=None) == L.DMN_EINVAL
    assert bw(c=None) == L.DMN_EINVAL
    assert bw(G=0) == L.DMN_EINVAL
    assert bw(o=off(0, 3, 2, 5)) == L.DMN_EINVAL
    assert bw() == L.DMN_EWORKSPACE


def test_missing_library_fails_loudly(monkeypatch):
    """No fallback: without the built library every call raises."""
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libdmn.so"))
    with pytest.raises(L.DmnError, match="no fallback"):
        L.lib()


def test_wrappers_refuse_host_tensors():
    """The bindings only marshal device tensors; host tensors are rejected
    before any library call (no CPU path)."""
    torch = pytest.importorskip("torch")
    from paper_2103_08253_amd import (dmn_homogenize_backward_groups, dmn_homogenize_linear,
                                      dmn_homogenize_linear_groups)
    w = torch.ones(8, dtype=torch.float64)
    n = torch.zeros(7, 3, dtype=torch.float64)
    C = torch.eye(6, dtype=torch.float64).expand(2, 6, 6).contiguous()
    with pytest.raises(TypeError, match="GPU tensor"):
        dmn_homogenize_linear(w, n, C, C)
    with pytest.raises(TypeError, match="GPU tensor"):
        dmn_homogenize_linear_groups(w, n[None], [0, 2], C, C)
    with pytest.raises(TypeError, match="GPU tensor"):
        dmn_homogenize_backward_groups(w, n[None], [0, 2], C, C, C)


def test_unrun_depths_are_switched_off():
    """Depths up to 10 pass argument validation, but calls whose kernels have
    not run on the device at that depth return DMN_EUNSUPPORTED: the
    Gauss-point update and the linear map above depth 9, the linear VJP and
    the adjoint above depth 8.  Below, the call goes on to the workspace
    check."""
    lib = L.lib()
    fib = L.DmnElastic(72000.0, 0.22)
    mat = L.DmnJ2(2800.0, 0.35, 50.0, 200.0, 30.0, 60.0)
    opts = L.DmnNewtonOpts(1e-10, 25, 10, 1e-4)
    big = 1 << 34
    off = (ctypes.c_int64 * 2)(0, 4)
    expect = lambda depth, top: L.DMN_EUNSUPPORTED if depth > top else L.DMN_EWORKSPACE
    for depth in (8, 9, 10):
        arr = (L.DmnPointGroup * 1)(group(depth))
        rc = lib.dmn_update_gauss_points(arr, 1, ctypes.byref(fib), ctypes.byref(mat), L.DMN_F64,
                                         ctypes.byref(opts), None, 0, None)
        assert rc == expect(depth, 9), (depth, rc)
        rc = lib.dmn_homogenize_linear(ctypes.byref(net(depth)), 4, L.DMN_F64, FAKE, FAKE, None,
                                       FAKE, None, big, None)
        assert rc == expect(depth, 9), (depth, rc)
        rc = lib.dmn_homogenize_linear_groups(depth, 1, off, L.DMN_F64, FAKE, FAKE, FAKE, FAKE,
                                              FAKE, None, big, None)
        assert rc == expect(depth, 9), (depth, rc)
        ag = L.DmnAdjointGroup(net(depth), 4, FAKE.value, FAKE.value, FAKE.value, FAKE.value,
                               None, ALIGNED.value, FAKE.value, FAKE.value)
        arr_a = (L.DmnAdjointGroup * 1)(ag)
        rc = lib.dmn_update_adjoint(arr_a, 1, ctypes.byref(fib), ctypes.byref(mat), L.DMN_F64,
                                    None, 0, None)
        assert rc == expect(depth, 8), (depth, rc)
        rc = lib.dmn_homogenize_backward(ctypes.byref(net(depth)), 4, L.DMN_F64, FAKE, FAKE, None,
                                         FAKE, FAKE, FAKE, None, None, None, big, None)
        assert rc == expect(depth, 8), (depth, rc)
        rc = lib.dmn_homogenize_backward_groups(depth, 1, off, L.DMN_F64, FAKE, FAKE, FAKE, FAKE,
                                                FAKE, FAKE, FAKE, None, big, None)
        assert rc == expect(depth, 8), (depth, rc)
