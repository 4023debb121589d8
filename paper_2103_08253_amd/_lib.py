"""ctypes view of libdmn.so (the C ABI declared in include/dmn.h).

The library is built in-tree by ``python -m paper_2103_08253_amd.build``.
Loading fails loudly when it is missing: there is no fallback path.
"""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdmn.so")

DMN_OK, DMN_EINVAL, DMN_EWORKSPACE, DMN_EHIP, DMN_EUNSUPPORTED = 0, -1, -2, -3, -4
DMN_F64, DMN_F32, DMN_F32_STATE = 0, 1, 2
DMN_ORI = {"none": 0, "linear": 1, "trilinear": 2, "quadratic": 3}
ORI_COUNT = {"linear": 3, "trilinear": 4, "quadratic": 6}
STATUS = {0: "ok", 1: "maxiter", 2: "nonfinite", 3: "notspd", 4: "local", 5: "badparam"}
ERRORS = {DMN_EINVAL: "DMN_EINVAL", DMN_EWORKSPACE: "DMN_EWORKSPACE", DMN_EHIP: "DMN_EHIP",
          DMN_EUNSUPPORTED: "DMN_EUNSUPPORTED"}


class DmnNet(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("w", ctypes.c_void_p), ("n", ctypes.c_void_p),
                ("ori_shape", ctypes.c_int32), ("ori_p", ctypes.c_void_p),
                ("ori_q", ctypes.c_void_p)]


class DmnElastic(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("nu", ctypes.c_double)]


class DmnJ2(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("nu", ctypes.c_double), ("sigma0", ctypes.c_double),
                ("k_inf", ctypes.c_double), ("dsigma", ctypes.c_double), ("b", ctypes.c_double)]


class DmnNewtonOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("max_backtrack", ctypes.c_int32), ("armijo", ctypes.c_double),
                ("local_max_iter", ctypes.c_int32), ("polish", ctypes.c_int32)]


class DmnPointGroup(ctypes.Structure):
    _fields_ = [("net", DmnNet), ("P", ctypes.c_int64),
                ("E", ctypes.c_void_p), ("z_in", ctypes.c_void_p), ("z_out", ctypes.c_void_p),
                ("a_in", ctypes.c_void_p), ("a_out", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("tangent", ctypes.c_void_p),
                ("iters", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("lam", ctypes.c_void_p)]


class DmnAdjointGroup(ctypes.Structure):
    _fields_ = [("net", DmnNet), ("P", ctypes.c_int64),
                ("E", ctypes.c_void_p), ("z_in", ctypes.c_void_p), ("a_conv", ctypes.c_void_p),
                ("g_sigma", ctypes.c_void_p), ("g_z_next", ctypes.c_void_p),
                ("g_z_prev", ctypes.c_void_p), ("gw", ctypes.c_void_p), ("gn", ctypes.c_void_p)]


class DmnGpTuning(ctypes.Structure):
    _fields_ = [("lanes_per_point", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32)]


class DmnLossOpts(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double), ("q", ctypes.c_double)]


class DmnAmsgradOpts(ctypes.Structure):
    _fields_ = [("lr_min", ctypes.c_double), ("lr_max", ctypes.c_double),
                ("lr_decay", ctypes.c_double), ("half_period", ctypes.c_int32),
                ("steps_per_epoch", ctypes.c_int32), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("penalty", ctypes.c_double)]


class DmnTrainParams(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("v", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("beta", ctypes.c_void_p), ("w", ctypes.c_void_p), ("n", ctypes.c_void_p),
                ("state", ctypes.c_void_p), ("step", ctypes.c_void_p)]


class DmnTrainParamsOriented(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("ori_shape", ctypes.c_int32), ("v", ctypes.c_void_p),
                ("p", ctypes.c_void_p), ("q", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("state", ctypes.c_void_p), ("step", ctypes.c_void_p)]


DMN_TRAIN_STATS = 8

# exported functions and their signatures
_SIGS = {
    "dmn_training_loss_workspace_size": (ctypes.c_size_t, [ctypes.c_int64]),
    "dmn_training_loss": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.POINTER(DmnLossOpts),
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dmn_training_update": (ctypes.c_int, [ctypes.POINTER(DmnTrainParams), ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.POINTER(DmnAmsgradOpts), ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "dmn_training_refresh": (ctypes.c_int, [ctypes.POINTER(DmnTrainParams), ctypes.c_int,
                                            ctypes.c_void_p]),
    "dmn_orientation_group_normals": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32,
                                                     ctypes.c_int32, ctypes.c_int,
                                                     ctypes.c_void_p, ctypes.c_void_p,
                                                     ctypes.c_void_p, ctypes.c_void_p,
                                                     ctypes.c_void_p]),
    "dmn_orientation_group_chain": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p]),
    "dmn_training_update_oriented": (ctypes.c_int, [ctypes.POINTER(DmnTrainParamsOriented),
                                                    ctypes.c_int, ctypes.c_void_p,
                                                    ctypes.c_void_p,
                                                    ctypes.POINTER(DmnAmsgradOpts),
                                                    ctypes.c_void_p, ctypes.c_void_p]),
    "dmn_training_refresh_oriented": (ctypes.c_int, [ctypes.POINTER(DmnTrainParamsOriented),
                                                     ctypes.c_int, ctypes.c_void_p]),
    "dmn_sample_stiffness": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "dmn_version": (ctypes.c_char_p, []),
    "dmn_homogenize_linear_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(DmnNet),
                                                               ctypes.c_int64, ctypes.c_int]),
    "dmn_homogenize_linear": (ctypes.c_int, [ctypes.POINTER(DmnNet), ctypes.c_int64, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                             ctypes.c_void_p]),
    "dmn_homogenize_backward_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(DmnNet),
                                                                 ctypes.c_int64, ctypes.c_int]),
    "dmn_homogenize_backward": (ctypes.c_int, [ctypes.POINTER(DmnNet), ctypes.c_int64, ctypes.c_int,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_size_t, ctypes.c_void_p]),
    "dmn_homogenize_linear_groups_workspace_size": (ctypes.c_size_t, [ctypes.c_int32,
                                                                      ctypes.c_int32,
                                                                      ctypes.c_int]),
    "dmn_homogenize_linear_groups": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                                    ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_size_t, ctypes.c_void_p]),
    "dmn_homogenize_backward_groups_workspace_size": (ctypes.c_size_t, [
        ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
    "dmn_homogenize_backward_groups": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32,
                                                      ctypes.POINTER(ctypes.c_int64),
                                                      ctypes.c_int, ctypes.c_void_p,
                                                      ctypes.c_void_p, ctypes.c_void_p,
                                                      ctypes.c_void_p, ctypes.c_void_p,
                                                      ctypes.c_void_p, ctypes.c_void_p,
                                                      ctypes.c_void_p, ctypes.c_size_t,
                                                      ctypes.c_void_p]),
    "dmn_update_gauss_points_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(DmnPointGroup),
                                                                 ctypes.c_int32, ctypes.c_int]),
    "dmn_update_gauss_points": (ctypes.c_int, [ctypes.POINTER(DmnPointGroup), ctypes.c_int32,
                                               ctypes.POINTER(DmnElastic), ctypes.POINTER(DmnJ2),
                                               ctypes.c_int, ctypes.POINTER(DmnNewtonOpts),
                                               ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dmn_update_gauss_points_noalloc": (ctypes.c_int, [ctypes.POINTER(DmnPointGroup),
                                                       ctypes.c_int32, ctypes.POINTER(DmnElastic),
                                                       ctypes.POINTER(DmnJ2), ctypes.c_int,
                                                       ctypes.POINTER(DmnNewtonOpts),
                                                       ctypes.c_void_p]),
    "dmn_gp_set_tuning": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(DmnGpTuning)]),
    "dmn_gp_get_tuning": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(DmnGpTuning)]),
    "dmn_gp_lane_variants": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.c_int32]),
    "dmn_update_adjoint_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(DmnAdjointGroup),
                                                            ctypes.c_int32, ctypes.c_int]),
    "dmn_update_adjoint": (ctypes.c_int, [ctypes.POINTER(DmnAdjointGroup), ctypes.c_int32,
                                          ctypes.POINTER(DmnElastic), ctypes.POINTER(DmnJ2),
                                          ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p]),
}

_lib = None


class DmnError(RuntimeError):
    pass


def lib():
    """Load libdmn.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DmnError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2103_08253_amd.build` (no fallback exists)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(rc, what):
    if rc != DMN_OK:
        raise DmnError(f"{what} returned {ERRORS.get(rc, rc)}")
