"""ctypes loader of libctrex.so (the C ABI in include/ctrex.h).

The library is built in-tree by ``paper_2609_30166_amd.build``.  There is no
fallback: if the shared object is missing or cannot be loaded, every entry
point raises.
"""

from __future__ import annotations

import ctypes
import os
import threading

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libctrex.so")
_lock = threading.Lock()
_lib = None

OK = 0
STATUS = {
    -1: "CTREX_EINVAL", -2: "CTREX_ESHAPE", -3: "CTREX_ESINGULAR", -4: "CTREX_ESOURCE_INSIDE",
    -5: "CTREX_EDEVICE", -6: "CTREX_EWORKSPACE", -7: "CTREX_ESTATE", -8: "CTREX_ENONFINITE",
}
F32, BF16, F16 = 0, 1, 2
NONNEG, BF16_GATHER, F16_GATHER, RECOMPUTE_WEIGHTS, VOXEL_BP = 1, 2, 4, 8, 16
NN_RELU, NN_ACCUMULATE, NN_OUT_F32 = 1, 2, 4


class CtrexError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


def library_path():
    return _PATH


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_PATH):
            raise ImportError(
                "libctrex.so is not built; run `python -c \"import __graft_entry__ as g; "
                "g.build()\"` (or python -m paper_2609_30166_amd.build) first")
        L = ctypes.CDLL(_PATH)
        vp, i32, u32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
        ip = ctypes.POINTER(ctypes.c_int32)
        dp = ctypes.POINTER(ctypes.c_double)
        sigs = {
            "ctrex_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int]),
            "ctrex_destroy": (None, [vp]),
            "ctrex_last_error": (ctypes.c_char_p, [vp]),
            "ctrex_set_geometry": (ctypes.c_int, [vp, dp, i32, i32, i32, i32, i32, i32, i32, d]),
            "ctrex_set_motion": (ctypes.c_int, [vp, vp, i32, i32, i32, dp]),
            "ctrex_set_voxel_weights": (ctypes.c_int, [vp, vp]),
            "ctrex_forward_project": (ctypes.c_int, [vp, vp, i32, vp, i32, ip, i32, vp]),
            "ctrex_back_project": (ctypes.c_int, [vp, vp, i32, vp, i32, ip, i32, vp]),
            "ctrex_back_project_scaled": (ctypes.c_int, [vp, vp, i32, ctypes.c_float, vp, i32, ip,
                                                         i32, vp]),
            "ctrex_back_project_noalloc": (ctypes.c_int, [vp, vp, i32, vp, i32, ip, i32, vp]),
            "ctrex_scratch_bytes": (ctypes.c_int, [vp, i32, ctypes.POINTER(ctypes.c_size_t)]),
            "ctrex_set_scratch": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
            "ctrex_data_residual": (ctypes.c_int, [vp, vp, i32, vp, vp, i32, ctypes.c_float, ip,
                                                   i32, vp, vp]),
            "ctrex_back_project_voxel": (ctypes.c_int, [vp, vp, i32, vp, i32, ip, i32, vp]),
            "ctrex_set_cylinder": (ctypes.c_int, [vp, i32, i32, i32, ctypes.c_double,
                                                  ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
            "ctrex_forward_project_cyl": (ctypes.c_int, [vp, vp, i32, vp, i32, ip, i32, vp]),
            "ctrex_back_project_cyl": (ctypes.c_int, [vp, vp, i32, vp, i32, ip, i32, vp]),
            "ctrex_sample_count_cyl": (ctypes.c_int, [vp, ip, i32, ctypes.POINTER(ctypes.c_int64),
                                                      vp]),
            "ctrex_sirt_workspace_bytes_cyl": (ctypes.c_int, [vp, i32,
                                                              ctypes.POINTER(ctypes.c_size_t)]),
            "ctrex_sirt_iterate_cyl": (ctypes.c_int, [vp, vp, vp, i32, i32, ctypes.c_float,
                                                      ctypes.c_uint32, ip, i32, vp, ctypes.c_size_t,
                                                      ctypes.POINTER(ctypes.c_double), vp]),
            "ctrex_sirt_workspace_bytes": (ctypes.c_int, [vp, i32, u32,
                                                          ctypes.POINTER(ctypes.c_size_t)]),
            "ctrex_sirt_iterate": (ctypes.c_int, [vp, vp, vp, i32, i32, ctypes.c_float, u32, ip,
                                                  i32, vp, ctypes.c_size_t, dp, vp]),
            "ctrex_residual_norm": (ctypes.c_int, [vp, vp, i32, vp, i32, ip, i32, dp, vp]),
            "ctrex_sample_count": (ctypes.c_int, [vp, ip, i32, ctypes.POINTER(ctypes.c_int64), vp]),
            "ctrex_convert": (ctypes.c_int, [vp, vp, i32, vp, i32, ctypes.c_int64, vp]),
            "ctrex_profile_enable": (ctypes.c_int, [vp, i32]),
            "ctrex_tv": (ctypes.c_int, [vp, vp, i32, i32, i32, ctypes.c_float, ctypes.c_float, dp,
                                        vp, vp]),
            "ctrex_profile_read": (ctypes.c_int, [vp, dp, ctypes.POINTER(ctypes.c_int64)]),
            # learned-correction kernels (include/ctrex_nn.h)
            "ctrex_nn_scratch_bytes": (ctypes.c_int, [i32, i32, ctypes.c_int64,
                                                      ctypes.POINTER(ctypes.c_size_t)]),
            "ctrex_nn_conv3": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, vp, vp, i32, i32, i32,
                                              i32, i32, i32, u32, vp]),
            "ctrex_nn_conv3_wgrad": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, i32, i32, i32,
                                                    i32, i32, i32, vp, vp, vp]),
            "ctrex_nn_conv3_cat": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, i32, i32, i32, vp,
                                                  vp, vp, i32, i32, i32, vp, i32, i32, i32, vp,
                                                  i32, i32, i32, i32, i32, u32, vp]),
            "ctrex_nn_conv3_head": (ctypes.c_int, [vp, vp, i32, i32, vp, vp, vp, i32, i32, vp, vp,
                                                   vp, ctypes.c_float, vp, vp, i32, i32, i32,
                                                   vp]),
            "ctrex_nn_conv3_wgrad_cat": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, i32, i32, i32,
                                                        vp, i32, i32, i32, i32, i32, i32, vp, vp,
                                                        vp]),
            "ctrex_nn_upconv2": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, vp, vp, i32, i32, i32,
                                                i32, i32, i32, u32, vp]),
            "ctrex_nn_upconv2_dgrad": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, vp, i32, i32,
                                                      i32, i32, i32, i32, u32, vp]),
            "ctrex_nn_upconv2_wgrad": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, i32, i32, i32,
                                                      i32, i32, i32, vp, vp, vp]),
            "ctrex_nn_maxpool2": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, i32, i32, i32, vp]),
            "ctrex_nn_maxpool2_backward": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, vp, i32, i32,
                                                          i32, vp]),
            "ctrex_nn_maxpool2_relu_backward": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, vp, i32,
                                                               i32, i32, vp]),
            "ctrex_nn_relu_backward": (ctypes.c_int, [vp, vp, vp, i32, i32, i32, ctypes.c_int64,
                                                      vp]),
            "ctrex_nn_input": (ctypes.c_int, [vp, vp, ctypes.c_float, vp, ctypes.c_int64, vp]),
            "ctrex_nn_head": (ctypes.c_int, [vp, vp, i32, vp, vp, vp, ctypes.c_float, vp, vp,
                                             ctypes.c_int64, vp]),
            "ctrex_nn_head_backward": (ctypes.c_int, [vp, vp, i32, vp, ctypes.c_float, vp, vp, vp,
                                                      vp, vp, ctypes.c_int64, vp]),
            "ctrex_nn_head_relu_backward": (ctypes.c_int, [vp, vp, i32, vp, ctypes.c_float, vp,
                                                           vp, vp, vp, vp, ctypes.c_int64, vp]),
            "ctrex_nn_mse": (ctypes.c_int, [vp, vp, vp, ctypes.c_int64, ctypes.c_float, dp, vp,
                                            vp]),
            "ctrex_nn_adam": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float,
                                             ctypes.c_float, ctypes.c_float, ctypes.c_float, i32,
                                             vp]),
            "ctrex_nn_pack_conv3": (ctypes.c_int, [vp, vp, i32, i32, vp, vp, vp]),
            "ctrex_nn_pack_upconv2": (ctypes.c_int, [vp, vp, i32, i32, vp, vp, vp]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        return _lib


def check(ctx, code):
    if code != OK:
        msg = lib().ctrex_last_error(ctx)
        raise CtrexError(code, msg.decode() if msg else "")
