"""ctypes declarations of the C ABI in include/wf.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwf.so")

WF_OK, WF_EINVAL, WF_ENOMEM, WF_EBUDGET, WF_EHIP, WF_ENOTSUP = range(6)
STATUS_NAMES = {0: "WF_OK", 1: "WF_EINVAL", 2: "WF_ENOMEM", 3: "WF_EBUDGET", 4: "WF_EHIP",
                5: "WF_ENOTSUP"}
STORE = {"f32": 0, "f16": 1, "bf16": 2}
STRATEGY = {"auto": 0, "G": 1, "H": 2, "otf": 3}
OTF_FORM = {"auto": 0, "rebuilt": 1, "factorised": 2}


class WfImageShape(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("cell_rad", ctypes.c_double)]


class WfOptions(ctypes.Structure):
    _fields_ = [("J", ctypes.c_int32), ("beta", ctypes.c_double),
                ("oversample", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("smax", ctypes.c_int32), ("eps_w", ctypes.c_double),
                ("nbins", ctypes.c_int32), ("strategy", ctypes.c_int32),
                ("store", ctypes.c_int32), ("plan_fraction", ctypes.c_double),
                ("budget_fraction", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("tile", ctypes.c_int32), ("max_rows_per_item", ctypes.c_int32),
                ("branches", ctypes.c_int32), ("surrogate", ctypes.c_void_p),
                ("surrogate_tol", ctypes.c_double), ("weights", ctypes.c_void_p),
                ("flags", ctypes.c_void_p), ("otf_form", ctypes.c_int32)]


class WfPlanInfo(ctypes.Structure):
    _fields_ = [("nchan", ctypes.c_int32), ("nbins", ctypes.c_int32),
                ("strategy", ctypes.c_int32), ("store", ctypes.c_int32),
                ("Kx", ctypes.c_int32), ("Ky", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("p_wsclean", ctypes.c_int32), ("p_star", ctypes.c_int32),
                ("nrows", ctypes.c_int64), ("ntaps", ctypes.c_int64),
                ("nwork", ctypes.c_int64), ("k_estimate", ctypes.c_double),
                ("mem_g_bytes", ctypes.c_double), ("mem_model_bytes", ctypes.c_double),
                ("cost_model", ctypes.c_double), ("capped_fraction", ctypes.c_double),
                ("max_dropped_energy", ctypes.c_double), ("build_seconds", ctypes.c_double),
                ("max_rows_per_item", ctypes.c_int32), ("branch", ctypes.c_int32),
                ("surrogate_fraction", ctypes.c_double), ("mem_h_bytes", ctypes.c_double),
                ("nflagged", ctypes.c_int64), ("mem_transient_bytes", ctypes.c_double),
                ("value_pass_flops", ctypes.c_double), ("mem_khat_bytes", ctypes.c_double),
                ("otf_form", ctypes.c_int32)]


class WfTuneInfo(ctypes.Structure):
    _fields_ = [("branches", ctypes.c_int32), ("retuned_chans", ctypes.c_int32),
                ("sweep_ms_before", ctypes.c_double), ("sweep_ms_after", ctypes.c_double),
                ("wide_tile_bins", ctypes.c_int32)]


APPLY = {"forward": 0, "adjoint": 1, "psf": 2, "psf_re": 3}


_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double

SIGNATURES = {
    "wf_default_options": (None, [ctypes.POINTER(WfOptions)]),
    "wf_briggs_weights": (_I32, [_P, _I64, _P, _P, _I32, WfImageShape, ctypes.c_double, _P,
                                 _P, _P, _P]),
    "wf_briggs_weights_noalloc": (_I32, [_P, _I64, _D, WfImageShape, ctypes.c_double, _P, _P,
                                         _P, _P]),
    "wf_build_operator": (_I32, [_P, _I64, _P, _P, _I32, WfImageShape, ctypes.c_uint64,
                                 ctypes.POINTER(WfOptions), _P, ctypes.POINTER(_P)]),
    "wf_forward": (_I32, [_P, _P, _P, _P]),
    "wf_adjoint": (_I32, [_P, _P, _P, _P]),
    "wf_psf_apply": (_I32, [_P, _P, _P, _P]),
    "wf_psf_apply_re": (_I32, [_P, _P, _P, _P]),
    "wf_plan": (_I32, [_P, _I64, _D, WfImageShape, ctypes.c_uint64,
                       ctypes.POINTER(WfOptions), ctypes.POINTER(WfPlanInfo), _P, _I32]),
    "wf_get_plan": (_I32, [_P, _I32, ctypes.POINTER(WfPlanInfo)]),
    "wf_get_centroids": (_I32, [_P, _I32, _P, _I32]),
    "wf_get_bin_rows": (_I32, [_P, _I32, _P, _I32]),
    "wf_get_row": (_I32, [_P, _I32, _I64, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                          ctypes.POINTER(_I32), ctypes.POINTER(_I32), _P, _I32]),
    "wf_layer_grid": (_I32, [_P, _I32, _I32, _P, _P, _P]),
    "wf_profile_enable": (_I32, [_P, _I32, _I32]),
    "wf_profile_read": (_I32, [_P, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    "wf_set_branches": (_I32, [_P, _I32]),
    "wf_set_sweep": (_I32, [_P, _I32]),
    "wf_graph_capture": (_I32, [_P, _I32, _P, _P, _P, ctypes.POINTER(_P)]),
    "wf_graph_launch": (_I32, [_P, _P]),
    "wf_graph_destroy": (_I32, [_P]),
    "wf_graph_nodes": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "wf_latency_enable": (_I32, [_P, _I32]),
    "wf_read_latency": (_I32, [_P, _P, _I32]),
    "wf_autotune": (_I32, [_P, _P, _P, _P, _I32, ctypes.POINTER(WfTuneInfo)]),
    "wf_get_bin_tiles": (_I32, [_P, _I32, _P, _I32]),
    "wf_set_bin_tiles": (_I32, [_P, _I32, _P, _I32]),
    "wf_dirty_image": (_I32, [_P, _P, _P, _P]),
    "wf_op_norm": (_I32, [_P, _I32, ctypes.POINTER(_D), _P]),
    "wf_fb_iterate": (_I32, [_P, _P, _P, _I32, _D, _D, _P]),
    "wf_mlp_create": (_I32, [ctypes.c_uint64, ctypes.POINTER(_P)]),
    "wf_mlp_destroy": (_I32, [_P]),
    "wf_mlp_num_params": (_I64, []),
    "wf_mlp_get_params": (_I32, [_P, _P, _I64]),
    "wf_mlp_set_params": (_I32, [_P, _P, _I64]),
    "wf_mlp_inputs": (_I32, [_P, _P, _P, _P, _I64, ctypes.POINTER(WfOptions), _P, _P, _P]),
    "wf_mlp_targets": (_I32, [_P, _P, _I64, ctypes.POINTER(WfOptions), _P, _P]),
    "wf_mlp_loss_grad": (_I32, [_P, _P, _P, _I32, _P, _P, _P]),
    "wf_mlp_adam_step": (_I32, [_P, ctypes.c_float, _P]),
    "wf_mlp_train": (_I32, [_P, _P, _P, _I64, _I32, _I32, _D, _D, ctypes.c_uint64, _P, _P]),
    "wf_mlp_infer": (_I32, [_P, _P, _I64, _I32, _P, _P]),
    "wf_destroy": (_I32, [_P]),
    "wf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libwf.so (built by build_lib); raise if it is missing -- there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2605_26347_amd/build_lib.py` (no CPU fallback exists)")
    # torch first: the library then binds to the HIP runtime torch has loaded (same
    # soname), so that one runtime owns the device, the tensors' memory and the streams
    import torch  # noqa: F401
    _lib = bind(ctypes.CDLL(LIB_PATH))
    return _lib


def bind(lib):
    """Declare the C signatures of every entry point on a loaded library."""
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


class WfError(RuntimeError):
    def __init__(self, status, where):
        msg = load().wf_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, where):
    if status != WF_OK:
        raise WfError(status, where)
