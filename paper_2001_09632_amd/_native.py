"""ctypes loader and prototypes of libabcs.so (include/abcs.h)."""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libabcs.so")

ABCS_OK, ABCS_EINVAL, ABCS_EDOMAIN, ABCS_EUNSUPPORTED, ABCS_ENOSPACE, ABCS_EHIP = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EDOMAIN", -3: "EUNSUPPORTED", -4: "ENOSPACE", -5: "EHIP"}

EXPORTS = [
    "abcs_plan_create", "abcs_plan_create_ex", "abcs_plan_destroy", "abcs_plan_totals", "abcs_plan_image",
    "abcs_budget", "abcs_sense", "abcs_reconstruct", "abcs_dct_basis", "abcs_last_error",
    "ida_workspace_bytes", "ida_refine", "ida_iterate", "abcs_denoise_workspace_bytes", "abcs_denoise",
    "abcs_cnn_param_count", "abcs_cnn_train_workspace_bytes", "abcs_cnn_train_step",
    "ida_graph_create", "ida_graph_launch", "ida_graph_destroy", "amp_workspace_bytes", "amp_refine",
    "abcs_threshold_workspace_bytes", "abcs_threshold", "abcs_budget_correlation",
    "abcs_bbv_samples", "ida_refine_bbv",
    "abcs_dncnn_param_count", "abcs_dncnn_running_count", "abcs_dncnn_train_workspace_bytes",
    "abcs_dncnn_train_step", "abcs_workspace_part", "abcs_encode", "abcs_sense_decode", "abcs_encode_workspace_bytes",
    "ida_noalloc_scratch_bytes", "ida_refine_noalloc",
    "abcs_image_totals", "abcs_set_launch_table", "abcs_launch_split", "abcs_plan_size_class", "abcs_time_splits", "abcs_build_id",
]


class LaunchEntry(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("transform", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("size_class", ctypes.c_int32), ("split", ctypes.c_int32)]


class AbcsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class ImageDesc(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("row_pitch", ctypes.c_int32),
        ("block", ctypes.c_int32), ("subrate", ctypes.c_double), ("method", ctypes.c_int32),
        ("transform", ctypes.c_int32), ("pixel_offset", ctypes.c_int64),
        ("block_offset", ctypes.c_int64), ("meas_offset", ctypes.c_int64),
        ("out_offset", ctypes.c_int64), ("n_meas", ctypes.c_int64),
        ("cropped_height", ctypes.c_int32), ("cropped_width", ctypes.c_int32),
        ("bbv_offset", ctypes.c_int64), ("n_bbv", ctypes.c_int64),
    ]


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2001_09632_amd.build`")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7 and the
    # library's dependency of the same name must resolve to it, so torch is
    # loaded first (loading the library first would bind torch to the system
    # runtime instead, and torch then finds no GPU).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    P64 = ctypes.POINTER(ctypes.c_int64)
    L.abcs_plan_create.argtypes = [ctypes.POINTER(ImageDesc), i32, ctypes.POINTER(vp)]
    L.abcs_plan_create_ex.argtypes = [ctypes.POINTER(ImageDesc), i32, ctypes.c_uint, ctypes.POINTER(vp)]
    L.abcs_plan_destroy.argtypes = [vp]
    L.abcs_plan_destroy.restype = None
    L.abcs_plan_totals.argtypes = [vp, P64, P64, P64]
    L.abcs_plan_image.argtypes = [vp, i32, ctypes.POINTER(ImageDesc)]
    L.abcs_image_totals.argtypes = [ctypes.POINTER(ImageDesc), P64, P64, P64]
    L.abcs_budget.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.abcs_sense.argtypes = [vp, vp, i64, vp, vp, vp, i32, vp]
    L.abcs_reconstruct.argtypes = [vp, vp, vp, vp, vp, i32, vp]
    L.abcs_encode.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, i32, vp, sz, vp]
    L.abcs_encode_workspace_bytes.argtypes = [vp]
    L.abcs_encode_workspace_bytes.restype = sz
    L.abcs_sense_decode.argtypes = [vp, vp, i64, vp, vp, vp, vp, i32, vp]
    L.abcs_dct_basis.argtypes = [i32, ctypes.POINTER(ctypes.c_double)]
    L.abcs_last_error.restype = ctypes.c_char_p
    L.ida_workspace_bytes.argtypes = [vp, i32]
    L.ida_workspace_bytes.restype = sz
    L.ida_refine.argtypes = [vp, vp, vp, vp, i32, ctypes.c_double, i32, vp, vp, vp, vp, sz, vp]
    L.ida_iterate.argtypes = [vp, vp, vp, vp, i32, i32, ctypes.c_double, i32, vp, vp, vp, vp, vp, sz, vp]
    L.abcs_denoise_workspace_bytes.argtypes = [vp, i32]
    L.abcs_denoise_workspace_bytes.restype = sz
    L.abcs_denoise.argtypes = [vp, i32, vp, vp, vp, vp, vp, sz, vp]
    L.abcs_cnn_param_count.argtypes = []
    L.abcs_cnn_param_count.restype = sz
    L.abcs_cnn_train_workspace_bytes.argtypes = [vp]
    L.abcs_cnn_train_workspace_bytes.restype = sz
    L.abcs_cnn_train_step.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, vp, vp, vp, vp, vp, vp, sz, vp]
    L.ida_graph_create.argtypes = [vp, vp, vp, vp, i32, ctypes.c_double, i32, vp, vp, vp, vp, sz,
                                   ctypes.POINTER(vp)]
    L.ida_graph_launch.argtypes = [vp, vp]
    L.amp_workspace_bytes.argtypes = [vp, i32]
    L.amp_workspace_bytes.restype = sz
    L.amp_refine.argtypes = [vp, vp, vp, vp, i32, ctypes.c_double, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.abcs_threshold_workspace_bytes.argtypes = [vp]
    L.abcs_threshold_workspace_bytes.restype = sz
    L.abcs_threshold.argtypes = [vp, vp, i64, i32, vp, vp, vp, sz, vp]
    L.abcs_budget_correlation.argtypes = [vp, vp, vp, vp, vp, vp]
    L.abcs_bbv_samples.argtypes = [vp, vp, i64, vp, vp]
    L.ida_refine_bbv.argtypes = [vp, vp, vp, vp, vp, i32, ctypes.c_double, i32, vp, vp, vp, vp, sz, vp]
    L.abcs_dncnn_param_count.argtypes = []
    L.abcs_dncnn_param_count.restype = sz
    L.abcs_dncnn_running_count.argtypes = []
    L.abcs_dncnn_running_count.restype = sz
    L.abcs_dncnn_train_workspace_bytes.argtypes = [vp]
    L.abcs_dncnn_train_workspace_bytes.restype = sz
    L.abcs_dncnn_train_step.argtypes = [vp, vp, vp, vp, vp, i64, ctypes.c_float, vp, vp, vp, vp, vp, vp, sz, vp]
    L.ida_noalloc_scratch_bytes.argtypes = []
    L.ida_noalloc_scratch_bytes.restype = sz
    L.ida_refine_noalloc.argtypes = [vp, vp, vp, vp, i32, ctypes.c_double, i32, vp, vp, vp, vp]
    L.abcs_workspace_part.argtypes = [vp, i32, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.abcs_set_launch_table.argtypes = [ctypes.POINTER(LaunchEntry), i32]
    L.abcs_launch_split.argtypes = [i32, i32, i32, i32]
    L.abcs_plan_size_class.argtypes = [vp, i32, i32]
    L.abcs_time_splits.argtypes = [vp, vp, i64, vp, vp, vp, vp, i32, i32, ctypes.POINTER(ctypes.c_float), vp]
    L.abcs_build_id.argtypes = []
    L.ida_graph_destroy.argtypes = [vp]
    L.ida_graph_destroy.restype = None
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("abcs_plan_destroy", "abcs_last_error", "ida_workspace_bytes", "ida_graph_destroy",
                        "amp_workspace_bytes", "abcs_threshold_workspace_bytes",
                        "abcs_dncnn_param_count", "abcs_dncnn_running_count", "abcs_dncnn_train_workspace_bytes",
                        "abcs_denoise_workspace_bytes", "abcs_cnn_param_count",
                        "abcs_cnn_train_workspace_bytes", "ida_noalloc_scratch_bytes",
                        "abcs_encode_workspace_bytes", "abcs_build_id"):
            f.restype = ctypes.c_int
    L.abcs_build_id.restype = ctypes.c_char_p
    _install_tuned_launches(L)
    _lib = L
    return L


TUNED_PATH = os.path.join(_PKG, "tuned_launch.json")
_TRANSFORMS = {"dct": 0, "wht": 1}
_PRECISIONS = {"fp32": 0, "bf16x3": 1, "fp16x3": 2, "bf16": 3, "fp16": 4}


def _install_tuned_launches(L):
    """Install the launch splits measured for this build (tune.py), if the
    stored table belongs to it; otherwise every split stays 0."""
    import json
    try:
        with open(TUNED_PATH) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return
    if table.get("build_id") != L.abcs_build_id().decode():
        return
    ents = [e for e in table.get("entries", []) if e.get("split", 0) != 0]
    arr = (LaunchEntry * max(1, len(ents)))()
    for i, e in enumerate(ents):
        arr[i] = LaunchEntry(int(e["block"]), _TRANSFORMS[e["transform"]], _PRECISIONS[e["precision"]],
                             int(e["size_class"]), int(e["split"]))
    L.abcs_set_launch_table(arr, len(ents))


def check(status):
    if status != ABCS_OK:
        raise AbcsError(status, lib().abcs_last_error().decode(errors="replace"))
