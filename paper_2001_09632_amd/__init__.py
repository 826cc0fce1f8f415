"""MI355X-native adaptive block compressive sensing (AL-DCT-BBV / AL-DCT-DD,
masked inverse 2D-DCT, IDA post-processing).

Thin Python binding of the C ABI in include/abcs.h: it marshals torch device
tensors to raw pointers and the current HIP stream; every step of the method
runs in the gfx950 kernels of libabcs.so.  There is no CPU fallback: calls
raise if the library is missing.
"""
from .api import (ZZ, BBV, DD, Plan, AbcsError, budget, sense, reconstruct, encode, sense_decode, encode_workspace_bytes,  # noqa: F401
                  dct_basis, METHODS, ida_refine, ida_iterate, ida_workspace_bytes, DENOISERS,
                  denoise, denoise_workspace_bytes, cnn_param_count, cnn_train_step,
                  cnn_train_workspace_bytes, IdaGraph, PRECISIONS,
                  amp_refine, amp_workspace_bytes, ALGORITHMS, threshold,
                  threshold_workspace_bytes, budget_correlation, RULES, TRANSFORMS,
                  bbv_samples, ida_refine_bbv, dncnn_param_count, dncnn_running_count,
                  dncnn_train_workspace_bytes, dncnn_train_step, workspace_part,
                  ida_refine_noalloc, ida_noalloc_scratch_bytes, denoiser_params,
                  set_launch_table, launch_split, plan_size_class, time_splits, build_id, image_totals)
from .admission import Admission  # noqa: F401
