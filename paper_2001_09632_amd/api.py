"""Python binding of libabcs (argument marshalling only)."""
import ctypes

from ._native import ImageDesc, AbcsError, check, lib  # noqa: F401

ZZ, BBV, DD = 0, 1, 2
METHODS = {"zz": ZZ, "bbv": BBV, "dd": DD}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


TRANSFORMS = {"dct": 0, "wht": 1}


def _fill_desc(out, d, offset=0):
    """Fill an ImageDesc from a dict (see Plan); returns the next packed
    pixel offset."""
    m = d["method"]
    m = METHODS[m] if isinstance(m, str) else int(m)
    pitch = int(d.get("row_pitch", (int(d["width"]) + 3) // 4 * 4))
    po = d.get("pixel_offset")
    if po is None:
        po = offset
        offset += pitch * int(d["height"])
        offset = (offset + 3) // 4 * 4
    out.height, out.width, out.row_pitch = int(d["height"]), int(d["width"]), pitch
    out.block, out.subrate, out.method = int(d["block"]), float(d["subrate"]), m
    xf = d.get("transform", "dct")
    out.transform = TRANSFORMS[xf] if isinstance(xf, str) else int(xf)
    out.pixel_offset = int(po)
    return offset


def image_totals(d):
    """abcs_image_totals: (blocks, coefficients, decoded pixels) one
    descriptor dict (as for Plan) adds to a plan; host only."""
    desc = ImageDesc()
    _fill_desc(desc, d)
    b, m, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(lib().abcs_image_totals(ctypes.byref(desc), ctypes.byref(b), ctypes.byref(m), ctypes.byref(p)))
    return b.value, m.value, p.value


class Plan:
    """A validated batch of images (abcs_plan_create).

    images: iterable of dicts with keys height, width, block, subrate,
    method (0/1/2 or 'zz'/'bbv'/'dd'), and optionally transform ('dct'
    (default) or 'wht', or 0/1), row_pitch (default width rounded up to 4)
    and pixel_offset (default: images packed one after the other).  Create it
    with the target device current.  `features` names the optional tables to
    build ('denoise': every non-identity denoiser, D-AMP and training;
    'bounds': THI / THB); an encoder/decoder-only plan passes ().
    """

    FEATURES = {"denoise": 1, "bounds": 2}

    def __init__(self, images, features=("denoise", "bounds")):
        imgs = list(images)
        arr = (ImageDesc * max(1, len(imgs)))()
        offset = 0
        for i, d in enumerate(imgs):
            offset = _fill_desc(arr[i], d, offset)
        self._h = ctypes.c_void_p()
        flags = 0
        for f in features:
            flags |= self.FEATURES[f]
        check(lib().abcs_plan_create_ex(arr, len(imgs), flags, ctypes.byref(self._h)))
        self.n = len(imgs)
        b, m, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib().abcs_plan_totals(self._h, ctypes.byref(b), ctypes.byref(m), ctypes.byref(p)))
        self.blocks, self.meas, self.pixels = b.value, m.value, p.value
        self.images = []
        for i in range(self.n):
            out = ImageDesc()
            check(lib().abcs_plan_image(self._h, i, ctypes.byref(out)))
            self.images.append({f: getattr(out, f) for f, _ in ImageDesc._fields_})
        self.bbv_total = sum(d["n_bbv"] for d in self.images)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().abcs_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def budget(plan, px, k, offsets, stat, stream=None):
    """abcs_budget: px uint8 device tensor; k int32[blocks], offsets
    int64[blocks], stat int32[blocks] device tensors (written)."""
    check(lib().abcs_budget(plan.handle, _ptr(px), px.numel() * px.element_size(), _ptr(k),
                            _ptr(offsets), _ptr(stat), _stream(stream)))


PRECISIONS = {"fp32": 0, "bf16x3": 1, "fp16x3": 2, "bf16": 3, "fp16": 4}


def _prec(precision):
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def sense(plan, px, k, offsets, y, stream=None, precision="fp32"):
    """abcs_sense: y float32[meas] device tensor (written); precision one of
    PRECISIONS (the B = 16 transform's arithmetic)."""
    check(lib().abcs_sense(plan.handle, _ptr(px), px.numel() * px.element_size(), _ptr(k),
                           _ptr(offsets), _ptr(y), _prec(precision), _stream(stream)))


def reconstruct(plan, y, k, offsets, out, stream=None, precision="fp32"):
    """abcs_reconstruct: out float32[pixels] device tensor (written)."""
    check(lib().abcs_reconstruct(plan.handle, _ptr(y), _ptr(k), _ptr(offsets), _ptr(out),
                                 _prec(precision), _stream(stream)))


IDENTITY, BM3D, CNN, DNCNN = 0, 1, 2, 3
DENOISERS = {"identity": IDENTITY, "bm3d": BM3D, "cnn": CNN, "dncnn": DNCNN}


def encode_workspace_bytes(plan):
    return int(lib().abcs_encode_workspace_bytes(plan.handle))


def encode(plan, px, k, offsets, stat, y, out=None, stream=None, precision="fp32", workspace=None):
    """abcs_encode: budget + sense (+ the decoder's image into out, float32
    [pixels], when given) in one call; with a workspace of
    encode_workspace_bytes(plan) bytes an eligible plan runs in one
    launch."""
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().abcs_encode(plan.handle, _ptr(px), px.numel() * px.element_size(), _ptr(k), _ptr(offsets),
                            _ptr(stat), _ptr(y), _ptr(out), _prec(precision), _ptr(workspace), ws_bytes,
                            _stream(stream)))


def sense_decode(plan, px, k, offsets, y, out, stream=None, precision="fp32"):
    """abcs_sense_decode: sensing and the decoder's image (budgets given)."""
    check(lib().abcs_sense_decode(plan.handle, _ptr(px), px.numel() * px.element_size(), _ptr(k), _ptr(offsets),
                                  _ptr(y), _ptr(out), _prec(precision), _stream(stream)))


def ida_workspace_bytes(plan, denoiser):
    d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
    return int(lib().ida_workspace_bytes(plan.handle, d))


def ida_refine(plan, y, k, offsets, x, iters, damping=2.0, denoiser="identity", params=None,
               sigma_trace=None, workspace=None, stream=None):
    """ida_refine: x float32[pixels] (written with x^iters); workspace a
    uint8 device tensor of at least ida_workspace_bytes(plan, denoiser)."""
    d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().ida_refine(plan.handle, _ptr(y), _ptr(k), _ptr(offsets), int(iters), float(damping), d,
                           _ptr(params), _ptr(x), _ptr(sigma_trace), _ptr(workspace), ws_bytes,
                           _stream(stream)))


def ida_noalloc_scratch_bytes():
    return int(lib().ida_noalloc_scratch_bytes())


def ida_refine_noalloc(plan, y, k, offsets, x, iters, damping=2.0, denoiser="identity", params=None,
                       sigma_trace=None, stream=None):
    """ida_refine_noalloc: ida_refine with the library's fixed per-device
    scratch in place of a workspace (no allocation)."""
    d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
    check(lib().ida_refine_noalloc(plan.handle, _ptr(y), _ptr(k), _ptr(offsets), int(iters), float(damping), d,
                                   _ptr(params), _ptr(x), _ptr(sigma_trace), _stream(stream)))


def bbv_samples(plan, px, out, stream=None):
    """abcs_bbv_samples: out float32[plan.bbv_total] <- the signed BBV samples."""
    check(lib().abcs_bbv_samples(plan.handle, _ptr(px), px.numel() * px.element_size(), _ptr(out),
                                 _stream(stream)))


def ida_refine_bbv(plan, y, k, offsets, bbv, x, iters, damping=2.0, denoiser="identity", params=None,
                   sigma_trace=None, workspace=None, stream=None):
    """ida_refine_bbv: ida_refine with the BBV samples (float32[plan.bbv_total])
    as extra difference rows of A."""
    d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().ida_refine_bbv(plan.handle, _ptr(y), _ptr(k), _ptr(offsets), _ptr(bbv), int(iters), float(damping),
                               d, _ptr(params), _ptr(x), _ptr(sigma_trace), _ptr(workspace), ws_bytes,
                               _stream(stream)))


ALGORITHMS = {"damp": 1, "damp-d": 2}


def amp_workspace_bytes(plan, denoiser):
    d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
    return int(lib().amp_workspace_bytes(plan.handle, d))


def amp_refine(plan, y, k, offsets, x, iters, probe, damping=2.0, algorithm="damp", denoiser="identity",
               params=None, sigma_trace=None, alpha_trace=None, workspace=None, stream=None):
    """amp_refine: D-AMP ("damp") or DAMP-D ("damp-d"); probe float32[pixels]
    (the Monte-Carlo divergence probe, drawn by the caller)."""
    d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
    a = ALGORITHMS[algorithm] if isinstance(algorithm, str) else int(algorithm)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().amp_refine(plan.handle, _ptr(y), _ptr(k), _ptr(offsets), int(iters), float(damping), a, d,
                           _ptr(params), _ptr(probe), _ptr(x), _ptr(sigma_trace), _ptr(alpha_trace),
                           _ptr(workspace), ws_bytes, _stream(stream)))


class IdaGraph:
    """ida_graph_create / ida_graph_launch / ida_graph_destroy: the whole
    ida_refine loop recorded once as a HIP graph and replayed per launch().
    The tensors passed here are the ones every replay uses; this object keeps
    references to them (and to the plan) until close()."""

    def __init__(self, plan, y, k, offsets, x, iters, damping=2.0, denoiser="identity", params=None,
                 sigma_trace=None, workspace=None):
        d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
        ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
        self._keep = (plan, y, k, offsets, x, params, sigma_trace, workspace)
        self._h = ctypes.c_void_p()
        check(lib().ida_graph_create(plan.handle, _ptr(y), _ptr(k), _ptr(offsets), int(iters), float(damping), d,
                                     _ptr(params), _ptr(x), _ptr(sigma_trace), _ptr(workspace), ws_bytes,
                                     ctypes.byref(self._h)))

    def launch(self, stream=None):
        if not self._h:
            raise RuntimeError("graph is closed")
        check(lib().ida_graph_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            lib().ida_graph_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ida_iterate(plan, y, k, offsets, x, t_begin, t_end, damping=2.0, denoiser="identity", params=None,
                sigma_trace=None, v_last=None, workspace=None, stream=None):
    """ida_iterate: resumable IDA iterations t_begin .. t_end-1."""
    d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().ida_iterate(plan.handle, _ptr(y), _ptr(k), _ptr(offsets), int(t_begin), int(t_end),
                            float(damping), d, _ptr(params), _ptr(x), _ptr(sigma_trace), _ptr(v_last),
                            _ptr(workspace), ws_bytes, _stream(stream)))


def denoise_workspace_bytes(plan, denoiser):
    d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
    return int(lib().abcs_denoise_workspace_bytes(plan.handle, d))


def denoise(plan, x_in, sigma, x_out, denoiser="bm3d", params=None, workspace=None, stream=None):
    """abcs_denoise: x_in, x_out float32[pixels]; sigma float32[n] device tensors."""
    d = DENOISERS[denoiser] if isinstance(denoiser, str) else int(denoiser)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().abcs_denoise(plan.handle, d, _ptr(params), _ptr(x_in), _ptr(sigma), _ptr(x_out),
                             _ptr(workspace), ws_bytes, _stream(stream)))


def denoiser_params(weights, sigma_range):
    """Parameter block of a learned denoiser as abcs_denoise / ida_refine take
    it: the network's float32 weights (for DnCNN followed by its running
    statistics), then the range [lo, hi] of sigma the network accepts (hi
    may be inf; images whose sigma lies outside it are denoised by BM3D)."""
    import numpy as np
    lo, hi = sigma_range
    return np.concatenate([np.asarray(weights, dtype=np.float32).reshape(-1),
                           np.array([lo, hi], dtype=np.float32)])


def cnn_param_count():
    return int(lib().abcs_cnn_param_count())


def cnn_train_workspace_bytes(plan):
    return int(lib().abcs_cnn_train_workspace_bytes(plan.handle))


def cnn_train_step(plan, params, adam_m, adam_v, step, lr, x_in, sigma, target, loss, grad=None,
                   workspace=None, stream=None):
    """abcs_cnn_train_step on device tensors (float32); updates params, adam_m,
    adam_v in place when lr > 0; loss float32[1]; grad float32[params] or None."""
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().abcs_cnn_train_step(plan.handle, _ptr(params), _ptr(adam_m), _ptr(adam_v), int(step),
                                    float(lr), _ptr(x_in), _ptr(sigma), _ptr(target), _ptr(loss), _ptr(grad),
                                    _ptr(workspace), ws_bytes, _stream(stream)))


THI, THB = 1, 2
RULES = {"thi": THI, "thb": THB}


def threshold_workspace_bytes(plan):
    return int(lib().abcs_threshold_workspace_bytes(plan.handle))


def threshold(plan, px, m, out=None, rule="thi", workspace=None, stream=None):
    """abcs_threshold: full-sensing bound THI ("thi") or THB ("thb"); px uint8
    pixels, m int32[blocks] (kept per block), out float32[pixels] or None."""
    r = RULES[rule] if isinstance(rule, str) else int(rule)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().abcs_threshold(plan.handle, _ptr(px), px.numel() * px.element_size(), r, _ptr(m), _ptr(out), _ptr(workspace),
                               ws_bytes, _stream(stream)))


def budget_correlation(plan, m, m_hat, rho, p=None, stream=None):
    """abcs_budget_correlation: rho float64[n] <- Pearson(m, m_hat) per image,
    p float64[n] (or None) <- two-sided p-value of rho = 0."""
    check(lib().abcs_budget_correlation(plan.handle, _ptr(m), _ptr(m_hat), _ptr(rho), _ptr(p), _stream(stream)))


def dncnn_param_count():
    return int(lib().abcs_dncnn_param_count())


def dncnn_running_count():
    return int(lib().abcs_dncnn_running_count())


def dncnn_train_workspace_bytes(plan):
    return int(lib().abcs_dncnn_train_workspace_bytes(plan.handle))


def dncnn_train_step(plan, params, adam_m, adam_v, running, step, lr, x_in, sigma, target, loss, grad=None,
                     workspace=None, stream=None):
    """abcs_dncnn_train_step on device tensors (float32); running (or None)
    float32[running_count] is moved towards the batch statistics."""
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().abcs_dncnn_train_step(plan.handle, _ptr(params), _ptr(adam_m), _ptr(adam_v), _ptr(running),
                                      int(step), float(lr), _ptr(x_in), _ptr(sigma), _ptr(target), _ptr(loss),
                                      _ptr(grad), _ptr(workspace), ws_bytes, _stream(stream)))


WS_KINDS = {"cnn_train": 1, "dncnn_train": 2, "bm3d": 3}
WS_PARTS = {"activations": 1, "prenorm": 2, "output": 3, "groups": 4, "basic": 5}


def workspace_part(plan, kind, part):
    """abcs_workspace_part: (byte offset, bytes) of a named part of a
    workspace ('cnn_train' / 'dncnn_train' / 'bm3d'; 'activations',
    'prenorm', 'output', 'groups', 'basic')."""
    off, nb = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().abcs_workspace_part(plan.handle, WS_KINDS[kind], WS_PARTS[part], ctypes.byref(off),
                                    ctypes.byref(nb)))
    return off.value, nb.value


def dct_basis(block):
    """Host float64 DCT-II basis used by the library (B x B nested list)."""
    buf = (ctypes.c_double * (block * block))()
    check(lib().abcs_dct_basis(int(block), buf))
    return [[buf[u * block + j] for j in range(block)] for u in range(block)]


def set_launch_table(entries):
    """abcs_set_launch_table: entries of dicts with block, transform ('dct' /
    'wht' or 0 / 1), precision (PRECISIONS name or value), size_class,
    split; every split not named becomes 0 (an empty list resets)."""
    from ._native import LaunchEntry
    arr = (LaunchEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        tr = e.get("transform", "dct")
        arr[i] = LaunchEntry(int(e["block"]), TRANSFORMS[tr] if isinstance(tr, str) else int(tr),
                             _prec(e["precision"]), int(e["size_class"]), int(e["split"]))
    check(lib().abcs_set_launch_table(arr, len(entries)))


def launch_split(block, transform, precision, size_class):
    """abcs_launch_split: the split in force for a launch kind."""
    r = lib().abcs_launch_split(int(block), TRANSFORMS[transform] if isinstance(transform, str) else int(transform),
                                _prec(precision), int(size_class))
    if r < 0:
        check(r)
    return r


def plan_size_class(plan, block, transform="dct"):
    """abcs_plan_size_class: size class of the plan's tiles of one kind, or
    -1 when the plan has none."""
    r = lib().abcs_plan_size_class(plan.handle, int(block),
                                   TRANSFORMS[transform] if isinstance(transform, str) else int(transform))
    if r < -1:
        check(r)
    return r


def time_splits(plan, px, k, offsets, y, out, precision="fp32", reps=10, stream=None):
    """abcs_time_splits: mean ms per abcs_sense_decode call at splits 0, 1, 2."""
    ms = (ctypes.c_float * 3)()
    check(lib().abcs_time_splits(plan.handle, _ptr(px), px.numel() * px.element_size(), _ptr(k), _ptr(offsets),
                                 _ptr(y), _ptr(out), _prec(precision), int(reps), ms, _stream(stream)))
    return [float(v) for v in ms]


def build_id():
    """abcs_build_id: hash of the library's sources and compiler flags."""
    return lib().abcs_build_id().decode()
