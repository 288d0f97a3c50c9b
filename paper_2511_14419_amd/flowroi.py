"""ctypes binding of libflowroi.so (C ABI in include/flowroi.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the path runs in the library's kernels.
The library must have been built (``python -m paper_2511_14419_amd.build``
or ``__graft_entry__.build()``); without it every call raises.
"""
from __future__ import annotations

import ctypes
import os
import time

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libflowroi.so")
_lib = None

ROI_OK, ROI_PRIMED, ROI_EINVAL, ROI_ENOMEM, ROI_EDEVICE, ROI_EUNSUPPORTED = 0, 1, -1, -2, -3, -4
ROI_U8, ROI_U16, ROI_F32 = 0, 1, 2
ROI_THRESH_ABS, ROI_THRESH_TOP = 0, 1
ROI_SE_SQUARE, ROI_SE_DISC = 0, 1
ROI_USE_INITIAL_FLOW, ROI_FP16_STORAGE, ROI_STABILIZE = 1, 2, 4
ROI_RULE_MAGNITUDE, ROI_RULE_SALIENCY = 0, 1

EXPORTED = [
    "roi_default_params", "roi_validate", "roi_workspace_size", "roi_mask", "roi_read_tau2",
    "roi_flow_mask_workspace_size", "roi_mask_from_flow", "roi_read_shift", "roi_phase_size",
    "roi_phase_workspace_size", "roi_phase_correlation", "roi_stream_read_shift",
    "roi_pyr_down", "roi_poly_expand", "roi_denoise", "roi_batched_workspace_size", "roi_mask_batched",
    "roi_stream_create", "roi_stream_push", "roi_stream_reset", "roi_stream_state_bytes",
    "roi_stream_destroy", "roi_stream_push_many", "roi_timing_enable", "roi_timing_read", "roi_timing_sample",
    "roi_timing_reset", "roi_timing_records", "roi_autotune", "roi_set_strip", "roi_tuned_strip", "roi_status_str",
    "roi_server_create", "roi_server_open_stream", "roi_server_close_stream", "roi_server_stream_bytes",
    "roi_server_submit", "roi_server_poll", "roi_server_drain", "roi_server_destroy",
]


class RoiError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, status_str(status), status))


class RoiParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("winsize", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("poly_n", ctypes.c_int32), ("poly_sigma", ctypes.c_float), ("eps", ctypes.c_float),
                ("thresh_mode", ctypes.c_int32), ("thresh", ctypes.c_float),
                ("dilate_radius", ctypes.c_int32), ("se_shape", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("denoise", ctypes.c_int32), ("median_radius", ctypes.c_int32), ("bilateral_radius", ctypes.c_int32),
                ("sigma_space", ctypes.c_float), ("sigma_range", ctypes.c_float), ("adjacent", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("sal_weight", ctypes.c_float), ("morph_radius", ctypes.c_int32),
                ("min_area", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RoiServerConfig(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int32), ("w", ctypes.c_int32), ("dtype", ctypes.c_int32), ("params", RoiParams),
                ("hbm_budget", ctypes.c_size_t), ("max_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("queue_depth", ctypes.c_int32)]


class RoiServerResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("stream", ctypes.c_int32), ("status", ctypes.c_int32),
                ("t_arrival", ctypes.c_double), ("t_done", ctypes.c_double), ("batch", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class RoiPair(ctypes.Structure):
    _fields_ = [("prev", ctypes.c_void_p), ("next", ctypes.c_void_p), ("flow", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("pitch", ctypes.c_int64)]


def lib():
    """Load libflowroi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libflowroi.so is not built (%s); run python -m paper_2511_14419_amd.build"
                               % _LIB_PATH)
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        pp = ctypes.POINTER(RoiParams)
        L.roi_default_params.argtypes = [pp]
        L.roi_default_params.restype = None
        L.roi_validate.argtypes = [i32, i32, i32, pp]
        L.roi_validate.restype = i32
        L.roi_workspace_size.argtypes = [i32, i32, i32, pp]
        L.roi_workspace_size.restype = sz
        L.roi_mask.argtypes = [vp, vp, i32, i32, i64, i32, pp, vp, vp, vp, sz, vp]
        L.roi_mask.restype = i32
        L.roi_read_tau2.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_float), vp]
        L.roi_read_tau2.restype = i32
        L.roi_flow_mask_workspace_size.argtypes = [i32, i32, pp]
        L.roi_flow_mask_workspace_size.restype = sz
        L.roi_mask_from_flow.argtypes = [vp, i32, i32, pp, vp, vp, vp, sz, vp]
        L.roi_mask_from_flow.restype = i32
        L.roi_read_shift.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float),
                                     vp]
        L.roi_read_shift.restype = i32
        L.roi_stream_read_shift.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                            ctypes.POINTER(ctypes.c_float), vp]
        L.roi_stream_read_shift.restype = i32
        L.roi_phase_size.argtypes = [i32, i32]
        L.roi_phase_size.restype = i32
        L.roi_phase_workspace_size.argtypes = [i32, i32]
        L.roi_phase_workspace_size.restype = sz
        L.roi_phase_correlation.argtypes = [vp, vp, i32, i32, i64, i32, vp, vp, vp, sz, vp]
        L.roi_phase_correlation.restype = i32
        L.roi_pyr_down.argtypes = [vp, i32, i32, vp, vp]
        L.roi_pyr_down.restype = i32
        L.roi_poly_expand.argtypes = [vp, i32, i32, i64, i32, pp, vp, vp]
        L.roi_poly_expand.restype = i32
        L.roi_denoise.argtypes = [vp, i32, i32, i64, i32, pp, vp, vp]
        L.roi_denoise.restype = i32
        L.roi_batched_workspace_size.argtypes = [i32, ctypes.POINTER(RoiPair), i32, pp]
        L.roi_batched_workspace_size.restype = sz
        L.roi_mask_batched.argtypes = [i32, ctypes.POINTER(RoiPair), i32, pp, vp, sz, vp]
        L.roi_mask_batched.restype = i32
        L.roi_stream_create.argtypes = [i32, i32, i32, pp, ctypes.POINTER(vp)]
        L.roi_stream_create.restype = i32
        L.roi_stream_push.argtypes = [vp, vp, i64, vp, vp, vp]
        L.roi_stream_push.restype = i32
        L.roi_stream_reset.argtypes = [vp]
        L.roi_stream_reset.restype = i32
        L.roi_stream_state_bytes.argtypes = [i32, i32, i32, pp]
        L.roi_stream_state_bytes.restype = sz
        L.roi_stream_destroy.argtypes = [vp]
        L.roi_stream_destroy.restype = None
        L.roi_stream_push_many.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64),
                                           ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i32), vp]
        L.roi_stream_push_many.restype = i32
        L.roi_timing_enable.argtypes = [i32]
        L.roi_timing_enable.restype = None
        L.roi_timing_sample.argtypes = [i32]
        L.roi_timing_sample.restype = None
        L.roi_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                      ctypes.POINTER(ctypes.c_double)]
        L.roi_timing_read.restype = i32
        L.roi_timing_records.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                         ctypes.POINTER(ctypes.c_double), i32]
        L.roi_timing_records.restype = i32
        L.roi_timing_reset.argtypes = []
        L.roi_timing_reset.restype = None
        L.roi_autotune.argtypes = [i32]
        L.roi_autotune.restype = None
        L.roi_set_strip.argtypes = [i32]
        L.roi_set_strip.restype = i32
        L.roi_tuned_strip.argtypes = [i32, i32, i32, i32]
        L.roi_tuned_strip.restype = i32
        sp = ctypes.POINTER(RoiServerConfig)
        L.roi_server_create.argtypes = [sp, ctypes.POINTER(vp)]
        L.roi_server_create.restype = i32
        L.roi_server_open_stream.argtypes = [vp, ctypes.POINTER(i32)]
        L.roi_server_open_stream.restype = i32
        L.roi_server_close_stream.argtypes = [vp, i32]
        L.roi_server_close_stream.restype = i32
        L.roi_server_stream_bytes.argtypes = [sp]
        L.roi_server_stream_bytes.restype = sz
        L.roi_server_submit.argtypes = [vp, i32, vp, i64, vp, vp, ctypes.c_uint64]
        L.roi_server_submit.restype = i32
        L.roi_server_poll.argtypes = [vp, ctypes.POINTER(RoiServerResult), i32]
        L.roi_server_poll.restype = i32
        L.roi_server_drain.argtypes = [vp]
        L.roi_server_drain.restype = i32
        L.roi_server_destroy.argtypes = [vp]
        L.roi_server_destroy.restype = None
        L.roi_status_str.argtypes = [i32]
        L.roi_status_str.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_str(s):
    return lib().roi_status_str(int(s)).decode()


def _check(s, where):
    if s < 0:
        raise RoiError(s, where)
    return s


def default_params(**kw):
    """roi_params with the library defaults, then ``kw`` overrides."""
    p = RoiParams()
    lib().roi_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def dtype_code(t):
    if t == torch.uint8:
        return ROI_U8
    if t == torch.uint16:
        return ROI_U16
    if t == torch.float32:
        return ROI_F32
    raise TypeError("frames must be uint8, uint16 or float32, got %s" % t)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _frame_pitch(t):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("frames must be 2-D with unit column stride")
    return t.stride(0)


def validate(h, w, dtype, params):
    return lib().roi_validate(h, w, dtype, ctypes.byref(params))


def workspace_size(h, w, dtype, params):
    n = lib().roi_workspace_size(h, w, dtype, ctypes.byref(params))
    if n == 0:
        raise RoiError(validate(h, w, dtype, params) or ROI_EINVAL, "roi_workspace_size")
    return n


def alloc_workspace(nbytes, device):
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def roi_mask(prev, next, params=None, flow=None, mask=None, ws=None, stream=None, want_mask=True):
    """Flow prev -> next and the RoI mask of one frame pair (device tensors).

    Returns (flow (h, w, 2) float32, mask (h, w) uint8 or None, ws)."""
    params = params or default_params()
    if prev.shape != next.shape or prev.dtype != next.dtype or prev.stride() != next.stride():
        raise ValueError("prev and next must share shape, dtype and strides")
    h, w = prev.shape
    dt = dtype_code(prev.dtype)
    dev = prev.device
    if flow is None:
        flow = torch.empty((h, w, 2), dtype=torch.float32, device=dev)
    if want_mask and mask is None:
        mask = torch.empty((h, w), dtype=torch.uint8, device=dev)
    need = workspace_size(h, w, dt, params)
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, dev)
    _check(lib().roi_mask(ctypes.c_void_p(prev.data_ptr()), ctypes.c_void_p(next.data_ptr()), h, w,
                          _frame_pitch(prev), dt, ctypes.byref(params), ctypes.c_void_p(flow.data_ptr()),
                          ctypes.c_void_p(mask.data_ptr() if mask is not None else 0),
                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "roi_mask")
    return flow, mask, ws


def read_tau2(ws, index=0, stream=None):
    v = ctypes.c_float(0.0)
    _check(lib().roi_read_tau2(ctypes.c_void_p(ws.data_ptr()), index, ctypes.byref(v), _stream(stream)),
           "roi_read_tau2")
    return v.value


def mask_from_flow(flow, params=None, want_saliency=False, ws=None, stream=None, mask=None):
    """The mask stage alone on a device flow field (h, w, 2) float32.

    Returns (mask (h, w) uint8, normalised saliency (h, w) float32 or None, ws)."""
    params = params or default_params()
    if flow.dtype != torch.float32 or flow.dim() != 3 or flow.shape[2] != 2 or not flow.is_contiguous():
        raise ValueError("flow must be a contiguous (h, w, 2) float32 tensor")
    h, w = flow.shape[:2]
    dev = flow.device
    if mask is None:
        mask = torch.empty((h, w), dtype=torch.uint8, device=dev)
    elif mask.shape != (h, w) or mask.dtype != torch.uint8 or not mask.is_contiguous():
        raise ValueError("mask must be a contiguous (h, w) uint8 tensor")
    sal = torch.empty((h, w), dtype=torch.float32, device=dev) if want_saliency else None
    need = lib().roi_flow_mask_workspace_size(h, w, ctypes.byref(params))
    if need == 0:
        raise RoiError(ROI_EINVAL, "roi_flow_mask_workspace_size")
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, dev)
    _check(lib().roi_mask_from_flow(ctypes.c_void_p(flow.data_ptr()), h, w, ctypes.byref(params),
                                    ctypes.c_void_p(mask.data_ptr()),
                                    ctypes.c_void_p(sal.data_ptr() if sal is not None else 0),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)),
           "roi_mask_from_flow")
    return mask, sal, ws


def read_shift(ws, index=0, stream=None):
    """(sy, sx, peak) of the last stabilised call on this workspace."""
    sy, sx, pk = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0.0)
    _check(lib().roi_read_shift(ctypes.c_void_p(ws.data_ptr()), index, ctypes.byref(sy), ctypes.byref(sx),
                                ctypes.byref(pk), _stream(stream)), "roi_read_shift")
    return sy.value, sx.value, pk.value


def phase_size(h, w):
    return lib().roi_phase_size(h, w)


def phase_correlation(prev, next, want_surface=True, want_aligned=True, ws=None, stream=None):
    """Stabilisation step alone on two device frames.

    Returns (sy, sx, peak, surface (P, P) float32 or None, aligned (h, w) float32 or None)."""
    if prev.shape != next.shape or prev.dtype != next.dtype or prev.stride() != next.stride():
        raise ValueError("prev and next must share shape, dtype and strides")
    h, w = prev.shape
    dev = prev.device
    P = phase_size(h, w)
    surface = torch.empty((P, P), dtype=torch.float32, device=dev) if want_surface and P > 0 else None
    aligned = torch.empty((h, w), dtype=torch.float32, device=dev) if want_aligned else None
    need = lib().roi_phase_workspace_size(h, w)
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, dev)
    _check(lib().roi_phase_correlation(ctypes.c_void_p(prev.data_ptr()), ctypes.c_void_p(next.data_ptr()), h, w,
                                       _frame_pitch(prev), dtype_code(prev.dtype),
                                       ctypes.c_void_p(surface.data_ptr() if surface is not None else 0),
                                       ctypes.c_void_p(aligned.data_ptr() if aligned is not None else 0),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)),
           "roi_phase_correlation")
    sy, sx, pk = read_shift(ws, 0, stream)
    return sy, sx, pk, surface, aligned


def pyr_down(src, stream=None):
    h, w = src.shape
    dst = torch.empty(((h + 1) // 2, (w + 1) // 2), dtype=torch.float32, device=src.device)
    _check(lib().roi_pyr_down(ctypes.c_void_p(src.data_ptr()), h, w, ctypes.c_void_p(dst.data_ptr()),
                              _stream(stream)), "roi_pyr_down")
    return dst


def poly_expand(img, params=None, stream=None):
    """(5, h, w) float32: b_x, b_y, A_xx, A_yy, A_xy."""
    params = params or default_params()
    h, w = img.shape
    coef = torch.empty((5, h, w), dtype=torch.float32, device=img.device)
    _check(lib().roi_poly_expand(ctypes.c_void_p(img.data_ptr()), h, w, _frame_pitch(img),
                                 dtype_code(img.dtype), ctypes.byref(params), ctypes.c_void_p(coef.data_ptr()),
                                 _stream(stream)), "roi_poly_expand")
    return coef


def denoise(img, params=None, stream=None):
    """Median then bilateral filter of one device frame -> (h, w) float32."""
    params = params or default_params()
    h, w = img.shape
    out = torch.empty((h, w), dtype=torch.float32, device=img.device)
    _check(lib().roi_denoise(ctypes.c_void_p(img.data_ptr()), h, w, _frame_pitch(img), dtype_code(img.dtype),
                             ctypes.byref(params), ctypes.c_void_p(out.data_ptr()), _stream(stream)), "roi_denoise")
    return out


def make_pairs(prevs, nexts, flows, masks):
    arr = (RoiPair * len(prevs))()
    for i, (p, q, f, m) in enumerate(zip(prevs, nexts, flows, masks)):
        arr[i] = RoiPair(p.data_ptr(), q.data_ptr(), f.data_ptr(), m.data_ptr(), p.shape[0], p.shape[1],
                         _frame_pitch(p))
    return arr


def batched_workspace_size(pairs, dtype, params):
    n = lib().roi_batched_workspace_size(len(pairs), pairs, dtype, ctypes.byref(params))
    if n == 0:
        raise RoiError(ROI_EINVAL, "roi_batched_workspace_size")
    return n


def roi_mask_batched(pairs, dtype, params, ws, stream=None):
    _check(lib().roi_mask_batched(len(pairs), pairs, dtype, ctypes.byref(params), ctypes.c_void_p(ws.data_ptr()),
                                  ws.numel(), _stream(stream)), "roi_mask_batched")


class Stream:
    """One camera stream: previous frame's expansion resident on the device."""

    def __init__(self, h, w, dtype, params=None):
        self.params = params or default_params()
        self.h, self.w, self.dtype = h, w, dtype
        ctx = ctypes.c_void_p()
        _check(lib().roi_stream_create(h, w, dtype, ctypes.byref(self.params), ctypes.byref(ctx)),
               "roi_stream_create")
        self.ctx = ctx

    @staticmethod
    def state_bytes(h, w, dtype, params):
        return lib().roi_stream_state_bytes(h, w, dtype, ctypes.byref(params))

    def push(self, frame, flow=None, mask=None, stream=None):
        """Returns ROI_PRIMED (first frame) or ROI_OK."""
        return _check(lib().roi_stream_push(self.ctx, ctypes.c_void_p(frame.data_ptr()), _frame_pitch(frame),
                                            ctypes.c_void_p(flow.data_ptr() if flow is not None else 0),
                                            ctypes.c_void_p(mask.data_ptr() if mask is not None else 0),
                                            _stream(stream)), "roi_stream_push")

    def read_shift(self, stream=None):
        """(sy, sx, peak) that stabilisation applied to the last pushed frame."""
        sy, sx, pk = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0.0)
        _check(lib().roi_stream_read_shift(self.ctx, ctypes.byref(sy), ctypes.byref(sx), ctypes.byref(pk),
                                           _stream(stream)), "roi_stream_read_shift")
        return sy.value, sx.value, pk.value

    def reset(self):
        _check(lib().roi_stream_reset(self.ctx), "roi_stream_reset")

    def close(self):
        if self.ctx:
            lib().roi_stream_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def push_many(streams, frames, flows, masks, stream=None):
    n = len(streams)
    V = ctypes.c_void_p * n
    st = (ctypes.c_int32 * n)()
    _check(lib().roi_stream_push_many(n, V(*[s.ctx for s in streams]), V(*[f.data_ptr() for f in frames]),
                                      (ctypes.c_int64 * n)(*[_frame_pitch(f) for f in frames]),
                                      V(*[f.data_ptr() for f in flows]), V(*[m.data_ptr() for m in masks]),
                                      st, _stream(stream)), "roi_stream_push_many")
    return list(st)


def timing_enable(on=True, per_call=False, every=1):
    """Iteration-kernel timing: off, per launch, or (per_call) one bracket
    around each call's run of iteration launches, on every `every`-th call."""
    lib().roi_timing_sample(every)
    lib().roi_timing_enable((2 if per_call else 1) if on else 0)


def timing_reset():
    lib().roi_timing_reset()


def timing_read():
    """(kernel ms, launches, output pixels, algorithmic bytes) of the iteration kernel."""
    ms, n, px, b = ctypes.c_double(0), ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_double(0)
    _check(lib().roi_timing_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(px), ctypes.byref(b)),
           "roi_timing_read")
    return ms.value, n.value, px.value, b.value


def timing_records():
    """[(kernel ms, output pixels, algorithmic bytes)] of every timed iteration launch."""
    n = lib().roi_timing_records(None, None, None, 0)
    if n < 0:
        raise RoiError(ROI_EDEVICE, "roi_timing_records")
    ms, px, b = (ctypes.c_double * n)(), (ctypes.c_int64 * n)(), (ctypes.c_double * n)()
    lib().roi_timing_records(ms, px, b, n)
    return list(zip(ms, px, b))


def autotune(mode=1):
    lib().roi_autotune(int(mode))


def set_strip(strip):
    _check(lib().roi_set_strip(int(strip)), "roi_set_strip")


def tuned_strip(h, w, winsize=15, fp16=False):
    return lib().roi_tuned_strip(h, w, winsize, 1 if fp16 else 0)


def server_config(h, w, dtype, params=None, hbm_budget=1 << 36, max_streams=64, max_batch=64, max_inflight=2,
                  queue_depth=8):
    return RoiServerConfig(h, w, dtype, params or default_params(), hbm_budget, max_streams, max_batch,
                           max_inflight, queue_depth)


class Server:
    """Continuous-batching server over camera streams (roi_server_* in the C ABI)."""

    def __init__(self, cfg):
        self.cfg = cfg
        srv = ctypes.c_void_p()
        _check(lib().roi_server_create(ctypes.byref(cfg), ctypes.byref(srv)), "roi_server_create")
        self.srv = srv

    @staticmethod
    def stream_bytes(cfg):
        return lib().roi_server_stream_bytes(ctypes.byref(cfg))

    def open_stream(self):
        """Stream id, or None when the HBM budget is exhausted."""
        i = ctypes.c_int32(-1)
        st = lib().roi_server_open_stream(self.srv, ctypes.byref(i))
        if st == ROI_ENOMEM:
            return None
        _check(st, "roi_server_open_stream")
        return i.value

    def close_stream(self, sid):
        _check(lib().roi_server_close_stream(self.srv, sid), "roi_server_close_stream")

    def submit(self, sid, host_frame, flow, mask, tag=0):
        """host_frame: pinned torch CPU tensor or numpy array (kept alive by the
        caller until its result is polled). Returns False when the stream's
        queue is full."""
        if hasattr(host_frame, "data_ptr"):
            ptr, pitch = host_frame.data_ptr(), host_frame.stride(0)
        else:
            ptr, pitch = host_frame.ctypes.data, host_frame.strides[0] // host_frame.itemsize
        st = lib().roi_server_submit(self.srv, sid, ctypes.c_void_p(ptr), pitch, ctypes.c_void_p(flow.data_ptr()),
                                     ctypes.c_void_p(mask.data_ptr() if mask is not None else 0), tag)
        if st == ROI_ENOMEM:
            return False
        _check(st, "roi_server_submit")
        return True

    def poll(self, max_results=1024):
        buf = (RoiServerResult * max_results)()
        n = lib().roi_server_poll(self.srv, buf, max_results)
        return [{"tag": buf[i].tag, "stream": buf[i].stream, "status": buf[i].status,
                 "t_arrival": buf[i].t_arrival, "t_done": buf[i].t_done, "batch": buf[i].batch} for i in range(n)]

    def drain(self):
        _check(lib().roi_server_drain(self.srv), "roi_server_drain")

    def close(self):
        if self.srv:
            lib().roi_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def steady_now():
    """Seconds on the same steady clock as the server's time stamps."""
    return time.monotonic()
