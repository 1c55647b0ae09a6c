"""ctypes binding of libcwth (include/cwt.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  PyTorch supplies device memory and streams.  Importing this
module loads libcwth.so and raises ImportError if it has not been built
(``python -c "import __graft_entry__ as g; g.build()"``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcwth.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libcwth.so is not built (%s); run paper_2408_14302_amd/build.py" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

_c_plan = ctypes.c_void_p
_i32, _i64, _dbl, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p

_SIGS = {
    "cwt_plan_create": (_i32, [_dbl, _i32, _vp, _i32, _i32, _i32, ctypes.POINTER(_c_plan)]),
    "cwt_plan_set_output": (_i32, [_c_plan, _i32]),
    "cwt_plan_destroy": (_i32, [_c_plan]),
    "cwt_num_frames": (_i64, [_c_plan, _i64]),
    "cwt_plan_num_scales": (_i32, [_c_plan]),
    "cwt_plan_hop": (_i32, [_c_plan]),
    "cwt_scale_frequencies": (_i32, [_c_plan, _vp]),
    "cwt_execute": (_i32, [_c_plan, _vp, _i64, _vp, _vp]),
    "cwt_execute_batch": (_i32, [_vp, _vp, _vp, _vp, _i32, _vp]),
    "cwt_execute_batch_noalloc": (_i32, [_vp, _vp, _vp, _vp, _i32, _vp]),
    "cwt_batch_create": (_i32, [_i32, ctypes.POINTER(_vp)]),
    "cwt_batch_destroy": (_i32, [_vp]),
    "cwt_batch_execute": (_i32, [_vp, _vp, _vp, _vp, _vp, _i32, _i32, _vp]),
    "cwt_autotune": (_i32, [_c_plan, _i64, ctypes.POINTER(_i32)]),
    "cwt_autotune_batch": (_i32, [_vp, _vp, _i32, ctypes.POINTER(_i32)]),
    "cwt_plan_config": (_i32, [_c_plan]),
    "cwt_plan_num_configs": (_i32, [_c_plan]),
    "cwt_plan_config_kind": (_i32, [_c_plan, _i32]),
    "cwt_plan_launch_config": (_i32, [_c_plan, _i64, _i32]),
    "cwt_plan_set_config": (_i32, [_c_plan, _i32]),
    "cwt_plan_bank_taps": (_i32, [_c_plan, _i32, _vp, _i64]),
    "cwt_image_workspace_bytes": (_i64, []),
    "cwt_scalogram_image": (_i32, [_vp, _i32, _i64, ctypes.c_float, _vp, _i32, _i32, _vp, _vp]),
    "cwt_decimated_length": (_i64, [_i64, _i32]),
    "cwt_lowpass_fir": (_i32, [_i32, _i32, _vp]),
    "cwt_decimate": (_i32, [_vp, _i64, _i32, _vp, _i32, _vp, _vp]),
    "cwt_daubechies": (_i32, [_i32, _vp]),
    "cwt_dwt_pyramid_length": (_i64, [_i64, _i32]),
    "cwt_dwt_scalogram": (_i32, [_vp, _i64, _i32, _vp, _i32, _i32, _vp, _vp, _vp]),
    "cwt_status_string": (ctypes.c_char_p, [_i32]),
    "cwt_last_error": (ctypes.c_char_p, []),
    "cwt_version": (ctypes.c_char_p, []),
}
EXPORTS = tuple(_SIGS)
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

OK, INVALID_ARG, UNSUPPORTED, OUT_OF_MEMORY, DEVICE, INTERNAL = range(6)
DTYPES = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16x3": 3, "fp8": 4}
MORLET = 0


class CwtError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        name = _lib.cwt_status_string(self.status).decode()
        msg = _lib.cwt_last_error().decode()
        super().__init__("%s: %s (%s)" % (where, name, msg))


def _check(st: int, where: str) -> None:
    if st != OK:
        raise CwtError(st, where)


def version() -> str:
    return _lib.cwt_version().decode()


def status_string(st: int) -> str:
    return _lib.cwt_status_string(int(st)).decode()


def _alloc_stream(stream):
    """A context under which torch allocates for work queued on `stream`
    (None: the current stream).  The caching allocator ties a block to the
    stream it was allocated on; a buffer that a kernel on another stream
    writes must belong to that stream, or its memory can be handed out again
    while the kernel still runs."""
    import contextlib
    import torch
    if stream is None:
        return contextlib.nullcontext()
    if isinstance(stream, int):
        if stream == torch.cuda.current_stream().cuda_stream:
            return contextlib.nullcontext()
        return torch.cuda.stream(torch.cuda.ExternalStream(stream))
    return torch.cuda.stream(stream)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check_signal(x):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32:
        raise TypeError("x must be a float32 CUDA tensor")
    if x.dim() != 1 or not x.is_contiguous():
        raise ValueError("x must be 1-D and contiguous")


def _check_buffer(t, device, numel, name, dtype=None):
    """A caller's output or workspace: a contiguous tensor of `numel` elements
    of `dtype` (float32 by default) in the memory of `device` (the input's
    GPU).  The library receives a bare pointer, so a host tensor or another
    GPU's must be refused here."""
    import torch
    dtype = torch.float32 if dtype is None else dtype
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.device != device:
        raise ValueError("%s must be a CUDA tensor on %s" % (name, device))
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError("%s must be a contiguous %s tensor of %d elements" % (name, dtype, numel))


class Plan:
    """A resident plan: scales (samples), hop, operand dtype and output mode.

    ``plan(x)`` returns the scalogram |W| (or signed W) as a [n_scales, K]
    float32 tensor on x's device, K = ceil(len(x) / hop)."""

    def __init__(self, fs: float, scales: Sequence[float], hop: int, dtype: str = "bf16",
                 signed: bool = False):
        sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64).reshape(-1))
        if dtype not in DTYPES:
            raise ValueError("dtype must be one of %s" % sorted(DTYPES))
        h = _c_plan()
        _check(_lib.cwt_plan_create(float(fs), MORLET, sc.ctypes.data_as(_vp), int(sc.size), int(hop),
                                    DTYPES[dtype], ctypes.byref(h)), "cwt_plan_create")
        self._h = h
        self.fs = float(fs)
        self.scales = sc.copy()
        self.hop = int(hop)
        self.dtype = dtype
        self.signed = bool(signed)
        if signed:
            _check(_lib.cwt_plan_set_output(self._h, 1), "cwt_plan_set_output")

    @property
    def handle(self):
        return self._h

    @property
    def num_scales(self) -> int:
        return int(_lib.cwt_plan_num_scales(self._h))

    def num_frames(self, n: int) -> int:
        return int(_lib.cwt_num_frames(self._h, int(n)))

    def set_signed(self, signed: bool) -> None:
        _check(_lib.cwt_plan_set_output(self._h, 1 if signed else 0), "cwt_plan_set_output")
        self.signed = bool(signed)

    def frequencies(self) -> np.ndarray:
        hz = np.zeros(self.num_scales, dtype=np.float64)
        _check(_lib.cwt_scale_frequencies(self._h, hz.ctypes.data_as(_vp)), "cwt_scale_frequencies")
        return hz

    def bank_taps(self, i: int) -> np.ndarray:
        M = int(np.floor(8.0 * self.scales[i]))
        t = np.zeros(2 * M + 1, dtype=np.float64)
        _check(_lib.cwt_plan_bank_taps(self._h, int(i), t.ctypes.data_as(_vp), t.size), "cwt_plan_bank_taps")
        return t

    @property
    def config(self) -> int:
        return int(_lib.cwt_plan_config(self._h))

    def launch_config(self, n: int, clips: int = 1) -> int:
        """The configuration a launch of `clips` clips of n samples runs."""
        return int(_lib.cwt_plan_launch_config(self._h, int(n), int(clips)))

    def config_kind(self, i: int) -> int:
        """0: 32-scale-block tiles, 1: Toeplitz tiles (hop 1), -1: none."""
        return int(_lib.cwt_plan_config_kind(self._h, int(i)))

    @property
    def num_configs(self) -> int:
        return int(_lib.cwt_plan_num_configs(self._h))

    def set_config(self, i: int) -> None:
        _check(_lib.cwt_plan_set_config(self._h, int(i)), "cwt_plan_set_config")

    def autotune(self, n: int) -> int:
        """Tune the one-clip launch of n samples (cwt_autotune); returns the
        configuration such launches now run."""
        c = _i32()
        _check(_lib.cwt_autotune(self._h, int(n), ctypes.byref(c)), "cwt_autotune")
        return int(c.value)

    def output(self, n: int, device=None):
        """An uninitialised [n_scales, K] float32 output on `device` (default:
        the current GPU)."""
        import torch
        if device is None:
            device = torch.device("cuda", torch.cuda.current_device())
        return torch.empty((self.num_scales, self.num_frames(n)), dtype=torch.float32, device=device)

    def execute(self, x, out, stream=None) -> None:
        """Queue the transform of x into out (both CUDA tensors on one device)
        on `stream`."""
        _check_signal(x)
        n = x.numel()
        _check_buffer(out, x.device, self.num_scales * self.num_frames(n), "out")
        _check(_lib.cwt_execute(self._h, x.data_ptr() if n else None, n, out.data_ptr() if n else None,
                                _stream_ptr(stream)), "cwt_execute")

    def __call__(self, x, out=None, stream=None):
        """Transform x on `stream` (default: the current stream).  x must be
        ready on that stream (ordered after the work that produced it); a new
        output is allocated for that stream."""
        if out is None:
            with _alloc_stream(stream):
                out = self.output(x.numel(), device=x.device)
        self.execute(x, out, stream)
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.cwt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _arrays(plans, xs, outs):
    n = len(plans)
    if not (len(xs) == len(outs) == n):
        raise ValueError("plans, xs and outs differ in length")
    for i, (p, x, o) in enumerate(zip(plans, xs, outs)):
        _check_buffer(o, x.device, p.num_scales * p.num_frames(x.numel()), "outs[%d]" % i)
    P = (_vp * n)(*[p.handle.value for p in plans])
    X = (_vp * n)(*[x.data_ptr() if x.numel() else None for x in xs])
    L = (_i64 * n)(*[x.numel() for x in xs])
    O = (_vp * n)(*[o.data_ptr() if o.numel() else None for o in outs])
    return n, P, X, L, O


def _outs_for(plans, xs, stream=None):
    import torch
    with _alloc_stream(stream):
        return [torch.empty((p.num_scales, p.num_frames(x.numel())), dtype=torch.float32, device=x.device)
                for p, x in zip(plans, xs)]


def autotune_batch(plans, lens) -> int:
    """Tune the persistent launch of these plans and lengths
    (cwt_autotune_batch); returns the configuration such launches now run."""
    n = len(plans)
    if n != len(lens) or n < 1:
        raise ValueError("need as many lengths as plans, at least one")
    P = (_vp * n)(*[p.handle.value for p in plans])
    L = (_i64 * n)(*[int(v) for v in lens])
    c = _i32()
    _check(_lib.cwt_autotune_batch(P, L, n, ctypes.byref(c)), "cwt_autotune_batch")
    return int(c.value)


def execute_batch(plans, xs, outs=None, stream=None):
    """All clips in one persistent launch (library-owned batch context)."""
    for x in xs:
        _check_signal(x)
    if outs is None:
        outs = _outs_for(plans, xs, stream)
    n, P, X, L, O = _arrays(plans, xs, outs)
    _check(_lib.cwt_execute_batch(P, X, L, O, n, _stream_ptr(stream)), "cwt_execute_batch")
    return outs


def execute_batch_noalloc(plans, xs, outs, stream=None):
    """cwt_execute_batch_noalloc: one persistent launch that allocates no
    device memory (caller-owned outputs; at most 512 clips)."""
    for x in xs:
        _check_signal(x)
    n, P, X, L, O = _arrays(plans, xs, outs)
    _check(_lib.cwt_execute_batch_noalloc(P, X, L, O, n, _stream_ptr(stream)), "cwt_execute_batch_noalloc")
    return outs


class Batch:
    """Explicit batch context (pinned descriptors + captured HIP graph)."""

    def __init__(self, max_clips: int):
        h = _vp()
        _check(_lib.cwt_batch_create(int(max_clips), ctypes.byref(h)), "cwt_batch_create")
        self._h = h
        self.max_clips = int(max_clips)

    def __call__(self, plans, xs, outs=None, stream=None, graph: bool = True):
        for x in xs:
            _check_signal(x)
        if outs is None:
            outs = _outs_for(plans, xs, stream)
        n, P, X, L, O = _arrays(plans, xs, outs)
        _check(_lib.cwt_batch_execute(self._h, P, X, L, O, n, 1 if graph else 0, _stream_ptr(stream)),
               "cwt_batch_execute")
        return outs

    def prepare(self, plans, xs, outs=None) -> "PreparedBatch":
        """Validate and marshal a batch once.  The returned object runs it again
        (same plans and buffers) with a single library call per run."""
        for x in xs:
            _check_signal(x)
        if outs is None:
            outs = _outs_for(plans, xs)
        return PreparedBatch(self, list(plans), list(xs), list(outs))

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.cwt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PreparedBatch:
    """A marshalled batch bound to its Batch context; keeps its tensors alive."""

    def __init__(self, batch: Batch, plans, xs, outs):
        self.batch = batch
        self.plans, self.xs, self.outs = plans, xs, outs
        self._n, self._P, self._X, self._L, self._O = _arrays(plans, xs, outs)

    def run(self, stream=None, graph: bool = True):
        _check(_lib.cwt_batch_execute(self.batch._h, self._P, self._X, self._L, self._O, self._n,
                                      1 if graph else 0, _stream_ptr(stream)), "cwt_batch_execute")
        return self.outs


def decimated_length(n: int, factor: int) -> int:
    return int(_lib.cwt_decimated_length(int(n), int(factor)))


def lowpass_fir(factor: int, n_taps: int):
    """Anti-alias filter taps (numpy float64[n_taps], unit DC gain) for
    decimation by `factor` (cwt_lowpass_fir)."""
    import numpy as np
    h = np.empty(int(n_taps), dtype=np.float64)
    _check(_lib.cwt_lowpass_fir(int(factor), int(n_taps), h.ctypes.data_as(_vp)), "cwt_lowpass_fir")
    return h


def decimate(x, factor: int, h=None, out=None, stream=None):
    """y[n] = sum_j h[j] x~[n*factor + j - (len(h)-1)/2] on the device
    (cwt_decimate).  h: None (plain decimation) or a float32 CUDA tensor of odd
    length."""
    import torch
    _check_signal(x)
    if h is None:
        h = torch.ones(1, dtype=torch.float32, device=x.device)
    if not (isinstance(h, torch.Tensor) and h.is_cuda and h.device == x.device and h.dtype == torch.float32
            and h.dim() == 1 and h.is_contiguous()):
        raise TypeError("h must be a contiguous 1-D float32 tensor on the signal's GPU")
    n = x.numel()
    ny = decimated_length(n, factor)
    if ny < 0:
        raise CwtError(INVALID_ARG, "cwt_decimate")
    if out is None:
        out = torch.empty(ny, dtype=torch.float32, device=x.device)
    else:
        _check_buffer(out, x.device, ny, "out")
    _check(_lib.cwt_decimate(x.data_ptr() if n else None, n, int(factor), h.data_ptr(), h.numel(),
                             out.data_ptr() if n else None, _stream_ptr(stream)), "cwt_decimate")
    return out


def scalogram_image(w, height: int, width: int, amin: float = 1e-6, out=None, workspace=None, stream=None):
    """The scalogram as a [height, width] image in [0, 1] (cwt_scalogram_image):
    dB of |W| floored at amin, bilinear resize, min-max over the full scalogram.
    w: float32 CUDA tensor [n_scales, n_frames]."""
    import torch
    if not (isinstance(w, torch.Tensor) and w.is_cuda and w.dtype == torch.float32 and w.dim() == 2
            and w.is_contiguous()):
        raise TypeError("w must be a contiguous 2-D float32 CUDA tensor")
    if int(height) < 1 or int(width) < 1:
        raise CwtError(INVALID_ARG, "cwt_scalogram_image")
    ws_bytes = int(_lib.cwt_image_workspace_bytes())
    if out is None:
        out = torch.empty((int(height), int(width)), dtype=torch.float32, device=w.device)
    else:
        _check_buffer(out, w.device, int(height) * int(width), "out")
    if workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=w.device)
    else:
        _check_buffer(workspace, w.device, ws_bytes, "workspace", torch.uint8)
    _check(_lib.cwt_scalogram_image(w.data_ptr(), w.shape[0], w.shape[1], float(amin), out.data_ptr(), int(height),
                                    int(width), workspace.data_ptr(), _stream_ptr(stream)), "cwt_scalogram_image")
    return out


def daubechies(order: int):
    """Lowpass Daubechies filter, numpy float64[2*order] (cwt_daubechies)."""
    h = np.empty(2 * int(order), dtype=np.float64)
    _check(_lib.cwt_daubechies(int(order), h.ctypes.data_as(_vp)), "cwt_daubechies")
    return h


def dwt_pyramid_length(n: int, levels: int) -> int:
    return int(_lib.cwt_dwt_pyramid_length(int(n), int(levels)))


def dwt_levels(pyramid, n: int, levels: int):
    """Views [(a_1, d_1), .., (a_J, d_J)] into a level record (last dim)."""
    out, off = [], 0
    for j in range(1, int(levels) + 1):
        lj = (int(n) - 1 >> j) + 1
        out.append((pyramid[..., off:off + lj], pyramid[..., off + lj:off + 2 * lj]))
        off += 2 * lj
    return out


def dwt_scalogram(x, h, levels: int, out=None, pyramid=None, matrix: bool = True, stream=None):
    """DWT scalogram on the device (cwt_dwt_scalogram).  x: contiguous float32
    CUDA tensor [len] or [clips, len]; h: lowpass taps (host sequence, even
    length).  Returns (S, pyramid): S is [levels, len] or [clips, levels, len]
    (None when matrix is False), pyramid the per-level (a_j, d_j) record."""
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.dim() in (1, 2)
            and x.is_contiguous()):
        raise TypeError("x must be a contiguous 1-D or 2-D float32 CUDA tensor")
    hh = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(-1))
    clips, n = (1, x.shape[0]) if x.dim() == 1 else (x.shape[0], x.shape[1])
    plen = dwt_pyramid_length(n, levels)
    if plen < 0 or clips < 1:
        raise CwtError(INVALID_ARG, "cwt_dwt_scalogram")
    lead = () if x.dim() == 1 else (clips,)
    if pyramid is None:
        pyramid = torch.empty(lead + (plen,), dtype=torch.float32, device=x.device)
    else:
        _check_buffer(pyramid, x.device, clips * plen, "pyramid")
    if matrix and out is None:
        out = torch.empty(lead + (int(levels), n), dtype=torch.float32, device=x.device)
    elif matrix:
        _check_buffer(out, x.device, clips * int(levels) * n, "out")
    _check(_lib.cwt_dwt_scalogram(x.data_ptr(), n, clips, hh.ctypes.data_as(_vp), hh.size, int(levels),
                                  pyramid.data_ptr(), out.data_ptr() if matrix else None, _stream_ptr(stream)),
           "cwt_dwt_scalogram")
    return (out if matrix else None), pyramid


def raw():
    """The ctypes library object (for ABI-level tests)."""
    return _lib
