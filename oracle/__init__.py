"""FP64 CPU oracle for the hop-strided Morlet CWT (CWTH).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package; the library never does, and
the two share no code.

Two independent routes to the same definition (paper, Sec. II-A Eq. (1) and its
discretisation; Sec. II-B for the hop):

* ``cwt`` / ``points`` / ``taps`` call the plain C direct sum in
  ``cwt_oracle.c`` (FP64, ascending tap order per coefficient).
* ``dense_cwt`` builds the dense analysis matrix Psi[k, n] = psi((n - k*hop)/s)/sqrt(s)
  (zero where |n - k*hop| > floor(8 s)) with numpy and multiplies it by x.  It
  is meant for tiny inputs and is the brute-force cross-check of the C route.

Readings (the paper leaves these open): real Morlet psi(t) = exp(-t^2/2) cos(5t)
truncated to |t| <= 8 inclusive; scales in samples; zero padding outside
[0, N); frame k centred on sample k*hop; K = ceil(N / hop); no sampling-interval
factor.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cwt_oracle.c")
_LIB = os.path.join(_HERE, "libcwt_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O3, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    d, i32, i64, vp = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.cwto_half_width.argtypes = [d]
    lib.cwto_half_width.restype = i64
    lib.cwto_num_frames.argtypes = [i64, i32]
    lib.cwto_num_frames.restype = i64
    lib.cwto_taps.argtypes = [d, vp, i64]
    lib.cwto_taps.restype = i64
    lib.cwto_cwt.argtypes = [vp, i64, vp, i32, i32, vp]
    lib.cwto_cwt.restype = ctypes.c_int
    lib.cwto_points.argtypes = [vp, i64, vp, i32, i32, vp, vp, i64, vp]
    lib.cwto_points.restype = ctypes.c_int
    lib.cwto_max_threads.restype = ctypes.c_int
    lib.cwto_set_threads.argtypes = [ctypes.c_int]
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def half_width(s: float) -> int:
    """M = floor(8 s): the truncated support is m = -M .. M (L = 2M + 1 taps)."""
    return int(_load().cwto_half_width(float(s)))


def num_frames(n: int, hop: int) -> int:
    """K = ceil(n / hop) frames; frame k is centred on sample k*hop."""
    return int(_load().cwto_num_frames(int(n), int(hop)))


def taps(s: float) -> np.ndarray:
    """FP64 taps t[m + M] = psi(|m|/s)/sqrt(s), m = -M .. M (Eq. (1) with 1/sqrt(a))."""
    L = 2 * half_width(s) + 1
    t = np.empty(L, dtype=np.float64)
    r = _load().cwto_taps(float(s), _ptr(t), L)
    if r != L:
        raise ValueError("invalid scale %r" % (s,))
    return t


def _prep(x, scales, hop):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64).reshape(-1))
    if sc.size < 1 or int(hop) < 1:
        raise ValueError("need at least one scale and hop >= 1")
    return x, sc, int(hop)


def cwt(x, scales, hop: int) -> np.ndarray:
    """Signed FP64 coefficients W, row-major [n_scales][ceil(N / hop)].

    W[i, k] = sum_{m=-M_i}^{M_i} t_i[m] * x~[k*hop + m], x~ = x inside [0, N), 0 outside.
    The scalogram is abs(W).
    """
    x, sc, hop = _prep(x, scales, hop)
    K = num_frames(x.size, hop)
    W = np.zeros((sc.size, K), dtype=np.float64)
    rc = _load().cwto_cwt(_ptr(x), x.size, _ptr(sc), sc.size, hop, _ptr(W))
    if rc != 0:
        raise ValueError("oracle rejected arguments (rc=%d)" % rc)
    return W


def points(x, scales, hop: int, scale_idx, frame_idx) -> np.ndarray:
    """Signed FP64 W at the listed (scale index, frame index) pairs."""
    x, sc, hop = _prep(x, scales, hop)
    ii = np.ascontiguousarray(np.asarray(scale_idx, dtype=np.int32).reshape(-1))
    kk = np.ascontiguousarray(np.asarray(frame_idx, dtype=np.int64).reshape(-1))
    if ii.size != kk.size:
        raise ValueError("index arrays differ in length")
    out = np.zeros(ii.size, dtype=np.float64)
    rc = _load().cwto_points(_ptr(x), x.size, _ptr(sc), sc.size, hop, _ptr(ii), _ptr(kk),
                             ii.size, _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected arguments (rc=%d)" % rc)
    return out


def dense_cwt(x, scales, hop: int) -> np.ndarray:
    """Brute-force route for tiny inputs: W = Psi @ x with an explicit dense
    matrix Psi[k, n] = psi((n - k*hop)/s)/sqrt(s) * [|n - k*hop| <= floor(8 s)]."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    sc = np.asarray(scales, dtype=np.float64).reshape(-1)
    N = x.size
    K = -(-N // int(hop)) if N > 0 else 0
    W = np.zeros((sc.size, K), dtype=np.float64)
    n = np.arange(N, dtype=np.float64)
    b = np.arange(K, dtype=np.float64) * hop
    for i, s in enumerate(sc):
        d = n[None, :] - b[:, None]
        u = d / s
        psi = np.exp(-0.5 * u * u) * np.cos(5.0 * u) / np.sqrt(s)
        psi[np.abs(d) > np.floor(8.0 * s)] = 0.0
        W[i] = psi @ x
    return W


def max_threads() -> int:
    return int(_load().cwto_max_threads())


def set_threads(n: int) -> None:
    _load().cwto_set_threads(int(n))


class Variant:
    """The same API bound to another build of the C source (used by the tests
    that plant a mistake in a copy of the oracle and check the pins catch it)."""

    def __init__(self, so_path: str):
        self._lib = _bind(ctypes.CDLL(so_path))

    def half_width(self, s):
        return int(self._lib.cwto_half_width(float(s)))

    def num_frames(self, n, hop):
        return int(self._lib.cwto_num_frames(int(n), int(hop)))

    def taps(self, s):
        L = 2 * self.half_width(s) + 1
        t = np.empty(max(L, 1), dtype=np.float64)
        r = self._lib.cwto_taps(float(s), _ptr(t), L)
        if r != L:
            raise ValueError("invalid scale")
        return t

    def cwt(self, x, scales, hop):
        x, sc, hop = _prep(x, scales, hop)
        K = self.num_frames(x.size, hop)
        W = np.zeros((sc.size, K), dtype=np.float64)
        if self._lib.cwto_cwt(_ptr(x), x.size, _ptr(sc), sc.size, hop, _ptr(W)) != 0:
            raise ValueError("oracle rejected arguments")
        return W

    def points(self, x, scales, hop, scale_idx, frame_idx):
        x, sc, hop = _prep(x, scales, hop)
        ii = np.ascontiguousarray(np.asarray(scale_idx, dtype=np.int32).reshape(-1))
        kk = np.ascontiguousarray(np.asarray(frame_idx, dtype=np.int64).reshape(-1))
        out = np.zeros(ii.size, dtype=np.float64)
        if self._lib.cwto_points(_ptr(x), x.size, _ptr(sc), sc.size, hop, _ptr(ii), _ptr(kk),
                                 ii.size, _ptr(out)) != 0:
            raise ValueError("oracle rejected arguments")
        return out


def build_variant(src_text: str, out_dir: str) -> "Variant":
    """Compile a modified copy of the C source (test use only)."""
    src = os.path.join(out_dir, "variant.c")
    so = os.path.join(out_dir, "libvariant.so")
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                    "-shared", "-std=c11", "-o", so, src, "-lm"], check=True)
    return Variant(so)


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


DEFAULT = None


def default() -> "Variant":
    """The shipped oracle as a Variant object (same API as the module functions)."""
    global DEFAULT
    if DEFAULT is None:
        _load()
        DEFAULT = Variant(_LIB)
    return DEFAULT
