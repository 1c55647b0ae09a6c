"""FP64 CPU oracle for the steps next to the hop-strided CWT: decimation
(the decimate-then-transform reading of the paper's workflow, Sec. III-B),
the scalogram-to-image step (Sec. II-A, Fig. 1 and Sec. III-B: scalograms
become CNN input images) and the DWT scalogram (Sec. II-C, Fig. 1c).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's
baseline legs, never by the library; it shares no code with it.  Plain numpy
in float64, loops where they keep the definition visible.
"""
from __future__ import annotations

import math

import numpy as np

from . import cwt as _cwt


# ---------------------------------------------------------------------------
# Decimation (Sec. III-B: the signal is re-sampled, then transformed).

def decimated_length(n: int, factor: int) -> int:
    """ceil(n / factor): output sample j sits on input sample j * factor."""
    return -(-int(n) // int(factor))


def lowpass_fir(factor: int, ntaps: int) -> np.ndarray:
    """Anti-alias filter for decimation by `factor`: windowed sinc with cutoff
    fs / (2 factor), h[j] = w[j] * sinc((j - c) / factor) / factor with
    c = (ntaps - 1) / 2 and the Hamming window w[j] = 0.54 - 0.46 cos(2 pi j / (ntaps - 1)),
    scaled so that sum(h) = 1 (unit gain at DC)."""
    factor, ntaps = int(factor), int(ntaps)
    if ntaps < 1 or ntaps % 2 == 0:
        raise ValueError("ntaps must be odd and >= 1")
    if ntaps == 1:
        return np.ones(1)
    c = (ntaps - 1) / 2.0
    h = np.empty(ntaps)
    for j in range(ntaps):
        t = (j - c) / factor
        sinc = 1.0 if t == 0.0 else math.sin(math.pi * t) / (math.pi * t)
        w = 0.54 - 0.46 * math.cos(2.0 * math.pi * j / (ntaps - 1))
        h[j] = w * sinc / factor
    return h / h.sum()


def decimate(x, factor: int, h=None) -> np.ndarray:
    """y[n] = sum_j h[j] * x~[n*factor + j - c], c = (len(h) - 1) / 2, for
    n = 0 .. ceil(N / factor) - 1, x~ = x inside [0, N) and 0 outside.
    h = None is plain decimation (h = [1]: y[n] = x[n*factor])."""
    x = np.asarray(x, dtype=np.float64)
    h = np.ones(1) if h is None else np.asarray(h, dtype=np.float64)
    if len(h) % 2 == 0:
        raise ValueError("the filter length must be odd")
    factor = int(factor)
    c = (len(h) - 1) // 2
    n_out = decimated_length(len(x), factor)
    y = np.zeros(n_out)
    for n in range(n_out):
        lo = n * factor - c                      # input index of h[0]
        j0, j1 = max(0, -lo), min(len(h), len(x) - lo)
        if j1 > j0:
            y[n] = float(np.dot(h[j0:j1], x[lo + j0:lo + j1]))
    return y


def decimated_cwt(x, scales, factor: int, h=None) -> np.ndarray:
    """The decimate-then-transform route: the full (hop 1) CWT of the
    decimated signal at scales s / factor, i.e. the same scales in seconds."""
    y = decimate(x, factor, h)
    return _cwt(y, np.asarray(scales, dtype=np.float64) / factor, 1)


# ---------------------------------------------------------------------------
# Scalogram to image (Sec. II-A with Fig. 1, Sec. III-B: the scalograms are
# the CNN's input images).  Readings (the paper gives no formula): decibels
# of the magnitude with an amplitude floor, bilinear resampling with
# half-pixel centres and no anti-aliasing, min-max normalisation over the
# full-resolution image.

def to_db(w, amin: float) -> np.ndarray:
    """D = 20 log10(max(|W|, amin))."""
    return 20.0 * np.log10(np.maximum(np.abs(np.asarray(w, dtype=np.float64)), float(amin)))


def _axis_weights(n_in: int, n_out: int):
    """Source index pairs and weights of one axis: src = (dst + 0.5) * n_in / n_out - 0.5,
    clamped below at 0; i0 = floor(src), i1 = i0 + 1 unless i0 is the last index."""
    src = (np.arange(n_out, dtype=np.float64) + 0.5) * (n_in / n_out) - 0.5
    src = np.maximum(src, 0.0)
    i0 = np.floor(src).astype(np.int64)
    i0 = np.minimum(i0, n_in - 1)
    i1 = np.where(i0 < n_in - 1, i0 + 1, i0)
    lam = src - i0
    return i0, i1, lam


def bilinear(img, height: int, width: int) -> np.ndarray:
    """Bilinear resampling of a 2-D array to height x width (half-pixel centres)."""
    img = np.asarray(img, dtype=np.float64)
    r0, r1, wr = _axis_weights(img.shape[0], int(height))
    c0, c1, wc = _axis_weights(img.shape[1], int(width))
    top = img[r0][:, c0] * (1.0 - wc) + img[r0][:, c1] * wc
    bot = img[r1][:, c0] * (1.0 - wc) + img[r1][:, c1] * wc
    return top * (1.0 - wr)[:, None] + bot * wr[:, None]


def scalogram_image(w, amin: float, height: int, width: int) -> np.ndarray:
    """image = (bilinear(D) - min D) / (max D - min D), min and max over the
    full-resolution D = to_db(w, amin); all zeros when max D == min D."""
    d = to_db(w, amin)
    lo, hi = float(d.min()), float(d.max())
    b = bilinear(d, height, width)
    if hi == lo:
        return np.zeros_like(b)
    return (b - lo) / (hi - lo)
