"""FP64 CPU oracle for the steps next to the hop-strided CWT: decimation
(the decimate-then-transform reading of the paper's workflow, Sec. III-B),
the scalogram-to-image step (Sec. II-A, Fig. 1 and Sec. III-B: scalograms
become CNN input images) and the DWT scalogram (Sec. II-A, Fig. 1c).

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


# ---------------------------------------------------------------------------
# DWT scalogram (Sec. II-A, Fig. 1c: the dyadic transform computed by a filter
# bank with down-sampling, its coefficients spread back over the time axis to
# form a scale-by-time matrix).  Readings: orthogonal Daubechies filters dbN
# (2N taps); periodic extension at every level, where a level of odd length is
# first made even by repeating its last sample; filters applied in correlation
# form a'[n] = sum_k h[k] a[(2n + k) mod P], d'[n] likewise with the mirror
# filter g; matrix row j (level j = 1 is the finest) holds |d_j[t >> j]| for
# t < N, i.e. each coefficient repeated over the 2^j samples it covers.

def daubechies(order: int) -> np.ndarray:
    """Lowpass dbN (2N taps, sum = sqrt(2)) by spectral factorisation: the
    roots y_i of P(y) = sum_{k<N} C(N-1+k, k) y^k map through
    z + 1/z = 2 - 4y to the roots z_i inside the unit circle, and
    H(w) = sqrt(2) ((1 + w)/2)^N prod (w - z_i)/(1 - z_i), w = z^-1."""
    order = int(order)
    if order < 1:
        raise ValueError("order >= 1")
    p = [math.comb(order - 1 + k, k) for k in range(order)]        # ascending in y
    ys = np.roots(p[::-1]) if order > 1 else np.array([])
    zs = []
    for y in ys:
        b = 2.0 - 4.0 * y
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
        zs.append(z1 if abs(z1) < 1.0 else z2)
    q = np.poly(zs)[::-1] if zs else np.array([1.0 + 0j])            # ascending in w
    q = q / np.prod([1.0 - z for z in zs]) if zs else q
    binom = np.array([math.comb(order, k) for k in range(order + 1)], dtype=np.float64) / 2.0 ** order
    h = math.sqrt(2.0) * np.convolve(binom, q.real)
    return h


def highpass(h) -> np.ndarray:
    """g[k] = (-1)^k h[L-1-k] (quadrature mirror)."""
    h = np.asarray(h, dtype=np.float64)
    return np.array([(-1.0) ** k * h[len(h) - 1 - k] for k in range(len(h))])


def dwt_level(a, h):
    """One analysis step: returns (a', d), each of length ceil(len(a) / 2)."""
    a = np.asarray(a, dtype=np.float64)
    if len(a) % 2:
        a = np.append(a, a[-1])
    P = len(a)
    g = highpass(h)
    out_a, out_d = np.zeros(P // 2), np.zeros(P // 2)
    for n in range(P // 2):
        idx = [(2 * n + k) % P for k in range(len(h))]
        out_a[n] = float(np.dot(h, a[idx]))
        out_d[n] = float(np.dot(g, a[idx]))
    return out_a, out_d


def idwt_level(a, d, h, P: int):
    """Inverse of one analysis step for an even period P (orthogonal filters)."""
    g = highpass(h)
    out = np.zeros(P)
    for n in range(len(a)):
        for k in range(len(h)):
            out[(2 * n + k) % P] += h[k] * a[n] + g[k] * d[n]
    return out


def dwt(x, h, levels: int):
    """[d_1, .., d_J], a_J."""
    a, ds = np.asarray(x, dtype=np.float64), []
    for _ in range(int(levels)):
        a, d = dwt_level(a, h)
        ds.append(d)
    return ds, a


def dwt_scalogram(x, h, levels: int) -> np.ndarray:
    """S[j-1][t] = |d_j[t >> j]| for j = 1 .. levels, t < N."""
    x = np.asarray(x, dtype=np.float64)
    ds, _ = dwt(x, h, levels)
    t = np.arange(len(x))
    return np.stack([np.abs(d[t >> (j + 1)]) for j, d in enumerate(ds)])
