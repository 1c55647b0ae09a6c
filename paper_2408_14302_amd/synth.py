"""Seeded synthetic machine-noise clips (stand-ins for the paper's 10 s, 16 kHz
factory recordings at -6/0/6 dB SNR, Sec. III-A).

This module draws inputs only.  It holds none of the transform's arithmetic and
is shared by the library's tests, the oracle tests and the benchmark.

Recipe (one clip):
  tone  = sum_{k=1..H} (1/k) cos(2 pi k f0 n / fs + phi_k),  f0 ~ U[50, 500] Hz,
          H ~ U{1..10}, phi_k ~ U[0, 2 pi); harmonics with k f0 >= fs/2 dropped
  pink  = irfft(rfft(white Gaussian) * f^{-1/2}), DC bin set to 0
  x     = tone + g * pink,  g chosen so 10 log10(P_tone / P_noise) = SNR
          (P = mean square over the clip)
  x    /= max|x|  (peak-normalised to 1), then cast to float32.
Seeds go through numpy's PCG64.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1430200


def clip_seed(config: int, index: int) -> int:
    """Seed used for clip `index` of workload `config` (1-based configs)."""
    return SEED_BASE + 100 * int(config) + int(index)


def clip_parts(seed: int, n: int, fs: float = 16000.0, snr_db: float = 0.0):
    """The two components make_clip(seed, n, fs, snr_db) mixes, in float64 and
    before peak normalisation: (tone, noise), noise = g * pink already scaled
    to the SNR."""
    n = int(n)
    if n < 0:
        raise ValueError("n must be >= 0")
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    f0 = rng.uniform(50.0, 500.0)
    nh = int(rng.integers(1, 11))
    phases = rng.uniform(0.0, 2.0 * math.pi, size=nh)
    t = np.arange(n, dtype=np.float64) / fs
    tone = np.zeros(n, dtype=np.float64)
    for k in range(1, nh + 1):
        if k * f0 >= fs / 2.0:
            break
        tone += np.cos(2.0 * math.pi * k * f0 * t + phases[k - 1]) / k
    white = rng.standard_normal(n)
    spec = np.fft.rfft(white)
    f = np.fft.rfftfreq(n, d=1.0 / fs)
    shape = np.zeros_like(f)
    shape[1:] = 1.0 / np.sqrt(f[1:])
    pink = np.fft.irfft(spec * shape, n=n)
    p_tone = float(np.mean(tone * tone)) if n else 0.0
    p_pink = float(np.mean(pink * pink)) if n else 0.0
    if p_pink > 0.0 and p_tone > 0.0:
        g = math.sqrt(p_tone / (p_pink * 10.0 ** (snr_db / 10.0)))
    else:
        g = 1.0
    return tone, g * pink


def make_clip(seed: int, n: int, fs: float = 16000.0, snr_db: float = 0.0) -> np.ndarray:
    """One peak-normalised float32 clip of n samples."""
    n = int(n)
    if n < 0:
        raise ValueError("n must be >= 0")
    if n == 0:
        return np.zeros(0, dtype=np.float32)
    tone, noise = clip_parts(seed, n, fs, snr_db)
    x = tone + noise
    peak = float(np.max(np.abs(x)))
    if peak > 0.0:
        x = x / peak
    return x.astype(np.float32)


def clip_params(seed: int):
    """The tone parameters make_clip(seed, ...) draws: (f0, n_harmonics)."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    f0 = rng.uniform(50.0, 500.0)
    nh = int(rng.integers(1, 11))
    return f0, nh


def batch_lengths(seed: int, count: int, lo: int = 16000, hi: int = 160000) -> np.ndarray:
    """Clip lengths drawn uniformly from {lo .. hi} (batched workload)."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    return rng.integers(lo, hi + 1, size=int(count)).astype(np.int64)


def serving_lengths(seed: int, count: int, median_s: float = 4.0, sigma: float = 0.75,
                    fs: float = 16000.0, lo_s: float = 0.5, hi_s: float = 30.0) -> np.ndarray:
    """Lognormal request lengths (median 4 s, clipped to [0.5 s, 30 s])."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    z = rng.standard_normal(int(count))
    n = np.round(fs * np.exp(math.log(median_s) + sigma * z))
    return np.clip(n, lo_s * fs, hi_s * fs).astype(np.int64)


def linear_scales(count: int) -> np.ndarray:
    """Scales 1, 2, .., count (samples)."""
    return np.arange(1, int(count) + 1, dtype=np.float64)


def geometric_scales(count: int = 256, top: float = 1024.0) -> np.ndarray:
    """count scales from 1 to top, s_i = top^(i/(count-1)); endpoints exact."""
    i = np.arange(int(count), dtype=np.float64)
    s = np.exp2(np.log2(top) * i / (count - 1))
    s[0] = 1.0
    s[-1] = float(top)
    return s
