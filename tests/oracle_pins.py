"""Pins that tie the FP64 oracle to facts fixed by the paper's definition
(Sec. II-A Eq. (1) and its discretisation, Sec. II-B for the hop) and by
mathematics, not to the oracle itself.  Each pin takes an object with the
oracle's API (``taps``, ``cwt``, ``points``, ``half_width``) so that the same
checks can be run on copies of the oracle with a planted mistake.

Every function raises AssertionError when its pin fails.
"""
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "closed_forms.json")


def golden():
    with open(GOLDEN) as f:
        return {k: float(v["value"]) for k, v in json.load(f).items()}


def dense(x, scales, hop):
    """Independent brute force: explicit analysis matrix, numpy matmul."""
    import oracle
    return oracle.dense_cwt(x, scales, hop)


def pin_brute_force(o):
    """Whole W against the dense-matrix route on tiny inputs (non-integer
    scales, scales below 1/8, hops larger than N)."""
    rng = np.random.default_rng(11)
    scales = [0.1, 0.7, 1.0, 2.5, 3.7, 6.0]
    for n in (1, 2, 7, 33, 64):
        x = rng.standard_normal(n)
        for hop in (1, 2, 3, 5, 64, 100):
            a = o.cwt(x, scales, hop)
            b = dense(x, scales, hop)
            assert a.shape == b.shape == (len(scales), -(-n // hop))
            scale = max(1.0, float(np.abs(b).max()))
            assert np.abs(a - b).max() <= 1e-14 * scale, (n, hop, np.abs(a - b).max())


def pin_tap_energy(o):
    """sum_m t[m]^2 -> integral of psi^2 = (sqrt(pi)/2)(1 + e^-25) for s >= 4
    (the 1/sqrt(a) energy normalisation of Eq. (1))."""
    ref = golden()["tap_energy"]
    for s in (4.0, 6.5, 32.0, 128.0, 1024.0):
        t = o.taps(s)
        assert t.size == 2 * math.floor(8 * s) + 1
        assert abs(float(np.sum(t * t)) - ref) <= 1e-12, (s, float(np.sum(t * t)))


def pin_tap_dc(o):
    """sum_m t[m] -> sqrt(s) * sqrt(2 pi) e^-12.5 (response to a constant)."""
    ref = golden()["dc_gain_unit"]
    for s in (4.0, 16.0, 128.0, 500.3):
        t = o.taps(s)
        exp = math.sqrt(s) * ref
        assert abs(float(np.sum(t)) - exp) <= 1e-9 * exp, (s, float(np.sum(t)), exp)


def pin_impulse(o):
    """x = delta[n - n0] gives W[i, k] = t_i[n0 - k*hop] inside the support and
    0 outside: fixes tap alignment, the frame centre and the zero boundary."""
    N = 300
    scales = [0.3, 1.0, 2.0, 5.5, 17.0]
    for n0 in (0, 137, N - 1):
        x = np.zeros(N)
        x[n0] = 1.0
        for hop in (1, 4, 7, 64):
            W = o.cwt(x, scales, hop)
            K = -(-N // hop)
            for i, s in enumerate(scales):
                t = o.taps(s)
                M = (t.size - 1) // 2
                exp = np.zeros(K)
                for k in range(K):
                    d = n0 - k * hop
                    if abs(d) <= M:
                        exp[k] = t[d + M]
                assert np.array_equal(W[i], exp), (n0, hop, s)


def pin_impulse_values(o):
    """The impulse response equals psi(d/s)/sqrt(s) evaluated independently."""
    N = 129
    x = np.zeros(N)
    x[64] = 1.0
    for s in (1.0, 3.3, 8.0):
        W = o.cwt(x, [s], 1)[0]
        for k in range(N):
            d = 64 - k
            if abs(d) <= math.floor(8 * s):
                u = d / s
                exp = math.exp(-u * u / 2) * math.cos(5 * u) / math.sqrt(s)
            else:
                exp = 0.0
            assert abs(W[k] - exp) <= 1e-15 + 1e-14 * abs(exp), (s, k, W[k], exp)


def pin_hop_subsample(o, x):
    """CWTH at hop h equals the full CWT sampled every h-th column (Sec. II-B)."""
    scales = [1.0, 3.0, 8.0, 33.0, 64.0]
    full = o.cwt(x, scales, 1)
    for hop in (2, 3, 32, 64, 256, 512):
        assert np.array_equal(o.cwt(x, scales, hop), full[:, ::hop]), hop


def pin_linearity(o):
    rng = np.random.default_rng(5)
    x = rng.standard_normal(2000)
    y = rng.standard_normal(2000)
    a, b = 0.75, -2.5
    scales = [1.0, 7.0, 40.0]
    for hop in (1, 9):
        lhs = o.cwt(a * x + b * y, scales, hop)
        rhs = a * o.cwt(x, scales, hop) + b * o.cwt(y, scales, hop)
        assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


def pin_tone(o):
    """Interior response to cos(W n + phi):
    sqrt(s) sqrt(pi/2) [e^{-(sW-5)^2/2} + e^{-(sW+5)^2/2}] cos(W b + phi)."""
    g = golden()["tone_gain_unit"]
    N = 6000
    n = np.arange(N)
    for (s, Om, phi) in ((4.0, 1.25, 0.3), (16.0, 0.3, 1.1), (64.0, 0.08, -0.7), (9.5, 0.5, 2.0)):
        x = np.cos(Om * n + phi)
        hop = 3
        W = o.cwt(x, [s], hop)[0]
        M = math.floor(8 * s)
        env = math.sqrt(s) * g * (math.exp(-(s * Om - 5) ** 2 / 2) + math.exp(-(s * Om + 5) ** 2 / 2))
        ks = np.arange(W.size)
        inner = (ks * hop - M >= 0) & (ks * hop + M < N)
        exp = env * np.cos(Om * ks[inner] * hop + phi)
        err = np.abs(W[inner] - exp).max()
        assert err <= 1e-12 * max(env, 1e-3), (s, Om, err, env)


def pin_peak_scale(o):
    """|W| of a tone peaks over s at s* = ((5 + sqrt 27)/2) / W, i.e. about
    1.0196 f_c fs / f with f_c = 5/(2 pi)."""
    y = golden()["peak_y"]
    fs = 16000.0
    for f in (500.0, 320.0, 1234.0):
        Om = 2 * math.pi * f / fs
        s_star = y / Om
        scales = np.arange(max(1, int(s_star) - 6), int(s_star) + 8, dtype=np.float64)
        N = 4000
        x = np.cos(Om * np.arange(N))
        # amplitude = max over one period of |W| at interior frames
        W = o.cwt(x, scales, 1)
        c = N // 2
        per = int(math.ceil(2 * math.pi / Om)) + 2
        amp = np.abs(W[:, c:c + per]).max(axis=1)
        best = scales[int(np.argmax(amp))]
        assert best in (math.floor(s_star), math.ceil(s_star)), (f, s_star, best)
    ex = golden()["peak_example_500hz_16khz"]
    assert abs(ex - y / (2 * math.pi * 500 / 16000)) < 1e-9
    assert abs(ex / (5 / (2 * math.pi) * 16000 / 500) - 1.0196) < 5e-5


def pin_time_reversal(o):
    rng = np.random.default_rng(8)
    x = rng.standard_normal(777)
    scales = [0.5, 2.0, 13.0]
    a = o.cwt(x, scales, 1)
    b = o.cwt(x[::-1].copy(), scales, 1)[:, ::-1]
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


def pin_shift(o):
    """Delaying x by one hop moves every column by one frame (bitwise)."""
    rng = np.random.default_rng(9)
    for hop in (1, 5, 64):
        x = rng.standard_normal(1000)
        y = np.concatenate([np.zeros(hop), x])
        scales = [1.0, 6.0, 20.0]
        Wx = o.cwt(x, scales, hop)
        Wy = o.cwt(y, scales, hop)
        K = Wx.shape[1]
        assert np.array_equal(Wy[:, 1:K + 1], Wx), hop


def pin_degenerate(o):
    """N = 0 gives no frames; N = 1 gives t_i[0] x[0] = x[0]/sqrt(s);
    s < 1/8 leaves one tap."""
    assert o.cwt(np.zeros(0), [1.0, 2.0], 3).shape == (2, 0)
    W = o.cwt(np.array([0.5]), [1.0, 4.0, 0.1], 7)
    assert W.shape == (3, 1)
    assert np.allclose(W[:, 0], [0.5, 0.25, 0.5 / math.sqrt(0.1)], rtol=1e-15, atol=0)
    assert o.taps(0.1).size == 1 and o.taps(0.125).size == 3


def pin_points(o, x):
    scales = [1.0, 2.5, 30.0, 100.0]
    for hop in (1, 17, 512):
        W = o.cwt(x, scales, hop)
        rng = np.random.default_rng(hop)
        ii = rng.integers(0, len(scales), 200)
        kk = rng.integers(0, W.shape[1], 200)
        kk[:2] = [0, W.shape[1] - 1]
        assert np.array_equal(o.points(x, scales, hop, ii, kk), W[ii, kk])


ALL_PINS = [
    pin_brute_force, pin_tap_energy, pin_tap_dc, pin_impulse, pin_impulse_values,
    pin_linearity, pin_tone, pin_peak_scale, pin_time_reversal, pin_shift, pin_degenerate,
]
SIGNAL_PINS = [pin_hop_subsample, pin_points]
