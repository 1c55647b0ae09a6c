"""Pins of the oracle's DWT scalogram (Sec. II-A, Fig. 1c) on the CPU: the
Daubechies filters against their closed forms and defining properties, the
filter bank against the Haar closed form, perfect reconstruction, energy
conservation and polynomial annihilation, and the matrix layout against an
impulse whose scalogram is known level by level."""
import ctypes
import math

import numpy as np
import pytest

from oracle import transforms as T

R2 = math.sqrt(2.0)


def test_db1_db2_db3_closed_forms():
    np.testing.assert_allclose(T.daubechies(1), [1 / R2, 1 / R2], rtol=0, atol=2e-16)
    r3 = math.sqrt(3.0)
    db2 = np.array([1 - r3, 3 - r3, 3 + r3, 1 + r3]) / (4 * R2)
    np.testing.assert_allclose(T.daubechies(2), db2, rtol=0, atol=1e-15)
    # Daubechies' closed form for three vanishing moments, written from the
    # largest tap down; the oracle stores taps in the opposite order
    r10, q = math.sqrt(10.0), math.sqrt(5 + 2 * math.sqrt(10.0))
    db3 = np.array([1 + r10 + q, 5 + r10 + 3 * q, 10 - 2 * r10 + 2 * q,
                    10 - 2 * r10 - 2 * q, 5 + r10 - 3 * q, 1 + r10 - q]) / (16 * R2)
    np.testing.assert_allclose(T.daubechies(3), db3[::-1], rtol=0, atol=1e-15)


@pytest.mark.parametrize("order", range(1, 11))
def test_daubechies_defining_properties(order):
    # sum sqrt(2), double-shift orthonormality, `order` vanishing moments of the
    # mirror filter and minimum phase determine dbN uniquely
    h = T.daubechies(order)
    L = len(h)
    assert L == 2 * order
    assert abs(h.sum() - R2) < 1e-14
    for m in range(order):
        assert abs(np.dot(h[:L - 2 * m], h[2 * m:]) - (1.0 if m == 0 else 0.0)) < 1e-14
    g = T.highpass(h)
    u = np.arange(L) / L
    for p in range(order):
        assert abs(np.dot(g, u ** p)) < 1e-13
    # divide out (1 + w)^order; the quotient's zeros lie inside the unit circle
    q, r = np.polynomial.polynomial.polydiv(h, np.polynomial.polynomial.polypow([1.0, 1.0], order))
    assert np.abs(r).max() < 1e-8                       # division by (1+w)^N amplifies rounding
    if len(q) > 1:
        assert np.abs(np.polynomial.polynomial.polyroots(q)).max() < 1.0


def test_haar_levels_are_scaled_pair_differences_and_block_sums():
    x = np.random.default_rng(2).standard_normal(64)
    ds, a = T.dwt(x, T.daubechies(1), 3)
    np.testing.assert_allclose(ds[0], (x[0::2] - x[1::2]) / R2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(a, x.reshape(8, 8).sum(1) / R2 ** 3, rtol=0, atol=1e-14)
    b = x.reshape(16, 4)
    np.testing.assert_allclose(ds[1], (b[:, 0] + b[:, 1] - b[:, 2] - b[:, 3]) / 2, rtol=0, atol=1e-14)


@pytest.mark.parametrize("order", [1, 2, 4, 7])
def test_perfect_reconstruction_and_energy(order):
    h = T.daubechies(order)
    x = np.random.default_rng(order).standard_normal(256)
    ds, a = T.dwt(x, h, 4)
    assert [len(d) for d in ds] == [128, 64, 32, 16] and len(a) == 16
    energy = (a ** 2).sum() + sum((d ** 2).sum() for d in ds)
    assert abs(energy - (x ** 2).sum()) < 1e-10 * (x ** 2).sum()
    for d in reversed(ds):
        a = T.idwt_level(a, d, h, 2 * len(d))
    np.testing.assert_allclose(a, x, rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", [2, 3, 5])
def test_polynomials_below_the_moment_count_leave_no_interior_detail(order):
    h = T.daubechies(order)
    t = np.arange(200) / 200.0
    x = sum((-1.5) ** p * t ** p for p in range(order))        # degree order - 1
    _, d = T.dwt_level(x, h)
    interior = [n for n in range(len(d)) if 2 * n + len(h) <= len(x)]
    assert np.abs(d[interior]).max() < 1e-12
    assert np.abs(d).max() > 1e-3                          # the wrap does see the jump


def test_periodic_shift_by_two_shifts_the_coefficients_by_one():
    h = T.daubechies(4)
    x = np.random.default_rng(4).standard_normal(98)
    a0, d0 = T.dwt_level(x, h)
    a1, d1 = T.dwt_level(np.roll(x, -2), h)
    np.testing.assert_allclose(a1, np.roll(a0, -1), rtol=0, atol=1e-13)
    np.testing.assert_allclose(d1, np.roll(d0, -1), rtol=0, atol=1e-13)


def test_odd_lengths_keep_a_constant_exact():
    # repeating the last sample keeps a constant constant on every level
    for n in (1, 3, 77, 1001):
        ds, a = T.dwt(np.full(n, 0.5), T.daubechies(3), 5)
        lens = [len(d) for d in ds]
        assert lens == [math.ceil(n / 2 ** j) for j in range(1, 6)]
        assert max(np.abs(d).max() for d in ds) < 1e-14
        np.testing.assert_allclose(a, 0.5 * R2 ** 5, rtol=1e-14)


def test_scalogram_of_a_haar_impulse():
    # an impulse at t0 leaves on level j one detail coefficient of size
    # 2^(-j/2), spread over the 2^j samples of t0's dyadic block
    n, t0, J = 96, 37, 5
    x = np.zeros(n)
    x[t0] = 1.0
    S = T.dwt_scalogram(x, T.daubechies(1), J)
    assert S.shape == (J, n)
    for j in range(1, J + 1):
        ref = np.zeros(n)
        lo = (t0 >> j) << j
        ref[lo:lo + 2 ** j] = 2.0 ** (-j / 2)
        np.testing.assert_allclose(S[j - 1], ref[:n], rtol=0, atol=1e-15)


def test_scalogram_rows_repeat_each_detail_over_its_support():
    x = np.random.default_rng(8).standard_normal(333)
    h = T.daubechies(4)
    ds, _ = T.dwt(x, h, 6)
    S = T.dwt_scalogram(x, h, 6)
    for j, d in enumerate(ds, start=1):
        np.testing.assert_array_equal(S[j - 1], np.repeat(np.abs(d), 2 ** j)[:333])


def test_library_daubechies_matches_the_oracle(lib_or_skip):
    for order in range(1, 11):
        h = np.empty(2 * order)
        assert lib_or_skip.cwt_daubechies(order, h.ctypes.data_as(ctypes.c_void_p)) == 0
        np.testing.assert_allclose(h, T.daubechies(order), rtol=0, atol=1e-13)
    h = np.empty(64)
    assert lib_or_skip.cwt_daubechies(0, h.ctypes.data_as(ctypes.c_void_p)) == 1
    assert lib_or_skip.cwt_daubechies(11, h.ctypes.data_as(ctypes.c_void_p)) == 1
