"""Pins of the oracle's decimation route (decimate-then-transform reading of
Sec. III-B) and the library's host-side filter design, on the CPU."""
import numpy as np
import pytest
import scipy.signal as ss

import oracle
from oracle import transforms as T


@pytest.mark.parametrize("factor,ntaps", [(2, 17), (3, 25), (4, 33), (8, 65), (64, 513)])
def test_lowpass_fir_is_the_hamming_windowed_sinc(factor, ntaps):
    # scipy's window method with the cutoff at 1/factor of Nyquist and unit DC gain
    ref = ss.firwin(ntaps, 1.0 / factor, window="hamming")
    np.testing.assert_allclose(T.lowpass_fir(factor, ntaps), ref, rtol=0, atol=1e-15)


def test_plain_decimation_is_subsampling():
    x = np.random.default_rng(1).standard_normal(1003)
    for f in (1, 2, 5, 64, 2000):
        np.testing.assert_array_equal(T.decimate(x, f), x[::f])
        assert len(T.decimate(x, f)) == T.decimated_length(len(x), f)


@pytest.mark.parametrize("factor", [2, 3, 8])
def test_filtered_decimation_matches_upfirdn(factor):
    # symmetric filter: the centred correlation equals scipy's convolution
    # followed by downsampling, shifted by the filter's half length
    x = np.random.default_rng(factor).standard_normal(777)
    h = T.lowpass_fir(factor, 8 * factor + 1)
    c = (len(h) - 1) // 2
    full = ss.upfirdn(h, np.concatenate([x, np.zeros(c)]), up=1, down=1)
    ref = full[np.arange(T.decimated_length(len(x), factor)) * factor + c]
    np.testing.assert_allclose(T.decimate(x, factor, h), ref, rtol=0, atol=1e-13)


def test_asymmetric_filter_against_a_dense_matrix():
    # the definition as a matrix: D[n, i] = h[i - n*f + c] for the valid taps
    rng = np.random.default_rng(5)
    x, h, f = rng.standard_normal(50), rng.standard_normal(7), 3
    c = 3
    n_out = T.decimated_length(len(x), f)
    D = np.zeros((n_out, len(x)))
    for n in range(n_out):
        for i in range(len(x)):
            j = i - n * f + c
            if 0 <= j < len(h):
                D[n, i] = h[j]
    np.testing.assert_allclose(T.decimate(x, f, h), D @ x, rtol=0, atol=1e-13)


def test_unit_dc_gain_keeps_a_constant_in_the_interior():
    h = T.lowpass_fir(4, 33)
    y = T.decimate(np.full(400, 0.75), 4, h)
    np.testing.assert_allclose(y[5:-5], 0.75, rtol=0, atol=1e-14)


def test_decimated_cwt_is_the_cwt_of_the_decimated_signal_at_scaled_scales():
    x = np.random.default_rng(9).standard_normal(256)
    scales = np.array([2.0, 4.0, 8.0])
    got = T.decimated_cwt(x, scales, 2)
    ref = oracle.dense_cwt(x[::2], scales / 2, 1)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_library_filter_design_matches_the_oracle(lib_or_skip):
    import ctypes
    for f, n in ((2, 17), (5, 41), (512, 4097)):
        h = np.empty(n)
        assert lib_or_skip.cwt_lowpass_fir(f, n, h.ctypes.data_as(ctypes.c_void_p)) == 0
        np.testing.assert_allclose(h, T.lowpass_fir(f, n), rtol=0, atol=1e-15)
    h = np.empty(4)
    assert lib_or_skip.cwt_lowpass_fir(2, 4, h.ctypes.data_as(ctypes.c_void_p)) == 1   # even length
    assert lib_or_skip.cwt_lowpass_fir(0, 5, h.ctypes.data_as(ctypes.c_void_p)) == 1
    assert lib_or_skip.cwt_decimated_length(10, 3) == 4
    assert lib_or_skip.cwt_decimated_length(-1, 3) == -1


# ---------------------------------------------------------------------------
# Scalogram to image.

@pytest.mark.parametrize("shape,size", [((37, 1001), (224, 224)), ((128, 160), (64, 50)), ((8, 50), (224, 224)),
                                        ((5, 7), (5, 7)), ((1, 300), (1, 33))])
def test_bilinear_is_torch_interpolate(shape, size):
    torch = pytest.importorskip("torch")
    img = np.random.default_rng(sum(shape)).standard_normal(shape)
    ref = torch.nn.functional.interpolate(torch.from_numpy(img)[None, None], size=size, mode="bilinear",
                                          align_corners=False, antialias=False)[0, 0].numpy()
    np.testing.assert_allclose(T.bilinear(img, *size), ref, rtol=0, atol=1e-12)


def test_bilinear_reproduces_an_affine_image_when_downsampling():
    r, c = np.meshgrid(np.arange(40.0), np.arange(3000.0), indexing="ij")
    img = 0.3 * r - 0.002 * c + 7.0
    out = T.bilinear(img, 16, 200)
    rr = (np.arange(16) + 0.5) * 40 / 16 - 0.5
    cc = (np.arange(200) + 0.5) * 3000 / 200 - 0.5
    np.testing.assert_allclose(out, 0.3 * rr[:, None] - 0.002 * cc[None, :] + 7.0, rtol=0, atol=1e-11)


def test_image_identity_size_constant_and_floor():
    w = np.random.default_rng(3).standard_normal((6, 9))
    d = 20 * np.log10(np.abs(w))
    np.testing.assert_allclose(T.scalogram_image(w, 1e-12, 6, 9), (d - d.min()) / (d.max() - d.min()), atol=1e-14)
    assert np.all(T.scalogram_image(np.full((4, 5), 2.0), 1e-6, 3, 3) == 0.0)
    z = np.zeros((3, 4))
    z[1, 2] = 1.0                                   # one sample above the floor
    img = T.scalogram_image(z, 1e-3, 3, 4)          # floor -60 dB, peak 0 dB
    assert img[1, 2] == 1.0 and img.sum() == 1.0


def test_image_min_max_come_from_the_full_resolution_scalogram():
    # A 4 x 8 scalogram at -40 dB with one 0 dB coefficient, halved in both
    # directions: every output pixel averages a 2 x 2 block with weights 1/4,
    # so the spike shows at -30 dB.  Normalised over the full-resolution D
    # (-40 .. 0 dB) that pixel is 0.25 and no pixel reaches 1; normalised over
    # the resized image it would be 1.
    w = np.full((4, 8), 0.01)
    w[1, 3] = 1.0
    img = T.scalogram_image(w, 1e-6, 2, 4)
    assert img.shape == (2, 4)
    np.testing.assert_allclose(img[0, 1], 0.25, rtol=0, atol=1e-14)
    np.testing.assert_allclose(img.max(), 0.25, rtol=0, atol=1e-14)
    assert img.min() == 0.0
    # and the mirror case: a dip averaged away leaves the image minimum above 0
    w = np.full((4, 8), 1.0)
    w[2, 5] = 0.01
    img = T.scalogram_image(w, 1e-6, 2, 4)
    np.testing.assert_allclose(img[1, 2], 0.75, rtol=0, atol=1e-14)
    np.testing.assert_allclose(img.min(), 0.75, rtol=0, atol=1e-14)
    assert img.max() == 1.0


def test_decimated_cwt_reaches_the_hop_strided_transform_for_a_slow_signal():
    # Independent of the route's own code: for a signal whose spectrum lies far
    # below the decimated Nyquist rate, decimating by H and transforming at
    # scales s/H gives the hop-H transform divided by sqrt(H): both sums are
    # Riemann sums of the same integral (spacing H against 1, hence a factor
    # H), and the coarse taps carry 1/sqrt(s/H) instead of 1/sqrt(s).  For a
    # smooth, band-limited integrand the two agree to rounding at frames whose
    # support stays inside the clip; at the edges the zero padding is a jump
    # that the two spacings sample differently.
    n, H = 4096, 4
    t = np.arange(n)
    x = np.cos(2 * np.pi * t / 512.0) + 0.5 * np.sin(2 * np.pi * t / 300.0 + 0.3)
    scales = np.array([32.0, 48.0, 64.0])
    got = T.decimated_cwt(x, scales, H) * np.sqrt(H)
    ref = oracle.cwt(x, scales, H)
    k = np.arange(ref.shape[1])
    for i, s in enumerate(scales):
        M = int(8 * s)
        inner = (k * H - M >= 0) & (k * H + M < n)
        assert inner.sum() > 500
        np.testing.assert_allclose(got[i, inner], ref[i, inner], rtol=0, atol=1e-12)
