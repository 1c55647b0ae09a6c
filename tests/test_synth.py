"""The seeded input generator: determinism, achieved SNR, peak, dtype."""
import numpy as np

from paper_2408_14302_amd import synth


def test_deterministic_and_float32():
    a = synth.make_clip(123, 5000, 16000.0, 0.0)
    b = synth.make_clip(123, 5000, 16000.0, 0.0)
    c = synth.make_clip(124, 5000, 16000.0, 0.0)
    assert a.dtype == np.float32 and a.shape == (5000,)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_peak_normalised():
    for snr in (-6.0, 0.0, 6.0):
        x = synth.make_clip(7, 16000, 16000.0, snr)
        assert abs(float(np.abs(x).max()) - 1.0) < 1e-6


def test_snr_achieved():
    for snr in (-6.0, 0.0, 6.0, 3.3):
        assert abs(synth.achieved_snr_db(31, 160000, 16000.0, snr) - snr) < 0.01


def test_tone_parameters_in_range():
    for seed in range(50):
        f0, nh = synth.clip_params(seed)
        assert 50.0 <= f0 <= 500.0 and 1 <= nh <= 10


def test_lengths_and_scales():
    L = synth.batch_lengths(1, 256)
    assert L.min() >= 16000 and L.max() <= 160000 and L.size == 256
    S = synth.serving_lengths(2, 1000)
    assert S.min() >= 8000 and S.max() <= 480000
    assert 3.0 * 16000 < np.median(S) < 5.0 * 16000
    g = synth.geometric_scales(256, 1024.0)
    assert g[0] == 1.0 and g[-1] == 1024.0 and np.all(np.diff(g) > 0)
    assert np.allclose(g, 2.0 ** (10.0 * np.arange(256) / 255.0), rtol=1e-14)
    assert np.array_equal(synth.linear_scales(4), [1.0, 2.0, 3.0, 4.0])


def test_empty_clip():
    assert synth.make_clip(1, 0).size == 0
