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


def test_clip_is_the_normalised_mix_of_its_parts():
    for snr in (-6.0, 0.0, 6.0, 3.3):
        tone, noise = synth.clip_parts(31, 160000, 16000.0, snr)
        x = synth.make_clip(31, 160000, 16000.0, snr)
        mix = tone + noise
        np.testing.assert_array_equal(x, (mix / np.abs(mix).max()).astype(np.float32))
        # the mixing SNR, measured on the parts (mean-square ratio)
        assert abs(10 * np.log10(np.mean(tone ** 2) / np.mean(noise ** 2)) - snr) < 1e-9


def test_tone_is_harmonic_and_noise_is_pink():
    fs, n = 16000.0, 160000
    for seed in (5, 31, 77):
        f0, nh = synth.clip_params(seed)
        tone, noise = synth.clip_parts(seed, n, fs, 0.0)
        # Hann-windowed spectrum: a sinusoid of amplitude a puts energy
        # n a^2 sum(w^2) / 4 into the bins within a few of its frequency
        w = np.hanning(n)
        P = np.abs(np.fft.rfft(tone * w)) ** 2
        f = np.fft.rfftfreq(n, 1.0 / fs)
        e1 = n * float(np.sum(w * w)) / 4.0
        for k in range(1, nh + 1):
            if k * f0 >= fs / 2:
                break
            band = np.abs(f - k * f0) <= 0.5
            amp = float(np.sqrt(P[band].sum() / e1))
            assert abs(amp - 1.0 / k) < 1e-3 / k, (seed, k, amp)
        off = np.ones_like(f, dtype=bool)
        for k in range(1, nh + 1):
            off &= np.abs(f - k * f0) > 0.5
        assert P[off].sum() < 1e-4 * P.sum()
        # pink: equal power per octave (power density ~ 1/f), within 20% over
        # the octaves from 20 Hz to 5.12 kHz
        p = np.abs(np.fft.rfft(noise)) ** 2
        octs = [float(p[(f >= lo) & (f < 2 * lo)].sum()) for lo in 20.0 * 2.0 ** np.arange(8)]
        assert max(octs) / min(octs) < 1.2, octs


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
