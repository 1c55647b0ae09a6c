"""The FP64 oracle against what the paper's definition and mathematics fix.

The oracle is pinned here, before anything is compared with it: brute force on
tiny inputs, closed forms (tap energy, DC gain, sinusoid response, peak scale),
exact special cases (impulse), and invariants (hop subsampling, shift,
linearity, time reversal).  A second group plants typical mistakes in copies of
the C source and checks that at least one pin catches each of them.
"""
import numpy as np
import pytest

import oracle
import oracle_pins as P
from paper_2408_14302_amd import synth


@pytest.fixture(scope="module")
def o():
    return oracle.default()


@pytest.fixture(scope="module")
def clip():
    return synth.make_clip(synth.clip_seed(1, 0), 20000, 16000.0, 0.0).astype(np.float64)


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(o, pin):
    pin(o)


@pytest.mark.parametrize("pin", P.SIGNAL_PINS, ids=lambda f: f.__name__)
def test_signal_pin(o, pin, clip):
    pin(o, clip)


def test_module_functions_match_variant_api(o, clip):
    scales = [1.0, 5.0, 77.0]
    assert np.array_equal(oracle.cwt(clip, scales, 7), o.cwt(clip, scales, 7))
    assert np.array_equal(oracle.taps(3.3), o.taps(3.3))
    assert oracle.num_frames(0, 5) == 0 and oracle.num_frames(10, 5) == 2
    assert oracle.num_frames(11, 5) == 3 and oracle.num_frames(1, 512) == 1


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.cwt(np.ones(4), [1.0, -2.0], 1)
    with pytest.raises(ValueError):
        oracle.cwt(np.ones(4), [1.0], 0)
    with pytest.raises(ValueError):
        oracle.cwt(np.ones(4), [float("nan")], 1)
    with pytest.raises(ValueError):
        oracle.points(np.ones(4), [1.0], 1, [0], [4])


# Mistakes a transcription could plausibly make; each must trip some pin.
MUTATIONS = {
    "dropped_normalisation": ("t[m + M] = morlet(u) / rs;", "t[m + M] = morlet(u);"),
    "sqrt_to_linear": ("double rs = sqrt(s);", "double rs = s;"),
    "wrong_centre_freq": ("cos(5.0 * u)", "cos(6.0 * u)"),
    "gaussian_width": ("exp(-0.5 * u * u)", "exp(-u * u)"),
    "support_off_by_one": ("return (int64_t)floor(8.0 * s); }", "return (int64_t)floor(8.0 * s) - 1; }"),
    "frame_offset": ("acc[j] += tm * xp[(k0 + j) * (int64_t)hop + m];",
                     "acc[j] += tm * xp[(k0 + j) * (int64_t)hop + m + 1];"),
    "tap_reversed_index": ("double u = (double)llabs(m) / s;", "double u = (double)(m + 1) / s;"),
    "frames_floor": ("return (n + hop - 1) / hop;", "return n / hop;"),
    "hop_ignored_in_points": ("int64_t c = frame_idx[p] * (int64_t)hop;", "int64_t c = frame_idx[p];"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path, clip):
    old, new = MUTATIONS[name]
    src = oracle.source_text()
    assert old in src, name
    v = oracle.build_variant(src.replace(old, new), str(tmp_path))
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin(v)
        except (AssertionError, ValueError, IndexError):
            caught.append(pin.__name__)
    for pin in P.SIGNAL_PINS:
        try:
            pin(v, clip[:3000])
        except (AssertionError, ValueError, IndexError):
            caught.append(pin.__name__)
    assert caught, "no pin caught mutation %s" % name
