"""GPU parity of the steps next to the transform: decimate-then-transform
(Sec. III-B reading), against the FP64 oracle in oracle/transforms.py."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_close, errors, gain, torch_cuda
from oracle import transforms as T
from paper_2408_14302_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cw():
    from paper_2408_14302_amd import cwth
    return cwth


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _dec_bound(h, xmax):
    # L FP32 products summed in any fixed order (an ascending chain, or
    # interleaved partial sums and a butterfly for long filters) plus the FP32
    # rounding of the taps: |err| <= (L + 1) * 2^-24 * sum|h| * max|x|
    return (len(h) + 1) * 2.0 ** -24 * float(np.abs(h).sum()) * xmax


@pytest.mark.parametrize("n", [1, 2, 7, 16000, 160001])
@pytest.mark.parametrize("factor", [1, 2, 3, 8, 64, 512])
@pytest.mark.parametrize("filtered", [False, True])
def test_decimate_matches_oracle(torch, cw, n, factor, filtered):
    x = synth.make_clip(900 + n, n, 16000.0, 0.0)
    h = T.lowpass_fir(factor, 8 * factor + 1) if filtered else np.ones(1)
    ref = T.decimate(x.astype(np.float64), factor, h)
    got = cw.decimate(_dev(torch, x), factor, _dev(torch, h)).cpu().numpy()
    assert got.shape == ref.shape == (cw.decimated_length(n, factor),)
    rel, mab = errors(got, ref)
    bound = _dec_bound(h, float(np.abs(x).max()))
    print("decimate n=%d factor=%d filtered=%s max-abs %.2e (bound %.2e) rel-L2 %.2e" % (n, factor, filtered, mab,
                                                                                         bound, rel))
    assert mab <= bound
    if not filtered:
        np.testing.assert_array_equal(got, x[::factor])     # plain decimation is a copy


def test_decimate_empty_and_invalid(torch, cw):
    x = torch.zeros(10, device="cuda")
    h2 = torch.ones(2, device="cuda")
    with pytest.raises(cw.CwtError):
        cw.decimate(x, 2, h2)                                # even filter length
    with pytest.raises(cw.CwtError):
        cw.decimate(x, 0)
    assert cw.decimate(torch.zeros(0, device="cuda"), 3).numel() == 0


@pytest.mark.parametrize("factor,filtered", [(2, False), (4, True), (16, True), (64, False)])
def test_decimate_then_transform_matches_oracle(torch, cw, factor, filtered):
    n = 48000
    x = synth.make_clip(950 + factor, n, 16000.0, 0.0)
    scales = np.arange(1, 65, dtype=np.float64)
    h = T.lowpass_fir(factor, 8 * factor + 1) if filtered else None
    ref = T.decimated_cwt(x.astype(np.float64), scales, factor, h)
    y = cw.decimate(_dev(torch, x), factor, None if h is None else _dev(torch, h))
    plan = cw.Plan(16000.0 / factor, scales / factor, 1, "bf16", signed=True)
    got = plan(y).cpu().numpy()
    assert got.shape == ref.shape
    assert_close("bf16", got, ref, "decimate %d then transform" % factor,
                 scale=gain(scales / factor, float(np.abs(x).max())))


# ---------------------------------------------------------------------------
# Scalogram to image.  Same float32 scalogram in, so the bound is the FP32
# arithmetic: D carries a few ulp of its magnitude (log10f <= 2 ulp, x20, the
# bilinear sum), |D| <= 20 log10(1/amin) = 120 dB at amin = 1e-6 (ulp 7.6e-6),
# so pixels agree within 8 ulp(120) / (max D - min D) <= 2e-6 for a dB range
# of 30 or more; the test allows 2e-5.

IMG_TOL = 2e-5


@pytest.mark.parametrize("shape,size", [((128, 16000), (224, 224)), ((64, 313), (224, 224)), ((8, 50), (100, 300)),
                                        ((128, 160000), (224, 224)), ((1, 1), (3, 3)), ((32, 40), (32, 40))])
def test_image_matches_oracle_on_the_same_scalogram(torch, cw, shape, size):
    rng = np.random.default_rng(shape[1])
    w = (rng.standard_normal(shape) * np.exp(rng.uniform(-8, 0, shape))).astype(np.float32)
    w[0, 0] = 0.0                                     # below the floor
    ref = T.scalogram_image(w.astype(np.float64), 1e-6, *size)
    got = cw.scalogram_image(_dev(torch, w), *size, amin=1e-6).cpu().numpy()
    rel, mab = errors(got, ref)
    print("image %s -> %s max-abs %.2e rel-L2 %.2e" % (shape, size, mab, rel))
    assert got.shape == tuple(size) and mab <= IMG_TOL


def test_image_of_a_transform_end_to_end(torch, cw):
    # signal -> plain FP32 transform on the device -> image, against the FP64
    # oracle's transform and image: the FP32 path's relative error ~1e-6 moves
    # a dB value by ~1e-5 dB except next to zeros of W, which the floor bounds
    x = synth.make_clip(990, 32000, 16000.0, 0.0)
    scales = np.arange(1, 65, dtype=np.float64)
    plan = cw.Plan(16000.0, scales, 1, "fp32")
    got = cw.scalogram_image(plan(_dev(torch, x)), 224, 224, amin=1e-6).cpu().numpy()
    ref = T.scalogram_image(oracle.cwt(x.astype(np.float64), scales, 1), 1e-6, 224, 224)
    rel, mab = errors(got, ref)
    print("image end to end (fp32): max-abs %.2e rel-L2 %.2e" % (mab, rel))
    assert rel <= 1e-4 and np.median(np.abs(got - ref)) <= 1e-5


def test_image_invalid_arguments(torch, cw):
    w = torch.ones((4, 5), device="cuda")
    with pytest.raises(cw.CwtError):
        cw.scalogram_image(w, 0, 3)
    with pytest.raises(cw.CwtError):
        cw.scalogram_image(w, 3, 3, amin=0.0)
    img = cw.scalogram_image(w, 3, 3)
    torch.cuda.synchronize()
    assert float(img.abs().max()) == 0.0              # constant scalogram -> zeros
