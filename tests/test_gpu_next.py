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
