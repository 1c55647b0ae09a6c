"""GPU parity of the DWT scalogram (Sec. II-A, Fig. 1c) against the FP64
oracle in oracle/transforms.py, through the C ABI (cwt_dwt_scalogram).

Error bound, level by level.  Each coefficient is an FP32 FMA chain of L
terms over the FP32 level below, with FP32-rounded taps.  With E_j the
largest error of level j and M_j the largest |a_j| of the oracle,
    E_j <= sum|h| * (E_{j-1} + (L + 1) * 2^-24 * (M_{j-1} + E_{j-1})),  E_0 = 0
(the chain's rounding is at most L * 2^-24 * sum|h v|, the taps' one more
2^-24 * sum|h v|); the mirror filter g has the same sum|g|.  The matrix is a
copy of |d_j|, so it inherits the bound of its level."""
import numpy as np
import pytest

from gpu_util import torch_cuda
from oracle import transforms as T
from paper_2408_14302_amd import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cw():
    from paper_2408_14302_amd import cwth
    return cwth


def _oracle_levels(x, h, levels):
    a, out = np.asarray(x, dtype=np.float64), []
    for _ in range(levels):
        a_next, d = T.dwt_level(a, h)
        out.append((a, a_next, d))
        a = a_next
    return out


def _bounds(levels_ref, h):
    s, L = float(np.abs(h).sum()), len(h)
    E, out = 0.0, []
    for a_prev, _, _ in levels_ref:
        M = float(np.abs(a_prev).max())
        E = s * (E + (L + 1) * U * (M + E))
        out.append(E)
    return out


def _check_clip(cw, x, h, levels, S, pyr, label):
    ref = _oracle_levels(x.astype(np.float64), h, levels)
    bounds = _bounds(ref, h)
    worst = 0.0
    for j, ((ga, gd), (_, ra, rd), bound) in enumerate(zip(cw.dwt_levels(pyr, len(x), levels), ref, bounds), 1):
        assert ga.shape == ra.shape and gd.shape == rd.shape
        ea, ed = float(np.abs(ga - ra).max()), float(np.abs(gd - rd).max())
        worst = max(worst, max(ea, ed) / bound)
        assert ea <= bound and ed <= bound, "%s level %d: %.3e %.3e > %.3e" % (label, j, ea, ed, bound)
        if S is not None:
            np.testing.assert_array_equal(S[j - 1], np.repeat(np.abs(gd), 2 ** j)[:len(x)])
    print("%s: worst error / bound %.3f (deepest bound %.2e)" % (label, worst, bounds[-1]))


CASES = [  # (n, order, levels): ragged lengths, both sides of the LDS tail (8192), deep levels of length 1,
    # fused groups ending at the last level, and signals long enough for two fused groups
    (1, 1, 1), (2, 2, 3), (3, 4, 2), (7, 4, 5), (100, 2, 6), (1001, 10, 9), (8191, 4, 13), (8192, 4, 13),
    (8193, 3, 14), (16385, 4, 12), (40000, 7, 15), (70000, 10, 4), (99999, 1, 17), (270000, 2, 6),
    (300001, 4, 9),
]


@pytest.mark.parametrize("n,order,levels", CASES)
def test_dwt_matches_oracle(torch, cw, n, order, levels):
    x = synth.make_clip(1200 + n, n, 16000.0, 0.0)
    h = T.daubechies(order)
    S, pyr = cw.dwt_scalogram(torch.from_numpy(x).cuda(), h, levels)
    assert tuple(S.shape) == (levels, n) and pyr.numel() == cw.dwt_pyramid_length(n, levels)
    _check_clip(cw, x, h, levels, S.cpu().numpy(), pyr.cpu().numpy(), "n=%d db%d J=%d" % (n, order, levels))


def test_dwt_with_a_general_filter_and_clips(torch, cw):
    # no orthogonality: exercises the mirror filter's construction and the clip stride
    rng = np.random.default_rng(77)
    h = rng.standard_normal(6)
    xs = np.stack([synth.make_clip(1300 + c, 20001, 16000.0, 0.0) for c in range(3)])
    S, pyr = cw.dwt_scalogram(torch.from_numpy(xs).cuda(), h, 6)
    assert tuple(S.shape) == (3, 6, 20001)
    S, pyr = S.cpu().numpy(), pyr.cpu().numpy()
    for c in range(3):
        _check_clip(cw, xs[c], h, 6, S[c], pyr[c], "general filter clip %d" % c)


@pytest.mark.parametrize("L", [22, 64])
def test_dwt_filter_lengths_without_a_specialised_kernel(torch, cw, L):
    h = np.random.default_rng(L).standard_normal(L) / np.sqrt(L)
    x = synth.make_clip(1350 + L, 30001, 16000.0, 0.0)
    S, pyr = cw.dwt_scalogram(torch.from_numpy(x).cuda(), h, 7)
    _check_clip(cw, x, h, 7, S.cpu().numpy(), pyr.cpu().numpy(), "filter length %d" % L)


def test_dwt_misaligned_buffers_give_identical_bits(torch, cw):
    # offset views take the unpaired, unvectorised paths; every path runs the
    # same FMA chains, so the results agree bit for bit
    n, J = 40000, 12
    h = T.daubechies(4)
    base = torch.from_numpy(synth.make_clip(1360, n + 1, 16000.0, 0.0)).cuda()
    x = base[1:]
    assert x.data_ptr() % 8 != 0
    S0, p0 = cw.dwt_scalogram(x.clone(), h, J)
    pbuf = torch.empty(cw.dwt_pyramid_length(n, J) + 1, device="cuda")
    obuf = torch.empty(J * n + 1, device="cuda")
    S1, p1 = cw.dwt_scalogram(x, h, J, out=obuf[1:], pyramid=pbuf[1:])
    assert torch.equal(p0, p1) and torch.equal(S0.reshape(-1), S1.reshape(-1))
    n2 = 40002                                        # rows not a multiple of four floats
    x2 = torch.from_numpy(synth.make_clip(1361, n2, 16000.0, 0.0)).cuda()
    S2, p2 = cw.dwt_scalogram(x2, h, J)
    _check_clip(cw, x2.cpu().numpy(), h, J, S2.cpu().numpy(), p2.cpu().numpy(), "n=%d" % n2)


def test_dwt_full_clips_of_the_transform_workload(torch, cw):
    # three 10 s clips at 16 kHz, db4, 14 levels: the configuration timed by the benchmark
    xs = np.stack([synth.make_clip(synth.clip_seed(1, c), 160000, 16000.0, snr) for c, snr in enumerate((-6, 0, 6))])
    h = T.daubechies(4)
    S, pyr = cw.dwt_scalogram(torch.from_numpy(xs).cuda(), h, 14)
    S, pyr = S.cpu().numpy(), pyr.cpu().numpy()
    for c in range(3):
        _check_clip(cw, xs[c], h, 14, S[c], pyr[c], "160000 samples clip %d" % c)


def test_dwt_large_batch_sampled_and_energy(torch, cw):
    # 256 clips: two sampled clips against the oracle; every clip keeps the
    # energy of each even-length level (orthogonal filter, periodic extension)
    n, levels, clips = 160000, 14, 256
    xs = torch.from_numpy(np.stack([synth.make_clip(1400 + (c % 8), n, 16000.0, 0.0) for c in range(clips)])).cuda()
    xs *= torch.linspace(0.5, 2.0, clips, device="cuda")[:, None]
    h = T.daubechies(4)
    S, pyr = cw.dwt_scalogram(xs, h, levels)
    for c in (0, clips - 1):
        _check_clip(cw, xs[c].cpu().numpy(), h, levels, S[c].cpu().numpy(), pyr[c].cpu().numpy(),
                    "batch clip %d" % c)
    prev = xs.double()
    for j, (a, d) in enumerate(cw.dwt_levels(pyr, n, levels), 1):
        if prev.shape[1] % 2 == 0:
            e_in = (prev ** 2).sum(1)
            e_out = (a.double() ** 2).sum(1) + (d.double() ** 2).sum(1)
            rel = float(((e_out - e_in).abs() / e_in).max())
            assert rel < 1e-5, "level %d energy %.2e" % (j, rel)
        prev = a.double()
    full = S.view(clips, levels, n)
    for j, (_, d) in enumerate(cw.dwt_levels(pyr, n, levels), 1):
        rep = d.abs().repeat_interleave(2 ** j, dim=1)[:, :n]
        assert torch.equal(full[:, j - 1], rep)


def test_dwt_pyramid_only_and_invalid_arguments(torch, cw):
    x = torch.from_numpy(synth.make_clip(1500, 5000, 16000.0, 0.0)).cuda()
    h = T.daubechies(2)
    S, pyr = cw.dwt_scalogram(x, h, 4, matrix=False)
    assert S is None
    _, pyr2 = cw.dwt_scalogram(x, h, 4)
    assert torch.equal(pyr, pyr2)
    for bad in (dict(h=np.ones(3), levels=2), dict(h=np.ones(66), levels=2), dict(h=h, levels=0),
                dict(h=h, levels=31), dict(h=np.array([1.0, np.nan]), levels=2)):
        with pytest.raises(cw.CwtError):
            cw.dwt_scalogram(x, bad["h"], bad["levels"])
    with pytest.raises(cw.CwtError):
        cw.daubechies(11)
