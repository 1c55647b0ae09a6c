"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Every case prints rel-L2 and max-abs against the oracle beside its tolerance.
Inputs are the seeded synthetic clips (tone + pink noise, peak-normalised).
"""
import ctypes
import functools
import math

import numpy as np
import pytest

import oracle
from gpu_util import DTYPES, TOL, assert_close, errors, gain, torch_cuda
from paper_2408_14302_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cw():
    from paper_2408_14302_amd import cwth
    return cwth


def gpu_run(torch, plan, x):
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    out = plan(xd)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@functools.lru_cache(maxsize=64)
def clip(config, index, n, snr):
    return synth.make_clip(synth.clip_seed(config, index), n, 16000.0, snr)


@functools.lru_cache(maxsize=32)
def oracle_full(config, index, n, snr, nscales, hop):
    x = clip(config, index, n, snr).astype(np.float64)
    return oracle.cwt(x, np.arange(1, nscales + 1, dtype=np.float64), hop)


# ---------------------------------------------------------------------------
# Wavelet bank: the stored operand values against the FP64 taps rounded once.

def _e4m3_table():
    vals = []
    for code in range(0x7F):  # positive finite codes (0x7F is NaN)
        e, m = code >> 3, code & 7
        vals.append(m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7))
    return np.array(vals)


def _round_e4m3(v):
    """Nearest e4m3 value (ties to even code), saturating at 448."""
    tab = _e4m3_table()
    a = np.minimum(np.abs(v), 448.0)
    d = np.abs(a[:, None] - tab[None, :])
    best = d.min(axis=1, keepdims=True)
    cand = d == best
    codes = np.arange(tab.size)[None, :]
    even = cand & (codes % 2 == 0)
    pick = np.where(even.any(axis=1), np.argmax(even, axis=1), np.argmax(cand, axis=1))
    return np.sign(v) * tab[pick]


def _round_bf16(v):
    """RNE of float64 to bfloat16 by integer arithmetic on the IEEE bits."""
    b = np.asarray(v, dtype=np.float64).view(np.uint64)
    keep = b >> np.uint64(45)
    rem = b & np.uint64((1 << 45) - 1)
    half = np.uint64(1 << 44)
    up = (rem > half) | ((rem == half) & ((keep & np.uint64(1)) == np.uint64(1)))
    keep = keep + up.astype(np.uint64)
    return (keep << np.uint64(45)).view(np.float64)


def _expected_bank(dt, t, alpha=None):
    if dt == "fp32":
        return t.astype(np.float32).astype(np.float64)
    if dt == "fp16":
        return t.astype(np.float16).astype(np.float64)
    if dt == "bf16":
        return _round_bf16(t)
    if dt == "bf16x3":
        hi = _round_bf16(t)
        return hi + _round_bf16(t - hi)
    return _round_e4m3(t * alpha) / alpha


@pytest.mark.parametrize("dt", DTYPES)
def test_bank_matches_fp64_taps(torch, cw, dt):
    scales = [0.1, 1.0, 2.5, 7.3, 32.0, 128.0, 77.7, 300.0]
    plan = cw.Plan(16000.0, scales, 1, dt)
    for i, s in enumerate(scales):
        t = oracle.taps(s)
        got = plan.bank_taps(i)
        alpha = None
        if dt == "fp8":
            m, e = math.frexp(448.0 * math.sqrt(s))
            alpha = math.ldexp(1.0, e - 1)
        exp = _expected_bank(dt, t, alpha)
        # The device evaluates exp/cos in FP64 too; allow the neighbouring
        # value only where the FP64 tap sits within 1e-13 (relative) of a
        # rounding boundary of the operand format.
        bad = got != exp
        if bad.any():
            tt = t[bad]
            lo = _expected_bank(dt, tt * (1 - 1e-13), alpha)
            hi = _expected_bank(dt, tt * (1 + 1e-13), alpha)
            ok = (got[bad] == lo) | (got[bad] == hi)
            assert ok.all(), (dt, s, np.flatnonzero(bad)[~ok][:5], got[bad][~ok][:5], exp[bad][~ok][:5])
        print("bank %-6s s=%-6g taps %d mismatches-at-boundary %d" % (dt, s, t.size, int(bad.sum())))


# ---------------------------------------------------------------------------
# The measured configurations.

@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("hop", [1, 64])
def test_one_second_clip_32_scales(torch, cw, dt, hop):
    """1 s at 16 kHz, linear scales 1..32, hop 1 and 64, SNR 0 dB."""
    x = clip(1, 0, 16000, 0.0)
    ref = oracle_full(1, 0, 16000, 0.0, 32, hop)
    plan = cw.Plan(16000.0, np.arange(1, 33), hop, dt, signed=True)
    got = gpu_run(torch, plan, x)
    assert got.shape == ref.shape
    assert_close(dt, got, ref, "1s/32sc hop=%d" % hop, workload="1s32")


C2_CASES = ([(hop, snr) for hop in (1, 512) for snr in (-6.0, 0.0, 6.0)]
            + [(32, 0.0), (128, 0.0), (256, 0.0), (1024, 0.0)])


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("hop,snr", C2_CASES)
def test_ten_second_clip_128_scales(torch, cw, dt, hop, snr):
    """10 s at 16 kHz (160000 samples), linear scales 1..128 (up to 2049 taps)."""
    idx = {-6.0: 0, 0.0: 1, 6.0: 2}[snr]
    x = clip(2, idx, 160000, snr)
    ref = oracle_full(2, idx, 160000, snr, 128, hop)
    plan = cw.Plan(16000.0, np.arange(1, 129), hop, dt, signed=True)
    got = gpu_run(torch, plan, x)
    assert got.shape == ref.shape == (128, -(-160000 // hop))
    assert_close(dt, got, ref, "10s/128sc hop=%d snr=%g" % (hop, snr), workload="10s128")


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("hop", [1, 128, 512])
def test_ten_second_clip_magnitude_output(torch, cw, dt, hop):
    """The default output, the scalogram |W| (Sec. II-A: the image is the
    magnitude of the coefficients), against |oracle| on the 10 s / 128-scale
    clip; ||a| - |b|| <= |a - b|, so the signed bounds hold."""
    x = clip(2, 1, 160000, 0.0)
    ref = np.abs(oracle_full(2, 1, 160000, 0.0, 128, hop))
    plan = cw.Plan(16000.0, np.arange(1, 129), hop, dt)
    got = gpu_run(torch, plan, x)
    assert got.shape == ref.shape and got.min() >= 0.0
    assert_close(dt, got, ref, "10s/128sc |W| hop=%d" % hop, workload="10s128")


@pytest.mark.parametrize("hop", [1, 64])
def test_constant_input_dc_leakage(torch, cw, hop):
    """A constant input: away from the edges W = sum_m t[m], the wavelet's DC
    leakage, sqrt(2 pi s) exp(-12.5) (1.87e-5 at s = 4), a sum of taps up to
    ~0.4 that cancels to 1e-5 of their size.  BF16 operands carry 2^-9 of each
    tap and lose the value entirely; the hi+lo split keeps ~2^-17 and stays
    within its stated bound, as does FP32."""
    n = 24000
    x = np.ones(n, dtype=np.float32)
    scales = [4.0, 16.0, 64.0, 128.0]
    ref = oracle.cwt(x.astype(np.float64), scales, hop)
    K = ref.shape[1]
    k = np.arange(K) * hop
    inner = (k >= 1100) & (k < n - 1100)
    dc = np.array([math.sqrt(2 * math.pi * s) * math.exp(-12.5) for s in scales])
    np.testing.assert_allclose(ref[:, inner], np.repeat(dc[:, None], inner.sum(), 1), rtol=1e-6)
    err = {}
    for dt in ("fp32", "bf16x3", "bf16"):
        got = gpu_run(torch, cw.Plan(16000.0, scales, hop, dt, signed=True), x)
        # rel-L2 means nothing on a near-zero W: the max-abs bound (stated for
        # max|x| = 1) is the test
        mab = float(np.abs(got - ref).max())
        err[dt] = float(np.abs(got[:, inner] - ref[:, inner]).max())
        print("constant input hop=%d %-6s max-abs %.3e (tol %.1e), interior %.3e (DC %.3e .. %.3e)" % (
            hop, dt, mab, TOL[dt][1], err[dt], dc.min(), dc.max()))
        assert mab <= TOL[dt][1]
    # BF16 loses the DC value; the split products keep it
    assert err["bf16x3"] < dc.max() < err["bf16"]
    assert err["fp32"] < dc.min()


@pytest.mark.parametrize("hop", [1, 64, 512])
def test_fp8_faint_signal(torch, cw, hop):
    """A clip peak-normalised to 1e-37: 448 / max|x| exceeds 2^128, so the FP8
    signal scale is capped at 2^126 (the samples then reach 8.5, not 448).
    Results stay finite and, divided by 1e-37, meet the FP8 bound against the
    oracle of the same input."""
    x = (clip(1, 0, 16000, 0.0).astype(np.float64) * 1e-37).astype(np.float32)
    scales = np.arange(1, 33, dtype=np.float64)
    ref = oracle.cwt(x.astype(np.float64), scales, hop) * 1e37
    got = gpu_run(torch, cw.Plan(16000.0, scales, hop, "fp8", signed=True), x).astype(np.float64) * 1e37
    assert np.isfinite(got).all()
    assert_close("fp8", got, ref, "fp8 faint clip hop=%d" % hop)


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
@pytest.mark.parametrize("hop", [128, 512])
def test_sixty_second_48k_geometric_sampled(torch, cw, dt, hop):
    """60 s at 48 kHz (2.88 M samples), 256 geometric scales 1..1024 (up to
    16385 taps), checked on sampled coefficients the oracle computes one by one."""
    n = 2_880_000
    x = synth.make_clip(synth.clip_seed(5, 0), n, 48000.0, 0.0)
    scales = synth.geometric_scales(256, 1024.0)
    plan = cw.Plan(48000.0, scales, hop, dt, signed=True)
    got = gpu_run(torch, plan, x)
    K = -(-n // hop)
    assert got.shape == (256, K)
    rng = np.random.default_rng(hop)
    ii = rng.integers(0, 256, 3000)
    kk = rng.integers(0, K, 3000)
    ii[:8] = [0, 255, 255, 255, 128, 0, 255, 200]
    kk[:8] = [0, 0, K - 1, 1, K - 1, K - 1, K // 2, 3]
    ref = oracle.points(x.astype(np.float64), scales, hop, ii, kk)
    assert_close(dt, got[ii, kk], ref, "60s/48k/256geo hop=%d (3000 samples)" % hop, workload="60s256")


# ---------------------------------------------------------------------------
# Edge cases: ragged tails, tiny and huge hops, odd scale sets.

EDGE = [
    ("one sample", 1, [1.0, 2.0], 1),
    ("two samples", 2, [0.1, 3.0], 2),
    ("shorter than taps", 300, [100.0, 1.0], 1),
    ("hop > len", 50, [1.0, 4.0], 4099),
    ("hop = len", 4096, [2.0, 9.0], 4096),
    ("odd hop, 40 scales (2 blocks)", 5000, list(range(1, 41)), 3),
    ("hop 7, non-integer scales", 7001, list(np.linspace(0.3, 57.1, 37)), 7),
    ("hop 2", 3333, [1.0, 5.0, 30.0], 2),
    ("hop 8", 9000, [1.0, 64.0, 33.3], 8),
    ("hop 16", 9000, [1.0, 64.0, 33.3], 16),
    ("hop 24", 9000, [1.0, 64.0, 33.3], 24),
    ("hop 48 (rows staging)", 9000, [1.0, 64.0, 33.3], 48),
    ("hop 96 (even stride, unswizzled)", 20000, [1.0, 64.0, 33.3], 96),
    ("hop 192 (swizzled stride)", 40000, [1.0, 64.0, 33.3], 192),
    ("hop 384 (swizzled stride, 2 blocks)", 80000, list(range(1, 41)), 384),
    ("hop 1000", 40000, [1.0, 64.0, 128.0], 1000),
    ("duplicates, unsorted", 4000, [9.0, 1.0, 9.0, 0.05, 3.0], 5),
    ("tile tail", 128 * 3 + 5, list(range(1, 9)), 1),
    ("wide scale at hop 1 (chunked window)", 20000, [1.0, 300.0, 1024.0], 1),
    ("wide scale at hop 3 (chunked window)", 20000, [2.0, 700.0], 3),
    ("hop 2048 (row staging)", 40000, [1.0, 64.0, 512.0], 2048),
    ("hop 5000, wide scale (row staging)", 60000, [1.0, 64.0, 1024.0], 5000),
]


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("case", EDGE, ids=[e[0] for e in EDGE])
def test_edge_cases(torch, cw, dt, case):
    name, n, scales, hop = case
    x = synth.make_clip(77 + n, n, 16000.0, 0.0)
    ref = oracle.cwt(x.astype(np.float64), scales, hop)
    plan = cw.Plan(16000.0, scales, hop, dt, signed=True)
    got = gpu_run(torch, plan, x)
    assert got.shape == ref.shape
    assert_close(dt, got, ref, name, scale=gain(scales, np.abs(x).max()))


@pytest.mark.parametrize("dt", ["bf16", "fp8", "fp32"])
def test_more_than_four_blocks(torch, cw, dt):
    """200 geometric scales (7 blocks, two work-group groups), hop 96."""
    n = 50000
    x = clip(9, 0, n, 0.0)
    scales = np.geomspace(1.0, 512.0, 200)
    ref = oracle.cwt(x.astype(np.float64), scales, 96)
    plan = cw.Plan(16000.0, scales, 96, dt, signed=True)
    got = gpu_run(torch, plan, x)
    assert_close(dt, got, ref, "200 scales hop 96")


def test_empty_signal_is_noop(torch, cw):
    plan = cw.Plan(16000.0, [1.0, 2.0], 3, "bf16")
    out = plan(torch.zeros(0, device="cuda"))
    assert tuple(out.shape) == (2, 0)


@pytest.mark.parametrize("dt", ["bf16", "fp32", "fp8"])
def test_magnitude_is_abs_of_signed(torch, cw, dt):
    x = clip(1, 0, 16000, 0.0)
    p = cw.Plan(16000.0, np.arange(1, 33), 5, dt, signed=True)
    xd = torch.from_numpy(x).cuda()
    w = p(xd)
    p.set_signed(False)
    s = p(xd)
    torch.cuda.synchronize()
    assert torch.equal(s, w.abs())


# ---------------------------------------------------------------------------
# Closed forms on the device (tone response, impulse) under tolerance.

@pytest.mark.parametrize("dt", ["bf16x3", "fp32"])
def test_tone_response_on_device(torch, cw, dt):
    fs, f = 16000.0, 500.0
    Om = 2 * math.pi * f / fs
    n = 20000
    x = np.cos(Om * np.arange(n)).astype(np.float32)
    scales = np.arange(10, 42, dtype=np.float64)
    p = cw.Plan(fs, scales, 1, dt, signed=False)
    S = gpu_run(torch, p, x)
    amp = S[:, n // 2:n // 2 + 40].max(axis=1)
    s_star = (5 + math.sqrt(27)) / 2 / Om
    assert scales[int(np.argmax(amp))] in (math.floor(s_star), math.ceil(s_star))
    env = np.sqrt(scales) * math.sqrt(math.pi / 2) * (np.exp(-(scales * Om - 5) ** 2 / 2) + np.exp(-(scales * Om + 5) ** 2 / 2))
    assert np.abs(amp - env).max() < 2e-3 * env.max()


@pytest.mark.parametrize("dt", DTYPES)
def test_impulse_response_on_device(torch, cw, dt):
    n, n0 = 3000, 1234
    x = np.zeros(n, dtype=np.float32)
    x[n0] = 1.0
    scales = [1.0, 4.0, 25.0, 60.0]
    for hop in (1, 17):
        p = cw.Plan(16000.0, scales, hop, dt, signed=True)
        got = gpu_run(torch, p, x)
        for i, s in enumerate(scales):
            exp = p.bank_taps(i)
            M = (exp.size - 1) // 2
            row = np.zeros(got.shape[1])
            for k in range(row.size):
                d = n0 - k * hop
                if abs(d) <= M:
                    row[k] = exp[d + M]
            # one product per coefficient: exact except for the FP8 descale
            np.testing.assert_allclose(got[i], row, rtol=1e-6, atol=1e-30)


# ---------------------------------------------------------------------------
# Determinism: the summation order is fixed, so results are bit-identical
# run to run and across kernel configurations.

@pytest.mark.parametrize("dt", ["bf16", "fp16", "bf16x3", "fp8", "fp32"])
def test_bitwise_repeatable_and_config_independent(torch, cw, dt):
    """Bit-identical run to run and across the configurations of one kind;
    the two kinds (32-scale-block and, at hop 1, Toeplitz tiles) group each
    coefficient's products differently and agree within the tolerance."""
    x = clip(2, 1, 160000, 0.0)
    xd = torch.from_numpy(x).cuda()
    for hop in (1, 3, 256, 384):
        p = cw.Plan(16000.0, np.arange(1, 129), hop, dt, signed=True)
        a = p(xd)
        b = p(xd)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        first = {p.config_kind(p.config): a}
        for c in range(p.num_configs):
            try:
                p.set_config(c)
            except cw.CwtError:
                continue
            got = p(xd)
            kind = p.config_kind(c)
            if kind in first:
                assert torch.equal(got, first[kind]), (dt, hop, c)
            else:
                first[kind] = got
        if len(first) > 1:
            assert_close(dt, first[0].cpu().numpy(), first[1].cpu().numpy(), "hop %d block vs Toeplitz tiles" % hop)
        if dt in ("bf16", "fp16"):
            assert (hop == 1) == (1 in first), (dt, hop, sorted(first))


# ---------------------------------------------------------------------------
# Batching: one persistent launch, bit-identical to the clips run alone.

def _batch_inputs(torch, seed, count, hops, lo=2000, hi=60000):
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi, count)
    hs = rng.choice(hops, count)
    xs = [torch.from_numpy(synth.make_clip(seed * 1000 + i, int(n), 16000.0, float(rng.uniform(-6, 6)))).cuda()
          for i, n in enumerate(lens)]
    return xs, [int(h) for h in hs]


@pytest.mark.parametrize("dt", ["bf16", "fp16", "bf16x3", "fp8", "fp32"])
def test_batch_bitwise_equals_single(torch, cw, dt):
    xs, hs = _batch_inputs(torch, 3, 24, [1, 3, 64, 256, 512])
    xs.append(torch.zeros(0, device="cuda"))
    hs.append(64)
    scales = np.arange(1, 129)
    plans = {h: cw.Plan(16000.0, scales, h, dt, signed=True) for h in set(hs)}
    pl = [plans[h] for h in hs]
    alone = [p(x) for p, x in zip(pl, xs)]
    outs = cw.execute_batch(pl, xs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(alone, outs)):
        assert torch.equal(a, b), (dt, i, hs[i], xs[i].numel())


@pytest.mark.parametrize("dt", ["bf16", "fp8"])
def test_batch_mixed_layouts(torch, cw, dt):
    """Whole-window, chunked-window and row-staged clips in one launch."""
    scales = [1.0, 64.0, 1024.0]
    plans = {h: cw.Plan(16000.0, scales, h, dt, signed=True) for h in (1, 64, 5000)}
    xs, hs = _batch_inputs(torch, 21, 9, [1, 64, 5000], lo=3000, hi=30000)
    pl = [plans[h] for h in hs]
    alone = [p(x) for p, x in zip(pl, xs)]
    for graph in (False, True):
        outs = cw.Batch(16)(pl, xs, graph=graph)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(alone, outs)):
            assert torch.equal(a, b), (dt, graph, i, hs[i])


def test_prepared_batches_replay(torch, cw):
    """Two marshalled batches run alternately through one context."""
    scales = np.arange(1, 129)
    plans = {h: cw.Plan(16000.0, scales, h, "bf16") for h in (64, 256, 512)}
    B = cw.Batch(48)
    sets = []
    for seed, count in ((31, 40), (32, 17)):
        xs, hs = _batch_inputs(torch, seed, count, [64, 256, 512])
        pl = [plans[h] for h in hs]
        sets.append(([p(x) for p, x in zip(pl, xs)], B.prepare(pl, xs)))
    for rep in range(3):
        for j, (alone, prep) in enumerate(sets):
            for o in prep.outs:
                o.fill_(-1.0)
            outs = prep.run(graph=True)
            torch.cuda.synchronize()
            for a, b in zip(alone, outs):
                assert torch.equal(a, b), (rep, j)


@pytest.mark.parametrize("dt", ["bf16", "fp16"])
def test_batch_of_hop1_clips_in_one_toeplitz_grid(torch, cw, dt):
    """A batch of hop-1 clips only runs their single-clip Toeplitz tiles in
    one grid (the frame tiles of all clips in one sequence): bit-identical to
    the clips launched alone, directly and as graph replays, for clips
    shorter than one tile, spanning many, and empty; the same batch among a
    hop-256 clip runs the persistent kernel, with the same bits too."""
    scales = np.arange(1, 97)
    p = cw.Plan(16000.0, scales, 1, dt, signed=True)
    p256 = cw.Plan(16000.0, scales, 256, dt, signed=True)
    lens = [3000, 16384, 16385, 40000, 170000, 90001, 0, 12345]
    xs = [torch.from_numpy(clip(2, 70 + i, n, 0.0)).cuda() if n else torch.zeros(0, device="cuda")
          for i, n in enumerate(lens)]
    alone = [p(x) for x in xs]
    outs = cw.execute_batch([p] * len(xs), xs)
    B = cw.Batch(16)
    g = B([p] * len(xs), xs, graph=True)
    g2 = B([p] * len(xs), xs, graph=True)
    mixed = cw.execute_batch([p] * len(xs) + [p256], xs + [xs[4]])
    torch.cuda.synchronize()
    for i, a in enumerate(alone):
        for b in (outs[i], g[i], g2[i], mixed[i]):
            assert torch.equal(a, b), (dt, i, lens[i])
    assert p.launch_config(160000, len(xs)) == 13


@pytest.mark.parametrize("dt", ["bf16", "fp16"])
def test_small_hop1_batches_take_smaller_toeplitz_tiles(torch, cw, dt):
    """A batch of hop-1 clips too small to give four work-groups per CU with
    16384-frame tiles runs 8192- or 4096-frame tiles in its one grid
    (configurations 14, 15), with the same bits as the clips launched alone,
    directly and as graph replays."""
    scales = np.arange(1, 97)   # 48 scale groups
    p = cw.Plan(16000.0, scales, 1, dt, signed=True)
    assert p.launch_config(40000, 6) == 14 and p.launch_config(3000, 3) == 15
    for lens in ([40000] * 6, [3000, 16385, 40000]):
        xs = [torch.from_numpy(clip(2, 90 + i, n, 0.0)).cuda() for i, n in enumerate(lens)]
        alone = [p(x) for x in xs]
        outs = cw.execute_batch([p] * len(xs), xs)
        g = cw.Batch(8)([p] * len(xs), xs, graph=True)
        torch.cuda.synchronize()
        for i, a in enumerate(alone):
            assert torch.equal(a, outs[i]) and torch.equal(a, g[i]), (dt, lens, i)


def test_prepared_batch_follows_configuration_changes(torch, cw):
    """A context runs a prepared launch again without preparing it on the
    host only while its plans, buffers and the configuration state are those
    it was prepared from: a plan moved from Toeplitz tiles to 32-scale-block
    tiles between two runs of one prepared batch runs the new tiles (the two
    kinds group the products differently, so the results change), and a new
    input written into the same buffers is transformed anew."""
    scales = np.arange(1, 65)
    p = cw.Plan(16000.0, scales, 1, "bf16", signed=True)
    assert p.config_kind(p.config) == 1
    xs = [torch.from_numpy(clip(2, 60 + i, 12000 + 1000 * i, 0.0)).cuda() for i in range(4)]
    B = cw.Batch(8)
    prep = B.prepare([p] * 4, xs)
    first = [o.clone() for o in prep.run(graph=False)]
    again = [o.clone() for o in prep.run(graph=False)]
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(first, again))
    p.set_config(6)
    blocks = [o.clone() for o in prep.run(graph=False)]
    alone = [p(x) for x in xs]
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(alone, blocks))
    assert not all(torch.equal(a, b) for a, b in zip(first, blocks))
    for a, b in zip(first, blocks):
        assert_close("bf16", a.cpu().numpy(), b.cpu().numpy(), "Toeplitz vs block tiles")
    # doubling the input doubles every product and partial sum exactly (a
    # negation would not: the matrix cores' accumulation is not symmetric in
    # sign at the last bit)
    for x in xs:
        x.mul_(2.0)
    scaled = [o.clone() for o in prep.run(graph=True)]
    torch.cuda.synchronize()
    for a, b in zip(blocks, scaled):
        assert torch.equal(2.0 * a, b)


def test_prepared_batch_from_two_streams(torch, cw):
    """A prepared batch run again from a second stream: the run reuses the
    resident descriptors, and the launches that last read them on the first
    stream are waited for before any later upload overwrites them."""
    scales = np.arange(1, 65)
    plans = {h: cw.Plan(16000.0, scales, h, "bf16") for h in (1, 256, 512)}
    B = cw.Batch(16)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    sets = []
    for seed in (51, 52):
        xs, hs = _batch_inputs(torch, seed, 10, [1, 256, 512], lo=4000, hi=40000)
        pl = [plans[h] for h in hs]
        sets.append(([p(x) for p, x in zip(pl, xs)], B.prepare(pl, xs)))
    torch.cuda.synchronize()
    for rep in range(6):
        alone, prep = sets[rep % 2 if rep < 4 else 0]
        st = streams[(rep // 2) % 2]
        with torch.cuda.stream(st):
            for o in prep.outs:
                o.fill_(-1.0)
            outs = prep.run(stream=st, graph=bool(rep % 3 == 2))
        st.synchronize()
        for a, b in zip(alone, outs):
            assert torch.equal(a, b), rep


def test_batch_context_on_two_streams(torch, cw):
    """One context fed alternately from two streams with changing batches."""
    scales = np.arange(1, 65)
    plans = {h: cw.Plan(16000.0, scales, h, "bf16") for h in (1, 64, 512)}
    B = cw.Batch(32)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    runs = []
    for rep in range(6):
        xs, hs = _batch_inputs(torch, 40 + rep % 3, 12, [1, 64, 512], lo=2000, hi=20000)
        pl = [plans[h] for h in hs]
        alone = [p(x) for p, x in zip(pl, xs)]
        torch.cuda.synchronize()
        st = streams[rep % 2]
        with torch.cuda.stream(st):
            outs = B(pl, xs, stream=st, graph=bool(rep % 2))
        runs.append((alone, outs))
    torch.cuda.synchronize()
    for rep, (alone, outs) in enumerate(runs):
        for a, b in zip(alone, outs):
            assert torch.equal(a, b), rep


def test_batch_graph_replays(torch, cw):
    scales = np.arange(1, 129)
    plans = {h: cw.Plan(16000.0, scales, h, "bf16") for h in (64, 256, 512)}
    B = cw.Batch(64)
    for rep, (seed, count) in enumerate([(5, 40), (6, 40), (7, 9), (8, 40)]):
        xs, hs = _batch_inputs(torch, seed, count, [64, 256, 512])
        pl = [plans[h] for h in hs]
        alone = [p(x) for p, x in zip(pl, xs)]
        g = B(pl, xs, graph=True)
        ng = B(pl, xs, graph=False)
        torch.cuda.synchronize()
        for a, b, c in zip(alone, g, ng):
            assert torch.equal(a, b) and torch.equal(a, c), rep


def test_batch_against_oracle(torch, cw):
    xs, hs = _batch_inputs(torch, 11, 6, [64, 256, 512], lo=16000, hi=40000)
    scales = np.arange(1, 129)
    plans = {h: cw.Plan(16000.0, scales, h, "bf16", signed=True) for h in set(hs)}
    outs = cw.execute_batch([plans[h] for h in hs], xs)
    torch.cuda.synchronize()
    for x, h, o in zip(xs, hs, outs):
        ref = oracle.cwt(x.cpu().numpy().astype(np.float64), scales, h)
        assert_close("bf16", o.cpu().numpy(), ref, "batch hop=%d" % h)


def _sampled_check(dt, got, x, scales, hop, rng, count, what, magnitude):
    """got (host array [S][K]) against the oracle on `count` sampled
    coefficients (first and last frames always included)."""
    S, K = got.shape
    ii = rng.integers(0, S, count)
    kk = rng.integers(0, K, count)
    ii[:4] = [0, S - 1, 0, S - 1]
    kk[:4] = [0, 0, K - 1, K - 1]
    ref = oracle.points(np.asarray(x, dtype=np.float64), scales, hop, ii, kk)
    if magnitude:
        ref = np.abs(ref)
    return assert_close(dt, got[ii, kk], ref, what)


def test_batch_of_256_uneven_clips_mixed_hops_graph_replays(torch, cw):
    """The batching workload at its own shape: 256 clips, lengths uniform in
    [1 s, 10 s] at 16 kHz, SNR uniform in [-6, 6] dB, hop per clip from
    {64, 256, 512}, 128 scales, BF16, |W|, tile configuration tuned on the
    batch itself, one persistent launch replayed from a captured HIP graph.  Every clip is checked against the FP64 oracle on
    2,000 sampled coefficients and four clips in full; the graph is replayed
    three times with other device work in between, each replay compared bit
    for bit with the first and with a direct launch."""
    n = 256
    lens = synth.batch_lengths(synth.clip_seed(3, 0), n)
    rng = np.random.default_rng(synth.clip_seed(3, 1))
    snr = rng.uniform(-6.0, 6.0, n)
    hops = rng.choice([64, 256, 512], n)
    xs_h = [synth.make_clip(synth.clip_seed(3, 10 + i), int(lens[i]), 16000.0, float(snr[i])) for i in range(n)]
    xs = [torch.from_numpy(x).cuda() for x in xs_h]
    scales = np.arange(1, 129, dtype=np.float64)
    plans = {h: cw.Plan(16000.0, scales, h, "bf16") for h in (64, 256, 512)}
    pl = [plans[int(h)] for h in hops]
    B = cw.Batch(n)
    untuned = [o.clone() for o in B(pl, xs, graph=False)]
    chosen = cw.autotune_batch(pl, lens)               # the batch's own tile configuration
    print("256-clip batch: tuned configuration %d" % chosen)
    prep = B.prepare(pl, xs)
    first = [o.clone() for o in prep.run(graph=True)]
    torch.cuda.synchronize()
    for i in range(n):
        assert torch.equal(untuned[i], first[i]), i
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda") * 2.0      # eager work between replays
        for o in prep.outs:
            o.fill_(-1.0)
        outs = prep.run(graph=True)
        torch.cuda.synchronize()
        assert float(junk.abs().sum()) > 0
        for i in range(n):
            assert torch.equal(outs[i], first[i]), (rep, i)
    direct = B(pl, xs, graph=False)
    torch.cuda.synchronize()
    for i in range(n):
        assert torch.equal(direct[i], first[i]), i
    got = [o.cpu().numpy() for o in first]
    full = {0, n - 1, int(np.argmax(lens)), int(np.argmin(lens))}
    for i in range(n):
        h = int(hops[i])
        if i in full:
            ref = np.abs(oracle.cwt(xs_h[i].astype(np.float64), scales, h))
            assert_close("bf16", got[i], ref, "256-clip batch clip %d (len %d, hop %d, full)" % (i, lens[i], h))
        _sampled_check("bf16", got[i], xs_h[i], scales, h, rng, 2000,
                       "256-clip batch clip %d (len %d, hop %d, 2000 samples)" % (i, lens[i], h), True)


def test_batch_rejects_mixed_plans(torch, cw):
    a = cw.Plan(16000.0, [1.0, 2.0], 4, "bf16")
    b = cw.Plan(16000.0, [1.0, 3.0], 4, "bf16")
    c = cw.Plan(16000.0, [1.0, 2.0], 4, "fp16")
    x = torch.zeros(100, device="cuda")
    for other in (b, c):
        with pytest.raises(cw.CwtError) as e:
            cw.execute_batch([a, other], [x, x])
        assert e.value.status == cw.UNSUPPORTED


# ---------------------------------------------------------------------------
# ABI argument checks with a device present.

def test_invalid_arguments(torch, cw):
    lib = cw.raw()
    h = ctypes.c_void_p()
    sc = (ctypes.c_double * 2)(1.0, 2.0)
    bad = (ctypes.c_double * 2)(1.0, -2.0)
    nan = (ctypes.c_double * 1)(float("nan"))
    assert lib.cwt_plan_create(16000.0, 0, sc, 2, 0, 1, ctypes.byref(h)) == cw.INVALID_ARG
    assert lib.cwt_plan_create(16000.0, 0, bad, 2, 1, 1, ctypes.byref(h)) == cw.INVALID_ARG
    assert lib.cwt_plan_create(16000.0, 0, nan, 1, 1, 1, ctypes.byref(h)) == cw.INVALID_ARG
    assert lib.cwt_plan_create(16000.0, 0, sc, 0, 1, 1, ctypes.byref(h)) == cw.INVALID_ARG
    assert lib.cwt_plan_create(0.0, 0, sc, 2, 1, 1, ctypes.byref(h)) == cw.INVALID_ARG
    assert lib.cwt_plan_create(16000.0, 0, None, 2, 1, 1, ctypes.byref(h)) == cw.INVALID_ARG
    assert lib.cwt_plan_create(16000.0, 0, sc, 2, 1, 1, None) == cw.INVALID_ARG
    assert lib.cwt_plan_create(16000.0, 3, sc, 2, 1, 1, ctypes.byref(h)) == cw.UNSUPPORTED
    assert lib.cwt_plan_create(16000.0, 0, sc, 2, 1, 9, ctypes.byref(h)) == cw.UNSUPPORTED
    assert lib.cwt_plan_create(16000.0, 0, sc, 2, 3, 1, ctypes.byref(h)) == cw.OK
    x = torch.zeros(10, device="cuda")
    o = torch.zeros(2 * 4, device="cuda")
    assert lib.cwt_execute(h, x.data_ptr(), -1, o.data_ptr(), None) == cw.INVALID_ARG
    assert lib.cwt_execute(h, None, 10, o.data_ptr(), None) == cw.INVALID_ARG
    assert lib.cwt_execute(h, x.data_ptr(), 10, None, None) == cw.INVALID_ARG
    assert lib.cwt_execute(h, None, 0, None, None) == cw.OK
    assert lib.cwt_execute(None, x.data_ptr(), 10, o.data_ptr(), None) == cw.INVALID_ARG
    assert lib.cwt_num_frames(h, 10) == 4 and lib.cwt_num_frames(h, -1) == -1
    assert lib.cwt_execute(h, x.data_ptr(), 10, o.data_ptr(), None) == cw.OK
    torch.cuda.synchronize()
    assert lib.cwt_plan_destroy(h) == cw.OK
    assert lib.cwt_plan_destroy(None) == cw.OK


def test_launch_configuration_follows_the_launch(torch, cw):
    """A default plan picks the tile per launch: 128-frame tiles at hop 1,
    64-frame tiles for a 256-clip batch at hop 512 (the 128-frame window does
    not fit LDS), 32-frame tiles for one clip there (too few frames); a set
    configuration holds for every launch, and the results agree bit for bit."""
    scales = np.arange(1, 129)
    p1 = cw.Plan(16000.0, scales, 1, "bf16")
    assert p1.config_kind(p1.launch_config(160000)) == 1          # hop 1: Toeplitz tiles
    assert p1.launch_config(160000, 3) == 13                       # hop-1 batches: one grid of these tiles
    assert cw.Plan(16000.0, scales, 1, "bf16x3").config_kind(6) == 0
    p = cw.Plan(16000.0, scales, 512, "bf16", signed=True)
    assert p.config == 6
    assert p.launch_config(160000, 256) == 4 and p.launch_config(160000, 1) == 5
    assert p.launch_config(0, 1) == -1 and p.launch_config(100, 0) == -1
    xs = [torch.from_numpy(clip(2, i % 3, 160000, 0.0)).cuda() for i in range(256)]
    auto = cw.execute_batch([p] * 256, xs)
    p.set_config(5)
    assert p.launch_config(160000, 256) == 5
    fixed = cw.execute_batch([p] * 256, xs)
    torch.cuda.synchronize()
    for i in (0, 1, 2, 255):
        assert torch.equal(auto[i], fixed[i]), i
    # FP8: the per-launch choice up to hop 128 (a signal scale per 128-frame
    # segment), 32-frame tiles beyond (a scale per tile)
    assert cw.Plan(16000.0, scales, 1, "fp8").launch_config(160000, 3) == 6
    p8 = cw.Plan(16000.0, scales, 512, "fp8")
    assert p8.launch_config(160000, 256) == 5 and p8.launch_config(160000, 1) == 5


def test_frequencies_and_autotune(torch, cw):
    p = cw.Plan(16000.0, [1.0, 5.0, 100.0], 32, "bf16")
    hz = p.frequencies()
    np.testing.assert_allclose(hz, 5 / (2 * math.pi) * 16000.0 / np.array([1.0, 5.0, 100.0]), rtol=1e-15)
    x = torch.from_numpy(clip(1, 0, 16000, 0.0)).cuda()
    before = p(x)
    c = p.autotune(16000)
    # the plan stays automatic; its launches of this class run the tuned choice
    assert 0 <= c < p.num_configs and c == p.launch_config(16000, 1)
    after = p(x)
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    # a set configuration is never overridden by a tuned one
    q = cw.Plan(16000.0, [1.0, 5.0, 100.0], 32, "bf16")
    q.set_config(5)
    assert q.launch_config(16000, 1) == 5


def test_autotune_batch_keys_on_length_and_clip_count(torch, cw):
    """Tuning a batch records its choice for its own class only: the one-clip
    launch of another length keeps the per-launch choice, and the tuned batch
    gives the same bits as before tuning."""
    scales = np.arange(1, 65)
    plans = {h: cw.Plan(16000.0, scales, h, "bf16") for h in (64, 256)}
    p1 = cw.Plan(16000.0, scales, 64, "bf16")
    single_before = p1.launch_config(100000, 1)
    lens = [20000 + 1000 * i for i in range(40)]
    pl = [plans[64 if i % 2 else 256] for i in range(40)]
    xs = [torch.from_numpy(synth.make_clip(700 + i, n, 16000.0, 0.0)).cuda() for i, n in enumerate(lens)]
    before = cw.execute_batch(pl, xs)
    c = cw.autotune_batch(pl, lens)
    assert 0 <= c < plans[64].num_configs
    after = cw.execute_batch(pl, xs)
    torch.cuda.synchronize()
    for a, b in zip(before, after):
        assert torch.equal(a, b)
    assert p1.launch_config(100000, 1) == single_before
    with pytest.raises(cw.CwtError):
        cw.autotune_batch([plans[64], cw.Plan(16000.0, scales, 64, "fp16")], [1000, 1000])
