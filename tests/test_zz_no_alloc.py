"""The allocation-free batch entry point (cwt_execute_batch_noalloc) through
the raw C ABI: the same bits as cwt_execute_batch on two calls in a row, the
second with a smaller batch of shorter clips, so whatever the first call left
in the shared device array cannot leak into the second."""
import ctypes

import numpy as np
import pytest

from gpu_util import torch_cuda
from paper_2408_14302_amd import synth

pytestmark = pytest.mark.gpu


def _raw_batch(lib, fn, plans, xs, outs, stream):
    n = len(plans)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    P = (vp * n)(*[p.handle.value for p in plans])
    X = (vp * n)(*[x.data_ptr() if x.numel() else None for x in xs])
    L = (i64 * n)(*[x.numel() for x in xs])
    O = (vp * n)(*[o.data_ptr() if o.numel() else None for o in outs])
    return getattr(lib, fn)(P, X, L, O, n, stream)


@pytest.mark.parametrize("dt", ["bf16", "fp8", "fp32"])
def test_noalloc_batch_matches_execute_batch_twice(dt):
    torch = torch_cuda()
    from paper_2408_14302_amd import cwth
    lib = cwth.raw()
    scales = np.arange(1, 129, dtype=np.float64)
    plans = {h: cwth.Plan(16000.0, scales, h, dt, signed=True) for h in (1, 64, 256, 512)}
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(7)
    for call, (count, lo, hi) in enumerate(((300, 16000, 160000), (37, 2000, 30000))):
        lens = rng.integers(lo, hi, count)
        hops = rng.choice([64, 256, 512] if call == 0 else [1, 64, 512], count)
        xs = [torch.from_numpy(synth.make_clip(4000 + 1000 * call + i, int(n), 16000.0, 0.0)).cuda()
              for i, n in enumerate(lens)]
        xs.append(torch.zeros(0, device="cuda"))          # an empty clip in the batch
        hops = list(hops) + [64]
        pl = [plans[int(h)] for h in hops]
        ref = [torch.full((128, p.num_frames(x.numel())), -1.0, device="cuda") for p, x in zip(pl, xs)]
        got = [torch.full((128, p.num_frames(x.numel())), -2.0, device="cuda") for p, x in zip(pl, xs)]
        assert _raw_batch(lib, "cwt_execute_batch", pl, xs, ref, stream) == cwth.OK
        st = _raw_batch(lib, "cwt_execute_batch_noalloc", pl, xs, got, stream)
        assert st == cwth.OK, lib.cwt_last_error()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(ref, got)):
            assert torch.equal(a, b), (dt, call, i, int(hops[i]), xs[i].numel())
        print("noalloc %s call %d: %d clips bit-identical to cwt_execute_batch" % (dt, call, len(xs)))


def test_noalloc_batch_of_hop1_clips():
    """A batch of hop-1 clips only (one grid of Toeplitz tiles) through the
    allocation-free entry point: the bits of cwt_execute_batch."""
    torch = torch_cuda()
    from paper_2408_14302_amd import cwth
    lib = cwth.raw()
    p = cwth.Plan(16000.0, np.arange(1, 65, dtype=np.float64), 1, "bf16", signed=True)
    stream = torch.cuda.current_stream().cuda_stream
    lens = [20000, 4000, 100000, 0, 65000]
    xs = [torch.from_numpy(synth.make_clip(5000 + i, n, 16000.0, 0.0)).cuda() if n else torch.zeros(0, device="cuda")
          for i, n in enumerate(lens)]
    ref = [torch.full((64, p.num_frames(x.numel())), -1.0, device="cuda") for x in xs]
    got = [torch.full((64, p.num_frames(x.numel())), -2.0, device="cuda") for x in xs]
    assert _raw_batch(lib, "cwt_execute_batch", [p] * len(xs), xs, ref, stream) == cwth.OK
    st = _raw_batch(lib, "cwt_execute_batch_noalloc", [p] * len(xs), xs, got, stream)
    assert st == cwth.OK, lib.cwt_last_error()
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(ref, got)):
        assert torch.equal(a, b), (i, lens[i])


def test_noalloc_rejects_more_than_512_clips():
    torch = torch_cuda()
    from paper_2408_14302_amd import cwth
    lib = cwth.raw()
    p = cwth.Plan(16000.0, [1.0, 2.0], 4, "bf16")
    xs = [torch.zeros(100, device="cuda")] * 513
    outs = [torch.zeros((2, 25), device="cuda")] * 513
    st = _raw_batch(lib, "cwt_execute_batch_noalloc", [p] * 513, xs, outs, None)
    assert st == cwth.INVALID_ARG
    assert b"512" in lib.cwt_last_error()
    assert _raw_batch(lib, "cwt_execute_batch_noalloc", [p] * 0, [], [], None) == cwth.OK
