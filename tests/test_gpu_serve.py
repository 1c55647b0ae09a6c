"""Serving on the GPU: requests admitted while others run, overlapping
batches on several streams, every result bit-identical to the same request
run alone (the summation order does not depend on the batch) and within the
BF16 bound of the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, assert_close, errors, torch_cuda
from paper_2408_14302_amd import synth

pytestmark = pytest.mark.gpu


def test_results_same_alone_and_in_the_mix():
    torch = torch_cuda()
    from paper_2408_14302_amd import cwth, serve
    lens = np.clip(synth.serving_lengths(11, 16) // 4, 4000, 60000)
    clips = [torch.from_numpy(synth.make_clip(900 + i, int(n), 16000.0, 0.0)).cuda() for i, n in enumerate(lens)]
    plans = {(s, h): cwth.Plan(16000.0, synth.linear_scales(s), h, "bf16") for s in (64, 128) for h in (1, 256, 512)}
    stats, reqs = serve.serve_session(4000.0, 0.05, clips, plans, seed=3, keep_outputs=True, max_batch=16)
    sm = stats.summary()
    print(sm)
    assert sm["completed"] == len(reqs) and sm["rejected"] == 0
    assert sm["batches"] >= 2
    for r in reqs:
        x, p = r.payload
        alone = p(x)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.output), r.rid
    # and every served result against the FP64 oracle: |W| on 300 sampled
    # coefficients per request, two requests in full
    rng = np.random.default_rng(5)
    host = {}
    full = {reqs[0].rid, reqs[len(reqs) // 2].rid}
    worst = 0.0
    for r in reqs:
        x, p = r.payload
        key = id(x)
        if key not in host:
            host[key] = x.cpu().numpy().astype(np.float64)
        xh = host[key]
        got = r.output.cpu().numpy()
        S, K = got.shape
        if r.rid in full:
            ref = np.abs(oracle.cwt(xh, p.scales, p.hop))
            assert_close("bf16", got, ref, "served request %d (S %d, hop %d, full)" % (r.rid, S, p.hop))
        ii = rng.integers(0, S, 300)
        kk = rng.integers(0, K, 300)
        kk[:2] = [0, K - 1]
        ref = np.abs(oracle.points(xh, p.scales, p.hop, ii, kk))
        rel, mab = errors(got[ii, kk], ref)
        worst = max(worst, mab)
        assert rel <= TOL["bf16"][0] and mab <= TOL["bf16"][1], (r.rid, S, p.hop, rel, mab)
    print("served results against the oracle: worst sampled max-abs %.3e over %d requests" % (worst, len(reqs)))


def test_budget_and_rejection_on_gpu():
    torch = torch_cuda()
    from paper_2408_14302_amd import cwth, serve
    clips = [torch.from_numpy(synth.make_clip(950 + i, 20000, 16000.0, 0.0)).cuda() for i in range(4)]
    plans = {(s, h): cwth.Plan(16000.0, synth.linear_scales(s), h, "bf16") for s in (64, 128) for h in (1, 256, 512)}
    # a budget below one hop-1 request (64 x 20000 x 4 B) rejects those, serves the rest
    stats, reqs = serve.serve_session(2000.0, 0.05, clips, plans, seed=4, budget_bytes=4 << 20,
                                      keep_outputs=False)
    sm = stats.summary()
    assert sm["max_inflight_bytes"] <= 4 << 20
    assert sm["rejected"] == sum(1 for r in reqs if r.footprint > (4 << 20)) > 0
    assert sm["completed"] == len(reqs) - sm["rejected"]


def test_closed_loop_saturation_serves_every_request():
    torch = torch_cuda()
    from paper_2408_14302_amd import cwth, serve
    clips = [torch.from_numpy(synth.make_clip(970 + i, 16000 * (1 + i), 16000.0, 0.0)).cuda() for i in range(4)]
    plans = {(s, h): cwth.Plan(16000.0, synth.linear_scales(s), h, "bf16") for s in (64, 128) for h in (1, 256, 512)}
    stats, reqs = serve.saturation_session(200, clips, plans, max_batch=16)
    sm = stats.summary()
    print(sm, "saturation %.0f requests/s" % (sm["completed"] / sm["wall_s"]))
    assert sm["completed"] == len(reqs) == 200 and sm["rejected"] == 0
    assert sm["max_concurrent_batches"] >= 2          # a backlog keeps several batches in flight
