#!/usr/bin/env python3
"""Throughput of the hop-strided Morlet CWT on one MI355X.

Workload (the headline): 10 s clips at 16 kHz (160000 samples), 128 linear
Morlet scales s = 1..128 (up to 2049 taps), three clips per step at SNR -6/0/6
dB, hop 1 (the full CWT), BF16 operands on the matrix cores with FP32
accumulation, |W| written as FP32 [scale][frame].  `value` is coefficients per
second over the timed steps, inputs resident in HBM, outputs rotated over two
sets larger than the 256 MB Infinity Cache.

The same JSON line carries the other legs of the metric: the plain FP32 kernel
at hop 1, both paths at hop 512 (256 clips per persistent launch), their
ratios, the roofline of the dominant kernel, the serving session's p50/p99 at a
fixed Poisson arrival rate, and the FP64 CPU oracle as a timed baseline.

    python bench.py [--gpus 1] [--steps 50] [--warmup 200]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FS = 16000.0
N = 160000
S = 128
METRIC = "CWT coeffs/sec at hop 1 & 512, BF16-MFMA vs FP32 plain; serving p50/p99 ms"
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2408_14302_amd", "csrc", "mfma.hip")

# HBM bytes per launch of the three timed MFMA kernels, from two rocprofv3 --pmc
# runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over
# the dispatches of the leg; for the mixed batch its last eight, the tuned
# configuration's, after the autotuner's candidates), each scaled by what the counter reads for a plain
# device copy of known size (FETCH_SCALE, WRITE_SCALE).  They describe the
# kernel source whose SHA-256 is recorded and are reported only while it is
# unchanged.
FETCH_SCALE = 2.0
WRITE_SCALE = 1.0
TRAFFIC = {
    "bf16_hop1": {"kernel": "k_toep_batch<1, 4>", "config": 13, "fetch_kib": 8789.0, "write_kib": 240000.0,
                  "src_sha256": "3dd0011b8713270b373109099a81a6b4be475d4f737e1fe04817a4283beb8068"},
    "bf16_hop512": {"kernel": "k_mfma_persistent_win<1, 2>", "config": 4, "fetch_kib": 87342.5,
                    "write_kib": 55737.2, "src_sha256": "3dd0011b8713270b373109099a81a6b4be475d4f737e1fe04817a4283beb8068"},
    "bf16_mixed": {"kernel": "k_mfma_persistent_win<1, 2>", "config": 4, "fetch_kib": 58063.6,
                   "write_kib": 110719.6, "src_sha256": "3dd0011b8713270b373109099a81a6b4be475d4f737e1fe04817a4283beb8068"},
}


def kernel_sha():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_bytes(leg, config):
    """Counted HBM bytes per launch, while the kernel source and the launch's
    tile configuration are the ones the counters were taken with."""
    rec = TRAFFIC.get(leg)
    if not rec or rec["src_sha256"] != kernel_sha() or rec["config"] != config:
        return None
    return 1024.0 * (FETCH_SCALE * rec["fetch_kib"] + WRITE_SCALE * rec["write_kib"])


def hop1_kernel(config):
    """Kernel a hop-1 BF16 batch of several clips of this configuration runs:
    Toeplitz tiles in one grid over the clips (configuration 13, 4 x 4096
    frames per work-group) or 32-scale-block tiles in the persistent kernel."""
    return "k_toep_batch<bf16>" if config == 13 else "k_mfma_persistent<bf16>"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--batch512", type=int, default=256, help="clips per hop-512 launch")
    ap.add_argument("--qps", type=float, default=2000.0, help="serving arrival rate")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--qps-half", type=float, default=46000.0,
                    help="fixed arrival rate of the second serving session (half the calibrated saturation)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["bf16-hop1", "fp32-hop1", "bf16-hop512", "fp32-hop512", "bf16-hopmixed",
                                       "fp32-hopmixed"], default=None,
                    help="time one leg only (for profiling runs)")
    ap.add_argument("--hop-sweep", action="store_true",
                    help="cost curve over hops 1, 2, 4, .., 1024 (one JSON line per hop) instead of the metric")
    ap.add_argument("--decimate", action="store_true",
                    help="decimate-then-transform against the hop-strided transform, hops 2 .. 512 (JSON lines)")
    ap.add_argument("--image", action="store_true",
                    help="scalogram-to-image step (dB, min-max, bilinear to 224x224) timing (JSON lines)")
    ap.add_argument("--dwt", action="store_true",
                    help="DWT scalogram (db4, 14 levels) on 3 and 256 clips of 10 s, against the CWTH (JSON lines)")
    ap.add_argument("--long", action="store_true",
                    help="8 channels x 60 s at 48 kHz, 256 geometric scales 1..1024, hops 128 and 512, "
                         "BF16 / FP8 / FP32 (JSON lines)")
    ap.add_argument("--errors", action="store_true",
                    help="error of every path against the FP64 oracle per workload, dtype and hop (JSON lines)")
    ap.add_argument("--long-dtypes", default="bf16,fp8,fp32", help="paths timed by --long (comma separated)")
    ap.add_argument("--dwt-clips", default="3,256", help="batch sizes for --dwt (comma separated)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device-to-device copy of MB mebibytes (calibrates HBM byte counters)")
    return ap.parse_args()


def alg_flops_per_coeff(scales):
    """2 L_i flop per coefficient, L_i = 2 floor(8 s_i) + 1 (Eq. (1), one tap per sample)."""
    L = 2 * np.floor(8.0 * np.asarray(scales, dtype=np.float64)) + 1
    return 2.0 * L


def time_launches(torch, launch, nsets, steps, warmup, warm_ms=0.0):
    """launch(step_index) queues one step; returns (total_ms, [per-step ms]).
    Untimed first: `warmup` steps and, with warm_ms > 0, further steps until
    warm_ms of wall time have passed.  The GPU's clock ramps up over the first
    milliseconds of sustained load: after 5 steps (~1 ms) of hop-1 work the
    first timed steps still run ~20% slower than after 200.  The timed steps
    run back to back between one pair of events, and each step's time is
    their mean: a timing event recorded between two launches holds the next
    one back by several microseconds (13 us per 256-clip hop-512 launch with
    an event pair around each)."""
    st = torch.cuda.current_stream()
    t_start = time.perf_counter()
    for w in range(warmup):
        launch(w)
    w = warmup
    while warm_ms > 0 and (time.perf_counter() - t_start) * 1e3 < warm_ms:
        for _ in range(4):
            launch(w)
            w += 1
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(st)
    for s in range(steps):
        launch(s)
    t1.record(st)
    torch.cuda.synchronize()
    total = t0.elapsed_time(t1)
    return total, [total / steps] * steps


def hop_sweep(torch, cwth, synth, dev, scales, args):
    """Cost of the transform of 10 s clips (128 scales) at hops 1, 2, 4, .., 1024:
    BF16 MFMA (default configuration) and plain FP32, clips per launch growing
    with the hop (min(hop, 256): one single-clip launch at hop 1, one
    persistent batch launch beyond) so each launch holds a comparable amount
    of work; inputs resident, outputs rotated over two sets.
    Reports coefficients/s, microseconds per clip, and the fraction of the
    roof that binds at that hop (MFMA flops or HBM bytes, whichever takes
    longer at peak)."""
    fpc = alg_flops_per_coeff(scales)
    flop_per_frame = float(fpc.sum())
    base = [torch.from_numpy(synth.make_clip(synth.clip_seed(2, 40 + i), N, FS, float(np.linspace(-6, 6, 8)[i])))
            .to(dev) for i in range(8)]
    stream = torch.cuda.current_stream()
    for hop in [1 << k for k in range(11)]:
        nb = min(hop, 256)
        K = -(-N // hop)
        row = {"hop": hop, "clips_per_launch": nb, "frames_per_clip": K}
        for dt in ("bf16", "fp32"):
            plan = cwth.Plan(FS, scales, hop, dt)
            B = cwth.Batch(nb)
            sets = [[base[(j * 3 + k) % 8].clone() for k in range(nb)] for j in range(2)]
            outs = [[torch.empty((S, K), dtype=torch.float32, device=dev) for _ in range(nb)] for _ in range(2)]
            prep = [B.prepare([plan] * nb, sets[j], outs[j]) for j in range(2)]
            steps = max(3, min(args.steps, 20 if dt == "bf16" else 5))
            if nb == 1:
                def launch(s_):
                    plan.execute(sets[s_ % 2][0], outs[s_ % 2][0], stream)
            else:
                def launch(s_):
                    prep[s_ % 2].run(stream=stream.cuda_stream, graph=False)
            total, per = time_launches(torch, launch, 2, steps, min(args.warmup, 3), warm_ms=30.0)
            ms = float(np.mean(per))
            coeffs = nb * S * K
            t_flop = flop_per_frame * K * nb / (PEAK_BF16_TFLOPS * 1e12 if dt == "bf16" else 157.3e12)
            t_hbm = nb * (4.0 * N + 4.0 * S * K) / (PEAK_HBM_GBS * 1e9)
            bound = "mfma" if dt == "bf16" and t_flop >= t_hbm else ("hbm" if t_hbm >= t_flop else "valu")
            row[dt] = {"coeffs_per_s": coeffs / (ms * 1e-3), "us_per_clip": 1e3 * ms / nb, "ms_per_launch": ms,
                       "config": plan.launch_config(N, nb), "bound": bound,
                       "roof_frac": max(t_flop, t_hbm) / (ms * 1e-3)}
            del prep, sets, outs, B, plan
        row["ratio_bf16_over_fp32"] = row["bf16"]["coeffs_per_s"] / row["fp32"]["coeffs_per_s"]
        if not args.no_cpu:
            import oracle
            x0 = base[0].cpu().numpy().astype(np.float64)
            t0 = time.perf_counter()
            oracle.cwt(x0, scales, hop)
            sec = time.perf_counter() - t0
            row["cpu_baseline"] = {"value": S * K / sec, "unit": "coeffs/s", "cores": oracle.max_threads(),
                                   "kind": "oracle", "seconds": sec, "sample": "one of the clips, FP64"}
        print(json.dumps({"metric": "hop sweep: " + METRIC, **row}), flush=True)
        log("hop %4d: bf16 %.3e coeffs/s (%.1f us/clip, %.2f of %s roof), fp32 %.3e, ratio %.1f" % (
            hop, row["bf16"]["coeffs_per_s"], row["bf16"]["us_per_clip"], row["bf16"]["roof_frac"],
            row["bf16"]["bound"], row["fp32"]["coeffs_per_s"], row["ratio_bf16_over_fp32"]))


def decimate_sweep(torch, cwth, synth, dev, scales, args):
    """The two readings of the paper's hop on one 10 s clip (128 scales, BF16):
    the hop-strided transform (Sec. II-B) against decimating the signal by the
    hop (plain, and with a 8h+1-tap anti-alias filter) and transforming the
    decimated signal at hop 1 with scales s/h (Sec. III-B).  Reports the device
    time of each route and the deviation of sqrt(h) times the decimated route's
    signed W from the hop-strided W (the sqrt(h) is the 1/sqrt(s) normalisation
    at the coarser sampling)."""
    x = torch.from_numpy(synth.make_clip(synth.clip_seed(2, 60), N, FS, 0.0)).to(dev)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        t_start, n = time.perf_counter(), 0
        while n < 3 or time.perf_counter() - t_start < 0.03:   # 30 ms of load: the clock's ramp
            fn()
            n += 1
            if n % 8 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for hop in [1 << k for k in range(1, 10)]:
        ref_plan = cwth.Plan(FS, scales, hop, "bf16", signed=True)
        ref = ref_plan(x)
        t_ref = timed(lambda: ref_plan.execute(x, ref, stream), 20)
        row = {"hop": hop, "hop_strided_us": 1e3 * t_ref}
        dec_plan = cwth.Plan(FS / hop, scales / hop, 1, "bf16", signed=True)
        for name, h in (("plain", None), ("fir", torch.from_numpy(cwth.lowpass_fir(hop, 8 * hop + 1)
                                                                 .astype(np.float32)).to(dev))):
            y = cwth.decimate(x, hop, h)
            w = dec_plan(y)
            t = timed(lambda: (cwth.decimate(x, hop, h, out=y, stream=stream), dec_plan.execute(y, w, stream)), 20)
            d = (w.double() * math.sqrt(hop) - ref.double())
            rel = float(d.norm() / ref.double().norm())
            keep = torch.from_numpy(np.asarray(scales) >= 2 * hop).to(dev)   # scales resolved after decimation
            rel_res = float(d[keep].norm() / ref.double()[keep].norm()) if bool(keep.any()) else None
            row[name] = {"us": 1e3 * t, "rel_l2_vs_hop_strided": rel, "rel_l2_scales_ge_2hop": rel_res}
        if not args.no_cpu:
            import oracle
            from oracle import transforms as T
            xd = x.cpu().numpy().astype(np.float64)
            hd = cwth.lowpass_fir(hop, 8 * hop + 1)
            t0 = time.perf_counter()
            oracle.cwt(xd, scales, hop)
            t1 = time.perf_counter()
            T.decimated_cwt(xd, scales, hop, hd)
            t2 = time.perf_counter()
            row["cpu_baseline"] = {"value": 1e6 * (t1 - t0), "unit": "us per clip (hop-strided)",
                                   "fir_route_us": 1e6 * (t2 - t1), "cores": oracle.max_threads(), "kind": "oracle",
                                   "sample": "the same clip, FP64: hop-strided transform and the FIR route"}
        print(json.dumps({"metric": "decimate-then-transform vs hop-strided transform, 10 s clip, 128 scales, bf16",
                          **row}), flush=True)
        log("hop %3d: strided %.1f us; decimate+cwt %.1f us (plain, dev %.3f / %s), %.1f us (fir, dev %.3f / %s)" % (
            hop, row["hop_strided_us"], row["plain"]["us"], row["plain"]["rel_l2_vs_hop_strided"],
            row["plain"]["rel_l2_scales_ge_2hop"], row["fir"]["us"], row["fir"]["rel_l2_vs_hop_strided"],
            row["fir"]["rel_l2_scales_ge_2hop"]))


def image_bench(torch, cwth, synth, dev, scales, args):
    """The scalogram-to-image step on the scalograms of one 10 s clip
    (128 scales) at hops 1 and 512: device time per image and the HBM rate of
    its dominant pass (the min/max over the whole scalogram, 4 B per
    coefficient), against the 8 TB/s peak."""
    x = torch.from_numpy(synth.make_clip(synth.clip_seed(2, 70), N, FS, 0.0)).to(dev)
    stream = torch.cuda.current_stream()
    for hop in (1, 512):
        w = cwth.Plan(FS, scales, hop, "bf16")(x)
        ws = torch.empty(int(cwth.raw().cwt_image_workspace_bytes()), dtype=torch.uint8, device=dev)
        img = torch.empty((224, 224), dtype=torch.float32, device=dev)
        run = lambda: cwth.scalogram_image(w, 224, 224, amin=1e-6, out=img, workspace=ws, stream=stream)
        total, per = time_launches(torch, lambda s_: run(), 1, max(args.steps, 20), args.warmup)
        ms = float(np.mean(per))
        byt = 4.0 * w.numel() + 4.0 * 5 * 224 * 224
        row = {"hop": hop, "scalogram": list(w.shape), "image": [224, 224], "us_per_image": 1e3 * ms,
               "bytes": byt, "gb_per_s": byt / (ms * 1e-3) / 1e9, "hbm_frac": byt / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
        if not args.no_cpu:
            from oracle import transforms as T
            wd = w.cpu().numpy().astype(np.float64)
            t0 = time.perf_counter()
            T.scalogram_image(wd, 1e-6, 224, 224)
            row["cpu_baseline"] = {"value": 1e6 * (time.perf_counter() - t0), "unit": "us per image", "cores": 1,
                                   "kind": "oracle", "sample": "the same scalogram, FP64 numpy"}
        print(json.dumps({"metric": "scalogram to image (dB, min-max, bilinear 224x224)", **row}), flush=True)
        log("image hop %d: %.1f us, %.0f GB/s (%.2f of HBM)" % (hop, row["us_per_image"], row["gb_per_s"],
                                                                 row["hbm_frac"]))


def long_bench(torch, cwth, synth, dev, args):
    """Long multichannel recordings: 8 channels x 60 s at 48 kHz (2,880,000
    samples each), 256 geometric scales from 1 to 1024 samples, hops 128 and
    512, all channels in one persistent launch (prepared batch, direct launch,
    two input/output sets in alternation).  Reports coefficients/s, the
    algorithmic TFLOP/s and its fraction of the dtype's dense peak (BF16
    2.5 PFLOP/s, FP8 5.0, FP32 VALU 157.3 TFLOP/s), and FP8 and BF16 over FP32."""
    n, fs, ch = 2880000, 48000.0, 8
    scales = synth.geometric_scales(256, 1024.0)
    flop_per_frame = float(alg_flops_per_coeff(scales).sum())
    base = [torch.from_numpy(synth.make_clip(synth.clip_seed(5, c), n, fs, 0.0)).to(dev) for c in range(ch)]
    stream = torch.cuda.current_stream()
    peaks = {"bf16": PEAK_BF16_TFLOPS, "fp8": 2 * PEAK_BF16_TFLOPS, "fp32": 157.3}
    for hop in (128, 512):
        K = -(-n // hop)
        row = {"hop": hop, "channels": ch, "samples": n, "scales": 256, "frames": K}
        for dt in args.long_dtypes.split(","):
            plan = cwth.Plan(fs, scales, hop, dt)
            B = cwth.Batch(ch)
            sets = [base, [b.clone() for b in base]]
            outs = [[torch.empty((256, K), dtype=torch.float32, device=dev) for _ in range(ch)] for _ in range(2)]
            prep = [B.prepare([plan] * ch, sets[j], outs[j]) for j in range(2)]
            steps = max(3, min(args.steps, 20 if dt != "fp32" else 3))
            _, per = time_launches(torch, lambda s_: prep[s_ % 2].run(stream=stream.cuda_stream, graph=False), 2,
                                   steps, min(args.warmup, 2), warm_ms=30.0)
            ms = float(np.mean(per))
            tflops = flop_per_frame * K * ch / (ms * 1e-3) / 1e12
            row[dt] = {"ms_per_launch": ms, "coeffs_per_s": ch * 256 * K / (ms * 1e-3), "tflops": tflops,
                       "frac_of_peak": tflops / peaks[dt], "config": plan.launch_config(n, ch)}
            del prep, outs, B, plan
        if "fp32" in row and "bf16" in row:
            row["bf16_over_fp32"] = row["fp32"]["ms_per_launch"] / row["bf16"]["ms_per_launch"]
        if "fp8" in row and "bf16" in row:
            row["fp8_over_bf16"] = row["bf16"]["ms_per_launch"] / row["fp8"]["ms_per_launch"]
        if not args.no_cpu:
            import oracle
            x0 = base[0].cpu().numpy().astype(np.float64)
            t0 = time.perf_counter()
            oracle.cwt(x0, scales, hop)
            sec = time.perf_counter() - t0
            row["cpu_baseline"] = {"value": 256 * K / sec, "unit": "coeffs/s", "cores": oracle.max_threads(),
                                   "kind": "oracle", "seconds": sec, "sample": "one of the channels, FP64"}
        print(json.dumps({"metric": "8 x 60 s at 48 kHz, 256 geometric scales", **row}), flush=True)
        log("hop %d: " % hop + ", ".join("%s %.3f ms (%.0f TFLOP/s, %.2f of peak)" % (
            d, row[d]["ms_per_launch"], row[d]["tflops"], row[d]["frac_of_peak"])
            for d in args.long_dtypes.split(",")))


def dwt_bench(torch, cwth, synth, dev, scales, args):
    """The DWT scalogram (Sec. II-A, Fig. 1c) of 10 s clips at 16 kHz with db4
    and 14 levels (the deepest whose input still spans the 8 taps), for the
    3-clip batch of the transform workload and a 256-clip batch: device time
    per batch, the HBM rate of the whole call (algorithmic bytes: the signal
    read once, the level record and the 14 x 160000 matrix written once), and
    the CWTH of the same 3 clips (128 scales, BF16) at hops 1 and 512 beside it."""
    h = cwth.daubechies(4)
    levels = 14
    stream = torch.cuda.current_stream()
    plen = cwth.dwt_pyramid_length(N, levels)
    for clips in [int(c) for c in args.dwt_clips.split(",")]:
        xs = torch.from_numpy(np.stack([synth.make_clip(synth.clip_seed(2, 80 + (c % 16)), N, FS, 0.0)
                                        for c in range(clips)])).to(dev)
        pyr = torch.empty((clips, plen), dtype=torch.float32, device=dev)
        out = torch.empty((clips, levels, N), dtype=torch.float32, device=dev)
        run = lambda s_: cwth.dwt_scalogram(xs, h, levels, out=out, pyramid=pyr, stream=stream)
        _, per = time_launches(torch, run, 1, max(args.steps, 20), args.warmup)
        ms = float(np.mean(per))
        byt = 4.0 * clips * (N + plen + levels * N)
        row = {"clips": clips, "samples": N, "wavelet": "db4", "levels": levels, "us_per_batch": 1e3 * ms,
               "matrix_entries_per_s": clips * levels * N / (ms * 1e-3), "alg_bytes": byt,
               "gb_per_s": byt / (ms * 1e-3) / 1e9, "hbm_frac": byt / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
        if clips == 3:
            for hop in (1, 512):
                plan = cwth.Plan(FS, scales, hop, "bf16")
                ws = [plan(xs[c]) for c in range(clips)]
                go = lambda s_: [plan.execute(xs[c], ws[c], stream) for c in range(clips)]
                _, per_c = time_launches(torch, go, 1, max(args.steps, 20), args.warmup)
                row["cwth_hop%d_us" % hop] = 1e3 * float(np.mean(per_c))
        if clips == 3 and not args.no_cpu:
            from oracle import transforms as T
            x0 = xs[0].cpu().numpy().astype(np.float64)
            t0 = time.perf_counter()
            T.dwt_scalogram(x0, T.daubechies(4), levels)
            sec = time.perf_counter() - t0
            row["cpu_baseline"] = {"value": levels * N / sec, "unit": "matrix entries/s", "cores": 1, "kind": "oracle",
                                   "seconds": sec, "sample": "one of the clips, FP64 numpy (a Python loop per level)"}
        print(json.dumps({"metric": "DWT scalogram (filter bank, 14 levels, matrix)", **row}), flush=True)
        log("dwt %d clips: %.1f us, %.0f GB/s (%.2f of HBM)%s" % (
            clips, row["us_per_batch"], row["gb_per_s"], row["hbm_frac"],
            "; cwth hop 1 %.1f us, hop 512 %.1f us" % (row["cwth_hop1_us"], row["cwth_hop512_us"])
            if clips == 3 else ""))
        del xs, pyr, out


def error_report(torch, cwth, synth, dev, args):
    """Measured error of every floating-point path against the FP64 oracle,
    one JSON line per (workload, dtype, hop): rel-L2 and max-abs over the
    whole signed scalogram, the worst single scale's rel-L2, and the stated
    tolerance.  Workloads: 1 s / 32 scales (hops 1, 64); 10 s / 128 scales,
    SNR -6/0/6 dB (hops 1, 32, 128, 256, 512); 8 x 60 s at 48 kHz with 256
    geometric scales (hops 128, 512; BF16, FP8, BF16x3 and FP32).  Every
    coefficient is compared (the oracle runs on all host threads)."""
    import oracle
    # the bounds the parity tests assert; FP8's per workload (its error grows
    # with the dynamic range the transform spans: the widest scales' output
    # against the narrowest ones' quantisation)
    tol = {"fp32": (1e-5, 1e-4), "fp16": (2e-3, 2e-3), "bf16": (1e-2, 1e-2), "bf16x3": (5e-5, 5e-5)}
    work = [("1 s at 16 kHz, 32 linear scales, SNR 0 dB", 16000, 16000.0, synth.linear_scales(32),
             [synth.make_clip(synth.clip_seed(1, 0), 16000, 16000.0, 0.0)], (1, 64), tuple(tol) + ("fp8",),
             (2.5e-2, 0.12)),
            ("10 s at 16 kHz, 128 linear scales, SNR -6/0/6 dB", N, FS, synth.linear_scales(128),
             [synth.make_clip(synth.clip_seed(2, i), N, FS, snr) for i, snr in enumerate((-6.0, 0.0, 6.0))],
             (1, 32, 128, 256, 512), tuple(tol) + ("fp8",), (2.5e-2, 0.15)),
            ("8 x 60 s at 48 kHz, 256 geometric scales 1..1024", 2880000, 48000.0, synth.geometric_scales(256, 1024.0),
             [synth.make_clip(synth.clip_seed(5, c), 2880000, 48000.0, 0.0) for c in range(8)], (128, 512),
             ("bf16", "fp8", "bf16x3", "fp32"), (2.5e-2, 0.2))]
    for name, n, fs, scales, clips, hops, dts, fp8_tol in work:
        tol["fp8"] = fp8_tol
        xs = [torch.from_numpy(c).to(dev) for c in clips]
        for hop in hops:
            t0 = time.perf_counter()
            refs = [oracle.cwt(c.astype(np.float64), scales, hop) for c in clips]
            osec = time.perf_counter() - t0
            for dt in dts:
                plan = cwth.Plan(fs, scales, hop, dt, signed=True)
                outs = cwth.execute_batch([plan] * len(xs), xs) if len(xs) > 1 else [plan(xs[0])]
                torch.cuda.synchronize()
                num = den = 0.0
                mab = 0.0
                sn = np.zeros(len(scales))
                sd = np.zeros(len(scales))
                for o, ref in zip(outs, refs):
                    d = o.cpu().numpy().astype(np.float64) - ref
                    num += float(np.sum(d * d))
                    den += float(np.sum(ref * ref))
                    mab = max(mab, float(np.abs(d).max()))
                    sn += np.sum(d * d, axis=1)
                    sd += np.sum(ref * ref, axis=1)
                per_scale = np.sqrt(sn / np.maximum(sd, 1e-300))
                w = int(np.argmax(per_scale))
                row = {"metric": "error vs FP64 oracle (signed W, every coefficient)", "workload": name, "dtype": dt,
                       "hop": hop, "clips": len(clips), "coefficients": int(sum(r.size for r in refs)),
                       "rel_l2": math.sqrt(num / den), "max_abs": mab, "tol_rel_l2": tol[dt][0],
                       "tol_max_abs": tol[dt][1], "worst_scale": float(scales[w]),
                       "worst_scale_rel_l2": float(per_scale[w]), "oracle_seconds": osec}
                if dt == "fp8":
                    row["per_scale_rel_l2_quantiles"] = [float(q) for q in np.quantile(per_scale, [0.0, 0.5, 0.9, 1.0])]
                print(json.dumps(row), flush=True)
                log("%s hop %d %-6s rel-L2 %.3e (tol %.0e) max-abs %.3e (tol %.0e) worst scale %g: %.3e" % (
                    name[:22], hop, dt, row["rel_l2"], tol[dt][0], mab, tol[dt][1], scales[w], per_scale[w]))
                del outs, plan
            del refs


def main():
    args = parse()
    if args.gpus != 1:
        msg = ("bench.py measures one GPU: the transform runs on a single MI355X "
               "(the work shards by clip with no collective). Run with --gpus 1.")
        print(msg, file=sys.stderr)
        print(json.dumps({"metric": METRIC, "error": msg, "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2408_14302_amd import cwth, serve, synth

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 5}))
        return
    scales = synth.linear_scales(S)
    if args.hop_sweep:
        hop_sweep(torch, cwth, synth, dev, scales, args)
        return
    if args.decimate:
        decimate_sweep(torch, cwth, synth, dev, scales, args)
        return
    if args.image:
        image_bench(torch, cwth, synth, dev, scales, args)
        return
    if args.dwt:
        dwt_bench(torch, cwth, synth, dev, scales, args)
        return
    if args.long:
        long_bench(torch, cwth, synth, dev, args)
        return
    if args.errors:
        error_report(torch, cwth, synth, dev, args)
        return
    fpc = alg_flops_per_coeff(scales)
    flops_per_frame = float(fpc.sum())                  # all scales, one frame

    # ---------------- inputs (resident) ----------------
    clips = [torch.from_numpy(synth.make_clip(synth.clip_seed(2, i), N, FS, snr)).to(dev)
             for i, snr in enumerate((-6.0, 0.0, 6.0))]
    K1 = N
    out1 = [[torch.empty((S, K1), dtype=torch.float32, device=dev) for _ in clips] for _ in range(2)]
    result = {}
    stream = torch.cuda.current_stream()

    def leg_hop1(dt):
        """The three clips of a step in one launch of the prepared batch (for
        BF16 one grid of Toeplitz tiles over the three clips, k_toep_batch;
        for FP32 the flat direct-sum grid), outputs rotated over two sets."""
        plan = cwth.Plan(FS, scales, 1, dt)
        B = cwth.Batch(len(clips))
        prep = [B.prepare([plan] * len(clips), clips, out1[j]) for j in range(2)]

        def launch(s):
            prep[s % 2].run(stream=stream.cuda_stream, graph=False)
        steps = args.steps if dt == "bf16" else max(5, args.steps // 5)
        total, per = time_launches(torch, launch, 2, steps, args.warmup)
        ms = total / steps
        coeffs = len(clips) * S * K1
        return {"ms_per_step": ms, "coeffs_per_s": coeffs / (ms * 1e-3), "per_launch_ms": float(np.mean(per)),
                "clips_per_launch": len(clips), "steps": steps, "config": plan.launch_config(N, len(clips))}

    # hop 512: many clips per launch (one clip alone is ~0.1 us of work)
    nb = args.batch512
    K512 = -(-N // 512)

    def leg_hop512(dt):
        base = [synth.make_clip(synth.clip_seed(2, 10 + i), N, FS, float(np.linspace(-6, 6, 16)[i])) for i in range(16)]
        base = [torch.from_numpy(b).to(dev) for b in base]
        sets = [[base[(j * 7 + k) % 16].clone() for k in range(nb)] for j in range(2)]
        outs = [[torch.empty((S, K512), dtype=torch.float32, device=dev) for _ in range(nb)] for _ in range(2)]
        plan = cwth.Plan(FS, scales, 512, dt)
        plans = [plan] * nb
        B = cwth.Batch(nb)
        # resident buffers: each set is validated and marshalled once
        prepared = [B.prepare(plans, sets[j], outs[j]) for j in range(2)]
        sptr = stream.cuda_stream

        def launch(s):
            prepared[s % 2].run(stream=sptr, graph=False)

        def launch_graph(s):
            prepared[s % 2].run(stream=sptr, graph=True)
        steps = args.steps if dt == "bf16" else max(5, args.steps // 5)
        # direct launches of the prepared batch (descriptors already resident):
        # a graph replay of the same launch adds ~8 us of launch processing on
        # the device, reported beside it
        total, per = time_launches(torch, launch, 2, steps, args.warmup)
        ms = total / steps
        _, per_graph = time_launches(torch, launch_graph, 2, steps, args.warmup)
        coeffs = nb * S * K512
        return {"ms_per_step": ms, "coeffs_per_s": coeffs / (ms * 1e-3), "per_launch_ms": float(np.mean(per)),
                "per_launch_ms_graph": float(np.mean(per_graph)), "clips_per_launch": nb, "steps": steps,
                "config": plan.launch_config(N, nb)}

    def leg_mixed(dt):
        """The batching workload: 256 clips, lengths uniform in [1 s, 10 s],
        SNR uniform in [-6, 6] dB, hop per clip from {64, 256, 512}, 128
        scales, one persistent launch whose tile configuration is tuned on the
        batch itself (cwt_autotune_batch); timed as direct launches of the
        prepared batch and as graph replays."""
        nb = 256
        lens = synth.batch_lengths(synth.clip_seed(3, 0), nb)
        rng = np.random.default_rng(synth.clip_seed(3, 1))
        snr = rng.uniform(-6.0, 6.0, nb)
        hops = rng.choice([64, 256, 512], nb)
        plans = {h: cwth.Plan(FS, scales, h, dt) for h in (64, 256, 512)}
        pl = [plans[int(h)] for h in hops]
        base = [torch.from_numpy(synth.make_clip(synth.clip_seed(3, 10 + i), int(lens[i]), FS, float(snr[i]))).to(dev)
                for i in range(nb)]
        sets = [base, [b.clone() for b in base]]
        outs = [[torch.empty((S, p.num_frames(int(n))), dtype=torch.float32, device=dev) for p, n in zip(pl, lens)]
                for _ in range(2)]
        chosen = cwth.autotune_batch(pl, lens) if dt != "fp32" else 0
        B = cwth.Batch(nb)
        prepared = [B.prepare(pl, sets[j], outs[j]) for j in range(2)]
        sptr = stream.cuda_stream
        steps = args.steps if dt == "bf16" else max(5, args.steps // 5)
        total, per = time_launches(torch, lambda s_: prepared[s_ % 2].run(stream=sptr, graph=False), 2, steps,
                                   args.warmup)
        _, per_graph = time_launches(torch, lambda s_: prepared[s_ % 2].run(stream=sptr, graph=True), 2, steps,
                                     args.warmup)
        ms = total / steps
        K = np.array([p.num_frames(int(n)) for p, n in zip(pl, lens)], dtype=np.float64)
        coeffs = float(S * K.sum())
        return {"ms_per_step": ms, "coeffs_per_s": coeffs / (ms * 1e-3), "per_launch_ms": float(np.mean(per)),
                "per_launch_ms_graph": float(np.mean(per_graph)), "clips_per_launch": nb, "steps": steps,
                "config": chosen, "alg_bytes": float(4.0 * lens.sum() + 4.0 * coeffs),
                "alg_flop": float(alg_flops_per_coeff(scales).sum() * K.sum()), "samples": int(lens.sum())}

    legs = [("bf16", 1), ("fp32", 1), ("bf16", 512), ("fp32", 512), ("bf16", "mixed"), ("fp32", "mixed")]
    if args.only:
        d, h = args.only.split("-hop")
        legs = [(d, h if h == "mixed" else int(h))]
    for dt, hop in legs:
        log("leg %s hop %s ..." % (dt, hop))
        r = leg_hop1(dt) if hop == 1 else (leg_hop512(dt) if hop == 512 else leg_mixed(dt))
        result[(dt, hop)] = r
        log("  %s hop %s: %.3f ms/step, %.3e coeffs/s" % (dt, hop, r["ms_per_step"], r["coeffs_per_s"]))

    head = result.get(("bf16", 1)) or next(iter(result.values()))
    line = {
        "metric": METRIC,
        "value": head["coeffs_per_s"],
        "unit": "coeffs/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "10 s clips at 16 kHz (160000 samples), 128 linear Morlet scales 1..128, "
                               "hop 1, 3 clips per step (SNR -6/0/6 dB), |W| as FP32",
                   "clip_samples": N, "fs_hz": FS, "n_scales": S, "hop": 1, "clips_per_step": len(clips),
                   "operands": "bf16 (MFMA, FP32 accumulation)"},
    }
    legs_out = {}
    for (dt, hop), r in result.items():
        legs_out["%s_hop%s" % (dt, hop)] = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}
    for hop in (1, 512, "mixed"):
        if ("bf16", hop) in result and ("fp32", hop) in result:
            legs_out["ratio_bf16_over_fp32_hop%s" % hop] = result[("bf16", hop)]["coeffs_per_s"] / result[("fp32", hop)]["coeffs_per_s"]
    line["legs"] = legs_out

    # ---------------- roofline of the dominant kernel ----------------
    if ("bf16", 1) in result:
        r = result[("bf16", 1)]
        flops = flops_per_frame * K1 * len(clips)         # one launch = the step's three clips
        ach = flops / (r["per_launch_ms"] * 1e-3) / 1e12
        line["roofline"] = {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                            "frac": ach / PEAK_BF16_TFLOPS, "traffic": traffic_bytes("bf16_hop1", r["config"]),
                            "kernel": "%s (configuration %d tiles), hop 1, three 160000-sample clips x 128 "
                                      "scales per launch" % (hop1_kernel(r["config"]), r["config"]),
                            "alg_flop_per_launch": flops, "avg_launch_ms": r["per_launch_ms"]}
    if ("bf16", 512) in result:
        r = result[("bf16", 512)]
        byt = nb * (4.0 * N + 4.0 * S * K512)
        gbs = byt / (r["per_launch_ms"] * 1e-3) / 1e9
        line["roofline_hop512"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                   "frac": gbs / PEAK_HBM_GBS, "alg_bytes_per_launch": byt,
                                   "traffic": traffic_bytes("bf16_hop512", r["config"]), "avg_launch_ms": r["per_launch_ms"],
                                   "kernel": "k_mfma_persistent_win<bf16> (configuration %d), hop 512, %d clips "
                                             "per launch" % (r["config"], nb)}

    if ("bf16", "mixed") in result:
        r = result[("bf16", "mixed")]
        gbs = r["alg_bytes"] / (r["per_launch_ms"] * 1e-3) / 1e9
        tfl = r["alg_flop"] / (r["per_launch_ms"] * 1e-3) / 1e12
        line["roofline_mixed"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                  "frac": gbs / PEAK_HBM_GBS, "alg_bytes_per_launch": r["alg_bytes"],
                                  "mfma_tflops": tfl, "mfma_frac": tfl / PEAK_BF16_TFLOPS,
                                  "traffic": traffic_bytes("bf16_mixed", r["config"]),
                                  "avg_launch_ms": r["per_launch_ms"],
                                  "kernel": "k_mfma_persistent_win<bf16> (configuration %d), 256 clips of 1-10 s, "
                                            "hops 64/256/512, one launch" % r["config"]}

    # ---------------- serving ----------------
    if not args.no_serve and not args.only:
        log("serving session: %.0f QPS for %.1f s ..." % (args.qps, args.serve_seconds))
        lens = synth.serving_lengths(1430400, 48)
        sclips = [torch.from_numpy(synth.make_clip(1430500 + i, int(n), FS, 0.0)).to(dev) for i, n in enumerate(lens)]
        plans = {(s_, h): cwth.Plan(FS, synth.linear_scales(s_), h, "bf16") for s_ in (64, 128) for h in (1, 256, 512)}
        ex = serve.GpuExecutor(3, max_clips=64)
        # warm every plan and batch shape once, untimed
        serve.serve_session(400.0, 1.0, sclips, plans, seed=7, executor=ex)
        stats, reqs = serve.serve_session(args.qps, args.serve_seconds, sclips, plans, seed=1430401, executor=ex)
        sm = stats.summary()
        sm["qps_offered"] = args.qps
        sm["budget_bytes"] = 4 << 30
        sm["slots"] = 3
        log("  serving: p50 %.3f ms p99 %.3f ms" % (sm.get("p50_ms", float("nan")), sm.get("p99_ms", float("nan"))))
        # closed-loop saturation, then an open-loop session at half of it
        sat, _ = serve.saturation_session(4000, sclips, plans, executor=ex)
        sat_qps = len(sat.latencies_ms) / sat.wall_s
        # the second session runs at a FIXED rate: half of the saturation
        # calibrated once (92,400-94,300 requests/s over three MI355X runs of
        # this closed-loop burst); the live saturation is reported beside it
        half = args.qps_half
        log("  saturation %.0f requests/s; session at the fixed %.0f QPS ..." % (sat_qps, half))
        hs, _ = serve.serve_session(half, args.serve_seconds, sclips, plans, seed=1430403, executor=ex)
        hm = hs.summary()
        hm["qps_offered"] = half
        sm["saturation_qps"] = sat_qps
        sm["at_fixed_half_saturation"] = {k: hm[k] for k in ("qps_offered", "completed", "p50_ms", "p99_ms", "mean_ms",
                                                       "max_ms", "coeffs_per_s") if k in hm}
        line["serving"] = sm
        log("  at half saturation: p50 %.3f ms p99 %.3f ms" % (hm.get("p50_ms", float("nan")),
                                                                hm.get("p99_ms", float("nan"))))

    # ---------------- CPU baseline (FP64 oracle) ----------------
    if not args.no_cpu and not args.only:
        import oracle
        xs = [c.cpu().numpy().astype(np.float64) for c in clips]
        cores = oracle.max_threads()
        log("cpu baseline: FP64 oracle on %d threads ..." % cores)
        t = time.perf_counter()
        for x in xs:
            oracle.cwt(x, scales, 1)
        dt_s = time.perf_counter() - t
        oracle.set_threads(1)
        t = time.perf_counter()
        oracle.cwt(xs[0], scales, 1)
        one_s = time.perf_counter() - t
        oracle.set_threads(cores)
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
        except OSError:
            pass
        line["cpu_baseline"] = {"value": len(xs) * S * N / dt_s, "unit": "coeffs/s", "cores": cores,
                                "kind": "oracle", "seconds": dt_s,
                                "sample": "the full step: 3 clips x 160000 samples x 128 scales at hop 1, FP64",
                                "one_core": {"value": S * N / one_s, "seconds": one_s,
                                             "sample": "one of the clips on one thread"},
                                "cpu_model": model}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
