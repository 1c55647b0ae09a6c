"""Helpers shared by the GPU tests: device guard, error metrics, tolerances."""
import numpy as np
import pytest

# Whole-scalogram bounds on signed W: (rel-L2, max-abs).  max-abs is stated for
# an input with max|x| = 1 and taps of unit energy (sum t^2 = sqrt(pi)/2, every
# scale >= 1/2 or so); assert_close scales it by max|x| * max(1, sqrt(sum t^2 / (sqrt(pi)/2)))
# for the widest-gain scale in the set (a scale s < 1/8 has one tap of gain 1/sqrt(s)).
# Error model: each operand is rounded once, relative error uniform in
# +-u (u = half an ulp), so one coefficient's error has standard deviation
# about u/sqrt(3) * sqrt(2 * sum t^2) * max|x|; the bound is ~5 of those.
#   fp32    FP32 taps and FMA chains (u = 2^-24, plus accumulation): 1e-5 / 1e-4
#   fp16    u = 2^-11:  sigma ~ 4e-4                            -> 2e-3 / 2e-3
#   bf16    u = 2^-8 :  sigma ~ 3e-3 (of which half is cancelled) -> 1e-2 / 1e-2
#   bf16x3  hi+lo leaves u ~ 2^-16 per operand                  -> 5e-5 / 5e-5
#   fp8     e4m3, u = 2^-4: sigma ~ 4.8e-2                      -> 1.5e-1 / 2e-1
TOL = {"fp32": (1e-5, 1e-4), "fp16": (2e-3, 2e-3), "bf16": (1e-2, 1e-2),
       "bf16x3": (5e-5, 5e-5), "fp8": (1.5e-1, 2e-1)}
# FP8 on the measured workloads (generator clips, the whole scalogram, every
# hop): the blanket bound above assumes |x| = 1 at every sample; these clips
# have an RMS near 0.3, and the maxima grow with the coefficient count like
# sqrt(2 ln n).  Measured on MI355X (bench.py --errors), all hops:
#   1 s, 32 scales (5e5 coefficients):        rel-L2 1.6-1.7e-2, max-abs 0.057-0.082
#   10 s, 128 scales, 3 clips (6e7):          rel-L2 1.28e-2,    max-abs 0.070-0.100
#   8 x 60 s at 48 kHz, 256 geometric (4.6e7): rel-L2 1.46e-2,    max-abs 0.120-0.129
# bounds: 2.5e-2 on rel-L2 and about 1.5x the largest measured max-abs.
TOL_FP8_WORKLOAD = {"1s32": (2.5e-2, 0.12), "10s128": (2.5e-2, 0.15), "60s256": (2.5e-2, 0.2)}
DTYPES = ("fp32", "bf16", "fp16", "bf16x3", "fp8")


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def errors(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    nr = float(np.linalg.norm(ref))
    rel = float(np.linalg.norm(d) / nr) if nr > 0 else float(np.linalg.norm(d))
    mab = float(np.abs(d).max()) if d.size else 0.0
    return rel, mab


def gain(scales, xmax=1.0):
    """max|x| * max(1, sqrt(sum t^2 / (sqrt(pi)/2))) over the scale set."""
    import oracle
    e = max(float(np.sum(oracle.taps(s) ** 2)) for s in scales)
    return float(xmax) * max(1.0, (e / (np.sqrt(np.pi) / 2)) ** 0.5)


def tol_for(dt, workload=None):
    """(rel-L2, max-abs) bound of a path; FP8 has per-workload bounds."""
    if dt == "fp8" and workload is not None:
        return TOL_FP8_WORKLOAD[workload]
    return TOL[dt]


def assert_close(dt, got, ref, what="", scale=1.0, workload=None):
    """scale: see gain(); the bounds hold for max|x| = 1 and unit-energy taps.
    workload: a key of TOL_FP8_WORKLOAD for the measured workloads."""
    rel, mab = errors(got, ref)
    r_tol, a_tol = tol_for(dt, workload)
    print("%s %-6s rel-L2 %.3e (tol %.1e)  max-abs %.3e (tol %.1e)" % (what, dt, rel, r_tol, mab, a_tol * scale))
    assert rel <= r_tol, "%s %s rel-L2 %.3e > %.1e" % (what, dt, rel, r_tol)
    assert mab <= a_tol * scale, "%s %s max-abs %.3e > %.1e" % (what, dt, mab, a_tol * scale)
    return rel, mab
