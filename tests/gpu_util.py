"""Helpers shared by the GPU tests: device guard, error metrics, tolerances."""
import numpy as np
import pytest

# Whole-scalogram bounds on signed W for inputs with |x| <= 1: (rel-L2, max-abs).
# Derivation (one rounding of each operand, FP32 accumulation):
#   fp32    FP32 taps and FMA chains: ~1e-7 relative per term, tolerance 1e-5 / 1e-4
#   fp16    2^-11 relative rounding of taps and samples: 2e-3 / 2e-3
#   bf16    2^-8 relative rounding of taps and samples: 1e-2 / 1e-2
#   bf16x3  hi+lo split leaves ~2^-16 per operand, the dropped lo*lo term ~2^-17: 5e-5 / 5e-5
#   fp8     e4m3 keeps 3 mantissa bits (2^-4 relative): 1.5e-1 / 1e-1
TOL = {"fp32": (1e-5, 1e-4), "fp16": (2e-3, 2e-3), "bf16": (1e-2, 1e-2),
       "bf16x3": (5e-5, 5e-5), "fp8": (1.5e-1, 1e-1)}
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


def assert_close(dt, got, ref, what="", scale=1.0):
    """scale: max|x| of the input (tolerances are stated for |x| <= 1)."""
    rel, mab = errors(got, ref)
    r_tol, a_tol = TOL[dt]
    print("%s %-6s rel-L2 %.3e (tol %.1e)  max-abs %.3e (tol %.1e)" % (what, dt, rel, r_tol, mab, a_tol * scale))
    assert rel <= r_tol, "%s %s rel-L2 %.3e > %.1e" % (what, dt, rel, r_tol)
    assert mab <= a_tol * scale, "%s %s max-abs %.3e > %.1e" % (what, dt, mab, a_tol * scale)
    return rel, mab
