"""The device's binary64 division, square root and fused multiply-add round
as the host's do (to nearest, ties to even, subnormals kept).

The step is bitwise equal to the oracle only because every division, square
root and fma it evaluates rounds correctly on the device, as they do on the
host; this checks that directly through hydro_fp_check, which computes them
with the step kernels' compiler settings, over 10^8 operand pairs spread over
all binades (random bit patterns, so subnormals, overflow and underflow of
the quotient, zeros, infinities and NaN all occur), plus operands near 1 and
cancelling fma terms.  Expected values come from the host (numpy's IEEE
division and square root, the C library's fma)."""
import ctypes
import ctypes.util

import numpy as np
import pytest
import torch

from paper_2401_03378_amd import _hip

pytestmark = pytest.mark.gpu

CHUNK = 10_000_000
NCHUNK = 10
NFMA = 200_000


def _same_bits(x, y):
    """Bitwise equal, or both NaN (NaN payloads are not compared)."""
    nan = np.isnan(x) & np.isnan(y)
    return (x.view(np.int64) == y.view(np.int64)) | nan


def _dev(x):
    return torch.from_numpy(x).cuda()


def _run(a, b, c):
    q, r, f = _hip.fp_check(_dev(a), _dev(b), _dev(c))
    torch.cuda.synchronize()
    return q.cpu().numpy(), r.cpu().numpy(), f.cpu().numpy()


def _random_doubles(rng, n):
    return rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, size=n, dtype=np.int64,
                        endpoint=True).view(np.float64)


def test_division_and_sqrt_match_the_host_bit_for_bit():
    rng = np.random.default_rng(20240106)
    bad_q = bad_r = 0
    sub = 0
    with np.errstate(all="ignore"):
        for chunk in range(NCHUNK):
            if chunk % 2 == 0:
                a, b = _random_doubles(rng, CHUNK), _random_doubles(rng, CHUNK)
            else:
                # operands of ordinary size: quotients near 1, the common case of the step
                a = rng.uniform(0.5, 4.0, CHUNK) * rng.choice([-1.0, 1.0], CHUNK)
                b = rng.uniform(0.25, 8.0, CHUNK)
            c = np.zeros_like(a)
            q, r, _ = _run(a, b, c)
            hq, hr = a / b, np.sqrt(a)
            bad_q += int((~_same_bits(q, hq)).sum())
            bad_r += int((~_same_bits(r, hr)).sum())
            sub += int(((hq != 0) & (np.abs(hq) < np.finfo(np.float64).tiny)).sum())
            print(f"chunk {chunk}: division mismatches so far {bad_q}, sqrt {bad_r}", flush=True)
    assert sub > 1000, "the operand mix must produce subnormal quotients"
    assert bad_q == 0 and bad_r == 0, (bad_q, bad_r)


def test_special_operands():
    tiny, big = np.finfo(np.float64).tiny, np.finfo(np.float64).max
    sub_min = np.nextafter(0.0, 1.0)
    vals = np.array([0.0, -0.0, 1.0, -1.0, 2.0, 3.0, 0.1, 1e-300, 1e300, tiny, tiny / 2, sub_min, -sub_min,
                     big, -big, np.inf, -np.inf, np.nan, np.nextafter(1.0, 2.0), np.nextafter(1.0, 0.0),
                     4.0, 9.0, 1e-320, 2.5e-308])
    a = np.repeat(vals, len(vals))
    b = np.tile(vals, len(vals))
    c = np.tile(vals[::-1], len(vals))
    q, r, f = _run(a, b, c)
    libm = ctypes.CDLL(ctypes.util.find_library("m"))
    libm.fma.restype = ctypes.c_double
    libm.fma.argtypes = [ctypes.c_double] * 3
    with np.errstate(all="ignore"):
        assert _same_bits(q, a / b).all()
        assert _same_bits(r, np.sqrt(a)).all()
    hf = np.array([libm.fma(x, y, z) for x, y, z in zip(a, b, c)])
    assert _same_bits(f, hf).all()


def test_fma_matches_the_host_bit_for_bit():
    rng = np.random.default_rng(7)
    a = rng.uniform(-2.0, 2.0, NFMA) * np.exp2(rng.integers(-60, 60, NFMA))
    b = rng.uniform(-2.0, 2.0, NFMA) * np.exp2(rng.integers(-60, 60, NFMA))
    # half the terms cancel the product (the fma then returns its rounding error exactly)
    c = np.where(np.arange(NFMA) % 2 == 0, -(a * b), rng.uniform(-1.0, 1.0, NFMA))
    _, _, f = _run(a, b, c)
    libm = ctypes.CDLL(ctypes.util.find_library("m"))
    libm.fma.restype = ctypes.c_double
    libm.fma.argtypes = [ctypes.c_double] * 3
    hf = np.fromiter((libm.fma(x, y, z) for x, y, z in zip(a.tolist(), b.tolist(), c.tolist())),
                     dtype=np.float64, count=NFMA)
    assert int((hf[::2] != 0).sum()) > NFMA // 4, "cancelling terms must leave rounding errors"
    assert _same_bits(f, hf).all()
