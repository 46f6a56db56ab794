"""Helpers for element-by-element comparison of the GPU path with the oracle.

Tolerance: for every conserved field f over interior cells,
max|f_gpu - f_oracle| / max|f_oracle| <= 1e-12 (a field that is identically
zero in the oracle must be identically zero on the GPU).  Both sides follow
the same evaluation order with correctly rounded +,-,*,/,sqrt and explicit
fma only, so the expected outcome is bitwise equality; the count of cells
that differ in any bit is reported alongside.
"""
import numpy as np

from paper_2401_03378_amd import workloads as W

RTOL = 1e-12


def field_errors(prob, Ug, Uo):
    m = W.interior_mask(prob.blocks, prob.ncell, prob.ndim)
    out = []
    for v in range(prob.ndim + 2):
        a, b = Ug[v, m], Uo[v, m]
        scale = np.max(np.abs(b)) if b.size else 0.0
        diff = np.max(np.abs(a - b)) if b.size else 0.0
        rel = 0.0 if scale == 0.0 and diff == 0.0 else (np.inf if scale == 0.0 else diff / scale)
        nbits = int(np.count_nonzero(a.view(np.int64) != b.view(np.int64)))
        out.append((rel, nbits))
    return out


def assert_parity(prob, Ug, Uo, what="", bitwise=False):
    """The tolerance above; with bitwise, also no cell may differ in any bit
    (the forward step: same arithmetic in the same order on both sides)."""
    errs = field_errors(prob, Ug, Uo)
    for v, (rel, nbits) in enumerate(errs):
        assert rel <= RTOL, f"{what} field {v}: rel err {rel:.3e} ({nbits} cells differ)"
        assert not bitwise or nbits == 0, f"{what} field {v}: {nbits} cells differ in some bit (rel err {rel:.3e})"
    return errs
