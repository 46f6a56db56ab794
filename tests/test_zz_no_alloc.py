"""The allocation-free CFL entry point (hydro_cfl_dt_noalloc) against the
context's hydro_cfl_dt, through the C ABI (needs an MI355X).

Two calls in a row on one GPU share the library's static scratch; the second
has fewer blocks and slower waves, so a stale per-block maximum left by the
first call would lower its dt and show up as a mismatch."""
import math

import numpy as np
import pytest

from paper_2401_03378_amd import _hip
from paper_2401_03378_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx_dt(p, U):
    from paper_2401_03378_amd.solver import Solver
    S = Solver(p)
    dt = S.cfl_dt(U).clone()
    S.status()
    S.close()
    return dt


def _noalloc_dt(p, U):
    blocks = torch.frombuffer(bytearray(_hip.block_table_bytes(p)), dtype=torch.uint8).to(U.device)
    dt = torch.full((1,), -1.0, dtype=torch.float64, device=U.device)
    _hip.cfl_dt_noalloc(p, blocks, U, dt)
    torch.cuda.synchronize()
    return dt


def _bits(t):
    return np.frombuffer(t.cpu().numpy().tobytes(), dtype=np.uint64)


def test_noalloc_dt_equals_the_context_dt_on_two_calls_in_a_row():
    dev = torch.device("cuda:0")
    big = W.batched_uneven(nblocks=512, seed=3)              # 3D, uneven 8^3 / 16^3 / 32^3 blocks
    small = W.sod2d(N=32, n=16)                               # 2D, 4 blocks, slower waves
    dts = []
    for p in (big, small):
        U = torch.as_tensor(np.ascontiguousarray(p.U0), dtype=torch.float64).to(dev)
        want = _ctx_dt(p, U)
        got = _noalloc_dt(p, U)
        assert math.isfinite(float(got)) and float(got) > 0.0
        assert (_bits(got) == _bits(want)).all(), (p.name if hasattr(p, "name") else p, float(got), float(want))
        dts.append(float(got))
    assert dts[1] > dts[0]          # the second problem's dt is the larger one: no stale maximum leaked in


def test_noalloc_reports_a_nonphysical_cell_and_a_bad_descriptor_as_nan():
    dev = torch.device("cuda:0")
    p = W.sod2d(N=32, n=16)
    U0 = np.array(p.U0, copy=True)
    m = W.interior_mask(p.blocks, p.ncell, 2)
    first = int(np.flatnonzero(m)[5])
    U0[0, first] = -1.0                                      # rho <= 0 in one interior cell
    U = torch.as_tensor(U0, dtype=torch.float64).to(dev)
    assert math.isnan(float(_noalloc_dt(p, U)))
    q = W.sod2d(N=32, n=16)
    q.blocks = np.array(q.blocks, copy=True)
    q.blocks["offset"][2] = q.ncell                          # padded cells beyond the state: not read
    U = torch.as_tensor(np.ascontiguousarray(q.U0), dtype=torch.float64).to(dev)
    assert math.isnan(float(_noalloc_dt(q, U)))
    r = W.sod2d(N=32, n=16)
    r.blocks = np.array(r.blocks, copy=True)
    r.blocks["nx"][1] = 2 ** 31 - 1                          # an extent whose padded size would overflow 32 bits
    assert math.isnan(float(_noalloc_dt(r, U)))
    # the valid problem right after still gets its own dt
    U = torch.as_tensor(np.ascontiguousarray(p.U0), dtype=torch.float64).to(dev)
    assert (_bits(_noalloc_dt(p, U)) == _bits(_ctx_dt(p, U))).all()


def test_noalloc_dt_at_full_size():
    """4096 blocks of 16^3 (the 256^3 turbulence workload): the same dt as
    the context's, bit for bit."""
    dev = torch.device("cuda:0")
    p = W.turb3d()
    U = torch.as_tensor(np.ascontiguousarray(p.U0), dtype=torch.float64).to(dev)
    assert (_bits(_noalloc_dt(p, U)) == _bits(_ctx_dt(p, U))).all()
