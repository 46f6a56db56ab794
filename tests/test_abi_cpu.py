"""The C-ABI library loads on a host without a GPU, exports every symbol the
header declares, and its host-side validation rejects bad problems (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2401_03378_amd import _hip
from paper_2401_03378_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hydro.h")).read()
    return sorted(set(re.findall(r"\b(hydro_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("hydro_step", "hydro_rk_stage", "hydro_cfl_dt", "hydro_step_vjp", "hydro_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _hip.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_hip.EXPORTS) <= set(_declared())


def test_validate_accepts_workloads():
    for p in (W.sod2d(N=32), W.random_blocks(3, 6, 3, seed=0, recon=1, rk=3),
              W.batched_uneven(nblocks=16)):
        assert _hip.validate(p) == _hip.HYDRO_OK


def _mut(f):
    p = W.random_blocks(3, 6, 2, seed=0)
    f(p)
    return _hip.validate(p)


@pytest.mark.parametrize("f", [
    lambda p: p.blocks["offset"].__setitem__(1, int(p.blocks["offset"][0]) + 5),
    lambda p: p.blocks["offset"].__setitem__(0, -1),
    lambda p: p.blocks["offset"].__setitem__(2, p.ncell),
    lambda p: p.blocks["ng"].__setitem__(0, 1),
    lambda p: p.blocks["nx"].__setitem__(0, 0),
    lambda p: p.links["nbr"].__setitem__(0, [7, 9, -1, -1, -1, -1]),
    lambda p: p.links["nbr"].__setitem__(0, [-3, -1, -1, -1, -1, -1]),
    lambda p: setattr(p, "gamma", 1.0),
    lambda p: setattr(p, "cfl", 0.0),
    lambda p: setattr(p, "dx", -1.0),
    lambda p: setattr(p, "rk", 4),
    lambda p: setattr(p, "recon", 2),
    lambda p: setattr(p, "ndim", 1),
    lambda p: setattr(p, "weno_eps", 0.0),
    lambda p: setattr(p, "weno_eps", -1e-6),
    lambda p: setattr(p, "weno_eps", float("nan")),
    lambda p: setattr(p, "weno_eps", float("inf")),
    lambda p: setattr(p, "grav", (float("nan"), 0.0, 0.0)),
    lambda p: setattr(p, "grav", (0.0, 0.0, float("-inf"))),
    lambda p: setattr(p, "shock_thresh", -0.5),
    lambda p: setattr(p, "shock_thresh", float("nan")),
])
def test_validate_rejects(f):
    assert _mut(f) == _hip.HYDRO_EINVAL


def test_validate_mismatched_faces_and_weno_guards():
    blocks, ncell = W.make_table([(6, 6, 6), (6, 4, 6)], 2, 3)
    links = np.zeros(2, dtype=W.LINK_DTYPE)
    links["nbr"] = [1, 1, -2, -2, -2, -2]
    p = W.random_blocks(3, 6, 2, seed=0)
    p.blocks, p.links, p.ncell = blocks, links, ncell
    assert _hip.validate(p) == _hip.HYDRO_EINVAL
    q = W.random_blocks(3, 6, 2, seed=0, recon=W.WENO5, rk=3)
    assert _hip.validate(q) == _hip.HYDRO_EINVAL


def test_validate_plane_size_bound():
    """A 3D block's padded xy plane must hold fewer than 2^31 cells (the
    stage kernels step a halo cell's index from plane to plane by that
    size in 32 bits): one periodic block of 30000 x 30000 x 9000 cells
    passes with ng = 3 and is refused with ng = 9000 (48000^2 > 2^31)."""
    def one(ng):
        blocks, ncell = W.make_table([(30000, 30000, 9000)], ng, 3)
        links = np.zeros(1, dtype=W.LINK_DTYPE)
        links["nbr"] = [0, 0, 0, 0, 0, 0]
        p = W.random_blocks(3, 6, 2, seed=0)
        p.blocks, p.links, p.ncell = blocks, links, ncell
        return _hip.validate(p)
    assert one(3) == _hip.HYDRO_OK
    assert one(9000) == _hip.HYDRO_EINVAL


def test_validate_amr_meshes_and_broken_tables():
    """Host-only check of a mesh with refinement levels: generated meshes
    pass; a link that disagrees with the level table, a level gap, a wrong
    half-face offset and a plain hydro_validate of the same links fail."""
    from paper_2401_03378_amd import workloads as W
    for ndim, ng, recon in ((2, 2, 0), (3, 3, 1)):
        p = W.amr_problem(ndim, n=8, ng=ng, recon=recon, rk=2)
        assert _hip.validate(p) == _hip.HYDRO_OK
        plain = p.copy()
        plain.amr = None
        assert _hip.validate(plain) == _hip.HYDRO_EINVAL         # LEVEL_FACE links need the table
        i = int(np.flatnonzero(p.amr["kind"][:, 3] == 2)[0])
        q = p.copy()
        q.links[i]["nbr"][3] = 0
        assert _hip.validate(q) == _hip.HYDRO_EINVAL
        q = p.copy()
        q.amr[i]["level"] = 1
        assert _hip.validate(q) == _hip.HYDRO_EINVAL
        j = int(np.flatnonzero(p.amr["kind"][:, 2] == 1)[0])
        q = p.copy()
        q.amr[j]["nbr"][2][1] = 1
        assert _hip.validate(q) == _hip.HYDRO_EINVAL


def test_fp_check_rejects_bad_arguments_without_a_gpu():
    L = _hip.lib()
    assert L.hydro_fp_check(None, None, None, None, None, None, -1, None) == _hip.HYDRO_EINVAL
    assert L.hydro_fp_check(None, None, None, None, None, None, 4, None) == _hip.HYDRO_EINVAL


def test_step_vjp_stages_rejects_null_arguments_without_a_gpu():
    """Argument checks come before any HIP call: a null ctx or a null stage
    array is HYDRO_EINVAL on a host without a GPU."""
    L = _hip.lib()
    assert L.hydro_step_vjp_stages(None, None, None, None, None, None) == _hip.HYDRO_EINVAL
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.hydro_step_vjp_stages(None, None, arr, None, None, None) == _hip.HYDRO_EINVAL


def test_cfl_dt_noalloc_rejects_bad_arguments_without_a_gpu():
    """hydro_cfl_dt_noalloc checks its arguments before any HIP call: null
    pointers, bad params and block counts outside 1..HYDRO_NOALLOC_MAX_BLOCKS
    are HYDRO_EINVAL, with text in hydro_last_error(NULL)."""
    L = _hip.lib()
    p = W.sod2d(N=32)
    P, _, _, nb = _hip.tables(p)
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: every case fails validation first
    f = L.hydro_cfl_dt_noalloc
    assert f(None, fake, nb, p.ncell, fake, fake, None) == _hip.HYDRO_EINVAL
    assert f(ctypes.byref(P), None, nb, p.ncell, fake, fake, None) == _hip.HYDRO_EINVAL
    assert f(ctypes.byref(P), fake, nb, p.ncell, None, fake, None) == _hip.HYDRO_EINVAL
    assert f(ctypes.byref(P), fake, nb, p.ncell, fake, None, None) == _hip.HYDRO_EINVAL
    assert f(ctypes.byref(P), fake, 0, p.ncell, fake, fake, None) == _hip.HYDRO_EINVAL
    assert f(ctypes.byref(P), fake, 65537, p.ncell, fake, fake, None) == _hip.HYDRO_EINVAL
    assert b"HYDRO_NOALLOC_MAX_BLOCKS" in L.hydro_last_error(None)
    assert f(ctypes.byref(P), fake, nb, 0, fake, fake, None) == _hip.HYDRO_EINVAL
    for field, bad in (("gamma", 1.0), ("cfl", 0.0), ("dx", -1.0), ("ndim", 4)):
        Q = _hip.Params.from_buffer_copy(P)
        setattr(Q, field, bad)
        assert f(ctypes.byref(Q), fake, nb, p.ncell, fake, fake, None) == _hip.HYDRO_EINVAL


def test_validate_physics_flags():
    """Gravity and the shock detector: valid values pass, unknown flag bits
    fail, and a mesh with levels refuses either."""
    p = W.random_blocks(3, 6, 2, seed=0)
    p.grav = (0.0, -9.8, 1.0)
    p.shock_thresh = 0.0
    assert _hip.validate(p) == _hip.HYDRO_OK
    P, B, L, nb = _hip.tables(p)
    assert P.flags == _hip.FLAG_GRAVITY | _hip.FLAG_SHOCK_DETECT
    P.flags |= 8
    assert _hip.lib().hydro_validate(ctypes.byref(P), B, L, nb, int(p.ncell)) == _hip.HYDRO_EINVAL
    for attr, val in (("grav", (0.0, 1.0, 0.0)), ("shock_thresh", 0.5)):
        q = W.amr_problem(2, n=8, ng=2, recon=0, rk=2)
        assert _hip.validate(q) == _hip.HYDRO_OK
        setattr(q, attr, val)
        assert _hip.validate(q) == _hip.HYDRO_EINVAL
