"""Pins of the oracle's positivity fallback (the step's reconstruction,
calcLims in Algorithm "Intra stage calculations for Spark", read as: when
either face value of a cell along a direction has a density or a pressure
that is not positive, both faces of that cell, in that direction only, take
the cell's own primitive state for all five primitives).

The expected values come from that definition and from the reconstruction
formulas, which are pinned on their own (quadratic exactness, order of
accuracy, TVD), never from the fallback code.  The same checks run against
copies of the oracle with a plausible slip planted in the fallback (built
here with gcc in a temporary folder): each copy must fail them.
"""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")


def _weno_problem():
    return W.random_blocks(3, 6, 3, seed=0, recon=W.WENO5, rk=3)


def _plm_problem():
    return W.random_blocks(3, 6, 2, seed=0, recon=W.PLM_MC, rk=2)


def _stencils(kind, rng, n=64):
    """WENO5 stencils (n, 5 cells, 5 primitives) of positive cells whose
    pressure (kind 'p_right' / 'p_left') or density ('rho') reconstruction
    gives a non-positive value at one face, the other faces and variables
    staying positive; 'smooth' gives stencils with every face positive."""
    out = []
    while len(out) < n:
        cand = np.exp(rng.uniform(-12, 9, size=(4096, 5)))
        qm, qp = O.weno5(cand)
        if kind == "p_right" or kind == "rho":
            sel = cand[(qp <= 0.0) & (qm > 0.0)]
        elif kind == "p_left":
            sel = cand[(qm <= 0.0) & (qp > 0.0)]
        else:
            sel = cand[(qm > 0.0) & (qp > 0.0)]
        for s in sel[: n - len(out)]:
            w = np.empty((5, 5))
            x = np.arange(5) - 2.0
            w[:, 0] = 1.0 + 0.1 * x + 0.05 * rng.standard_normal()      # smooth positive density
            w[:, 1:4] = rng.standard_normal((5, 3))
            w[:, 4] = 2.0 + 0.2 * x                                       # smooth positive pressure
            if kind in ("p_right", "p_left"):
                w[:, 4] = s
            elif kind == "rho":
                w[:, 0] = s
            else:
                w[:, 4] = s
            out.append(w)
    return np.array(out)


def _recon(L, P, w):
    f = L.ora_recon_cell_n
    f.restype = None
    dp = C.POINTER(C.c_double)
    f.argtypes = [C.POINTER(O._Problem), C.c_int64, dp, dp, dp, C.POINTER(C.c_int)]
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = w.shape[0]
    qm, qp, fb = np.zeros((n, 5)), np.zeros((n, 5)), np.zeros(n, dtype=np.int32)
    f(P.ptr, n, w.ctypes.data_as(dp), qm.ctypes.data_as(dp), qp.ctypes.data_as(dp),
      fb.ctypes.data_as(C.POINTER(C.c_int)))
    return qm, qp, fb


def check_fallback_pointwise(L):
    """The point-wise pins of the fallback, on the oracle library L."""
    rng = np.random.default_rng(7)
    P = O.Problem(_weno_problem())
    # (1) a face going non-positive in p (right or left face) or rho: both
    # faces become the cell's primitives, all five of them, bit for bit
    for kind in ("p_right", "p_left", "rho"):
        w = _stencils(kind, rng)
        qm, qp, fb = _recon(L, P, w)
        assert np.all(fb == 1), kind
        assert np.array_equal(qm, w[:, 2, :]), kind
        assert np.array_equal(qp, w[:, 2, :]), kind
    # (2) every face positive: no fallback, every primitive's faces are the
    # plain WENO5 values of its own stencil
    w = _stencils("smooth", rng)
    qm, qp, fb = _recon(L, P, w)
    assert np.all(fb == 0)
    for v in range(5):
        em, ep = O.weno5(w[:, :, v])
        assert np.array_equal(qm[:, v], em) and np.array_equal(qp[:, v], ep), v
    # (3) PLM-MC on positive data never triggers it (its faces lie between
    # neighbouring cell values) and gives the plain PLM faces
    Pp = O.Problem(_plm_problem())
    w = np.exp(rng.uniform(-12, 9, size=(4096, 3, 5)))
    w[:, :, 1:4] = rng.standard_normal((4096, 3, 3))
    qm, qp, fb = _recon(L, Pp, w)
    assert np.all(fb == 0)
    for v in range(5):
        em, ep, _ = O.plm(w[:, :, v])
        assert np.array_equal(qm[:, v], em) and np.array_equal(qp[:, v], ep), v


def test_fallback_pointwise():
    check_fallback_pointwise(O.lib())


def _x_dip_problem():
    """One periodic 3D WENO5 block whose pressure varies along x only, with
    near-vacuum dips that drive x reconstructions non-positive, and whose
    density and velocities vary smoothly along y and z."""
    p = W.random_blocks(3, 8, 3, seed=3, recon=W.WENO5, rk=3)
    n = 8
    blocks, ncell = W.make_table([(n, n, n)], 3, 3)
    links = np.zeros(1, dtype=W.LINK_DTYPE)
    links["nbr"] = [-2] * 6
    x = np.arange(n)
    k = 2 * np.pi / n
    px = np.array([1e-5, 5000.0, 1e-5, 1e-5, 3.0, 1e-5, 800.0, 2.0])
    rho = (1.0 + 0.3 * np.sin(k * x)[None, None, :] * np.cos(k * x)[None, :, None]
           + 0.2 * np.sin(2 * k * x)[:, None, None])                       # (z, y, x)
    vel = [0.3 * np.cos(k * x)[:, None, None] * np.ones((n, n, n)),
           0.2 * np.sin(k * x)[None, :, None] * np.ones((n, n, n)),
           0.1 * np.cos(2 * k * x)[:, None, None] * np.sin(k * x)[None, :, None] * np.ones((n, n, n))]
    pr = np.broadcast_to(px[None, None, :], (n, n, n))
    U = W.empty_state(5, ncell)
    W.interior(U, blocks, 0, 3)[...] = W.conserved(rho, vel, pr, p.gamma)
    p.blocks, p.links, p.ncell, p.U0 = blocks, links, ncell, U
    return p


def test_fallback_acts_on_its_own_direction_only():
    """Cells whose x reconstruction falls back: x faces are the cell's
    primitives; the y and z faces of the same cells are the plain WENO5
    values of their y and z stencils (no fallback there)."""
    p = _x_dip_problem()
    U = p.U0.copy()
    O.fill_guards(p, U)
    Wc, _ = O.eos(p, U.T.copy())        # primitives of every padded cell (NaN where no guard)
    Wc = Wc.T                           # (5, ncell)
    B = p.blocks[0]
    n, ng = int(B["nx"]), int(B["ng"])
    idx = lambda i, j, k: int(B["offset"]) + ((k + ng) * (n + 2 * ng) + (j + ng)) * (n + 2 * ng) + (i + ng)
    fx = O.faces(p, U, 0)
    fy = O.faces(p, U, 1)
    fz = O.faces(p, U, 2)
    cells = [(i, j, k) for k in range(n) for j in range(n) for i in range(n) if fx[2][idx(i, j, k)]]
    assert len(cells) >= n * n, "the x dips must trigger the fallback"
    for (i, j, k) in cells:
        c = idx(i, j, k)
        assert np.array_equal(fx[0][:, c], Wc[:, c]) and np.array_equal(fx[1][:, c], Wc[:, c])
        for d, f in ((1, fy), (2, fz)):
            assert f[2][c] == 0
            st = np.array([Wc[:, idx(*[(i, j, k)[a] + (o if a == d else 0) for a in range(3)])]
                           for o in range(-2, 3)])                 # (5 cells, 5 primitives)
            for v in range(5):
                em, ep = O.weno5(st[None, :, v])
                assert f[0][v, c] == em[0] and f[1][v, c] == ep[0], (d, v)
        # the y and z faces differ from the cell value, so the comparison
        # above is not one with the fallback's result
        assert not np.array_equal(fy[0][:, c], Wc[:, c]) or not np.array_equal(fz[0][:, c], Wc[:, c])


def test_sedov_fallback_fires():
    """On the 32^3 Sedov problem the fallback fires from the second step on
    (the blast's pressure jump of ~5e8 drives WENO5 faces negative), the same
    number of times along x, y and z (the problem is symmetric under axis
    permutation), and the stage-by-stage run equals the oracle's step bit
    for bit (no non-physical state reaches the Riemann solver)."""
    p = W.sedov3d(N=32, n=16)
    U = p.U0.copy()
    V = p.U0.copy()
    total = 0
    for n in range(3):
        dt = O.cfl_dt(p, U)
        Un, Us = U.copy(), U.copy()
        for s in range(1, p.rk + 1):
            O.fill_guards(p, Us)
            hits = [int(np.count_nonzero(O.faces(p, Us, d)[2])) for d in range(3)]
            assert hits[0] == hits[1] == hits[2]
            total += hits[0]
            out = Un.copy()
            O.rk_stage(p, s, dt, Un, Us, out)
            Us = out
        U = Us
        assert O.step(p, V) == dt
    assert total > 0
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert np.array_equal(U[:, m], V[:, m])


# ---------------------------------------------------------------- mutations

_FALLBACK = """    int fb = shock || !(RE(qm[0]) > 0.0 && RE(qm[4]) > 0.0) || !(RE(qp[0]) > 0.0 && RE(qp[4]) > 0.0);
    if (fb)
        for (int q = 0; q < 5; q++) { qm[q] = w[q]; qp[q] = w[q]; }"""

MUTATIONS = {
    "offending_face_only": """    int fbm = !(RE(qm[0]) > 0.0 && RE(qm[4]) > 0.0), fbp = !(RE(qp[0]) > 0.0 && RE(qp[4]) > 0.0);
    int fb = shock || fbm || fbp;
    for (int q = 0; q < 5; q++) { if (fbm) qm[q] = w[q]; if (fbp) qp[q] = w[q]; }""",
    "density_and_pressure_only": """    int fb = shock || !(RE(qm[0]) > 0.0 && RE(qm[4]) > 0.0) || !(RE(qp[0]) > 0.0 && RE(qp[4]) > 0.0);
    if (fb)
        for (int q = 0; q < 5; q += 4) { qm[q] = w[q]; qp[q] = w[q]; }""",
    "neighbour_states": """    int fb = shock || !(RE(qm[0]) > 0.0 && RE(qm[4]) > 0.0) || !(RE(qp[0]) > 0.0 && RE(qp[4]) > 0.0);
    if (fb)
        for (int q = 0; q < 5; q++) { qm[q] = w[q - 5]; qp[q] = w[q + 5]; }""",
    "pressure_test_only": """    int fb = shock || !(RE(qm[4]) > 0.0) || !(RE(qp[4]) > 0.0);
    if (fb)
        for (int q = 0; q < 5; q++) { qm[q] = w[q]; qp[q] = w[q]; }""",
    "right_face_test_only": """    int fb = shock || !(RE(qp[0]) > 0.0 && RE(qp[4]) > 0.0);
    if (fb)
        for (int q = 0; q < 5; q++) { qm[q] = w[q]; qp[q] = w[q]; }""",
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_a_mutated_fallback(name, tmp_path):
    src = open(os.path.join(ORACLE_DIR, "forward_body.inc")).read()
    assert src.count(_FALLBACK) == 1, "the fallback's source changed: update the mutations"
    for f in ("oracle.c", "oracle_cs.c", "oracle_amr.c", "oracle.h"):
        shutil.copy(os.path.join(ORACLE_DIR, f), tmp_path / f)
    (tmp_path / "forward_body.inc").write_text(src.replace(_FALLBACK, MUTATIONS[name]))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=gnu11",
                    "-o", str(lib), "oracle.c", "oracle_cs.c", "oracle_amr.c", "-lm"],
                   check=True, cwd=tmp_path, capture_output=True)
    with pytest.raises(AssertionError):
        check_fallback_pointwise(C.CDLL(str(lib)))
