"""Pins of the oracle's AMR step (refinement ratio 2, flux correction at
coarse-fine faces; the paper's Sec. 4.2 flux-correction listings): exact
conservation with the correction and not without it, the two correction
orders agreeing bit for bit, a uniform state kept exactly, the guard rules
checked cell by cell, and the limits of no refinement and of refining
everything (CPU only)."""
import numpy as np
import pytest

import oracle as O
from paper_2401_03378_amd import workloads as W


def _totals(p, U):
    m = W.interior_mask(p.blocks, p.ncell, p.ndim)
    vol = p.cell_volumes()
    return np.array([np.sum(U[v, m] * vol[m]) for v in range(p.nvar)])


CASES = [(2, 0, 2, 8, 2), (2, 1, 3, 8, 3), (3, 0, 2, 8, 2), (3, 1, 3, 8, 3)]


@pytest.mark.parametrize("ndim,recon,rk,n,ng", CASES)
def test_generated_meshes_validate(ndim, recon, rk, n, ng):
    p = W.amr_problem(ndim, n=n, ng=ng, recon=recon, rk=rk)
    assert O.amr_validate(p) == O.ORA_OK


def test_broken_tables_are_rejected():
    p = W.amr_problem(2, n=8)
    i = int(np.flatnonzero(p.amr["kind"][:, 3] == 2)[0])           # a coarse block with fine +y neighbours
    for mutate in (lambda a: a[i]["nbr"].__setitem__((3, 0), a[i]["nbr"][3][1]),   # same fine block twice
                   lambda a: a[i].__setitem__("level", 1),                           # no level gap left
                   lambda a: a[i]["kind"].__setitem__(3, 1)):                        # wrong kind
        q = p.copy()
        mutate(q.amr)
        assert O.amr_validate(q) == O.ORA_EINVAL
    j = int(np.flatnonzero(p.amr["kind"][:, 2] == 1)[0])            # a fine block under a coarse one
    q = p.copy()
    q.amr[j]["nbr"][2][1] = 1                                       # offset not a half face
    assert O.amr_validate(q) == O.ORA_EINVAL


@pytest.mark.parametrize("ndim,recon,rk,n,ng", CASES)
def test_flux_correction_conserves(ndim, recon, rk, n, ng):
    """Periodic domain: with the correction every conserved total is kept to
    rounding; without it the coarse and fine fluxes through the coarse-fine
    faces differ and the totals drift."""
    p = W.amr_problem(ndim, n=n, ng=ng, recon=recon, rk=rk, flow="random", seed=3)
    t0 = _totals(p, p.U0)
    U = p.U0.copy()
    O.amr_run(p, U, 4)
    t1 = _totals(p, U)
    scale = np.abs(t0) + 1.0
    assert np.max(np.abs(t1 - t0) / scale) < 5e-15
    V = p.U0.copy()
    O.amr_run(p, V, 4, order=O.AMR_NO_CORRECTION)
    assert np.max(np.abs(_totals(p, V) - t0) / scale) > 1e-9


@pytest.mark.parametrize("ndim,recon,rk,n,ng", CASES)
def test_level_by_level_equals_all_levels(ndim, recon, rk, n, ng):
    p = W.amr_problem(ndim, n=n, ng=ng, recon=recon, rk=rk, seed=1)
    a, b = p.U0.copy(), p.U0.copy()
    da = O.amr_run(p, a, 3, order=O.AMR_ALL_LEVELS)
    db = O.amr_run(p, b, 3, order=O.AMR_LEVEL_BY_LEVEL)
    m = W.interior_mask(p.blocks, p.ncell, ndim)
    assert da == db and np.array_equal(a[:, m], b[:, m])


@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_state_is_kept_exactly(ndim):
    p = W.amr_problem(ndim, n=8, ng=3, recon=1, rk=3)
    m = W.interior_mask(p.blocks, p.ncell, ndim)
    vals = [1.3, 0.4, -0.7, 0.2, 2.9][:p.nvar - 1] + [2.9]
    for v, val in enumerate(vals):
        p.U0[v, m] = val
    U = p.U0.copy()
    O.amr_run(p, U, 3)
    assert np.array_equal(U[:, m], p.U0[:, m])


def test_guard_rules_cell_by_cell():
    """Fine guards behind a coarse face take the containing coarse cell; coarse
    guards behind fine faces take the pairwise sum of the covered fine cells
    times 2^-ndim (checked by brute force from block geometry)."""
    for ndim in (2, 3):
        p = W.amr_problem(ndim, n=8, ng=3, recon=1, rk=3, flow="random", seed=5)
        U = p.U0.copy()
        O.amr_fill_guards(p, U)
        n, ng = 8, 3
        def at(b, ijk):        # interior cell (i, j[, k]) of block b in the input state
            zyx = tuple(reversed(ijk)) if ndim == 3 else (0,) + tuple(reversed(ijk))
            return W.interior(p.U0, p.blocks, b, ndim)[(slice(None),) + zyx]
        checked = 0
        for b in range(p.nblocks):
            lev = int(p.amr[b]["level"])
            h = 0.5 ** lev
            for d in range(ndim):
                for side in range(2):
                    f = 2 * d + side
                    kind = int(p.amr[b]["kind"][f])
                    if kind == 0:
                        continue
                    nbr = p.amr[b]["nbr"][f]
                    for l in range(1, ng + 1):
                        for e in np.ndindex(*(n,) * (ndim - 1)):
                            idx = [0] * ndim
                            t = [a for a in range(ndim) if a != d]
                            idx[d] = -l if side == 0 else n - 1 + l
                            for a, ev in zip(t, e):
                                idx[a] = ev
                            nx, ny, nz, g, off = (int(p.blocks[b][k]) for k in ("nx", "ny", "nz", "ng", "offset"))
                            pz = nz + 2 * g if ndim == 3 else 1
                            blk = U[:, off:off + pz * (ny + 2 * g) * (nx + 2 * g)].reshape(p.nvar, pz, ny + 2 * g, nx + 2 * g)
                            gk = idx[2] + g if ndim == 3 else 0
                            got = blk[:, gk, idx[1] + g, idx[0] + g]
                            # physical centre of the guard cell
                            ctr = [p.origin[b][a] + (idx[a] + 0.5) * h for a in range(ndim)]
                            if kind == 1:
                                c = int(nbr[0])
                                ci = [int(np.floor(ctr[a] - p.origin[c][a])) for a in range(ndim)]
                                want = at(c, ci)
                            else:
                                # fine blocks covering the coarse guard cell: centres at +-1/4
                                vals = []
                                for q in np.ndindex(*(2,) * ndim):
                                    pt = [ctr[a] + (q[a] - 0.5) * 0.5 for a in range(ndim)]
                                    for fb in nbr[:2 ** (ndim - 1)]:
                                        fi = [int(np.floor((pt[a] - p.origin[fb][a]) * 2)) for a in range(ndim)]
                                        if all(0 <= x < n for x in fi):
                                            vals.append((q, at(fb, fi)))
                                assert len(vals) == 2 ** ndim
                                # pairwise: normal pair, then transverse 1, then transverse 2
                                def key(q):
                                    return tuple(q[a] for a in reversed(t)) + (q[d],)
                                vals.sort(key=lambda x: key(x[0]))
                                v = [x[1] for x in vals]
                                if ndim == 2:
                                    want = ((v[0] + v[1]) + (v[2] + v[3])) * 0.25
                                else:
                                    want = (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) * 0.125
                            assert np.array_equal(got, want), (ndim, b, f, l, e)
                            checked += 1
        assert checked > 0


def test_no_refinement_is_the_uniform_step():
    p = W.amr_problem(3, NBc=(2, 2, 2), n=8, ng=3, recon=1, rk=3, refine=[], flow="random", seed=2)
    q = W.random_blocks(3, 8, 3, seed=0, recon=1, rk=3, bc="periodic", NB=(2, 2, 2), cfl=p.cfl)
    q.U0 = p.U0.copy()
    a, b = p.U0.copy(), p.U0.copy()
    da = O.amr_run(p, a, 2)
    db = O.run(q, b, 2)
    m = W.interior_mask(p.blocks, p.ncell, 3)
    assert da == db and np.array_equal(a[:, m], b[:, m])


def test_refining_everything_is_the_fine_uniform_step():
    """All coarse blocks refined: the level-1 mesh is a uniform grid of half
    the cell width; the AMR step equals the uniform step on it bit for bit."""
    NBc = (2, 2)
    p = W.amr_problem(2, NBc=NBc, n=8, ng=2, recon=0, rk=2, refine=[(i, j) for i in range(2) for j in range(2)],
                      flow="random", seed=4)
    q = W.random_blocks(2, 8, 2, seed=0, recon=0, rk=2, bc="periodic", NB=(4, 4, 1), cfl=p.cfl)
    q.dx = q.dy = p.dx / 2
    # move the AMR blocks' states into the uniform grid's block order
    U = q.U0.copy()
    for b in range(p.nblocks):
        I, J = (int(round(p.origin[b][a] * 2 / 8)) for a in range(2))
        W.interior(U, q.blocks, J * 4 + I, 2)[...] = W.interior(p.U0, p.blocks, b, 2)
    a = p.U0.copy()
    da = O.amr_run(p, a, 3)
    db = O.run(q, U, 3)
    assert da == db
    for b in range(p.nblocks):
        I, J = (int(round(p.origin[b][a_] * 2 / 8)) for a_ in range(2))
        assert np.array_equal(W.interior(a, p.blocks, b, 2), W.interior(U, q.blocks, J * 4 + I, 2))


@pytest.mark.parametrize("recon,rk,nsteps", [(0, 2, 5), (1, 3, 2)])
def test_refined_patch_equals_the_fine_uniform_grid(recon, rk, nsteps):
    """A blast inside a refined patch, before its disturbance (grown by the
    stencil reach every stage) gets near the coarse-fine faces: the fine
    blocks' states equal those of a uniform grid of the fine width bit for
    bit (same dt: the CFL maximum lies in the blast), so the level scaling,
    the guard fill and the correction leave a locally uniform-grid
    computation untouched."""
    ng = 3 if recon == 1 else 2
    p = W.amr_problem(2, NBc=(8, 8), n=8, ng=ng, recon=recon, rk=rk, flow="blast",
                      refine=[(i, j) for i in range(2, 6) for j in range(2, 6)])
    q = W.random_blocks(2, 8, ng, seed=0, recon=recon, rk=rk, bc="outflow", NB=(16, 16, 1), cfl=p.cfl)
    q.dx = q.dy = p.dx / 2
    # uniform grid: the blast's fine cells where the patch is, the quiet state elsewhere
    quiet = np.array([1.0, 0.0, 0.0, 1e-5 / (p.gamma - 1.0)])
    U = q.U0.copy()
    for b in range(q.nblocks):
        W.interior(U, q.blocks, b, 2)[...] = quiet[:, None, None, None]
    where = {}
    for b in range(p.nblocks):
        if p.amr[b]["level"] == 1:
            I, J = (int(round(p.origin[b][a] * 2 / 8)) for a in range(2))
            where[b] = J * 16 + I
            W.interior(U, q.blocks, where[b], 2)[...] = W.interior(p.U0, p.blocks, b, 2)
    a = p.U0.copy()
    da = O.amr_run(p, a, nsteps)
    db = O.run(q, U, nsteps)
    assert da == db
    moved = 0
    for b, qb in where.items():
        fa, fb = W.interior(a, p.blocks, b, 2), W.interior(U, q.blocks, qb, 2)
        assert np.array_equal(fa, fb), b
        moved += int(np.any(fa != quiet[:, None, None, None]))
    assert moved >= 4          # the blast has spread over several fine blocks
