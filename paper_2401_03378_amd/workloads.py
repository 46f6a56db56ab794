"""Seeded synthetic workloads for the block-structured Euler step.

This module builds inputs only: the block descriptor table, the neighbour
links, and the initial conserved state on the guard-padded structure-of-arrays
layout.  It holds none of the solver's arithmetic (no EOS inversion,
reconstruction, Riemann solver or update); it is shared by the GPU path's
callers and by the CPU oracle's tests so that both see bit-identical inputs.

Layout (the paper's blocks, each surrounded by a halo of guard cells, Sec. 2.2
"Flash-X"): one float64 buffer of shape (nvar, ncell_total), variable-major.
Block b occupies cells [offset, offset + (nx+2ng)(ny+2ng)(nz+2ng)) of every
variable plane, x fastest; in 2D nz = 1 and there is no z padding.  Variables
are (rho, m_x, m_y[, m_z], E).  Every padding cell (guards, edges, corners) is
NaN on input, so a read of a cell the method must not use poisons the result.

Links: int32 nbr[6] per block in face order (-x, +x, -y, +y, -z, +z); a value
>= 0 is a neighbour block index, -1 outflow (zero-gradient), -2 periodic onto
the block itself.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

PLM_MC = 0
WENO5 = 1

OUTFLOW = -1
PERIODIC_SELF = -2

BLOCK_DTYPE = np.dtype([("nx", "<i4"), ("ny", "<i4"), ("nz", "<i4"),
                        ("ng", "<i4"), ("offset", "<i8")])
LINK_DTYPE = np.dtype([("nbr", "<i4", (6,))])

# Refinement: a face whose link is LEVEL_FACE touches another level; the AMR
# table says how (kind 1: one coarser block, nbr = (block, o1, o2, -1) with
# (o1, o2) where this face starts on the coarse face, in coarse cells along
# the two transverse axes in x, y, z order; kind 2: the 2^(ndim-1) finer
# blocks covering the face, nbr[h1 + 2 h2] by transverse half).
LEVEL_FACE = -3
AMR_DTYPE = np.dtype([("level", "<i4"), ("kind", "<i4", (6,)), ("nbr", "<i4", (6, 4))])


@dataclasses.dataclass
class Problem:
    name: str
    ndim: int
    recon: int            # PLM_MC or WENO5
    rk: int               # 2 or 3 SSP-RK stages
    gamma: float
    cfl: float
    dx: float
    dy: float
    dz: float
    blocks: np.ndarray    # BLOCK_DTYPE, shape (nblocks,)
    links: np.ndarray     # LINK_DTYPE, shape (nblocks,)
    ncell: int            # cells per variable plane, padding included
    nsteps: int
    U0: np.ndarray        # float64 (nvar, ncell), NaN in all padding
    seed: Optional[int] = None
    grid: Optional[tuple] = None   # (NBx, NBy, NBz, n) for uniform block grids
    amr: Optional[np.ndarray] = None   # AMR_DTYPE per block, for meshes with refinement levels
    origin: Optional[np.ndarray] = None   # (nblocks, 3) lower corner of each block (AMR meshes)
    weno_eps: float = 1e-6   # epsilon of the WENO5 nonlinear weights (Jiang & Shu 1996)
    grav: Optional[tuple] = None          # uniform gravitational acceleration (gx, gy, gz), or None
    shock_thresh: Optional[float] = None  # relative pressure jump of the shock detector, or None (off)

    @property
    def nvar(self) -> int:
        return self.ndim + 2

    @property
    def nblocks(self) -> int:
        return int(self.blocks.shape[0])

    @property
    def interior_zones(self) -> int:
        b = self.blocks
        return int(np.sum(b["nx"].astype(np.int64) * b["ny"] * b["nz"]))

    def copy(self) -> "Problem":
        return dataclasses.replace(self, U0=self.U0.copy(),
                                   blocks=self.blocks.copy(),
                                   links=self.links.copy(),
                                   amr=None if self.amr is None else self.amr.copy())

    def cell_volumes(self) -> np.ndarray:
        """Volume (area in 2D) of every cell of one variable plane (0 in the
        padding): dx dy dz / 2^(ndim level) per block."""
        vol = np.zeros((1, self.ncell))
        base = self.dx * self.dy * (self.dz if self.ndim == 3 else 1.0)
        for b in range(self.nblocks):
            lev = 0 if self.amr is None else int(self.amr[b]["level"])
            interior(vol, self.blocks, b, self.ndim)[...] = base / 2.0 ** (self.ndim * lev)
        return vol[0]


# ----------------------------------------------------------------------------
# block tables
# ----------------------------------------------------------------------------

def padded_shape(nx, ny, nz, ng, ndim):
    """(pz, py, px) extents of a guard-padded block."""
    pz = nz + 2 * ng if ndim == 3 else 1
    return pz, ny + 2 * ng, nx + 2 * ng


def make_table(sizes, ng, ndim):
    """Descriptor table with contiguous offsets in the given block order."""
    blocks = np.zeros(len(sizes), dtype=BLOCK_DTYPE)
    off = 0
    for b, (nx, ny, nz) in enumerate(sizes):
        pz, py, px = padded_shape(nx, ny, nz, ng, ndim)
        blocks[b] = (nx, ny, nz, ng, off)
        off += pz * py * px
    return blocks, off


def uniform_grid(NB, n, ng, ndim, bc):
    """Blocks of n^ndim cells on an NBx x NBy (x NBz) block grid.

    Block index b = (bk*NBy + bj)*NBx + bi (x fastest).  bc is 'outflow' or
    'periodic' (neighbours wrap around the block grid).
    """
    NBx, NBy, NBz = NB
    nz = n if ndim == 3 else 1
    sizes = [(n, n, nz)] * (NBx * NBy * NBz)
    blocks, ncell = make_table(sizes, ng, ndim)
    links = np.zeros(len(sizes), dtype=LINK_DTYPE)
    dims = (NBx, NBy, NBz)
    for bk in range(NBz):
        for bj in range(NBy):
            for bi in range(NBx):
                b = (bk * NBy + bj) * NBx + bi
                pos = [bi, bj, bk]
                nbr = [-1] * 6
                for d in range(ndim):
                    for side, step in ((0, -1), (1, +1)):
                        q = list(pos)
                        q[d] += step
                        if 0 <= q[d] < dims[d]:
                            nbr[2 * d + side] = (q[2] * NBy + q[1]) * NBx + q[0]
                        elif bc == "periodic":
                            q[d] %= dims[d]
                            nb = (q[2] * NBy + q[1]) * NBx + q[0]
                            nbr[2 * d + side] = PERIODIC_SELF if nb == b else nb
                        else:
                            nbr[2 * d + side] = OUTFLOW
                links[b]["nbr"] = nbr
    return blocks, links, ncell


def empty_state(nvar, ncell):
    return np.full((nvar, ncell), np.nan, dtype=np.float64)


def interior(U, blocks, b, ndim):
    """View (nvar, nz, ny, nx) of block b's interior cells."""
    nx, ny, nz, ng, off = (int(blocks[b][f]) for f in ("nx", "ny", "nz", "ng", "offset"))
    pz, py, px = padded_shape(nx, ny, nz, ng, ndim)
    blk = U[:, off:off + pz * py * px].reshape(U.shape[0], pz, py, px)
    gz = ng if ndim == 3 else 0
    return blk[:, gz:gz + nz, ng:ng + ny, ng:ng + nx]


def scatter_global(U, G, blocks, grid, ndim):
    """Write a global (nvar, Nz, Ny, Nx) array into the blocks' interiors."""
    NBx, NBy, NBz, n = grid
    for b in range(len(blocks)):
        bi = b % NBx
        bj = (b // NBx) % NBy
        bk = b // (NBx * NBy)
        nz = n if ndim == 3 else 1
        interior(U, blocks, b, ndim)[...] = G[:, bk * nz:(bk + 1) * nz,
                                              bj * n:(bj + 1) * n,
                                              bi * n:(bi + 1) * n]


def gather_global(U, blocks, grid, ndim):
    """Inverse of scatter_global: global (nvar, Nz, Ny, Nx) interior array."""
    NBx, NBy, NBz, n = grid
    nz = n if ndim == 3 else 1
    G = np.empty((U.shape[0], NBz * nz, NBy * n, NBx * n), dtype=U.dtype)
    for b in range(len(blocks)):
        bi = b % NBx
        bj = (b // NBx) % NBy
        bk = b // (NBx * NBy)
        G[:, bk * nz:(bk + 1) * nz, bj * n:(bj + 1) * n,
          bi * n:(bi + 1) * n] = interior(U, blocks, b, ndim)
    return G


def interior_mask(blocks, ncell, ndim):
    """Boolean mask over one variable plane: True on interior cells."""
    m = np.zeros((1, ncell), dtype=bool)
    for b in range(len(blocks)):
        interior(m, blocks, b, ndim)[...] = True
    return m[0]


def conserved(rho, vel, p, gamma):
    """Initial conserved variables from primitive fields (input set-up only).

    vel is a list of ndim velocity component arrays.
    """
    kin = np.zeros_like(rho)
    for v in vel:
        kin += v * v
    E = p / (gamma - 1.0) + 0.5 * rho * kin
    return np.stack([rho] + [rho * v for v in vel] + [E])


def _streams(seed, k):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


# ----------------------------------------------------------------------------
# the five workloads (and their small variants)
# ----------------------------------------------------------------------------

def sod2d(N=64, n=16, ng=2, axis=0, nsteps=100, cfl=0.8, recon=PLM_MC, rk=2):
    """2D Sod tube: (rho, p) = (1, 1) where the cell centre's coordinate along
    `axis` is < 0.5, else (0.125, 0.1); at rest; outflow on all sides."""
    gamma = 1.4
    NB = N // n
    blocks, links, ncell = uniform_grid((NB, NB, 1), n, ng, 2, "outflow")
    xc = (np.arange(N) + 0.5) / N
    left = xc < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    if axis == 0:
        rho = np.broadcast_to(rho[None, :], (N, N)).copy()
        p = np.broadcast_to(p[None, :], (N, N)).copy()
    else:
        rho = np.broadcast_to(rho[:, None], (N, N)).copy()
        p = np.broadcast_to(p[:, None], (N, N)).copy()
    z = np.zeros((N, N))
    G = conserved(rho, [z, z], p, gamma)[:, None]   # (4, 1, N, N)
    U = empty_state(4, ncell)
    scatter_global(U, G, blocks, (NB, NB, 1, n), 2)
    return Problem("sod2d", 2, recon, rk, gamma, cfl, 1.0 / N, 1.0 / N, 1.0,
                   blocks, links, ncell, nsteps, U, None, (NB, NB, 1, n))


def sedov3d(N=128, n=16, ng=3, nsteps=20, cfl=0.5, recon=WENO5, rk=3,
            radius_cells=3.5):
    """3D Sedov blast: rho = 1, p = 1e-5, at rest; total energy 1 spread
    uniformly over the cells whose centres lie within radius_cells*dx of the
    domain centre; outflow boundaries."""
    gamma = 1.4
    NB = N // n
    blocks, links, ncell = uniform_grid((NB, NB, NB), n, ng, 3, "outflow")
    xc = (np.arange(N) + 0.5) / N - 0.5
    r2 = (xc[:, None, None] ** 2 + xc[None, :, None] ** 2 + xc[None, None, :] ** 2) * N * N
    hot = r2 < radius_cells ** 2
    nhot = int(hot.sum())
    dV = (1.0 / N) ** 3
    rho = np.ones((N, N, N))
    p = np.full((N, N, N), 1e-5)
    z = np.zeros((N, N, N))
    G = conserved(rho, [z, z, z], p, gamma)
    G[4][hot] += 1.0 / (nhot * dV)
    U = empty_state(5, ncell)
    scatter_global(U, G, blocks, (NB, NB, NB, n), 3)
    prob = Problem("sedov3d", 3, recon, rk, gamma, cfl, 1.0 / N, 1.0 / N, 1.0 / N,
                   blocks, links, ncell, nsteps, U, None, (NB, NB, NB, n))
    prob.nhot = nhot
    return prob


def batched_uneven(nblocks=4096, fractions=(0.5, 0.4, 0.1), sizes=(8, 16, 32),
                   ng=2, seed=0, nsteps=10, cfl=0.8, recon=PLM_MC, rk=2,
                   dx=1.0 / 32):
    """Independent periodic blocks of uneven sizes advanced together.

    Counts per size are floor(f*nblocks) for all but the last size, which
    takes the remainder (4096 -> 2048, 1638, 410); the size sequence is a seeded permutation and offsets follow it.  Per
    cell, independently: rho = exp(0.3 N(0,1)), p = exp(0.3 N(0,1)),
    u_d = 0.3 c N(0,1) with c = sqrt(gamma p / rho); gamma = 5/3.
    """
    gamma = 5.0 / 3.0
    counts = [int(math.floor(f * nblocks)) for f in fractions[:-1]]
    counts.append(nblocks - sum(counts))
    r_perm, r_field = _streams(seed, 2)
    seq = np.concatenate([np.full(c, s) for c, s in zip(counts, sizes)])
    seq = seq[r_perm.permutation(len(seq))]
    blocks, ncell = make_table([(s, s, s) for s in seq], ng, 3)
    links = np.zeros(nblocks, dtype=LINK_DTYPE)
    links["nbr"] = PERIODIC_SELF
    U = empty_state(5, ncell)
    for b, s in enumerate(seq):
        shp = (s, s, s)
        rho = np.exp(0.3 * r_field.standard_normal(shp))
        p = np.exp(0.3 * r_field.standard_normal(shp))
        c = np.sqrt(gamma * p / rho)
        vel = [0.3 * c * r_field.standard_normal(shp) for _ in range(3)]
        interior(U, blocks, b, 3)[...] = conserved(rho, vel, p, gamma)
    return Problem("batched_uneven", 3, recon, rk, gamma, cfl, dx, dx, dx,
                   blocks, links, ncell, nsteps, U, seed, None)


def kh2d(N=256, n=16, ng=2, seed=0, nsteps=50, cfl=0.8, recon=PLM_MC, rk=2):
    """2D Kelvin-Helmholtz: rho = 2, u_x = +0.5 in the strip |y - 0.5| < 0.25,
    else rho = 1, u_x = -0.5; p = 2.5; v_y = 0.01 * s(x)/max|s| with
    s(x) = sum_{m=1..4} a_m sin(2 pi m x + phi_m), a_m ~ N(0,1),
    phi_m ~ U(0, 2 pi) (seeded); periodic."""
    gamma = 1.4
    NB = N // n
    blocks, links, ncell = uniform_grid((NB, NB, 1), n, ng, 2, "periodic")
    (r,) = _streams(seed, 1)
    a = r.standard_normal(4)
    phi = r.uniform(0.0, 2.0 * np.pi, 4)
    xc = (np.arange(N) + 0.5) / N
    s = sum(a[m] * np.sin(2.0 * np.pi * (m + 1) * xc + phi[m]) for m in range(4))
    vy1 = 0.01 * s / np.max(np.abs(s))
    strip = np.abs(xc - 0.5) < 0.25                     # by y index
    rho = np.where(strip[:, None], 2.0, 1.0) * np.ones((N, N))
    ux = np.where(strip[:, None], 0.5, -0.5) * np.ones((N, N))
    vy = np.broadcast_to(vy1[None, :], (N, N)).copy()
    p = np.full((N, N), 2.5)
    G = conserved(rho, [ux, vy], p, gamma)[:, None]
    U = empty_state(4, ncell)
    scatter_global(U, G, blocks, (NB, NB, 1, n), 2)
    return Problem("kh2d", 2, recon, rk, gamma, cfl, 1.0 / N, 1.0 / N, 1.0,
                   blocks, links, ncell, nsteps, U, seed, (NB, NB, 1, n))


def turb3d(N=256, n=16, ng=3, seed=0, nsteps=20, cfl=0.5, recon=WENO5, rk=3,
           mach=0.5):
    """3D turbulence-like field: rho = 1, p = 1/gamma (so c = 1), velocity
    components from seeded white noise filtered by |k|^-2 in Fourier space
    (power ~ |k|^-4), mean removed, one common factor giving rms |u| = mach;
    periodic."""
    gamma = 1.4
    NB = N // n
    blocks, links, ncell = uniform_grid((NB, NB, NB), n, ng, 3, "periodic")
    rs = _streams(seed, 3)
    k1 = np.fft.fftfreq(N) * N
    kr = np.fft.rfftfreq(N) * N
    k2 = k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kr[None, None, :] ** 2
    filt = np.zeros_like(k2)
    filt[k2 > 0] = 1.0 / k2[k2 > 0]
    vel = []
    for d in range(3):
        w = rs[d].standard_normal((N, N, N))
        vel.append(np.fft.irfftn(np.fft.rfftn(w) * filt, s=(N, N, N), axes=(0, 1, 2)))
    rms = math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)))
    vel = [v * (mach / rms) for v in vel]
    rho = np.ones((N, N, N))
    p = np.full((N, N, N), 1.0 / gamma)
    G = conserved(rho, vel, p, gamma)
    U = empty_state(5, ncell)
    scatter_global(U, G, blocks, (NB, NB, NB, n), 3)
    return Problem("turb3d", 3, recon, rk, gamma, cfl, 1.0 / N, 1.0 / N, 1.0 / N,
                   blocks, links, ncell, nsteps, U, seed, (NB, NB, NB, n))


def random_blocks(ndim, sizes, ng, seed, recon=PLM_MC, rk=2, gamma=1.4, cfl=0.8,
                  bc="periodic", NB=None, amp=0.3):
    """Small random smooth-free state on a block grid (test fixtures).

    sizes: n (cells per block side).  NB: block grid (defaults to 2 per dim).
    """
    n = sizes
    if NB is None:
        NB = (2, 2, 2 if ndim == 3 else 1)
    blocks, links, ncell = uniform_grid(NB, n, ng, ndim, bc)
    (r,) = _streams(seed, 1)
    nz = n * NB[2] if ndim == 3 else 1
    shp = (nz, n * NB[1], n * NB[0])
    rho = np.exp(amp * r.standard_normal(shp))
    p = np.exp(amp * r.standard_normal(shp))
    c = np.sqrt(gamma * p / rho)
    vel = [amp * c * r.standard_normal(shp) for _ in range(ndim)]
    G = conserved(rho, vel, p, gamma)
    U = empty_state(ndim + 2, ncell)
    scatter_global(U, G, blocks, (NB[0], NB[1], NB[2], n), ndim)
    dx = 1.0 / (n * NB[0])
    return Problem("random", ndim, recon, rk, gamma, cfl, dx, dx,
                   dx if ndim == 3 else 1.0, blocks, links, ncell, 1, U, seed,
                   (NB[0], NB[1], NB[2], n))


def rectilinear(ndim, widths, ng, seed, recon=PLM_MC, rk=2, gamma=1.4, cfl=0.8, bc="periodic", amp=0.3):
    """Random smooth-free state on a block grid whose columns, rows (and
    layers) have their own widths (test fixtures): widths = (wx, wy[, wz]),
    block (i, j, k) has wx[i] x wy[j] x wz[k] cells, so neighbours across a
    face share that face's size but not their extent along its normal (nor
    their padded plane size).  Block index (k*NBy + j)*NBx + i."""
    wx, wy = list(widths[0]), list(widths[1])
    wz = list(widths[2]) if ndim == 3 else [1]
    NB = (len(wx), len(wy), len(wz))
    sizes = [(wx[i], wy[j], wz[k]) for k in range(NB[2]) for j in range(NB[1]) for i in range(NB[0])]
    blocks, ncell = make_table(sizes, ng, ndim)
    _, links, _ = uniform_grid(NB, 1, ng, ndim, bc)       # the same block graph
    (r,) = _streams(seed, 1)
    shp = (sum(wz), sum(wy), sum(wx))
    rho = np.exp(amp * r.standard_normal(shp))
    p = np.exp(amp * r.standard_normal(shp))
    c = np.sqrt(gamma * p / rho)
    vel = [amp * c * r.standard_normal(shp) for _ in range(ndim)]
    G = conserved(rho, vel, p, gamma)
    U = empty_state(ndim + 2, ncell)
    ox, oy, oz = np.cumsum([0] + wx), np.cumsum([0] + wy), np.cumsum([0] + wz)
    for b in range(len(sizes)):
        i, j, k = b % NB[0], (b // NB[0]) % NB[1], b // (NB[0] * NB[1])
        interior(U, blocks, b, ndim)[...] = G[:, oz[k]:oz[k + 1], oy[j]:oy[j + 1], ox[i]:ox[i + 1]]
    dx = 1.0 / sum(wx)
    return Problem("rectilinear", ndim, recon, rk, gamma, cfl, dx, dx, dx if ndim == 3 else 1.0,
                   blocks, links, ncell, 1, U, seed)


def free_fall(ndim, n=8, ng=2, recon=PLM_MC, rk=2, NB=None, grav=(0.3, -2.0, 0.5), rho=1.3,
              vel=(0.2, -0.1, 0.3), p=0.7, gamma=1.4, cfl=0.8):
    """A uniform gas in a periodic box under a uniform gravitational
    acceleration: every cell holds the same (rho, u, p)."""
    if NB is None:
        NB = (2, 2, 2 if ndim == 3 else 1)
    blocks, links, ncell = uniform_grid(NB, n, ng, ndim, "periodic")
    nz = n * NB[2] if ndim == 3 else 1
    shp = (nz, n * NB[1], n * NB[0])
    G = conserved(np.full(shp, rho), [np.full(shp, v) for v in vel[:ndim]], np.full(shp, p), gamma)
    U = empty_state(ndim + 2, ncell)
    scatter_global(U, G, blocks, (NB[0], NB[1], NB[2], n), ndim)
    dx = 1.0 / (n * NB[0])
    return Problem("free_fall", ndim, recon, rk, gamma, cfl, dx, dx, dx if ndim == 3 else 1.0,
                   blocks, links, ncell, 1, U, None, (NB[0], NB[1], NB[2], n), grav=tuple(grav))


def atmosphere2d(N=64, n=16, ng=2, g=1.0, recon=PLM_MC, rk=2, gamma=1.4, cfl=0.8):
    """Isothermal atmosphere at rest in the unit square: rho = p = exp(-g y)
    at cell centres (hydrostatic for an acceleration of g along -y), periodic
    along x, outflow at the bottom and top faces."""
    NB = N // n
    blocks, links, ncell = uniform_grid((NB, NB, 1), n, ng, 2, "periodic")
    for b in range(len(links)):
        nbr = links[b]["nbr"].copy()
        bj = (b // NB) % NB
        if bj == 0:
            nbr[2] = OUTFLOW
        if bj == NB - 1:
            nbr[3] = OUTFLOW
        links[b]["nbr"] = nbr
    yc = (np.arange(N) + 0.5) / N
    rho = np.broadcast_to(np.exp(-g * yc)[:, None], (N, N)).copy()
    z = np.zeros((N, N))
    G = conserved(rho, [z, z], rho.copy(), gamma)[:, None]
    U = empty_state(4, ncell)
    scatter_global(U, G, blocks, (NB, NB, 1, n), 2)
    return Problem("atmosphere2d", 2, recon, rk, gamma, cfl, 1.0 / N, 1.0 / N, 1.0,
                   blocks, links, ncell, 1, U, None, (NB, NB, 1, n), grav=(0.0, -g, 0.0))


def amr_mesh(ndim, NBc, n, ng, refine, bc="periodic"):
    """Two-level mesh: a periodic NBc block grid of n^ndim-cell blocks at level
    0, where the coarse blocks at the positions in `refine` are replaced by
    their 2^ndim children (level 1, n^ndim cells of half the width).

    Returns (blocks, links, amr, origin, ncell); origin is each block's lower
    corner in units of level-0 cells.  Block order: the unrefined coarse blocks
    (x fastest), then the children of each refined block (x fastest).  bc:
    'periodic' (the block grid wraps) or 'outflow' on the domain faces.
    """
    NB = tuple(NBc) + (1,) * (3 - len(NBc))
    if ndim == 2:
        NB = (NB[0], NB[1], 1)
    refine = {tuple(r) + (0,) * (3 - len(r)) for r in refine}
    order = []              # (level, position in that level's block grid)
    for K in range(NB[2]):
        for J in range(NB[1]):
            for I in range(NB[0]):
                if (I, J, K) not in refine:
                    order.append((0, (I, J, K)))
    for (I, J, K) in sorted(refine, key=lambda q: (q[2], q[1], q[0])):
        for c in range(2 ** ndim):
            a, b_, e = c & 1, (c >> 1) & 1, (c >> 2) & 1
            order.append((1, (2 * I + a, 2 * J + b_, 2 * K + e if ndim == 3 else 0)))
    index = {key: i for i, key in enumerate(order)}
    nz = n if ndim == 3 else 1
    blocks, ncell = make_table([(n, n, nz)] * len(order), ng, ndim)
    links = np.zeros(len(order), dtype=LINK_DTYPE)
    amr = np.zeros(len(order), dtype=AMR_DTYPE)
    amr["nbr"] = -1
    origin = np.zeros((len(order), 3))
    for i, (lev, pos) in enumerate(order):
        dims = [NB[d] * 2 ** lev for d in range(3)]
        amr[i]["level"] = lev
        origin[i] = [pos[d] * n / 2 ** lev if d < ndim else 0.0 for d in range(3)]
        nbr = [OUTFLOW] * 6
        for d in range(ndim):
            t = [e for e in range(3) if e != d]          # transverse axes, x, y, z order
            for side, step in ((0, -1), (1, 1)):
                f = 2 * d + side
                q = list(pos)
                q[d] = q[d] + step
                if not 0 <= q[d] < dims[d]:
                    if bc == "outflow":
                        nbr[f] = OUTFLOW
                        continue
                    q[d] %= dims[d]
                if (lev, tuple(q)) in index:
                    nb = index[(lev, tuple(q))]
                    nbr[f] = PERIODIC_SELF if nb == i else nb
                elif lev == 1 and (0, tuple(x // 2 for x in q)) in index:
                    nbr[f] = LEVEL_FACE
                    amr[i]["kind"][f] = 1
                    amr[i]["nbr"][f] = [index[(0, tuple(x // 2 for x in q))],
                                        (pos[t[0]] % 2) * (n // 2),
                                        (pos[t[1]] % 2) * (n // 2) if ndim == 3 else 0, -1]
                elif lev == 0:
                    nbr[f] = LEVEL_FACE
                    amr[i]["kind"][f] = 2
                    fine = []
                    for h in range(2 ** (ndim - 1)):
                        r = [0, 0, 0]
                        r[d] = 2 * q[d] + (1 if side == 0 else 0)
                        r[t[0]] = 2 * pos[t[0]] + (h & 1)
                        r[t[1]] = (2 * pos[t[1]] + (h >> 1)) if ndim == 3 else 0
                        fine.append(index[(1, tuple(r))])
                    amr[i]["nbr"][f] = fine + [-1] * (4 - len(fine))
                else:
                    raise ValueError("levels may differ by one across a face")
        links[i]["nbr"] = nbr
    return blocks, links, amr, origin, ncell


def amr_problem(ndim, NBc=(4, 4, 4), n=8, ng=2, refine=None, seed=0, recon=PLM_MC, rk=2,
                gamma=1.4, cfl=0.5, nsteps=5, flow="blob", bc=None):
    """A two-level mesh (see amr_mesh; by default the central 2^ndim coarse
    blocks are refined) with a smooth state: a density and pressure bump
    moving diagonally through the refined patch ("blob"), seeded smooth random
    fields ("random"), both periodic; or a Sedov-like blast at the domain
    centre, inside the refined patch, with outflow faces ("blast": rho = 1,
    p = 1e-5, total energy 1 spread over the level-0 cell volume within 3.5
    level-0 cells of the centre).  dx = 1 / (NBc[0] n) at level 0."""
    NBc = tuple(NBc[:ndim])
    if refine is None:
        refine = [tuple(c // 2 - 1 + a for c, a in zip(NBc, idx))
                  for idx in np.ndindex(*(2,) * ndim)]
    if bc is None:
        bc = "outflow" if flow == "blast" else "periodic"
    blocks, links, amr, origin, ncell = amr_mesh(ndim, NBc, n, ng, refine, bc)
    nb = len(blocks)
    U = empty_state(ndim + 2, ncell)
    L = [NBc[d] * n for d in range(ndim)]                 # domain extent in level-0 cells
    (r,) = _streams(seed, 1)
    modes = [(r.integers(1, 3, ndim), r.uniform(0, 2 * np.pi), r.uniform(-1, 1)) for _ in range(4)]
    dx0 = 1.0 / L[0]
    if flow == "blast":
        # volume (physical units) of the cells whose centres lie in the deposit
        blast_volume = 0.0
        for b in range(nb):
            lev = int(amr[b]["level"])
            h = 1.0 / 2 ** lev
            c = [origin[b][d] + (np.arange(n) + 0.5) * h for d in range(ndim)]
            g = np.meshgrid(*c, indexing="ij")
            r2 = sum((gg - 0.5 * L[0]) ** 2 for gg in g)
            blast_volume += np.count_nonzero(r2 < 3.5 ** 2) * (h * dx0) ** ndim
    for b in range(nb):
        lev = int(amr[b]["level"])
        h = 1.0 / 2 ** lev
        c = [origin[b][d] + (np.arange(n) + 0.5) * h for d in range(ndim)]     # cell centres
        if ndim == 3:
            X = np.meshgrid(c[0] / L[0], c[1] / L[1], c[2] / L[2], indexing="ij")
            X = [x.transpose(2, 1, 0) for x in X]                 # (z, y, x)
        else:
            X = np.meshgrid(c[0] / L[0], c[1] / L[1], indexing="ij")
            X = [x.T[None] for x in X]                            # (1, y, x)
        if flow == "blast":
            r2 = sum(((x - 0.5) * L[0]) ** 2 for x in X)          # in level-0 cells (cubic domain)
            hot = r2 < 3.5 ** 2
            rho = np.ones_like(r2)
            p = np.full_like(r2, 1e-5)
            vel = [np.zeros_like(r2) for _ in range(ndim)]
            U_b = conserved(rho, vel, p, gamma)
            # energy density making the deposit's total 1 over its volume
            vol0 = blast_volume
            U_b[-1] = np.where(hot, U_b[-1] + 1.0 / vol0, U_b[-1])
            interior(U, blocks, b, ndim)[...] = U_b
            continue
        if flow == "blob":
            r2 = sum((np.minimum(np.abs(x - 0.3), 1 - np.abs(x - 0.3))) ** 2 for x in X)
            bump = np.exp(-r2 / 0.02)
            rho = 1.0 + 0.5 * bump
            p = 1.0 + 0.3 * bump
            vel = [np.full_like(rho, v) for v in (0.6, 0.4, 0.3)[:ndim]]
        else:
            field = lambda k: sum(a * np.sin(2 * np.pi * sum(int(m[d]) * X[d] for d in range(ndim)) + ph + k)
                                  for m, ph, a in modes)
            rho = np.exp(0.2 * field(0.0))
            p = np.exp(0.2 * field(1.0))
            vel = [0.3 * field(2.0 + d) for d in range(ndim)]
        interior(U, blocks, b, ndim)[...] = conserved(rho, vel, p, gamma)
    dx = 1.0 / L[0]
    return Problem(f"amr{ndim}d", ndim, recon, rk, gamma, cfl, dx, dx, dx if ndim == 3 else 1.0,
                   blocks, links, ncell, nsteps, U, seed, None, amr, origin)


def config(i: int, seed: int = 0) -> Problem:
    """The five named workloads, numbered 0..4."""
    if i == 0:
        return sod2d()
    if i == 1:
        return sedov3d()
    if i == 2:
        return batched_uneven(seed=seed)
    if i == 3:
        return kh2d(seed=seed)
    if i == 4:
        return turb3d(seed=seed)
    raise ValueError(f"no workload {i}")
