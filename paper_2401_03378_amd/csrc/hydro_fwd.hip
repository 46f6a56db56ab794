// Forward kernels of the FP64 Euler step on gfx950.
//
//  k_stage      fused stage: guard gather + EOS + reconstruction + HLLC +
//               flux difference + SSP-RK combine, one launch for all blocks
//               (the paper's per-stage block loop with the intra-stage chain
//               calcLims -> calcFlux -> updSoln -> calcEos, Sec. 4.2).
//  k_cfl_*      CFL time step: per-workgroup max of the wave-speed sum,
//               then a one-workgroup reduction to dt on the device.
//  k_stage_cfl  the stage kernel that also records those maxima for the
//               state it writes (the last stage of a step whose successor
//               takes its dt from them).
//  k_fill_guards  materialised guard fill (the listing's fill_guardcells)
//               for callers that want guards in the array, and for the
//               plain per-block launch form.
//  k_stage_lv, k_amr_fill, k_amr_correct  meshes with refinement levels
//               (the paper's flux-correction listings, Sec. 4.2): the stage
//               kernel that also writes the fluxes through faces to another
//               level into flux registers, the guard layers of those faces,
//               and the correction of the coarse cells next to finer faces.
//  k_tele_*     thick block copies of the telescoping step.
//
// Work decomposition of k_stage.  A work item is an xy tile (TX x TY cells)
// of one block over a run of z planes.  The workgroup marches through the
// planes: each thread owns one column and keeps the primitive variables of a
// (2R+1)-cell window along z in registers, so z-faces are reconstructed and
// solved once and the flux of the lower face is carried to the next plane.
// The current plane, with its x and y halo of R+1 cells, is staged in LDS as
// primitives; x and y reconstruction read their stencils from there.  Guard
// cells are never read from the state array: a halo cell outside the block
// is gathered from the cell it is a copy of (neighbour interior, periodic
// wrap, outflow copy); only the guard layers of faces to another refinement
// level are read from the array, after k_amr_fill has written them.  A
// persistent grid walks the work list with a fixed stride.
#include "hydro_kernels.h"

namespace hydro {

// Wave priority (0..3) for the issue arbiter of the SIMD.
__device__ __forceinline__ void set_prio(int p)
{
    if (p >= 3) __builtin_amdgcn_s_setprio(3);
    else if (p == 2) __builtin_amdgcn_s_setprio(2);
    else if (p == 1) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

template <int NDIM, int RECON, int TX, int TY, bool GATHER, bool PF, bool LV = false, bool CFLO = false,
          bool PHYS = false>
__device__ __forceinline__ void stage_body(const StageArgs &A)
{
    constexpr int R = (RECON == kWENO) ? 2 : 1;
    constexpr int H = R + 1;
    constexpr int NV = NDIM + 2;
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;
    constexpr int NT = TX * TY;
    constexpr int NW = 2 * R + 1;   // z window
    __shared__ double sW[5][LY][LX];
    __shared__ double sQx[5][TY][TX + 1];
    __shared__ double sQy[5][TY + 1][TX];
    // the face fluxes take the place of the face states: each slot is read
    // (its left state) and then written (its flux) by the one thread that
    // solves that face, and the next write of a state follows a barrier
    auto &sFx = sQx;
    auto &sFy = sQy;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int64_t nc = A.nc;
    const Consts K{A.gamma, A.g1, A.ig1};
    const double dt = *A.dt;
    bool bad = false;
    // PHYS: the shock detector's flags decide first-order faces; gravity adds
    // its source in the update (both uniform over the launch)
    const bool shk = PHYS && (A.phys & kShock);
    const bool grv = PHYS && (A.phys & kGravity);
    // CFLO: each thread's maximum of the CFL wave-speed sum of the cells it writes
    __shared__ double sCfl[CFLO ? NT : 1];
    if constexpr (CFLO) sCfl[tid] = 0.0;

    for (int w = blockIdx.x; w < A.nitems; w += gridDim.x) {
        const WorkItem it = A.items[w];
        const DevBlock B = A.blocks[it.block];
        const FaceSrc *F6 = A.faces + 6 * (int64_t)it.block;
        const int x0 = it.xy & 0xffff, y0 = it.xy >> 16;
        const int z0 = it.z & 0xffff, nzc = it.z >> 16;
        const int wx = min(TX, B.nx - x0), wy = min(TY, B.ny - y0);
        // inverse cell widths: this block's level on a mesh with levels
        const double idxb = LV ? B.ix : A.idx, idyb = LV ? B.iy : A.idy, idzb = LV ? B.iz : A.idz;
        // flux through block face f at transverse cell (e1, e2) to its register slot, if any
        auto reg_put = [&](int f, int e1, int e2, const double (&Fv)[5]) {
            if constexpr (!LV) return;       // meshes without levels keep no face fluxes
            const int slot = F6[f].reg;
            if (slot < 0) return;
            const int n1 = (f < 2) ? B.ny : B.nx;
            double *r = A.freg + (int64_t)slot * NV * A.nface + (int64_t)e2 * n1 + e1;
#pragma unroll
            for (int v = 0; v < NV; ++v) r[(int64_t)v * A.nface] = Fv[v];
        };
        const bool own = (tx < wx) && (ty < wy);
        const int i = x0 + tx, j = y0 + ty;
        const int nhalo = 2 * H * (wx + wy);
        const int nextra = 2 * (wx + wy);

        double zw[NW][5];     // primitives of cells k+1-R .. k+1+R along z
        double qpz[5];        // right-face state of cell k (z)
        double Flo[5];        // z flux at k-1/2
        // prefetch schedule (PF): raw values of the next plane, loaded one plane ahead
        constexpr int NSLOT = (2 * H * (TX + TY) + NT - 1) / NT;
        double pz[5], ph[NSLOT][5], pus[5], pun[5];
        auto halo_cell = [&](int e, int k, int &li, int &lj) -> int64_t {
            if (e < 2 * H * wy) {
                const int row = e / (2 * H), c = e % (2 * H);
                const int off = (c < H) ? c - H : wx + (c - H);
                li = off + H;
                lj = row + H;
                return src_cell<0, GATHER>(B, F6, x0 + off, y0 + row, k);
            }
            const int e2 = e - 2 * H * wy;
            const int c = e2 / wx, col = e2 % wx;
            const int off = (c < H) ? c - H : wy + (c - H);
            li = col + H;
            lj = off + H;
            return src_cell<1, GATHER>(B, F6, x0 + col, y0 + off, k);
        };
        // The halo cells a thread loads, as the index in the item's first plane,
        // the plane stride and the LDS slot: a halo cell's index is affine in
        // the plane (its source block and transverse position do not change
        // along z), so two evaluations per work item replace the per-plane
        // gather arithmetic.  The stride is a source block's padded plane
        // size, below 2^31 (checked on the host); 2D items have one plane.
        int64_t hc0[NSLOT];
        int32_t hst[NSLOT];
        int hls[NSLOT];
#pragma unroll
        for (int q = 0; q < NSLOT; ++q) {
            const int e = tid + q * NT;
            hc0[q] = 0;
            hst[q] = 0;
            hls[q] = 0;
            if (e < nhalo) {
                int li, lj;
                hc0[q] = halo_cell(e, z0, li, lj);
                if constexpr (NDIM == 3) hst[q] = (int32_t)(halo_cell(e, z0 + 1, li, lj) - hc0[q]);
                hls[q] = lj * LX + li;
            }
        }
        auto halo_at = [&](int q, int kk) -> int64_t {
            if constexpr (NDIM == 3) return hc0[q] + (int64_t)kk * hst[q];
            return hc0[q];
        };
        auto prefetch = [&](int k) {
            if (own) {
                if constexpr (NDIM == 3)
                    load_cons<NDIM>(A.Us, nc, src_cell<2, GATHER>(B, F6, i, j, k + H), pz);
                else
                    load_cons<NDIM>(A.Us, nc, cell_at(B, i, j, k), pz);
                const int64_t ci = cell_at(B, i, j, k);
                load_cons<NDIM>(A.Us, nc, ci, pus);
                if (A.stage != 1) load_cons<NDIM>(A.Un, nc, ci, pun);
            }
#pragma unroll
            for (int q = 0; q < NSLOT; ++q) {
                const int e = tid + q * NT;
                if (e < nhalo) load_cons<NDIM>(A.Us, nc, halo_at(q, k - z0), ph[q]);
            }
        };
        if constexpr (!PF) set_prio(3);
        if constexpr (NDIM == 3) {
            if (own) {
                double Wt[NW + 1][5];
#pragma unroll
                for (int c = 0; c < NW + 1; ++c) {
                    double u[5];
                    load_cons<NDIM>(A.Us, nc, src_cell<2, GATHER>(B, F6, i, j, z0 - H + c), u);
                    bad |= eos<NDIM>(u, Wt[c], K.g1);
                }
                double s0[NW][5], s1[NW][5];
#pragma unroll
                for (int c = 0; c < NW; ++c)
#pragma unroll
                    for (int v = 0; v < 5; ++v) { s0[c][v] = Wt[c][v]; s1[c][v] = Wt[c + 1][v]; }
                double qa[5], qb[5], qm[5];
                recon_cell<NDIM, RECON>(s0, qa, qpz, A.eps, shk && shock_flag<2, R>(s0, A.sthresh));  // cell z0-1: keep its right face
                recon_cell<NDIM, RECON>(s1, qm, qb, A.eps, shk && shock_flag<2, R>(s1, A.sthresh));   // cell z0
                bad |= hllc<NDIM, 2, RECON == kPLM>(qpz, qm, Flo, K);
                if (z0 == 0) reg_put(4, i, j, Flo);
#pragma unroll
                for (int v = 0; v < 5; ++v) qpz[v] = qb[v];
#pragma unroll
                for (int c = 0; c < NW - 1; ++c)
#pragma unroll
                    for (int v = 0; v < 5; ++v) zw[c][v] = Wt[c + 2][v];
            }
        }

        if constexpr (PF) prefetch(z0);
        for (int kk = 0; kk < nzc; ++kk) {
            const int k = z0 + kk;
            // Two workgroups share a CU; the arbiter favours the older one's waves,
            // so the younger would finish last and run alone.  Lowering the
            // priority over the last planes of an item lets a lagging
            // co-resident workgroup catch up.
            if constexpr (!PF) set_prio((kk < nzc - 8) ? 3 : ((kk < nzc - 4) ? 2 : ((kk < nzc - 2) ? 1 : 0)));
            double Dz[5];
            double cus[5], cun[5], chalo[NSLOT][5], cz[5];
            if constexpr (PF) {
#pragma unroll
                for (int v = 0; v < 5; ++v) { cus[v] = pus[v]; cun[v] = pun[v]; cz[v] = pz[v]; }
#pragma unroll
                for (int q = 0; q < NSLOT; ++q)
#pragma unroll
                    for (int v = 0; v < 5; ++v) chalo[q][v] = ph[q][v];
                if (kk + 1 < nzc) prefetch(k + 1);
            }
            // z face k+1/2 of the own column: the new cell k+H enters the z
            // window, cell k+1 is reconstructed and the face solved
            auto zface = [&]() {
                double u[5];
                if constexpr (PF) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) u[v] = cz[v];
                } else {
                    load_cons<NDIM>(A.Us, nc, src_cell<2, GATHER>(B, F6, i, j, k + H), u);
                }
                bad |= eos<NDIM>(u, zw[NW - 1], K.g1);
                double qm[5], qp[5], Fhi[5];
                recon_cell<NDIM, RECON>(zw, qm, qp, A.eps, shk && shock_flag<2, R>(zw, A.sthresh));   // cell k+1
                bad |= hllc<NDIM, 2, RECON == kPLM>(qpz, qm, Fhi, K);
                if (k == B.nz - 1) reg_put(5, i, j, Fhi);
#pragma unroll
                for (int v = 0; v < NV; ++v) { Dz[v] = Fhi[v] - Flo[v]; Flo[v] = Fhi[v]; }
#pragma unroll
                for (int v = 0; v < 5; ++v) qpz[v] = qp[v];
#pragma unroll
                for (int c = 0; c < NW - 1; ++c)
#pragma unroll
                    for (int v = 0; v < 5; ++v) zw[c][v] = zw[c + 1][v];
            };
            if (own) {
                if constexpr (NDIM == 3) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) sW[v][ty + H][tx + H] = zw[R - 1][v];   // cell k
                    zface();
                } else {
                    double u[5], wv[5];
                    if constexpr (PF) {
#pragma unroll
                        for (int v = 0; v < 5; ++v) u[v] = cz[v];
                    } else {
                        load_cons<NDIM>(A.Us, nc, cell_at(B, i, j, k), u);
                    }
                    bad |= eos<NDIM>(u, wv, K.g1);
#pragma unroll
                    for (int v = 0; v < 5; ++v) sW[v][ty + H][tx + H] = wv[v];
                }
            }
            // x and y halo of plane k
            if constexpr (NDIM == 3 || PF) {
#pragma unroll
                for (int q = 0; q < NSLOT; ++q) {
                    if (tid + q * NT < nhalo) {
                        double u[5], wv[5];
                        if constexpr (PF) {
#pragma unroll
                            for (int v = 0; v < 5; ++v) u[v] = chalo[q][v];
                        } else {
                            load_cons<NDIM>(A.Us, nc, halo_at(q, kk), u);
                        }
                        bad |= eos<NDIM>(u, wv, K.g1);
                        double *d = &sW[0][0][0] + hls[q];
#pragma unroll
                        for (int v = 0; v < 5; ++v) d[v * LY * LX] = wv[v];
                    }
                }
            } else {
                // a 2D item is one plane: its halo is gathered once
                for (int e = tid; e < nhalo; e += NT) {
                    int li, lj;
                    double u[5], wv[5];
                    load_cons<NDIM>(A.Us, nc, halo_cell(e, k, li, lj), u);
                    bad |= eos<NDIM>(u, wv, K.g1);
#pragma unroll
                    for (int v = 0; v < 5; ++v) sW[v][lj][li] = wv[v];
                }
            }
            __syncthreads();

            // x and y reconstruction: own cells, then the cells just outside the tile
            double qmx[5], qmy[5], qme[5];
            if (own) {
                double s[NW][5], qp[5];
#pragma unroll
                for (int c = 0; c < NW; ++c)
#pragma unroll
                    for (int v = 0; v < 5; ++v) s[c][v] = sW[v][ty + H][tx + H - R + c];
                recon_cell<NDIM, RECON>(s, qmx, qp, A.eps, shk && shock_flag<0, R>(s, A.sthresh));
#pragma unroll
                for (int v = 0; v < 5; ++v) sQx[v][ty][tx + 1] = qp[v];
#pragma unroll
                for (int c = 0; c < NW; ++c)
#pragma unroll
                    for (int v = 0; v < 5; ++v) s[c][v] = sW[v][ty + H - R + c][tx + H];
                recon_cell<NDIM, RECON>(s, qmy, qp, A.eps, shk && shock_flag<1, R>(s, A.sthresh));
#pragma unroll
                for (int v = 0; v < 5; ++v) sQy[v][ty + 1][tx] = qp[v];
            }
            int etype = -1, epos = 0;
            if (tid < nextra) {
                double s[NW][5], qm[5], qp[5];
                int e = tid;
                if (e < 2 * wy) {          // x: cell -1 (type 0) or cell wx (type 1) of row epos
                    etype = (e < wy) ? 0 : 1;
                    epos = (e < wy) ? e : e - wy;
                    const int cx = (etype == 0) ? -1 : wx;
#pragma unroll
                    for (int c = 0; c < NW; ++c)
#pragma unroll
                        for (int v = 0; v < 5; ++v) s[c][v] = sW[v][epos + H][cx + H - R + c];
                } else {                   // y: cell -1 (type 2) or cell wy (type 3) of column epos
                    e -= 2 * wy;
                    etype = (e < wx) ? 2 : 3;
                    epos = (e < wx) ? e : e - wx;
                    const int cy = (etype == 2) ? -1 : wy;
#pragma unroll
                    for (int c = 0; c < NW; ++c)
#pragma unroll
                        for (int v = 0; v < 5; ++v) s[c][v] = sW[v][cy + H - R + c][epos + H];
                }
                recon_cell<NDIM, RECON>(s, qm, qp, A.eps, shk && shock_flag_xy<R>(s, etype >= 2, A.sthresh));
                if (etype == 0) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) sQx[v][epos][0] = qp[v];
                } else if (etype == 2) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) sQy[v][0][epos] = qp[v];
                } else {
#pragma unroll
                    for (int v = 0; v < 5; ++v) qme[v] = qm[v];
                }
            }
            __syncthreads();

            if constexpr (!PF) {
                // operands of the RK update: issued here, consumed after the Riemann
                // problems (loaded at plane start they would hold registers through
                // the reconstruction, where pressure peaks)
                if (own) {
                    const int64_t ci = cell_at(B, i, j, k);
                    load_cons<NDIM>(A.Us, nc, ci, cus);
                    if (A.stage != 1) load_cons<NDIM>(A.Un, nc, ci, cun);
                }
            }
            // Riemann problems at the faces
            if (own) {
                double WL[5], Fv[5];
#pragma unroll
                for (int v = 0; v < 5; ++v) WL[v] = sQx[v][ty][tx];
                bad |= hllc<NDIM, 0, RECON == kPLM>(WL, qmx, Fv, K);
#pragma unroll
                for (int v = 0; v < NV; ++v) sFx[v][ty][tx] = Fv[v];
                if (i == 0) reg_put(0, j, (NDIM == 3) ? k : 0, Fv);
#pragma unroll
                for (int v = 0; v < 5; ++v) WL[v] = sQy[v][ty][tx];
                bad |= hllc<NDIM, 1, RECON == kPLM>(WL, qmy, Fv, K);
#pragma unroll
                for (int v = 0; v < NV; ++v) sFy[v][ty][tx] = Fv[v];
                if (j == 0) reg_put(2, i, (NDIM == 3) ? k : 0, Fv);
            }
            if (etype == 1 || etype == 3) {
                // The high x and y edge faces in one pass: a y face is solved as
                // an x face with the x and y velocity components exchanged in both
                // states and in the flux.  The bits are the same (the only sum over
                // these components, the kinetic energy's, starts with their pair).
                const bool fy = (etype == 3);
                constexpr int sx = TY * (TX + 1), sy = (TY + 1) * TX;   // per-variable strides
                const double *ql = fy ? &sQy[0][wy][epos] : &sQx[0][epos][wx];
                double *fo = fy ? &sFy[0][wy][epos] : &sFx[0][epos][wx];
                const int st = fy ? sy : sx;
                auto xch = [fy](double (&q)[5]) {
                    const double a = q[1], b = q[2];
                    q[1] = fy ? b : a;
                    q[2] = fy ? a : b;
                };
                double WL[5], Fv[5];
#pragma unroll
                for (int v = 0; v < 5; ++v) WL[v] = ql[v * st];
                xch(WL);
                xch(qme);
                bad |= hllc<NDIM, 0, RECON == kPLM>(WL, qme, Fv, K);
                xch(Fv);
#pragma unroll
                for (int v = 0; v < NV; ++v) fo[v * st] = Fv[v];
                if (fy ? (y0 + wy == B.ny) : (x0 + wx == B.nx))
                    reg_put(fy ? 3 : 1, (fy ? x0 : y0) + epos, (NDIM == 3) ? k : 0, Fv);
            }
            __syncthreads();

            // flux differences and the SSP-RK combination
            if (own) {
                const int64_t ci = cell_at(B, i, j, k);
                // gravity source from the stage input's cell: rho g_d, m . g
                double src[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                if (grv) {
#pragma unroll
                    for (int d = 0; d < NDIM; ++d) src[1 + d] = cus[0] * A.grav[d];
                    double mg = cus[1] * A.grav[0] + cus[2] * A.grav[1];
                    if constexpr (NDIM == 3) mg = mg + cus[3] * A.grav[2];
                    src[NV - 1] = mg;
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double Dx = sFx[v][ty][tx + 1] - sFx[v][ty][tx];
                    const double Dy = sFy[v][ty + 1][tx] - sFy[v][ty][tx];
                    double acc = Dx * idxb + Dy * idyb;
                    if constexpr (NDIM == 3) acc = acc + Dz[v] * idzb;
                    const double L = (grv && v > 0) ? src[v] - acc : -acc;
                    const double T = fma(dt, L, cus[v]);
                    double out;
                    if (A.stage == 1)
                        out = T;
                    else
                        out = fma(A.b, T, A.a * cun[v]);
                    A.Uout[v * nc + ci] = out;
                    if constexpr (CFLO) cus[v] = out;
                }
                if constexpr (CFLO) {
                    // the CFL wave-speed sum of the new state, as the dt reduction
                    // would take it from the array at the next step
                    double wv[5];
                    bad |= eos<NDIM>(cus, wv, K.g1);
                    const double r = 1.0 / cus[0];
                    const double c = sqrt((A.gamma * wv[4]) * r);
                    double sig = ((fabs(wv[1]) + c) * idxb) + ((fabs(wv[2]) + c) * idyb);
                    if constexpr (NDIM == 3) sig = sig + ((fabs(wv[3]) + c) * idzb);
                    const double m = sCfl[tid];
                    sCfl[tid] = (sig > m) ? sig : m;
                }
            }
        }
    }
    if constexpr (CFLO) {
        __syncthreads();
        double m = sCfl[tid];
        for (int sh = 32; sh > 0; sh >>= 1) {
            const double o = __shfl_xor(m, sh, 64);
            m = (o > m) ? o : m;
        }
        __syncthreads();
        if ((tid & 63) == 0) sCfl[tid >> 6] = m;
        __syncthreads();
        if (tid == 0) {
            for (int q = 1; q < NT / 64; ++q) m = (sCfl[q] > m) ? sCfl[q] : m;
            A.cfl_partial[blockIdx.x] = m;
        }
    }
    if (bad) atomicAdd(A.nbad, 1ull);
}

// Entry points of the two schedules.  The plain schedule is held to two
// waves per SIMD (its register use fits without spills; the 16x16 tile would
// otherwise fall to one); the prefetching schedule keeps the compiler's choice.
template <int NDIM, int RECON, int TX, int TY, bool GATHER>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(2))) k_stage(StageArgs A)
{
    stage_body<NDIM, RECON, TX, TY, GATHER, false>(A);
}

template <int NDIM, int RECON, int TX, int TY, bool GATHER>
__global__ void __launch_bounds__(TX *TY) k_stage_pf(StageArgs A)
{
    stage_body<NDIM, RECON, TX, TY, GATHER, true>(A);
}

// The plain schedule that also reduces the CFL wave-speed sum of the state it
// writes (the last stage of a step whose successor takes dt from it).
template <int NDIM, int RECON, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(2))) k_stage_cfl(StageArgs A)
{
    stage_body<NDIM, RECON, TX, TY, true, false, false, true>(A);
}

// Stages with gravity or the shock detector: the plain schedule (and its
// form that records the CFL maxima) with those parts compiled in.
template <int NDIM, int RECON, int TX, int TY, bool GATHER>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(2))) k_stage_phys(StageArgs A)
{
    stage_body<NDIM, RECON, TX, TY, GATHER, false, false, false, true>(A);
}

template <int NDIM, int RECON, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(2))) k_stage_cfl_phys(StageArgs A)
{
    stage_body<NDIM, RECON, TX, TY, true, false, false, true, true>(A);
}

// Meshes with refinement levels: the plain schedule that also writes the
// fluxes through faces to another level into their flux registers.
template <int NDIM, int RECON, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(2))) k_stage_lv(StageArgs A)
{
    stage_body<NDIM, RECON, TX, TY, true, false, true>(A);
}

// Per-workgroup maximum of the unsplit wave-speed sum over the interior
// cells of its work items.
template <int NDIM, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_cfl_partial(CflArgs A)
{
    constexpr int NT = TX * TY;
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    double m = 0.0;
    bool bad = false;
    for (int w = blockIdx.x; w < A.nitems; w += gridDim.x) {
        const WorkItem it = A.items[w];
        const DevBlock B = A.blocks[it.block];
        const int x0 = it.xy & 0xffff, y0 = it.xy >> 16;
        const int z0 = it.z & 0xffff, nzc = it.z >> 16;
        const int i = x0 + tx, j = y0 + ty;
        const double idxb = B.ix, idyb = B.iy, idzb = B.iz;
        if (i < B.nx && j < B.ny) {
            for (int k = z0; k < z0 + nzc; ++k) {
                double u[5], wv[5];
                load_cons<NDIM>(A.U, A.nc, cell_at(B, i, j, k), u);
                bad |= eos<NDIM>(u, wv, A.g1);
                const double r = 1.0 / u[0];
                const double c = sqrt((A.gamma * wv[4]) * r);
                double sig = ((fabs(wv[1]) + c) * idxb) + ((fabs(wv[2]) + c) * idyb);
                if constexpr (NDIM == 3) sig = sig + ((fabs(wv[3]) + c) * idzb);
                m = (sig > m) ? sig : m;
            }
        }
    }
    for (int s = 32; s > 0; s >>= 1) {
        const double o = __shfl_xor(m, s, 64);
        m = (o > m) ? o : m;
    }
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        for (int q = 1; q < NT / 64; ++q) m = (red[q] > m) ? red[q] : m;
        A.partial[blockIdx.x] = m;
    }
    if (bad) atomicAdd(A.nbad, 1ull);
}

__global__ void __launch_bounds__(256) k_cfl_final(const double *__restrict__ partial, int n, double cfl,
                                                   double *__restrict__ dt)
{
    __shared__ double red[4];
    const int tid = threadIdx.x;
    double m = 0.0;
    for (int q = tid; q < n; q += 256) m = (partial[q] > m) ? partial[q] : m;
    for (int s = 32; s > 0; s >>= 1) {
        const double o = __shfl_xor(m, s, 64);
        m = (o > m) ? o : m;
    }
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        for (int q = 1; q < 4; ++q) m = (red[q] > m) ? red[q] : m;
        *dt = cfl / m;
    }
}

// Guard layers of faces to another refinement level (ratio 2), one
// workgroup per (block, face) of the list.  Behind a coarser neighbour a
// guard cell takes the coarse cell containing it; behind finer neighbours it
// takes the 2^NDIM fine cells it covers, summed in pairs (the normal pair,
// then along the first and the second transverse axis) times 2^-NDIM.
template <int NDIM>
__global__ void __launch_bounds__(256) k_amr_fill(AmrArgs A)
{
    constexpr int NV = NDIM + 2;
    const int64_t nc = A.nc;
    // fchunks workgroups per face of the list; the face's items (guard layer
    // l = 1 .. ng, cell of the face) are numbered with the layer fastest, so
    // the layers of one row (adjacent doubles behind an x face) fall to
    // neighbouring lanes, and each workgroup takes one 256-item chunk
    for (int w = blockIdx.x; w < A.nlist * A.fchunks; w += gridDim.x) {
        const int b = A.list[w / A.fchunks].x, f = A.list[w / A.fchunks].y;
        const int t0 = (w % A.fchunks) * (int)blockDim.x;
        const int d = f >> 1, side = f & 1;
        const int o1 = (d == 0) ? 1 : 0, o2 = (d == 2) ? 1 : 2;
        const DevBlock B = A.blocks[b];
        const DevAmr &M = A.amr[b];
        const int ext[3] = {B.nx, B.ny, B.nz};
        const int n = ext[d], n1 = ext[o1], n2 = (NDIM == 3) ? ext[o2] : 1;
        {
            const int t = t0 + (int)threadIdx.x;
            if (t >= n1 * n2 * A.ng) continue;
            const int l = 1 + t % A.ng, e = t / A.ng;
            const int e1 = e % n1, e2 = e / n1;
            int g[3] = {0, 0, 0};
            g[d] = (side == 0) ? -l : n - 1 + l;
            g[o1] = e1;
            if (NDIM == 3) g[o2] = e2;
            const int64_t gi = cell_at(B, g[0], g[1], g[2]);
            if (M.kind[f] == 1) {
                const DevBlock C = A.blocks[M.nbr[f][0]];
                const int cext[3] = {C.nx, C.ny, C.nz};
                const int half = (l + 1) / 2;
                int s[3] = {0, 0, 0};
                s[d] = (side == 0) ? cext[d] - half : half - 1;
                s[o1] = M.nbr[f][1] + e1 / 2;
                if (NDIM == 3) s[o2] = M.nbr[f][2] + e2 / 2;
                const int64_t si = cell_at(C, s[0], s[1], s[2]);
#pragma unroll
                for (int v = 0; v < NV; ++v) A.U[v * nc + gi] = A.U[v * nc + si];
            } else {
                const int h1n = n1 / 2, h2n = (NDIM == 3) ? n2 / 2 : 1;
                const int h1 = e1 / h1n, h2 = (NDIM == 3) ? e2 / h2n : 0;
                const DevBlock F = A.blocks[M.nbr[f][h1 + 2 * h2]];
                const int fext[3] = {F.nx, F.ny, F.nz};
                const int p0 = (side == 0) ? fext[d] - 2 * l : 2 * (l - 1);
                const int f1 = 2 * (e1 - h1 * h1n), f2 = (NDIM == 3) ? 2 * (e2 - h2 * h2n) : 0;
                auto fine = [&](int v, int in, int i1, int i2) {
                    int s[3] = {0, 0, 0};
                    s[d] = p0 + in;
                    s[o1] = f1 + i1;
                    if (NDIM == 3) s[o2] = f2 + i2;
                    return A.U[v * nc + cell_at(F, s[0], s[1], s[2])];
                };
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double val;
                    if constexpr (NDIM == 3)
                        val = (((fine(v, 0, 0, 0) + fine(v, 1, 0, 0)) + (fine(v, 0, 1, 0) + fine(v, 1, 1, 0))) +
                               ((fine(v, 0, 0, 1) + fine(v, 1, 0, 1)) + (fine(v, 0, 1, 1) + fine(v, 1, 1, 1)))) * 0.125;
                    else
                        val = ((fine(v, 0, 0, 0) + fine(v, 1, 0, 0)) + (fine(v, 0, 1, 0) + fine(v, 1, 1, 0))) * 0.25;
                    A.U[v * nc + gi] = val;
                }
            }
        }
    }
}

// Flux correction of the coarse blocks of the list, one workgroup per block:
// faces with finer neighbours in the order -x, +x, -y, +y, -z, +z (a barrier
// between faces, so a cell next to two of them takes its corrections in that
// order); the coarse cell next to a face gets sigma b (dt ((Fbar - Fc) / dx)),
// Fbar the fine fluxes through the face averaged in pairs, Fc its own flux,
// sigma = +1 on a low and -1 on a high face.
template <int NDIM>
__global__ void __launch_bounds__(256) k_amr_correct(AmrArgs A)
{
    constexpr int NV = NDIM + 2;
    const int64_t nc = A.nc;
    const double dt = *A.dt;
    for (int w = blockIdx.x; w < A.nlist; w += gridDim.x) {
        const int b = A.list[w].x;
        const DevBlock B = A.blocks[b];
        const DevAmr &M = A.amr[b];
        const int ext[3] = {B.nx, B.ny, B.nz};
        for (int f = 0; f < 2 * NDIM; ++f) {
            if (M.kind[f] != 2) continue;
            const int d = f >> 1, side = f & 1;
            const int o1 = (d == 0) ? 1 : 0, o2 = (d == 2) ? 1 : 2;
            const int n = ext[d], n1 = ext[o1], n2 = (NDIM == 3) ? ext[o2] : 1;
            const double id = (d == 0) ? B.ix : ((d == 1) ? B.iy : B.iz);
            const int ff = 2 * d + 1 - side;              // the fine blocks' face
            const double *Rc = A.freg + (int64_t)A.faces[6 * (int64_t)b + f].reg * NV * A.nface;
            for (int t = threadIdx.x; t < n1 * n2; t += blockDim.x) {
                const int e1 = t % n1, e2 = t / n1;
                const int h1n = n1 / 2, h2n = (NDIM == 3) ? n2 / 2 : 1;
                const int h1 = e1 / h1n, h2 = (NDIM == 3) ? e2 / h2n : 0;
                const int fb = M.nbr[f][h1 + 2 * h2];
                const int f1 = 2 * (e1 - h1 * h1n), f2 = (NDIM == 3) ? 2 * (e2 - h2 * h2n) : 0;
                const double *Rf = A.freg + (int64_t)A.faces[6 * (int64_t)fb + ff].reg * NV * A.nface;
                int c[3] = {0, 0, 0};
                c[d] = (side == 0) ? 0 : n - 1;
                c[o1] = e1;
                if (NDIM == 3) c[o2] = e2;
                const int64_t ci = cell_at(B, c[0], c[1], c[2]);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double *rf = Rf + (int64_t)v * A.nface;
                    double Fbar;
                    if constexpr (NDIM == 3)
                        Fbar = ((rf[f2 * n1 + f1] + rf[f2 * n1 + f1 + 1]) + (rf[(f2 + 1) * n1 + f1] + rf[(f2 + 1) * n1 + f1 + 1])) * 0.25;
                    else
                        Fbar = (rf[f1] + rf[f1 + 1]) * 0.5;
                    const double Fc = Rc[(int64_t)v * A.nface + e2 * n1 + e1];
                    const double corr = A.b * (dt * ((Fbar - Fc) * id));
                    A.U[v * nc + ci] = (side == 0) ? A.U[v * nc + ci] + corr : A.U[v * nc + ci] - corr;
                }
            }
            __syncthreads();
        }
    }
}

// Materialised guard fill for blocks [b0, b0 + gridDim.x / (2 NDIM)):
// workgroup = (block, face); threads walk layers x transverse cells with the
// index that is contiguous in memory fastest: the layer on x faces (the ng
// guard cells of a row), the x index on y and z faces.
template <int NDIM>
__global__ void __launch_bounds__(256) k_fill_guards(GuardArgs A)
{
    const int b = A.b0 + blockIdx.x / (2 * NDIM);
    const int f = blockIdx.x % (2 * NDIM);
    const int d = f / 2, side = f % 2;
    const DevBlock B = A.blocks[b];
    const FaceSrc S = A.faces[6 * (int64_t)b + f];
    const int n = (d == 0) ? B.nx : ((d == 1) ? B.ny : B.nz);
    const int n1 = (d == 0) ? B.ny : B.nx;
    const int n2 = (NDIM == 3) ? ((d == 2) ? B.ny : B.nz) : 1;
    const int count = B.ng * n1 * n2;
    for (int e = threadIdx.x; e < count; e += blockDim.x) {
        int l, r;
        if (d == 0) { l = e % B.ng + 1; r = e / B.ng; }
        else { l = e / (n1 * n2) + 1; r = e % (n1 * n2); }
        const int e1 = r % n1, e2 = r / n1;
        const int pos = (side == 0) ? -l : n - 1 + l;
        const int sp = S.A + S.B * pos;
        int g[3], s[3];
        if (d == 0) { g[0] = pos; g[1] = e1; g[2] = e2; s[0] = sp; s[1] = e1; s[2] = e2; }
        else if (d == 1) { g[0] = e1; g[1] = pos; g[2] = e2; s[0] = e1; s[1] = sp; s[2] = e2; }
        else { g[0] = e1; g[1] = e2; g[2] = pos; s[0] = e1; s[1] = e2; s[2] = sp; }
        const int64_t gi = cell_at(B, g[0], g[1], g[2]);
        const int64_t si = S.off + ((int64_t)(s[2] + B.gz) * S.py + (s[1] + B.ng)) * S.px + (s[0] + B.ng);
#pragma unroll
        for (int v = 0; v < NDIM + 2; ++v) A.U[v * A.nc + gi] = A.U[v * A.nc + si];
    }
}

// ------------------------------------------------------- telescoping step
//
// The paper's telescoping RK variant (Sec. 4.2, second listing): one guard
// fill per step into thick copies of the blocks, then every stage updates the
// block and the part of its halo later stages still read.  The thick halo is
// filled one direction after the other (one launch per direction): direction
// d copies ng layers over the already-filled extents of the directions
// before it, so edges and corners come from neighbours of neighbours.

// Interior copy between the caller's layout and the thick layout.
template <int NDIM>
__global__ void __launch_bounds__(256) k_tele_copy(TeleArgs A, int to_thick)
{
    const int b = blockIdx.x;
    const DevBlock Bt = A.tb[b], Bu = A.ub[b];
    const int n = Bu.nx * Bu.ny * Bu.nz;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int i = q % Bu.nx, j = (q / Bu.nx) % Bu.ny, k = q / (Bu.nx * Bu.ny);
        const int64_t ct = cell_at(Bt, i, j, k), cu = cell_at(Bu, i, j, k);
#pragma unroll
        for (int v = 0; v < NDIM + 2; ++v) {
            if (to_thick) A.T[v * A.nct + ct] = A.U[v * A.ncu + cu];
            else A.U[v * A.ncu + cu] = A.T[v * A.nct + ct];
        }
    }
}

// Halo layers of direction A.d: workgroup = (block, side).
template <int NDIM>
__global__ void __launch_bounds__(256) k_tele_fill(TeleArgs A)
{
    const int b = blockIdx.x / 2, side = blockIdx.x % 2, d = A.d;
    const DevBlock B = A.tb[b];
    const FaceSrc S = A.tf[6 * (int64_t)b + 2 * d + side];
    const int g = B.ng;
    const int n3[3] = {B.nx, B.ny, B.nz};
    int lo[3], len[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        if (e >= NDIM || e == d) { lo[e] = 0; len[e] = 1; }
        else if (e < d) { lo[e] = -g; len[e] = n3[e] + 2 * g; }
        else { lo[e] = 0; len[e] = n3[e]; }
    }
    const int n = n3[d];
    const int plane = len[0] * len[1] * len[2];
    const int count = g * plane;
    for (int q = threadIdx.x; q < count; q += blockDim.x) {
        const int l = q / plane + 1;
        const int r = q % plane;
        int c[3];
        c[0] = lo[0] + r % len[0];
        c[1] = lo[1] + (r / len[0]) % len[1];
        c[2] = lo[2] + r / (len[0] * len[1]);
        const int pos = (side == 0) ? -l : n - 1 + l;
        int s[3] = {c[0], c[1], c[2]};
        c[d] = pos;
        s[d] = S.A + S.B * pos;
        const int64_t gi = cell_at(B, c[0], c[1], c[2]);
        const int64_t si = S.off + ((int64_t)(s[2] + B.gz) * S.py + (s[1] + B.ng)) * S.px + (s[0] + B.ng);
#pragma unroll
        for (int v = 0; v < NDIM + 2; ++v) A.T[v * A.nct + gi] = A.T[v * A.nct + si];
    }
}

hipError_t launch_tele_fill(const TeleArgs &a, int ndim, int nblk, hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    if (ndim == 3) k_tele_fill<3><<<2 * nblk, 256, 0, st>>>(a);
    else k_tele_fill<2><<<2 * nblk, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_tele_copy(const TeleArgs &a, int ndim, int nblk, bool to_thick, hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    if (ndim == 3) k_tele_copy<3><<<nblk, 256, 0, st>>>(a, to_thick ? 1 : 0);
    else k_tele_copy<2><<<nblk, 256, 0, st>>>(a, to_thick ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------------- launchers

template <int NDIM, int RECON, int TX, int TY, bool GATHER>
static hipError_t launch_stage_t(const StageArgs &a, int variant, int grid, hipStream_t st)
{
    if (a.phys) {           // meshes without levels only (the context refuses the rest)
        if constexpr (GATHER) {
            if (a.cfl_partial != nullptr) {
                k_stage_cfl_phys<NDIM, RECON, TX, TY><<<grid, TX * TY, 0, st>>>(a);
                return hipGetLastError();
            }
        }
        k_stage_phys<NDIM, RECON, TX, TY, GATHER><<<grid, TX * TY, 0, st>>>(a);
        return hipGetLastError();
    }
    if constexpr (GATHER) {
        if (a.freg != nullptr) {
            k_stage_lv<NDIM, RECON, TX, TY><<<grid, TX * TY, 0, st>>>(a);
            return hipGetLastError();
        }
        if (a.cfl_partial != nullptr) {
            k_stage_cfl<NDIM, RECON, TX, TY><<<grid, TX * TY, 0, st>>>(a);
            return hipGetLastError();
        }
    }
    if (variant == 1)
        k_stage_pf<NDIM, RECON, TX, TY, GATHER><<<grid, TX * TY, 0, st>>>(a);
    else
        k_stage<NDIM, RECON, TX, TY, GATHER><<<grid, TX * TY, 0, st>>>(a);
    return hipGetLastError();
}

template <int NDIM, int RECON, bool GATHER>
static hipError_t launch_stage_r(const StageArgs &a, int tile, int variant, int grid, hipStream_t st)
{
    switch (tile) {
    case 0: return launch_stage_t<NDIM, RECON, 8, 8, GATHER>(a, variant, grid, st);
    case 1: return launch_stage_t<NDIM, RECON, 16, 8, GATHER>(a, variant, grid, st);
    default: return launch_stage_t<NDIM, RECON, 16, 16, GATHER>(a, variant, grid, st);
    }
}

hipError_t launch_stage(const StageArgs &a, int ndim, int recon, int tile, int variant, bool gather, int grid,
                        hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    if (ndim == 3) {
        if (recon == kWENO)
            return gather ? launch_stage_r<3, kWENO, true>(a, tile, variant, grid, st)
                          : launch_stage_r<3, kWENO, false>(a, tile, variant, grid, st);
        return gather ? launch_stage_r<3, kPLM, true>(a, tile, variant, grid, st)
                      : launch_stage_r<3, kPLM, false>(a, tile, variant, grid, st);
    }
    if (recon == kWENO)
        return gather ? launch_stage_r<2, kWENO, true>(a, tile, variant, grid, st)
                      : launch_stage_r<2, kWENO, false>(a, tile, variant, grid, st);
    return gather ? launch_stage_r<2, kPLM, true>(a, tile, variant, grid, st)
                  : launch_stage_r<2, kPLM, false>(a, tile, variant, grid, st);
}

template <int NDIM>
static hipError_t launch_cfl_n(const CflArgs &a, int tile, int grid, hipStream_t st)
{
    switch (tile) {
    case 0: k_cfl_partial<NDIM, 8, 8><<<grid, 64, 0, st>>>(a); break;
    case 1: k_cfl_partial<NDIM, 16, 8><<<grid, 128, 0, st>>>(a); break;
    default: k_cfl_partial<NDIM, 16, 16><<<grid, 256, 0, st>>>(a); break;
    }
    return hipGetLastError();
}

hipError_t launch_cfl_final(const double *partial, int n, double cfl, double *dt, hipStream_t st)
{
    k_cfl_final<<<1, 256, 0, st>>>(partial, n, cfl, dt);
    return hipGetLastError();
}

hipError_t launch_cfl(const CflArgs &a, int ndim, int tile, int grid, double cfl, double *dt, hipStream_t st)
{
    hipError_t e = (ndim == 3) ? launch_cfl_n<3>(a, tile, grid, st) : launch_cfl_n<2>(a, tile, grid, st);
    if (e != hipSuccess) return e;
    k_cfl_final<<<1, 256, 0, st>>>(a.partial, grid, cfl, dt);
    return hipGetLastError();
}

hipError_t launch_fill_guards(const GuardArgs &a, int ndim, int nblk, hipStream_t st)
{
    if (nblk <= 0) return hipSuccess;
    if (ndim == 3)
        k_fill_guards<3><<<nblk * 6, 256, 0, st>>>(a);
    else
        k_fill_guards<2><<<nblk * 4, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_amr_fill(const AmrArgs &a, int ndim, hipStream_t st)
{
    if (a.nlist <= 0) return hipSuccess;
    if (ndim == 3) k_amr_fill<3><<<a.nlist * a.fchunks, 256, 0, st>>>(a);
    else k_amr_fill<2><<<a.nlist * a.fchunks, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_amr_correct(const AmrArgs &a, int ndim, hipStream_t st)
{
    if (a.nlist <= 0) return hipSuccess;
    if (ndim == 3) k_amr_correct<3><<<a.nlist, 256, 0, st>>>(a);
    else k_amr_correct<2><<<a.nlist, 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace hydro
