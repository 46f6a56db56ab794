// C ABI of the FP64 Euler step (declared in include/hydro.h): validation,
// device tables, the work-item list, stage buffers, the SSP-RK step driver
// and its hipGraph replay, the telescoping step, meshes with refinement
// levels (coarse-fine guard fill and flux correction) and the step VJP.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "hydro.h"
#include "hydro_kernels.h"

using namespace hydro;

struct hydro_ctx {
    int device = 0;
    hipStream_t stream = nullptr;       // caller's stream
    hipStream_t cap = nullptr;          // private stream used only for graph capture
    hydro_params_t prm{};
    int32_t nblocks = 0;
    int64_t ncell = 0;
    int nv = 0;
    std::vector<hydro_block_t> hb;
    std::vector<hydro_link_t> hl;
    DevBlock *d_blocks = nullptr;
    FaceSrc *d_faces = nullptr;
    std::vector<DevBlock> h_dev;
    std::vector<FaceSrc> h_faces;
    // work list (persistent order) and per-block order with ranges
    WorkItem *d_items = nullptr;
    int nitems = 0;
    WorkItem *d_items_pb = nullptr;
    std::vector<int> pb_start;
    double *d_buf[2] = {nullptr, nullptr};
    double *d_partial = nullptr;
    int partial_cap = 0;
    // CFL maxima of the state the last fused step wrote (compute_dt 2): the
    // per-workgroup maxima of its final stage, valid for cfl_next_U until
    // another call may have changed that state
    double *d_cflnext = nullptr;
    int ncflnext = 0;
    const double *cfl_next_U = nullptr;
    unsigned long long *d_nbad = nullptr;
    hydro_tuning_t tune{};
    std::string err;
    // captured step
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    const double *g_U = nullptr;
    const double *g_dt = nullptr;
    int g_cdt = -1;
    const double *l_U = nullptr;    // arguments of the previous hydro_step call
    const double *l_dt = nullptr;
    int l_cdt = -1;
    // adjoint: line work lists per direction, 16x4 cell tiles, inverse links, scratch
    WorkItem *d_lines = nullptr;  // lines of every direction (cost field = direction | segment << 4)
    int nlines = 0;
    int nseg = 1;                 // segments per line
    WorkItem *d_citems = nullptr;
    int ncitems = 0;
    WorkItem *d_xitems = nullptr;  // tiles of the x-line transpose
    int nxitems = 0;
    int *d_inc_start = nullptr;
    int4 *d_inc = nullptr;
    double *d_vjp = nullptr;     // gW per direction and segment | gS | UsT | gOutT, each nvar x ncell
    // telescoping: thick block copies, per-stage virtual (extended) blocks and work lists
    int tele_ready = 0;
    int ngt = 0;
    int64_t ncell_t = 0;
    DevBlock *d_tblocks = nullptr;
    FaceSrc *d_tfaces = nullptr;
    DevBlock *d_vblocks[3] = {nullptr, nullptr, nullptr};
    WorkItem *d_titems[3] = {nullptr, nullptr, nullptr};
    int ntitems[3] = {0, 0, 0};
    double *d_tbuf = nullptr;    // U^n | A | B in the thick layout
    // refinement levels: faces to other levels, flux registers, per-level work
    bool amr = false;
    std::vector<hydro_amr_t> ha;
    DevAmr *d_amr = nullptr;
    double *d_freg = nullptr;    // register slots x nvar x nface
    int32_t nface = 0;
    int2 *d_afill = nullptr;     // (block, face) of every face to another level
    int nafill = 0;
    int2 *d_acorr = nullptr;     // (block, 0) of the blocks with faces to finer neighbours, by level
    std::vector<int> acorr_start;  // blocks of level L: [acorr_start[L], acorr_start[L + 1])
    int nlev = 1;
    std::vector<int> lvl_first, lvl_count;   // work items of level L in the persistent list
};

namespace {

int fail(hydro_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(hydro_ctx *c, hipError_t e, const char *where)
{
    return fail(c, HYDRO_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                  \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return hip_fail((c), _e, #expr); \
    } while (0)

int extent(const hydro_block_t &b, int d) { return d == 0 ? b.nx : (d == 1 ? b.ny : b.nz); }

int64_t padded_cells(const hydro_block_t &b, int ndim)
{
    int64_t pz = (ndim == 3) ? b.nz + 2 * b.ng : 1;
    return (int64_t)(b.nx + 2 * b.ng) * (b.ny + 2 * b.ng) * pz;
}

std::string check_problem(const hydro_params_t *p, const hydro_block_t *blocks, const hydro_link_t *links,
                          int32_t nblocks, int64_t ncell)
{
    if (!p) return "null params";
    if (nblocks < 0 || ncell < 0) return "negative sizes";
    if (nblocks > 0 && (!blocks || !links)) return "null descriptor table";
    if (p->ndim != 2 && p->ndim != 3) return "ndim must be 2 or 3";
    if (p->recon != HYDRO_PLM_MC && p->recon != HYDRO_WENO5) return "unknown reconstruction";
    if (p->rk != 2 && p->rk != 3) return "rk must be 2 or 3";
    if (!(p->gamma > 1.0)) return "gamma must be > 1";
    if (!(p->cfl > 0.0) || !(p->dx > 0.0) || !(p->dy > 0.0) || !(p->dz > 0.0)) return "cfl and cell widths must be > 0";
    if (!(p->weno_eps > 0.0) || !std::isfinite(p->weno_eps)) return "weno_eps must be finite and > 0";
    if (p->flags & ~(HYDRO_FLAG_LEVEL_BY_LEVEL | HYDRO_FLAG_GRAVITY | HYDRO_FLAG_SHOCK_DETECT)) return "unknown flags";
    if ((p->flags & HYDRO_FLAG_GRAVITY) &&
        !(std::isfinite(p->grav[0]) && std::isfinite(p->grav[1]) && std::isfinite(p->grav[2])))
        return "grav must be finite";
    if ((p->flags & HYDRO_FLAG_SHOCK_DETECT) && !(p->shock_thresh >= 0.0 && std::isfinite(p->shock_thresh)))
        return "shock_thresh must be finite and >= 0";
    const int ngmin = (p->recon == HYDRO_WENO5) ? 3 : 2;
    std::vector<std::pair<int64_t, int64_t>> span(nblocks);
    for (int b = 0; b < nblocks; ++b) {
        const hydro_block_t &B = blocks[b];
        if (B.nx < 1 || B.ny < 1 || B.nz < 1) return "block " + std::to_string(b) + ": extent < 1";
        if (B.nx > 32767 || B.ny > 32767 || B.nz > 32767) return "block " + std::to_string(b) + ": extent too large";
        if (B.ng < ngmin) return "block " + std::to_string(b) + ": ng below the stencil's need";
        if (p->ndim == 2 && B.nz != 1) return "block " + std::to_string(b) + ": 2D block with nz != 1";
        if (p->ndim == 3 && (int64_t)(B.nx + 2 * (int64_t)B.ng) * (B.ny + 2 * (int64_t)B.ng) > INT32_MAX)
            return "block " + std::to_string(b) + ": padded plane of 2^31 cells or more";
        const int64_t sz = padded_cells(B, p->ndim);
        if (B.offset < 0 || B.offset + sz > ncell) return "block " + std::to_string(b) + ": offset out of range";
        span[b] = {B.offset, B.offset + sz};
    }
    std::sort(span.begin(), span.end());
    for (int b = 1; b < nblocks; ++b)
        if (span[b].first < span[b - 1].second) return "blocks overlap";
    for (int b = 0; b < nblocks; ++b) {
        const hydro_block_t &B = blocks[b];
        for (int d = 0; d < p->ndim; ++d)
            for (int side = 0; side < 2; ++side) {
                const int nb = links[b].nbr[2 * d + side];
                if (nb >= nblocks || nb < -2) return "block " + std::to_string(b) + ": link out of range";
                if (nb == HYDRO_OUTFLOW) continue;
                const hydro_block_t &S = (nb >= 0) ? blocks[nb] : B;
                for (int e = 0; e < p->ndim; ++e)
                    if (e != d && extent(S, e) != extent(B, e))
                        return "block " + std::to_string(b) + ": neighbour face size mismatch";
                if (extent(S, d) < B.ng) return "block " + std::to_string(b) + ": neighbour shallower than ng";
                if (S.ng != B.ng) return "block " + std::to_string(b) + ": neighbour ng differs";
            }
    }
    return "";
}

// A mesh with refinement levels: the same-level checks on the links with
// every face to another level taken as outflow, then the level table.
std::string check_amr(const hydro_params_t *p, const hydro_block_t *blocks, const hydro_link_t *links,
                      const hydro_amr_t *amr, int32_t nblocks, int64_t ncell)
{
    if (!p) return "null params";
    if (nblocks > 0 && (!blocks || !links || !amr)) return "null descriptor table";
    if (p->flags & (HYDRO_FLAG_GRAVITY | HYDRO_FLAG_SHOCK_DETECT))
        return "gravity and the shock detector apply to meshes without levels only";
    if (p->flags & ~HYDRO_FLAG_LEVEL_BY_LEVEL) return "unknown flags";
    const int nd = p->ndim;
    std::vector<hydro_link_t> same(links, links + std::max(0, nblocks));
    for (int b = 0; b < nblocks; ++b)
        for (int f = 0; f < 6; ++f) {
            const bool level_face = (f < 2 * nd) && amr[b].kind[f] != 0;
            if ((links[b].nbr[f] == HYDRO_LEVEL_FACE) != level_face)
                return "block " + std::to_string(b) + ": link and level table disagree";
            if (level_face) same[b].nbr[f] = HYDRO_OUTFLOW;
        }
    hydro_params_t q = *p;
    q.flags = 0;
    std::string why = check_problem(&q, blocks, same.data(), nblocks, ncell);
    if (!why.empty()) return why;
    for (int b = 0; b < nblocks; ++b) {
        const hydro_block_t &B = blocks[b];
        if (B.nx != blocks[0].nx || B.ny != blocks[0].ny || B.nz != blocks[0].nz || B.ng != blocks[0].ng)
            return "blocks of an AMR mesh must share nx, ny, nz and ng";
        for (int d = 0; d < nd; ++d)
            if (extent(B, d) % 2 != 0 || extent(B, d) < 2 * B.ng)
                return "block " + std::to_string(b) + ": extents must be even and at least 2 ng";
        if (amr[b].level < 0 || amr[b].level > 20) return "block " + std::to_string(b) + ": level out of range";
    }
    for (int b = 0; b < nblocks; ++b)
        for (int d = 0; d < nd; ++d) {
            const int o1 = (d == 0) ? 1 : 0, o2 = (d == 2) ? 1 : 2;
            const int h1n = extent(blocks[b], o1) / 2, h2n = (nd == 3) ? extent(blocks[b], o2) / 2 : 0;
            for (int side = 0; side < 2; ++side) {
                const int f = 2 * d + side, opp = 2 * d + 1 - side;
                const std::string at = "block " + std::to_string(b) + " face " + std::to_string(f) + ": ";
                const int kind = amr[b].kind[f];
                if (kind == 1) {
                    const int cb = amr[b].nbr[f][0], q1 = amr[b].nbr[f][1], q2 = amr[b].nbr[f][2];
                    if (cb < 0 || cb >= nblocks) return at + "coarser block out of range";
                    if (amr[cb].level != amr[b].level - 1 || amr[cb].kind[opp] != 2) return at + "coarser block does not match";
                    if (!(q1 == 0 || q1 == h1n) || !((nd == 2) ? q2 == 0 : (q2 == 0 || q2 == h2n)))
                        return at + "face offset not a half face";
                    const int h = q1 / h1n + 2 * ((nd == 3) ? q2 / h2n : 0);
                    if (amr[cb].nbr[opp][h] != b) return at + "coarser block does not list this block";
                } else if (kind == 2) {
                    for (int h = 0; h < (1 << (nd - 1)); ++h) {
                        const int fb = amr[b].nbr[f][h];
                        if (fb < 0 || fb >= nblocks) return at + "finer block out of range";
                        if (amr[fb].level != amr[b].level + 1 || amr[fb].kind[opp] != 1 || amr[fb].nbr[opp][0] != b ||
                            amr[fb].nbr[opp][1] != (h & 1) * h1n || amr[fb].nbr[opp][2] != (h >> 1) * h2n)
                            return at + "finer block does not match";
                    }
                } else if (kind != 0) {
                    return at + "unknown kind";
                }
            }
        }
    return "";
}

// Host tables: geometry and, per face, the source of its guard layers.
void build_tables(hydro_ctx *c)
{
    const int nd = c->prm.ndim;
    c->h_dev.resize(c->nblocks);
    c->h_faces.assign((size_t)c->nblocks * 6, FaceSrc{0, 0, 0, 0, 0, -1, 0});
    for (int b = 0; b < c->nblocks; ++b) {
        const hydro_block_t &B = c->hb[b];
        DevBlock D{};
        D.off = B.offset;
        D.nx = B.nx; D.ny = B.ny; D.nz = B.nz; D.ng = B.ng;
        D.px = B.nx + 2 * B.ng;
        D.py = B.ny + 2 * B.ng;
        D.gz = (nd == 3) ? B.ng : 0;
        D.lev = c->amr ? c->ha[b].level : 0;
        D.ix = std::ldexp(1.0 / c->prm.dx, D.lev);
        D.iy = std::ldexp(1.0 / c->prm.dy, D.lev);
        D.iz = std::ldexp(1.0 / c->prm.dz, D.lev);
        c->h_dev[b] = D;
    }
    int slot = 0;
    for (int b = 0; b < c->nblocks; ++b) {
        const hydro_block_t &B = c->hb[b];
        for (int d = 0; d < nd; ++d)
            for (int side = 0; side < 2; ++side) {
                const int nb = c->hl[b].nbr[2 * d + side];
                const int n = extent(B, d);
                FaceSrc f{};
                f.reg = -1;
                const hydro_block_t &S = (nb >= 0) ? c->hb[nb] : B;
                f.off = S.offset;
                f.px = S.nx + 2 * S.ng;
                f.py = S.ny + 2 * S.ng;
                if (nb == HYDRO_LEVEL_FACE) {        // another level: the block's own (filled) guard layers
                    f.A = 0;
                    f.B = 1;
                    f.reg = slot++;
                } else if (nb == HYDRO_OUTFLOW) {    // nearest interior cell
                    f.A = (side == 0) ? 0 : n - 1;
                    f.B = 0;
                } else {                             // neighbour or periodic: distance l-1 from the face
                    const int m = extent(S, d);
                    f.A = (side == 0) ? m : -n;
                    f.B = 1;
                }
                c->h_faces[(size_t)b * 6 + 2 * d + side] = f;
            }
    }
}

// Order a list of independent work items (in block order) for a launch of
// one workgroup per item, which the hardware deals round-robin onto the 8
// XCDs by workgroup index: each XCD gets a contiguous range of whole blocks,
// about an eighth of the items, and the 8 ranges are interleaved item by
// item.  A block's items then share one L2, and so do most neighbouring
// blocks (adjacent indices), whose halo lines the items read.  Only the
// order changes, so results do not.
void interleave_block_ranges(std::vector<WorkItem> &xi)
{
    std::vector<std::vector<WorkItem>> lane(8);
    const size_t n = xi.size();
    size_t q = 0;
    for (int l = 0; l < 8; ++l) {
        const size_t end = n * (size_t)(l + 1) / 8;
        // past the lane's share only to finish the block in hand
        while (q < n && (q < end || (!lane[l].empty() && xi[q].block == xi[q - 1].block)))
            lane[l].push_back(xi[q++]);
    }
    std::vector<WorkItem> o;
    o.reserve(n);
    size_t maxl = 0;
    for (auto &l : lane) maxl = std::max(maxl, l.size());
    for (size_t r = 0; r < maxl; ++r)
        for (int l = 0; l < 8; ++l)
            if (r < lane[l].size()) o.push_back(lane[l][r]);
    xi.swap(o);
}

int tile_x(int t) { return t == 0 ? 8 : 16; }
int tile_y(int t) { return t == 2 ? 16 : 8; }

// Work items: xy tiles of every block over z chunks.  The persistent list is
// sorted by decreasing size (largest first).  With xcd != 0 the items of one
// block are placed at list positions congruent modulo 8, so that workgroups
// dealt round-robin onto the 8 XCDs (one per item, or a persistent grid of a
// multiple of 8) keep them on one XCD: xcd = 1 deals the blocks round-robin
// onto the 8 positions; xcd = 2 gives each position a contiguous range of
// block indices of about equal work, so blocks that are neighbours in the
// block order also share an L2 and one's halo reads can hit the lines the
// other brought in.
void build_items(hydro_ctx *c, std::vector<WorkItem> &list, std::vector<WorkItem> &perblock, std::vector<int> &start)
{
    const int TX = tile_x(c->tune.tile), TY = tile_y(c->tune.tile);
    const int nd = c->prm.ndim;
    perblock.clear();
    start.assign(c->nblocks + 1, 0);
    for (int b = 0; b < c->nblocks; ++b) {
        const hydro_block_t &B = c->hb[b];
        const int nz = (nd == 3) ? B.nz : 1;
        const int zc = (nd == 3 && c->tune.zchunk > 0) ? c->tune.zchunk : nz;
        start[b] = (int)perblock.size();
        for (int z0 = 0; z0 < nz; z0 += zc)
            for (int y0 = 0; y0 < B.ny; y0 += TY)
                for (int x0 = 0; x0 < B.nx; x0 += TX) {
                    WorkItem w{};
                    w.block = b;
                    w.xy = x0 | (y0 << 16);
                    const int nzi = std::min(zc, nz - z0);
                    w.z = z0 | (nzi << 16);
                    w.cost = std::min(TX, B.nx - x0) * std::min(TY, B.ny - y0) * nzi;
                    perblock.push_back(w);
                }
    }
    start[c->nblocks] = (int)perblock.size();
    list = perblock;
    std::stable_sort(list.begin(), list.end(), [](const WorkItem &a, const WorkItem &b) { return a.cost > b.cost; });
    if (c->amr) {
        // levels finest first, each level's items largest first
        std::stable_sort(list.begin(), list.end(), [c](const WorkItem &a, const WorkItem &b) {
            return c->ha[a.block].level > c->ha[b.block].level;
        });
        c->lvl_first.assign(c->nlev, 0);
        c->lvl_count.assign(c->nlev, 0);
        for (size_t q = 0; q < list.size(); ++q) {
            const int L = c->ha[list[q].block].level;
            if (c->lvl_count[L]++ == 0) c->lvl_first[L] = (int)q;
        }
        return;
    }
    if (c->tune.xcd) {
        // deal blocks round-robin onto 8 lanes, keep each lane's items in
        // order, then interleave the lanes position by position
        std::vector<std::vector<WorkItem>> lane(8);
        std::vector<int> lane_of(c->nblocks, -1);
        if (c->tune.xcd == 2) {
            std::vector<double> cost(c->nblocks, 0.0);
            double total = 0.0;
            for (const WorkItem &w : perblock) { cost[w.block] += w.cost; total += w.cost; }
            double before = 0.0;
            for (int b = 0; b < c->nblocks; ++b) {
                const double mid = before + 0.5 * cost[b];
                lane_of[b] = std::min(7, (int)(8.0 * mid / std::max(total, 1.0)));
                before += cost[b];
            }
        } else {
            int next = 0;
            for (const WorkItem &w : list)
                if (lane_of[w.block] < 0) lane_of[w.block] = (next++) % 8;
        }
        for (const WorkItem &w : list) lane[lane_of[w.block]].push_back(w);
        std::vector<WorkItem> out;
        out.reserve(list.size());
        size_t maxl = 0;
        for (auto &l : lane) maxl = std::max(maxl, l.size());
        for (size_t r = 0; r < maxl; ++r)
            for (int q = 0; q < 8; ++q)
                if (r < lane[q].size()) out.push_back(lane[q][r]);
        list.swap(out);
    }
}

int upload_items(hydro_ctx *c)
{
    std::vector<WorkItem> list, pb;
    build_items(c, list, pb, c->pb_start);
    if (c->d_items) (void)hipFree(c->d_items);
    if (c->d_items_pb) (void)hipFree(c->d_items_pb);
    c->d_items = c->d_items_pb = nullptr;
    c->nitems = (int)list.size();
    const size_t bytes = sizeof(WorkItem) * std::max<size_t>(1, list.size());
    HIP_TRY(c, hipMalloc(&c->d_items, bytes));
    HIP_TRY(c, hipMalloc(&c->d_items_pb, bytes));
    if (!list.empty()) {
        HIP_TRY(c, hipMemcpy(c->d_items, list.data(), sizeof(WorkItem) * list.size(), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_items_pb, pb.data(), sizeof(WorkItem) * pb.size(), hipMemcpyHostToDevice));
    }
    const int need = std::max(1, c->nitems);
    if (need > c->partial_cap) {
        if (c->d_partial) (void)hipFree(c->d_partial);
        c->d_partial = nullptr;
        HIP_TRY(c, hipMalloc(&c->d_partial, sizeof(double) * need));
        if (c->d_cflnext) (void)hipFree(c->d_cflnext);
        c->d_cflnext = nullptr;
        HIP_TRY(c, hipMalloc(&c->d_cflnext, sizeof(double) * need));
        c->partial_cap = need;
    }
    c->cfl_next_U = nullptr;     // the work list (and grid) may have changed
    return HYDRO_OK;
}

void drop_graph(hydro_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->g_U = c->g_dt = nullptr;
    c->g_cdt = -1;
}

void rk_coeffs(int rk, int s, double &a, double &b)
{
    a = 0.0;
    b = 1.0;
    if (rk == 2 && s == 2) { a = 0.5; b = 0.5; }
    if (rk == 3 && s == 2) { a = 0.75; b = 0.25; }
    if (rk == 3 && s == 3) { a = 1.0 / 3.0; b = 2.0 / 3.0; }
}

// Gravity and the shock detector of a problem (kGravity | kShock).
void phys_args(const hydro_ctx *c, int32_t &phys, double (&grav)[3], double &sthresh)
{
    phys = 0;
    grav[0] = grav[1] = grav[2] = 0.0;
    sthresh = 0.0;
    if (c->prm.flags & HYDRO_FLAG_GRAVITY) {
        phys |= kGravity;
        for (int d = 0; d < 3; ++d) grav[d] = c->prm.grav[d];
    }
    if (c->prm.flags & HYDRO_FLAG_SHOCK_DETECT) {
        phys |= kShock;
        sthresh = c->prm.shock_thresh;
    }
}

StageArgs stage_args(hydro_ctx *c, int s, const double *dt, const double *Un, const double *Us, double *Uout)
{
    StageArgs a{};
    a.blocks = c->d_blocks;
    a.faces = c->d_faces;
    a.items = c->d_items;
    a.nitems = c->nitems;
    a.stage = s;
    a.nc = c->ncell;
    a.gamma = c->prm.gamma;
    a.g1 = c->prm.gamma - 1.0;
    a.ig1 = 1.0 / (c->prm.gamma - 1.0);
    a.idx = 1.0 / c->prm.dx;
    a.idy = 1.0 / c->prm.dy;
    a.idz = 1.0 / c->prm.dz;
    rk_coeffs(c->prm.rk, s, a.a, a.b);
    a.eps = c->prm.weno_eps;
    a.dt = dt;
    a.Un = Un;
    a.Us = Us;
    a.Uout = Uout;
    a.nbad = c->d_nbad;
    a.freg = c->d_freg;
    a.nface = c->nface;
    phys_args(c, a.phys, a.grav, a.sthresh);
    return a;
}

AmrArgs amr_args(hydro_ctx *c, double *U)
{
    AmrArgs g{};
    g.blocks = c->d_blocks;
    g.amr = c->d_amr;
    g.faces = c->d_faces;
    g.nc = c->ncell;
    g.ng = (c->nblocks > 0) ? c->hb[0].ng : 1;
    if (c->nblocks > 0) {
        // every block of a mesh with levels has the same extents
        const hydro_block_t &B = c->hb[0];
        const int face = (c->prm.ndim == 3) ? std::max(B.ny * B.nz, std::max(B.nx * B.nz, B.nx * B.ny))
                                            : std::max(B.nx, B.ny);
        g.fchunks = (face * g.ng + 255) / 256;
    } else {
        g.fchunks = 1;
    }
    g.nface = c->nface;
    g.idx = 1.0 / c->prm.dx;
    g.idy = 1.0 / c->prm.dy;
    g.idz = 1.0 / c->prm.dz;
    g.freg = c->d_freg;
    g.U = U;
    return g;
}

// Guard layers of faces to another level, from the interiors of U.
int enqueue_amr_fill(hydro_ctx *c, double *U, hipStream_t st)
{
    AmrArgs g = amr_args(c, U);
    g.list = c->d_afill;
    g.nlist = c->nafill;
    hipError_t e = launch_amr_fill(g, c->prm.ndim, st);
    if (e != hipSuccess) return hip_fail(c, e, "level guard launch");
    return HYDRO_OK;
}

// Flux corrections of stage s on Uout for the coarse blocks of levels
// [l0, l1) (each block's faces in the order -x .. +z).
int enqueue_amr_correct(hydro_ctx *c, int s, const double *dt, double *Uout, int l0, int l1, hipStream_t st)
{
    AmrArgs g = amr_args(c, Uout);
    double a;
    rk_coeffs(c->prm.rk, s, a, g.b);
    g.dt = dt;
    g.list = c->d_acorr + c->acorr_start[l0];
    g.nlist = c->acorr_start[l1] - c->acorr_start[l0];
    hipError_t e = launch_amr_correct(g, c->prm.ndim, st);
    if (e != hipSuccess) return hip_fail(c, e, "flux correction launch");
    return HYDRO_OK;
}

int persistent_grid(hydro_ctx *c)
{
    int g = c->tune.grid > 0 ? std::min(c->tune.grid, c->nitems) : c->nitems;
    return g;
}

int enqueue_cfl(hydro_ctx *c, const double *U, double *dt, hipStream_t st)
{
    CflArgs a{};
    a.blocks = c->d_blocks;
    a.items = c->d_items;
    a.nitems = c->nitems;
    a.nc = c->ncell;
    a.gamma = c->prm.gamma;
    a.g1 = c->prm.gamma - 1.0;
    a.idx = 1.0 / c->prm.dx;
    a.idy = 1.0 / c->prm.dy;
    a.idz = 1.0 / c->prm.dz;
    a.U = U;
    a.partial = c->d_partial;
    a.nbad = c->d_nbad;
    const int grid = std::max(1, std::min(persistent_grid(c), c->partial_cap));
    hipError_t e = launch_cfl(a, c->prm.ndim, c->tune.tile, grid, c->prm.cfl, dt, st);
    if (e != hipSuccess) return hip_fail(c, e, "cfl launch");
    return HYDRO_OK;
}

int enqueue_guards(hydro_ctx *c, double *U, int b0, int nblk, hipStream_t st)
{
    GuardArgs g{};
    g.blocks = c->d_blocks;
    g.faces = c->d_faces;
    g.b0 = b0;
    g.nc = c->ncell;
    g.U = U;
    hipError_t e = launch_fill_guards(g, c->prm.ndim, nblk, st);
    if (e != hipSuccess) return hip_fail(c, e, "guard launch");
    return HYDRO_OK;
}

// One stage in the configured form.  In the per-block and materialised
// forms Us must be writable (its guard cells are filled before the stage
// kernel reads them, block by block or in one launch).
int enqueue_stage(hydro_ctx *c, int s, const double *dt, const double *Un, const double *Us, double *Uout,
                  hipStream_t st, double *cflo = nullptr)
{
    StageArgs a = stage_args(c, s, dt, Un, Us, Uout);
    if (c->tune.mode == HYDRO_MODE_MATERIALISED) {
        // one fill launch over every block, then the persistent stage launch
        // reading the filled guard cells (the stage's CFL record needs the
        // gathering kernel, so cflo is never set in this form)
        int rc = enqueue_guards(c, const_cast<double *>(Us), 0, c->nblocks, st);
        if (rc) return rc;
        hipError_t e = launch_stage(a, c->prm.ndim, c->prm.recon, c->tune.tile, c->tune.variant, false,
                                    persistent_grid(c), st);
        if (e != hipSuccess) return hip_fail(c, e, "stage launch");
        return HYDRO_OK;
    }
    if (c->tune.mode == HYDRO_MODE_PERBLOCK) {
        for (int b = 0; b < c->nblocks; ++b) {
            int rc = enqueue_guards(c, const_cast<double *>(Us), b, 1, st);
            if (rc) return rc;
            a.items = c->d_items_pb + c->pb_start[b];
            a.nitems = c->pb_start[b + 1] - c->pb_start[b];
            hipError_t e = launch_stage(a, c->prm.ndim, c->prm.recon, c->tune.tile, c->tune.variant, false, a.nitems, st);
            if (e != hipSuccess) return hip_fail(c, e, "stage launch");
        }
        return HYDRO_OK;
    }
    if (c->amr) {
        int rc = enqueue_amr_fill(c, const_cast<double *>(Us), st);
        if (rc) return rc;
        if (c->prm.flags & HYDRO_FLAG_LEVEL_BY_LEVEL) {
            for (int L = c->nlev - 1; L >= 0; --L) {
                a.items = c->d_items + c->lvl_first[L];
                a.nitems = c->lvl_count[L];
                const int grid = c->tune.grid > 0 ? std::min(c->tune.grid, a.nitems) : a.nitems;
                hipError_t e = launch_stage(a, c->prm.ndim, c->prm.recon, c->tune.tile, c->tune.variant, true, grid, st);
                if (e != hipSuccess) return hip_fail(c, e, "stage launch");
                if ((rc = enqueue_amr_correct(c, s, dt, Uout, L, L + 1, st))) return rc;
            }
            return HYDRO_OK;
        }
        hipError_t e = launch_stage(a, c->prm.ndim, c->prm.recon, c->tune.tile, c->tune.variant, true, persistent_grid(c), st);
        if (e != hipSuccess) return hip_fail(c, e, "stage launch");
        return enqueue_amr_correct(c, s, dt, Uout, 0, c->nlev, st);
    }
    a.cfl_partial = cflo;
    hipError_t e = launch_stage(a, c->prm.ndim, c->prm.recon, c->tune.tile, c->tune.variant, true, persistent_grid(c), st);
    if (e != hipSuccess) return hip_fail(c, e, "stage launch");
    return HYDRO_OK;
}

// Stage buffers: RK2 U -> B0 -> U ; RK3 U -> B0 -> B1 -> U.  The final stage
// writes U in place (it reads U^n only at the cell it writes).
int enqueue_step_tele(hydro_ctx *c, double *U, double *dt, int compute_dt, hipStream_t st);

// dt modes of a step: 0 the caller's dt; 1 the CFL dt of U; 2 the CFL dt
// from the maxima the previous fused step's final stage recorded for U, and
// 3 the CFL dt of U; in modes 2 and 3 the final stage records the maxima of
// the state it writes for the next step.
int enqueue_step(hydro_ctx *c, double *U, double *dt, int mode, hipStream_t st)
{
    if (c->tune.mode == HYDRO_MODE_TELESCOPING) return enqueue_step_tele(c, U, dt, mode, st);
    int rc;
    if (mode == 2) {
        hipError_t e = launch_cfl_final(c->d_cflnext, c->ncflnext, c->prm.cfl, dt, st);
        if (e != hipSuccess) return hip_fail(c, e, "cfl launch");
    } else if (mode && (rc = enqueue_cfl(c, U, dt, st))) {
        return rc;
    }
    const int S = c->prm.rk;
    double *in = U;
    for (int s = 1; s <= S; ++s) {
        double *out = (s == S) ? U : c->d_buf[(s - 1) & 1];
        double *cflo = (s == S && mode >= 2) ? c->d_cflnext : nullptr;
        if ((rc = enqueue_stage(c, s, dt, U, in, out, st, cflo))) return rc;
        in = out;
    }
    if (mode >= 2) c->ncflnext = persistent_grid(c);
    return HYDRO_OK;
}

// Work lists and tables of the adjoint (built on first use).
int setup_vjp(hydro_ctx *c)
{
    if (c->d_vjp) return HYDRO_OK;
    const int nd = c->prm.ndim;
    // lines along each direction, grouped by 64 within a block; small
    // problems cut each line into up to 4 segments for more threads
    int64_t total_lines = 0;
    for (int b = 0; b < c->nblocks; ++b)
        for (int d = 0; d < nd; ++d) {
            const hydro_block_t &B = c->hb[b];
            total_lines += (int64_t)((d == 0) ? B.ny : B.nx) * ((nd == 3) ? ((d == 2) ? B.ny : B.nz) : 1);
        }
    const int64_t want = 131072;  // about two waves per SIMD
    c->nseg = (int)std::max<int64_t>(1, std::min<int64_t>(4, (want + total_lines - 1) / std::max<int64_t>(1, total_lines)));
    std::vector<WorkItem> v;
    for (int s = 0; s < c->nseg; ++s)
    for (int d = 0; d < nd; ++d) {
        for (int b = 0; b < c->nblocks; ++b) {
            const hydro_block_t &B = c->hb[b];
            const int n1 = (d == 0) ? B.ny : B.nx;
            const int n2 = (nd == 3) ? ((d == 2) ? B.ny : B.nz) : 1;
            const int nl = n1 * n2;
            for (int l0 = 0; l0 < nl; l0 += 64) {
                WorkItem w{};
                w.block = b;
                w.xy = l0;
                w.z = std::min(64, nl - l0);
                w.cost = d | (s << 4);
                v.push_back(w);
            }
        }
    }
    c->nlines = (int)v.size();
    HIP_TRY(c, hipMalloc(&c->d_lines, sizeof(WorkItem) * std::max<size_t>(1, v.size())));
    if (!v.empty())
        HIP_TRY(c, hipMemcpy(c->d_lines, v.data(), sizeof(WorkItem) * v.size(), hipMemcpyHostToDevice));
    // cell tiles of 16 x 4 (a 128-byte row segment per tile row) over runs of
    // at most 4 z planes, so that every wave has independent rows to load
    std::vector<WorkItem> ci;
    for (int b = 0; b < c->nblocks; ++b) {
        const hydro_block_t &B = c->hb[b];
        const int nz = (nd == 3) ? B.nz : 1;
        for (int z0 = 0; z0 < nz; z0 += 4)
            for (int y0 = 0; y0 < B.ny; y0 += 4)
                for (int x0 = 0; x0 < B.nx; x0 += 16) {
                    WorkItem w{};
                    w.block = b;
                    w.xy = x0 | (y0 << 16);
                    w.z = z0 | (std::min(4, nz - z0) << 16);
                    ci.push_back(w);
                }
    }
    // The row tiles of one plane run share the cache lines of the transposed
    // x-line array (rows of ny doubles) and the lines that padded rows
    // straddle; guard copies read the neighbouring blocks' arrays.
    interleave_block_ranges(ci);
    c->ncitems = (int)ci.size();
    HIP_TRY(c, hipMalloc(&c->d_citems, sizeof(WorkItem) * std::max<size_t>(1, ci.size())));
    if (!ci.empty())
        HIP_TRY(c, hipMemcpy(c->d_citems, ci.data(), sizeof(WorkItem) * ci.size(), hipMemcpyHostToDevice));
    // x-line transpose: 16 positions x 16 rows of one plane per tile, positions -H .. nx+H-1
    {
        const int Hs = (c->prm.recon == HYDRO_WENO5) ? 3 : 2;
        std::vector<WorkItem> xi;
        for (int b = 0; b < c->nblocks; ++b) {
            const hydro_block_t &B = c->hb[b];
            const int nz = (nd == 3) ? B.nz : 1;
            for (int k = 0; k < nz; ++k)
                for (int j0 = 0; j0 < B.ny; j0 += 16)
                    for (int p0 = 0; p0 < B.nx + 2 * Hs; p0 += 16) {
                        WorkItem w{};
                        w.block = b;
                        w.xy = p0 | (j0 << 16);
                        w.z = k;
                        xi.push_back(w);
                    }
        }
        // a tile reads its x halo from the neighbouring blocks
        interleave_block_ranges(xi);
        c->nxitems = (int)xi.size();
        HIP_TRY(c, hipMalloc(&c->d_xitems, sizeof(WorkItem) * std::max<size_t>(1, xi.size())));
        if (!xi.empty())
            HIP_TRY(c, hipMemcpy(c->d_xitems, xi.data(), sizeof(WorkItem) * xi.size(), hipMemcpyHostToDevice));
    }
    // inverse links: for block b, every (block X, dir, side, kind) whose guards copy cells of b
    std::vector<std::vector<int4>> inc(c->nblocks);
    for (int x = 0; x < c->nblocks; ++x)
        for (int d = 0; d < nd; ++d)
            for (int side = 0; side < 2; ++side) {
                const int nb = c->hl[x].nbr[2 * d + side];
                if (nb >= 0) inc[nb].push_back(make_int4(x, d, side, 0));
                else if (nb == HYDRO_PERIODIC_SELF) inc[x].push_back(make_int4(x, d, side, 0));
                else inc[x].push_back(make_int4(x, d, side, 1));
            }
    std::vector<int> start(c->nblocks + 1, 0);
    std::vector<int4> flat;
    for (int b = 0; b < c->nblocks; ++b) {
        start[b] = (int)flat.size();
        flat.insert(flat.end(), inc[b].begin(), inc[b].end());
    }
    start[c->nblocks] = (int)flat.size();
    HIP_TRY(c, hipMalloc(&c->d_inc_start, sizeof(int) * start.size()));
    HIP_TRY(c, hipMemcpy(c->d_inc_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMalloc(&c->d_inc, sizeof(int4) * std::max<size_t>(1, flat.size())));
    if (!flat.empty())
        HIP_TRY(c, hipMemcpy(c->d_inc, flat.data(), sizeof(int4) * flat.size(), hipMemcpyHostToDevice));
    const size_t per = (size_t)c->nv * (size_t)std::max<int64_t>(1, c->ncell);
    if (hipMalloc(&c->d_vjp, sizeof(double) * per * (size_t)(nd * c->nseg + 3)) != hipSuccess) {
        c->d_vjp = nullptr;
        return fail(c, HYDRO_ENOMEM, "adjoint scratch");
    }
    return HYDRO_OK;
}

// Telescoping step tables (built when that mode is selected).
int setup_tele(hydro_ctx *c)
{
    const int nd = c->prm.ndim, S = c->prm.rk;
    const int H = (c->prm.recon == HYDRO_WENO5) ? 3 : 2;
    const int ngt = S * H;
    for (int b = 0; b < c->nblocks; ++b)
        for (int d = 0; d < nd; ++d)
            for (int side = 0; side < 2; ++side) {
                const int nb = c->hl[b].nbr[2 * d + side];
                const hydro_block_t &Src = (nb >= 0) ? c->hb[nb] : c->hb[b];
                if (nb != HYDRO_OUTFLOW && extent(Src, d) < ngt)
                    return fail(c, HYDRO_EINVAL, "telescoping halo (" + std::to_string(ngt) +
                                " layers) deeper than a source block");
            }
    if (c->tele_ready) return HYDRO_OK;
    std::vector<DevBlock> tb(c->nblocks);
    int64_t off = 0;
    for (int b = 0; b < c->nblocks; ++b) {
        const hydro_block_t &B = c->hb[b];
        DevBlock D{};
        D.off = off;
        D.nx = B.nx; D.ny = B.ny; D.nz = B.nz; D.ng = ngt;
        D.px = B.nx + 2 * ngt;
        D.py = B.ny + 2 * ngt;
        D.gz = (nd == 3) ? ngt : 0;
        D.ix = 1.0 / c->prm.dx;
        D.iy = 1.0 / c->prm.dy;
        D.iz = 1.0 / c->prm.dz;
        tb[b] = D;
        off += (int64_t)D.px * D.py * ((nd == 3) ? B.nz + 2 * ngt : 1);
    }
    c->ncell_t = off;
    c->ngt = ngt;
    std::vector<FaceSrc> tf((size_t)c->nblocks * 6, FaceSrc{0, 0, 0, 0, 0, -1, 0});
    for (int b = 0; b < c->nblocks; ++b)
        for (int d = 0; d < nd; ++d)
            for (int side = 0; side < 2; ++side) {
                const int nb = c->hl[b].nbr[2 * d + side];
                const int n = extent(c->hb[b], d);
                const int src = (nb >= 0) ? nb : b;
                FaceSrc f{};
                f.reg = -1;
                f.off = tb[src].off;
                f.px = tb[src].px;
                f.py = tb[src].py;
                if (nb == HYDRO_OUTFLOW) { f.A = (side == 0) ? 0 : n - 1; f.B = 0; }
                else { f.A = (side == 0) ? extent(c->hb[src], d) : -n; f.B = 1; }
                tf[(size_t)b * 6 + 2 * d + side] = f;
            }
    HIP_TRY(c, hipMalloc(&c->d_tblocks, sizeof(DevBlock) * std::max(1, c->nblocks)));
    HIP_TRY(c, hipMalloc(&c->d_tfaces, sizeof(FaceSrc) * std::max(1, c->nblocks) * 6));
    if (c->nblocks) {
        HIP_TRY(c, hipMemcpy(c->d_tblocks, tb.data(), sizeof(DevBlock) * c->nblocks, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(c->d_tfaces, tf.data(), sizeof(FaceSrc) * c->nblocks * 6, hipMemcpyHostToDevice));
    }
    const int TX = tile_x(c->tune.tile), TY = tile_y(c->tune.tile);
    for (int s = 1; s <= S; ++s) {
        const int m = (S - s) * H;
        std::vector<DevBlock> vb(c->nblocks);
        std::vector<WorkItem> items;
        for (int b = 0; b < c->nblocks; ++b) {
            DevBlock V = tb[b];
            V.nx += 2 * m;
            V.ny += 2 * m;
            if (nd == 3) V.nz += 2 * m;
            V.ng = ngt - m;
            V.gz = (nd == 3) ? ngt - m : 0;
            vb[b] = V;
            for (int y0 = 0; y0 < V.ny; y0 += TY)
                for (int x0 = 0; x0 < V.nx; x0 += TX) {
                    WorkItem w{};
                    w.block = b;
                    w.xy = x0 | (y0 << 16);
                    w.z = 0 | (V.nz << 16);
                    w.cost = std::min(TX, V.nx - x0) * std::min(TY, V.ny - y0) * V.nz;
                    items.push_back(w);
                }
        }
        std::stable_sort(items.begin(), items.end(), [](const WorkItem &x, const WorkItem &y) { return x.cost > y.cost; });
        HIP_TRY(c, hipMalloc(&c->d_vblocks[s - 1], sizeof(DevBlock) * std::max(1, c->nblocks)));
        HIP_TRY(c, hipMalloc(&c->d_titems[s - 1], sizeof(WorkItem) * std::max<size_t>(1, items.size())));
        if (c->nblocks)
            HIP_TRY(c, hipMemcpy(c->d_vblocks[s - 1], vb.data(), sizeof(DevBlock) * c->nblocks, hipMemcpyHostToDevice));
        if (!items.empty())
            HIP_TRY(c, hipMemcpy(c->d_titems[s - 1], items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
        c->ntitems[s - 1] = (int)items.size();
    }
    const size_t per = (size_t)c->nv * (size_t)std::max<int64_t>(1, c->ncell_t);
    if (hipMalloc(&c->d_tbuf, sizeof(double) * per * (S == 3 ? 3 : 2)) != hipSuccess) {
        c->d_tbuf = nullptr;
        return fail(c, HYDRO_ENOMEM, "telescoping buffers");
    }
    c->tele_ready = 1;
    return HYDRO_OK;
}

void free_tele(hydro_ctx *c)
{
    (void)hipFree(c->d_tblocks);
    (void)hipFree(c->d_tfaces);
    for (int s = 0; s < 3; ++s) {
        (void)hipFree(c->d_vblocks[s]);
        (void)hipFree(c->d_titems[s]);
        c->d_vblocks[s] = nullptr;
        c->d_titems[s] = nullptr;
        c->ntitems[s] = 0;
    }
    (void)hipFree(c->d_tbuf);
    c->d_tblocks = nullptr;
    c->d_tfaces = nullptr;
    c->d_tbuf = nullptr;
    c->tele_ready = 0;
}

// Telescoping step: CFL dt on U, one thick fill, S stages on the shrinking
// extended blocks (the last writes the thick U^n copy in place), copy back.
int enqueue_step_tele(hydro_ctx *c, double *U, double *dt, int compute_dt, hipStream_t st)
{
    int rc;
    if (compute_dt && (rc = enqueue_cfl(c, U, dt, st))) return rc;
    const int nd = c->prm.ndim, S = c->prm.rk;
    const size_t per = (size_t)c->nv * (size_t)c->ncell_t;
    double *Tn = c->d_tbuf, *TA = c->d_tbuf + per, *TB = (S == 3) ? c->d_tbuf + 2 * per : nullptr;
    TeleArgs t{};
    t.tb = c->d_tblocks;
    t.tf = c->d_tfaces;
    t.ub = c->d_blocks;
    t.nct = c->ncell_t;
    t.ncu = c->ncell;
    t.T = Tn;
    t.U = U;
    hipError_t e = launch_tele_copy(t, nd, c->nblocks, true, st);
    if (e != hipSuccess) return hip_fail(c, e, "telescoping load");
    for (int d = 0; d < nd; ++d) {
        t.d = d;
        e = launch_tele_fill(t, nd, c->nblocks, st);
        if (e != hipSuccess) return hip_fail(c, e, "telescoping fill");
    }
    const double *in = Tn;
    for (int s = 1; s <= S; ++s) {
        double *out = (s == S) ? Tn : ((s == 1) ? TA : TB);
        StageArgs a = stage_args(c, s, dt, Tn, in, out);
        a.blocks = c->d_vblocks[s - 1];
        a.items = c->d_titems[s - 1];
        a.nitems = c->ntitems[s - 1];
        a.nc = c->ncell_t;
        const int grid = c->tune.grid > 0 ? std::min(c->tune.grid, a.nitems) : a.nitems;
        e = launch_stage(a, nd, c->prm.recon, c->tune.tile, c->tune.variant, false, grid, st);
        if (e != hipSuccess) return hip_fail(c, e, "telescoping stage launch");
        in = out;
    }
    e = launch_tele_copy(t, nd, c->nblocks, false, st);
    if (e != hipSuccess) return hip_fail(c, e, "telescoping store");
    return HYDRO_OK;
}

// Device tables of a mesh with refinement levels: the level table, flux
// registers for every face to another level, the list of those faces (guard
// fill) and the coarse faces with finer neighbours by face and level
// (correction).  Returns non-zero with c->err set on failure.
int setup_amr(hydro_ctx *c)
{
    const int nd = c->prm.ndim;
    int nslots = 0;
    for (const FaceSrc &f : c->h_faces) nslots += (f.reg >= 0);
    c->nface = 1;
    if (c->nblocks > 0) {
        const hydro_block_t &B = c->hb[0];
        c->nface = std::max(B.ny * B.nz, B.nx * B.nz);
        if (nd == 3) c->nface = std::max(c->nface, B.nx * B.ny);
        if (nd == 2) c->nface = std::max(B.nx, B.ny);
    }
    std::vector<DevAmr> da(std::max(1, c->nblocks));
    std::vector<int2> fill;
    for (int b = 0; b < c->nblocks; ++b) {
        for (int f = 0; f < 6; ++f) {
            da[b].kind[f] = c->ha[b].kind[f];
            for (int h = 0; h < 4; ++h) da[b].nbr[f][h] = c->ha[b].nbr[f][h];
            if (f < 2 * nd && c->ha[b].kind[f] != 0) fill.push_back(make_int2(b, f));
        }
    }
    std::vector<int2> corr;
    c->acorr_start.assign((size_t)c->nlev + 1, 0);
    for (int L = 0; L <= c->nlev; ++L) {
        c->acorr_start[L] = (int)corr.size();
        if (L == c->nlev) continue;
        for (int b = 0; b < c->nblocks; ++b) {
            bool finer = false;
            for (int f = 0; f < 2 * nd; ++f) finer |= (c->ha[b].kind[f] == 2);
            if (c->ha[b].level == L && finer) corr.push_back(make_int2(b, 0));
        }
    }
    c->nafill = (int)fill.size();
    const size_t regs = (size_t)std::max(1, nslots) * c->nv * c->nface;
    if (hipMalloc(&c->d_amr, sizeof(DevAmr) * da.size()) != hipSuccess ||
        hipMalloc(&c->d_freg, sizeof(double) * regs) != hipSuccess ||
        hipMalloc(&c->d_afill, sizeof(int2) * std::max<size_t>(1, fill.size())) != hipSuccess ||
        hipMalloc(&c->d_acorr, sizeof(int2) * std::max<size_t>(1, corr.size())) != hipSuccess) {
        c->err = "device tables (levels)";
        return 1;
    }
    if (hipMemcpy(c->d_amr, da.data(), sizeof(DevAmr) * da.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (!fill.empty() && hipMemcpy(c->d_afill, fill.data(), sizeof(int2) * fill.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        (!corr.empty() && hipMemcpy(c->d_acorr, corr.data(), sizeof(int2) * corr.size(), hipMemcpyHostToDevice) != hipSuccess)) {
        c->err = "level table upload";
        return 1;
    }
    return 0;
}

}  // namespace

// Element-wise division, square root and fused multiply-add, compiled with
// the settings of the step kernels (the device-arithmetic check).
static __global__ void __launch_bounds__(256) k_fp_check(const double *__restrict__ a, const double *__restrict__ b,
                                                  const double *__restrict__ c, double *__restrict__ quot,
                                                  double *__restrict__ root, double *__restrict__ fmad, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = a[i], y = b[i];
        quot[i] = x / y;
        root[i] = sqrt(x);
        fmad[i] = fma(x, y, c[i]);
    }
}

static hipError_t launch_fp_check(const double *a, const double *b, const double *c, double *quot, double *root,
                           double *fmad, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 255) / 256;
    const int grid = (int)std::min<int64_t>(want, 65536);
    k_fp_check<<<grid, 256, 0, st>>>(a, b, c, quot, root, fmad, n);
    return hipGetLastError();
}

extern "C" {

int hydro_validate(const hydro_params_t *params, const hydro_block_t *blocks, const hydro_link_t *links,
                   int32_t nblocks, int64_t ncell_total)
{
    return check_problem(params, blocks, links, nblocks, ncell_total).empty() ? HYDRO_OK : HYDRO_EINVAL;
}

// Text of the last error of a call without a context (hydro_create,
// hydro_create_amr, hydro_cfl_dt_noalloc), per thread.
thread_local std::string g_noctx_err;

int hydro_validate_amr(const hydro_params_t *params, const hydro_block_t *blocks, const hydro_link_t *links,
                       const hydro_amr_t *amr, int32_t nblocks, int64_t ncell_total)
{
    return check_amr(params, blocks, links, amr, nblocks, ncell_total).empty() ? HYDRO_OK : HYDRO_EINVAL;
}

static int create_ctx(const hydro_params_t *params, const hydro_block_t *blocks, const hydro_link_t *links,
                      const hydro_amr_t *amr, int32_t nblocks, int64_t ncell_total, void *stream, hydro_ctx_t **out)
{
    if (!out) return HYDRO_EINVAL;
    *out = nullptr;
    std::string why = amr ? check_amr(params, blocks, links, amr, nblocks, ncell_total)
                          : check_problem(params, blocks, links, nblocks, ncell_total);
    if (!why.empty()) {
        g_noctx_err = why;
        return HYDRO_EINVAL;
    }
    hydro_ctx *c = new hydro_ctx();
    c->prm = *params;
    c->nblocks = nblocks;
    c->ncell = ncell_total;
    c->nv = params->ndim + 2;
    c->hb.assign(blocks, blocks + nblocks);
    c->hl.assign(links, links + nblocks);
    c->stream = (hipStream_t)stream;
    if (amr) {
        c->amr = true;
        c->ha.assign(amr, amr + nblocks);
        for (int b = 0; b < nblocks; ++b) c->nlev = std::max(c->nlev, amr[b].level + 1);
    }
    auto bail = [&](int code) {
        g_noctx_err = c->err;
        hydro_destroy(c);
        return code;
    };
    if (hipGetDevice(&c->device) != hipSuccess) { c->err = "no HIP device"; return bail(HYDRO_EHIP); }
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        c->err = "capture stream";
        return bail(HYDRO_EHIP);
    }
    build_tables(c);
    const size_t nb = std::max<int>(1, nblocks);
    if (hipMalloc(&c->d_blocks, sizeof(DevBlock) * nb) != hipSuccess ||
        hipMalloc(&c->d_faces, sizeof(FaceSrc) * nb * 6) != hipSuccess ||
        hipMalloc(&c->d_nbad, sizeof(unsigned long long)) != hipSuccess) {
        c->err = "device tables";
        return bail(HYDRO_ENOMEM);
    }
    if (nblocks > 0) {
        if (hipMemcpy(c->d_blocks, c->h_dev.data(), sizeof(DevBlock) * nblocks, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->d_faces, c->h_faces.data(), sizeof(FaceSrc) * nblocks * 6, hipMemcpyHostToDevice) != hipSuccess) {
            c->err = "table upload";
            return bail(HYDRO_EHIP);
        }
    }
    if (hipMemset(c->d_nbad, 0, sizeof(unsigned long long)) != hipSuccess) { c->err = "memset"; return bail(HYDRO_EHIP); }
    const size_t sbytes = sizeof(double) * (size_t)c->nv * (size_t)std::max<int64_t>(1, ncell_total);
    const int nbuf = (params->rk == 3) ? 2 : 1;
    for (int q = 0; q < nbuf; ++q)
        if (hipMalloc(&c->d_buf[q], sbytes) != hipSuccess) { c->err = "stage buffers"; return bail(HYDRO_ENOMEM); }
    // default tuning: the tile with the best lane use (ties: larger), persistent, graph
    double best = -1.0;
    int tbest = 0;
    for (int t = 0; t < 3; ++t) {
        const int TX = tile_x(t), TY = tile_y(t);
        double used = 0.0, paid = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            const auto &B = blocks[b];
            used += (double)B.nx * B.ny;
            paid += (double)((B.nx + TX - 1) / TX) * TX * ((B.ny + TY - 1) / TY) * TY;
        }
        const double u = paid > 0 ? used / paid : 1.0;
        if (u >= best - 1e-12) { best = u; tbest = t; }
    }
    c->tune.mode = HYDRO_MODE_PERSISTENT;
    c->tune.tile = tbest;
    c->tune.grid = 0;
    c->tune.zchunk = 0;
    c->tune.use_graph = 1;
    c->tune.xcd = 0;
    c->tune.variant = 0;
    if (c->amr) {
        if (setup_amr(c)) return bail(c->err.rfind("device", 0) == 0 ? HYDRO_ENOMEM : HYDRO_EHIP);
    }
    int rc = upload_items(c);
    if (rc) return bail(rc);
    *out = c;
    return HYDRO_OK;
}

int hydro_create(const hydro_params_t *params, const hydro_block_t *blocks, const hydro_link_t *links,
                 int32_t nblocks, int64_t ncell_total, void *stream, hydro_ctx_t **out)
{
    return create_ctx(params, blocks, links, nullptr, nblocks, ncell_total, stream, out);
}

int hydro_create_amr(const hydro_params_t *params, const hydro_block_t *blocks, const hydro_link_t *links,
                     const hydro_amr_t *amr, int32_t nblocks, int64_t ncell_total, void *stream, hydro_ctx_t **out)
{
    if (!amr && nblocks > 0) {
        g_noctx_err = "null level table";
        return HYDRO_EINVAL;
    }
    hydro_amr_t none{};
    return create_ctx(params, blocks, links, amr ? amr : &none, nblocks, ncell_total, stream, out);
}

int hydro_set_tuning(hydro_ctx_t *c, const hydro_tuning_t *t)
{
    if (!c || !t) return HYDRO_EINVAL;
    if (t->mode != HYDRO_MODE_PERSISTENT && t->mode != HYDRO_MODE_PERBLOCK && t->mode != HYDRO_MODE_TELESCOPING &&
        t->mode != HYDRO_MODE_MATERIALISED)
        return fail(c, HYDRO_EINVAL, "mode");
    if (t->tile < 0 || t->tile > 2 || t->grid < 0 || t->zchunk < 0 || t->variant < 0 || t->variant > 1 ||
        t->xcd < 0 || t->xcd > 2)
        return fail(c, HYDRO_EINVAL, "tuning range");
    if (c->amr && t->mode != HYDRO_MODE_PERSISTENT)
        return fail(c, HYDRO_EINVAL, "a mesh with refinement levels runs in the persistent mode only");
    if ((c->prm.flags & HYDRO_FLAG_SHOCK_DETECT) && t->mode == HYDRO_MODE_TELESCOPING)
        return fail(c, HYDRO_EINVAL, "the telescoping step runs the block initialisation (shock detector) once "
                                     "per step: not built with the detector");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    const int old_tile = c->tune.tile;
    c->tune = *t;
    int rc = upload_items(c);
    if (rc) return rc;
    if (c->tele_ready && old_tile != t->tile) free_tele(c);
    if (t->mode == HYDRO_MODE_TELESCOPING) {
        rc = setup_tele(c);
        if (rc) {
            c->tune.mode = HYDRO_MODE_PERSISTENT;
            return rc;
        }
    }
    return HYDRO_OK;
}

int hydro_get_tuning(hydro_ctx_t *c, hydro_tuning_t *t)
{
    if (!c || !t) return HYDRO_EINVAL;
    *t = c->tune;
    return HYDRO_OK;
}

int hydro_fill_guards(hydro_ctx_t *c, double *U)
{
    if (!c || !U) return HYDRO_EINVAL;
    int rc = enqueue_guards(c, U, 0, c->nblocks, c->stream);
    if (rc || !c->amr) return rc;
    return enqueue_amr_fill(c, U, c->stream);
}

int hydro_cfl_dt(hydro_ctx_t *c, const double *U, double *dt_dev)
{
    if (!c || !U || !dt_dev) return fail(c, HYDRO_EINVAL, "null pointer");
    if (c->nitems == 0) return fail(c, HYDRO_EINVAL, "no cells");
    return enqueue_cfl(c, U, dt_dev, c->stream);
}

int hydro_rk_stage(hydro_ctx_t *c, int32_t stage, const double *dt_dev, const double *Un, const double *Us,
                   double *Uout)
{
    if (!c || !dt_dev || !Un || !Us || !Uout) return fail(c, HYDRO_EINVAL, "null pointer");
    if (stage < 1 || stage > c->prm.rk) return fail(c, HYDRO_EINVAL, "stage out of range");
    if (c->tune.mode == HYDRO_MODE_TELESCOPING)
        return fail(c, HYDRO_EINVAL, "single stages are not defined in the telescoping mode");
    if (Uout == Us) return fail(c, HYDRO_EINVAL, "Uout aliases Us");
    c->cfl_next_U = nullptr;     // it may write the state a fused step recorded
    return enqueue_stage(c, stage, dt_dev, Un, Us, Uout, c->stream);
}

}  // extern "C"

namespace {

// Enqueue one step with dt mode cdt (see enqueue_step), directly or through
// the ctx's graph.
int step_launch(hydro_ctx *c, double *U, double *dt_dev, int cdt)
{
    if (!c->tune.use_graph || c->tune.mode == HYDRO_MODE_PERBLOCK) return enqueue_step(c, U, dt_dev, cdt, c->stream);
    // The graph is bound to (U, dt, dt mode).  A call with other arguments
    // is launched directly; it is captured only when the same arguments come
    // twice in a row, so callers that step ever-new buffers (a recomputation
    // from checkpoints) pay no capture per step.
    const bool repeat = (c->l_U == U && c->l_dt == dt_dev && c->l_cdt == cdt);
    c->l_U = U;
    c->l_dt = dt_dev;
    c->l_cdt = cdt;
    const bool bound = c->gexec && c->g_U == U && c->g_dt == dt_dev && c->g_cdt == cdt;
    if (!bound && !repeat) return enqueue_step(c, U, dt_dev, cdt, c->stream);
    if (!bound) {
        drop_graph(c);
        HIP_TRY(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_step(c, U, dt_dev, cdt, c->cap);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(c, e, "end capture");
        c->graph = g;
        e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(c);
            return hip_fail(c, e, "graph instantiate");
        }
        c->g_U = U;
        c->g_dt = dt_dev;
        c->g_cdt = cdt;
    }
    HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
    return HYDRO_OK;
}

}  // namespace

extern "C" {

int hydro_step(hydro_ctx_t *c, double *U, double *dt_dev, int32_t compute_dt)
{
    if (!c || !U || !dt_dev) return fail(c, HYDRO_EINVAL, "null pointer");
    if (c->nitems == 0) return HYDRO_OK;
    // dt mode (see enqueue_step): fused only in the persistent form on a mesh
    // without levels, where the final stage covers every cell in one launch
    int cdt = compute_dt ? 1 : 0;
    if ((compute_dt == HYDRO_DT_FROM_PREVIOUS || compute_dt == HYDRO_DT_RECORD) &&
        c->tune.mode == HYDRO_MODE_PERSISTENT && !c->amr)
        cdt = (compute_dt == HYDRO_DT_FROM_PREVIOUS && c->cfl_next_U == U) ? 2 : 3;
    // the recorded maxima describe U only once this step is enqueued
    c->cfl_next_U = nullptr;
    const int rc = step_launch(c, U, dt_dev, cdt);
    if (rc == HYDRO_OK && cdt >= 2) c->cfl_next_U = U;
    return rc;
}

// The step VJP; stages (S-1 device pointers) holds the stage inputs U_2 ..
// U_S, or is null, and then they are recomputed from Un into the ctx's
// stage buffers.
static int step_vjp(hydro_ctx_t *c, const double *Un, const double *const *stages, const double *dt_dev,
                    const double *gUnext, double *gUn)
{
    if (!c || !Un || !dt_dev || !gUnext || !gUn) return fail(c, HYDRO_EINVAL, "null pointer");
    if (gUn == gUnext) return fail(c, HYDRO_EINVAL, "gUn aliases gUnext");
    if (gUn == Un) return fail(c, HYDRO_EINVAL, "gUn aliases Un");
    if (c->tune.mode == HYDRO_MODE_TELESCOPING)
        return fail(c, HYDRO_EINVAL, "the adjoint is defined for the per-stage-fill step only");
    if (c->amr) return fail(c, HYDRO_EINVAL, "the adjoint is defined on meshes without refinement levels");
    const int S = c->prm.rk, nd = c->prm.ndim;
    if (stages)
        for (int s = 0; s < S - 1; ++s) {
            if (!stages[s]) return fail(c, HYDRO_EINVAL, "null stage input pointer");
            if (stages[s] == gUn) return fail(c, HYDRO_EINVAL, "gUn aliases a stage input");
        }
    if (c->nitems == 0) return HYDRO_OK;
    int rc = setup_vjp(c);
    if (rc) return rc;
    hipStream_t st = c->stream;
    const size_t per = (size_t)c->nv * (size_t)c->ncell;
    const double *Us_of[4] = {nullptr, Un, c->d_buf[0], c->d_buf[1]};
    if (stages) {
        for (int s = 2; s <= S; ++s) Us_of[s] = stages[s - 2];
    } else {
        // forward recomputation of the stage inputs U_2 .. U_S
        for (int s = 1; s < S; ++s) {
            StageArgs a = stage_args(c, s, dt_dev, Un, Us_of[s], c->d_buf[s - 1]);
            hipError_t e = launch_stage(a, nd, c->prm.recon, c->tune.tile, c->tune.variant, true,
                                        persistent_grid(c), st);
            if (e != hipSuccess) return hip_fail(c, e, "stage launch");
        }
    }
    HIP_TRY(c, hipMemsetAsync(gUn, 0, sizeof(double) * per, st));
    const size_t narr = (size_t)nd * c->nseg;
    // one stage-cotangent array: the last stage reads the caller's gUnext and
    // writes gS; every earlier stage reads and writes gS in place (the cell
    // kernel reads a cell's output cotangent before writing the same cell's
    // input cotangent, and the transpose and line kernels, which read the
    // output cotangents of other cells, have finished by then)
    double *gW = c->d_vjp, *gS = c->d_vjp + narr * per;
    double *UsT = c->d_vjp + (narr + 1) * per, *gOutT = c->d_vjp + (narr + 2) * per;
    const double *g = gUnext;
    for (int s = S; s >= 1; --s) {
        VjpArgs v{};
        v.blocks = c->d_blocks;
        v.faces = c->d_faces;
        v.citems = c->d_citems;
        v.ncitems = c->ncitems;
        v.nc = c->ncell;
        v.gamma = c->prm.gamma;
        v.g1 = c->prm.gamma - 1.0;
        v.ig1 = 1.0 / (c->prm.gamma - 1.0);
        v.idx = 1.0 / c->prm.dx;
        v.idy = 1.0 / c->prm.dy;
        v.idz = 1.0 / c->prm.dz;
        rk_coeffs(S, s, v.a, v.b);
        v.eps = c->prm.weno_eps;
        v.dt = dt_dev;
        v.Us = Us_of[s];
        v.gOut = g;
        v.gW = gW;
        v.gUs = gS;
        v.gUn = gUn;                 // s >= 2: += a gOut; s = 1: += gU_1
        v.last = (s == 1) ? 1 : 0;
        v.inc_start = c->d_inc_start;
        v.inc = c->d_inc;
        v.nseg = c->nseg;
        v.items = c->d_lines;
        v.nitems = c->nlines;
        v.xitems = c->d_xitems;
        v.nxitems = c->nxitems;
        v.UsT = UsT;
        v.gOutT = gOutT;
        phys_args(c, v.phys, v.grav, v.sthresh);
        hipError_t ex = launch_vjp_xpose(v, nd, c->prm.recon, st);
        if (ex != hipSuccess) return hip_fail(c, ex, "adjoint transpose launch");
        hipError_t el = launch_vjp_lines(v, nd, c->prm.recon, c->nlines, st);
        if (el != hipSuccess) return hip_fail(c, el, "adjoint line launch");
        hipError_t e = launch_vjp_cells(v, nd, c->prm.recon, c->ncitems, st);
        if (e != hipSuccess) return hip_fail(c, e, "adjoint cell launch");
        g = gS;
    }
    return HYDRO_OK;
}

int hydro_step_vjp(hydro_ctx_t *c, const double *Un, const double *dt_dev, const double *gUnext, double *gUn)
{
    return step_vjp(c, Un, nullptr, dt_dev, gUnext, gUn);
}

int hydro_step_vjp_stages(hydro_ctx_t *c, const double *Un, const double *const *stages, const double *dt_dev,
                          const double *gUnext, double *gUn)
{
    if (!stages) return fail(c, HYDRO_EINVAL, "null pointer");
    return step_vjp(c, Un, stages, dt_dev, gUnext, gUn);
}

int hydro_status(hydro_ctx_t *c, int64_t *n_nonphys)
{
    if (!c) return HYDRO_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unsigned long long n = 0;
    HIP_TRY(c, hipMemcpy(&n, c->d_nbad, sizeof(n), hipMemcpyDeviceToHost));
    if (n) HIP_TRY(c, hipMemset(c->d_nbad, 0, sizeof(n)));
    if (n_nonphys) *n_nonphys = (int64_t)n;
    if (n) return fail(c, HYDRO_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or NaN) met " + std::to_string(n) + " times");
    return HYDRO_OK;
}

const char *hydro_last_error(hydro_ctx_t *c)
{
    if (!c) return g_noctx_err.c_str();
    return c->err.c_str();
}

int hydro_fp_check(const double *a, const double *b, const double *c, double *quot, double *root, double *fmad,
                   int64_t n, void *stream)
{
    if (n < 0) return HYDRO_EINVAL;
    if (n > 0 && (!a || !b || !c || !quot || !root || !fmad)) return HYDRO_EINVAL;
    hipError_t e = launch_fp_check(a, b, c, quot, root, fmad, n, (hipStream_t)stream);
    return e == hipSuccess ? HYDRO_OK : HYDRO_EHIP;
}

void hydro_destroy(hydro_ctx_t *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    drop_graph(c);
    (void)hipFree(c->d_blocks);
    (void)hipFree(c->d_faces);
    (void)hipFree(c->d_items);
    (void)hipFree(c->d_items_pb);
    (void)hipFree(c->d_buf[0]);
    (void)hipFree(c->d_buf[1]);
    (void)hipFree(c->d_partial);
    (void)hipFree(c->d_cflnext);
    (void)hipFree(c->d_nbad);
    (void)hipFree(c->d_vjp);
    (void)hipFree(c->d_lines);
    (void)hipFree(c->d_citems);
    (void)hipFree(c->d_xitems);
    (void)hipFree(c->d_amr);
    (void)hipFree(c->d_freg);
    (void)hipFree(c->d_afill);
    (void)hipFree(c->d_acorr);
    (void)hipFree(c->d_inc_start);
    (void)hipFree(c->d_inc);
    free_tele(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
}

}  // extern "C"
