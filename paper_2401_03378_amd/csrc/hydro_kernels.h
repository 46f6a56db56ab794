// Kernel argument blocks and launchers shared by the library's host code.
#pragma once
#include "hydro_common.h"

namespace hydro {

struct StageArgs {
    const DevBlock *blocks;
    const FaceSrc *faces;
    const WorkItem *items;
    int32_t nitems;
    int32_t stage;              // 1-based SSP-RK stage
    int64_t nc;                 // cells per variable plane
    double gamma, g1, ig1;
    double idx, idy, idz;
    double a, b;                // U_out = b T + a U^n for stage >= 2
    double eps;                 // WENO5 weight epsilon
    const double *dt;           // device scalar
    const double *Un;
    const double *Us;
    double *Uout;
    unsigned long long *nbad;
    double *freg;               // flux registers (faces with FaceSrc::reg >= 0)
    int32_t nface;              // cells per register slot and variable
    double *cfl_partial;        // non-null: per-workgroup maxima of the CFL wave-speed sum of Uout
    int32_t phys;               // kGravity | kShock, or 0
    double grav[3];             // uniform gravitational acceleration (kGravity)
    double sthresh;             // relative pressure jump of the shock detector (kShock)
};

// Coarse-fine faces: guard fill across levels and the flux correction.
struct AmrArgs {
    const DevBlock *blocks;
    const DevAmr *amr;
    const FaceSrc *faces;
    const int2 *list;           // fill: (block, face); correction: (block, -)
    int32_t nlist;
    int32_t ng;                 // guard layers (shared by all blocks of a mesh with levels)
    int32_t fchunks;            // guard fill: workgroups per face (chunks of its layer x cell items)
    int64_t nc;
    int32_t nface;
    double idx, idy, idz;
    double b;                   // stage coefficient of the correction
    const double *dt;
    const double *freg;
    double *U;                  // state whose guards are filled / stage output corrected
};

struct CflArgs {
    const DevBlock *blocks;
    const WorkItem *items;
    int32_t nitems;
    int64_t nc;
    double gamma, g1, idx, idy, idz;
    const double *U;
    double *partial;
    unsigned long long *nbad;
};

struct GuardArgs {
    const DevBlock *blocks;
    const FaceSrc *faces;
    int32_t b0;
    int64_t nc;
    double *U;
};

// Telescoping step: thick copies of the blocks (T) and the caller's layout (U).
struct TeleArgs {
    const DevBlock *tb;         // thick blocks (ng = halo width of the step)
    const FaceSrc *tf;          // per face: source of the thick halo layers
    const DevBlock *ub;         // blocks in the caller's layout
    int64_t nct, ncu;           // cells per variable plane: thick, caller
    int32_t d;                  // direction filled by this launch
    double *T;
    double *U;
};

struct VjpArgs {
    const DevBlock *blocks;
    const FaceSrc *faces;
    const WorkItem *items;      // line work items: block, first line (xy), line count (z)
    int32_t nitems;
    const WorkItem *citems;     // cell work items (16x4 tiles over runs of z planes)
    int32_t ncitems;
    int64_t nc;
    double gamma, g1, ig1;
    double idx, idy, idz;
    double a, b;
    double eps;                 // WENO5 weight epsilon
    const double *dt;
    const double *Us;           // stage input (forward state)
    const double *gOut;         // cotangent of the stage output (interior)
    double *gW;                 // padded primitive cotangents, nvar x nc
    double *gUs;                // cotangent of the stage input (interior)
    double *gUn;                // += a gOut (null: skip)
    int32_t last;               // first stage: gU_s goes straight into gUn (gUn += gU_s), gUs unused
    const int *inc_start;       // per block: range in inc
    const int4 *inc;            // guard positions copying this block: (block, dir, side, kind)
    int32_t nseg;               // requested segments per line (arrays per direction)
    const WorkItem *xitems;     // transpose tiles: block, p tile | j tile << 16, k
    int32_t nxitems;
    double *UsT;                // Us along x lines, j fastest (positions -H .. nx+H-1)
    double *gOutT;              // gOut along x lines, j fastest (interior positions)
    int32_t phys;               // kGravity | kShock, or 0 (as StageArgs)
    double grav[3];
    double sthresh;
};

hipError_t launch_stage(const StageArgs &a, int ndim, int recon, int tile, int variant, bool gather, int grid,
                        hipStream_t st);
hipError_t launch_cfl(const CflArgs &a, int ndim, int tile, int grid, double cfl, double *dt, hipStream_t st);
hipError_t launch_cfl_final(const double *partial, int n, double cfl, double *dt, hipStream_t st);
hipError_t launch_fill_guards(const GuardArgs &a, int ndim, int nblk, hipStream_t st);
hipError_t launch_tele_fill(const TeleArgs &a, int ndim, int nblk, hipStream_t st);
hipError_t launch_tele_copy(const TeleArgs &a, int ndim, int nblk, bool to_thick, hipStream_t st);
hipError_t launch_amr_fill(const AmrArgs &a, int ndim, hipStream_t st);
hipError_t launch_amr_correct(const AmrArgs &a, int ndim, hipStream_t st);
hipError_t launch_vjp_xpose(const VjpArgs &a, int ndim, int recon, hipStream_t st);
hipError_t launch_vjp_lines(const VjpArgs &a, int ndim, int recon, int nitems, hipStream_t st);
hipError_t launch_vjp_cells(const VjpArgs &a, int ndim, int recon, int grid, hipStream_t st);

}  // namespace hydro
