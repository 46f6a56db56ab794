/*
 * CPU oracle for the block-structured compressible-Euler step -- TEST
 * INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, constant or helper with the GPU path.
 *
 * The oracle is a plain, slow, obviously-correct FP64 transcription of the
 * method: the non-telescoping SSP-RK step of the paper's Sec. 4.2 ("Variants
 * for Flash-X hydrodynamics simulations", the traditional RK listing: per
 * stage fill the guard cells, then for every block run the intra-stage
 * calculations), with the intra-stage dependency chain of the paper's
 * Algorithm "Intra stage calculations for Spark" (calcLims -> calcFlux ->
 * updSoln -> calcEos).  The paper names those steps but does not give their
 * formulas; the formulas follow the textbook methods they stand for:
 * ideal-gas EOS, MC-limited PLM (van Leer 1977), WENO5-JS (Jiang & Shu 1996),
 * HLLC with Davis wave speeds (Toro 2009, Sec. 10.4-10.5), Shu-Osher SSP-RK2/3
 * (Gottlieb & Shu 1998).
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

typedef struct {            /* one block: interior extents, guard width, offset */
    int32_t nx, ny, nz, ng;
    int64_t offset;         /* first padded cell within one variable plane */
} ora_block;

typedef struct { int32_t nbr[6]; } ora_link;   /* -x,+x,-y,+y,-z,+z; >=0 block, -1 outflow, -2 periodic self */

typedef struct {
    int32_t ndim;           /* 2 or 3 */
    int32_t recon;          /* 0 PLM-MC, 1 WENO5-JS */
    int32_t rk;             /* 2 or 3 stages */
    int32_t nblocks;
    int64_t ncell;          /* cells per variable plane (padding included) */
    double gamma, cfl, dx, dy, dz;
    const ora_block *blocks;
    const ora_link *links;
    double weno_eps;        /* epsilon of the WENO5 weights (Jiang & Shu: 1e-6) */
    double grav[3];         /* uniform gravitational acceleration (ORA_GRAVITY; z ignored in 2D) */
    double shock_thresh;    /* relative pressure jump of the shock detector (ORA_SHOCK), >= 0 */
    int32_t phys;           /* ORA_GRAVITY | ORA_SHOCK, or 0 */
} ora_problem;

/* Optional parts of the intra-stage chain and the block initialisation
 * (the grvAccel and shockDet nodes of the paper's Algorithms "Intra stage
 * calculations for Spark" and "Block initializations for Spark"). */
#define ORA_GRAVITY 1
#define ORA_SHOCK 2

/* Two-level-ratio block AMR (refinement ratio 2, levels differ by at most
 * one across a face).  A face whose link is ORA_LEVEL_FACE touches blocks of
 * another level: kind 1, one coarser block, of whose face this block's face
 * covers the part starting at coarse cells (o1, o2) along the face's two
 * transverse axes (x, y, z order); kind 2, the 2^(ndim-1) finer blocks that
 * cover the face, listed as nbr[face][h1 + 2 h2] by transverse half.  All
 * blocks of an AMR problem share nx, ny, nz and ng. */
#define ORA_LEVEL_FACE (-3)
typedef struct {
    int32_t level;          /* 0 = coarsest; cell widths dx / 2^level */
    int32_t kind[6];        /* 0 as the link says, 1 coarser neighbour, 2 finer neighbours */
    int32_t nbr[6][4];      /* kind 1: {coarse block, o1, o2, -1}; kind 2: fine blocks by half */
} ora_amr;

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ENONPHYS (-3)
#define ORA_ENOMEM (-4)

#endif
