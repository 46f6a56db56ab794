/*
 * hydro.h -- C ABI of the MI355X (gfx950) FP64 block-structured
 * compressible-Euler step.
 *
 * What it computes.  One explicit time step of the unsplit finite-volume
 * method for the Euler equations of an ideal gas, on a table of blocks each
 * surrounded by guard cells (the paper's block-structured mesh, Sec. 2.2
 * "Flash-X").  The step is the non-telescoping SSP-RK loop of the paper's
 * Sec. 4.2 (the "traditional" listing: per stage, fill guard cells, then for
 * every block do the intra-stage calculations), with the intra-stage chain of
 * the paper's Algorithm "Intra stage calculations for Spark": reconstruction
 * (calcLims), Riemann fluxes (calcFlux), solution update (updSoln) and EOS
 * (calcEos).  The paper names these steps only; the formulas are the textbook
 * methods they stand for: ideal-gas EOS; MC-limited piecewise-linear
 * (van Leer 1977) or WENO5-JS (Jiang & Shu 1996) reconstruction of primitive
 * variables; HLLC fluxes with Davis wave speeds (Toro 2009, Sec. 10.4);
 * Shu-Osher SSP-RK2/RK3 (Gottlieb & Shu 1998); CFL time step from the
 * unsplit wave-speed sum.
 *
 * Data layout (all state arrays).  One float64 array of nvar x ncell_total,
 * variable-major (v * ncell_total + cell), nvar = ndim + 2, variables
 * (rho, m_x, m_y[, m_z], E).  Block b owns the padded cells
 * [offset, offset + (nx+2ng)(ny+2ng)(nz+2ng)) of every variable plane, x
 * fastest; in 2D nz = 1 and there is no z padding.  Only interior cells are
 * results; guard, edge and corner cells of the caller's arrays are never
 * read by the step kernels (guards are gathered from their source cells).
 *
 * Ownership.  Arrays passed to the ctx functions are DEVICE pointers on the
 * ctx's device, owned by the caller, and must stay valid until the work
 * enqueued on the ctx's stream completes.  Descriptor tables passed to
 * hydro_create / hydro_validate are HOST pointers, copied.  The ctx owns its
 * device tables, stage buffers, partial-reduction buffers and graphs.  A ctx
 * is bound to one stream and is not thread-safe.
 *
 * Errors.  Every int-returning function returns HYDRO_OK or a negative code;
 * hydro_last_error(ctx) gives text.  Kernel-detected non-physical states
 * (rho <= 0, p <= 0, NaN) are counted on the device and reported by
 * hydro_status (HYDRO_ENONPHYS); no floors are applied.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRO_OK 0
#define HYDRO_EINVAL (-1)     /* bad argument, descriptor table or dt <= 0  */
#define HYDRO_EHIP (-2)       /* HIP runtime error (text in hydro_last_error) */
#define HYDRO_ENONPHYS (-3)   /* non-physical state met by a kernel         */
#define HYDRO_ENOMEM (-4)     /* device allocation failed                   */

#define HYDRO_PLM_MC 0
#define HYDRO_WENO5 1

#define HYDRO_OUTFLOW (-1)        /* zero-gradient copy of the nearest interior cell */
#define HYDRO_PERIODIC_SELF (-2)  /* periodic wrap onto the block itself */
#define HYDRO_LEVEL_FACE (-3)     /* face to another refinement level (hydro_amr_t) */

/* One block: interior extents, guard width, first padded cell (per plane). */
typedef struct {
    int32_t nx, ny, nz, ng;
    int64_t offset;
} hydro_block_t;

/* Face links in order (-x, +x, -y, +y, -z, +z): >= 0 neighbour block index,
 * HYDRO_OUTFLOW or HYDRO_PERIODIC_SELF.  Neighbours must match in the
 * transverse extents and in ng, and be at least ng cells deep. */
typedef struct {
    int32_t nbr[6];
} hydro_link_t;

typedef struct {
    int32_t ndim;     /* 2 or 3 */
    int32_t recon;    /* HYDRO_PLM_MC (needs ng >= 2) or HYDRO_WENO5 (ng >= 3) */
    int32_t rk;       /* 2 or 3 SSP-RK stages */
    int32_t flags;    /* 0 or an OR of HYDRO_FLAG_LEVEL_BY_LEVEL (AMR context),
                         HYDRO_FLAG_GRAVITY, HYDRO_FLAG_SHOCK_DETECT */
    double gamma;     /* ratio of specific heats, > 1 */
    double cfl;       /* Courant number of the unsplit sum, > 0 */
    double dx, dy, dz;  /* cell widths (dz ignored in 2D but must be > 0) */
    double weno_eps;  /* epsilon of the WENO5 nonlinear weights alpha_k = d_k/(eps+beta_k)^2,
                         finite and > 0 (Jiang & Shu 1996 use 1e-6); ignored by PLM-MC */
    double grav[3];   /* HYDRO_FLAG_GRAVITY: uniform gravitational acceleration (finite;
                         grav[2] unused in 2D) */
    double shock_thresh;  /* HYDRO_FLAG_SHOCK_DETECT: relative pressure jump, finite and >= 0 */
} hydro_params_t;

/* Gravity (the grvAccel node that heads the paper's Algorithm "Intra stage
 * calculations for Spark"; the paper gives no field).  The acceleration is
 * the uniform vector grav, and its source enters the update of every stage
 * from the stage input's own cell values: L(U_s) gains rho g_d in momentum d
 * and (m_x g_x + m_y g_y) + m_z g_z in energy (2D: m_x g_x + m_y g_y), as
 * L_v = S_v - (flux differences)_v for v >= 1.  The CFL dt is unchanged.
 *
 * Shock detector (the shockDet node of the paper's Algorithm "Block
 * initializations for Spark", which the non-telescoping RK listing of Sec.
 * 4.2 runs per stage before the intra-stage chain; no formula in the paper).
 * From the stage input's primitives, a cell is flagged along direction d
 * when u_d(next) - u_d(previous) < 0 (compression along d) and
 * |p(next) - p(previous)| > shock_thresh * min(p(previous), p(next)); a
 * flagged cell reconstructs at first order along d (both faces take its own
 * primitives, as the positivity fallback does).  Per direction, because the
 * cells just outside a block face would need edge cells for a divergence.
 *
 * Both apply to meshes without levels in the persistent, per-block and
 * materialised modes, and to hydro_step_vjp / hydro_step_vjp_stages.
 * Gravity also applies in HYDRO_MODE_TELESCOPING; the detector does not
 * (that listing runs the block initialisation once per step), and
 * hydro_set_tuning refuses the telescoping mode for it; hydro_create_amr
 * refuses either flag.  Stages with either flag run the plain schedule
 * whatever hydro_tuning_t.variant says. */
#define HYDRO_FLAG_GRAVITY 2
#define HYDRO_FLAG_SHOCK_DETECT 4

/* Refinement levels (hydro_create_amr).  Flash-X's block-structured AMR
 * (the paper's Sec. 2.2 mesh and Sec. 4.2 flux-correction listings) with
 * refinement ratio 2 and levels that differ by at most one across a face.
 * Per block: its level (cell widths dx / 2^level) and, for every face whose
 * link is HYDRO_LEVEL_FACE, what lies behind it:
 *   kind 1: one coarser block; nbr = {block, o1, o2, -1}, where this face
 *           starts on the coarse block's face at coarse cell (o1, o2) along the
 *           face's two transverse axes in x, y, z order (o = 0 or half the
 *           transverse extent; o2 = 0 in 2D);
 *   kind 2: the 2^(ndim-1) finer blocks covering the face, nbr[h1 + 2 h2] the
 *           one over transverse half (h1, h2).
 * All blocks of an AMR problem share nx, ny, nz and ng; every extent is even
 * and at least 2 ng.  Guard cells behind a coarser face take the coarse cell
 * that contains them; behind finer faces, the pairwise sum of the 2^ndim
 * fine cells they cover times 2^-ndim (normal pair, then first, then second
 * transverse axis).  One dt for all levels.  After every stage each coarse
 * cell next to a finer face is corrected by sigma b_s (dt ((Fbar - Fc)/dx)):
 * Fc its own flux through the face, Fbar the fine fluxes through it averaged
 * in pairs, sigma = +1 on a low face and -1 on a high one, faces in the order
 * -x, +x, -y, +y, -z, +z.  HYDRO_FLAG_LEVEL_BY_LEVEL runs the levels finest
 * first with their corrections in between (the paper's level-by-level
 * listing) instead of all blocks, then all corrections (all-levels listing);
 * both give the same result bit for bit. */
#define HYDRO_FLAG_LEVEL_BY_LEVEL 1
typedef struct {
    int32_t level;
    int32_t kind[6];      /* 0: the link says; 1: coarser block; 2: finer blocks */
    int32_t nbr[6][4];
} hydro_amr_t;

/* Launch configuration of the stage kernels (chosen by an autotuner). */
#define HYDRO_MODE_PERSISTENT 0  /* one launch per stage over all blocks; guards gathered on load */
#define HYDRO_MODE_PERBLOCK 1    /* per block: guard-fill launch + stage launch */
#define HYDRO_MODE_TELESCOPING 2 /* one thick guard fill per step, stages on the extended blocks */
#define HYDRO_MODE_MATERIALISED 3 /* one guard-fill launch over all blocks + one stage launch */
/* In the per-block and materialised modes a stage first writes the guard
 * cells of its input state (the paper's per-stage fill), so hydro_step and
 * hydro_rk_stage then write the guard cells of U and Us; the interiors they
 * produce are the same bit for bit in every mode. */
typedef struct {
    int32_t mode;       /* HYDRO_MODE_* */
    int32_t tile;       /* xy tile of a work item: 0 = 8x8, 1 = 16x8, 2 = 16x16 */
    int32_t grid;       /* workgroups of a persistent launch; 0 = one per work item */
    int32_t zchunk;     /* z planes per work item; 0 = the whole block */
    int32_t use_graph;  /* replay hydro_step from a captured hipGraph */
    int32_t xcd;        /* 0: list order; 1: a block's work items on one XCD (L2), blocks
                           dealt round-robin; 2: the same with contiguous ranges of
                           block indices per XCD (neighbours share an L2) */
    int32_t variant;    /* stage schedule: 0 plain, 1 loads of the next plane issued a plane ahead
                           (meshes with levels always run the plain schedule) */
} hydro_tuning_t;

typedef struct hydro_ctx hydro_ctx_t;

/* Host-only check of a problem description (no GPU use).  Returns HYDRO_OK
 * or HYDRO_EINVAL: null pointer, ndim/recon/rk out of range, gamma <= 1,
 * cfl or dx <= 0, weno_eps not finite and > 0, extents outside 1..32767, ng
 * below the stencil's need, 2D block with nz != 1, 3D block whose padded xy
 * plane (nx+2ng)(ny+2ng) holds 2^31 cells or more, offsets out of range or
 * overlapping, link index out of range, neighbour faces that do not match. */
int hydro_validate(const hydro_params_t *params, const hydro_block_t *blocks,
                   const hydro_link_t *links, int32_t nblocks, int64_t ncell_total);

/* Create a context on the current HIP device for the given problem; work is
 * enqueued on `stream` (a hipStream_t; NULL = default stream).  Validates as
 * hydro_validate, uploads the tables, allocates stage buffers and picks a
 * default tuning.  *out receives the context (NULL on error).  A problem with
 * no blocks is valid: hydro_step, hydro_rk_stage, hydro_fill_guards and
 * hydro_step_vjp then enqueue nothing and leave their arrays untouched, and
 * hydro_cfl_dt returns HYDRO_EINVAL (no cell bounds the step). */
int hydro_create(const hydro_params_t *params, const hydro_block_t *blocks,
                 const hydro_link_t *links, int32_t nblocks, int64_t ncell_total,
                 void *stream, hydro_ctx_t **out);

/* hydro_validate / hydro_create for a mesh with refinement levels (amr: one
 * entry per block, HOST pointer, copied; see hydro_amr_t).  In an AMR context
 * the guard layers of faces to another level are materialised in the state
 * array of each stage input (hydro_step, hydro_rk_stage and
 * hydro_fill_guards write them into the caller's array too), only the
 * persistent launch mode is accepted by hydro_set_tuning, and
 * hydro_step_vjp returns HYDRO_EINVAL. */
int hydro_validate_amr(const hydro_params_t *params, const hydro_block_t *blocks,
                       const hydro_link_t *links, const hydro_amr_t *amr, int32_t nblocks,
                       int64_t ncell_total);
int hydro_create_amr(const hydro_params_t *params, const hydro_block_t *blocks,
                     const hydro_link_t *links, const hydro_amr_t *amr, int32_t nblocks,
                     int64_t ncell_total, void *stream, hydro_ctx_t **out);

/* Replace / read the launch configuration.  Invalidates captured graphs.
 * HYDRO_EINVAL for a mode other than the four HYDRO_MODE_* values or a field
 * out of range.  HYDRO_MODE_PERSISTENT, _PERBLOCK and _MATERIALISED give the
 * same interiors bit for bit (the latter two write guard cells, see above).
 * HYDRO_MODE_TELESCOPING is the paper's telescoping RK variant (Sec. 4.2,
 * second RK listing): per step one guard fill into thick block copies with
 * S*(R+1) layers (R = 1 PLM, 2 WENO5; edges and corners included), then all
 * stages update the blocks together with the halo later stages read.  It
 * equals the per-stage-fill step bit for bit on domains without outflow
 * faces and differs at outflow faces.  It needs every neighbour / periodic
 * source block to be at least S*(R+1) cells deep (else HYDRO_EINVAL); in it,
 * hydro_rk_stage and hydro_step_vjp return HYDRO_EINVAL. */
int hydro_set_tuning(hydro_ctx_t *ctx, const hydro_tuning_t *tuning);
int hydro_get_tuning(hydro_ctx_t *ctx, hydro_tuning_t *tuning);

/* Fill the ng face guard layers of every block of U in place (neighbour
 * interior, periodic wrap or outflow copy; edges and corners untouched). */
int hydro_fill_guards(hydro_ctx_t *ctx, double *U);

/* CFL time step dt = cfl / max over interior cells of
 * sum_d (|u_d| + c) / dx_d (the unsplit wave-speed sum of every direction,
 * sound speed c = sqrt(gamma p / rho)), computed from U; written to dt_dev
 * (one device double).  The paper gives no time-step rule; this is the
 * usual CFL bound of an explicit unsplit finite-volume step, taken once per
 * step of Sec. 4.2's RK loop, before its stages.  Asynchronous. */
int hydro_cfl_dt(hydro_ctx_t *ctx, const double *U, double *dt_dev);

/* One SSP-RK stage s (1-based), the body of the stage loop of the paper's
 * non-telescoping RK listing (Sec. 4.2): fill guard cells, then for every
 * block the intra-stage chain of Algorithm "Intra stage calculations for
 * Spark" (calcEos, calcLims, calcFlux, updSoln), here L(Us) = minus the flux
 * differences of HLLC fluxes between reconstructed face states, combined as
 * T = Us + dt L(Us);  Uout = T for s = 1,
 * else Uout = b_s T + a_s Un with (a,b) = (1/2,1/2) [RK2], (3/4,1/4) and
 * (1/3,2/3) [RK3].  Reads the interiors of Un and Us (guards are gathered
 * from their sources; in the per-block and materialised modes they are
 * first written into Us's guard cells), writes the interior of Uout.  Uout
 * may alias Un, not Us.  dt is read from dt_dev on the device. */
int hydro_rk_stage(hydro_ctx_t *ctx, int32_t stage, const double *dt_dev,
                   const double *Un, const double *Us, double *Uout);

/* One full step in place on U: the non-telescoping SSP-RK step of the
 * paper's Sec. 4.2 (per stage: guard fill, then every block's intra-stage
 * chain of Algorithm "Intra stage calculations for Spark"), preceded by the
 * CFL time step.  If compute_dt != 0 the CFL dt of U is first written to
 * dt_dev; otherwise the value already in dt_dev is used.
 * compute_dt = HYDRO_DT_RECORD (3) computes the CFL dt from U as 1 does, and
 * the final stage also records the CFL maxima of the state it writes;
 * compute_dt = HYDRO_DT_FROM_PREVIOUS (2) then gives the next step of the
 * same state the same dt, bit for bit, from those maxima instead of reading
 * U again, and records again.  The ctx recognises "the same state" by its
 * address only, so the caller must pass HYDRO_DT_FROM_PREVIOUS only for the
 * very allocation the previous recording step wrote, not freed since, and
 * must not have written its interior by other means than this library (the
 * ctx itself forgets the maxima on hydro_rk_stage, hydro_set_tuning, any
 * other hydro_step call or a different U, and then acts as with
 * HYDRO_DT_RECORD).  Both apply to HYDRO_MODE_PERSISTENT on meshes without
 * levels; elsewhere they act as 1.  With use_graph, the step is captured into
 * a hipGraph bound to (U, dt_dev, dt mode) once the same arguments arrive in
 * two consecutive calls, and replayed while they stay the same; other calls
 * launch the kernels directly.  Either way the result is the same bit for
 * bit. */
#define HYDRO_DT_FROM_PREVIOUS 2
#define HYDRO_DT_RECORD 3
int hydro_step(hydro_ctx_t *ctx, double *U, double *dt_dev, int32_t compute_dt);

/* Vector-Jacobian product of one step with dt held fixed (the branch
 * decisions of limiters, fallback and Riemann solver are those of the forward
 * step at Un): gUn = (dU^{n+1}/dU^n)^T gUnext over interior cells; the
 * padding of gUn is set to 0.  gUn must alias neither gUnext nor Un
 * (HYDRO_EINVAL: gUn is cleared before Un is read).  It recomputes the
 * stage inputs from Un (no tape), is asynchronous, and is deterministic (no
 * atomics; linear in gUnext bit for bit).  It equals the exact transpose up
 * to rounding (summation order and reciprocal-based quotients in the
 * derivative arithmetic; relative error near 1e-15 per field), not bit for
 * bit.  The first call allocates the
 * ctx's adjoint scratch, (ndim x line segments + 3) x nvar x ncell_total
 * doubles, kept until hydro_destroy (HYDRO_ENOMEM if it cannot). */
int hydro_step_vjp(hydro_ctx_t *ctx, const double *Un, const double *dt_dev,
                   const double *gUnext, double *gUn);

/* hydro_step_vjp with the stage inputs of the step supplied instead of
 * recomputed (the stages of the Sec. 4.2 step, reversed one by one).
 * stages is a host array of S-1 device pointers (S = params.rk):
 * stages[s-2] holds U_s, the output of hydro_rk_stage stage s-1 for this Un
 * and dt_dev (interiors are read; guard values are
 * gathered from their sources, as in the step).  The caller owns the buffers
 * and keeps them alive until the enqueued work completes.  For a caller that
 * has just run the step stage by stage (a checkpointed rollout recomputing a
 * segment) it saves the S-1 stage launches; with those stage inputs the
 * result is bit for bit that of hydro_step_vjp.  HYDRO_EINVAL if stages or
 * one of its pointers is null or gUn aliases gUnext, Un or a stage input. */
int hydro_step_vjp_stages(hydro_ctx_t *ctx, const double *Un, const double *const *stages,
                          const double *dt_dev, const double *gUnext, double *gUn);

/* The CFL time step of hydro_cfl_dt, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, harnesses
 * that forbid hipMalloc): no context and no allocation of any kind.  Its
 * scratch, one double per block, is a fixed array inside the library
 * (HYDRO_NOALLOC_MAX_BLOCKS doubles, 512 KiB, held on each GPU the library
 * runs on until the process ends).
 *   params      HOST pointer; ndim, gamma, cfl, dx, dy, dz are used and checked
 *               as in hydro_validate (recon, rk, flags, weno_eps are ignored).
 *   blocks_dev  DEVICE pointer to nblocks hydro_block_t entries, laid out as the host table's
 *               are, 1 <= nblocks <= HYDRO_NOALLOC_MAX_BLOCKS; read only.
 *   U           DEVICE state of nvar x ncell_total doubles (the layout above);
 *               interiors are read.
 *   dt_dev      DEVICE double that receives dt.
 *   stream      hipStream_t (NULL: the default stream); asynchronous.
 * On valid blocks and physical states dt equals hydro_cfl_dt's for the same
 * problem bit for bit.  A block whose descriptor the kernel finds out of
 * range (extents outside 1..32767, ng outside 0..32767, 2D nz != 1,
 * offset < 0 or its padded cells beyond ncell_total; none of its cells is
 * then read) or a non-physical cell
 * (rho <= 0, p <= 0, NaN) makes dt NaN: with no context, that is the report.
 * Returns HYDRO_EINVAL for a null pointer, bad params, nblocks out of range
 * or ncell_total < 1 (text in hydro_last_error(NULL)), HYDRO_EHIP if the
 * scratch cannot be resolved or a launch fails.  Every call on one GPU
 * shares the scratch, which keeps the last call's contents: calls that
 * overlap on one GPU (other streams or threads) race and must be ordered by
 * the caller.  Each call writes the entries it reads, so none need
 * clearing. */
#define HYDRO_NOALLOC_MAX_BLOCKS 65536
int hydro_cfl_dt_noalloc(const hydro_params_t *params, const hydro_block_t *blocks_dev, int32_t nblocks,
                         int64_t ncell_total, const double *U, double *dt_dev, void *stream);

/* Wait for the ctx's stream; *n_nonphys (may be NULL) receives the number of
 * non-physical events counted since the last call, then the count is reset.
 * Returns HYDRO_ENONPHYS if that number is non-zero. */
int hydro_status(hydro_ctx_t *ctx, int64_t *n_nonphys);

/* Text of the last error on this ctx (valid until the next call on it);
 * with ctx NULL, of the last failed call without a context on this thread
 * (hydro_create, hydro_create_amr, hydro_cfl_dt_noalloc). */
const char *hydro_last_error(hydro_ctx_t *ctx);

/* Wait for the ctx's stream, then release the ctx and all device memory it
 * owns.  NULL is ignored. */
void hydro_destroy(hydro_ctx_t *ctx);

/* Arithmetic check of the device.  The step's results are reproducible bit
 * for bit on any host only if the device's binary64 division, square root
 * and fused multiply-add round correctly (to nearest, ties to even, with
 * subnormals kept), as the step kernels use them.  For i < n this computes,
 * with the kernels' compiler settings, quot[i] = a[i] / b[i],
 * root[i] = sqrt(a[i]) and fmad[i] = fma(a[i], b[i], c[i]); all six are
 * DEVICE pointers of n doubles on the current device, owned by the caller.
 * Enqueued on `stream` (a hipStream_t; NULL: the default stream) and
 * asynchronous.  Returns HYDRO_EINVAL for n < 0 or a null pointer with
 * n > 0, HYDRO_EHIP if the launch fails. */
int hydro_fp_check(const double *a, const double *b, const double *c, double *quot, double *root,
                   double *fmad, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HYDRO_H */
