/*
 * CPU oracle, AMR part: the step of oracle.c on a mesh whose blocks sit on
 * refinement levels (ratio 2), with the flux correction at coarse-fine faces
 * that the paper's Sec. 4.2 describes for Flash-X's two AMR back ends: the
 * face fluxes of the coarse side of a coarse-fine face are replaced by those
 * of the fine side, either for all levels at once after all blocks are updated
 * (Paramesh, the "all levels" listing) or level by level, finest first
 * (AMReX, the "level by level" listing).  With one time step for all levels
 * both orders give the same numbers.  TEST INFRASTRUCTURE ONLY (see oracle.c).
 *
 * The paper gives the structure only; the parts it leaves open are read as:
 *  - guard cells of a fine block behind a coarse neighbour take the value of
 *    the coarse cell that contains them (piecewise-constant prolongation);
 *  - guard cells of a coarse block behind fine neighbours take the average of
 *    the 2^ndim fine cells they cover, summed pairwise (conservative
 *    restriction; exact for a uniform state);
 *  - one dt for all levels (no subcycling), the CFL bound taken over every
 *    block with its own cell widths dx / 2^level;
 *  - in every stage, after the blocks' updates, each coarse cell next to a
 *    coarse-fine face gets U += sigma * b_s * (dt * ((Fbar - Fc) / dx)),
 *    Fc the coarse flux through its face, Fbar the average of the 2^(ndim-1)
 *    fine fluxes through the same face (pairwise), sigma = +1 on the coarse
 *    block's low face and -1 on its high face; faces in order x low, x high,
 *    y low, y high, z low, z high.
 *
 * Build: with oracle.c (gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#pragma GCC diagnostic ignored "-Wunused-function"   /* parts of the shared body this file does not use */

#define REAL double
#define FN(name) ora_a_##name
#define RE(x) (x)
#define RSQRT(x) sqrt(x)
#define RFMA(a, b, c) fma((a), (b), (c))
#define RABS(x) fabs(x)
#define RCOPYSIGN(m, a) copysign((m), (a))
static inline double RMIN(double a, double b) { return (a <= b) ? a : b; }
static inline double RMAX(double a, double b) { return (a >= b) ? a : b; }
#include "forward_body.inc"

int ora_validate(const ora_problem *P);

/* The problem with every coarse-fine face turned into an outflow face, so the
 * same-level machinery (validation, guard fill) applies to the rest. */
typedef struct {
    ora_problem Q;
    ora_link *links;
} amr_base;

static int base_of(const ora_problem *P, const ora_amr *A, amr_base *out)
{
    out->links = NULL;
    if (!P || !A || (P->nblocks > 0 && !P->links)) return ORA_EINVAL;
    out->Q = *P;
    out->links = malloc(sizeof(ora_link) * (size_t)(P->nblocks > 0 ? P->nblocks : 1));
    if (!out->links) return ORA_ENOMEM;
    for (int b = 0; b < P->nblocks; b++)
        for (int f = 0; f < 6; f++) {
            int nb = P->links[b].nbr[f];
            if ((nb == ORA_LEVEL_FACE) != (f < 2 * P->ndim && A[b].kind[f] != 0)) return ORA_EINVAL;
            out->links[b].nbr[f] = (nb == ORA_LEVEL_FACE) ? -1 : nb;
        }
    out->Q.links = out->links;
    return ORA_OK;
}

/* The transverse axes of a face normal to d, in x, y, z order. */
static void axes(int d, int *o1, int *o2)
{
    *o1 = (d == 0) ? 1 : 0;
    *o2 = (d == 2) ? 1 : 2;
}

static int amr_validate(const ora_problem *P, const ora_amr *A, amr_base *base)
{
    int rc = base_of(P, A, base);
    if (rc) return rc;
    rc = ora_validate(&base->Q);
    if (rc) return rc;
    if (P->phys) return ORA_EINVAL;     /* gravity and the shock detector: meshes without levels only */
    const int nd = P->ndim;
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b], *B0 = &P->blocks[0];
        if (B->nx != B0->nx || B->ny != B0->ny || B->nz != B0->nz || B->ng != B0->ng) return ORA_EINVAL;
        for (int d = 0; d < nd; d++) {
            int n = ora_a_extent(B, d);
            if (n % 2 != 0 || n < 2 * B->ng) return ORA_EINVAL;
        }
        if (A[b].level < 0 || A[b].level > 20) return ORA_EINVAL;
    }
    for (int b = 0; b < P->nblocks; b++)
        for (int d = 0; d < nd; d++) {
            int o1, o2;
            axes(d, &o1, &o2);
            const ora_block *B = &P->blocks[b];
            int h1n = ora_a_extent(B, o1) / 2, h2n = (nd == 3) ? ora_a_extent(B, o2) / 2 : 0;
            for (int side = 0; side < 2; side++) {
                int f = 2 * d + side, opp = 2 * d + 1 - side;
                if (A[b].kind[f] == 1) {
                    int c = A[b].nbr[f][0], q1 = A[b].nbr[f][1], q2 = A[b].nbr[f][2];
                    if (c < 0 || c >= P->nblocks || A[c].level != A[b].level - 1 || A[c].kind[opp] != 2) return ORA_EINVAL;
                    if (!(q1 == 0 || q1 == h1n) || !(nd == 2 ? q2 == 0 : (q2 == 0 || q2 == h2n))) return ORA_EINVAL;
                    int h = (q1 / h1n) + 2 * ((nd == 3) ? q2 / h2n : 0);
                    if (A[c].nbr[opp][h] != b) return ORA_EINVAL;
                } else if (A[b].kind[f] == 2) {
                    int nq = (nd == 3) ? 4 : 2;
                    for (int h = 0; h < nq; h++) {
                        int fb = A[b].nbr[f][h];
                        if (fb < 0 || fb >= P->nblocks || A[fb].level != A[b].level + 1 || A[fb].kind[opp] != 1) return ORA_EINVAL;
                        if (A[fb].nbr[opp][0] != b || A[fb].nbr[opp][1] != (h % 2) * h1n ||
                            A[fb].nbr[opp][2] != (h / 2) * h2n) return ORA_EINVAL;
                    }
                } else if (A[b].kind[f] != 0) {
                    return ORA_EINVAL;
                }
            }
        }
    return ORA_OK;
}

/* Guard layers of coarse-fine faces (after the same-level fill). */
static void amr_fill(const ora_problem *Q, const ora_amr *A, double *U)
{
    const int nd = Q->ndim, nv = nd + 2;
    const int64_t nc = Q->ncell;
#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < Q->nblocks; b++) {
        const ora_block *B = &Q->blocks[b];
        for (int d = 0; d < nd; d++) {
            int o1, o2;
            axes(d, &o1, &o2);
            const int n = ora_a_extent(B, d), n1 = ora_a_extent(B, o1);
            const int n2 = (nd == 3) ? ora_a_extent(B, o2) : 1;
            for (int side = 0; side < 2; side++) {
                const int f = 2 * d + side;
                if (A[b].kind[f] == 0) continue;
                for (int l = 1; l <= B->ng; l++)
                    for (int e2 = 0; e2 < n2; e2++)
                        for (int e1 = 0; e1 < n1; e1++) {
                            int g[3];
                            g[d] = (side == 0) ? -l : n - 1 + l;
                            g[o1] = e1;
                            g[o2] = e2;
                            if (nd == 2) g[2] = 0;
                            const int64_t gi = ora_a_cell(B, nd, g[0], g[1], g[2]);
                            if (A[b].kind[f] == 1) {
                                /* coarse cell containing the guard cell */
                                const int c = A[b].nbr[f][0];
                                const ora_block *C = &Q->blocks[c];
                                const int m = ora_a_extent(C, d), half = (l + 1) / 2;
                                int s[3];
                                s[d] = (side == 0) ? m - half : half - 1;
                                s[o1] = A[b].nbr[f][1] + e1 / 2;
                                s[o2] = (nd == 3) ? A[b].nbr[f][2] + e2 / 2 : 0;
                                if (nd == 2) s[2] = 0;
                                const int64_t si = ora_a_cell(C, nd, s[0], s[1], s[2]);
                                for (int v = 0; v < nv; v++) U[v * nc + gi] = U[v * nc + si];
                            } else {
                                /* average of the fine cells the guard cell covers */
                                const int h1n = n1 / 2, h2n = (nd == 3) ? n2 / 2 : 1;
                                const int h1 = e1 / h1n, h2 = (nd == 3) ? e2 / h2n : 0;
                                const int fb = A[b].nbr[f][h1 + 2 * h2];
                                const ora_block *F = &Q->blocks[fb];
                                const int mf = ora_a_extent(F, d);
                                const int p0 = (side == 0) ? mf - 2 * l : 2 * (l - 1);
                                const int f1 = 2 * (e1 - h1 * h1n), f2 = (nd == 3) ? 2 * (e2 - h2 * h2n) : 0;
                                for (int v = 0; v < nv; v++) {
                                    double a[2][2][2];
                                    for (int i2 = 0; i2 < 2; i2++)
                                        for (int i1 = 0; i1 < 2; i1++)
                                            for (int in = 0; in < 2; in++) {
                                                int s[3];
                                                s[d] = p0 + in;
                                                s[o1] = f1 + i1;
                                                s[o2] = f2 + i2;
                                                if (nd == 2) s[2] = 0;
                                                a[i2][i1][in] = (nd == 2 && i2 == 1)
                                                    ? 0.0 : U[v * nc + ora_a_cell(F, nd, s[0], s[1], s[2])];
                                            }
                                    double val;
                                    if (nd == 3)
                                        val = (((a[0][0][0] + a[0][0][1]) + (a[0][1][0] + a[0][1][1])) +
                                               ((a[1][0][0] + a[1][0][1]) + (a[1][1][0] + a[1][1][1]))) * 0.125;
                                    else
                                        val = ((a[0][0][0] + a[0][0][1]) + (a[0][1][0] + a[0][1][1])) * 0.25;
                                    U[v * nc + gi] = val;
                                }
                            }
                        }
            }
        }
    }
}

/* The problem seen from one level: cell widths dx / 2^level. */
static ora_problem at_level(const ora_problem *Q, int level)
{
    ora_problem L = *Q;
    L.dx = ldexp(Q->dx, -level);
    L.dy = ldexp(Q->dy, -level);
    L.dz = ldexp(Q->dz, -level);
    return L;
}

static void rk_coeffs(int rk, int s, double *a, double *b)
{
    *a = 0.0;
    *b = 1.0;
    if (rk == 2 && s == 2) { *a = 0.5; *b = 0.5; }
    if (rk == 3 && s == 2) { *a = 0.75; *b = 0.25; }
    if (rk == 3 && s == 3) { *a = 1.0 / 3.0; *b = 2.0 / 3.0; }
}

/* The stage update of one block (as in the uniform-mesh stage), recording
 * the fluxes through the block's faces. */
static int64_t block_update(const ora_problem *Q, const ora_amr *A, int b, int s, double dt,
                            const double *Un, const double *Us, double *Uout, double *bflux)
{
    const int nd = Q->ndim, nv = nd + 2;
    const int64_t nc = Q->ncell;
    const ora_block *B = &Q->blocks[b];
    const ora_problem L = at_level(Q, A[b].level);
    double a, bcoef;
    rk_coeffs(Q->rk, s, &a, &bcoef);
    const int64_t nint = (int64_t)B->nx * B->ny * B->nz;
    double *acc = malloc(sizeof(double) * nv * nint);
    int64_t bad = ora_a_block_rhs(&L, b, Us, NULL, acc, bflux);
    for (int k = 0; k < B->nz; k++)
        for (int j = 0; j < B->ny; j++)
            for (int i = 0; i < B->nx; i++) {
                const int64_t li = ((int64_t)k * B->ny + j) * B->nx + i;
                const int64_t ci = ora_a_cell(B, nd, i, j, k);
                for (int v = 0; v < nv; v++) {
                    const double Lv = -acc[v * nint + li];
                    const double T = fma(dt, Lv, Us[v * nc + ci]);
                    Uout[v * nc + ci] = (s == 1) ? T : fma(bcoef, T, a * Un[v * nc + ci]);
                }
            }
    free(acc);
    return bad;
}

/* Flux correction of the coarse cells next to the coarse-fine faces of block b. */
static void block_correct(const ora_problem *Q, const ora_amr *A, int b, int s, double dt,
                          const double *bflux, int64_t nface, double *Uout)
{
    const int nd = Q->ndim, nv = nd + 2;
    const int64_t nc = Q->ncell;
    const ora_block *B = &Q->blocks[b];
    const ora_problem L = at_level(Q, A[b].level);
    const double id[3] = {1.0 / L.dx, 1.0 / L.dy, 1.0 / L.dz};
    const int64_t rec = (int64_t)2 * nd * nface * 5;      /* face-flux record of one block */
    double a, bcoef;
    rk_coeffs(Q->rk, s, &a, &bcoef);
    (void)a;
    for (int d = 0; d < nd; d++) {
        int o1, o2;
        axes(d, &o1, &o2);
        const int n = ora_a_extent(B, d), n1 = ora_a_extent(B, o1);
        const int n2 = (nd == 3) ? ora_a_extent(B, o2) : 1;
        const int h1n = n1 / 2, h2n = (nd == 3) ? n2 / 2 : 1;
        for (int side = 0; side < 2; side++) {
            const int f = 2 * d + side;
            if (A[b].kind[f] != 2) continue;
            const int ff = 2 * d + 1 - side;                  /* the fine blocks' face */
            for (int e2 = 0; e2 < n2; e2++)
                for (int e1 = 0; e1 < n1; e1++) {
                    const int h1 = e1 / h1n, h2 = (nd == 3) ? e2 / h2n : 0;
                    const int fb = A[b].nbr[f][h1 + 2 * h2];
                    const int f1 = 2 * (e1 - h1 * h1n), f2 = (nd == 3) ? 2 * (e2 - h2 * h2n) : 0;
                    const double *Fc = &bflux[b * rec + ((int64_t)f * nface + (int64_t)e2 * n1 + e1) * 5];
                    int pos[3];
                    pos[d] = (side == 0) ? 0 : n - 1;
                    pos[o1] = e1;
                    pos[o2] = e2;
                    if (nd == 2) pos[2] = 0;
                    const int64_t ci = ora_a_cell(B, nd, pos[0], pos[1], pos[2]);
                    for (int v = 0; v < nv; v++) {
#define FFINE(i1, i2) bflux[fb * rec + ((int64_t)ff * nface + (int64_t)(f2 + (i2)) * n1 + (f1 + (i1))) * 5 + v]
                        double Fbar;
                        if (nd == 3)
                            Fbar = ((FFINE(0, 0) + FFINE(1, 0)) + (FFINE(0, 1) + FFINE(1, 1))) * 0.25;
                        else
                            Fbar = (FFINE(0, 0) + FFINE(1, 0)) * 0.5;
#undef FFINE
                        const double corr = bcoef * (dt * ((Fbar - Fc[v]) * id[d]));
                        Uout[v * nc + ci] = (side == 0) ? Uout[v * nc + ci] + corr : Uout[v * nc + ci] - corr;
                    }
                }
        }
    }
}

/* One stage on the AMR mesh.  order: 0 all levels at once, 1 level by level
 * (finest first), 2 all levels without the flux correction (a check only). */
static int64_t amr_stage(const ora_problem *Q, const ora_amr *A, int s, double dt, const double *Un,
                         double *Us, double *Uout, int order, double *bflux, int64_t nface)
{
    const int nd = Q->ndim;
    const int64_t rec = (int64_t)2 * nd * nface * 5;
    ora_a_fill_guards(Q, Us);
    amr_fill(Q, A, Us);
    int maxlev = 0;
    for (int b = 0; b < Q->nblocks; b++) maxlev = A[b].level > maxlev ? A[b].level : maxlev;
    int64_t bad = 0;
    if (order == 1) {
        for (int lev = maxlev; lev >= 0; lev--) {
#pragma omp parallel for schedule(dynamic) reduction(+ : bad)
            for (int b = 0; b < Q->nblocks; b++)
                if (A[b].level == lev) bad += block_update(Q, A, b, s, dt, Un, Us, Uout, &bflux[b * rec]);
#pragma omp parallel for schedule(dynamic)
            for (int b = 0; b < Q->nblocks; b++)
                if (A[b].level == lev) block_correct(Q, A, b, s, dt, bflux, nface, Uout);
        }
    } else {
#pragma omp parallel for schedule(dynamic) reduction(+ : bad)
        for (int b = 0; b < Q->nblocks; b++) bad += block_update(Q, A, b, s, dt, Un, Us, Uout, &bflux[b * rec]);
        if (order == 0) {
#pragma omp parallel for schedule(dynamic)
            for (int b = 0; b < Q->nblocks; b++) block_correct(Q, A, b, s, dt, bflux, nface, Uout);
        }
    }
    return bad;
}

int ora_amr_validate(const ora_problem *P, const ora_amr *A)
{
    amr_base base;
    int rc = amr_validate(P, A, &base);
    free(base.links);
    return rc;
}

int ora_amr_fill_guards(const ora_problem *P, const ora_amr *A, double *U)
{
    amr_base base;
    int rc = amr_validate(P, A, &base);
    if (!rc) {
        ora_a_fill_guards(&base.Q, U);
        amr_fill(&base.Q, A, U);
    }
    free(base.links);
    return rc;
}

/* CFL time step over all levels: dt = cfl / max over interior cells of
 * sum_d (|u_d| + c) / dx_d with each block's own cell widths. */
int ora_amr_cfl_dt(const ora_problem *P, const ora_amr *A, const double *U, double *dt)
{
    amr_base base;
    int rc = amr_validate(P, A, &base);
    free(base.links);
    if (rc) return rc;
    const int nd = P->ndim, nv = nd + 2;
    const int64_t nc = P->ncell;
    double smax = 0.0;
    int64_t bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(max : smax) reduction(+ : bad)
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        const ora_problem L = at_level(P, A[b].level);
        const double idx = 1.0 / L.dx, idy = 1.0 / L.dy, idz = 1.0 / L.dz;
        for (int k = 0; k < B->nz; k++)
            for (int j = 0; j < B->ny; j++)
                for (int i = 0; i < B->nx; i++) {
                    const int64_t ci = ora_a_cell(B, nd, i, j, k);
                    double Uc[5], W[5];
                    for (int v = 0; v < nv; v++) Uc[v] = U[v * nc + ci];
                    bad += ora_a_eos(P, Uc, W);
                    const double r = 1.0 / Uc[0];
                    const double c = sqrt((P->gamma * W[4]) * r);
                    double sig;
                    if (nd == 3)
                        sig = (((fabs(W[1]) + c) * idx) + ((fabs(W[2]) + c) * idy)) + ((fabs(W[3]) + c) * idz);
                    else
                        sig = ((fabs(W[1]) + c) * idx) + ((fabs(W[2]) + c) * idy);
                    if (sig > smax) smax = sig;
                }
    }
    if (bad) return ORA_ENONPHYS;
    *dt = P->cfl / smax;
    return ORA_OK;
}

/* One step in place on U.  compute_dt: *dt receives the CFL step of U;
 * otherwise *dt is used.  order as for amr_stage. */
int ora_amr_step(const ora_problem *P, const ora_amr *A, double *U, double *dt, int compute_dt, int order)
{
    if (order < 0 || order > 2) return ORA_EINVAL;
    amr_base base;
    int rc = amr_validate(P, A, &base);
    if (rc) { free(base.links); return rc; }
    if (compute_dt) {
        rc = ora_amr_cfl_dt(P, A, U, dt);
        if (rc) { free(base.links); return rc; }
    }
    if (!(*dt > 0.0)) { free(base.links); return ORA_EINVAL; }
    const ora_problem *Q = &base.Q;
    const int64_t nface = (P->nblocks > 0) ? ora_a_nface(&P->blocks[0], P->ndim) : 1;
    size_t bytes = sizeof(double) * (size_t)(P->ndim + 2) * (size_t)P->ncell;
    double *Us = malloc(bytes), *Uo = malloc(bytes);
    double *bflux = malloc(sizeof(double) * (size_t)(P->nblocks > 0 ? P->nblocks : 1) * 2 * P->ndim * nface * 5);
    if (!Us || !Uo || !bflux) { free(Us); free(Uo); free(bflux); free(base.links); return ORA_ENOMEM; }
    memcpy(Us, U, bytes);
    memcpy(Uo, U, bytes);
    int64_t bad = 0;
    for (int s = 1; s <= P->rk && !bad; s++) {
        bad += amr_stage(Q, A, s, *dt, U, Us, Uo, order, bflux, nface);
        double *t = Us; Us = Uo; Uo = t;
    }
    if (!bad) memcpy(U, Us, bytes);
    free(Us); free(Uo); free(bflux); free(base.links);
    return bad ? ORA_ENONPHYS : ORA_OK;
}
