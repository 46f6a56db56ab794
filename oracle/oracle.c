/*
 * CPU oracle, double precision: forward step, CFL time step, and the
 * hand-written adjoint (vector-Jacobian product) of a step with the time step
 * held fixed.  TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke
 * check and the benchmark's CPU-baseline leg; never by the product path.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define REAL double
#define FN(name) ora_r_##name
#define RE(x) (x)
#define RSQRT(x) sqrt(x)
#define RFMA(a, b, c) fma((a), (b), (c))
#define RABS(x) fabs(x)
#define RCOPYSIGN(m, a) copysign((m), (a))
static inline double RMIN(double a, double b) { return (a <= b) ? a : b; }
static inline double RMAX(double a, double b) { return (a >= b) ? a : b; }
#include "forward_body.inc"

/* ------------------------------------------------------------ validation */

static int validate(const ora_problem *P)
{
    if (!P || !P->blocks || !P->links) return ORA_EINVAL;
    if (P->ndim != 2 && P->ndim != 3) return ORA_EINVAL;
    if (P->recon != 0 && P->recon != 1) return ORA_EINVAL;
    if (P->rk != 2 && P->rk != 3) return ORA_EINVAL;
    if (P->nblocks < 0 || P->ncell < 0) return ORA_EINVAL;
    if (!(P->gamma > 1.0) || !(P->cfl > 0.0) || !(P->dx > 0.0) || !(P->dy > 0.0) || !(P->dz > 0.0))
        return ORA_EINVAL;
    if (!(P->weno_eps > 0.0) || !isfinite(P->weno_eps)) return ORA_EINVAL;
    if (P->phys & ~(ORA_GRAVITY | ORA_SHOCK)) return ORA_EINVAL;
    if ((P->phys & ORA_GRAVITY) &&
        !(isfinite(P->grav[0]) && isfinite(P->grav[1]) && isfinite(P->grav[2])))
        return ORA_EINVAL;
    if ((P->phys & ORA_SHOCK) && !(P->shock_thresh >= 0.0 && isfinite(P->shock_thresh))) return ORA_EINVAL;
    int ngmin = (P->recon == 1) ? 3 : 2;
    /* extents, guard width, range of offsets */
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        if (B->nx < 1 || B->ny < 1 || B->nz < 1 || B->ng < ngmin) return ORA_EINVAL;
        if (P->ndim == 2 && B->nz != 1) return ORA_EINVAL;
        int64_t pz = (P->ndim == 3) ? B->nz + 2 * B->ng : 1;
        int64_t sz = (int64_t)(B->nx + 2 * B->ng) * (B->ny + 2 * B->ng) * pz;
        if (B->offset < 0 || B->offset + sz > P->ncell) return ORA_EINVAL;
    }
    /* no two blocks overlap: sort by offset and compare neighbours */
    int64_t *ord = malloc(sizeof(int64_t) * 2 * (size_t)(P->nblocks > 0 ? P->nblocks : 1));
    if (!ord) return ORA_ENOMEM;
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        int64_t pz = (P->ndim == 3) ? B->nz + 2 * B->ng : 1;
        ord[2 * b] = B->offset;
        ord[2 * b + 1] = B->offset + (int64_t)(B->nx + 2 * B->ng) * (B->ny + 2 * B->ng) * pz;
    }
    /* insertion sort on pairs (fine for test sizes; O(n^2) worst case) */
    for (int i = 1; i < P->nblocks; i++) {
        int64_t a = ord[2 * i], e = ord[2 * i + 1];
        int j = i - 1;
        while (j >= 0 && ord[2 * j] > a) { ord[2 * j + 2] = ord[2 * j]; ord[2 * j + 3] = ord[2 * j + 1]; j--; }
        ord[2 * j + 2] = a; ord[2 * j + 3] = e;
    }
    for (int i = 1; i < P->nblocks; i++)
        if (ord[2 * i] < ord[2 * i - 1]) { free(ord); return ORA_EINVAL; }
    free(ord);
    /* links: index range, matching faces, enough interior to feed the guards */
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        for (int d = 0; d < P->ndim; d++)
            for (int side = 0; side < 2; side++) {
                int nb = P->links[b].nbr[2 * d + side];
                if (nb >= P->nblocks || nb < -2) return ORA_EINVAL;
                const ora_block *S = (nb >= 0) ? &P->blocks[nb] : B;
                if (nb == -1) continue;
                for (int e = 0; e < P->ndim; e++)
                    if (e != d && ora_r_extent(S, e) != ora_r_extent(B, e)) return ORA_EINVAL;
                if (ora_r_extent(S, d) < B->ng) return ORA_EINVAL;
                if (S->ng != B->ng) return ORA_EINVAL;
            }
    }
    return ORA_OK;
}

int ora_validate(const ora_problem *P) { return validate(P); }

/* ------------------------------------------------------------ forward API */

int ora_fill_guards(const ora_problem *P, double *U)
{
    int rc = validate(P);
    if (rc) return rc;
    ora_r_fill_guards(P, U);
    return ORA_OK;
}

/* CFL time step: dt = cfl / max over interior cells of
 * sum_d (|u_d| + c)/dx_d, from the cell averages of U (unsplit form). */
int ora_cfl_dt(const ora_problem *P, const double *U, double *dt)
{
    int rc = validate(P);
    if (rc) return rc;
    const int nd = P->ndim, nv = nd + 2;
    const int64_t nc = P->ncell;
    const double idx = 1.0 / P->dx, idy = 1.0 / P->dy, idz = 1.0 / P->dz;
    double smax = 0.0;
    int64_t bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(max : smax) reduction(+ : bad)
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        for (int k = 0; k < B->nz; k++)
            for (int j = 0; j < B->ny; j++)
                for (int i = 0; i < B->nx; i++) {
                    int64_t ci = ora_r_cell(B, nd, i, j, k);
                    double Uc[5], W[5];
                    for (int v = 0; v < nv; v++) Uc[v] = U[v * nc + ci];
                    bad += ora_r_eos(P, Uc, W);
                    double r = 1.0 / Uc[0];
                    double c = sqrt((P->gamma * W[4]) * r);
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

/* One stage: fills the guards of Us in place, writes the interior of Uout. */
int ora_rk_stage(const ora_problem *P, int s, double dt, const double *Un, double *Us, double *Uout)
{
    int rc = validate(P);
    if (rc) return rc;
    if (s < 1 || s > P->rk || !(dt > 0.0)) return ORA_EINVAL;
    ora_r_fill_guards(P, Us);
    int64_t bad = ora_r_stage(P, s, dt, Un, Us, Uout);
    return bad ? ORA_ENONPHYS : ORA_OK;
}

/* One time step in place on U (interior).  If compute_dt, *dt receives the
 * CFL step computed from U; otherwise *dt is used as given. */
int ora_step(const ora_problem *P, double *U, double *dt, int compute_dt)
{
    int rc = validate(P);
    if (rc) return rc;
    if (compute_dt) {
        rc = ora_cfl_dt(P, U, dt);
        if (rc) return rc;
    }
    if (!(*dt > 0.0)) return ORA_EINVAL;
    size_t bytes = sizeof(double) * (size_t)(P->ndim + 2) * (size_t)P->ncell;
    double *Us = malloc(bytes), *Uo = malloc(bytes);
    if (!Us || !Uo) { free(Us); free(Uo); return ORA_ENOMEM; }
    memcpy(Us, U, bytes);
    memcpy(Uo, U, bytes);
    int64_t bad = 0;
    for (int s = 1; s <= P->rk && !bad; s++) {
        ora_r_fill_guards(P, Us);
        bad += ora_r_stage(P, s, *dt, U, Us, Uo);
        double *t = Us; Us = Uo; Uo = t;
    }
    if (!bad) memcpy(U, Us, bytes);
    free(Us); free(Uo);
    return bad ? ORA_ENONPHYS : ORA_OK;
}

/* ------------------------------------------------------ telescoping step */

/* Telescoping variant of the SSP-RK step (the paper's second RK listing in
 * Sec. 4.2): the guard cells are filled once per step, with a halo thick
 * enough for all stages (S*(R+1) layers, edges and corners included), and
 * every stage then updates the block together with the part of its halo
 * that later stages still read, instead of refilling guards between stages.
 *
 * Thick copies of the blocks live in a separate buffer.  The halo is filled
 * one direction after the other: direction d fills its layers over the
 * already-filled extents of the directions before it, which fills edges and
 * corners from the neighbours of neighbours (or by wrap / nearest-cell copy).
 * Stage s then runs on "virtual" blocks that are the interior extended by
 * m = (S - s)(R + 1) cells on every side. */

static int tele_width(const ora_problem *P) { return P->rk * ((P->recon == 1) ? 3 : 2); }

static void thick_table(const ora_problem *P, int ngt, ora_block *T, int64_t *ncell_t)
{
    int64_t off = 0;
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        T[b].nx = B->nx; T[b].ny = B->ny; T[b].nz = B->nz; T[b].ng = ngt; T[b].offset = off;
        int64_t pz = (P->ndim == 3) ? B->nz + 2 * ngt : 1;
        off += (int64_t)(B->nx + 2 * ngt) * (B->ny + 2 * ngt) * pz;
    }
    *ncell_t = off;
}

/* Copy the interior of U into the thick buffer and fill its halo. */
static void thick_fill(const ora_problem *P, const ora_block *T, int64_t nct, const double *U, double *Ut)
{
    const int nd = P->ndim, nv = nd + 2;
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        for (int k = 0; k < B->nz; k++)
            for (int j = 0; j < B->ny; j++)
                for (int i = 0; i < B->nx; i++)
                    for (int v = 0; v < nv; v++)
                        Ut[v * nct + ora_r_cell(&T[b], nd, i, j, k)] = U[v * P->ncell + ora_r_cell(B, nd, i, j, k)];
    }
    for (int d = 0; d < nd; d++)
        for (int b = 0; b < P->nblocks; b++) {
            const ora_block *B = &T[b];
            const int g = B->ng;
            int lo[3], hi[3];        /* ranges of the other coordinates */
            for (int e = 0; e < 3; e++) {
                int n = ora_r_extent(B, e);
                if (e >= nd) { lo[e] = 0; hi[e] = 1; }
                else if (e < d) { lo[e] = -g; hi[e] = n + g; }
                else { lo[e] = 0; hi[e] = n; }
            }
            int n = ora_r_extent(B, d);
            for (int side = 0; side < 2; side++) {
                int nb = P->links[b].nbr[2 * d + side];
                for (int l = 1; l <= g; l++) {
                    int gpos = (side == 0) ? -l : n - 1 + l;
                    int sb = b, spos;
                    if (nb >= 0) { sb = nb; spos = (side == 0) ? ora_r_extent(&T[nb], d) - l : l - 1; }
                    else if (nb == -2) spos = (side == 0) ? n - l : l - 1;
                    else spos = (side == 0) ? 0 : n - 1;
                    lo[d] = 0; hi[d] = 1;
                    for (int c2 = lo[2]; c2 < hi[2]; c2++)
                        for (int c1 = lo[1]; c1 < hi[1]; c1++)
                            for (int c0 = lo[0]; c0 < hi[0]; c0++) {
                                int gc[3] = {c0, c1, c2}, sc[3] = {c0, c1, c2};
                                gc[d] = gpos;
                                sc[d] = spos;
                                int64_t gi = ora_r_cell(B, nd, gc[0], gc[1], gc[2]);
                                int64_t si = ora_r_cell(&T[sb], nd, sc[0], sc[1], sc[2]);
                                for (int v = 0; v < nv; v++) Ut[v * nct + gi] = Ut[v * nct + si];
                            }
                }
            }
        }
}

/* One telescoping step in place on U. */
int ora_step_telescoping(const ora_problem *P, double *U, double *dt, int compute_dt)
{
    int rc = validate(P);
    if (rc) return rc;
    /* the telescoping listing runs the block initialisation (shockDet) once
     * per step, before all stages: not built with the detector */
    if (P->phys & ORA_SHOCK) return ORA_EINVAL;
    const int H = (P->recon == 1) ? 3 : 2, S = P->rk, ngt = tele_width(P);
    for (int b = 0; b < P->nblocks; b++)
        for (int d = 0; d < P->ndim; d++) {
            int nb = P->links[b].nbr[2 * d], nb2 = P->links[b].nbr[2 * d + 1];
            if ((nb >= 0 && ora_r_extent(&P->blocks[nb], d) < ngt) ||
                (nb2 >= 0 && ora_r_extent(&P->blocks[nb2], d) < ngt) ||
                ((nb == -2 || nb2 == -2) && ora_r_extent(&P->blocks[b], d) < ngt))
                return ORA_EINVAL;             /* halo deeper than the source block */
        }
    if (compute_dt) {
        rc = ora_cfl_dt(P, U, dt);
        if (rc) return rc;
    }
    if (!(*dt > 0.0)) return ORA_EINVAL;
    const int nv = P->ndim + 2;
    ora_block *T = malloc(sizeof(ora_block) * (size_t)(P->nblocks > 0 ? P->nblocks : 1));
    ora_block *V = malloc(sizeof(ora_block) * (size_t)(P->nblocks > 0 ? P->nblocks : 1));
    int64_t nct;
    thick_table(P, ngt, T, &nct);
    size_t bytes = sizeof(double) * (size_t)nv * (size_t)nct;
    double *Un = malloc(bytes), *Ua = malloc(bytes), *Ub = malloc(bytes);
    if (!T || !V || !Un || !Ua || !Ub) { free(T); free(V); free(Un); free(Ua); free(Ub); return ORA_ENOMEM; }
    for (size_t q = 0; q < bytes / sizeof(double); q++) Un[q] = NAN;
    thick_fill(P, T, nct, U, Un);
    memcpy(Ua, Un, bytes);
    memcpy(Ub, Un, bytes);
    int64_t bad = 0;
    const double *in = Un;
    double *out = Ua;
    for (int s = 1; s <= S; s++) {
        const int m = (S - s) * H;          /* cells beyond the interior still needed */
        for (int b = 0; b < P->nblocks; b++) {
            const int mz = (P->ndim == 3) ? m : 0;
            V[b].nx = T[b].nx + 2 * m; V[b].ny = T[b].ny + 2 * m; V[b].nz = T[b].nz + 2 * mz;
            V[b].ng = ngt - m;           /* same memory and strides; interior grown by m */
            V[b].offset = T[b].offset;
        }
        ora_problem Q = *P;
        Q.blocks = V;
        Q.ncell = nct;
        bad += ora_r_stage(&Q, s, *dt, Un, in, out);
        in = out;
        out = (out == Ua) ? Ub : Ua;
    }
    if (!bad)
        for (int b = 0; b < P->nblocks; b++) {
            const ora_block *B = &P->blocks[b];
            for (int k = 0; k < B->nz; k++)
                for (int j = 0; j < B->ny; j++)
                    for (int i = 0; i < B->nx; i++)
                        for (int v = 0; v < nv; v++)
                            U[v * P->ncell + ora_r_cell(B, P->ndim, i, j, k)] = in[v * nct + ora_r_cell(&T[b], P->ndim, i, j, k)];
        }
    free(T); free(V); free(Un); free(Ua); free(Ub);
    return bad ? ORA_ENONPHYS : ORA_OK;
}

/* ------------------------------------------------------------- adjoint */

/* Reverse of the EOS: gU (nvar) += (dW/dU)^T gW. */
static void eos_vjp(const ora_problem *P, const double *Uc, const double *W, const double *gW, double *gU)
{
    const double g1 = P->gamma - 1.0;
    int nd = P->ndim;
    double r = 1.0 / Uc[0];
    double gke = -g1 * gW[4];
    double gr = 0.0;
    gU[nd + 1] += g1 * gW[4];
    for (int d = 0; d < nd; d++) {
        double gu = gW[1 + d] + 0.5 * Uc[1 + d] * gke;   /* u_d = m_d r, ke = sum m_d u_d / 2 */
        gU[1 + d] += 0.5 * W[1 + d] * gke + r * gu;
        gr += Uc[1 + d] * gu;
    }
    gU[0] += gW[0] - r * r * gr;
}

/* Reverse of the limited linear reconstruction with the recorded branch. */
static void plm_vjp(int code, double gqm, double gqp, double *ga, double *g0, double *gb)
{
    double gs = 0.5 * gqp - 0.5 * gqm;
    double gdm = 0.0, gdp = 0.0;
    if (code == 1) { gdm = 0.5 * gs; gdp = 0.5 * gs; }     /* s = (dm+dp)/2 */
    else if (code == 2) gdm = 2.0 * gs;
    else if (code == 3) gdp = 2.0 * gs;
    *g0 += gqm + gqp + gdm - gdp;
    *ga -= gdm;
    *gb += gdp;
}

/* Reverse of WENO5-JS (both faces share the smoothness indicators). */
static void weno5_vjp(const double *q, double eps, double gqm, double gqp, double *g)
{
    const double k13 = 13.0 / 12.0, k6 = 1.0 / 6.0;
    double a = q[0], b = q[1], c = q[2], d = q[3], e = q[4];
    double t[3], w[3], be[3], s[3], o[3];
    t[0] = (a - 2.0 * b) + c;  w[0] = (a - 4.0 * b) + 3.0 * c;
    t[1] = (b - 2.0 * c) + d;  w[1] = b - d;
    t[2] = (c - 2.0 * d) + e;  w[2] = (3.0 * c - 4.0 * d) + e;
    for (int k = 0; k < 3; k++) {
        be[k] = k13 * (t[k] * t[k]) + 0.25 * (w[k] * w[k]);
        s[k] = (eps + be[k]) * (eps + be[k]);
    }
    /* unnormalised weights as in the forward: o_k = product of the other s_j */
    o[0] = s[1] * s[2];  o[1] = s[0] * s[2];  o[2] = s[0] * s[1];
    double go[3] = {0.0, 0.0, 0.0};
    /* right face */
    {
        double p[3], al[3];
        p[0] = ((2.0 * a - 7.0 * b) + 11.0 * c) * k6;
        p[1] = ((-b + 5.0 * c) + 2.0 * d) * k6;
        p[2] = ((2.0 * c + 5.0 * d) - e) * k6;
        al[0] = 0.1 * o[0];  al[1] = 0.6 * o[1];  al[2] = 0.3 * o[2];
        double iS = 1.0 / ((al[0] + al[1]) + al[2]);
        double gS = gqp * iS;
        double qv = ((al[0] * p[0] + al[1] * p[1]) + al[2] * p[2]) * iS;
        double gp[3];
        for (int k = 0; k < 3; k++) gp[k] = gS * al[k];
        go[0] += 0.1 * gS * (p[0] - qv);
        go[1] += 0.6 * gS * (p[1] - qv);
        go[2] += 0.3 * gS * (p[2] - qv);
        g[0] += k6 * (2.0 * gp[0]);
        g[1] += k6 * (-7.0 * gp[0] - gp[1]);
        g[2] += k6 * (11.0 * gp[0] + 5.0 * gp[1] + 2.0 * gp[2]);
        g[3] += k6 * (2.0 * gp[1] + 5.0 * gp[2]);
        g[4] += k6 * (-gp[2]);
    }
    /* left face: mirrored candidates, weights (0.1 o2, 0.6 o1, 0.3 o0) */
    {
        double p[3], al[3];
        p[0] = ((2.0 * e - 7.0 * d) + 11.0 * c) * k6;
        p[1] = ((-d + 5.0 * c) + 2.0 * b) * k6;
        p[2] = ((2.0 * c + 5.0 * b) - a) * k6;
        al[0] = 0.1 * o[2];  al[1] = 0.6 * o[1];  al[2] = 0.3 * o[0];
        double iS = 1.0 / ((al[0] + al[1]) + al[2]);
        double gS = gqm * iS;
        double qv = ((al[0] * p[0] + al[1] * p[1]) + al[2] * p[2]) * iS;
        double gp[3];
        for (int k = 0; k < 3; k++) gp[k] = gS * al[k];
        go[2] += 0.1 * gS * (p[0] - qv);
        go[1] += 0.6 * gS * (p[1] - qv);
        go[0] += 0.3 * gS * (p[2] - qv);
        g[4] += k6 * (2.0 * gp[0]);
        g[3] += k6 * (-7.0 * gp[0] - gp[1]);
        g[2] += k6 * (11.0 * gp[0] + 5.0 * gp[1] + 2.0 * gp[2]);
        g[1] += k6 * (2.0 * gp[1] + 5.0 * gp[2]);
        g[0] += k6 * (-gp[2]);
    }
    /* o_0 = s_1 s_2, o_1 = s_0 s_2, o_2 = s_0 s_1; s_k = (eps + beta_k)^2;
     * beta_k = k13 t_k^2 + w_k^2 / 4 */
    double gs[3];
    gs[0] = go[1] * s[2] + go[2] * s[1];
    gs[1] = go[0] * s[2] + go[2] * s[0];
    gs[2] = go[0] * s[1] + go[1] * s[0];
    double gt[3], gw[3];
    for (int k = 0; k < 3; k++) {
        double gbe = 2.0 * (eps + be[k]) * gs[k];
        gt[k] = 2.0 * k13 * t[k] * gbe;
        gw[k] = 0.5 * w[k] * gbe;
    }
    g[0] += gt[0] + gw[0];
    g[1] += -2.0 * gt[0] - 4.0 * gw[0] + gt[1] + gw[1];
    g[2] += gt[0] + 3.0 * gw[0] - 2.0 * gt[1] + gt[2] + 3.0 * gw[2];
    g[3] += gt[1] - gw[1] - 2.0 * gt[2] - 4.0 * gw[2];
    g[4] += gt[2] + gw[2];
}

/* Reverse of state_flux: gW (5) += contributions of gU, gF (nvar), gc, gr. */
static void state_flux_vjp(const ora_problem *P, const double *W, int n,
                           const double *gU, const double *gF, double gc, double gr, double *gW)
{
    const double g = P->gamma, ig1 = 1.0 / (g - 1.0);
    int nd = P->ndim, nv = nd + 2;
    double rho = W[0], p = W[4], un = W[1 + n];
    double u2;
    if (nd == 3) u2 = (W[1] * W[1] + W[2] * W[2]) + W[3] * W[3];
    else u2 = W[1] * W[1] + W[2] * W[2];
    double E = p * ig1 + 0.5 * (rho * u2);
    double fr = rho * un;
    double grho = 0.0, gp = 0.0, gE = 0.0, gu[3] = {0.0, 0.0, 0.0};
    /* F */
    double gfr = gF[0];
    for (int d = 0; d < nd; d++) { gfr += gF[1 + d] * W[1 + d]; gu[d] += gF[1 + d] * fr; }
    gp += gF[1 + n];
    gE += gF[nv - 1] * un;
    gp += gF[nv - 1] * un;
    gu[n] += gF[nv - 1] * (E + p);
    grho += gfr * un;
    gu[n] += gfr * rho;
    /* U */
    grho += gU[0];
    for (int d = 0; d < nd; d++) { grho += gU[1 + d] * W[1 + d]; gu[d] += gU[1 + d] * rho; }
    gE += gU[nv - 1];
    /* E = p/(g-1) + rho |u|^2 / 2 */
    gp += gE * ig1;
    grho += gE * 0.5 * u2;
    for (int d = 0; d < nd; d++) gu[d] += gE * rho * W[1 + d];
    /* r = 1/rho, c = sqrt(g p r) */
    double r = 1.0 / rho, c = sqrt((g * p) * r);
    double gx = gc / (2.0 * c);
    gp += gx * g * r;
    double grt = gr + gx * g * p;
    grho += -r * r * grt;
    gW[0] += grho;
    for (int d = 0; d < nd; d++) gW[1 + d] += gu[d];
    gW[4] += gp;
}

/* Reverse of HLLC at one face with the recorded tape. */
static void hllc_vjp(const ora_problem *P, const double *WL, const double *WR, int n, int tape,
                     const double *gF, double *gWL, double *gWR)
{
    int nd = P->ndim, nv = nd + 2;
    double UL[5], UR[5], FL[5], FR[5], cL, cR, rL, rR;
    ora_r_state_flux(P, WL, n, UL, FL, &cL, &rL);
    ora_r_state_flux(P, WR, n, UR, FR, &cR, &rR);
    double gUL[5] = {0}, gUR[5] = {0}, gFL[5] = {0}, gFR[5] = {0};
    double gcL = 0.0, gcR = 0.0, grL = 0.0, grR = 0.0;
    int region = tape & 3;
    if (region == 0) {
        for (int v = 0; v < nv; v++) gFL[v] += gF[v];
    } else if (region == 3) {
        for (int v = 0; v < nv; v++) gFR[v] += gF[v];
    } else {
        double uL = WL[1 + n], uR = WR[1 + n];
        double SL = (tape & 4) ? uR - cR : uL - cL;
        double SR = (tape & 8) ? uR + cR : uL + cL;
        double mL = WL[0] * (SL - uL), mR = WR[0] * (SR - uR);
        double Num = (WR[4] - WL[4]) + (mL * uL - mR * uR), Den = mL - mR;
        double Ss = Num / Den;
        int K = (region == 1) ? 0 : 1;
        const double *W = K ? WR : WL, *UK = K ? UR : UL;
        double *gW = K ? gWR : gWL, *gUK = K ? gUR : gUL, *gFK = K ? gFR : gFL;
        double SK = K ? SR : SL, mK = K ? mR : mL, rK = K ? rR : rL, uK = W[1 + n];
        double den = SK - Ss, chi = mK / den;
        double Us[5];
        Us[0] = chi;
        for (int d = 0; d < nd; d++) Us[1 + d] = chi * W[1 + d];
        Us[1 + n] = chi * Ss;
        double q = W[4] / mK;
        double Bq = UK[nv - 1] * rK + (Ss - uK) * (Ss + q);
        Us[nv - 1] = chi * Bq;
        /* F = F_K + S_K (U* - U_K) */
        double gSK = 0.0, gUs[5];
        for (int v = 0; v < nv; v++) {
            gFK[v] += gF[v];
            gSK += gF[v] * (Us[v] - UK[v]);
            gUs[v] = SK * gF[v];
            gUK[v] -= SK * gF[v];
        }
        /* U* */
        double gchi = gUs[0] + gUs[1 + n] * Ss + gUs[nv - 1] * Bq;
        for (int d = 0; d < nd; d++)
            if (d != n) { gchi += gUs[1 + d] * W[1 + d]; gW[1 + d] += gUs[1 + d] * chi; }
        double gSs = gUs[1 + n] * chi;
        double gB = gUs[nv - 1] * chi;
        gUK[nv - 1] += gB * rK;
        double grK = gB * UK[nv - 1];
        gSs += gB * (Ss + q) + gB * (Ss - uK);
        gW[1 + n] -= gB * (Ss + q);
        double gq = gB * (Ss - uK);
        gW[4] += gq / mK;
        double gmK = -gq * q / mK;
        /* chi = m_K / (S_K - S*) */
        gmK += gchi / den;
        double gden = -gchi * chi / den;
        gSK += gden;
        gSs -= gden;
        if (K) grR += grK; else grL += grK;
        double gSL = 0.0, gSR = 0.0, gmL = 0.0, gmR = 0.0;
        if (K) { gSR += gSK; gmR += gmK; } else { gSL += gSK; gmL += gmK; }
        /* S* = Num / Den */
        double gN = gSs / Den, gD = -gSs * Ss / Den;
        gWR[4] += gN;
        gWL[4] -= gN;
        gmL += gN * uL + gD;
        gmR += -gN * uR - gD;
        double guL = gN * mL, guR = -gN * mR;
        /* m_L = rho_L (S_L - u_L), m_R = rho_R (S_R - u_R) */
        gWL[0] += gmL * (SL - uL);  gSL += gmL * WL[0];  guL -= gmL * WL[0];
        gWR[0] += gmR * (SR - uR);  gSR += gmR * WR[0];  guR -= gmR * WR[0];
        /* Davis bounds */
        if (tape & 4) { guR += gSL; gcR -= gSL; } else { guL += gSL; gcL -= gSL; }
        if (tape & 8) { guR += gSR; gcR += gSR; } else { guL += gSR; gcL += gSR; }
        gWL[1 + n] += guL;
        gWR[1 + n] += guR;
    }
    state_flux_vjp(P, WL, n, gUL, gFL, gcL, grL, gWL);
    state_flux_vjp(P, WR, n, gUR, gFR, gcR, grR, gWR);
}

/* Adjoint of the spatial part of one block's stage.  gacc is the cotangent
 * of acc = sum_d D_d/dx_d (nvar x interior, x fastest); gPad receives the
 * cotangents of every padded cell the block's stencils read. */
static void block_rhs_vjp(const ora_problem *P, int b, const double *U, const double *gacc, double *gPad)
{
    unsigned char *shock = NULL;
    if (P->phys & ORA_SHOCK) {
        shock = malloc((size_t)(P->ndim * ora_r_npad(&P->blocks[b], P->ndim)));
        ora_r_shock_detect(P, b, U, shock);
    }
    const int nd = P->ndim, nv = nd + 2;
    const int64_t nc = P->ncell;
    const ora_block *B = &P->blocks[b];
    const int R = (P->recon == 1) ? 2 : 1;
    const double id[3] = {1.0 / P->dx, 1.0 / P->dy, 1.0 / P->dz};
    const int64_t nint = (int64_t)B->nx * B->ny * B->nz;
    int nmax = B->nx > B->ny ? B->nx : B->ny;
    if (B->nz > nmax) nmax = B->nz;
    int len = nmax + 2 * (R + 1);
    double *Uln = malloc(sizeof(double) * 5 * len), *W = malloc(sizeof(double) * 5 * len);
    double *gW = malloc(sizeof(double) * 5 * len);
    double *qm = malloc(sizeof(double) * 5 * (nmax + 2)), *qp = malloc(sizeof(double) * 5 * (nmax + 2));
    double *gqm = malloc(sizeof(double) * 5 * (nmax + 2)), *gqp = malloc(sizeof(double) * 5 * (nmax + 2));
    int *code = malloc(sizeof(int) * 5 * (nmax + 2)), *fb = malloc(sizeof(int) * (nmax + 2));
    double *gF = malloc(sizeof(double) * 5 * (nmax + 1));
    for (int d = 0; d < nd; d++) {
        int n = ora_r_extent(B, d);
        int o1 = (d == 0) ? 1 : 0, o2 = (d == 2) ? 1 : 2;
        int n1 = ora_r_extent(B, o1), n2 = (nd == 3) ? ora_r_extent(B, o2) : 1;
        for (int e2 = 0; e2 < n2; e2++)
            for (int e1 = 0; e1 < n1; e1++) {
                /* forward recomputation of the line */
                for (int t = -1 - R; t <= n + R; t++) {
                    int pos[3];
                    pos[d] = t;  pos[o1] = e1;  pos[o2] = e2;
                    if (nd == 2) pos[2] = 0;
                    int64_t ci = ora_r_cell(B, nd, pos[0], pos[1], pos[2]);
                    for (int v = 0; v < nv; v++) Uln[5 * (t + 1 + R) + v] = U[v * nc + ci];
                    ora_r_eos(P, &Uln[5 * (t + 1 + R)], &W[5 * (t + 1 + R)]);
                }
                for (int t = -1; t <= n; t++) {
                    int sh = 0;
                    if (shock) {
                        int pos[3];
                        pos[d] = t;  pos[o1] = e1;  pos[o2] = e2;
                        if (nd == 2) pos[2] = 0;
                        sh = shock[d * ora_r_npad(B, nd) + ora_r_cell(B, nd, pos[0], pos[1], pos[2]) - B->offset];
                    }
                    fb[t + 1] = ora_r_recon_cell(P, &W[5 * (t + 1 + R)], sh, &qm[5 * (t + 1)], &qp[5 * (t + 1)],
                                                 &code[5 * (t + 1)]);
                }
                /* reverse: flux differences -> face flux cotangents */
                for (int i = 0; i < 5 * (n + 1); i++) gF[i] = 0.0;
                for (int t = 0; t < n; t++) {
                    int pos[3];
                    pos[d] = t;  pos[o1] = e1;  pos[o2] = e2;
                    if (nd == 2) pos[2] = 0;
                    int64_t li = ((int64_t)pos[2] * B->ny + pos[1]) * B->nx + pos[0];
                    for (int v = 0; v < nv; v++) {
                        double gD = gacc[v * nint + li] * id[d];
                        gF[5 * (t + 1) + v] += gD;
                        gF[5 * t + v] -= gD;
                    }
                }
                /* HLLC -> face states */
                for (int i = 0; i < 5 * (n + 2); i++) { gqm[i] = 0.0; gqp[i] = 0.0; }
                for (int t = 0; t <= n; t++) {
                    double Ftmp[5];
                    int tape;
                    ora_r_hllc(P, &qp[5 * t], &qm[5 * (t + 1)], d, Ftmp, &tape);
                    double gFv[5] = {0};
                    for (int v = 0; v < nv; v++) gFv[v] = gF[5 * t + v];
                    hllc_vjp(P, &qp[5 * t], &qm[5 * (t + 1)], d, tape, gFv, &gqp[5 * t], &gqm[5 * (t + 1)]);
                }
                /* reconstruction -> cell primitives */
                for (int i = 0; i < 5 * len; i++) gW[i] = 0.0;
                for (int t = -1; t <= n; t++) {
                    int c0 = t + 1 + R;
                    const double *gm = &gqm[5 * (t + 1)], *gp = &gqp[5 * (t + 1)];
                    if (fb[t + 1]) {
                        for (int q = 0; q < 5; q++) gW[5 * c0 + q] += gm[q] + gp[q];
                        continue;
                    }
                    for (int q = 0; q < 5; q++) {
                        if (q == 3 && nd == 2) continue;
                        if (R == 1) {
                            plm_vjp(code[5 * (t + 1) + q], gm[q], gp[q],
                                    &gW[5 * (c0 - 1) + q], &gW[5 * c0 + q], &gW[5 * (c0 + 1) + q]);
                        } else {
                            double st[5], gs[5] = {0, 0, 0, 0, 0};
                            for (int k = 0; k < 5; k++) st[k] = W[5 * (c0 - 2 + k) + q];
                            weno5_vjp(st, P->weno_eps, gm[q], gp[q], gs);
                            for (int k = 0; k < 5; k++) gW[5 * (c0 - 2 + k) + q] += gs[k];
                        }
                    }
                }
                /* EOS -> conserved cell values, accumulated into the block's padded cells */
                for (int t = -1 - R; t <= n + R; t++) {
                    int pos[3];
                    pos[d] = t;  pos[o1] = e1;  pos[o2] = e2;
                    if (nd == 2) pos[2] = 0;
                    int64_t ci = ora_r_cell(B, nd, pos[0], pos[1], pos[2]);
                    double gU[5] = {0, 0, 0, 0, 0};
                    eos_vjp(P, &Uln[5 * (t + 1 + R)], &W[5 * (t + 1 + R)], &gW[5 * (t + 1 + R)], gU);
                    for (int v = 0; v < nv; v++) gPad[v * nc + ci] += gU[v];
                }
            }
    }
    free(Uln); free(W); free(gW); free(qm); free(qp); free(gqm); free(gqp); free(code); free(fb); free(gF);
    free(shock);
}

/* Adjoint of guard filling: each guard cell's cotangent moves onto the
 * interior cell it was copied from; the guard's own entry is cleared. */
static void fill_guards_vjp(const ora_problem *P, double *gPad)
{
    const int nd = P->ndim, nv = nd + 2;
    const int64_t nc = P->ncell;
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        for (int d = 0; d < nd; d++) {
            int o1 = (d == 0) ? 1 : 0, o2 = (d == 2) ? 1 : 2;
            int n1 = ora_r_extent(B, o1), n2 = (nd == 3) ? ora_r_extent(B, o2) : 1;
            for (int side = 0; side < 2; side++)
                for (int l = 1; l <= B->ng; l++) {
                    int sb, spos;
                    ora_r_guard_source(P, b, d, side, l, &sb, &spos);
                    int gpos = (side == 0) ? -l : ora_r_extent(B, d) - 1 + l;
                    for (int e2 = 0; e2 < n2; e2++)
                        for (int e1 = 0; e1 < n1; e1++) {
                            int g[3], s[3];
                            g[d] = gpos;  g[o1] = e1;  g[o2] = e2;
                            s[d] = spos;  s[o1] = e1;  s[o2] = e2;
                            if (nd == 2) { g[2] = 0; s[2] = 0; }
                            int64_t gi = ora_r_cell(B, nd, g[0], g[1], g[2]);
                            int64_t si = ora_r_cell(&P->blocks[sb], nd, s[0], s[1], s[2]);
                            for (int v = 0; v < nv; v++) {
                                gPad[v * nc + si] += gPad[v * nc + gi];
                                gPad[v * nc + gi] = 0.0;
                            }
                        }
                }
        }
    }
}

/* Cotangent of one stage.  Us: guard-filled stage input.  gOut: cotangent of
 * the stage output's interior.  Writes gUs (interior; padding zero) and adds
 * a_s gOut to gUn's interior. */
static void stage_vjp(const ora_problem *P, int s, double dt, const double *Us, const double *gOut,
                      double *gUs, double *gUn, double *gPad)
{
    const int nd = P->ndim, nv = nd + 2;
    const int64_t nc = P->ncell;
    double a = 0.0, bcoef = 1.0;
    if (P->rk == 2 && s == 2) { a = 0.5; bcoef = 0.5; }
    if (P->rk == 3 && s == 2) { a = 0.75; bcoef = 0.25; }
    if (P->rk == 3 && s == 3) { a = 1.0 / 3.0; bcoef = 2.0 / 3.0; }
    memset(gPad, 0, sizeof(double) * (size_t)nv * (size_t)nc);
#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        int64_t nint = (int64_t)B->nx * B->ny * B->nz;
        double *gacc = malloc(sizeof(double) * nv * nint);
        for (int k = 0; k < B->nz; k++)
            for (int j = 0; j < B->ny; j++)
                for (int i = 0; i < B->nx; i++) {
                    int64_t li = ((int64_t)k * B->ny + j) * B->nx + i;
                    int64_t ci = ora_r_cell(B, nd, i, j, k);
                    for (int v = 0; v < nv; v++) {
                        double gT = bcoef * gOut[v * nc + ci];
                        gacc[v * nint + li] = -(dt * gT);     /* L = -acc, T = U_s + dt L */
                    }
                }
        block_rhs_vjp(P, b, Us, gacc, gPad);
        free(gacc);
    }
    fill_guards_vjp(P, gPad);
    memset(gUs, 0, sizeof(double) * (size_t)nv * (size_t)nc);
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        for (int k = 0; k < B->nz; k++)
            for (int j = 0; j < B->ny; j++)
                for (int i = 0; i < B->nx; i++) {
                    int64_t ci = ora_r_cell(B, nd, i, j, k);
                    /* gravity source: T_{m_d} gains dt rho g_d, T_E gains dt (m . g) */
                    double gsrc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                    if (P->phys & ORA_GRAVITY) {
                        double g[3];
                        ora_r_grav_accel(P, b, i, j, k, g);
                        double gTE = bcoef * gOut[(nd + 1) * nc + ci];
                        for (int d = 0; d < nd; d++) {
                            double gTm = bcoef * gOut[(1 + d) * nc + ci];
                            gsrc[0] += dt * (g[d] * gTm);
                            gsrc[1 + d] = dt * (g[d] * gTE);
                        }
                    }
                    for (int v = 0; v < nv; v++) {
                        double go = gOut[v * nc + ci];
                        double gs = bcoef * go + gPad[v * nc + ci];
                        if (P->phys & ORA_GRAVITY) gs = gs + gsrc[v];
                        gUs[v * nc + ci] = gs;
                        gUn[v * nc + ci] += a * go;
                    }
                }
    }
}

/* Vector-Jacobian product of one step with dt held fixed:
 * gUn = (d U^{n+1} / d U^n)^T gUnext, interior cells (padding of gUn = 0). */
int ora_step_vjp(const ora_problem *P, const double *Un, double dt, const double *gUnext, double *gUn)
{
    int rc = validate(P);
    if (rc) return rc;
    if (!(dt > 0.0)) return ORA_EINVAL;
    const int S = P->rk, nv = P->ndim + 2;
    size_t bytes = sizeof(double) * (size_t)nv * (size_t)P->ncell;
    double *stg = malloc(bytes * (size_t)(S + 1));
    double *g = malloc(bytes), *gs = malloc(bytes), *gPad = malloc(bytes);
    if (!stg || !g || !gs || !gPad) { free(stg); free(g); free(gs); free(gPad); return ORA_ENOMEM; }
    /* forward recomputation, keeping every guard-filled stage input */
    memcpy(stg, Un, bytes);
    int64_t bad = 0;
    for (int s = 1; s <= S; s++) {
        double *Us = stg + (size_t)(s - 1) * (bytes / sizeof(double));
        double *Uo = stg + (size_t)s * (bytes / sizeof(double));
        ora_r_fill_guards(P, Us);
        memcpy(Uo, Us, bytes);
        bad += ora_r_stage(P, s, dt, Un, Us, Uo);
    }
    if (bad) { free(stg); free(g); free(gs); free(gPad); return ORA_ENONPHYS; }
    memset(gUn, 0, bytes);
    memcpy(g, gUnext, bytes);
    for (int s = S; s >= 1; s--) {
        double *Us = stg + (size_t)(s - 1) * (bytes / sizeof(double));
        stage_vjp(P, s, dt, Us, g, gs, gUn, gPad);
        double *t = g; g = gs; gs = t;
    }
    /* g now holds the cotangent of U_1 = U^n */
    const int nd = P->ndim;
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        for (int k = 0; k < B->nz; k++)
            for (int j = 0; j < B->ny; j++)
                for (int i = 0; i < B->nx; i++) {
                    int64_t ci = ora_r_cell(B, nd, i, j, k);
                    for (int v = 0; v < nv; v++) gUn[v * P->ncell + ci] += g[v * P->ncell + ci];
                }
    }
    free(stg); free(g); free(gs); free(gPad);
    return ORA_OK;
}

/* ------------------------------------------- point-wise entry points (pins) */

int ora_eos_n(const ora_problem *P, int64_t n, const double *U, double *W)
{
    int bad = 0, nv = P->ndim + 2;
    for (int64_t i = 0; i < n; i++) bad += ora_r_eos(P, &U[nv * i], &W[5 * i]);
    return bad;
}

void ora_plm_n(int64_t n, const double *q, double *qm, double *qp, int *code)
{
    for (int64_t i = 0; i < n; i++) ora_r_plm(q[3 * i], q[3 * i + 1], q[3 * i + 2], &qm[i], &qp[i], &code[i]);
}

void ora_weno5_n(int64_t n, const double *q, double eps, double *qm, double *qp)
{
    for (int64_t i = 0; i < n; i++)
        ora_r_weno5(q[5 * i], q[5 * i + 1], q[5 * i + 2], q[5 * i + 3], q[5 * i + 4], eps, &qm[i], &qp[i]);
}

/* Reconstruction of n cells along a line with the positivity fallback (the
 * step's calcLims for one cell and direction): w holds, per cell, the
 * primitives (rho, u_x, u_y, u_z, p) of its 2R+1 stencil cells (R = 1 PLM-MC,
 * 2 WENO5), the cell itself in the middle; qm, qp receive its left- and
 * right-face values (5 each), fb whether the fallback fired. */
void ora_recon_cell_n(const ora_problem *P, int64_t n, const double *w, double *qm, double *qp, int *fb)
{
    const int R = (P->recon == 1) ? 2 : 1;
    for (int64_t i = 0; i < n; i++)
        fb[i] = ora_r_recon_cell(P, &w[5 * ((2 * R + 1) * i + R)], 0, &qm[5 * i], &qp[5 * i], NULL);
}

/* Face values of every interior cell along direction d, from a state whose
 * guard cells are filled (ora_fill_guards): qm, qp (5 x ncell, primitives,
 * padded layout; entries outside the interior are left as they are) and fb
 * (ncell; 1 where the positivity fallback fired, 0 elsewhere in the
 * interior).  The same line walk as the stage: primitives from the EOS,
 * then the reconstruction of each cell. */
int ora_faces(const ora_problem *P, const double *U, int d, double *qm, double *qp, int *fb)
{
    int rc = validate(P);
    if (rc) return rc;
    if (d < 0 || d >= P->ndim) return ORA_EINVAL;
    const int nd = P->ndim, nv = nd + 2, R = (P->recon == 1) ? 2 : 1;
    const int64_t nc = P->ncell;
    int64_t bad = 0;
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        int n = ora_r_extent(B, d);
        int o1 = (d == 0) ? 1 : 0, o2 = (d == 2) ? 1 : 2;
        int n1 = ora_r_extent(B, o1), n2 = (nd == 3) ? ora_r_extent(B, o2) : 1;
        unsigned char *shock = NULL;
        if (P->phys & ORA_SHOCK) {
            shock = malloc((size_t)(nd * ora_r_npad(B, nd)));
            ora_r_shock_detect(P, b, U, shock);
        }
        double *W = malloc(sizeof(double) * 5 * (n + 2 * R));
        for (int e2 = 0; e2 < n2; e2++)
            for (int e1 = 0; e1 < n1; e1++) {
                int pos[3];
                for (int t = -R; t < n + R; t++) {
                    pos[d] = t;  pos[o1] = e1;  pos[o2] = e2;
                    if (nd == 2) pos[2] = 0;
                    int64_t ci = ora_r_cell(B, nd, pos[0], pos[1], pos[2]);
                    double Uc[5];
                    for (int v = 0; v < nv; v++) Uc[v] = U[v * nc + ci];
                    bad += ora_r_eos(P, Uc, &W[5 * (t + R)]);
                }
                for (int t = 0; t < n; t++) {
                    pos[d] = t;  pos[o1] = e1;  pos[o2] = e2;
                    if (nd == 2) pos[2] = 0;
                    int64_t ci = ora_r_cell(B, nd, pos[0], pos[1], pos[2]);
                    double m[5], p[5];
                    int sh = shock ? shock[d * ora_r_npad(B, nd) + ci - B->offset] : 0;
                    fb[ci] = ora_r_recon_cell(P, &W[5 * (t + R)], sh, m, p, NULL);
                    for (int q = 0; q < 5; q++) { qm[q * nc + ci] = m[q]; qp[q * nc + ci] = p[q]; }
                }
            }
        free(W);
        free(shock);
    }
    return bad ? ORA_ENONPHYS : ORA_OK;
}

/* The shock detector's flags along direction d (the block initialisation of
 * a stage) for every interior cell of a guard-filled state: flag (ncell)
 * receives 1 or 0 in the interior; other entries are left as they are.  The
 * problem's shock_thresh is used whether or not ORA_SHOCK is set. */
int ora_shock_flags(const ora_problem *P, const double *U, int d, int *flag)
{
    int rc = validate(P);
    if (rc) return rc;
    if (d < 0 || d >= P->ndim || !(P->shock_thresh >= 0.0)) return ORA_EINVAL;
    const int nd = P->ndim;
    for (int b = 0; b < P->nblocks; b++) {
        const ora_block *B = &P->blocks[b];
        const int64_t np = ora_r_npad(B, nd);
        unsigned char *sh = malloc((size_t)(nd * np));
        ora_r_shock_detect(P, b, U, sh);
        for (int k = 0; k < B->nz; k++)
            for (int j = 0; j < B->ny; j++)
                for (int i = 0; i < B->nx; i++) {
                    int64_t ci = ora_r_cell(B, nd, i, j, k);
                    flag[ci] = sh[d * np + ci - B->offset];
                }
        free(sh);
    }
    return ORA_OK;
}

int ora_hllc_n(const ora_problem *P, int64_t n, int dir, const double *WL, const double *WR, double *F, int *tape)
{
    int bad = 0, nv = P->ndim + 2;
    for (int64_t i = 0; i < n; i++) bad += ora_r_hllc(P, &WL[5 * i], &WR[5 * i], dir, &F[nv * i], &tape[i]);
    return bad;
}

void ora_state_flux_n(const ora_problem *P, int64_t n, int dir, const double *W, double *U, double *F, double *c)
{
    int nv = P->ndim + 2;
    for (int64_t i = 0; i < n; i++) {
        double r;
        ora_r_state_flux(P, &W[5 * i], dir, &U[nv * i], &F[nv * i], &c[i], &r);
    }
}

void ora_eos_vjp_n(const ora_problem *P, int64_t n, const double *U, const double *gW, double *gU)
{
    int nv = P->ndim + 2;
    for (int64_t i = 0; i < n; i++) {
        double W[5];
        ora_r_eos(P, &U[nv * i], W);
        for (int v = 0; v < nv; v++) gU[nv * i + v] = 0.0;
        eos_vjp(P, &U[nv * i], W, &gW[5 * i], &gU[nv * i]);
    }
}

void ora_plm_vjp_n(int64_t n, const double *q, const double *gqm, const double *gqp, double *gq)
{
    for (int64_t i = 0; i < n; i++) {
        double m, p;
        int code;
        ora_r_plm(q[3 * i], q[3 * i + 1], q[3 * i + 2], &m, &p, &code);
        gq[3 * i] = gq[3 * i + 1] = gq[3 * i + 2] = 0.0;
        plm_vjp(code, gqm[i], gqp[i], &gq[3 * i], &gq[3 * i + 1], &gq[3 * i + 2]);
    }
}

void ora_weno5_vjp_n(int64_t n, const double *q, double eps, const double *gqm, const double *gqp, double *gq)
{
    for (int64_t i = 0; i < n; i++) {
        for (int k = 0; k < 5; k++) gq[5 * i + k] = 0.0;
        weno5_vjp(&q[5 * i], eps, gqm[i], gqp[i], &gq[5 * i]);
    }
}

void ora_hllc_vjp_n(const ora_problem *P, int64_t n, int dir, const double *WL, const double *WR,
                    const double *gF, double *gWL, double *gWR)
{
    int nv = P->ndim + 2;
    for (int64_t i = 0; i < n; i++) {
        double F[5];
        int tape;
        ora_r_hllc(P, &WL[5 * i], &WR[5 * i], dir, F, &tape);
        for (int k = 0; k < 5; k++) { gWL[5 * i + k] = 0.0; gWR[5 * i + k] = 0.0; }
        double g[5] = {0};
        for (int v = 0; v < nv; v++) g[v] = gF[nv * i + v];
        hllc_vjp(P, &WL[5 * i], &WR[5 * i], dir, tape, g, &gWL[5 * i], &gWR[5 * i]);
    }
}
