/*
 * Complex-step instance of the oracle's forward method -- TEST
 * INFRASTRUCTURE ONLY.  Evaluating the forward step at U + i h V with a tiny h
 * gives Im(.)/h = J V, the exact directional derivative to rounding (Squire &
 * Trapp 1998; Martins, Sturdza & Alonso 2003), with every branch decided on
 * real parts.  It pins the hand-written adjoint through the dot-product
 * identity <w, J v> = <J^T w, v>.
 *
 * Non-analytic operations are complexified in the usual way: |x| and
 * copysign act on the sign of the real part; min/max compare real parts and
 * keep the first argument on a tie; the square root is expanded to first
 * order so its real part is the double-precision square root.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef double complex cplx;

static inline cplx cs_sqrt(cplx z)
{
    double s = sqrt(creal(z));
    return s + I * (cimag(z) / (2.0 * s));
}
static inline cplx cs_abs(cplx x) { return signbit(creal(x)) ? -x : x; }
static inline cplx cs_copysign(cplx m, cplx a) { return (signbit(creal(m)) != signbit(creal(a))) ? -m : m; }
static inline cplx RMIN(cplx a, cplx b) { return (creal(a) <= creal(b)) ? a : b; }
static inline cplx RMAX(cplx a, cplx b) { return (creal(a) >= creal(b)) ? a : b; }

#define REAL cplx
#define FN(name) ora_c_##name
#define RE(x) creal(x)
#define RSQRT(x) cs_sqrt(x)
#define RFMA(a, b, c) ((a) * (b) + (c))
#define RABS(x) cs_abs(x)
#define RCOPYSIGN(m, a) cs_copysign((m), (a))
#include "forward_body.inc"

static void pack(int64_t n, const double *re, const double *im, cplx *z)
{
    for (int64_t i = 0; i < n; i++) z[i] = re[i] + I * im[i];
}
static void unpack(int64_t n, const cplx *z, double *re, double *im)
{
    for (int64_t i = 0; i < n; i++) { re[i] = creal(z[i]); im[i] = cimag(z[i]); }
}

/* One step at fixed dt on the complex state (re, im), in place. */
int ora_cs_step(const ora_problem *P, double *re, double *im, double dt)
{
    const int nv = P->ndim + 2;
    int64_t N = (int64_t)nv * P->ncell;
    cplx *Un = malloc(sizeof(cplx) * N), *Us = malloc(sizeof(cplx) * N), *Uo = malloc(sizeof(cplx) * N);
    if (!Un || !Us || !Uo) { free(Un); free(Us); free(Uo); return ORA_ENOMEM; }
    pack(N, re, im, Un);
    memcpy(Us, Un, sizeof(cplx) * N);
    memcpy(Uo, Un, sizeof(cplx) * N);
    int64_t bad = 0;
    for (int s = 1; s <= P->rk; s++) {
        ora_c_fill_guards(P, Us);
        bad += ora_c_stage(P, s, dt, Un, Us, Uo);
        cplx *t = Us; Us = Uo; Uo = t;
    }
    unpack(N, Us, re, im);
    free(Un); free(Us); free(Uo);
    return bad ? ORA_ENONPHYS : ORA_OK;
}

void ora_cs_eos_n(const ora_problem *P, int64_t n, const double *ur, const double *ui, double *wr, double *wi)
{
    int nv = P->ndim + 2;
    for (int64_t i = 0; i < n; i++) {
        cplx U[5], W[5];
        pack(nv, &ur[nv * i], &ui[nv * i], U);
        ora_c_eos(P, U, W);
        unpack(5, W, &wr[5 * i], &wi[5 * i]);
    }
}

void ora_cs_plm_n(int64_t n, const double *qr, const double *qi, double *mr, double *mi, double *pr, double *pi)
{
    for (int64_t i = 0; i < n; i++) {
        cplx q[3], m, p;
        int code;
        pack(3, &qr[3 * i], &qi[3 * i], q);
        ora_c_plm(q[0], q[1], q[2], &m, &p, &code);
        mr[i] = creal(m); mi[i] = cimag(m); pr[i] = creal(p); pi[i] = cimag(p);
    }
}

void ora_cs_weno5_n(int64_t n, const double *qr, const double *qi, double eps, double *mr, double *mi, double *pr,
                    double *pi)
{
    for (int64_t i = 0; i < n; i++) {
        cplx q[5], m, p;
        pack(5, &qr[5 * i], &qi[5 * i], q);
        ora_c_weno5(q[0], q[1], q[2], q[3], q[4], eps, &m, &p);
        mr[i] = creal(m); mi[i] = cimag(m); pr[i] = creal(p); pi[i] = cimag(p);
    }
}

void ora_cs_hllc_n(const ora_problem *P, int64_t n, int dir, const double *lr, const double *li,
                   const double *rr, const double *ri, double *fr, double *fi)
{
    int nv = P->ndim + 2;
    for (int64_t i = 0; i < n; i++) {
        cplx WL[5], WR[5], F[5];
        int tape;
        pack(5, &lr[5 * i], &li[5 * i], WL);
        pack(5, &rr[5 * i], &ri[5 * i], WR);
        ora_c_hllc(P, WL, WR, dir, F, &tape);
        unpack(nv, F, &fr[nv * i], &fi[nv * i]);
    }
}
