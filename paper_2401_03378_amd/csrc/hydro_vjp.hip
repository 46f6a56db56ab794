// Adjoint (vector-Jacobian product) of one SSP-RK stage on gfx950, with the
// time step held fixed and every branch (limiter slope, positivity fallback,
// HLLC region, Davis min/max argument) taken as the forward step takes it at
// the same state.
//
// A stage is U_{s+1} = b (U_s + dt L(U_s)) + a U^n with
// L = -sum_d (F_{d,i+1/2} - F_{d,i-1/2})/dx_d.  Its transpose splits into
//  k_vjp_lines     one thread per 1D line (or segment of a line, on small
//                  problems) of a block, every direction in one launch,
//                  streaming along it: it recomputes
//                  primitives, reconstruction (with fallback) and the HLLC
//                  branch, then reverses face flux -> face states -> stencil
//                  primitives, and writes the primitive cotangent of every
//                  position the line's stencils read (interior and guard
//                  positions) into a padded array of its own direction, so no
//                  two threads write one element.  Lines along x work on a
//                  transposed copy of their inputs (k_vjp_xpose), so that the
//                  lines of a wave read and write consecutive addresses.
//  k_vjp_cells     one thread per interior cell: sums the arrays of the
//                  directions and line segments that cover it in a fixed
//                  order (x, y, z; segments in order), adds the cotangents of the
//                  guard positions that are copies of the cell (through the
//                  inverse link table; neighbour, periodic and outflow
//                  copies), applies the EOS transpose and forms
//                  gU_s = b gOut + (dW/dU)^T gW, gU^n += a gOut (for the
//                  first stage, whose input is U^n: gU^n += gU_s).
// The guard-fill transpose is thus a deterministic gather, not an atomic
// scatter.
#include "hydro_kernels.h"

namespace hydro {

// ------------------------------------------------------- point-wise VJPs

// 1/x for the derivative arithmetic, which is held to a tolerance, not to the
// forward's bits (values that decide a branch keep correctly rounded
// divisions): the hardware reciprocal estimate refined by two Newton-Raphson
// steps, r <- r + r (1 - x r), each of which squares the relative error.
// Finite non-zero x of moderate exponent only (physical states).
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// Reverse of the wave-speed part of a face state: c = sqrt(gamma p r),
// r = 1/rho (both as the forward computed them), given cotangents gc and gr.
__device__ __forceinline__ void wave_vjp(const double (&w)[5], double r, double c, double gc, double gr,
                                         double (&gW)[5], const Consts &K)
{
    const double p = w[4];
    const double gxg = (gc * rcp_nr(2.0 * c)) * K.gamma;
    gW[4] = fma(gxg, r, gW[4]);
    const double grt = fma(gxg, p, gr);
    gW[0] = fma(-r * r, grt, gW[0]);
}

// Reverse of U and F of a face state (state_flux without c and r).
template <int NDIM, int N>
__device__ __forceinline__ void cons_flux_vjp(const double (&w)[5], const double (&gU)[5], const double (&gF)[5],
                                              double (&gW)[5], const Consts &K)
{
    constexpr int NV = NDIM + 2;
    const double rho = w[0], p = w[4], un = w[1 + N];
    double u2;
    if constexpr (NDIM == 3)
        u2 = (w[1] * w[1] + w[2] * w[2]) + w[3] * w[3];
    else
        u2 = w[1] * w[1] + w[2] * w[2];
    const double E = p * K.ig1 + 0.5 * (rho * u2);
    const double fr = rho * un;
    // the derivative arithmetic in fused multiply-adds
    double gu[3] = {0.0, 0.0, 0.0};
    double gfr = gF[0];
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        gfr = fma(gF[1 + d], w[1 + d], gfr);
        gu[d] = gF[1 + d] * fr;
    }
    double gp = fma(gF[NV - 1], un, gF[1 + N]);
    double gE = fma(gF[NV - 1], un, gU[NV - 1]);
    gu[N] = fma(gF[NV - 1], E + p, fma(gfr, rho, gu[N]));
    double grho = fma(gfr, un, gU[0]);
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        grho = fma(gU[1 + d], w[1 + d], grho);
        gu[d] = fma(gU[1 + d], rho, gu[d]);
    }
    gp = fma(gE, K.ig1, gp);
    grho = fma(gE * 0.5, u2, grho);
    const double gEr = gE * rho;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) gu[d] = fma(gEr, w[1 + d], gu[d]);
    gW[0] += grho;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) gW[1 + d] += gu[d];
    gW[4] += gp;
}

// Reverse of the HLLC flux: recomputes the forward face solution (region and
// Davis arguments included) and accumulates gWL, gWR.  Only the side whose
// U and F enter the flux has them formed and transposed; the other side
// contributes through its wave speed, pressure, density and normal velocity.
template <int NDIM, int N>
__device__ __forceinline__ void hllc_vjp(const double (&WL)[5], const double (&WR)[5], const double (&gF)[5],
                                         double (&gWL)[5], double (&gWR)[5], const Consts &K)
{
    constexpr int NV = NDIM + 2;
    const double rL = 1.0 / WL[0], cL = sqrt((K.gamma * WL[4]) * rL);
    const double rR = 1.0 / WR[0], cR = sqrt((K.gamma * WR[4]) * rR);
    const double uL = WL[1 + N], uR = WR[1 + N];
    const double sl0 = uL - cL, sl1 = uR - cR, sr0 = uL + cL, sr1 = uR + cR;
    if (sl0 <= sl1 ? sl0 >= 0.0 : sl1 >= 0.0) {           // F = F_L
        const double zero[5] = {0, 0, 0, 0, 0};
        cons_flux_vjp<NDIM, N>(WL, zero, gF, gWL, K);
        return;
    }
    const bool slR = !(sl0 <= sl1);
    const bool srR = !(sr0 >= sr1);
    const double SL = slR ? sl1 : sl0, SR = srR ? sr1 : sr0;
    const double mL = WL[0] * (SL - uL), mR = WR[0] * (SR - uR);
    const double Num = (WR[4] - WL[4]) + (mL * uL - mR * uR), Den = mL - mR;
    const double Ss = Num / Den;
    if (!(Ss >= 0.0 || SR > 0.0)) {                       // F = F_R
        const double zero[5] = {0, 0, 0, 0, 0};
        cons_flux_vjp<NDIM, N>(WR, zero, gF, gWR, K);
        return;
    }
    double gcL = 0.0, gcR = 0.0, grL = 0.0, grR = 0.0;
    const bool right = !(Ss >= 0.0);
    const double(&W)[5] = right ? WR : WL;
    double UK[5], FK[5];
    {
        const double rho = W[0], p = W[4], un = W[1 + N];
        double ke;
        if constexpr (NDIM == 3)
            ke = 0.5 * (rho * ((W[1] * W[1] + W[2] * W[2]) + W[3] * W[3]));
        else
            ke = 0.5 * (rho * (W[1] * W[1] + W[2] * W[2]));
        const double E = p * K.ig1 + ke;
        UK[0] = rho;
#pragma unroll
        for (int d = 0; d < NDIM; ++d) UK[1 + d] = rho * W[1 + d];
        UK[NV - 1] = E;
        const double fr = rho * un;
        FK[0] = fr;
#pragma unroll
        for (int d = 0; d < NDIM; ++d) FK[1 + d] = (d == N) ? (fr * un) + p : fr * W[1 + d];
        FK[NV - 1] = (E + p) * un;
    }
    const double SK = right ? SR : SL, mK = right ? mR : mL, rK = right ? rR : rL;
    const double uK = W[1 + N];
    // chi and q enter only derivatives: reciprocals, not divisions
    const double den = SK - Ss, iden = rcp_nr(den), imK = rcp_nr(mK), chi = mK * iden;
    const double q = W[4] * imK;
    const double Bq = UK[NV - 1] * rK + (Ss - uK) * (Ss + q);
    double Us[5];
    Us[0] = chi;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) Us[1 + d] = (d == N) ? chi * Ss : chi * W[1 + d];
    Us[NV - 1] = chi * Bq;
    // the derivative arithmetic in fused multiply-adds
    double gSK = 0.0, gUs[5], gUK[5];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        gSK = fma(gF[v], Us[v] - UK[v], gSK);
        gUs[v] = SK * gF[v];
        gUK[v] = -gUs[v];
    }
    double gWK[5] = {0, 0, 0, 0, 0};
    double gchi = fma(gUs[NV - 1], Bq, fma(gUs[1 + N], Ss, gUs[0]));
#pragma unroll
    for (int d = 0; d < NDIM; ++d)
        if (d != N) {
            gchi = fma(gUs[1 + d], W[1 + d], gchi);
            gWK[1 + d] = gUs[1 + d] * chi;
        }
    const double gB = gUs[NV - 1] * chi;
    gUK[NV - 1] = fma(gB, rK, gUK[NV - 1]);
    const double grK = gB * UK[NV - 1];
    double gSs = fma(gB, (Ss + q) + (Ss - uK), gUs[1 + N] * chi);
    gWK[1 + N] = -(gB * (Ss + q));
    const double gq = gB * (Ss - uK);
    gWK[4] = gq * imK;
    const double gmK = fma(-gq * q, imK, gchi * iden);
    const double gden = -(gchi * chi) * iden;
    gSK += gden;
    gSs -= gden;
    cons_flux_vjp<NDIM, N>(W, gUK, gF, gWK, K);          // F_K + terms through U_K
    double gSL = 0.0, gSR = 0.0, gmL = 0.0, gmR = 0.0;
    if (right) {
        gSR += gSK; gmR += gmK; grR += grK;
#pragma unroll
        for (int v = 0; v < 5; ++v) gWR[v] += gWK[v];
    } else {
        gSL += gSK; gmL += gmK; grL += grK;
#pragma unroll
        for (int v = 0; v < 5; ++v) gWL[v] += gWK[v];
    }
    const double iDen = rcp_nr(Den);
    const double gN = gSs * iDen, gD = -(gSs * Ss) * iDen;
    gWR[4] += gN;
    gWL[4] -= gN;
    gmL += fma(gN, uL, gD);
    gmR -= fma(gN, uR, gD);
    double guL = gN * mL, guR = -(gN * mR);
    gWL[0] = fma(gmL, SL - uL, gWL[0]);
    gSL = fma(gmL, WL[0], gSL);
    guL = fma(-gmL, WL[0], guL);
    gWR[0] = fma(gmR, SR - uR, gWR[0]);
    gSR = fma(gmR, WR[0], gSR);
    guR = fma(-gmR, WR[0], guR);
    if (slR) { guR += gSL; gcR -= gSL; } else { guL += gSL; gcL -= gSL; }
    if (srR) { guR += gSR; gcR += gSR; } else { guL += gSR; gcL += gSR; }
    gWL[1 + N] += guL;
    gWR[1 + N] += guR;
    wave_vjp(WL, rL, cL, gcL, grL, gWL, K);
    wave_vjp(WR, rR, cR, gcR, grR, gWR, K);
}

// Reverse of the limited linear slope of (qa, q0, qb): adds to g[0..2].
__device__ __forceinline__ void plm_vjp(double qa, double q0, double qb, double gqm, double gqp, double *g)
{
    const double dm = q0 - qa, dp = qb - q0;
    const double gs = 0.5 * gqp - 0.5 * gqm;
    double gdm = 0.0, gdp = 0.0;
    if ((dm > 0.0 && dp > 0.0) || (dm < 0.0 && dp < 0.0)) {
        const double a = 0.5 * (dm + dp);
        const double aa = fabs(a), m2 = 2.0 * fabs(dm), p2 = 2.0 * fabs(dp);
        const double side = dmin(m2, p2);
        if (aa <= side) { gdm = 0.5 * gs; gdp = 0.5 * gs; }
        else if (m2 <= p2) gdm = 2.0 * gs;
        else gdp = 2.0 * gs;
    }
    g[0] -= gdm;
    g[1] += gqm + gqp + gdm - gdp;
    g[2] += gdp;
}

// Reverse of WENO5-JS on (a,b,c,d,e): adds to g[0..4].
//
// Forward: beta_k = 13/12 t_k^2 + 1/4 w_k^2, sq_k = eps + beta_k,
// s_k = sq_k^2, o_k = the product of the two other s_j, and per face the
// value sum(d_k o_k p_k) / sum(d_k o_k) of the candidates p_k (the left face
// mirrors the stencil and takes the weights in the order o_2, o_1, o_0).
// The face values are recomputed here for their derivatives only (one
// reciprocal per face), and the derivative arithmetic, which is held to a
// tolerance rather than to the forward's bits, uses fused multiply-adds.
// The recomputed indicators and candidates stay in separate multiplies and
// adds, unlike the forward reconstruction's fused expressions: written alike,
// the compiler would carry the forward's values of a cell over to its
// reverse one position later, which does not fit in the registers of two
// waves per SIMD; and fused in another grouping, their rounding departs
// from the reference reverse's where a candidate nearly equals the face
// value (p_k - q cancels), which costs two to three digits of agreement.
__device__ __forceinline__ void weno5_vjp(const double *q, double eps, double gqm, double gqp, double *g)
{
    const double k13 = 13.0 / 12.0, k6 = 1.0 / 6.0;
    const double a = q[0], b = q[1], c = q[2], d = q[3], e = q[4];
    double t[3], w[3], sq[3], s[3];
    t[0] = (a - 2.0 * b) + c;
    w[0] = (a - 4.0 * b) + 3.0 * c;
    t[1] = (b - 2.0 * c) + d;
    w[1] = b - d;
    t[2] = (c - 2.0 * d) + e;
    w[2] = (3.0 * c - 4.0 * d) + e;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        sq[k] = eps + (k13 * (t[k] * t[k]) + 0.25 * (w[k] * w[k]));
        s[k] = sq[k] * sq[k];
    }
    const double o[3] = {s[1] * s[2], s[0] * s[2], s[0] * s[1]};
    double go0, go1, go2;
    {   // right face; u_k: the cotangents of the candidates p_k over 6
        const double p0 = ((2.0 * a - 7.0 * b) + 11.0 * c) * k6;
        const double p1 = ((-b + 5.0 * c) + 2.0 * d) * k6;
        const double p2 = ((2.0 * c + 5.0 * d) - e) * k6;
        const double a0 = 0.1 * o[0], a1 = 0.6 * o[1], a2 = 0.3 * o[2];
        const double iS = rcp_nr((a0 + a1) + a2);
        const double gS = gqp * iS;
        const double qv = ((a0 * p0 + a1 * p1) + a2 * p2) * iS;
        go0 = (0.1 * gS) * (p0 - qv);
        go1 = (0.6 * gS) * (p1 - qv);
        go2 = (0.3 * gS) * (p2 - qv);
        const double gSk = gS * k6;
        const double u0 = gSk * a0, u1 = gSk * a1, u2 = gSk * a2;
        g[0] = fma(2.0, u0, g[0]);
        g[1] = g[1] - fma(7.0, u0, u1);
        g[2] = fma(11.0, u0, fma(5.0, u1, fma(2.0, u2, g[2])));
        g[3] = fma(2.0, u1, fma(5.0, u2, g[3]));
        g[4] = g[4] - u2;
    }
    {   // left face: mirrored candidates, weights (0.1 o2, 0.6 o1, 0.3 o0)
        const double p0 = ((2.0 * e - 7.0 * d) + 11.0 * c) * k6;
        const double p1 = ((-d + 5.0 * c) + 2.0 * b) * k6;
        const double p2 = ((2.0 * c + 5.0 * b) - a) * k6;
        const double a0 = 0.1 * o[2], a1 = 0.6 * o[1], a2 = 0.3 * o[0];
        const double iS = rcp_nr((a0 + a1) + a2);
        const double gS = gqm * iS;
        const double qv = ((a0 * p0 + a1 * p1) + a2 * p2) * iS;
        go2 = fma(0.1 * gS, p0 - qv, go2);
        go1 = fma(0.6 * gS, p1 - qv, go1);
        go0 = fma(0.3 * gS, p2 - qv, go0);
        const double gSk = gS * k6;
        const double u0 = gSk * a0, u1 = gSk * a1, u2 = gSk * a2;
        g[4] = fma(2.0, u0, g[4]);
        g[3] = g[3] - fma(7.0, u0, u1);
        g[2] = fma(11.0, u0, fma(5.0, u1, fma(2.0, u2, g[2])));
        g[1] = fma(2.0, u1, fma(5.0, u2, g[1]));
        g[0] = g[0] - u2;
    }
    // o -> s -> beta: beta_k receives 2 sq_k gs_k (gs_k: the cotangent of
    // s_k); with G_k = sq_k gs_k, t_k receives 4 k13 t_k G_k and w_k w_k G_k
    const double G0 = sq[0] * fma(go1, s[2], go2 * s[1]);
    const double G1 = sq[1] * fma(go0, s[2], go2 * s[0]);
    const double G2 = sq[2] * fma(go0, s[1], go1 * s[0]);
    const double k4 = 4.0 * k13;
    const double gt0 = (k4 * t[0]) * G0, gw0 = w[0] * G0;
    const double gt1 = (k4 * t[1]) * G1, gw1 = w[1] * G1;
    const double gt2 = (k4 * t[2]) * G2, gw2 = w[2] * G2;
    // the indicators' stencils: t_0 = a - 2b + c, w_0 = a - 4b + 3c,
    // t_1 = b - 2c + d, w_1 = b - d, t_2 = c - 2d + e, w_2 = 3c - 4d + e
    g[0] = g[0] + (gt0 + gw0);
    g[1] = fma(-2.0, gt0, fma(-4.0, gw0, g[1] + (gt1 + gw1)));
    g[2] = fma(-2.0, gt1, fma(3.0, gw0 + gw2, g[2] + (gt0 + gt2)));
    g[3] = fma(-2.0, gt2, fma(-4.0, gw2, g[3] + (gt1 - gw1)));
    g[4] = g[4] + (gt2 + gw2);
}

// Reverse of one cell's reconstruction along a line: s[c][v] stencil
// (2R+1 cells); fb: the positivity fallback fired (faces = cell value).
template <int NDIM, int RECON, int S>
__device__ __forceinline__ void recon_cell_vjp(const double (&s)[S][5], bool fb, const double (&gqm)[5],
                                               const double (&gqp)[5], double (&g)[S][5], double eps)
{
    constexpr int R = (RECON == kWENO) ? 2 : 1;
    if (fb) {
#pragma unroll
        for (int v = 0; v < 5; ++v) g[R][v] += gqm[v] + gqp[v];
        return;
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        if (NDIM == 2 && v == 3) continue;
        double st[2 * R + 1], gs[2 * R + 1];
#pragma unroll
        for (int k = 0; k < 2 * R + 1; ++k) { st[k] = s[k][v]; gs[k] = 0.0; }
        if constexpr (RECON == kWENO)
            weno5_vjp(st, eps, gqm[v], gqp[v], gs);
        else
            plm_vjp(st[0], st[1], st[2], gqm[v], gqp[v], gs);
#pragma unroll
        for (int k = 0; k < 2 * R + 1; ++k) g[k][v] += gs[k];
    }
}

// primitive slot of the padded cotangent array: rho, u_1..u_nd, p
template <int NDIM>
__device__ __forceinline__ int wslot(int v) { return v == 4 ? NDIM + 1 : v; }

// Segments of a line: a line of n cells (faces 0..n) is cut into k segments
// of L = ceil(n/k) faces; segment s owns faces [f0, f1] and writes the
// cotangents of positions [f0-1-R, f1+R] into its own array.  k is the
// requested count, reduced so every segment spans at least 2R+1 cells.
template <int R>
__device__ __forceinline__ int seg_count(int n, int nseg)
{
    const int cap = n / (2 * R + 1);
    return max(1, min(nseg, cap));
}

template <int R>
__device__ __forceinline__ void seg_range(int n, int k, int s, int &f0, int &f1)
{
    const int L = (n + k - 1) / k;
    f0 = (s == 0) ? 0 : s * L + 1;
    f1 = min((s + 1) * L, n);
}

// Lines along x are read and written in a transposed order: element
// (p, j, k) of block B, p in [-H, nx+H), sits at
// off + (k (nx + 2H) + p + H) ny + j, so the lines of one wave (consecutive
// j) touch consecutive addresses.  The block's padded footprint holds this
// (H <= ng), so the transposed arrays share the state's block offsets.
template <int H>
__device__ __forceinline__ int64_t xt_at(const DevBlock &B, int p, int j, int k)
{
    return B.off + ((int64_t)k * (B.nx + 2 * H) + (p + H)) * B.ny + j;
}

// ------------------------------------------------------------ line kernel

template <int D>
__device__ __forceinline__ void line_coords(int t, int e1, int e2, int &i, int &j, int &k)
{
    if (D == 0) { i = t; j = e1; k = e2; }
    else if (D == 1) { i = e1; j = t; k = e2; }
    else { i = e1; j = e2; k = t; }
}

template <int NDIM, int RECON, int D, bool SHOCK>
__device__ __forceinline__ void vjp_line(const VjpArgs &A, const WorkItem &it, int lane)
{
    constexpr int R = (RECON == kWENO) ? 2 : 1;
    constexpr int H = R + 1;
    constexpr int NV = NDIM + 2;
    constexpr int NS = 2 * R + 1;     // stencil
    constexpr int NWIN = 2 * R + 2;   // primitives at positions t-2R-1 .. t
    const int nl = it.z;               // lines in this item
    if (lane >= nl) return;
    const int seg = it.cost >> 4;
    const DevBlock B = A.blocks[it.block];
    const FaceSrc *F6 = A.faces + 6 * (int64_t)it.block;
    const int L = it.xy + lane;
    const int n1 = (D == 0) ? B.ny : B.nx;
    const int e1 = L % n1, e2 = L / n1;
    const int n = (D == 0) ? B.nx : ((D == 1) ? B.ny : B.nz);
    const int64_t nc = A.nc;
    const Consts K{A.gamma, A.g1, A.ig1};
    const double dt = *A.dt;
    const double id = (D == 0) ? A.idx : ((D == 1) ? A.idy : A.idz);
    const int kseg = seg_count<R>(n, A.nseg);
    if (seg >= kseg) return;
    int f0, f1;
    seg_range<R>(n, kseg, seg, f0, f1);
    if (f0 > f1) return;

    double Wwin[NWIN][5];
    double gWwin[NS][5];
    double qp_prev[5], gqm_prev[5], gD_prev[5];
    bool fb_prev = false;
#pragma unroll
    for (int c = 0; c < NWIN; ++c)
#pragma unroll
        for (int v = 0; v < 5; ++v) Wwin[c][v] = 0.0;
#pragma unroll
    for (int c = 0; c < NS; ++c)
#pragma unroll
        for (int v = 0; v < 5; ++v) gWwin[c][v] = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) { qp_prev[v] = 0.0; gqm_prev[v] = 0.0; gD_prev[v] = 0.0; }
    if (f0 >= 1) {        // flux difference of the cell left of the first face
        int i, j, k;
        line_coords<D>(f0 - 1, e1, e2, i, j, k);
        const int64_t ci = (D == 0) ? xt_at<H>(B, i, j, k) : cell_at(B, i, j, k);
        const double *gO = (D == 0) ? A.gOutT : A.gOut;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double gT = A.b * gO[v * nc + ci];
            gD_prev[v] = -(dt * gT) * id;
        }
    }

    double *gWd = A.gW + ((int64_t)D * A.nseg + seg) * NV * nc;   // this direction's and segment's array
    auto emit = [&](int p, const double (&gw)[5]) {
        int i, j, k;
        line_coords<D>(p, e1, e2, i, j, k);
        const int64_t ci = (D == 0) ? xt_at<H>(B, i, j, k) : cell_at(B, i, j, k);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            if (NDIM == 2 && v == 3) continue;
            gWd[(int64_t)wslot<NDIM>(v) * nc + ci] = gw[v];
        }
    };

    for (int t = f0 - H; t <= f1 + R; ++t) {
        // primitives at the new position
#pragma unroll
        for (int c = 0; c < NWIN - 1; ++c)
#pragma unroll
            for (int v = 0; v < 5; ++v) Wwin[c][v] = Wwin[c + 1][v];
        {
            int i, j, k;
            line_coords<D>(t, e1, e2, i, j, k);
            double u[5];
            if constexpr (D == 0)
                load_cons<NDIM>(A.UsT, nc, xt_at<H>(B, i, j, k), u);
            else
                load_cons<NDIM>(A.Us, nc, src_cell<D, true>(B, F6, i, j, k), u);
            eos<NDIM>(u, Wwin[NWIN - 1], K.g1);
        }
        const int c = t - R;          // reconstruction cell completed by this position
        if (c >= f0 - 1) {
            double s[NS][5], qm[5], qp[5];
#pragma unroll
            for (int q = 0; q < NS; ++q)
#pragma unroll
                for (int v = 0; v < 5; ++v) s[q][v] = Wwin[q + 1][v];
            // the forward's branches: positivity fallback and (SHOCK) the detector's flag
            const bool fb = recon_cell<NDIM, RECON>(s, qm, qp, A.eps, SHOCK && shock_flag<D, R>(s, A.sthresh));
            double gqp_c1[5] = {0, 0, 0, 0, 0}, gqm_c[5] = {0, 0, 0, 0, 0};
            if (c >= f0) {
                // cotangent of face c-1/2: gD_{c-1} - gD_c
                double gD[5] = {0, 0, 0, 0, 0};
                if (c < n) {
                    int i, j, k;
                    line_coords<D>(c, e1, e2, i, j, k);
                    const int64_t ci = (D == 0) ? xt_at<H>(B, i, j, k) : cell_at(B, i, j, k);
                    const double *gO = (D == 0) ? A.gOutT : A.gOut;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const double gT = A.b * gO[v * nc + ci];
                        gD[v] = -(dt * gT) * id;
                    }
                }
                double gF[5] = {0, 0, 0, 0, 0};
#pragma unroll
                for (int v = 0; v < NV; ++v) gF[v] = gD_prev[v] - gD[v];
                hllc_vjp<NDIM, D>(qp_prev, qm, gF, gqp_c1, gqm_c, K);
#pragma unroll
                for (int v = 0; v < 5; ++v) gD_prev[v] = gD[v];
                // cell c-1 now has both face cotangents
                double s1[NS][5], g1[NS][5];
#pragma unroll
                for (int q = 0; q < NS; ++q)
#pragma unroll
                    for (int v = 0; v < 5; ++v) { s1[q][v] = Wwin[q][v]; g1[q][v] = 0.0; }
                recon_cell_vjp<NDIM, RECON>(s1, fb_prev, gqm_prev, gqp_c1, g1, A.eps);
#pragma unroll
                for (int q = 0; q < NS; ++q)
#pragma unroll
                    for (int v = 0; v < 5; ++v) gWwin[q][v] += g1[q][v];
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) { qp_prev[v] = qp[v]; gqm_prev[v] = gqm_c[v]; }
            fb_prev = fb;
        }
        // position t-2R-1 receives nothing more
        const int pout = t - 2 * R - 1;
        if (pout >= f0 - H) emit(pout, gWwin[0]);
#pragma unroll
        for (int q = 0; q < NS - 1; ++q)
#pragma unroll
            for (int v = 0; v < 5; ++v) gWwin[q][v] = gWwin[q + 1][v];
#pragma unroll
        for (int v = 0; v < 5; ++v) gWwin[NS - 1][v] = 0.0;
    }
    // last reconstruction cell (f1): its right face is not this segment's
    {
        double s1[NS][5], g1[NS][5];
        const double zero[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
            for (int v = 0; v < 5; ++v) { s1[q][v] = Wwin[q + 1][v]; g1[q][v] = 0.0; }
        recon_cell_vjp<NDIM, RECON>(s1, fb_prev, gqm_prev, zero, g1, A.eps);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
#pragma unroll
            for (int v = 0; v < 5; ++v) gWwin[q][v] += g1[q][v];
            emit(f1 - R + q, gWwin[q]);
        }
    }
}

// One launch for every direction and segment: work item cost field =
// direction | segment << 4.  SHOCK: the shock detector's flags are among the
// branches the reverse pass follows.
template <int NDIM, int RECON, bool SHOCK>
__global__ void __launch_bounds__(64) k_vjp_lines(VjpArgs A)
{
    const WorkItem it = A.items[blockIdx.x];
    const int dir = it.cost & 15;
    if (dir == 0) vjp_line<NDIM, RECON, 0, SHOCK>(A, it, threadIdx.x);
    else if (dir == 1) vjp_line<NDIM, RECON, 1, SHOCK>(A, it, threadIdx.x);
    else if constexpr (NDIM == 3) vjp_line<NDIM, RECON, 2, SHOCK>(A, it, threadIdx.x);
}

// ------------------------------------------------------------ cell kernel

// Reverse of the EOS at one cell: gU (nvar) = (dW/dU)^T gW.
template <int NDIM>
__device__ __forceinline__ void eos_vjp(const double (&u)[5], const double (&gw)[5], double (&gu)[5], double g1)
{
    const double r = 1.0 / u[0];
    const double gke = -g1 * gw[4];
    double gr = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) gu[v] = 0.0;
    gu[NDIM + 1] = g1 * gw[4];
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        const double ud = u[1 + d] * r;
        const double g = gw[1 + d] + 0.5 * u[1 + d] * gke;
        gu[1 + d] = 0.5 * ud * gke + r * g;
        gr += u[1 + d] * g;
    }
    gu[0] = gw[0] - r * r * gr;
}

template <int NDIM, int H, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_vjp_cells(VjpArgs A)
{
    constexpr int NV = NDIM + 2;
    constexpr int R = H - 1;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int64_t nc = A.nc;
    const int64_t astride = (int64_t)NV * nc;
    // sum of the segment arrays of direction d whose ranges contain position p
    auto seg_sum = [&](const DevBlock &X, int d, int p, int64_t cell, double (&gw)[5]) {
        const int n = (d == 0) ? X.nx : ((d == 1) ? X.ny : X.nz);
        const int k = seg_count<R>(n, A.nseg);
        for (int s = 0; s < k; ++s) {
            int f0, f1;
            seg_range<R>(n, k, s, f0, f1);
            if (f0 > f1 || p < f0 - 1 - R || p > f1 + R) continue;
            const double *g = A.gW + ((int64_t)d * A.nseg + s) * astride;
#pragma unroll
            for (int v = 0; v < NV; ++v) gw[v == NDIM + 1 ? 4 : v] += g[v * nc + cell];
        }
    };
    for (int w = blockIdx.x; w < A.ncitems; w += gridDim.x) {
        const WorkItem it = A.citems[w];
        const DevBlock B = A.blocks[it.block];
        const int x0 = it.xy & 0xffff, y0 = it.xy >> 16;
        const int z0 = it.z & 0xffff, nzc = it.z >> 16;
        const int i = x0 + tx, j = y0 + ty;
        if (i >= B.nx || j >= B.ny) continue;
        const int inc0 = A.inc_start[it.block], inc1 = A.inc_start[it.block + 1];
        for (int k = z0; k < z0 + nzc; ++k) {
            const int64_t ci = cell_at(B, i, j, k);
            // the cell's own operands first, so their loads overlap the sums below
            double u[5], go[5], gn[5];
            load_cons<NDIM>(A.Us, nc, ci, u);
#pragma unroll
            for (int v = 0; v < NV; ++v) go[v] = A.gOut[v * nc + ci];
            if (A.gUn) {
#pragma unroll
                for (int v = 0; v < NV; ++v) gn[v] = A.gUn[v * nc + ci];
            }
            double gw[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) gw[v] = 0.0;
            if (A.nseg == 1) {
                // one segment per line: every direction's array covers the cell;
                // all loads issued before the sums (same order of additions)
                double gd[NDIM][NV];
                const int64_t xi = xt_at<H>(B, i, j, k);
#pragma unroll
                for (int d = 0; d < NDIM; ++d)
#pragma unroll
                    for (int v = 0; v < NV; ++v) gd[d][v] = A.gW[(int64_t)d * astride + v * nc + (d == 0 ? xi : ci)];
#pragma unroll
                for (int d = 0; d < NDIM; ++d)
#pragma unroll
                    for (int v = 0; v < NV; ++v) gw[v == NDIM + 1 ? 4 : v] += gd[d][v];
            } else {
                seg_sum(B, 0, i, xt_at<H>(B, i, j, k), gw);
                seg_sum(B, 1, j, ci, gw);
                if constexpr (NDIM == 3) seg_sum(B, 2, k, ci, gw);
            }
            // guard positions (of this or other blocks) that copy this cell
            for (int e = inc0; e < inc1; ++e) {
                const int4 q = A.inc[e];                 // x = block, y = dir, z = side, w = kind
                const DevBlock &X = A.blocks[q.x];    // read in place: a local copy with fields picked at run time would go to LDS
                const int d = q.y;
                const int pos = (d == 0) ? i : ((d == 1) ? j : k);
                const int nb = (d == 0) ? B.nx : ((d == 1) ? B.ny : B.nz);
                const int nx_ = (d == 0) ? X.nx : ((d == 1) ? X.ny : X.nz);
                int lo = 1, hi = 0, gp0 = 0, step = 0;
                if (q.w == 0) {                          // copy: layer l <-> one position
                    if (q.z == 0) { const int l = nb - pos; if (l >= 1 && l <= H) { lo = hi = l; } gp0 = 0; step = -1; }
                    else { const int l = pos + 1; if (l <= H) { lo = hi = l; } gp0 = nx_ - 1; step = 1; }
                } else {                                 // outflow: every layer copies the boundary cell
                    if (q.z == 0 && pos == 0) { lo = 1; hi = H; gp0 = 0; step = -1; }
                    if (q.z == 1 && pos == nb - 1) { lo = 1; hi = H; gp0 = nx_ - 1; step = 1; }
                }
                for (int l = lo; l <= hi; ++l) {
                    const int gpos = gp0 + step * l;
                    const int gi = (d == 0) ? gpos : i, gj = (d == 1) ? gpos : j, gk = (d == 2) ? gpos : k;
                    seg_sum(X, d, gpos, (d == 0) ? xt_at<H>(X, gi, gj, gk) : cell_at(X, gi, gj, gk), gw);
                }
            }
            double gu[5];
            eos_vjp<NDIM>(u, gw, gu, A.g1);
            // gravity source: T_{m_d} gains dt rho g_d and T_E gains dt (m . g)
            const bool grv = (A.phys & kGravity) != 0;
            double gsrc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (grv) {
                const double dtv = *A.dt;
                const double gTE = A.b * go[NV - 1];
#pragma unroll
                for (int d = 0; d < NDIM; ++d) {
                    const double gTm = A.b * go[1 + d];
                    gsrc[0] += dtv * (A.grav[d] * gTm);
                    gsrc[1 + d] = dtv * (A.grav[d] * gTE);
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double gs = A.b * go[v] + gu[v];
                if (grv) gs = gs + gsrc[v];
                if (A.last) {
                    A.gUn[v * nc + ci] = gn[v] + gs;
                } else {
                    A.gUs[v * nc + ci] = gs;
                    if (A.gUn) A.gUn[v * nc + ci] = gn[v] + A.a * go[v];
                }
            }
        }
    }
}

// Stage input and output cotangent of every block in the transposed x-line
// order (see xt_at): Us at positions -H .. nx+H-1, guard positions gathered
// from their sources, and gOut at the interior positions.  A workgroup takes
// a 16-position x 16-row tile of one plane through LDS, reading along x and
// writing along y.
template <int NDIM, int H>
__global__ void __launch_bounds__(256) k_vjp_xpose(VjpArgs A)
{
    constexpr int NV = NDIM + 2;
    __shared__ double sU[NV][16][17];
    __shared__ double sG[NV][16][17];
    const int tid = threadIdx.x;
    const int64_t nc = A.nc;
    for (int w = blockIdx.x; w < A.nxitems; w += gridDim.x) {
        const WorkItem it = A.xitems[w];
        const DevBlock B = A.blocks[it.block];
        const FaceSrc *F6 = A.faces + 6 * (int64_t)it.block;
        const int p0 = (it.xy & 0xffff) - H, j0 = it.xy >> 16, k = it.z;
        {
            const int tp = tid % 16, tj = tid / 16;
            const int p = p0 + tp, j = j0 + tj;
            if (p < B.nx + H && j < B.ny) {
                const int64_t src = src_cell<0, true>(B, F6, p, j, k);
#pragma unroll
                for (int v = 0; v < NV; ++v) sU[v][tj][tp] = A.Us[v * nc + src];
                if (p >= 0 && p < B.nx) {
                    const int64_t ci = cell_at(B, p, j, k);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sG[v][tj][tp] = A.gOut[v * nc + ci];
                }
            }
        }
        __syncthreads();
        {
            const int tj = tid % 16, tp = tid / 16;
            const int p = p0 + tp, j = j0 + tj;
            if (p < B.nx + H && j < B.ny) {
                const int64_t ti = xt_at<H>(B, p, j, k);
#pragma unroll
                for (int v = 0; v < NV; ++v) A.UsT[v * nc + ti] = sU[v][tj][tp];
                if (p >= 0 && p < B.nx) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) A.gOutT[v * nc + ti] = sG[v][tj][tp];
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- launchers

hipError_t launch_vjp_xpose(const VjpArgs &a, int ndim, int recon, hipStream_t st)
{
    if (a.nxitems <= 0) return hipSuccess;
    if (ndim == 3) {
        if (recon == kWENO) k_vjp_xpose<3, 3><<<a.nxitems, 256, 0, st>>>(a);
        else k_vjp_xpose<3, 2><<<a.nxitems, 256, 0, st>>>(a);
    } else {
        if (recon == kWENO) k_vjp_xpose<2, 3><<<a.nxitems, 256, 0, st>>>(a);
        else k_vjp_xpose<2, 2><<<a.nxitems, 256, 0, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_lines(const VjpArgs &a, int ndim, int recon, int nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    const bool shock = (a.phys & kShock) != 0;
    if (ndim == 3) {
        if (recon == kWENO) {
            if (shock) k_vjp_lines<3, kWENO, true><<<nitems, 64, 0, st>>>(a);
            else k_vjp_lines<3, kWENO, false><<<nitems, 64, 0, st>>>(a);
        } else {
            if (shock) k_vjp_lines<3, kPLM, true><<<nitems, 64, 0, st>>>(a);
            else k_vjp_lines<3, kPLM, false><<<nitems, 64, 0, st>>>(a);
        }
    } else {
        if (recon == kWENO) {
            if (shock) k_vjp_lines<2, kWENO, true><<<nitems, 64, 0, st>>>(a);
            else k_vjp_lines<2, kWENO, false><<<nitems, 64, 0, st>>>(a);
        } else {
            if (shock) k_vjp_lines<2, kPLM, true><<<nitems, 64, 0, st>>>(a);
            else k_vjp_lines<2, kPLM, false><<<nitems, 64, 0, st>>>(a);
        }
    }
    return hipGetLastError();
}

hipError_t launch_vjp_cells(const VjpArgs &a, int ndim, int recon, int grid, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    if (ndim == 3) {
        if (recon == kWENO) k_vjp_cells<3, 3, 16, 4><<<grid, 64, 0, st>>>(a);
        else k_vjp_cells<3, 2, 16, 4><<<grid, 64, 0, st>>>(a);
    } else {
        if (recon == kWENO) k_vjp_cells<2, 3, 16, 4><<<grid, 64, 0, st>>>(a);
        else k_vjp_cells<2, 2, 16, 4><<<grid, 64, 0, st>>>(a);
    }
    return hipGetLastError();
}

}  // namespace hydro
