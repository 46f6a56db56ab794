// Device-side building blocks of the FP64 Euler step for gfx950.
//
// Point-wise pieces of the method (the paper's intra-stage chain calcLims ->
// calcFlux -> updSoln -> calcEos, Algorithm "Intra stage calculations for
// Spark"): ideal-gas EOS, MC-limited PLM (van Leer 1977), WENO5-JS (Jiang &
// Shu 1996), HLLC with Davis wave speeds (Toro 2009, Sec. 10.4).  Every
// expression is written in the evaluation order the library fixes for
// bit-reproducibility; the file is compiled with -ffp-contract=off, so an
// fma occurs only where fma() is written.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hydro {

constexpr int kPLM = 0;
constexpr int kWENO = 1;
// optional parts of a stage: gravity source, shock detector
constexpr int kGravity = 1;
constexpr int kShock = 2;

// Geometry of one block as the kernels see it.
struct DevBlock {
    int64_t off;            // first padded cell in a variable plane
    int32_t nx, ny, nz, ng;
    int32_t px, py;         // padded x and y extents
    int32_t gz;             // z guard width (ng in 3D, 0 in 2D)
    int32_t lev;            // refinement level: cell widths dx / 2^lev
    double ix, iy, iz;      // inverse cell widths of the level: (1/dx) 2^lev (exact scaling)
};

// Where the guard layers of one block face are gathered from: the source
// block's padded geometry and the map pos -> A + B*pos of the coordinate
// along the face normal (neighbour interior, periodic wrap, or outflow copy;
// on a face to another refinement level, the block's own guard layers).
// reg >= 0: the fluxes through this face go to flux-register slot reg.
struct FaceSrc {
    int64_t off;
    int32_t px, py;
    int32_t A, B;
    int32_t reg, pad;
};

// A block's faces to other refinement levels: kind 1, one coarser block,
// nbr = {block, o1, o2, -1}; kind 2, the finer blocks, nbr[h1 + 2 h2].
struct DevAmr {
    int32_t kind[6];
    int32_t nbr[6][4];
};

// A work item: an xy tile of one block over a range of z planes.
struct WorkItem {
    int32_t block;
    int32_t xy;      // x0 | y0 << 16
    int32_t z;       // z0 | nz << 16
    int32_t cost;
};

struct Consts {
    double gamma, g1, ig1;
};

__device__ __forceinline__ double dmin(double a, double b) { return (a <= b) ? a : b; }
__device__ __forceinline__ double dmax(double a, double b) { return (a >= b) ? a : b; }

__device__ __forceinline__ int64_t cell_at(const DevBlock &B, int i, int j, int k)
{
    return B.off + ((int64_t)(k + B.gz) * B.py + (j + B.ng)) * B.px + (i + B.ng);
}

// Cell index of (i,j,k) where at most the coordinate along D lies outside
// the block: a face guard is mapped onto the cell it is a copy of.
template <int D, bool GATHER>
__device__ __forceinline__ int64_t src_cell(const DevBlock &B, const FaceSrc *F, int i, int j, int k)
{
    if constexpr (!GATHER) {
        return cell_at(B, i, j, k);
    } else {
        const int pos = (D == 0) ? i : ((D == 1) ? j : k);
        const int n = (D == 0) ? B.nx : ((D == 1) ? B.ny : B.nz);
        if (pos >= 0 && pos < n) return cell_at(B, i, j, k);
        const FaceSrc f = F[2 * D + (pos < 0 ? 0 : 1)];
        const int sp = f.A + f.B * pos;
        int si = i, sj = j, sk = k;
        if (D == 0) si = sp;
        if (D == 1) sj = sp;
        if (D == 2) sk = sp;
        return f.off + ((int64_t)(sk + B.gz) * f.py + (sj + B.ng)) * f.px + (si + B.ng);
    }
}

template <int NDIM>
__device__ __forceinline__ void load_cons(const double *__restrict__ U, int64_t nc, int64_t ci, double (&u)[5])
{
#pragma unroll
    for (int v = 0; v < NDIM + 2; ++v) u[v] = U[v * nc + ci];
}

// Conserved -> primitive (rho, u_x, u_y, u_z, p); returns true if not
// (rho > 0 and p > 0).
template <int NDIM>
__device__ __forceinline__ bool eos(const double (&u)[5], double (&w)[5], double g1)
{
    const double r = 1.0 / u[0];
    w[0] = u[0];
    w[1] = u[1] * r;
    w[2] = u[2] * r;
    double ke;
    if constexpr (NDIM == 3) {
        w[3] = u[3] * r;
        ke = 0.5 * ((u[1] * w[1] + u[2] * w[2]) + u[3] * w[3]);
    } else {
        w[3] = 0.0;
        ke = 0.5 * (u[1] * w[1] + u[2] * w[2]);
    }
    w[4] = g1 * (u[NDIM + 1] - ke);
    return !(w[0] > 0.0 && w[4] > 0.0);
}

// MC-limited linear reconstruction: left-face (qm) and right-face (qp)
// values of the middle cell of (qa, q0, qb).
__device__ __forceinline__ void plm(double qa, double q0, double qb, double &qm, double &qp)
{
    const double dm = q0 - qa, dp = qb - q0;
    // the limited slope, evaluated for every lane and kept where the one-sided
    // differences have the same strict sign (else 0): no divergent branch
    const bool same = (dm > 0.0 && dp > 0.0) || (dm < 0.0 && dp < 0.0);
    const double a = 0.5 * (dm + dp);
    const double aa = fabs(a), m2 = 2.0 * fabs(dm), p2 = 2.0 * fabs(dp);
    // the hardware minimum: where its result is kept, its operands are >= 0
    // and never NaN (the differences passed strict sign tests), and there it
    // equals the (a <= b) ? a : b rule of the method bit for bit
    const double lim = fmin(aa, fmin(m2, p2));
    const double s = same ? copysign(lim, a) : 0.0;
    qp = q0 + 0.5 * s;
    qm = q0 - 0.5 * s;
}

// WENO5-JS on (a,b,c,d,e) = q_{i-2..i+2}; both faces share beta_k.
// Candidates and indicators are evaluated with fused multiply-adds in the
// order written; the weights are alpha_k = d_k / s_k, s_k = (eps + beta_k)^2
// (eps: the problem's weno_eps, 1e-6 in Jiang & Shu),
// scaled by s_0 s_1 s_2 (the normalised weights are unchanged), so the only
// divisions are one per face.
__device__ __forceinline__ void weno5(double a, double b, double c, double d, double e, double eps, double &qm,
                                      double &qp)
{
    const double k13 = 13.0 / 12.0;
    const double c13 = 1.0 / 3.0, c16 = 1.0 / 6.0, c56 = 5.0 / 6.0, c76 = 7.0 / 6.0, c116 = 11.0 / 6.0;
    double t, w;
    t = fma(-2.0, b, a) + c;
    w = fma(3.0, c, fma(-4.0, b, a));
    const double b0 = fma(k13 * t, t, 0.25 * (w * w));
    t = fma(-2.0, c, b) + d;
    w = b - d;
    const double b1 = fma(k13 * t, t, 0.25 * (w * w));
    t = fma(-2.0, d, c) + e;
    w = fma(3.0, c, fma(-4.0, d, e));
    const double b2 = fma(k13 * t, t, 0.25 * (w * w));
    const double s0 = (eps + b0) * (eps + b0);
    const double s1 = (eps + b1) * (eps + b1);
    const double s2 = (eps + b2) * (eps + b2);
    const double o0 = s1 * s2, o1 = s0 * s2, o2 = s0 * s1;
    {
        const double p0 = fma(c116, c, fma(-c76, b, c13 * a));
        const double p1 = fma(c13, d, fma(c56, c, -c16 * b));
        const double p2 = fma(c13, c, fma(c56, d, -c16 * e));
        const double a0 = 0.1 * o0, a1 = 0.6 * o1, a2 = 0.3 * o2;
        qp = fma(a2, p2, fma(a1, p1, a0 * p0)) / ((a0 + a1) + a2);
    }
    {
        const double p0 = fma(c116, c, fma(-c76, d, c13 * e));
        const double p1 = fma(c13, b, fma(c56, c, -c16 * d));
        const double p2 = fma(c13, c, fma(c56, b, -c16 * a));
        const double a0 = 0.1 * o2, a1 = 0.6 * o1, a2 = 0.3 * o0;
        qm = fma(a2, p2, fma(a1, p1, a0 * p0)) / ((a0 + a1) + a2);
    }
}

// Shock detector of the middle cell of a line stencil s (2R+1 cells along
// direction D): compression along D (u_D of the next cell below u_D of the
// previous one) and a pressure jump across the cell larger than thresh times
// the smaller of the two pressures.
template <int D, int R, int S>
__device__ __forceinline__ bool shock_flag(const double (&s)[S][5], double thresh)
{
    const double du = s[R + 1][1 + D] - s[R - 1][1 + D];
    const double pa = s[R - 1][4], pb = s[R + 1][4];
    const double jump = fabs(pb - pa);
    const double lim = thresh * dmin(pa, pb);
    return (du < 0.0) && (jump > lim);
}

// The same along x (y = false) or y (y = true), chosen at run time.
template <int R, int S>
__device__ __forceinline__ bool shock_flag_xy(const double (&s)[S][5], bool y, double thresh)
{
    const double dux = s[R + 1][1] - s[R - 1][1];
    const double duy = s[R + 1][2] - s[R - 1][2];
    const double du = y ? duy : dux;
    const double pa = s[R - 1][4], pb = s[R + 1][4];
    const double jump = fabs(pb - pa);
    const double lim = thresh * dmin(pa, pb);
    return (du < 0.0) && (jump > lim);
}

// Reconstruct all primitives of one cell along a line; s[c][v] is the
// stencil (2R+1 cells).  Applies the positivity fallback (both faces become
// the cell value when either face has non-positive density or pressure);
// a cell the shock detector flagged along this line (shock) takes the same
// first-order faces.  Returns true if the faces are first order.  eps: the
// WENO5 weight epsilon.
template <int NDIM, int RECON, int S>
__device__ __forceinline__ bool recon_cell(const double (&s)[S][5], double (&qm)[5], double (&qp)[5], double eps,
                                           bool shock = false)
{
    constexpr int R = (RECON == kWENO) ? 2 : 1;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        if (NDIM == 2 && v == 3) { qm[v] = 0.0; qp[v] = 0.0; continue; }
        if constexpr (RECON == kWENO)
            weno5(s[R - 2][v], s[R - 1][v], s[R][v], s[R + 1][v], s[R + 2][v], eps, qm[v], qp[v]);
        else
            plm(s[R - 1][v], s[R][v], s[R + 1][v], qm[v], qp[v]);
    }
    const bool fb = shock || !(qm[0] > 0.0 && qm[4] > 0.0) || !(qp[0] > 0.0 && qp[4] > 0.0);
    if (fb) {
#pragma unroll
        for (int v = 0; v < 5; ++v) { qm[v] = s[R][v]; qp[v] = s[R][v]; }
    }
    return fb;
}

// Face state -> conserved U and normal flux F (direction N).
template <int NDIM, int N>
__device__ __forceinline__ void state_flux(const double (&w)[5], double (&u)[5], double (&f)[5], const Consts &K)
{
    const double rho = w[0], p = w[4], un = w[1 + N];
    double ke;
    if constexpr (NDIM == 3)
        ke = 0.5 * (rho * ((w[1] * w[1] + w[2] * w[2]) + w[3] * w[3]));
    else
        ke = 0.5 * (rho * (w[1] * w[1] + w[2] * w[2]));
    const double E = p * K.ig1 + ke;
    u[0] = rho;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) u[1 + d] = rho * w[1 + d];
    u[NDIM + 1] = E;
    const double fr = rho * un;
    f[0] = fr;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) f[1 + d] = (d == N) ? (fr * un) + p : fr * w[1 + d];
    f[NDIM + 1] = (E + p) * un;
}

// The same, also giving 1/rho and the sound speed.
template <int NDIM, int N>
__device__ __forceinline__ void state_flux_rc(const double (&w)[5], double (&u)[5], double (&f)[5], double &r,
                                              double &c, const Consts &K)
{
    state_flux<NDIM, N>(w, u, f, K);
    r = 1.0 / w[0];
    c = sqrt((K.gamma * w[4]) * r);
}

// Flux of the HLLC star region on side K: F*_K = F_K + S_K (U*_K - U_K).
template <int NDIM, int N>
__device__ __forceinline__ void star_flux(const double (&W)[5], const double (&UK)[5], const double (&FK)[5],
                                          double SK, double mK, double rK, double Ss, double (&F)[5])
{
    constexpr int NV = NDIM + 2;
    const double uK = W[1 + N];
    const double chi = mK / (SK - Ss);
    double Us[5];
    Us[0] = chi;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) Us[1 + d] = (d == N) ? chi * Ss : chi * W[1 + d];
    Us[NV - 1] = chi * (UK[NV - 1] * rK + (Ss - uK) * (Ss + W[4] / mK));
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = fma(SK, (Us[v] - UK[v]), FK[v]);
}

// HLLC flux at a face normal to N from left/right primitive states, with
// Davis bounds S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R)
// and the contact speed S*.  Region: S_L >= 0 -> F_L; S* >= 0 -> F*_L;
// S_R > 0 -> F*_R; else F_R.  Every region needs the conserved state and
// flux of one side only (K = L for the first two, R for the others).  With
// ONE_SIDE a lane builds those of its side after the wave speeds and the star
// regions of both sides share one evaluation (fewer instructions and no
// divergent second star flux); otherwise both sides are built and the region
// picks one, which the compiler schedules better in the WENO5 kernels.  Both
// give the same bits.  Returns true if either state is non-physical.
template <int NDIM, int N, bool ONE_SIDE = false>
__device__ __forceinline__ bool hllc(const double (&WL)[5], const double (&WR)[5], double (&F)[5], const Consts &K)
{
    constexpr int NV = NDIM + 2;
    const bool bad = !(WL[0] > 0.0 && WL[4] > 0.0) || !(WR[0] > 0.0 && WR[4] > 0.0);
    const double uL = WL[1 + N], uR = WR[1 + N];
    if constexpr (ONE_SIDE) {
        const double rL = 1.0 / WL[0], rR = 1.0 / WR[0];
        const double cL = sqrt((K.gamma * WL[4]) * rL), cR = sqrt((K.gamma * WR[4]) * rR);
        // hardware min/max: for physical states the speeds are finite and
        // never -0 (c > 0), where they equal the (a <= b) ? a : b rule bit for
        // bit; a non-physical state is reported whatever the flux
        const double SL = fmin(uL - cL, uR - cR);
        const double SR = fmax(uL + cL, uR + cR);
        const double mL = WL[0] * (SL - uL), mR = WR[0] * (SR - uR);
        const double Ss = ((WR[4] - WL[4]) + (mL * uL - mR * uR)) / (mL - mR);
        const bool subL = !(SL >= 0.0);
        const bool right = subL && !(Ss >= 0.0);          // F*_R or F_R
        const bool star = subL && ((Ss >= 0.0) || (SR > 0.0));
        double W[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) W[v] = right ? WR[v] : WL[v];
        double UK[5], FK[5];
        state_flux<NDIM, N>(W, UK, FK, K);
        if (star) {
            star_flux<NDIM, N>(W, UK, FK, right ? SR : SL, right ? mR : mL, right ? rR : rL, Ss, F);
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v] = FK[v];
        }
    } else {
        double UL[5], UR[5], FL[5], FR[5], rL, rR, cL, cR;
        state_flux_rc<NDIM, N>(WL, UL, FL, rL, cL, K);
        state_flux_rc<NDIM, N>(WR, UR, FR, rR, cR, K);
        const double SL = fmin(uL - cL, uR - cR);   // as in the one-sided form
        const double SR = fmax(uL + cL, uR + cR);
        const double mL = WL[0] * (SL - uL), mR = WR[0] * (SR - uR);
        const double Ss = ((WR[4] - WL[4]) + (mL * uL - mR * uR)) / (mL - mR);
        if (SL >= 0.0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v] = FL[v];
        } else if (Ss >= 0.0) {
            star_flux<NDIM, N>(WL, UL, FL, SL, mL, rL, Ss, F);
        } else if (SR > 0.0) {
            star_flux<NDIM, N>(WR, UR, FR, SR, mR, rR, Ss, F);
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v] = FR[v];
        }
    }
    return bad;
}

}  // namespace hydro
