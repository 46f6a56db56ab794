// hydro_cfl_dt_noalloc: the CFL time step without a context and without any
// device allocation.  The per-block maxima of the wave-speed sum live in a
// file-scope device array of the library (one copy per GPU, resolved with
// hipGetSymbolAddress on the first call on a device) instead of a context's
// partial-reduction buffer.
#include <cmath>
#include <mutex>
#include <string>

#include "hydro.h"
#include "hydro_common.h"

using namespace hydro;

// One double per block: the maximum of the block's wave-speed sum, or NaN
// when the block's descriptor is out of range or one of its cells is
// non-physical.  Shared by every call on a GPU; each call writes the first
// nblocks entries before reading them, so nothing needs clearing.
static __device__ __align__(256) double scratch[HYDRO_NOALLOC_MAX_BLOCKS];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double *g_scratch_dev[kMaxDevices] = {};   // device address of `scratch` per device

// One workgroup per block: the largest sum_d (|u_d| + c) / dx_d over the
// block's interior cells, the expression of the context's CFL kernels in
// the same order.  The descriptor is checked before any cell is read.
template <int NDIM>
__global__ void __launch_bounds__(256) k_cfl_blocks(const hydro_block_t *__restrict__ blocks, int64_t nc,
                                                    double gamma, double g1, double idx, double idy, double idz,
                                                    const double *__restrict__ U, double *__restrict__ part)
{
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const hydro_block_t B = blocks[blockIdx.x];
    // extents bounded as hydro_validate bounds them, so the padded sizes below
    // cannot overflow
    constexpr int32_t kMaxExtent = 32767;
    bool ok = B.nx >= 1 && B.ny >= 1 && B.nz >= 1 && B.nx <= kMaxExtent && B.ny <= kMaxExtent &&
              B.nz <= kMaxExtent && B.ng >= 0 && B.ng <= kMaxExtent && B.offset >= 0 && B.offset < nc &&
              (NDIM == 3 || B.nz == 1);
    const int64_t gz = (NDIM == 3) ? B.ng : 0;
    const int64_t px = (int64_t)B.nx + 2 * (int64_t)B.ng, py = (int64_t)B.ny + 2 * (int64_t)B.ng;
    const int64_t pz = (int64_t)B.nz + 2 * gz;
    if (ok) ok = (nc - B.offset) / (px * py) >= pz;   // offset + px py pz <= nc, without overflow
    double m = 0.0;
    bool bad = !ok;
    if (ok) {
        const int64_t ncell = (int64_t)B.nx * B.ny * B.nz;
        for (int64_t q = tid; q < ncell; q += 256) {
            const int i = (int)(q % B.nx);
            const int64_t r = q / B.nx;
            const int j = (int)(r % B.ny);
            const int k = (int)(r / B.ny);
            const int64_t ci = B.offset + ((k + gz) * py + (j + B.ng)) * px + (i + B.ng);
            double u[5], wv[5];
            load_cons<NDIM>(U, nc, ci, u);
            bad |= eos<NDIM>(u, wv, g1);
            const double rr = 1.0 / u[0];
            const double c = sqrt((gamma * wv[4]) * rr);
            double sig = ((fabs(wv[1]) + c) * idx) + ((fabs(wv[2]) + c) * idy);
            if constexpr (NDIM == 3) sig = sig + ((fabs(wv[3]) + c) * idz);
            m = (sig > m) ? sig : m;
        }
    }
    for (int s = 32; s > 0; s >>= 1) {
        const double o = __shfl_xor(m, s, 64);
        m = (o > m) ? o : m;
    }
    if ((tid & 63) == 0) red[tid >> 6] = m;
    const int anybad = __syncthreads_or(bad ? 1 : 0);
    if (tid == 0) {
        for (int q = 1; q < 4; ++q) m = (red[q] > m) ? red[q] : m;
        part[blockIdx.x] = anybad ? __builtin_nan("") : m;
    }
}

// dt = cfl / (largest block maximum); NaN if any block reported NaN.
__global__ void __launch_bounds__(256) k_cfl_blocks_final(const double *__restrict__ part, int n, double cfl,
                                                          double *__restrict__ dt)
{
    __shared__ double red[4];
    const int tid = threadIdx.x;
    double m = 0.0;
    bool nan = false;
    for (int q = tid; q < n; q += 256) {
        const double v = part[q];
        nan |= (v != v);
        m = (v > m) ? v : m;
    }
    for (int s = 32; s > 0; s >>= 1) {
        const double o = __shfl_xor(m, s, 64);
        m = (o > m) ? o : m;
    }
    if ((tid & 63) == 0) red[tid >> 6] = m;
    const int anynan = __syncthreads_or(nan ? 1 : 0);
    if (tid == 0) {
        for (int q = 1; q < 4; ++q) m = (red[q] > m) ? red[q] : m;
        *dt = anynan ? __builtin_nan("") : cfl / m;
    }
}

}  // namespace


extern "C" {

extern thread_local std::string g_noctx_err;   // defined with hydro_last_error

int hydro_cfl_dt_noalloc(const hydro_params_t *params, const hydro_block_t *blocks_dev, int32_t nblocks,
                         int64_t ncell_total, const double *U, double *dt_dev, void *stream)
{
    auto fail = [](int code, const char *msg) {
        g_noctx_err = msg;
        return code;
    };
    if (!params || !blocks_dev || !U || !dt_dev) return fail(HYDRO_EINVAL, "null argument");
    const hydro_params_t &p = *params;
    if (p.ndim != 2 && p.ndim != 3) return fail(HYDRO_EINVAL, "ndim must be 2 or 3");
    if (!(p.gamma > 1.0) || !std::isfinite(p.gamma)) return fail(HYDRO_EINVAL, "gamma must be finite and > 1");
    if (!(p.cfl > 0.0) || !std::isfinite(p.cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0");
    if (!(p.dx > 0.0) || !(p.dy > 0.0) || !(p.dz > 0.0)) return fail(HYDRO_EINVAL, "cell widths must be > 0");
    if (nblocks < 1) return fail(HYDRO_EINVAL, "no blocks: no cell bounds the step");
    if (nblocks > HYDRO_NOALLOC_MAX_BLOCKS) return fail(HYDRO_EINVAL, "more blocks than HYDRO_NOALLOC_MAX_BLOCKS");
    if (ncell_total < 1) return fail(HYDRO_EINVAL, "ncell_total must be >= 1");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(HYDRO_EHIP, "no HIP device");
    if (dev < 0 || dev >= kMaxDevices) return fail(HYDRO_EINVAL, "device index beyond the library's table");
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[dev]) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) {
                g_noctx_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
                return HYDRO_EHIP;
            }
            g_scratch_dev[dev] = static_cast<double *>(ptr);
        }
        part = g_scratch_dev[dev];
    }
    hipStream_t st = (hipStream_t)stream;
    const double idx = std::ldexp(1.0 / p.dx, 0), idy = std::ldexp(1.0 / p.dy, 0), idz = std::ldexp(1.0 / p.dz, 0);
    if (p.ndim == 3)
        k_cfl_blocks<3><<<nblocks, 256, 0, st>>>(blocks_dev, ncell_total, p.gamma, p.gamma - 1.0, idx, idy, idz, U,
                                                 part);
    else
        k_cfl_blocks<2><<<nblocks, 256, 0, st>>>(blocks_dev, ncell_total, p.gamma, p.gamma - 1.0, idx, idy, idz, U,
                                                 part);
    k_cfl_blocks_final<<<1, 256, 0, st>>>(part, nblocks, p.cfl, dt_dev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_noctx_err = std::string("cfl launch: ") + hipGetErrorString(e);
        return HYDRO_EHIP;
    }
    return HYDRO_OK;
}

}  // extern "C"
