// spmv_rm.hip -- launcher of the SpMV for right-hand sides stored row by
// row (element (i, r) at X[i*ldx + r]): one workgroup per row tile
// (spmv_tile_rm.h), tiles optionally regrouped over the 8 XCDs.
#include "internal.h"
#include "spmv_tile_rm.h"

namespace mhdc {
namespace {

using KernelFn = void (*)(SpmvArgs);

// Row-major right-hand sides: one tile of WG rows per workgroup.  256-lane
// tiles are held to four waves per SIMD, what their LDS allows (at 16
// columns with both parts the compiler took 132 VGPRs and three fitted; the
// cap costs a 20-byte spill and took the partially diagonal 192^3 case at
// 16 columns from 2.47 to 2.13 ms).  64-lane tiles are LDS-bound at one.
template <int WG, int KC, bool HAS_DIA, bool HAS_REM, bool RG>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WG == 256 ? 4 : 1, 8))) void k_spmm_rm(SpmvArgs a)
{
    __shared__ double s_lds[HAS_REM ? (TileShapeRm<WG, KC>::LDS_BYTES + 7) / 8 : 1];
    const int tile = a.remap ? xcd_tile(blockIdx.x, gridDim.x, a.remap) : (int)blockIdx.x;
    spmv_tile_rm<WG, KC, HAS_DIA, HAS_REM, RG>(a, tile, s_lds);
}

// parts: 1 = DIA part, 2 = CSR part, 4 = CSR part by row gathers
template <int WG, int KC>
KernelFn pick_rm_parts(int parts)
{
    switch (parts) {
    case 1:
    case 5: return (KernelFn)k_spmm_rm<WG, KC, true, false, false>;
    case 2: return (KernelFn)k_spmm_rm<WG, KC, false, true, false>;
    case 3: return (KernelFn)k_spmm_rm<WG, KC, true, true, false>;
    case 6: return (KernelFn)k_spmm_rm<WG, KC, false, true, true>;
    case 7: return (KernelFn)k_spmm_rm<WG, KC, true, true, true>;
    }
    return nullptr;
}

template <int WG>
KernelFn pick_rm_kc(int kc, int parts)
{
    switch (kc) {
    case 2: return pick_rm_parts<WG, 2>(parts);
    case 4: return pick_rm_parts<WG, 4>(parts);
    case 8: return pick_rm_parts<WG, 8>(parts);
    case 16: return pick_rm_parts<WG, 16>(parts);
    }
    return nullptr;
}

KernelFn pick_rm(int wg, int kc, int parts)
{
    switch (wg) {
    case 64: return pick_rm_kc<64>(kc, parts);
    case 256: return pick_rm_kc<256>(kc, parts);
    }
    return nullptr;
}

// Fills the first k entries of n rows of a row-major Y with zeros.
__global__ __launch_bounds__(256) void k_zero_rows(double *Y, int64_t ldy, int32_t n, int32_t k)
{
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < (int64_t)n * k;
         s += (int64_t)gridDim.x * 256) {
        const int64_t i = s / k, r = s - i * k;
        Y[i * ldy + r] = 0.0;
    }
}

}  // namespace

int check_operands_rm(const BdcMatrix &m, const double *X, int64_t ldx, const double *Y,
                      int64_t ldy, int32_t k)
{
    if (k < 1 || k > 16)
        return set_error(MHDC_ERR_INVALID_ARG, "k must be in [1, 16]");
    if (m.n > 0 && (!X || !Y))
        return set_error(MHDC_ERR_INVALID_ARG, "X/Y is NULL");
    if (ldx < k || ldy < k)
        return set_error(MHDC_ERR_INVALID_ARG, "ldx/ldy must be >= k");
    if (m.n == 0)
        return MHDC_OK;
    const char *xb = (const char *)X, *xe = (const char *)(X + (int64_t)(m.n - 1) * ldx + k);
    const char *yb = (const char *)Y, *ye = (const char *)(Y + (int64_t)(m.n - 1) * ldy + k);
    if (xb < ye && yb < xe)
        return set_error(MHDC_ERR_INVALID_ARG, "X and Y overlap");
    return MHDC_OK;
}

bool rm_row_gather(const BdcMatrix &m)
{
    if (m.launch.csr_mode == 0)
        return m.row_repeat >= 0.5;
    return m.launch.csr_mode == 2;
}

bool rm_pairs(const double *X, int64_t ldx, const double *Y, int64_t ldy)
{
    return ((uintptr_t)X & 15) == 0 && ((uintptr_t)Y & 15) == 0 && (ldx & 1) == 0 &&
           (ldy & 1) == 0;
}

int rm_columns(int32_t k)
{
    const int kc = kc_for(k);
    return kc < 2 ? 2 : kc;
}

int launch_spmm_rm(const BdcMatrix &m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                   int32_t k, hipStream_t stream)
{
    int rc = check_operands_rm(m, X, ldx, Y, ldy, k);
    if (rc || m.n == 0)
        return rc;
    // one right-hand side with unit strides is a plain vector: the
    // single-column kernel, same bits
    if (k == 1 && ldx == 1 && ldy == 1)
        return launch_spmv(m, X, m.n, Y, m.n, 1, stream);
    const int32_t wg = m.launch.wg_size;
    const bool has_dia = m.K > 0;
    const bool has_rem = m.R > 0;
    if (!has_dia && !has_rem) {
        const int64_t g = ((int64_t)m.n * k + 255) / 256;
        k_zero_rows<<<dim3((unsigned)(g > 65536 ? 65536 : g)), dim3(256), 0, stream>>>(Y, ldy,
                                                                                      m.n, k);
    } else {
        KernelFn fn = pick_rm(wg, rm_columns(k), (has_dia ? 1 : 0) | (has_rem ? 2 : 0) |
                                                     (rm_row_gather(m) ? 4 : 0));
        if (!fn)
            return set_error(MHDC_ERR_NOT_SUPPORTED, "no kernel variant for this launch shape");
        SpmvArgs a = make_args(m, X, ldx, Y, ldy, k, 1);
        a.pairs = rm_pairs(X, ldx, Y, ldy);
        const int64_t tiles = ((int64_t)m.n + wg - 1) / wg;
        if (tiles > INT32_MAX)
            return set_error(MHDC_ERR_SIZE, "too many tiles");
        hipLaunchKernelGGL(fn, dim3((unsigned)tiles), dim3(wg), 0, stream, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string("row-major spmm launch: ") + hipGetErrorString(e));
    return MHDC_OK;
}

}  // namespace mhdc
