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
// YC: Y stored by column (the workspace route of column-major products).
template <int WG, int KC, bool HAS_DIA, bool HAS_REM, bool RG, bool YC>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WG == 256 ? 4 : 1, 8))) void k_spmm_rm(SpmvArgs a)
{
    __shared__ double s_lds[HAS_REM ? (TileShapeRm<WG, KC>::LDS_BYTES + 7) / 8 : 1];
    const int tile = a.remap ? xcd_tile(blockIdx.x, gridDim.x, a.remap) : (int)blockIdx.x;
    spmv_tile_rm<WG, KC, HAS_DIA, HAS_REM, RG, YC>(a, tile, s_lds);
}

// parts: 1 = DIA part, 2 = CSR part, 4 = CSR part by row gathers
template <int WG, int KC, bool YC>
KernelFn pick_rm_parts(int parts)
{
    switch (parts) {
    case 1:
    case 5: return (KernelFn)k_spmm_rm<WG, KC, true, false, false, YC>;
    case 2: return (KernelFn)k_spmm_rm<WG, KC, false, true, false, YC>;
    case 3: return (KernelFn)k_spmm_rm<WG, KC, true, true, false, YC>;
    case 6: return (KernelFn)k_spmm_rm<WG, KC, false, true, true, YC>;
    case 7: return (KernelFn)k_spmm_rm<WG, KC, true, true, true, YC>;
    }
    return nullptr;
}

template <int WG, bool YC>
KernelFn pick_rm_kc(int kc, int parts)
{
    switch (kc) {
    case 2: return pick_rm_parts<WG, 2, YC>(parts);
    case 4: return pick_rm_parts<WG, 4, YC>(parts);
    case 8: return pick_rm_parts<WG, 8, YC>(parts);
    case 16: return pick_rm_parts<WG, 16, YC>(parts);
    }
    return nullptr;
}

KernelFn pick_rm(int wg, int kc, int parts, bool y_cols)
{
    switch (wg) {
    case 64: return y_cols ? pick_rm_kc<64, true>(kc, parts) : pick_rm_kc<64, false>(kc, parts);
    case 256: return y_cols ? pick_rm_kc<256, true>(kc, parts) : pick_rm_kc<256, false>(kc, parts);
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

// Transposition of column-major right-hand sides (column r at X + r*ldx)
// into a row-major copy W (element (i, r) at W[i*ld + r], ld = k rounded up
// to even, so rows start 16-byte aligned).  One workgroup moves TR_ROWS
// rows through LDS so that both sides are read and written in contiguous
// runs: a column's TR_ROWS doubles in, the rows' TR_ROWS*ld doubles out as
// 16-byte pairs.  The pad column of an odd k is written as zero and never
// read as data.
constexpr int TR_ROWS = 256;
constexpr int TR_PAD = TR_ROWS + 1;  // LDS row stride of one column

template <int KC>
__global__ __launch_bounds__(TR_ROWS) void k_cols_to_rows(const double *__restrict__ X,
                                                          int64_t ldx, double *__restrict__ W,
                                                          int32_t ld, int32_t n, int32_t k)
{
    __shared__ double t[KC * TR_PAD];
    const int64_t r0 = (int64_t)blockIdx.x * TR_ROWS;
    const int rows = (int)min((int64_t)TR_ROWS, (int64_t)n - r0);
    const int tid = threadIdx.x;
    if (tid < rows) {
#pragma unroll
        for (int c = 0; c < KC; ++c)
            if (c < k)
                t[c * TR_PAD + tid] = __builtin_nontemporal_load(X + c * ldx + r0 + tid);
    }
    __syncthreads();
    const int half = ld / 2;
    rm_pair *w = reinterpret_cast<rm_pair *>(W + r0 * ld);
    for (int e = tid; e < rows * half; e += TR_ROWS) {
        const int row = e / half, c = 2 * (e - row * half);
        rm_pair v;
        v.x = t[c * TR_PAD + row];
        v.y = c + 1 < k ? t[(c + 1) * TR_PAD + row] : 0.0;
        w[e] = v;
    }
}

using TransposeFn = void (*)(const double *, int64_t, double *, int32_t, int32_t, int32_t);

TransposeFn pick_cols_to_rows(int kc)
{
    switch (kc) {
    case 2: return k_cols_to_rows<2>;
    case 4: return k_cols_to_rows<4>;
    case 8: return k_cols_to_rows<8>;
    case 16: return k_cols_to_rows<16>;
    }
    return nullptr;
}

// Row stride of the row-major copy of X.
int32_t ws_ld(int32_t k) { return (k + 1) & ~1; }

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

// Default (csr_mode 0): row gathers where rows repeat their neighbours'
// offsets, where the CSR part is light (at most 6 entries per row: its
// values and columns then stage in a few large chunks, where staged
// products at 16 columns take 256 entries per chunk and two barriers each)
// and at an accumulator width of 8 columns (k = 5..8), where each lane's
// four gathers of 16 bytes in flight beat the staged products' LDS round
// trip.  Measured on MI355X: 1.1-5.1 entries per row next to a DIA part
// 2-5 % faster on average at 4, 8 and 16 columns; at 8 columns 5-20 %
// faster on every handle tried with 7.7-19.9 entries per row, whole-matrix
// CSR handles included; at 4 columns such CSR parts keep staged products
// (up to 15 % ahead), as they do at 16.
bool rm_row_gather(const BdcMatrix &m, int kc)
{
    if (m.launch.csr_mode == 0)
        return m.row_repeat >= 0.5 || (m.R > 0 && m.R <= 6 * (int64_t)m.n) || kc == 8;
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

namespace {

// The row-major kernel on checked operands; y_cols: Y by column (ldy >= n)
// instead of by row.  A matrix without entries takes the zero fill, which
// writes Y by row: callers with y_cols handle it themselves.
int launch_rm_kernel(const BdcMatrix &m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                     int32_t k, bool y_cols, hipStream_t stream)
{
    const int32_t wg = m.launch.wg_size;
    const bool has_dia = m.K > 0;
    const bool has_rem = m.R > 0;
    if (!has_dia && !has_rem) {
        const int64_t g = ((int64_t)m.n * k + 255) / 256;
        k_zero_rows<<<dim3((unsigned)(g > 65536 ? 65536 : g)), dim3(256), 0, stream>>>(Y, ldy,
                                                                                      m.n, k);
    } else {
        KernelFn fn = pick_rm(wg, rm_columns(k),
                              (has_dia ? 1 : 0) | (has_rem ? 2 : 0) |
                                  (rm_row_gather(m, rm_columns(k)) ? 4 : 0),
                              y_cols);
        if (!fn)
            return set_error(MHDC_ERR_NOT_SUPPORTED, "no kernel variant for this launch shape");
        SpmvArgs a = make_args(m, X, ldx, Y, ldy, k, 1);
        a.pairs = rm_pairs(X, ldx, y_cols ? X : Y, y_cols ? ldx : ldy);
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

}  // namespace

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
    return launch_rm_kernel(m, X, ldx, Y, ldy, k, false, stream);
}

size_t spmm_ws_bytes(const BdcMatrix &m, int32_t k)
{
    return (size_t)m.n * ws_ld(k) * 8;
}

// Lone gathers cost one cache line per column from column-major X and about
// one line per row from the row-major copy (k <= 16 doubles), against 2k
// extra doubles per row of transposition.  Measured on MI355X: at 1 lone
// entry per row the route through the row-major kernel gained 1.13x at k = 2
// and 1.4-1.7x at k = 4..16; at 2-2.4 per row 1.07-1.33x at k = 2 and
// 1.4-2.4x beyond; with almost none (stencil remainders) it ranged from
// 0.5x to 1.07x.
bool spmm_ws_prefers_rm(const BdcMatrix &m, int32_t k)
{
    return k >= 2 && m.R > 0 && m.lone_per_row * k >= 2.0;
}

int launch_spmm_ws(const BdcMatrix &m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                   int32_t k, int32_t route, void *ws, size_t ws_bytes, hipStream_t stream)
{
    int rc = check_operands(m, X, ldx, Y, ldy, k);
    if (rc)
        return rc;
    if (route < 0 || route > 2)
        return set_error(MHDC_ERR_INVALID_ARG, "route must be 0, 1 or 2");
    const bool via_rm = route == 2 || (route == 0 && spmm_ws_prefers_rm(m, k));
    // a matrix without entries only zeroes Y: no detour
    if (!via_rm || m.n == 0 || (m.K == 0 && m.R == 0))
        return launch_spmv(m, X, ldx, Y, ldy, k, stream);
    const size_t need = spmm_ws_bytes(m, k);
    if (!ws || ws_bytes < need)
        return set_error(MHDC_ERR_INVALID_ARG,
                         "workspace smaller than mhdc_spmm_workspace_bytes (" +
                             std::to_string(need) + " bytes)");
    if (((uintptr_t)ws & 255) != 0)
        return set_error(MHDC_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    const char *wb = (const char *)ws, *we = wb + need;
    const char *xb = (const char *)X, *xe = (const char *)(X + (int64_t)(k - 1) * ldx + m.n);
    const char *yb = (const char *)Y, *ye = (const char *)(Y + (int64_t)(k - 1) * ldy + m.n);
    if ((wb < xe && xb < we) || (wb < ye && yb < we))
        return set_error(MHDC_ERR_INVALID_ARG, "workspace overlaps X or Y");
    const int32_t ld = ws_ld(k);
    double *Xr = (double *)ws;
    const unsigned blocks = (unsigned)(((int64_t)m.n + TR_ROWS - 1) / TR_ROWS);
    hipLaunchKernelGGL(pick_cols_to_rows(rm_columns(k)), dim3(blocks), dim3(TR_ROWS), 0, stream,
                       X, ldx, Xr, ld, m.n, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string("transpose launch: ") + hipGetErrorString(e));
    // the row-major kernel on the copy, storing Y by column
    return launch_rm_kernel(m, Xr, ld, Y, ldy, k, true, stream);
}

}  // namespace mhdc
