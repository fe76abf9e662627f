// spmv.hip -- single-matrix SpMV / SpMM launcher: one workgroup per row
// tile (spmv_tile.h), tiles optionally regrouped over the 8 XCDs.
#include "internal.h"
#include "spmv_tile.h"

namespace mhdc {
namespace {

template <int WG, int V, int KC, bool HAS_DIA, bool HAS_REM, bool RG>
__global__ __launch_bounds__(WG) void k_spmv(SpmvArgs a)
{
    __shared__ double s_lds[HAS_REM ? (TileShape<WG, KC, RG>::LDS_BYTES + 7) / 8 : 1];
    const int tile = a.remap ? xcd_tile(blockIdx.x, gridDim.x, a.remap) : (int)blockIdx.x;
    spmv_tile<WG, V, KC, HAS_DIA, HAS_REM, RG>(a, tile, s_lds);
}

using KernelFn = void (*)(SpmvArgs);

// parts: 1 = DIA part, 2 = CSR part, 4 = CSR part with staged values/columns
template <int WG, int V, int KC>
KernelFn pick_rem(int parts)
{
    switch (parts) {
    case 1:
    case 5: return (KernelFn)k_spmv<WG, V, KC, true, false, false>;
    case 3: return (KernelFn)k_spmv<WG, V, KC, true, true, false>;
    case 7: return (KernelFn)k_spmv<WG, V, KC, true, true, true>;
    case 2: return (KernelFn)k_spmv<WG, V, KC, false, true, false>;
    case 6: return (KernelFn)k_spmv<WG, V, KC, false, true, true>;
    }
    return nullptr;
}

template <int WG, int V>
KernelFn pick_kc(int kc, int parts)
{
    switch (kc) {
    case 1: return pick_rem<WG, V, 1>(parts);
    case 2: return pick_rem<WG, V, 2>(parts);
    case 4: return pick_rem<WG, V, 4>(parts);
    case 8: return pick_rem<WG, V, 8>(parts);
    case 16: return pick_rem<WG, V, 16>(parts);
    }
    return nullptr;
}

template <int WG>
KernelFn pick_v(int v, int kc, int parts)
{
    switch (v) {
    case 1: return pick_kc<WG, 1>(kc, parts);
    case 2:
        if (kc == 1)
            return pick_rem<WG, 2, 1>(parts);
        if (kc == 2)
            return pick_rem<WG, 2, 2>(parts);
        if (kc == 4)
            return pick_rem<WG, 2, 4>(parts);
        if (kc == 8)
            return pick_rem<WG, 2, 8>(parts);
        if (kc == 16)
            return pick_rem<WG, 2, 16>(parts);
        return nullptr;
    case 4: return kc == 1 ? pick_rem<WG, 4, 1>(parts) : nullptr;
    }
    return nullptr;
}

KernelFn pick(int wg, int v, int kc, int parts)
{
    switch (wg) {
    case 64: return pick_v<64>(v, kc, parts);
    case 256: return pick_v<256>(v, kc, parts);
    }
    return nullptr;
}

// Fills Y with zeros (a matrix without stored entries).
__global__ __launch_bounds__(256) void k_zero_cols(double *Y, int64_t ldy, int32_t n, int32_t k)
{
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < (int64_t)n * k;
         s += (int64_t)gridDim.x * 256) {
        const int64_t r = s / n, i = s - r * n;
        Y[r * ldy + i] = 0.0;
    }
}

}  // namespace

bool row_gather(int32_t csr_mode, int kc)
{
    return csr_mode == 2 || (csr_mode == 0 && kc > 1);
}

int kc_for(int k)
{
    return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
}

int check_launch(const mhdc_launch &cfg)
{
    if (cfg.wg_size != 64 && cfg.wg_size != 256)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "wg_size must be 64 or 256");
    if (cfg.rows_per_lane != 1 && cfg.rows_per_lane != 2 && cfg.rows_per_lane != 4)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "rows_per_lane must be 1, 2 or 4");
    if (cfg.csr_mode < 0 || cfg.csr_mode > 2)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "csr_mode must be 0, 1 or 2");
    const int r = cfg.xcd_remap;
    if (r < 0 || r > 64)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "xcd_remap must lie in [0, 64]");
    const int g = cfg.rhs_group;
    if (g != 0 && g != 1 && g != 2 && g != 4 && g != 8 && g != 16)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "rhs_group must be 0, 1, 2, 4, 8 or 16");
    return MHDC_OK;
}

SpmvArgs make_args(const BdcMatrix &m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                   int32_t k, int32_t v)
{
    SpmvArgs a;
    a.n = m.n;
    a.n_b = m.n_b > 0 ? m.n_b : 1;
    a.dia_ptr = m.dia_ptr;
    a.dia_off = m.dia_off;
    a.dia_val = m.dia_val;
    a.rem_ptr = m.rem_ptr;
    a.rem_mask = m.rem_mask;
    a.rem_col = m.rem_col;
    a.rem_val = m.rem_val;
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.ldy = ldy;
    a.k = k;
    a.has_dia = m.K > 0;
    a.has_rem = m.R > 0;
    a.uniform = a.has_dia && (m.n_blk == 1 || (m.n_b % (64 * v)) == 0);
    a.remap = m.launch.xcd_remap;
    a.pairs = 0;
    return a;
}

int check_operands(const BdcMatrix &m, const double *X, int64_t ldx, const double *Y,
                   int64_t ldy, int32_t k)
{
    if (k < 1 || k > 16)
        return set_error(MHDC_ERR_INVALID_ARG, "k must be in [1, 16]");
    if (m.n > 0 && (!X || !Y))
        return set_error(MHDC_ERR_INVALID_ARG, "x/y is NULL");
    if (k > 1 && (ldx < m.n || ldy < m.n))
        return set_error(MHDC_ERR_INVALID_ARG, "ldx/ldy must be >= n");
    if (m.n == 0)
        return MHDC_OK;
    // x and y must not overlap (y is written while x is still being read).
    const char *xb = (const char *)X, *xe = (const char *)(X + (int64_t)(k - 1) * ldx + m.n);
    const char *yb = (const char *)Y, *ye = (const char *)(Y + (int64_t)(k - 1) * ldy + m.n);
    if (xb < ye && yb < xe)
        return set_error(MHDC_ERR_INVALID_ARG, "x and y overlap");
    return MHDC_OK;
}

int launch_spmv(const BdcMatrix &m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                int32_t k, hipStream_t stream)
{
    int rc = check_operands(m, X, ldx, Y, ldy, k);
    if (rc || m.n == 0)
        return rc;
    int32_t v = m.launch.rows_per_lane, wg = m.launch.wg_size, remap = m.launch.xcd_remap;
    const int group = m.launch.rhs_group > 0 ? m.launch.rhs_group : 16;
    const int kc = kc_for(k < group ? k : group);
    // Several right-hand sides on a handle with a DIA part and no CSR part,
    // still in its default launch of 256-lane tiles: two adjacent rows per
    // lane (16-byte x and y accesses per column; 1.24x at 16 columns on the
    // 256^3 stencil), XCD runs chosen for the 512-row tiles.  Next to a CSR
    // part the pairs lose (the lanes' remainder gathers no longer fall on
    // neighbouring rows: 1.14x slower at 16 columns on the partially
    // diagonal 192^3 matrix).
    const mhdc_launch &L = m.launch, &D = m.dflt;
    const bool is_default = L.rows_per_lane == D.rows_per_lane && L.wg_size == D.wg_size &&
                            L.xcd_remap == D.xcd_remap && L.csr_mode == D.csr_mode &&
                            L.rhs_group == D.rhs_group;
    if (kc > 1 && wg == 256 && m.K > 0 && m.R == 0 && is_default && remap >= 2) {
        v = 2;
        remap = xcd_run(m.far_offset, 2 * wg);
    }
    // registers: 4 rows per lane only for one right-hand side
    if (kc > 1 && v > 2)
        v = 2;
    const bool has_dia = m.K > 0;
    const bool has_rem = m.R > 0;
    if (!has_dia && !has_rem) {
        const int64_t tot = (int64_t)m.n * k;
        int64_t g = (tot + 255) / 256;
        k_zero_cols<<<dim3((unsigned)(g > 65536 ? 65536 : g)), dim3(256), 0, stream>>>(Y, ldy, m.n,
                                                                                      k);
    } else {
        const int parts = (has_dia ? 1 : 0) | (has_rem ? 2 : 0) |
                          (row_gather(m.launch.csr_mode, kc) ? 4 : 0);
        KernelFn fn = pick(wg, v, kc, parts);
        if (!fn)
            return set_error(MHDC_ERR_NOT_SUPPORTED, "no kernel variant for this launch shape");
        SpmvArgs a = make_args(m, X, ldx, Y, ldy, k, v);
        a.remap = remap;
        const int64_t T = (int64_t)wg * v;
        const int64_t tiles = ((int64_t)m.n + T - 1) / T;
        if (tiles > INT32_MAX)
            return set_error(MHDC_ERR_SIZE, "too many tiles");
        hipLaunchKernelGGL(fn, dim3((unsigned)tiles), dim3(wg), 0, stream, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string("spmv launch: ") + hipGetErrorString(e));
    return MHDC_OK;
}

int launch_rem_part(const BdcMatrix &m, const double *x, double *y, hipStream_t stream)
{
    int rc = check_operands(m, x, m.n, y, m.n, 1);
    if (rc || m.n == 0)
        return rc;
    if (m.R == 0) {
        const int64_t g = ((int64_t)m.n + 255) / 256;
        k_zero_cols<<<dim3((unsigned)(g > 65536 ? 65536 : g)), dim3(256), 0, stream>>>(y, m.n,
                                                                                      m.n, 1);
    } else {
        const int32_t v = m.launch.rows_per_lane, wg = m.launch.wg_size;
        KernelFn fn = pick(wg, v, 1, 2 | (row_gather(m.launch.csr_mode, 1) ? 4 : 0));
        if (!fn)
            return set_error(MHDC_ERR_NOT_SUPPORTED, "no kernel variant for this launch shape");
        SpmvArgs a = make_args(m, x, m.n, y, m.n, 1, v);
        a.has_dia = 0;
        const int64_t T = (int64_t)wg * v;
        const int64_t tiles = ((int64_t)m.n + T - 1) / T;
        hipLaunchKernelGGL(fn, dim3((unsigned)tiles), dim3(wg), 0, stream, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string("remainder launch: ") + hipGetErrorString(e));
    return MHDC_OK;
}

}  // namespace mhdc
