// spmv.hip -- the fused SpMV kernel for row-blocked DIA + CSR remainder.
//
// One kernel serves the three handle kinds: M-HDC (Sec. 4.3, Fig. 16), HDC
// in its cache-blocked form (Sec. 4.2, Fig. 13; one block of n rows) and
// plain CSR (no DIA part, Fig. 3).  Per row it computes, in this order,
//     acc  = sum of the row's remainder entries (ascending column),
//     acc += dia_val[k*n_b + t] * x[i + off_k]  for the block's diagonals k
//            in ascending order, only where 0 <= i + off_k < n,
// and stores acc once: the CSR part first, then the diagonals, as in Fig. 16.
//
// Work mapping (gfx950, 64-lane wavefronts):
//   * a workgroup of WG lanes owns a tile of WG*V consecutive rows; lane l of
//     wave w owns rows tile_base + w*64*V + v*64 + l (v < V), so every load
//     and store of the DIA part is 64 consecutive doubles per instruction;
//   * the DIA value stream and the remainder arrays are read once, with
//     non-temporal loads so they do not evict x from L2; y is written with
//     non-temporal stores; x goes through the caches (its reuse across the
//     diagonals of neighbouring rows is what the blocking buys);
//   * when every wavefront's rows fall in one block (n_b a multiple of 64*V,
//     or a single block) the block index, its diagonal range and each offset
//     are wave-uniform values;
//   * the tile's remainder entries are contiguous in rem_col/rem_val: they
//     are staged through LDS in chunks with coalesced loads, then each lane
//     sums its own rows' entries from LDS in column order;
//   * workgroups are remapped so that each XCD (dispatch is round-robin over
//     the 8 XCDs) walks one contiguous range of tiles and its L2 sees the x
//     window of its rows.
#include "internal.h"

namespace mhdc {
namespace {

struct SpmvArgs {
    int32_t n;
    int32_t n_b;
    const int32_t *__restrict__ dia_ptr;
    const int32_t *__restrict__ dia_off;
    const double *__restrict__ dia_val;
    const int32_t *__restrict__ rem_ptr;
    const int32_t *__restrict__ rem_col;
    const double *__restrict__ rem_val;
    const double *__restrict__ X;
    int64_t ldx;
    double *__restrict__ Y;
    int64_t ldy;
    int32_t k;
    int32_t has_dia;
    int32_t uniform;
    int32_t remap;
};

__device__ inline int xcd_tile(int w, int G)
{
    const int x = w & 7, idx = w >> 3, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + idx;
}

template <int WG, int V, int KC, bool HAS_REM>
__global__ __launch_bounds__(WG) void k_spmv(SpmvArgs a)
{
    constexpr int T = WG * V;
    constexpr int CH = WG * 8;
    const int n = a.n;
    const int tile = a.remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int64_t tile_base = (int64_t)tile * T;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wave_base = tile_base + (int64_t)wave * 64 * V;

    double acc[V][KC];
#pragma unroll
    for (int v = 0; v < V; v++)
#pragma unroll
        for (int r = 0; r < KC; r++)
            acc[v][r] = 0.0;

    if constexpr (HAS_REM) {
        __shared__ double s_val[CH];
        __shared__ int32_t s_col[CH];
        const int64_t tile_end = tile_base + T < n ? tile_base + T : n;
        const int32_t e_beg = a.rem_ptr[tile_base];
        const int32_t e_end = a.rem_ptr[tile_end];
        if (e_beg < e_end) {
            int32_t rs[V], re[V];
#pragma unroll
            for (int v = 0; v < V; v++) {
                const int64_t row = wave_base + v * 64 + lane;
                rs[v] = row < n ? a.rem_ptr[row] : 0;
                re[v] = row < n ? a.rem_ptr[row + 1] : 0;
            }
            for (int32_t cb = e_beg; cb < e_end; cb += CH) {
                const int32_t ce = cb + CH < e_end ? cb + CH : e_end;
                for (int32_t e = cb + (int32_t)threadIdx.x; e < ce; e += WG) {
                    s_val[e - cb] = __builtin_nontemporal_load(a.rem_val + e);
                    s_col[e - cb] = __builtin_nontemporal_load(a.rem_col + e);
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < V; v++) {
                    const int32_t lo = rs[v] > cb ? rs[v] : cb;
                    const int32_t hi = re[v] < ce ? re[v] : ce;
                    for (int32_t e = lo; e < hi; e++) {
                        const double w = s_val[e - cb];
                        const int32_t c = s_col[e - cb];
#pragma unroll
                        for (int r = 0; r < KC; r++)
                            if (r < a.k)
                                acc[v][r] += w * a.X[r * a.ldx + c];
                    }
                }
                __syncthreads();
            }
        }
    }

    if (a.has_dia && wave_base < n) {
        if (a.uniform) {
            // All rows of this wavefront lie in block ib.
            const int64_t ib = wave_base / a.n_b;
            const int64_t t0 = wave_base - ib * a.n_b;
            const int32_t kb0 = a.dia_ptr[ib], kb1 = a.dia_ptr[ib + 1];
            for (int32_t kk = kb0; kk < kb1; kk++) {
                const int64_t off = a.dia_off[kk];
                const double *seg = a.dia_val + (int64_t)kk * a.n_b + t0;
#pragma unroll
                for (int v = 0; v < V; v++) {
                    const int64_t row = wave_base + v * 64 + lane;
                    const int64_t j = row + off;
                    if (row < n && j >= 0 && j < n) {
                        const double w = __builtin_nontemporal_load(seg + v * 64 + lane);
#pragma unroll
                        for (int r = 0; r < KC; r++)
                            if (r < a.k)
                                acc[v][r] += w * a.X[r * a.ldx + j];
                    }
                }
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; v++) {
                const int64_t row = wave_base + v * 64 + lane;
                if (row < n) {
                    const int64_t ib = row / a.n_b;
                    const int64_t t = row - ib * a.n_b;
                    const int32_t kb0 = a.dia_ptr[ib], kb1 = a.dia_ptr[ib + 1];
                    for (int32_t kk = kb0; kk < kb1; kk++) {
                        const int64_t j = row + a.dia_off[kk];
                        if (j >= 0 && j < n) {
                            const double w =
                                __builtin_nontemporal_load(a.dia_val + (int64_t)kk * a.n_b + t);
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < a.k)
                                    acc[v][r] += w * a.X[r * a.ldx + j];
                        }
                    }
                }
            }
        }
    }

#pragma unroll
    for (int v = 0; v < V; v++) {
        const int64_t row = wave_base + v * 64 + lane;
        if (row < n) {
#pragma unroll
            for (int r = 0; r < KC; r++)
                if (r < a.k)
                    __builtin_nontemporal_store(acc[v][r], a.Y + r * a.ldy + row);
        }
    }
}

using KernelFn = void (*)(SpmvArgs);

template <int WG, int V, int KC>
KernelFn pick_rem(bool has_rem)
{
    return has_rem ? (KernelFn)k_spmv<WG, V, KC, true> : (KernelFn)k_spmv<WG, V, KC, false>;
}

template <int WG, int V>
KernelFn pick_kc(int kc, bool has_rem)
{
    switch (kc) {
    case 1: return pick_rem<WG, V, 1>(has_rem);
    case 2: return pick_rem<WG, V, 2>(has_rem);
    case 4: return pick_rem<WG, V, 4>(has_rem);
    case 8: return pick_rem<WG, V, 8>(has_rem);
    case 16: return pick_rem<WG, V, 16>(has_rem);
    }
    return nullptr;
}

template <int WG>
KernelFn pick_v(int v, int kc, bool has_rem)
{
    switch (v) {
    case 1: return pick_kc<WG, 1>(kc, has_rem);
    case 2: return pick_kc<WG, 2>(kc, has_rem);
    case 4: return kc == 1 ? pick_rem<WG, 4, 1>(has_rem) : nullptr;
    }
    return nullptr;
}

KernelFn pick(int wg, int v, int kc, bool has_rem)
{
    switch (wg) {
    case 64: return pick_v<64>(v, kc, has_rem);
    case 256: return pick_v<256>(v, kc, has_rem);
    }
    return nullptr;
}

int kc_for(int k)
{
    return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
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

int check_launch(const mhdc_launch &cfg)
{
    if (cfg.wg_size != 64 && cfg.wg_size != 256)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "wg_size must be 64 or 256");
    if (cfg.rows_per_lane != 1 && cfg.rows_per_lane != 2 && cfg.rows_per_lane != 4)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "rows_per_lane must be 1, 2 or 4");
    return MHDC_OK;
}

int launch_spmv(const BdcMatrix &m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                int32_t k, hipStream_t stream)
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
    {
        const char *xb = (const char *)X, *xe = (const char *)(X + (int64_t)(k - 1) * ldx + m.n);
        const char *yb = (const char *)Y, *ye = (const char *)(Y + (int64_t)(k - 1) * ldy + m.n);
        if (xb < ye && yb < xe)
            return set_error(MHDC_ERR_INVALID_ARG, "x and y overlap");
    }
    int32_t v = m.launch.rows_per_lane, wg = m.launch.wg_size;
    int kc = kc_for(k);
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
        KernelFn fn = pick(wg, v, kc, has_rem);
        if (!fn)
            return set_error(MHDC_ERR_NOT_SUPPORTED, "no kernel variant for this launch shape");
        SpmvArgs a;
        a.n = m.n;
        a.n_b = m.n_b > 0 ? m.n_b : 1;
        a.dia_ptr = m.dia_ptr;
        a.dia_off = m.dia_off;
        a.dia_val = m.dia_val;
        a.rem_ptr = m.rem_ptr;
        a.rem_col = m.rem_col;
        a.rem_val = m.rem_val;
        a.X = X;
        a.ldx = ldx;
        a.Y = Y;
        a.ldy = ldy;
        a.k = k;
        a.has_dia = has_dia;
        a.uniform = has_dia && (m.n_blk == 1 || (m.n_b % (64 * v)) == 0);
        a.remap = m.launch.xcd_remap;
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

}  // namespace mhdc
