// spmv_tile.h -- one row tile of the fused SpMV for row-blocked DIA + CSR
// remainder, shared by the single-matrix kernel (spmv.hip) and the batched
// persistent kernel (batch.hip).
//
// One device routine serves the three handle kinds: M-HDC (Sec. 4.3, Fig. 16),
// HDC in its cache-blocked form (Sec. 4.2, Fig. 13; one block of n rows) and
// plain CSR (no DIA part, Fig. 3).  Per row and right-hand side it computes,
// in this order,
//     acc = 0;  acc = acc + round(val * x[col])   for the row's remainder
//                                                  entries in column order,
//     acc = acc + round(dia_val[k*n_b + t] * x[i + off_k])
//                      for the block's diagonals k in ascending order, only
//                      where 0 <= i + off_k < n,
// and stores acc once.  Every product is rounded before it is added (no fused
// multiply-add), so a row's value is bit-identical to the sequential kernels
// of Figs. 3, 8 and 16 and does not depend on the launch shape.
//
// Work mapping (gfx950, 64-lane wavefronts):
//   * a workgroup of WG lanes owns a tile of WG*V consecutive rows; lane l of
//     wave w owns rows tile_base + w*64*V + v*64 + l (v < V), so each DIA load
//     and y store covers 64 consecutive doubles per instruction;
//   * the DIA value stream and the remainder arrays are read once with
//     non-temporal loads, y is written with non-temporal stores, x goes
//     through the caches (its reuse across neighbouring diagonals is what the
//     row blocking buys);
//   * when all rows of a wavefront fall in one block the block's diagonal
//     range and offsets are wave-uniform; diagonals are processed U at a time
//     so that U*V value loads and U*V x loads are in flight per lane;
//   * the tile's remainder entries are contiguous: each chunk is read with
//     coalesced loads, multiplied by the gathered x on the spot (CH/WG
//     independent gathers per lane) and the products are staged in LDS; each
//     lane then sums its own rows' products from LDS in column order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mhdc {

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
    int32_t has_rem;
    int32_t uniform;
    int32_t remap;
};

// Workgroups are dispatched round-robin over the 8 XCDs; map workgroup w so
// that XCD (w mod 8) walks one contiguous range of the G tiles.  A bijection
// on [0, G) for any G.
__device__ inline int xcd_tile(int w, int G)
{
    const int x = w & 7, idx = w >> 3, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + idx;
}

template <int WG, int KC>
struct TileShape {
    // remainder entries staged per chunk; LDS = KC * CH doubles
    static constexpr int CH = (WG * 8 / KC) < WG ? WG : WG * 8 / KC;
    // diagonals processed together in the uniform DIA path
    static constexpr int U = KC == 1 ? 4 : (KC <= 4 ? 2 : 1);
};

template <int WG, int V, int KC, bool HAS_REM>
__device__ inline void spmv_tile(const SpmvArgs &a, int64_t tile, double *s_prod)
{
    // products are rounded before they are added: no multiply-add fusion
#pragma clang fp contract(off)
    constexpr int T = WG * V;
    constexpr int CH = TileShape<WG, KC>::CH;
    constexpr int U = TileShape<WG, KC>::U;
    const int n = a.n;
    const int64_t tile_base = tile * T;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wave_base = tile_base + (int64_t)wave * 64 * V;

    double acc[V][KC];
#pragma unroll
    for (int v = 0; v < V; v++)
#pragma unroll
        for (int r = 0; r < KC; r++)
            acc[v][r] = 0.0;

    if (HAS_REM && a.has_rem) {
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
#pragma unroll
                for (int j = 0; j < CH / WG; j++) {
                    const int32_t e = cb + j * WG + (int32_t)threadIdx.x;
                    if (e < ce) {
                        const double w = __builtin_nontemporal_load(a.rem_val + e);
                        const int32_t c = __builtin_nontemporal_load(a.rem_col + e);
#pragma unroll
                        for (int r = 0; r < KC; r++)
                            if (r < a.k)
                                s_prod[r * CH + (e - cb)] = __dmul_rn(w, a.X[r * a.ldx + c]);
                    }
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < V; v++) {
                    const int32_t lo = rs[v] > cb ? rs[v] : cb;
                    const int32_t hi = re[v] < ce ? re[v] : ce;
                    for (int32_t e = lo; e < hi; e++)
#pragma unroll
                        for (int r = 0; r < KC; r++)
                            if (r < a.k)
                                acc[v][r] = __dadd_rn(acc[v][r], s_prod[r * CH + (e - cb)]);
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
            for (int32_t kk = kb0; kk < kb1; kk += U) {
                int64_t off[U];
                bool live[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    live[u] = kk + u < kb1;
                    off[u] = live[u] ? a.dia_off[kk + u] : 0;
                }
                double w[U][V], xv[U][V][KC];
                bool in[U][V];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const double *seg = a.dia_val + (int64_t)(kk + u) * a.n_b + t0;
#pragma unroll
                    for (int v = 0; v < V; v++) {
                        const int64_t row = wave_base + v * 64 + lane;
                        const int64_t j = row + off[u];
                        in[u][v] = live[u] && row < n && j >= 0 && j < n;
                        w[u][v] = 0.0;
#pragma unroll
                        for (int r = 0; r < KC; r++)
                            xv[u][v][r] = 0.0;
                        if (in[u][v]) {
                            w[u][v] = __builtin_nontemporal_load(seg + v * 64 + lane);
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < a.k)
                                    xv[u][v][r] = a.X[r * a.ldx + j];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < U; u++)
#pragma unroll
                    for (int v = 0; v < V; v++)
                        if (in[u][v])
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < a.k)
                                    acc[v][r] = __dadd_rn(acc[v][r], __dmul_rn(w[u][v], xv[u][v][r]));
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
                                    acc[v][r] = __dadd_rn(acc[v][r], __dmul_rn(w, a.X[r * a.ldx + j]));
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

}  // namespace mhdc
