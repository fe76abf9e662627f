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
// of Figs. 3, 8 and 16 and does not depend on the launch shape or variant.
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
//   * the tile's remainder entries are contiguous and read in chunks with
//     coalesced loads into LDS.  Two variants (RG):
//       RG = false: the staging lane multiplies its entries by the gathered
//         x on the spot (CH/WG independent gathers per lane) and stages the
//         rounded products; each lane then adds its rows' products;
//       RG = true: values and columns are staged (12 bytes per entry, for
//         any number of right-hand sides) and each lane gathers x for its
//         own rows' entries -- for rows of similar structure (stencils) the
//         lanes of a wavefront then read neighbouring x.
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
    const uint32_t *rem_mask;  // one bit per 64 rows, or null: test rem_ptr
    int32_t pairs;             // row-major kernel: 16-byte accesses of column pairs
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  remap = 1: XCD (w mod 8) walks one contiguous eighth of the G tiles.
// remap = C >= 2: runs of C consecutive tiles go to one XCD and the XCDs
// take the runs in turn, so a row tile's neighbours (whose x entries it
// shares through near diagonals) mostly sit in the same L2 while all XCDs
// still sweep the rows together; tile t + 8*C*j is on t's XCD, so a C that
// divides the far diagonals' distance in tiles by 8 keeps those x rows in
// the same L2 too.  Tiles past the last whole round of 8*C keep dispatch
// order.  Both forms are bijections on [0, G).
__device__ inline int xcd_tile(int w, int G, int remap)
{
    const int x = w & 7, idx = w >> 3;
    if (remap == 1) {
        const int q = G >> 3, r = G & 7;
        return x * q + (x < r ? x : r) + idx;
    }
    const int span = remap * 8;
    if (w >= (G / span) * span)
        return w;
    const int run = idx / remap;
    return (run * 8 + x) * remap + (idx - run * remap);
}

// Wave-uniform read of data no kernel writes while it runs (block and
// remainder pointers, offsets, the remainder mask, batch descriptors),
// through the constant address space so that it becomes a scalar load even
// after a workgroup barrier (after which the compiler can no longer prove on
// its own that global memory is unchanged, and falls back to one vector
// load and wait per value).
template <typename E>
__device__ inline E uniform_load(const E *p, int64_t i)
{
    using const_e = const __attribute__((address_space(4))) E;
    return ((const_e *)p)[i];
}

// Format metadata read through uniform_load (SCALAR) or as plain loads.
template <bool SCALAR, typename E>
__device__ inline E meta_load(const E *p, int64_t i)
{
    if constexpr (SCALAR)
        return uniform_load(p, i);
    else
        return p[i];
}

template <int WG, int KC, bool RG>
struct TileShape {
    // remainder entries staged per chunk
    static constexpr int CH = RG ? WG * 8 : ((WG * 8 / KC) < WG ? WG : WG * 8 / KC);
    static constexpr int LDS_BYTES = RG ? CH * 12 : KC * CH * 8;
    // diagonals processed together in the uniform DIA path (8 and 16
    // columns: the U8 argument of spmv_tile_cols)
    static constexpr int U = KC == 1 ? 8 : 2;
    // remainder entries gathered together per row in the RG variant
    static constexpr int UR = KC == 1 ? 4 : (KC <= 4 ? 2 : 1);
};

// HAS_DIA / HAS_REM compile the DIA part / the CSR part in (a kernel's
// register budget is that of everything it contains); a.has_dia and
// a.has_rem still switch them per matrix at run time.
// U8: diagonals in flight in the uniform DIA path for 8 and 16 columns (two
// in the single-matrix kernel; one in the batched kernel, which keeps four
// waves per SIMD and would spill with two).
template <int WG, int V, int KC, bool HAS_DIA, bool HAS_REM, bool RG, int U8 = 2>
__device__ inline void spmv_tile_cols(const SpmvArgs &a, int64_t tile, void *lds,
                                      const double *__restrict__ Xg, double *__restrict__ Yg,
                                      int32_t kc_n)
{
    // products are rounded before they are added: no multiply-add fusion
#pragma clang fp contract(off)
    using Shape = TileShape<WG, KC, RG>;
    constexpr int T = WG * V;
    constexpr int CH = Shape::CH;
    // Several right-hand sides at two rows per lane: the lane's rows are
    // adjacent, so each column's x pair and y pair move as one 16-byte
    // access (half the load instructions per diagonal); otherwise the rows
    // of a lane lie one wavefront apart.  The arithmetic per row is the same.
    constexpr bool ADJ = KC >= 2 && V == 2;
    typedef double pair8 __attribute__((ext_vector_type(2), aligned(8)));
    // eight diagonals in flight for pure DIA tiles, four next to a CSR part;
    // one at 8 and 16 columns with adjacent rows (registers)
    constexpr int U = (KC == 1 && HAS_REM) ? 4 : (KC >= 8 ? (ADJ ? 1 : U8) : Shape::U);
    constexpr int UR = Shape::UR;
    const int n = a.n;
    const int64_t tile_base = tile * T;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wave_base = tile_base + (int64_t)wave * 64 * V;
    // row of the lane's slot v
    auto row_of = [&](int v) -> int64_t {
        return ADJ ? wave_base + 2 * lane + v : wave_base + v * 64 + lane;
    };

    double acc[V][KC];
#pragma unroll
    for (int v = 0; v < V; v++)
#pragma unroll
        for (int r = 0; r < KC; r++)
            acc[v][r] = 0.0;

    // Scalar metadata loads up to 4 columns; at 8 and 16 the scalar
    // registers are taken by the column addresses.
    constexpr bool SM = KC <= 4;
    // Wave-uniform DIA range, loaded before the remainder pointers are
    // looked at so that the two scalar loads share one memory round trip
    // (most tiles of a mostly-diagonal matrix have no remainder entries).
    const bool dia_uniform = HAS_DIA && a.has_dia && a.uniform && wave_base < n;
    int64_t u_ib = 0;
    int32_t u_kb0 = 0, u_kb1 = 0;
    if (SM && dia_uniform) {
        u_ib = wave_base / a.n_b;
        u_kb0 = uniform_load(a.dia_ptr, u_ib);
        u_kb1 = uniform_load(a.dia_ptr, u_ib + 1);
    }

    // A tile covers T/64 whole groups of 64 rows inside one mask word.
    static_assert(T % 64 == 0 && 32 % (T / 64) == 0, "tile must cover 64-row groups of one word");
    bool tile_rem = HAS_REM && a.has_rem;
    if (tile_rem && a.rem_mask) {
        const int64_t g0 = tile_base >> 6;
        const uint32_t word = meta_load<SM>(a.rem_mask, g0 >> 5);
        tile_rem = ((word >> (g0 & 31)) & (T == 2048 ? 0xffffffffu : ((1u << (T / 64)) - 1u))) != 0;
    }
    if (tile_rem) {
        const int64_t tile_end = tile_base + T < n ? tile_base + T : n;
        const int32_t e_beg = meta_load<SM>(a.rem_ptr, tile_base);
        const int32_t e_end = meta_load<SM>(a.rem_ptr, tile_end);
        if (e_beg < e_end) {
            int32_t rs[V], re[V];
#pragma unroll
            for (int v = 0; v < V; v++) {
                const int64_t row = row_of(v);
                rs[v] = row < n ? a.rem_ptr[row] : 0;
                re[v] = row < n ? a.rem_ptr[row + 1] : 0;
            }
            double *s_val = static_cast<double *>(lds);
            int32_t *s_col = reinterpret_cast<int32_t *>(s_val + CH);
            for (int32_t cb = e_beg; cb < e_end; cb += CH) {
                const int32_t ce = cb + CH < e_end ? cb + CH : e_end;
#pragma unroll
                for (int j = 0; j < CH / WG; j++) {
                    const int32_t e = cb + j * WG + (int32_t)threadIdx.x;
                    if (e < ce) {
                        const double w = __builtin_nontemporal_load(a.rem_val + e);
                        const int32_t c = __builtin_nontemporal_load(a.rem_col + e);
                        if constexpr (RG) {
                            s_val[e - cb] = w;
                            s_col[e - cb] = c;
                        } else {
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < kc_n)
                                    s_val[r * CH + (e - cb)] = __dmul_rn(w, Xg[r * a.ldx + c]);
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < V; v++) {
                    const int32_t lo = rs[v] > cb ? rs[v] : cb;
                    const int32_t hi = re[v] < ce ? re[v] : ce;
                    if constexpr (RG) {
                        int32_t e = lo;
                        for (; e + UR <= hi; e += UR) {
                            double w[UR], xv[UR][KC];
#pragma unroll
                            for (int u = 0; u < UR; u++) {
                                w[u] = s_val[e + u - cb];
                                const int32_t c = s_col[e + u - cb];
#pragma unroll
                                for (int r = 0; r < KC; r++)
                                    xv[u][r] = r < kc_n ? Xg[r * a.ldx + c] : 0.0;
                            }
#pragma unroll
                            for (int u = 0; u < UR; u++)
#pragma unroll
                                for (int r = 0; r < KC; r++)
                                    if (r < kc_n)
                                        acc[v][r] = __dadd_rn(acc[v][r], __dmul_rn(w[u], xv[u][r]));
                        }
                        for (; e < hi; e++) {
                            const double w = s_val[e - cb];
                            const int32_t c = s_col[e - cb];
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < kc_n)
                                    acc[v][r] = __dadd_rn(acc[v][r], __dmul_rn(w, Xg[r * a.ldx + c]));
                        }
                    } else {
                        for (int32_t e = lo; e < hi; e++)
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < kc_n)
                                    acc[v][r] = __dadd_rn(acc[v][r], s_val[r * CH + (e - cb)]);
                    }
                }
                __syncthreads();
            }
        }
    }

    if (HAS_DIA && a.has_dia && wave_base < n) {
        // (a.uniform where the range is loaded here: the compiler's register
        // allocation of the 8- and 16-column kernels is much worse with the
        // hoisted flag)
        if (SM ? dia_uniform : a.uniform != 0) {
            // All rows of this wavefront lie in block u_ib.
            if (!SM) {
                u_ib = wave_base / a.n_b;
                u_kb0 = a.dia_ptr[u_ib];
                u_kb1 = a.dia_ptr[u_ib + 1];
            }
            const int64_t t0 = wave_base - u_ib * a.n_b;
            const int32_t kb1 = u_kb1;
            for (int32_t kk = u_kb0; kk < kb1; kk += U) {
                int64_t off[U];
                bool live[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    live[u] = kk + u < kb1;
                    // clamped index: unconditional loads that issue together
                    off[u] = meta_load<SM>(a.dia_off, live[u] ? kk + u : kb1 - 1);
                }
                double w[U][V], xv[U][V][KC];
                bool in[U][V];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const double *seg = a.dia_val + (int64_t)(kk + u) * a.n_b + t0;
                    if constexpr (ADJ) {
                        // rows row0 and row0 + 1: 16-byte loads where both are in range
                        const int64_t row0 = wave_base + 2 * lane;
                        const int64_t j0 = row0 + off[u];
                        in[u][0] = live[u] && row0 < n && j0 >= 0 && j0 < n;
                        in[u][V - 1] = live[u] && row0 + 1 < n && j0 + 1 >= 0 && j0 + 1 < n;
                        w[u][0] = 0.0;
                        w[u][V - 1] = 0.0;
#pragma unroll
                        for (int r = 0; r < KC; r++) {
                            xv[u][0][r] = 0.0;
                            xv[u][V - 1][r] = 0.0;
                        }
                        if (in[u][0] && in[u][V - 1]) {
                            const pair8 wv = __builtin_nontemporal_load(reinterpret_cast<const pair8 *>(seg + 2 * lane));
                            w[u][0] = wv.x;
                            w[u][V - 1] = wv.y;
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < kc_n) {
                                    const pair8 xx = *reinterpret_cast<const pair8 *>(Xg + r * a.ldx + j0);
                                    xv[u][0][r] = xx.x;
                                    xv[u][V - 1][r] = xx.y;
                                }
                        } else {
                            if (in[u][0]) {
                                w[u][0] = __builtin_nontemporal_load(seg + 2 * lane);
#pragma unroll
                                for (int r = 0; r < KC; r++)
                                    if (r < kc_n)
                                        xv[u][0][r] = Xg[r * a.ldx + j0];
                            }
                            if (in[u][V - 1]) {
                                w[u][V - 1] = __builtin_nontemporal_load(seg + 2 * lane + 1);
#pragma unroll
                                for (int r = 0; r < KC; r++)
                                    if (r < kc_n)
                                        xv[u][V - 1][r] = Xg[r * a.ldx + j0 + 1];
                            }
                        }
                        continue;
                    }
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
                                if (r < kc_n)
                                    xv[u][v][r] = Xg[r * a.ldx + j];
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
                                if (r < kc_n)
                                    acc[v][r] = __dadd_rn(acc[v][r], __dmul_rn(w[u][v], xv[u][v][r]));
            }
        } else {
            // Rows of one wavefront span several blocks: each row walks its
            // own block's list, two diagonals at a time.
#pragma unroll
            for (int v = 0; v < V; v++) {
                const int64_t row = row_of(v);
                if (row < n) {
                    const int64_t ib = row / a.n_b;
                    const int64_t t = row - ib * a.n_b;
                    const int32_t kb0 = a.dia_ptr[ib], kb1 = a.dia_ptr[ib + 1];
                    int32_t kk = kb0;
                    for (; kk + 2 <= kb1; kk += 2) {
                        const int64_t j0 = row + a.dia_off[kk], j1 = row + a.dia_off[kk + 1];
                        const bool in0 = j0 >= 0 && j0 < n, in1 = j1 >= 0 && j1 < n;
                        double w0 = 0.0, w1 = 0.0, x0[KC], x1[KC];
#pragma unroll
                        for (int r = 0; r < KC; r++)
                            x0[r] = x1[r] = 0.0;
                        if (in0) {
                            w0 = __builtin_nontemporal_load(a.dia_val + (int64_t)kk * a.n_b + t);
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < kc_n)
                                    x0[r] = Xg[r * a.ldx + j0];
                        }
                        if (in1) {
                            w1 = __builtin_nontemporal_load(a.dia_val + (int64_t)(kk + 1) * a.n_b + t);
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < kc_n)
                                    x1[r] = Xg[r * a.ldx + j1];
                        }
#pragma unroll
                        for (int r = 0; r < KC; r++)
                            if (r < kc_n) {
                                if (in0)
                                    acc[v][r] = __dadd_rn(acc[v][r], __dmul_rn(w0, x0[r]));
                                if (in1)
                                    acc[v][r] = __dadd_rn(acc[v][r], __dmul_rn(w1, x1[r]));
                            }
                    }
                    if (kk < kb1) {
                        const int64_t j = row + a.dia_off[kk];
                        if (j >= 0 && j < n) {
                            const double w =
                                __builtin_nontemporal_load(a.dia_val + (int64_t)kk * a.n_b + t);
#pragma unroll
                            for (int r = 0; r < KC; r++)
                                if (r < kc_n)
                                    acc[v][r] = __dadd_rn(acc[v][r], __dmul_rn(w, Xg[r * a.ldx + j]));
                        }
                    }
                }
            }
        }
    }

    if constexpr (ADJ) {
        const int64_t row0 = wave_base + 2 * lane;
#pragma unroll
        for (int r = 0; r < KC; r++)
            if (r < kc_n) {
                if (row0 + 1 < n) {
                    pair8 yv;
                    yv.x = acc[0][r];
                    yv.y = acc[V - 1][r];
                    __builtin_nontemporal_store(yv, reinterpret_cast<pair8 *>(Yg + r * a.ldy + row0));
                } else if (row0 < n) {
                    __builtin_nontemporal_store(acc[0][r], Yg + r * a.ldy + row0);
                }
            }
        return;
    }
#pragma unroll
    for (int v = 0; v < V; v++) {
        const int64_t row = wave_base + v * 64 + lane;
        if (row < n) {
#pragma unroll
            for (int r = 0; r < KC; r++)
                if (r < kc_n)
                    __builtin_nontemporal_store(acc[v][r], Yg + r * a.ldy + row);
        }
    }
}

// All right-hand sides of the tile, KC columns per pass (the tile's share
// of A is read again from the caches for every further pass).
template <int WG, int V, int KC, bool HAS_DIA, bool HAS_REM, bool RG, int U8 = 2>
__device__ inline void spmv_tile(const SpmvArgs &a, int64_t tile, void *lds)
{
    for (int32_t r0 = 0; r0 < a.k; r0 += KC) {
        const int32_t kc_n = a.k - r0 < KC ? a.k - r0 : KC;
        spmv_tile_cols<WG, V, KC, HAS_DIA, HAS_REM, RG, U8>(a, tile, lds, a.X + r0 * a.ldx,
                                                            a.Y + r0 * a.ldy, kc_n);
    }
}

}  // namespace mhdc
