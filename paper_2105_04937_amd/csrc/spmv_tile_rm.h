// spmv_tile_rm.h -- one row tile of the fused SpMV for 2 to 16 right-hand
// sides stored row by row (element (i, r) of X at X[i*ldx + r], ldx >= k),
// shared by the single-matrix launcher (spmv.hip) and the batched kernel
// (batch.hip).
//
// The arithmetic and its order are those of spmv_tile.h: per row and
// column, the remainder entries in column order, then the block's diagonals
// in ascending order, every product rounded before it is added -- so every
// column equals the column-major kernel's bits and the sequential kernels'
// (Figs. 3, 8, 16).
//
// Work mapping (64-lane wavefronts): a wavefront owns 64 consecutive rows.
// Each lane carries P = 2 adjacent columns, so a row takes LC = KC/2 lanes and
// the wavefront splits into RPI = 64/LC row slots: lane (s, c) =
// (lane / LC, lane % LC) accumulates columns 2c and 2c + 1 of the rows
// wave_base + s + RPI*q, q < LC.  One load of X then covers RPI consecutive
// rows times KC columns -- 128 consecutive doubles when ldx = KC -- for a
// diagonal, and a remainder entry brings its column's row of X (KC
// doubles, one cache line at KC = 16) instead of KC lines of KC separate
// column vectors.  When X and Y are 16-byte aligned with even leading
// dimensions (a.pairs) a lane moves its two columns with one 16-byte load
// or store, otherwise with two 8-byte ones.  Against one column per lane
// this halves the load instructions and cross-lane reads per diagonal and
// doubles the bytes of each gather in flight.
//   * DIA part: each lane loads the value of row wave_base + lane (one
//     coalesced load per diagonal, non-temporal) and the lanes of row slot s
//     read the value of their row q from lane s + RPI*q (cross-lane read).
//   * CSR part, staged products: per chunk of the tile's entries, the
//     wavefronts form the rounded products w * X[col*ldx + c'] and store
//     them in LDS, with four columns per lane from KC = 4 on (independent
//     gathers of two 16-byte loads each, eight or more loads in flight per
//     lane; each value and column index is then read by KC/4 lanes instead
//     of KC/2; the DIA part keeps pairs, since with four columns per lane
//     each 16-byte load instruction covers only half of every row's cache
//     line); each lane then adds the products of its rows' entries in
//     column order, finding them through the tile's row pointers, which
//     are staged in LDS once per tile.
//   * CSR part, row gathers (RG): values and columns are staged instead and
//     each lane gathers the X rows of its own rows' entries, four at once up
//     to KC = 8 (the launcher's choice between the two is rm_row_gather).
#pragma once

#include "spmv_tile.h"

namespace mhdc {

template <int WG, int KC>
struct TileShapeRm {
    static_assert(KC >= 2 && KC <= 16 && (KC & (KC - 1)) == 0, "2..16 columns");
    static constexpr int P = 2;          // columns per lane
    static constexpr int LC = KC / P;    // lanes per row
    static constexpr int RPI = 64 / LC;  // rows per load instruction
    // remainder entries per chunk: 32 KB of products (staged products), or
    // 8 entries per lane of values and columns (row gathers); then the
    // tile's WG + 1 remainder row pointers
    static constexpr int CH = 4096 / KC;
    static constexpr int CHR = WG * 8;
    static constexpr int STAGE_BYTES = CH * KC * 8 > CHR * 12 ? CH * KC * 8 : CHR * 12;
    static constexpr int LDS_BYTES = STAGE_BYTES + (WG + 1) * 4;
    // staged products are formed with GP columns per lane (a lane's two
    // 16-byte loads per entry at 4 columns: half as many value and column
    // loads per product as with pairs), entry slots of GRPI entries per load
    static constexpr int GP = KC >= 4 ? 4 : 2;
    static constexpr int GLC = KC / GP;
    static constexpr int GRPI = 64 / GLC;
    static_assert(CH % (WG / 64 * GRPI) == 0, "chunk splits evenly over the slots");
    // products per lane and chunk
    static constexpr int PER_LANE = CH / (WG / 64) / GRPI;
    // diagonals in flight: four up to 8 columns (at 8 the DIA-only kernel
    // then holds 4 instead of 6 waves per SIMD and is still 8 % faster than
    // with two on the 7-point 256^3 matrix; 1-2 % at 3 and 4 columns), one
    // at 16 (two gained nothing there: registers)
    static constexpr int U = KC >= 16 ? 1 : 4;
};

typedef double rm_pair __attribute__((ext_vector_type(2)));

// The lane's P columns of one row of X at p, of which the first nl exist
// (the others read as zero): 16-byte loads of column pairs when pairs (p is
// then 16-byte aligned), 8-byte loads otherwise.
template <int P>
__device__ inline void rm_load(const double *__restrict__ p, int nl, bool pairs, double (&v)[P])
{
#pragma unroll
    for (int h = 0; h < P; h += 2) {
        if (pairs && nl >= h + 2) {
            const rm_pair t = *reinterpret_cast<const rm_pair *>(p + h);
            v[h] = t.x;
            v[h + 1] = t.y;
        } else {
            v[h] = nl > h ? p[h] : 0.0;
            v[h + 1] = nl > h + 1 ? p[h + 1] : 0.0;
        }
    }
}

// Stores the first nl of the lane's P columns to y (non-temporal), as
// rm_load reads them.
template <int P>
__device__ inline void rm_store(double *p, int nl, bool pairs, const double (&v)[P])
{
#pragma unroll
    for (int h = 0; h < P; h += 2) {
        if (pairs && nl >= h + 2) {
            rm_pair t;
            t.x = v[h];
            t.y = v[h + 1];
            __builtin_nontemporal_store(t, reinterpret_cast<rm_pair *>(p + h));
        } else {
            if (nl > h)
                __builtin_nontemporal_store(v[h], p + h);
            if (nl > h + 1)
                __builtin_nontemporal_store(v[h + 1], p + h + 1);
        }
    }
}

// RG: the CSR part's values and columns are staged and each lane gathers X
// for its own rows' entries (rows of similar structure, such as stencils,
// then read neighbouring rows of X in one load); otherwise the rounded
// products are staged (independent gathers, best for scattered columns).
// YC: Y is stored by column (element (i, r) at Y[r*ldy + i]) instead of by
// row; a template parameter, so that the kernels storing by row carry no
// trace of it (a runtime branch cost the 16-column kernel 3 %).
template <int WG, int KC, bool HAS_DIA, bool HAS_REM, bool RG, bool YC = false>
__device__ inline void spmv_tile_rm(const SpmvArgs &a, int64_t tile, void *lds)
{
    // products are rounded before they are added: no multiply-add fusion
#pragma clang fp contract(off)
    using Sh = TileShapeRm<WG, KC>;
    constexpr int P = Sh::P;
    constexpr int LC = Sh::LC;
    constexpr int RPI = Sh::RPI;
    constexpr int CH = Sh::CH;
    constexpr int U = Sh::U;
    const int n = a.n;
    const int64_t tile_base = tile * WG;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wave_base = tile_base + (int64_t)wave * 64;
    const int s = lane / LC, c0 = (lane % LC) * P;
    // the lane's columns that exist: nl of its P
    const int nl = a.k - c0 < 0 ? 0 : a.k - c0 > P ? P : a.k - c0;
    const bool l0 = nl > 0;
    const bool pairs = a.pairs;
    const double *__restrict__ X = a.X;
    const int64_t ldx = a.ldx;

    double acc[LC][P];
#pragma unroll
    for (int q = 0; q < LC; q++)
#pragma unroll
        for (int p = 0; p < P; p++)
            acc[q][p] = 0.0;

    static_assert(WG % 64 == 0 && 32 % (WG / 64) == 0, "tile must cover 64-row groups of one word");
    bool tile_rem = HAS_REM && a.has_rem;
    if (tile_rem && a.rem_mask) {
        const int64_t g0 = tile_base >> 6;
        const uint32_t word = uniform_load(a.rem_mask, g0 >> 5);
        tile_rem = ((word >> (g0 & 31)) & ((1u << (WG / 64)) - 1u)) != 0;
    }
    if (tile_rem) {
        const int64_t tile_end = tile_base + WG < n ? tile_base + WG : n;
        const int32_t e_beg = uniform_load(a.rem_ptr, tile_base);
        const int32_t e_end = uniform_load(a.rem_ptr, tile_end);
        if (e_beg < e_end) {
            double *s_prod = static_cast<double *>(lds);
            // the tile's row pointers, read once (each chunk looks them up)
            int32_t *s_rp = reinterpret_cast<int32_t *>(static_cast<char *>(lds) + Sh::STAGE_BYTES);
            for (int i = threadIdx.x; i <= WG; i += WG)
                s_rp[i] = tile_base + i <= n ? a.rem_ptr[tile_base + i] : e_end;
            if constexpr (RG) {
                constexpr int CHR = Sh::CHR;
                double *s_val = s_prod;
                int32_t *s_col = reinterpret_cast<int32_t *>(s_val + CHR);
                for (int32_t cb = e_beg; cb < e_end; cb += CHR) {
                    const int32_t ce = cb + CHR < e_end ? cb + CHR : e_end;
#pragma unroll
                    for (int j = 0; j < CHR / WG; j++) {
                        const int32_t e = cb + j * WG + (int32_t)threadIdx.x;
                        if (e < ce) {
                            s_val[e - cb] = __builtin_nontemporal_load(a.rem_val + e);
                            s_col[e - cb] = __builtin_nontemporal_load(a.rem_col + e);
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < LC; q++) {
                        const int64_t row = wave_base + s + RPI * q;
                        if (row < n && l0) {
                            const int r = (int)(row - tile_base);
                            const int32_t rs = s_rp[r], re = s_rp[r + 1];
                            const int32_t lo = rs > cb ? rs : cb;
                            const int32_t hi = re < ce ? re : ce;
                            int32_t e = lo;
                            // four entries at once up to 8 columns (twice the
                            // gathers in flight; at 16 columns the registers
                            // are spent), then two, then one: ascending order
                            if constexpr (KC <= 8) {
                                for (; e + 4 <= hi; e += 4) {
                                    double x0[P], x1[P], x2[P], x3[P];
                                    rm_load<P>(X + (int64_t)s_col[e - cb] * ldx + c0, nl, pairs, x0);
                                    rm_load<P>(X + (int64_t)s_col[e + 1 - cb] * ldx + c0, nl, pairs, x1);
                                    rm_load<P>(X + (int64_t)s_col[e + 2 - cb] * ldx + c0, nl, pairs, x2);
                                    rm_load<P>(X + (int64_t)s_col[e + 3 - cb] * ldx + c0, nl, pairs, x3);
                                    const double w0 = s_val[e - cb], w1 = s_val[e + 1 - cb];
                                    const double w2 = s_val[e + 2 - cb], w3 = s_val[e + 3 - cb];
#pragma unroll
                                    for (int p = 0; p < P; p++) {
                                        acc[q][p] = __dadd_rn(acc[q][p], __dmul_rn(w0, x0[p]));
                                        acc[q][p] = __dadd_rn(acc[q][p], __dmul_rn(w1, x1[p]));
                                        acc[q][p] = __dadd_rn(acc[q][p], __dmul_rn(w2, x2[p]));
                                        acc[q][p] = __dadd_rn(acc[q][p], __dmul_rn(w3, x3[p]));
                                    }
                                }
                            }
                            for (; e + 2 <= hi; e += 2) {
                                const double w0 = s_val[e - cb], w1 = s_val[e + 1 - cb];
                                double x0[P], x1[P];
                                rm_load<P>(X + (int64_t)s_col[e - cb] * ldx + c0, nl, pairs, x0);
                                rm_load<P>(X + (int64_t)s_col[e + 1 - cb] * ldx + c0, nl, pairs, x1);
#pragma unroll
                                for (int p = 0; p < P; p++) {
                                    acc[q][p] = __dadd_rn(acc[q][p], __dmul_rn(w0, x0[p]));
                                    acc[q][p] = __dadd_rn(acc[q][p], __dmul_rn(w1, x1[p]));
                                }
                            }
                            if (e < hi) {
                                double x0[P];
                                rm_load<P>(X + (int64_t)s_col[e - cb] * ldx + c0, nl, pairs, x0);
#pragma unroll
                                for (int p = 0; p < P; p++)
                                    acc[q][p] = __dadd_rn(acc[q][p], __dmul_rn(s_val[e - cb], x0[p]));
                            }
                        }
                    }
                    __syncthreads();
                }
            } else {
                for (int32_t cb = e_beg; cb < e_end; cb += CH) {
                    const int32_t ce = cb + CH < e_end ? cb + CH : e_end;
                    // products: wavefront w takes chunk positions [w*CH/W, (w+1)*CH/W);
                    // eight gathers in flight per lane
                    const int32_t wb = cb + wave * (CH / (WG / 64));
                    constexpr int GP = Sh::GP;
                    const int gs = lane / Sh::GLC, gc0 = (lane % Sh::GLC) * GP;
                    const int gnl = a.k - gc0 < 0 ? 0 : a.k - gc0 > GP ? GP : a.k - gc0;
#pragma unroll 8
                    for (int j = 0; j < Sh::PER_LANE; j++) {
                        const int32_t e = wb + gs + Sh::GRPI * j;
                        if (e < ce) {
                            const double w = __builtin_nontemporal_load(a.rem_val + e);
                            const int32_t col = __builtin_nontemporal_load(a.rem_col + e);
                            double xv[GP];
                            rm_load<GP>(X + (int64_t)col * ldx + gc0, gnl, pairs, xv);
#pragma unroll
                            for (int p = 0; p < GP; p++)
                                s_prod[(e - cb) * KC + gc0 + p] = __dmul_rn(w, xv[p]);
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < LC; q++) {
                        const int64_t row = wave_base + s + RPI * q;
                        if (row < n && l0) {
                            const int r = (int)(row - tile_base);
                            const int32_t rs = s_rp[r], re = s_rp[r + 1];
                            const int32_t lo = rs > cb ? rs : cb;
                            const int32_t hi = re < ce ? re : ce;
                            for (int32_t e = lo; e < hi; e++)
#pragma unroll
                                for (int p = 0; p < P; p++)
                                    acc[q][p] = __dadd_rn(acc[q][p], s_prod[(e - cb) * KC + c0 + p]);
                        }
                    }
                    __syncthreads();
                }
            }
        }
    }

    if (HAS_DIA && a.has_dia && wave_base < n) {
        if (a.uniform) {
            // all rows of this wavefront lie in block ib
            const int64_t ib = wave_base / a.n_b;
            const int32_t kb0 = uniform_load(a.dia_ptr, ib);
            const int32_t kb1 = uniform_load(a.dia_ptr, ib + 1);
            const int64_t t0 = wave_base - ib * a.n_b;
            // the one-block (HDC) layout has no slots past row n - 1
            const bool lrow = wave_base + lane < n;
            for (int32_t kk = kb0; kk < kb1; kk += U) {
                int64_t off[U];
                double wl[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const bool live = kk + u < kb1;
                    off[u] = uniform_load(a.dia_off, live ? kk + u : kb1 - 1);
                    wl[u] = live && lrow ? __builtin_nontemporal_load(
                                                   a.dia_val + (int64_t)(kk + u) * a.n_b + t0 + lane)
                                         : 0.0;
                }
                double xv[U][LC][P];
                bool in[U][LC];
#pragma unroll
                for (int u = 0; u < U; u++)
#pragma unroll
                    for (int q = 0; q < LC; q++) {
                        const int64_t row = wave_base + s + RPI * q;
                        const int64_t j = row + off[u];
                        in[u][q] = kk + u < kb1 && row < n && j >= 0 && j < n && l0;
                        rm_load<P>(X + (in[u][q] ? j : 0) * ldx + c0, in[u][q] ? nl : 0, pairs,
                                   xv[u][q]);
                    }
#pragma unroll
                for (int u = 0; u < U; u++)
#pragma unroll
                    for (int q = 0; q < LC; q++) {
                        // one lane per row: the lane's own value
                        const double w = LC == 1 ? wl[u] : __shfl(wl[u], s + RPI * q, 64);
                        if (in[u][q])
#pragma unroll
                            for (int p = 0; p < P; p++)
                                acc[q][p] = __dadd_rn(acc[q][p], __dmul_rn(w, xv[u][q][p]));
                    }
            }
        } else {
            // rows of one wavefront span several blocks: each row walks its
            // own block's list
#pragma unroll
            for (int q = 0; q < LC; q++) {
                const int64_t row = wave_base + s + RPI * q;
                if (row < n && l0) {
                    const int64_t ib = row / a.n_b;
                    const int64_t t = row - ib * a.n_b;
                    const int32_t kb0 = a.dia_ptr[ib], kb1 = a.dia_ptr[ib + 1];
                    for (int32_t kk = kb0; kk < kb1; kk++) {
                        const int64_t j = row + a.dia_off[kk];
                        if (j >= 0 && j < n) {
                            const double w = a.dia_val[(int64_t)kk * a.n_b + t];
                            double xv[P];
                            rm_load<P>(X + j * ldx + c0, nl, pairs, xv);
#pragma unroll
                            for (int p = 0; p < P; p++)
                                acc[q][p] = __dadd_rn(acc[q][p], __dmul_rn(w, xv[p]));
                        }
                    }
                }
            }
        }
    }

    if constexpr (YC) {
        if constexpr (HAS_REM) {
            // Y by column through LDS: the wavefront puts its 64 rows x KC
            // columns in its own region (column stride 65 doubles), then
            // stores each column's 64 rows as one contiguous 512-byte run.
            // The CSR part's staging area is free: its last chunk ended on
            // a barrier, and its row pointers are no longer read.
            static_assert(Sh::LDS_BYTES >= WG / 64 * KC * 65 * 8, "Y staging fits");
            __syncthreads();
            double *s_y = static_cast<double *>(lds) + wave * (KC * 65);
#pragma unroll
            for (int q = 0; q < LC; q++)
#pragma unroll
                for (int p = 0; p < P; p++)
                    if (p < nl)
                        s_y[(c0 + p) * 65 + s + RPI * q] = acc[q][p];
            __syncthreads();
            const int64_t row = wave_base + lane;
            if (row < n)
                for (int c = 0; c < a.k; c++)
                    __builtin_nontemporal_store(s_y[c * 65 + lane], a.Y + (int64_t)c * a.ldy + row);
        } else {
            // no LDS in this variant: the RPI row slots of one store write
            // RPI consecutive rows of each of the wavefront's columns
#pragma unroll
            for (int q = 0; q < LC; q++) {
                const int64_t row = wave_base + s + RPI * q;
                if (row < n && l0) {
#pragma unroll
                    for (int p = 0; p < P; p++)
                        if (p < nl)
                            __builtin_nontemporal_store(acc[q][p],
                                                        a.Y + (int64_t)(c0 + p) * a.ldy + row);
                }
            }
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < LC; q++) {
        const int64_t row = wave_base + s + RPI * q;
        if (row < n && l0) {
            rm_store<P>(a.Y + row * a.ldy + c0, nl, pairs, acc[q]);
        }
    }
}

}  // namespace mhdc
