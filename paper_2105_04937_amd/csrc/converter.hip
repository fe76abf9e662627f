// converter.hip -- CSR -> M-HDC / HDC / CSR handles, and M-HDC -> CSR.
//
// Steps (M-HDC, Sec. 4.3; HDC, Sec. 3.4), each a HIP kernel:
//   1. validate the CSR arrays (one lane per row, error bits in a flag);
//   2. census: for each row block count the nonzeros of every offset
//      d = j - i in an open-addressing hash table (in LDS, 512 to 8192
//      slots, the smallest that holds the largest block, when the
//      block holds fewer entries than that, else a per-block region of a
//      global table); only integer atomics on counts, so the counted set
//      does not depend on the order of the atomics;
//   3. select offsets with count/rows >= theta and order each block's list
//      ascending (rank sort: the kept offsets are distinct);
//   4. scan the per-block counts into dia_ptr;
//   5. scatter the kept nonzeros into dia_val[k*n_b + (i - ib*n_b)] and
//      count, then scan and write, the CSR remainder row by row.
// HDC counts N(d) over the whole matrix (per-chunk tables flushed into one
// dense count array), keeps d with N(d)/n >= theta by an order-preserving
// compaction, and is then laid out as one block of n rows.
#include "census.h"
#include "internal.h"

#include <climits>
#include <vector>

namespace mhdc {
namespace {

constexpr int CV_WG = CENSUS_WG;
constexpr int HDC_CENSUS_ROWS = 256;        // rows per HDC census chunk

inline unsigned grid_for(int64_t items, int per_block, int64_t cap = 1 << 22)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1)
        g = 1;
    if (g > cap)
        g = cap;
    return (unsigned)g;
}

// ---------------------------------------------------------------- validate
__global__ __launch_bounds__(CV_WG) void k_validate(int32_t n, int64_t nnz,
                                                    const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ colind,
                                                    int32_t *flag)
{
    for (int64_t i = (int64_t)blockIdx.x * CV_WG + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * CV_WG) {
        int64_t a = rowptr[i], b = rowptr[i + 1];
        if (a > b || a < 0 || b > nnz) {
            atomicOr(flag, 1);
            continue;
        }
        int32_t prev = -1;
        for (int64_t k = a; k < b; k++) {
            int32_t c = colind[k];
            if (c < 0 || c >= n || c <= prev) {
                atomicOr(flag, 2);
                break;
            }
            prev = c;
        }
    }
}

// Largest number of stored entries in one block of n_b rows.
__global__ __launch_bounds__(CV_WG) void k_block_max(int32_t n, int32_t n_b, int64_t n_blk,
                                                     const int32_t *__restrict__ rowptr,
                                                     int32_t *out)
{
    int32_t best = 0;
    for (int64_t ib = (int64_t)blockIdx.x * CV_WG + threadIdx.x; ib < n_blk;
         ib += (int64_t)gridDim.x * CV_WG) {
        int64_t r0 = ib * n_b, r1 = min((int64_t)n, r0 + n_b);
        best = max(best, rowptr[r1] - rowptr[r0]);
    }
    atomicMax(out, best);
}

// ---------------------------------------------------------------- census
// mode 0 (M-HDC): per block, select and sort the kept offsets:
//   Kb[ib] = number kept, sel_tmp[e0 .. e0+Kb) = kept offsets ascending,
//   with e0 = rowptr[ib*n_b] (a block keeps at most its entry count).
// mode 1 (HDC census): add each block's counts into hdc_count[d + n - 1].
// SLOTS: LDS hash-table slots, the smallest of 512 / 2048 / 4096 / 8192 that
// holds the largest block (small tables leave LDS for more resident workgroups:
// with 8192 slots only two fit per CU).
template <int SLOTS>
__global__ __launch_bounds__(CV_WG) void k_census(int mode, int32_t n, int32_t n_b, int64_t n_blk,
                                                  const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colind,
                                                  const double *__restrict__ val, double theta,
                                                  int32_t *Kb, int32_t *sel_tmp, int32_t *list_tmp,
                                                  int32_t *gkeys, int32_t *gcnts,
                                                  int32_t *hdc_count)
{
    static_assert(SLOTS >= 64 && SLOTS <= CENSUS_LDS_SLOTS && (SLOTS & (SLOTS - 1)) == 0,
                  "table slots");
    __shared__ int32_t s_keys[SLOTS];
    __shared__ int32_t s_cnts[SLOTS];
    __shared__ int32_t s_nsel;

    for (int64_t ib = blockIdx.x; ib < n_blk; ib += gridDim.x) {
        const int64_t r0 = ib * n_b, r1 = min((int64_t)n, r0 + n_b);
        const int64_t rows = r1 - r0;
        const int64_t e0 = rowptr[r0], e1 = rowptr[r1];

        if (threadIdx.x == 0)
            s_nsel = 0;
        int32_t *keys, *cnts;
        const uint32_t cap = census_block(r0, r1, e0, e1, rowptr, colind, val, s_keys, s_cnts,
                                          SLOTS, gkeys, gcnts, &keys, &cnts);

        for (uint32_t s = threadIdx.x; s < cap; s += CV_WG) {
            const int32_t key = keys[s];
            if (key == EMPTY_KEY)
                continue;
            const int32_t c = cnts[s];
            if (mode == 1) {
                atomicAdd(&hdc_count[(int64_t)key + n - 1], c);
            } else if (c >= 1 && (double)c / (double)rows >= theta) {
                int32_t p = atomicAdd(&s_nsel, 1);
                list_tmp[e0 + p] = key;
            }
        }
        __syncthreads();

        if (mode == 0) {
            const int32_t nsel = s_nsel;
            for (int32_t s = threadIdx.x; s < nsel; s += CV_WG) {
                const int32_t key = list_tmp[e0 + s];
                int32_t rank = 0;
                for (int32_t t = 0; t < nsel; t++)
                    rank += list_tmp[e0 + t] < key;
                sel_tmp[e0 + rank] = key;
            }
            if (threadIdx.x == 0)
                Kb[ib] = nsel;
        }
        __syncthreads();
    }
}

// dia_off[dia_ptr[ib] + t] = sel_tmp[rowptr[ib*n_b] + t]
__global__ __launch_bounds__(CV_WG) void k_gather_offsets(int32_t n_b, int64_t n_blk,
                                                          const int32_t *__restrict__ rowptr,
                                                          const int32_t *__restrict__ dia_ptr,
                                                          const int32_t *__restrict__ sel_tmp,
                                                          int32_t *dia_off)
{
    for (int64_t ib = blockIdx.x; ib < n_blk; ib += gridDim.x) {
        const int64_t e0 = rowptr[ib * n_b];
        const int32_t k0 = dia_ptr[ib], kb = dia_ptr[ib + 1] - k0;
        for (int32_t t = threadIdx.x; t < kb; t += CV_WG)
            dia_off[k0 + t] = sel_tmp[e0 + t];
    }
}

// HDC: flag[q] = 1 iff offset q - (n-1) is kept (N(d)/n >= theta).
__global__ __launch_bounds__(CV_WG) void k_hdc_flags(int32_t n, int64_t span,
                                                     const int32_t *__restrict__ cnt,
                                                     double theta, int32_t *flag)
{
    for (int64_t q = (int64_t)blockIdx.x * CV_WG + threadIdx.x; q < span;
         q += (int64_t)gridDim.x * CV_WG) {
        const int32_t c = cnt[q];
        flag[q] = (c >= 1 && (double)c / (double)n >= theta) ? 1 : 0;
    }
}

__global__ __launch_bounds__(CV_WG) void k_hdc_compact(int32_t n, int64_t span,
                                                       const int32_t *__restrict__ flag,
                                                       const int32_t *__restrict__ pos,
                                                       int32_t *dia_off)
{
    for (int64_t q = (int64_t)blockIdx.x * CV_WG + threadIdx.x; q < span;
         q += (int64_t)gridDim.x * CV_WG)
        if (flag[q])
            dia_off[pos[q]] = (int32_t)(q - (n - 1));
}

__global__ __launch_bounds__(CV_WG) void k_fill_f64(double *p, int64_t count, double v)
{
    for (int64_t s = (int64_t)blockIdx.x * CV_WG + threadIdx.x; s < count;
         s += (int64_t)gridDim.x * CV_WG)
        p[s] = v;
}

// Position of offset d in the block's ascending list dia_off[lo, hi), or -1.
__device__ inline int32_t find_offset(const int32_t *__restrict__ dia_off, int32_t lo,
                                      int32_t hi, int32_t d)
{
    int32_t a = lo, b = hi;
    while (a < b) {
        int32_t mid = (a + b) >> 1;
        if (dia_off[mid] < d)
            a = mid + 1;
        else
            b = mid;
    }
    return (a < hi && dia_off[a] == d) ? a : -1;
}

// Scatter the kept nonzeros of every row into its segment slot and count
// the entries left for the remainder.
__global__ __launch_bounds__(CV_WG) void k_split_rows(int32_t n, int32_t n_b,
                                                      const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ colind,
                                                      const double *__restrict__ val,
                                                      const int32_t *__restrict__ dia_ptr,
                                                      const int32_t *__restrict__ dia_off,
                                                      double *dia_val, int32_t *remcnt)
{
    for (int64_t i = (int64_t)blockIdx.x * CV_WG + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * CV_WG) {
        const int64_t ib = i / n_b, t = i - ib * n_b;
        const int32_t kb0 = dia_ptr[ib], kb1 = dia_ptr[ib + 1];
        int32_t cnt = 0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; k++) {
            const double v = val[k];
            int32_t p = -1;
            if (v != 0.0 && kb1 > kb0)
                p = find_offset(dia_off, kb0, kb1, colind[k] - (int32_t)i);
            if (p >= 0)
                dia_val[(int64_t)p * n_b + t] = v;
            else
                cnt++;
        }
        remcnt[i] = cnt;
    }
}

__global__ __launch_bounds__(CV_WG) void k_scatter_rem(int32_t n, int32_t n_b,
                                                       const int32_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ colind,
                                                       const double *__restrict__ val,
                                                       const int32_t *__restrict__ dia_ptr,
                                                       const int32_t *__restrict__ dia_off,
                                                       const int32_t *__restrict__ rem_ptr,
                                                       int32_t *rem_col, double *rem_val)
{
    for (int64_t i = (int64_t)blockIdx.x * CV_WG + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * CV_WG) {
        const int64_t ib = i / n_b;
        const int32_t kb0 = dia_ptr[ib], kb1 = dia_ptr[ib + 1];
        int32_t q = rem_ptr[i];
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; k++) {
            const double v = val[k];
            const int32_t c = colind[k];
            int32_t p = -1;
            if (v != 0.0 && kb1 > kb0)
                p = find_offset(dia_off, kb0, kb1, c - (int32_t)i);
            if (p < 0) {
                rem_col[q] = c;
                rem_val[q] = v;
                q++;
            }
        }
    }
}

// One lane per 32-bit word of the remainder mask: bit b of word w is set
// when rows [64(32w+b), 64(32w+b)+64) hold remainder entries.
__global__ __launch_bounds__(CV_WG) void k_rem_mask(int32_t n, int64_t words,
                                                    const int32_t *__restrict__ rem_ptr,
                                                    uint32_t *__restrict__ mask)
{
    for (int64_t w = (int64_t)blockIdx.x * CV_WG + threadIdx.x; w < words;
         w += (int64_t)gridDim.x * CV_WG) {
        uint32_t bits = 0;
        for (int b = 0; b < 32; b++) {
            const int64_t r0 = (w * 32 + b) * 64;
            if (r0 >= n)
                break;
            const int64_t r1 = r0 + 64 < n ? r0 + 64 : n;
            if (rem_ptr[r1] > rem_ptr[r0])
                bits |= 1u << b;
        }
        mask[w] = bits;
    }
}

// Largest |offset| over the K selected diagonals (offsets lie in (-n, n), so
// the absolute value fits int32): one atomic per wavefront.
__global__ __launch_bounds__(CV_WG) void k_max_abs_offset(int64_t K, const int32_t *__restrict__ off,
                                                          int32_t *out)
{
    int32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * CV_WG + threadIdx.x; i < K;
         i += (int64_t)gridDim.x * CV_WG) {
        const int32_t v = off[i] < 0 ? -off[i] : off[i];
        m = v > m ? v : m;
    }
    for (int sh = 32; sh >= 1; sh >>= 1) {
        const int32_t o = __shfl_xor(m, sh, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m > 0)
        atomicMax(out, m);
}

// Columns within LONE_REACH (16 doubles, one 128-byte line) count as near.
constexpr int32_t LONE_REACH = 16;

// Advances p over the ascending columns col[p, e) below j - LONE_REACH and
// reports whether the next one lies within LONE_REACH of j.  For ascending
// j the pointer only moves forward: one merge pass over the row.
__device__ inline bool near_merge(const int32_t *__restrict__ col, int32_t &p, int32_t e, int32_t j)
{
    const int64_t lo_col = (int64_t)j - LONE_REACH;
    while (p < e && (int64_t)col[p] < lo_col)
        p++;
    return p < e && (int64_t)col[p] <= (int64_t)j + LONE_REACH;
}

// One lane per row of a CSR-shaped pair (ptr, col): cnt[0] counts the rows
// with entries, cnt[1] those of them whose column offsets col - row repeat
// the previous row's (same length, same offsets in order), cnt[2] the lone
// entries: those with no column within LONE_REACH (16 doubles, one 128-byte
// line) in either of the two previous rows.  Where most rows repeat
// (stencils), the lanes of a wavefront gathering x for their own rows read
// neighbouring elements; a lone entry's gather shares no cache line with
// its neighbours' rows, one line per right-hand side stored by column.
__global__ __launch_bounds__(CV_WG) void k_row_repeat(int32_t n, const int32_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ col,
                                                      unsigned long long *cnt)
{
    uint32_t ne = 0, rep = 0;
    unsigned long long lone = 0;
    for (int64_t i = (int64_t)blockIdx.x * CV_WG + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * CV_WG) {
        const int32_t b1 = ptr[i], e1 = ptr[i + 1];
        if (e1 == b1)
            continue;
        ne++;
        {
            // rows before the first hold no columns
            const int32_t bm1 = i >= 1 ? ptr[i - 1] : b1, bm2 = i >= 2 ? ptr[i - 2] : bm1;
            int32_t p1 = bm1, p2 = bm2;
            for (int32_t e = b1; e < e1; e++) {
                const int32_t j = col[e];
                const bool n1 = near_merge(col, p1, b1, j);
                const bool n2 = near_merge(col, p2, bm1, j);
                lone += n1 || n2 ? 0u : 1u;
            }
        }
        if (i == 0)
            continue;
        const int32_t b0 = ptr[i - 1];
        if (b1 - b0 != e1 - b1)
            continue;
        // no early exit: the loads of a row issue together
        bool same = true;
        for (int32_t e = 0; e < e1 - b1; e++)
            same &= (int64_t)col[b1 + e] - i == (int64_t)col[b0 + e] - (i - 1);
        rep += same ? 1u : 0u;
    }
    // one pair of atomics per workgroup (on a few thousand workgroups):
    // per-wavefront atomics on the two counters serialised for milliseconds
    for (int sh = 32; sh >= 1; sh >>= 1) {
        ne += __shfl_xor(ne, sh, 64);
        rep += __shfl_xor(rep, sh, 64);
        lone += __shfl_xor(lone, sh, 64);
    }
    __shared__ unsigned long long s_sum[3][CV_WG / 64];
    if ((threadIdx.x & 63) == 0) {
        s_sum[0][threadIdx.x >> 6] = ne;
        s_sum[1][threadIdx.x >> 6] = rep;
        s_sum[2][threadIdx.x >> 6] = lone;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0, c = 0;
        for (int w = 0; w < CV_WG / 64; w++) {
            a += s_sum[0][w];
            b += s_sum[1][w];
            c += s_sum[2][w];
        }
        atomicAdd(cnt, a);
        atomicAdd(cnt + 1, b);
        atomicAdd(cnt + 2, c);
    }
}

// ---------------------------------------------------------------- decode
__global__ __launch_bounds__(CV_WG) void k_decode_count(int32_t n, int32_t n_b,
                                                        const int32_t *__restrict__ dia_ptr,
                                                        const int32_t *__restrict__ dia_off,
                                                        const double *__restrict__ dia_val,
                                                        const int32_t *__restrict__ rem_ptr,
                                                        int32_t *cnt)
{
    for (int64_t i = (int64_t)blockIdx.x * CV_WG + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * CV_WG) {
        const int64_t ib = i / n_b, t = i - ib * n_b;
        int32_t c = rem_ptr[i + 1] - rem_ptr[i];
        for (int32_t k = dia_ptr[ib]; k < dia_ptr[ib + 1]; k++) {
            const int64_t j = i + dia_off[k];
            if (j >= 0 && j < n && dia_val[(int64_t)k * n_b + t] != 0.0)
                c++;
        }
        cnt[i] = c;
    }
}

__global__ __launch_bounds__(CV_WG) void k_decode_write(int32_t n, int32_t n_b,
                                                        const int32_t *__restrict__ dia_ptr,
                                                        const int32_t *__restrict__ dia_off,
                                                        const double *__restrict__ dia_val,
                                                        const int32_t *__restrict__ rem_ptr,
                                                        const int32_t *__restrict__ rem_col,
                                                        const double *__restrict__ rem_val,
                                                        const int32_t *__restrict__ out_ptr,
                                                        int32_t *out_col, double *out_val)
{
    for (int64_t i = (int64_t)blockIdx.x * CV_WG + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * CV_WG) {
        const int64_t ib = i / n_b, t = i - ib * n_b;
        int32_t k = dia_ptr[ib];
        const int32_t kend = dia_ptr[ib + 1];
        int32_t q = rem_ptr[i];
        const int32_t qend = rem_ptr[i + 1];
        int32_t e = out_ptr[i];
        for (;;) {
            while (k < kend) {
                const int64_t j = i + dia_off[k];
                if (j >= 0 && j < n && dia_val[(int64_t)k * n_b + t] != 0.0)
                    break;
                k++;
            }
            const bool hd = k < kend, hr = q < qend;
            if (!hd && !hr)
                break;
            const bool take_d = hd && (!hr || (int64_t)i + dia_off[k] < rem_col[q]);
            if (take_d) {
                out_col[e] = (int32_t)(i + dia_off[k]);
                out_val[e] = dia_val[(int64_t)k * n_b + t];
                k++;
            } else {
                out_col[e] = rem_col[q];
                out_val[e] = rem_val[q];
                q++;
            }
            e++;
        }
    }
}

// Frees every pointer registered with it unless release() was called.
struct TempSet {
    std::vector<void *> ptrs;
    void *add(void *p)
    {
        ptrs.push_back(p);
        return p;
    }
    ~TempSet()
    {
        for (void *p : ptrs)
            dfree(p);
    }
};

int launch_ok(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return MHDC_OK;
}

int sync_ok(const char *what)
{
    hipError_t e = hipStreamSynchronize(0);
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return launch_ok(what);
}

}  // namespace

// ---------------------------------------------------------------- host side
int validate_csr(int32_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                 int64_t *nnz_out)
{
    if (n < 0)
        return set_error(MHDC_ERR_INVALID_ARG, "n must be >= 0");
    if (!rowptr)
        return set_error(MHDC_ERR_INVALID_ARG, "rowptr is NULL");
    int32_t ends[2] = {0, 0};
    MHDC_HIP_CHECK(hipMemcpy(&ends[0], rowptr, sizeof(int32_t), hipMemcpyDeviceToHost));
    MHDC_HIP_CHECK(hipMemcpy(&ends[1], rowptr + n, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (ends[0] != 0)
        return set_error(MHDC_ERR_BAD_CSR, "rowptr[0] must be 0");
    if (ends[1] < 0)
        return set_error(MHDC_ERR_BAD_CSR, "rowptr[n] (nnz) is negative");
    const int64_t nnz = ends[1];
    if (nnz > MAX_NNZ)
        return set_error(MHDC_ERR_SIZE, "nnz must be at most 2^31 - 4097");
    if (nnz > 0 && (!colind || !val))
        return set_error(MHDC_ERR_INVALID_ARG, "colind/val is NULL");
    if (n > 0) {
        int32_t *flag = nullptr;
        int rc = dmalloc((void **)&flag, sizeof(int32_t), "validation flag");
        if (rc)
            return rc;
        (void)hipMemsetAsync(flag, 0, sizeof(int32_t), 0);
        k_validate<<<grid_for(n, CV_WG, 1 << 16), CV_WG, 0, 0>>>(n, nnz, rowptr, colind, flag);
        int32_t h = 0;
        hipError_t e = hipMemcpy(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost);
        dfree(flag);
        if (e != hipSuccess)
            return set_error(MHDC_ERR_HIP, std::string("validation: ") + hipGetErrorString(e));
        if (h & 1)
            return set_error(MHDC_ERR_BAD_CSR, "rowptr is not non-decreasing within [0, nnz]");
        if (h & 2)
            return set_error(MHDC_ERR_BAD_CSR,
                             "column index out of range, unsorted or duplicated in a row");
    }
    *nnz_out = nnz;
    return MHDC_OK;
}

// Largest |offset| of the K diagonals in off (k_max_abs_offset).
int max_abs_offset(int64_t K, const int32_t *off, int32_t *far)
{
    *far = 0;
    if (K <= 0)
        return MHDC_OK;
    int32_t *d = nullptr;
    int rc = dmalloc((void **)&d, sizeof(int32_t), "offset maximum");
    if (rc)
        return rc;
    TempSet tmp;
    tmp.add(d);
    MHDC_HIP_CHECK(hipMemset(d, 0, sizeof(int32_t)));
    k_max_abs_offset<<<grid_for(K, CV_WG, 1 << 10), CV_WG, 0, 0>>>(K, off, d);
    if ((rc = launch_ok("offset maximum")))
        return rc;
    MHDC_HIP_CHECK(hipMemcpy(far, d, sizeof(int32_t), hipMemcpyDeviceToHost));
    return MHDC_OK;
}

// Share of the CSR part's nonempty rows that repeat the previous row's
// column offsets, and its lone entries per row (k_row_repeat); both 0 for
// an empty CSR part.
int row_repeat_share(int32_t n, const int32_t *ptr, const int32_t *col, double *share,
                     double *lone_per_row)
{
    *share = 0.0;
    *lone_per_row = 0.0;
    if (n < 1)
        return MHDC_OK;
    unsigned long long *cnt = nullptr;
    int rc = dmalloc((void **)&cnt, 3 * sizeof(unsigned long long), "row repeat counts");
    if (rc)
        return rc;
    TempSet tmp;
    tmp.add(cnt);
    MHDC_HIP_CHECK(hipMemset(cnt, 0, 3 * sizeof(unsigned long long)));
    k_row_repeat<<<grid_for(n, CV_WG, 1 << 12), CV_WG, 0, 0>>>(n, ptr, col, cnt);
    if ((rc = launch_ok("row repeat")))
        return rc;
    unsigned long long h[3] = {0, 0, 0};
    MHDC_HIP_CHECK(hipMemcpy(h, cnt, sizeof(h), hipMemcpyDeviceToHost));
    *share = h[0] > 0 ? (double)h[1] / (double)h[0] : 0.0;
    *lone_per_row = (double)h[2] / (double)n;
    return MHDC_OK;
}

void free_matrix(BdcMatrix &m)
{
    dfree(m.dia_ptr);
    dfree(m.dia_off);
    dfree(m.dia_val);
    dfree(m.rem_ptr);
    dfree(m.rem_col);
    dfree(m.rem_val);
    dfree(m.rem_mask);
    m.dia_ptr = m.dia_off = m.rem_ptr = m.rem_col = nullptr;
    m.dia_val = m.rem_val = nullptr;
    m.rem_mask = nullptr;
}

// Census launch with the smallest LDS table that holds a block of hmax
// entries (more entries than 8191 go to the global table).
void launch_census(int64_t grid, int64_t hmax, int mode, int32_t n, int32_t n_b, int64_t n_blk,
                   const int32_t *rowptr, const int32_t *colind, const double *val, double theta,
                   int32_t *Kb, int32_t *sel_tmp, int32_t *list_tmp, int32_t *gkeys,
                   int32_t *gcnts, int32_t *hdc_count)
{
    const unsigned g = grid_for(grid, 1, 1 << 20);
    if (hmax < 256)
        k_census<512><<<g, CV_WG, 0, 0>>>(mode, n, n_b, n_blk, rowptr, colind, val, theta, Kb,
                                            sel_tmp, list_tmp, gkeys, gcnts, hdc_count);
    else if (hmax < 1024)
        k_census<2048><<<g, CV_WG, 0, 0>>>(mode, n, n_b, n_blk, rowptr, colind, val, theta, Kb,
                                             sel_tmp, list_tmp, gkeys, gcnts, hdc_count);
    else if (hmax < 2048)
        k_census<4096><<<g, CV_WG, 0, 0>>>(mode, n, n_b, n_blk, rowptr, colind, val, theta, Kb,
                                             sel_tmp, list_tmp, gkeys, gcnts, hdc_count);
    else
        k_census<CENSUS_LDS_SLOTS><<<g, CV_WG, 0, 0>>>(mode, n, n_b, n_blk, rowptr, colind, val,
                                                         theta, Kb, sel_tmp, list_tmp, gkeys,
                                                         gcnts, hdc_count);
}

int build_blocked(BdcMatrix &m, const int32_t *rowptr, const int32_t *colind, const double *val)
{
    const int32_t n = m.n;
    int64_t nnz = 0;
    int rc = validate_csr(n, rowptr, colind, val, &nnz);
    if (rc)
        return rc;
    m.nnz = nnz;
    if (m.kind == KIND_HDC)
        m.n_b = n > 0 ? n : 1;
    const int32_t n_b = m.n_b;
    const int64_t n_blk = n == 0 ? 0 : ((int64_t)n + n_b - 1) / n_b;
    m.n_blk = n_blk;

    TempSet tmp;
    rc = dmalloc((void **)&m.dia_ptr, sizeof(int32_t) * (size_t)(n_blk + 1), "dia_ptr");
    if (rc)
        return rc;
    rc = dmalloc((void **)&m.rem_ptr, sizeof(int32_t) * (size_t)(n + 1), "rem_ptr");
    if (rc)
        return rc;
    if (n == 0) {
        MHDC_HIP_CHECK(hipMemset(m.dia_ptr, 0, sizeof(int32_t)));
        MHDC_HIP_CHECK(hipMemset(m.rem_ptr, 0, sizeof(int32_t)));
        return MHDC_OK;
    }
    const size_t nz1 = (size_t)(nnz > 0 ? nnz : 1);

    int64_t K = 0;
    if (m.kind == KIND_MHDC) {
        int32_t *Kb = nullptr, *sel_tmp = nullptr, *list_tmp = nullptr, *bmax = nullptr;
        int32_t *gkeys = nullptr, *gcnts = nullptr;
        if ((rc = dmalloc((void **)&Kb, sizeof(int32_t) * (size_t)n_blk, "block counts")))
            return rc;
        tmp.add(Kb);
        if ((rc = dmalloc((void **)&sel_tmp, sizeof(int32_t) * nz1, "census list")))
            return rc;
        tmp.add(sel_tmp);
        if ((rc = dmalloc((void **)&list_tmp, sizeof(int32_t) * nz1, "census list")))
            return rc;
        tmp.add(list_tmp);
        if ((rc = dmalloc((void **)&bmax, sizeof(int32_t), "block max")))
            return rc;
        tmp.add(bmax);
        MHDC_HIP_CHECK(hipMemsetAsync(bmax, 0, sizeof(int32_t), 0));
        k_block_max<<<grid_for(n_blk, CV_WG, 1 << 14), CV_WG, 0, 0>>>(n, n_b, n_blk, rowptr, bmax);
        int32_t hmax = 0;
        MHDC_HIP_CHECK(hipMemcpy(&hmax, bmax, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (hmax >= CENSUS_LDS_SLOTS) {
            if ((rc = dmalloc((void **)&gkeys, sizeof(int32_t) * 2 * nz1, "census table")))
                return rc;
            tmp.add(gkeys);
            if ((rc = dmalloc((void **)&gcnts, sizeof(int32_t) * 2 * nz1, "census table")))
                return rc;
            tmp.add(gcnts);
        }
        launch_census(n_blk, hmax, 0, n, n_b, n_blk, rowptr, colind, val, m.theta, Kb, sel_tmp,
                      list_tmp, gkeys, gcnts, nullptr);
        if ((rc = launch_ok("census")))
            return rc;
        if ((rc = exclusive_scan_i32(Kb, m.dia_ptr, n_blk, &K, 0)))
            return rc;
        m.K = K;
        if (K > 0) {
            if ((rc = dmalloc((void **)&m.dia_off, sizeof(int32_t) * (size_t)K, "dia_off")))
                return rc;
            k_gather_offsets<<<grid_for(n_blk, 1, 1 << 20), CV_WG, 0, 0>>>(
                n_b, n_blk, rowptr, m.dia_ptr, sel_tmp, m.dia_off);
            if ((rc = launch_ok("gather offsets")))
                return rc;
        }
    } else {
        // HDC: global census over chunks, then select over all offsets.
        const int64_t span = 2 * (int64_t)n - 1;
        const int64_t n_chunk = ((int64_t)n + HDC_CENSUS_ROWS - 1) / HDC_CENSUS_ROWS;
        int32_t *gcount = nullptr, *flag = nullptr, *pos = nullptr, *gkeys = nullptr,
                *gcnts = nullptr, *bmax = nullptr;
        if ((rc = dmalloc((void **)&gcount, sizeof(int32_t) * (size_t)span, "offset counts")))
            return rc;
        tmp.add(gcount);
        MHDC_HIP_CHECK(hipMemsetAsync(gcount, 0, sizeof(int32_t) * (size_t)span, 0));
        if ((rc = dmalloc((void **)&bmax, sizeof(int32_t), "block max")))
            return rc;
        tmp.add(bmax);
        MHDC_HIP_CHECK(hipMemsetAsync(bmax, 0, sizeof(int32_t), 0));
        k_block_max<<<grid_for(n_chunk, CV_WG, 1 << 14), CV_WG, 0, 0>>>(n, HDC_CENSUS_ROWS,
                                                                        n_chunk, rowptr, bmax);
        int32_t hmax = 0;
        MHDC_HIP_CHECK(hipMemcpy(&hmax, bmax, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (hmax >= CENSUS_LDS_SLOTS) {
            if ((rc = dmalloc((void **)&gkeys, sizeof(int32_t) * 2 * nz1, "census table")))
                return rc;
            tmp.add(gkeys);
            if ((rc = dmalloc((void **)&gcnts, sizeof(int32_t) * 2 * nz1, "census table")))
                return rc;
            tmp.add(gcnts);
        }
        launch_census(n_chunk, hmax, 1, n, HDC_CENSUS_ROWS, n_chunk, rowptr, colind, val, m.theta,
                      nullptr, nullptr, nullptr, gkeys, gcnts, gcount);
        if ((rc = launch_ok("hdc census")))
            return rc;
        if ((rc = dmalloc((void **)&flag, sizeof(int32_t) * (size_t)span, "offset flags")))
            return rc;
        tmp.add(flag);
        if ((rc = dmalloc((void **)&pos, sizeof(int32_t) * (size_t)(span + 1), "offset pos")))
            return rc;
        tmp.add(pos);
        k_hdc_flags<<<grid_for(span, CV_WG, 1 << 16), CV_WG, 0, 0>>>(n, span, gcount, m.theta,
                                                                     flag);
        if ((rc = exclusive_scan_i32(flag, pos, span, &K, 0)))
            return rc;
        m.K = K;
        int32_t hptr[2] = {0, (int32_t)K};
        MHDC_HIP_CHECK(hipMemcpy(m.dia_ptr, hptr, sizeof(hptr), hipMemcpyHostToDevice));
        if (K > 0) {
            if ((rc = dmalloc((void **)&m.dia_off, sizeof(int32_t) * (size_t)K, "dia_off")))
                return rc;
            k_hdc_compact<<<grid_for(span, CV_WG, 1 << 16), CV_WG, 0, 0>>>(n, span, flag, pos,
                                                                           m.dia_off);
            if ((rc = launch_ok("hdc compact")))
                return rc;
        }
    }

    if ((rc = max_abs_offset(K, m.dia_off, &m.far_offset)))
        return rc;

    // DIA values: K * n_b slots, +0.0 padding.
    m.S = K * (int64_t)n_b;
    if (m.S > 0) {
        size_t fr = 0, tot = 0;
        MHDC_HIP_CHECK(hipMemGetInfo(&fr, &tot));
        const double need = 8.0 * (double)m.S;
        if (need > (double)fr)
            return set_error(MHDC_ERR_OOM, "DIA part needs " + std::to_string(need / 1e9) +
                                               " GB, " + std::to_string(fr / 1e9) + " GB free");
        if ((rc = dmalloc((void **)&m.dia_val, sizeof(double) * (size_t)m.S, "dia_val")))
            return rc;
        k_fill_f64<<<grid_for(m.S, CV_WG, 1 << 16), CV_WG, 0, 0>>>(m.dia_val, m.S, 0.0);
    }

    int32_t *remcnt = nullptr;
    if ((rc = dmalloc((void **)&remcnt, sizeof(int32_t) * (size_t)n, "remainder counts")))
        return rc;
    tmp.add(remcnt);
    k_split_rows<<<grid_for(n, CV_WG, 1 << 16), CV_WG, 0, 0>>>(n, n_b, rowptr, colind, val,
                                                               m.dia_ptr, m.dia_off, m.dia_val,
                                                               remcnt);
    if ((rc = launch_ok("split rows")))
        return rc;
    int64_t R = 0;
    if ((rc = exclusive_scan_i32(remcnt, m.rem_ptr, n, &R, 0)))
        return rc;
    m.R = R;
    if (R > 0) {
        if ((rc = dmalloc((void **)&m.rem_col, sizeof(int32_t) * (size_t)R, "rem_col")))
            return rc;
        if ((rc = dmalloc((void **)&m.rem_val, sizeof(double) * (size_t)R, "rem_val")))
            return rc;
        k_scatter_rem<<<grid_for(n, CV_WG, 1 << 16), CV_WG, 0, 0>>>(
            n, n_b, rowptr, colind, val, m.dia_ptr, m.dia_off, m.rem_ptr, m.rem_col, m.rem_val);
        const int64_t words = rem_mask_words(n);
        if ((rc = dmalloc((void **)&m.rem_mask, sizeof(uint32_t) * (size_t)words, "rem_mask")))
            return rc;
        k_rem_mask<<<grid_for(words, CV_WG, 1 << 16), CV_WG, 0, 0>>>(n, words, m.rem_ptr,
                                                                     m.rem_mask);
        if ((rc = launch_ok("remainder mask")))
            return rc;
        // Keep the mask only where most row groups have no remainder: where
        // most have one, testing it first would only add a round trip.
        std::vector<uint32_t> h((size_t)words);
        MHDC_HIP_CHECK(hipMemcpy(h.data(), m.rem_mask, sizeof(uint32_t) * (size_t)words,
                                 hipMemcpyDeviceToHost));
        int64_t set = 0;
        for (uint32_t w : h)
            set += __builtin_popcount(w);
        if (2 * set > ((int64_t)n + 63) / 64) {
            dfree(m.rem_mask);
            m.rem_mask = nullptr;
        }
        if ((rc = row_repeat_share(n, m.rem_ptr, m.rem_col, &m.row_repeat, &m.lone_per_row)))
            return rc;
    }
    return sync_ok("conversion");
}

int build_csr(BdcMatrix &m, const int32_t *rowptr, const int32_t *colind, const double *val)
{
    const int32_t n = m.n;
    int64_t nnz = 0;
    int rc = validate_csr(n, rowptr, colind, val, &nnz);
    if (rc)
        return rc;
    m.nnz = nnz;
    m.n_b = 0;
    m.n_blk = 0;
    m.K = m.S = 0;
    m.R = nnz;
    if ((rc = dmalloc((void **)&m.rem_ptr, sizeof(int32_t) * (size_t)(n + 1), "rowptr")))
        return rc;
    MHDC_HIP_CHECK(hipMemcpy(m.rem_ptr, rowptr, sizeof(int32_t) * (size_t)(n + 1),
                             hipMemcpyDeviceToDevice));
    if (nnz > 0) {
        if ((rc = dmalloc((void **)&m.rem_col, sizeof(int32_t) * (size_t)nnz, "colind")))
            return rc;
        if ((rc = dmalloc((void **)&m.rem_val, sizeof(double) * (size_t)nnz, "val")))
            return rc;
        MHDC_HIP_CHECK(hipMemcpy(m.rem_col, colind, sizeof(int32_t) * (size_t)nnz,
                                 hipMemcpyDeviceToDevice));
        MHDC_HIP_CHECK(hipMemcpy(m.rem_val, val, sizeof(double) * (size_t)nnz,
                                 hipMemcpyDeviceToDevice));
        if ((rc = row_repeat_share(n, m.rem_ptr, m.rem_col, &m.row_repeat, &m.lone_per_row)))
            return rc;
    }
    return sync_ok("csr copy");
}

int decode_to_csr(const BdcMatrix &m, int32_t *rowptr, int32_t *colind, double *val)
{
    const int32_t n = m.n;
    if (!rowptr)
        return set_error(MHDC_ERR_INVALID_ARG, "rowptr is NULL");
    if (n == 0) {
        MHDC_HIP_CHECK(hipMemset(rowptr, 0, sizeof(int32_t)));
        return MHDC_OK;
    }
    if (m.nnz > 0 && (!colind || !val))
        return set_error(MHDC_ERR_INVALID_ARG, "colind/val is NULL");
    TempSet tmp;
    int32_t *cnt = nullptr;
    int rc = dmalloc((void **)&cnt, sizeof(int32_t) * (size_t)n, "decode counts");
    if (rc)
        return rc;
    tmp.add(cnt);
    k_decode_count<<<grid_for(n, CV_WG, 1 << 16), CV_WG, 0, 0>>>(n, m.n_b, m.dia_ptr, m.dia_off,
                                                                 m.dia_val, m.rem_ptr, cnt);
    int64_t total = 0;
    if ((rc = exclusive_scan_i32(cnt, rowptr, n, &total, 0)))
        return rc;
    if (total != m.nnz)
        return set_error(MHDC_ERR_BAD_CSR, "decoded entry count differs from nnz");
    k_decode_write<<<grid_for(n, CV_WG, 1 << 16), CV_WG, 0, 0>>>(
        n, m.n_b, m.dia_ptr, m.dia_off, m.dia_val, m.rem_ptr, m.rem_col, m.rem_val, rowptr,
        colind, val);
    return sync_ok("decode");
}

}  // namespace mhdc
