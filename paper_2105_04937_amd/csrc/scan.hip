// scan.hip -- exclusive prefix sum used by the converter to lay out the
// per-block diagonal lists (dia_ptr) and the CSR remainder (rem_ptr).
//
// Three passes over chunks of SCAN_CHUNK elements: per-chunk totals, one
// workgroup scanning those totals (int64, so an overflow of the int32
// result is detected), and a per-chunk scan that adds the chunk's offset.
#include "internal.h"

namespace mhdc {
namespace {

constexpr int SCAN_WG = 256;
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_CHUNK = SCAN_WG * SCAN_PER_THREAD;

// Exclusive scan of one int64 value per thread across the workgroup;
// returns the thread's exclusive prefix and writes the workgroup total.
__device__ int64_t wg_exclusive_scan(int64_t v, int64_t *wave_tot, int64_t *total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int64_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t o = __shfl_up(inc, d, 64);
        if (lane >= d)
            inc += o;
    }
    if (lane == 63)
        wave_tot[wave] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < SCAN_WG / 64; w++) {
        if (w < wave)
            before += wave_tot[w];
        all += wave_tot[w];
    }
    *total = all;
    __syncthreads();
    return before + inc - v;
}

__global__ __launch_bounds__(SCAN_WG) void scan_chunk_totals(const int32_t *cnt, int64_t N,
                                                             int64_t *part)
{
    __shared__ int64_t wave_tot[SCAN_WG / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER_THREAD; j++) {
        int64_t e = base + (int64_t)j * SCAN_WG + threadIdx.x;
        if (e < N)
            s += cnt[e];
    }
    int64_t total;
    wg_exclusive_scan(s, wave_tot, &total);
    if (threadIdx.x == 0)
        part[blockIdx.x] = total;
}

// One workgroup: part[b] <- sum of part[0..b), total -> *tot and out[N].
__global__ __launch_bounds__(SCAN_WG) void scan_chunk_offsets(int64_t *part, int64_t nb,
                                                              int64_t *tot, int32_t *out,
                                                              int64_t N)
{
    __shared__ int64_t wave_tot[SCAN_WG / 64];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_WG) {
        int64_t b = b0 + threadIdx.x;
        int64_t v = b < nb ? part[b] : 0;
        int64_t total;
        int64_t ex = wg_exclusive_scan(v, wave_tot, &total);
        if (b < nb)
            part[b] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        *tot = carry;
        out[N] = (int32_t)carry;
    }
}

__global__ __launch_bounds__(SCAN_WG) void scan_chunk_apply(const int32_t *cnt, int64_t N,
                                                            const int64_t *part, int32_t *out)
{
    __shared__ int64_t wave_tot[SCAN_WG / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int32_t v[SCAN_PER_THREAD];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER_THREAD; j++) {
        int64_t e = base + j;
        v[j] = e < N ? cnt[e] : 0;
        s += v[j];
    }
    int64_t total;
    int64_t run = part[blockIdx.x] + wg_exclusive_scan(s, wave_tot, &total);
#pragma unroll
    for (int j = 0; j < SCAN_PER_THREAD; j++) {
        int64_t e = base + j;
        if (e < N)
            out[e] = (int32_t)run;
        run += v[j];
    }
}

}  // namespace

int exclusive_scan_i32(const int32_t *cnt, int32_t *out, int64_t N, int64_t *total,
                       hipStream_t stream)
{
    int64_t nb = (N + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nb < 1)
        nb = 1;
    int64_t *part = nullptr;
    int rc = dmalloc((void **)&part, sizeof(int64_t) * (size_t)(nb + 1), "scan partials");
    if (rc)
        return rc;
    int64_t *tot = part + nb;
    if (N > 0)
        scan_chunk_totals<<<dim3((unsigned)nb), dim3(SCAN_WG), 0, stream>>>(cnt, N, part);
    else
        (void)hipMemsetAsync(part, 0, sizeof(int64_t), stream);
    scan_chunk_offsets<<<1, SCAN_WG, 0, stream>>>(part, N > 0 ? nb : 1, tot, out, N);
    if (N > 0)
        scan_chunk_apply<<<dim3((unsigned)nb), dim3(SCAN_WG), 0, stream>>>(cnt, N, part, out);
    int64_t h_tot = 0;
    hipError_t e = hipMemcpyAsync(&h_tot, tot, sizeof(int64_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);
    dfree(part);
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string("scan: ") + hipGetErrorString(e));
    e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string("scan launch: ") + hipGetErrorString(e));
    if (h_tot >= (int64_t)INT32_MAX)
        return set_error(MHDC_ERR_SIZE, "prefix sum exceeds the int32 index range");
    *total = h_tot;
    return MHDC_OK;
}

}  // namespace mhdc
