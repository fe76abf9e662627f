// membench.hip -- the memory benchmark kernels of Sec. 6.2 (Figs. 19-20),
// used to measure the achievable HBM bandwidth (the w_mem of Eq. 2) and to
// calibrate the hardware byte counters.
//
//   direct:   C[i] = C[i] + A[i] * B[i]       32 bytes per element
//   indirect: C[i] = C[i] + A[i] * B[I[i]]    36 bytes per element
//
// Each lane handles pairs of consecutive elements with 16-byte non-temporal
// loads and stores (every byte is used once), several pairs per lane in
// flight; an element with an odd index at the end, or arrays that are not
// 16-byte aligned, take a scalar path.  The product is rounded before the
// add, as in the sequential loop.
#include "internal.h"

namespace mhdc {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef int32_t i2 __attribute__((ext_vector_type(2)));
constexpr int MB_WG = 256;
constexpr int MB_PAIRS = 4;  // pairs per lane per step

__global__ __launch_bounds__(MB_WG) void k_direct_pairs(int64_t P, const d2 *__restrict__ A,
                                                        const d2 *__restrict__ B,
                                                        d2 *__restrict__ C)
{
#pragma clang fp contract(off)
    const int64_t stride = (int64_t)gridDim.x * MB_WG * MB_PAIRS;
    for (int64_t base = (int64_t)blockIdx.x * MB_WG * MB_PAIRS + threadIdx.x; base < P;
         base += stride) {
        d2 a[MB_PAIRS], b[MB_PAIRS], c[MB_PAIRS];
#pragma unroll
        for (int j = 0; j < MB_PAIRS; j++) {
            const int64_t p = base + (int64_t)j * MB_WG;
            if (p < P) {
                a[j] = __builtin_nontemporal_load(A + p);
                b[j] = __builtin_nontemporal_load(B + p);
                c[j] = __builtin_nontemporal_load(C + p);
            }
        }
#pragma unroll
        for (int j = 0; j < MB_PAIRS; j++) {
            const int64_t p = base + (int64_t)j * MB_WG;
            if (p < P) {
                d2 r;
                r.x = __dadd_rn(c[j].x, __dmul_rn(a[j].x, b[j].x));
                r.y = __dadd_rn(c[j].y, __dmul_rn(a[j].y, b[j].y));
                __builtin_nontemporal_store(r, C + p);
            }
        }
    }
}

// B holds N elements; an index outside [0, N) leaves its C element unchanged.
__device__ inline double gather_term(double c, double a, const double *__restrict__ B,
                                     int32_t i, int64_t N)
{
#pragma clang fp contract(off)
    return (i >= 0 && i < N) ? __dadd_rn(c, __dmul_rn(a, B[i])) : c;
}

__global__ __launch_bounds__(MB_WG) void k_indirect_pairs(int64_t P, int64_t N,
                                                          const d2 *__restrict__ A,
                                                          const double *__restrict__ B,
                                                          const i2 *__restrict__ I,
                                                          d2 *__restrict__ C)
{
#pragma clang fp contract(off)
    const int64_t stride = (int64_t)gridDim.x * MB_WG * MB_PAIRS;
    for (int64_t base = (int64_t)blockIdx.x * MB_WG * MB_PAIRS + threadIdx.x; base < P;
         base += stride) {
        d2 a[MB_PAIRS], c[MB_PAIRS];
        i2 idx[MB_PAIRS];
#pragma unroll
        for (int j = 0; j < MB_PAIRS; j++) {
            const int64_t p = base + (int64_t)j * MB_WG;
            if (p < P) {
                a[j] = __builtin_nontemporal_load(A + p);
                idx[j] = __builtin_nontemporal_load(I + p);
                c[j] = __builtin_nontemporal_load(C + p);
            }
        }
#pragma unroll
        for (int j = 0; j < MB_PAIRS; j++) {
            const int64_t p = base + (int64_t)j * MB_WG;
            if (p < P) {
                d2 r;
                r.x = gather_term(c[j].x, a[j].x, B, idx[j].x, N);
                r.y = gather_term(c[j].y, a[j].y, B, idx[j].y, N);
                __builtin_nontemporal_store(r, C + p);
            }
        }
    }
}

// scalar path for elements [i0, N)
__global__ __launch_bounds__(MB_WG) void k_direct_scalar(int64_t i0, int64_t N,
                                                         const double *__restrict__ A,
                                                         const double *__restrict__ B,
                                                         double *__restrict__ C)
{
#pragma clang fp contract(off)
    for (int64_t i = i0 + (int64_t)blockIdx.x * MB_WG + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * MB_WG)
        C[i] = __dadd_rn(C[i], __dmul_rn(A[i], B[i]));
}

__global__ __launch_bounds__(MB_WG) void k_indirect_scalar(int64_t i0, int64_t N,
                                                           const double *__restrict__ A,
                                                           const double *__restrict__ B,
                                                           const int32_t *__restrict__ I,
                                                           double *__restrict__ C)
{
#pragma clang fp contract(off)
    for (int64_t i = i0 + (int64_t)blockIdx.x * MB_WG + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * MB_WG)
        C[i] = gather_term(C[i], A[i], B, I[i], N);
}

unsigned grid_of(int64_t items, int per_wg)
{
    int64_t g = (items + per_wg - 1) / per_wg;
    if (g > 256 * 32)
        g = 256 * 32;
    return (unsigned)(g < 1 ? 1 : g);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace
}  // namespace mhdc

using namespace mhdc;

extern "C" int mhdc_stream_direct(int64_t N, const double *A, const double *B, double *C,
                                  hipStream_t stream)
{
    clear_error();
    if (N < 0 || (N > 0 && (!A || !B || !C)))
        return set_error(MHDC_ERR_INVALID_ARG, "bad stream_direct arguments");
    if (N == 0)
        return MHDC_OK;
    int64_t done = 0;
    if (aligned16(A) && aligned16(B) && aligned16(C) && N >= 2) {
        const int64_t P = N / 2;
        k_direct_pairs<<<grid_of(P, MB_WG * MB_PAIRS), MB_WG, 0, stream>>>(
            P, (const d2 *)A, (const d2 *)B, (d2 *)C);
        done = 2 * P;
    }
    if (done < N)
        k_direct_scalar<<<grid_of(N - done, MB_WG), MB_WG, 0, stream>>>(done, N, A, B, C);
    MHDC_HIP_CHECK(hipGetLastError());
    return MHDC_OK;
}

extern "C" int mhdc_stream_indirect(int64_t N, const double *A, const double *B,
                                    const int32_t *I, double *C, hipStream_t stream)
{
    clear_error();
    if (N < 0 || (N > 0 && (!A || !B || !I || !C)))
        return set_error(MHDC_ERR_INVALID_ARG, "bad stream_indirect arguments");
    if (N == 0)
        return MHDC_OK;
    int64_t done = 0;
    if (aligned16(A) && aligned16(C) && ((uintptr_t)I & 7) == 0 && N >= 2) {
        const int64_t P = N / 2;
        k_indirect_pairs<<<grid_of(P, MB_WG * MB_PAIRS), MB_WG, 0, stream>>>(
            P, N, (const d2 *)A, B, (const i2 *)I, (d2 *)C);
        done = 2 * P;
    }
    if (done < N)
        k_indirect_scalar<<<grid_of(N - done, MB_WG), MB_WG, 0, stream>>>(done, N, A, B, I, C);
    MHDC_HIP_CHECK(hipGetLastError());
    return MHDC_OK;
}
