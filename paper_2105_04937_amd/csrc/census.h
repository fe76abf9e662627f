// census.h -- per-block count of nonzeros per diagonal offset (the
// N~(d, ib) of Sec. 4.3), shared by the converter and the selector's
// feature kernel.
//
// One workgroup counts one block of rows in an open-addressing hash table
// keyed by d = j - i: in LDS when the block holds fewer than
// CENSUS_LDS_SLOTS stored entries, else in the block's own region
// [2*e0, 2*e1) of a global table (e0, e1 = the block's entry range).  The
// table always has more slots than the block has entries, so probing ends.
// Only integer atomics are used; the resulting (key, count) set does not
// depend on their order.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace mhdc {

constexpr int CENSUS_WG = 256;
constexpr int CENSUS_LDS_SLOTS = 8192;    // 64 KB of keys + counts
constexpr int32_t EMPTY_KEY = INT32_MIN;  // offsets lie in [-(n-1), n-1]

__device__ inline uint32_t census_hash(int32_t d, uint32_t cap)
{
    return ((uint32_t)d * 2654435761u) % cap;
}

__device__ inline void census_add(int32_t *keys, int32_t *cnts, uint32_t cap, int32_t d)
{
    uint32_t h = census_hash(d, cap);
    for (;;) {
        const int32_t prev = atomicCAS(&keys[h], EMPTY_KEY, d);
        if (prev == EMPTY_KEY || prev == d) {
            atomicAdd(&cnts[h], 1);
            return;
        }
        h = (h + 1 == cap) ? 0 : h + 1;
    }
}

// Count block [r0, r1) (entries [e0, e1)) into a table chosen as described
// above; returns its capacity and sets keys/cnts.  Ends with a barrier.
__device__ inline uint32_t census_block(int64_t r0, int64_t r1, int64_t e0, int64_t e1,
                                        const int32_t *__restrict__ rowptr,
                                        const int32_t *__restrict__ colind,
                                        const double *__restrict__ val, int32_t *s_keys,
                                        int32_t *s_cnts, int32_t *gkeys, int32_t *gcnts,
                                        int32_t **keys_out, int32_t **cnts_out)
{
    const int64_t m = e1 - e0;
    int32_t *keys, *cnts;
    uint32_t cap;
    if (m < CENSUS_LDS_SLOTS) {
        keys = s_keys;
        cnts = s_cnts;
        uint32_t c = 64;
        while (c < 2 * (uint32_t)m && c < CENSUS_LDS_SLOTS)
            c <<= 1;
        cap = c > (uint32_t)m ? c : (uint32_t)CENSUS_LDS_SLOTS;
    } else {
        keys = gkeys + 2 * e0;
        cnts = gcnts + 2 * e0;
        cap = (uint32_t)(2 * m);
    }
    for (uint32_t s = threadIdx.x; s < cap; s += CENSUS_WG) {
        keys[s] = EMPTY_KEY;
        cnts[s] = 0;
    }
    __syncthreads();
    for (int64_t i = r0 + threadIdx.x; i < r1; i += CENSUS_WG) {
        const int32_t a = rowptr[i], b = rowptr[i + 1];
        for (int32_t k = a; k < b; k++)
            if (val[k] != 0.0)
                census_add(keys, cnts, cap, colind[k] - (int32_t)i);
    }
    __syncthreads();
    *keys_out = keys;
    *cnts_out = cnts;
    return cap;
}

}  // namespace mhdc
