// census.h -- per-block count of nonzeros per diagonal offset (the
// N~(d, ib) of Sec. 4.3), shared by the converter and the selector's
// feature kernel.
//
// One workgroup counts one block of rows in an open-addressing hash table
// keyed by d = j - i: in LDS when the block's distinct offsets fit the
// kernel's LDS table (at most CENSUS_LDS_SLOTS slots), else in the block's
// own region [2*e0, 2*e1) of a global table (e0, e1 = the block's entry
// range), which has more slots than the block has entries.  Probing is
// bounded by the table size.
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

// Count d; false if all cap slots hold other keys, or if d is a new key
// beyond the first `limit` ones (counted in *nkeys; nkeys == null: no limit).
__device__ inline bool census_add(int32_t *keys, int32_t *cnts, uint32_t cap, int32_t d,
                                  int32_t *nkeys, int32_t limit)
{
    uint32_t h = census_hash(d, cap);
    for (uint32_t probe = 0; probe < cap; probe++) {
        const int32_t prev = atomicCAS(&keys[h], EMPTY_KEY, d);
        if (prev == EMPTY_KEY && nkeys && atomicAdd(nkeys, 1) >= limit)
            return false;
        if (prev == EMPTY_KEY || prev == d) {
            atomicAdd(&cnts[h], 1);
            return true;
        }
        h = (h + 1 == cap) ? 0 : h + 1;
    }
    return false;
}

// Clear a table and count rows [r0, r1) into it; true if every entry found
// a slot and (with `limited`) the block has at most cap / 2 distinct
// offsets -- a trial table is given up at half load rather than probed
// ever longer.  Ends with a barrier.
__device__ inline bool census_fill(int64_t r0, int64_t r1, const int32_t *__restrict__ rowptr,
                                   const int32_t *__restrict__ colind,
                                   const double *__restrict__ val, int32_t *keys, int32_t *cnts,
                                   uint32_t cap, bool limited, int32_t *s_full, int32_t *s_nkeys)
{
    if (threadIdx.x == 0) {
        *s_full = 0;
        *s_nkeys = 0;
    }
    for (uint32_t s = threadIdx.x; s < cap; s += CENSUS_WG) {
        keys[s] = EMPTY_KEY;
        cnts[s] = 0;
    }
    __syncthreads();
    int32_t *nk = limited ? s_nkeys : nullptr;
    const int32_t limit = (int32_t)(cap / 2);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += CENSUS_WG) {
        if (*(volatile int32_t *)s_full)
            break;  // the table is given up: the rest of the work is wasted
        const int32_t a = rowptr[i], b = rowptr[i + 1];
        for (int32_t k = a; k < b; k++)
            if (val[k] != 0.0 && !census_add(keys, cnts, cap, colind[k] - (int32_t)i, nk, limit))
                *(volatile int32_t *)s_full = 1;
    }
    __syncthreads();
    const bool ok = *s_full == 0;
    // every lane has read the flag before a further fill resets it
    __syncthreads();
    return ok;
}

// Count block [r0, r1) (entries [e0, e1)) into a table chosen as described
// above; returns its capacity and sets keys/cnts.  A block with more
// entries than the largest LDS table first tries that table anyway (its
// distinct offsets are usually few: 7 for a 7-point grid) and moves to its
// global region once more than half the table's slots would be taken.
// Ends with a barrier.
// lds_slots: slots of the LDS table s_keys / s_cnts (a power of two, at
// least 64).
__device__ inline uint32_t census_block(int64_t r0, int64_t r1, int64_t e0, int64_t e1,
                                        const int32_t *__restrict__ rowptr,
                                        const int32_t *__restrict__ colind,
                                        const double *__restrict__ val, int32_t *s_keys,
                                        int32_t *s_cnts, uint32_t lds_slots, int32_t *gkeys,
                                        int32_t *gcnts, int32_t **keys_out, int32_t **cnts_out)
{
    __shared__ int32_t s_full, s_nkeys;
    const int64_t m = e1 - e0;
    if (m < (int64_t)lds_slots || lds_slots == (uint32_t)CENSUS_LDS_SLOTS) {
        uint32_t cap = lds_slots;
        const bool trial = m >= (int64_t)lds_slots;
        if (!trial) {
            uint32_t c = 64;
            while (c < 2 * (uint32_t)m && c < lds_slots)
                c <<= 1;
            cap = c > (uint32_t)m ? c : lds_slots;
        }
        if (census_fill(r0, r1, rowptr, colind, val, s_keys, s_cnts, cap, trial, &s_full,
                        &s_nkeys)) {
            *keys_out = s_keys;
            *cnts_out = s_cnts;
            return cap;
        }
        // only a trial (a block with at least lds_slots entries) gives up
    }
    int32_t *keys = gkeys + 2 * e0, *cnts = gcnts + 2 * e0;
    const uint32_t cap = (uint32_t)(2 * m);
    census_fill(r0, r1, rowptr, colind, val, keys, cnts, cap, false, &s_full, &s_nkeys);
    *keys_out = keys;
    *cnts_out = cnts;
    return cap;
}

}  // namespace mhdc
