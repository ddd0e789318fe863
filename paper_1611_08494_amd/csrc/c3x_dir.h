// c3x_dir.h -- the cell directory of an index: dir[q] = the first sorted
// position whose key lies in bucket q (key >> dshift) or a later one, for
// every bucket q < dsize (dir[dsize - 1] = n). Shared by the index build and
// the batched form; each translation unit gets its own (static) copy of the
// kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace c3x {

// The directory from the sorted keys: position s (0 <= s <= n; s = n stands
// for the end) is the first key of every bucket q with bucket(keys[s-1]) < q
// <= bucket(keys[s]) (the end: every bucket up to dsize - 1), so it writes
// dir[q] = s for those q. Longer gaps are listed (first, last, s) for
// k_dir_fill_gaps: up to kDirBig buckets one workgroup each, longer ones
// (empty stretches of sky) by the whole grid, so that no lane and no
// workgroup walks a long gap alone. gaps[0, gap_cap) holds the former,
// gaps[gap_cap, gap_cap + big_cap) the latter; n_gaps[0], n_gaps[1] count
// them.
static constexpr uint32_t kDirGap = 64;
static constexpr uint32_t kDirBig = 65536;

// List capacities for dsize buckets: every listed gap spans more than
// kDirGap (kDirBig) buckets, and the gaps are disjoint.
static inline uint32_t dir_gap_cap(uint32_t dsize) { return dsize / kDirGap + 2; }
static inline uint32_t dir_big_cap(uint32_t dsize) { return dsize / kDirBig + 2; }

static __global__ void k_dir_fill(const uint32_t *__restrict__ keys, int64_t n, int dshift,
                                  uint32_t dsize, uint32_t *__restrict__ dir,
                                  uint3 *__restrict__ gaps, uint32_t *__restrict__ n_gaps,
                                  uint32_t gap_cap, uint32_t big_cap)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n) return;
    // buckets clamped to the directory: keys out of order or out of range
    // (a sort that gave up, whose index is discarded) still write in bounds
    const int64_t top = (int64_t)dsize - 1;
    const int64_t hi = t < n ? std::min<int64_t>(keys[t] >> dshift, top) : top;
    const int64_t lo = t > 0 ? std::min<int64_t>(keys[t - 1] >> dshift, top) : -1;
    if (hi - lo <= (int64_t)kDirGap) {
        for (int64_t q = lo + 1; q <= hi; ++q) dir[q] = (uint32_t)t;
    } else if (hi - lo <= (int64_t)kDirBig) {
        const uint32_t slot = atomicAdd(n_gaps, 1u);
        if (slot < gap_cap) gaps[slot] = make_uint3((uint32_t)(lo + 1), (uint32_t)hi, (uint32_t)t);
    } else {
        const uint32_t slot = atomicAdd(n_gaps + 1, 1u);
        if (slot < big_cap)
            gaps[gap_cap + slot] = make_uint3((uint32_t)(lo + 1), (uint32_t)hi, (uint32_t)t);
    }
}

static __global__ void k_dir_fill_gaps(const uint3 *__restrict__ gaps,
                                       const uint32_t *__restrict__ n_gaps, uint32_t gap_cap,
                                       uint32_t big_cap, uint32_t *__restrict__ dir)
{
    const uint32_t ng = min(n_gaps[0], gap_cap);
    for (uint32_t g = blockIdx.x; g < ng; g += gridDim.x) {
        const uint3 v = gaps[g];
        for (uint32_t q = v.x + threadIdx.x; q <= v.y && q >= v.x; q += blockDim.x) dir[q] = v.z;
    }
    const uint32_t nbig = min(n_gaps[1], big_cap);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint32_t g = 0; g < nbig; ++g) {
        const uint3 v = gaps[gap_cap + g];
        for (uint64_t q = (uint64_t)v.x + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
             q <= v.y; q += stride)
            dir[q] = v.z;
    }
}

}  // namespace c3x
