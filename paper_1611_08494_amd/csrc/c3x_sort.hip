// c3x_sort.hip -- LSD radix sort of (u32 key, u32 value) pairs and prefix
// scans, written for 64-wide CDNA wavefronts.
//
// Sort: 8-bit digits, only as many passes as the key range needs. One
// kernel first counts every pass's digits over the whole input (the keys are
// read once for all passes). Each pass is then one launch over 8192-element
// tiles taken in order from a counter: a tile ranks its elements (each
// wavefront ranks its quarter with ballots -- eight ballots match the lanes
// that share a digit, mbcnt ranks them -- against its own digit counters),
// publishes its digit counts, and finds how many elements of each digit the
// earlier tiles hold by looking back over their published counts (a chained
// scan with decoupled look-back); the tile is staged in LDS in digit order
// so that the global writes of a digit run are contiguous. Inputs below
// 8M elements (and of 2^30 or more) instead count each pass's digits per
// tile into a table, scan it, and scatter: there the table is small enough
// to scan with one workgroup per digit, and the three launches a pass cost
// less than the look-back.
//
// A look-back waits only on tiles that took their numbers earlier (so are
// running or done), but every wait is bounded: a tile that polls an
// unpublished predecessor more than the spin limit gives up, and its pass
// then writes a wrong order (every access still in bounds). The give-up is
// recorded in a device word the caller passes and checks at its next
// synchronisation; the caller then redoes its work with the table schedule,
// which never waits. A sort given no such word always takes the table
// schedule.
#include <stdlib.h>

#include <algorithm>

#include "c3x_internal.h"
#include "c3x_sort.h"

namespace c3x {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;  // 4096
constexpr int kWaves = kSortBlock / 64;
constexpr int64_t kRowScanTiles = 8192;  // 32M elements
// Sorts of this many 4096-element tiles (8M elements) and more take the
// one-sweep schedule where the caller can observe a give-up: at 10M
// elements it measured 7 us a pass faster than the table, at 200M 0.7 ms.
constexpr int64_t kOneSweepMinTiles = 2048;

__device__ __forceinline__ uint64_t lanemask_lt()
{
    unsigned lane = __lane_id();
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__device__ __forceinline__ unsigned rank_in_mask(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__global__ __launch_bounds__(kSortBlock) void k_digit_hist(const uint32_t *__restrict__ keys,
                                                           int64_t n, int shift,
                                                           uint32_t *__restrict__ hist,
                                                           int nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    uint32_t kk[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        int64_t e = base + r * kSortBlock + threadIdx.x;
        kk[r] = e < n ? keys[e] : 0xffffffffu;
    }
    // a wavefront whose valid lanes share the digit adds them with one atomic
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t e = base + r * kSortBlock + threadIdx.x;
        const bool valid = e < n;
        const uint64_t vm = __ballot(valid);
        if (vm == 0) continue;
        const int lead = __builtin_ffsll((long long)vm) - 1;
        const uint32_t d = (kk[r] >> shift) & 255u;
        const uint32_t d0 = (uint32_t)__shfl((int)d, lead);
        if (__ballot(valid && d != d0) == 0) {
            if ((int)__lane_id() == lead) atomicAdd(&h[d0], (uint32_t)__popcll(vm));
        } else if (valid) {
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ __forceinline__ uint32_t block256_excl_scan(uint32_t x, uint32_t *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    __syncthreads();
    return pre + inc - x;
}

// Stable scatter of one 4096-element tile. The tile's own digit histogram
// (from k_digit_hist) gives where each digit's run starts inside the tile.
// Each wavefront ranks its own contiguous quarter of the tile, 64 elements
// a round, with no barrier between rounds: eight ballots match the lanes
// that share a digit, mbcnt ranks them, and a per-wavefront digit counter in
// LDS (read by the group, advanced by its last lane) gives the group's place
// among the wavefront's earlier elements of that digit. One prefix over the
// four wavefronts' counters then places every element in LDS in (digit,
// original order); the tile leaves LDS in order, so consecutive threads
// write consecutive addresses of one digit run. Keys and then values pass
// through one LDS buffer (22 KB a workgroup).
__global__ __launch_bounds__(kSortBlock) void k_digit_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const uint32_t *__restrict__ offs, const uint32_t *__restrict__ tot,
    const uint32_t *__restrict__ hist, int nblocks)
{
    constexpr int kPerWave = kSortTile / kWaves;  // 1024
    constexpr int kRounds = kPerWave / 64;        // 16
    __shared__ uint32_t sbuf[kSortTile];  // the tile in digit order: keys, then values
    __shared__ uint32_t gbase[256], tstart[256];
    __shared__ uint32_t wc[kWaves][256];
    __shared__ uint32_t wsum[kWaves];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int64_t tbase = (int64_t)blockIdx.x * kSortTile;
    const int64_t wbase = tbase + (int64_t)wave * kPerWave + __lane_id();
    uint32_t hc = hist[(int64_t)tid * nblocks + blockIdx.x];
    uint32_t gb = offs[(int64_t)tid * nblocks + blockIdx.x];
    // offsets within each digit's row of tiles (tot: the rows' totals, whose
    // prefix places the digits), or global offsets (tot null)
    if (tot) gb += block256_excl_scan(tot[tid], wsum);
    gbase[tid] = gb;
    uint32_t ts = block256_excl_scan(hc, wsum);
    tstart[tid] = ts;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wc[w][tid] = 0;
    // all of this thread's elements are loaded up front (memory-level
    // parallelism); the ranking rounds then work from registers
    uint32_t kk[kRounds], vv[kRounds], loc[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t e = wbase + r * 64;
        kk[r] = e < n ? kin[e] : 0u;
        vv[r] = e < n ? (vin ? vin[e] : (uint32_t)e) : 0u;  // no vin: the index
    }
    __syncthreads();
    uint32_t *cnt = wc[wave];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const bool valid = wbase + r * 64 < n;
        const uint32_t d = (kk[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const unsigned rank = rank_in_mask(peers & lanemask_lt());
        const unsigned grp = (unsigned)__popcll(peers);
        // the group's read of its counter comes before its last lane's update
        // (one wavefront's LDS operations complete in order)
        const uint32_t c = valid ? cnt[d] : 0u;
        loc[r] = c + rank;
        if (valid && rank + 1 == grp) cnt[d] = c + grp;
    }
    __syncthreads();
    {  // thread tid = digit: where each wavefront's elements of it start
        uint32_t acc = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t t = wc[w][tid];
            wc[w][tid] = acc;
            acc += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        if (wbase + r * 64 < n) {
            const uint32_t d = (kk[r] >> shift) & 255u;
            loc[r] += tstart[d] + cnt[d];
            sbuf[loc[r]] = kk[r];
        }
    }
    __syncthreads();
    // keys out; each lane keeps the digits of its places (four to a
    // register) for the values
    const int nt = (int)min<int64_t>(kSortTile, n - tbase);
    uint32_t dg[kRounds / 4];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int q = tid + r * kSortBlock;
        uint32_t d = 0;
        if (q < nt) {
            const uint32_t k = sbuf[q];
            d = (k >> shift) & 255u;
            const uint32_t dst = gbase[d] + (uint32_t)(q - tstart[d]);
            if (dst < (uint64_t)n) kout[dst] = k;
        }
        if (r % 4 == 0) dg[r / 4] = d; else dg[r / 4] |= d << (8 * (r % 4));
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
        if (wbase + r * 64 < n) sbuf[loc[r]] = vv[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int q = tid + r * kSortBlock;
        const uint32_t d = (dg[r / 4] >> (8 * (r % 4))) & 255u;
        const uint32_t dst = gbase[d] + (uint32_t)(q - tstart[d]);
        if (q < nt && dst < (uint64_t)n) vout[dst] = sbuf[q];
    }
}

// Every pass's digit counts over the whole input, accumulated per wavefront
// in LDS and added to ghist[pass][digit] once per block. Where the valid
// lanes of a wavefront share a digit (grouped input, such as a batch's
// job-major keys) one lane adds them all: 64 atomics on one LDS address
// would serialise.
__global__ __launch_bounds__(kSortBlock) void k_digit_hist_all(const uint32_t *__restrict__ keys,
                                                               int64_t n, int lo_bit, int npass,
                                                               uint32_t *__restrict__ ghist)
{
    __shared__ uint32_t h[kWaves][4][256];
    const int tid = threadIdx.x, wave = tid >> 6;
    for (int w = 0; w < kWaves; ++w)
#pragma unroll
        for (int p = 0; p < 4; ++p) h[w][p][tid] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kSortBlock * 4;
    for (int64_t b = (int64_t)blockIdx.x * kSortBlock * 4 + tid; b < n; b += stride) {
        uint32_t kk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = b + u * kSortBlock;
            kk[u] = e < n ? keys[e] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool valid = b + u * kSortBlock < n;
            const uint64_t vm = __ballot(valid);
            if (vm == 0) break;  // wavefront-uniform
            const int lead = __builtin_ffsll((long long)vm) - 1;
            for (int p = 0; p < npass; ++p) {
                const uint32_t d = (kk[u] >> (lo_bit + 8 * p)) & 255u;
                const uint32_t d0 = (uint32_t)__shfl((int)d, lead);
                if (__ballot(valid && d != d0) == 0) {
                    if ((int)__lane_id() == lead) atomicAdd(&h[wave][p][d0], (uint32_t)__popcll(vm));
                } else if (valid) {
                    atomicAdd(&h[wave][p][d], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int p = 0; p < npass; ++p) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) c += h[w][p][tid];
        if (c) atomicAdd(&ghist[p * 256 + tid], c);
    }
}

// Look-back status word of one (tile, digit): the flag in the top two bits
// (0 not yet published, 1 the tile's own count, 2 the count of this and
// every earlier tile), the count in the low 30.
constexpr uint32_t kStAgg = 1u << 30, kStInc = 2u << 30, kStVal = (1u << 30) - 1u;
constexpr uint32_t kSpinLimit = 1u << 20;  // polls before a look-back gives up

__device__ __forceinline__ void st_publish(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t st_read(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One pass over the tiles: stable scatter of the tile counter's next tile
// by the digit at `shift`. ghist: this pass's digit totals; tctr: this
// pass's tile counter; status: nb x 256 look-back words (all zero at entry).
// A tile waits only on tiles that took their numbers before it (and so are
// running or done); a wait that exceeds spin_limit polls gives up, leaving
// a wrong order but no access out of bounds, and sets *fail. spin_limit 0
// (a test setting) makes every tile but the first give up at once. A tile is
// kSortBlock * ITEMS elements (longer tiles: longer runs per digit in the
// scatter, fewer look-backs). The tile passes through LDS twice, keys then
// values, in one buffer: at 32 items 38 KB a workgroup, so the registers
// (three wavefronts a SIMD) bound the workgroups a CU holds, not the LDS.
template <int ITEMS>
__global__ __launch_bounds__(kSortBlock) void k_onesweep(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const uint32_t *__restrict__ ghist, uint32_t *__restrict__ tctr, uint32_t *status, int nb,
    uint32_t spin_limit, uint32_t *__restrict__ fail)
{
    constexpr int kTile = kSortBlock * ITEMS;
    constexpr int kPerWave = kTile / kWaves;  // 64 * ITEMS
    constexpr int kRounds = kPerWave / 64;    // ITEMS
    // one buffer stages the tile in digit order: its keys, then its values
    // (38 KB of LDS a workgroup, four workgroups a CU)
    __shared__ uint32_t sbuf[kTile];
    __shared__ uint32_t gbase[256], tstart[256];
    __shared__ uint32_t wc[kWaves][256];
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(tctr, 1u);
    // where each digit starts in the output
    const uint32_t dbase = block256_excl_scan(ghist[tid], wsum);
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wc[w][tid] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= (uint32_t)nb) return;  // the counter was not cleared: nothing is touched
    const int64_t tbase = (int64_t)tile * kTile;
    const int64_t wbase = tbase + (int64_t)wave * kPerWave + __lane_id();
    uint32_t kk[kRounds], loc[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int64_t e = wbase + r * 64;
        kk[r] = e < n ? kin[e] : 0u;
    }
    uint32_t *cnt = wc[wave];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const bool valid = wbase + r * 64 < n;
        const uint32_t d = (kk[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const unsigned rank = rank_in_mask(peers & lanemask_lt());
        const unsigned grp = (unsigned)__popcll(peers);
        // the group's read of its counter comes before its last lane's update
        // (one wavefront's LDS operations complete in order)
        const uint32_t c = valid ? cnt[d] : 0u;
        loc[r] = c + rank;
        if (valid && rank + 1 == grp) cnt[d] = c + grp;
    }
    __syncthreads();
    // thread tid = digit: where each wavefront's elements of it start, and
    // the tile's count of it
    uint32_t acc = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t t = wc[w][tid];
        wc[w][tid] = acc;
        acc += t;
    }
    // publish the tile's digit counts, stage its keys in digit order, then
    // look back (the staging overlaps the predecessors' publishing)
    uint32_t *mine = status + (size_t)tile * 256 + tid;
    st_publish(mine, (tile == 0 ? kStInc : kStAgg) | acc);
    tstart[tid] = block256_excl_scan(acc, wsum);
    __syncthreads();
    // loc becomes each element's place in the tile's digit order
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        if (wbase + r * 64 < n) {
            const uint32_t d = (kk[r] >> shift) & 255u;
            loc[r] += tstart[d] + cnt[d];
            sbuf[loc[r]] = kk[r];
        }
    }
    // the values (no vin: the element's index), loaded while the tile looks
    // back; only they and the places stay live
    uint32_t vv[kRounds];
    if (vin) {
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const int64_t e = wbase + r * 64;
            vv[r] = e < n ? vin[e] : 0u;
        }
    } else {
#pragma unroll
        for (int r = 0; r < kRounds; ++r) vv[r] = (uint32_t)(wbase + r * 64);
    }
    uint32_t excl = 0;
    if (tile != 0) {
        int64_t p = spin_limit ? (int64_t)tile - 1 : -1;
        uint32_t spins = 0;
        bool gave_up = spin_limit == 0;
        while (p >= 0) {
            const uint32_t v = st_read(status + (size_t)p * 256 + tid);
            const uint32_t fl = v & ~kStVal;
            if (fl == 0u) {
                if (++spins > spin_limit) {
                    gave_up = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += v & kStVal;
            if (fl == kStInc) break;
            --p;
        }
        if (gave_up) atomicOr(fail, 1u);
        st_publish(mine, kStInc | ((excl + acc) & kStVal));
    }
    gbase[tid] = dbase + excl;
    __syncthreads();
    // keys out; each lane keeps the digits of its ITEMS places (four to a
    // register) for the values
    const int nt = (int)min<int64_t>(kTile, n - tbase);
    uint32_t dg[kRounds / 4];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int q = tid + r * kSortBlock;
        uint32_t d = 0;
        if (q < nt) {
            const uint32_t k = sbuf[q];
            d = (k >> shift) & 255u;
            const uint32_t dst = gbase[d] + (uint32_t)(q - tstart[d]);
            if (dst < (uint64_t)n) kout[dst] = k;
        }
        if (r % 4 == 0) dg[r / 4] = d; else dg[r / 4] |= d << (8 * (r % 4));
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
        if (wbase + r * 64 < n) sbuf[loc[r]] = vv[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int q = tid + r * kSortBlock;
        const uint32_t d = (dg[r / 4] >> (8 * (r % 4))) & 255u;
        const uint32_t dst = gbase[d] + (uint32_t)(q - tstart[d]);
        if (q < nt && dst < (uint64_t)n) vout[dst] = sbuf[q];
    }
}

__global__ void k_sort_iota(uint32_t *__restrict__ p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = (uint32_t)t;
}

__global__ void k_sort_clear(uint32_t *__restrict__ p, int64_t n, uint32_t v)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// ---------------------------------------------------------------------------- scans

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T &total)
{
    __shared__ T ws[kScanBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    T inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    T pre = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / 64; ++w) {
        if (w < wave) pre += ws[w];
        total += ws[w];
    }
    __syncthreads();
    return pre + inc - x;
}

// Strided input (compact != null): the tile's values are also kept, packed,
// at the start of the tile's own output range (compact = the output as Ti,
// To twice as wide), so that the final pass reads them there instead of
// the strided records again.
template <typename Ti, typename To>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const Ti *__restrict__ in,
                                                            int64_t stride, Ti mask, int64_t n,
                                                            To *__restrict__ part,
                                                            Ti *__restrict__ compact)
{
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    To s = 0;
    for (int r = 0; r < kScanItems; ++r) {
        int64_t e = base + r * kScanBlock + threadIdx.x;
        if (e < n) {
            const Ti v = in[e * stride] & mask;
            s += (To)v;
            if (compact) compact[2 * base + r * kScanBlock + threadIdx.x] = v;
        }
    }
    To tot;
    block_excl_scan<To>(s, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One workgroup over the tiles' totals, kScanTile of them a round (each lane
// a run of kScanItems consecutive ones).
template <typename To>
__global__ __launch_bounds__(kScanBlock) void k_scan_partials(To *part, int64_t np, To *total)
{
    To carry = 0;
    for (int64_t b = 0; b < np; b += kScanTile) {
        const int64_t e0 = b + (int64_t)threadIdx.x * kScanItems;
        To v[kScanItems];
        To sum = 0;
#pragma unroll
        for (int r = 0; r < kScanItems; ++r) {
            v[r] = e0 + r < np ? part[e0 + r] : (To)0;
            sum += v[r];
        }
        To tot;
        To run = carry + block_excl_scan<To>(sum, tot);
#pragma unroll
        for (int r = 0; r < kScanItems; ++r) {
            if (e0 + r < np) part[e0 + r] = run;
            run += v[r];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename Ti, typename To>
__global__ __launch_bounds__(kScanBlock) void k_scan_final(const Ti *__restrict__ in,
                                                           int64_t stride, Ti mask, int64_t n,
                                                           const To *__restrict__ part,
                                                           To *out, const Ti *compact)
{
    __shared__ To tile[kScanTile];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int r = 0; r < kScanItems; ++r) {
        int i = r * kScanBlock + threadIdx.x;
        int64_t e = base + i;
        tile[i] = e < n ? (To)(compact ? compact[2 * base + i] : (in[e * stride] & mask)) : (To)0;
    }
    __syncthreads();  // the tile's packed values are read before its outputs overwrite them
    To v[kScanItems];
    To s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        v[r] = tile[threadIdx.x * kScanItems + r];
        s += v[r];
    }
    To tot;
    To run = block_excl_scan<To>(s, tot) + part[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        tile[threadIdx.x * kScanItems + r] = run;
        run += v[r];
    }
    __syncthreads();
    for (int r = 0; r < kScanItems; ++r) {
        int i = r * kScanBlock + threadIdx.x;
        int64_t e = base + i;
        if (e < n) out[e] = tile[i];
    }
}

// Per digit (one workgroup each): the exclusive prefix of its row of tile
// counts, and the row's total. With the digits' totals the scatter places
// each tile's runs; three launches a pass instead of a full-table scan.
__global__ __launch_bounds__(kScanBlock) void k_digit_rows(const uint32_t *__restrict__ hist,
                                                           int nb, uint32_t *__restrict__ offs,
                                                           uint32_t *__restrict__ tot)
{
    const uint32_t *row = hist + (int64_t)blockIdx.x * nb;
    uint32_t *orow = offs + (int64_t)blockIdx.x * nb;
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kScanBlock) {
        const int t = base + (int)threadIdx.x;
        const uint32_t x = t < nb ? row[t] : 0u;
        uint32_t chunk;
        const uint32_t ex = block_excl_scan<uint32_t>(x, chunk);
        if (t < nb) orow[t] = carry + ex;
        carry += chunk;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

size_t scan_ws_bytes(int64_t n)
{
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * sizeof(int64_t);
}

template <typename Ti, typename To>
static hipError_t scan_impl(const Ti *in, int64_t stride, Ti mask, To *out, int64_t n, To *total,
                            void *ws, hipStream_t s)
{
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    To *part = (To *)ws;
    if (n == 0) {
        if (total) return hipMemsetAsync(total, 0, sizeof(To), s);
        return hipSuccess;
    }
    // strided input: its values packed into the output's own tiles (To is
    // twice Ti's width) by the first pass
    Ti *compact = (stride != 1 && sizeof(To) == 2 * sizeof(Ti)) ? (Ti *)out : nullptr;
    hipLaunchKernelGGL((k_scan_reduce<Ti, To>), dim3((unsigned)nb), dim3(kScanBlock), 0, s, in,
                       stride, mask, n, part, compact);
    hipLaunchKernelGGL((k_scan_partials<To>), dim3(1), dim3(kScanBlock), 0, s, part, nb, total);
    hipLaunchKernelGGL((k_scan_final<Ti, To>), dim3((unsigned)nb), dim3(kScanBlock), 0, s, in,
                       stride, mask, n, part, out, (const Ti *)compact);
    return hipGetLastError();
}

hipError_t scan_u32_to_i64(const uint32_t *in, int64_t stride, uint32_t mask, int64_t *out,
                           int64_t n, int64_t *total, void *ws, hipStream_t s)
{
    return scan_impl<uint32_t, int64_t>(in, stride, mask, out, n, total, ws, s);
}

hipError_t scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *ws,
                    hipStream_t s)
{
    return scan_impl<uint32_t, uint32_t>(in, 1, ~0u, out, n, total, ws, s);
}

// One-sweep workspace: ghist[4][256], tile counters[64], status[4][nb][256].
constexpr int64_t kOneSweepMax = (int64_t)1 << 30;  // counts fit the status words
static size_t onesweep_words(int64_t nb, int npass)
{
    return (size_t)4 * 256 + 64 + (size_t)npass * 256 * (size_t)nb;
}

size_t radix_ws_bytes(int64_t n)
{
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb < 1) nb = 1;
    size_t hist = (size_t)256 * (size_t)nb * sizeof(uint32_t);
    const size_t table = 2 * hist + 256 * sizeof(uint32_t) + scan_ws_bytes(256 * nb) + 256;
    return std::max(table, onesweep_words(nb, 4) * sizeof(uint32_t));
}

hipError_t radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *ktmp, uint32_t *vtmp,
                            int64_t n, int nbits, void *ws, hipStream_t s, int *in_tmp,
                            bool vals_are_index, uint32_t *fail)
{
    return radix_sort_pairs_bits(keys, vals, ktmp, vtmp, n, 0, nbits, ws, s, in_tmp,
                                 vals_are_index, fail);
}

// Test settings: C3X_DEBUG_ONESWEEP_TILES=t takes the one-sweep schedule
// from t tiles up (default kOneSweepMinTiles); C3X_DEBUG_SORT_SPIN=k sets the
// look-back's spin limit (0: every tile but the first gives up).
static int64_t onesweep_min_tiles()
{
    if (const char *e = getenv("C3X_DEBUG_ONESWEEP_TILES")) return std::max(1LL, atoll(e));
    return kOneSweepMinTiles;
}

// Elements per thread of a one-sweep tile: 32 (8192-element tiles; over
// 200M elements 0.16 ms less per pass than 4096, whose digit runs are half
// as long though six wavefronts a SIMD fit, and level with 6144 at four);
// C3X_ONESWEEP_ITEMS=16 or 24 overrides it (for timing).
static int onesweep_items()
{
    if (const char *e = getenv("C3X_ONESWEEP_ITEMS")) {
        const int v = atoi(e);
        if (v == 16 || v == 24 || v == 32) return v;
    }
    return 32;
}

static uint32_t spin_limit()
{
    if (const char *e = getenv("C3X_DEBUG_SORT_SPIN")) return (uint32_t)std::max(0LL, atoll(e));
    return kSpinLimit;
}

hipError_t radix_sort_pairs_bits(uint32_t *keys, uint32_t *vals, uint32_t *ktmp, uint32_t *vtmp,
                                 int64_t n, int lo_bit, int nbits, void *ws, hipStream_t s,
                                 int *in_tmp, bool vals_are_index, uint32_t *fail)
{
    *in_tmp = 0;
    if (n <= 0) return hipSuccess;
    if (n == 1 || nbits <= lo_bit) {  // nothing to order: the values as they stand
        if (vals_are_index)
            hipLaunchKernelGGL(k_sort_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                               vals, n);
        return hipGetLastError();
    }
    // the first pass reads no values when they are the elements' own indices
    const uint32_t *vfirst = vals_are_index ? nullptr : vals;
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    // below kOneSweepMinTiles tiles the table's launches cost less than the
    // look-back's latency; above, one sweep is faster (when the caller can
    // observe a give-up), and from kRowScanTiles on the table would need a
    // full scan
    if (fail && nb >= onesweep_min_tiles() && n < kOneSweepMax) {
        const uint32_t spins = spin_limit();
        const int items = onesweep_items();
        const int64_t tile = (int64_t)kSortBlock * items;
        nb = (n + tile - 1) / tile;  // <= the 4096-element count the workspace is sized for
        const int npass = (nbits - lo_bit + 7) / 8;  // at most 4
        uint32_t *ghist = (uint32_t *)ws;
        uint32_t *tctr = ghist + 4 * 256;
        uint32_t *status = tctr + 64;
        const int64_t words = (int64_t)onesweep_words(nb, npass);
        hipLaunchKernelGGL(k_sort_clear, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                           ghist, words, 0u);
        const unsigned hb = (unsigned)std::min<int64_t>((n + 4 * kSortBlock - 1) / (4 * kSortBlock),
                                                        2048);
        hipLaunchKernelGGL(k_digit_hist_all, dim3(hb), dim3(kSortBlock), 0, s, keys, n, lo_bit,
                           npass, ghist);
        uint32_t *ka = keys, *va = vals, *kb = ktmp, *vb = vtmp;
        // with a test spin limit, every output slot starts as 0xffffffff, so
        // that the slots a pass that gave up leaves unwritten always hold an
        // out-of-range value (what every reader must survive)
        const bool poison = getenv("C3X_DEBUG_SORT_SPIN") != nullptr;
        const unsigned fb = (unsigned)((n + 255) / 256);
        for (int p = 0; p < npass; ++p) {
            if (poison) {
                hipLaunchKernelGGL(k_sort_clear, dim3(fb), dim3(256), 0, s, kb, n, 0xffffffffu);
                hipLaunchKernelGGL(k_sort_clear, dim3(fb), dim3(256), 0, s, vb, n, 0xffffffffu);
            }
#define C3X_ONESWEEP(IT)                                                                          \
    hipLaunchKernelGGL(k_onesweep<IT>, dim3((unsigned)nb), dim3(kSortBlock), 0, s, ka,             \
                       p == 0 ? vfirst : va, kb, vb, n, lo_bit + 8 * p, ghist + 256 * p, tctr + p, \
                       status + (size_t)p * 256 * (size_t)nb, (int)nb, spins, fail)
            if (items == 32) C3X_ONESWEEP(32);
            else if (items == 24) C3X_ONESWEEP(24);
            else C3X_ONESWEEP(16);
#undef C3X_ONESWEEP
            std::swap(ka, kb);
            std::swap(va, vb);
            *in_tmp ^= 1;
        }
        return hipGetLastError();
    }
    uint32_t *hist = (uint32_t *)ws;
    uint32_t *offs = hist + 256 * nb;
    uint32_t *tot = offs + 256 * nb;
    void *sws = (void *)(tot + 256);
    // up to this many tiles, one workgroup per digit scans its row
    const bool rows = nb <= kRowScanTiles;
    uint32_t *ka = keys, *va = vals, *kb = ktmp, *vb = vtmp;
    for (int shift = lo_bit; shift < nbits; shift += 8) {
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)nb), dim3(kSortBlock), 0, s, ka, n, shift,
                           hist, (int)nb);
        hipError_t e = hipSuccess;
        if (rows)
            hipLaunchKernelGGL(k_digit_rows, dim3(256), dim3(kScanBlock), 0, s, hist, (int)nb,
                               offs, tot);
        else
            e = scan_u32(hist, offs, 256 * nb, nullptr, sws, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)nb), dim3(kSortBlock), 0, s, ka,
                           shift == lo_bit ? vfirst : va, kb, vb, n, shift, offs,
                           rows ? tot : nullptr, hist, (int)nb);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint32_t *t = ka;
        ka = kb;
        kb = t;
        t = va;
        va = vb;
        vb = t;
        *in_tmp ^= 1;
    }
    return hipSuccess;
}

}  // namespace c3x
