// c3x_sort.hip -- LSD radix sort of (u32 key, u32 value) pairs and prefix
// scans, written for 64-wide CDNA wavefronts.
//
// Sort: 8-bit digits, only as many passes as the key range needs. Each pass
// is a digit histogram per 4096-element tile (LDS atomics), a scan of the
// digit-major histogram table, and a stable scatter: each wavefront ranks
// its quarter of the tile with ballots (eight ballots match the lanes that
// share a digit; mbcnt gives the rank among them) against its own digit
// counters, one prefix over the wavefronts orders the quarters, and the
// whole tile is staged in LDS in digit order so that the global writes of a
// digit run are contiguous (about 16 elements per run).
#include "c3x_internal.h"
#include "c3x_sort.h"

namespace c3x {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;  // 4096
constexpr int kWaves = kSortBlock / 64;
constexpr int64_t kRowScanTiles = 8192;  // 32M elements

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
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        int64_t e = base + r * kSortBlock + threadIdx.x;
        if (e < n) atomicAdd(&h[(kk[r] >> shift) & 255u], 1u);
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
// write consecutive addresses of one digit run.
__global__ __launch_bounds__(kSortBlock) void k_digit_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const uint32_t *__restrict__ offs, const uint32_t *__restrict__ tot,
    const uint32_t *__restrict__ hist, int nblocks)
{
    constexpr int kPerWave = kSortTile / kWaves;  // 1024
    constexpr int kRounds = kPerWave / 64;        // 16
    __shared__ uint32_t sk[kSortTile], sv[kSortTile];
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
        vv[r] = e < n ? vin[e] : 0u;
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
            const uint32_t slot = tstart[d] + cnt[d] + loc[r];
            sk[slot] = kk[r];
            sv[slot] = vv[r];
        }
    }
    __syncthreads();
    int nt = (int)min<int64_t>(kSortTile, n - tbase);
    for (int p = tid; p < nt; p += kSortBlock) {
        uint32_t k = sk[p];
        uint32_t d = (k >> shift) & 255u;
        uint32_t dst = gbase[d] + (uint32_t)(p - tstart[d]);
        if (dst < (uint64_t)n) {
            kout[dst] = k;
            vout[dst] = sv[p];
        }
    }
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

template <typename Ti, typename To>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const Ti *__restrict__ in,
                                                            int64_t stride, int64_t n,
                                                            To *__restrict__ part)
{
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    To s = 0;
    for (int r = 0; r < kScanItems; ++r) {
        int64_t e = base + r * kScanBlock + threadIdx.x;
        if (e < n) s += (To)in[e * stride];
    }
    To tot;
    block_excl_scan<To>(s, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename To>
__global__ __launch_bounds__(kScanBlock) void k_scan_partials(To *part, int64_t np, To *total)
{
    To carry = 0;
    for (int64_t b = 0; b < np; b += kScanBlock) {
        int64_t e = b + threadIdx.x;
        To x = e < np ? part[e] : (To)0;
        To tot;
        To ex = block_excl_scan<To>(x, tot);
        if (e < np) part[e] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename Ti, typename To>
__global__ __launch_bounds__(kScanBlock) void k_scan_final(const Ti *__restrict__ in,
                                                           int64_t stride, int64_t n,
                                                           const To *__restrict__ part,
                                                           To *__restrict__ out)
{
    __shared__ To tile[kScanTile];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int r = 0; r < kScanItems; ++r) {
        int i = r * kScanBlock + threadIdx.x;
        int64_t e = base + i;
        tile[i] = e < n ? (To)in[e * stride] : (To)0;
    }
    __syncthreads();
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
static hipError_t scan_impl(const Ti *in, int64_t stride, To *out, int64_t n, To *total, void *ws,
                            hipStream_t s)
{
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    To *part = (To *)ws;
    if (n == 0) {
        if (total) return hipMemsetAsync(total, 0, sizeof(To), s);
        return hipSuccess;
    }
    hipLaunchKernelGGL((k_scan_reduce<Ti, To>), dim3((unsigned)nb), dim3(kScanBlock), 0, s, in,
                       stride, n, part);
    hipLaunchKernelGGL((k_scan_partials<To>), dim3(1), dim3(kScanBlock), 0, s, part, nb, total);
    hipLaunchKernelGGL((k_scan_final<Ti, To>), dim3((unsigned)nb), dim3(kScanBlock), 0, s, in,
                       stride, n, part, out);
    return hipGetLastError();
}

hipError_t scan_u32_to_i64(const uint32_t *in, int64_t stride, int64_t *out, int64_t n,
                           int64_t *total, void *ws, hipStream_t s)
{
    return scan_impl<uint32_t, int64_t>(in, stride, out, n, total, ws, s);
}

hipError_t scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *ws,
                    hipStream_t s)
{
    return scan_impl<uint32_t, uint32_t>(in, 1, out, n, total, ws, s);
}

size_t radix_ws_bytes(int64_t n)
{
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    size_t hist = (size_t)256 * (size_t)(nb > 0 ? nb : 1) * sizeof(uint32_t);
    return 2 * hist + 256 * sizeof(uint32_t) + scan_ws_bytes(256 * (nb > 0 ? nb : 1)) + 256;
}

hipError_t radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *ktmp, uint32_t *vtmp,
                            int64_t n, int nbits, void *ws, hipStream_t s, int *in_tmp)
{
    return radix_sort_pairs_bits(keys, vals, ktmp, vtmp, n, 0, nbits, ws, s, in_tmp);
}

hipError_t radix_sort_pairs_bits(uint32_t *keys, uint32_t *vals, uint32_t *ktmp, uint32_t *vtmp,
                                 int64_t n, int lo_bit, int nbits, void *ws, hipStream_t s,
                                 int *in_tmp)
{
    *in_tmp = 0;
    if (n <= 1 || nbits <= lo_bit) return hipSuccess;
    int64_t nb = (n + kSortTile - 1) / kSortTile;
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
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)nb), dim3(kSortBlock), 0, s, ka, va, kb,
                           vb, n, shift, offs, rows ? tot : nullptr, hist, (int)nb);
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
