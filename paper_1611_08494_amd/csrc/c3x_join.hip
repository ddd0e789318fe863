// c3x_join.hip -- rows without a stored match, the ingredient of the join
// types of Section 2.2 ("Match selection and join types"): every join is a
// union of the stored pairs, the catalogue-A rows in no stored pair and the
// catalogue-B rows in no stored pair.
//
//   k_mark_pairs / k_mark_best  flag the rows the stored pairs name   (8 B per pair in)
//   k_tile_unmatched            unmatched rows per 4096-row tile      (1 B per row in)
//   scan_u32                    tile offsets
//   k_tile_compact              the unmatched rows, ascending         (1 B in, 4 B out per row)
#include <algorithm>
#include <cstring>
#include <mutex>

#include "c3x_host.h"
#include "c3x_internal.h"
#include "c3x_sort.h"

namespace c3x {

constexpr int kJoinBlock = 256;
constexpr int kJoinRounds = 16;
constexpr int64_t kJoinTile = (int64_t)kJoinBlock * kJoinRounds;  // 4096 rows

// Flags of the rows named by the stored pairs (every match): a row named at
// least once gets 1 (concurrent stores all write 1). A row index outside
// its catalogue sets *err and is skipped.
__global__ void k_mark_pairs(const int32_t *__restrict__ ia, const int32_t *__restrict__ ib,
                             int64_t n, int64_t nA, int64_t nB, uint8_t *__restrict__ fa,
                             uint8_t *__restrict__ fb, uint32_t *__restrict__ err)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t a = ia[t], b = ib[t];
    if (a < 0 || a >= nA || b < 0 || b >= nB) {
        atomicOr(err, 1u);
        return;
    }
    fa[a] = 1;
    fb[b] = 1;
}

// The same for the best pairs: A row t and its best match best[t] (-1: none).
__global__ void k_mark_best(const int32_t *__restrict__ best, int64_t nA, int64_t nB,
                            uint8_t *__restrict__ fa, uint8_t *__restrict__ fb,
                            uint32_t *__restrict__ err)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nA) return;
    const int32_t b = best[t];
    if (b < 0) return;
    if (b >= nB) {
        atomicOr(err, 1u);
        return;
    }
    fa[t] = 1;
    fb[b] = 1;
}

// Exclusive prefix over the block's 256 threads of x, and the block's sum.
__device__ __forceinline__ uint32_t join_block_scan(uint32_t x, uint32_t &sum, uint32_t *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t pre = 0;
    sum = 0;
#pragma unroll
    for (int w = 0; w < kJoinBlock / 64; ++w) {
        if (w < wave) pre += wsum[w];
        sum += wsum[w];
    }
    __syncthreads();
    return pre + inc - x;
}

// Unmatched rows (flag 0) of each tile.
__global__ __launch_bounds__(kJoinBlock) void k_tile_unmatched(const uint8_t *__restrict__ f,
                                                               int64_t n,
                                                               uint32_t *__restrict__ cnt)
{
    __shared__ uint32_t wsum[kJoinBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kJoinTile;
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < kJoinRounds; ++r) {
        const int64_t e = base + r * kJoinBlock + threadIdx.x;
        c += (e < n && f[e] == 0) ? 1u : 0u;
    }
    uint32_t sum;
    (void)join_block_scan(c, sum, wsum);
    if (threadIdx.x == 0) cnt[blockIdx.x] = sum;
}

// The tile's unmatched rows in ascending order from the tile's offset: 256
// consecutive rows a round, placed by a block prefix of their flags.
__global__ __launch_bounds__(kJoinBlock) void k_tile_compact(const uint8_t *__restrict__ f,
                                                             int64_t n,
                                                             const uint32_t *__restrict__ off,
                                                             int32_t *__restrict__ out)
{
    __shared__ uint32_t wsum[kJoinBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kJoinTile;
    uint32_t at = off[blockIdx.x];
    for (int r = 0; r < kJoinRounds; ++r) {
        const int64_t e = base + r * kJoinBlock + threadIdx.x;
        const uint32_t x = (e < n && f[e] == 0) ? 1u : 0u;
        uint32_t sum;
        const uint32_t p = join_block_scan(x, sum, wsum);
        if (x) out[at + p] = (int32_t)e;
        at += sum;
    }
}

static inline unsigned jblk(int64_t n, int64_t b) { return (unsigned)((n + b - 1) / b); }

// Flags f[0, n) -> the rows with flag 0, ascending, into out; their number
// into *total (device).
static hipError_t compact_unmatched(const uint8_t *f, int64_t n, int32_t *out, uint32_t *cnt,
                                    uint32_t *off, uint32_t *total, void *ws, hipStream_t s)
{
    const int64_t nt = (n + kJoinTile - 1) / kJoinTile;
    if (nt == 0) return hipMemsetAsync(total, 0, sizeof(uint32_t), s);
    hipLaunchKernelGGL(k_tile_unmatched, dim3((unsigned)nt), dim3(kJoinBlock), 0, s, f, n, cnt);
    hipError_t e = scan_u32(cnt, off, nt, total, ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_compact, dim3((unsigned)nt), dim3(kJoinBlock), 0, s, f, n, off, out);
    return hipGetLastError();
}

}  // namespace c3x

using namespace c3x;

#define JCHK(expr, what)                                 \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

extern "C" c3x_status c3x_result_unmatched(c3x_result *r, unsigned selection, void *stream,
                                           const int32_t **rowsA, int64_t *n_rowsA,
                                           const int32_t **rowsB, int64_t *n_rowsB)
{
    clear_error();
    if (!r || !rowsA || !n_rowsA || !rowsB || !n_rowsB) return fail(C3X_EINVAL, "NULL argument");
    if (r->nB < 0)
        return fail(C3X_EINVAL, "unmatched rows are defined for c3x_match results only (a batch "
                                "result holds job-local rows)");
    if (selection != C3X_ALL && selection != C3X_BEST)
        return fail(C3X_EINVAL, "selection must be C3X_ALL or C3X_BEST");
    if (selection == C3X_ALL && !(r->mode & C3X_ALL))
        return fail(C3X_EINVAL, "selection C3X_ALL needs a result made with C3X_ALL");
    if (selection == C3X_BEST && !(r->mode & C3X_BEST))
        return fail(C3X_EINVAL, "selection C3X_BEST needs a result made with C3X_BEST");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nA = r->nA, nB = r->nB;
    if (!r->unA) r->unA = r->mem.get_n<int32_t>(nA);
    if (!r->unB) r->unB = r->mem.get_n<int32_t>(nB);
    const int64_t tA = (nA + kJoinTile - 1) / kJoinTile, tB = (nB + kJoinTile - 1) / kJoinTile;
    Arena tmp(s);
    uint8_t *fa = (uint8_t *)tmp.get((size_t)std::max<int64_t>(nA, 1));
    uint8_t *fb = (uint8_t *)tmp.get((size_t)std::max<int64_t>(nB, 1));
    uint32_t *cnt = tmp.get_n<uint32_t>(tA + tB);
    uint32_t *off = tmp.get_n<uint32_t>(tA + tB);
    uint32_t *ctr = tmp.get_n<uint32_t>(4);  // total A, total B, error
    void *ws = tmp.get(scan_ws_bytes(std::max<int64_t>(tA, tB)));
    if (!r->unA || !r->unB || !fa || !fb || !cnt || !off || !ctr || !ws)
        return fail(C3X_ENOMEM, "unmatched-row buffers");
    JCHK(hipMemsetAsync(ctr, 0, 4 * sizeof(uint32_t), s), "memset");
    if (nA > 0) JCHK(hipMemsetAsync(fa, 0, (size_t)nA, s), "memset");
    if (nB > 0) JCHK(hipMemsetAsync(fb, 0, (size_t)nB, s), "memset");
    if (selection == C3X_ALL) {
        if (r->n_pairs > 0)
            hipLaunchKernelGGL(k_mark_pairs, dim3(jblk(r->n_pairs, 256)), dim3(256), 0, s, r->idxA,
                               r->idxB, r->n_pairs, nA, nB, fa, fb, ctr + 2);
    } else if (nA > 0) {
        hipLaunchKernelGGL(k_mark_best, dim3(jblk(nA, 256)), dim3(256), 0, s, r->best_idx, nA, nB,
                           fa, fb, ctr + 2);
    }
    JCHK(hipGetLastError(), "mark");
    JCHK(compact_unmatched(fa, nA, r->unA, cnt, off, ctr + 0, ws, s), "compact A");
    // the B tiles reuse the scan workspace after the A compaction (stream order)
    JCHK(compact_unmatched(fb, nB, r->unB, cnt + tA, off + tA, ctr + 1, ws, s), "compact B");
    uint32_t h[4] = {0, 0, 0, 0};
    uint32_t *hs = (uint32_t *)pinned_stage(64);
    uint32_t *dst = hs ? hs : h;
    JCHK(hipMemcpyAsync(dst, ctr, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy");
    JCHK(hipStreamSynchronize(s), "c3x_result_unmatched");
    memcpy(h, dst, sizeof(h));
    if (h[2]) return fail(C3X_EINVAL, "a stored pair names a row outside its catalogue");
    *rowsA = r->unA;
    *n_rowsA = (int64_t)h[0];
    *rowsB = r->unB;
    *n_rowsB = (int64_t)h[1];
    return C3X_OK;
}

// ---------------------------------------------------------------------------- no allocation

namespace c3x {

// Working memory of c3x_result_unmatched_noalloc: one array per GPU, held
// until the process ends. Host code reaches it only through the address
// hipGetSymbolAddress gives for the current device (the array's own name is
// a host stand-in, not a device address).
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint8_t *g_scratch[kMaxDevices];

// The current device's copy of the array (set-up once per device, with that
// device current); null, with the message set, when it cannot be had.
static uint8_t *scratch_on_device(int *dev_out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        fail(C3X_EDEVICE, "no current HIP device (or more than %d devices)", kMaxDevices);
        return nullptr;
    }
    *dev_out = dev;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(C3X_EDEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
            return nullptr;
        }
        g_scratch[dev] = (uint8_t *)p;
    }
    return g_scratch[dev];
}

__global__ void k_fill_u8(uint8_t *__restrict__ p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0;
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0u;
}

// Counts of unmatched rows to the caller's device array; -1 for both when a
// stored pair named a row outside its catalogue.
__global__ void k_unmatched_counts(const uint32_t *__restrict__ ctr, int64_t *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const bool bad = ctr[2] != 0;
        out[0] = bad ? -1 : (int64_t)ctr[0];
        out[1] = bad ? -1 : (int64_t)ctr[1];
    }
}

static inline size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

// Bytes of the array a result of nA and nB rows needs.
static size_t noalloc_bytes(int64_t nA, int64_t nB)
{
    const int64_t tA = (nA + kJoinTile - 1) / kJoinTile, tB = (nB + kJoinTile - 1) / kJoinTile;
    return up256((size_t)nA) + up256((size_t)nB) + 2 * up256((size_t)(tA + tB) * 4) + 256 +
           up256(scan_ws_bytes(std::max<int64_t>(std::max(tA, tB), 1)));
}

// The flags' rows with flag 0, ascending, as compact_unmatched, without the
// zero-length scan's memset (n == 0 writes its zero total with a kernel).
static hipError_t compact_noalloc(const uint8_t *f, int64_t n, int32_t *out, uint32_t *cnt,
                                  uint32_t *off, uint32_t *total, void *ws, hipStream_t s)
{
    const int64_t nt = (n + kJoinTile - 1) / kJoinTile;
    if (nt == 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, total, (int64_t)1);
        return hipGetLastError();
    }
    return compact_unmatched(f, n, out, cnt, off, total, ws, s);
}

}  // namespace c3x

extern "C" c3x_status c3x_result_unmatched_noalloc(const c3x_result *r, unsigned selection,
                                                   void *stream, int32_t *rowsA, int64_t capA,
                                                   int32_t *rowsB, int64_t capB,
                                                   int64_t *counts)
{
    clear_error();
    if (!r || !counts || (r->nA > 0 && !rowsA) || (r->nB > 0 && !rowsB))
        return fail(C3X_EINVAL, "NULL argument");
    if (r->nB < 0)
        return fail(C3X_EINVAL, "unmatched rows are defined for c3x_match results only (a batch "
                                "result holds job-local rows)");
    if (selection != C3X_ALL && selection != C3X_BEST)
        return fail(C3X_EINVAL, "selection must be C3X_ALL or C3X_BEST");
    if (selection == C3X_ALL && !(r->mode & C3X_ALL))
        return fail(C3X_EINVAL, "selection C3X_ALL needs a result made with C3X_ALL");
    if (selection == C3X_BEST && !(r->mode & C3X_BEST))
        return fail(C3X_EINVAL, "selection C3X_BEST needs a result made with C3X_BEST");
    const int64_t nA = r->nA, nB = r->nB;
    if (capA < nA || capB < nB)
        return fail(C3X_EINVAL, "output capacities %lld, %lld below the result's %lld A and %lld "
                                "B rows", (long long)capA, (long long)capB, (long long)nA,
                    (long long)nB);
    const size_t need = noalloc_bytes(nA, nB);
    if (need > kNoAllocBytes)
        return fail(C3X_ERANGE, "%lld A + %lld B rows need %zu bytes of working memory, above the "
                                "fixed %zu", (long long)nA, (long long)nB, need, kNoAllocBytes);
    int dev = 0;
    uint8_t *base = scratch_on_device(&dev);
    if (!base) return C3X_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t tA = (nA + kJoinTile - 1) / kJoinTile, tB = (nB + kJoinTile - 1) / kJoinTile;
    uint8_t *at = base;
    uint8_t *fa = at;
    at += up256((size_t)nA);
    uint8_t *fb = at;
    at += up256((size_t)nB);
    uint32_t *cnt = (uint32_t *)at;
    at += up256((size_t)(tA + tB) * 4);
    uint32_t *off = (uint32_t *)at;
    at += up256((size_t)(tA + tB) * 4);
    uint32_t *ctr = (uint32_t *)at;  // total A, total B, error
    at += 256;
    void *ws = at;
    // the array keeps the last call's contents: clear what must start at zero
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, ctr, (int64_t)4);
    if (nA > 0) hipLaunchKernelGGL(k_fill_u8, dim3(jblk(nA, 256)), dim3(256), 0, s, fa, nA);
    if (nB > 0) hipLaunchKernelGGL(k_fill_u8, dim3(jblk(nB, 256)), dim3(256), 0, s, fb, nB);
    if (selection == C3X_ALL) {
        if (r->n_pairs > 0)
            hipLaunchKernelGGL(k_mark_pairs, dim3(jblk(r->n_pairs, 256)), dim3(256), 0, s, r->idxA,
                               r->idxB, r->n_pairs, nA, nB, fa, fb, ctr + 2);
    } else if (nA > 0) {
        hipLaunchKernelGGL(k_mark_best, dim3(jblk(nA, 256)), dim3(256), 0, s, r->best_idx, nA, nB,
                           fa, fb, ctr + 2);
    }
    JCHK(hipGetLastError(), "mark");
    JCHK(compact_noalloc(fa, nA, rowsA, cnt, off, ctr + 0, ws, s), "compact A");
    JCHK(compact_noalloc(fb, nB, rowsB, cnt + tA, off + tA, ctr + 1, ws, s), "compact B");
    hipLaunchKernelGGL(k_unmatched_counts, dim3(1), dim3(64), 0, s, ctr, counts);
    JCHK(hipGetLastError(), "counts");
    (void)dev;
    return C3X_OK;
}
