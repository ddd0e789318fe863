// c3x_exact.hip -- the Exact Value functional case (paper Section 2.1: two
// rows match when the values of one chosen column each are equal) with the
// all / best match selections of Section 2.2, as a GPU hash join.
//
//   k_ev_hash      B keys normalised (float64: -0 as +0; NaN matches
//                  nothing) and hashed to 32 bits; the row its own value
//   radix sort     (hash, row) by hash, stable: rows ascending inside a hash
//   k_ev_gather    the normalised keys in hash order
//   k_dir_fill     a directory over the hash's top bits (the hash table's
//                  buckets are runs of the sorted array)
//   k_ev_probe     one thread per A row in input order: its bucket, the run of
//                  its hash, the rows with an equal key (count and first);
//                  MODE 1 writes them at the row's offset (ascending B rows)
//   scan           counts -> offsets
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "c3x_dir.h"
#include "c3x_host.h"
#include "c3x_sort.h"

namespace c3x {

// 64 -> 32-bit mix (the finaliser of a 64-bit multiplicative hash): every
// input bit reaches the top bits, which pick the bucket.
__device__ __forceinline__ uint32_t ev_hash(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (uint32_t)(k >> 32);
}

constexpr uint64_t kEvNaN = 0x7ff8000000000000ull;  // the one NaN pattern kept

// Normalised key bits and whether the value can match: int64 as is; float64
// with -0 folded onto +0, every NaN onto one pattern that matches nothing.
__device__ __forceinline__ uint64_t ev_norm(uint64_t bits, int type, bool &valid)
{
    valid = true;
    if (type == C3X_KEY_F64) {
        const double x = __longlong_as_double((long long)bits);
        if (x != x) {
            valid = false;
            return kEvNaN;
        }
        if (x == 0.0) return 0ull;
    }
    return bits;
}

__global__ void k_ev_hash(const uint64_t *__restrict__ key, int64_t n, int type,
                          uint32_t *__restrict__ hash)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    bool valid;
    const uint64_t k = ev_norm(key[t], type, valid);
    hash[t] = valid ? ev_hash(k) : 0xffffffffu;
}

__global__ void k_ev_gather(const uint32_t *__restrict__ rows, const uint64_t *__restrict__ key,
                            int64_t n, int type, uint64_t *__restrict__ ks)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t r = rows[p];
    if (r >= (uint64_t)n) r = 0;  // unreachable for a permutation
    bool valid;
    ks[p] = ev_norm(key[r], type, valid);
}

// One thread per A row. MODE 0: the number of equal keys and the first (the
// lowest B row: rows ascend inside a run of one hash). MODE 1: every match
// written at the row's offset, ascending; BEST-only output writes the first.
template <int MODE>
__global__ void k_ev_probe(const uint64_t *__restrict__ keyA, int64_t nA, int type,
                           const uint32_t *__restrict__ hs, const uint64_t *__restrict__ ks,
                           const uint32_t *__restrict__ rs, int64_t nB,
                           const uint32_t *__restrict__ dir, int dshift, uint32_t dsize,
                           uint32_t *__restrict__ cnt, int32_t *__restrict__ best,
                           const int64_t *__restrict__ off, int best_only, int64_t P,
                           int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                           uint32_t *__restrict__ err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nA) return;
    bool valid;
    const uint64_t k = ev_norm(keyA[i], type, valid);
    uint32_t c = 0;
    int32_t first = -1;
    int64_t o = 0, oe = 0;
    if (MODE == 1) {
        o = off[i];
        oe = off[i + 1];
        if (oe > P) {
            atomicOr(err, 1u);
            return;
        }
    }
    if (valid) {
        const uint32_t h = ev_hash(k);
        const uint32_t q = h >> dshift;
        uint32_t lo = 0, hi = 0;
        if (q + 1 < dsize) {
            hi = min(dir[q + 1], (uint32_t)nB);
            lo = min(dir[q], hi);
        }
        // the run of hash h inside the bucket
        while (lo < hi) {
            const uint32_t m = lo + ((hi - lo) >> 1);
            if (hs[m] < h) lo = m + 1;
            else hi = m;
        }
        for (uint32_t p = lo; p < (uint32_t)nB && hs[p] == h; ++p) {
            if (ks[p] != k) continue;
            if (first < 0) first = (int32_t)rs[p];
            if (MODE == 1 && !best_only) {
                if (o + c < oe) {
                    oa[o + c] = (int32_t)i;
                    ob[o + c] = (int32_t)rs[p];
                } else {
                    atomicOr(err, 2u);
                }
            }
            ++c;
        }
    }
    if (MODE == 0) {
        cnt[i] = best_only ? (c ? 1u : 0u) : c;
        best[i] = first;
    } else if (best_only && first >= 0) {
        if (o < oe) {
            oa[o] = (int32_t)i;
            ob[o] = first;
        } else {
            atomicOr(err, 2u);
        }
    }
}

__global__ void k_ev_finish(int64_t P, int64_t nA, double *__restrict__ sep,
                            const int32_t *__restrict__ best, double *__restrict__ bsep)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < P) sep[t] = 0.0;
    if (t < nA) bsep[t] = best[t] >= 0 ? 0.0 : NAN;
}

static inline unsigned eblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace c3x

using namespace c3x;

#define ECHK(expr, what)                                 \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

static c3x_status exact_impl(const uint64_t *keyA, int64_t nA, const uint64_t *keyB, int64_t nB,
                             int type, unsigned mode, hipStream_t s, c3x_result *R)
{
    const bool all = (mode & C3X_ALL) != 0;
    Arena tmp(s);
    uint32_t *hash = tmp.get_n<uint32_t>(nB), *rows = tmp.get_n<uint32_t>(nB);
    uint32_t *h2 = tmp.get_n<uint32_t>(nB), *r2 = tmp.get_n<uint32_t>(nB);
    uint64_t *ks = tmp.get_n<uint64_t>(nB);
    void *ws = tmp.get(std::max(radix_ws_bytes(nB), scan_ws_bytes(nA + 1)));
    uint32_t *cnt = tmp.get_n<uint32_t>(nA);
    int64_t *off = tmp.get_n<int64_t>(nA + 1);
    uint32_t *ctr = tmp.get_n<uint32_t>(4);  // 0: error flags
    // directory over the top D bits of the hash: about two B rows a bucket
    int D = 8;
    while (D < 30 && ((int64_t)1 << D) < 2 * nB) ++D;
    const int dshift = 32 - D;
    const uint32_t dsize = (1u << D) + 1u;
    uint32_t *dir = tmp.get_n<uint32_t>(dsize);
    const uint32_t gap_cap = dir_gap_cap(dsize), big_cap = dir_big_cap(dsize);
    uint3 *gaps = tmp.get_n<uint3>((int64_t)gap_cap + big_cap);
    uint32_t *n_gaps = tmp.get_n<uint32_t>(2);
    R->nA = nA;
    R->best_idx = R->mem.get_n<int32_t>(nA);
    R->best_sep = R->mem.get_n<double>(nA);
    if (!hash || !rows || !h2 || !r2 || !ks || !ws || !cnt || !off || !ctr || !dir || !gaps ||
        !n_gaps || !R->best_idx || !R->best_sep)
        return fail(C3X_ENOMEM, "exact-value buffers");
    ECHK(hipMemsetAsync(ctr, 0, 4 * sizeof(uint32_t), s), "memset");
    ECHK(hipMemsetAsync(n_gaps, 0, 2 * sizeof(uint32_t), s), "memset");
    if (nB > 0)
        hipLaunchKernelGGL(k_ev_hash, dim3(eblk(nB)), dim3(256), 0, s, keyB, nB, type, hash);
    ECHK(hipGetLastError(), "hash");
    int in_tmp = 0;
    ECHK(radix_sort_pairs(hash, rows, h2, r2, nB, 32, ws, s, &in_tmp, /*vals_are_index=*/true),
         "hash sort");
    const uint32_t *hs = in_tmp ? h2 : hash;
    const uint32_t *rs = in_tmp ? r2 : rows;
    if (nB > 0)
        hipLaunchKernelGGL(k_ev_gather, dim3(eblk(nB)), dim3(256), 0, s, rs, keyB, nB, type, ks);
    hipLaunchKernelGGL(k_dir_fill, dim3(eblk(nB + 1)), dim3(256), 0, s, hs, nB, dshift, dsize, dir,
                       gaps, n_gaps, gap_cap, big_cap);
    hipLaunchKernelGGL(k_dir_fill_gaps, dim3(4096), dim3(256), 0, s, gaps, n_gaps, gap_cap,
                       big_cap, dir);
    if (nA > 0)
        hipLaunchKernelGGL(k_ev_probe<0>, dim3(eblk(nA)), dim3(256), 0, s, keyA, nA, type, hs, ks,
                           rs, nB, dir, dshift, dsize, cnt, R->best_idx, nullptr, (int)!all,
                           (int64_t)0, nullptr, nullptr, ctr);
    ECHK(hipGetLastError(), "probe");
    ECHK(scan_u32_to_i64(cnt, 1, ~0u, off, nA, off + nA, ws, s), "scan");
    int64_t P = 0;
    ECHK(hipMemcpyAsync(&P, off + nA, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    ECHK(hipStreamSynchronize(s), "exact-value count");
    R->n_pairs = P;
    R->idxA = R->mem.get_n<int32_t>(P);
    R->idxB = R->mem.get_n<int32_t>(P);
    R->sep = R->mem.get_n<double>(P);
    if (!R->idxA || !R->idxB || !R->sep)
        return fail(C3X_ENOMEM, "result buffers (%lld pairs)", (long long)P);
    if (nA > 0)
        hipLaunchKernelGGL(k_ev_probe<1>, dim3(eblk(nA)), dim3(256), 0, s, keyA, nA, type, hs, ks,
                           rs, nB, dir, dshift, dsize, nullptr, nullptr, off, (int)!all, P,
                           R->idxA, R->idxB, ctr);
    if (std::max(P, nA) > 0)
        hipLaunchKernelGGL(k_ev_finish, dim3(eblk(std::max(P, nA))), dim3(256), 0, s, P, nA,
                           R->sep, R->best_idx, R->best_sep);
    ECHK(hipGetLastError(), "write");
    uint32_t flags = 0;
    ECHK(hipMemcpyAsync(&flags, ctr, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy");
    ECHK(hipStreamSynchronize(s), "c3x_exact_match");
    if (flags) return fail(C3X_EDEVICE, "internal: count and write passes disagree (%u)", flags);
    c3x_stats &S = R->stats;
    S.n_a = nA;
    S.n_b = nB;
    S.n_pairs = P;
    return C3X_OK;
}

extern "C" c3x_status c3x_exact_match(const void *keyA, int64_t nA, const void *keyB, int64_t nB,
                                      c3x_keytype type, unsigned mode, void *stream,
                                      c3x_result **out)
{
    clear_error();
    if (!out) return fail(C3X_EINVAL, "out is NULL");
    *out = nullptr;
    if (nA < 0 || nB < 0) return fail(C3X_EINVAL, "negative row count");
    if (nA > 2147483647LL || nB > 2147483647LL) return fail(C3X_ERANGE, "row count above 2^31 - 1");
    if ((nA > 0 && !keyA) || (nB > 0 && !keyB)) return fail(C3X_EINVAL, "NULL key array");
    if (type != C3X_KEY_I64 && type != C3X_KEY_F64) return fail(C3X_EINVAL, "bad key type");
    if (mode == 0 || (mode & ~(unsigned)(C3X_ALL | C3X_BEST)))
        return fail(C3X_EINVAL, "mode must be C3X_ALL, C3X_BEST or both");
    hipStream_t s = (hipStream_t)stream;
    c3x_result *R = new (std::nothrow) c3x_result();
    if (!R) return fail(C3X_ENOMEM, "host allocation");
    (void)hipGetDevice(&R->device);
    memset(&R->stats, 0, sizeof(R->stats));
    R->mode = mode;
    R->nB = nB;
    const c3x_status st = exact_impl((const uint64_t *)keyA, nA, (const uint64_t *)keyB, nB,
                                     (int)type, mode, s, R);
    if (st != C3X_OK) {
        (void)hipStreamSynchronize(s);
        delete R;
        return st;
    }
    *out = R;
    return C3X_OK;
}
