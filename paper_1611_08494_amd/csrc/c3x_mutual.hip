// c3x_mutual.hip -- symmetric best pairs of a cross-match (Section 2.2: the
// "best" match selection keeps only the best pairs; read here as the pairs
// that are each other's nearest match). Besides each A row's best match,
// every B row gets its nearest A row among the A rows whose areas hold it
// (exact ties to the lower A row), and (i, j) is a symmetric best pair when
// best(i) = j and best_a_of_b(j) = i.
//
//   k_mu_fill     per B row: no minimum yet, no candidate          (16 B out)
//   k_mu_min      per pair: its separation's bits, atomicMin at its B row (12 B in)
//   k_mu_near     per pair within the error band of its row's minimum: count
//                 and lowest A row                                  (20 B in)
//   k_mu_list     B rows with two or more candidates in the band: listed for
//                 the exact ranking; the others keep their single candidate
//   k_mu_collect  the band candidates of the listed rows, with coordinates
//   host          binary128 ranking of each listed row (c3x_q_best, the B row
//                 as the centre: the angle is symmetric), winners patched
//   k_mu_flag     per A row: symmetric when its best's nearest A row is itself
//   scan_u32 + k_mu_write  the symmetric pairs in ascending A row
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "c3x_host.h"
#include "c3x_internal.h"
#include "c3x_sort.h"

namespace c3x {

// Error band of the stored separations: those from FP64 unit vectors carry
// at most ~1.3e-14 rad (2.7e-9 arcsec) absolute, the ones from the haversine
// form a few ulps relative. Two candidates further apart than twice the
// bound are ordered by their FP64 values; closer ones are ranked exactly.
constexpr double kMuAbs = 2.5e-8;              // arcsec, about 4 x 2 x 2.7e-9
constexpr double kMuRel = 3.637978807091713e-12;  // 2^-38

struct alignas(16) MuEnt {
    uint32_t slot, i;
    double ra, dec;
};

__global__ void k_mu_fill(int64_t nB, unsigned long long *__restrict__ minbits,
                          int32_t *__restrict__ first, uint32_t *__restrict__ cnt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nB) return;
    minbits[t] = 0x7ff0000000000000ull;  // +inf
    first[t] = 0x7fffffff;
    cnt[t] = 0u;
}

// Non-negative doubles order as their bit patterns.
__global__ void k_mu_min(const int32_t *__restrict__ ib, const double *__restrict__ sep,
                         int64_t P, int64_t nB, unsigned long long *__restrict__ minbits,
                         uint32_t *__restrict__ err)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P) return;
    const int32_t b = ib[t];
    const double s = sep[t];
    if (b < 0 || b >= nB || !(s >= 0.0)) {
        atomicOr(err, 1u);
        return;
    }
    atomicMin(minbits + b, (unsigned long long)__double_as_longlong(s));
}

__global__ void k_mu_near(const int32_t *__restrict__ ia, const int32_t *__restrict__ ib,
                          const double *__restrict__ sep, int64_t P, int64_t nB,
                          const unsigned long long *__restrict__ minbits,
                          int32_t *__restrict__ first, uint32_t *__restrict__ cnt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P) return;
    const int32_t b = ib[t];
    if (b < 0 || b >= nB) return;
    const double m = __longlong_as_double((long long)minbits[b]);
    if (sep[t] <= m + (kMuAbs + kMuRel * m)) {
        atomicAdd(cnt + b, 1u);
        atomicMin(first + b, ia[t]);
    }
}

// best_a_of_b: the single band candidate, -1 for rows without a match;
// rows with several are listed (slot[b] = their place in the list).
__global__ void k_mu_list(int64_t nB, const int32_t *__restrict__ first,
                          const uint32_t *__restrict__ cnt, int32_t *__restrict__ bab,
                          uint32_t *__restrict__ slot, uint32_t *__restrict__ list,
                          uint32_t *__restrict__ n_list, uint32_t cap)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nB) return;
    const uint32_t c = cnt[t];
    bab[t] = c == 0 ? -1 : first[t];
    slot[t] = 0xffffffffu;
    if (c >= 2) {
        const uint32_t s = atomicAdd(n_list, 1u);
        if (s < cap) {
            list[s] = (uint32_t)t;
            slot[t] = s;
        }
    }
}

__global__ void k_mu_collect(const int32_t *__restrict__ ia, const int32_t *__restrict__ ib,
                             const double *__restrict__ sep, int64_t P, int64_t nA, int64_t nB,
                             const unsigned long long *__restrict__ minbits,
                             const uint32_t *__restrict__ slot, const double *__restrict__ raA,
                             const double *__restrict__ decA, MuEnt *__restrict__ ent,
                             uint32_t *__restrict__ n_ent, uint32_t cap)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P) return;
    const int32_t b = ib[t], a = ia[t];
    if (b < 0 || b >= nB || a < 0 || a >= nA) return;
    const uint32_t s = slot[b];
    if (s == 0xffffffffu) return;
    const double m = __longlong_as_double((long long)minbits[b]);
    if (!(sep[t] <= m + (kMuAbs + kMuRel * m))) return;
    const uint32_t k = atomicAdd(n_ent, 1u);
    if (k < cap) {
        MuEnt e;
        e.slot = s;
        e.i = (uint32_t)a;
        e.ra = raA[a];
        e.dec = decA[a];
        ent[k] = e;
    }
}

__global__ void k_mu_gather_b(const uint32_t *__restrict__ rows, uint32_t n,
                              const double *__restrict__ raB, const double *__restrict__ decB,
                              double2 *__restrict__ out)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = make_double2(raB[rows[t]], decB[rows[t]]);
}

__global__ void k_mu_patch(const uint32_t *__restrict__ rows, const int32_t *__restrict__ win,
                           uint32_t n, int32_t *__restrict__ bab)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) bab[rows[t]] = win[t];
}

__global__ void k_mu_flag(const int32_t *__restrict__ best, int64_t nA, int64_t nB,
                          const int32_t *__restrict__ bab, uint32_t *__restrict__ flag)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nA) return;
    const int32_t b = best[t];
    flag[t] = (b >= 0 && b < nB && bab[b] == (int32_t)t) ? 1u : 0u;
}

__global__ void k_mu_write(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ off,
                           int64_t nA, const int32_t *__restrict__ best,
                           const double *__restrict__ bsep, int32_t *__restrict__ oa,
                           int32_t *__restrict__ ob, double *__restrict__ os)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nA || !flag[t]) return;
    const uint32_t p = off[t];
    oa[p] = (int32_t)t;
    ob[p] = best[t];
    os[p] = bsep[t];
}

static inline unsigned mblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace c3x

using namespace c3x;

#define MCHK(expr, what)                                 \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

extern "C" c3x_status c3x_result_mutual(c3x_result *r, const double *raA, const double *decA,
                                        const double *raB, const double *decB, void *stream,
                                        const int32_t **idxA, const int32_t **idxB,
                                        const double **sep, int64_t *n_pairs,
                                        const int32_t **best_a_of_b)
{
    clear_error();
    if (!r || !idxA || !idxB || !sep || !n_pairs) return fail(C3X_EINVAL, "NULL argument");
    if (r->nB < 0)
        return fail(C3X_EINVAL, "symmetric best pairs are defined for c3x_match results only "
                                "(a batch result holds job-local rows)");
    if ((r->mode & (C3X_ALL | C3X_BEST)) != (C3X_ALL | C3X_BEST))
        return fail(C3X_EINVAL, "symmetric best pairs need a result made with C3X_ALL | C3X_BEST");
    const int64_t nA = r->nA, nB = r->nB, P = r->n_pairs;
    if ((nA > 0 && (!raA || !decA)) || (nB > 0 && (!raB || !decB)))
        return fail(C3X_EINVAL, "NULL coordinate array");
    hipStream_t s = (hipStream_t)stream;
    if (!r->muA) r->muA = r->mem.get_n<int32_t>(nA);
    if (!r->muB) r->muB = r->mem.get_n<int32_t>(nA);
    if (!r->muS) r->muS = r->mem.get_n<double>(nA);
    if (!r->muBA) r->muBA = r->mem.get_n<int32_t>(nB);
    Arena tmp(s);
    unsigned long long *minbits = tmp.get_n<unsigned long long>(nB);
    int32_t *first = tmp.get_n<int32_t>(nB);
    uint32_t *cnt = tmp.get_n<uint32_t>(nB);
    uint32_t *slot = tmp.get_n<uint32_t>(nB);
    uint32_t *flag = tmp.get_n<uint32_t>(nA);
    uint32_t *off = tmp.get_n<uint32_t>(nA);
    uint32_t *ctr = tmp.get_n<uint32_t>(4);  // listed rows, entries, error, pairs
    void *ws = tmp.get(scan_ws_bytes(std::max<int64_t>(nA, 1)));
    uint32_t cap = (uint32_t)std::min<int64_t>(std::max<int64_t>(nB, 1), 1 << 24);
    uint32_t *list = tmp.get_n<uint32_t>(cap);
    if (!r->muA || !r->muB || !r->muS || !r->muBA || !minbits || !first || !cnt || !slot ||
        !flag || !off || !ctr || !ws || !list)
        return fail(C3X_ENOMEM, "symmetric best-pair buffers");
    MCHK(hipMemsetAsync(ctr, 0, 4 * sizeof(uint32_t), s), "memset");
    if (nB > 0) {
        hipLaunchKernelGGL(k_mu_fill, dim3(mblk(nB)), dim3(256), 0, s, nB, minbits, first, cnt);
        if (P > 0) {
            hipLaunchKernelGGL(k_mu_min, dim3(mblk(P)), dim3(256), 0, s, r->idxB, r->sep, P, nB,
                               minbits, ctr + 2);
            hipLaunchKernelGGL(k_mu_near, dim3(mblk(P)), dim3(256), 0, s, r->idxA, r->idxB,
                               r->sep, P, nB, minbits, first, cnt);
        }
        hipLaunchKernelGGL(k_mu_list, dim3(mblk(nB)), dim3(256), 0, s, nB, first, cnt, r->muBA,
                           slot, list, ctr, cap);
    }
    MCHK(hipGetLastError(), "nearest A rows");
    uint32_t h[4] = {0, 0, 0, 0};
    MCHK(hipMemcpyAsync(h, ctr, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy");
    MCHK(hipStreamSynchronize(s), "nearest A rows");
    if (h[2]) return fail(C3X_EINVAL, "a stored pair names a row outside its catalogue");
    if (h[0] > cap) return fail(C3X_ENOMEM, "more than %u B rows need exact ranking", cap);
    const uint32_t nl = h[0];
    if (nl > 0) {
        // band candidates of the listed rows, ranked in binary128 on the host
        uint32_t ecap = (uint32_t)std::min<int64_t>(std::max<int64_t>(4 * (int64_t)nl, 64), P);
        std::vector<MuEnt> ent;
        for (int attempt = 0; attempt < 2; ++attempt) {
            MuEnt *dent = (MuEnt *)tmp.get((size_t)ecap * sizeof(MuEnt));
            if (!dent) return fail(C3X_ENOMEM, "exact ranking list");
            MCHK(hipMemsetAsync(ctr + 1, 0, sizeof(uint32_t), s), "memset");
            hipLaunchKernelGGL(k_mu_collect, dim3(mblk(P)), dim3(256), 0, s, r->idxA, r->idxB,
                               r->sep, P, nA, nB, minbits, slot, raA, decA, dent, ctr + 1, ecap);
            uint32_t ne = 0;
            MCHK(hipMemcpyAsync(&ne, ctr + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy");
            MCHK(hipStreamSynchronize(s), "exact ranking list");
            if (ne > ecap) {
                ecap = ne;
                continue;
            }
            ent.resize(ne);
            MCHK(hipMemcpyAsync(ent.data(), dent, ne * sizeof(MuEnt), hipMemcpyDeviceToHost, s),
                 "copy");
            break;
        }
        double2 *dcb = tmp.get_n<double2>(nl);
        if (!dcb) return fail(C3X_ENOMEM, "exact ranking list");
        hipLaunchKernelGGL(k_mu_gather_b, dim3(mblk(nl)), dim3(256), 0, s, list, nl, raB, decB,
                           dcb);
        std::vector<double2> cb(nl);
        MCHK(hipMemcpyAsync(cb.data(), dcb, nl * sizeof(double2), hipMemcpyDeviceToHost, s),
             "copy");
        MCHK(hipStreamSynchronize(s), "exact ranking list");
        std::vector<std::vector<const MuEnt *>> per(nl);
        for (const MuEnt &e : ent)
            if (e.slot < nl) per[e.slot].push_back(&e);
        std::vector<int32_t> win(nl, -1);
        for (uint32_t k = 0; k < nl; ++k) {
            auto &v = per[k];
            if (v.empty()) continue;
            std::vector<double> ra2(v.size()), dec2(v.size());
            std::vector<int32_t> idx(v.size());
            for (size_t q = 0; q < v.size(); ++q) {
                ra2[q] = v[q]->ra;
                dec2[q] = v[q]->dec;
                idx[q] = (int32_t)v[q]->i;
            }
            const int w = c3x_q_best(cb[k].x, cb[k].y, (int)v.size(), ra2.data(), dec2.data(),
                                     idx.data());
            win[k] = idx[w];
        }
        int32_t *dwin = tmp.get_n<int32_t>(nl);
        if (!dwin) return fail(C3X_ENOMEM, "exact ranking list");
        MCHK(hipMemcpyAsync(dwin, win.data(), nl * sizeof(int32_t), hipMemcpyHostToDevice, s),
             "copy");
        hipLaunchKernelGGL(k_mu_patch, dim3(mblk(nl)), dim3(256), 0, s, list, dwin, nl, r->muBA);
    }
    if (nA > 0) {
        hipLaunchKernelGGL(k_mu_flag, dim3(mblk(nA)), dim3(256), 0, s, r->best_idx, nA, nB,
                           r->muBA, flag);
        MCHK(scan_u32(flag, off, nA, ctr + 3, ws, s), "scan");
        hipLaunchKernelGGL(k_mu_write, dim3(mblk(nA)), dim3(256), 0, s, flag, off, nA,
                           r->best_idx, r->best_sep, r->muA, r->muB, r->muS);
    }
    MCHK(hipGetLastError(), "symmetric pairs");
    uint32_t np = 0;
    MCHK(hipMemcpyAsync(&np, ctr + 3, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy");
    MCHK(hipStreamSynchronize(s), "c3x_result_mutual");
    *idxA = r->muA;
    *idxB = r->muB;
    *sep = r->muS;
    *n_pairs = nA > 0 ? (int64_t)np : 0;
    if (best_a_of_b) *best_a_of_b = r->muBA;
    r->n_mutual = *n_pairs;
    return C3X_OK;
}
