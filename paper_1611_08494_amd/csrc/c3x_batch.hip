// c3x_batch.hip -- many independent circular cross-matches in one graph.
//
// Each job (a slice of catalogue A, a slice of catalogue B and a radius) is
// a "Sky" cross-match of its own (paper Section 2.1, all and best matches of
// Section 2.2). The paper runs such work as independent processes over a
// partition of the input; here every job of a batch shares one index and
// one launch of each kernel:
//   plan     per job, its mean direction c and the largest distance D of
//            its sources from c (device reductions); a local frame (c, east,
//            north) in which the job's sky is a small box around (0, 0), with
//            no pole and no RA seam; a grid of square cells of side h over
//            that box, h picked per job from its density and radius (the
//            autotuner times a few cell scales and keeps the fastest); the
//            jobs' cells numbered in one key space (key_base per job)
//   pipeline keys of every (job, row) entry of B and A, one radix sort of
//            each, directory over the keys, candidate ranges per A source,
//            then the match kernels of the single call in their batch form
//            (per-source job thresholds, FP32 offsets from the job centre),
//            the FP64 band recheck, the rare binary128 decisions in a host
//            node, FP64 best re-ranking, scan, placement, canonical order,
//            and job-local indices
//   graph    the pipeline is captured once into a hipGraph; c3x_batch_run
//            replays it (one launch); capacities come from the plan's own
//            first run, and any overflow on a replay is reported, never
//            written past.
// Batches are circular (fixed radius per job, at most 1 degree); a job's
// sources must lie within 10 degrees of their mean direction (the local box
// stays small). This file is compiled as part of c3x_match.hip, whose match
// kernels it launches in their batch form.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "c3x_batch_kernels.h"
#include "c3x_dir.h"

namespace c3x {

constexpr double kMaxJobExtentDeg = 10.0;
constexpr double kMaxBatchRadiusArcsec = 3600.0;

// ---------------------------------------------------------------------------- device helpers

// Job of entry e: the last j with pref[j] <= e (pref ascending, pref[0] = 0).
__device__ __forceinline__ uint32_t job_of(const uint32_t *__restrict__ pref, int nj, uint32_t e)
{
    int lo = 0, hi = nj;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= e) lo = mid;
        else hi = mid;
    }
    return (uint32_t)lo;
}

// Caller row of entry e of job jb (A side or B side).
__device__ __forceinline__ int64_t entry_row(const BJob &jb, uint32_t e, bool isB)
{
    return isB ? jb.b_off + (int64_t)(e - jb.b_ent) : jb.a_off + (int64_t)(e - jb.a_ent);
}

// (ra', dec') in degrees of unit vector p in job jb's local frame.
// Tangent-plane coordinates of unit vector p in job jb's frame.
__device__ __forceinline__ void local_plane(const BJob &jb, double x, double y, double z,
                                            double &px, double &py)
{
    const double u = x * jb.cx + y * jb.cy + z * jb.cz;
    const double v = x * jb.ex + y * jb.ey + z * jb.ez;
    const double w = x * jb.nx + y * jb.ny + z * jb.nz;
    const double iu = 1.0 / u;
    px = v * iu;
    py = w * iu;
}

__device__ __forceinline__ uint32_t clampu(double t, uint32_t n)
{
    if (!(t >= 0.0)) return 0;
    if (t >= (double)n) return n - 1;
    return (uint32_t)t;
}

__global__ void k_bfill(uint32_t *p, int64_t n, uint32_t v)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

__global__ void k_bfill64(unsigned long long *p, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0ull;
}

// Sum of the unit vectors of every (job, row) entry, per job (A and B
// entries; a wavefront of one job adds once).
__global__ void k_bsum(const BJob *__restrict__ jobs, const uint32_t *__restrict__ pref, int nj,
                       const double *__restrict__ ra, const double *__restrict__ dec, int64_t n,
                       bool isB, double *__restrict__ sums, uint32_t *__restrict__ bad)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = e < n;
    uint32_t j = 0;
    double x = 0.0, y = 0.0, z = 0.0;
    if (valid) {
        j = job_of(pref, nj, (uint32_t)e);
        const int64_t row = entry_row(jobs[j], (uint32_t)e, isB);
        const double a = ra[row], d = dec[row];
        if (!(isfinite(a) && isfinite(d) && a >= 0.0 && a < 360.0 && fabs(d) <= 90.0)) {
            atomicMin(bad, (uint32_t)j);
        } else {
            unit_vec(a, d, x, y, z);
        }
    }
    const uint32_t j0 = (uint32_t)__shfl((int)j, 0);
    if (__all(!valid || j == j0)) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            x += __shfl_xor(x, o);
            y += __shfl_xor(y, o);
            z += __shfl_xor(z, o);
        }
        if (__lane_id() == 0 && (x != 0.0 || y != 0.0 || z != 0.0)) {
            atomicAdd(&sums[3 * j0], x);
            atomicAdd(&sums[3 * j0 + 1], y);
            atomicAdd(&sums[3 * j0 + 2], z);
        }
    } else if (valid) {
        atomicAdd(&sums[3 * j], x);
        atomicAdd(&sums[3 * j + 1], y);
        atomicAdd(&sums[3 * j + 2], z);
    }
}

// Job of every entry (entries of job j: [pref[j], pref[j + 1])).
__global__ void k_bjob_fill(const uint32_t *__restrict__ pref, int nj, int64_t n,
                            uint32_t *__restrict__ ejob)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) ejob[e] = job_of(pref, nj, (uint32_t)e);
}

// Largest angle (deg, as ordered bits of a non-negative double) between an
// entry and its job's centre.
__global__ void k_bext(const BJob *__restrict__ jobs, const uint32_t *__restrict__ pref, int nj,
                       const double *__restrict__ ra, const double *__restrict__ dec, int64_t n,
                       bool isB, unsigned long long *__restrict__ ext)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint32_t j = job_of(pref, nj, (uint32_t)e);
    const BJob &jb = jobs[j];
    const int64_t row = entry_row(jb, (uint32_t)e, isB);
    double x, y, z;
    unit_vec(ra[row], dec[row], x, y, z);
    const double cx = y * jb.cz - z * jb.cy, cy = z * jb.cx - x * jb.cz, cz = x * jb.cy - y * jb.cx;
    const double ang = atan2(sqrt(cx * cx + cy * cy + cz * cz), x * jb.cx + y * jb.cy + z * jb.cz) *
                       (180.0 / kPi);
    atomicMax(&ext[j], (unsigned long long)__double_as_longlong(ang));
}

// Cell key of every entry (its value in the sort: the entry number). Entries outside
// their job's planned box are reported (the plan no longer fits the data).
__global__ void k_bkeys(const BJob *__restrict__ jobs, const uint32_t *__restrict__ ejob,
                        const double *__restrict__ ra, const double *__restrict__ dec, int64_t n,
                        bool isB, uint32_t *__restrict__ keys, double2 *__restrict__ packed,
                        uint32_t *__restrict__ flags)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint32_t j = ejob[e];
    const BJob &jb = jobs[j];
    const int64_t row = entry_row(jb, (uint32_t)e, isB);
    double a = ra[row], d = dec[row];
    if (!(isfinite(a) && isfinite(d) && a >= 0.0 && a < 360.0 && fabs(d) <= 90.0)) {
        atomicOr(flags, kBFlagStale);
        a = 0.0;
        d = 0.0;
    }
    packed[e] = make_double2(a, d);  // one 16-byte record per entry for the gathers
    double x, y, z, px, py;
    unit_vec(a, d, x, y, z);
    local_plane(jb, x, y, z, px, py);
    const double tr = (py + jb.T) * jb.inv_h, tc = (px + jb.T) * jb.inv_h;
    if (!(tr >= 0.0 && tr < (double)jb.nrow && tc >= 0.0 && tc < (double)jb.ncol))
        atomicOr(flags, kBFlagStale);
    const uint32_t r = clampu(tr, jb.nrow), c = clampu(tc, jb.ncol);
    keys[e] = jb.key_base + r * jb.ncol + c;
}

// Sorted B payloads: FP64 unit vector, FP32 offset from the job centre; idx
// is the B entry (its coordinates stay in packB, in entry order).
__global__ void k_bgather_b(const uint32_t *__restrict__ rows, const BJob *__restrict__ jobs,
                            const uint32_t *__restrict__ ejob, const double2 *__restrict__ packed,
                            int64_t n, Pay64 *__restrict__ p64, Pay32 *__restrict__ p32)
{
    // a job's sorted entries take its own entries' places (keys are job-major),
    // and one XCD reads one job's rows
    const int64_t s = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t e = rows[s];
    if (e >= (uint64_t)n) e = 0;  // unreachable for a permutation
    const BJob &jb = jobs[ejob[s]];
    const double2 ad = packed[e];
    const double a = ad.x, d = ad.y;
    double x, y, z;
    unit_vec(a, d, x, y, z);
    if (p64) {
        Pay64 q;
        q.x = x;
        q.y = y;
        q.z = z;
        q.idx = e;
        q.pad = 0;
        p64[s] = q;
    }
    if (p32) {
        Pay32 f;
        f.x = (float)(x - jb.cx);
        f.y = (float)(y - jb.cy);
        f.z = (float)(z - jb.cz);
        f.idx = e;
        p32[s] = f;
    }
}

// Sorted A records and candidate ranges: up to three grid rows within the
// radius (h exceeds the radius), in each the columns within
// asin(sin r / cos dec'_max) of ra', padded for rounding, as sorted B
// positions.
__global__ void k_bgather_a(const uint32_t *__restrict__ rows, const BJob *__restrict__ jobs,
                            const uint32_t *__restrict__ ejob, const double2 *__restrict__ packed,
                            int64_t n, Grid g, double2 *__restrict__ arad,
                            uint32_t *__restrict__ aidx, uint32_t *__restrict__ ajob,
                            ARange *__restrict__ arng)
{
    const int64_t s = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t e = rows[s];
    if (e >= (uint64_t)n) e = 0;
    const uint32_t j = ejob[s];
    const BJob &jb = jobs[j];
    const double2 ad = packed[e];  // checked (else zeroed) by the key pass
    const double a = ad.x, d = ad.y;
    arad[s] = ad;
    aidx[s] = e;
    ajob[s] = j;
    double x, y, z, px, py;
    unit_vec(a, d, x, y, z);
    local_plane(jb, x, y, z, px, py);
    // B within the radius of A lies within wd of it on the plane along each
    // axis (wd bounds the projection's stretch over the job's cap, with pads)
    const uint32_t r0 = clampu((py - jb.wd + jb.T) * jb.inv_h, jb.nrow);
    const uint32_t r1 = clampu((py + jb.wd + jb.T) * jb.inv_h, jb.nrow);
    const uint32_t c0 = clampu((px - jb.wd + jb.T) * jb.inv_h, jb.ncol);
    const uint32_t c1 = clampu((px + jb.wd + jb.T) * jb.inv_h, jb.ncol);
    ARange rg;
    rg.wide = 0;
    rg.zlo = (int32_t)r0;
    bool ok = r1 - r0 < (uint32_t)kRZ;
#pragma unroll
    for (int q = 0; q < kRZ; ++q) {
        uint32_t j0 = 0, j1 = 0;
        if (ok && r0 + q <= r1) {
            const uint32_t kb = jb.key_base + (r0 + q) * jb.ncol;
            j0 = key_lower_bound(g, kb + c0);
            j1 = key_lower_bound(g, kb + c1 + 1);
        }
        if (j1 < j0) j1 = j0;
        ok = ok && j1 - j0 < 65535u;
        rg.j0[q] = j0;
        rg.n[q] = (uint16_t)(ok ? j1 - j0 : 0u);
    }
    if (!ok) rg.zlo = -1;
    arng[s] = rg;
}

// FP64 relative recheck of the band candidates (one thread each). IN goes to
// the band-match list, still undecided to the host list (binary128).
__global__ void k_brecheck(const uint2 *__restrict__ band, const uint32_t *__restrict__ n_band,
                           uint32_t cap, const double2 *__restrict__ arad,
                           const uint32_t *__restrict__ aidx, const uint32_t *__restrict__ ajob,
                           const BJob *__restrict__ jobs, const double2 *__restrict__ coordB,
                           BRows brows, uint4 *__restrict__ bin,
                           uint32_t *__restrict__ n_bin, uint32_t bin_cap,
                           BAmb *__restrict__ hl, uint32_t *__restrict__ n_hl, uint32_t hl_cap,
                           uint32_t *__restrict__ flags)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= min(*n_band, cap)) return;
    const uint2 q = band[t];
    const double2 ad = arad[q.x];
    const uint32_t idxB = brows(q.y);
    const double2 rb = coordB[idxB];
    const BJob &jb = jobs[ajob[q.x]];
    ARec a;
    a.ra = ad.x;
    a.dec = ad.y;
    unit_vec(a.ra, a.dec, a.x, a.y, a.z);
    a.cosd = cos_dec_acc(a.dec);
    a.reach_deg = 0.0;
    a.idx = aidx[q.x];
    a.pad = 0;
    const int d = recheck_circle(a, rb, jb.h_r);
    if (d == IN) {
        const uint32_t s = atomicAdd(n_bin, 1u);
        if (s < bin_cap) bin[s] = make_uint4(q.x, a.idx, idxB, q.y);
        else atomicOr(flags, kBFlagCap);
    } else if (d == AMBIG) {
        const uint32_t s = atomicAdd(n_hl, 1u);
        if (s < hl_cap) {
            BAmb h;
            h.raA = ad.x;
            h.decA = ad.y;
            h.raB = rb.x;
            h.decB = rb.y;
            h.r_arcsec = jb.r_arcsec;
            h.i = q.x;
            h.j = q.y;
            h.idxA = a.idx;
            h.idxB = idxB;
            hl[s] = h;
        } else {
            atomicOr(flags, kBFlagCap);
        }
    }
}

// Host decisions back on the device: the undecided candidates the host found
// inside join the band-match list.
__global__ void k_bapply(const BAmb *__restrict__ hl, const uint32_t *__restrict__ n_hl,
                         uint32_t hl_cap, const uint8_t *__restrict__ hin, uint4 *__restrict__ bin,
                         uint32_t *__restrict__ n_bin, uint32_t bin_cap,
                         uint32_t *__restrict__ flags)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= min(*n_hl, hl_cap) || !hin[t]) return;
    const BAmb h = hl[t];
    const uint32_t s = atomicAdd(n_bin, 1u);
    if (s < bin_cap) bin[s] = make_uint4(h.i, h.idxA, h.idxB, h.j);
    else atomicOr(flags, kBFlagCap);
}

// Band matches: counted in their row's record, and listed as the k-th
// match of their row.
__global__ void k_badd(const uint4 *__restrict__ bin, const uint32_t *__restrict__ n_bin,
                       uint32_t cap, RowRec *rec, WEnt *__restrict__ out)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= min(*n_bin, cap)) return;
    const uint4 q = bin[t];
    const uint32_t k = atomicAdd(&rec[q.y].n, 1u) & kCountMask;
    out[t] = WEnt{q.x, k, q.z, q.w};
}

// Rows to re-rank: near-tie rows of the count pass, then rows with a band
// match.
__global__ void k_brows(const uint2 *__restrict__ tie, const uint32_t *__restrict__ n_tie,
                        uint32_t tie_cap, const uint4 *__restrict__ bin,
                        const uint32_t *__restrict__ n_bin, uint32_t bin_cap,
                        uint32_t *__restrict__ pos, uint32_t *__restrict__ n_pos)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nt = min(*n_tie, tie_cap), nb = min(*n_bin, bin_cap);
    if (t < nt) pos[t] = tie[t].x;
    else if (t < nt + nb) pos[t] = bin[t - nt].x;
    if (t == 0) *n_pos = nt + nb;
}

// Pair and best outputs in job-local rows.
__global__ void k_blocal_pairs(const BJob *__restrict__ jobs, const uint32_t *__restrict__ ejobA,
                               const int64_t *__restrict__ P, int64_t cap, int64_t nA,
                               int32_t *__restrict__ ia, int32_t *__restrict__ ib)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= min(*P, cap)) return;
    const uint32_t a = (uint32_t)ia[p];
    // the slots of rows above 2048 matches are written after the graph (and
    // renumbered then): whatever they hold now is skipped
    if (a >= (uint64_t)nA) return;
    const BJob &jb = jobs[ejobA[a]];
    ia[p] = (int32_t)(a - jb.a_ent);
    ib[p] = (int32_t)((uint32_t)ib[p] - jb.b_ent);
}

__global__ void k_blocal_best(const BJob *__restrict__ jobs, const uint32_t *__restrict__ ejobA,
                              int64_t n, int32_t *__restrict__ best)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n || best[a] < 0) return;
    const BJob &jb = jobs[ejobA[a]];
    best[a] = (int32_t)((uint32_t)best[a] - jb.b_ent);
}

// Job-local rows of the pairs of rows listed in `rows` (ordered after the
// graph, by finish_huge): one workgroup per row, grid-stride.
__global__ void k_blocal_rows(const uint32_t *__restrict__ rows, uint32_t n,
                              const int64_t *__restrict__ off, const BJob *__restrict__ jobs,
                              const uint32_t *__restrict__ ejobA, int64_t nA,
                              int32_t *__restrict__ ia, int32_t *__restrict__ ib)
{
    for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
        const uint32_t a = rows[r];
        if (a >= (uint64_t)nA) continue;
        const BJob &jb = jobs[ejobA[a]];
        for (int64_t q = off[a] + threadIdx.x; q < off[a + 1]; q += blockDim.x) {
            ia[q] = (int32_t)(a - jb.a_ent);
            ib[q] = (int32_t)((uint32_t)ib[q] - jb.b_ent);
        }
    }
}

// New best of a row the host ranked: job-local index and separation.
__global__ void k_bpatch(const uint32_t *__restrict__ pos, const uint32_t *__restrict__ bj,
                         uint32_t n, const uint32_t *__restrict__ aidx,
                         const double2 *__restrict__ arad, const double2 *__restrict__ coordB,
                         BRows brows, const BJob *__restrict__ jobs,
                         const uint32_t *__restrict__ ajob, int32_t *__restrict__ best,
                         double *__restrict__ bsep)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t i = pos[t], j = bj[t];
    const uint32_t a = aidx[i];
    const BJob &jb = jobs[ajob[i]];
    const uint32_t e = brows(j);
    best[a] = (int32_t)(e - jb.b_ent);
    const double2 ra = arad[i], rb = coordB[e];
    bsep[a] = sep_arcsec_rd(ra.x, ra.y, rb.x, rb.y);
}

// Pair offset of each job: off at the job's first A entry.
__global__ void k_bjob_off(const BJob *__restrict__ jobs, int nj, const int64_t *__restrict__ off,
                           int64_t nA, int64_t *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nj) out[t] = off[jobs[t].a_ent];
    if (t == nj) out[t] = off[nA];
}

}  // namespace c3x

// ---------------------------------------------------------------------------- host side

using namespace c3x;

struct c3x_batch {
    int device = 0;
    c3x_precision prec = C3X_FP64;
    int32_t nj = 0;
    int64_t NA = 0, NB = 0;
    const double *raA = nullptr, *decA = nullptr, *raB = nullptr, *decB = nullptr;
    std::vector<c3x_job> jobs;
    std::vector<BJob> hjobs;
    hipStream_t s = nullptr;
    Arena mem;
    // job table
    BJob *djobs = nullptr;
    uint32_t *prefA = nullptr, *prefB = nullptr;
    uint32_t *ejobA = nullptr, *ejobB = nullptr;  // job of each entry (and sorted position)
    // B index
    uint32_t *bk = nullptr, *bv = nullptr, *bk2 = nullptr, *bv2 = nullptr;
    void *bws = nullptr;
    Pay64 *p64 = nullptr;
    Pay32 *p32 = nullptr;
    double2 *coordB = nullptr;  // B coordinates in entry order (packB)
    double2 *packA = nullptr, *packB = nullptr;  // entry-order coordinates
    uint32_t *dir = nullptr;
    uint3 *gaps = nullptr;  // directory gaps longer than kDirGap buckets
    uint32_t *n_gaps = nullptr, gap_cap = 0, big_cap = 0;
    int key_bits = 32;
    Grid g{};
    // A
    uint32_t *ak = nullptr, *av = nullptr, *ak2 = nullptr, *av2 = nullptr;
    void *aws = nullptr;
    double2 *arad = nullptr;
    uint32_t *aidx = nullptr, *ajob = nullptr;
    ARange *arng = nullptr;
    RowRec *rec = nullptr;
    int32_t *best2 = nullptr;
    // lists
    uint2 *amb = nullptr, *tie = nullptr;
    uint32_t amb_cap = 0, tie_cap = 0;
    OvEnt *ovl = nullptr;
    uint32_t *octr = nullptr, ov_pool = 0;
    uint4 *bin = nullptr;
    uint32_t bin_cap = 0;
    BAmb *hl = nullptr;
    uint32_t hl_cap = 0;
    WEnt *xent = nullptr;
    uint32_t *pos = nullptr, *unc = nullptr;
    // host decisions: pinned mirrors and device copies
    BAmb *h_hl = nullptr;
    uint32_t *h_cnt = nullptr;     // [1] undecided count
    uint8_t *h_in = nullptr;       // [hl_cap]
    unsigned long long *h_vk = nullptr;
    uint8_t *h_vi = nullptr;
    uint32_t *h_nv = nullptr;      // [1]
    uint8_t *d_hin = nullptr, *d_vi = nullptr;
    unsigned long long *d_vk = nullptr;
    uint32_t *d_nv = nullptr;
    // counters: 0 flags, 1 amb_n, 2 tie_n, 3 unc_n, 4 err, 5 ov_flag, 6-7 seg_n,
    // 8 n_bin, 9 n_hl, 10 n_pos, 11 bad job, 12 collect count, 13 sort give-up
    uint32_t *ctr = nullptr;
    unsigned long long *c64 = nullptr;  // statistics copies (tests, band, placed)
    // outputs
    int64_t *off = nullptr;
    void *sws = nullptr;
    PairTmp *pt = nullptr;
    int64_t P_cap = 0, P = 0;
    int32_t *oa = nullptr, *ob = nullptr, *obest = nullptr;
    double *os = nullptr, *obsep = nullptr;
    uint32_t *seg_list = nullptr, *seg_huge = nullptr, seg_cap = 0;
    int64_t *joboff = nullptr;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool ran = false;
    // large sorts may take the one-sweep schedule; cleared for good once a
    // look-back gave up (the graph is then captured again without it)
    bool onesweep = true;
    c3x_stats stats{};
    double cell_scale = 1.0;       // the scale the autotuner set for every class first
    // per density class of job (by its B rows, see job_class): the cell
    // scale, and the count kernel's tile (A sources per workgroup)
    double kappa_class[4] = {1.0, 1.0, 1.0, 1.0};
    int tile = 256;
    // count pass as a persistent kernel taking tiles costliest first (else
    // one workgroup per tile, in order); its tile cost keys, order, counter
    bool queue = false;
    unsigned queue_blocks = 0;     // workgroups of the persistent kernel
    uint32_t *qk = nullptr, *qv = nullptr, *qk2 = nullptr, *qv2 = nullptr, *qctr = nullptr;
    float *jcost = nullptr;
    void *qws = nullptr;
    std::vector<int64_t> hjoboff;

    ~c3x_batch()
    {
        if (s) (void)hipStreamSynchronize(s);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (h_hl) (void)hipHostFree(h_hl);
        if (h_cnt) (void)hipHostFree(h_cnt);
        if (h_in) (void)hipHostFree(h_in);
        if (h_vk) (void)hipHostFree(h_vk);
        if (h_vi) (void)hipHostFree(h_vi);
        if (h_nv) (void)hipHostFree(h_nv);
        mem.release_all();
        if (s) (void)hipStreamDestroy(s);
    }
};

namespace c3x {

// Host node: binary128 decisions of the candidates the FP64 recheck left
// open, and the sorted verdict table the re-ranking kernels consult.
static void batch_host_decide(void *arg)
{
    c3x_batch *b = (c3x_batch *)arg;
    const uint32_t n = std::min(*b->h_cnt, b->hl_cap);
    std::vector<std::pair<unsigned long long, uint8_t>> v(n);
    for (uint32_t t = 0; t < n; ++t) {
        const BAmb &h = b->h_hl[t];
        const int in = c3x_q_circle(h.raA, h.decA, h.raB, h.decB, h.r_arcsec);
        b->h_in[t] = (uint8_t)(in ? 1 : 0);
        v[t] = {((unsigned long long)h.i << 32) | h.j, (uint8_t)(in ? 1 : 0)};
    }
    std::sort(v.begin(), v.end());
    for (uint32_t t = 0; t < n; ++t) {
        b->h_vk[t] = v[t].first;
        b->h_vi[t] = v[t].second;
    }
    *b->h_nv = n;
}

static MatchArgs batch_args(c3x_batch *b)
{
    MatchArgs m;
    memset(&m, 0, sizeof(m));
    m.g = b->g;
    m.pay64 = b->p64;
    m.pay32 = b->p32;
    m.coordB = b->coordB;
    m.arad = b->arad;
    m.aidx = b->aidx;
    m.arng = b->arng;
    m.jobs = b->djobs;
    m.ajob = b->ajob;
    m.nA = (int32_t)b->NA;
    m.best2 = b->best2;
    m.rec_zeroed = 1;  // cleared by a fill kernel before the count pass
    m.best_only = 0;
    m.rec = b->rec;
    m.amb_n = b->ctr + 1;
    m.amb = b->amb;
    m.amb_cap = b->amb_cap;
    m.tie_n = b->ctr + 2;
    m.tie = b->tie;
    m.tie_cap = b->tie_cap;
    m.ver_key = b->d_vk;
    m.ver_in = b->d_vi;
    m.n_ver = b->hl_cap;
    m.n_ver_dev = b->d_nv;
    m.ovl = b->ovl;
    m.octr = b->octr;
    m.ov_pool = b->ov_pool;
    m.ov_flag = b->ctr + 5;
    m.n_placed = b->c64 + 2;
    m.n_tests = b->c64;
    m.n_band = b->c64 + 1;
    m.err_flag = b->ctr + 4;
    return m;
}

// Index and count half of the pipeline: everything up to the scan of the
// per-row counts (off[NA] = P). Stream-ordered, no host synchronisation.
static hipError_t batch_front(c3x_batch *b)
{
    hipStream_t s = b->s;
    const int nj = b->nj;
    hipLaunchKernelGGL(k_bfill, dim3(1), dim3(64), 0, s, b->ctr, (int64_t)16, 0u);
    hipLaunchKernelGGL(k_bfill64, dim3(kStatSlots * kStatStride / 64), dim3(64), 0, s, b->c64,
                       (int64_t)kStatSlots * kStatStride);
    hipLaunchKernelGGL(k_bfill, dim3(nblk(kEmitPools * kEmitPoolStride, 256)), dim3(256), 0, s,
                       b->octr, (int64_t)kEmitPools * kEmitPoolStride, 0u);
    // B: keys, sort, payloads, directory
    const int64_t NB = b->NB, NA = b->NA;
    if (NB > 0)
        hipLaunchKernelGGL(k_bkeys, dim3(nblk(NB, 256)), dim3(256), 0, s, b->djobs, b->ejobB,
                           b->raB, b->decB, NB, true, b->bk, b->packB, b->ctr);
    int in_tmp = 0;
    uint32_t *sort_fail = b->onesweep ? b->ctr + 13 : nullptr;
    hipError_t e = radix_sort_pairs(b->bk, b->bv, b->bk2, b->bv2, NB, b->key_bits, b->bws, s,
                                    &in_tmp, /*vals_are_index=*/true, sort_fail);
    if (e != hipSuccess) return e;
    const uint32_t *skeys = in_tmp ? b->bk2 : b->bk;
    const uint32_t *srows = in_tmp ? b->bv2 : b->bv;
    b->g.keys = skeys;
    if (NB > 0)
        hipLaunchKernelGGL(k_bgather_b, dim3(nblk(NB, 256)), dim3(256), 0, s, srows, b->djobs,
                           b->ejobB, b->packB, NB, b->p64, b->p32);
    // the directory straight from the sorted keys (the gap counter cleared by
    // a kernel: this runs inside the graph)
    hipLaunchKernelGGL(k_bfill, dim3(1), dim3(64), 0, s, b->n_gaps, (int64_t)2, 0u);
    hipLaunchKernelGGL(k_dir_fill, dim3(nblk(NB + 1, 256)), dim3(256), 0, s, skeys, NB,
                       b->g.dshift, b->g.dsize, b->dir, b->gaps, b->n_gaps, b->gap_cap,
                       b->big_cap);
    hipLaunchKernelGGL(k_dir_fill_gaps, dim3(4096), dim3(256), 0, s, b->gaps, b->n_gaps,
                       b->gap_cap, b->big_cap, b->dir);
    // A: keys, sort, records and candidate ranges
    if (NA > 0)
        hipLaunchKernelGGL(k_bkeys, dim3(nblk(NA, 256)), dim3(256), 0, s, b->djobs, b->ejobA,
                           b->raA, b->decA, NA, false, b->ak, b->packA, b->ctr);
    // A in the order of its top key bits (its order changes no result)
    // (a job's entries stay together: keys are job-major and the sort stable)
    const int a_lo = std::max(0, b->key_bits - kAKeyBits);
    e = radix_sort_pairs_bits(b->ak, b->av, b->ak2, b->av2, NA, a_lo, b->key_bits, b->aws, s,
                              &in_tmp, /*vals_are_index=*/true, sort_fail);
    if (e != hipSuccess) return e;
    const uint32_t *arows = in_tmp ? b->av2 : b->av;
    if (NA > 0)
        hipLaunchKernelGGL(k_bgather_a, dim3(nblk(NA, 256)), dim3(256), 0, s, arows, b->djobs,
                           b->ejobA, b->packA, NA, b->g, b->arad, b->aidx, b->ajob, b->arng);
    // count + emit
    MatchArgs m = batch_args(b);
    const unsigned grid = nblk(NA, b->tile);
    if (grid && b->queue) {
        // tiles of the costliest jobs first (a job's cost: the candidates of
        // its rows), each job's tiles together and in order, taken from a
        // counter by a persistent grid
        hipLaunchKernelGGL(k_bfill, dim3(nblk(NA * kRecWords, 256)), dim3(256), 0, s,
                           (uint32_t *)b->rec, NA * kRecWords, 0u);
        hipLaunchKernelGGL(k_job_cost, dim3(std::min(nj, 4096)), dim3(256), 0, s, b->djobs, nj,
                           b->arng, b->jcost);
        hipLaunchKernelGGL(k_tile_cost, dim3(nblk(grid, 256)), dim3(256), 0, s, b->ajob, b->jcost,
                           NA, (uint32_t)b->tile, grid, b->qk, b->qv);
        int qin = 0;
        e = radix_sort_pairs(b->qk, b->qv, b->qk2, b->qv2, grid, 16, b->qws, s, &qin, false,
                             nullptr);
        if (e != hipSuccess) return e;
        const uint32_t *order = qin ? b->qv2 : b->qv;
        hipLaunchKernelGGL(k_bfill, dim3(1), dim3(64), 0, s, b->qctr, (int64_t)1, 0u);
        const unsigned pg = std::max(1u, std::min(grid, b->queue_blocks));
        // about eight takes per workgroup: few atomics on the one counter,
        // and the last chunks still short
        const uint32_t chunk = std::max(1u, grid / (8u * pg));
        if (b->prec == C3X_FP64)
            hipLaunchKernelGGL(k_match_queue<C3X_FP64>, dim3(pg), dim3(b->tile), 0, s, m, order,
                               grid, chunk, b->qctr);
        else
            hipLaunchKernelGGL(k_match_queue<C3X_MIXED>, dim3(pg), dim3(b->tile), 0, s, m, order,
                               grid, chunk, b->qctr);
    } else if (grid) {
        hipLaunchKernelGGL(k_bfill, dim3(nblk(NA * kRecWords, 256)), dim3(256), 0, s,
                           (uint32_t *)b->rec, NA * kRecWords, 0u);
        if (b->prec == C3X_FP64)
            hipLaunchKernelGGL((k_match<C3X_CIRCLE, C3X_FP64, 2, true>), dim3(grid),
                               dim3(b->tile), 0, s, m);
        else
            hipLaunchKernelGGL((k_match<C3X_CIRCLE, C3X_MIXED, 2, true>), dim3(grid),
                               dim3(b->tile), 0, s, m);
    }
    // band candidates: FP64 recheck, then the host decides what is left
    hipLaunchKernelGGL(k_brecheck, dim3(nblk(b->amb_cap, 256)), dim3(256), 0, s, b->amb,
                       b->ctr + 1, b->amb_cap, b->arad, b->aidx, b->ajob, b->djobs, b->coordB,
                       BRows{b->p64, b->p32}, b->bin, b->ctr + 8, b->bin_cap, b->hl, b->ctr + 9,
                       b->hl_cap,
                       b->ctr);
    e = hipMemcpyAsync(b->h_cnt, b->ctr + 9, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_hl, b->hl, b->hl_cap * sizeof(BAmb), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipLaunchHostFunc(s, batch_host_decide, b);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_hin, b->h_in, b->hl_cap, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_vk, b->h_vk, b->hl_cap * sizeof(unsigned long long),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_vi, b->h_vi, b->hl_cap, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_nv, b->h_nv, sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bapply, dim3(nblk(b->hl_cap, 256)), dim3(256), 0, s, b->hl, b->ctr + 9,
                       b->hl_cap, b->d_hin, b->bin, b->ctr + 8, b->bin_cap, b->ctr);
    hipLaunchKernelGGL(k_badd, dim3(nblk(b->bin_cap, 256)), dim3(256), 0, s, b->bin, b->ctr + 8,
                       b->bin_cap, b->rec, b->xent);
    // best matches the filter cannot rank: FP64 on the GPU; what FP64 cannot
    // separate is listed (c3x_batch_result ranks it in binary128)
    const uint32_t npos = b->tie_cap + b->bin_cap;
    const unsigned rr_grid = std::min<uint32_t>(npos, 8192u);
    hipLaunchKernelGGL(k_brows, dim3(nblk(npos, 256)), dim3(256), 0, s, b->tie, b->ctr + 2,
                       b->tie_cap, b->bin, b->ctr + 8, b->bin_cap, b->pos, b->ctr + 10);
    if (b->prec == C3X_FP64)
        hipLaunchKernelGGL((k_rerank<C3X_CIRCLE, C3X_FP64, true>), dim3(rr_grid), dim3(64), 0, s, m,
                           b->pos, npos, b->ctr + 10, b->ctr + 3, b->unc);
    else
        hipLaunchKernelGGL((k_rerank<C3X_CIRCLE, C3X_MIXED, true>), dim3(rr_grid), dim3(64), 0, s, m,
                           b->pos, npos, b->ctr + 10, b->ctr + 3, b->unc);
    // counts -> offsets (off[NA] = P)
    if (NA > 0) {
        e = scan_u32_to_i64(&b->rec->n, kRecWords, kCountMask, b->off, NA, b->off + NA, b->sws,
                            s);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_bfill64, dim3(1), dim3(64), 0, s, (unsigned long long *)b->off,
                           (int64_t)1);
    }
    return hipGetLastError();
}

// What the finishing kernels need, for the batch's buffers.
static FinishArgs batch_fin_args(c3x_batch *b)
{
    FinishArgs fa{};
    fa.nA = b->NA;
    fa.nB = b->NB;
    fa.pcap = b->P_cap;
    fa.off = b->off;
    fa.rec = b->rec;
    fa.best2 = b->best2;
    fa.use_rec = 1;
    fa.defer = b->prec == C3X_MIXED ? 1 : 0;
    fa.tmp = b->pt;
    fa.coordA = b->packA;  // A coordinates in entry order
    fa.coordB = b->coordB;
    fa.best_idx = b->obest;
    fa.oa = b->oa;
    fa.ob = b->ob;
    fa.os = b->os;
    fa.bsep = b->obsep;
    fa.err = b->ctr + 4;
    fa.open_flag = b->ctr + 14;
    fa.sort_fail = nullptr;  // rows above 2048 matches: table-schedule sorts
    fa.seg_n = b->ctr + 6;
    fa.cap = b->seg_cap;
    fa.list = b->seg_list;
    fa.huge = b->seg_huge;
    return fa;
}

// Placement and output half (capacity P_cap).
static hipError_t batch_back(c3x_batch *b)
{
    hipStream_t s = b->s;
    const int64_t NA = b->NA;
    if (b->ov_pool)
        hipLaunchKernelGGL(k_place_ov, dim3(nblk(b->ov_pool, 256), kEmitPools), dim3(256), 0, s,
                           b->ovl, b->ov_pool, b->octr, NA, b->off, b->P_cap, b->pt, b->c64 + 2,
                           b->ctr + 4);
    hipLaunchKernelGGL(k_place_x, dim3(nblk(b->bin_cap, 256)), dim3(256), 0, s, b->xent,
                       b->bin_cap, b->ctr + 8, b->aidx, b->arad, b->coordB, NA, b->NB,
                       b->off,
                       b->P_cap, b->rec, 1, b->pt, b->c64 + 2, b->ctr + 4);
    const FinishArgs fa = batch_fin_args(b);
    finish_segments(fa, s);
    hipLaunchKernelGGL(k_blocal_pairs, dim3(nblk(std::max<int64_t>(b->P_cap, 1), 256)), dim3(256),
                       0, s, b->djobs, b->ejobA, b->off + NA, b->P_cap, NA, b->oa, b->ob);
    hipLaunchKernelGGL(k_blocal_best, dim3(nblk(std::max<int64_t>(NA, 1), 256)), dim3(256), 0, s,
                       b->djobs, b->ejobA, NA, b->obest);
    hipLaunchKernelGGL(k_bjob_off, dim3(nblk(b->nj + 1, 256)), dim3(256), 0, s, b->djobs, b->nj,
                       b->off, NA, b->joboff);
    return hipGetLastError();
}

// Density class of a job, by its number of B rows: below 4k, 40k, 400k,
// and above (the autotuner picks a cell scale per class).
static inline int job_class(uint32_t nB)
{
    return nB < 4000u ? 0 : (nB < 40000u ? 1 : (nB < 400000u ? 2 : 3));
}

// Grids of every job for the cell scale of its class (tangent-plane
// units): the cell side is kappa times the mean spacing of the job's B
// sources, at least the window half-width (so a window spans at most three
// rows) and at least 1e-4 arcsec; all cells must fit 32-bit keys. kappa > 0
// sets every class to it first.
static c3x_status batch_grids(c3x_batch *b, double kappa_all)
{
    if (kappa_all > 0.0)
        for (double &k : b->kappa_class) k = kappa_all;
    uint64_t base = 0;
    for (int j = 0; j < b->nj; ++j) {
        BJob &jb = b->hjobs[j];
        const double kappa = b->kappa_class[job_class(jb.nB)];
        const double T = jb.T;  // box half-side, set by the plan
        const double area = 4.0 * T * T;
        const double spacing = sqrt(area / (double)std::max<uint32_t>(jb.nB, 1u));
        double h = std::max(kappa * spacing, jb.wd * (1.0 + 1e-6) + 1e-12);
        h = std::max(h, 1e-4 / 3600.0 * kDeg);
        double nr = ceil(2.0 * T / h), nc = nr;
        // keep each job's grid modest: at most ~4 cells per B source + 1024
        const double lim = 4.0 * (double)jb.nB + 1024.0;
        while (nr * nc > lim && h < T) {
            h *= 1.25;
            nr = ceil(2.0 * T / h);
            nc = nr;
        }
        jb.h = h;
        jb.inv_h = 1.0 / h;
        jb.nrow = (uint32_t)std::max(1.0, nr);
        jb.ncol = (uint32_t)std::max(1.0, nc);
        jb.key_base = (uint32_t)std::min<uint64_t>(base, 0xffffffffull);
        base += (uint64_t)jb.nrow * jb.ncol;
    }
    if (base >= 0xffffffffull) return fail(C3X_ERANGE, "batch grids need more than 2^32 cells");
    uint64_t maxkey = base ? base - 1 : 0;
    int bits = 0;
    while (bits < 32 && (maxkey >> bits)) ++bits;
    b->key_bits = std::max(bits, 1);
    uint64_t want = std::max<uint64_t>(1024, (uint64_t)b->NB * 2);
    int sh = 0;
    while (sh < 31 && (maxkey >> sh) + 1 > want) ++sh;
    b->g.dshift = sh;
    b->g.dsize = (uint32_t)((maxkey >> sh) + 2);
    b->g.nB = (int32_t)b->NB;
    if (kappa_all > 0.0) b->cell_scale = kappa_all;
    hipError_t e = hipMemcpyAsync(b->djobs, b->hjobs.data(), b->nj * sizeof(BJob),
                                  hipMemcpyHostToDevice, b->s);
    if (e != hipSuccess) return fail_hip(e, "batch job table");
    return C3X_OK;
}

}  // namespace c3x

// Workgroups of the persistent count kernel: as many as fit on the device
// at once for the current tile.
static c3x_status set_queue_blocks(c3x_batch *b)
{
    int dev = 0, ncu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) {
        if (b->prec == C3X_FP64)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_match_queue<C3X_FP64>,
                                                             b->tile, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_match_queue<C3X_MIXED>,
                                                             b->tile, 0);
    }
    if (e != hipSuccess) return fail_hip(e, "persistent count kernel occupancy");
    b->queue_blocks = (unsigned)std::max(1, ncu) * (unsigned)std::max(1, per);
    return C3X_OK;
}

#define BCHK(expr, what)                                   \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return fail_hip(e_, what);   \
    } while (0)

// Runs the front half and grows every list that overflowed, until none does.
static c3x_status batch_size_lists(c3x_batch *b)
{
    hipStream_t s = b->s;
    auto &M = b->mem;
    for (int attempt = 0;; ++attempt) {
        BCHK(batch_front(b), "batch pipeline");
        uint32_t hc[16];
        std::vector<uint32_t> oc(kEmitPools * kEmitPoolStride);
        BCHK(hipMemcpyAsync(hc, b->ctr, sizeof(hc), hipMemcpyDeviceToHost, s), "copy");
        BCHK(hipMemcpyAsync(oc.data(), b->octr, oc.size() * 4, hipMemcpyDeviceToHost, s), "copy");
        BCHK(hipStreamSynchronize(s), "batch pipeline");
        if (hc[13]) return kSortGaveUp;
        uint32_t ov_need = 0;
        for (int q = 0; q < kEmitPools; ++q) ov_need = std::max(ov_need, oc[q * kEmitPoolStride]);
        const bool grow_amb = hc[1] > b->amb_cap, grow_tie = hc[2] > b->tie_cap;
        const bool grow_bin = hc[8] > b->bin_cap, grow_hl = hc[9] > b->hl_cap;
        const bool grow_ov = ov_need > b->ov_pool;
        if (!(grow_amb || grow_tie || grow_bin || grow_hl || grow_ov)) break;
        if (attempt >= 3) return fail(C3X_ENOMEM, "batch lists keep growing");
        if (grow_amb) {
            b->amb_cap = hc[1] + hc[1] / 8 + 1024;
            b->amb = M.get_n<uint2>(b->amb_cap);
        }
        if (grow_tie) {
            b->tie_cap = hc[2] + hc[2] / 8 + 1024;
            b->tie = M.get_n<uint2>(b->tie_cap);
        }
        if (grow_bin || grow_amb) {
            b->bin_cap = std::max(b->amb_cap, hc[8] + hc[8] / 8 + 1024);
            b->bin = M.get_n<uint4>(b->bin_cap);
            b->xent = M.get_n<WEnt>(b->bin_cap);
        }
        if (grow_hl) return fail(C3X_ENOMEM, "more than %u candidates need binary128 in one "
                                             "batch", b->hl_cap);
        if (grow_ov) {
            b->ov_pool = ov_need + ov_need / 8 + 4096;
            b->ovl = M.get_n<OvEnt>((int64_t)b->ov_pool * kEmitPools);
        }
        b->pos = M.get_n<uint32_t>((int64_t)b->tie_cap + b->bin_cap);
        b->unc = M.get_n<uint32_t>((int64_t)b->tie_cap + b->bin_cap);
        if (!b->amb || !b->tie || !b->bin || !b->xent || !b->ovl || !b->pos || !b->unc)
            return fail(C3X_ENOMEM, "batch lists");
    }
    return C3X_OK;
}

// The whole pipeline as one graph (replacing any earlier capture).
static c3x_status batch_capture(c3x_batch *b)
{
    hipStream_t s = b->s;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    BCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture");
    hipError_t e = batch_front(b);
    if (e == hipSuccess) e = batch_back(b);
    hipGraph_t gr = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &gr);
    if (e != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return fail_hip(e, "graph capture");
    }
    if (e2 != hipSuccess) return fail_hip(e2, "graph capture");
    b->graph = gr;
    BCHK(hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0), "graph instantiate");
    return C3X_OK;
}

static c3x_status batch_plan_impl(c3x_batch *b)
{
    hipStream_t s = b->s;
    const int nj = b->nj;
    const int64_t NA = b->NA, NB = b->NB;
    Arena tmp(s);
    // job table and entry prefixes
    std::vector<uint32_t> pa(nj + 1), pb(nj + 1);
    b->hjobs.assign(nj, BJob{});
    for (int j = 0; j < nj; ++j) {
        const c3x_job &q = b->jobs[j];
        pa[j + 1] = pa[j] + (uint32_t)q.nA;
        pb[j + 1] = pb[j] + (uint32_t)q.nB;
        BJob &jb = b->hjobs[j];
        jb.a_off = q.a_off;
        jb.b_off = q.b_off;
        jb.a_ent = pa[j];
        jb.b_ent = pb[j];
        jb.nA = (uint32_t)q.nA;
        jb.nB = (uint32_t)q.nB;
        jb.cx = 1.0;
        jb.ey = 1.0;
        jb.nz = 1.0;
    }
    b->djobs = b->mem.get_n<BJob>(nj);
    b->prefA = b->mem.get_n<uint32_t>(nj + 1);
    b->prefB = b->mem.get_n<uint32_t>(nj + 1);
    double *sums = tmp.get_n<double>(3 * nj);
    unsigned long long *ext = tmp.get_n<unsigned long long>(nj);
    uint32_t *bad = tmp.get_n<uint32_t>(1);
    if (!b->djobs || !b->prefA || !b->prefB || !sums || !ext || !bad)
        return fail(C3X_ENOMEM, "batch plan buffers");
    BCHK(hipMemcpyAsync(b->prefA, pa.data(), (nj + 1) * 4, hipMemcpyHostToDevice, s), "copy");
    BCHK(hipMemcpyAsync(b->prefB, pb.data(), (nj + 1) * 4, hipMemcpyHostToDevice, s), "copy");
    b->ejobA = b->mem.get_n<uint32_t>(std::max<int64_t>(NA, 1));
    b->ejobB = b->mem.get_n<uint32_t>(std::max<int64_t>(NB, 1));
    if (!b->ejobA || !b->ejobB) return fail(C3X_ENOMEM, "batch job tables");
    if (NA > 0)
        hipLaunchKernelGGL(k_bjob_fill, dim3(nblk(NA, 256)), dim3(256), 0, s, b->prefA, nj, NA,
                           b->ejobA);
    if (NB > 0)
        hipLaunchKernelGGL(k_bjob_fill, dim3(nblk(NB, 256)), dim3(256), 0, s, b->prefB, nj, NB,
                           b->ejobB);
    BCHK(hipMemcpyAsync(b->djobs, b->hjobs.data(), nj * sizeof(BJob), hipMemcpyHostToDevice, s),
         "copy");
    BCHK(hipMemsetAsync(sums, 0, 3 * nj * sizeof(double), s), "memset");
    BCHK(hipMemsetAsync(ext, 0, nj * sizeof(unsigned long long), s), "memset");
    BCHK(hipMemsetAsync(bad, 0xff, 4, s), "memset");
    // mean direction of each job
    if (NA > 0)
        hipLaunchKernelGGL(k_bsum, dim3(nblk(NA, 256)), dim3(256), 0, s, b->djobs, b->prefA, nj,
                           b->raA, b->decA, NA, false, sums, bad);
    if (NB > 0)
        hipLaunchKernelGGL(k_bsum, dim3(nblk(NB, 256)), dim3(256), 0, s, b->djobs, b->prefB, nj,
                           b->raB, b->decB, NB, true, sums, bad);
    std::vector<double> hs(3 * nj);
    uint32_t hbad = 0;
    BCHK(hipMemcpyAsync(hs.data(), sums, 3 * nj * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    BCHK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s), "copy");
    BCHK(hipStreamSynchronize(s), "batch plan");
    if (hbad != 0xffffffffu)
        return fail(C3X_EINVAL, "batch job %u: a coordinate outside RA [0,360), |Dec| <= 90 or not "
                                "finite", hbad);
    for (int j = 0; j < nj; ++j) {
        BJob &jb = b->hjobs[j];
        double cx = hs[3 * j], cy = hs[3 * j + 1], cz = hs[3 * j + 2];
        double nrm = sqrt(cx * cx + cy * cy + cz * cz);
        if (!(nrm > 1e-9 * (double)std::max<uint32_t>(jb.nA + jb.nB, 1u))) {
            cx = 1.0;
            cy = 0.0;
            cz = 0.0;
            nrm = 1.0;
        }
        cx /= nrm;
        cy /= nrm;
        cz /= nrm;
        // east = z x c (x axis when c is a pole), north = c x east
        double ex = -cy, ey = cx, ez = 0.0;
        double en = sqrt(ex * ex + ey * ey);
        if (en < 1e-6) {
            ex = 0.0;
            ey = 1.0;
            ez = 0.0;
            en = 1.0;
        }
        ex /= en;
        ey /= en;
        const double nx = cy * ez - cz * ey, ny = cz * ex - cx * ez, nz = cx * ey - cy * ex;
        jb.cx = cx;
        jb.cy = cy;
        jb.cz = cz;
        jb.ex = ex;
        jb.ey = ey;
        jb.ez = ez;
        jb.nx = nx;
        jb.ny = ny;
        jb.nz = nz;
    }
    BCHK(hipMemcpyAsync(b->djobs, b->hjobs.data(), nj * sizeof(BJob), hipMemcpyHostToDevice, s),
         "copy");
    if (NA > 0)
        hipLaunchKernelGGL(k_bext, dim3(nblk(NA, 256)), dim3(256), 0, s, b->djobs, b->prefA, nj,
                           b->raA, b->decA, NA, false, ext);
    if (NB > 0)
        hipLaunchKernelGGL(k_bext, dim3(nblk(NB, 256)), dim3(256), 0, s, b->djobs, b->prefB, nj,
                           b->raB, b->decB, NB, true, ext);
    std::vector<unsigned long long> hx(nj);
    BCHK(hipMemcpyAsync(hx.data(), ext, nj * 8, hipMemcpyDeviceToHost, s), "copy");
    BCHK(hipStreamSynchronize(s), "batch plan");
    for (int j = 0; j < nj; ++j) {
        BJob &jb = b->hjobs[j];
        double D;
        memcpy(&D, &hx[j], 8);
        const double r = b->jobs[j].radius_arcsec;
        if (D > kMaxJobExtentDeg)
            return fail(C3X_EINVAL, "batch job %d: sources lie %.3g deg from their mean "
                                    "direction (at most %g deg in a batch; use c3x_match)",
                        j, D, kMaxJobExtentDeg);
        jb.reach_deg = r / 3600.0;
        jb.r_arcsec = r;
        // on the tangent plane: the box holds every source (angle <= D) with a
        // margin of two radii; the window half-width is the radius times the
        // largest stretch of the projection within angle D + radius
        // (sec^2), padded for rounding
        const double Dmax = (D * (1.0 + 1e-6) + jb.reach_deg * 2.0 + 1e-9) * kDeg;
        jb.T = tan(Dmax);
        const double cmax = cos(Dmax);
        jb.wd = jb.reach_deg * kDeg / (cmax * cmax) * (1.0 + 1e-9) + 1e-12;
        CircleThresholds t;
        jb.L = 2.0 * sin(0.5 * (D + 1e-6) * kDeg) + 1e-12;
        t = circle_thresholds(r, jb.L);
        jb.cr2 = t.cr2;
        jb.h_r = t.h_r;
        jb.t64_in = t.t64_in;
        jb.t64_out = t.t64_out;
        jb.t32_in = t.t32_in;
        jb.t32_out = t.t32_out;
        jb.r_zero = r == 0.0;
    }
    // buffers (sizes do not depend on the cell scale)
    auto &M = b->mem;
    b->bk = M.get_n<uint32_t>(NB);
    b->bv = M.get_n<uint32_t>(NB);
    b->bk2 = M.get_n<uint32_t>(NB);
    b->bv2 = M.get_n<uint32_t>(NB);
    b->bws = M.get(radix_ws_bytes(NB));
    // one payload: FP64 unit vectors, or FP32 offsets from the job centres
    if (b->prec == C3X_MIXED) b->p32 = M.get_n<Pay32>(NB);
    else b->p64 = M.get_n<Pay64>(NB);
    b->packB = M.get_n<double2>(std::max<int64_t>(NB, 1));
    b->coordB = b->packB;  // B coordinates in entry order, reached through the payload's row
    b->packA = M.get_n<double2>(std::max<int64_t>(NA, 1));
    const int64_t dmax = std::max<int64_t>(1024, 2 * NB) + 2;
    b->dir = M.get_n<uint32_t>(dmax);
    b->gap_cap = dir_gap_cap((uint32_t)dmax);
    b->big_cap = dir_big_cap((uint32_t)dmax);
    b->gaps = M.get_n<uint3>((int64_t)b->gap_cap + b->big_cap);
    b->n_gaps = M.get_n<uint32_t>(2);
    b->ak = M.get_n<uint32_t>(NA);
    b->av = M.get_n<uint32_t>(NA);
    b->ak2 = M.get_n<uint32_t>(NA);
    b->av2 = M.get_n<uint32_t>(NA);
    b->aws = M.get(radix_ws_bytes(NA));
    b->arad = M.get_n<double2>(NA);
    b->aidx = M.get_n<uint32_t>(NA);
    b->ajob = M.get_n<uint32_t>(NA);
    b->arng = M.get_n<ARange>(NA);
    b->rec = M.get_n<RowRec>(NA);
    b->best2 = M.get_n<int32_t>(NA);
    b->amb_cap = (uint32_t)std::min<int64_t>(NA / 16 + 4096, 1 << 26);
    b->tie_cap = (uint32_t)std::min<int64_t>(NA / 16 + 4096, 1 << 26);
    b->bin_cap = b->amb_cap;
    b->hl_cap = 4096;
    b->ov_pool = (uint32_t)std::max<int64_t>(NA / 8 / kEmitPools, 4096);
    b->amb = M.get_n<uint2>(b->amb_cap);
    b->tie = M.get_n<uint2>(b->tie_cap);
    b->ovl = M.get_n<OvEnt>((int64_t)b->ov_pool * kEmitPools);
    b->octr = M.get_n<uint32_t>(kEmitPools * kEmitPoolStride);
    b->bin = M.get_n<uint4>(b->bin_cap);
    b->hl = M.get_n<BAmb>(b->hl_cap);
    b->xent = M.get_n<WEnt>(b->bin_cap);
    b->pos = M.get_n<uint32_t>((int64_t)b->tie_cap + b->bin_cap);
    b->unc = M.get_n<uint32_t>((int64_t)b->tie_cap + b->bin_cap);
    b->d_hin = M.get_n<uint8_t>(b->hl_cap);
    b->d_vi = M.get_n<uint8_t>(b->hl_cap);
    b->d_vk = M.get_n<unsigned long long>(b->hl_cap);
    b->d_nv = M.get_n<uint32_t>(1);
    b->ctr = M.get_n<uint32_t>(16);
    b->c64 = M.get_n<unsigned long long>(kStatSlots * kStatStride);
    b->off = M.get_n<int64_t>(NA + 1);
    b->sws = M.get(scan_ws_bytes(NA + 1));
    b->seg_cap = (uint32_t)std::min<int64_t>(std::max<int64_t>(NA, 1), 1 << 22);
    b->seg_list = M.get_n<uint32_t>(b->seg_cap);
    b->seg_huge = M.get_n<uint32_t>(b->seg_cap);
    b->obest = M.get_n<int32_t>(NA);
    b->obsep = M.get_n<double>(NA);
    b->joboff = M.get_n<int64_t>(nj + 1);
    // the persistent count pass: tiles of at least 64 rows
    const int64_t qmax = (NA + 63) / 64 + 1;
    b->qk = M.get_n<uint32_t>(qmax);
    b->qv = M.get_n<uint32_t>(qmax);
    b->qk2 = M.get_n<uint32_t>(qmax);
    b->qv2 = M.get_n<uint32_t>(qmax);
    b->qws = M.get(radix_ws_bytes(qmax));
    b->qctr = M.get_n<uint32_t>(1);
    b->jcost = M.get_n<float>(std::max(nj, 1));
    bool ok = b->bk && b->bv && b->bk2 && b->bv2 && b->bws && (b->p64 || b->p32) &&
              b->qk && b->qv && b->qk2 && b->qv2 && b->qws && b->qctr && b->jcost &&
              b->coordB && b->packA && b->packB &&
              b->dir && b->gaps && b->n_gaps &&
              b->ak && b->av && b->ak2 && b->av2 && b->aws && b->arad && b->aidx && b->ajob &&
              b->arng && b->best2 && b->rec && b->amb && b->tie && b->ovl && b->octr && b->bin &&
              b->hl && b->xent && b->pos && b->unc && b->d_hin && b->d_vi && b->d_vk &&
              b->d_nv && b->ctr && b->c64 && b->off && b->sws && b->seg_list && b->seg_huge &&
              b->obest && b->obsep && b->joboff;
    if (!ok) return fail(C3X_ENOMEM, "batch buffers");
    BCHK(hipHostMalloc((void **)&b->h_hl, b->hl_cap * sizeof(BAmb)), "pinned buffers");
    BCHK(hipHostMalloc((void **)&b->h_cnt, sizeof(uint32_t)), "pinned buffers");
    BCHK(hipHostMalloc((void **)&b->h_in, b->hl_cap), "pinned buffers");
    BCHK(hipHostMalloc((void **)&b->h_vk, b->hl_cap * sizeof(unsigned long long)), "pinned buffers");
    BCHK(hipHostMalloc((void **)&b->h_vi, b->hl_cap), "pinned buffers");
    BCHK(hipHostMalloc((void **)&b->h_nv, sizeof(uint32_t)), "pinned buffers");
    b->g.dir = b->dir;
    b->g.nB = (int32_t)NB;

    // lists sized at the default cell scale first, so that the timed runs
    // below do not overflow them
    {
        c3x_status st = batch_grids(b, 1.0);
        if (st == C3X_OK) {
            st = batch_size_lists(b);
            if (st != C3X_OK) return st;
        }
        clear_error();
    }

    // autotuner: times the index + count half (the best of two runs of each
    // setting): first one cell scale for every job, then the count kernel's
    // tile, then each density class's own cell scale in turn. Settings only
    // change the speed, never the answer. C3X_BATCH_CELL_SCALE fixes one
    // scale for all classes, C3X_BATCH_CELL_SCALES "k0,k1,k2,k3" one per
    // class, C3X_BATCH_TILE the tile (64, 128 or 256).
    hipEvent_t e0, e1;
    BCHK(hipEventCreate(&e0), "events");
    BCHK(hipEventCreate(&e1), "events");
    auto timed = [&](double &ms) -> c3x_status {
        ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            BCHK(hipEventRecord(e0, s), "events");
            BCHK(batch_front(b), "batch pipeline");
            BCHK(hipEventRecord(e1, s), "events");
            BCHK(hipEventSynchronize(e1), "events");
            float t = 0.f;
            BCHK(hipEventElapsedTime(&t, e0, e1), "events");
            ms = std::min(ms, (double)t);
        }
        return C3X_OK;
    };
    const std::vector<double> scales = {0.5, 1.0, 2.0, 4.0};
    const char *fixed = getenv("C3X_BATCH_CELL_SCALE");
    const char *fixed_cls = getenv("C3X_BATCH_CELL_SCALES");
    const char *fixed_tile = getenv("C3X_BATCH_TILE");
    bool present[4] = {false, false, false, false};
    for (const BJob &jb : b->hjobs) present[job_class(jb.nB)] = true;
    double best_ms = 1e300;
    c3x_status st = C3X_OK;
    if (fixed_cls) {
        double k[4] = {1.0, 1.0, 1.0, 1.0};
        sscanf(fixed_cls, "%lf,%lf,%lf,%lf", &k[0], &k[1], &k[2], &k[3]);
        for (int c = 0; c < 4; ++c) b->kappa_class[c] = std::max(0.05, k[c]);
        st = batch_grids(b, 0.0);
        if (st != C3X_OK) return st;
    } else if (fixed) {
        st = batch_grids(b, std::max(0.05, atof(fixed)));
        if (st != C3X_OK) return st;
    } else {
        double best_k = 1.0;
        for (double k : scales) {
            if (batch_grids(b, k) != C3X_OK) continue;
            double ms;
            st = timed(ms);
            if (st != C3X_OK) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best_k = k;
            }
        }
        st = batch_grids(b, best_k);
        if (st != C3X_OK) return st;
    }
    if (fixed_tile) {
        const int t = atoi(fixed_tile);
        b->tile = (t == 64 || t == 128) ? t : 256;
    } else {
        int best_t = b->tile;
        double tms = 1e300;
        for (int t : {64, 128, 256}) {
            b->tile = t;
            double ms;
            st = timed(ms);
            if (st != C3X_OK) return st;
            if (ms < tms) {
                tms = ms;
                best_t = t;
            }
        }
        b->tile = best_t;
        best_ms = tms;
    }
    // the count pass's mapping: one workgroup per tile in order, or the
    // persistent kernel taking tiles costliest first (C3X_BATCH_QUEUE=0/1)
    st = set_queue_blocks(b);
    if (st != C3X_OK) return st;
    if (const char *q = getenv("C3X_BATCH_QUEUE")) {
        b->queue = atoi(q) != 0;
    } else {
        b->queue = false;
        double ms_grid, ms_queue;
        st = timed(ms_grid);
        if (st != C3X_OK) return st;
        b->queue = true;
        st = timed(ms_queue);
        if (st != C3X_OK) return st;
        b->queue = ms_queue < ms_grid;
        best_ms = std::min(ms_grid, ms_queue);
    }
    if (!fixed && !fixed_cls) {
        // each class's own scale, the others held (kept when 2% faster)
        for (int c = 0; c < 4; ++c) {
            if (!present[c]) continue;
            const double keep = b->kappa_class[c];
            double bk = keep, bms = best_ms;
            for (double k : scales) {
                if (k == keep) continue;
                b->kappa_class[c] = k;
                if (batch_grids(b, 0.0) != C3X_OK) continue;
                double ms;
                st = timed(ms);
                if (st != C3X_OK) return st;
                if (ms < bms * 0.98) {
                    bms = ms;
                    bk = k;
                }
            }
            b->kappa_class[c] = bk;
            best_ms = bms;
        }
        st = batch_grids(b, 0.0);
        if (st != C3X_OK) return st;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    clear_error();

    // first run: sizes the lists (grown and run again while one overflows)
    // and the outputs
    st = batch_size_lists(b);
    if (st != C3X_OK) return st;
    int64_t P = 0;
    BCHK(hipMemcpyAsync(&P, b->off + NA, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    BCHK(hipStreamSynchronize(s), "batch pipeline");
    b->P_cap = P;
    b->pt = M.get_n<PairTmp>(P);
    b->oa = M.get_n<int32_t>(P);
    b->ob = M.get_n<int32_t>(P);
    b->os = M.get_n<double>(P);
    if (!b->pt || !b->oa || !b->ob || !b->os) return fail(C3X_ENOMEM, "batch outputs");
    BCHK(batch_back(b), "batch pipeline");
    BCHK(hipStreamSynchronize(s), "batch pipeline");
    b->ran = true;

    return batch_capture(b);
}

// Reads the run's flags and counts; ranks on the host (binary128) the rows
// the FP64 re-ranking left open, and patches their best match.
static c3x_status batch_finish(c3x_batch *b)
{
    hipStream_t s = b->s;
    uint32_t hc[16];
    std::vector<unsigned long long> hs(kStatSlots * kStatStride);
    unsigned long long h64[3];
    int64_t P = 0;
    BCHK(hipMemcpyAsync(hc, b->ctr, sizeof(hc), hipMemcpyDeviceToHost, s), "copy");
    BCHK(hipMemcpyAsync(hs.data(), b->c64, hs.size() * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s), "copy");
    BCHK(hipMemcpyAsync(&P, b->off + b->NA, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    BCHK(hipStreamSynchronize(s), "batch result");
    stat_sums(hs.data(), h64);
    if (hc[13]) return kSortGaveUp;  // nothing of this run is used
    if (hc[0] & kBFlagStale)
        return fail(C3X_EINVAL, "batch inputs moved outside the planned sky boxes: plan again");
    if ((hc[0] & kBFlagCap) || hc[1] > b->amb_cap || hc[2] > b->tie_cap || hc[5] ||
        hc[9] > b->hl_cap || P != b->P_cap)
        return fail(C3X_EINVAL,
                    "batch inputs changed since the plan (pairs %lld of %lld planned; band list "
                    "%u of %u, tie list %u of %u, overflow %u): plan again",
                    (long long)P, (long long)b->P_cap, hc[1], b->amb_cap, hc[2], b->tie_cap,
                    hc[5]);
    if (h64[2] != (unsigned long long)P)
        return fail(C3X_EDEVICE, "internal: batch placement flags %u, %llu of %lld placed", hc[4],
                    h64[2], (long long)P);
    if (hc[7]) {
        // rows with more than 2048 matches: ordered by one segmented sort of
        // all of them after the graph, then renumbered job-locally
        const FinishArgs fa = batch_fin_args(b);
        c3x_status st = finish_huge(fa, hc + 6, s);
        if (st != C3X_OK) return st;
        const uint32_t nh = std::min(hc[7], b->seg_cap);
        hipLaunchKernelGGL(k_blocal_rows, dim3(std::min<uint32_t>(nh, 4096)), dim3(256), 0, s,
                           b->seg_huge, nh, b->off, b->djobs, b->ejobA, b->NA, b->oa, b->ob);
        BCHK(hipGetLastError(), "long rows");
        BCHK(hipMemcpyAsync(&hc[4], b->ctr + 4, sizeof(uint32_t), hipMemcpyDeviceToHost, s),
             "copy");
        BCHK(hipStreamSynchronize(s), "long rows");
    }
    if (hc[4])
        return fail(C3X_EDEVICE, "internal: batch placement flags %u, %llu of %lld placed", hc[4],
                    h64[2], (long long)P);
    b->P = P;
    b->stats.n_tests = (int64_t)h64[0];
    b->stats.n_band = (int64_t)h64[1];
    b->stats.n_ambiguous = hc[9];
    b->stats.n_best_ties = hc[2];
    const uint32_t nc = std::min(hc[3], b->tie_cap + b->bin_cap);
    if (nc == 0) return C3X_OK;
    // rows FP64 could not rank: every match listed, ranked in binary128
    Arena tmp(s);
    MatchArgs m = batch_args(b);
    uint32_t col_cap = 64 * nc + 1024;
    std::vector<ColEnt> col;
    for (int attempt = 0; attempt < 2; ++attempt) {
        ColEnt *dcol = (ColEnt *)tmp.get(col_cap * sizeof(ColEnt));
        if (!dcol) return fail(C3X_ENOMEM, "collect buffers");
        BCHK(hipMemsetAsync(b->ctr + 12, 0, 4, s), "memset");
        m.col_pos = b->unc;
        m.n_col = nc;
        m.col_n = b->ctr + 12;
        m.col = dcol;
        m.col_cap = col_cap;
        if (b->prec == C3X_FP64)
            hipLaunchKernelGGL((k_collect<C3X_CIRCLE, C3X_FP64, true>), dim3(nc), dim3(64), 0, s, m);
        else
            hipLaunchKernelGGL((k_collect<C3X_CIRCLE, C3X_MIXED, true>), dim3(nc), dim3(64), 0, s, m);
        uint32_t ncol = 0;
        BCHK(hipMemcpyAsync(&ncol, b->ctr + 12, 4, hipMemcpyDeviceToHost, s), "copy");
        BCHK(hipStreamSynchronize(s), "collect");
        if (ncol > col_cap) {
            col_cap = ncol;
            continue;
        }
        col.resize(ncol);
        BCHK(hipMemcpy(col.data(), dcol, ncol * sizeof(ColEnt), hipMemcpyDeviceToHost), "copy");
        break;
    }
    std::vector<uint32_t> upos(nc);
    std::vector<double2> ad(nc);
    BCHK(hipMemcpy(upos.data(), b->unc, nc * 4, hipMemcpyDeviceToHost), "copy");
    for (uint32_t k = 0; k < nc; ++k)
        BCHK(hipMemcpy(&ad[k], b->arad + upos[k], sizeof(double2), hipMemcpyDeviceToHost), "copy");
    std::vector<std::vector<const ColEnt *>> per(nc);
    for (const ColEnt &c : col)
        if (c.t < nc) per[c.t].push_back(&c);
    std::vector<uint32_t> prow, pbj;
    for (uint32_t k = 0; k < nc; ++k) {
        auto &v = per[k];
        if (v.empty()) continue;
        std::vector<double> r2(v.size()), d2(v.size());
        std::vector<int32_t> ib(v.size());
        for (size_t q = 0; q < v.size(); ++q) {
            r2[q] = v[q]->ra;
            d2[q] = v[q]->dec;
            ib[q] = (int32_t)v[q]->idxB;
        }
        const int w = c3x_q_best(ad[k].x, ad[k].y, (int)v.size(), r2.data(), d2.data(), ib.data());
        prow.push_back(upos[k]);
        pbj.push_back(v[w]->j);
    }
    if (!prow.empty()) {
        const uint32_t np = (uint32_t)prow.size();
        uint32_t *d1 = tmp.get_n<uint32_t>(np), *d2 = tmp.get_n<uint32_t>(np);
        if (!d1 || !d2) return fail(C3X_ENOMEM, "best patch");
        BCHK(hipMemcpyAsync(d1, prow.data(), np * 4, hipMemcpyHostToDevice, s), "copy");
        BCHK(hipMemcpyAsync(d2, pbj.data(), np * 4, hipMemcpyHostToDevice, s), "copy");
        hipLaunchKernelGGL(k_bpatch, dim3(nblk(np, 256)), dim3(256), 0, s, d1, d2, np, b->aidx,
                           b->arad, b->coordB, BRows{b->p64, b->p32}, b->djobs, b->ajob, b->obest,
                           b->obsep);
        BCHK(hipGetLastError(), "best patch");
        BCHK(hipStreamSynchronize(s), "best patch");
    }
    return C3X_OK;
}

extern "C" c3x_status c3x_batch_plan(const c3x_job *jobs, int32_t n_jobs, const double *raA,
                                     const double *decA, const double *raB, const double *decB,
                                     c3x_frame frame, const c3x_opts *opts, c3x_batch **out)
{
    clear_error();
    if (!out) return fail(C3X_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_jobs < 1 || n_jobs > (1 << 22)) return fail(C3X_EINVAL, "n_jobs must be in [1, 2^22]");
    if (!jobs) return fail(C3X_EINVAL, "jobs is NULL");
    if (frame != C3X_EQUATORIAL && frame != C3X_GALACTIC) return fail(C3X_EINVAL, "bad frame");
    c3x_opts o{};
    if (opts) o = *opts;
    if (o.precision != C3X_FP64 && o.precision != C3X_MIXED)
        return fail(C3X_EINVAL, "bad precision");
    int64_t SA = 0, SB = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const c3x_job &q = jobs[j];
        if (q.a_off < 0 || q.nA < 0 || q.b_off < 0 || q.nB < 0)
            return fail(C3X_EINVAL, "batch job %d: negative offset or count", j);
        if (!(q.radius_arcsec >= 0.0) || !(q.radius_arcsec <= kMaxBatchRadiusArcsec))
            return fail(C3X_EINVAL, "batch job %d: radius must be in [0, %g] arcsec", j,
                        kMaxBatchRadiusArcsec);
        if (q.radius_arcsec > 0.0 && q.radius_arcsec < 1e-6)
            return fail(C3X_EINVAL, "batch job %d: radius below 1e-6 arcsec", j);
        SA += q.nA;
        SB += q.nB;
    }
    if (SA > 2147483647LL || SB > 2147483647LL)
        return fail(C3X_ERANGE, "batch totals above 2^31 - 1 entries");
    if ((SA > 0 && (!raA || !decA)) || (SB > 0 && (!raB || !decB)))
        return fail(C3X_EINVAL, "NULL coordinate array");
    // the inputs may still be in flight on another stream
    if (hipDeviceSynchronize() != hipSuccess) return fail(C3X_EDEVICE, "device synchronize");
    c3x_batch *b = nullptr;
    c3x_status st = C3X_OK;
    // a plan whose one-sweep sort gave up its look-back is made again with
    // the table schedule
    for (int attempt = 0; attempt < 2; ++attempt) {
        b = new (std::nothrow) c3x_batch();
        if (!b) return fail(C3X_ENOMEM, "host allocation");
        (void)hipGetDevice(&b->device);
        b->onesweep = attempt == 0;
        b->prec = o.precision;
        b->nj = n_jobs;
        b->NA = SA;
        b->NB = SB;
        b->raA = raA;
        b->decA = decA;
        b->raB = raB;
        b->decB = decB;
        b->jobs.assign(jobs, jobs + n_jobs);
        if (hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return fail(C3X_EDEVICE, "stream");
        }
        st = batch_plan_impl(b);
        if (st == C3X_OK) st = batch_finish(b);
        if (st != kSortGaveUp) break;
        delete b;
        b = nullptr;
    }
    if (st != C3X_OK) {
        delete b;
        return st == kSortGaveUp ? fail(C3X_EDEVICE, "internal: sort gave up twice") : st;
    }
    b->stats.n_sort_retries = b->onesweep ? 0 : 1;
    b->stats.n_a = SA;
    b->stats.n_b = SB;
    b->stats.n_pairs = b->P;
    b->stats.precision = o.precision;
    b->stats.tile = b->tile;
    b->stats.queue = b->queue ? 1 : 0;
    b->stats.cell_arcsec = b->cell_scale;
    *out = b;
    return C3X_OK;
}

extern "C" c3x_status c3x_batch_run(c3x_batch *b, void *stream)
{
    clear_error();
    if (!b || !b->exec) return fail(C3X_EINVAL, "batch not planned");
    hipStream_t cs = (hipStream_t)stream;
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return fail(C3X_EDEVICE, "event");
    // order after the caller's stream, then run on the batch's own stream
    hipError_t e = hipEventRecord(ev, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->s, ev, 0);
    hipEvent_t t0, t1;
    bool timed = hipEventCreate(&t0) == hipSuccess && hipEventCreate(&t1) == hipSuccess;
    if (e == hipSuccess && timed) e = hipEventRecord(t0, b->s);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->s);
    if (e == hipSuccess && timed) e = hipEventRecord(t1, b->s);
    if (e == hipSuccess) e = hipEventRecord(ev, b->s);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
    c3x_status st = e == hipSuccess ? C3X_OK : fail_hip(e, "c3x_batch_run");
    if (st == C3X_OK) st = batch_finish(b);
    const bool retried = st == kSortGaveUp;
    if (retried) {
        // a one-sweep look-back gave up during the replay: the graph is
        // captured again with the table schedule and replayed
        b->onesweep = false;
        b->stats.n_sort_retries = 1;
        st = batch_capture(b);
        if (st == C3X_OK) {
            e = hipGraphLaunch(b->exec, b->s);
            if (e == hipSuccess) e = hipEventRecord(ev, b->s);
            if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
            st = e == hipSuccess ? batch_finish(b) : fail_hip(e, "c3x_batch_run");
        }
        if (st == kSortGaveUp) st = fail(C3X_EDEVICE, "internal: table sort reported a give-up");
    }
    if (st == C3X_OK && timed && !retried) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t0, t1) == hipSuccess) b->stats.ms_total = ms;
    }
    if (timed) {
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
    }
    (void)hipEventDestroy(ev);
    b->stats.n_pairs = b->P;
    return st;
}

extern "C" c3x_status c3x_batch_result(const c3x_batch *b, c3x_result **out)
{
    clear_error();
    if (!b || !out) return fail(C3X_EINVAL, "NULL argument");
    *out = nullptr;
    c3x_result *R = new (std::nothrow) c3x_result();
    if (!R) return fail(C3X_ENOMEM, "host allocation");
    R->device = b->device;
    R->n_pairs = b->P;
    R->nA = b->NA;
    R->mode = C3X_ALL | C3X_BEST;
    R->idxA = R->mem.get_n<int32_t>(b->P);
    R->idxB = R->mem.get_n<int32_t>(b->P);
    R->sep = R->mem.get_n<double>(b->P);
    R->best_idx = R->mem.get_n<int32_t>(b->NA);
    R->best_sep = R->mem.get_n<double>(b->NA);
    if (!R->idxA || !R->idxB || !R->sep || !R->best_idx || !R->best_sep) {
        delete R;
        return fail(C3X_ENOMEM, "batch result buffers");
    }
    hipError_t e = hipSuccess;
    if (b->P > 0) {
        e = hipMemcpyAsync(R->idxA, b->oa, b->P * 4, hipMemcpyDeviceToDevice, b->s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(R->idxB, b->ob, b->P * 4, hipMemcpyDeviceToDevice, b->s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(R->sep, b->os, b->P * 8, hipMemcpyDeviceToDevice, b->s);
    }
    if (b->NA > 0 && e == hipSuccess) {
        e = hipMemcpyAsync(R->best_idx, b->obest, b->NA * 4, hipMemcpyDeviceToDevice, b->s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(R->best_sep, b->obsep, b->NA * 8, hipMemcpyDeviceToDevice, b->s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->s);
    if (e != hipSuccess) {
        delete R;
        return fail_hip(e, "c3x_batch_result");
    }
    R->stats = b->stats;
    *out = R;
    return C3X_OK;
}

extern "C" c3x_status c3x_batch_offsets(const c3x_batch *b, int64_t *pair_off)
{
    clear_error();
    if (!b || !pair_off) return fail(C3X_EINVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(pair_off, b->joboff, (b->nj + 1) * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, b->s);
    if (e == hipSuccess) e = hipStreamSynchronize(b->s);
    if (e != hipSuccess) return fail_hip(e, "c3x_batch_offsets");
    return C3X_OK;
}

extern "C" c3x_status c3x_batch_stats(const c3x_batch *b, c3x_stats *st)
{
    if (!b || !st) return fail(C3X_EINVAL, "NULL argument");
    *st = b->stats;
    return C3X_OK;
}

extern "C" void c3x_batch_free(c3x_batch *b) { delete b; }
