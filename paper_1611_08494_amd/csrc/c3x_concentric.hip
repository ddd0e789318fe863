// c3x_concentric.hip -- concentric ellipses of ClumpPopulator (Section 3):
// each source's ellipse taken at several scale factors; a pair's level is
// the smallest scale whose ellipse holds the B source.
//
// The scaled ellipses are nested (axes fl(k a) and fl(k b) grow with k, same
// centre and PA), so the largest one's certified match holds every pair.
// One c3x_match at the largest scale gives the pairs; one thread per pair
// then finds its level. The pair's parts of the FP64 ellipse recheck
// (theta / sin theta and the sines along and across the orientation) do not
// depend on the axes: they are computed once, and the smaller scales, in
// increasing order, are decided against them with the recheck's margin. A
// pair whose scale the margin leaves open is decided from that scale up in
// binary128 on the host.
//
//   k_scale_axes     axes of the largest scale              16 B in, 16 B out per source
//   c3x_match        the certified elliptical match at that scale
//   k_check_scaled   the smaller scales' axes inside the ellipse domain
//   k_levels         a pair's level, or the pair listed for the host
//                    (8 B of indices, 40 B of A and B coordinates and
//                    ellipse, 4 B out per pair)
//   k_level_patch    the host's levels written back
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "c3x_host.h"
#include "c3x_internal.h"

namespace c3x {

constexpr int kMaxScales = 64;

// The scale factors, by value.
struct LevelScales {
    double k[kMaxScales];
    int32_t n;
};

// A pair whose level the FP64 margin left open at scale m (every smaller
// scale decided outside): what the host's binary128 decision needs.
struct LevelAmb {
    double raA, decA, raB, decB, a, b, pa;
    int64_t p;
    int32_t m, pad;
};

__global__ void k_scale_axes(const double *__restrict__ a, const double *__restrict__ b,
                             int64_t n, double k, double *__restrict__ ka,
                             double *__restrict__ kb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    ka[t] = a[t] * k;
    kb[t] = b[t] * k;
}

// The smaller scales' axes fl(k a), fl(k b) inside the domain of an ellipse
// (1e-6 <= b <= a <= 324000 arcsec, a <= 1000 b); the largest failing scale
// and its first row: the minimum of ((n - 2 - m) << 32 | row) in *first.
__global__ void k_check_scaled(const double *__restrict__ a, const double *__restrict__ b,
                               int64_t n, LevelScales sc, unsigned long long *__restrict__ first)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double A = a[t], B = b[t];
    for (int m = sc.n - 2; m >= 0; --m) {
        const double ka = A * sc.k[m], kb = B * sc.k[m];
        const bool ok = isfinite(ka) && isfinite(kb) && kb >= 1e-6 && kb <= ka &&
                        ka <= 324000.0 && ka <= 1000.0 * kb;
        if (!ok) {
            atomicMin(first, ((unsigned long long)(sc.n - 2 - m) << 32) | (uint64_t)t);
            return;
        }
    }
}

// One thread per pair p of the largest ellipses (A row ia[p], B row ib[p]):
// level[p] = the smallest scale whose ellipse holds B, or -1 with the pair
// listed for the host (every pair with a smaller scale to decide, under
// force_host). The orientation is taken as when A is prepared for a match
// (T = pa_zero + pa_sense PA).
__global__ void k_levels(const int32_t *__restrict__ ia, const int32_t *__restrict__ ib,
                         int64_t P, const double *__restrict__ ra, const double *__restrict__ dec,
                         const double *__restrict__ sa, const double *__restrict__ sb,
                         const double *__restrict__ pa, double pa_zero, int pa_sense,
                         const double2 *__restrict__ coordB, LevelScales sc,
                         int32_t *__restrict__ level, LevelAmb *__restrict__ amb,
                         uint32_t *__restrict__ n_amb, uint32_t cap, int force_host)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int32_t i = ia[p], j = ib[p];
    ARec a;
    a.ra = ra[i];
    a.dec = dec[i];
    unit_vec(a.ra, a.dec, a.x, a.y, a.z);
    a.cosd = cos_dec_acc(a.dec);
    a.reach_deg = 0.0;
    a.idx = (uint32_t)i;
    a.pad = 0;
    const double2 rb = coordB[j];
    const double cd2 = cos_dec_acc(rb.y);
    const double h = haversine(a.ra, a.dec, a.cosd, rb.x, rb.y, cd2);
    int32_t lv = sc.n - 1;
    if (h == 0.0) {
        lv = 0;
    } else if (sc.n > 1) {
        const double T = pa_zero + (double)pa_sense * pa[i];
        double st, ct;
        sincos(T * kDeg, &st, &ct);
        double f, su, sv;
        ell_parts(a, ct, st, rb, cd2, h, f, su, sv);
        const double A = sa[i], B = sb[i];
        for (int m = 0; m < sc.n - 1; ++m) {
            const int d =
                force_host ? AMBIG : ell_decide(f, su, sv, A * sc.k[m], B * sc.k[m]);
            if (d == OUT) continue;
            if (d == IN) {
                lv = m;
            } else {
                lv = -1;
                const uint32_t slot = atomicAdd(n_amb, 1u);
                if (slot < cap) {
                    LevelAmb e;
                    e.raA = a.ra;
                    e.decA = a.dec;
                    e.raB = rb.x;
                    e.decB = rb.y;
                    e.a = A;
                    e.b = B;
                    e.pa = pa[i];
                    e.p = p;
                    e.m = m;
                    e.pad = 0;
                    amb[slot] = e;
                }
            }
            break;
        }
    }
    level[p] = lv;
}

__global__ void k_level_patch(const int64_t *__restrict__ pos, const int32_t *__restrict__ lv,
                              uint32_t n, int64_t P, int32_t *__restrict__ level)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && pos[t] >= 0 && pos[t] < P) level[pos[t]] = lv[t];
}

static inline unsigned cblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace c3x

using namespace c3x;

#define CCHK(expr, what)                                 \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

namespace {
struct ResultGuard {
    c3x_result *r = nullptr;
    ~ResultGuard()
    {
        if (r) c3x_result_free(r);
    }
};
}  // namespace

extern "C" c3x_status c3x_match_concentric(const c3x_index *ix, const double *ra_deg,
                                           const double *dec_deg, int64_t nA, c3x_frame frame,
                                           const c3x_area *area, const double *scales,
                                           int32_t n_scales, unsigned mode,
                                           const c3x_opts *opts, c3x_result **out)
{
    clear_error();
    if (!out) return fail(C3X_EINVAL, "NULL out");
    *out = nullptr;
    if (!ix || !area || !scales) return fail(C3X_EINVAL, "NULL argument");
    if (area->shape != C3X_ELLIPSE) return fail(C3X_EINVAL, "concentric areas need an ellipse");
    if (!(mode & C3X_ALL)) return fail(C3X_EINVAL, "concentric levels need mode C3X_ALL");
    if (n_scales < 1 || n_scales > kMaxScales)
        return fail(C3X_EINVAL, "n_scales must be in [1, %d]", kMaxScales);
    for (int m = 0; m < n_scales; ++m) {
        if (!(std::isfinite(scales[m]) && scales[m] > 0.0) || (m && !(scales[m] > scales[m - 1])))
            return fail(C3X_EINVAL, "scales must be finite, positive and strictly increasing");
    }
    if (nA < 0) return fail(C3X_EINVAL, "nA < 0");
    if (nA > 0 && (!area->semi_major_arcsec || !area->semi_minor_arcsec || !area->pa_deg))
        return fail(C3X_EINVAL, "NULL ellipse array");
    if (frame != C3X_EQUATORIAL && frame != C3X_GALACTIC) return fail(C3X_EINVAL, "bad frame");
    if (nA > 0 && (!ra_deg || !dec_deg)) return fail(C3X_EINVAL, "NULL coordinate array");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    Arena tmp(s);
    // catalogue A in the index's frame (as the match itself would convert
    // it): the levels read the same positions and orientations
    c3x_area ea = *area;
    {
        const c3x_status cs = convert_catalogue_a((int)frame, (int)ix->frame, nA, &ra_deg,
                                                  &dec_deg, &ea, tmp, s);
        if (cs != C3X_OK) return cs;
        frame = (c3x_frame)ix->frame;
    }
    LevelScales sc{};
    for (int m = 0; m < n_scales; ++m) sc.k[m] = scales[m];
    sc.n = n_scales;
    double *ka = tmp.get_n<double>(nA), *kb = tmp.get_n<double>(nA);
    unsigned long long *first = tmp.get_n<unsigned long long>(1);
    uint32_t *n_amb = tmp.get_n<uint32_t>(1);
    if (!ka || !kb || !first || !n_amb) return fail(C3X_ENOMEM, "scaled axes");
    c3x_area sa = ea;
    sa.semi_major_arcsec = ka;
    sa.semi_minor_arcsec = kb;
    const int top = n_scales - 1;
    if (nA > 0)
        hipLaunchKernelGGL(k_scale_axes, dim3(cblk(nA)), dim3(256), 0, s, ea.semi_major_arcsec,
                           ea.semi_minor_arcsec, nA, scales[top], ka, kb);
    CCHK(hipGetLastError(), "scale axes");
    // the largest ellipses: the stored pairs (and, if asked, the best matches)
    ResultGuard outer;
    c3x_status st = c3x_match(ix, ra_deg, dec_deg, nA, frame, &sa, mode, opts, &outer.r);
    if (st != C3X_OK) {
        const std::string why = c3x_last_error();  // the message buffer is reused below
        return fail(st, "scale %d (%g): %s", top, scales[top], why.c_str());
    }
    // the smaller scales' axes inside the ellipse domain, as a match at each
    // scale would require (the largest one failing first)
    if (nA > 0 && n_scales > 1) {
        CCHK(hipMemsetAsync(first, 0xff, sizeof(unsigned long long), s), "memset");
        hipLaunchKernelGGL(k_check_scaled, dim3(cblk(nA)), dim3(256), 0, s,
                           ea.semi_major_arcsec, ea.semi_minor_arcsec, nA, sc, first);
        CCHK(hipGetLastError(), "scaled axes check");
        unsigned long long hf = ~0ull;
        CCHK(hipMemcpyAsync(&hf, first, sizeof(hf), hipMemcpyDeviceToHost, s), "copy");
        CCHK(hipStreamSynchronize(s), "scaled axes check");
        if (hf != ~0ull) {
            const int m = n_scales - 2 - (int)(hf >> 32);
            return fail(C3X_EINVAL,
                        "scale %d (%g): catalogue A row %u: ellipse axes outside 1e-6 <= b <= "
                        "a <= 324000 arcsec, a <= 1000 b",
                        m, scales[m], (unsigned)(hf & 0xffffffffu));
        }
    }
    c3x_result *R = outer.r;
    const int64_t P = R->n_pairs;
    R->level = R->mem.get_n<int32_t>(P);
    if (!R->level) return fail(C3X_ENOMEM, "levels");
    if (P > 0) {
        // test setting: every level with a smaller scale decided on the host
        const bool force_host = env_on("C3X_DEBUG_FORCE_AMBIG");
        uint32_t cap = (uint32_t)std::min<int64_t>(std::max<int64_t>(1024, P / 256), 1 << 26);
        uint32_t hn = 0;
        LevelAmb *amb = nullptr;
        for (int attempt = 0; attempt < 2; ++attempt) {
            amb = tmp.get_n<LevelAmb>(cap);
            if (!amb) return fail(C3X_ENOMEM, "level list");
            CCHK(hipMemsetAsync(n_amb, 0, sizeof(uint32_t), s), "memset");
            hipLaunchKernelGGL(k_levels, dim3(cblk(P)), dim3(256), 0, s, R->idxA, R->idxB, P,
                               ra_deg, dec_deg, ea.semi_major_arcsec, ea.semi_minor_arcsec,
                               ea.pa_deg, ea.pa_zero_deg, ea.pa_sense, ix->radec, sc, R->level,
                               amb, n_amb, cap, (int)force_host);
            CCHK(hipGetLastError(), "levels");
            CCHK(hipMemcpyAsync(&hn, n_amb, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy");
            CCHK(hipStreamSynchronize(s), "levels");
            if (hn <= cap) break;
            cap = hn;  // the list ran out: the pass again with room for all
        }
        if (hn > cap) return fail(C3X_EDEVICE, "level list: %u entries for %u slots", hn, cap);
        // pairs the FP64 margin left open: binary128 from their scale up
        if (hn > 0) {
            std::vector<LevelAmb> h(hn);
            CCHK(hipMemcpyAsync(h.data(), amb, hn * sizeof(LevelAmb), hipMemcpyDeviceToHost, s),
                 "copy");
            CCHK(hipStreamSynchronize(s), "level list");
            std::vector<int64_t> pos(hn);
            std::vector<int32_t> lv(hn);
            for (uint32_t t = 0; t < hn; ++t) {
                const LevelAmb &e = h[t];
                int32_t l = top;
                for (int m = e.m; m < top; ++m) {
                    if (c3x_q_ellipse(e.raA, e.decA, e.raB, e.decB, e.a * scales[m],
                                      e.b * scales[m], e.pa, ea.pa_zero_deg, ea.pa_sense)) {
                        l = m;
                        break;
                    }
                }
                pos[t] = e.p;
                lv[t] = l;
            }
            int64_t *dpos = tmp.get_n<int64_t>(hn);
            int32_t *dlv = tmp.get_n<int32_t>(hn);
            if (!dpos || !dlv) return fail(C3X_ENOMEM, "level patch");
            CCHK(hipMemcpyAsync(dpos, pos.data(), hn * sizeof(int64_t), hipMemcpyHostToDevice, s),
                 "copy");
            CCHK(hipMemcpyAsync(dlv, lv.data(), hn * sizeof(int32_t), hipMemcpyHostToDevice, s),
                 "copy");
            hipLaunchKernelGGL(k_level_patch, dim3(cblk(hn)), dim3(256), 0, s, dpos, dlv, hn, P,
                               R->level);
            CCHK(hipGetLastError(), "level patch");
            CCHK(hipStreamSynchronize(s), "level patch");  // before the host vectors go
        }
        R->stats.n_ambiguous += hn;  // host decisions, as for the band
    }
    CCHK(hipStreamSynchronize(s), "c3x_match_concentric");
    R->n_scales = n_scales;
    *out = R;
    outer.r = nullptr;
    return C3X_OK;
}

extern "C" c3x_status c3x_result_levels(const c3x_result *r, const int32_t **level)
{
    if (!r || !level) return fail(C3X_EINVAL, "NULL argument");
    if (r->n_scales < 1) return fail(C3X_EINVAL, "not a result of c3x_match_concentric");
    *level = r->level;
    return C3X_OK;
}
