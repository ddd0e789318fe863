// c3x_concentric.hip -- concentric ellipses of ClumpPopulator (Section 3):
// each source's ellipse taken at several scale factors; a pair's level is
// the smallest scale whose ellipse holds the B source.
//
// The scaled ellipses are nested (axes fl(k a) and fl(k b) grow with k, same
// centre and PA), so the largest one's certified match holds every pair,
// and a pair's level is the smallest scale whose own certified match holds
// it. Each scale is one c3x_match over the same index:
//
//   k_scale_axes   axes of scale k                         16 B in, 16 B out per source
//   c3x_match      the certified elliptical match at that scale
//   k_level_mark   its pairs located in the largest scale's pairs (binary
//                  search over the canonical (idxA, idxB) order), level set
#include <cmath>
#include <string>

#include "c3x_host.h"
#include "c3x_internal.h"

namespace c3x {

constexpr int kMaxScales = 64;

__global__ void k_scale_axes(const double *__restrict__ a, const double *__restrict__ b,
                             int64_t n, double k, double *__restrict__ ka,
                             double *__restrict__ kb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    ka[t] = a[t] * k;
    kb[t] = b[t] * k;
}

__global__ void k_level_fill(int32_t *__restrict__ level, int64_t n, int32_t v)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) level[t] = v;
}

// Pairs (ia, ib)[0, n) of scale m, each found among the outer pairs (oa, ob)
// [0, P) (both in canonical order): its level becomes m. A pair missing from
// the outer set (the scales would not be nested) sets *err.
__global__ void k_level_mark(const int32_t *__restrict__ ia, const int32_t *__restrict__ ib,
                             int64_t n, const int32_t *__restrict__ oa,
                             const int32_t *__restrict__ ob, int64_t P, int32_t m,
                             int32_t *__restrict__ level, uint32_t *__restrict__ err)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t x = ia[t], y = ib[t];
    int64_t lo = 0, hi = P;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const int32_t u = oa[mid], v = ob[mid];
        if (u < x || (u == x && v < y)) lo = mid + 1;
        else hi = mid;
    }
    if (lo < P && oa[lo] == x && ob[lo] == y) level[lo] = m;
    else atomicOr(err, 1u);
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
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    Arena tmp(s);
    double *ka = tmp.get_n<double>(nA), *kb = tmp.get_n<double>(nA);
    uint32_t *err = tmp.get_n<uint32_t>(1);
    if (!ka || !kb || !err) return fail(C3X_ENOMEM, "scaled axes");
    CCHK(hipMemsetAsync(err, 0, sizeof(uint32_t), s), "memset");
    c3x_area sa = *area;
    sa.semi_major_arcsec = ka;
    sa.semi_minor_arcsec = kb;
    auto scaled_match = [&](int m, unsigned md, c3x_result **res) -> c3x_status {
        if (nA > 0)
            hipLaunchKernelGGL(k_scale_axes, dim3(cblk(nA)), dim3(256), 0, s,
                               area->semi_major_arcsec, area->semi_minor_arcsec, nA, scales[m],
                               ka, kb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail_hip(e, "scale axes");
        c3x_status st = c3x_match(ix, ra_deg, dec_deg, nA, frame, &sa, md, opts, res);
        if (st != C3X_OK) {
            const std::string why = c3x_last_error();  // the message buffer is reused below
            return fail(st, "scale %d (%g): %s", m, scales[m], why.c_str());
        }
        return C3X_OK;
    };
    // the largest ellipse: the stored pairs (and, if asked, the best matches)
    ResultGuard outer;
    c3x_status st = scaled_match(n_scales - 1, mode, &outer.r);
    if (st != C3X_OK) return st;
    c3x_result *R = outer.r;
    const int64_t P = R->n_pairs;
    R->level = R->mem.get_n<int32_t>(P);
    if (!R->level) return fail(C3X_ENOMEM, "levels");
    if (P > 0)
        hipLaunchKernelGGL(k_level_fill, dim3(cblk(P)), dim3(256), 0, s, R->level, P,
                           (int32_t)(n_scales - 1));
    // smaller scales, from the largest down: each overwrites its pairs' level
    for (int m = n_scales - 2; m >= 0 && P > 0; --m) {
        ResultGuard inner;
        st = scaled_match(m, C3X_ALL, &inner.r);
        if (st != C3X_OK) return st;
        const int64_t n = inner.r->n_pairs;
        if (n > 0)
            hipLaunchKernelGGL(k_level_mark, dim3(cblk(n)), dim3(256), 0, s, inner.r->idxA,
                               inner.r->idxB, n, R->idxA, R->idxB, P, (int32_t)m, R->level, err);
        CCHK(hipGetLastError(), "level mark");
        CCHK(hipStreamSynchronize(s), "level mark");  // before the inner result is freed
    }
    uint32_t herr = 0;
    CCHK(hipMemcpyAsync(&herr, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy");
    CCHK(hipStreamSynchronize(s), "c3x_match_concentric");
    if (herr) return fail(C3X_EDEVICE, "a smaller ellipse held a pair the largest did not");
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
