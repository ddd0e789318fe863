// c3x_match.hip -- cross-match of catalogue A against a sky index.
//
// Paper Section 2.1 ("Sky" case): a region is centred on each A source and
// the B sources inside it are found "by comparing their distance from the
// central object and the limits of the area"; Section 2.2: the matches are
// kept as rows, all of them or only the best; Section 2.3: each source is
// tested only against the cells around it. Phases on one stream:
//   A prep      validate, key, sort A by cell, sorted A records
//   count       per A: enumerate cells in reach, decide every candidate
//               (fast filter -> FP64 haversine recheck -> ambiguous list)
//   [host]      ambiguous pairs decided in binary128, verdict table uploaded
//   scan        per-A counts -> int64 offsets in idxA order
//   write       same enumeration and decisions; writes (idxA, idxB, sep) and
//               the best match (min separation, lower idxB on equal values);
//               near-tie best matches are listed for the host
//   order       each A's segment sorted by idxB (canonical order)
// The decisions of the count and write passes come from the same device
// function compiled with -ffp-contract=off, so they agree bit for bit.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "c3x_host.h"
#include "c3x_sort.h"

namespace c3x {

constexpr int kMatchBlock = 256;
constexpr double kTieRel = kE40;  // best matches closer than this (relative) go to the host

struct alignas(16) ColEnt {
    uint32_t t, idxB, j, pad;
    double sep, ra, dec;
};
struct AmbInfo {
    double raA, decA, raB, decB, a, b, pa;
    uint32_t i, j, idxA, idxB;
};
struct alignas(16) TieEnt {
    uint32_t i, idxA;
    double s1;
};

// ---------------------------------------------------------------------------- A preparation

__global__ void k_prep_a(const double *__restrict__ ra, const double *__restrict__ dec, int64_t n,
                         Grid g, int shape, const double *__restrict__ sa,
                         const double *__restrict__ sb, const double *__restrict__ pa,
                         uint32_t *__restrict__ keys, uint32_t *__restrict__ rows,
                         uint32_t *__restrict__ bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = ra[i], d = dec[i];
    bool ok = isfinite(a) && isfinite(d) && a >= 0.0 && a < 360.0 && fabs(d) <= 90.0;
    if (shape == C3X_ELLIPSE) {
        double A = sa[i], B = sb[i], P = pa[i];
        ok = ok && isfinite(A) && isfinite(B) && isfinite(P) && B >= 1e-6 && B <= A &&
             A <= 324000.0 && A <= 1000.0 * B;
    }
    if (!ok) {
        atomicMin(bad, (uint32_t)i);
        a = 0.0;
        d = 0.0;
    }
    int z = zone_of(d, g);
    keys[i] = g.zbase[z] + cell_of(z, a, g);
    rows[i] = (uint32_t)i;
}

// Margin on the ellipse form Q for a filter whose tangent-plane components
// carry an absolute error <= c * kappa + lambda (c the chord). Covers the
// rounding of Q, the truncation of (theta / sin theta)^2 ~ 1 + c^2 / 3 and a
// factor-2 safety; returns a huge value when the filter cannot decide.
__device__ __forceinline__ double ell_margin(double ar, double br, double kappa, double lambda,
                                             double u_round)
{
    double ia = 1.0 / ar, ib = 1.0 / br;
    double k1 = kappa * (1.0 + ar / br) * 1.01;
    double l1 = 1.5 * lambda * (ia + ib);
    double rho = 2.0 * k1 + 2.0 * l1 + (k1 + l1) * (k1 + l1) + 6.0 * u_round;
    double trunc = 0.2 * (ar * ar) * (ar * ar);
    double m = 2.0 * (2.0 * rho + trunc);
    return m > 0.25 ? 1e30 : m;
}

template <int SHAPE>
__global__ void k_gather_a(const uint32_t *__restrict__ rows, const double *__restrict__ ra,
                           const double *__restrict__ dec, int64_t n, double radius_arcsec,
                           const double *__restrict__ sa, const double *__restrict__ sb,
                           const double *__restrict__ pa, double pa_zero, int pa_sense,
                           double L_rad, ARec *__restrict__ arec, AEll *__restrict__ aell,
                           AEllR *__restrict__ aellr)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t row = rows[i];
    if (row >= (uint64_t)n) row = 0;  // unreachable for a permutation; keeps reads in bounds
    ARec r;
    r.ra = ra[row];
    r.dec = dec[row];
    unit_vec(r.ra, r.dec, r.x, r.y, r.z);
    r.cosd = cos_dec_acc(r.dec);
    r.idx = row;
    double reach_as = SHAPE == C3X_ELLIPSE ? sa[row] : radius_arcsec;
    r.reach_deg = reach_as / 3600.0;
    arec[i] = r;
    if (SHAPE == C3X_ELLIPSE) {
        double A = sa[row], B = sb[row];
        double T = pa_zero + (double)pa_sense * pa[row];
        double st, ct;
        sincos(T * kDeg, &st, &ct);
        double sdd = r.z;           // sin dec
        double sra, cra;
        sincos(r.ra * kDeg, &sra, &cra);
        // local north and east at A
        double nx = -sdd * cra, ny = -sdd * sra, nz = r.cosd;
        double ex = -sra, ey = cra;
        AEll e;
        e.ux = nx * ct + ex * st;
        e.uy = ny * ct + ey * st;
        e.uz = nz * ct;
        e.vx = ex * ct - nx * st;
        e.vy = ey * ct - ny * st;
        e.vz = -nz * st;
        double ar = kDeg * (A / 3600.0), br = kDeg * (B / 3600.0);
        e.ia = 1.0 / ar;
        e.ib = 1.0 / br;
        aell[i] = e;
        AEllR q;
        q.a_arcsec = A;
        q.b_arcsec = B;
        q.ct = ct;
        q.st = st;
        const double ev = 32.0 * kU;              // unit-vector component error
        const double s3 = 1.7320508075688772;
        double kappa64 = s3 * 64.0 * kU + s3 * kU + 4.0 * kU;
        double lambda64 = 2.0 * s3 * ev;
        q.m64 = ell_margin(ar, br, kappa64, lambda64, kU);
        const double e32 = kU32 * 1.0001;
        double kappa32 = s3 * (e32 + 64.0 * kU) + 2.0 * s3 * e32 + 4.0 * e32;
        double lambda32 = 2.0 * s3 * e32 * L_rad + 2.0 * s3 * ev;
        double m32 = ell_margin(ar, br, kappa32, lambda32, e32);
        q.m32 = m32 > 0.25 ? 0.0f : (float)(m32 * 1.0001);
        q.pad = 0.f;
        aellr[i] = q;
    }
}

// ---------------------------------------------------------------------------- match

__device__ __forceinline__ int verdict(const MatchArgs &m, uint32_t i, uint32_t j)
{
    unsigned long long k = ((unsigned long long)i << 32) | j;
    uint32_t lo = 0, hi = m.n_ver;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (m.ver_key[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    if (lo < m.n_ver && m.ver_key[lo] == k) return m.ver_in[lo] ? IN : OUT;
    atomicOr(m.err_flag, 4u);
    return OUT;
}

// MODE 0: count, 1: write, 2: collect near-best candidates.
template <int SHAPE, int PREC, int MODE>
__global__ __launch_bounds__(kMatchBlock) void k_match(MatchArgs m)
{
    __shared__ unsigned long long s_tests, s_band;
    if (threadIdx.x == 0) {
        s_tests = 0;
        s_band = 0;
    }
    __syncthreads();
    uint32_t t = blockIdx.x * kMatchBlock + threadIdx.x;
    uint32_t nwork = MODE == 2 ? m.n_col : (uint32_t)m.nA;
    unsigned long long tests = 0, band = 0;
    if (t < nwork) {
        uint32_t i = MODE == 2 ? m.col_pos[t] : t;
        const ARec a = m.arec[i];
        AEll e{};
        AEllR er{};
        if (SHAPE == C3X_ELLIPSE) {
            e = m.aell[i];
            er = m.aellr[i];
        }
        float ux = (float)e.ux, uy = (float)e.uy, uz = (float)e.uz;
        float vx = (float)e.vx, vy = (float)e.vy, vz = (float)e.vz;
        float ia32 = (float)e.ia, ib32 = (float)e.ib;
        double lim = MODE == 2 ? m.col_lim[t] : 0.0;
        uint32_t cnt = 0;
        int64_t o = 0, oe = 0;
        if (MODE == 1) {
            o = m.off[a.idx];
            oe = m.off[a.idx + 1];
        }
        double s1 = INFINITY, s2 = INFINITY;
        int32_t bidx = -1;
        for_each_range(m.g, a.ra, a.dec, a.cosd, a.reach_deg, [&](int z, uint32_t j0, uint32_t j1) {
            uint32_t curkey = 0xffffffffu;
            float ax = 0.f, ay = 0.f, az = 0.f;
            for (uint32_t j = j0; j < j1; ++j) {
                ++tests;
                int d;
                uint32_t idxB;
                if (PREC == C3X_FP64) {
                    const Pay64 b = m.pay64[j];
                    idxB = b.idx;
                    double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
                    double c2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    if (SHAPE == C3X_CIRCLE) {
                        d = c2 <= m.t64_in ? IN : (c2 > m.t64_out ? OUT : AMBIG);
                    } else {
                        double su = fma(dx, e.ux, fma(dy, e.uy, dz * e.uz));
                        double sv = fma(dx, e.vx, fma(dy, e.vy, dz * e.vz));
                        double xu = su * e.ia, xv = sv * e.ib;
                        double q = fma(xu, xu, xv * xv);
                        double qf = q * fma(c2, 1.0 / 3.0, 1.0);
                        d = qf <= 1.0 - er.m64 ? IN : (qf > 1.0 + er.m64 ? OUT : AMBIG);
                    }
                } else {
                    uint32_t key = m.g.keys[j];
                    if (key != curkey) {
                        curkey = key;
                        double rx, ry, rz;
                        cell_ref(z, key - m.g.zbase[z], m.g, rx, ry, rz);
                        ax = (float)(a.x - rx);
                        ay = (float)(a.y - ry);
                        az = (float)(a.z - rz);
                    }
                    const Pay32 b = m.pay32[j];
                    idxB = b.idx;
                    float dx = b.x - ax, dy = b.y - ay, dz = b.z - az;
                    float c2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    if (SHAPE == C3X_CIRCLE) {
                        d = c2 <= m.t32_in ? IN : (c2 > m.t32_out ? OUT : AMBIG);
                    } else {
                        float su = fmaf(dx, ux, fmaf(dy, uy, dz * uz));
                        float sv = fmaf(dx, vx, fmaf(dy, vy, dz * vz));
                        float xu = su * ia32, xv = sv * ib32;
                        float q = fmaf(xu, xu, xv * xv);
                        float qf = q * fmaf(c2, 1.0f / 3.0f, 1.0f);
                        float mm = er.m32;
                        d = mm == 0.0f ? AMBIG
                                       : (qf <= 1.0f - mm ? IN : (qf > 1.0f + mm ? OUT : AMBIG));
                    }
                }
                double2 rb;
                bool have_rb = false;
                if (d == AMBIG) {
                    ++band;
                    rb = m.radecB[j];
                    have_rb = true;
                    if (SHAPE == C3X_CIRCLE)
                        d = m.r_zero ? (same_point(a, rb) ? IN : OUT) : recheck_circle(a, rb, m.h_r);
                    else
                        d = recheck_ellipse(a, er, rb);
                    if (d == AMBIG) {
                        if (MODE == 0) {
                            uint32_t slot = atomicAdd(m.amb_n, 1u);
                            if (slot < m.amb_cap) m.amb[slot] = make_uint2(i, j);
                            d = OUT;
                        } else {
                            d = verdict(m, i, j);
                        }
                    }
                }
                if (d != IN) continue;
                if (MODE == 0) {
                    ++cnt;
                    continue;
                }
                if (!have_rb) rb = m.radecB[j];
                double sp = sep_arcsec(a, rb.x, rb.y);
                if (MODE == 2) {
                    if (sp <= lim) {
                        uint32_t slot = atomicAdd(m.col_n, 1u);
                        if (slot < m.col_cap) {
                            ColEnt c;
                            c.t = t;
                            c.idxB = idxB;
                            c.j = j;
                            c.pad = 0;
                            c.sep = sp;
                            c.ra = rb.x;
                            c.dec = rb.y;
                            ((ColEnt *)m.col)[slot] = c;
                        }
                    }
                    continue;
                }
                if (m.write_pairs) {
                    int64_t p = o + cnt;
                    if (p < oe) {
                        m.out_a[p] = (int32_t)a.idx;
                        m.out_b[p] = (int32_t)idxB;
                        m.out_sep[p] = sp;
                    } else {
                        atomicOr(m.err_flag, 1u);
                    }
                }
                ++cnt;
                if (sp < s1 || (sp == s1 && (int32_t)idxB < bidx)) {
                    s2 = s1;
                    s1 = sp;
                    bidx = (int32_t)idxB;
                } else if (sp < s2) {
                    s2 = sp;
                }
            }
        });
        if (MODE == 0) m.cnt[a.idx] = cnt;
        if (MODE == 1) {
            if (m.write_pairs && o + cnt != oe) atomicOr(m.err_flag, 2u);
            m.best_idx[a.idx] = cnt ? bidx : -1;
            m.best_sep[a.idx] = cnt ? s1 : NAN;
            if (cnt >= 2 && s2 <= s1 * (1.0 + kTieRel) + 1e-300) {
                uint32_t slot = atomicAdd(m.tie_n, 1u);
                if (slot < m.tie_cap) {
                    TieEnt te;
                    te.i = i;
                    te.idxA = a.idx;
                    te.s1 = s1;
                    ((TieEnt *)m.tie)[slot] = te;
                }
            }
        }
    }
    if (tests) atomicAdd(&s_tests, tests);
    if (band) atomicAdd(&s_band, band);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_tests) atomicAdd(m.n_tests, s_tests);
        if (s_band) atomicAdd(m.n_band, s_band);
    }
}

__global__ void k_amb_info(const uint2 *__restrict__ amb, uint32_t n, const ARec *__restrict__ arec,
                           const double2 *__restrict__ radecB, const Pay64 *__restrict__ p64,
                           const Pay32 *__restrict__ p32, const double *__restrict__ sa,
                           const double *__restrict__ sb, const double *__restrict__ pa,
                           AmbInfo *__restrict__ out)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint2 q = amb[t];
    ARec a = arec[q.x];
    double2 b = radecB[q.y];
    AmbInfo r;
    r.raA = a.ra;
    r.decA = a.dec;
    r.raB = b.x;
    r.decB = b.y;
    r.a = sa ? sa[a.idx] : 0.0;
    r.b = sb ? sb[a.idx] : 0.0;
    r.pa = pa ? pa[a.idx] : 0.0;
    r.i = q.x;
    r.j = q.y;
    r.idxA = a.idx;
    r.idxB = p64 ? p64[q.y].idx : p32[q.y].idx;
    out[t] = r;
}

__global__ void k_add_counts(const uint32_t *__restrict__ rows, uint32_t n, uint32_t *cnt)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) atomicAdd(&cnt[rows[t]], 1u);
}

__global__ void k_nonzero(const uint32_t *__restrict__ cnt, int64_t n, uint32_t *__restrict__ f)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) f[t] = cnt[t] ? 1u : 0u;
}

__global__ void k_best_pairs(int64_t n, int64_t P, const int64_t *__restrict__ off,
                             const int32_t *__restrict__ bidx, const double *__restrict__ bsep,
                             int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                             double *__restrict__ os, uint32_t *__restrict__ err)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || bidx[t] < 0) return;
    int64_t p = off[t];
    if (p >= P || off[t + 1] != p + 1) {
        atomicOr(err, 8u);
        return;
    }
    oa[p] = (int32_t)t;
    ob[p] = bidx[t];
    os[p] = bsep[t];
}

// ---------------------------------------------------------------------------- canonical order

constexpr int kSegSmall = 32;
constexpr int kSegLds = 2048;

__global__ void k_seg_small(const int64_t *__restrict__ off, int64_t n, int32_t *__restrict__ ob,
                            double *__restrict__ os, uint32_t *__restrict__ big_n,
                            uint32_t *__restrict__ big, uint32_t big_cap)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int64_t o = off[t];
    int64_t len = off[t + 1] - o;
    if (len < 2) return;
    if (len > kSegSmall) {
        uint32_t s = atomicAdd(big_n, 1u);
        if (s < big_cap) big[s] = (uint32_t)t;
        return;
    }
    int32_t kb[kSegSmall];
    double ks[kSegSmall];
    for (int k = 0; k < len; ++k) {
        kb[k] = ob[o + k];
        ks[k] = os[o + k];
    }
    bool sorted = true;
    for (int k = 1; k < len; ++k) sorted &= kb[k - 1] < kb[k];
    if (sorted) return;
    for (int k = 1; k < len; ++k) {
        int32_t b = kb[k];
        double s = ks[k];
        int q = k - 1;
        while (q >= 0 && kb[q] > b) {
            kb[q + 1] = kb[q];
            ks[q + 1] = ks[q];
            --q;
        }
        kb[q + 1] = b;
        ks[q + 1] = s;
    }
    for (int k = 0; k < len; ++k) {
        ob[o + k] = kb[k];
        os[o + k] = ks[k];
    }
}

// One workgroup per segment of up to kSegLds pairs: bitonic sort in LDS.
__global__ __launch_bounds__(256) void k_seg_lds(const int64_t *__restrict__ off,
                                                 const uint32_t *__restrict__ big, uint32_t nbig,
                                                 int32_t *__restrict__ ob, double *__restrict__ os,
                                                 uint32_t *__restrict__ huge_n,
                                                 uint32_t *__restrict__ huge, uint32_t huge_cap)
{
    __shared__ uint32_t key[kSegLds];
    __shared__ uint32_t pos[kSegLds];
    __shared__ double sep[kSegLds];
    uint32_t a = big[blockIdx.x];
    int64_t o = off[a];
    int len = (int)(off[a + 1] - o);
    if (len > kSegLds) {
        if (threadIdx.x == 0) {
            uint32_t s = atomicAdd(huge_n, 1u);
            if (s < huge_cap) huge[s] = a;
        }
        return;
    }
    int p2 = 1;
    while (p2 < len) p2 <<= 1;
    for (int k = threadIdx.x; k < p2; k += blockDim.x) {
        key[k] = k < len ? (uint32_t)ob[o + k] : 0xffffffffu;
        pos[k] = (uint32_t)k;
        if (k < len) sep[k] = os[o + k];
    }
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int k = threadIdx.x; k < p2; k += blockDim.x) {
                int l = k ^ stride;
                if (l > k) {
                    bool up = (k & size) == 0;
                    uint32_t x = key[k], y = key[l];
                    if ((x > y) == up) {
                        key[k] = y;
                        key[l] = x;
                        uint32_t t = pos[k];
                        pos[k] = pos[l];
                        pos[l] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int k = threadIdx.x; k < len; k += blockDim.x) {
        ob[o + k] = (int32_t)key[k];
        os[o + k] = sep[pos[k]];
    }
}

__global__ void k_iota(uint32_t *v, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) v[t] = (uint32_t)t;
}

__global__ void k_permute_seg(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ pos,
                              const double *__restrict__ sin_, int64_t n, int32_t *__restrict__ ob,
                              double *__restrict__ os)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    ob[t] = (int32_t)keys[t];
    os[t] = sin_[pos[t]];
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Sorts every A segment of (ob, os) by idxB.
static c3x_status order_segments(const int64_t *off, int64_t nA, int32_t *ob, double *os,
                                 hipStream_t s, double &ms)
{
    if (nA == 0) return C3X_OK;
    Arena tmp(s);
    uint32_t cap = (uint32_t)std::min<int64_t>(std::max<int64_t>(nA, 1), 1 << 22);
    uint32_t *cnt = tmp.get_n<uint32_t>(2);
    uint32_t *big = tmp.get_n<uint32_t>(cap);
    uint32_t *huge = tmp.get_n<uint32_t>(cap);
    if (!cnt || !big || !huge) return fail(C3X_ENOMEM, "segment order buffers");
    hipError_t e = hipMemsetAsync(cnt, 0, 2 * sizeof(uint32_t), s);
    hipLaunchKernelGGL(k_seg_small, dim3(nblk(nA, 256)), dim3(256), 0, s, off, nA, ob, os, cnt,
                       big, cap);
    uint32_t h[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "segment order");
    if (h[0] > cap) return fail(C3X_ENOMEM, "too many long segments");
    if (h[0]) {
        hipLaunchKernelGGL(k_seg_lds, dim3(h[0]), dim3(256), 0, s, off, big, h[0], ob, os, cnt + 1,
                           huge, cap);
        e = hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail_hip(e, "segment order");
    }
    if (h[1]) {
        std::vector<uint32_t> hv(h[1]);
        e = hipMemcpy(hv.data(), huge, h[1] * sizeof(uint32_t), hipMemcpyDeviceToHost);
        std::vector<int64_t> offs(2);
        for (uint32_t k = 0; k < h[1] && e == hipSuccess; ++k) {
            e = hipMemcpy(offs.data(), off + hv[k], 2 * sizeof(int64_t), hipMemcpyDeviceToHost);
            if (e != hipSuccess) break;
            int64_t o = offs[0], len = offs[1] - offs[0];
            Arena t2(s);
            uint32_t *k1 = t2.get_n<uint32_t>(len), *v1 = t2.get_n<uint32_t>(len);
            uint32_t *k2 = t2.get_n<uint32_t>(len), *v2 = t2.get_n<uint32_t>(len);
            double *sv = t2.get_n<double>(len);
            void *ws = t2.get(radix_ws_bytes(len));
            if (!k1 || !v1 || !k2 || !v2 || !sv || !ws) return fail(C3X_ENOMEM, "segment sort");
            e = hipMemcpyAsync(k1, ob + o, len * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(sv, os + o, len * sizeof(double), hipMemcpyDeviceToDevice, s);
            hipLaunchKernelGGL(k_iota, dim3(nblk(len, 256)), dim3(256), 0, s, v1, len);
            int in_tmp = 0;
            if (e == hipSuccess) e = radix_sort_pairs(k1, v1, k2, v2, len, 31, ws, s, &in_tmp);
            if (e == hipSuccess)
                hipLaunchKernelGGL(k_permute_seg, dim3(nblk(len, 256)), dim3(256), 0, s,
                                   in_tmp ? k2 : k1, in_tmp ? v2 : v1, sv, len, ob + o, os + o);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        if (e != hipSuccess) return fail_hip(e, "segment order");
    }
    (void)ms;
    return C3X_OK;
}

// Margins of the circle filters on the squared chord (see the library notes):
// FP64 unit vectors carry <= 32 u per component; FP32 offsets from a cell
// reference carry 2^-24 of their size (<= L + c). Factor 4 of safety.
struct CircleThresholds {
    double cr2, h_r, t64_in, t64_out;
    float t32_in, t32_out;
};

static CircleThresholds circle_thresholds(double r_arcsec, double L)
{
    CircleThresholds t;
    c3x_q_thresholds(r_arcsec, &t.h_r, &t.cr2);
    const double s3 = 1.7320508075688772;
    double c = sqrt(t.cr2) * 1.5;
    double ev = 32.0 * kU;
    double eta = s3 * (2.0 * ev + kU * c);
    double err = 2.0 * c * eta + eta * eta + 3.0 * kU * (c + eta) * (c + eta);
    double M64 = 4.0 * err;
    if (r_arcsec == 0.0 || M64 > 0.25 * t.cr2) {
        t.t64_in = -1.0;
        t.t64_out = INFINITY;
    } else {
        t.t64_in = t.cr2 - M64;
        t.t64_out = t.cr2 + M64;
    }
    double e32 = kU32 * 1.0001;
    double eta32 = s3 * e32 * (2.0 * L + 2.0 * c) + 2.0 * s3 * ev;
    double err32 = 2.0 * c * eta32 + eta32 * eta32 + 3.0 * e32 * (c + eta32) * (c + eta32);
    double M32 = 4.0 * err32;
    if (r_arcsec == 0.0 || M32 > 0.25 * t.cr2) {
        t.t32_in = -1.0f;
        t.t32_out = INFINITY;
    } else {
        float lo = (float)(t.cr2 - M32), hi = (float)(t.cr2 + M32);
        if ((double)lo > t.cr2 - M32) lo = nextafterf(lo, -INFINITY);
        if ((double)hi < t.cr2 + M32) hi = nextafterf(hi, INFINITY);
        t.t32_in = lo;
        t.t32_out = hi;
    }
    return t;
}

template <int MODE>
static void launch_match(const MatchArgs &m, int shape, int prec, unsigned grid, hipStream_t s)
{
    if (grid == 0) return;
    if (shape == C3X_CIRCLE) {
        if (prec == C3X_FP64)
            hipLaunchKernelGGL((k_match<C3X_CIRCLE, C3X_FP64, MODE>), dim3(grid), dim3(kMatchBlock), 0,
                               s, m);
        else
            hipLaunchKernelGGL((k_match<C3X_CIRCLE, C3X_MIXED, MODE>), dim3(grid),
                               dim3(kMatchBlock), 0, s, m);
    } else {
        if (prec == C3X_FP64)
            hipLaunchKernelGGL((k_match<C3X_ELLIPSE, C3X_FP64, MODE>), dim3(grid),
                               dim3(kMatchBlock), 0, s, m);
        else
            hipLaunchKernelGGL((k_match<C3X_ELLIPSE, C3X_MIXED, MODE>), dim3(grid),
                               dim3(kMatchBlock), 0, s, m);
    }
}

}  // namespace c3x

using namespace c3x;

#define HIPCHK(expr, what)                       \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

static c3x_status match_impl(const c3x_index *ix, const double *ra, const double *dec, int64_t nA,
                             const c3x_area *area, unsigned mode, hipStream_t s, c3x_result *R)
{
    const int shape = area->shape;
    const int prec = ix->precision;
    Timer tm(s);
    tm.mark();  // 0
    Arena tmp(s);
    // ---- A preparation
    uint32_t *keys = tmp.get_n<uint32_t>(nA), *rows = tmp.get_n<uint32_t>(nA);
    uint32_t *ktmp = tmp.get_n<uint32_t>(nA), *rtmp = tmp.get_n<uint32_t>(nA);
    void *ws = tmp.get(std::max(radix_ws_bytes(nA), scan_ws_bytes(nA + 1)));
    uint32_t *ctr = tmp.get_n<uint32_t>(8);  // bad, amb_n, tie_n, col_n, err
    unsigned long long *c64 = tmp.get_n<unsigned long long>(2);
    ARec *arec = tmp.get_n<ARec>(nA);
    AEll *aell = nullptr;
    AEllR *aellr = nullptr;
    if (shape == C3X_ELLIPSE) {
        aell = tmp.get_n<AEll>(nA);
        aellr = tmp.get_n<AEllR>(nA);
        if (!aell || !aellr) return fail(C3X_ENOMEM, "A buffers");
    }
    if (!keys || !rows || !ktmp || !rtmp || !ws || !ctr || !c64 || !arec)
        return fail(C3X_ENOMEM, "A buffers");
    HIPCHK(hipMemsetAsync(ctr, 0, 8 * sizeof(uint32_t), s), "memset");
    HIPCHK(hipMemsetAsync(ctr, 0xff, sizeof(uint32_t), s), "memset");
    HIPCHK(hipMemsetAsync(c64, 0, 2 * sizeof(unsigned long long), s), "memset");
    const double *sa = area->semi_major_arcsec, *sb = area->semi_minor_arcsec, *pa = area->pa_deg;
    if (nA > 0)
        hipLaunchKernelGGL(k_prep_a, dim3(nblk(nA, 256)), dim3(256), 0, s, ra, dec, nA, ix->grid,
                           shape, sa, sb, pa, keys, rows, ctr);
    HIPCHK(hipGetLastError(), "A keys");
    int in_tmp = 0;
    HIPCHK(radix_sort_pairs(keys, rows, ktmp, rtmp, nA, ix->plan.key_bits, ws, s, &in_tmp), "A sort");
    uint32_t *srows = in_tmp ? rtmp : rows;
    if (nA > 0) {
        if (shape == C3X_CIRCLE)
            hipLaunchKernelGGL(k_gather_a<C3X_CIRCLE>, dim3(nblk(nA, 256)), dim3(256), 0, s, srows,
                               ra, dec, nA, area->radius_arcsec, sa, sb, pa, area->pa_zero_deg,
                               area->pa_sense, ix->plan.L_rad, arec, aell, aellr);
        else
            hipLaunchKernelGGL(k_gather_a<C3X_ELLIPSE>, dim3(nblk(nA, 256)), dim3(256), 0, s,
                               srows, ra, dec, nA, area->radius_arcsec, sa, sb, pa,
                               area->pa_zero_deg, area->pa_sense, ix->plan.L_rad, arec, aell,
                               aellr);
    }
    HIPCHK(hipGetLastError(), "A records");
    uint32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, ctr, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(hipStreamSynchronize(s), "A preparation");
    if (bad != 0xffffffffu)
        return fail(C3X_EINVAL,
                    "catalogue A row %u: coordinate outside RA [0,360), |Dec| <= 90, not finite, "
                    "or ellipse axes outside 1e-6 <= b <= a <= 324000 arcsec, a <= 1000 b",
                    bad);
    tm.mark();  // 1

    // ---- thresholds and common arguments
    MatchArgs m;
    memset(&m, 0, sizeof(m));
    m.g = ix->grid;
    m.pay64 = ix->pay64;
    m.pay32 = ix->pay32;
    m.radecB = ix->radec;
    m.arec = arec;
    m.aell = aell;
    m.aellr = aellr;
    m.nA = (int32_t)nA;
    if (shape == C3X_CIRCLE) {
        CircleThresholds t = circle_thresholds(area->radius_arcsec, ix->plan.L_rad);
        m.cr2 = t.cr2;
        m.h_r = t.h_r;
        m.t64_in = t.t64_in;
        m.t64_out = t.t64_out;
        m.t32_in = t.t32_in;
        m.t32_out = t.t32_out;
        m.r_zero = area->radius_arcsec == 0.0;
    }
    m.n_tests = c64;
    m.n_band = c64 + 1;
    m.err_flag = ctr + 4;
    unsigned grid = nblk(nA, kMatchBlock);

    // ---- count pass
    uint32_t *cnt = tmp.get_n<uint32_t>(nA);
    uint32_t amb_cap = (uint32_t)std::max<int64_t>(4096, nA / 256);
    uint2 *amb = tmp.get_n<uint2>(amb_cap);
    if (!cnt || !amb) return fail(C3X_ENOMEM, "count buffers");
    m.cnt = cnt;
    m.amb_n = ctr + 1;
    m.amb = amb;
    m.amb_cap = amb_cap;
    uint32_t hctr[8];
    unsigned long long h64[2];
    for (int attempt = 0; attempt < 2; ++attempt) {
        launch_match<0>(m, shape, prec, grid, s);
        HIPCHK(hipGetLastError(), "count pass");
        HIPCHK(hipMemcpyAsync(hctr, ctr, sizeof(hctr), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(hipMemcpyAsync(h64, c64, sizeof(h64), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(hipStreamSynchronize(s), "count pass");
        if (hctr[1] <= amb_cap) break;
        // the ambiguous list overflowed: grow it and count again
        amb_cap = hctr[1];
        amb = tmp.get_n<uint2>(amb_cap);
        if (!amb) return fail(C3X_ENOMEM, "ambiguous list");
        m.amb = amb;
        m.amb_cap = amb_cap;
        HIPCHK(hipMemsetAsync(ctr + 1, 0, sizeof(uint32_t), s), "memset");
        HIPCHK(hipMemsetAsync(c64, 0, 2 * sizeof(unsigned long long), s), "memset");
    }
    uint32_t n_amb = hctr[1];
    R->stats.n_tests = (int64_t)h64[0];
    R->stats.n_band = (int64_t)h64[1];
    R->stats.n_ambiguous = n_amb;
    tm.mark();  // 2

    // ---- host decisions of the ambiguous pairs
    if (n_amb > 0) {
        AmbInfo *dinfo = tmp.get_n<AmbInfo>(n_amb);
        if (!dinfo) return fail(C3X_ENOMEM, "ambiguous info");
        hipLaunchKernelGGL(k_amb_info, dim3(nblk(n_amb, 256)), dim3(256), 0, s, amb, n_amb, arec,
                           ix->radec, ix->pay64, ix->pay32, shape == C3X_ELLIPSE ? sa : nullptr,
                           shape == C3X_ELLIPSE ? sb : nullptr, shape == C3X_ELLIPSE ? pa : nullptr,
                           dinfo);
        std::vector<AmbInfo> info(n_amb);
        HIPCHK(hipMemcpyAsync(info.data(), dinfo, n_amb * sizeof(AmbInfo), hipMemcpyDeviceToHost, s),
               "copy");
        HIPCHK(hipStreamSynchronize(s), "ambiguous info");
        std::vector<std::pair<unsigned long long, uint8_t>> ver(n_amb);
        std::vector<uint32_t> add;
        for (uint32_t k = 0; k < n_amb; ++k) {
            const AmbInfo &q = info[k];
            int in = shape == C3X_CIRCLE
                         ? c3x_q_circle(q.raA, q.decA, q.raB, q.decB, area->radius_arcsec)
                         : c3x_q_ellipse(q.raA, q.decA, q.raB, q.decB, q.a, q.b, q.pa,
                                         area->pa_zero_deg, area->pa_sense);
            ver[k] = {((unsigned long long)q.i << 32) | q.j, (uint8_t)(in ? 1 : 0)};
            if (in) add.push_back(q.idxA);
        }
        std::sort(ver.begin(), ver.end());
        std::vector<unsigned long long> vk(n_amb);
        std::vector<uint8_t> vi(n_amb);
        for (uint32_t k = 0; k < n_amb; ++k) {
            vk[k] = ver[k].first;
            vi[k] = ver[k].second;
        }
        unsigned long long *dvk = tmp.get_n<unsigned long long>(n_amb);
        uint8_t *dvi = tmp.get_n<uint8_t>(n_amb);
        uint32_t *dadd = tmp.get_n<uint32_t>(add.size());
        if (!dvk || !dvi || !dadd) return fail(C3X_ENOMEM, "verdict table");
        HIPCHK(hipMemcpyAsync(dvk, vk.data(), n_amb * 8, hipMemcpyHostToDevice, s), "copy");
        HIPCHK(hipMemcpyAsync(dvi, vi.data(), n_amb, hipMemcpyHostToDevice, s), "copy");
        if (!add.empty()) {
            HIPCHK(hipMemcpyAsync(dadd, add.data(), add.size() * 4, hipMemcpyHostToDevice, s), "copy");
            hipLaunchKernelGGL(k_add_counts, dim3(nblk(add.size(), 256)), dim3(256), 0, s, dadd,
                               (uint32_t)add.size(), cnt);
        }
        m.ver_key = dvk;
        m.ver_in = dvi;
        m.n_ver = n_amb;
        HIPCHK(hipStreamSynchronize(s), "verdict upload");  // host vectors go out of scope
    }

    // ---- scan of the per-A counts (idxA order)
    const bool all = (mode & C3X_ALL) != 0;
    int64_t *off = tmp.get_n<int64_t>(nA + 1);
    if (!off) return fail(C3X_ENOMEM, "offsets");
    const uint32_t *scan_in = cnt;
    if (!all) {
        uint32_t *f = tmp.get_n<uint32_t>(nA);
        if (!f) return fail(C3X_ENOMEM, "offsets");
        if (nA > 0)
            hipLaunchKernelGGL(k_nonzero, dim3(nblk(nA, 256)), dim3(256), 0, s, cnt, nA, f);
        scan_in = f;
    }
    HIPCHK(scan_u32_to_i64(scan_in, off, nA, off + nA, ws, s), "scan");
    int64_t P = 0;
    HIPCHK(hipMemcpyAsync(&P, off + nA, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(hipStreamSynchronize(s), "scan");
    tm.mark();  // 3

    // ---- outputs
    R->n_pairs = P;
    R->nA = nA;
    R->idxA = R->mem.get_n<int32_t>(P);
    R->idxB = R->mem.get_n<int32_t>(P);
    R->sep = R->mem.get_n<double>(P);
    R->best_idx = R->mem.get_n<int32_t>(nA);
    R->best_sep = R->mem.get_n<double>(nA);
    if (!R->idxA || !R->idxB || !R->sep || !R->best_idx || !R->best_sep)
        return fail(C3X_ENOMEM, "result buffers (%lld pairs)", (long long)P);

    // ---- write pass
    uint32_t tie_cap = (uint32_t)std::max<int64_t>(4096, nA / 256);
    TieEnt *tie = (TieEnt *)tmp.get(tie_cap * sizeof(TieEnt));
    if (!tie) return fail(C3X_ENOMEM, "tie list");
    m.off = all ? off : nullptr;
    m.write_pairs = all ? 1 : 0;
    m.out_a = R->idxA;
    m.out_b = R->idxB;
    m.out_sep = R->sep;
    m.best_idx = R->best_idx;
    m.best_sep = R->best_sep;
    m.tie_n = ctr + 2;
    m.tie = (uint2 *)tie;
    m.tie_cap = tie_cap;
    if (!all) {
        // offsets are not used by the write pass in this mode
        m.off = off;
    }
    launch_match<1>(m, shape, prec, grid, s);
    HIPCHK(hipGetLastError(), "write pass");
    HIPCHK(hipMemcpyAsync(hctr, ctr, sizeof(hctr), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(hipStreamSynchronize(s), "write pass");
    tm.mark();  // 4
    if (hctr[4] & (all ? 7u : 4u))
        return fail(C3X_EDEVICE, "internal: count and write passes disagree (flags %u)", hctr[4]);
    uint32_t n_tie = hctr[2];

    // ---- best matches closer than the FP64 separation can rank: binary128
    if ((mode & C3X_BEST) && n_tie > 0) {
        if (n_tie > tie_cap) {
            // rerun the write pass with room for every near-tie
            tie_cap = n_tie;
            tie = (TieEnt *)tmp.get(tie_cap * sizeof(TieEnt));
            if (!tie) return fail(C3X_ENOMEM, "tie list");
            m.tie = (uint2 *)tie;
            m.tie_cap = tie_cap;
            HIPCHK(hipMemsetAsync(ctr + 2, 0, sizeof(uint32_t), s), "memset");
            launch_match<1>(m, shape, prec, grid, s);
            HIPCHK(hipGetLastError(), "write pass");
        }
        std::vector<TieEnt> ties(n_tie);
        HIPCHK(hipMemcpyAsync(ties.data(), tie, n_tie * sizeof(TieEnt), hipMemcpyDeviceToHost, s),
               "copy");
        HIPCHK(hipStreamSynchronize(s), "ties");
        std::vector<uint32_t> cpos(n_tie);
        std::vector<double> clim(n_tie);
        for (uint32_t k = 0; k < n_tie; ++k) {
            cpos[k] = ties[k].i;
            clim[k] = ties[k].s1 * (1.0 + 2.0 * kTieRel) + 1e-300;
        }
        uint32_t *dpos = tmp.get_n<uint32_t>(n_tie);
        double *dlim = tmp.get_n<double>(n_tie);
        if (!dpos || !dlim) return fail(C3X_ENOMEM, "tie buffers");
        HIPCHK(hipMemcpyAsync(dpos, cpos.data(), n_tie * 4, hipMemcpyHostToDevice, s), "copy");
        HIPCHK(hipMemcpyAsync(dlim, clim.data(), n_tie * 8, hipMemcpyHostToDevice, s), "copy");
        uint32_t col_cap = 4 * n_tie + 64;
        std::vector<ColEnt> col;
        for (int attempt = 0; attempt < 2; ++attempt) {
            ColEnt *dcol = (ColEnt *)tmp.get(col_cap * sizeof(ColEnt));
            if (!dcol) return fail(C3X_ENOMEM, "tie candidates");
            HIPCHK(hipMemsetAsync(ctr + 3, 0, sizeof(uint32_t), s), "memset");
            m.col_pos = dpos;
            m.col_lim = dlim;
            m.n_col = n_tie;
            m.col_n = ctr + 3;
            m.col = (uint4 *)dcol;
            m.col_cap = col_cap;
            launch_match<2>(m, shape, prec, nblk(n_tie, kMatchBlock), s);
            HIPCHK(hipGetLastError(), "collect pass");
            uint32_t ncol = 0;
            HIPCHK(hipMemcpyAsync(&ncol, ctr + 3, 4, hipMemcpyDeviceToHost, s), "copy");
            HIPCHK(hipStreamSynchronize(s), "collect pass");
            if (ncol > col_cap) {
                col_cap = ncol;
                continue;
            }
            col.resize(ncol);
            HIPCHK(hipMemcpy(col.data(), dcol, ncol * sizeof(ColEnt), hipMemcpyDeviceToHost), "copy");
            break;
        }
        std::vector<std::vector<const ColEnt *>> per(n_tie);
        for (const ColEnt &c : col) per[c.t].push_back(&c);
        std::vector<ARec> ar(1);
        for (uint32_t k = 0; k < n_tie; ++k) {
            auto &v = per[k];
            if (v.size() < 2) continue;
            HIPCHK(hipMemcpy(ar.data(), arec + ties[k].i, sizeof(ARec), hipMemcpyDeviceToHost), "copy");
            std::vector<double> r2(v.size()), d2(v.size());
            std::vector<int32_t> ib(v.size());
            for (size_t q = 0; q < v.size(); ++q) {
                r2[q] = v[q]->ra;
                d2[q] = v[q]->dec;
                ib[q] = (int32_t)v[q]->idxB;
            }
            int w = c3x_q_best(ar[0].ra, ar[0].dec, (int)v.size(), r2.data(), d2.data(), ib.data());
            int32_t bi = ib[w];
            double bs = v[w]->sep;
            uint32_t ia = ties[k].idxA;
            HIPCHK(hipMemcpy(R->best_idx + ia, &bi, sizeof(int32_t), hipMemcpyHostToDevice), "copy");
            HIPCHK(hipMemcpy(R->best_sep + ia, &bs, sizeof(double), hipMemcpyHostToDevice), "copy");
        }
        R->stats.n_best_ties = n_tie;
    }
    tm.mark();  // 5

    // ---- canonical order / best-only pairs
    if (all) {
        double ms = 0;
        c3x_status st = order_segments(off, nA, R->idxB, R->sep, s, ms);
        if (st != C3X_OK) return st;
    } else if (nA > 0) {
        hipLaunchKernelGGL(k_best_pairs, dim3(nblk(nA, 256)), dim3(256), 0, s, nA, P, off,
                           R->best_idx, R->best_sep, R->idxA, R->idxB, R->sep, ctr + 4);
        HIPCHK(hipGetLastError(), "best pairs");
    }
    tm.mark();  // 6
    HIPCHK(hipMemcpyAsync(hctr, ctr, sizeof(hctr), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(hipStreamSynchronize(s), "c3x_match");
    if (hctr[4]) return fail(C3X_EDEVICE, "internal: inconsistent best-match output (%u)", hctr[4]);
    c3x_stats &S = R->stats;
    S.n_a = nA;
    S.n_b = ix->nB;
    S.n_pairs = P;
    S.n_cells = (int64_t)ix->plan.ncells;
    S.cell_arcsec = ix->plan.cell_arcsec;
    S.ms_a_prep = tm.ms(0, 1);
    S.ms_count = tm.ms(1, 2);
    S.ms_scan = tm.ms(2, 3);
    S.ms_write = tm.ms(3, 4);
    S.ms_sort_pairs = tm.ms(5, 6);
    S.ms_total = tm.ms(0, 6);
    S.precision = prec;
    S.tile = kMatchBlock;
    return C3X_OK;
}

extern "C" c3x_status c3x_match(const c3x_index *ix, const double *ra_deg, const double *dec_deg,
                                int64_t nA, c3x_frame frame, const c3x_area *area, unsigned mode,
                                const c3x_opts *opts, c3x_result **out)
{
    clear_error();
    if (!out) return fail(C3X_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ix || !area) return fail(C3X_EINVAL, "NULL index or area");
    if (nA < 0) return fail(C3X_EINVAL, "nA < 0");
    if (nA > 2147483647LL) return fail(C3X_ERANGE, "nA above 2^31 - 1");
    if (nA > 0 && (!ra_deg || !dec_deg)) return fail(C3X_EINVAL, "NULL coordinate array");
    if (frame != C3X_EQUATORIAL && frame != C3X_GALACTIC) return fail(C3X_EINVAL, "bad frame");
    if (frame != ix->frame) return fail(C3X_EFRAME, "catalogue A frame differs from the index's");
    if (mode == 0 || (mode & ~(unsigned)(C3X_ALL | C3X_BEST)))
        return fail(C3X_EINVAL, "mode must be C3X_ALL, C3X_BEST or both");
    if (area->shape == C3X_CIRCLE) {
        double r = area->radius_arcsec;
        if (!(r == 0.0 || (r >= 1e-6 && r <= 324000.0)))
            return fail(C3X_EINVAL, "radius must be 0 or in [1e-6, 324000] arcsec");
    } else if (area->shape == C3X_ELLIPSE) {
        if (nA > 0 && (!area->semi_major_arcsec || !area->semi_minor_arcsec || !area->pa_deg))
            return fail(C3X_EINVAL, "ellipse parameter arrays are NULL");
        if (!isfinite(area->pa_zero_deg)) return fail(C3X_EINVAL, "pa_zero_deg not finite");
        if (area->pa_sense != 1 && area->pa_sense != -1)
            return fail(C3X_EINVAL, "pa_sense must be +1 or -1");
    } else {
        return fail(C3X_EINVAL, "bad shape");
    }
    if (opts && opts->precision != ix->precision)
        return fail(C3X_EINVAL, "precision differs from the index's");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    c3x_result *R = new (std::nothrow) c3x_result();
    if (!R) return fail(C3X_ENOMEM, "host allocation");
    (void)hipGetDevice(&R->device);
    memset(&R->stats, 0, sizeof(R->stats));
    R->mode = mode;
    c3x_status st = match_impl(ix, ra_deg, dec_deg, nA, area, mode, s, R);
    if (st != C3X_OK) {
        (void)hipStreamSynchronize(s);
        delete R;
        return st;
    }
    *out = R;
    return C3X_OK;
}

extern "C" c3x_status c3x_result_sizes(const c3x_result *r, int64_t *n_pairs, int64_t *nA)
{
    if (!r) return fail(C3X_EINVAL, "NULL result");
    if (n_pairs) *n_pairs = r->n_pairs;
    if (nA) *nA = r->nA;
    return C3X_OK;
}

extern "C" c3x_status c3x_result_copy(const c3x_result *r, int32_t *idxA, int32_t *idxB,
                                      double *sep_arcsec, int32_t *best_idxB,
                                      double *best_sep_arcsec, void *stream)
{
    if (!r) return fail(C3X_EINVAL, "NULL result");
    hipStream_t s = (hipStream_t)stream;
    size_t P = (size_t)r->n_pairs, n = (size_t)r->nA;
    if (idxA && P) HIPCHK(hipMemcpyAsync(idxA, r->idxA, P * 4, hipMemcpyDefault, s), "copy");
    if (idxB && P) HIPCHK(hipMemcpyAsync(idxB, r->idxB, P * 4, hipMemcpyDefault, s), "copy");
    if (sep_arcsec && P)
        HIPCHK(hipMemcpyAsync(sep_arcsec, r->sep, P * 8, hipMemcpyDefault, s), "copy");
    if (best_idxB && n)
        HIPCHK(hipMemcpyAsync(best_idxB, r->best_idx, n * 4, hipMemcpyDefault, s), "copy");
    if (best_sep_arcsec && n)
        HIPCHK(hipMemcpyAsync(best_sep_arcsec, r->best_sep, n * 8, hipMemcpyDefault, s), "copy");
    HIPCHK(hipStreamSynchronize(s), "c3x_result_copy");
    return C3X_OK;
}

extern "C" c3x_status c3x_result_stats(const c3x_result *r, c3x_stats *st)
{
    if (!r || !st) return fail(C3X_EINVAL, "NULL argument");
    *st = r->stats;
    return C3X_OK;
}

extern "C" void c3x_result_free(c3x_result *r) { delete r; }
