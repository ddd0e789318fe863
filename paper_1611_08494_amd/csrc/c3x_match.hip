// c3x_match.hip -- cross-match of catalogue A against a sky index.
//
// Paper Section 2.1 ("Sky" case): a region is centred on each A source and
// the B sources inside it are found by comparing their distance from the
// central object with the limits of the area; Section 2.2: the matches are
// kept as rows, all of them or only the best; Section 2.3: each source is
// tested only against the cells around it. Phases on one stream:
//   A prep     validate, key, sort A by cell (LDS radix sort), sorted
//              coordinates (+ ellipse frames)
//   count      wavefront tiles of 64 consecutive sorted A sources: per zone,
//              the union of the lanes' cell windows is one key range of B,
//              found with two directory lookups and staged through LDS; each
//              lane binary-searches its own cells in LDS and decides its
//              candidates with the certified filter; candidates inside the
//              filter's error band are listed. Counts and the best match go
//              to idxA order.
//   recheck    one thread per listed candidate: FP64 relative-accuracy form;
//              what it cannot certify is decided on the host in binary128
//   [host]     verdict table; near-tie best matches re-ranked in binary128
//              from a collect pass
//   scan       counts -> int64 offsets (idxA order)
//   write      same tiles and decisions; each lane writes (idxB, B position)
//              into its own idxA segment
//   finalize   one thread per pair: rank inside its segment by idxB
//              (canonical order), separation in FP64, final write
//   best       one thread per A: separation of the best match
// Decisions of the count, write and collect passes come from one device
// function compiled with -ffp-contract=off, so they agree bit for bit.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <type_traits>
#include <vector>

#include "c3x_host.h"
#include "c3x_sort.h"

namespace c3x {

constexpr int kMatchBlock = 256;
constexpr int kWavesPerBlock = kMatchBlock / 64;
constexpr int kShortSeg = 16;   // segments up to this long are ordered by the finalize kernel
constexpr int kSegLds = 2048;   // segments up to this long are sorted in LDS
constexpr int kTileZones = 5;   // zones a cooperative tile may span; wider tiles go per lane
static_assert(6 * kTileZones <= 64, "one lane per hull end");

struct alignas(16) ColEnt {
    uint32_t t, idxB, j, pad;
    double ra, dec;
};
struct AmbInfo {
    double raA, decA, raB, decB, a, b, pa;
    uint32_t i, j, idxA, idxB;
};

template <int PREC>
using PayOf = typename std::conditional<PREC == C3X_FP64, Pay64, Pay32>::type;

// ---------------------------------------------------------------------------- A preparation

__global__ void k_prep_a(const double *__restrict__ ra, const double *__restrict__ dec, int64_t n,
                         Grid g, int shape, const double *__restrict__ sa,
                         const double *__restrict__ sb, const double *__restrict__ pa,
                         uint32_t *__restrict__ keys, uint32_t *__restrict__ rows,
                         double2 *__restrict__ packed, uint32_t *__restrict__ bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = ra[i], d = dec[i];
    packed[i] = make_double2(a, d);  // one 16-byte record per row for the gather
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
    const ZoneInfo zi = g.zinfo[z];
    keys[i] = zi.base + cell_in(zi, a);
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

// Invalid rows (already reported through k_prep_a's flag) are given the
// position (0, 0) and, for ellipses, a 1" circle, so every later loop stays
// bounded even before the host sees the error.
template <int SHAPE>
__global__ void k_gather_a(const uint32_t *__restrict__ rows, const double2 *__restrict__ packed,
                           int64_t n,
                           const double *__restrict__ sa, const double *__restrict__ sb,
                           const double *__restrict__ pa, double pa_zero, int pa_sense,
                           double L_rad, double2 *__restrict__ arad, uint32_t *__restrict__ aidx,
                           AEll *__restrict__ aell, AEllR *__restrict__ aellr)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t row = rows[i];
    if (row >= (uint64_t)n) row = 0;  // unreachable for a permutation; keeps reads in bounds
    const double2 rd = packed[row];
    double r = rd.x, d = rd.y;
    bool ok = isfinite(r) && isfinite(d) && r >= 0.0 && r < 360.0 && fabs(d) <= 90.0;
    double A = 1.0, B = 1.0, P = 0.0;
    if (SHAPE == C3X_ELLIPSE) {
        A = sa[row];
        B = sb[row];
        P = pa[row];
        ok = ok && isfinite(A) && isfinite(B) && isfinite(P) && B >= 1e-6 && B <= A &&
             A <= 324000.0 && A <= 1000.0 * B;
    }
    if (!ok) {
        r = 0.0;
        d = 0.0;
        A = 1.0;
        B = 1.0;
        P = 0.0;
    }
    arad[i] = make_double2(r, d);
    aidx[i] = row;
    if (SHAPE == C3X_ELLIPSE) {
        double T = pa_zero + (double)pa_sense * P;
        double st, ct;
        sincos(T * kDeg, &st, &ct);
        double sdd, cdd, sra, cra;
        sincos(d * kDeg, &sdd, &cdd);
        sincos(r * kDeg, &sra, &cra);
        // local north and east at A
        double nx = -sdd * cra, ny = -sdd * sra, nz = cos_dec_acc(d);
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

// ---------------------------------------------------------------------------- decisions

// A lane's source. cosd here is only a lower bound of cos Dec for the
// window (from the unit vector, no extra trigonometry); the recheck kernel
// rebuilds the source with the accurate cos Dec.
__device__ __forceinline__ ARec load_a(const MatchArgs &m, uint32_t i, double reach_deg)
{
    ARec a;
    double2 rd = m.arad[i];
    a.ra = rd.x;
    a.dec = rd.y;
    unit_vec(a.ra, a.dec, a.x, a.y, a.z);
    a.cosd = sqrt(a.x * a.x + a.y * a.y) * (1.0 - 1e-12) - 1e-15;
    a.reach_deg = reach_deg;
    a.idx = m.aidx[i];
    a.pad = 0;
    return a;
}

struct LaneF32 {            // FP32 copies of the ellipse frame
    float ux, uy, uz, vx, vy, vz, ia, ib;
};

struct CellCache {          // A's offset from the reference of the current B cell
    uint32_t key;
    float ax, ay, az;
};

// Fast certified filter of one candidate: IN, OUT, or AMBIG when the pair
// lies inside the filter's error band (then the FP64 relative-accuracy
// recheck decides it, in k_recheck). Also returns the filter's squared chord.
// Radius 0 is decided structurally here (same point), without a band.
template <int SHAPE, int PREC>
__device__ __forceinline__ int decide(const MatchArgs &m, const ARec &a, const AEll &e,
                                      const AEllR &er, const LaneF32 &f, CellCache &cc, int z,
                                      uint32_t key, const PayOf<PREC> &b, uint32_t j, double &c2o)
{
    int d;
    if constexpr (PREC == C3X_FP64) {
        double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
        double c2 = fma(dx, dx, fma(dy, dy, dz * dz));
        c2o = c2;
        if constexpr (SHAPE == C3X_CIRCLE) {
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
        if (key != cc.key) {
            cc.key = key;
            double rx, ry, rz;
            cell_ref(z, key - m.g.zinfo[z].base, m.g, rx, ry, rz);
            cc.ax = (float)(a.x - rx);
            cc.ay = (float)(a.y - ry);
            cc.az = (float)(a.z - rz);
        }
        float dx = b.x - cc.ax, dy = b.y - cc.ay, dz = b.z - cc.az;
        float c2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        c2o = (double)c2;
        if constexpr (SHAPE == C3X_CIRCLE) {
            d = c2 <= m.t32_in ? IN : (c2 > m.t32_out ? OUT : AMBIG);
        } else {
            float su = fmaf(dx, f.ux, fmaf(dy, f.uy, dz * f.uz));
            float sv = fmaf(dx, f.vx, fmaf(dy, f.vy, dz * f.vz));
            float xu = su * f.ia, xv = sv * f.ib;
            float q = fmaf(xu, xu, xv * xv);
            float qf = q * fmaf(c2, 1.0f / 3.0f, 1.0f);
            float mm = er.m32;
            d = mm == 0.0f ? AMBIG : (qf <= 1.0f - mm ? IN : (qf > 1.0f + mm ? OUT : AMBIG));
        }
    }
    if constexpr (SHAPE == C3X_CIRCLE) {
        if (m.r_zero) d = same_point(a, m.radecB[j]) ? IN : OUT;
    }
    return d;
}

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

// Error bound of the filter's squared chord at chord c (see circle_thresholds).
template <int PREC>
__device__ __forceinline__ double c2_err(double c, double L)
{
    const double s3 = 1.7320508075688772;
    if constexpr (PREC == C3X_FP64) {
        double eta = s3 * (64.0 * kU + kU * c);
        return 2.0 * c * eta + eta * eta + 3.0 * kU * (c + eta) * (c + eta);
    } else {
        const double e32 = kU32 * 1.0001;
        double eta = s3 * e32 * (2.0 * L + 2.0 * c) + 2.0 * s3 * 32.0 * kU;
        return 2.0 * c * eta + eta * eta + 3.0 * e32 * (c + eta) * (c + eta);
    }
}

__device__ __forceinline__ uint32_t lds_lower_bound(const uint32_t *k, uint32_t n, uint32_t v)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (k[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------- count / write

// A match's separation as the match passes leave it, without trigonometry:
// from the FP64 chord c < 1.38 the code -c^2 (the separation is 2 asin(c / 2),
// error ~1e-14 rad), 0 for c = 0, otherwise NaN (computed later from the
// coordinates).
__device__ __forceinline__ double sep_code(double c2)
{
    if (c2 < 1.9) return c2 > 0.0 ? -c2 : 0.0;
    return NAN;
}

__device__ __forceinline__ double sep_from_chord2(double c2)
{
    return 2.0 * asin(0.5 * sqrt(c2)) * (180.0 / kPi * 3600.0);
}

// MODE 0: count + best; MODE 1: write every filter match into the
// offsets from the count; MODE 2: count + best, each filter match written
// to its row's table slot (the first kTab) or to the overflow list.
template <int SHAPE, int PREC, int MODE>
__global__ __launch_bounds__(kMatchBlock) void k_match(MatchArgs m)
{
    using PayT = PayOf<PREC>;
    constexpr int kStage = PREC == C3X_FP64 ? 192 : 256;  // B staged per wavefront
    __shared__ uint32_t s_key[kWavesPerBlock][kStage];
    __shared__ PayT s_pay[kWavesPerBlock][kStage];
    __shared__ unsigned long long s_tests, s_band, s_placed;
    if (threadIdx.x == 0) {
        s_tests = 0;
        s_band = 0;
        s_placed = 0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const PayT *pay;
    if constexpr (PREC == C3X_FP64) pay = m.pay64;
    else pay = m.pay32;
    uint32_t *sk = s_key[wave];
    PayT *sp = s_pay[wave];

    const uint32_t i = blockIdx.x * kMatchBlock + threadIdx.x;
    const bool active = i < (uint32_t)m.nA;
    ARec a{};
    AEll e{};
    AEllR er{};
    LaneF32 f{};
    Window w{0, -1, false, 0.0};
    if (active) {
        double reach = m.reach_deg;
        if constexpr (SHAPE == C3X_ELLIPSE) {
            e = m.aell[i];
            er = m.aellr[i];
            reach = er.a_arcsec / 3600.0;
            f = LaneF32{(float)e.ux, (float)e.uy, (float)e.uz, (float)e.vx,
                        (float)e.vy, (float)e.vz, (float)e.ia, (float)e.ib};
        }
        a = load_a(m, i, reach);
        w = window_of(m.g, a.dec, a.cosd, a.reach_deg);
    }
    uint32_t zlo_all = wave_min_u32(active ? (uint32_t)w.zlo : 0xffffffffu);
    uint32_t zhi_all = wave_max_u32(active ? (uint32_t)w.zhi : 0u);

    uint32_t cnt = 0;
    double b1 = INFINITY, b2 = INFINITY;
    uint32_t bidx = 0xffffffffu, bj = 0;
    int64_t o = 0, oe = 0;
    if (MODE == 1 && active) {
        o = m.off[a.idx];
        oe = o + m.astat[a.idx].nf;  // band matches are placed separately
    }
    unsigned long long tests = 0, band = 0, placed = 0;
    CellCache cc{0xffffffffu, 0.f, 0.f, 0.f};

    // A filter match as written: the separation coded from the FP64 chord
    // (the FP64 path's filter chord; the mixed path recomputes it from the
    // FP64 unit vectors).
    auto coded = [&](const PayT &b, uint32_t j, double c2) -> PairTmp {
        double c64 = c2;
        if constexpr (PREC != C3X_FP64) {
            const Pay64 b8 = m.pay64[j];
            const double dx = b8.x - a.x, dy = b8.y - a.y, dz = b8.z - a.z;
            c64 = fma(dx, dx, fma(dy, dy, dz * dz));
        }
        PairTmp t;
        t.idxB = b.idx;
        t.j = j;
        t.sep = sep_code(c64);
        return t;
    };

    // The k-th filter match of this lane's row beyond its table slots:
    // appended to the block's region of the overflow list, one atomic per
    // group of lanes calling together (possibly inside divergent loops).
    auto overflow = [&](uint32_t k, const PairTmp &t) {
        const unsigned long long hm = __ballot(1);
        const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(hm >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)hm, 0u));
        const uint32_t pool = blockIdx.x & (kEmitPools - 1);
        uint32_t base = 0;
        if (r == 0) base = atomicAdd(m.octr + pool * kEmitPoolStride, (uint32_t)__popcll(hm));
        base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
        const uint32_t slot = base + r;
        if (slot < m.ov_pool) {
            OvEnt v;
            v.idxA = a.idx;
            v.k = k;
            v.idxB = t.idxB;
            v.j = t.j;
            v.code = t.sep;
            m.ovl[(size_t)pool * m.ov_pool + slot] = v;
        } else {
            atomicOr(m.ov_flag, 1u);
        }
    };

    // One candidate: decide it, then count / rank it (MODE 0), write it
    // (MODE 1), or both (MODE 2). Band candidates are only listed.
    auto visit = [&](int z, uint32_t key, const PayT &b, uint32_t j) {
        ++tests;
        double c2;
        int d = decide<SHAPE, PREC>(m, a, e, er, f, cc, z, key, b, j, c2);
        if (d == AMBIG) {
            if (MODE != 1) {
                ++band;
                uint32_t slot = atomicAdd(m.amb_n, 1u);
                if (slot < m.amb_cap) m.amb[slot] = make_uint2(i, j);
            }
            return;
        }
        if (d != IN) return;
        if (MODE == 2) {
            const PairTmp t = coded(b, j, c2);
            if (cnt < (uint32_t)kTab) {
                m.table[(size_t)a.idx * kTab + cnt] = t;
                ++placed;
            } else {
                overflow(cnt, t);
            }
        }
        if (MODE != 1) {
            ++cnt;
            if (c2 < b1 || (c2 == b1 && b.idx < bidx)) {
                b2 = b1;
                b1 = c2;
                bidx = b.idx;
                bj = j;
            } else if (c2 < b2) {
                b2 = c2;
            }
        } else {
            int64_t p = o + cnt;
            if (p < oe) {
                m.tmp[p] = coded(b, j, c2);
                ++placed;
            } else {
                atomicOr(m.err_flag, 1u);
            }
            ++cnt;
        }
    };

    if (zhi_all >= zlo_all && zhi_all - zlo_all >= (uint32_t)kTileZones) {
        // A tile spread over many zones (sparse sky near the poles): each
        // lane walks its own few zones with direct loads.
        if (active)
            for_each_range(m.g, a.ra, a.dec, a.cosd, a.reach_deg, [&](int z, uint32_t j0, uint32_t j1) {
                cc.key = 0xffffffffu;
                for (uint32_t j = j0; j < j1; ++j) {
                    const PayT b = pay[j];
                    visit(z, m.g.keys[j], b, j);
                }
            });
    } else if (zhi_all >= zlo_all) {
        // Cooperative tile. In each of the tile's zones the lanes' cell
        // windows are gathered into up to three hulls -- plain windows, the
        // [0, b] pieces and the [a, n-1] pieces of windows split at RA 0/360
        // (so a tile near RA 0 does not stage its whole zone) -- each one key
        // range of B. All range ends are looked up at once (lane 6q+2h and
        // 6q+2h+1 for hull h of zone q), every range is staged in LDS behind
        // one wave barrier, and each lane binary-searches its own cells in
        // the segment of the matching hull. Lane windows are recomputed per
        // zone rather than kept in registers.
        const uint32_t zb = (uint32_t)__builtin_amdgcn_readfirstlane((int)zlo_all);
        const int nzt = __builtin_amdgcn_readfirstlane((int)(zhi_all - zlo_all)) + 1;
        ZoneInfo zq[kTileZones];
#pragma unroll
        for (int q = 0; q < kTileZones; ++q) zq[q] = m.g.zinfo[min((int)zb + q, m.g.nz - 1)];
        uint32_t lkey = 0;
        bool lvalid = false, lend = false;
#pragma unroll
        for (int q = 0; q < kTileZones; ++q) {
            if (q >= nzt) break;
            const int z = (int)zb + q;
            const ZoneInfo zi = zq[q];
            uint32_t c0[2], c1[2];
            int nr = 0;
            if (active && z >= w.zlo && z <= w.zhi) nr = zone_ranges(zi, w, a.ra, c0, c1);
            const int nh = __ballot(nr == 2) ? 3 : 1;  // wrap hulls only if a lane wraps
            for (int h = 0; h < nh; ++h) {
                uint32_t lo = 0xffffffffu, hi = 0;
                if (h == 0 && nr == 1) {
                    lo = c0[0];
                    hi = c1[0];
                } else if (h > 0 && nr == 2) {
                    lo = c0[h - 1];
                    hi = c1[h - 1];
                }
                lo = wave_min_u32(lo);
                hi = wave_max_u32(hi);
                if (lane >> 1 == 3 * q + h && lo <= hi) {
                    lvalid = true;
                    lend = lane & 1;
                    lkey = lend ? zi.base + hi + 1 : zi.base + lo;
                }
            }
        }
        const uint32_t lres = lvalid ? key_bound(m.g, lkey, lend) : 0u;
        // ends of hull h of zone q (wave-uniform)
        auto ends = [&](int q, int h, uint32_t &j0, uint32_t &j1) {
            j0 = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)lres, 2 * (3 * q + h)));
            j1 = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)lres, 2 * (3 * q + h) + 1));
            if (j1 < j0) j1 = j0;
        };
        uint32_t T = 0;
        for (int q = 0; q < nzt; ++q)
#pragma unroll
            for (int h = 0; h < 3; ++h) {
                uint32_t j0, j1;
                ends(q, h, j0, j1);
                T += j1 - j0;
            }
        if (T <= (uint32_t)kStage) {
            uint32_t seg = 0;
            for (int q = 0; q < nzt; ++q)
#pragma unroll
                for (int h = 0; h < 3; ++h) {
                    uint32_t j0, j1;
                    ends(q, h, j0, j1);
                    for (uint32_t s = lane; s < j1 - j0; s += 64) {
                        sk[seg + s] = m.g.keys[j0 + s];
                        sp[seg + s] = pay[j0 + s];
                    }
                    seg += j1 - j0;
                }
            wave_sync();
            seg = 0;
            for (int q = 0; q < nzt; ++q) {
                const int z = (int)zb + q;
                const ZoneInfo zi = m.g.zinfo[z];
                uint32_t c0[2], c1[2];
                int nr = 0;
                if (active && z >= w.zlo && z <= w.zhi) nr = zone_ranges(zi, w, a.ra, c0, c1);
                cc.key = 0xffffffffu;
#pragma unroll
                for (int h = 0; h < 3; ++h) {
                    uint32_t j0, j1;
                    ends(q, h, j0, j1);
                    const uint32_t segn = j1 - j0;
                    int k = -1;
                    if (h == 0 && nr == 1) k = 0;
                    else if (h > 0 && nr == 2) k = h - 1;
                    if (segn > 0 && k >= 0) {
                        const uint32_t ka = k ? c0[1] : c0[0], kb = k ? c1[1] : c1[0];
                        uint32_t s0 = seg + lds_lower_bound(sk + seg, segn, zi.base + ka);
                        uint32_t s1 = seg + lds_lower_bound(sk + seg, segn, zi.base + kb + 1);
                        for (uint32_t s = s0; s < s1; ++s) {
                            const PayT b = sp[s];
                            visit(z, sk[s], b, j0 + (s - seg));
                        }
                    }
                    seg += segn;
                }
            }
        } else {
            // more than fits in LDS at once: hull by hull, in chunks
            for (int q = 0; q < nzt; ++q) {
                const int z = (int)zb + q;
                const ZoneInfo zi = m.g.zinfo[z];
                uint32_t c0[2], c1[2];
                int nr = 0;
                if (active && z >= w.zlo && z <= w.zhi) nr = zone_ranges(zi, w, a.ra, c0, c1);
#pragma unroll
                for (int h = 0; h < 3; ++h) {
                    uint32_t j0, j1;
                    ends(q, h, j0, j1);
                    int k = -1;
                    if (h == 0 && nr == 1) k = 0;
                    else if (h > 0 && nr == 2) k = h - 1;
                    const uint32_t ka = k == 1 ? c0[1] : c0[0], kb = k == 1 ? c1[1] : c1[0];
                    cc.key = 0xffffffffu;
                    for (uint32_t c = j0; c < j1; c += kStage) {
                        const uint32_t nst = min((uint32_t)kStage, j1 - c);
                        wave_sync();
                        for (uint32_t s = lane; s < nst; s += 64) {
                            sk[s] = m.g.keys[c + s];
                            sp[s] = pay[c + s];
                        }
                        wave_sync();
                        if (k >= 0) {
                            uint32_t s0 = lds_lower_bound(sk, nst, zi.base + ka);
                            uint32_t s1 = lds_lower_bound(sk, nst, zi.base + kb + 1);
                            for (uint32_t s = s0; s < s1; ++s) {
                                const PayT b = sp[s];
                                visit(z, sk[s], b, c + s);
                            }
                        }
                    }
                }
            }
        }
    }
    if (active) {
        if (MODE != 1) {
            AStat st;
            st.cnt = cnt;
            st.nf = cnt;
            st.best_j = bj;
            st.pad = 0;
            m.astat[a.idx] = st;
            m.best_idx[a.idx] = cnt ? (int32_t)bidx : -1;
            if (cnt >= 2 && b2 - b1 <= 4.0 * c2_err<PREC>(sqrt(b2), m.L_rad)) {
                uint32_t slot = atomicAdd(m.tie_n, 1u);
                if (slot < m.tie_cap) m.tie[slot] = make_uint2(i, a.idx);
            }
        } else {
            if (o + cnt != oe) atomicOr(m.err_flag, 2u);
        }
    }
    if (placed) atomicAdd(&s_placed, placed);
    if (tests) atomicAdd(&s_tests, tests);
    if (band) atomicAdd(&s_band, band);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_tests && MODE != 1) atomicAdd(m.n_tests, s_tests);
        if (s_band && MODE != 1) atomicAdd(m.n_band, s_band);
        if (s_placed) atomicAdd(m.n_placed, s_placed);
    }
}

// Every match of the listed sorted A positions (best-match re-ranking): one
// wavefront per listed source, lanes striding over its candidate ranges.
template <int SHAPE, int PREC>
__global__ __launch_bounds__(64) void k_collect(MatchArgs m)
{
    using PayT = PayOf<PREC>;
    const uint32_t t = blockIdx.x;
    if (t >= m.n_col) return;
    const PayT *pay;
    if constexpr (PREC == C3X_FP64) pay = m.pay64;
    else pay = m.pay32;
    uint32_t i = m.col_pos[t];
    AEll e{};
    AEllR er{};
    LaneF32 f{};
    double reach = m.reach_deg;
    if constexpr (SHAPE == C3X_ELLIPSE) {
        e = m.aell[i];
        er = m.aellr[i];
        reach = er.a_arcsec / 3600.0;
        f = LaneF32{(float)e.ux, (float)e.uy, (float)e.uz, (float)e.vx,
                    (float)e.vy, (float)e.vz, (float)e.ia, (float)e.ib};
    }
    ARec a = load_a(m, i, reach);
    CellCache cc{0xffffffffu, 0.f, 0.f, 0.f};
    for_each_range(m.g, a.ra, a.dec, a.cosd, a.reach_deg, [&](int z, uint32_t j0, uint32_t j1) {
        for (uint32_t j = j0 + threadIdx.x; j < j1; j += 64) {
            const PayT b = pay[j];
            double c2;
            int d = decide<SHAPE, PREC>(m, a, e, er, f, cc, z, m.g.keys[j], b, j, c2);
            if (d == AMBIG) d = verdict(m, i, j);
            if (d != IN) continue;
            uint32_t slot = atomicAdd(m.col_n, 1u);
            if (slot < m.col_cap) {
                double2 rb = m.radecB[j];
                ColEnt ce;
                ce.t = t;
                ce.idxB = b.idx;
                ce.j = j;
                ce.pad = 0;
                ce.ra = rb.x;
                ce.dec = rb.y;
                ((ColEnt *)m.col)[slot] = ce;
            }
        }
    });
}

// ---------------------------------------------------------------------------- small kernels

// One thread per band candidate: the FP64 relative-accuracy recheck (error
// <= ~90 u against a 2^-40 margin). Writes 0 (out), 1 (in) or 2 (still
// undecided: the host decides it in binary128), with what the host needs.
template <int SHAPE>
__global__ void k_recheck(const uint2 *__restrict__ band, uint32_t n, const double2 *__restrict__ arad,
                          const uint32_t *__restrict__ aidx, const AEllR *__restrict__ aellr,
                          const double2 *__restrict__ radecB, const Pay64 *__restrict__ p64,
                          const Pay32 *__restrict__ p32, double h_r, const double *__restrict__ sa,
                          const double *__restrict__ sb, const double *__restrict__ pa,
                          AmbInfo *__restrict__ out, uint8_t *__restrict__ v)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint2 q = band[t];
    double2 ad = arad[q.x];
    uint32_t row = aidx[q.x];
    double2 rb = radecB[q.y];
    ARec a;
    a.ra = ad.x;
    a.dec = ad.y;
    unit_vec(a.ra, a.dec, a.x, a.y, a.z);
    a.cosd = cos_dec_acc(a.dec);
    a.reach_deg = 0.0;
    a.idx = row;
    a.pad = 0;
    int d;
    if (SHAPE == C3X_CIRCLE) d = recheck_circle(a, rb, h_r);
    else d = recheck_ellipse(a, aellr[q.x], rb);
    v[t] = (uint8_t)d;
    AmbInfo r;
    r.raA = ad.x;
    r.decA = ad.y;
    r.raB = rb.x;
    r.decB = rb.y;
    r.a = sa ? sa[row] : 0.0;
    r.b = sb ? sb[row] : 0.0;
    r.pa = pa ? pa[row] : 0.0;
    r.i = q.x;
    r.j = q.y;
    r.idxA = row;
    r.idxB = p64 ? p64[q.y].idx : p32[q.y].idx;
    out[t] = r;
}

__global__ void k_gather_pos(const uint32_t *__restrict__ pos, uint32_t n,
                             const double2 *__restrict__ arad, const uint32_t *__restrict__ aidx,
                             double2 *__restrict__ oad, uint32_t *__restrict__ orow)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    oad[t] = arad[pos[t]];
    orow[t] = aidx[pos[t]];
}

// Band candidates found inside (sorted A position, idxA, idxB, sorted B
// position): each is counted, and listed as the k-th match of its source.
__global__ void k_add_pairs(const uint4 *__restrict__ in, uint32_t n, AStat *st,
                            WEnt *__restrict__ out)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint4 q = in[t];
    uint32_t k = atomicAdd(&st[q.y].cnt, 1u);
    if (out) out[t] = WEnt{q.x, k, q.z, q.w};
}

// Separation from the coordinates, out of line: only the rare paths (band
// matches, separations the write pass leaves undefined) need it.
__device__ __noinline__ double sep_rare(double ra1, double dec1, double ra2, double dec2)
{
    return sep_arcsec_rd(ra1, dec1, ra2, dec2);
}

// One thread per used slot of overflow region blockIdx.y: the k-th match of
// row idxA to offset off[idxA] + k of the segments.
__global__ void k_place_ov(const OvEnt *__restrict__ ovl, uint32_t ov_pool,
                           const uint32_t *__restrict__ octr, int64_t nA,
                           const int64_t *__restrict__ off, int64_t P, PairTmp *__restrict__ tmp,
                           unsigned long long *__restrict__ placed, uint32_t *__restrict__ err)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= min(octr[blockIdx.y * kEmitPoolStride], ov_pool)) return;
    const OvEnt v = ovl[(size_t)blockIdx.y * ov_pool + t];
    if (v.idxA >= (uint64_t)nA) {
        atomicOr(err, 16u);
        return;
    }
    const int64_t o = off[v.idxA], oe = off[v.idxA + 1];
    const int64_t p = o + v.k;
    if (v.k < (uint32_t)kTab || p >= oe || oe > P) {
        atomicOr(err, 1u);
        return;
    }
    PairTmp x;
    x.idxB = v.idxB;
    x.j = v.j;
    x.sep = v.code;
    tmp[p] = x;
    atomicAdd(placed, 1ull);
}

// One thread per band match found inside: to its row's table slot (k <
// kTab, when the single pass filled the table) or its place in the
// idxA-order segments, with its separation.
__global__ void k_place_x(const WEnt *__restrict__ xent, uint32_t nx,
                          const uint32_t *__restrict__ aidx, const double2 *__restrict__ arad,
                          const double2 *__restrict__ radecB, int64_t nA, int64_t nB,
                          const int64_t *__restrict__ off, int64_t P, PairTmp *__restrict__ table,
                          PairTmp *__restrict__ tmp, unsigned long long *__restrict__ placed,
                          uint32_t *__restrict__ err)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nx) return;
    const WEnt e = xent[t];
    if (e.i >= (uint64_t)nA || e.j >= (uint64_t)nB) {
        atomicOr(err, 16u);
        return;
    }
    const uint32_t a = aidx[e.i];
    const int64_t o = off[a], oe = off[a + 1];
    const int64_t p = o + e.k;
    if (p >= oe || oe > P) {
        atomicOr(err, 1u);
        return;
    }
    const double2 ra = arad[e.i], rb = radecB[e.j];
    PairTmp x;
    x.idxB = e.idxB;
    x.j = e.j;
    x.sep = sep_rare(ra.x, ra.y, rb.x, rb.y);
    if (table && e.k < (uint32_t)kTab) table[(size_t)a * kTab + e.k] = x;
    else tmp[p] = x;
    atomicAdd(placed, 1ull);
}

__global__ void k_patch_best(const uint32_t *__restrict__ rows, const int32_t *__restrict__ bi,
                             const uint32_t *__restrict__ bj, uint32_t n, int32_t *best_idx,
                             AStat *st)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    best_idx[rows[t]] = bi[t];
    st[rows[t]].best_j = bj[t];
}

__global__ void k_counts(const AStat *__restrict__ st, int64_t n, int nonzero,
                         uint32_t *__restrict__ out, double *__restrict__ bsep)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint32_t c = st[t].cnt;
    out[t] = nonzero ? (c ? 1u : 0u) : c;
    if (bsep) bsep[t] = NAN;
}

// Final record of one match: idxA, idxB and the separation (computed here
// when the pass that placed it left it undefined), and the best match's
// separation.
__device__ __forceinline__ void final_write(int64_t q, int64_t a, const PairTmp &x, int64_t nB,
                                            const double *__restrict__ raA,
                                            const double *__restrict__ decA,
                                            const double2 *__restrict__ radecB,
                                            const int32_t *__restrict__ bidx,
                                            int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                                            double *__restrict__ os, double *__restrict__ bsep,
                                            uint32_t *__restrict__ err)
{
    double s = x.sep;
    if (s < 0.0) {  // coded by the write pass (see sep_code)
        s = sep_from_chord2(-s);
    } else if (isnan(s)) {
        if (x.j >= (uint64_t)nB) {
            atomicOr(err, 16u);
            return;
        }
        double2 rb = radecB[x.j];
        s = sep_rare(raA[a], decA[a], rb.x, rb.y);
    }
    oa[q] = (int32_t)a;
    ob[q] = (int32_t)x.idxB;
    os[q] = s;
    if (bidx[a] == (int32_t)x.idxB) bsep[a] = s;
}

// One thread per A row. A row's k-th match is in its table slot for k <
// kTab (when the single pass filled the table) and at offset off + k of its
// segment otherwise. A short segment (<= kShortSeg) is finished here: the
// canonical position of each match is its rank by idxB (unique in a
// segment). A longer one has its table slots copied into the segment, which
// k_seg_lds then finishes.
__global__ void k_finalize(int64_t nA, int64_t nB, const int64_t *__restrict__ off,
                           const PairTmp *__restrict__ table, PairTmp *__restrict__ tmp,
                           const double *__restrict__ raA, const double *__restrict__ decA,
                           const double2 *__restrict__ radecB, const int32_t *__restrict__ bidx,
                           int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                           double *__restrict__ os, double *__restrict__ bsep,
                           uint32_t *__restrict__ err)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nA) return;
    const int64_t o = off[a], len = off[a + 1] - o;
    if (len <= 0) return;
    const int nt = table ? (int)min<int64_t>(len, kTab) : 0;
    const PairTmp *row = table + (table ? a * kTab : 0);
    if (len > kShortSeg) {
        for (int q = 0; q < nt; ++q) tmp[o + q] = row[q];
        return;
    }
    if (len == 1) {
        final_write(o, a, nt ? row[0] : tmp[o], nB, raA, decA, radecB, bidx, oa, ob, os, bsep, err);
        return;
    }
    for (int q = 0; q < len; ++q) {
        const PairTmp x = q < nt ? row[q] : tmp[o + q];
        int r = 0;
        for (int y = 0; y < len; ++y) r += (y < nt ? row[y].idxB : tmp[o + y].idxB) < x.idxB;
        final_write(o + r, a, x, nB, raA, decA, radecB, bidx, oa, ob, os, bsep, err);
    }
}

// One thread per A row: separation of the best match; in BEST-only mode also
// the compacted (idxA, idxB, sep) pair.
__global__ void k_best_sep(int64_t n, int64_t nB, const int32_t *__restrict__ bidx,
                           const AStat *__restrict__ st, const double *__restrict__ raA,
                           const double *__restrict__ decA, const double2 *__restrict__ radecB,
                           double *__restrict__ bsep, const int64_t *__restrict__ off, int64_t P,
                           int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                           double *__restrict__ os, uint32_t *__restrict__ err)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int32_t b = bidx[t];
    if (b < 0) {
        bsep[t] = NAN;
        return;
    }
    uint32_t bj = st[t].best_j;
    if (bj >= (uint64_t)nB) {
        atomicOr(err, 16u);
        return;
    }
    double2 rb = radecB[bj];
    double s = sep_arcsec_rd(raA[t], decA[t], rb.x, rb.y);
    bsep[t] = s;
    if (off) {
        int64_t p = off[t];
        if (p < P && off[t + 1] == p + 1) {
            oa[p] = (int32_t)t;
            ob[p] = b;
            os[p] = s;
        } else {
            atomicOr(err, 8u);
        }
    }
}

// ---------------------------------------------------------------------------- long segments

__global__ void k_seg_list(const int64_t *__restrict__ off, int64_t n, uint32_t *__restrict__ cnt,
                           uint32_t *__restrict__ list, uint32_t cap)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    if (off[t + 1] - off[t] > kShortSeg) {
        uint32_t s = atomicAdd(cnt, 1u);
        if (s < cap) list[s] = (uint32_t)t;
    }
}

// Segments longer than kShortSeg, one workgroup at a time over the list
// (the grid does not depend on the list's length): segments of up to
// kSegLds matches are sorted by idxB in LDS (bitonic network over
// idxB << 32 | position; idxB is unique in a segment) and written out in
// final form; longer ones are listed for the host-driven radix sort.
__global__ __launch_bounds__(256) void k_seg_lds(const int64_t *__restrict__ off,
                                                 const uint32_t *__restrict__ cnt,
                                                 const uint32_t *__restrict__ list, uint32_t cap,
                                                 const PairTmp *__restrict__ tmp, int64_t nB,
                                                 const double *__restrict__ raA,
                                                 const double *__restrict__ decA,
                                                 const double2 *__restrict__ radecB,
                                                 const int32_t *__restrict__ bidx,
                                                 int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                                                 double *__restrict__ os, double *__restrict__ bsep,
                                                 uint32_t *__restrict__ huge_n,
                                                 uint32_t *__restrict__ huge,
                                                 uint32_t *__restrict__ err)
{
    __shared__ unsigned long long v[kSegLds];
    const uint32_t nseg = min(*cnt, cap);
    for (uint32_t b = blockIdx.x; b < nseg; b += gridDim.x) {
        const uint32_t a = list[b];
        const int64_t o = off[a];
        const int len = (int)min<int64_t>(off[a + 1] - o, 1 << 30);
        if (len > kSegLds) {
            if (threadIdx.x == 0) {
                uint32_t s = atomicAdd(huge_n, 1u);
                if (s < cap) huge[s] = a;
            }
            continue;  // uniform over the workgroup
        }
        int p2 = 1;
        while (p2 < len) p2 <<= 1;
        for (int k = threadIdx.x; k < p2; k += blockDim.x)
            v[k] = k < len ? ((unsigned long long)tmp[o + k].idxB << 32) | (unsigned)k : ~0ull;
        __syncthreads();
        for (int size = 2; size <= p2; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int k = threadIdx.x; k < p2; k += blockDim.x) {
                    int l = k ^ stride;
                    if (l > k) {
                        bool up = (k & size) == 0;
                        unsigned long long x = v[k], y = v[l];
                        if ((x > y) == up) {
                            v[k] = y;
                            v[l] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int k = threadIdx.x; k < len; k += blockDim.x)
            final_write(o + k, a, tmp[o + (uint32_t)v[k]], nB, raA, decA, radecB, bidx, oa, ob, os,
                        bsep, err);
        __syncthreads();  // v is reused by the next segment
    }
}

// Final records of a segment already sorted in place (host-driven path).
__global__ void k_seg_copy(int64_t o, int64_t len, int64_t a, const PairTmp *__restrict__ tmp,
                           int64_t nB, const double *__restrict__ raA,
                           const double *__restrict__ decA, const double2 *__restrict__ radecB,
                           const int32_t *__restrict__ bidx, int32_t *__restrict__ oa,
                           int32_t *__restrict__ ob, double *__restrict__ os,
                           double *__restrict__ bsep, uint32_t *__restrict__ err)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len)
        final_write(o + k, a, tmp[o + k], nB, raA, decA, radecB, bidx, oa, ob, os, bsep, err);
}

__global__ void k_split(const PairTmp *__restrict__ t, int64_t n, uint32_t *__restrict__ k,
                        uint32_t *__restrict__ v)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    k[p] = t[p].idxB;
    v[p] = (uint32_t)p;
}

__global__ void k_merge(const uint32_t *__restrict__ v, const PairTmp *__restrict__ copy, int64_t n,
                        PairTmp *__restrict__ t)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n && v[p] < (uint64_t)n) t[p] = copy[v[p]];
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// What the finishing kernels need.
struct FinishArgs {
    int64_t nA, nB;
    const int64_t *off;
    const PairTmp *table;
    PairTmp *tmp;
    const double *raA, *decA;
    const double2 *radecB;
    const int32_t *bidx;
    int32_t *oa, *ob;
    double *os, *bsep;
    uint32_t *err;
    uint32_t *seg_n;   // [2]: listed long segments, listed huge segments
    uint32_t *list, *huge;
    uint32_t cap;
};

constexpr unsigned kSegGrid = 1024;

// Final records of every segment: short ones per A row, long ones per
// workgroup; segments above kSegLds are only listed (finish_huge).
static void finish_segments(const FinishArgs &f, hipStream_t s)
{
    if (f.nA == 0) return;
    hipLaunchKernelGGL(k_finalize, dim3(nblk(f.nA, 256)), dim3(256), 0, s, f.nA, f.nB, f.off,
                       f.table, f.tmp, f.raA, f.decA, f.radecB, f.bidx, f.oa, f.ob, f.os, f.bsep,
                       f.err);
    hipLaunchKernelGGL(k_seg_list, dim3(nblk(f.nA, 256)), dim3(256), 0, s, f.off, f.nA, f.seg_n,
                       f.list, f.cap);
    hipLaunchKernelGGL(k_seg_lds, dim3(kSegGrid), dim3(256), 0, s, f.off, f.seg_n, f.list, f.cap,
                       f.tmp, f.nB, f.raA, f.decA, f.radecB, f.bidx, f.oa, f.ob, f.os, f.bsep,
                       f.seg_n + 1, f.huge, f.err);
}

// Segments longer than kSegLds (counts already on the host): radix sort by
// idxB, one segment at a time, then their final records.
static c3x_status finish_huge(const FinishArgs &f, const uint32_t *hseg, hipStream_t s)
{
    if (hseg[0] > f.cap || hseg[1] > f.cap) return fail(C3X_ENOMEM, "too many long segments");
    uint32_t nh = hseg[1];
    if (nh == 0) return C3X_OK;
    std::vector<uint32_t> hv(nh);
    hipError_t e = hipMemcpy(hv.data(), f.huge, nh * sizeof(uint32_t), hipMemcpyDeviceToHost);
    for (uint32_t k = 0; k < nh && e == hipSuccess; ++k) {
        int64_t ob[2];
        e = hipMemcpy(ob, f.off + hv[k], 2 * sizeof(int64_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) break;
        int64_t o = ob[0], len = ob[1] - ob[0];
        Arena t2(s);
        uint32_t *k1 = t2.get_n<uint32_t>(len), *v1 = t2.get_n<uint32_t>(len);
        uint32_t *k2 = t2.get_n<uint32_t>(len), *v2 = t2.get_n<uint32_t>(len);
        PairTmp *copy = t2.get_n<PairTmp>(len);
        void *ws = t2.get(radix_ws_bytes(len));
        if (!k1 || !v1 || !k2 || !v2 || !copy || !ws) return fail(C3X_ENOMEM, "segment sort");
        e = hipMemcpyAsync(copy, f.tmp + o, len * sizeof(PairTmp), hipMemcpyDeviceToDevice, s);
        hipLaunchKernelGGL(k_split, dim3(nblk(len, 256)), dim3(256), 0, s, f.tmp + o, len, k1, v1);
        int in_tmp = 0;
        if (e == hipSuccess) e = radix_sort_pairs(k1, v1, k2, v2, len, 31, ws, s, &in_tmp);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_merge, dim3(nblk(len, 256)), dim3(256), 0, s, in_tmp ? v2 : v1,
                               copy, len, f.tmp + o);
            hipLaunchKernelGGL(k_seg_copy, dim3(nblk(len, 256)), dim3(256), 0, s, o, len,
                               (int64_t)hv[k], f.tmp, f.nB, f.raA, f.decA, f.radecB, f.bidx, f.oa,
                               f.ob, f.os, f.bsep, f.err);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) return fail_hip(e, "segment order");
    return C3X_OK;
}

// Margins of the circle filters on the squared chord: FP64 unit vectors
// carry <= 32 u per component; FP32 offsets from a cell reference carry
// 2^-24 of their size (<= L + c). Factor 4 of safety on the error at 1.5 r.
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
#define C3X_LAUNCH(SH, PR) \
    hipLaunchKernelGGL((k_match<SH, PR, MODE>), dim3(grid), dim3(kMatchBlock), 0, s, m)
    if (shape == C3X_CIRCLE) {
        if (prec == C3X_FP64) C3X_LAUNCH(C3X_CIRCLE, C3X_FP64);
        else C3X_LAUNCH(C3X_CIRCLE, C3X_MIXED);
    } else {
        if (prec == C3X_FP64) C3X_LAUNCH(C3X_ELLIPSE, C3X_FP64);
        else C3X_LAUNCH(C3X_ELLIPSE, C3X_MIXED);
    }
#undef C3X_LAUNCH
}

static void launch_collect(const MatchArgs &m, int shape, int prec, hipStream_t s)
{
    unsigned grid = m.n_col;
    if (grid == 0) return;
    if (shape == C3X_CIRCLE) {
        if (prec == C3X_FP64)
            hipLaunchKernelGGL((k_collect<C3X_CIRCLE, C3X_FP64>), dim3(grid), dim3(64), 0, s, m);
        else
            hipLaunchKernelGGL((k_collect<C3X_CIRCLE, C3X_MIXED>), dim3(grid), dim3(64), 0, s, m);
    } else {
        if (prec == C3X_FP64)
            hipLaunchKernelGGL((k_collect<C3X_ELLIPSE, C3X_FP64>), dim3(grid), dim3(64), 0, s, m);
        else
            hipLaunchKernelGGL((k_collect<C3X_ELLIPSE, C3X_MIXED>), dim3(grid), dim3(64), 0, s, m);
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
    const bool all = (mode & C3X_ALL) != 0;
    Timer tm(s);
    tm.mark();  // 0
    Arena tmp(s);
    // ---- A preparation
    uint32_t *keys = tmp.get_n<uint32_t>(nA), *rows = tmp.get_n<uint32_t>(nA);
    uint32_t *ktmp = tmp.get_n<uint32_t>(nA), *rtmp = tmp.get_n<uint32_t>(nA);
    void *ws = tmp.get(std::max(radix_ws_bytes(nA), scan_ws_bytes(nA + 1)));
    uint32_t *ctr = tmp.get_n<uint32_t>(8);  // bad, amb_n, tie_n, col_n, err, emit overflow
    unsigned long long *c64 = tmp.get_n<unsigned long long>(3);  // tests, band, placed
    double2 *arad = tmp.get_n<double2>(nA);
    double2 *packed = tmp.get_n<double2>(nA);
    uint32_t *aidx = tmp.get_n<uint32_t>(nA);
    AStat *astat = tmp.get_n<AStat>(nA);
    AEll *aell = nullptr;
    AEllR *aellr = nullptr;
    if (shape == C3X_ELLIPSE) {
        aell = tmp.get_n<AEll>(nA);
        aellr = tmp.get_n<AEllR>(nA);
        if (!aell || !aellr) return fail(C3X_ENOMEM, "A buffers");
    }
    if (!keys || !rows || !ktmp || !rtmp || !ws || !ctr || !c64 || !arad || !packed || !aidx ||
        !astat)
        return fail(C3X_ENOMEM, "A buffers");
    R->nA = nA;
    R->best_idx = R->mem.get_n<int32_t>(nA);
    R->best_sep = R->mem.get_n<double>(nA);
    if (!R->best_idx || !R->best_sep) return fail(C3X_ENOMEM, "best buffers");
    HIPCHK(hipMemsetAsync(ctr, 0, 8 * sizeof(uint32_t), s), "memset");
    HIPCHK(hipMemsetAsync(ctr, 0xff, sizeof(uint32_t), s), "memset");
    HIPCHK(hipMemsetAsync(c64, 0, 3 * sizeof(unsigned long long), s), "memset");
    const double *sa = area->semi_major_arcsec, *sb = area->semi_minor_arcsec, *pa = area->pa_deg;
    if (nA > 0)
        hipLaunchKernelGGL(k_prep_a, dim3(nblk(nA, 256)), dim3(256), 0, s, ra, dec, nA, ix->grid,
                           shape, sa, sb, pa, keys, rows, packed, ctr);
    HIPCHK(hipGetLastError(), "A keys");
    int in_tmp = 0;
    HIPCHK(radix_sort_pairs(keys, rows, ktmp, rtmp, nA, ix->plan.key_bits, ws, s, &in_tmp), "A sort");
    uint32_t *srows = in_tmp ? rtmp : rows;
    if (nA > 0) {
        if (shape == C3X_CIRCLE)
            hipLaunchKernelGGL(k_gather_a<C3X_CIRCLE>, dim3(nblk(nA, 256)), dim3(256), 0, s, srows,
                               packed, nA, sa, sb, pa, area->pa_zero_deg, area->pa_sense,
                               ix->plan.L_rad, arad, aidx, aell, aellr);
        else
            hipLaunchKernelGGL(k_gather_a<C3X_ELLIPSE>, dim3(nblk(nA, 256)), dim3(256), 0, s,
                               srows, packed, nA, sa, sb, pa, area->pa_zero_deg, area->pa_sense,
                               ix->plan.L_rad, arad, aidx, aell, aellr);
    }
    HIPCHK(hipGetLastError(), "A records");
    tm.mark();  // 1

    // ---- thresholds and common arguments
    MatchArgs m;
    memset(&m, 0, sizeof(m));
    m.g = ix->grid;
    m.pay64 = ix->pay64;
    m.pay32 = ix->pay32;
    m.radecB = ix->radec;
    m.arad = arad;
    m.aidx = aidx;
    m.aell = aell;
    m.aellr = aellr;
    m.nA = (int32_t)nA;
    m.L_rad = ix->plan.L_rad;
    if (shape == C3X_CIRCLE) {
        CircleThresholds t = circle_thresholds(area->radius_arcsec, ix->plan.L_rad);
        m.reach_deg = area->radius_arcsec / 3600.0;
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
    m.astat = astat;
    m.best_idx = R->best_idx;
    unsigned grid = nblk(nA, kMatchBlock);

    // ---- count pass (+ best by the filter's chord, near-ties listed)
    uint32_t amb_cap = (uint32_t)std::max<int64_t>(4096, nA / 256);
    uint32_t tie_cap = (uint32_t)std::max<int64_t>(4096, nA / 256);
    uint2 *amb = tmp.get_n<uint2>(amb_cap);
    uint2 *tie = tmp.get_n<uint2>(tie_cap);
    if (!amb || !tie) return fail(C3X_ENOMEM, "count buffers");
    m.amb_n = ctr + 1;
    m.amb = amb;
    m.amb_cap = amb_cap;
    m.tie_n = ctr + 2;
    m.tie = tie;
    m.tie_cap = tie_cap;
    // All matches: the pass that counts also writes them -- a row's first
    // kTab matches into its table slots, later ones into the overflow list
    // (kEmitPools regions; block b uses region b mod kEmitPools). If a
    // region runs out, the count stands and the write pass puts every
    // match into the offsets instead.
    m.n_placed = c64 + 2;
    m.ov_flag = ctr + 5;
    bool emit = false;
    const int kPoolWords = kEmitPools * kEmitPoolStride;
    if (all && nA > 0) {
        uint64_t per = (uint64_t)std::max<int64_t>(nA / 8 / kEmitPools, 4096);
        // test hook: C3X_DEBUG_OVERFLOW_SLOTS=k gives each region k slots (0: no table)
        if (const char *ev = getenv("C3X_DEBUG_OVERFLOW_SLOTS"))
            per = (uint64_t)std::max<long long>(atoll(ev), -1);
        const bool no_table = getenv("C3X_DEBUG_OVERFLOW_SLOTS") && per == 0;
        if (!no_table && per < (1ull << 26)) {
            m.table = tmp.get_n<PairTmp>((size_t)nA * kTab);
            m.ovl = tmp.get_n<OvEnt>(per * kEmitPools);
            m.octr = tmp.get_n<uint32_t>(kPoolWords);
            m.ov_pool = (uint32_t)per;
            emit = m.table && m.ovl && m.octr;
            if (emit) HIPCHK(hipMemsetAsync(m.octr, 0, kPoolWords * sizeof(uint32_t), s), "memset");
        }
    }
    uint32_t hctr[8];
    unsigned long long h64[3];
    std::vector<uint32_t> hoctr(kPoolWords);
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (emit) launch_match<2>(m, shape, prec, grid, s);
        else launch_match<0>(m, shape, prec, grid, s);
        HIPCHK(hipGetLastError(), "count pass");
        HIPCHK(hipMemcpyAsync(hctr, ctr, sizeof(hctr), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(hipMemcpyAsync(h64, c64, sizeof(h64), hipMemcpyDeviceToHost, s), "copy");
        if (emit)
            HIPCHK(hipMemcpyAsync(hoctr.data(), m.octr, kPoolWords * sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(hipStreamSynchronize(s), "count pass");
        if (hctr[0] != 0xffffffffu)
            return fail(C3X_EINVAL,
                        "catalogue A row %u: coordinate outside RA [0,360), |Dec| <= 90, not "
                        "finite, or ellipse axes outside 1e-6 <= b <= a <= 324000 arcsec, "
                        "a <= 1000 b",
                        hctr[0]);
        if (hctr[1] <= amb_cap && hctr[2] <= tie_cap) break;
        // a list overflowed: grow it and count again
        if (hctr[1] > amb_cap) {
            amb_cap = hctr[1];
            amb = tmp.get_n<uint2>(amb_cap);
        }
        if (hctr[2] > tie_cap) {
            tie_cap = hctr[2];
            tie = tmp.get_n<uint2>(tie_cap);
        }
        if (!amb || !tie) return fail(C3X_ENOMEM, "count lists");
        m.amb = amb;
        m.amb_cap = amb_cap;
        m.tie = tie;
        m.tie_cap = tie_cap;
        HIPCHK(hipMemsetAsync(ctr + 1, 0, 2 * sizeof(uint32_t), s), "memset");
        HIPCHK(hipMemsetAsync(ctr + 5, 0, sizeof(uint32_t), s), "memset");
        HIPCHK(hipMemsetAsync(c64, 0, 3 * sizeof(unsigned long long), s), "memset");
        if (emit) HIPCHK(hipMemsetAsync(m.octr, 0, kPoolWords * sizeof(uint32_t), s), "memset");
    }
    // the table and list hold every filter match unless a region ran out
    const bool emitted = emit && hctr[5] == 0;
    uint32_t ov_used = 0;
    if (emitted)
        for (int q = 0; q < kEmitPools; ++q)
            ov_used = std::max(ov_used, std::min(hoctr[q * kEmitPoolStride], m.ov_pool));
    if (!emitted) {
        m.table = nullptr;
        HIPCHK(hipMemsetAsync(c64 + 2, 0, sizeof(unsigned long long), s), "memset");
    }
    uint32_t n_amb = hctr[1], n_tie = hctr[2];
    R->stats.n_tests = (int64_t)h64[0];
    R->stats.n_band = (int64_t)h64[1];
    tm.mark();  // 2

    // ---- band candidates: FP64 recheck on the GPU, the rest in binary128 on the host
    std::vector<uint32_t> recheck_pos;  // sorted A positions whose best must be re-ranked
    uint32_t n_host = 0;
    WEnt *xent = nullptr;  // band matches found inside (all-matches mode)
    uint32_t n_x = 0;
    if (n_amb > 0) {
        AmbInfo *dinfo = tmp.get_n<AmbInfo>(n_amb);
        uint8_t *dv = tmp.get_n<uint8_t>(n_amb);
        if (!dinfo || !dv) return fail(C3X_ENOMEM, "band buffers");
        if (shape == C3X_CIRCLE)
            hipLaunchKernelGGL(k_recheck<C3X_CIRCLE>, dim3(nblk(n_amb, 256)), dim3(256), 0, s, amb,
                               n_amb, arad, aidx, aellr, ix->radec, ix->pay64, ix->pay32, m.h_r,
                               nullptr, nullptr, nullptr, dinfo, dv);
        else
            hipLaunchKernelGGL(k_recheck<C3X_ELLIPSE>, dim3(nblk(n_amb, 256)), dim3(256), 0, s, amb,
                               n_amb, arad, aidx, aellr, ix->radec, ix->pay64, ix->pay32, m.h_r,
                               sa, sb, pa, dinfo, dv);
        HIPCHK(hipGetLastError(), "band recheck");
        std::vector<AmbInfo> info(n_amb);
        std::vector<uint8_t> vv(n_amb);
        HIPCHK(hipMemcpyAsync(info.data(), dinfo, n_amb * sizeof(AmbInfo), hipMemcpyDeviceToHost, s),
               "copy");
        HIPCHK(hipMemcpyAsync(vv.data(), dv, n_amb, hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(hipStreamSynchronize(s), "band recheck");
        std::vector<std::pair<unsigned long long, uint8_t>> ver(n_amb);
        std::vector<uint4> add;
        for (uint32_t k = 0; k < n_amb; ++k) {
            const AmbInfo &q = info[k];
            int in = vv[k];
            if (in == AMBIG) {
                ++n_host;
                in = shape == C3X_CIRCLE
                         ? c3x_q_circle(q.raA, q.decA, q.raB, q.decB, area->radius_arcsec)
                         : c3x_q_ellipse(q.raA, q.decA, q.raB, q.decB, q.a, q.b, q.pa,
                                         area->pa_zero_deg, area->pa_sense);
            }
            ver[k] = {((unsigned long long)q.i << 32) | q.j, (uint8_t)(in ? 1 : 0)};
            if (in) {
                add.push_back(make_uint4(q.i, q.idxA, q.idxB, q.j));
                recheck_pos.push_back(q.i);
            }
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
        uint4 *dadd = tmp.get_n<uint4>(add.size());
        if (!dvk || !dvi || !dadd) return fail(C3X_ENOMEM, "verdict table");
        if (all && !add.empty()) {
            xent = tmp.get_n<WEnt>(add.size());
            if (!xent) return fail(C3X_ENOMEM, "verdict table");
            n_x = (uint32_t)add.size();
        }
        HIPCHK(hipMemcpyAsync(dvk, vk.data(), n_amb * 8, hipMemcpyHostToDevice, s), "copy");
        HIPCHK(hipMemcpyAsync(dvi, vi.data(), n_amb, hipMemcpyHostToDevice, s), "copy");
        if (!add.empty()) {
            HIPCHK(hipMemcpyAsync(dadd, add.data(), add.size() * sizeof(uint4),
                                  hipMemcpyHostToDevice, s), "copy");
            hipLaunchKernelGGL(k_add_pairs, dim3(nblk(add.size(), 256)), dim3(256), 0, s, dadd,
                               (uint32_t)add.size(), astat, xent);
        }
        m.ver_key = dvk;
        m.ver_in = dvi;
        m.n_ver = n_amb;
        HIPCHK(hipStreamSynchronize(s), "verdict upload");  // host vectors go out of scope
    }
    R->stats.n_ambiguous = n_host;

    // ---- best matches the filter cannot rank: every match re-ranked in binary128
    if (n_tie > 0) {
        std::vector<uint2> ties(n_tie);
        HIPCHK(hipMemcpyAsync(ties.data(), tie, n_tie * sizeof(uint2), hipMemcpyDeviceToHost, s),
               "copy");
        HIPCHK(hipStreamSynchronize(s), "ties");
        for (const uint2 &t : ties) recheck_pos.push_back(t.x);
    }
    if (!recheck_pos.empty()) {
        std::sort(recheck_pos.begin(), recheck_pos.end());
        recheck_pos.erase(std::unique(recheck_pos.begin(), recheck_pos.end()), recheck_pos.end());
        uint32_t nc = (uint32_t)recheck_pos.size();
        uint32_t *dpos = tmp.get_n<uint32_t>(nc);
        if (!dpos) return fail(C3X_ENOMEM, "collect buffers");
        HIPCHK(hipMemcpyAsync(dpos, recheck_pos.data(), nc * 4, hipMemcpyHostToDevice, s), "copy");
        uint32_t col_cap = 8 * nc + 64;
        std::vector<ColEnt> col;
        for (int attempt = 0; attempt < 2; ++attempt) {
            ColEnt *dcol = (ColEnt *)tmp.get(col_cap * sizeof(ColEnt));
            if (!dcol) return fail(C3X_ENOMEM, "collect buffers");
            HIPCHK(hipMemsetAsync(ctr + 3, 0, sizeof(uint32_t), s), "memset");
            m.col_pos = dpos;
            m.n_col = nc;
            m.col_n = ctr + 3;
            m.col = dcol;
            m.col_cap = col_cap;
            launch_collect(m, shape, prec, s);
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
        std::vector<std::vector<const ColEnt *>> per(nc);
        for (const ColEnt &c : col) per[c.t].push_back(&c);
        std::vector<double2> ad(nc);
        std::vector<uint32_t> arow(nc);
        {
            double2 *dad = tmp.get_n<double2>(nc);
            uint32_t *drow = tmp.get_n<uint32_t>(nc);
            if (!dad || !drow) return fail(C3X_ENOMEM, "collect buffers");
            hipLaunchKernelGGL(k_gather_pos, dim3(nblk(nc, 256)), dim3(256), 0, s, dpos, nc, arad,
                               aidx, dad, drow);
            HIPCHK(hipMemcpyAsync(ad.data(), dad, nc * sizeof(double2), hipMemcpyDeviceToHost, s),
                   "copy");
            HIPCHK(hipMemcpyAsync(arow.data(), drow, nc * 4, hipMemcpyDeviceToHost, s), "copy");
            HIPCHK(hipStreamSynchronize(s), "collect gather");
        }
        std::vector<uint32_t> prow;
        std::vector<int32_t> pbi;
        std::vector<uint32_t> pbj;
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
            int w = c3x_q_best(ad[k].x, ad[k].y, (int)v.size(), r2.data(), d2.data(), ib.data());
            prow.push_back(arow[k]);
            pbi.push_back(ib[w]);
            pbj.push_back(v[w]->j);
        }
        if (!prow.empty()) {
            uint32_t np = (uint32_t)prow.size();
            uint32_t *d1 = tmp.get_n<uint32_t>(np), *d3 = tmp.get_n<uint32_t>(np);
            int32_t *d2 = tmp.get_n<int32_t>(np);
            if (!d1 || !d2 || !d3) return fail(C3X_ENOMEM, "best patch");
            HIPCHK(hipMemcpyAsync(d1, prow.data(), np * 4, hipMemcpyHostToDevice, s), "copy");
            HIPCHK(hipMemcpyAsync(d2, pbi.data(), np * 4, hipMemcpyHostToDevice, s), "copy");
            HIPCHK(hipMemcpyAsync(d3, pbj.data(), np * 4, hipMemcpyHostToDevice, s), "copy");
            hipLaunchKernelGGL(k_patch_best, dim3(nblk(np, 256)), dim3(256), 0, s, d1, d2, d3, np,
                               R->best_idx, astat);
            HIPCHK(hipStreamSynchronize(s), "best patch");
        }
        R->stats.n_best_ties = nc;
    }

    // ---- scan of the per-A counts (idxA order)
    int64_t *off = tmp.get_n<int64_t>(nA + 1);
    uint32_t *cnts = tmp.get_n<uint32_t>(nA);
    if (!off || !cnts) return fail(C3X_ENOMEM, "offsets");
    if (nA > 0)
        hipLaunchKernelGGL(k_counts, dim3(nblk(nA, 256)), dim3(256), 0, s, astat, nA, all ? 0 : 1,
                           cnts, all ? R->best_sep : nullptr);
    HIPCHK(scan_u32_to_i64(cnts, off, nA, off + nA, ws, s), "scan");
    int64_t P = 0;
    HIPCHK(hipMemcpyAsync(&P, off + nA, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(hipStreamSynchronize(s), "scan");
    tm.mark();  // 3

    // ---- outputs
    R->n_pairs = P;
    R->idxA = R->mem.get_n<int32_t>(P);
    R->idxB = R->mem.get_n<int32_t>(P);
    R->sep = R->mem.get_n<double>(P);
    if (!R->idxA || !R->idxB || !R->sep)
        return fail(C3X_ENOMEM, "result buffers (%lld pairs)", (long long)P);

    FinishArgs fa{};
    if (all) {
        // ---- overflow list and band matches to their places, or the write pass
        PairTmp *pt = tmp.get_n<PairTmp>(P);
        if (!pt) return fail(C3X_ENOMEM, "pair buffer (%lld pairs)", (long long)P);
        if (emitted) {
            if (ov_used > 0)
                hipLaunchKernelGGL(k_place_ov, dim3(nblk(ov_used, 256), kEmitPools), dim3(256), 0,
                                   s, m.ovl, m.ov_pool, m.octr, nA, off, P, pt, c64 + 2, ctr + 4);
        } else {
            m.off = off;
            m.tmp = pt;
            launch_match<1>(m, shape, prec, grid, s);
        }
        HIPCHK(hipGetLastError(), "write pass");
        if (n_x > 0)
            hipLaunchKernelGGL(k_place_x, dim3(nblk(n_x, 256)), dim3(256), 0, s, xent, n_x, aidx,
                               arad, ix->radec, nA, ix->nB, off, P, m.table, pt, c64 + 2, ctr + 4);
        HIPCHK(hipGetLastError(), "band matches");
        tm.mark();  // 4
        // ---- canonical order inside each segment, final records
        fa.nA = nA;
        fa.nB = ix->nB;
        fa.off = off;
        fa.table = m.table;
        fa.tmp = pt;
        fa.raA = ra;
        fa.decA = dec;
        fa.radecB = ix->radec;
        fa.bidx = R->best_idx;
        fa.oa = R->idxA;
        fa.ob = R->idxB;
        fa.os = R->sep;
        fa.bsep = R->best_sep;
        fa.err = ctr + 4;
        fa.seg_n = ctr + 6;
        fa.cap = (uint32_t)std::min<int64_t>(std::max<int64_t>(nA, 1), 1 << 22);
        fa.list = tmp.get_n<uint32_t>(fa.cap);
        fa.huge = tmp.get_n<uint32_t>(fa.cap);
        if (!fa.list || !fa.huge) return fail(C3X_ENOMEM, "segment lists");
        finish_segments(fa, s);
        HIPCHK(hipGetLastError(), "finalize");
        tm.mark();  // 5
    } else {
        tm.mark();  // 4
        tm.mark();  // 5
    }
    if (nA > 0 && !all)
        hipLaunchKernelGGL(k_best_sep, dim3(nblk(nA, 256)), dim3(256), 0, s, nA, ix->nB,
                           R->best_idx, astat, ra, dec, ix->radec, R->best_sep, off, P, R->idxA,
                           R->idxB, R->sep, ctr + 4);
    HIPCHK(hipGetLastError(), "best separations");
    tm.mark();  // 6
    HIPCHK(hipMemcpyAsync(hctr, ctr, sizeof(hctr), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(hipMemcpyAsync(h64, c64, sizeof(h64), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(hipStreamSynchronize(s), "c3x_match");
    if (all) {
        c3x_status st = finish_huge(fa, hctr + 6, s);
        if (st != C3X_OK) return st;
        if (hctr[7]) {
            HIPCHK(hipMemcpyAsync(hctr + 4, ctr + 4, sizeof(uint32_t), hipMemcpyDeviceToHost, s),
                   "copy");
            HIPCHK(hipStreamSynchronize(s), "c3x_match");
        }
    }
    if (hctr[4]) return fail(C3X_EDEVICE, "internal: count and write passes disagree (flags %u)",
                             hctr[4]);
    if (all && h64[2] != (unsigned long long)P)
        return fail(C3X_EDEVICE, "internal: %llu of %lld matches placed", h64[2], (long long)P);
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
    S.ms_sort_pairs = tm.ms(4, 6);
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
