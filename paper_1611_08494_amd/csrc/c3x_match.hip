// c3x_match.hip -- cross-match of catalogue A against a sky index.
//
// Paper Section 2.1 ("Sky" case): a region is centred on each A source and
// the B sources inside it are found by comparing their distance from the
// central object with the limits of the area; Section 2.2: the matches are
// kept as rows, all of them or only the best; Section 2.3: each source is
// tested only against the cells around it. Phases on one stream:
//   A prep     validate, key, sort A by cell (LDS radix sort); in sorted
//              order the coordinates, each source's candidate ranges of
//              sorted B positions (up to three zones, from the cell
//              directory) and ellipse frames; sources with many candidates
//              are listed for a wavefront each
//   count      one lane per sorted source (a wavefront per listed one): its
//              candidates decided by the certified filter, those inside the
//              filter's error band listed; the row's record (count, first
//              match, best) stored once in idxA order, later matches
//              appended to the overflow list
//   recheck    one thread per listed candidate: FP64 relative-accuracy form;
//              what it cannot certify is decided on the host in binary128
//   [host]     verdict table; near-tie best matches re-ranked in FP64, and
//              in binary128 from a collect pass where FP64 cannot rank them
//   scan       record counts -> int64 offsets (idxA order)
//   place      overflow-list and band matches to their segments (a write
//              pass repeats the count's decisions into the segments when an
//              overflow region ran out)
//   finalize   one thread per A row: best, the record's match, ranks by idxB
//              (canonical order) and separations; long segments sorted in
//              LDS or by the radix sort
//   best       best-only calls: one thread per A, the best's separation
// Decisions of the count, write and collect passes come from one device
// function compiled with -ffp-contract=off, so they agree bit for bit.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "c3x_host.h"
#include "c3x_sort.h"

namespace c3x {

constexpr int kMatchBlock = 256;
constexpr uint32_t kWideMin = 32;  // candidates from which a row gets a wavefront of its own
constexpr int64_t kFewRows = 1 << 21;  // fewer A rows: one lane each leaves the device idle
constexpr int kAKeyBits = 24;          // key bits that order catalogue A

// Key bits that order catalogue A in single calls: kAKeyBits, or
// C3X_A_KEY_BITS (8 to 32, for timing: fewer bits, fewer radix passes,
// longer unordered runs).
static int a_key_bits()
{
    if (const char *e = getenv("C3X_A_KEY_BITS")) {
        const int v = atoi(e);
        if (v >= 8 && v <= 32) return v;
    }
    return kAKeyBits;
}

constexpr uint32_t kNoKey = 0xffffffffu;  // no cell key: the lane's FP32 offsets are set
constexpr int kWavesPerBlock = kMatchBlock / 64;
constexpr int kShortSeg = 16;   // segments up to this long are ordered by the finalize kernel
constexpr int kSegLds = 2048;   // segments up to this long are sorted in LDS

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
                         uint32_t *__restrict__ keys, double2 *__restrict__ packed,
                         uint32_t *__restrict__ bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = ra[i], d = dec[i];
    packed[i] = make_double2(a, d);  // one 16-byte record per row for the gather
    bool ok = isfinite(a) && isfinite(d) && a >= 0.0 && a < 360.0 && fabs(d) <= 90.0;
    if (shape != C3X_CIRCLE) {
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
    keys[i] = zi.base + cell_in(zi, a);  // its value in the sort: the row i itself
}

// Margin on the ellipse form Q (or on each of the rectangle's forms Qu, Qv)
// for a filter whose tangent-plane components carry an absolute error
// <= c * kappa + lambda (c the chord, at most cmax where a decision is near:
// a for the ellipse, the half-diagonal for the rectangle). The error of
// su / a is then <= (c kappa + lambda) / a <= kappa cmax / a + lambda / a and
// that of sv / b <= kappa cmax / b + lambda / b; cmax / b <= 1 + a / b for
// both shapes. Covers the rounding of Q, the truncation of
// (theta / sin theta)^2 ~ 1 + c^2 / 3 and a factor-2 safety; returns a huge
// value when the filter cannot decide.
__device__ __forceinline__ double ell_margin(double ar, double br, double cmax, double kappa,
                                             double lambda, double u_round)
{
    double ia = 1.0 / ar, ib = 1.0 / br;
    double k1 = kappa * (1.0 + ar / br) * 1.01;
    double l1 = 1.5 * lambda * (ia + ib);
    double rho = 2.0 * k1 + 2.0 * l1 + (k1 + l1) * (k1 + l1) + 6.0 * u_round;
    double trunc = 0.2 * (cmax * cmax) * (cmax * cmax);
    double m = 2.0 * (2.0 * rho + trunc);
    return m > 0.25 ? 1e30 : m;
}

// Candidate ranges of a source at (ra, dec) with reach reach_deg: the
// window the match kernels would walk (same functions, same inputs), its
// cell ranges turned into sorted B positions now, with every zone's
// directory lookups independent of the others.
// Also flags, per zone, how its cells lie on the FP32 reference steps: a
// window inside one step, or across two (the source's own step and the one
// above or below it), is told apart by the parity each B payload carries;
// multi is set when a window crosses more than two steps.
__device__ __forceinline__ ARange a_ranges(const Grid &g, double ra, double dec, double reach_deg,
                                           bool &multi)
{
    ARange rg;
    rg.zlo = -1;
    rg.wide = 0;
    multi = false;
    double x, y, z;
    unit_vec(ra, dec, x, y, z);
    const double cosd = sqrt(x * x + y * y) * (1.0 - 1e-12) - 1e-15;
    const Window w = window_of(g, dec, cosd, reach_deg);
    bool ok = w.zhi - w.zlo < kRZ;
    uint32_t k0[kRZ], k1[kRZ];
#pragma unroll
    for (int q = 0; q < kRZ; ++q) {
        k0[q] = k1[q] = 0;
        const int zz = w.zlo + q;
        if (zz <= w.zhi && ok) {
            const ZoneInfo zi = g.zinfo[zz];
            uint32_t c0[2], c1[2];
            const int nr = zone_ranges(zi, w, ra, c0, c1);
            ok = nr == 1;
            k0[q] = zi.base + c0[0];
            k1[q] = zi.base + c1[0] + 1;
            const uint32_t s0 = ref_step(zi, c0[0]), s1 = ref_step(zi, c1[0]);
            const uint32_t sa = ref_step(zi, cell_in(zi, ra));
            if (s1 > s0 + 1u) multi = true;
            if (s1 != s0) rg.wide |= (uint16_t)((sa == s1 ? 3u : 1u) << (2 * q + 2));
        }
    }
#pragma unroll
    for (int q = 0; q < kRZ; ++q) {
        uint32_t j0 = 0, j1 = 0;
        if (w.zlo + q <= w.zhi && ok) {
            j0 = key_lower_bound(g, k0[q]);
            j1 = key_lower_bound(g, k1[q]);
        }
        if (j1 < j0) j1 = j0;
        ok = ok && j1 - j0 < 65535u;
        rg.j0[q] = j0;
        rg.n[q] = (uint16_t)(ok ? j1 - j0 : 0u);
    }
    if (ok) rg.zlo = w.zlo;
    return rg;
}

// Sorted A position i: its coordinates, candidate ranges and ellipse frame.
// rows (the sort's values) stay the sorted sources' idxA list. Invalid rows
// (already reported through k_prep_a's flag) are given the position (0, 0)
// and, for ellipses, a 1" circle, so every later loop stays bounded even
// before the host sees the error.
template <int SHAPE>
__global__ void k_gather_a(uint32_t *__restrict__ rows, const double2 *__restrict__ packed,
                           int64_t n,
                           const double *__restrict__ sa, const double *__restrict__ sb,
                           const double *__restrict__ pa, double pa_zero, int pa_sense,
                           double L_rad, Grid g, double reach_deg,
                           double2 *__restrict__ arad,
                           AEll *__restrict__ aell, AEllR *__restrict__ aellr,
                           ARange *__restrict__ arng, uint32_t wide_min, bool few,
                           uint32_t *__restrict__ wide, uint32_t *__restrict__ wide_n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t row = rows[i];
    if (row >= (uint64_t)n) {  // unreachable for a permutation; keeps every later use in bounds
        row = 0;
        rows[i] = 0;
    }
    const double2 rd = packed[row];
    double r = rd.x, d = rd.y;
    bool ok = isfinite(r) && isfinite(d) && r >= 0.0 && r < 360.0 && fabs(d) <= 90.0;
    double A = 1.0, B = 1.0, P = 0.0;
    if (SHAPE != C3X_CIRCLE) {
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
    bool multi;
    ARange rg = a_ranges(g, r, d, SHAPE == C3X_CIRCLE ? reach_deg : area_reach_deg(SHAPE, A, B),
                         multi);
    if (multi) rg.wide |= 2u;  // the mixed filter reads this row's cell keys
    if (wide_min) {
        // rows for the wavefront-per-source kernel: a window walked cell by
        // cell, 16 wide_min candidates or more, or wide_min or more and either
        // at least 4 times the mean of the wavefront's rows (one lane each, the
        // wavefront would wait on it) or too few rows (few) for one lane each
        // to fill the device
        const uint32_t nc = (uint32_t)rg.n[0] + rg.n[1] + rg.n[2];
        uint32_t sum = rg.zlo < 0 ? 0u : nc, cnt = 1;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            sum += __shfl_xor(sum, o);
            cnt += __shfl_xor(cnt, o);
        }
        const bool wd = rg.zlo < 0 || nc >= 16 * wide_min ||
                        (nc >= wide_min && (few || (uint64_t)nc * cnt >= 4ull * sum));
        rg.wide = (uint16_t)((rg.wide & ~1u) | (wd ? 1u : 0u));
        const unsigned long long wm = __ballot(wd);
        if (wm) {
            const int l0 = __builtin_ffsll((long long)wm) - 1;
            const int lane = (int)(threadIdx.x & 63u);
            uint32_t base = 0;
            if (lane == l0) base = atomicAdd(wide_n, (uint32_t)__popcll(wm));
            base = (uint32_t)__builtin_amdgcn_readlane((int)base, l0);
            if (wd)
                wide[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(wm >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)wm, 0u))] =
                    (uint32_t)i;
        }
    }
    arng[i] = rg;
    if (SHAPE != C3X_CIRCLE) {
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
        const double cmax = SHAPE == C3X_RECT ? sqrt(ar * ar + br * br) : ar;
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
        q.m64 = ell_margin(ar, br, cmax, kappa64, lambda64, kU);
        const double e32 = kU32 * 1.0001;
        double kappa32 = s3 * (e32 + 64.0 * kU) + 2.0 * s3 * e32 + 4.0 * e32;
        double lambda32 = 2.0 * s3 * e32 * L_rad + 2.0 * s3 * ev;
        double m32 = ell_margin(ar, br, cmax, kappa32, lambda32, e32);
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

// Thresholds and FP32 error bound of sorted A position i: the call's, or
// its job's in a batch.
template <bool BATCH>
__device__ __forceinline__ Thr lane_thr(const MatchArgs &m, uint32_t i, double &L)
{
    Thr t;
    if constexpr (BATCH) {
        const BJob &jb = m.jobs[m.ajob[i]];
        t.t64_in = jb.t64_in;
        t.t64_out = jb.t64_out;
        t.t32_in = jb.t32_in;
        t.t32_out = jb.t32_out;
        t.r_zero = jb.r_zero;
        L = jb.L;
    } else {
        t.t64_in = m.t64_in;
        t.t64_out = m.t64_out;
        t.t32_in = m.t32_in;
        t.t32_out = m.t32_out;
        t.r_zero = m.r_zero;
        L = m.L_rad;
    }
    return t;
}

struct LaneF32 {            // FP32 copies of the ellipse frame
    float ux, uy, uz, vx, vy, vz, ia, ib;
};

struct CellCache {          // A's offset from the reference of the current B cell
    uint32_t key;          // cell key last seen
    uint32_t ref;          // its reference: zone << kRefBits | RA-grid step (zones < 2^22:
                           // square-ish cells and fewer than 2^31 of them)
    float ax, ay, az;
};

// Batch: every B offset is from the job's centre, so is the lane's.
__device__ __forceinline__ void batch_ref(const MatchArgs &m, uint32_t i, const ARec &a,
                                          CellCache &cc)
{
    const BJob &jb = m.jobs[m.ajob[i]];
    cc.ax = (float)(a.x - jb.cx);
    cc.ay = (float)(a.y - jb.cy);
    cc.az = (float)(a.z - jb.cz);
}

// Calls f(z, j0, j1) for each candidate range of sorted A position i: the
// ranges found when A was prepared, else (single calls only) a walk of the
// cells. Returns false for a batch source without ranges.
template <bool BATCH, typename F>
__device__ __forceinline__ bool cand_ranges(const MatchArgs &m, uint32_t i, const ARec &a, F &&f)
{
    const ARange rg = m.arng[i];
    if (rg.zlo >= 0) {
#pragma unroll 1
        for (int q = 0; q < kRZ; ++q) {
            const uint32_t j0 = q == 0 ? rg.j0[0] : (q == 1 ? rg.j0[1] : rg.j0[2]);
            const uint32_t nq = q == 0 ? rg.n[0] : (q == 1 ? rg.n[1] : rg.n[2]);
            if (nq) f(rg.zlo + q, j0, j0 + nq);
        }
        return true;
    }
    if constexpr (BATCH) {
        return false;
    } else {
        for_each_range(m.g, a.ra, a.dec, a.cosd, a.reach_deg, f);
        return true;
    }
}

// Residual word of sorted B position j where decide uses it (single calls
// of the mixed path), else zero.
template <int PREC, bool BATCH>
__device__ __forceinline__ uint2 res_word(const MatchArgs &m, uint32_t j)
{
    if constexpr (PREC != C3X_FP64 && !BATCH) return m.res[j];
    else return make_uint2(0u, 0u);
}

// Fast certified filter of one candidate: IN, OUT, or AMBIG when the pair
// lies inside the filter's error band (then the FP64 relative-accuracy
// recheck decides it, in k_recheck). Also returns a squared chord: for a
// match of a single call its FP64 chord (the mixed filter's from the FP32
// payload and its residual, see chord_err), which ranks it and codes its
// separation; otherwise the filter's. Radius 0 is decided structurally here
// (same point), without a band. rw (have_rw): the candidate's residual word
// where the caller loaded it with the payload (the one-lane count pass: a
// match's chord then waits on no further load); otherwise it is loaded for
// matches only.
template <int SHAPE, int PREC, bool BATCH>
__device__ __forceinline__ int decide(const MatchArgs &m, const ARec &a, const AEll &e,
                                      const AEllR &er, const LaneF32 &f, CellCache &cc,
                                      const Thr &th, int z, const ZoneInfo &zi, double2 zr,
                                      uint32_t key, const PayOf<PREC> &b, uint32_t j, uint2 rw,
                                      bool have_rw, double &c2o)
{
    int d;
    if constexpr (PREC == C3X_FP64) {
        double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
        double c2 = fma(dx, dx, fma(dy, dy, dz * dz));
        c2o = c2;
        if constexpr (SHAPE == C3X_CIRCLE) {
            d = c2 <= th.t64_in ? IN : (c2 > th.t64_out ? OUT : AMBIG);
        } else {
            double su = fma(dx, e.ux, fma(dy, e.uy, dz * e.uz));
            double sv = fma(dx, e.vx, fma(dy, e.vy, dz * e.vz));
            double xu = su * e.ia, xv = sv * e.ib;
            const double t = fma(c2, 1.0 / 3.0, 1.0);
            if constexpr (SHAPE == C3X_ELLIPSE) {
                double qf = fma(xu, xu, xv * xv) * t;
                d = qf <= 1.0 - er.m64 ? IN : (qf > 1.0 + er.m64 ? OUT : AMBIG);
            } else {  // rectangle: |u| <= a and |v| <= b, each form on its own
                double qu = (xu * xu) * t, qv = (xv * xv) * t;
                d = (qu > 1.0 + er.m64 || qv > 1.0 + er.m64)
                        ? OUT
                        : ((qu <= 1.0 - er.m64 && qv <= 1.0 - er.m64) ? IN : AMBIG);
            }
        }
    } else {
        // batch: the offsets are from the job's centre, set once per lane
        if (!BATCH && key != cc.key) {
            cc.key = key;
            const uint32_t st = ref_step(zi, key - zi.base);
            const uint32_t rf = ((uint32_t)z << kRefBits) | st;
            if (rf != cc.ref) {
                cc.ref = rf;
                double rx, ry, rz;
                ref_vec(zr, st, rx, ry, rz);
                cc.ax = (float)(a.x - rx);
                cc.ay = (float)(a.y - ry);
                cc.az = (float)(a.z - rz);
            }
        }
        float dx = b.x - cc.ax, dy = b.y - cc.ay, dz = b.z - cc.az;
        float c2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        c2o = (double)c2;
        // single calls: the FP64 chord of a match, from the B offset restored
        // from the payload and its residual and A's FP64 offset from the same
        // reference
        auto chord64 = [&]() {
            double rx, ry, rz;
            ref_vec(zr, cc.ref & ((1u << kRefBits) - 1u), rx, ry, rz);
            const uint2 w = have_rw ? rw : m.res[j];
            const double ex = res_off(b.x, w, 0) - (a.x - rx);
            const double ey = res_off(b.y, w, 1) - (a.y - ry);
            const double ez = res_off(b.z, w, 2) - (a.z - rz);
            return fma(ex, ex, fma(ey, ey, ez * ez));
        };
        if constexpr (SHAPE == C3X_CIRCLE) {
            d = c2 <= th.t32_in ? IN : (c2 > th.t32_out ? OUT : AMBIG);
        } else {
            float su = fmaf(dx, f.ux, fmaf(dy, f.uy, dz * f.uz));
            float sv = fmaf(dx, f.vx, fmaf(dy, f.vy, dz * f.vz));
            float xu = su * f.ia, xv = sv * f.ib;
            const float t = fmaf(c2, 1.0f / 3.0f, 1.0f);
            float mm = er.m32;
            if constexpr (SHAPE == C3X_ELLIPSE) {
                float qf = fmaf(xu, xu, xv * xv) * t;
                d = mm == 0.0f ? AMBIG : (qf <= 1.0f - mm ? IN : (qf > 1.0f + mm ? OUT : AMBIG));
            } else {
                float qu = (xu * xu) * t, qv = (xv * xv) * t;
                d = mm == 0.0f ? AMBIG
                               : ((qu > 1.0f + mm || qv > 1.0f + mm)
                                      ? OUT
                                      : ((qu <= 1.0f - mm && qv <= 1.0f - mm) ? IN : AMBIG));
            }
        }
        if constexpr (!BATCH) {
            if (d == IN) c2o = chord64();
        }
    }
    if constexpr (SHAPE == C3X_CIRCLE) {
        if (th.r_zero) {
            d = same_point(a, m.coordB[pay_row(b)]) ? IN : OUT;
            if constexpr (!BATCH) {
                if (d == IN) c2o = 0.0;  // the same point: no angle
            }
        }
    }
    return d;
}

__device__ __forceinline__ int verdict(const MatchArgs &m, uint32_t i, uint32_t j)
{
    unsigned long long k = ((unsigned long long)i << 32) | j;
    const uint32_t n = m.n_ver_dev ? min(*m.n_ver_dev, m.n_ver) : m.n_ver;
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (m.ver_key[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    if (lo < n && m.ver_key[lo] == k) return m.ver_in[lo] ? IN : OUT;
    atomicOr(m.err_flag, 4u);
    return OUT;
}

// Verdict of a band candidate: the FP64 recheck again (the decision the
// recheck kernel took), then the table of host decisions for what it leaves
// open.
template <int SHAPE, bool BATCH>
__device__ __forceinline__ int band_verdict(const MatchArgs &m, uint32_t i, uint32_t j,
                                            const ARec &a)
{
    ARec q = a;
    q.cosd = cos_dec_acc(a.dec);
    int d;
    const double2 rb = m.coordB[brow(m, j)];
    if constexpr (SHAPE == C3X_ELLIPSE) d = recheck_ellipse(q, m.aellr[i], rb);
    else if constexpr (SHAPE == C3X_RECT) d = recheck_rect(q, m.aellr[i], rb);
    else d = recheck_circle(q, rb, BATCH ? m.jobs[m.ajob[i]].h_r : m.h_r);
    if (d != AMBIG && !m.force_host) return d;
    return verdict(m, i, j);
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

// Error bound of a single call's FP64 match chord at chord c (the ranking
// of its best matches): the FP64 unit vectors carry <= 32 u per component;
// L > 0: the B point restored from an FP32 offset of size <= L and its
// residual (within 2^-44 L, plus roundings of size u L), so 2^-43 L more
// per component; L = 0: the FP64 payload.
__device__ __forceinline__ double chord_err(double c, double L)
{
    const double s3 = 1.7320508075688772;
    const double eta = s3 * (64.0 * kU + kU * c + 0x1p-43 * L);
    return 2.0 * c * eta + eta * eta + 3.0 * kU * (c + eta) * (c + eta);
}

// ---------------------------------------------------------------------------- count / write

// A match's separation as the match passes leave it, without trigonometry:
// from the FP64 chord c < 1.38 the code -c^2 (the separation is 2 asin(c / 2),
// error ~1e-14 rad), 0 for c = 0, otherwise a quiet NaN: the separation is
// then computed from the coordinates of A and of the match's B row (the
// batch's mixed path codes every match so: it has no FP64 chord of its
// matches). Non-negative values are separations in arcsec.
__device__ __forceinline__ double sep_code(double c2)
{
    if (c2 < 1.9) return c2 > 0.0 ? -c2 : 0.0;
    return __longlong_as_double((long long)0x7ff8000000000000ull);
}
__device__ __forceinline__ double sep_code_coords()
{
    return __longlong_as_double((long long)0x7ff8000000000000ull);
}

__device__ __forceinline__ double sep_from_chord2(double c2)
{
    return 2.0 * asin(0.5 * sqrt(c2)) * (180.0 / kPi * 3600.0);
}

// ---------------------------------------------------------------------------- wavefront helpers

// Lane l's value, for every lane (l wavefront-uniform).
__device__ __forceinline__ uint32_t rl_u32(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ double rl_f64(double v, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = rl_u32((uint32_t)u, l), hi = rl_u32((uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// Lane rank among the lanes of mask hm below this one.
__device__ __forceinline__ uint32_t lane_rank(unsigned long long hm)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(hm >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)hm, 0u));
}

// One sorted A row of the count / write pass (one lane each), its counters
// added to tests, band and placed.
// MODE 0: count + best; MODE 1: write every filter match into the
// offsets from the count; MODE 2: count + best, the row's first kTab filter
// matches kept for its record, later ones written to the overflow list.
// BATCH: a batch of jobs (per-source thresholds and centre, local grids).
template <int SHAPE, int PREC, int MODE, bool BATCH>
__device__ __forceinline__ void match_row(const MatchArgs &m, uint32_t i,
                                          unsigned long long &tests, unsigned long long &band,
                                          unsigned long long &placed)
{
    using PayT = PayOf<PREC>;
    const PayT *pay;
    if constexpr (PREC == C3X_FP64) pay = m.pay64;
    else pay = m.pay32;

    bool active = i < (uint32_t)m.nA;
    ARec a{};
    AEll e{};
    AEllR er{};
    LaneF32 f{};
    ARange rg{};
    if (active) {
        double reach = m.reach_deg;
        if constexpr (SHAPE != C3X_CIRCLE) {
            e = m.aell[i];
            er = m.aellr[i];
            reach = area_reach_deg(SHAPE, er.a_arcsec, er.b_arcsec);
            f = LaneF32{(float)e.ux, (float)e.uy, (float)e.uz, (float)e.vx,
                        (float)e.vy, (float)e.vz, (float)e.ia, (float)e.ib};
        }
        rg = m.arng[i];
        a = load_a(m, i, reach);
    }
    // rows listed for the wavefront-per-source kernel are its to count
    if (MODE != 1 && !BATCH && active && m.wide_min && wide_row(rg)) active = false;
    double Lr = 0.0;
    const Thr th = lane_thr<BATCH>(m, active ? i : 0u, Lr);

    uint32_t cnt = 0;
    double b1 = INFINITY, b2 = INFINITY;
    uint32_t bidx = 0xffffffffu;
    uint32_t tb0 = 0;  // MODE 2: the row's first match
    double tc0 = 0.0;
    static_assert(kTab == 1, "one record slot");
    int64_t o = 0, oe = 0;
    if (MODE == 1 && active) {
        o = m.off[a.idx];
        oe = m.off[a.idx + 1];
    }
    CellCache cc{0xffffffffu, 0xffffffffu, 0.f, 0.f, 0.f};
    if (BATCH && active) batch_ref(m, i, a, cc);

    // A filter match as written: the separation coded from its FP64 chord;
    // the batch's mixed path leaves it to the coordinates (a pass after the
    // canonical order computes it from both rows' positions).
    auto coded = [&](const PayT &b, uint32_t j, double c2) -> PairTmp {
        PairTmp t;
        t.idxB = pay_row(b);
        t.j = j;
        if constexpr (PREC == C3X_FP64 || !BATCH) t.sep = sep_code(c2);
        else t.sep = sep_code_coords();
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
        }
        // a full region: one flag write per group, not one per match
        if (__ballot(slot >= m.ov_pool) && r == 0) atomicOr(m.ov_flag, 1u);
    };

    // One candidate: decide it, then count / rank it (MODE 0), write it
    // (MODE 1), or both (MODE 2). Band candidates are only listed.
    auto visit = [&](int z, const ZoneInfo &zi, double2 zr, uint32_t key, const PayT &b,
                     uint32_t j, uint2 rw, bool have_rw) {
        ++tests;
        double c2;
        int d = decide<SHAPE, PREC, BATCH>(m, a, e, er, f, cc, th, z, zi, zr, key, b, j, rw,
                                           have_rw, c2);
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
            if (cnt == 0) {
                tb0 = t.idxB;
                tc0 = t.sep;
            } else {
                overflow(cnt, t);
            }
        }
        if (MODE != 1) {
            ++cnt;
            if (c2 < b1 || (c2 == b1 && pay_row(b) < bidx)) {
                b2 = b1;
                b1 = c2;
                bidx = pay_row(b);
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

    if (active) {
        if (rg.zlo >= 0) {
            // the ranges found when A was prepared; candidates are loaded
            // kBatch at a time so that their loads overlap
            constexpr int kBatch = (PREC != C3X_FP64 && !BATCH) ? 2 : 4;
#pragma unroll 1
            for (int q = 0; q < kRZ; ++q) {
                const uint32_t j0 = q == 0 ? rg.j0[0] : (q == 1 ? rg.j0[1] : rg.j0[2]);
                const uint32_t nq = q == 0 ? rg.n[0] : (q == 1 ? rg.n[1] : rg.n[2]);
                if (nq == 0) continue;
                const int z = rg.zlo + q;
                ZoneInfo zi{};
                double2 zr{};
                if (!BATCH) zi = m.g.zinfo[z];
                if (!BATCH && PREC != C3X_FP64) zr = m.g.zref[z];
                // mixed: the zone's cells lie on one or two FP32 reference
                // steps (the source's own, and the one above or below it);
                // the lane's offsets from both are formed once here, and
                // each candidate's parity bit picks one -- no cell keys
                const bool par = PREC != C3X_FP64 && !BATCH && !(rg.wide & 2u);
                float oax = 0.f, oay = 0.f, oaz = 0.f, oox = 0.f, ooy = 0.f, ooz = 0.f;
                uint32_t pa = 0, rfa = 0, rfo = 0;
                if (par) {
                    const uint32_t sa = ref_step(zi, cell_in(zi, a.ra));
                    const uint32_t bits = (rg.wide >> (2 * q + 2)) & 3u;
                    const uint32_t so = bits == 1u ? sa + 1u : (bits == 3u ? sa - 1u : sa);
                    double rx, ry, rz;
                    ref_vec(zr, sa, rx, ry, rz);
                    oax = (float)(a.x - rx);
                    oay = (float)(a.y - ry);
                    oaz = (float)(a.z - rz);
                    oox = oax;
                    ooy = oay;
                    ooz = oaz;
                    if (so != sa) {
                        ref_vec(zr, so, rx, ry, rz);
                        oox = (float)(a.x - rx);
                        ooy = (float)(a.y - ry);
                        ooz = (float)(a.z - rz);
                    }
                    pa = sa & 1u;
                    rfa = ((uint32_t)z << kRefBits) | sa;
                    rfo = ((uint32_t)z << kRefBits) | (so & ((1u << kRefBits) - 1u));
                    cc.key = kNoKey;
                }
                for (uint32_t t = 0; t < nq; t += kBatch) {
                    PayT bb[kBatch];
                    uint32_t kk[kBatch];
                    uint2 rr[kBatch];
#pragma unroll
                    for (int u = 0; u < kBatch; ++u) {
                        const uint32_t jj = j0 + min(t + u, nq - 1);
                        bb[u] = pay[jj];
                        rr[u] = res_word<PREC, BATCH>(m, jj);
                        kk[u] = (PREC == C3X_FP64 || BATCH || par) ? kNoKey : m.g.keys[jj];
                    }
#pragma unroll
                    for (int u = 0; u < kBatch; ++u)
                        if (t + u < nq) {
                            if (par) {
                                const bool other = (bb[u].idx >> 31) != pa;
                                cc.ax = other ? oox : oax;
                                cc.ay = other ? ooy : oay;
                                cc.az = other ? ooz : oaz;
                                cc.ref = other ? rfo : rfa;
                            }
                            visit(z, zi, zr, kk[u], bb[u], j0 + t + u, rr[u], true);
                        }
                }
            }
        } else if constexpr (BATCH) {
            atomicOr(m.err_flag, 64u);  // the plan guarantees ranges
        } else {
            // split at RA 0/360, many zones or long ranges: walk the cells
            for_each_range(m.g, a.ra, a.dec, a.cosd, a.reach_deg, [&](int z, uint32_t j0, uint32_t j1) {
                const ZoneInfo zi = m.g.zinfo[z];
                const double2 zr = PREC != C3X_FP64 ? m.g.zref[z] : double2{};
                cc.key = cc.ref = 0xffffffffu;
                for (uint32_t j = j0; j < j1; ++j) {
                    const PayT b = pay[j];
                    visit(z, zi, zr, m.g.keys[j], b, j, make_uint2(0u, 0u), false);
                }
            });
        }
    }
    // a row's record is a scattered store (idxA order), the costliest of
    // the pass: rows without a match skip it when the records start at zero
    if (active && MODE != 1 && (cnt || !m.rec_zeroed)) {
        // the record keeps the first match (MODE 2): a second one puts the
        // best in the side table
        const bool side = MODE == 2 && cnt >= 2;
        RowRec r;
        r.n = cnt | (side ? kBestSide : 0u);
        r.b0 = MODE == 0 ? bidx : tb0;
        r.c0 = tc0;
        m.rec[a.idx] = r;
        if (side) m.best2[a.idx] = (int32_t)bidx;
        if (MODE == 2) placed += min(cnt, (uint32_t)kTab);
        if (cnt >= 2) {  // a near tie: the two best chords within 4 error bounds
            const double c = sqrt(b2);
            const double terr = PREC == C3X_FP64 ? c2_err<C3X_FP64>(c, Lr)
                                : (BATCH ? c2_err<C3X_MIXED>(c, Lr) : chord_err(c, Lr));
            if (b2 - b1 <= (4.0 + m.tie_widen) * terr) {
                uint32_t slot = atomicAdd(m.tie_n, 1u);
                if (slot < m.tie_cap) m.tie[slot] = make_uint2(i, a.idx);
            }
        }
    }
}

// A workgroup's counters: summed in LDS, then one atomic per counter.
template <int MODE>
__device__ __forceinline__ void add_counters(const MatchArgs &m, unsigned long long tests,
                                             unsigned long long band, unsigned long long placed)
{
    __shared__ unsigned long long s_tests, s_band, s_placed;
    if (threadIdx.x == 0) {
        s_tests = 0;
        s_band = 0;
        s_placed = 0;
    }
    __syncthreads();
    if (placed) atomicAdd(&s_placed, placed);
    if (tests) atomicAdd(&s_tests, tests);
    if (band) atomicAdd(&s_band, band);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_tests && MODE != 1) atomicAdd(stat_slot(m.n_tests), s_tests);
        if (s_band && MODE != 1) atomicAdd(stat_slot(m.n_band), s_band);
        if (s_placed) atomicAdd(stat_slot(m.n_placed), s_placed);
    }
}

// One lane per sorted A row, rows in order.
template <int SHAPE, int PREC, int MODE, bool BATCH>
__global__ __launch_bounds__(kMatchBlock) void k_match(MatchArgs m)
{
    unsigned long long tests = 0, band = 0, placed = 0;
    match_row<SHAPE, PREC, MODE, BATCH>(m, blockIdx.x * blockDim.x + threadIdx.x, tests, band,
                                        placed);  // blockDim.x <= kMatchBlock
    add_counters<MODE>(m, tests, band, placed);
}

// The batch's count pass as a persistent kernel: each workgroup takes
// `chunk` consecutive entries of `order` at a time from a counter (one
// atomic per chunk, not per tile: a single counter serialises its atomics),
// each entry a tile of blockDim.x consecutive sorted A rows, the costliest
// first, until none is left; the take is workgroup-uniform, so every lane
// of a workgroup leaves the loop together.
template <int PREC>
__global__ __launch_bounds__(kMatchBlock) void k_match_queue(MatchArgs m,
                                                             const uint32_t *__restrict__ order,
                                                             uint32_t n_items, uint32_t chunk,
                                                             uint32_t *__restrict__ qctr)
{
    __shared__ uint32_t s_item;
    unsigned long long tests = 0, band = 0, placed = 0;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(qctr, chunk);
        __syncthreads();
        const uint32_t it0 = s_item;
        __syncthreads();  // every lane has read it before the next take
        if (it0 >= n_items) break;
        const uint32_t it1 = min(it0 + chunk, n_items);
        for (uint32_t it = it0; it < it1; ++it) {
            const uint32_t tile = min(order[it], n_items - 1u);
            match_row<C3X_CIRCLE, PREC, 2, true>(m, tile * blockDim.x + threadIdx.x, tests, band,
                                                 placed);
        }
    }
    add_counters<2>(m, tests, band, placed);
}

// Cost of each job (the candidates its rows test, plus one per row): one
// workgroup per job over its sorted rows (a job's sorted rows take its own
// entries' places: [a_ent, a_ent + nA)).
__global__ void k_job_cost(const BJob *__restrict__ jobs, int nj, const ARange *__restrict__ arng,
                           float *__restrict__ cost)
{
    __shared__ float part[kMatchBlock / 64];
    for (int j = blockIdx.x; j < nj; j += gridDim.x) {
        const uint32_t a0 = jobs[j].a_ent, na = jobs[j].nA;
        float c = 0.f;
        for (uint32_t k = threadIdx.x; k < na; k += blockDim.x) {
            const ARange g = arng[a0 + k];
            c += 1.0f + (float)((uint32_t)g.n[0] + g.n[1] + g.n[2]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
        if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.f;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
            cost[j] = t;
        }
        __syncthreads();
    }
}

// Sort key of each tile of `tile` sorted A rows: its job's cost (the job of
// its first row) as the top 16 bits of a float (monotone), complemented, so
// that a stable sort puts the costliest jobs first and keeps each job's
// tiles together and in order (their B candidates stay close in memory).
__global__ void k_tile_cost(const uint32_t *__restrict__ ajob, const float *__restrict__ jcost,
                            int64_t nA, uint32_t tile, uint32_t n_items,
                            uint32_t *__restrict__ key, uint32_t *__restrict__ val)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_items) return;
    const int64_t r0 = min<int64_t>((int64_t)t * tile, nA - 1);
    key[t] = 0xffffu - (__float_as_uint(jcost[ajob[r0]]) >> 16);
    val[t] = t;
}

// Sources with many candidates (large areas, dense fields): one wavefront
// per listed source, lanes striding over its candidate ranges, so that the
// loads of a range are coalesced and no lane waits for a longer neighbour.
// Same outputs as k_match in MODE 0 / 2 for those rows: count, best by the
// filter's chord (near-ties listed), band candidates listed, the first kTab
// matches in the record and later ones in the overflow list.

template <int SHAPE, int PREC, int MODE>
__global__ __launch_bounds__(256) void k_match_wide(MatchArgs m)
{
    static_assert(MODE == 0 || MODE == 2, "count (+ emit) passes only");
    using PayT = PayOf<PREC>;
    __shared__ unsigned long long s_tests, s_band, s_placed;
    if (threadIdx.x == 0) {
        s_tests = 0;
        s_band = 0;
        s_placed = 0;
    }
    __syncthreads();
    const PayT *pay;
    if constexpr (PREC == C3X_FP64) pay = m.pay64;
    else pay = m.pay32;
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t nw = min(*m.wide_n, (uint32_t)m.nA);
    const uint32_t pool = wave & (kEmitPools - 1);
    unsigned long long tests = 0, band = 0, placed = 0;

    for (uint32_t w = wave; w < nw; w += nwaves) {
        const uint32_t i = min(m.wide[w], (uint32_t)m.nA - 1u);
        double reach = m.reach_deg;
        AEll e{};
        AEllR er{};
        LaneF32 f{};
        if constexpr (SHAPE != C3X_CIRCLE) {
            e = m.aell[i];
            er = m.aellr[i];
            reach = area_reach_deg(SHAPE, er.a_arcsec, er.b_arcsec);
            f = LaneF32{(float)e.ux, (float)e.uy, (float)e.uz, (float)e.vx,
                        (float)e.vy, (float)e.vz, (float)e.ia, (float)e.ib};
        }
        const ARec a = load_a(m, i, reach);
        double Lr = 0.0;
        const Thr th = lane_thr<false>(m, i, Lr);
        CellCache cc{0xffffffffu, 0xffffffffu, 0.f, 0.f, 0.f};
        uint32_t cnt = 0;  // wave-uniform
        double b1 = INFINITY, b2 = INFINITY;
        uint32_t bidx = 0xffffffffu;
        uint32_t tb0 = 0;
        double tc0 = 0.0;

        auto range = [&](int z, uint32_t j0, uint32_t j1) {
            const ZoneInfo zi = m.g.zinfo[z];
            const double2 zr = PREC != C3X_FP64 ? m.g.zref[z] : double2{};
            for (uint32_t t = j0; t < j1; t += 64) {
                const uint32_t j = t + (uint32_t)lane;
                const bool on = j < j1;
                int d = OUT;
                double c2 = INFINITY;
                PayT b{};
                if (on) {
                    b = pay[j];
                    const uint32_t key = PREC == C3X_FP64 ? 0u : m.g.keys[j];
                    ++tests;
                    d = decide<SHAPE, PREC, false>(m, a, e, er, f, cc, th, z, zi, zr, key, b, j,
                                                   make_uint2(0u, 0u), false, c2);
                }
                const unsigned long long am = __ballot(d == AMBIG);
                if (am) {
                    uint32_t base = 0;
                    if (lane == __builtin_ffsll((long long)am) - 1)
                        base = atomicAdd(m.amb_n, (uint32_t)__popcll(am));
                    base = rl_u32(base, __builtin_ffsll((long long)am) - 1);
                    if (d == AMBIG) {
                        ++band;
                        const uint32_t slot = base + lane_rank(am);
                        if (slot < m.amb_cap) m.amb[slot] = make_uint2(i, j);
                    }
                }
                const unsigned long long im = __ballot(d == IN);
                if (!im) continue;
                if (d == IN) {
                    if (c2 < b1 || (c2 == b1 && pay_row(b) < bidx)) {
                        b2 = b1;
                        b1 = c2;
                        bidx = pay_row(b);
                    } else if (c2 < b2) {
                        b2 = c2;
                    }
                }
                if (MODE == 2) {
                    const uint32_t k = cnt + lane_rank(im);
                    PairTmp pt{};
                    if (d == IN) {
                        pt.idxB = pay_row(b);
                        pt.j = j;
                        pt.sep = sep_code(c2);
                    }
                    if (cnt == 0) {  // the record's slot: the group's first lane
                        const int l = __builtin_ffsll((long long)im) - 1;
                        tb0 = rl_u32(pt.idxB, l);
                        tc0 = rl_f64(pt.sep, l);
                    }
                    const unsigned long long om = __ballot(d == IN && k >= (uint32_t)kTab);
                    if (om) {
                        const int l0 = __builtin_ffsll((long long)om) - 1;
                        uint32_t base = 0;
                        if (lane == l0)
                            base = atomicAdd(m.octr + pool * kEmitPoolStride,
                                             (uint32_t)__popcll(om));
                        base = rl_u32(base, l0);
                        const uint32_t slot = base + lane_rank(om);
                        const bool mine = d == IN && k >= (uint32_t)kTab;
                        if (mine && slot < m.ov_pool) {
                            OvEnt v;
                            v.idxA = a.idx;
                            v.k = k;
                            v.idxB = pt.idxB;
                            v.j = pt.j;
                            v.code = pt.sep;
                            m.ovl[(size_t)pool * m.ov_pool + slot] = v;
                        }
                        if (__ballot(mine && slot >= m.ov_pool) && lane == l0)
                            atomicOr(m.ov_flag, 1u);
                    }
                }
                cnt += (uint32_t)__popcll(im);
            }
        };
        const ARange rg = m.arng[i];
        if (rg.zlo >= 0) {
#pragma unroll 1
            for (int q = 0; q < kRZ; ++q) {
                const uint32_t j0 = q == 0 ? rg.j0[0] : (q == 1 ? rg.j0[1] : rg.j0[2]);
                const uint32_t nq = q == 0 ? rg.n[0] : (q == 1 ? rg.n[1] : rg.n[2]);
                if (nq) range(rg.zlo + q, j0, j0 + nq);
            }
        } else {
            for_each_range(m.g, a.ra, a.dec, a.cosd, a.reach_deg, range);
        }

        // the best two chords of the wave: minimum by (chord, idxB), then the
        // smallest of the rest
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double ob1 = __shfl_xor(b1, o), ob2 = __shfl_xor(b2, o);
            const uint32_t oidx = __shfl_xor(bidx, o);
            if (ob1 < b1 || (ob1 == b1 && oidx < bidx)) {
                b2 = fmin(b1, fmin(b2, ob2));
                b1 = ob1;
                bidx = oidx;
            } else {
                b2 = fmin(ob1, fmin(b2, ob2));
            }
        }
        if (lane == 0) {
            const bool side = MODE == 2 && cnt >= 2;
            RowRec r;
            r.n = cnt | (side ? kBestSide : 0u);
            r.b0 = MODE == 0 ? bidx : tb0;
            r.c0 = tc0;
            m.rec[a.idx] = r;
            if (side) m.best2[a.idx] = (int32_t)bidx;
            if (MODE == 2) placed += min(cnt, (uint32_t)kTab);
            if (cnt >= 2 &&
                b2 - b1 <= (4.0 + m.tie_widen) * (PREC == C3X_FP64 ? c2_err<C3X_FP64>(sqrt(b2), Lr)
                                                                   : chord_err(sqrt(b2), Lr))) {
                const uint32_t slot = atomicAdd(m.tie_n, 1u);
                if (slot < m.tie_cap) m.tie[slot] = make_uint2(i, a.idx);
            }
        }
    }
    if (placed) atomicAdd(&s_placed, placed);
    if (tests) atomicAdd(&s_tests, tests);
    if (band) atomicAdd(&s_band, band);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_tests) atomicAdd(stat_slot(m.n_tests), s_tests);
        if (s_band) atomicAdd(stat_slot(m.n_band), s_band);
        if (s_placed) atomicAdd(stat_slot(m.n_placed), s_placed);
    }
}

// Every match of the listed sorted A positions (best-match re-ranking): one
// wavefront per listed source, lanes striding over its candidate ranges.
template <int SHAPE, int PREC, bool BATCH>
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
    if constexpr (SHAPE != C3X_CIRCLE) {
        e = m.aell[i];
        er = m.aellr[i];
        reach = area_reach_deg(SHAPE, er.a_arcsec, er.b_arcsec);
        f = LaneF32{(float)e.ux, (float)e.uy, (float)e.uz, (float)e.vx,
                    (float)e.vy, (float)e.vz, (float)e.ia, (float)e.ib};
    }
    ARec a = load_a(m, i, reach);
    CellCache cc{0xffffffffu, 0xffffffffu, 0.f, 0.f, 0.f};
    if (BATCH) batch_ref(m, i, a, cc);
    double Lr;
    const Thr th = lane_thr<BATCH>(m, i, Lr);
    cand_ranges<BATCH>(m, i, a, [&](int z, uint32_t j0, uint32_t j1) {
        ZoneInfo zi{};
        double2 zr{};
        if (!BATCH) zi = m.g.zinfo[z];
        if (!BATCH && PREC != C3X_FP64) zr = m.g.zref[z];
        for (uint32_t j = j0 + threadIdx.x; j < j1; j += 64) {
            const PayT b = pay[j];
            double c2;
            int d = decide<SHAPE, PREC, BATCH>(m, a, e, er, f, cc, th, z, zi, zr, m.g.keys[j], b, j,
                                               make_uint2(0u, 0u), false, c2);
            if (d == AMBIG) d = band_verdict<SHAPE, BATCH>(m, i, j, a);
            if (d != IN) continue;
            uint32_t slot = atomicAdd(m.col_n, 1u);
            if (slot < m.col_cap) {
                double2 rb = m.coordB[pay_row(b)];
                ColEnt ce;
                ce.t = t;
                ce.idxB = pay_row(b);
                ce.j = j;
                ce.pad = 0;
                ce.ra = rb.x;
                ce.dec = rb.y;
                ((ColEnt *)m.col)[slot] = ce;
            }
        }
    });
}

// (c2, idxB, j) candidates of the FP64 re-ranking, ordered by (c2, idxB).
struct Cand {
    double c2;
    uint32_t idxB, j;
};
__device__ __forceinline__ bool cand_less(const Cand &x, const Cand &y)
{
    return x.c2 < y.c2 || (x.c2 == y.c2 && x.idxB < y.idxB);
}
__device__ __forceinline__ Cand cand_shfl_xor(const Cand &x, int o)
{
    Cand y;
    const long long b = __double_as_longlong(x.c2);
    y.c2 = __longlong_as_double(((long long)(uint32_t)__shfl_xor((int)(b >> 32), o) << 32) |
                                (uint32_t)__shfl_xor((int)(uint32_t)b, o));
    y.idxB = (uint32_t)__shfl_xor((int)x.idxB, o);
    y.j = (uint32_t)__shfl_xor((int)x.j, o);
    return y;
}

// Best-match re-ranking of the listed sorted A positions (rows whose two
// nearest filter matches are within the filter's error, and rows with band
// matches found inside): one wavefront per row. Every match is re-decided
// (filter, then the band verdicts) and ranked by its FP64 squared chord
// from the FP64 unit vectors (error c2_err<FP64>); when the runner-up is
// further than 4 such errors the best is certain and written to the side
// table (the row's record flagged kBestSide), otherwise the row is listed
// for the host's binary128 ranking.
template <int SHAPE, int PREC, bool BATCH>
__device__ __forceinline__ void rerank_one(const MatchArgs &m, uint32_t i,
                                           uint32_t *__restrict__ unc_n,
                                           uint32_t *__restrict__ unc)
{
    using PayT = PayOf<PREC>;
    const PayT *pay;
    if constexpr (PREC == C3X_FP64) pay = m.pay64;
    else pay = m.pay32;
    AEll e{};
    AEllR er{};
    LaneF32 f{};
    double reach = m.reach_deg;
    if constexpr (SHAPE != C3X_CIRCLE) {
        e = m.aell[i];
        er = m.aellr[i];
        reach = area_reach_deg(SHAPE, er.a_arcsec, er.b_arcsec);
        f = LaneF32{(float)e.ux, (float)e.uy, (float)e.uz, (float)e.vx,
                    (float)e.vy, (float)e.vz, (float)e.ia, (float)e.ib};
    }
    const ARec a = load_a(m, i, reach);
    CellCache cc{0xffffffffu, 0xffffffffu, 0.f, 0.f, 0.f};
    if (BATCH) batch_ref(m, i, a, cc);
    double Lr;
    const Thr th = lane_thr<BATCH>(m, i, Lr);
    Cand b1{INFINITY, 0xffffffffu, 0u}, b2{INFINITY, 0xffffffffu, 0u};
    cand_ranges<BATCH>(m, i, a, [&](int z, uint32_t j0, uint32_t j1) {
        ZoneInfo zi{};
        double2 zr{};
        if (!BATCH) zi = m.g.zinfo[z];
        if (!BATCH && PREC != C3X_FP64) zr = m.g.zref[z];
        for (uint32_t j = j0 + threadIdx.x; j < j1; j += 64) {
            const PayT b = pay[j];
            double c2;
            int d = decide<SHAPE, PREC, BATCH>(m, a, e, er, f, cc, th, z, zi, zr, m.g.keys[j], b, j,
                                               make_uint2(0u, 0u), false, c2);
            if (d == AMBIG) d = band_verdict<SHAPE, BATCH>(m, i, j, a);
            if (d != IN) continue;
            // the FP64 unit vector: the FP64 payload's, or made the same way
            // (unit_vec of the row's coordinates) for the mixed index
            double bx, by, bz;
            if constexpr (PREC == C3X_FP64) {
                bx = b.x;
                by = b.y;
                bz = b.z;
            } else {
                const double2 rb = m.coordB[pay_row(b)];
                unit_vec(rb.x, rb.y, bx, by, bz);
            }
            const double dx = bx - a.x, dy = by - a.y, dz = bz - a.z;
            const Cand c{fma(dx, dx, fma(dy, dy, dz * dz)), pay_row(b), j};
            if (cand_less(c, b1)) {
                b2 = b1;
                b1 = c;
            } else if (cand_less(c, b2)) {
                b2 = c;
            }
        }
    });
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const Cand y1 = cand_shfl_xor(b1, o), y2 = cand_shfl_xor(b2, o);
        const bool mine = cand_less(b1, y1);
        const Cand lo = mine ? b1 : y1, hi = mine ? y1 : b1;
        Cand s2 = cand_less(b2, y2) ? b2 : y2;
        if (cand_less(hi, s2)) s2 = hi;
        b1 = lo;
        b2 = s2;
    }
    if (threadIdx.x == 0 && b1.idxB != 0xffffffffu) {
        const uint32_t row = a.idx;
        const bool sure = b2.idxB == 0xffffffffu ||
                          b2.c2 - b1.c2 > (4.0 + m.tie_widen) * c2_err<C3X_FP64>(sqrt(b2.c2), 0.0);
        if (sure) {
            m.best2[row] = (int32_t)b1.idxB;
            atomicOr(&m.rec[row].n, kBestSide);
        } else {
            unc[atomicAdd(unc_n, 1u)] = i;
        }
    }
}

// One wavefront per listed row (grid-stride over the list; the count may
// live on the device).
template <int SHAPE, int PREC, bool BATCH>
__global__ __launch_bounds__(64) void k_rerank(MatchArgs m, const uint32_t *__restrict__ pos,
                                               uint32_t n, const uint32_t *__restrict__ n_dev,
                                               uint32_t *__restrict__ unc_n,
                                               uint32_t *__restrict__ unc)
{
    const uint32_t nn = n_dev ? min(n, *n_dev) : n;
    for (uint32_t t = blockIdx.x; t < nn; t += gridDim.x)
        rerank_one<SHAPE, PREC, BATCH>(m, pos[t], unc_n, unc);
}

// ---------------------------------------------------------------------------- small kernels

// One thread per band candidate: the FP64 relative-accuracy recheck (error
// <= ~90 u against a 2^-40 margin). Writes 0 (out), 1 (in) or 2 (still
// undecided: the host decides it in binary128), with what the host needs.
// FP64 recheck of the band candidates the count pass listed (their number
// is on the device): those it finds inside join the matches list `in`, those
// it cannot decide go to `hl` for binary128 on the host; outside ones drop.
// force_host (a forced path for tests): every one goes to `hl`.
template <int SHAPE>
__global__ void k_recheck(const uint2 *__restrict__ band, const uint32_t *__restrict__ n_band,
                          uint32_t cap, const double2 *__restrict__ arad,
                          const uint32_t *__restrict__ aidx, const AEllR *__restrict__ aellr,
                          const double2 *__restrict__ coordB, const Pay64 *__restrict__ p64,
                          const Pay32 *__restrict__ p32, double h_r, const double *__restrict__ sa,
                          const double *__restrict__ sb, const double *__restrict__ pa,
                          uint4 *__restrict__ in, uint32_t *__restrict__ n_in,
                          AmbInfo *__restrict__ hl, uint32_t *__restrict__ n_hl, int force_host)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= min(*n_band, cap)) return;
    uint2 q = band[t];
    double2 ad = arad[q.x];
    uint32_t row = aidx[q.x];
    const uint32_t idxB = BRows{p64, p32}(q.y);
    double2 rb = coordB[idxB];
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
    else if (SHAPE == C3X_RECT) d = recheck_rect(a, aellr[q.x], rb);
    else d = recheck_ellipse(a, aellr[q.x], rb);
    if (force_host) d = AMBIG;
    if (d == OUT) return;
    if (d == IN) {
        in[atomicAdd(n_in, 1u)] = make_uint4(q.x, row, idxB, q.y);  // at most one per band entry
        return;
    }
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
    r.idxB = idxB;
    hl[atomicAdd(n_hl, 1u)] = r;
}

// Forced band (a test path): ellipse and rectangle margins of 3 make the
// filter decide nothing inside and nothing within twice the axes outside, so
// every such candidate is listed for the FP64 recheck.
// A margin was at most 1/4 where the filter may decide (an FP32 margin of 0
// marks a row the FP32 filter leaves wholly to the recheck, and stays), so a
// candidate it still finds outside lies truly outside.
__global__ void k_force_band_margins(AEllR *__restrict__ er, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    er[t].m64 = fmax(er[t].m64, 3.0);
    if (er[t].m32 != 0.0f) er[t].m32 = fmaxf(er[t].m32, 3.0f);
}

// Sorted A positions whose best match is re-ranked: the near-ties, then the
// rows that gained a band match.
__global__ void k_rerank_rows(const uint2 *__restrict__ tie, uint32_t n_tie,
                              const uint4 *__restrict__ bin, uint32_t n_bin,
                              uint32_t *__restrict__ pos)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tie) pos[t] = tie[t].x;
    else if (t < n_tie + n_bin) pos[t] = bin[t - n_tie].x;
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
// position): each is counted in its row's record, and listed as the k-th
// match of its source.
__global__ void k_add_pairs(const uint4 *__restrict__ in, uint32_t n, RowRec *rec,
                            WEnt *__restrict__ out)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint4 q = in[t];
    const uint32_t k = atomicAdd(&rec[q.y].n, 1u) & kCountMask;
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
    bool ok = t < min(octr[blockIdx.y * kEmitPoolStride], ov_pool);
    if (ok) {
        const OvEnt v = ovl[(size_t)blockIdx.y * ov_pool + t];
        if (v.idxA >= (uint64_t)nA) {
            atomicOr(err, 16u);
            ok = false;
        } else {
            const int64_t o = off[v.idxA], oe = off[v.idxA + 1];
            const int64_t p = o + v.k;
            if (v.k < (uint32_t)kTab || p >= oe || oe > P) {
                atomicOr(err, 1u);
                ok = false;
            } else {
                PairTmp x;
                x.idxB = v.idxB;
                x.j = v.j;
                x.sep = v.code;
                tmp[p] = x;
            }
        }
    }
    // one count per wavefront
    const unsigned long long pm = __ballot(ok);
    if (pm && (threadIdx.x & 63u) == (uint32_t)(__builtin_ffsll((long long)pm) - 1))
        atomicAdd(stat_slot(placed), (unsigned long long)__popcll(pm));
}

// One thread per band match found inside: to its row's record (k < kTab,
// when the single pass filled the records) or its place in the idxA-order
// segments, with its separation.
__global__ void k_place_x(const WEnt *__restrict__ xent, uint32_t nx,
                          const uint32_t *__restrict__ nx_dev,
                          const uint32_t *__restrict__ aidx, const double2 *__restrict__ arad,
                          const double2 *__restrict__ coordB, int64_t nA, int64_t nB,
                          const int64_t *__restrict__ off, int64_t P, RowRec *__restrict__ rec,
                          int use_rec, PairTmp *__restrict__ tmp,
                          unsigned long long *__restrict__ placed,
                          uint32_t *__restrict__ err)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nx || (nx_dev && t >= *nx_dev)) return;
    const WEnt e = xent[t];
    if (e.i >= (uint64_t)nA || e.idxB >= (uint64_t)nB) {
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
    const double2 ra = arad[e.i], rb = coordB[e.idxB];
    PairTmp x;
    x.idxB = e.idxB;
    x.j = e.j;
    x.sep = sep_rare(ra.x, ra.y, rb.x, rb.y);
    if (use_rec && e.k < (uint32_t)kTab) {
        rec[a].b0 = x.idxB;
        rec[a].c0 = x.sep;
    } else {
        tmp[p] = x;
    }
    atomicAdd(stat_slot(placed), 1ull);
}

__global__ void k_patch_best(const uint32_t *__restrict__ rows, const int32_t *__restrict__ bi,
                             uint32_t n, RowRec *rec, int32_t *__restrict__ best2)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    best2[rows[t]] = bi[t];
    atomicOr(&rec[rows[t]].n, kBestSide);
}

// Best matches decided on the host after the outputs exist: the row's best
// idxB, and its separation as written in the row's segment (ordered by idxB).
__global__ void k_patch_out(const uint32_t *__restrict__ rows, const int32_t *__restrict__ bi,
                            uint32_t n, const int64_t *__restrict__ off,
                            const int32_t *__restrict__ ob, const double *__restrict__ os,
                            int32_t *__restrict__ best_idx, double *__restrict__ best_sep,
                            uint32_t *__restrict__ err)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t a = rows[t];
    int64_t lo = off[a], hi = off[a + 1];
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (ob[mid] < bi[t]) lo = mid + 1;
        else hi = mid;
    }
    if (lo < off[a + 1] && ob[lo] == bi[t]) {
        best_idx[a] = bi[t];
        best_sep[a] = os[lo];
    } else {
        atomicOr(err, 128u);
    }
}

// BEST-only output: one record per row that has a match.
__global__ void k_nonzero(const RowRec *__restrict__ rec, int64_t n, uint32_t *__restrict__ out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = (rec[t].n & kCountMask) ? 1u : 0u;
}

// Separation (arcsec) of a coded match (see sep_code). A chord below 0.1
// uses the Maclaurin series of arcsin, 2 asin(x) = 2x (1 + x^2/6 + 3x^4/40
// + ...), x = c/2, to x^15 (truncation below 1e-20 relative); larger chords
// and the coordinate form are left to final_write.
__device__ __forceinline__ double theta_small(double c2)
{
    const double x2 = 0.25 * c2;
    double p = 143.0 / 10240.0;
    p = fma(p, x2, 231.0 / 13312.0);
    p = fma(p, x2, 63.0 / 2816.0);
    p = fma(p, x2, 35.0 / 1152.0);
    p = fma(p, x2, 5.0 / 112.0);
    p = fma(p, x2, 3.0 / 40.0);
    p = fma(p, x2, 1.0 / 6.0);
    p = fma(p, x2, 1.0);
    return sqrt(c2) * p * (180.0 / kPi * 3600.0);
}

// Separation (arcsec) from the coordinates of A (pa) and of B (pb): the
// FP64 chord of their unit vectors (a few units of rounding per component:
// ~1e-10 arcsec), the full formula near the antipode.
__device__ __noinline__ double sep_from_coords(double2 pa, double2 pb)
{
    double ax, ay, az, bx, by, bz;
    unit_vec(pa.x, pa.y, ax, ay, az);
    unit_vec(pb.x, pb.y, bx, by, bz);
    const double dx = bx - ax, dy = by - ay, dz = bz - az;
    const double c2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (c2 < 0.01) return theta_small(c2);
    if (c2 < 1.9) return 2.0 * asin(0.5 * sqrt(c2)) * (180.0 / kPi * 3600.0);
    return sep_arcsec_rd(pa.x, pa.y, pb.x, pb.y);
}

// Final record of one match: idxA, idxB and the decoded separation; the
// best match's separation too. coordA: A coordinates by output row a;
// coordB: B coordinates by output idxB (before any job-local renumbering).
// defer: a separation to take from the coordinates is left as the code
// (NaN) for k_sep_fix, which computes them all in one parallel pass. Used
// by the segment kernels; k_finalize writes its common cases itself.
__device__ __forceinline__ void final_write(int64_t q, int64_t a, const PairTmp &x, int64_t nB,
                                            const double2 *__restrict__ coordA,
                                            const double2 *__restrict__ coordB, int32_t best,
                                            int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                                            double *__restrict__ os, double *__restrict__ bsep,
                                            uint32_t *__restrict__ err, bool defer)
{
    double s = x.sep;
    if (!(s >= 0.0)) {
        if (s > -0.01) {
            s = theta_small(-s);
        } else if (s < 0.0) {
            s = 2.0 * asin(0.5 * sqrt(-s)) * (180.0 / kPi * 3600.0);
        } else if (defer) {
            oa[q] = (int32_t)a;
            ob[q] = (int32_t)x.idxB;
            os[q] = sep_code_coords();
            return;
        } else if (x.idxB < (uint64_t)nB) {
            s = sep_from_coords(coordA[a], coordB[x.idxB]);
        } else {
            atomicOr(err, 16u);
            s = NAN;
        }
    }
    oa[q] = (int32_t)a;
    ob[q] = (int32_t)x.idxB;
    os[q] = s;
    if (best == (int32_t)x.idxB) bsep[a] = s;
}

// One thread per A row: its best match and, in all-matches mode, its
// segment. A row's k-th match is in its record for k < kTab (when the
// single pass filled the records) and at offset off + k of its segment
// otherwise. A short segment (<= kShortSeg) is finished here: the
// canonical position of each match is its rank by idxB (unique in a
// segment). A longer one has its record's match copied into the segment
// and is listed (seg_n, seg_list) for k_seg_lds, which finishes it.
__global__ void k_finalize(int64_t nA, int64_t nB, int64_t pcap, const int64_t *__restrict__ off,
                           const RowRec *__restrict__ rec, const int32_t *__restrict__ best2,
                           int use_rec, PairTmp *__restrict__ tmp,
                           int32_t *__restrict__ best_idx,
                           int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                           double *__restrict__ os, double *__restrict__ bsep,
                           uint32_t *__restrict__ err, uint32_t *__restrict__ open_flag,
                           uint32_t *__restrict__ seg_n,
                           uint32_t *__restrict__ seg_list, uint32_t seg_cap)
{
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nA) return;
    const int64_t o = off[a], len = off[a + 1] - o;
    bsep[a] = NAN;
    if (o + len > pcap) {  // outputs sized for fewer pairs (a batch replay)
        atomicOr(err, 1u);
        return;
    }
    if (len <= 0) {
        best_idx[a] = -1;
        return;
    }
    const RowRec r = rec[a];
    const int32_t best = row_best(r, best2, a);
    best_idx[a] = best;
    const int nt = use_rec ? (int)min<int64_t>(len, kTab) : 0;
    PairTmp x0;  // the record's slot
    x0.idxB = r.b0;
    x0.j = 0;
    x0.sep = r.c0;
    if (len > kShortSeg) {  // the record's match joins the segment; listed for k_seg_lds
        if (nt > 0) tmp[o] = x0;
        const uint32_t slot = atomicAdd(seg_n, 1u);  // (long segments are few)
        if (slot < seg_cap) seg_list[slot] = (uint32_t)a;
        return;
    }
    // canonical position of a match: its rank by idxB (unique in a row)
    auto rank_of = [&](uint32_t ib) {
        int rk = 0;
        if (nt > 0) rk += x0.idxB < ib;
        for (int y = nt; y < len; ++y) rk += tmp[o + y].idxB < ib;
        return rk;
    };
    // a separation that needs more than the small-chord series (a chord of
    // 0.1 or more, or a NaN code: the coordinates') keeps its code for
    // k_sep_fix; keeping those paths out of this kernel halves its registers
    auto put = [&](const PairTmp &x) {
        const int64_t q = o + rank_of(x.idxB);
        double sp = x.sep;
        const bool open = !(sp >= 0.0) && !(sp > -0.01);
        if (!(sp >= 0.0) && !open) sp = theta_small(-sp);
        oa[q] = (int32_t)a;
        ob[q] = (int32_t)x.idxB;
        os[q] = sp;
        if (!open) {
            if (best == (int32_t)x.idxB) bsep[a] = sp;
        } else if (x.idxB >= (uint64_t)nB) {
            atomicOr(err, 16u);
        }
        // one plain store of the flag per wavefront (every writer writes 1)
        const unsigned long long om = __ballot(open);
        if (open_flag && om && (int)__lane_id() == __builtin_ffsll((long long)om) - 1)
            *open_flag = 1u;
    };
    if (nt > 0) put(x0);
    for (int q = nt; q < len; ++q) put(tmp[o + q]);
}

// BEST-only mode, one thread per A row: the best match, its separation and
// the compacted (idxA, idxB, sep) pair.
__global__ void k_best_sep(int64_t n, int64_t nB, const RowRec *__restrict__ rec,
                           const int32_t *__restrict__ best2,
                           const double *__restrict__ raA, const double *__restrict__ decA,
                           const double2 *__restrict__ coordB,
                           int32_t *__restrict__ bidx,
                           double *__restrict__ bsep, const int64_t *__restrict__ off, int64_t P,
                           int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                           double *__restrict__ os, uint32_t *__restrict__ err)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t b = off[t + 1] > off[t] ? row_best(rec[t], best2, t) : -1;
    bidx[t] = b;
    if (b < 0) {
        bsep[t] = NAN;
        return;
    }
    if (b >= nB) {
        atomicOr(err, 16u);
        return;
    }
    const double2 rb = coordB[b];
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

// Segments longer than kShortSeg (listed by the finalize kernel), one workgroup at a time over the list
// (the grid does not depend on the list's length): segments of up to
// kSegLds matches are sorted by idxB in LDS (bitonic network over
// idxB << 32 | position; idxB is unique in a segment) and written out in
// final form; longer ones are listed for the host-driven radix sort.
__global__ __launch_bounds__(256) void k_seg_lds(const int64_t *__restrict__ off,
                                                 const uint32_t *__restrict__ cnt,
                                                 const uint32_t *__restrict__ list, uint32_t cap,
                                                 const PairTmp *__restrict__ tmp, int64_t nB,
                                                 int64_t pcap,
                                                 const double2 *__restrict__ coordA,
                                                 const double2 *__restrict__ coordB,
                                                 const RowRec *__restrict__ rec,
                                                 const int32_t *__restrict__ best2,
                                                 int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                                                 double *__restrict__ os, double *__restrict__ bsep,
                                                 uint32_t *__restrict__ huge_n,
                                                 uint32_t *__restrict__ huge,
                                                 uint32_t *__restrict__ err, int defer)
{
    __shared__ unsigned long long v[kSegLds];
    const uint32_t nseg = min(*cnt, cap);
    for (uint32_t b = blockIdx.x; b < nseg; b += gridDim.x) {
        const uint32_t a = list[b];
        const int64_t o = off[a];
        if (off[a + 1] > pcap) continue;  // reported by the finalize kernel
        const int len = (int)min<int64_t>(off[a + 1] - o, 1 << 30);
        if (len > kSegLds) {
            if (threadIdx.x == 0) {
                uint32_t s = atomicAdd(huge_n, 1u);
                if (s < cap) huge[s] = a;
            }
            // until finish_huge writes them, the segment's slots say "no row"
            // (k_sep_fix skips them)
            for (int k = threadIdx.x; k < len; k += blockDim.x) oa[o + k] = -1;
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
        const int32_t best = row_best(rec[a], best2, a);
        for (int k = threadIdx.x; k < len; k += blockDim.x)
            final_write(o + k, a, tmp[o + (uint32_t)v[k]], nB, coordA, coordB, best, oa, ob, os,
                        bsep, err, defer != 0);
        __syncthreads();  // v is reused by the next segment
    }
}

// The separations the final passes left as codes: a chord of 0.1 or more
// (the arcsine) and NaN codes, taken from both rows' coordinates (the
// batch's mixed matches, which carry no FP64 chord, and separations near
// 90 deg or more); the best match's separation with them. Grid-stride over
// the pairs written (ptot: their count; P: the outputs' capacity); with
// open_flag given, nothing is done unless the finalize kernel set it. The
// slots of rows that finish_huge orders later say idxA -1 and are skipped.
__global__ void k_sep_fix(int64_t P, const int64_t *__restrict__ ptot, int64_t nA, int64_t nB,
                          const int32_t *__restrict__ oa,
                          const int32_t *__restrict__ ob, double *__restrict__ os,
                          const double2 *__restrict__ coordA,
                          const double2 *__restrict__ coordB,
                          const int32_t *__restrict__ best_idx, double *__restrict__ bsep,
                          const uint32_t *__restrict__ open_flag)
{
    if (open_flag && *open_flag == 0u) return;  // nothing was left open
    const int64_t n = min(P, max(*ptot, (int64_t)0));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const double c = os[q];
        if (c >= 0.0) continue;  // final
        const int32_t a = oa[q], b = ob[q];
        if (a < 0 || a >= nA || b < 0 || b >= nB) continue;
        double sp;
        if (c > -0.01) sp = theta_small(-c);
        else if (c < 0.0) sp = 2.0 * asin(0.5 * sqrt(-c)) * (180.0 / kPi * 3600.0);
        else sp = sep_from_coords(coordA[a], coordB[b]);
        os[q] = sp;
        if (best_idx[a] == b) bsep[a] = sp;
    }
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// What the finishing kernels need.
struct FinishArgs {
    int64_t nA, nB;
    int64_t pcap;          // pairs the outputs hold
    const int64_t *off;
    const RowRec *rec;
    const int32_t *best2;   // bests of the rows flagged kBestSide
    int use_rec;
    int defer;              // every separation from the coordinates, by k_sep_fix (a batch's mixed path)
    PairTmp *tmp;
    const double2 *coordA;  // A coordinates by output row
    const double2 *coordB;  // B coordinates by output idxB
    int32_t *best_idx;
    int32_t *oa, *ob;
    double *os, *bsep;
    uint32_t *err;
    uint32_t *open_flag;  // cleared device word: separations left to k_sep_fix (unused with defer)
    uint32_t *sort_fail;  // cleared device word for the segment sorts (null: table schedule)
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
    // with defer every pair is left to k_sep_fix, which then runs over all
    // of them; otherwise the few left open raise a flag
    uint32_t *flag = f.defer ? nullptr : f.open_flag;
    hipLaunchKernelGGL(k_finalize, dim3(nblk(f.nA, 256)), dim3(256), 0, s, f.nA, f.nB, f.pcap,
                       f.off, f.rec, f.best2, f.use_rec, f.tmp, f.best_idx, f.oa, f.ob, f.os,
                       f.bsep, f.err, flag, f.seg_n, f.list, f.cap);
    hipLaunchKernelGGL(k_seg_lds, dim3(kSegGrid), dim3(256), 0, s, f.off, f.seg_n, f.list, f.cap,
                       f.tmp, f.nB, f.pcap, f.coordA, f.coordB, f.rec, f.best2, f.oa, f.ob, f.os,
                       f.bsep, f.seg_n + 1, f.huge, f.err, f.defer);
    if (f.pcap > 0) {
        const unsigned g = flag ? kSegGrid : nblk(f.pcap, 256);
        hipLaunchKernelGGL(k_sep_fix, dim3(g), dim3(256), 0, s, f.pcap, f.off + f.nA, f.nA, f.nB,
                           f.oa, f.ob, f.os, f.coordA, f.coordB, f.best_idx, f.bsep, flag);
    }
}

// Segments longer than kSegLds (their count already on the host), all at
// once: their entries gathered into one array (key idxB, value the entry's
// place in that array), sorted by idxB, then stably by segment, and each
// written to its place in its segment.
__global__ void k_huge_len(const uint32_t *__restrict__ huge, uint32_t nh,
                           const int64_t *__restrict__ off, uint32_t *__restrict__ len)
{
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= nh) return;
    const uint32_t a = huge[h];
    len[h] = (uint32_t)(off[a + 1] - off[a]);
}

__global__ void k_huge_gather(const uint32_t *__restrict__ huge, uint32_t nh,
                              const int64_t *__restrict__ off, const uint32_t *__restrict__ base,
                              const PairTmp *__restrict__ tmp, uint32_t *__restrict__ key,
                              uint32_t *__restrict__ val, uint32_t *__restrict__ seg)
{
    for (uint32_t h = blockIdx.x; h < nh; h += gridDim.x) {
        const uint32_t a = huge[h];
        const int64_t o = off[a], len = off[a + 1] - o;
        const uint32_t b = base[h];
        for (int64_t k = threadIdx.x; k < len; k += blockDim.x) {
            key[b + k] = tmp[o + k].idxB;
            val[b + k] = b + (uint32_t)k;
            seg[b + k] = h;
        }
    }
}

// val is a permutation of [0, n) unless the sort by idxB gave up (the call
// is then redone and its slots may hold anything): other values get key 0.
__global__ void k_huge_segkey(const uint32_t *__restrict__ val, const uint32_t *__restrict__ seg,
                              uint32_t n, uint32_t *__restrict__ key)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t v = val[t];
    key[t] = v < n ? seg[v] : 0u;
}

// Entry i of the final order: gathered entry e = val[i] of segment h, whose
// row is huge[h]; it goes to rank i - base[h] of that row's segment.
__global__ void k_huge_write(const uint32_t *__restrict__ val, uint32_t n,
                             const uint32_t *__restrict__ seg, const uint32_t *__restrict__ base,
                             const uint32_t *__restrict__ huge, const int64_t *__restrict__ off,
                             const PairTmp *__restrict__ tmp, int64_t nB,
                             const double2 *__restrict__ coordA,
                             const double2 *__restrict__ coordB,
                             const RowRec *__restrict__ rec,
                             const int32_t *__restrict__ best2,
                             int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                             double *__restrict__ os, double *__restrict__ bsep,
                             uint32_t *__restrict__ err)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t e = val[i];
    if (e >= n) {
        atomicOr(err, 16u);
        return;
    }
    const uint32_t h = seg[e];
    const uint32_t a = huge[h];
    const int64_t o = off[a], len = off[a + 1] - o;
    // ranks outside the segment only come from a sort that gave up (the
    // call is then redone): nothing is written
    const int64_t rk = (int64_t)i - (int64_t)base[h], src = (int64_t)e - (int64_t)base[h];
    if (rk < 0 || rk >= len || src < 0 || src >= len) {
        atomicOr(err, 16u);
        return;
    }
    final_write(o + rk, a, tmp[o + src], nB, coordA, coordB, row_best(rec[a], best2, a), oa, ob,
                os, bsep, err, false);
}

static c3x_status finish_huge(const FinishArgs &f, const uint32_t *hseg, hipStream_t s)
{
    if (hseg[0] > f.cap || hseg[1] > f.cap) return fail(C3X_ENOMEM, "too many long segments");
    const uint32_t nh = hseg[1];
    if (nh == 0) return C3X_OK;
    Arena t2(s);
    uint32_t *len = t2.get_n<uint32_t>(nh), *base = t2.get_n<uint32_t>(nh);
    uint32_t *tot = t2.get_n<uint32_t>(1);
    void *sws = t2.get(scan_ws_bytes(nh));
    if (!len || !base || !tot || !sws) return fail(C3X_ENOMEM, "segment order");
    hipLaunchKernelGGL(k_huge_len, dim3(nblk(nh, 256)), dim3(256), 0, s, f.huge, nh, f.off, len);
    hipError_t e = scan_u32(len, base, nh, tot, sws, s);
    uint32_t n = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&n, tot, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "segment order");
    uint32_t *k1 = t2.get_n<uint32_t>(n), *v1 = t2.get_n<uint32_t>(n);
    uint32_t *k2 = t2.get_n<uint32_t>(n), *v2 = t2.get_n<uint32_t>(n);
    uint32_t *seg = t2.get_n<uint32_t>(n);
    void *ws = t2.get(radix_ws_bytes(n));
    if (!k1 || !v1 || !k2 || !v2 || !seg || !ws) return fail(C3X_ENOMEM, "segment order");
    hipLaunchKernelGGL(k_huge_gather, dim3(std::min<uint32_t>(nh, 4096)), dim3(256), 0, s, f.huge,
                       nh, f.off, base, f.tmp, k1, v1, seg);
    // by idxB (stable), then by segment (stable): each segment in idxB order
    int in1 = 0, in2 = 0;
    e = radix_sort_pairs(k1, v1, k2, v2, n, 31, ws, s, &in1, false, f.sort_fail);
    uint32_t *ka = in1 ? k2 : k1, *va = in1 ? v2 : v1;  // sorted by idxB
    uint32_t *kb = in1 ? k1 : k2, *vb = in1 ? v1 : v2;  // free
    int segbits = 1;
    while (segbits < 32 && (nh - 1) >> segbits) ++segbits;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_huge_segkey, dim3(nblk(n, 256)), dim3(256), 0, s, va, seg, n, kb);
        e = radix_sort_pairs(kb, va, ka, vb, n, segbits, ws, s, &in2, false, f.sort_fail);
    }
    if (e == hipSuccess) {
        const uint32_t *vf = in2 ? vb : va;
        hipLaunchKernelGGL(k_huge_write, dim3(nblk(n, 256)), dim3(256), 0, s, vf, n, seg, base,
                           f.huge, f.off, f.tmp, f.nB, f.coordA, f.coordB, f.rec, f.best2, f.oa,
                           f.ob, f.os, f.bsep, f.err);
        e = hipGetLastError();
    }
    uint32_t gave_up = 0;
    if (e == hipSuccess && f.sort_fail)
        e = hipMemcpyAsync(&gave_up, f.sort_fail, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "segment order");
    return gave_up ? kSortGaveUp : C3X_OK;
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

// Dispatch of a (shape, precision) pair to a launch macro L(SHAPE, PREC).
#define C3X_SHAPES(L)                                                 \
    do {                                                              \
        if (shape == C3X_CIRCLE) {                                    \
            if (prec == C3X_FP64) L(C3X_CIRCLE, C3X_FP64);            \
            else L(C3X_CIRCLE, C3X_MIXED);                            \
        } else if (shape == C3X_ELLIPSE) {                            \
            if (prec == C3X_FP64) L(C3X_ELLIPSE, C3X_FP64);           \
            else L(C3X_ELLIPSE, C3X_MIXED);                           \
        } else {                                                      \
            if (prec == C3X_FP64) L(C3X_RECT, C3X_FP64);              \
            else L(C3X_RECT, C3X_MIXED);                              \
        }                                                             \
    } while (0)

template <int MODE>
static void launch_match(const MatchArgs &m, int shape, int prec, unsigned grid, hipStream_t s)
{
    if (grid == 0) return;
#define C3X_LAUNCH(SH, PR) \
    hipLaunchKernelGGL((k_match<SH, PR, MODE, false>), dim3(grid), dim3(kMatchBlock), 0, s, m)
    C3X_SHAPES(C3X_LAUNCH);
#undef C3X_LAUNCH
}

template <int MODE>
static void launch_wide(const MatchArgs &m, int shape, int prec, hipStream_t s)
{
    if (!m.wide_min || m.nA == 0) return;
    // a fixed grid of wavefronts striding over the list (its length is on
    // the device): 16 per compute unit, what stays resident
    const unsigned grid = (unsigned)std::min<int64_t>((m.nA + 3) / 4, 1024);
#define C3X_LAUNCH(SH, PR) \
    hipLaunchKernelGGL((k_match_wide<SH, PR, MODE>), dim3(grid), dim3(256), 0, s, m)
    C3X_SHAPES(C3X_LAUNCH);
#undef C3X_LAUNCH
}

static void launch_rerank(const MatchArgs &m, int shape, int prec, const uint32_t *pos,
                          uint32_t n, uint32_t *unc_n, uint32_t *unc, hipStream_t s)
{
    if (n == 0) return;
#define C3X_RR(SH, PR) \
    hipLaunchKernelGGL((k_rerank<SH, PR, false>), dim3(n), dim3(64), 0, s, m, pos, n, nullptr, \
                       unc_n, unc)
    C3X_SHAPES(C3X_RR);
#undef C3X_RR
}

static void launch_collect(const MatchArgs &m, int shape, int prec, hipStream_t s)
{
    unsigned grid = m.n_col;
    if (grid == 0) return;
#define C3X_COL(SH, PR) \
    hipLaunchKernelGGL((k_collect<SH, PR, false>), dim3(grid), dim3(64), 0, s, m)
    C3X_SHAPES(C3X_COL);
#undef C3X_COL
}

}  // namespace c3x

using namespace c3x;

#define HIPCHK(expr, what)                       \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

// Sums of the statistics copies: out[0] tests, out[1] band, out[2] placed.
static void stat_sums(const unsigned long long *h, unsigned long long out[3])
{
    out[0] = out[1] = out[2] = 0;
    for (int q = 0; q < kStatSlots; ++q)
        for (int f = 0; f < 3; ++f) out[f] += h[q * kStatStride + f];
}

// Overflow-list demand of recent calls, in entries per 1024 A rows: sizes the
// next call's regions so that steady workloads keep the single pass.
static std::atomic<uint64_t> g_ov_hint{0};
constexpr uint64_t kOvFloorBytes = 1ull << 30;  // overflow regions: floor of 256 entries a row up to this
constexpr uint64_t kOvMaxBytes = 4ull << 30;    // and never more than this

// onesweep: large sorts may take the one-sweep schedule; kSortGaveUp when
// one of them gave up its look-back (the caller then redoes the call
// without it).
// s_keys (may be s): the stream that keys and sorts catalogue A. ib: an index
// still being built on s (c3x_cross_match): it is checked, and handed to
// *ix_built, once A is sorted.
static c3x_status match_impl(const c3x_index *ix, const double *ra, const double *dec, int64_t nA,
                             const c3x_area *area, unsigned mode, hipStream_t s, bool onesweep,
                             c3x_result *R, hipStream_t s_keys = nullptr, IndexBuild *ib = nullptr,
                             c3x_index **ix_built = nullptr)
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
    // bad, amb_n, tie_n, col_n, err, emit overflow, segments (2), wide rows
    // one block of counters, read back with one copy: 16 u32, the statistics
    // copies (tests, band, placed), then the overflow regions' counters
    constexpr int kPoolWords = kEmitPools * kEmitPoolStride;
    constexpr size_t kStatBytes = kStatSlots * kStatStride * sizeof(unsigned long long);
    constexpr size_t kOctrAt = 128 + kStatBytes;
    constexpr size_t kCtrBytes = kOctrAt + kPoolWords * sizeof(uint32_t);
    uint8_t *cblk = (uint8_t *)tmp.get(kCtrBytes);
    uint32_t *ctr = (uint32_t *)cblk;
    unsigned long long *c64 = (unsigned long long *)(cblk + 128);
    double2 *arad = tmp.get_n<double2>(nA);
    double2 *packed = tmp.get_n<double2>(nA);
    ARange *arng = tmp.get_n<ARange>(nA);
    int32_t *best2 = tmp.get_n<int32_t>(nA);
    RowRec *rec = tmp.get_n<RowRec>(nA);
    AEll *aell = nullptr;
    AEllR *aellr = nullptr;
    if (shape != C3X_CIRCLE) {
        aell = tmp.get_n<AEll>(nA);
        aellr = tmp.get_n<AEllR>(nA);
        if (!aell || !aellr) return fail(C3X_ENOMEM, "A buffers");
    }
    if (!keys || !rows || !ktmp || !rtmp || !ws || !ctr || !c64 || !arad || !packed ||
        !best2 || !rec || !arng)
        return fail(C3X_ENOMEM, "A buffers");
    R->nA = nA;
    R->best_idx = R->mem.get_n<int32_t>(nA);
    R->best_sep = R->mem.get_n<double>(nA);
    if (!R->best_idx || !R->best_sep) return fail(C3X_ENOMEM, "best buffers");
    // catalogue A keyed and sorted on its own stream when the index is still
    // being built on s (from the moment its grid is on the device; the two
    // only meet at the gather)
    StreamFork fork(s, s_keys ? s_keys : s, ib ? ib->grid_ready : nullptr);
    HIPCHK(fork.e, "stream fork");
    const hipStream_t s_a = fork.a;
    HIPCHK(hipMemsetAsync(cblk, 0, kCtrBytes, s_a), "memset");
    HIPCHK(hipMemsetAsync(ctr, 0xff, sizeof(uint32_t), s_a), "memset");
    const double *sa = area->semi_major_arcsec, *sb = area->semi_minor_arcsec, *pa = area->pa_deg;
    if (nA > 0)
        hipLaunchKernelGGL(k_prep_a, dim3(nblk(nA, 256)), dim3(256), 0, s_a, ra, dec, nA, ix->grid,
                           shape, sa, sb, pa, keys, packed, ctr);
    HIPCHK(hipGetLastError(), "A keys");
    int in_tmp = 0;
    // A is ordered by its top 24 key bits only (three passes): runs of up to
    // 2^(bits - 24) cells along a zone keep a wavefront's sources together,
    // and no result depends on the order of A
    const int a_lo = std::max(0, ix->plan.key_bits - a_key_bits());
    // ctr[11]: set when a one-sweep sort gave up (read back after the count)
    HIPCHK(radix_sort_pairs_bits(keys, rows, ktmp, rtmp, nA, a_lo, ix->plan.key_bits, ws, s_a,
                                 &in_tmp, /*vals_are_index=*/true, onesweep ? ctr + 11 : nullptr),
           "A sort");
    HIPCHK(fork.join(), "stream join");
    if (ib) {  // the index: its rows and its sort checked before anything reads it
        const c3x_status st = index_build_end(*ib, ix_built);
        if (st != C3X_OK) return st;
    }
    // the sorted rows are the sorted sources' idxA (the gather clamps them)
    uint32_t *srows = in_tmp ? rtmp : rows;
    const uint32_t *aidx = srows;
    // rows with at least wide_min candidates (or a window walked cell by
    // cell) are counted by one wavefront each; C3X_WIDE_MIN=0 turns it off
    uint32_t wide_min = kWideMin;
    if (const char *ev = getenv("C3X_WIDE_MIN")) wide_min = (uint32_t)std::max(0, atoi(ev));
    const bool few = nA < kFewRows;
    uint32_t *wide = wide_min ? ktmp : nullptr;  // the key buffer is free after the sort
    if (in_tmp) wide = wide_min ? keys : nullptr;
    if (nA > 0) {
        const double reach = shape == C3X_CIRCLE ? area->radius_arcsec / 3600.0 : 0.0;
#define C3X_GATHER(SH)                                                                            \
    hipLaunchKernelGGL(k_gather_a<SH>, dim3(nblk(nA, 256)), dim3(256), 0, s, srows, packed, nA, sa, \
                       sb, pa, area->pa_zero_deg, area->pa_sense, ix->plan.L_rad, ix->grid, reach,  \
                       arad, aell, aellr, arng, wide_min, few, wide, ctr + 8)
        if (shape == C3X_CIRCLE) C3X_GATHER(C3X_CIRCLE);
        else if (shape == C3X_ELLIPSE) C3X_GATHER(C3X_ELLIPSE);
        else C3X_GATHER(C3X_RECT);
#undef C3X_GATHER
    }
    // forced paths (tests; the answer must not change): C3X_DEBUG_FORCE_BAND
    // lists every candidate within twice the area for the FP64 recheck;
    // C3X_DEBUG_FORCE_AMBIG sends every band candidate, and the best match of
    // every row with two or more matches, to binary128 on the host
    const bool force_band = env_on("C3X_DEBUG_FORCE_BAND");
    const bool force_ambig = env_on("C3X_DEBUG_FORCE_AMBIG");
    if (force_band && shape != C3X_CIRCLE && nA > 0)
        hipLaunchKernelGGL(k_force_band_margins, dim3(nblk(nA, 256)), dim3(256), 0, s, aellr, nA);
    HIPCHK(hipGetLastError(), "A records");
    tm.mark();  // 1

    // ---- thresholds and common arguments
    MatchArgs m;
    memset(&m, 0, sizeof(m));
    m.g = ix->grid;
    m.pay64 = ix->pay64;
    m.pay32 = ix->pay32;
    m.res = ix->res;
    m.coordB = ix->radec;
    m.arad = arad;
    m.aidx = aidx;
    m.aell = aell;
    m.aellr = aellr;
    m.arng = arng;
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
        if (force_band && !m.r_zero) {  // nothing inside, nothing within 2 r outside
            m.t64_in = -1.0;
            m.t32_in = -1.0f;
            m.t64_out = std::max(m.t64_out, 4.0 * m.cr2);
            m.t32_out = std::max(m.t32_out, (float)(4.0 * m.cr2));
        }
    }
    if (force_ambig) {
        m.force_host = 1;
        m.tie_widen = 1e300;
    }
    m.n_tests = c64;
    m.n_band = c64 + 1;
    m.err_flag = ctr + 4;
    m.best2 = best2;
    m.rec_zeroed = 1;
    m.best_only = !all;
    m.rec = rec;
    m.wide = wide;
    m.wide_n = ctr + 8;
    m.wide_min = wide_min;
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
    // kTab matches into its record, later ones into the overflow list
    // (kEmitPools regions; block b uses region b mod kEmitPools). If a
    // region runs out, the count stands and the write pass puts every
    // match into the offsets instead.
    m.n_placed = c64 + 2;
    m.ov_flag = ctr + 5;
    bool emit = false;
    if (all && nA > 0) {
        // regions sized from the need seen by recent calls (entries per 1024
        // A rows); at least 256 entries per row while that stays within
        // kOvFloorBytes, at least nA / 8 in all, and at most kOvMaxBytes (an
        // unused entry costs nothing but memory; a full region costs a
        // second, write-only pass)
        const uint64_t hint = g_ov_hint.load(std::memory_order_relaxed);
        const uint64_t floor_n = std::min<uint64_t>((uint64_t)nA * 256,
                                                    kOvFloorBytes / sizeof(OvEnt));
        uint64_t per = (uint64_t)std::max<int64_t>(nA / 8 / kEmitPools, 4096);
        per = std::max<uint64_t>(per, (floor_n + kEmitPools - 1) / kEmitPools);
        per = std::max<uint64_t>(per, ((uint64_t)nA * hint / 1024 + kEmitPools - 1) / kEmitPools);
        per = std::min<uint64_t>(per, kOvMaxBytes / sizeof(OvEnt) / kEmitPools);
        // test hook: C3X_DEBUG_OVERFLOW_SLOTS=k gives each region k slots (0: none,
        // every match goes through the write pass)
        if (const char *ev = getenv("C3X_DEBUG_OVERFLOW_SLOTS"))
            per = (uint64_t)std::max<long long>(atoll(ev), -1);
        if (per > 0 && per < (1ull << 26)) {
            m.ovl = tmp.get_n<OvEnt>(per * kEmitPools);
            m.octr = (uint32_t *)(cblk + kOctrAt);
            m.ov_pool = (uint32_t)per;
            emit = m.ovl && m.octr;
        }
    }
    // band candidates decided by the FP64 recheck right after the count:
    // inside ones (bin) join the matches, open ones (hl) go to the host
    uint4 *bin = tmp.get_n<uint4>(amb_cap);
    AmbInfo *hl = tmp.get_n<AmbInfo>(amb_cap);
    if (!bin || !hl) return fail(C3X_ENOMEM, "band buffers");
    auto recheck = [&]() {
        if (shape == C3X_CIRCLE)
            hipLaunchKernelGGL(k_recheck<C3X_CIRCLE>, dim3(nblk(amb_cap, 256)), dim3(256), 0, s,
                               m.amb, ctr + 1, amb_cap, arad, aidx, aellr, ix->radec, ix->pay64,
                               ix->pay32, m.h_r, nullptr, nullptr, nullptr, bin, ctr + 9, hl,
                               ctr + 10, m.force_host);
        else if (shape == C3X_ELLIPSE)
            hipLaunchKernelGGL(k_recheck<C3X_ELLIPSE>, dim3(nblk(amb_cap, 256)), dim3(256), 0, s,
                               m.amb, ctr + 1, amb_cap, arad, aidx, aellr, ix->radec, ix->pay64,
                               ix->pay32, m.h_r, sa, sb, pa, bin, ctr + 9, hl, ctr + 10,
                               m.force_host);
        else
            hipLaunchKernelGGL(k_recheck<C3X_RECT>, dim3(nblk(amb_cap, 256)), dim3(256), 0, s,
                               m.amb, ctr + 1, amb_cap, arad, aidx, aellr, ix->radec, ix->pay64,
                               ix->pay32, m.h_r, sa, sb, pa, bin, ctr + 9, hl, ctr + 10,
                               m.force_host);
    };
    std::vector<uint8_t> hvec;
    uint8_t *hb = pinned_stage(kCtrBytes + 64);
    if (!hb) {
        hvec.resize(kCtrBytes + 64);
        hb = hvec.data();
    }
    uint32_t hctr[16];
    unsigned long long h64[3];
    std::vector<uint32_t> hoctr(kPoolWords);
    if (nA > 0) HIPCHK(hipMemsetAsync(rec, 0, (size_t)nA * sizeof(RowRec), s), "memset");
    Timer tk(s);  // the count kernel alone (the last attempt's launch)
    for (int attempt = 0; attempt < 2; ++attempt) {
        tk.n = 0;
        tk.mark();
        if (emit) launch_match<2>(m, shape, prec, grid, s);
        else launch_match<0>(m, shape, prec, grid, s);
        tk.mark();
        if (emit) launch_wide<2>(m, shape, prec, s);
        else launch_wide<0>(m, shape, prec, s);
        HIPCHK(hipGetLastError(), "count pass");
        if (nA > 0) recheck();
        HIPCHK(hipGetLastError(), "band recheck");
        HIPCHK(hipMemcpyAsync(hb, cblk, emit ? kCtrBytes : kOctrAt,
                              hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(hipStreamSynchronize(s), "count pass");
        memcpy(hctr, hb, sizeof(hctr));
        stat_sums((const unsigned long long *)(hb + 128), h64);
        if (emit) memcpy(hoctr.data(), hb + kOctrAt, kPoolWords * sizeof(uint32_t));
        if (hctr[11]) return kSortGaveUp;
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
            bin = tmp.get_n<uint4>(amb_cap);
            hl = tmp.get_n<AmbInfo>(amb_cap);
        }
        if (hctr[2] > tie_cap) {
            tie_cap = hctr[2];
            tie = tmp.get_n<uint2>(tie_cap);
        }
        if (!amb || !tie || !bin || !hl) return fail(C3X_ENOMEM, "count lists");
        m.amb = amb;
        m.amb_cap = amb_cap;
        m.tie = tie;
        m.tie_cap = tie_cap;
        HIPCHK(hipMemsetAsync(ctr + 1, 0, 2 * sizeof(uint32_t), s), "memset");
        HIPCHK(hipMemsetAsync(ctr + 5, 0, sizeof(uint32_t), s), "memset");
        HIPCHK(hipMemsetAsync(ctr + 9, 0, 2 * sizeof(uint32_t), s), "memset");
        HIPCHK(hipMemsetAsync(c64, 0, kStatBytes, s), "memset");
        if (emit) HIPCHK(hipMemsetAsync(m.octr, 0, kPoolWords * sizeof(uint32_t), s), "memset");
    }
    // the records and the list hold every filter match unless a region ran out
    const bool emitted = emit && hctr[5] == 0;
    if (emit && nA > 0 && !getenv("C3X_DEBUG_OVERFLOW_SLOTS")) {
        // the busiest region's demand (counted even past its end), with a margin
        uint64_t need = 0;
        for (int q = 0; q < kEmitPools; ++q) need = std::max<uint64_t>(need, hoctr[q * kEmitPoolStride]);
        const uint64_t obs = need * kEmitPools * 1024 * 5 / 4 / (uint64_t)nA;
        const uint64_t old = g_ov_hint.load(std::memory_order_relaxed);
        g_ov_hint.store(std::min<uint64_t>(std::max(obs, old / 2), 1024 * 1024),
                        std::memory_order_relaxed);
    }
    uint32_t ov_used = 0;
    if (emitted)
        for (int q = 0; q < kEmitPools; ++q)
            ov_used = std::max(ov_used, std::min(hoctr[q * kEmitPoolStride], m.ov_pool));
    // (tests and band are read; the write pass counts the placed matches anew)
    if (!emitted) HIPCHK(hipMemsetAsync(c64, 0, kStatBytes, s), "memset");
    const uint32_t n_tie = hctr[2];
    uint32_t n_bin = std::min(hctr[9], amb_cap);
    const uint32_t n_host = std::min(hctr[10], amb_cap);
    R->stats.n_tests = (int64_t)h64[0];
    R->stats.n_band = (int64_t)h64[1];
    tm.mark();  // 2

    // ---- band candidates the FP64 recheck left open: binary128 on the host;
    // its verdicts go to a sorted table the re-ranking passes look up. The
    // host vectors live to the end of the call (the copies are asynchronous).
    std::vector<AmbInfo> info;
    std::vector<unsigned long long> vk;
    std::vector<uint8_t> vi;
    std::vector<uint4> hadd;
    if (n_host > 0) {
        info.resize(n_host);
        HIPCHK(hipMemcpyAsync(info.data(), hl, n_host * sizeof(AmbInfo), hipMemcpyDeviceToHost, s),
               "copy");
        HIPCHK(hipStreamSynchronize(s), "band recheck");
        std::vector<std::pair<unsigned long long, uint8_t>> ver(n_host);
        for (uint32_t k = 0; k < n_host; ++k) {
            const AmbInfo &q = info[k];
            const int in =
                shape == C3X_CIRCLE
                    ? c3x_q_circle(q.raA, q.decA, q.raB, q.decB, area->radius_arcsec)
                : shape == C3X_ELLIPSE
                    ? c3x_q_ellipse(q.raA, q.decA, q.raB, q.decB, q.a, q.b, q.pa,
                                    area->pa_zero_deg, area->pa_sense)
                    : c3x_q_rect(q.raA, q.decA, q.raB, q.decB, q.a, q.b, q.pa, area->pa_zero_deg,
                                 area->pa_sense);
            ver[k] = {((unsigned long long)q.i << 32) | q.j, (uint8_t)(in ? 1 : 0)};
            if (in) hadd.push_back(make_uint4(q.i, q.idxA, q.idxB, q.j));
        }
        std::sort(ver.begin(), ver.end());
        vk.resize(n_host);
        vi.resize(n_host);
        for (uint32_t k = 0; k < n_host; ++k) {
            vk[k] = ver[k].first;
            vi[k] = ver[k].second;
        }
        unsigned long long *dvk = tmp.get_n<unsigned long long>(n_host);
        uint8_t *dvi = tmp.get_n<uint8_t>(n_host);
        if (!dvk || !dvi) return fail(C3X_ENOMEM, "verdict table");
        HIPCHK(hipMemcpyAsync(dvk, vk.data(), n_host * 8, hipMemcpyHostToDevice, s), "copy");
        HIPCHK(hipMemcpyAsync(dvi, vi.data(), n_host, hipMemcpyHostToDevice, s), "copy");
        if (!hadd.empty()) {  // the band list has room: each entry joins at most once
            HIPCHK(hipMemcpyAsync(bin + n_bin, hadd.data(), hadd.size() * sizeof(uint4),
                                  hipMemcpyHostToDevice, s), "copy");
            n_bin += (uint32_t)hadd.size();
        }
        m.ver_key = dvk;
        m.ver_in = dvi;
        m.n_ver = n_host;
    }
    R->stats.n_ambiguous = n_host;
    // band matches: counted, and listed as the k-th match of their row
    WEnt *xent = nullptr;
    const uint32_t n_x = all ? n_bin : 0;
    if (n_bin > 0) {
        if (all) {
            xent = tmp.get_n<WEnt>(n_bin);
            if (!xent) return fail(C3X_ENOMEM, "band matches");
        }
        hipLaunchKernelGGL(k_add_pairs, dim3(nblk(n_bin, 256)), dim3(256), 0, s, bin, n_bin, rec,
                           xent);
    }

    // ---- best matches the filter cannot rank (near-ties, rows with a band
    // match): re-ranked in FP64 on the GPU; rows FP64 cannot separate are
    // listed (ctr[3]) for binary128 on the host
    const uint32_t nr = n_tie + n_bin;
    R->stats.n_best_ties = nr;
    uint32_t *dpos = nullptr;
    if (nr > 0) {
        uint32_t *dall = tmp.get_n<uint32_t>(nr);
        dpos = tmp.get_n<uint32_t>(nr);
        if (!dall || !dpos) return fail(C3X_ENOMEM, "re-ranking buffers");
        hipLaunchKernelGGL(k_rerank_rows, dim3(nblk(nr, 256)), dim3(256), 0, s, tie, n_tie, bin,
                           n_bin, dall);
        HIPCHK(hipMemsetAsync(ctr + 3, 0, sizeof(uint32_t), s), "memset");
        launch_rerank(m, shape, prec, dall, nr, ctr + 3, dpos, s);
        HIPCHK(hipGetLastError(), "re-ranking");
    }

    // ---- rows FP64 could not rank (nc of them, listed in dpos): every match
    // listed, ranked in binary128 on the host, and their best patched -- in
    // the records before the outputs exist, or in the outputs afterwards
    int64_t *off = nullptr;
    auto resolve_unranked = [&](uint32_t nc, bool after_outputs) -> c3x_status {

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
        }
        if (!prow.empty()) {
            uint32_t np = (uint32_t)prow.size();
            uint32_t *d1 = tmp.get_n<uint32_t>(np);
            int32_t *d2 = tmp.get_n<int32_t>(np);
            if (!d1 || !d2) return fail(C3X_ENOMEM, "best patch");
            HIPCHK(hipMemcpyAsync(d1, prow.data(), np * 4, hipMemcpyHostToDevice, s), "copy");
            HIPCHK(hipMemcpyAsync(d2, pbi.data(), np * 4, hipMemcpyHostToDevice, s), "copy");
            if (after_outputs)
                hipLaunchKernelGGL(k_patch_out, dim3(nblk(np, 256)), dim3(256), 0, s, d1, d2, np,
                                   off, R->idxB, R->sep, R->best_idx, R->best_sep, ctr + 4);
            else
                hipLaunchKernelGGL(k_patch_best, dim3(nblk(np, 256)), dim3(256), 0, s, d1, d2, np,
                                   rec, best2);
            HIPCHK(hipStreamSynchronize(s), "best patch");
        }
        return C3X_OK;
    };

    // ---- scan of the per-A counts (idxA order). In all-matches mode with
    // every filter match emitted, the total is known from the count pass
    // (first matches in the records, the overflow list, the band matches)
    // and the outputs go ahead without waiting for the scan.
    off = tmp.get_n<int64_t>(nA + 1);
    // the counts are the records' first words (the flag bit masked off)
    const uint32_t *scan_in = &rec->n;
    int64_t scan_stride = kRecWords;
    if (!all) {  // one output row per A row with a match
        uint32_t *nz = tmp.get_n<uint32_t>(nA);
        if (!nz) return fail(C3X_ENOMEM, "offsets");
        if (nA > 0)
            hipLaunchKernelGGL(k_nonzero, dim3(nblk(nA, 256)), dim3(256), 0, s, rec, nA, nz);
        scan_in = nz;
        scan_stride = 1;
    }
    if (!off) return fail(C3X_ENOMEM, "offsets");
    HIPCHK(scan_u32_to_i64(scan_in, scan_stride, kCountMask, off, nA, off + nA, ws, s), "scan");
    const bool early = all && emitted;
    int64_t P = 0;
    int64_t *hP = (int64_t *)(hb + kCtrBytes);
    if (early) {
        uint64_t ov_total = 0;
        for (int q = 0; q < kEmitPools; ++q) ov_total += hoctr[q * kEmitPoolStride];
        P = (int64_t)(h64[2] + ov_total + n_bin);
    } else {
        uint32_t *hnc = (uint32_t *)(hb + kCtrBytes + 8);
        *hnc = 0;
        HIPCHK(hipMemcpyAsync(hP, off + nA, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
        if (nr > 0)
            HIPCHK(hipMemcpyAsync(hnc, ctr + 3, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy");
        HIPCHK(hipStreamSynchronize(s), "scan");
        P = *hP;
        const uint32_t nc = std::min(*hnc, nr);
        if (nc > 0) {
            c3x_status st = resolve_unranked(nc, false);
            if (st != C3X_OK) return st;
        }
    }

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
            hipLaunchKernelGGL(k_place_x, dim3(nblk(n_x, 256)), dim3(256), 0, s, xent, n_x, nullptr,
                               aidx,
                               arad, ix->radec, nA, ix->nB, off, P, rec, emitted ? 1 : 0, pt, c64 + 2,
                               ctr + 4);
        HIPCHK(hipGetLastError(), "band matches");
        tm.mark();  // 4
        // ---- canonical order inside each segment, final records
        fa.nA = nA;
        fa.nB = ix->nB;
        fa.pcap = P;
        fa.off = off;
        fa.rec = rec;
        fa.best2 = best2;
        fa.use_rec = emitted ? 1 : 0;
        fa.defer = 0;  // every match's separation is coded from its FP64 chord
        fa.tmp = pt;
        fa.coordA = packed;  // A coordinates in input order (the key pass's copy)
        fa.coordB = ix->radec;
        fa.best_idx = R->best_idx;
        fa.oa = R->idxA;
        fa.ob = R->idxB;
        fa.os = R->sep;
        fa.bsep = R->best_sep;
        fa.err = ctr + 4;
        fa.open_flag = ctr + 14;
        fa.sort_fail = onesweep ? ctr + 11 : nullptr;
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
        hipLaunchKernelGGL(k_best_sep, dim3(nblk(nA, 256)), dim3(256), 0, s, nA, ix->nB, rec,
                           best2, ra, dec, ix->radec, R->best_idx, R->best_sep, off, P, R->idxA,
                           R->idxB, R->sep, ctr + 4);
    HIPCHK(hipGetLastError(), "best separations");
    tm.mark();  // 6
    HIPCHK(hipMemcpyAsync(hb, cblk, kOctrAt, hipMemcpyDeviceToHost, s), "copy");
    if (early) HIPCHK(hipMemcpyAsync(hP, off + nA, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    HIPCHK(hipStreamSynchronize(s), "c3x_match");
    memcpy(hctr, hb, sizeof(hctr));
    stat_sums((const unsigned long long *)(hb + 128), h64);
    if (early && *hP != P)
        return fail(C3X_EDEVICE, "internal: %lld matches counted, %lld expected", (long long)*hP,
                    (long long)P);
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
    if (early) {  // rows FP64 could not rank, now that the outputs exist
        const uint32_t nc = std::min(hctr[3], nr);
        if (nc > 0) {
            c3x_status st = resolve_unranked(nc, true);
            if (st != C3X_OK) return st;
            HIPCHK(hipMemcpyAsync(hctr + 4, ctr + 4, sizeof(uint32_t), hipMemcpyDeviceToHost, s),
                   "copy");
            HIPCHK(hipStreamSynchronize(s), "c3x_match");
            if (hctr[4]) return fail(C3X_EDEVICE, "internal: best patch (flags %u)", hctr[4]);
        }
    }
    c3x_stats &S = R->stats;
    S.n_a = nA;
    S.n_b = ix->nB;
    S.n_pairs = P;
    S.n_cells = (int64_t)ix->plan.ncells;
    S.cell_arcsec = ix->plan.cell_arcsec;
    S.ms_a_prep = tm.ms(0, 1);
    S.ms_count = tm.ms(1, 2);
    S.ms_count_kernel = tk.ms(0, 1);
    S.ms_scan = tm.ms(2, 3);
    S.ms_write = tm.ms(3, 4);
    S.ms_sort_pairs = tm.ms(4, 6);
    S.ms_total = tm.ms(0, 6);
    S.precision = prec;
    S.tile = kMatchBlock;
    return C3X_OK;
}

// Checks of catalogue A, its area and the mode, shared by c3x_match and
// c3x_cross_match.
static c3x_status check_match_args(const double *ra_deg, const double *dec_deg, int64_t nA,
                                   c3x_frame frame, const c3x_area *area, unsigned mode)
{
    if (!area) return fail(C3X_EINVAL, "NULL area");
    if (nA < 0) return fail(C3X_EINVAL, "nA < 0");
    if (nA > 2147483647LL) return fail(C3X_ERANGE, "nA above 2^31 - 1");
    if (nA > 0 && (!ra_deg || !dec_deg)) return fail(C3X_EINVAL, "NULL coordinate array");
    if (frame != C3X_EQUATORIAL && frame != C3X_GALACTIC) return fail(C3X_EINVAL, "bad frame");

    if (mode == 0 || (mode & ~(unsigned)(C3X_ALL | C3X_BEST)))
        return fail(C3X_EINVAL, "mode must be C3X_ALL, C3X_BEST or both");
    if (area->shape == C3X_CIRCLE) {
        double r = area->radius_arcsec;
        if (!(r == 0.0 || (r >= 1e-6 && r <= 324000.0)))
            return fail(C3X_EINVAL, "radius must be 0 or in [1e-6, 324000] arcsec");
    } else if (area->shape == C3X_ELLIPSE || area->shape == C3X_RECT) {
        if (nA > 0 && (!area->semi_major_arcsec || !area->semi_minor_arcsec || !area->pa_deg))
            return fail(C3X_EINVAL, "ellipse or rectangle parameter arrays are NULL");
        if (!isfinite(area->pa_zero_deg)) return fail(C3X_EINVAL, "pa_zero_deg not finite");
        if (area->pa_sense != 1 && area->pa_sense != -1)
            return fail(C3X_EINVAL, "pa_sense must be +1 or -1");
    } else {
        return fail(C3X_EINVAL, "bad shape");
    }
    return C3X_OK;
}

static c3x_result *new_result(unsigned mode, int64_t nB)
{
    c3x_result *R = new (std::nothrow) c3x_result();
    if (!R) return nullptr;
    (void)hipGetDevice(&R->device);
    memset(&R->stats, 0, sizeof(R->stats));
    R->mode = mode;
    R->nB = nB;
    return R;
}

extern "C" c3x_status c3x_match(const c3x_index *ix, const double *ra_deg, const double *dec_deg,
                                int64_t nA, c3x_frame frame, const c3x_area *area, unsigned mode,
                                const c3x_opts *opts, c3x_result **out)
{
    clear_error();
    if (!out) return fail(C3X_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ix || !area) return fail(C3X_EINVAL, "NULL index or area");
    {
        const c3x_status cs = check_match_args(ra_deg, dec_deg, nA, frame, area, mode);
        if (cs != C3X_OK) return cs;
    }
    if (opts && opts->precision != ix->precision)
        return fail(C3X_EINVAL, "precision differs from the index's");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    c3x_result *R = new_result(mode, ix->nB);
    if (!R) return fail(C3X_ENOMEM, "host allocation");
    // catalogue A in the other frame: converted into the index's frame by the
    // fixed FP64 rule (orientations turned with it); the converted doubles
    // are A's inputs
    Arena conv(s);
    c3x_area ar = *area;
    {
        const c3x_status cs = convert_catalogue_a((int)frame, (int)ix->frame, nA, &ra_deg,
                                                  &dec_deg, &ar, conv, s);
        if (cs != C3X_OK) {
            delete R;
            return cs;
        }
        area = &ar;
    }
    c3x_status st = match_impl(ix, ra_deg, dec_deg, nA, area, mode, s, true, R);
    if (st == kSortGaveUp) {
        // a one-sweep sort gave up its look-back: the call again, with the
        // table schedule (which never waits), into a fresh result
        (void)hipStreamSynchronize(s);
        delete R;
        R = new_result(mode, ix->nB);
        if (!R) return fail(C3X_ENOMEM, "host allocation");
        st = match_impl(ix, ra_deg, dec_deg, nA, area, mode, s, false, R);
        R->stats.n_sort_retries = 1;
    }
    if (st != C3X_OK) {
        (void)hipStreamSynchronize(s);
        delete R;
        return st;
    }
    *out = R;
    return C3X_OK;
}

// The stream that keys and sorts catalogue A in c3x_cross_match: one per
// device, created on first use (default priority, not synchronising with
// the null stream) and kept to the end of the process. Calls that overlap on
// one device share it: their work on it runs one call after the other,
// still ordered by each call's own events. Null when it cannot be created
// (the call then runs both halves on its own stream).
static hipStream_t keys_stream()
{
    constexpr int kDevices = 64;
    static std::mutex mu;
    static hipStream_t streams[kDevices];
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> g(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        streams[dev] = nullptr;
    }
    return streams[dev];
}

extern "C" c3x_status c3x_cross_match(const double *raB, const double *decB, int64_t nB,
                                      c3x_frame frameB, double reach_hint_arcsec,
                                      const double *raA, const double *decA, int64_t nA,
                                      c3x_frame frameA, const c3x_area *area, unsigned mode,
                                      const c3x_opts *opts, c3x_index **index_out,
                                      c3x_result **out)
{
    clear_error();
    if (!out) return fail(C3X_EINVAL, "out is NULL");
    *out = nullptr;
    if (index_out) *index_out = nullptr;
    {
        const c3x_status cs = check_match_args(raA, decA, nA, frameA, area, mode);
        if (cs != C3X_OK) return cs;
    }
    if (frameB != C3X_EQUATORIAL && frameB != C3X_GALACTIC) return fail(C3X_EINVAL, "bad frame");
    hipStream_t s = opts ? (hipStream_t)opts->stream : nullptr;
    // catalogue A in B's frame, as the match converts it
    Arena conv(s);
    c3x_area ar = *area;
    c3x_status st = convert_catalogue_a((int)frameA, (int)frameB, nA, &raA, &decA, &ar, conv, s);
    if (st != C3X_OK) return st;
    c3x_index *ix = nullptr;
    c3x_result *R = nullptr;
    {
        IndexBuild b(s);
        st = index_build_begin(raB, decB, nB, frameB, reach_hint_arcsec, opts, true, b);
        if (st == C3X_OK) {
            R = new_result(mode, nB);
            if (!R) st = fail(C3X_ENOMEM, "host allocation");
        }
        // A is keyed and sorted on the device's second stream while the index
        // is built on s; without one, the two run one after the other
        if (st == C3X_OK) {
            hipStream_t s_keys = keys_stream();
            if (s_keys == s) s_keys = nullptr;
            st = match_impl(b.ix, raA, decA, nA, &ar, mode, s, true, R, s_keys, &b, &ix);
        }
        (void)hipStreamSynchronize(s);
    }  // (an index not handed over is freed here, its kernels done)
    if (st == kSortGaveUp) {
        // a one-sweep sort gave up its look-back: the index build and the
        // match again, one after the other, each redoing what gave up
        delete R;
        R = nullptr;
        delete ix;
        ix = nullptr;
        st = c3x_build_index(raB, decB, nB, frameB, reach_hint_arcsec, opts, &ix);
        if (st == C3X_OK) st = c3x_match(ix, raA, decA, nA, frameB, &ar, mode, opts, &R);
        if (st == C3X_OK) R->stats.n_sort_retries = 1;
    }
    if (st != C3X_OK) {
        delete R;
        delete ix;
        return st;
    }
    R->stats.ms_index = ix->stats.ms_index;
    if (index_out) *index_out = ix;
    else delete ix;
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

extern "C" c3x_status c3x_result_views(const c3x_result *r, const int32_t **idxA,
                                       const int32_t **idxB, const double **sep_arcsec,
                                       const int32_t **best_idxB, const double **best_sep_arcsec)
{
    if (!r) return fail(C3X_EINVAL, "NULL result");
    if (idxA) *idxA = r->idxA;
    if (idxB) *idxB = r->idxB;
    if (sep_arcsec) *sep_arcsec = r->sep;
    if (best_idxB) *best_idxB = r->best_idx;
    if (best_sep_arcsec) *best_sep_arcsec = r->best_sep;
    return C3X_OK;
}

extern "C" void c3x_result_free(c3x_result *r)
{
    if (!r) return;
    // views may still be read by queued work on any stream: its blocks go
    // back to the cache only when the device is idle
    (void)hipDeviceSynchronize();
    delete r;
}

// The batched form: its kernels and entry points use the ones above.
#include "c3x_batch.hip"
