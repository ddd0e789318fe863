// c3x_internal.h -- shared declarations of the MI355X cross-match library.
//
// Data layout in HBM (all device arrays, catalogue B sorted by cell key):
//   keys[nB]   u32   cell key = zbase[zone] + RA cell (zone-major)
//   pay64[nB]  {f64 x, y, z; u32 idx; u32 pad}   FP64 unit vector (32 B),
//                                                 FP64 index only
//   pay32[nB]  {f32 dx, dy, dz; u32 idx}          FP32 offset from the cell's
//                                                 reference vector (16 B), mixed
//                                                 index only
//   radec[nB]  {f64 ra, dec}                      coordinates in input order
//                                                 (sorted position j: row brow(j))
//   dir[Q+1]   u32   dir[q] = #keys with (key >> dshift) < q
// Catalogue A is keyed on the same grid and sorted, so a wavefront of
// threads covers neighbouring sky and reads neighbouring cells of B.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/c3x.h"

namespace c3x {

constexpr double kPi = 3.14159265358979323846;
constexpr double kDeg = kPi / 180.0;     // degrees -> radians
constexpr double kHalfDeg = kPi / 360.0; // half of it (haversines)
constexpr double kU = 1.1102230246251565e-16;   // 2^-53
constexpr double kU32 = 5.9604644775390625e-08; // 2^-24
constexpr double kE40 = 9.094947017729282e-13;  // 2^-40
constexpr double kE38 = 3.637978807091713e-12;  // 2^-38
constexpr int kRefBits = 10;                     // RA reference grid, 2^10 points

enum Decision : int { OUT = 0, IN = 1, AMBIG = 2 };

// One zone of the grid: first key, number of RA cells, cells per degree.
struct alignas(16) ZoneInfo {
    uint32_t base, n;
    double f;              // n / 360
    double g;              // 2^kRefBits / n
    double pad;
};

// Grid of declination zones split into RA cells (the paper's cells,
// restated for the sphere). Passed by value to kernels.
struct Grid {
    double h_deg;          // zone height (degrees)
    double inv_h;          // 1 / h_deg
    int32_t nz;            // number of zones
    uint32_t ncells;       // total cells
    const ZoneInfo *zinfo; // [nz]
    const double2 *zref;   // [nz] cos, sin of the zone's reference Dec
    const uint32_t *keys;  // [nB] sorted keys of B
    const uint32_t *dir;   // [dsize] coarse directory over key >> dshift
    int32_t dshift;
    uint32_t dsize;        // Q + 1
    int32_t nB;
};

struct alignas(32) Pay64 {
    double x, y, z;
    uint32_t idx, pad;
};
struct alignas(16) Pay32 {
    float x, y, z;
    uint32_t idx;          // B row | (low bit of the reference's RA step) << 31
};
__device__ __forceinline__ uint32_t pay_row(const Pay32 &b) { return b.idx & 0x7fffffffu; }
__device__ __forceinline__ uint32_t pay_row(const Pay64 &b) { return b.idx; }

// FP64 residual of an FP32 payload (8 bytes per sorted row, read only for
// filter matches): for each FP64 offset o whose FP32 value is f = fl32(o),
// the remainder o - f (exact in FP64, at most half an FP32 ulp of o) as a
// 21-bit signed multiple of 2^(s - 43), s the binary exponent of f (at
// least -100), the three packed into one 64-bit word. f plus its residual
// restores o to within 2^(s - 44) <= 2^-44 |o|: the FP64 chord of a match
// without an FP64 payload.
__device__ __forceinline__ int res_exp(float f)
{
    const int s = (int)((__float_as_uint(f) >> 23) & 0xffu) - 127;  // zero, subnormal: -127
    return s < -100 ? -100 : s;
}
__device__ __forceinline__ double pow2(int k)  // 2^k, -1022 <= k <= 1023
{
    return __longlong_as_double((long long)(k + 1023) << 52);
}
__device__ __forceinline__ unsigned long long res_part(double o, float f)
{
    const double q = rint((o - (double)f) * pow2(43 - res_exp(f)));
    const int v = (int)fmin(fmax(q, -1048576.0), 1048575.0);
    return (unsigned long long)((uint32_t)v & 0x1fffffu);
}
__device__ __forceinline__ uint2 res_pack(double ox, double oy, double oz, float fx, float fy,
                                          float fz)
{
    const unsigned long long w = res_part(ox, fx) | (res_part(oy, fy) << 21) |
                                 (res_part(oz, fz) << 42);
    return make_uint2((uint32_t)w, (uint32_t)(w >> 32));
}
// Offset k (0: x, 1: y, 2: z) of payload f with residual word w.
__device__ __forceinline__ double res_off(float f, uint2 w, int k)
{
    const unsigned long long u = ((unsigned long long)w.y << 32) | w.x;
    const int v = ((int)((uint32_t)(u >> (21 * k)) << 11)) >> 11;  // sign-extended 21 bits
    return (double)f + (double)v * pow2(res_exp(f) - 43);
}

// One A source as a match lane sees it: position, unit vector (z = sin Dec),
// cos Dec with small relative error near the poles, reach of its area.
// Rebuilt from (ra, dec) inside each kernel, so every pass gets the same bits.
struct ARec {
    double ra, dec, x, y, z, cosd, reach_deg;
    uint32_t idx, pad;
};

// Per-A ellipse parameters (sorted order).
struct alignas(64) AEll {
    double ux, uy, uz;     // major-axis direction in the tangent plane
    double vx, vy, vz;     // minor-axis direction
    double ia, ib;         // 1/a, 1/b in radians^-1
};
struct AEllR {             // what the FP64 recheck needs
    double a_arcsec, b_arcsec, ct, st;
    double m64;            // FP64 filter margin on Q
    float m32;             // FP32 filter margin on Q (0: FP32 filter unusable)
    float pad;
};

// One match as the write pass leaves it: B row, sorted B position and the
// separation in arcsec (NaN: computed later from the coordinates).
struct alignas(16) PairTmp {
    uint32_t idxB, j;
    double sep;
};

// A band candidate found inside, listed as the k-th match of the A source
// at sorted position i.
struct alignas(16) WEnt {
    uint32_t i, k, idxB, j;
};
// A match beyond a row's table slots: the k-th match of A row idxA, with
// its coded separation (see sep_code).
struct alignas(8) OvEnt {
    uint32_t idxA, k, idxB, j;
    double code;
};
constexpr int kTab = 1;              // table slots per A row
// Statistics counters (candidates tested, band candidates, matches placed):
// 64 copies on separate 128-byte lines, block b adding to copy b mod 64, so
// that one address does not take every block's atomic; the host sums them.
constexpr int kStatSlots = 64;
constexpr int kStatStride = 16;      // u64 words per copy
enum { kStatTests = 0, kStatBand = 1, kStatPlaced = 2 };
__device__ __forceinline__ unsigned long long *stat_slot(unsigned long long *field)
{
    return field + (size_t)(blockIdx.x & (kStatSlots - 1)) * kStatStride;
}
constexpr int kEmitPools = 64;       // overflow-list counters (spread contention)
constexpr int kEmitPoolStride = 32;  // u32 words between two counters (128 B)

// Per-A record of the count pass (idxA order): the row's match count (the
// scan's input), its first match and, where that settles it, its best. It
// is one aligned 16-byte store per matched row, and the only one: the
// records are written scattered, in idxA order, and each scattered store
// costs a memory transaction of its own. A row whose best is not the
// record's match (two or more matches when the record keeps the first one,
// or a best re-ranked after the count) has kBestSide set and its best in a
// side table (best2), written for those rows only.
struct alignas(16) RowRec {
    uint32_t n;            // matches (filter, then band ones added) | kBestSide
    uint32_t b0;           // idxB of the row's first match (count-only passes:
                           // of its best)
    double c0;             // the first match's coded separation (see sep_code)
};
static_assert(sizeof(RowRec) == 16, "one 16-byte store per row");
static_assert(kTab == 1, "one match slot in the record");
constexpr uint32_t kBestSide = 1u << 31;       // RowRec.n: the best is in best2
constexpr uint32_t kCountMask = kBestSide - 1u;  // RowRec.n: the count
constexpr int64_t kRecWords = sizeof(RowRec) / sizeof(uint32_t);

// Best match (idxB) of idxA row a from its record: -1 for a row without
// matches.
__device__ __forceinline__ int32_t row_best(const RowRec &r, const int32_t *__restrict__ best2,
                                            int64_t a)
{
    if ((r.n & kCountMask) == 0u) return -1;
    return (r.n & kBestSide) ? best2[a] : (int32_t)r.b0;
}

// Candidate B ranges of one sorted A source, found once when A is prepared:
// zone zlo + q holds the sorted B positions [j0[q], j0[q] + n[q]). zlo < 0:
// not precomputed (an RA window split at 0/360, more than kRZ zones, or a
// range longer than 65535); the match kernels then walk the cells on the fly.
constexpr int kRZ = 3;
struct alignas(8) ARange {
    uint32_t j0[kRZ];
    uint16_t n[kRZ];
    uint16_t wide;         // bit 0: counted by a wavefront of its own; bits 2q+2, 2q+3:
                           // zone q's cells span two FP32 reference steps, and the
                           // other one is below the source's own (see a_ranges)
    int32_t zlo;
};
static_assert(sizeof(ARange) == 24, "24-byte range record");

// A row counted by a wavefront of its own (marked when A is prepared).
__device__ __forceinline__ bool wide_row(const ARange &r)
{
    return (r.wide & 1u) != 0;
}

// One job of a batch (device job table). Its A and B rows are projected on
// the plane tangent to the job's mean direction c (gnomonic: p -> (p.e / p.c,
// p.n / p.c), e and n the east and north axes at c), where the job's data lie
// within tan(10 deg) of the origin, without poles or RA wrap; a grid of
// square cells of side h covers the box [-T, T)^2. Cell (row, col) has key
// key_base + row * ncol + col in one key space shared by all jobs.
struct alignas(16) BJob {
    int64_t a_off, b_off;          // caller rows of the job
    uint32_t a_ent, b_ent;         // first A / B entry of the job
    uint32_t nA, nB;
    uint32_t key_base, ncol, nrow, pad0;
    double cx, cy, cz, ex, ey, ez, nx, ny, nz;
    double T, wd, h, inv_h;        // box half-side, window half-width, cell side
                                   // (tangent-plane units)
    double reach_deg, h_r, cr2, L; // radius, sin^2(r/2), 4 sin^2(r/2), max |p - c|
    double r_arcsec;               // the radius as given
    double t64_in, t64_out;
    float t32_in, t32_out;
    int32_t r_zero, pad1;
};

// Thresholds of the circle filters of one source.
struct Thr {
    double t64_in, t64_out;
    float t32_in, t32_out;
    int32_t r_zero;
};

// Everything a match kernel needs; passed by value.
struct MatchArgs {
    Grid g;
    const Pay64 *pay64;
    const Pay32 *pay32;
    const uint2 *res;      // FP64 residuals of pay32 (mixed)
    const double2 *coordB;
    const double2 *arad;   // sorted A coordinates
    const uint32_t *aidx;  // sorted A rows
    const AEll *aell;
    const AEllR *aellr;
    const ARange *arng;    // [nA] sorted A order
    const BJob *jobs;      // batch: job table, and the job of each sorted A
    const uint32_t *ajob;
    int32_t nA;
    double reach_deg;      // circle reach
    // circle thresholds on the squared chord
    double cr2;            // 4 sin^2(r/2)
    double t64_in, t64_out;
    float t32_in, t32_out;
    double h_r;            // sin^2(r/2) for the haversine recheck
    int32_t r_zero;        // radius exactly 0
    double L_rad;          // bound on |p - cell reference| (FP32 error model)
    // count pass
    RowRec *rec;           // [nA] idxA order
    int32_t *best2;        // [nA] idxA order: bests of rows flagged kBestSide
    int32_t best_only;     // no pairs kept: only the best of each row
    int32_t rec_zeroed;    // records cleared beforehand: rows without a filter
                           // match store no record (every reader of a record
                           // checks the row's count first)
    uint32_t *amb_n;       // band candidates: (sorted A pos, sorted B pos)
    uint2 *amb;
    uint32_t amb_cap;
    uint32_t *tie_n;       // near-tie best matches: (sorted A pos, row)
    uint2 *tie;
    uint32_t tie_cap;
    // forced paths of single calls (zero otherwise): tie_widen is added to
    // the factor 4 of the near-tie tests (a huge value lists every row with
    // two or more matches and lets no FP64 ranking stand); force_host makes
    // every band candidate take the host's binary128 verdict
    double tie_widen;
    int32_t force_host;
    // verdicts of the band candidates: sorted keys (i << 32 | j); in a batch
    // only the host-decided ones, their count in n_ver_dev
    const unsigned long long *ver_key;
    const uint8_t *ver_in;
    uint32_t n_ver;
    const uint32_t *n_ver_dev;
    // write pass
    const int64_t *off;    // [nA + 1] idxA order
    PairTmp *tmp;          // matches in enumeration order
    // count + emit (MODE 2): a row's first kTab matches go to its record,
    // later ones to the overflow list
    OvEnt *ovl;            // kEmitPools regions of ov_pool entries
    uint32_t *octr;        // [kEmitPools * kEmitPoolStride] entries taken per region
    uint32_t ov_pool;      // entries per region
    uint32_t *ov_flag;     // set when a region ran out
    unsigned long long *n_placed;  // matches written (table, list or segments)
    // collect pass: sorted A positions; every match of each is listed
    const uint32_t *col_pos;
    uint32_t n_col;
    uint32_t *col_n;
    void *col;
    uint32_t col_cap;
    // rows counted by the wavefront-per-source kernel (sorted A positions)
    const uint32_t *wide;
    const uint32_t *wide_n;
    uint32_t wide_min;     // 0: none
    // counters
    unsigned long long *n_tests;
    unsigned long long *n_band;
    uint32_t *err_flag;    // 1: write overflow, 2: count mismatch, 4: missing verdict
};

// B row of sorted position j: from the FP64 payload when the index has one,
// else from the FP32 payload (the mixed index keeps no FP64 payload: its
// matches take FP64 chords from the payload's residual, and the rechecks
// FP64 geometry from the coordinates, coordB[row]).
struct BRows {
    const Pay64 *p64;
    const Pay32 *p32;
    __device__ __forceinline__ uint32_t operator()(uint32_t j) const
    {
        return p64 ? p64[j].idx : (p32[j].idx & 0x7fffffffu);
    }
};
__device__ __forceinline__ uint32_t brow(const MatchArgs &m, uint32_t j)
{
    return BRows{m.pay64, m.pay32}(j);
}

// ----------------------------------------------------------------------------
// device geometry
// ----------------------------------------------------------------------------

// Logical block of a 1-D grid such that each XCD takes one contiguous
// share: the dispatcher deals workgroups to the 8 XCDs in turn, so block b
// runs on XCD b % 8, and neighbouring data (one catalogue slice, one L2)
// stays on one XCD.
__device__ __forceinline__ uint32_t xcd_block()
{
    const uint32_t n = gridDim.x, b = blockIdx.x;
    const uint32_t per = n >> 3, rem = n & 7u, x = b & 7u;
    return x * per + min(x, rem) + (b >> 3);
}

__device__ __forceinline__ int zone_of(double dec, const Grid &g)
{
    double t = floor((dec + 90.0) * g.inv_h);
    if (!(t >= 0.0)) return 0;
    if (t >= (double)g.nz) return g.nz - 1;
    return (int)t;
}

__device__ __forceinline__ uint32_t cell_in(const ZoneInfo &zi, double ra)
{
    double t = floor(ra * zi.f);
    if (!(t >= 0.0)) return 0;
    if (t >= (double)zi.n) return zi.n - 1;
    return (uint32_t)t;
}

__device__ __forceinline__ uint32_t cell_of(int z, double ra, const Grid &g)
{
    return cell_in(g.zinfo[z], ra);
}

// Reference vectors of the FP32 filter: in zone z, the zone's reference Dec
// (table) and the centre of the step of a 2^kRefBits-step RA grid that holds
// the cell's centre (one FP64 product, then an FP32 sincospi of the exact
// dyadic angle). Cells of one grid step share their reference. It is only a
// fixed point near the cell shared by every kernel: its accuracy does not
// matter, only that all kernels get the same bits and that |p - ref| stays
// below L.
__device__ __forceinline__ uint32_t ref_step(const ZoneInfo &zi, uint32_t c)
{
    return (uint32_t)(((double)c + 0.5) * zi.g) & ((1u << kRefBits) - 1u);
}

__device__ __forceinline__ void ref_vec(double2 zr, uint32_t step, double &rx, double &ry,
                                        double &rz)
{
    float sa, ca;
    sincospif((float)(2u * step + 1u) * (1.0f / (float)(1u << kRefBits)), &sa, &ca);
    rx = zr.x * (double)ca;
    ry = zr.x * (double)sa;
    rz = zr.y;
}

// Unit vector of (ra, dec) in degrees. The angles go to sincospi in half
// turns (x / 180): its reduction is exact, so there is no large-argument
// path; each component carries a few units of FP64 rounding.
__device__ __forceinline__ void unit_vec(double ra, double dec, double &x, double &y, double &z)
{
    double sa, ca, sd, cd;
    sincospi(ra * (1.0 / 180.0), &sa, &ca);
    sincospi(dec * (1.0 / 180.0), &sd, &cd);
    x = cd * ca;
    y = cd * sa;
    z = sd;
}

// cos(dec) with small relative error also near the poles.
__device__ __forceinline__ double cos_dec_acc(double dec)
{
    double ad = fabs(dec);
    if (ad > 45.0) return sin(kDeg * (90.0 - ad));
    return cos(kDeg * dec);
}

// ra2 - ra1 reduced to (-180, 180] keeping relative accuracy (360 - ra is
// exact for ra > 180).
__device__ __forceinline__ double wrap_dra(double ra1, double ra2)
{
    double d = ra2 - ra1;
    if (d > 180.0) return -((360.0 - ra2) + ra1);
    if (d < -180.0) return (360.0 - ra1) + ra2;
    return d;
}

__device__ __forceinline__ double haversine(double ra1, double dec1, double cd1, double ra2,
                                            double dec2, double cd2)
{
    double s1 = sin(kHalfDeg * (dec2 - dec1));
    double s2 = sin(kHalfDeg * wrap_dra(ra1, ra2));
    return s1 * s1 + (cd1 * cd2) * (s2 * s2);
}

// Tangent-plane components (north, east) of point 2 seen from point 1.
__device__ __forceinline__ void tangent_ne(double ra1, double dec1, double sd1, double ra2,
                                           double dec2, double cd2, double &tn, double &te)
{
    double da = wrap_dra(ra1, ra2);
    double s2 = sin(kHalfDeg * da);
    tn = sin(kDeg * (dec2 - dec1)) + 2.0 * sd1 * cd2 * (s2 * s2);
    te = cd2 * sin(kDeg * da);
}

// Separation in arcsec between two positions given in degrees, accurate to
// a few ulps at every angle.
__device__ __forceinline__ double sep_arcsec_rd(double ra1, double dec1, double ra2, double dec2)
{
    double cd1 = cos_dec_acc(dec1), cd2 = cos_dec_acc(dec2);
    double sd1 = sin(kDeg * dec1);
    double tn, te;
    tangent_ne(ra1, dec1, sd1, ra2, dec2, cd2, tn, te);
    double h = haversine(ra1, dec1, cd1, ra2, dec2, cd2);
    double th = atan2(sqrt(tn * tn + te * te), 1.0 - 2.0 * h);
    return th * (180.0 / kPi * 3600.0);
}

// FP64 relative-accuracy recheck of the circle: the haversine carries at
// most ~90 u of error (a few units per trigonometric call and product), far
// inside its 2^-40 margin.
__device__ __forceinline__ int recheck_circle(const ARec &a, double2 rb, double h_r)
{
    double cd2 = cos_dec_acc(rb.y);
    double h = haversine(a.ra, a.dec, a.cosd, rb.x, rb.y, cd2);
    if (h <= h_r * (1.0 - kE40)) return IN;
    if (h > h_r * (1.0 + kE40)) return OUT;
    return AMBIG;
}

// What the ellipse recheck computes from the pair alone (not from the
// axes): theta / sin theta and the sines of the offset along (su) and
// across (sv) the orientation (cos, sin of the orientation ct, st), for a
// pair at haversine h > 0 (cd2: cos Dec of B).
__device__ __forceinline__ void ell_parts(const ARec &a, double ct, double st, double2 rb,
                                          double cd2, double h, double &f, double &su,
                                          double &sv)
{
    double tn, te;
    tangent_ne(a.ra, a.dec, a.z, rb.x, rb.y, cd2, tn, te);
    double th = 2.0 * asin(sqrt(h));
    double sth = 2.0 * sqrt(h) * sqrt(1.0 - h);
    f = th / sth;
    su = tn * ct + te * st;
    sv = te * ct - tn * st;
}

// The ellipse of semi-axes a, b (arcsec) against those parts:
// Q = (theta / sin theta)^2 ((su / a)^2 + (sv / b)^2), within its margin.
__device__ __forceinline__ int ell_decide(double f, double su, double sv, double a_arcsec,
                                          double b_arcsec)
{
    double x = su / (kDeg * (a_arcsec / 3600.0));
    double y = sv / (kDeg * (b_arcsec / 3600.0));
    double q = (f * f) * (x * x + y * y);
    double m = kE38 * (1.0 + a_arcsec / b_arcsec);
    if (q <= 1.0 - m) return IN;
    if (q > 1.0 + m) return OUT;
    return AMBIG;
}

__device__ __forceinline__ int recheck_ellipse(const ARec &a, const AEllR &e, double2 rb)
{
    double cd2 = cos_dec_acc(rb.y);
    double h = haversine(a.ra, a.dec, a.cosd, rb.x, rb.y, cd2);
    if (h == 0.0) return IN;
    double sa = sin(kHalfDeg * (e.a_arcsec / 3600.0));
    if (h > (sa * sa) * (1.0 + kE40)) return OUT;
    double f, su, sv;
    ell_parts(a, e.ct, e.st, rb, cd2, h, f, su, sv);
    return ell_decide(f, su, sv, e.a_arcsec, e.b_arcsec);
}

// Rectangle of half-sides a (along the orientation) and b (across):
// |u| <= a and |v| <= b, each form (theta / sin theta)^2 (su / a)^2 and
// (theta / sin theta)^2 (sv / b)^2 decided on its own, with the ellipse's
// relative accuracy and margin (near the u side |su| ~ a and sin theta <=
// 1.42 a, near the v side |sv| ~ b and sin theta <= a + b).
__device__ __forceinline__ int recheck_rect(const ARec &a, const AEllR &e, double2 rb)
{
    double cd2 = cos_dec_acc(rb.y);
    double h = haversine(a.ra, a.dec, a.cosd, rb.x, rb.y, cd2);
    if (h == 0.0) return IN;
    const double diag = sqrt(e.a_arcsec * e.a_arcsec + e.b_arcsec * e.b_arcsec) * (1.0 + 1e-15);
    double sa = sin(kHalfDeg * (diag / 3600.0));
    if (h > (sa * sa) * (1.0 + kE40)) return OUT;
    double tn, te;
    tangent_ne(a.ra, a.dec, a.z, rb.x, rb.y, cd2, tn, te);
    double th = 2.0 * asin(sqrt(h));
    double sth = 2.0 * sqrt(h) * sqrt(1.0 - h);
    double f = th / sth;
    double su = tn * e.ct + te * e.st;
    double sv = te * e.ct - tn * e.st;
    double x = su / (kDeg * (e.a_arcsec / 3600.0));
    double y = sv / (kDeg * (e.b_arcsec / 3600.0));
    double qu = (f * f) * (x * x), qv = (f * f) * (y * y);
    double m = kE38 * (1.0 + e.a_arcsec / e.b_arcsec);
    if (qu > 1.0 + m || qv > 1.0 + m) return OUT;
    if (qu <= 1.0 - m && qv <= 1.0 - m) return IN;
    return AMBIG;
}

// Reach (degrees) of a per-source area: the semi-major axis of an ellipse,
// the half-diagonal of a rectangle (padded for its rounding).
__device__ __host__ __forceinline__ double area_reach_deg(int shape, double a_arcsec,
                                                          double b_arcsec)
{
    if (shape == C3X_RECT)
        return sqrt(a_arcsec * a_arcsec + b_arcsec * b_arcsec) * (1.0 + 1e-15) / 3600.0;
    return a_arcsec / 3600.0;
}

__device__ __forceinline__ bool same_point(const ARec &a, double2 rb)
{
    return a.dec == rb.y && (a.ra == rb.x || fabs(a.dec) == 90.0);
}

// First sorted position whose key is >= k (keys ascending). The result
// never exceeds nB, whatever the directory holds (an index whose sort gave
// up is discarded, but the kernels already queued on it stay in bounds).
__device__ __forceinline__ uint32_t key_lower_bound(const Grid &g, uint32_t k)
{
    uint32_t q = k >> g.dshift;
    if (q + 1 >= g.dsize) return (uint32_t)g.nB;
    uint32_t hi = min(g.dir[q + 1], (uint32_t)g.nB), lo = min(g.dir[q], hi);
    while (lo < hi) {
        uint32_t m = lo + ((hi - lo) >> 1);
        if (g.keys[m] < k) lo = m + 1;
        else hi = m;
    }
    return lo;
}

// Window of one source: the zones within reach in Dec and, unless the
// whole zone is needed (a cap holding a pole, or a wide RA window), an upper
// bound on the RA half-width of the cap. The exact half-width is
// asin(sin R / cos dec); with y = R / cos_lb >= sin R / cos dec (R in
// radians, cos_lb <= cos dec) it is at most asin(y) <= y / sqrt(1 - y^2).
// The pads absorb every rounding of this arithmetic, and zone_of / cell_of
// are monotone, so the cells found are an exact superset.
struct Window {
    int zlo, zhi;
    bool full;
    double dra;
};

__device__ __forceinline__ Window window_of(const Grid &g, double dec, double cos_lb,
                                            double reach_deg)
{
    Window w;
    double rp = reach_deg * (1.0 + 1e-9) + 1e-12;
    w.zlo = zone_of(dec - rp, g);
    w.zhi = zone_of(dec + rp, g);
    w.full = false;
    w.dra = 0.0;
    if (fabs(dec) + rp >= 90.0 || !(cos_lb > 0.0)) {
        w.full = true;
    } else {
        double y = (kDeg * rp) / cos_lb;
        if (y >= 0.9) {
            w.full = true;
        } else {
            w.dra = y / sqrt(1.0 - y * y) / kDeg * (1.0 + 1e-9) + 1e-12;
            if (w.dra >= 180.0) w.full = true;
        }
    }
    return w;
}

// Cell ranges [c0[k], c1[k]] of zone z covering [ra - dRA, ra + dRA], split
// at RA = 0/360 (at most two, disjoint). Returns how many.
__device__ __forceinline__ int zone_ranges(const ZoneInfo &zi, const Window &w, double ra,
                                           uint32_t c0[2], uint32_t c1[2])
{
    const uint32_t n = zi.n;
    if (!w.full) {
        double lo = ra - w.dra, hi = ra + w.dra;
        if (lo < 0.0) {
            uint32_t a0 = cell_in(zi, lo + 360.0), b1 = cell_in(zi, hi);
            if (a0 > b1) {
                c0[0] = 0;
                c1[0] = b1;
                c0[1] = a0;
                c1[1] = n - 1;
                return 2;
            }
        } else if (hi >= 360.0) {
            uint32_t a0 = cell_in(zi, lo), b1 = cell_in(zi, hi - 360.0);
            if (a0 > b1) {
                c0[0] = 0;
                c1[0] = b1;
                c0[1] = a0;
                c1[1] = n - 1;
                return 2;
            }
        } else {
            c0[0] = cell_in(zi, lo);
            c1[0] = cell_in(zi, hi);
            return 1;
        }
    }
    c0[0] = 0;
    c1[0] = n - 1;
    return 1;
}

// Calls f(zone, j0, j1) for every contiguous range of sorted B positions
// whose cells can hold a source within reach_deg of (ra, dec).
template <typename F>
__device__ __forceinline__ void for_each_range(const Grid &g, double ra, double dec, double cosd,
                                               double reach_deg, F &&f)
{
    Window w = window_of(g, dec, cosd, reach_deg);
    for (int z = w.zlo; z <= w.zhi; ++z) {
        const ZoneInfo zi = g.zinfo[z];
        const uint32_t base = zi.base;
        uint32_t c0[2], c1[2];
        int nr = zone_ranges(zi, w, ra, c0, c1);
        for (int k = 0; k < nr; ++k) {
            uint32_t j0 = key_lower_bound(g, base + c0[k]);
            uint32_t j1 = key_lower_bound(g, base + c1[k] + 1);
            if (j0 < j1) f(z, j0, j1);
        }
    }
}

}  // namespace c3x

// ----------------------------------------------------------------------------
// host-side pieces shared between translation units
// ----------------------------------------------------------------------------
namespace c3x {

void set_error(const char *fmt, ...);

// binary128 fallback (exact128.cpp, compiled without HIP)
extern "C" int c3x_q_circle(double ra1, double dec1, double ra2, double dec2, double r_arcsec);
extern "C" int c3x_q_ellipse(double ra1, double dec1, double ra2, double dec2, double a_arcsec,
                             double b_arcsec, double pa_deg, double pa_zero_deg, int pa_sense);
extern "C" int c3x_q_rect(double ra1, double dec1, double ra2, double dec2, double a_arcsec,
                          double b_arcsec, double pa_deg, double pa_zero_deg, int pa_sense);
extern "C" int c3x_q_best(double ra1, double dec1, int n, const double *ra2, const double *dec2,
                          const int32_t *idx);
extern "C" void c3x_q_thresholds(double r_arcsec, double *h_r, double *cr2);
extern "C" void c3x_frame_matrix(int src, int dst, double *M);

}  // namespace c3x
