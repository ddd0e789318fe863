// c3x_index.hip -- sky index over catalogue B (paper Section 2.3: each row
// of the second catalogue is put in the partition cell its coordinates fall
// in).
//
// The flat grid of the paper becomes declination zones of height h, each cut
// into n_z RA cells of true width >= h at the zone's edge nearest the
// equator; key = zbase[zone] + cell is zone-major, so the cells an A source
// needs in one zone are one contiguous key range. Phases (one stream):
//   k_prep_b    validate rows, key + packed copy         16 B in, 4 + 16 B out
//   radix sort  (key, row) by key, ceil(bits/8) passes   16 B per pass
//   k_gather_b  payload in sorted order                   20 B in, 32 or 16 + 8 B out
//   k_dir_fill  dir[q] = number of keys in buckets below q, written straight
//               from the sorted keys: each position fills the buckets between
//               its predecessor's and its own (long gaps by k_dir_fill_gaps)
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "c3x_dir.h"
#include "c3x_host.h"
#include "c3x_sort.h"

namespace c3x {

constexpr double kSkyArcsec2 = 4.0 * kPi * (180.0 / kPi * 3600.0) * (180.0 / kPi * 3600.0);
constexpr double kMinCellArcsec = 16.0;  // keeps the key space below 2^31 cells

static void build_zones(ZoneTables &p, double cell_arcsec)
{
    p.cell_arcsec = cell_arcsec;
    p.h_deg = cell_arcsec / 3600.0;
    p.nz = (int32_t)std::max(1.0, ceil(180.0 / p.h_deg));
    p.zinfo.assign(p.nz, ZoneInfo{0, 1, 0.0, 0.0, 0.0});
    p.zref.assign(p.nz, make_double2(0.0, 0.0));
    uint64_t tot = 0;
    double L = 0.0;
    for (int z = 0; z < p.nz; ++z) {
        double lo = -90.0 + z * p.h_deg;
        double hi = std::min(90.0, lo + p.h_deg);
        if (z == p.nz - 1) hi = 90.0;
        double deq = (lo <= 0.0 && hi >= 0.0) ? 0.0 : (fabs(lo) < fabs(hi) ? lo : hi);
        double ceq = cos(deq * kDeg);
        double nzf = floor(360.0 * ceq / p.h_deg);
        uint32_t n = (uint32_t)std::max(1.0, std::min(nzf, 4.0e9));
        p.zinfo[z].base = (uint32_t)std::min<uint64_t>(tot, 0xffffffffull);
        p.zinfo[z].n = n;
        p.zinfo[z].f = (double)n / 360.0;
        p.zinfo[z].g = ldexp(1.0, kRefBits) / (double)n;
        tot += n;
        double dc = std::max(-90.0, std::min(90.0, 0.5 * (lo + hi)));
        p.zref[z] = make_double2(cos(dc * kDeg), sin(dc * kDeg));
        // largest distance from a point of a cell to its reference: RA
        // half-cell + half a reference-grid step (+1e-6 rad of slack for the
        // FP32 sine/cosine of the grid point)
        double ddec = std::max(hi - dc, dc - lo);
        double dra = (180.0 / n + 180.0 / (1 << kRefBits)) * ceq + 1e-6 / kDeg;
        double ang = sqrt(ddec * ddec + dra * dra) * kDeg;
        L = std::max(L, ang);
    }
    p.ncells = tot;
    p.L_rad = L * 1.01 + 1e-12;
    uint64_t maxkey = tot ? tot - 1 : 0;
    int bits = 0;
    while (bits < 32 && (maxkey >> bits)) ++bits;
    p.key_bits = bits;
}

namespace {
struct TableCache {
    std::mutex mu;
    std::map<double, std::unique_ptr<ZoneTables>> host;
    std::map<std::pair<int, const ZoneTables *>, std::pair<ZoneInfo *, double2 *>> dev;
};
TableCache &tables()
{
    static TableCache *c = new TableCache();  // never destroyed: outlives static teardown
    return *c;
}
}  // namespace

static const ZoneTables *zone_tables(double cell_arcsec)
{
    TableCache &c = tables();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.host.find(cell_arcsec);
    if (it != c.host.end()) return it->second.get();
    std::unique_ptr<ZoneTables> t(new (std::nothrow) ZoneTables());
    if (!t) return nullptr;
    build_zones(*t, cell_arcsec);
    const ZoneTables *r = t.get();
    c.host[cell_arcsec] = std::move(t);
    return r;
}

c3x_status device_zone_tables(const ZoneTables *zt, const ZoneInfo **zinfo, const double2 **zref)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    TableCache &c = tables();
    std::lock_guard<std::mutex> g(c.mu);
    auto key = std::make_pair(dev, zt);
    auto it = c.dev.find(key);
    if (it == c.dev.end()) {
        ZoneInfo *zi = nullptr;
        double2 *zr = nullptr;
        hipError_t e = hipMalloc(&zi, zt->nz * sizeof(ZoneInfo));
        if (e == hipSuccess) e = hipMalloc(&zr, zt->nz * sizeof(double2));
        if (e == hipSuccess)
            e = hipMemcpy(zi, zt->zinfo.data(), zt->nz * sizeof(ZoneInfo), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(zr, zt->zref.data(), zt->nz * sizeof(double2), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (zi) (void)hipFree(zi);
            if (zr) (void)hipFree(zr);
            return fail_hip(e, "zone tables");
        }
        it = c.dev.emplace(key, std::make_pair(zi, zr)).first;
    }
    *zinfo = it->second.first;
    *zref = it->second.second;
    return C3X_OK;
}

// Chooses the cell side and the directory resolution. The cell is the
// reach (the paper sizes cells by the largest matching region), floored so
// that the key space stays below 2^31 cells.
c3x_status plan_grid(GridPlan &p, int64_t nB, double reach_arcsec, double cell_req)
{
    double cell = cell_req > 0.0 ? cell_req : std::max(reach_arcsec, kMinCellArcsec);
    cell = std::max(cell, 1e-3);
    cell = std::min(cell, 180.0 * 3600.0);
    // skip, without building their tables, the cell sizes whose cell count
    // (sky area / cell^2, within a zone count of the exact one) is far above 2^31
    while (kSkyArcsec2 / (cell * cell) > 4.0 * 2147483648.0) cell *= 1.25;
    const ZoneTables *zt = nullptr;
    for (int it = 0; it < 64; ++it) {
        zt = zone_tables(cell);
        if (!zt) return fail(C3X_ENOMEM, "zone tables");
        if (zt->ncells < (1ull << 31)) break;
        cell *= 1.25;
    }
    if (!zt || zt->ncells >= (1ull << 31)) return fail(C3X_EINVAL, "grid plan failed");
    p.zt = zt;
    p.cell_arcsec = zt->cell_arcsec;
    p.h_deg = zt->h_deg;
    p.nz = zt->nz;
    p.ncells = zt->ncells;
    p.key_bits = zt->key_bits;
    p.L_rad = zt->L_rad;
    uint64_t maxkey = p.ncells - 1;
    // directory: about two entries per B row, so that a bucket of the
    // uniform sky holds about one key and a lookup is one or two loads
    uint64_t want = std::max<uint64_t>(1024, (uint64_t)nB * 2);
    int sh = 0;
    while (sh < 31 && (maxkey >> sh) + 1 > want) ++sh;
    p.dshift = sh;
    p.dsize = (uint32_t)((maxkey >> sh) + 2);
    return C3X_OK;
}

// ---------------------------------------------------------------------------- kernels

// Keys of the B rows, and the coordinates packed in pairs so that the
// gather after the sort reads one 16-byte record per row.
__global__ void k_prep_b(const double *__restrict__ ra, const double *__restrict__ dec, int64_t n,
                         Grid g, uint32_t *__restrict__ keys, double2 *__restrict__ packed,
                         uint32_t *__restrict__ bad)
{
    // two rows a thread, j0 and j0 + ceil(n / 2), both loads issued first
    // (0.2 ms less over 200M rows than one row a thread)
    const int64_t h = (n + 1) / 2;
    const int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j0 >= h) return;
    const int64_t j1 = j0 + h;
    const bool two = j1 < n;
    double a0 = ra[j0], d0 = dec[j0];
    double a1 = two ? ra[j1] : 0.0, d1 = two ? dec[j1] : 0.0;
    packed[j0] = make_double2(a0, d0);
    if (two) packed[j1] = make_double2(a1, d1);
    const bool ok0 = isfinite(a0) && isfinite(d0) && a0 >= 0.0 && a0 < 360.0 && fabs(d0) <= 90.0;
    const bool ok1 = isfinite(a1) && isfinite(d1) && a1 >= 0.0 && a1 < 360.0 && fabs(d1) <= 90.0;
    if (!ok0) {
        atomicMin(bad, (uint32_t)j0);
        a0 = 0.0;
        d0 = 0.0;
    }
    if (two && !ok1) {
        atomicMin(bad, (uint32_t)j1);
        a1 = 0.0;
        d1 = 0.0;
    }
    const ZoneInfo zi0 = g.zinfo[zone_of(d0, g)];
    const ZoneInfo zi1 = g.zinfo[zone_of(d1, g)];
    keys[j0] = zi0.base + cell_in(zi0, a0);  // its value in the sort: the row itself
    if (two) keys[j1] = zi1.base + cell_in(zi1, a1);
}

template <int PREC>
__global__ void k_gather_b(const uint32_t *__restrict__ rows, const double2 *__restrict__ packed,
                           int64_t n, Grid g, Pay64 *__restrict__ p64, Pay32 *__restrict__ p32,
                           uint2 *__restrict__ res)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t row = rows[s];
    if (row >= (uint64_t)n) row = 0;  // unreachable for a permutation; keeps reads in bounds
    const double2 rd = packed[row];
    const double a = rd.x, d = rd.y;
    double x, y, z;
    unit_vec(a, d, x, y, z);
    if (PREC == C3X_FP64) {
        Pay64 q8;
        q8.x = x;
        q8.y = y;
        q8.z = z;
        q8.idx = row;
        q8.pad = 0;
        p64[s] = q8;
    } else {
        int zz = zone_of(d, g);
        uint32_t c = cell_of(zz, a, g);
        double rx, ry, rz;
        const uint32_t st = ref_step(g.zinfo[zz], c);
        ref_vec(g.zref[zz], st, rx, ry, rz);
        const double ox = x - rx, oy = y - ry, oz = z - rz;
        Pay32 q;
        q.x = (float)ox;
        q.y = (float)oy;
        q.z = (float)oz;
        q.idx = row | ((st & 1u) << 31);  // the step's parity: a window spans at most two
        p32[s] = q;
        res[s] = res_pack(ox, oy, oz, q.x, q.y, q.z);
    }
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Points the index's grid at the (shared, cached) device zone tables.
c3x_status upload_grid(c3x_index *ix, hipStream_t s)
{
    (void)s;
    GridPlan &p = ix->plan;
    Grid &g = ix->grid;
    const ZoneInfo *zinfo = nullptr;
    const double2 *zref = nullptr;
    c3x_status st = device_zone_tables(p.zt, &zinfo, &zref);
    if (st != C3X_OK) return st;
    g.h_deg = p.h_deg;
    g.inv_h = 1.0 / p.h_deg;
    g.nz = p.nz;
    g.ncells = (uint32_t)p.ncells;
    g.zinfo = zinfo;
    g.zref = zref;
    g.dshift = p.dshift;
    g.dsize = p.dsize;
    return C3X_OK;
}

}  // namespace c3x

using namespace c3x;

// onesweep: large sorts may take the one-sweep schedule (kSortGaveUp if its
// look-back gave up; the caller then builds again without it).
namespace c3x {

c3x_status index_build_begin(const double *ra_deg, const double *dec_deg, int64_t nB,
                             c3x_frame frame, double reach_hint_arcsec, const c3x_opts *opts,
                             bool onesweep, IndexBuild &b)
{
    if (nB < 0) return fail(C3X_EINVAL, "nB < 0");
    if (nB > 2147483647LL) return fail(C3X_ERANGE, "nB above 2^31 - 1");
    if (nB > 0 && (!ra_deg || !dec_deg)) return fail(C3X_EINVAL, "NULL coordinate array");
    if (frame != C3X_EQUATORIAL && frame != C3X_GALACTIC) return fail(C3X_EINVAL, "bad frame");
    if (!(reach_hint_arcsec >= 0.0) || !isfinite(reach_hint_arcsec))
        return fail(C3X_EINVAL, "reach_hint_arcsec must be finite and >= 0");
    c3x_opts o{};
    if (opts) o = *opts;
    if (o.precision != C3X_FP64 && o.precision != C3X_MIXED)
        return fail(C3X_EINVAL, "bad precision");
    if (!(o.cell_arcsec >= 0.0) || !isfinite(o.cell_arcsec))
        return fail(C3X_EINVAL, "cell_arcsec must be finite and >= 0");
    hipStream_t s = b.s;

    c3x_index *ix = new (std::nothrow) c3x_index();
    if (!ix) return fail(C3X_ENOMEM, "host allocation");
    b.ix = ix;
    (void)hipGetDevice(&ix->device);
    ix->frame = frame;
    ix->precision = o.precision;
    ix->nB = nB;
    ix->reach_hint_arcsec = reach_hint_arcsec;
    memset(&ix->stats, 0, sizeof(ix->stats));
    c3x_status st = plan_grid(ix->plan, nB, reach_hint_arcsec, o.cell_arcsec);
    if (st != C3X_OK) return st;
    b.tm.mark();
    st = upload_grid(ix, s);
    if (st != C3X_OK) return st;
    // work that needs only the grid may start here on another stream
    if (hipEventCreateWithFlags(&b.grid_ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(b.grid_ready, s) != hipSuccess)
        return fail(C3X_EDEVICE, "event");
    Arena &tmp = b.tmp;
    int64_t n = nB;
    uint32_t *keys = ix->mem.get_n<uint32_t>(n);
    uint32_t *rows = tmp.get_n<uint32_t>(n);
    uint32_t *ktmp = tmp.get_n<uint32_t>(n);
    uint32_t *rtmp = tmp.get_n<uint32_t>(n);
    void *ws = tmp.get(radix_ws_bytes(n));
    uint32_t *bad = tmp.get_n<uint32_t>(2);  // first bad row; sort give-up
    b.bad = bad;
    // the coordinates in input order: the gathers' source, then kept by the
    // index (the band recheck reads them through the payload's row)
    double2 *packed = ix->mem.get_n<double2>(n);
    Pay64 *p64 = nullptr;
    Pay32 *p32 = nullptr;
    uint2 *res = nullptr;
    // one payload per index: FP64 unit vectors, or FP32 offsets from the
    // cell references (the mixed filter) with their FP64 residuals (the
    // chords of its matches)
    if (o.precision == C3X_FP64) {
        p64 = ix->mem.get_n<Pay64>(n);
    } else {
        p32 = ix->mem.get_n<Pay32>(n);
        res = ix->mem.get_n<uint2>(n);
    }
    uint32_t *dir = ix->mem.get_n<uint32_t>(ix->plan.dsize);
    const uint32_t gap_cap = dir_gap_cap(ix->plan.dsize), big_cap = dir_big_cap(ix->plan.dsize);
    uint3 *gaps = tmp.get_n<uint3>((int64_t)gap_cap + big_cap);
    uint32_t *n_gaps = tmp.get_n<uint32_t>(2);
    if (!keys || !rows || !ktmp || !rtmp || !ws || !bad || !packed || !dir || !gaps || !n_gaps ||
        (!p64 && !(p32 && res)))
        return fail(C3X_ENOMEM, "index buffers");
    hipError_t e = hipMemsetAsync(bad, 0xff, sizeof(uint32_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(bad + 1, 0, sizeof(uint32_t), s);
    Grid g = ix->grid;
    g.nB = (int32_t)n;
    if (n > 0)
        hipLaunchKernelGGL(k_prep_b, dim3(nblk((n + 1) / 2, 256)), dim3(256), 0, s, ra_deg, dec_deg,
                           n, g,
                           keys, packed, bad);
    int in_tmp = 0;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess)
        e = radix_sort_pairs(keys, rows, ktmp, rtmp, n, ix->plan.key_bits, ws, s, &in_tmp,
                             /*vals_are_index=*/true, onesweep ? bad + 1 : nullptr);
    if (e == hipSuccess && in_tmp) {
        e = hipMemcpyAsync(keys, ktmp, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        rows = rtmp;
    }
    if (e == hipSuccess && n > 0) {
        if (o.precision == C3X_FP64)
            hipLaunchKernelGGL(k_gather_b<C3X_FP64>, dim3(nblk(n, 256)), dim3(256), 0, s, rows,
                               packed, n, g, p64, p32, res);
        else
            hipLaunchKernelGGL(k_gather_b<C3X_MIXED>, dim3(nblk(n, 256)), dim3(256), 0, s, rows,
                               packed, n, g, p64, p32, res);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemsetAsync(n_gaps, 0, 2 * sizeof(uint32_t), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_dir_fill, dim3(nblk(n + 1, 256)), dim3(256), 0, s, keys, n,
                           ix->plan.dshift, ix->plan.dsize, dir, gaps, n_gaps, gap_cap, big_cap);
        hipLaunchKernelGGL(k_dir_fill_gaps, dim3(4096), dim3(256), 0, s, gaps, n_gaps, gap_cap,
                           big_cap, dir);
        e = hipGetLastError();
    }
    b.tm.mark();
    ix->keys = keys;
    ix->pay64 = p64;
    ix->pay32 = p32;
    ix->res = res;
    ix->radec = packed;
    ix->grid.keys = keys;
    ix->grid.dir = dir;
    ix->grid.nB = (int32_t)n;
    ix->stats.precision = (int32_t)o.precision;
    b.e = e;
    if (e != hipSuccess) return fail_hip(e, "c3x_build_index");
    return C3X_OK;
}

c3x_status index_build_end(IndexBuild &b, c3x_index **out)
{
    hipError_t e = b.e;
    uint32_t bad_h[2] = {0xffffffffu, 0u};
    uint32_t *hbad = (uint32_t *)pinned_stage(64);
    if (!hbad) hbad = bad_h;
    hbad[0] = 0xffffffffu;
    hbad[1] = 0u;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(hbad, b.bad, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, b.s);
    if (e == hipSuccess) e = hipStreamSynchronize(b.s);
    const uint32_t sort_gave_up = hbad[1];
    bad_h[0] = hbad[0];
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(b.s);
        return fail_hip(e, "c3x_build_index");
    }
    if (sort_gave_up) return kSortGaveUp;
    if (bad_h[0] != 0xffffffffu)
        return fail(C3X_EINVAL, "catalogue B row %u: coordinate outside RA [0,360), |Dec| <= 90 "
                                "or not finite", bad_h[0]);
    c3x_index *ix = b.ix;
    c3x_stats &S = ix->stats;
    S.n_b = ix->nB;
    S.n_cells = (int64_t)ix->plan.ncells;
    S.cell_arcsec = ix->plan.cell_arcsec;
    S.ms_index = b.tm.ms(0, 1);
    S.ms_total = S.ms_index;
    b.ix = nullptr;
    *out = ix;
    return C3X_OK;
}

}  // namespace c3x

static c3x_status build_index_impl(const double *ra_deg, const double *dec_deg, int64_t nB,
                                   c3x_frame frame, double reach_hint_arcsec,
                                   const c3x_opts *opts, bool onesweep, c3x_index **out)
{
    IndexBuild b(opts ? (hipStream_t)opts->stream : nullptr);
    c3x_status st = index_build_begin(ra_deg, dec_deg, nB, frame, reach_hint_arcsec, opts,
                                      onesweep, b);
    if (st != C3X_OK) {
        (void)hipStreamSynchronize(b.s);
        return st;
    }
    return index_build_end(b, out);
}

extern "C" c3x_status c3x_build_index(const double *ra_deg, const double *dec_deg, int64_t nB,
                                      c3x_frame frame, double reach_hint_arcsec,
                                      const c3x_opts *opts, c3x_index **out)
{
    clear_error();
    if (!out) return fail(C3X_EINVAL, "out is NULL");
    *out = nullptr;
    c3x_status st = build_index_impl(ra_deg, dec_deg, nB, frame, reach_hint_arcsec, opts, true, out);
    if (st != kSortGaveUp) return st;
    // the one-sweep sort gave up its look-back: build again with the table
    // schedule, which never waits
    st = build_index_impl(ra_deg, dec_deg, nB, frame, reach_hint_arcsec, opts, false, out);
    if (st == C3X_OK) (*out)->stats.n_sort_retries = 1;
    return st;
}

extern "C" void c3x_index_free(c3x_index *ix) { delete ix; }

extern "C" c3x_status c3x_index_stats(const c3x_index *ix, c3x_stats *s)
{
    if (!ix || !s) return fail(C3X_EINVAL, "NULL argument");
    *s = ix->stats;
    return C3X_OK;
}
