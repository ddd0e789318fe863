// c3x_host.h -- host-side objects of the library: index, result, device
// memory cache, error reporting and phase timers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "c3x_internal.h"

namespace c3x {

// Internal status (never returned across the ABI): a one-sweep radix sort
// gave up its look-back, so the call's work is redone with the table
// schedule.
constexpr c3x_status kSortGaveUp = (c3x_status)7;  // within the enum's value range

// Thread-local error message; returns the status for convenience.
c3x_status fail(c3x_status st, const char *fmt, ...);
c3x_status fail_hip(hipError_t e, const char *what);
void clear_error();

// Device memory cache. Blocks are returned to the cache, not to HIP, and
// reused by size class; every API call synchronises its stream before it
// returns, so a block is never handed out while a kernel may still use it.
void *dev_alloc(size_t bytes);
void dev_free(void *p);
// Pinned host staging for a call's small read-backs (one buffer per host
// thread, kept for the process); null if it cannot be had.
uint8_t *pinned_stage(size_t bytes);

// RAII owner of device blocks allocated during one call.
// With a stream set, the destructor first waits for that stream, so blocks
// freed on an early error return are never reused while a kernel runs.
struct Arena {
    std::vector<void *> blocks;
    hipStream_t sync_stream = nullptr;
    bool sync_on_release = false;
    Arena() = default;
    explicit Arena(hipStream_t s) : sync_stream(s), sync_on_release(true) {}
    void *get(size_t bytes)
    {
        void *p = dev_alloc(bytes ? bytes : 16);
        if (p) blocks.push_back(p);
        return p;
    }
    template <typename T>
    T *get_n(int64_t n)
    {
        return (T *)get((size_t)(n > 0 ? n : 1) * sizeof(T));
    }
    void release_all()
    {
        if (sync_on_release && !blocks.empty()) (void)hipStreamSynchronize(sync_stream);
        for (void *p : blocks) dev_free(p);
        blocks.clear();
    }
    // Hand a block over to a longer-lived owner.
    void detach(void *p)
    {
        for (auto &b : blocks)
            if (b == p) {
                b = blocks.back();
                blocks.pop_back();
                return;
            }
    }
    ~Arena() { release_all(); }
};

// HIP events around phases of one call.
struct Timer {
    hipEvent_t ev[16];
    int n = 0;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st)
    {
        for (auto &e : ev) e = nullptr;
    }
    void mark()
    {
        if (n < 16) {
            if (!ev[n]) (void)hipEventCreate(&ev[n]);
            (void)hipEventRecord(ev[n], s);
            n++;
        }
    }
    double ms(int a, int b)
    {
        float t = 0.f;
        if (a < n && b < n) (void)hipEventElapsedTime(&t, ev[a], ev[b]);
        return (double)t;
    }
    ~Timer()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Zone tables of one cell size. Built once per cell size and process, and
// uploaded once per device; immutable and shared by every index using that
// cell size (a few MB per cell size, kept until the process ends).
struct ZoneTables {
    double cell_arcsec;
    double h_deg;
    int32_t nz;
    uint64_t ncells;
    int key_bits;
    double L_rad;                 // bound on |p - cell reference| (radians, chord)
    std::vector<ZoneInfo> zinfo;  // nz
    std::vector<double2> zref;    // nz
};

struct GridPlan {
    const ZoneTables *zt = nullptr;
    double cell_arcsec;
    double h_deg;
    int32_t nz;
    uint64_t ncells;
    int key_bits;
    double L_rad;
    int32_t dshift;
    uint32_t dsize;
};

// Catalogue positions converted from frame src to frame dst by the fixed
// FP64 rule (c3x_frames.hip); with orient given, also the area orientations
// T = pa_zero + pa_sense * pa[i] turned into the target frame; the first
// out-of-domain row goes to *bad (atomicMin). Stream-ordered.
hipError_t frame_convert(int src, int dst, const double *ra, const double *dec, int64_t n,
                         double *ra_out, double *dec_out, double *gamma_out, const double *pa,
                         double pa_zero, int pa_sense, double *orient, uint32_t *bad,
                         hipStream_t s);

// An environment switch (test settings): set and not "0".
inline bool env_on(const char *name)
{
    const char *e = getenv(name);
    return e && *e && strcmp(e, "0") != 0;
}

// Catalogue A (n rows, frame src) made ready for a cross-match in frame dst:
// nothing when the frames agree; otherwise its positions converted by the
// fixed rule into arrays of conv, and an oriented area's orientations turned
// with them (then taken with zero offset and sense +1). *ra, *dec and *area
// are replaced; C3X_EINVAL names the first row outside the domain.
// Synchronises the stream.
c3x_status convert_catalogue_a(int src, int dst, int64_t n, const double **ra, const double **dec,
                               c3x_area *area, Arena &conv, hipStream_t s);

// Device copies of a cell size's zone tables on the current device.
c3x_status device_zone_tables(const ZoneTables *zt, const ZoneInfo **zinfo, const double2 **zref);

}  // namespace c3x

struct c3x_index {
    int device;
    c3x_frame frame;
    c3x_precision precision;
    int64_t nB;
    double reach_hint_arcsec;
    c3x::GridPlan plan;
    c3x::Grid grid;               // device pointers
    c3x::Arena mem;               // owns everything below
    uint32_t *keys = nullptr;
    c3x::Pay64 *pay64 = nullptr;
    c3x::Pay32 *pay32 = nullptr;
    uint2 *res = nullptr;           // FP64 residuals of pay32 (mixed)
    double2 *radec = nullptr;  // B coordinates in input order (row pay64[j].idx)
    c3x_stats stats;
};

namespace c3x {

// An index build enqueued on its stream and not yet checked: index_build_begin
// validates and plans, allocates and enqueues every kernel;
// index_build_end waits for them, checks the rows and the sorts and hands
// the index over (or frees it; kSortGaveUp when a one-sweep sort gave up).
// c3x_build_index runs the two in a row; c3x_cross_match enqueues the A
// preparation on a second stream between them.
struct IndexBuild {
    c3x_index *ix = nullptr;
    hipStream_t s;
    Arena tmp;                // the kernels' working buffers
    Timer tm;
    uint32_t *bad = nullptr;  // [2]: first bad row, one-sweep give-up
    hipEvent_t grid_ready = nullptr;  // recorded on s once the grid is on the device
    hipError_t e = hipSuccess;
    explicit IndexBuild(hipStream_t st) : s(st), tmp(st), tm(st) {}
    ~IndexBuild()
    {
        delete ix;  // an index not handed over
        if (grid_ready) (void)hipEventDestroy(grid_ready);
    }
};
c3x_status index_build_begin(const double *ra_deg, const double *dec_deg, int64_t nB,
                             c3x_frame frame, double reach_hint_arcsec, const c3x_opts *opts,
                             bool onesweep, IndexBuild &b);
c3x_status index_build_end(IndexBuild &b, c3x_index **out);

// Work forked from stream s onto a second stream a: the constructor makes a
// wait for what s has queued so far (or, given `after`, for that event of
// s), join() makes s wait for what a has queued since, and the destructor
// waits for a (an early error return must not free buffers that a's
// kernels still use). a == s: all of it nothing.
struct StreamFork {
    hipStream_t s, a;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipSuccess;
    StreamFork(hipStream_t s_, hipStream_t a_, hipEvent_t after = nullptr) : s(s_), a(a_)
    {
        if (a == s) return;
        e = hipEventCreateWithFlags(&ev[0], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[1], hipEventDisableTiming);
        if (e == hipSuccess && !after) e = hipEventRecord(ev[0], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(a, after ? after : ev[0], 0);
    }
    hipError_t join()
    {
        if (a == s || e != hipSuccess) return e;
        e = hipEventRecord(ev[1], a);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ev[1], 0);
        return e;
    }
    ~StreamFork()
    {
        if (a != s) (void)hipStreamSynchronize(a);
        for (auto &x : ev)
            if (x) (void)hipEventDestroy(x);
    }
    StreamFork(const StreamFork &) = delete;
    StreamFork &operator=(const StreamFork &) = delete;
};

}  // namespace c3x

struct c3x_result {
    int device;
    int64_t n_pairs;
    int64_t nA;
    int64_t nB = -1;  // rows of catalogue B (c3x_match results; -1 for a batch)
    unsigned mode;
    c3x::Arena mem;
    int32_t *idxA = nullptr, *idxB = nullptr;
    double *sep = nullptr;
    int32_t *best_idx = nullptr;
    double *best_sep = nullptr;
    int32_t *unA = nullptr, *unB = nullptr;  // unmatched rows (c3x_result_unmatched)
    int32_t *level = nullptr;  // per pair: smallest scale holding it (c3x_match_concentric)
    // symmetric best pairs (c3x_result_mutual): pairs and each B row's nearest A row
    int32_t *muA = nullptr, *muB = nullptr, *muBA = nullptr;
    double *muS = nullptr;
    int64_t n_mutual = 0;
    int n_scales = 0;
    c3x_stats stats;
};
