/*
 * c3x.h -- C ABI of the MI355X positional cross-match library (libc3x.so).
 *
 * The library implements the "Sky" functional case of the C^3 cross-match
 * (Riccio et al., ADASS XXVI, arXiv:1611.08494, Section 2.1): for every
 * source of catalogue A it finds the catalogue-B sources inside a region
 * centred on that source -- a circle of fixed radius, or an ellipse whose
 * semi-axes and position angle come from per-source catalogue parameters --
 * with the "all" and "best" match selections of Section 2.2, on equatorial or
 * galactic coordinates (Section 2). The sky partitioning of Section 2.3
 * (catalogue B assigned to cells, each A source tested only against the
 * cells around it) is restated for the sphere as declination zones split
 * into RA cells.
 *
 * Semantics (the exact pair set). Inputs are IEEE doubles taken as exact
 * reals and theta(i, j) is the exact great-circle angle.
 *   circle : j matches i  <=>  theta(i, j) <= r.
 *   ellipse: j matches i  <=>  (u/a_i)^2 + (v/b_i)^2 <= 1, where
 *            (u, v) = theta * (cos(phi - T_i), sin(phi - T_i)), phi is the
 *            bearing of j seen from i from local north (+Dec, or +b for
 *            galactic input) towards local east (+RA / +l), and
 *            T_i = pa_zero_deg + pa_sense * pa_deg[i] is the direction of
 *            the semi-major axis (Section 2.1: the PA has a zero-point and a
 *            direction of rotation). a = b gives theta <= a.
 *   rectangle: j matches i  <=>  |u| <= a_i and |v| <= b_i (half-sides).
 *   Boundaries are inclusive. best(i) is the match with the smallest exact
 *   theta; an exact tie goes to the lower B row.
 * Every decision is certified: the GPU decides in FP32 (MIXED) or FP64 with
 * proven error margins, re-decides band cases with a relative-accuracy FP64
 * formula, and resolves what is still undecided on the host in binary128.
 * Pairs whose exact value lies within 2^-96 (relative) of the threshold are
 * treated as on the boundary, so inside.
 *
 * Memory and ownership. Catalogue and area arrays are caller-owned, C-
 * contiguous float64 DEVICE pointers on the current HIP device; they only
 * need to stay valid for the duration of the call. An index owns copies of
 * what it needs and is immutable: several c3x_match calls may share it
 * concurrently on different streams. Results own their device buffers until
 * c3x_result_free. All work is ordered on opts->stream (NULL: the null
 * stream); c3x_match synchronises that stream to size its outputs.
 *
 * Errors. Every call returns a status; on error *out is NULL and nothing
 * leaks. c3x_last_error() gives a thread-local message (for bad input rows it
 * names the first offending row). The library never throws or aborts.
 *
 * Input domain: RA (or l) in [0, 360), Dec (or b) in [-90, 90], finite;
 * radius 0 or in [1e-6", 324000"]; ellipse 1e-6" <= b <= a <= 324000",
 * a <= 1000 b, PA finite; pa_sense +1 or -1; row counts <= 2^31 - 1.
 */
#ifndef C3X_H
#define C3X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define C3X_ABI_VERSION 2

typedef enum {
    C3X_OK = 0,
    C3X_EINVAL = 1,   /* bad argument or out-of-domain input value */
    C3X_ERANGE = 2,   /* a row count above 2^31 - 1 */
    C3X_ENOMEM = 3,   /* device or host allocation failed */
    C3X_EDEVICE = 4,  /* HIP runtime error (message holds the HIP string) */
    C3X_EFRAME = 5    /* kept for the ABI; frames that differ are converted */
} c3x_status;

/* Coordinate frame of a catalogue (Section 2: equatorial and galactic). It
 * fixes what "north" means for the position angle. A catalogue A in the
 * other frame than the index's is converted into the index's frame (see
 * c3x_frame_convert). */
typedef enum { C3X_EQUATORIAL = 0, C3X_GALACTIC = 1 } c3x_frame;

/* Region shape (Section 2.1: an elliptical, circular -- the special ellipse
 * -- or rectangular region). C3X_RECT: |u| <= a and |v| <= b in the
 * ellipse's frame (see the semantics above), a the half-side along the
 * orientation T, b across it; the area arrays and their domain are the
 * ellipse's (semi_major_arcsec = a, semi_minor_arcsec = b). */
typedef enum { C3X_CIRCLE = 0, C3X_ELLIPSE = 1, C3X_RECT = 2 } c3x_shape;

/* Match selection (Section 2.2). OR-able. ALL writes every pair; BEST fills
 * the per-A best arrays; BEST alone writes one pair per matched A row. */
enum { C3X_ALL = 1u, C3X_BEST = 2u };

/* Arithmetic of the GPU filter. Both give the same pair set. */
typedef enum { C3X_FP64 = 0, C3X_MIXED = 1 } c3x_precision;

/* The matching area centred on each A source (Section 2.1). */
typedef struct {
    c3x_shape shape;
    double radius_arcsec;            /* CIRCLE: fixed radius */
    const double *semi_major_arcsec; /* ELLIPSE, RECT: device, nA entries */
    const double *semi_minor_arcsec; /* ELLIPSE, RECT: device, nA entries */
    const double *pa_deg;            /* ELLIPSE, RECT: device, nA entries */
    double pa_zero_deg;              /* T = pa_zero_deg + pa_sense * PA */
    int pa_sense;                    /* +1 or -1 */
} c3x_area;

/* Options. Zero-initialised fields mean "choose automatically".
 * cell_arcsec: side of the sky cells (the partition resolution the paper
 *   lets users tune, Section 4); 0 lets the planner pick it. It never
 *   changes the answer.
 * tile: A sources per workgroup in the match kernels (64 or 256; 0 = auto).
 * stream: hipStream_t to order all work on (NULL = null stream). */
typedef struct {
    c3x_precision precision;
    double cell_arcsec;
    int tile;
    void *stream;
} c3x_opts;

typedef struct c3x_index c3x_index;
typedef struct c3x_result c3x_result;
typedef struct c3x_batch c3x_batch;

/* One job of a batch: rows [a_off, a_off + nA) of catalogue A against rows
 * [b_off, b_off + nB) of catalogue B, circle of radius_arcsec (0 or in
 * [1e-6, 3600]). Jobs are independent; their row ranges may overlap. */
typedef struct {
    int64_t a_off, nA, b_off, nB;
    double radius_arcsec;
} c3x_job;

/* Catalogues in different frames (Section 2: equatorial and galactic
 * coordinates). c3x_match (and c3x_match_concentric) accept catalogue A in
 * the other frame than the index's: A's positions are first converted into
 * the index's frame by the fixed FP64 rule of c3x_frame_convert, the area
 * orientations T = pa_zero + pa_sense * PA turned with them, and the
 * converted doubles are A's inputs of the match (the result's rows are
 * still A's own).
 *
 * c3x_frame_matrix: the rule's rotation from frame src to frame dst (host,
 * row-major, 9 doubles): fixed by the galactic north pole at RA 192.85948
 * deg, Dec 27.12825 deg and the galactic longitude 122.93192 deg of the
 * north celestial pole, taken as exact decimals, each entry the double
 * nearest its exact value.
 *
 * c3x_frame_convert: n positions (device float64 arrays, degrees) from frame
 * src to frame dst by the rule, which uses only correctly rounded +, -, *,
 * / and exact floor, frexp, ldexp in a fixed order (series sine, cosine and
 * arctangent, a Newton square root), so any IEEE FP64 machine following it
 * gets the same bits; it is within 1e-11 deg of the exact rotation.
 * gamma_out (may be NULL) receives for every row the angle (degrees) that
 * turns an orientation measured in frame src (from local north towards local
 * east) into one measured in frame dst. Output arrays are caller-owned
 * device memory; the call synchronises `stream`. Errors: C3X_EINVAL (bad
 * frame, NULL array, an input row outside RA [0, 360), |Dec| <= 90 or not
 * finite: the message names the first), C3X_ENOMEM, C3X_EDEVICE. */
void c3x_frame_matrix(int src, int dst, double *M);
c3x_status c3x_frame_convert(const double *ra, const double *dec, int64_t n, c3x_frame src,
                             c3x_frame dst, double *ra_out, double *dec_out, double *gamma_out,
                             void *stream);

/* Counters and phase times of one call (milliseconds from HIP events). */
typedef struct {
    int64_t n_a, n_b;
    int64_t n_pairs;          /* pairs written (ALL) or matched A rows (BEST only) */
    int64_t n_tests;          /* candidate (A, B) pairs examined by the match kernel */
    int64_t n_band;           /* candidates re-decided by the FP64 haversine form */
    int64_t n_ambiguous;      /* pairs resolved on the host in binary128 */
    int64_t n_best_ties;      /* best matches re-ranked on the host */
    int64_t n_cells;          /* cells of the sky grid */
    double cell_arcsec;       /* cell side used */
    double ms_index;          /* build_index phases (index stats only) */
    double ms_a_prep;         /* A keys, sort, records */
    double ms_count;          /* count pass */
    double ms_scan;
    double ms_write;          /* write pass + best */
    double ms_sort_pairs;     /* per-A segment ordering */
    double ms_total;
    int32_t precision;
    int32_t tile;
    double ms_count_kernel;   /* the count kernel's own launch (one lane per source) */
    int32_t n_sort_retries;   /* 1: a large radix sort's look-back gave up and the call's
                                 work was redone with the table schedule */
    int32_t queue;            /* batch: 1 when its count pass runs as the persistent kernel
                                 taking tiles costliest first (0: one workgroup per tile) */
} c3x_stats;

/* Builds the sky index over catalogue B: validates the rows, puts each row
 * in the zone/RA cell its coordinates fall in (the partition of Section
 * 2.3), sorts B by cell with an LDS radix sort, and builds the cell
 * directory. A large sort whose bounded look-back gave up is redone with the
 * table schedule (stats n_sort_retries = 1), never returned out of order. ra_deg/dec_deg: device float64[nB].
 * reach_hint_arcsec: the largest radius or semi-major axis expected (sizes
 * the cells; any reach still works). opts may be NULL.
 * Errors: C3X_EINVAL (bad row: message names it; bad frame or options),
 * C3X_ERANGE (nB > 2^31 - 1), C3X_ENOMEM, C3X_EDEVICE. */
c3x_status c3x_build_index(const double *ra_deg, const double *dec_deg, int64_t nB,
                           c3x_frame frame, double reach_hint_arcsec, const c3x_opts *opts,
                           c3x_index **out);

/* Cross-matches catalogue A against an index (Section 2.1 region test,
 * Section 2.2 selection). ra_deg/dec_deg: device float64[nA]; area as
 * above; mode: C3X_ALL, C3X_BEST or both. opts->precision must be the one
 * the index was built with (opts NULL: the index's).
 * Output (via c3x_result_copy): pairs in canonical (idxA, idxB) ascending
 * order, 0-based rows of the caller's arrays; sep in arcsec (float64, within
 * 1e-6" of exact); best_idxB[nA] (-1 if unmatched), best_sep[nA] (NaN).
 * frame: catalogue A's frame; when it differs from the index's, A's
 * positions and area orientations are converted into the index's frame by
 * the rule of c3x_frame_convert before the match.
 * Errors: C3X_EINVAL, C3X_ERANGE, C3X_ENOMEM, C3X_EDEVICE. */
c3x_status c3x_match(const c3x_index *ix, const double *ra_deg, const double *dec_deg,
                     int64_t nA, c3x_frame frame, const c3x_area *area, unsigned mode,
                     const c3x_opts *opts, c3x_result **out);

/* The whole cross-match of Section 2 in one call: c3x_build_index over
 * catalogue B (raB/decB, nB, frameB, reach_hint_arcsec) and c3x_match of
 * catalogue A (raA/decA, nA, frameA, area, mode) against it, with the same
 * checks, errors and outputs as the two calls in a row. The difference is
 * only in time: catalogue A is keyed and sorted on a second stream while
 * B's index is built on opts->stream, and the two meet where A's candidate
 * ranges are taken from the index. The second stream (default priority,
 * not synchronising with the null stream) is the library's own, one per
 * device, kept to the end of the process; calls that overlap on one device
 * share it and run their A halves one after the other. index_out (may be NULL: the index is freed) receives the index
 * for later c3x_match calls. Synchronises opts->stream; *out and *index_out
 * are left NULL on an error. */
c3x_status c3x_cross_match(const double *raB, const double *decB, int64_t nB, c3x_frame frameB,
                           double reach_hint_arcsec, const double *raA, const double *decA,
                           int64_t nA, c3x_frame frameA, const c3x_area *area, unsigned mode,
                           const c3x_opts *opts, c3x_index **index_out, c3x_result **out);

/* Sizes of a result: number of pairs and of A rows. */
c3x_status c3x_result_sizes(const c3x_result *r, int64_t *n_pairs, int64_t *nA);

/* Copies result arrays into caller buffers (device or host pointers; any may
 * be NULL to skip it). idxA/idxB/sep_arcsec take n_pairs entries,
 * best_idxB/best_sep_arcsec nA entries. Ordered on `stream`, synchronous
 * with respect to the host when any destination is host memory. */
c3x_status c3x_result_copy(const c3x_result *r, int32_t *idxA, int32_t *idxB,
                           double *sep_arcsec, int32_t *best_idxB, double *best_sep_arcsec,
                           void *stream);

/* Device views of a result's arrays, owned by the result: valid until
 * c3x_result_free (which first waits for the device, so that no queued work
 * still reads them). Layout as for c3x_result_copy; any output may be NULL.
 * The arrays are complete once the stream of the call that made the result
 * has reached the point where that call returned. */
c3x_status c3x_result_views(const c3x_result *r, const int32_t **idxA, const int32_t **idxB,
                            const double **sep_arcsec, const int32_t **best_idxB,
                            const double **best_sep_arcsec);

/* Concentric ellipses (Section 3, ClumpPopulator): each A source's ellipse
 * (area->shape must be C3X_ELLIPSE) is also taken at the scale factors
 * scales[0] < scales[1] < ... < scales[n_scales - 1] (host array, finite,
 * > 0, 1 <= n_scales <= 64): ellipse m has semi-axes a * scales[m] and
 * b * scales[m] (FP64 products), the source's centre and position angle.
 * The result is c3x_match's for the largest ellipse (mode must include
 * C3X_ALL; C3X_BEST adds the best matches within it), and each of its pairs
 * has a level: the smallest m whose ellipse holds the B source (the
 * ellipses are nested), read with c3x_result_levels. The largest ellipse
 * is one certified c3x_match over the index; each pair's level is then
 * decided exactly as a certified match at every smaller scale would decide
 * it (FP64 with a proven margin, else binary128 on the host), so every
 * scale's axes must satisfy c3x_match's ellipse domain. The returned
 * result's stats are those of the largest ellipse's call, with the level
 * decisions taken on the host added to n_ambiguous. Errors: those of
 * c3x_match (prefixed with the failing scale); C3X_EINVAL also for a
 * circle, a mode without C3X_ALL, or bad scales. */
c3x_status c3x_match_concentric(const c3x_index *ix, const double *ra_deg, const double *dec_deg,
                                int64_t nA, c3x_frame frame, const c3x_area *area,
                                const double *scales, int32_t n_scales, unsigned mode,
                                const c3x_opts *opts, c3x_result **out);

/* Per-pair levels of a c3x_match_concentric result: int32 device array of
 * n_pairs entries in the pairs' order, owned by r. EINVAL for other
 * results. */
c3x_status c3x_result_levels(const c3x_result *r, const int32_t **level);

/* Column type of the Exact Value case. */
typedef enum { C3X_KEY_I64 = 0, C3X_KEY_F64 = 1 } c3x_keytype;

/* The Exact Value case (Section 2.1): A row i and B row j match when the
 * chosen columns hold equal values, keyA[i] == keyB[j] (int64: equal
 * integers; float64: numerically equal, +0 equal to -0, a NaN equal to
 * nothing). keyA, keyB: device arrays of nA and nB 8-byte values of `type`
 * (caller-owned, read during the call). mode: C3X_ALL and/or C3X_BEST
 * (Section 2.2); every match of a row is equally good, so its best match is
 * its lowest matching B row. The result reads like c3x_match's: pairs in
 * (idxA, idxB) order with separation 0, best_idxB (-1 if unmatched) and
 * best_sep (0, NaN if unmatched); BEST alone stores one pair per matched A
 * row; c3x_result_unmatched gives its join types (Section 2.2). A GPU hash
 * join: B hashed and ordered by hash (LDS radix sort), a directory over the
 * hash's top bits as the buckets, one probe per A row, count, scan, write.
 * Work is ordered on `stream` (NULL: the null stream), synchronised to size
 * the outputs. Errors: C3X_EINVAL, C3X_ERANGE (a count above 2^31 - 1),
 * C3X_ENOMEM, C3X_EDEVICE. */
c3x_status c3x_exact_match(const void *keyA, int64_t nA, const void *keyB, int64_t nB,
                           c3x_keytype type, unsigned mode, void *stream, c3x_result **out);

/* Rows without a stored match, from which every join type of Section 2.2
 * ("Match selection and join types") is assembled with the stored pairs:
 *   1 and 2        the stored pairs;
 *   1 or 2         the pairs, the unmatched A rows and the unmatched B rows;
 *   All from 1 (2) the pairs and the unmatched A (B) rows;
 *   1 not 2 (2 not 1)  the unmatched A (B) rows;
 *   1 xor 2        the unmatched A rows and the unmatched B rows.
 * selection picks the stored pairs: C3X_ALL, every match (r made with
 * C3X_ALL); C3X_BEST, each matched A row with its best match (r made with
 * C3X_BEST). An A row is unmatched when it has no match (under either
 * selection); a B row when no stored pair names it (under C3X_BEST: it is
 * no A row's best match). On return *rowsA (*rowsB) points to the ascending
 * int32 row indices of the unmatched A (B) rows, *n_rowsA (*n_rowsB) of
 * them: device arrays owned by r, valid until c3x_result_free and
 * overwritten by the next call on r. Work is ordered on `stream` (NULL: the
 * null stream), which is synchronised before the call returns. Only
 * results of c3x_match qualify (a batch result holds job-local rows).
 * Errors: C3X_EINVAL (NULL argument, batch result, selection not C3X_ALL or
 * C3X_BEST or not in r's mode), C3X_ENOMEM, C3X_EDEVICE. */
c3x_status c3x_result_unmatched(c3x_result *r, unsigned selection, void *stream,
                                const int32_t **rowsA, int64_t *n_rowsA,
                                const int32_t **rowsB, int64_t *n_rowsB);

/* No-allocation form of c3x_result_unmatched, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The unmatched rows of r (same meaning,
 * selection and order as c3x_result_unmatched) go to the caller's device
 * arrays rowsA[capA] and rowsB[capB] (capA >= nA and capB >= nB of r), and
 * their numbers to counts[0] (A) and counts[1] (B), a caller device array of
 * two int64 (-1 in both if a stored pair names a row outside its
 * catalogue). No memory is allocated: the working memory is one fixed
 * library array of 64 MiB per GPU, held from the library's load to the end
 * of the process, which takes about nA + nB bytes for a result of nA and nB
 * rows; larger results fail with C3X_ERANGE and nothing is written. All work
 * is queued on `stream` (NULL: the null stream) and the call returns
 * without waiting for it. Every call on one GPU shares that GPU's array and
 * leaves it holding its data: calls that overlap in time on one GPU
 * (different streams or host threads) race and must not be made. Errors:
 * C3X_EINVAL (NULL argument, batch result, selection not C3X_ALL or
 * C3X_BEST or not in r's mode, capacity below nA or nB), C3X_ERANGE,
 * C3X_EDEVICE. */
c3x_status c3x_result_unmatched_noalloc(const c3x_result *r, unsigned selection, void *stream,
                                        int32_t *rowsA, int64_t capA, int32_t *rowsB,
                                        int64_t capB, int64_t *counts);

/* Symmetric best pairs (Section 2.2, the "best" match selection, read as
 * the pairs that are each other's nearest match). Seen from catalogue B,
 * each B row's nearest A row is the one at the smallest exact angle among
 * the A rows whose areas hold it (an exact tie goes to the lower A row);
 * (i, j) is a symmetric best pair when j is the best match of A row i and i
 * is the nearest A row of B row j. Each row of either catalogue is in at
 * most one such pair. r must come from c3x_match with mode C3X_ALL |
 * C3X_BEST; raA/decA and raB/decB are the device arrays of that call (nA
 * and nB entries), read only to rank, in binary128 on the host, the B rows
 * whose nearest A rows the stored FP64 separations cannot tell apart (within
 * 2.5e-8" + 2^-38 relative). On return *idxA, *idxB, *sep (device arrays
 * owned by r, valid until c3x_result_free and overwritten by the next call
 * on r) hold the *n_pairs symmetric pairs in ascending A row, with the
 * pair's stored separation (arcsec); *best_a_of_b (may be NULL) the nearest
 * A row of every B row (-1: in no pair). Work is ordered on `stream` (NULL:
 * the null stream), which is synchronised before the call returns.
 * Errors: C3X_EINVAL (NULL argument, batch result, mode without both
 * C3X_ALL and C3X_BEST), C3X_ENOMEM, C3X_EDEVICE. */
c3x_status c3x_result_mutual(c3x_result *r, const double *raA, const double *decA,
                             const double *raB, const double *decB, void *stream,
                             const int32_t **idxA, const int32_t **idxB, const double **sep,
                             int64_t *n_pairs, const int32_t **best_a_of_b);

/* Counters and timings of the call that produced r (or of an index). */
c3x_status c3x_result_stats(const c3x_result *r, c3x_stats *s);
c3x_status c3x_index_stats(const c3x_index *ix, c3x_stats *s);

void c3x_result_free(c3x_result *r);
void c3x_index_free(c3x_index *ix);

/* Batched form: many independent circular cross-matches (each one the
 * "Sky" case of Section 2.1 with all and best matches, Section 2.2) in one
 * graph launch; the paper's partition of the work over concurrent processes
 * (Section 2.3) becomes one shared index and one launch of each kernel.
 *
 * c3x_batch_plan: raA/decA and raB/decB are device FP64 arrays (degrees)
 * holding every row the jobs name; jobs is a host array of n_jobs entries
 * (1 <= n_jobs <= 2^22; total nA and total nB each <= 2^31 - 1). The
 * arrays must stay valid and unchanged in size until c3x_batch_free; the
 * plan reads them again on every run. Each job's sources must lie within
 * 10 degrees of their mean direction. opts: precision (FP64 or MIXED);
 * cell_arcsec, tile and stream are not used (the plan picks cell sizes by
 * timing a few scales, C3X_BATCH_CELL_SCALE fixes one, and works on a
 * stream of its own). The plan runs the batch once (its result is ready)
 * and captures the pipeline into a hipGraph. Errors: EINVAL (bad job, bad
 * coordinate, a job too spread out), ERANGE (totals), ENOMEM, EDEVICE.
 * The batch owns its device memory until c3x_batch_free.
 *
 * c3x_batch_run: replays the graph after the work already queued on
 * `stream` (hipStream_t, NULL = null stream) and waits for it. Fails with
 * EINVAL when the inputs no longer fit the plan (a source outside its
 * job's planned sky box, or list sizes that changed): plan again.
 *
 * c3x_batch_result: a new result holding the last run's output; pairs in
 * (job, idxA, idxB) order with job-local row indices, best_idxB job-local
 * (-1: none). c3x_batch_offsets fills n_jobs + 1 host entries: job j's
 * pairs are [pair_off[j], pair_off[j + 1]); job j's best entries start at
 * the sum of nA over the jobs before it. */
c3x_status c3x_batch_plan(const c3x_job *jobs, int32_t n_jobs, const double *raA,
                          const double *decA, const double *raB, const double *decB,
                          c3x_frame frame, const c3x_opts *opts, c3x_batch **out);
c3x_status c3x_batch_run(c3x_batch *b, void *stream);
c3x_status c3x_batch_result(const c3x_batch *b, c3x_result **out);
c3x_status c3x_batch_offsets(const c3x_batch *b, int64_t *pair_off);
c3x_status c3x_batch_stats(const c3x_batch *b, c3x_stats *s);
void c3x_batch_free(c3x_batch *b);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *c3x_last_error(void);
const char *c3x_version(void);
int c3x_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* C3X_H */
