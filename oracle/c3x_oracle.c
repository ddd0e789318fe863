/*
 * c3x_oracle.c -- plain CPU oracle for the positional ("Sky") cross-match.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. The GPU library does not
 * include, link or call anything here, and this file shares no code with it.
 *
 * What is computed (paper Section 2.1, "Sky" functional case, and Section 2.2,
 * match selection): for every source i of catalogue A a region is centred on
 * its position, a circle of fixed radius r or an ellipse with per-source
 * semi-axes a_i >= b_i and position angle PA_i (a circle is the ellipse with
 * a = b); source j of catalogue B matches i when its distance from the centre
 * is within the limits of the area. Inputs are IEEE doubles taken as exact
 * reals; theta_ij is the exact great-circle angle between the exact points.
 *
 *   circle : (i, j) in S  <=>  theta_ij <= r                      (inclusive)
 *   ellipse: (i, j) in S  <=>  (u/a_i)^2 + (v/b_i)^2 <= 1         (inclusive)
 *            where (u, v) = theta_ij * (cos(phi - T_i), sin(phi - T_i)),
 *            phi is the bearing of j seen from i, measured from local north
 *            (+Dec, or +b in the galactic frame) towards local east (+RA /
 *            +l), and T_i = pa_zero + pa_sense * PA_i is the orientation of
 *            the semi-major axis (the zero-point and the direction of
 *            rotation are the two extra PA parameters of Section 2.1).
 *            This is the azimuthal-equidistant reading: distances along the
 *            sphere, so a = b gives back theta <= a exactly.
 *   rectangle: (i, j) in S  <=>  |u| <= a_i and |v| <= b_i           (inclusive)
 *            with (u, v) as for the ellipse: a_i and b_i are the half-sides
 *            along and across the orientation T_i (Section 2.1 names the
 *            rectangular region beside the ellipse and the circle).
 *
 * How: each candidate is decided in FP64 with a proven error bound. The
 * computed quantity (the haversine of theta, or the ellipse form Q) carries a
 * relative error of at most ~45 u for the circle (u = 2^-53, derivation
 * below); the decision is taken only when the computed value is further than
 * E64 = 2^-40 (relative) from the threshold. Otherwise the pair is returned
 * as AMBIGUOUS and the caller re-decides it in extended precision (mpmath,
 * 60 digits; see exact.py). The pair set is therefore the exact one and does
 * not depend on the host's libm.
 *
 * Error budget, circle. hav = sin^2(dDec/2) + cos d1 cos d2 sin^2(dRA/2).
 *   dDec = fl(d2 - d1): 1 rounding. dRA: wrap-safe (360 - ra_hi is exact by
 *   Sterbenz when ra_hi > 180), 1 rounding. k = pi/360 factor: 2u. sin of a
 *   small argument (condition number <= 1), libm allowance 2 ulp: 7u, squared
 *   15u. cos d: sin(k (90 - |d|)) when |d| > 45 (90 - |d| exact), else
 *   cos(k d) (condition <= 0.79): 6u each. Product term 29u, sum of two
 *   non-negative terms 30u. Threshold sin^2(k r / 7200): 15u. Total 45u
 *   = 2^-47.5 against E64 = 2^-40: a 180x margin. Values that drive the
 *   terms subnormal are excluded by the input domain (r = 0 or r >= 1e-6").
 *
 * Error budget, ellipse. q.n = sin dDec + 2 sin d1 cos d2 sin^2(dRA/2) and
 *   q.e = cos d2 sin dRA (the tangent-plane components of B at A) each have
 *   absolute error <= ~30 u sin(theta) (every term is bounded by 2 sin
 *   theta, see below), T adds ~17u, so su, sv carry <= ~100 u sin(theta);
 *   Q then has relative error <= ~(300 + 200 a/b) u near Q = 1. The margin
 *   E_ell = 2^-38 (1 + a/b) keeps a ~64x safety factor. Rectangle: the two
 *   forms Qu = (theta/sin theta)^2 (su/a)^2 and Qv (the same with sv/b) are
 *   decided separately against 1; near Qu = 1, |su| ~ a and sin theta <=
 *   sqrt(a^2 + b^2) <= 1.42 a, near Qv = 1, |sv| ~ b and sin theta <= a + b,
 *   so each carries at most ~300 (1 + a/b) u relative and the same margin
 *   E_ell keeps a ~100x safety factor. (Bound on the second
 *   term of q.n: for |dRA| <= 90 deg, cos d2 sin^2(dRA/2) <= sin theta /
 *   sqrt 2; for |dRA| > 90 deg theta is the largest side of the triangle
 *   (pole, A, B), so cos d2 <= sin theta.)
 *
 * Enumeration. method 0 ("brute"): every (i, j). method 1 ("zones"): the sky
 * partitioning of Section 2.3 restated for the sphere: B is split into
 * declination zones of height h (>= the largest reach is not needed for
 * correctness, only for speed) and sorted by RA inside each zone; an A source
 * visits the zones within its reach in Dec and, in each, the RA interval
 * [ra - dRA, ra + dRA] with dRA = asin(sin R / cos dec) (the widest RA extent
 * of a cap of radius R), split at RA = 0/360; a cap that contains a pole, or
 * an interval of 180 deg or more, takes the whole zone. Catalogue A is split
 * into contiguous chunks, one per thread (Section 2.3: a subsample of the
 * first catalogue per concurrent process). Brute force and zones must return
 * identical results; the tests check it.
 *
 * Parity pins: closed forms (meridian, equator/RA wrap, through-the-pole,
 * ellipse axes at known PA), mpmath brute force on small catalogues, and the
 * invariants listed in the tests.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_OUT 0
#define O_IN 1
#define O_AMBIG 2

static const double KDEG = M_PI / 180.0;   /* degrees -> radians */
static const double KHALF = M_PI / 360.0;  /* half of it, for haversines */

typedef struct {
    double ra, dec, cosd, sind;
} opt;

typedef struct {
    int64_t n_in;
    int32_t *in_a, *in_b;
    double *in_sep;          /* FP64 separation of each in-pair, arcsec */
    int64_t n_amb;
    int32_t *amb_a, *amb_b;
    int64_t n_tests;         /* candidate pairs examined */
    int32_t threads_used;
} c3o_out;

typedef struct {
    int shape;               /* 0 circle, 1 ellipse, 2 rectangle */
    double radius_arcsec;
    const double *a_arcsec, *b_arcsec, *pa_deg;
    double pa_zero_deg;
    int pa_sense;
} c3o_area;

/* ------------------------------------------------------------------------ */
/* geometry                                                                 */
/* ------------------------------------------------------------------------ */

static double cos_dec(double d)
{
    double ad = fabs(d);
    if (ad > 45.0) return sin(KDEG * (90.0 - ad));
    return cos(KDEG * d);
}

static opt mkpt(double ra, double dec)
{
    opt p;
    p.ra = ra;
    p.dec = dec;
    p.cosd = cos_dec(dec);
    p.sind = sin(KDEG * dec);
    return p;
}

/* ra2 - ra1 reduced to (-180, 180] without losing relative accuracy. */
static double wrap_dra(double ra1, double ra2)
{
    double d = ra2 - ra1;
    if (d > 180.0) return -((360.0 - ra2) + ra1);
    if (d < -180.0) return (360.0 - ra1) + ra2;
    return d;
}

static double hav_of(const opt *p, const opt *q)
{
    double dd = q->dec - p->dec;
    double da = wrap_dra(p->ra, q->ra);
    double s1 = sin(KHALF * dd);
    double s2 = sin(KHALF * da);
    return s1 * s1 + (p->cosd * q->cosd) * (s2 * s2);
}

static int same_point(const opt *p, const opt *q)
{
    return p->dec == q->dec && (p->ra == q->ra || fabs(p->dec) == 90.0);
}

/* Tangent-plane components of q seen from p: north (tn) and east (te). */
static void tangent(const opt *p, const opt *q, double *tn, double *te)
{
    double dd = q->dec - p->dec;
    double da = wrap_dra(p->ra, q->ra);
    double s2 = sin(KHALF * da);
    *tn = sin(KDEG * dd) + 2.0 * p->sind * q->cosd * (s2 * s2);
    *te = q->cosd * sin(KDEG * da);
}

static double sep_rad(const opt *p, const opt *q)
{
    double tn, te;
    tangent(p, q, &tn, &te);
    double h = hav_of(p, q);
    double y = sqrt(tn * tn + te * te);
    double x = 1.0 - 2.0 * h;
    return atan2(y, x);
}

static const double E64 = 9.094947017729282e-13;  /* 2^-40 */
static const double E38 = 3.637978807091713e-12;  /* 2^-38 */

static int decide_circle(const opt *p, const opt *q, double h_r)
{
    if (h_r == 0.0) return same_point(p, q) ? O_IN : O_OUT;
    double h = hav_of(p, q);
    if (h <= h_r * (1.0 - E64)) return O_IN;
    if (h > h_r * (1.0 + E64)) return O_OUT;
    return O_AMBIG;
}

typedef struct {
    double h_a;       /* haversine of the semi-major axis */
    double ar, br;    /* semi-axes in radians */
    double ct, st;    /* cos, sin of the orientation T */
    double e;         /* decision margin */
} ell_par;

static ell_par mk_ell(double a_arcsec, double b_arcsec, double pa, double pa_zero, int sense)
{
    ell_par e;
    double s = sin(KHALF * (a_arcsec / 3600.0));
    e.h_a = s * s;
    e.ar = KDEG * (a_arcsec / 3600.0);
    e.br = KDEG * (b_arcsec / 3600.0);
    double T = pa_zero + (double)sense * pa;
    e.ct = cos(KDEG * T);
    e.st = sin(KDEG * T);
    e.e = E38 * (1.0 + a_arcsec / b_arcsec);
    return e;
}

static int decide_ellipse(const opt *p, const opt *q, const ell_par *e)
{
    double h = hav_of(p, q);
    if (h == 0.0) return O_IN;
    /* outside the circle of radius a: outside the ellipse */
    if (h > e->h_a * (1.0 + E64)) return O_OUT;
    double tn, te;
    tangent(p, q, &tn, &te);
    double th = 2.0 * asin(sqrt(h));
    double sth = 2.0 * sqrt(h) * sqrt(1.0 - h);
    double f = th / sth;
    double su = tn * e->ct + te * e->st;
    double sv = te * e->ct - tn * e->st;
    double x = su / e->ar, y = sv / e->br;
    double Q = (f * f) * (x * x + y * y);
    if (Q <= 1.0 - e->e) return O_IN;
    if (Q > 1.0 + e->e) return O_OUT;
    return O_AMBIG;
}

/* Rectangle of half-sides a (along T) and b (across): |u| <= a and
 * |v| <= b. ep->h_a is the haversine of the half-diagonal here. */
static ell_par mk_rect(double a_arcsec, double b_arcsec, double pa, double pa_zero, int sense)
{
    ell_par e = mk_ell(a_arcsec, b_arcsec, pa, pa_zero, sense);
    double d = sqrt(a_arcsec * a_arcsec + b_arcsec * b_arcsec) * (1.0 + 1e-15);
    double s = sin(KHALF * (d / 3600.0));
    e.h_a = s * s;
    return e;
}

static int decide_rect(const opt *p, const opt *q, const ell_par *e)
{
    double h = hav_of(p, q);
    if (h == 0.0) return O_IN;
    /* beyond the half-diagonal: outside the rectangle */
    if (h > e->h_a * (1.0 + E64)) return O_OUT;
    double tn, te;
    tangent(p, q, &tn, &te);
    double th = 2.0 * asin(sqrt(h));
    double sth = 2.0 * sqrt(h) * sqrt(1.0 - h);
    double f = th / sth;
    double su = tn * e->ct + te * e->st;
    double sv = te * e->ct - tn * e->st;
    double x = su / e->ar, y = sv / e->br;
    double Qu = (f * f) * (x * x), Qv = (f * f) * (y * y);
    if (Qu > 1.0 + e->e || Qv > 1.0 + e->e) return O_OUT;
    if (Qu <= 1.0 - e->e && Qv <= 1.0 - e->e) return O_IN;
    return O_AMBIG;
}

static int decide_area(const opt *p, const opt *q, int shape, const ell_par *e, double h_r)
{
    if (shape == 1) return decide_ellipse(p, q, e);
    if (shape == 2) return decide_rect(p, q, e);
    return decide_circle(p, q, h_r);
}

/* ------------------------------------------------------------------------ */
/* growable per-thread buffers                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t *a, *b;
    double *s;
    int64_t n, cap;
} vec3;

static int vpush(vec3 *v, int32_t a, int32_t b, double s)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 1024;
        int32_t *na = realloc(v->a, nc * sizeof(int32_t));
        if (!na) return -1;
        v->a = na;
        int32_t *nb = realloc(v->b, nc * sizeof(int32_t));
        if (!nb) return -1;
        v->b = nb;
        double *ns = realloc(v->s, nc * sizeof(double));
        if (!ns) return -1;
        v->s = ns;
        v->cap = nc;
    }
    v->a[v->n] = a;
    v->b[v->n] = b;
    v->s[v->n] = s;
    v->n++;
    return 0;
}

static void vfree(vec3 *v)
{
    free(v->a);
    free(v->b);
    free(v->s);
    memset(v, 0, sizeof(*v));
}

/* ------------------------------------------------------------------------ */
/* zone index over B                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    double h;
    int nz;
    int64_t *zoff;     /* nz + 1 */
    int64_t *order;    /* B rows sorted by (zone, ra, row) */
    double *zra;       /* ra of order[] */
} zindex;

static int zone_of(double dec, double h, int nz)
{
    double t = floor((dec + 90.0) / h);
    if (t < 0.0) return 0;
    if (t >= (double)nz) return nz - 1;
    return (int)t;
}

typedef struct {
    double ra;
    int64_t row;
} rarow;

static int cmp_rarow(const void *x, const void *y)
{
    const rarow *a = x, *b = y;
    if (a->ra < b->ra) return -1;
    if (a->ra > b->ra) return 1;
    return (a->row > b->row) - (a->row < b->row);
}

static int build_zones(const opt *B, int64_t nB, double h, zindex *z)
{
    memset(z, 0, sizeof(*z));
    z->h = h;
    double nzf = ceil(180.0 / h);
    if (nzf < 1.0) nzf = 1.0;
    if (nzf > 50000000.0) return -1;
    z->nz = (int)nzf;
    z->zoff = calloc((size_t)z->nz + 1, sizeof(int64_t));
    z->order = malloc((size_t)(nB > 0 ? nB : 1) * sizeof(int64_t));
    z->zra = malloc((size_t)(nB > 0 ? nB : 1) * sizeof(double));
    int *zz = malloc((size_t)(nB > 0 ? nB : 1) * sizeof(int));
    rarow *tmp = malloc((size_t)(nB > 0 ? nB : 1) * sizeof(rarow));
    if (!z->zoff || !z->order || !z->zra || !zz || !tmp) {
        free(zz);
        free(tmp);
        return -1;
    }
    for (int64_t j = 0; j < nB; j++) {
        zz[j] = zone_of(B[j].dec, h, z->nz);
        z->zoff[zz[j] + 1]++;
    }
    for (int k = 0; k < z->nz; k++) z->zoff[k + 1] += z->zoff[k];
    int64_t *fill = malloc((size_t)z->nz * sizeof(int64_t));
    if (!fill) {
        free(zz);
        free(tmp);
        return -1;
    }
    memcpy(fill, z->zoff, (size_t)z->nz * sizeof(int64_t));
    for (int64_t j = 0; j < nB; j++) {
        int64_t pos = fill[zz[j]]++;
        tmp[pos].ra = B[j].ra;
        tmp[pos].row = j;
    }
    for (int k = 0; k < z->nz; k++) {
        int64_t lo = z->zoff[k], hi = z->zoff[k + 1];
        if (hi - lo > 1) qsort(tmp + lo, (size_t)(hi - lo), sizeof(rarow), cmp_rarow);
    }
    for (int64_t j = 0; j < nB; j++) {
        z->order[j] = tmp[j].row;
        z->zra[j] = tmp[j].ra;
    }
    free(fill);
    free(zz);
    free(tmp);
    return 0;
}

static void free_zones(zindex *z)
{
    free(z->zoff);
    free(z->order);
    free(z->zra);
    memset(z, 0, sizeof(*z));
}

static int64_t lower_ra(const double *ra, int64_t lo, int64_t hi, double x)
{
    while (lo < hi) {
        int64_t m = lo + (hi - lo) / 2;
        if (ra[m] < x) lo = m + 1;
        else hi = m;
    }
    return lo;
}

static int64_t upper_ra(const double *ra, int64_t lo, int64_t hi, double x)
{
    while (lo < hi) {
        int64_t m = lo + (hi - lo) / 2;
        if (ra[m] <= x) lo = m + 1;
        else hi = m;
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* the join                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    const opt *A, *B;
    int64_t nB;
    const c3o_area *area;
    const zindex *zi;
    int method;
    int64_t a0, a1;
    vec3 in, amb;
    int64_t tests;
    int err;
} job;

typedef struct {
    int32_t j;
    int kind;
    double sep;
} hit;

static int cmp_hit(const void *x, const void *y)
{
    const hit *a = x, *b = y;
    return (a->j > b->j) - (a->j < b->j);
}

static double reach_deg(const c3o_area *ar, int64_t i)
{
    if (ar->shape == 1) return ar->a_arcsec[i] / 3600.0;
    if (ar->shape == 2) {
        double a = ar->a_arcsec[i], b = ar->b_arcsec[i];
        return sqrt(a * a + b * b) * (1.0 + 1e-15) / 3600.0;  /* the half-diagonal */
    }
    return ar->radius_arcsec / 3600.0;
}

static void *run_chunk(void *arg)
{
    job *jb = arg;
    const c3o_area *ar = jb->area;
    double h_r = 0.0;
    if (ar->shape == 0) {
        double s = sin(KHALF * (ar->radius_arcsec / 3600.0));
        h_r = s * s;
    }
    hit *hits = NULL;
    int64_t hcap = 0;
    for (int64_t i = jb->a0; i < jb->a1 && !jb->err; i++) {
        const opt *p = &jb->A[i];
        ell_par ep;
        memset(&ep, 0, sizeof(ep));
        if (ar->shape == 1)
            ep = mk_ell(ar->a_arcsec[i], ar->b_arcsec[i], ar->pa_deg[i], ar->pa_zero_deg, ar->pa_sense);
        else if (ar->shape == 2)
            ep = mk_rect(ar->a_arcsec[i], ar->b_arcsec[i], ar->pa_deg[i], ar->pa_zero_deg, ar->pa_sense);
        int64_t nh = 0;
#define CONSIDER(J)                                                              \
    do {                                                                         \
        int64_t jj_ = (J);                                                       \
        const opt *q_ = &jb->B[jj_];                                             \
        int k_ = decide_area(p, q_, ar->shape, &ep, h_r);                       \
        jb->tests++;                                                             \
        if (k_ != O_OUT) {                                                       \
            if (nh == hcap) {                                                    \
                int64_t nc_ = hcap ? 2 * hcap : 256;                             \
                hit *nh_ = realloc(hits, (size_t)nc_ * sizeof(hit));             \
                if (!nh_) { jb->err = 1; break; }                                \
                hits = nh_;                                                      \
                hcap = nc_;                                                      \
            }                                                                    \
            hits[nh].j = (int32_t)jj_;                                           \
            hits[nh].kind = k_;                                                  \
            hits[nh].sep = sep_rad(p, q_) / KDEG * 3600.0;                       \
            nh++;                                                                \
        }                                                                        \
    } while (0)

        if (jb->method == 0) {
            for (int64_t j = 0; j < jb->nB; j++) CONSIDER(j);
        } else {
            const zindex *z = jb->zi;
            double R = reach_deg(ar, i);
            double Rp = R * (1.0 + 1e-9) + 1e-12;
            int zlo = zone_of(p->dec - Rp, z->h, z->nz);
            int zhi = zone_of(p->dec + Rp, z->h, z->nz);
            int full = 0;
            double dra = 0.0;
            if (fabs(p->dec) + Rp >= 90.0) {
                full = 1;
            } else {
                double x = sin(KDEG * Rp) / cos_dec(p->dec);
                if (x >= 0.9999) full = 1;
                else {
                    dra = asin(x) / KDEG * (1.0 + 1e-9) + 1e-12;
                    if (dra >= 180.0) full = 1;
                }
            }
            for (int zk = zlo; zk <= zhi && !jb->err; zk++) {
                int64_t lo = z->zoff[zk], hi = z->zoff[zk + 1];
                if (lo == hi) continue;
                int64_t r0[2], r1[2];
                int nr = 0;
                if (full) {
                    r0[0] = lo;
                    r1[0] = hi;
                    nr = 1;
                } else {
                    double a_lo = p->ra - dra, a_hi = p->ra + dra;
                    if (a_lo < 0.0) {
                        r0[nr] = lower_ra(z->zra, lo, hi, a_lo + 360.0);
                        r1[nr] = hi;
                        nr++;
                        r0[nr] = lo;
                        r1[nr] = upper_ra(z->zra, lo, hi, a_hi);
                        nr++;
                    } else if (a_hi >= 360.0) {
                        r0[nr] = lower_ra(z->zra, lo, hi, a_lo);
                        r1[nr] = hi;
                        nr++;
                        r0[nr] = lo;
                        r1[nr] = upper_ra(z->zra, lo, hi, a_hi - 360.0);
                        nr++;
                    } else {
                        r0[nr] = lower_ra(z->zra, lo, hi, a_lo);
                        r1[nr] = upper_ra(z->zra, lo, hi, a_hi);
                        nr++;
                    }
                }
                for (int k = 0; k < nr && !jb->err; k++)
                    for (int64_t t = r0[k]; t < r1[k]; t++) CONSIDER(z->order[t]);
            }
            if (nh > 1) qsort(hits, (size_t)nh, sizeof(hit), cmp_hit);
        }
#undef CONSIDER
        for (int64_t k = 0; k < nh && !jb->err; k++) {
            vec3 *v = hits[k].kind == O_IN ? &jb->in : &jb->amb;
            if (vpush(v, (int32_t)i, hits[k].j, hits[k].sep)) jb->err = 1;
        }
    }
    free(hits);
    return NULL;
}

static int64_t cat3(vec3 *parts, int np, int32_t **oa, int32_t **ob, double **os)
{
    int64_t tot = 0;
    for (int k = 0; k < np; k++) tot += parts[k].n;
    size_t m = (size_t)(tot > 0 ? tot : 1);
    *oa = malloc(m * sizeof(int32_t));
    *ob = malloc(m * sizeof(int32_t));
    if (os) *os = malloc(m * sizeof(double));
    if (!*oa || !*ob || (os && !*os)) return -1;
    int64_t o = 0;
    for (int k = 0; k < np; k++) {
        if (parts[k].n) {
            memcpy(*oa + o, parts[k].a, (size_t)parts[k].n * sizeof(int32_t));
            memcpy(*ob + o, parts[k].b, (size_t)parts[k].n * sizeof(int32_t));
            if (os) memcpy(*os + o, parts[k].s, (size_t)parts[k].n * sizeof(double));
        }
        o += parts[k].n;
    }
    return tot;
}

/* Returns 0 on success, -1 on allocation failure, -2 on a bad argument. */
int c3o_match(const double *raA, const double *decA, int64_t nA,
              const double *raB, const double *decB, int64_t nB,
              const c3o_area *area, int method, double zone_deg, int nthreads,
              c3o_out *out)
{
    memset(out, 0, sizeof(*out));
    if (nA < 0 || nB < 0 || nA > 2147483647LL || nB > 2147483647LL) return -2;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nA < nthreads) nthreads = nA > 0 ? (int)nA : 1;
    opt *A = malloc((size_t)(nA > 0 ? nA : 1) * sizeof(opt));
    opt *B = malloc((size_t)(nB > 0 ? nB : 1) * sizeof(opt));
    if (!A || !B) {
        free(A);
        free(B);
        return -1;
    }
    for (int64_t i = 0; i < nA; i++) A[i] = mkpt(raA[i], decA[i]);
    for (int64_t j = 0; j < nB; j++) B[j] = mkpt(raB[j], decB[j]);
    zindex zi;
    memset(&zi, 0, sizeof(zi));
    if (method == 1) {
        if (!(zone_deg > 0.0)) {
            free(A);
            free(B);
            return -2;
        }
        if (build_zones(B, nB, zone_deg, &zi)) {
            free_zones(&zi);
            free(A);
            free(B);
            return -1;
        }
    }
    job *jobs = calloc((size_t)nthreads, sizeof(job));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    int rc = 0;
    if (!jobs || !th) rc = -1;
    char *created = calloc((size_t)nthreads, 1);
    if (!created) rc = -1;
    for (int t = 0; t < nthreads && !rc; t++) {
        jobs[t].A = A;
        jobs[t].B = B;
        jobs[t].nB = nB;
        jobs[t].area = area;
        jobs[t].zi = &zi;
        jobs[t].method = method;
        jobs[t].a0 = nA * t / nthreads;
        jobs[t].a1 = nA * (t + 1) / nthreads;
        if (nthreads > 1 && pthread_create(&th[t], NULL, run_chunk, &jobs[t]) == 0)
            created[t] = 1;
        else
            run_chunk(&jobs[t]);
    }
    for (int t = 0; t < nthreads && created; t++)
        if (created[t]) pthread_join(th[t], NULL);
    free(created);
    if (!rc) {
        vec3 *ins = malloc((size_t)nthreads * sizeof(vec3));
        vec3 *ams = malloc((size_t)nthreads * sizeof(vec3));
        if (!ins || !ams) rc = -1;
        for (int t = 0; t < nthreads && !rc; t++) {
            if (jobs[t].err) rc = -1;
            ins[t] = jobs[t].in;
            ams[t] = jobs[t].amb;
            out->n_tests += jobs[t].tests;
        }
        if (!rc) {
            out->n_in = cat3(ins, nthreads, &out->in_a, &out->in_b, &out->in_sep);
            out->n_amb = cat3(ams, nthreads, &out->amb_a, &out->amb_b, NULL);
            if (out->n_in < 0 || out->n_amb < 0) rc = -1;
        }
        free(ins);
        free(ams);
    }
    for (int t = 0; jobs && t < nthreads; t++) {
        vfree(&jobs[t].in);
        vfree(&jobs[t].amb);
    }
    out->threads_used = nthreads;
    free(jobs);
    free(th);
    free_zones(&zi);
    free(A);
    free(B);
    return rc;
}

void c3o_free(c3o_out *out)
{
    free(out->in_a);
    free(out->in_b);
    free(out->in_sep);
    free(out->amb_a);
    free(out->amb_b);
    memset(out, 0, sizeof(*out));
}

/* Single-pair decision, for tests: 0 out, 1 in, 2 ambiguous. */
int c3o_decide(double ra1, double dec1, double ra2, double dec2, const c3o_area *area, int64_t i)
{
    opt p = mkpt(ra1, dec1), q = mkpt(ra2, dec2);
    if (area->shape == 1) {
        ell_par e = mk_ell(area->a_arcsec[i], area->b_arcsec[i], area->pa_deg[i],
                           area->pa_zero_deg, area->pa_sense);
        return decide_ellipse(&p, &q, &e);
    }
    if (area->shape == 2) {
        ell_par e = mk_rect(area->a_arcsec[i], area->b_arcsec[i], area->pa_deg[i],
                            area->pa_zero_deg, area->pa_sense);
        return decide_rect(&p, &q, &e);
    }
    double s = sin(KHALF * (area->radius_arcsec / 3600.0));
    return decide_circle(&p, &q, s * s);
}

/* FP64 separation in arcsec for a list of pairs. */
void c3o_seps(const double *raA, const double *decA, const double *raB, const double *decB,
              const int32_t *ia, const int32_t *ib, int64_t n, double *out)
{
    for (int64_t k = 0; k < n; k++) {
        opt p = mkpt(raA[ia[k]], decA[ia[k]]);
        opt q = mkpt(raB[ib[k]], decB[ib[k]]);
        out[k] = sep_rad(&p, &q) / KDEG * 3600.0;
    }
}

int c3o_abi_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* frame conversion rule (catalogues in different frames)                   */
/* ------------------------------------------------------------------------ */
/*
 * Reading taken for mixed frames (Section 2: equatorial and galactic
 * coordinates): catalogue A's positions (and area orientations) are first
 * converted into catalogue B's frame by the fixed FP64 rule below, and the
 * converted doubles are A's inputs of the cross-match in B's frame. The rule
 * uses only correctly rounded +, -, *, /, exact floor, frexp and ldexp, in a
 * fixed order (no fused operations, no library trigonometry), so any IEEE
 * FP64 machine evaluating it gets the same bits. M is the rotation between
 * the frames, each entry the double nearest the exact value fixed by the
 * galactic pole (RA 192.85948 deg, Dec 27.12825 deg) and the galactic
 * longitude of the north celestial pole (122.93192 deg), taken as exact
 * decimals; it is passed in by the caller.
 *
 * sin, cos: x in degrees = r + 90 q with q = floor((x + 45) / 90); t = r pi/180
 *   (|t| <= pi/4 + tiny); Taylor series to t^17 (sin) and t^18 (cos), Horner
 *   in t^2; quadrant by q mod 4.
 * atan2: t = min(|x|,|y|) / max(|x|,|y|); above tan(pi/12), t' = (t sqrt3 - 1) /
 *   (t + sqrt3) and pi/6 added; Taylor series of atan to t'^29; quadrant by
 *   the signs and the swap; degrees.
 * sqrt: frexp to [0.5, 2) with an even exponent, a linear first guess, five
 *   Newton steps, ldexp.
 */

static const double R_KDEG = 0.017453292519943295;  /* pi / 180 */
static const double R_KRAD = 57.29577951308232;     /* 180 / pi */
static const double R_PI = 3.141592653589793;
static const double R_HALF_PI = 1.5707963267948966;
static const double R_PI_6 = 0.5235987755982988;
static const double R_SQRT3 = 1.7320508075688772;
static const double R_TAN_PI_12 = 0.2679491924311227;

static double r_sqrt(double x)
{
    if (!(x > 0.0)) return 0.0;
    int e;
    double m = frexp(x, &e);          /* x = m 2^e, m in [0.5, 1) */
    if (e & 1) {
        m = m * 2.0;
        e = e - 1;
    }
    double y = 0.41731 + 0.59016 * m;
    for (int k = 0; k < 5; k++) y = 0.5 * (y + m / y);
    return ldexp(y, e / 2);
}

static void r_sincos_deg(double x, double *s_out, double *c_out)
{
    double qf = floor((x + 45.0) / 90.0);
    double r = x - 90.0 * qf;
    double t = r * R_KDEG;
    double z = t * t;
    /* sin t = t (1 - z/3! + z^2/5! - ... + z^8/17!), Horner from the top */
    double s = 1.0 / 355687428096000.0;
    s = -1.0 / 1307674368000.0 + z * s;
    s = 1.0 / 6227020800.0 + z * s;
    s = -1.0 / 39916800.0 + z * s;
    s = 1.0 / 362880.0 + z * s;
    s = -1.0 / 5040.0 + z * s;
    s = 1.0 / 120.0 + z * s;
    s = -1.0 / 6.0 + z * s;
    s = 1.0 + z * s;
    s = t * s;
    /* cos t = 1 - z/2! + z^2/4! - ... - z^9/18! */
    double c = -1.0 / 6402373705728000.0;
    c = 1.0 / 20922789888000.0 + z * c;
    c = -1.0 / 87178291200.0 + z * c;
    c = 1.0 / 479001600.0 + z * c;
    c = -1.0 / 3628800.0 + z * c;
    c = 1.0 / 40320.0 + z * c;
    c = -1.0 / 720.0 + z * c;
    c = 1.0 / 24.0 + z * c;
    c = -0.5 + z * c;
    c = 1.0 + z * c;
    long q = (long)qf;
    int k = (int)(((q % 4) + 4) % 4);
    if (k == 0) { *s_out = s; *c_out = c; }
    else if (k == 1) { *s_out = c; *c_out = -s; }
    else if (k == 2) { *s_out = -s; *c_out = -c; }
    else { *s_out = -c; *c_out = s; }
}

static double r_atan2_deg(double y, double x)
{
    double ax = fabs(x), ay = fabs(y);
    if (ax == 0.0 && ay == 0.0) return 0.0;
    int swap = ay > ax;
    double t = swap ? ax / ay : ay / ax;
    double off = 0.0;
    if (t > R_TAN_PI_12) {
        t = (t * R_SQRT3 - 1.0) / (t + R_SQRT3);
        off = R_PI_6;
    }
    double z = t * t;
    double p = 1.0 / 29.0;
    p = -1.0 / 27.0 + z * p;
    p = 1.0 / 25.0 + z * p;
    p = -1.0 / 23.0 + z * p;
    p = 1.0 / 21.0 + z * p;
    p = -1.0 / 19.0 + z * p;
    p = 1.0 / 17.0 + z * p;
    p = -1.0 / 15.0 + z * p;
    p = 1.0 / 13.0 + z * p;
    p = -1.0 / 11.0 + z * p;
    p = 1.0 / 9.0 + z * p;
    p = -1.0 / 7.0 + z * p;
    p = 1.0 / 5.0 + z * p;
    p = -1.0 / 3.0 + z * p;
    p = 1.0 + z * p;
    double a = off + t * p;
    if (swap) a = R_HALF_PI - a;
    if (x < 0.0) a = R_PI - a;
    if (y < 0.0) a = -a;
    return a * R_KRAD;
}

/* rows of M times v: ((m0 v0 + m1 v1) + m2 v2) */
static void r_rot(const double *M, const double *v, double *o)
{
    o[0] = (M[0] * v[0] + M[1] * v[1]) + M[2] * v[2];
    o[1] = (M[3] * v[0] + M[4] * v[1]) + M[5] * v[2];
    o[2] = (M[6] * v[0] + M[7] * v[1]) + M[8] * v[2];
}

/* Converts n positions (degrees) with the rule; gamma_out (may be NULL)
 * receives, per position, the angle (degrees) from the target frame's local
 * north to the source frame's local north, measured towards the target's
 * local east: an orientation T in the source frame is T + gamma in the
 * target frame. */
void c3o_frame_convert(const double *M, const double *ra, const double *dec, int64_t n,
                       double *ra_out, double *dec_out, double *gamma_out)
{
    for (int64_t i = 0; i < n; i++) {
        double sa, ca, sd, cd;
        r_sincos_deg(ra[i], &sa, &ca);
        r_sincos_deg(dec[i], &sd, &cd);
        double p[3] = {cd * ca, cd * sa, sd}, q[3];
        r_rot(M, p, q);
        double a2 = r_atan2_deg(q[1], q[0]);
        if (a2 < 0.0) a2 = a2 + 360.0;
        if (a2 >= 360.0) a2 = 0.0;
        double d2 = r_atan2_deg(q[2], r_sqrt(q[0] * q[0] + q[1] * q[1]));
        if (d2 > 90.0) d2 = 90.0;
        if (d2 < -90.0) d2 = -90.0;
        ra_out[i] = a2;
        dec_out[i] = d2;
        if (gamma_out) {
            double nA[3] = {-(sd * ca), -(sd * sa), cd}, nq[3];
            r_rot(M, nA, nq);
            double sa2, ca2, sd2, cd2;
            r_sincos_deg(a2, &sa2, &ca2);
            r_sincos_deg(d2, &sd2, &cd2);
            double ue = nq[0] * (-sa2) + nq[1] * ca2;
            double un = (nq[0] * (-(sd2 * ca2)) + nq[1] * (-(sd2 * sa2))) + nq[2] * cd2;
            gamma_out[i] = r_atan2_deg(ue, un);
        }
    }
}
