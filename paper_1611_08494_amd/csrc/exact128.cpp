// exact128.cpp -- host binary128 decisions for the few cases the GPU's
// certified FP64 arithmetic leaves undecided.
//
// The predicates are those of the "Sky" case (paper Section 2.1): theta <= r
// for the circle, the azimuthal-equidistant ellipse form Q <= 1 for the
// ellipse (PA from north through east, T = pa_zero + pa_sense * PA), and the
// exact argmin of (theta, index) for the best match (Section 2.2).
// binary128 carries 113 bits; every value below is computed to a relative
// error of about 2^-106, so a difference from the threshold under 2^-96
// (relative) is taken as an exact tie, which the inclusive boundary puts
// inside and the best-match rule breaks by the lower index.
#include <math.h>
#include <quadmath.h>
#include <stdint.h>

typedef __float128 q128;

static const q128 kTie = 1.2621774483536188886587657044524579674771e-29Q;  // 2^-96

static inline q128 qdeg() { return M_PIq / 180; }

struct QPts {
    q128 d1, d2, dd, da;
};

static inline QPts pieces(double ra1, double dec1, double ra2, double dec2)
{
    QPts p;
    q128 k = qdeg();
    p.d1 = (q128)dec1 * k;
    p.d2 = (q128)dec2 * k;
    p.dd = ((q128)dec2 - (q128)dec1) * k;
    p.da = ((q128)ra2 - (q128)ra1) * k;
    return p;
}

static inline q128 qhav(const QPts &p)
{
    q128 s1 = sinq(p.dd / 2), s2 = sinq(p.da / 2);
    return s1 * s1 + cosq(p.d1) * cosq(p.d2) * s2 * s2;
}

static inline q128 qtheta(double ra1, double dec1, double ra2, double dec2)
{
    QPts p = pieces(ra1, dec1, ra2, dec2);
    q128 h = qhav(p);
    if (h < 0) h = 0;
    if (h > 1) h = 1;
    return 2 * asinq(sqrtq(h));
}

static inline bool same_point(double ra1, double dec1, double ra2, double dec2)
{
    return dec1 == dec2 && (ra1 == ra2 || dec1 == 90.0 || dec1 == -90.0);
}

extern "C" int c3x_q_circle(double ra1, double dec1, double ra2, double dec2, double r_arcsec)
{
    if (r_arcsec == 0.0) return same_point(ra1, dec1, ra2, dec2) ? 1 : 0;
    q128 th = qtheta(ra1, dec1, ra2, dec2);
    q128 R = (q128)r_arcsec / 3600 * qdeg();
    q128 d = th - R;
    if (fabsq(d) <= kTie * R) return 1;
    return d < 0 ? 1 : 0;
}

extern "C" int c3x_q_ellipse(double ra1, double dec1, double ra2, double dec2, double a_arcsec,
                             double b_arcsec, double pa_deg, double pa_zero_deg, int pa_sense)
{
    QPts p = pieces(ra1, dec1, ra2, dec2);
    q128 h = qhav(p);
    if (h <= 0) return 1;
    q128 th = 2 * asinq(sqrtq(h));
    q128 s2 = sinq(p.da / 2);
    q128 tn = sinq(p.dd) + 2 * sinq(p.d1) * cosq(p.d2) * s2 * s2;
    q128 te = cosq(p.d2) * sinq(p.da);
    q128 T = ((q128)pa_zero_deg + (q128)pa_sense * (q128)pa_deg) * qdeg();
    q128 ct = cosq(T), st = sinq(T);
    q128 su = tn * ct + te * st;
    q128 sv = te * ct - tn * st;
    q128 A = (q128)a_arcsec / 3600 * qdeg();
    q128 B = (q128)b_arcsec / 3600 * qdeg();
    q128 f = th / sinq(th);
    q128 x = su / A, y = sv / B;
    q128 Q = f * f * (x * x + y * y);
    q128 d = Q - 1;
    if (fabsq(d) <= kTie) return 1;
    return d < 0 ? 1 : 0;
}

// Rectangle of half-sides a (along T) and b (across): |u| <= a and |v| <= b,
// u, v the ellipse's axis coordinates; a side within kTie counts as on it.
extern "C" int c3x_q_rect(double ra1, double dec1, double ra2, double dec2, double a_arcsec,
                          double b_arcsec, double pa_deg, double pa_zero_deg, int pa_sense)
{
    QPts p = pieces(ra1, dec1, ra2, dec2);
    q128 h = qhav(p);
    if (h <= 0) return 1;
    q128 th = 2 * asinq(sqrtq(h));
    q128 s2 = sinq(p.da / 2);
    q128 tn = sinq(p.dd) + 2 * sinq(p.d1) * cosq(p.d2) * s2 * s2;
    q128 te = cosq(p.d2) * sinq(p.da);
    q128 T = ((q128)pa_zero_deg + (q128)pa_sense * (q128)pa_deg) * qdeg();
    q128 ct = cosq(T), st = sinq(T);
    q128 su = tn * ct + te * st;
    q128 sv = te * ct - tn * st;
    q128 A = (q128)a_arcsec / 3600 * qdeg();
    q128 B = (q128)b_arcsec / 3600 * qdeg();
    q128 f = th / sinq(th);
    q128 x = fabsq(f * su / A), y = fabsq(f * sv / B);
    if ((x > 1 && x - 1 > kTie) || (y > 1 && y - 1 > kTie)) return 0;
    return 1;
}

// Index (into the candidate list) of the exact argmin of (theta, idx).
// Haversine sin^2(theta/2) in FP64 with a relative error below 2^-45 (a few
// dozen roundings of 2^-53 and the host libm's sine/cosine, each within an
// ulp or two): RA difference taken across the 0/360 seam by an exact shift,
// cos(dec) as the sine of the exact co-latitude above |dec| = 45.
static double hav64(double ra1, double dec1, double ra2, double dec2)
{
    const double k = 0.017453292519943295;  // pi / 180
    if (ra2 - ra1 > 180.0) ra2 -= 360.0;
    else if (ra1 - ra2 > 180.0) ra1 -= 360.0;
    double sa = sin((ra2 - ra1) * k * 0.5);
    double sd = sin((dec2 - dec1) * k * 0.5);
    double c1 = fabs(dec1) > 45.0 ? sin((90.0 - fabs(dec1)) * k) : cos(dec1 * k);
    double c2 = fabs(dec2) > 45.0 ? sin((90.0 - fabs(dec2)) * k) : cos(dec2 * k);
    return sd * sd + c1 * c2 * (sa * sa);
}

// Index (into the candidate list) of the exact argmin of (theta, idx).
// An FP64 pass first drops every candidate whose haversine is above the
// smallest by more than 2^-36 (relative; far outside the FP64 error, so the
// exact order is certain); the survivors are ranked in binary128.
extern "C" int c3x_q_best(double ra1, double dec1, int n, const double *ra2, const double *dec2,
                          const int32_t *idx)
{
    const double kKeep = 1.0 + 0x1p-36, kTiny = 0x1p-900;
    double hmin = 0.0;
    if (n > 1) {
        hmin = hav64(ra1, dec1, ra2[0], dec2[0]);
        for (int k = 1; k < n; ++k) {
            double h = hav64(ra1, dec1, ra2[k], dec2[k]);
            if (h < hmin) hmin = h;
        }
    }
    double lim = hmin * kKeep > kTiny ? hmin * kKeep : kTiny;
    if (n > 1) {
        int keep = 0, last = -1;
        for (int k = 0; k < n; ++k)
            if (hav64(ra1, dec1, ra2[k], dec2[k]) <= lim) ++keep, last = k;
        if (keep == 1) return last;
    }
    int best = -1;
    q128 bt = 0;
    for (int k = 0; k < n; ++k) {
        if (n > 1 && !(hav64(ra1, dec1, ra2[k], dec2[k]) <= lim)) continue;
        q128 t = qtheta(ra1, dec1, ra2[k], dec2[k]);
        if (best < 0) {
            best = k;
            bt = t;
            continue;
        }
        q128 scale = bt > t ? bt : t;
        bool tie = fabsq(t - bt) <= kTie * scale;
        if (tie ? idx[k] < idx[best] : t < bt) {
            best = k;
            bt = tie ? (bt < t ? bt : t) : t;
        }
    }
    return best;
}

// sin^2(r/2) and the squared chord 4 sin^2(r/2), r in arcsec, each rounded
// to the nearest double.
extern "C" void c3x_q_thresholds(double r_arcsec, double *h_r, double *cr2)
{
    q128 s = sinq((q128)r_arcsec / 7200 * qdeg());
    *h_r = (double)(s * s);
    *cr2 = (double)(4 * s * s);
}

// Rotation between the equatorial and galactic frames (Section 2 names both
// coordinate systems), fixed by the galactic north pole (RA 192.85948 deg,
// Dec 27.12825 deg) and the galactic longitude of the north celestial pole
// (122.93192 deg) taken as exact decimals: the galactic basis vectors in
// equatorial coordinates, computed in binary128 and rounded to doubles.
// src == dst gives the identity; equatorial -> galactic has the basis
// vectors as rows, galactic -> equatorial is the transpose. Row-major.
extern "C" void c3x_frame_matrix(int src, int dst, double *M)
{
    for (int k = 0; k < 9; ++k) M[k] = (k % 4 == 0) ? 1.0 : 0.0;
    if (src == dst) return;
    const q128 k = qdeg();
    const q128 a = strtoflt128("192.85948", nullptr) * k;
    const q128 d = strtoflt128("27.12825", nullptr) * k;
    const q128 l = strtoflt128("122.93192", nullptr) * k;
    const q128 zg[3] = {cosq(d) * cosq(a), cosq(d) * sinq(a), sinq(d)};
    // the north celestial pole: galactic longitude l, latitude d
    q128 q[3];
    for (int i = 0; i < 3; ++i) q[i] = ((i == 2 ? (q128)1 : (q128)0) - sinq(d) * zg[i]) / cosq(d);
    const q128 qp[3] = {zg[1] * q[2] - zg[2] * q[1], zg[2] * q[0] - zg[0] * q[2],
                        zg[0] * q[1] - zg[1] * q[0]};
    q128 xg[3], yg[3];
    for (int i = 0; i < 3; ++i) {
        xg[i] = cosq(l) * q[i] - sinq(l) * qp[i];
        yg[i] = sinq(l) * q[i] + cosq(l) * qp[i];
    }
    const q128 *rows[3] = {xg, yg, zg};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            const double v = (double)rows[r][c];
            if (src == 0) M[3 * r + c] = v;  // equatorial -> galactic
            else M[3 * c + r] = v;           // galactic -> equatorial
        }
}
