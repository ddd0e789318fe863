// c3x_frames.hip -- catalogues in different frames (paper Section 2:
// equatorial and galactic coordinate systems).
//
// A catalogue given in the other frame is converted into the index's frame
// by a fixed FP64 rule, and the converted doubles are its inputs of the
// cross-match, which then runs in one frame. The rule uses only correctly
// rounded +, -, *, /, exact floor, frexp and ldexp in a fixed order (no
// fused operations: the library is compiled without contraction; no
// library trigonometry), so every IEEE FP64 machine that follows it gets
// the same bits. Its steps:
//   sin, cos of x degrees: x = r + 90 q, q = floor((x + 45) / 90);
//     t = r * (pi / 180); Taylor series to t^17 (sin) and t^18 (cos), Horner
//     in t^2 from the top term; the quadrant by q mod 4;
//   atan2 (degrees): t = min(|x|, |y|) / max(|x|, |y|); above tan(pi / 12)
//     t' = (t sqrt3 - 1) / (t + sqrt3) and pi / 6 added; Taylor series of
//     atan to t'^29; pi / 2 - a when |y| > |x|, pi - a when x < 0, -a when
//     y < 0; times 180 / pi;
//   sqrt: frexp to [0.5, 2) with an even exponent, first guess
//     0.41731 + 0.59016 m, five Newton steps y = 0.5 (y + m / y), ldexp;
//   position: p = (cos d cos a, cos d sin a, sin d); p' = M p row by row as
//     (m0 p0 + m1 p1) + m2 p2; a' = atan2(p'1, p'0), plus 360 if negative,
//     0 if it reaches 360; d' = atan2(p'2, sqrt(p'0^2 + p'1^2)) within
//     [-90, 90];
//   orientation turn gamma: the source frame's local north
//     (-sin d cos a, -sin d sin a, cos d) rotated by M, as a bearing from
//     the target frame's local north towards its local east at (a', d'):
//     atan2(n'.e, n'.n), e = (-sin a', cos a', 0), n = (-sin d' cos a',
//     -sin d' sin a', cos d'), dot products ((u0 v0 + u1 v1) + u2 v2).
// M (c3x_frame_matrix) is the rotation fixed by the galactic north pole and
// the north celestial pole's galactic longitude, rounded to doubles.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "c3x_host.h"

namespace c3x {

constexpr double kRDeg = 0.017453292519943295;  // pi / 180
constexpr double kRRad = 57.29577951308232;     // 180 / pi
constexpr double kRPi = 3.141592653589793;
constexpr double kRHalfPi = 1.5707963267948966;
constexpr double kRPi6 = 0.5235987755982988;
constexpr double kRSqrt3 = 1.7320508075688772;
constexpr double kRTanPi12 = 0.2679491924311227;

struct Rot {
    double m[9];
};

__device__ double rule_sqrt(double x)
{
    if (!(x > 0.0)) return 0.0;
    int e;
    double m = frexp(x, &e);
    if (e & 1) {
        m = m * 2.0;
        e = e - 1;
    }
    double y = 0.41731 + 0.59016 * m;
    for (int k = 0; k < 5; ++k) y = 0.5 * (y + m / y);
    return ldexp(y, e / 2);
}

__device__ void rule_sincos_deg(double x, double &s_out, double &c_out)
{
    const double qf = floor((x + 45.0) / 90.0);
    const double r = x - 90.0 * qf;
    const double t = r * kRDeg;
    const double z = t * t;
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
    const long q = (long)qf;
    const int k = (int)(((q % 4) + 4) % 4);
    if (k == 0) {
        s_out = s;
        c_out = c;
    } else if (k == 1) {
        s_out = c;
        c_out = -s;
    } else if (k == 2) {
        s_out = -s;
        c_out = -c;
    } else {
        s_out = -c;
        c_out = s;
    }
}

__device__ double rule_atan2_deg(double y, double x)
{
    const double ax = fabs(x), ay = fabs(y);
    if (ax == 0.0 && ay == 0.0) return 0.0;
    const bool swap = ay > ax;
    double t = swap ? ax / ay : ay / ax;
    double off = 0.0;
    if (t > kRTanPi12) {
        t = (t * kRSqrt3 - 1.0) / (t + kRSqrt3);
        off = kRPi6;
    }
    const double z = t * t;
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
    if (swap) a = kRHalfPi - a;
    if (x < 0.0) a = kRPi - a;
    if (y < 0.0) a = -a;
    return a * kRRad;
}

__device__ __forceinline__ void rule_rot(const Rot &M, const double v[3], double o[3])
{
    o[0] = (M.m[0] * v[0] + M.m[1] * v[1]) + M.m[2] * v[2];
    o[1] = (M.m[3] * v[0] + M.m[4] * v[1]) + M.m[5] * v[2];
    o[2] = (M.m[6] * v[0] + M.m[7] * v[1]) + M.m[8] * v[2];
}

// One thread per row: the converted position, and (when orient is given)
// the area orientation T = pa_zero + sense * pa turned by gamma. Rows
// outside the input domain are reported (the first one) and converted as
// (0, 0).
__global__ void k_frame_convert(Rot M, const double *__restrict__ ra,
                                const double *__restrict__ dec, int64_t n,
                                double *__restrict__ ra_out, double *__restrict__ dec_out,
                                double *__restrict__ gamma_out, const double *__restrict__ pa,
                                double pa_zero, int pa_sense, double *__restrict__ orient,
                                uint32_t *__restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = ra[i], d = dec[i];
    if (!(isfinite(a) && isfinite(d) && a >= 0.0 && a < 360.0 && fabs(d) <= 90.0)) {
        if (bad) atomicMin(bad, (uint32_t)i);
        a = 0.0;
        d = 0.0;
    }
    double sa, ca, sd, cd;
    rule_sincos_deg(a, sa, ca);
    rule_sincos_deg(d, sd, cd);
    const double p[3] = {cd * ca, cd * sa, sd};
    double q[3];
    rule_rot(M, p, q);
    double a2 = rule_atan2_deg(q[1], q[0]);
    if (a2 < 0.0) a2 = a2 + 360.0;
    if (a2 >= 360.0) a2 = 0.0;
    double d2 = rule_atan2_deg(q[2], rule_sqrt(q[0] * q[0] + q[1] * q[1]));
    if (d2 > 90.0) d2 = 90.0;
    if (d2 < -90.0) d2 = -90.0;
    ra_out[i] = a2;
    dec_out[i] = d2;
    if (gamma_out || orient) {
        const double nA[3] = {-(sd * ca), -(sd * sa), cd};
        double nq[3];
        rule_rot(M, nA, nq);
        double sa2, ca2, sd2, cd2;
        rule_sincos_deg(a2, sa2, ca2);
        rule_sincos_deg(d2, sd2, cd2);
        const double ue = nq[0] * (-sa2) + nq[1] * ca2;
        const double un = (nq[0] * (-(sd2 * ca2)) + nq[1] * (-(sd2 * sa2))) + nq[2] * cd2;
        const double g = rule_atan2_deg(ue, un);
        if (gamma_out) gamma_out[i] = g;
        if (orient) orient[i] = (pa_zero + (double)pa_sense * pa[i]) + g;
    }
}

static inline unsigned fblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t frame_convert(int src, int dst, const double *ra, const double *dec, int64_t n,
                         double *ra_out, double *dec_out, double *gamma_out, const double *pa,
                         double pa_zero, int pa_sense, double *orient, uint32_t *bad,
                         hipStream_t s)
{
    Rot M;
    c3x_frame_matrix(src, dst, M.m);
    if (n > 0)
        hipLaunchKernelGGL(k_frame_convert, dim3(fblk(n)), dim3(256), 0, s, M, ra, dec, n, ra_out,
                           dec_out, gamma_out, pa, pa_zero, pa_sense, orient, bad);
    return hipGetLastError();
}

c3x_status convert_catalogue_a(int src, int dst, int64_t n, const double **ra, const double **dec,
                               c3x_area *area, Arena &conv, hipStream_t s)
{
    if (src == dst || n <= 0) return C3X_OK;
    const bool oriented = area->shape != C3X_CIRCLE;
    double *ra2 = conv.get_n<double>(n), *dec2 = conv.get_n<double>(n);
    double *t2 = oriented ? conv.get_n<double>(n) : nullptr;
    uint32_t *bad = conv.get_n<uint32_t>(1);
    if (!ra2 || !dec2 || (oriented && !t2) || !bad) return fail(C3X_ENOMEM, "frame conversion");
    uint32_t hbad = 0xffffffffu;
    hipError_t e = hipMemsetAsync(bad, 0xff, sizeof(uint32_t), s);
    if (e == hipSuccess)
        e = frame_convert(src, dst, *ra, *dec, n, ra2, dec2, nullptr,
                          oriented ? area->pa_deg : nullptr, area->pa_zero_deg, area->pa_sense, t2,
                          bad, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "frame conversion");
    if (hbad != 0xffffffffu)
        return fail(C3X_EINVAL, "catalogue A row %u: coordinate outside RA [0,360), |Dec| <= "
                                "90 or not finite", hbad);
    *ra = ra2;
    *dec = dec2;
    if (oriented) {
        area->pa_deg = t2;
        area->pa_zero_deg = 0.0;
        area->pa_sense = 1;
    }
    return C3X_OK;
}

}  // namespace c3x

extern "C" c3x_status c3x_frame_convert(const double *ra, const double *dec, int64_t n,
                                        c3x_frame src, c3x_frame dst, double *ra_out,
                                        double *dec_out, double *gamma_out, void *stream)
{
    using namespace c3x;
    clear_error();
    if (n < 0) return fail(C3X_EINVAL, "n < 0");
    if (n > 0 && (!ra || !dec || !ra_out || !dec_out)) return fail(C3X_EINVAL, "NULL array");
    if ((src != C3X_EQUATORIAL && src != C3X_GALACTIC) ||
        (dst != C3X_EQUATORIAL && dst != C3X_GALACTIC))
        return fail(C3X_EINVAL, "bad frame");
    hipStream_t s = (hipStream_t)stream;
    Arena tmp(s);
    uint32_t *bad = tmp.get_n<uint32_t>(1);
    if (!bad) return fail(C3X_ENOMEM, "frame conversion");
    hipError_t e = hipMemsetAsync(bad, 0xff, sizeof(uint32_t), s);
    if (e == hipSuccess)
        e = frame_convert((int)src, (int)dst, ra, dec, n, ra_out, dec_out, gamma_out, nullptr,
                          0.0, 1, nullptr, bad, s);
    uint32_t h = 0xffffffffu;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "c3x_frame_convert");
    if (h != 0xffffffffu)
        return fail(C3X_EINVAL, "row %u: coordinate outside RA [0,360), |Dec| <= 90 or not "
                                "finite", h);
    return C3X_OK;
}
