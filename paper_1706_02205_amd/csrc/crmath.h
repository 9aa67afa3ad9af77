// Correctly rounded exponential and the Matern closed forms for gfx950.
//
// The factorization must start from bit-identical covariance entries for its
// results to be reproducible entry by entry, so exp is evaluated to about 100
// bits in double-double arithmetic and rounded once:
//   x = k ln2 + r            Cody-Waite reduction, ln2 split into three parts
//   r' = r / 2^8             exact
//   expm1(r') = r' + r'^2 P(r'),  P the Taylor series to degree 10 (double-double)
//   expm1(2s) = 2 expm1(s) + expm1(s)^2, eight times
//   exp(x) = 2^k (1 + expm1(r))
// The double-double result (hi, lo) is normalised, so hi is the correctly
// rounded value unless the true value lies within the evaluation error of a
// rounding midpoint; such cases are reported through `hard` (probability about
// 2^-40 per call).  Results below the normal range are rounded onto the
// subnormal grid with integer arithmetic so they are correctly rounded too.
// The extra arithmetic (~300 FP64 operations per entry) is cheap next to the
// memory traffic of the factorization it feeds.
#pragma once

#include <hip/hip_runtime.h>

namespace kcdev {

struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ __forceinline__ dd quick_two_sum(double a, double b) {  // |a| >= |b|
    double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
    double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo = __builtin_fma(a.hi, b.lo, __builtin_fma(a.lo, b.hi, p.lo));
    return quick_two_sum(p.hi, p.lo);
}

// ln 2 = C1 + C2 + C3; C1 has 42 significant bits so k*C1 is exact for |k| < 2^11.
constexpr double kLn2C1 = 0x1.62e42fefa3800p-1;
constexpr double kLn2C2 = 0x1.ef35793c76730p-45;
constexpr double kLn2C3 = 0x1.f97b57a079a19p-103;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;

__device__ __forceinline__ dd expm1_small(dd r) {
    // 1/n! for n = 2..10 as double-double
    const dd c[9] = {{0x1.0000000000000p-1, 0.0},
                     {0x1.5555555555555p-3, 0x1.5555555555555p-57},
                     {0x1.5555555555555p-5, 0x1.5555555555555p-59},
                     {0x1.1111111111111p-7, 0x1.1111111111111p-63},
                     {0x1.6c16c16c16c17p-10, -0x1.f49f49f49f49fp-65},
                     {0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-73},
                     {0x1.a01a01a01a01ap-16, 0x1.a01a01a01a01ap-76},
                     {0x1.71de3a556c734p-19, -0x1.c154f8ddc6c00p-73},
                     {0x1.27e4fb7789f5cp-22, 0x1.cbbc05b4fa99ap-76}};
    dd p = c[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) p = dd_add(c[i], dd_mul(r, p));
    return dd_add(r, dd_mul(dd_mul(r, r), p));
}

// Correctly rounded exp(x).  hard |= 1 when the rounding could not be certified.
__device__ inline double cr_exp(double x, int& hard) {
    if (x != x) return x;
    if (x < -745.2) return 0.0;          // below half the smallest subnormal
    if (x > 709.79) return __builtin_inf();
    double kd = __builtin_rint(x * kInvLn2);
    int k = int(kd);
    double t1 = x - kd * kLn2C1;         // exact
    dd p2 = two_prod(kd, kLn2C2);
    dd r = two_sum(t1, -p2.hi);
    r.lo = (r.lo - p2.lo) - kd * kLn2C3;
    r = quick_two_sum(r.hi, r.lo);
    r.hi *= 0x1p-8;
    r.lo *= 0x1p-8;
    dd e = expm1_small(r);
#pragma unroll
    for (int i = 0; i < 8; ++i) {        // expm1(2s) = 2 expm1(s) + expm1(s)^2
        dd e2 = dd_mul(e, e);
        e = dd_add({2.0 * e.hi, 2.0 * e.lo}, e2);
    }
    dd v = dd_add({1.0, 0.0}, e);        // exp(r), normalised: |lo| <= ulp(hi)/2
    if (k >= -1021) {  // 2^k * [0.7, 1.42] is a normal number: the scaling is exact
        // hi is RN(v) unless |lo| is within the error bound of half an ulp
        long long bits = __double_as_longlong(v.hi);
        int ex = int((bits >> 52) & 0x7ff);
        double ulp = __longlong_as_double((long long)(ex - 52) << 52);
        bool pow2 = (bits & 0xfffffffffffffLL) == 0;
        double half = (v.lo < 0.0 && pow2) ? 0.25 * ulp : 0.5 * ulp;
        double tol = v.hi * 0x1p-92;
        if (half - __builtin_fabs(v.lo) <= tol) hard = 1;
        return __builtin_ldexp(v.hi, k);
    }
    // result below 2^-1021 * 1.42: round (hi + lo) * 2^(k+1074) to an integer number
    // of 2^-1074 (the spacing of subnormals and of normals below 2^-1021; z < 2^53)
    int s = k + 1074;
    double z = __builtin_ldexp(v.hi, s);
    double zl = __builtin_ldexp(v.lo, s);
    double nn = __builtin_rint(z);
    dd h = two_sum(z - nn, zl);
    if (h.hi > 0.5 || (h.hi == 0.5 && h.lo > 0.0)) nn += 1.0;
    else if (h.hi < -0.5 || (h.hi == -0.5 && h.lo < 0.0)) nn -= 1.0;
    else if (h.hi == 0.5 && h.lo == 0.0) nn = (__builtin_fmod(nn, 2.0) == 0.0) ? nn : nn + 1.0;
    else if (h.hi == -0.5 && h.lo == 0.0) nn = (__builtin_fmod(nn, 2.0) == 0.0) ? nn : nn - 1.0;
    if (__builtin_fabs(__builtin_fabs(h.hi) - 0.5) < 0x1p-40) hard = 1;
    return nn * 0x1p-1074;
}

// Euclidean distance, coordinates summed in ascending order without fusion
// (the library is compiled with -ffp-contract=off).
__device__ __forceinline__ double dist(const double* __restrict__ a, const double* __restrict__ b, int d) {
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double df = a[t] - b[t];
        s = s + df * df;
    }
    return __builtin_sqrt(s);
}

// Matern covariance with unit variance at nu = TWONU/2 (Section 4.4 closed forms).
template <int TWONU>
__device__ __forceinline__ double matern(double r, double ell, int& hard) {
    if constexpr (TWONU == 1) {
        double a = r / ell;
        return cr_exp(-a, hard);
    } else if constexpr (TWONU == 3) {
        double a = (0x1.bb67ae8584caap+0 * r) / ell;  // sqrt(3), correctly rounded
        return (1.0 + a) * cr_exp(-a, hard);
    } else {
        double a = (0x1.1e3779b97f4a8p+1 * r) / ell;  // sqrt(5), correctly rounded
        return ((1.0 + a) + (a * a) / 3.0) * cr_exp(-a, hard);
    }
}

// FP32 Matern for the mixed-precision factorization.
template <int TWONU>
__device__ __forceinline__ float matern_f32(float r, float ell) {
    if constexpr (TWONU == 1) {
        return expf(-(r / ell));
    } else if constexpr (TWONU == 3) {
        float a = (1.7320508f * r) / ell;
        return (1.0f + a) * expf(-a);
    } else {
        float a = (2.2360680f * r) / ell;
        return ((1.0f + a) + (a * a) * (1.0f / 3.0f)) * expf(-a);
    }
}

}  // namespace kcdev
