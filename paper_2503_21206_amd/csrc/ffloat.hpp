// Compensated (float-float) distance arithmetic for the device.
//
// The search compares single-precision distances (section 6.1).  A plain fp32 sum depends
// on the order of its terms, so two kernels, or a kernel and the host, that sum in
// different orders can disagree in the last bit, and a last-bit difference can flip a
// decision of Algorithm 1 when two candidates nearly tie.  Here a distance is carried as an
// unevaluated sum hi + lo of two floats: every product and every difference is split
// exactly (fma-based two-product, two-sum), the running sum keeps its rounding error in lo,
// and the final value is hi + lo rounded once.  The pair is accurate to about 2^-44 of
// the sum of |terms|, so the fp32 result is the correctly rounded exact distance except
// when the exact value lies within that margin of a midpoint between two floats, and it
// no longer depends on the order in which partial sums are combined.  No fp64 is used.
#pragma once

#include <hip/hip_runtime.h>

namespace pa {

struct ff32 {
    float hi, lo;
};

// s + e == a + b exactly (Knuth's two-sum; no ordering assumption on |a|, |b|).  e is the
// exact rounding error, so the pair does not depend on the order of a and b.
//
// Every function below turns off fp contraction: fusing a product into a following sum
// (d * d + acc into one fma) would break the exactness of the two-sum steps.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Accumulates one L2 term (q - x)^2 into acc.
__device__ __forceinline__ void ff_add_sqdiff(ff32& acc, float q, float x) {
#pragma clang fp contract(off)
    float d, dl;
    two_sum(q, -x, d, dl);                      // q - x == d + dl
    const float p = d * d;
    const float pe = __builtin_fmaf(d, d, -p);  // d*d == p + pe
    const float tail = __builtin_fmaf(2.0f * d, dl, pe);  // (d + dl)^2 - p, without dl^2
    float s, e;
    two_sum(acc.hi, p, s, e);
    acc.hi = s;
    acc.lo += e + tail;
}

// Accumulates one inner-product term q * x into acc.
__device__ __forceinline__ void ff_add_prod(ff32& acc, float q, float x) {
#pragma clang fp contract(off)
    const float p = q * x;
    const float pe = __builtin_fmaf(q, x, -p);
    float s, e;
    two_sum(acc.hi, p, s, e);
    acc.hi = s;
    acc.lo += e + pe;
}

// Renormalises a pair so that hi is hi + lo rounded to fp32.
__device__ __forceinline__ ff32 ff_norm(ff32 a) {
    ff32 r;
    two_sum(a.hi, a.lo, r.hi, r.lo);
    return r;
}

// a + b for two pairs, renormalised.  Symmetric in a and b, bit for bit: the two-sum error
// is exact and the low parts are combined with one commutative addition.
__device__ __forceinline__ ff32 ff_add(ff32 a, ff32 b) {
#pragma clang fp contract(off)
    float s, e;
    two_sum(a.hi, b.hi, s, e);
    const float lo = e + (a.lo + b.lo);
    ff32 r;
    two_sum(s, lo, r.hi, r.lo);
    return r;
}

}  // namespace pa
