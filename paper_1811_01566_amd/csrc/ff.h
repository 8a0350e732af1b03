// Float-float ("double-FP32") arithmetic for the delay geometry.
//
// A value is an unevaluated sum hi + lo of two floats with |lo| <= ulp(hi)/2,
// carrying about 48 significand bits.  The error-free transformations are
// the classical ones: Knuth's TwoSum, Dekker's Fast-TwoSum, and the product
// error recovered with a fused multiply-add (Dekker 1971; Ogita, Rump and
// Oishi 2005).  The square root takes the hardware estimate and corrects it
// with one Newton step on the float-float residual.
//
// Every kernel source including this header is compiled with floating-point
// contraction off, so that the error terms below are evaluated as written;
// fused multiply-adds appear only where fmaf() is called explicitly.
#pragma once

#include <hip/hip_runtime.h>

struct ff {
    float hi, lo;
};

__device__ __forceinline__ ff ff_make(float hi, float lo) { return ff{hi, lo}; }

__device__ __forceinline__ ff two_sum(float a, float b) {
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return ff{s, e};
}

// requires |a| >= |b| (or a == 0)
__device__ __forceinline__ ff fast_two_sum(float a, float b) {
    float s = a + b;
    float e = b - (s - a);
    return ff{s, e};
}

__device__ __forceinline__ ff two_prod(float a, float b) {
    float p = a * b;
    float e = fmaf(a, b, -p);
    return ff{p, e};
}

__device__ __forceinline__ ff ff_add(ff a, ff b) {
    ff s = two_sum(a.hi, b.hi);
    float e = s.lo + (a.lo + b.lo);
    return fast_two_sum(s.hi, e);
}

__device__ __forceinline__ ff ff_add_f(ff a, float b) {
    ff s = two_sum(a.hi, b);
    float e = s.lo + a.lo;
    return fast_two_sum(s.hi, e);
}

__device__ __forceinline__ ff ff_mul(ff a, ff b) {
    ff p = two_prod(a.hi, b.hi);
    float e = fmaf(a.hi, b.lo, fmaf(a.lo, b.hi, p.lo));
    return fast_two_sum(p.hi, e);
}

__device__ __forceinline__ ff ff_mul_f(ff a, float b) {
    ff p = two_prod(a.hi, b);
    float e = fmaf(a.lo, b, p.lo);
    return fast_two_sum(p.hi, e);
}

__device__ __forceinline__ ff ff_sqr(ff a) {
    ff p = two_prod(a.hi, a.hi);
    float e = fmaf(2.0f * a.hi, a.lo, p.lo);
    return fast_two_sum(p.hi, e);
}

// sqrt of a non-negative float-float.
__device__ __forceinline__ ff ff_sqrt(ff a) {
    if (!(a.hi > 0.0f)) return ff{0.0f, 0.0f};
    float s = __builtin_amdgcn_sqrtf(a.hi);
    ff p = two_prod(s, s);
    float r = ((a.hi - p.hi) - p.lo) + a.lo;  // a - s^2
    float corr = r * (0.5f * __builtin_amdgcn_rcpf(s));
    return fast_two_sum(s, corr);
}

// (float)i * b for an integer i exactly representable in float.
__device__ __forceinline__ ff ff_scale_i(ff b, int i) { return ff_mul_f(b, (float)i); }
