// Phase rotations exp(j th) without a general-argument sine: quadrant
// reduction, then Taylor polynomials on [-pi/4, pi/4].
#pragma once
#include <hip/hip_runtime.h>

namespace dbp {

// sin and cos of r for |r| <= pi/4 from their Taylor series (terms to r^11 and
// r^10; the first omitted terms are below 1.2e-10 there), Horner in FP32.
__device__ __forceinline__ void sincos_reduced(float r, float& s, float& c) {
    const float r2 = r * r;
    float ps = fmaf(r2, -2.50521084e-8f, 2.75573192e-6f);     // -1/11!, 1/9!
    ps = fmaf(r2, ps, -1.98412698e-4f);                          // -1/7!
    ps = fmaf(r2, ps, 8.33333333e-3f);                           // 1/5!
    ps = fmaf(r2, ps, -1.66666667e-1f);                          // -1/3!
    s = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, -2.75573192e-7f, 2.48015873e-5f);     // -1/10!, 1/8!
    pc = fmaf(r2, pc, -1.38888889e-3f);                          // -1/6!
    pc = fmaf(r2, pc, 4.16666667e-2f);                           // 1/4!
    pc = fmaf(r2, pc, -0.5f);                                    // -1/2!
    c = fmaf(r2, pc, 1.0f);
}

// (cos th, sin th) from th = q pi/2 + r, |r| <= pi/4: a quarter-turn rotation of
// (cos r, sin r) selected by q mod 4.
__device__ __forceinline__ float2 rotate_quadrant(int q, float s, float c) {
    const float cs = (q & 1) ? -s : c, sn = (q & 1) ? c : s;
    return (q & 2) ? make_float2(-cs, -sn) : make_float2(cs, sn);
}

// (cos th, sin th) for an FP32 argument, reduced with pi/2 split in two FP32
// parts (Cody-Waite): exact to well below an FP32 ulp of the reduced argument
// for |th| < 1e3 rad.
__device__ __forceinline__ float2 expj(float th) {
    const float k = rintf(th * 0.636619772f);
    float r = fmaf(-k, 1.57079637e+0f, th);
    r = fmaf(-k, -4.37113883e-8f, r);
    float s, c;
    sincos_reduced(r, s, c);
    return rotate_quadrant((int)k, s, c);
}

}  // namespace dbp
