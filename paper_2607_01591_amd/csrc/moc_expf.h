// FP32 evaluation of 1 - exp(-tau) shared by the planar and the DGMOC sweeps.
#pragma once

#include <hip/hip_runtime.h>

namespace moc {

// FP32, MOC_EXP_POLY, evaluated from x = -tau log2(e) (folded into the per-polar
// constant, so one multiply forms x) as the larger of two lower bounds of 1 - 2^x:
//  * P4, the degree-4 Taylor polynomial of 1 - e^-tau: the Lagrange remainder
//    tau^5 e^-xi / 120 is positive, so P4 never exceeds the true value, and it is
//    accurate for small tau (relative error <= tau^4 / 120);
//  * 1 - 2^x from the hardware exponential, lowered by kExpBias (four units in the last
//    place of 1, more than that instruction's error), so it never exceeds the true value
//    either, with an absolute error below 3.1e-7.
// The maximum is within min(tau^5 / 120, 3.1e-7) of 1 - e^-tau: relative error <= 2.7e-6
// (worst near tau = 0.13, with the exponential one unit off), and 0 for tau = 0. Relative accuracy matters because the
// tally takes (psi - qhat) * F directly.
constexpr float kLn2 = 0.69314718055994531f;
constexpr float kPolyC1 = -kLn2;
constexpr float kPolyC2 = -kLn2 * kLn2 / 2.0f;
constexpr float kPolyC3 = -kLn2 * kLn2 * kLn2 / 6.0f;
constexpr float kPolyC4 = -kLn2 * kLn2 * kLn2 * kLn2 / 24.0f;
constexpr float kExpBias = 2.384185791015625e-7f;   // 4 * 2^-24
__device__ __forceinline__ float one_minus_exp2_poly(float x) {
    const float small = x * (kPolyC1 + x * (kPolyC2 + x * (kPolyC3 + x * kPolyC4)));
    const float big = (1.0f - kExpBias) - __builtin_amdgcn_exp2f(x);
    return fmaxf(small, big);
}

}  // namespace moc
