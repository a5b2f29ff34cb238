// hz_device.h -- device-side primitives shared by the real and complex
// kernels of the blocked implicit Hari-Zimmermann GSVD (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hz {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// One v_mfma_f64_16x16x4_f64: C(16x16) += A(16x4) * B(4x16).
// Lane layout (checked on gfx950): A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k, C[i][j] in lane j + 16*(i%4), element i/4 of the d4.
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Sum over aligned groups of W lanes by a xor butterfly.  IEEE addition is
// commutative, so every lane of a group ends with the bitwise same value and
// the association order is fixed: the result is reproducible run to run.
template <int W>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int m = 1; m < W; m <<= 1)
        v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }

// Scheduling fence between LDS traffic of lanes of one wave (LDS executes a
// wave's operations in order; this only stops the compiler from moving
// accesses across it).
__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double sign1(double b) { return copysign(1.0, b); }

// cos and sin of an angle in (-pi/2, pi/2] from its tangent; an infinite
// tangent gives cos = 0 and sin = sign of the tangent.
__device__ __forceinline__ void cs_from_tan(double tn, double &c, double &s)
{
    if (isinf(tn)) {
        c = 0.0;
        s = sign1(tn);
    } else {
        c = 1.0 / sqrt(fma(tn, tn, 1.0));
        s = tn * c;
    }
}

// Real 2x2 implicit Hari-Zimmermann transformation (paper, Section 2.1.2)
// for the pivot pair A' = [[aii, aij], [aij, ajj]], B' = [[1, x], [x, 1]]:
// returns Z' = (1/t)[[cos phi, sin phi], [-sin psi, cos psi]] as
// (z11, z21, z12, z22), z11/z22 being the scaled cosines used by criterion
// C1.  When A' and B' are proportional (cot 2theta = 0/0) the exceptional
// congruence of that section is returned, with the sign of x carried onto
// the off-diagonal entries so that it is a congruence to I for x < 0 too.
__device__ __forceinline__ void hz_real_2x2(double aii, double ajj, double aij, double x,
                                            double &z11, double &z21, double &z12, double &z22)
{
    const double t = sqrt(fma(-x, x, 1.0));
    const double h = ajj - aii;
    const double den = 2.0 * aij - (aii + ajj) * x;
    if (h == 0.0 && den == 0.0) {
        const double ax = fabs(x), s = (x < 0.0) ? -1.0 : 1.0;
        const double r2 = 0.70710678118654752440;
        const double p = r2 / sqrt(1.0 + ax), q = r2 / sqrt(1.0 - ax);
        z11 = p;
        z21 = s * p;
        z12 = -s * q;
        z22 = q;
        return;
    }
    const double sp = sqrt(1.0 + x), sm = sqrt(1.0 - x);
    const double xi = x / (sp + sm);
    const double eta = x / ((1.0 + sp) * (1.0 + sm));
    const double cot2 = (t * h) / den;
    const double tn = sign1(cot2) / (fabs(cot2) + sqrt(fma(cot2, cot2, 1.0)));
    double c, s;
    cs_from_tan(tn, c, s);
    const double cphi = c + xi * (s - eta * c);
    const double cpsi = c - xi * (s + eta * c);
    const double sphi = s - xi * (c + eta * s);
    const double spsi = s + xi * (c - eta * s);
    z11 = cphi / t;
    z21 = -spsi / t;
    z12 = sphi / t;
    z22 = cpsi / t;
}

}  // namespace hz
