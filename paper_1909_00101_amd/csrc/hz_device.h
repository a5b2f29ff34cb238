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

// DPP lane exchange of a double within a row of 16 lanes (two 32-bit moves).
// Every pattern used here reads a lane of the same row, so bound_ctrl (read
// 0 from an invalid source lane) never applies; it lets the move write a
// fresh register instead of one tied to, and first copied from, the source.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Sum over aligned groups of L = 2, 4, 8 or 16 lanes with DPP only (no LDS
// traffic): quad xor-1 and xor-2 permutations, then the 8-lane half mirror
// and the 16-lane mirror.  Each stage adds a lane's value to its partner's
// (commutative), so all lanes of a group hold the bitwise same sum.
template <int L>
__device__ __forceinline__ double dpp_group_sum(double v)
{
    static_assert(L == 2 || L == 4 || L == 8 || L == 16, "group of 2..16 lanes");
    v += dpp_d<0xB1>(v);                      // quad_perm [1,0,3,2]
    if (L >= 4) v += dpp_d<0x4E>(v);          // quad_perm [2,3,0,1]
    if (L >= 8) v += dpp_d<0x141>(v);         // row_half_mirror
    if (L >= 16) v += dpp_d<0x140>(v);        // row_mirror
    return v;
}

// Broadcast lane l's double to the wave (two v_readlane_b32; l uniform).
__device__ __forceinline__ double readlane_d(double v, int l)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Copy n int16 entries (the inner ordering table) from global memory to
// LDS with a workgroup of NT threads, four loads of a thread in flight
// before its stores.
template <int NT>
__device__ __forceinline__ void copy_table(int16_t *__restrict__ dst, const int16_t *__restrict__ src,
                                           int n)
{
    const int tid = threadIdx.x;
    for (int e0 = tid; e0 < n; e0 += 4 * NT) {
        int16_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = (e0 + k * NT < n) ? src[e0 + k * NT] : (int16_t)0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (e0 + k * NT < n) dst[e0 + k * NT] = v[k];
    }
}

// Reciprocal square root from the hardware estimate y0 = v_rsq_f64(x)
// (relative error e0 about 2^-22) refined by one third-order step
// y = y0 (1 + e/2 + 3e^2/8), e = 1 - x y0^2, which leaves O(e0^3) -- below
// double rounding -- with a dependency depth of four operations.  About one
// ulp for positive normal finite x; exactly 1 for x = 1.  Deterministic.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    const double p = fma(0.375, e, 0.5);
    return fma(y * e, p, y);
}

__device__ __forceinline__ double sqrt_nr(double x) { return x * rsqrt_nr(x); }

// a / b for finite b != 0: hardware reciprocal estimate r0 refined by one
// third-order step r = r0 (1 + e + e^2), e = 1 - b r0, then a * r with one
// residual correction.
__device__ __forceinline__ double div_nr(double a, double b)
{
    const double r0 = __builtin_amdgcn_rcp(b);
    const double e = fma(-b, r0, 1.0);
    const double r = fma(r0, fma(e, e, e), r0);
    const double q = a * r;
    return fma(r, fma(-b, q, a), q);
}

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

// The real 2x2 transformation of Section 2.1.2 arranged for a short
// dependency chain on gfx950 (used by the inner solver).  With
// N = t (a_jj - a_ii) and D = 2 a_ij - (a_ii + a_jj) x, cot 2theta = N / D,
// and the printed tan theta = sign(cot)/(|cot| + sqrt(1 + cot^2)) equals
// sign(N) D / q with q = |N| + sqrt(N^2 + D^2) for every (N, D) != (0, 0),
// including D = 0 (tan = 0) and N = 0 (tan = sign D), so no infinities
// arise.  Then cos theta = q / sqrt(q^2 + D^2) and sin theta = sign(N) D /
// sqrt(q^2 + D^2); when D^2 is below the rounding of q^2 the correctly
// rounded cosine is exactly 1 and is set so (criterion C1 depends on exact
// ones, as with the printed 1/sqrt(1 + tan^2)).  N^2 is formed as
// t^2 h^2 so that sqrt(N^2 + D^2) does not wait for t.  The cosines and
// sines of phi and psi follow as printed, scaled by 1/t.  The exception
// (N = D = 0, A' proportional to B') returns the signed form of
// hz_real_2x2.  Returns z11, z21, z12, z22 of Z' (column-major).
__device__ __forceinline__ void hz_real_2x2_fast(double aii, double ajj, double aij, double x,
                                                 double &z11, double &z21, double &z12,
                                                 double &z22, bool &c2small)
{
    const double t2 = fma(-x, x, 1.0);
    const double h = ajj - aii;
    const double D = fma(-(aii + ajj), x, 2.0 * aij);
    if (h == 0.0 && D == 0.0) {
        const double r2 = 0.70710678118654752440;
        const double ax = fabs(x), s = (x < 0.0) ? -1.0 : 1.0;
        const double p = r2 * rsqrt_nr(1.0 + ax), q = r2 * rsqrt_nr(1.0 - ax);
        z11 = p;
        z21 = s * p;
        z12 = -s * q;
        z22 = q;
        c2small = false;
        return;
    }
    const double rt = rsqrt_nr(t2);                       // 1/t
    const double D2 = D * D;
    const double hyp = sqrt_nr(fma(t2 * h, h, D2));       // sqrt(N^2 + D^2)
    const double q = fma(t2 * rt, fabs(h), hyp);          // |N| + hyp
    const double q2 = q * q;
    const double qd = q2 + D2;
    const double r = rsqrt_nr(qd);
    const double sD = (h < 0.0) ? -D : D;                 // sign(N) D
    const bool tiny = (qd == q2);
    const double c = tiny ? 1.0 : q * r;
    const double s = sD * r;
    // sqrt(1 + x) from one reciprocal square root and sqrt(1 - x) =
    // t/sqrt(1 + x) with t = t2 * (1/t), both to a few ulps.  xi is divided
    // out rather than taken as (sqrt(1+x) - sqrt(1-x))/2: for tiny x that
    // difference cancels, and xi enters the sines of tiny transformations
    // directly, so it needs relative accuracy.
    const double rp = rsqrt_nr(1.0 + x);
    const double sp = (1.0 + x) * rp, sm = (t2 * rt) * rp;
    const double xi = div_nr(x, sp + sm);
    const double eta = div_nr(x, (1.0 + sp) * (1.0 + sm));
    const double cphi = fma(xi, fma(-eta, c, s), c);
    const double cpsi = fma(-xi, fma(eta, c, s), c);
    const double sphi = fma(-xi, fma(eta, s, c), s);
    const double spsi = fma(xi, fma(-eta, s, c), s);
    z11 = cphi * rt;
    z21 = -spsi * rt;
    z12 = sphi * rt;
    z22 = cpsi * rt;
    c2small = (cphi == 1.0 && cpsi == 1.0);     // criterion C2 (Section 2.5)
}

// The complex 2x2 transformation of Section 2.1.1 without infinities, for
// A' = [[aii, a], [conj(a), ajj]], B' = [[1, b], [conj(b), 1]], |b| < 1.
// x = |b|, e^{i zeta} = b/|b| (1 for b = 0), z = e^{-i zeta} a = u + i v,
// h = ajj - aii, tau = sign(1, h), s = aii + ajj, t = sqrt(1 - x^2).
// With P = tau (2u - s x), R = sqrt(h^2 + 4 v^2) and Q = t R,
// tan 2theta = P / Q gives cos 2theta = Q / sqrt(P^2 + Q^2) and
// sin 2theta = P / sqrt(P^2 + Q^2); tan gamma = 2v / h gives cos gamma =
// |h| / R and sin gamma = tau 2v / R (so h = 0, v != 0 yields cos 0 and
// sin = sign(v)).  Then, as printed,
//   cos phi = sqrt((1 + x s2 + t cg c2) / 2), cos psi = sqrt((1 - x s2 + t cg c2) / 2),
//   e^{i alpha} sin phi = e^{i zeta} ((s2 - x) + i t sg c2) / (2 cos psi),
//   e^{-i beta} sin psi = e^{-i zeta} ((s2 + x) - i t sg c2) / (2 cos phi),
// and Z' = (1/t)[[cos phi, e^{ia} sin phi], [-e^{-ib} sin psi, cos psi]].
// The exception v = h = 0 returns the printed congruence.  Cosines that
// round to 1 are exactly 1 (criterion C1).  Output: z11, z22 real; z21 =
// (z21r, z21i), z12 = (z12r, z12i) (column-major Z).
__device__ __forceinline__ void hz_cplx_2x2_fast(double aii, double ajj, double ar, double ai,
                                                 double br, double bi, double &z11,
                                                 double &z21r, double &z21i, double &z12r,
                                                 double &z12i, double &z22, bool &c2small)
{
    const double x2 = fma(br, br, bi * bi);
    const bool bz = (x2 == 0.0);
    const double rx = bz ? 0.0 : rsqrt_nr(x2);
    const double x = x2 * rx;
    const double er = bz ? 1.0 : br * rx, ei = bz ? 0.0 : bi * rx;   // e^{i zeta}
    const double u = fma(er, ar, ei * ai), v = fma(er, ai, -ei * ar);  // e^{-i zeta} a
    const double h = ajj - aii;
    const double t2 = fma(-x, x, 1.0);
    const double rt = rsqrt_nr(t2);
    const double t = t2 * rt;
    if (v == 0.0 && h == 0.0) {
        const double r2 = 0.70710678118654752440;
        const double p = r2 * rsqrt_nr(1.0 + x), q = r2 * rsqrt_nr(1.0 - x);
        z11 = p;
        z21r = er * p;
        z21i = -ei * p;
        z12r = -er * q;
        z12i = -ei * q;
        z22 = q;
        c2small = false;
        return;
    }
    const double tau = (h < 0.0) ? -1.0 : 1.0;
    const double h2 = h * h, v4 = 4.0 * v * v;
    const double R2 = h2 + v4;
    const double rR = rsqrt_nr(R2);
    const double cg = (R2 == h2) ? 1.0 : fabs(h) * rR;
    const double sg = tau * 2.0 * v * rR;
    const double P = tau * fma(-(aii + ajj), x, 2.0 * u);
    const double Q2 = t2 * R2;
    const double PQ = fma(P, P, Q2);
    const double rPQ = rsqrt_nr(PQ);
    const double c2 = (PQ == Q2) ? 1.0 : sqrt_nr(Q2) * rPQ;
    const double s2 = P * rPQ;
    const double tcc = t * cg * c2;
    const double cphi = sqrt_nr(0.5 * (fma(x, s2, 1.0) + tcc));
    const double cpsi = sqrt_nr(0.5 * (fma(-x, s2, 1.0) + tcc));
    const double im = t * sg * c2;
    const double dpsi = div_nr(rt, 2.0 * cpsi), dphi = div_nr(rt, 2.0 * cphi);
    // e^{i zeta} ((s2 - x) + i im) / (2 cos psi) / t
    const double ar_ = s2 - x, br_ = s2 + x;
    z12r = (er * ar_ - ei * im) * dpsi;
    z12i = (er * im + ei * ar_) * dpsi;
    // -e^{-i zeta} ((s2 + x) - i im) / (2 cos phi) / t
    z21r = -(er * br_ - ei * im) * dphi;
    z21i = -(-er * im - ei * br_) * dphi;
    z11 = cphi * rt;
    z22 = cpsi * rt;
    c2small = (cphi == 1.0 && cpsi == 1.0);     // criterion C2 (Section 2.5)
}

// Appendix A (enhanced dot products): a*b rounded toward -infinity, from the
// round-to-nearest product p and its exact error e = a*b - p (one FMA): the
// exact product rounds down to p when e >= 0, else to the double just below
// p.  The rounding mode register is left alone; contraction is off here so
// that the product and the sums stay separately rounded operations.
__device__ __forceinline__ double mul_rd(double a, double b)
{
#pragma clang fp contract(off)
    const double p = a * b;
    const double e = fma(a, b, -p);
    if (!(e < 0.0)) return p;
    long long bits = __double_as_longlong(p);
    if (p > 0.0) bits -= 1;
    else if (p < 0.0) bits += 1;
    else bits = (long long)0x8000000000000001ull;   // below +-0: -denorm_min
    return __longlong_as_double(bits);
}

// |re + i im|^2 by the simpler complex procedure of Appendix A: the
// rounded-down squares c_r, c_i and the sum e of their errors, combined as
// (e + min(c_r, c_i)) + max(c_r, c_i).
__device__ __forceinline__ double enh_abs2(double re, double im)
{
#pragma clang fp contract(off)
    const double cr = mul_rd(re, re), ci = mul_rd(im, im);
    const double e = fma(re, re, -cr) + fma(im, im, -ci);
    return (cr <= ci) ? (e + cr) + ci : (e + ci) + cr;
}

// Accumulate a*b into the pair (sum of rounded-down products, sum of their
// non-negative rounding errors).
__device__ __forceinline__ void edot_acc(double a, double b, double &sc, double &sd)
{
#pragma clang fp contract(off)
    const double c = mul_rd(a, b);
    sc = sc + c;
    sd = sd + fma(a, b, -c);
}

}  // namespace hz
