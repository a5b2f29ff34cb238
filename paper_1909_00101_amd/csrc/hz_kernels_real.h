// hz_kernels_real.h -- FP64 device bodies shared by the single-pair kernels
// (hz_real.hip) and the batched kernels (hz_batched.hip): the pivot Gram
// block of a block-column pair, the inner solve of one pivot block pair and
// the in-place block update of a row range.
#pragma once
#include "hz_device.h"
#include "hz_internal.h"

namespace hz {

// LDS (doubles) each body needs; the caller provides it, so one kernel can
// run several bodies over a single allocation.
// (gram: two regions for the waves' partial blocks with stride W2 + 2,
// which puts the 16 lanes of a tile row in distinct banks)
template <int W2> constexpr int gram_lds() { return 2 * W2 * (W2 + 2); }
template <int W2> constexpr int update_lds() { return W2 * (W2 + 1); }

// A pivot Gram block counts as numerically positive definite when every
// Cholesky pivot exceeds W2 * eps (eps = 2^-52) times that column's diagonal
// entry before the factorization: a smaller pivot is at the level of the
// factorization's own rounding errors (an exactly rank-deficient block, e.g.
// two equal columns, leaves pivots of either sign of about that size).
template <int W2> constexpr double PIV_REL() { return W2 * 2.220446049250313e-16; }
template <int W2> constexpr int inner_lds()
{
    return 3 * W2 * (W2 + 2) + 128 + W2 * W2 / 4 + (3 * (W2 / 2) + 1) / 2 + 2;
}

// Device body: four waves form the Gram block of the block-column pair
// (p, q) of Y (m rows, ld m) over the 64-row chunks [c0, c1) and write it to
// out (column-major W2 x W2, lower tiles).  The MFMA operands come straight
// from global memory, no LDS in the loop: for X^T X both operands of a
// product hold the same kind of value (lane l: row k of the chunk's slab,
// column l % 16 of a 16-column tile), and which rows feed which k-step is
// free, so wave w takes rows 16w .. 16w + 15 of every chunk and lane group
// g = l / 16 loads rows 2g, 2g + 1 of each 8-row half as one 16-byte load:
// a column's 64 bytes are contiguous per load and every 128-byte line is
// used whole by one wave.  A wave's k-steps are, per chunk, rows
// 16w + 8h + 2g + j for (h, j) = (0,0), (0,1), (1,0), (1,1); the four
// waves' partial tiles are summed as (w0 + w1) + (w2 + w3) (tile, gram_lds
// doubles).  Further waves of a larger workgroup only take part in the
// barriers, so the sums do not depend on the workgroup size.
template <int W2>
__device__ __forceinline__ void gram_block(const double *__restrict__ Y, int64_t m, int p, int q,
                                           int64_t c0, int64_t c1, double *__restrict__ out,
                                           double *__restrict__ tile)
{
    constexpr int W = W2 / 2, NB = W2 / 16, NTL = NB * (NB + 1) / 2, PF = 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    d4 acc[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    const double *colp[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        const int cc = 16 * a + (lane & 15);
        const int gc = (cc < W) ? p * W + cc : q * W + (cc - W);
        colp[a] = Y + (int64_t)gc * m + 16 * wave + 2 * (lane >> 4);
    }
    d2 buf[PF][NB][2];
    auto load = [&](d2 (&b)[NB][2], int64_t c) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int h = 0; h < 2; ++h) b[a][h] = *(const d2 *)(colp[a] + c * 64 + 8 * h);
    };
    auto mul = [&](const d2 (&b)[NB][2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                int t = 0;
#pragma unroll
                for (int a = 0; a < NB; ++a)
#pragma unroll
                    for (int b2 = 0; b2 <= a; ++b2, ++t)
                        acc[t] = mfma16(b[a][h][j], b[b2][h][j], acc[t]);
            }
    };
    // PF chunks in flight.  The main loop has no branch, so each chunk's
    // products wait only for that chunk's loads (a branch there made the
    // compiler wait for all of them); loads past the range are clamped to
    // its last chunk and left unused, and the remainder follows the loop.
    if (wave < 4 && c0 < c1) {
#pragma unroll
        for (int i = 0; i < PF; ++i) load(buf[i], c0 + i < c1 ? c0 + i : c1 - 1);
        int64_t c = c0;
        for (; c + PF <= c1; c += PF) {
#pragma unroll
            for (int i = 0; i < PF; ++i) {
                mul(buf[i]);
                load(buf[i], c + i + PF < c1 ? c + i + PF : c1 - 1);
            }
        }
#pragma unroll
        for (int i = 0; i < PF - 1; ++i)
            if (c + i < c1) mul(buf[i]);
    }
    // Sum the waves' partial tiles pairwise, (w0 + w1) + (w2 + w3): waves 1
    // and 3 leave theirs in two LDS regions (tile reused, ld W2 + 2), wave 2
    // adds its own into the second, and wave 0 adds both regions to its own
    // and stores the lower tiles straight from its registers.  Element r of
    // tile (a, b) in lane l is entry (16a + 4r + l/16, 16b + l%16).
    constexpr int LDSUM = W2 + 2;
    double *const R0 = tile, *const R1 = tile + W2 * LDSUM;
    auto at = [&](int a, int b, int r) {
        return (16 * b + (lane & 15)) * LDSUM + 16 * a + 4 * r + (lane >> 4);
    };
    __syncthreads();                     // the caller's previous use of tile is over
    if (wave == 1 || wave == 3) {
        double *const R = (wave == 1) ? R0 : R1;
        int t = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b, ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) R[at(a, b, r)] = acc[t][r];
    }
    __syncthreads();
    if (wave == 2) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b, ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) R1[at(a, b, r)] = acc[t][r] + R1[at(a, b, r)];
    }
    __syncthreads();
    if (wave == 0) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b, ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    out[(16 * b + (lane & 15)) * W2 + 16 * a + 4 * r + (lane >> 4)] =
                        (acc[t][r] + R0[at(a, b, r)]) + R1[at(a, b, r)];
    }
}

// The four pivot entries of a column pair held as RPL rows per lane by
// groups of LP lanes, summed over the group (every lane gets the sums):
// a_ii = f_i^T f_i, a_jj = f_j^T f_j, a_ij = f_i^T f_j, b_ij = g_i^T g_j
// (b_ii = b_jj = 1 after the prescaling, Section 2.1).  Odd variants use the
// enhanced dot products of Appendix A.
template <int LP, int RPL>
__device__ __forceinline__ void pair_dots(const double (&fi)[RPL], const double (&fj)[RPL],
                                          const double (&gi)[RPL], const double (&gj)[RPL],
                                          int variant, double &aii, double &ajj, double &aij,
                                          double &bij)
{
    aii = 0.0; ajj = 0.0; aij = 0.0; bij = 0.0;
    if (variant & 1) {
        // the rounded-down products and their errors are summed apart
        double ei = 0.0, ej = 0.0, eij = 0.0, eb = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            edot_acc(fi[r], fi[r], aii, ei);
            edot_acc(fj[r], fj[r], ajj, ej);
            edot_acc(fi[r], fj[r], aij, eij);
            edot_acc(gi[r], gj[r], bij, eb);
        }
        aii = dpp_group_sum<LP>(aii) + dpp_group_sum<LP>(ei);
        ajj = dpp_group_sum<LP>(ajj) + dpp_group_sum<LP>(ej);
        aij = dpp_group_sum<LP>(aij) + dpp_group_sum<LP>(eij);
        bij = dpp_group_sum<LP>(bij) + dpp_group_sum<LP>(eb);
    } else {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            aii = fma(fi[r], fi[r], aii);
            ajj = fma(fj[r], fj[r], ajj);
            aij = fma(fi[r], fj[r], aij);
            bij = fma(gi[r], gj[r], bij);
        }
        aii = dpp_group_sum<LP>(aii);
        ajj = dpp_group_sum<LP>(ajj);
        aij = dpp_group_sum<LP>(aij);
        bij = dpp_group_sum<LP>(bij);
    }
}

// One pointwise step of the inner solver on the pivot entries of column
// pair (i, j), i < j (Section 2.1): the relative orthogonality test, the 2x2
// transformation Z' (real case, Section 2.1.2), its classification (big
// unless criterion C1, or C2 for variants 4 and 5, says small, Section 2.5)
// and the sorting heuristic (swap the two columns when the transformed
// a''_11 < a''_22, or when an orthogonal pair has a_ii < a_jj).  Returns
// whether [f_i f_j] (and g, z) change: z11, z21, z12, z22 is then the 2x2
// matrix to postmultiply them by, swap included.
__device__ __forceinline__ bool pair_transform(double aii, double ajj, double aij, double bij,
                                               double tol, double tol2, int sort, int variant,
                                               double &z11, double &z21, double &z12,
                                               double &z22, unsigned &sw_all, unsigned &sw_big)
{
    z11 = 1.0; z21 = 0.0; z12 = 0.0; z22 = 1.0;
    bool swap;
    const bool orth = (aij * aij < aii * ajj * tol2) && (fabs(bij) < tol);
    if (orth) {
        swap = sort && (aii < ajj);
    } else {
        bool c2small;
        hz_real_2x2_fast(aii, ajj, aij, bij, z11, z21, z12, z22, c2small);
        sw_all += 1;
        // small: criterion C1 (variants 0, 1) or C2 (variants 4, 5), Section 2.5
        if ((variant & 4) ? !c2small : !(z11 == 1.0 && z22 == 1.0)) sw_big += 1;
        swap = false;
        if (sort) {
            const double a11 = fma(z11 * z11, aii, fma(2.0 * z11 * z21, aij, z21 * z21 * ajj));
            const double a22 = fma(z12 * z12, aii, fma(2.0 * z22 * z12, aij, z22 * z22 * ajj));
            swap = a11 < a22;
        }
    }
    if (swap) {
        double t;
        t = z11; z11 = z12; z12 = t;
        t = z21; z21 = z22; z22 = t;
    }
    return !orth || swap;
}

// [x_i x_j] <- [x_i x_j] [[z11, z12], [z21, z22]] on RPL rows per lane.
template <int RPL>
__device__ __forceinline__ void rotate_rows(double (&xi)[RPL], double (&xj)[RPL], double z11,
                                            double z21, double z12, double z22)
{
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const double ni = fma(xj[r], z21, xi[r] * z11);
        const double nj = fma(xi[r], z12, xj[r] * z22);
        xi[r] = ni;
        xj[r] = nj;
    }
}

// Device body: the workgroup (NT threads) solves the block pair whose Gram
// blocks are pa (F) and pb (G) (column-major W2 x W2, lower triangles),
// writes Z_tilde to zt, the counters (transformations, big ones, inner
// sweeps) to myc[0..2] and to myc[3] whether Z_tilde is the identity, and
// on a non-positive pivot sets FLAG_CHOL in status[ST_FLAGS] and failcode
// into status[ST_FAILPAIR] (minimum kept).  When no pair of the block was
// transformed or swapped, Z_tilde is the diagonal Theta-scaled prescale,
// which only renormalizes columns that already have ||f_j||^2 + ||g_j||^2 =
// 1 up to rounding; it is then set to I exactly and myc[3] = 1, so the
// block update may be skipped (Section 2.5).
template <int W2, int LP, bool RING = false>
__device__ __forceinline__ void inner_solve(
    const double *__restrict__ pa, const double *__restrict__ pb, int nsplit, size_t sstride,
    const int16_t *__restrict__ itab, int isteps, int inner_max, double tol, int sort, int variant,
    double *__restrict__ zt, unsigned long long *__restrict__ myc, int *__restrict__ status,
    int failcode, unsigned long long *__restrict__ ph, double *__restrict__ lds)
{
    constexpr int W = W2 / 2;         // column pairs per inner step
    constexpr int NT = W * LP;
    constexpr int RPL = W2 / LP;      // rows per lane
    constexpr int LDI = W2 + 2;
    static_assert(RPL >= 2 && RPL % 2 == 0 && NT >= 64, "bad inner geometry");
    double *const sF = lds;
    double *const sG = lds + W2 * LDI;
    double *const sZ = lds + 2 * W2 * LDI;
    double *const lbuf0 = lds + 3 * W2 * LDI;                 // 2 x 64 doubles
    int16_t *const stab = (int16_t *)(lbuf0 + 128);           // W2 * W2 entries
    unsigned *const s_cnt = (unsigned *)(lbuf0 + 128 + W2 * W2 / 4);
    int *const s_failp = (int *)(s_cnt + 3 * W);
#define s_fail (*s_failp)

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (ph && tid == 0) ph[0] = wall_clock64();
    // 1. load the Gram blocks (lower triangles) into LDS; with nsplit > 1 the
    // blocks arrive as nsplit row-split partials (stride sstride), added in
    // split order; with nsplit 0 they are the upper triangular factors
    // themselves (QR of the block-column pairs).
    if (nsplit <= 1) {
        // one summed block (or a factor): every load of a thread issued
        // before the first store, so the phase costs one memory latency
        constexpr int NIT = (W2 * W2) / (2 * NT);
        static_assert(NIT * 2 * NT == W2 * W2, "Gram load geometry");
        d2 va[NIT], vb[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int e = 2 * tid + 2 * NT * it;
            // upper tiles of a Gram are never read (zeros go to LDS); a factor
            // (nsplit 0) is upper
            const bool skip = nsplit > 0 && (e / W2) / 16 > (e % W2) / 16;
            va[it] = skip ? d2{0.0, 0.0} : *(const d2 *)(pa + e);
            vb[it] = skip ? d2{0.0, 0.0} : *(const d2 *)(pb + e);
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int e = 2 * tid + 2 * NT * it, col = e / W2, row = e % W2;
            *(d2 *)(sF + col * LDI + row) = va[it];
            *(d2 *)(sG + col * LDI + row) = vb[it];
        }
        if (!RING) copy_table<NT>(stab, itab, isteps * W * 2);
        if (tid == 0) s_fail = 0;
    } else {
        for (int e = 2 * tid; e < W2 * W2; e += 2 * NT) {
            // upper tiles of a Gram are never read
            if ((e / W2) / 16 > (e % W2) / 16) continue;
            d2 a = *(const d2 *)(pa + e), b = *(const d2 *)(pb + e);
            for (int sp = 1; sp < nsplit; ++sp) {
                a += *(const d2 *)(pa + sp * sstride + e);
                b += *(const d2 *)(pb + sp * sstride + e);
            }
            const int col = e / W2, row = e % W2;
            *(d2 *)(sF + col * LDI + row) = a;
            *(d2 *)(sG + col * LDI + row) = b;
        }
        if (!RING) copy_table<NT>(stab, itab, isteps * W * 2);
        if (tid == 0) s_fail = 0;
    }
    __syncthreads();
    if (ph && tid == 0) ph[1] = wall_clock64();

    // 2. Cholesky factorizations, lane = row, one wave per matrix.  With
    // nsplit 0 the factors came in (QR of the block-column pairs): only their
    // diagonals are checked for zeros and non-finite values.
    if (nsplit == 0) {
        if (tid < W2) {
            const double df = sF[tid * LDI + tid], dg = sG[tid * LDI + tid];
            if (!(fabs(df) > 0.0 && fabs(df) < INFINITY && fabs(dg) > 0.0 && fabs(dg) < INFINITY))
                s_fail = 1;
        }
    } else if constexpr (W2 >= 32 && NT >= 128) {
        // Blocked right-looking Cholesky, one wave per matrix, panels of 16
        // columns (2w = 32 or 64; lanes past the block's rows idle).  A
        // panel (its rows c0.. of columns c0..c0+15, lane = row) is factored
        // in registers, the entries of a column reaching the later panel
        // columns by readlane; the panel goes back to LDS and the trailing
        // lower tiles take the update A22 -= L21 L21^T as FP64 MFMA products
        // (tile (ti, tj): A operand L rows of ti, B operand L rows of tj,
        // four k-steps of 4 panel columns).
        constexpr int NBK = W2 / 16;
        if (wave < 2) {
            double *M = wave ? sG : sF;
            bool ok = true;
            // lane j (< 16) holds the diagonals of columns 16 kb + j before
            // the factorization; it tests the pivot of that column itself
            // once the panel is factored
            double d0[NBK];
#pragma unroll
            for (int kb = 0; kb < NBK; ++kb)
                d0[kb] = (lane < 16) ? M[(16 * kb + lane) * LDI + 16 * kb + lane] : 1.0;
#pragma unroll
            for (int kb = 0; kb < NBK; ++kb) {
                const int c0 = 16 * kb, row = c0 + lane;
                const bool live = row < W2;
                double pv[16];
#pragma unroll
                for (int t = 0; t < 16; ++t) pv[t] = live ? M[(c0 + t) * LDI + row] : 0.0;
                double own = 1.0;           // lane j: the pivot of column c0 + j
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const double piv = readlane_d(pv[j], j);
                    if (lane == j) own = pv[j];
                    const double inv = rsqrt_nr(piv);
                    const double l = (lane >= j) ? pv[j] * inv : 0.0;
                    pv[j] = l;
#pragma unroll
                    for (int t = j + 1; t < 16; ++t) pv[t] = fma(-l, readlane_d(l, t), pv[t]);
                }
                if (lane < 16) ok = ok && (own > PIV_REL<W2>() * d0[kb]) && (own < INFINITY);
                if (live) {
#pragma unroll
                    for (int t = 0; t < 16; ++t) M[(c0 + t) * LDI + row] = pv[t];
                }
                wave_fence();
                const int i16 = lane & 15, k4 = lane >> 4;
#pragma unroll
                for (int ti = kb + 1; ti < NBK; ++ti)
#pragma unroll
                    for (int tj = kb + 1; tj <= ti; ++tj) {
                        // element r of lane l: row 16 ti + 4 r + l/16, column 16 tj + l%16
                        double *const ct = M + (16 * tj + i16) * LDI + 16 * ti + k4;
                        d4 acc = d4{ct[0], ct[4], ct[8], ct[12]};
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const double *const lc = M + (c0 + 4 * s + k4) * LDI;
                            acc = mfma16(-lc[16 * ti + i16], lc[16 * tj + i16], acc);
                        }
                        ct[0] = acc[0];
                        ct[4] = acc[1];
                        ct[8] = acc[2];
                        ct[12] = acc[3];
                    }
                wave_fence();
            }
            // F_hat = L^T: column i of F_hat is row i of L.
            double a[W2];
            if (lane < W2) {
#pragma unroll
                for (int k = 0; k < W2; ++k) a[k] = M[k * LDI + lane];
            }
            wave_fence();
            if (lane < W2) {
#pragma unroll
                for (int k = 0; k < W2; ++k) M[lane * LDI + k] = (k <= lane) ? a[k] : 0.0;
            }
            if (!ok) s_fail = 1;
        }
    } else {
        constexpr bool two = (W2 == 64);
        const int mat = two ? wave : (lane >> 5);
        const int i = two ? lane : (lane & 31);
        if ((two ? (wave < 2) : (wave == 0)) && i < W2) {
            double *M = mat ? sG : sF;
            double *lb = lbuf0 + 64 * mat;
            double a[W2];
#pragma unroll
            for (int k = 0; k < W2; ++k) a[k] = M[k * LDI + i];
            const double d0 = M[i * LDI + i];    // column i's diagonal before the factorization
            double own = 1.0;                      // the pivot of column i, kept by lane i
#pragma unroll
            for (int j = 0; j < W2; ++j) {
                double piv;
                if (two) {
                    piv = readlane_d(a[j], j);
                } else {
                    const double p0 = readlane_d(a[j], j), p1 = readlane_d(a[j], 32 + j);
                    piv = mat ? p1 : p0;
                }
                if (i == j) own = a[j];
                const double inv = rsqrt_nr(piv);
                const double l = (i >= j) ? a[j] * inv : 0.0;
                a[j] = l;
                lb[i] = l;
                wave_fence();
#pragma unroll
                for (int k = j + 1; k < W2; k += 2) {
                    const d2 lk = *(const d2 *)(lb + k - (k & 1));
                    if (k & 1) {
                        a[k] = fma(-l, lk[1], a[k]);
                        if (k + 1 < W2) a[k + 1] = fma(-l, (*(const d2 *)(lb + k + 1))[0], a[k + 1]);
                    } else {
                        a[k] = fma(-l, lk[0], a[k]);
                        if (k + 1 < W2) a[k + 1] = fma(-l, lk[1], a[k + 1]);
                    }
                }
                wave_fence();
            }
            // F_hat = L^T: column i of F_hat is row i of L.
#pragma unroll
            for (int k = 0; k < W2; ++k) M[i * LDI + k] = (k <= i) ? a[k] : 0.0;
            if (!((own > PIV_REL<W2>() * d0) && (own < INFINITY))) s_fail = 1;
        }
    }
    __syncthreads();
    if (ph && tid == 0) ph[2] = wall_clock64();
    if (__builtin_amdgcn_readfirstlane(s_fail)) {      // uniform: every lane read the same word
        for (int e = tid; e < W2 * W2; e += NT) zt[e] = (e % W2 == e / W2) ? 1.0 : 0.0;
        if (tid == 0) {
            myc[0] = 0;
            myc[1] = 0;
            myc[2] = 0;
            myc[3] = 0;
            atomicOr(status + ST_FLAGS, FLAG_CHOL);
            atomicMin(status + ST_FAILPAIR, failcode);
        }
        return;
    }

    const int grp = tid / LP, gl = tid % LP, r0 = gl * RPL;
    // Row k (0 <= k < RPL) of a lane's share of a column: RPL consecutive
    // rows for the table orderings; for the ring ordering pairs of rows
    // 2 LP apart, so that the 16-byte accesses of a group's lanes are
    // contiguous in LDS.
    auto RI = [&](int k) { return RING ? (k >> 1) * 2 * LP + 2 * gl + (k & 1) : r0 + k; };
    // 3. prescale the factor pair: columns 2*grp and 2*grp+1 per group.
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = 2 * grp + h;
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const double g = sG[c * LDI + RI(r)];
            s = fma(g, g, s);
        }
        s = dpp_group_sum<LP>(s);
        const double d = rsqrt_nr(s);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            sF[c * LDI + RI(r)] *= d;
            sG[c * LDI + RI(r)] *= d;
            sZ[c * LDI + RI(r)] = (RI(r) == c) ? d : 0.0;
        }
    }
    __syncthreads();
    if (ph && tid == 0) ph[3] = wall_clock64();

    // 4. inner sweeps
    const double tol2 = tol * tol;
    unsigned my_all = 0, my_big = 0, my_chg = 0;
    int nsw = 0;
    auto load = [&](const double *M, int c, double (&x)[RPL]) {
#pragma unroll
        for (int r = 0; r < RPL; r += 2) {
            const d2 v = *(const d2 *)(M + c * LDI + RI(r));
            x[r] = v[0];
            x[r + 1] = v[1];
        }
    };
    auto store = [&](double *M, int c, const double (&x)[RPL]) {
#pragma unroll
        for (int r = 0; r < RPL; r += 2) *(d2 *)(M + c * LDI + RI(r)) = d2{x[r], x[r + 1]};
    };
    for (int sw = 0; sw < inner_max; ++sw) {
        unsigned sw_all = 0, sw_big = 0;
        ++nsw;
        if constexpr (RING) {
            // Ring ordering, level by level: the columns form blocks of size
            // 2h (h = W, W/2, ..., 1); group u of a block keeps column u of
            // the block's first half in registers for the whole level and
            // meets every column of the second half once.  The second half
            // is cut into sets of G = min(h, groups per wave) columns; in
            // phase p wave o of the block takes set (o + p) mod (h / G), and
            // in its sub-step t group g of the wave takes column g xor t of
            // that set.  A set stays inside one wave for a phase, so the
            // columns move between sub-steps through LDS in the wave's own
            // program order; only between phases and levels does the whole
            // workgroup synchronise.
            constexpr int GW = 64 / LP;             // groups per wave
            for (int h = W; h >= 1; h >>= 1) {
                const int blk = grp / h, u = grp % h;
                const int ci = blk * 2 * h + u;
                const int nset = (h >= GW) ? h / GW : 1, ssz = (h >= GW) ? GW : h;
                const int ow = u / ssz, gw = u % ssz;
                double fi[RPL], gi[RPL], zi[RPL];
                load(sF, ci, fi);
                load(sG, ci, gi);
                load(sZ, ci, zi);
                for (int p = 0; p < nset; ++p) {
                    for (int t = 0; t < ssz; ++t) {
                        const int cj = blk * 2 * h + h + ring_col(ssz, nset, ow, gw, p, t);
                        double fj[RPL], gj[RPL], zj[RPL];
                        load(sF, cj, fj);
                        load(sG, cj, gj);
                        load(sZ, cj, zj);
                        double aii, ajj, aij, bij, z11, z21, z12, z22;
                        pair_dots<LP, RPL>(fi, fj, gi, gj, variant, aii, ajj, aij, bij);
                        // Every group applies its 2x2 matrix, the identity when
                        // its pair is left alone (which reproduces the columns,
                        // a negative zero possibly turned positive): with one
                        // path through the step the columns stay in their
                        // registers, where a branch costs a copy of each.
                        if (pair_transform(aii, ajj, aij, bij, tol, tol2, sort, variant, z11, z21,
                                           z12, z22, sw_all, sw_big)) {
                            my_chg = 1;
                            rotate_rows<RPL>(fi, fj, z11, z21, z12, z22);
                            rotate_rows<RPL>(gi, gj, z11, z21, z12, z22);
                            rotate_rows<RPL>(zi, zj, z11, z21, z12, z22);
                            store(sF, cj, fj);
                            store(sG, cj, gj);
                            store(sZ, cj, zj);
                        }
                        if (t + 1 < ssz) wave_fence();
                    }
                    __syncthreads();
                }
                store(sF, ci, fi);
                store(sG, ci, gi);
                store(sZ, ci, zi);
                __syncthreads();
            }
        } else {
            for (int st = 0; st < isteps; ++st) {
                const int ci = stab[(st * W + grp) * 2], cj = stab[(st * W + grp) * 2 + 1];
                double fi[RPL], fj[RPL], gi[RPL], gj[RPL], zi[RPL], zj[RPL];
                load(sF, ci, fi);
                load(sF, cj, fj);
                load(sG, ci, gi);
                load(sG, cj, gj);
                load(sZ, ci, zi);
                load(sZ, cj, zj);
                double aii, ajj, aij, bij, z11, z21, z12, z22;
                pair_dots<LP, RPL>(fi, fj, gi, gj, variant, aii, ajj, aij, bij);
                if (pair_transform(aii, ajj, aij, bij, tol, tol2, sort, variant, z11, z21, z12,
                                   z22, sw_all, sw_big)) {
                    my_chg = 1;
                    rotate_rows<RPL>(fi, fj, z11, z21, z12, z22);
                    rotate_rows<RPL>(gi, gj, z11, z21, z12, z22);
                    rotate_rows<RPL>(zi, zj, z11, z21, z12, z22);
                    store(sF, ci, fi);
                    store(sF, cj, fj);
                    store(sG, ci, gi);
                    store(sG, cj, gj);
                    store(sZ, ci, zi);
                    store(sZ, cj, zj);
                }
                __syncthreads();
            }
        }
        my_all += sw_all;
        my_big += sw_big;
        const int any = __builtin_amdgcn_readfirstlane(__syncthreads_count(gl == 0 && sw_all > 0));
        if (any == 0) break;
    }

    if (ph && tid == 0) ph[4] = wall_clock64();
    // 5. Theta rescale and write Z_tilde (column-major W2 x W2); the
    // identity when nothing was transformed or swapped.
    const int nchg =
        __builtin_amdgcn_readfirstlane(__syncthreads_count(gl == 0 && my_chg != 0));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = 2 * grp + h;
        if (nchg == 0) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) zt[c * W2 + RI(r)] = (RI(r) == c) ? 1.0 : 0.0;
            continue;
        }
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const double f = sF[c * LDI + RI(r)], g = sG[c * LDI + RI(r)];
            s = fma(f, f, s);
            s = fma(g, g, s);
        }
        s = dpp_group_sum<LP>(s);
        const double th = rsqrt_nr(s);
#pragma unroll
        for (int r = 0; r < RPL; ++r) zt[c * W2 + RI(r)] = sZ[c * LDI + RI(r)] * th;
    }
    // counters: the groups' totals summed in group order
    if (gl == 0) {
        s_cnt[3 * grp] = my_all;
        s_cnt[3 * grp + 1] = my_big;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long ta = 0, tb = 0;
        for (int g = 0; g < W; ++g) {
            ta += s_cnt[3 * g];
            tb += s_cnt[3 * g + 1];
        }
        myc[0] = ta;
        myc[1] = tb;
        myc[2] = (unsigned long long)nsw;
        myc[3] = (nchg == 0) ? 1ull : 0ull;
        if (ph) ph[5] = wall_clock64();
    }
#undef s_fail
}

// Device body: one workgroup of NW waves updates the rows [rb, re) (a
// multiple of 16 rows) of a row sequence by zt (column-major W2 x W2),
// staged in LDS (sz, update_lds<W2>() doubles).  locate(v, Y, m, r) maps
// sequence row v (the first of a 16-row tile, which never straddles two
// matrices) to the matrix Y (ld m) and its row r; in Y the block-column
// pair (p, q) is updated.
template <int W2, int NW, class Locate>
__device__ __forceinline__ void update_row_seq(Locate locate, int p, int q, int64_t rb,
                                               int64_t re, const double *__restrict__ zt,
                                               double *__restrict__ sz)
{
    constexpr int W = W2 / 2, NB = W2 / 16, KS = W2 / 4, LDZ = W2 + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NTH = 64 * NW;
    if constexpr ((W2 * W2) % NTH == 0) {
        // every load of a thread issued before the first store: one memory
        // latency before the rows can start instead of one per element
        constexpr int NZ = (W2 * W2) / NTH;
        double zv[NZ];
#pragma unroll
        for (int it = 0; it < NZ; ++it) zv[it] = zt[tid + NTH * it];
#pragma unroll
        for (int it = 0; it < NZ; ++it) {
            const int e = tid + NTH * it;
            sz[(e / W2) * LDZ + (e % W2)] = zv[it];
        }
    } else {
        for (int e = tid; e < W2 * W2; e += NTH) sz[(e / W2) * LDZ + (e % W2)] = zt[e];
    }
    __syncthreads();
    // Lane (i, k) = (lane % 16, lane / 16).  Columns 0..W-1 of the pair are
    // block column p, W..2W-1 block column q; every k-step's column offset
    // is a uniform multiple of m.
    const int k4 = lane >> 4, i16 = lane & 15;
    for (int64_t v0 = rb + 16 * wave; v0 < re; v0 += 16 * NW) {
        // keep the Z_tilde fragment reads inside the loop (in LDS, not in
        // 128 registers hoisted out of it)
        __asm__ volatile("" ::: "memory");
        double *Y;
        int64_t m, r0;
        locate(v0, Y, m, r0);
        const double *bp = Y + ((int64_t)p * W + k4) * m + i16;
        const double *bq = Y + ((int64_t)q * W + k4) * m + i16;
        double xb[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s)
            xb[s] = (4 * s < W) ? bp[(int64_t)(4 * s) * m + r0] : bq[(int64_t)(4 * s - W) * m + r0];
        d4 acc[NB];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) acc[jb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                // A'[j][k] = Z_tilde[4s+k][16jb+j], lane j + 16k
                const double za = sz[(16 * jb + i16) * LDZ + 4 * s + k4];
                acc[jb] = mfma16(za, xb[s], acc[jb]);
            }
        // element r of acc[jb] in lane l is output column 16jb + 4r + l/16, row l%16
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c0 = 16 * jb + 4 * r;
                double *dst = (c0 < W) ? (double *)bp + (int64_t)c0 * m + r0
                                       : (double *)bq + (int64_t)(c0 - W) * m + r0;
                *dst = acc[jb][r];
            }
    }
}

// The same for the rows [rb, re) of one matrix Y (ld m).
template <int W2, int NW>
__device__ __forceinline__ void update_rows(double *__restrict__ Y, int64_t m, int p, int q,
                                            int64_t rb, int64_t re,
                                            const double *__restrict__ zt,
                                            double *__restrict__ sz)
{
    update_row_seq<W2, NW>(
        [=](int64_t v, double *&y, int64_t &ld, int64_t &r) {
            y = Y;
            ld = m;
            r = v;
        },
        p, q, rb, re, zt, sz);
}

}  // namespace hz
