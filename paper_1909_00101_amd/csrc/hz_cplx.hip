// hz_cplx.hip -- complex128 kernels of the blocked one-sided implicit
// Hari-Zimmermann GSVD on gfx950 (paper: the complex case of Sections 2.1.1
// and 3; matrices kept interleaved (re, im) in HBM and LDS).
//
// The structure mirrors the real path (hz_real.hip): prescale/copy-in,
// block steps of Gram -> inner solve -> update, then extraction and sort.
// Complex products on FP64 MFMA use four real products per complex
// multiply-accumulate.  No floating-point atomics; fixed reduction orders.
#include "hz_device.h"
#include "hz_internal.h"

namespace hz {

// Prescale and copy-in with bordering (Section 2, Section 3.1, Section 3.3).
__global__ __launch_bounds__(256) void k_prescale_copy_z(
    int64_t mf, int64_t mg, int64_t n, const d2 *__restrict__ F, int64_t ldf,
    const d2 *__restrict__ G, int64_t ldg, int64_t nw, int64_t mfw, int64_t mgw, int64_t nzw,
    d2 *__restrict__ Fw, d2 *__restrict__ Gw, d2 *__restrict__ Zw, int *__restrict__ status)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nw) return;
    d2 *fw = Fw + j * mfw, *gw = Gw + j * mgw, *zw = Zw + j * nzw;
    const d2 zero = {0.0, 0.0};
    if (j < n) {
        const d2 *f = F + j * ldf, *g = G + j * ldg;
        double s = 0.0;
        for (int64_t r = lane; r < mg; r += 64) {
            const d2 v = g[r];
            s = fma(v[0], v[0], s);
            s = fma(v[1], v[1], s);
        }
        s = wave_sum(s);
        const double d = 1.0 / sqrt(s);
        bool bad = !(s > 0.0) || !isfinite(s);
        for (int64_t r = lane; r < mfw; r += 64) {
            const d2 v = (r < mf) ? f[r] * d : zero;
            bad |= !isfinite(v[0]) || !isfinite(v[1]);
            fw[r] = v;
        }
        for (int64_t r = lane; r < mgw; r += 64) gw[r] = (r < mg) ? g[r] * d : zero;
        for (int64_t r = lane; r < nzw; r += 64) zw[r] = (r == j) ? d2{d, 0.0} : zero;
        if (bad) atomicOr(status + ST_FLAGS, FLAG_NONFINITE);
    } else {
        const int64_t k = j - n;
        const d2 one = {1.0, 0.0};
        for (int64_t r = lane; r < mfw; r += 64) fw[r] = (r == mf + k) ? one : zero;
        for (int64_t r = lane; r < mgw; r += 64) gw[r] = (r == mg + k) ? one : zero;
        for (int64_t r = lane; r < nzw; r += 64) zw[r] = (r == j) ? one : zero;
    }
}

// Hermitian pivot Gram blocks A_hat = X^H X (Section 2.3, ZHERK-like),
// lower-triangle 16x16 tiles, split-K partials (interleaved complex,
// column-major W2 x W2).  Re = Xr^T Xr + Xi^T Xi, Im = Xr^T Xi - Xi^T Xr.
// The MFMA operands come straight from memory: wave w takes rows
// 16w .. 16w + 15 of every 64-row chunk, its k-step s rows 16w + 4s + g
// (g = lane / 16), one 16-byte complex element per lane, so a column's
// 64 bytes are contiguous per load; two chunks in flight, with a
// branch-free main loop as in the real Gram.
template <int W2>
__global__ __launch_bounds__(256) void k_gram_z(const d2 *__restrict__ Fw,
                                                const d2 *__restrict__ Gw, int64_t mfw,
                                                int64_t mgw, const int *__restrict__ pairs,
                                                int splits, d2 *__restrict__ part)
{
    // LDR: row stride of the two regions that take the waves' partial
    // tiles (padded so that the 16 lanes of a tile row fall in distinct LDS
    // banks).
    constexpr int W = W2 / 2, NB = W2 / 16, LDR = W2 + 2, PF = 2;
    constexpr int NT = NB * (NB + 1) / 2;
    __shared__ __attribute__((aligned(16))) double tre[2 * W2 * LDR];
    __shared__ __attribute__((aligned(16))) double tim[2 * W2 * LDR];
    const int split = blockIdx.x, pr = blockIdx.y, mat = blockIdx.z;
    const d2 *Y = mat ? Gw : Fw;
    const int64_t m = mat ? mgw : mfw;
    const int p = pairs[2 * pr], q = pairs[2 * pr + 1];
    const int64_t nch = m / 64;
    const int64_t c0 = nch * split / splits, c1 = nch * (split + 1) / splits;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    d4 accr[NT], acci[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        accr[t] = d4{0.0, 0.0, 0.0, 0.0};
        acci[t] = d4{0.0, 0.0, 0.0, 0.0};
    }
    const d2 *colp[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        const int cc = 16 * a + (lane & 15);
        const int gc = (cc < W) ? p * W + cc : q * W + (cc - W);
        colp[a] = Y + (int64_t)gc * m + 16 * wave + (lane >> 4);
    }
    d2 buf[PF][NB][4];
    auto load = [&](d2 (&b)[NB][4], int64_t c) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int s = 0; s < 4; ++s) b[a][s] = colp[a][c * 64 + 4 * s];
    };
    auto mul = [&](const d2 (&b)[NB][4]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            int t = 0;
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int bb = 0; bb <= a; ++bb, ++t) {
                    accr[t] = mfma16(b[a][s][0], b[bb][s][0], accr[t]);
                    accr[t] = mfma16(b[a][s][1], b[bb][s][1], accr[t]);
                    acci[t] = mfma16(b[a][s][0], b[bb][s][1], acci[t]);
                    acci[t] = mfma16(-b[a][s][1], b[bb][s][0], acci[t]);
                }
        }
    };
    if (c0 < c1) {
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
    // The waves' partial tiles summed pairwise, (w0 + w1) + (w2 + w3), as
    // for the real Gram: waves 1 and 3 leave theirs in two regions, wave 2
    // adds its own into the second, wave 0 adds both and stores the lower
    // tiles (entry (16a + 4r + l/16, 16b + l%16) of tile (a, b) in lane l).
    auto at = [&](int reg, int a, int b, int r) {
        return reg * W2 * LDR + (16 * b + (lane & 15)) * LDR + 16 * a + 4 * r + (lane >> 4);
    };
    __syncthreads();
    if (wave == 1 || wave == 3) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b, ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    tre[at(wave >> 1, a, b, r)] = accr[t][r];
                    tim[at(wave >> 1, a, b, r)] = acci[t][r];
                }
    }
    __syncthreads();
    if (wave == 2) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b, ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    tre[at(1, a, b, r)] = accr[t][r] + tre[at(1, a, b, r)];
                    tim[at(1, a, b, r)] = acci[t][r] + tim[at(1, a, b, r)];
                }
    }
    __syncthreads();
    if (wave == 0) {
        d2 *out = part + ((size_t)(pr * 2 + mat) * splits + split) * (W2 * W2);
        int t = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b, ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    out[(16 * b + (lane & 15)) * W2 + 16 * a + 4 * r + (lane >> 4)] =
                        d2{(accr[t][r] + tre[at(0, a, b, r)]) + tre[at(1, a, b, r)],
                           (acci[t][r] + tim[at(0, a, b, r)]) + tim[at(1, a, b, r)]};
    }
}

// Sum of the split partials in split order (fixed association); the upper
// tiles, which no kernel forms, are written as zeros.
template <int W2>
__global__ __launch_bounds__(256) void k_gram_sum_z(const d2 *__restrict__ part, int splits,
                                                    d2 *__restrict__ gram)
{
    constexpr int MAXS = 16;
    const int pm = blockIdx.y;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= W2 * W2) return;
    if ((e % W2) / 16 < (e / W2) / 16) {       // upper tiles: not formed, left at zero
        gram[(size_t)pm * (W2 * W2) + e] = d2{0.0, 0.0};
        return;
    }
    const d2 *src = part + (size_t)pm * splits * (W2 * W2) + e;
    d2 v[MAXS];
#pragma unroll
    for (int s = 0; s < MAXS; ++s)
        if (s < splits) v[s] = src[(size_t)s * (W2 * W2)];
    d2 acc = v[0];
#pragma unroll
    for (int s = 1; s < MAXS; ++s)
        if (s < splits) acc += v[s];
    gram[(size_t)pm * (W2 * W2) + e] = acc;
}

// Inner solve of one complex pivot block pair: Hermitian Cholesky
// (A_hat = F_hat^H F_hat), factor prescale, inner sweeps of the complex
// pointwise method (Section 2.1.1), Theta rescale (Section 2.4).  Layout and
// phases as the real k_inner; columns of F_hat, G_hat, Z_hat are
// interleaved complex in LDS.
template <int W2, int LP, bool RING>
__global__ __launch_bounds__((W2 / 2) * LP) void k_inner_z(
    const d2 *__restrict__ gram, int factors, int npairs, int step,
    const int16_t *__restrict__ itab, int isteps, int inner_max, double tol, int sort, int variant,
    d2 *__restrict__ Zt, unsigned long long *__restrict__ cnt, int *__restrict__ status,
    unsigned long long *__restrict__ phase)
{
    constexpr int W = W2 / 2;
    constexpr int NT = W * LP;
    constexpr int RPL = W2 / LP;
    constexpr int LDI = W2 + 1;
    static_assert(RPL >= 1 && NT >= 64 && W2 <= 32, "bad complex inner geometry");
    __shared__ d2 sF[W2 * LDI];
    __shared__ d2 sG[W2 * LDI];
    __shared__ d2 sZ[W2 * LDI];
    __shared__ int16_t stab[W2 * W2];
    __shared__ d2 lbuf[2][32];
    __shared__ int s_fail;
    __shared__ unsigned s_cnt[2 * W];

    const int pr = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned long long *myc = cnt + ((size_t)step * npairs + pr) * 4;
    // with `phase`, the wall clock at the boundaries of the phases (load,
    // Cholesky, prescale, inner sweeps, Theta and store)
    unsigned long long *const ph = phase ? phase + ((size_t)step * npairs + pr) * 8 : nullptr;
    if (ph && tid == 0) ph[0] = wall_clock64();
    {
        // every load of a thread issued before the first store, so the
        // phase costs one memory latency
        const d2 *pa = gram + (size_t)(pr * 2) * (W2 * W2);
        const d2 *pb = pa + (W2 * W2);
        constexpr int NIT = (W2 * W2) / NT;
        static_assert(NIT * NT == W2 * W2, "Gram load geometry");
        d2 va[NIT], vb[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            va[it] = pa[tid + NT * it];
            vb[it] = pb[tid + NT * it];
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int e = tid + NT * it, col = e / W2, row = e % W2;
            sF[col * LDI + row] = va[it];
            sG[col * LDI + row] = vb[it];
        }
        if (!RING) copy_table<NT>(stab, itab, isteps * W * 2);   // the ring needs no table
        if (tid == 0) s_fail = 0;
    }
    __syncthreads();
    if (ph && tid == 0) ph[1] = wall_clock64();

    // Hermitian Cholesky, lane = row, A in lanes 0..31 and B in 32..63 of wave 0.
    // With `factors` the blocks are already the upper triangular factors (QR
    // of the block-column pairs, real diagonal): only the diagonals are
    // checked for zeros and non-finite values.
    if (factors) {
        if (tid < W2) {
            const double df = sF[tid * LDI + tid][0], dg = sG[tid * LDI + tid][0];
            if (!(fabs(df) > 0.0 && fabs(df) < INFINITY && fabs(dg) > 0.0 && fabs(dg) < INFINITY))
                s_fail = 1;
        }
    } else {
        const int mat = lane >> 5, i = lane & 31;
        if (wave == 0 && i < W2) {
            d2 *M = mat ? sG : sF;
            d2 *lb = lbuf[mat];
            d2 a[W2];
#pragma unroll
            for (int k = 0; k < W2; ++k) a[k] = M[k * LDI + i];
            const double d0 = M[i * LDI + i][0];   // column i's diagonal before the factorization
            double own = 1.0;                        // the pivot of column i, kept by lane i
#pragma unroll
            for (int j = 0; j < W2; ++j) {
                const double p0 = readlane_d(a[j][0], j), p1 = readlane_d(a[j][0], 32 + j);
                const double piv = mat ? p1 : p0;
                if (i == j) own = a[j][0];
                const double inv = rsqrt_nr(piv);
                d2 l = (i > j) ? a[j] * inv : d2{0.0, 0.0};
                if (i == j) l = d2{piv * inv, 0.0};
                a[j] = l;
                lb[i] = l;
                wave_fence();
#pragma unroll
                for (int k = j + 1; k < W2; ++k) {
                    const d2 lk = lb[k];
                    // a[k] -= l * conj(lk)
                    a[k][0] = fma(-l[0], lk[0], fma(-l[1], lk[1], a[k][0]));
                    a[k][1] = fma(-l[1], lk[0], fma(l[0], lk[1], a[k][1]));
                }
                wave_fence();
            }
            // F_hat = L^H: column i of F_hat is the conjugate of row i of L.
#pragma unroll
            for (int k = 0; k < W2; ++k)
                M[i * LDI + k] = (k <= i) ? d2{a[k][0], -a[k][1]} : d2{0.0, 0.0};
            // numerically positive definite: every pivot above W2 * eps times
            // its column's diagonal, each tested by the lane that holds it
            if (!((own > W2 * 2.220446049250313e-16 * d0) && (own < INFINITY))) s_fail = 1;
        }
    }
    __syncthreads();
    if (ph && tid == 0) ph[2] = wall_clock64();
    if (s_fail) {
        d2 *zt = Zt + (size_t)pr * (W2 * W2);
        for (int e = tid; e < W2 * W2; e += NT)
            zt[e] = (e % W2 == e / W2) ? d2{1.0, 0.0} : d2{0.0, 0.0};
        if (tid == 0) {
            myc[0] = 0;
            myc[1] = 0;
            myc[2] = 0;
            myc[3] = 0;
            atomicOr(status + ST_FLAGS, FLAG_CHOL);
            atomicMin(status + ST_FAILPAIR, step * 65536 + pr);
        }
        return;
    }

    const int grp = tid / LP, gl = tid % LP, r0 = gl * RPL;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = 2 * grp + h;
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const d2 g = sG[c * LDI + r0 + r];
            s = fma(g[0], g[0], fma(g[1], g[1], s));
        }
        s = dpp_group_sum<LP>(s);
        const double d = rsqrt_nr(s);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            sF[c * LDI + r0 + r] *= d;
            sG[c * LDI + r0 + r] *= d;
            sZ[c * LDI + r0 + r] = (r0 + r == c) ? d2{d, 0.0} : d2{0.0, 0.0};
        }
    }
    __syncthreads();
    if (ph && tid == 0) ph[3] = wall_clock64();

    const double tol2 = tol * tol;
    unsigned my_all = 0, my_big = 0, my_chg = 0;
    int nsw = 0;
    for (int sw = 0; sw < inner_max; ++sw) {
        unsigned sw_all = 0, sw_big = 0;
        ++nsw;
        // One pointwise step on column pair (i, j), i < j, held in registers:
        // the complex pivot entries, the orthogonality test, the 2x2
        // transformation of Section 2.1.1, criterion C1 (C2), the sorting
        // swap, and [y_i y_j] <- [y_i y_j] Z' applied to the arrays.  Returns
        // whether the columns changed.
        auto pair_step = [&](d2 (&fi)[RPL], d2 (&fj)[RPL], d2 (&gi)[RPL], d2 (&gj)[RPL],
                             d2 (&zi)[RPL], d2 (&zj)[RPL]) -> bool {
            double aii = 0.0, ajj = 0.0, ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
            if (variant & 1) {
                // variants 1 and 5: squared norms by the enhanced procedure
                // of Appendix A (the off-diagonal entries stay ordinary)
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    aii += enh_abs2(fi[r][0], fi[r][1]);
                    ajj += enh_abs2(fj[r][0], fj[r][1]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    aii = fma(fi[r][0], fi[r][0], fma(fi[r][1], fi[r][1], aii));
                    ajj = fma(fj[r][0], fj[r][0], fma(fj[r][1], fj[r][1], ajj));
                }
            }
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                ar = fma(fi[r][0], fj[r][0], fma(fi[r][1], fj[r][1], ar));
                ai = fma(fi[r][0], fj[r][1], fma(-fi[r][1], fj[r][0], ai));
                br = fma(gi[r][0], gj[r][0], fma(gi[r][1], gj[r][1], br));
                bi = fma(gi[r][0], gj[r][1], fma(-gi[r][1], gj[r][0], bi));
            }
            aii = dpp_group_sum<LP>(aii);
            ajj = dpp_group_sum<LP>(ajj);
            ar = dpp_group_sum<LP>(ar);
            ai = dpp_group_sum<LP>(ai);
            br = dpp_group_sum<LP>(br);
            bi = dpp_group_sum<LP>(bi);
            double z11 = 1.0, z22 = 1.0, z21r = 0.0, z21i = 0.0, z12r = 0.0, z12i = 0.0;
            bool swap;
            const bool orth = (fma(ar, ar, ai * ai) < aii * ajj * tol2) &&
                              (fma(br, br, bi * bi) < tol2);
            if (orth) {
                swap = sort && (aii < ajj);
            } else {
                bool c2small;
                hz_cplx_2x2_fast(aii, ajj, ar, ai, br, bi, z11, z21r, z21i, z12r, z12i, z22,
                                 c2small);
                sw_all += 1;
                // small: criterion C1 (variants 0, 1) or C2 (variants 4, 5), Section 2.5
                if ((variant & 4) ? !c2small : !(z11 == 1.0 && z22 == 1.0)) sw_big += 1;
                swap = false;
                if (sort) {
                    // diagonal of Z^H A Z
                    const double a11 = fma(z11 * z11, aii,
                                           fma(2.0 * z11, fma(ar, z21r, -ai * z21i),
                                               fma(z21r, z21r, z21i * z21i) * ajj));
                    const double a22 = fma(fma(z12r, z12r, z12i * z12i), aii,
                                           fma(2.0 * z22, fma(z12r, ar, z12i * ai),
                                               z22 * z22 * ajj));
                    swap = a11 < a22;
                }
            }
            if (!(!orth || swap)) return false;
            my_chg = 1;
            // [y_i y_j] <- [y_i y_j] Z (z11, z22 real), then the sorting swap
            auto rot = [&](d2 &yi, d2 &yj) {
                d2 a, b;
                a[0] = fma(yi[0], z11, fma(yj[0], z21r, -yj[1] * z21i));
                a[1] = fma(yi[1], z11, fma(yj[0], z21i, yj[1] * z21r));
                b[0] = fma(yj[0], z22, fma(yi[0], z12r, -yi[1] * z12i));
                b[1] = fma(yj[1], z22, fma(yi[0], z12i, yi[1] * z12r));
                yi = swap ? b : a;
                yj = swap ? a : b;
            };
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                rot(fi[r], fj[r]);
                rot(gi[r], gj[r]);
                rot(zi[r], zj[r]);
            }
            return true;
        };
        auto load = [&](const d2 *M, int c, d2 (&x)[RPL]) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) x[r] = M[c * LDI + r0 + r];
        };
        auto store = [&](d2 *M, int c, const d2 (&x)[RPL]) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) M[c * LDI + r0 + r] = x[r];
        };
        if constexpr (RING) {
            // the ring ordering of the real solver (HZ_ORD_RING): the first
            // column of a pair stays in registers for a level, the second
            // half of the block is visited in-wave between phase barriers
            constexpr int GW = 64 / LP;
            for (int h = W; h >= 1; h >>= 1) {
                const int blk = grp / h, u = grp % h;
                const int ci = blk * 2 * h + u;
                const int nset = (h >= GW) ? h / GW : 1, ssz = (h >= GW) ? GW : h;
                const int ow = u / ssz, gw = u % ssz;
                d2 fi[RPL], gi[RPL], zi[RPL];
                load(sF, ci, fi);
                load(sG, ci, gi);
                load(sZ, ci, zi);
                for (int p = 0; p < nset; ++p) {
                    for (int t = 0; t < ssz; ++t) {
                        const int cj = blk * 2 * h + h + ring_col(ssz, nset, ow, gw, p, t);
                        d2 fj[RPL], gj[RPL], zj[RPL];
                        load(sF, cj, fj);
                        load(sG, cj, gj);
                        load(sZ, cj, zj);
                        if (pair_step(fi, fj, gi, gj, zi, zj)) {
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
                d2 fi[RPL], fj[RPL], gi[RPL], gj[RPL], zi[RPL], zj[RPL];
                load(sF, ci, fi);
                load(sF, cj, fj);
                load(sG, ci, gi);
                load(sG, cj, gj);
                load(sZ, ci, zi);
                load(sZ, cj, zj);
                if (pair_step(fi, fj, gi, gj, zi, zj)) {
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
        const int any = __syncthreads_count(gl == 0 && sw_all > 0);
        if (any == 0) break;
    }

    if (ph && tid == 0) ph[4] = wall_clock64();
    // Z_tilde = Z_hat Theta, or exactly I when nothing was transformed or
    // swapped (the block update is then skipped, Section 2.5)
    d2 *zt = Zt + (size_t)pr * (W2 * W2);
    const int nchg = __syncthreads_count(gl == 0 && my_chg != 0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = 2 * grp + h;
        if (nchg == 0) {
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                zt[c * W2 + r0 + r] = d2{(r0 + r == c) ? 1.0 : 0.0, 0.0};
            continue;
        }
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const d2 f = sF[c * LDI + r0 + r], g = sG[c * LDI + r0 + r];
            s = fma(f[0], f[0], fma(f[1], f[1], s));
            s = fma(g[0], g[0], fma(g[1], g[1], s));
        }
        s = dpp_group_sum<LP>(s);
        const double th = rsqrt_nr(s);
#pragma unroll
        for (int r = 0; r < RPL; ++r) zt[c * W2 + r0 + r] = sZ[c * LDI + r0 + r] * th;
    }
    if (gl == 0) {
        s_cnt[2 * grp] = my_all;
        s_cnt[2 * grp + 1] = my_big;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long ta = 0, tb = 0;
        for (int g = 0; g < W; ++g) {
            ta += s_cnt[2 * g];
            tb += s_cnt[2 * g + 1];
        }
        myc[0] = ta;
        myc[1] = tb;
        myc[2] = (unsigned long long)nsw;
        myc[3] = (nchg == 0) ? 1ull : 0ull;
        if (ph) ph[5] = wall_clock64();
    }
}

// Complex block update [Y_p Y_q] <- [Y_p Y_q] Z_tilde in place
// (Section 2.3, Section 3.5.4): D' = Z_tilde^T X^T with
// Re = Zr^T Xr^T - Zi^T Xi^T, Im = Zi^T Xr^T + Zr^T Xi^T on FP64 MFMA.
// The rows of F, G and Z (each padded to a multiple of 64) are taken as one
// sequence cut into equal workgroup ranges of 4 * rows_per_wave; a 16-row
// tile never straddles two matrices, and its matrix is chosen per tile.
template <int W2>
__global__ __launch_bounds__(256) void k_update_z(d2 *__restrict__ Fw, d2 *__restrict__ Gw,
                                                  d2 *__restrict__ Zw, int64_t mfw, int64_t mgw,
                                                  int64_t nzw, const int *__restrict__ pairs,
                                                  const d2 *__restrict__ Zt, int rows_per_wave,
                                                  const unsigned long long *__restrict__ scnt)
{
    constexpr int W = W2 / 2, NB = W2 / 16, KS = W2 / 4, LDZ = W2 + 1;
    __shared__ d2 sz[W2 * LDZ];
    const int pr = blockIdx.y;
    if (scnt[(size_t)pr * 4 + 3]) return;   // Z_tilde = I: nothing to update
    const int p = pairs[2 * pr], q = pairs[2 * pr + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const d2 *zt = Zt + (size_t)pr * (W2 * W2);
    {
        // every load of a thread issued before the first store
        constexpr int NZ = (W2 * W2) / 256;
        static_assert(NZ * 256 == W2 * W2, "Z_tilde staging geometry");
        d2 zv[NZ];
#pragma unroll
        for (int it = 0; it < NZ; ++it) zv[it] = zt[tid + 256 * it];
#pragma unroll
        for (int it = 0; it < NZ; ++it) {
            const int e = tid + 256 * it;
            sz[(e / W2) * LDZ + (e % W2)] = zv[it];
        }
    }
    const int64_t span = 4 * (int64_t)rows_per_wave;
    const int64_t vb = (int64_t)blockIdx.x * span, total = mfw + mgw + nzw;
    const int64_t ve = (vb + span < total) ? vb + span : total;
    __syncthreads();
    const int k4 = lane >> 4, i16 = lane & 15;
    for (int64_t v0 = vb + 16 * wave; v0 < ve; v0 += 64) {
        __asm__ volatile("" ::: "memory");
        d2 *Y;
        int64_t m, r0;
        if (v0 < mfw) {
            Y = Fw;
            m = mfw;
            r0 = v0;
        } else if (v0 < mfw + mgw) {
            Y = Gw;
            m = mgw;
            r0 = v0 - mfw;
        } else {
            Y = Zw;
            m = nzw;
            r0 = v0 - mfw - mgw;
        }
        d2 *bp = Y + ((int64_t)p * W + k4) * m + i16;
        d2 *bq = Y + ((int64_t)q * W + k4) * m + i16;
        d2 xb[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s)
            xb[s] = (4 * s < W) ? bp[(int64_t)(4 * s) * m + r0] : bq[(int64_t)(4 * s - W) * m + r0];
        d4 accr[NB], acci[NB];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
            accr[jb] = d4{0.0, 0.0, 0.0, 0.0};
            acci[jb] = d4{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const d2 za = sz[(16 * jb + i16) * LDZ + 4 * s + k4];
                accr[jb] = mfma16(za[0], xb[s][0], accr[jb]);
                accr[jb] = mfma16(-za[1], xb[s][1], accr[jb]);
                acci[jb] = mfma16(za[1], xb[s][0], acci[jb]);
                acci[jb] = mfma16(za[0], xb[s][1], acci[jb]);
            }
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c0 = 16 * jb + 4 * r;
                d2 *dst = (c0 < W) ? bp + (int64_t)c0 * m + r0 : bq + (int64_t)(c0 - W) * m + r0;
                *dst = d2{accr[jb][r], acci[jb][r]};
            }
    }
}

// Extraction (Section 2.4, Section 3.4): norms and bordering flags.
__global__ __launch_bounds__(256) void k_colnorms_z(const d2 *__restrict__ Fw,
                                                    const d2 *__restrict__ Gw,
                                                    const d2 *__restrict__ Zw, int64_t mfw,
                                                    int64_t mgw, int64_t nzw, int64_t n,
                                                    int64_t nw, double *__restrict__ sf,
                                                    double *__restrict__ sg,
                                                    double *__restrict__ sig,
                                                    int *__restrict__ border,
                                                    int *__restrict__ status)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nw) return;
    const d2 *f = Fw + j * mfw, *g = Gw + j * mgw, *z = Zw + j * nzw;
    double a = 0.0, b = 0.0;
    for (int64_t r = lane; r < mfw; r += 64) a = fma(f[r][0], f[r][0], fma(f[r][1], f[r][1], a));
    for (int64_t r = lane; r < mgw; r += 64) b = fma(g[r][0], g[r][0], fma(g[r][1], g[r][1], b));
    int bz = 0;
    for (int64_t r = n + lane; r < nw; r += 64) bz |= (z[r][0] != 0.0 || z[r][1] != 0.0);
    a = wave_sum(a);
    b = wave_sum(b);
    const int isb = __any(bz) ? 1 : 0;
    if (lane == 0) {
        const double x = sqrt(a), y = sqrt(b);
        sf[j] = x;
        sg[j] = y;
        sig[j] = x / y;
        border[j] = isb;
        if (!isb && !(isfinite(x / y) && x > 0.0 && y > 0.0)) atomicOr(status + ST_FLAGS, FLAG_NONFINITE);
    }
}

__global__ __launch_bounds__(256) void k_scatter_z(
    const d2 *__restrict__ Fw, const d2 *__restrict__ Gw, const d2 *__restrict__ Zw, int64_t mfw,
    int64_t mgw, int64_t nzw, int64_t mf, int64_t mg, int64_t n, int64_t nw,
    const double *__restrict__ sf, const double *__restrict__ sg, const int *__restrict__ rank,
    d2 *__restrict__ U, int64_t ldu, d2 *__restrict__ V, int64_t ldv, d2 *__restrict__ Z,
    int64_t ldz, double *__restrict__ sigma, double *__restrict__ sigma_f,
    double *__restrict__ sigma_g)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nw) return;
    const int rk = rank[j];
    if (rk < 0 || rk >= n) return;
    const double x = sf[j], y = sg[j];
    const double th = 1.0 / sqrt(x * x + y * y);
    const double ix = 1.0 / x, iy = 1.0 / y;
    const d2 *f = Fw + j * mfw, *g = Gw + j * mgw, *z = Zw + j * nzw;
    d2 *u = U + (int64_t)rk * ldu, *v = V + (int64_t)rk * ldv, *zo = Z + (int64_t)rk * ldz;
    for (int64_t r = lane; r < mf; r += 64) u[r] = f[r] * ix;
    for (int64_t r = lane; r < mg; r += 64) v[r] = g[r] * iy;
    for (int64_t r = lane; r < n; r += 64) zo[r] = z[r] * th;
    if (lane == 0) {
        sigma[rk] = x / y;
        sigma_f[rk] = x * th;
        sigma_g[rk] = y * th;
    }
}

// n = 1 closed form (Section 2), complex.
__global__ __launch_bounds__(64) void k_n1_z(int64_t mf, int64_t mg, d2 *__restrict__ F,
                                             d2 *__restrict__ G, d2 *__restrict__ Z,
                                             double *__restrict__ sigma,
                                             double *__restrict__ sigma_f,
                                             double *__restrict__ sigma_g,
                                             int *__restrict__ status)
{
    const int lane = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t r = lane; r < mf; r += 64) a = fma(F[r][0], F[r][0], fma(F[r][1], F[r][1], a));
    for (int64_t r = lane; r < mg; r += 64) b = fma(G[r][0], G[r][0], fma(G[r][1], G[r][1], b));
    a = wave_sum(a);
    b = wave_sum(b);
    const double nf = sqrt(a), ng = sqrt(b), rr = sqrt(a + b);
    for (int64_t r = lane; r < mf; r += 64) F[r] = F[r] / nf;
    for (int64_t r = lane; r < mg; r += 64) G[r] = G[r] / ng;
    if (lane == 0) {
        Z[0] = d2{1.0 / rr, 0.0};
        sigma[0] = nf / ng;
        sigma_f[0] = nf / rr;
        sigma_g[0] = ng / rr;
        if (!(isfinite(nf / ng) && nf > 0.0 && ng > 0.0)) atomicOr(status + ST_FLAGS, FLAG_NONFINITE);
    }
}

// Diagnostic evaluation of hz_cplx_2x2_fast: in rows (aii, ajj, ar, ai, br,
// bi), out rows (z11, z21r, z21i, z12r, z12i, z22).
__global__ __launch_bounds__(256) void k_eval_2x2_z(int64_t count, const double *__restrict__ in,
                                                    double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const double *a = in + 6 * i;
    double *o = out + 6 * i;
    bool c2small;
    hz_cplx_2x2_fast(a[0], a[1], a[2], a[3], a[4], a[5], o[0], o[1], o[2], o[3], o[4], o[5],
                     c2small);
}

// ------------------------------------------------------------------ launchers

void launch_prescale_cplx(const Plan &P, const Ptrs &W, const double *F, int64_t ldf,
                          const double *G, int64_t ldg, hipStream_t s)
{
    const unsigned nb = (unsigned)((P.nw + 3) / 4);
    hipLaunchKernelGGL(k_prescale_copy_z, dim3(nb), dim3(256), 0, s, P.mf, P.mg, P.n,
                       (const d2 *)F, ldf, (const d2 *)G, ldg, P.nw, P.mfw, P.mgw, P.nzw,
                       (d2 *)W.Fw, (d2 *)W.Gw, (d2 *)W.Zw, W.status);
}

template <int W2>
static void step_impl_z(const Plan &P, const Ptrs &W, int step, const hz_params &prm,
                        double tol, hipStream_t s)
{
    const int *pairs = W.otab + (size_t)step * P.npairs * 2;
    prof_mark(K_GRAM, true, s);
    const int fac = prm.pivot_qr ? 1 : 0;
    if (fac) {
        launch_pivot_qr(P, W, step, s);
    } else {
        hipLaunchKernelGGL(k_gram_z<W2>, dim3(P.splits, P.npairs, 2), dim3(256), 0, s,
                           (const d2 *)W.Fw, (const d2 *)W.Gw, P.mfw, P.mgw, pairs, P.splits,
                           (d2 *)W.part);
        hipLaunchKernelGGL(k_gram_sum_z<W2>, dim3((W2 * W2 + 255) / 256, 2 * P.npairs),
                           dim3(256), 0, s, (const d2 *)W.part, P.splits, (d2 *)W.gram);
    }
    prof_mark(K_GRAM, false, s);
    prof_mark(K_INNER, true, s);
    const bool ring = (prm.inner_ordering == HZ_ORD_RING);
    auto go = [&](auto kern, int lp) {
        hipLaunchKernelGGL(kern, dim3(P.npairs), dim3((W2 / 2) * lp), 0, s, (const d2 *)W.gram,
                           fac, P.npairs, step, W.itab, P.isteps, prm.inner_max_sweeps, tol,
                           prm.sort, prm.variant, (d2 *)W.Zt, W.cnt, W.status, W.phase);
    };
    if (W2 == 32 && P.inner_lp == 16) {
        if (ring) go(k_inner_z<W2, 16, true>, 16);
        else go(k_inner_z<W2, 16, false>, 16);
    } else {
        if (ring) go(k_inner_z<W2, 8, true>, 8);
        else go(k_inner_z<W2, 8, false>, 8);
    }
    prof_mark(K_INNER, false, s);
    const int64_t rpt = 4 * (int64_t)P.upd_rows;
    const int nt = (int)((P.mfw + P.mgw + P.nzw + rpt - 1) / rpt);
    prof_mark(K_UPDATE, true, s);
    hipLaunchKernelGGL(k_update_z<W2>, dim3(nt, P.npairs), dim3(256), 0, s, (d2 *)W.Fw,
                       (d2 *)W.Gw, (d2 *)W.Zw, P.mfw, P.mgw, P.nzw, pairs, (const d2 *)W.Zt,
                       P.upd_rows, W.cnt + (size_t)step * P.npairs * 4);
    prof_mark(K_UPDATE, false, s);
}

void launch_step_cplx(const Plan &P, const Ptrs &W, int step, const hz_params &prm, double tol,
                      hipStream_t s)
{
    if (P.W2 == 16) step_impl_z<16>(P, W, step, prm, tol, s);
    else step_impl_z<32>(P, W, step, prm, tol, s);
}

void launch_finish_cplx(const Plan &P, const Ptrs &W, double *F, int64_t ldf, double *G,
                        int64_t ldg, double *Z, int64_t ldz, double *sigma, double *sigma_f,
                        double *sigma_g, hipStream_t s)
{
    const unsigned nb4 = (unsigned)((P.nw + 3) / 4);
    hipLaunchKernelGGL(k_colnorms_z, dim3(nb4), dim3(256), 0, s, (const d2 *)W.Fw,
                       (const d2 *)W.Gw, (const d2 *)W.Zw, P.mfw, P.mgw, P.nzw, P.n, P.nw, W.sf,
                       W.sg, W.sig, W.border, W.status);
    launch_rank(P, W, s);
    hipLaunchKernelGGL(k_scatter_z, dim3(nb4), dim3(256), 0, s, (const d2 *)W.Fw,
                       (const d2 *)W.Gw, (const d2 *)W.Zw, P.mfw, P.mgw, P.nzw, P.mf, P.mg, P.n,
                       P.nw, W.sf, W.sg, W.rank, (d2 *)F, ldf, (d2 *)G, ldg, (d2 *)Z, ldz, sigma,
                       sigma_f, sigma_g);
}

void launch_n1_cplx(int64_t mf, int64_t mg, double *F, double *G, double *Z, double *sigma,
                    double *sigma_f, double *sigma_g, int *status, hipStream_t s)
{
    hipLaunchKernelGGL(k_n1_z, dim3(1), dim3(64), 0, s, mf, mg, (d2 *)F, (d2 *)G, (d2 *)Z, sigma,
                       sigma_f, sigma_g, status);
}

void launch_eval_2x2_cplx(int64_t count, const double *in, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_eval_2x2_z, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       count, in, out);
}

}  // namespace hz
