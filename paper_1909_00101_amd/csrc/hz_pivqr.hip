// hz_pivqr.hip -- pivot factors from QR factorizations of the block-column
// pairs instead of Gram matrices and their Cholesky factorizations (paper,
// Section 2.3, and Appendix E: for ill-conditioned pairs the Grams of the
// block-column pairs can be numerically indefinite, and the pairs are then
// shortened by QR).  With R the triangular factor of [Y_p Y_q] = Q R,
// R^T R is the pivot Gram, so R takes the place of the Cholesky factor; Q
// is never formed.
//
// Tall-skinny QR as a reduction tree: every workgroup factors one tile of
// 2 * W2 rows and W2 columns with Householder reflections (the tile in
// registers, the reflectors through LDS) and writes its W2 x W2 triangle;
// the leaves are consecutive row chunks of [Y_p Y_q], each further level
// factors two stacked triangles of the level below, until one triangle per
// block pair and matrix is left.  All pivot pairs of
// a step, F and G, go in one launch per level.  The factor is not squared,
// so a block pair whose columns are independent to working accuracy gets a
// usable factor where its Gram would lose half the digits.
#include <math.h>

#include "hz_device.h"
#include "hz_internal.h"

namespace hz {

// One level of the tree.  Level 0 reads rows [c * 2W2, (c + 1) * 2W2) of
// the block columns p, q of Fw (matrix 0) or Gw (matrix 1); a further level
// reads the triangles 2c and 2c + 1 of the level below (a missing second
// one is zero).  Triangles are column-major W2 x W2 with zeros below the
// diagonal, at out + ((pair * 2 + matrix) * out_stride + node) * W2 * W2.
struct QRLevel {
    const double *Fw, *Gw;
    int64_t mfw, mgw;
    const int *pairs;          // this step's (p, q) per pivot pair
    const double *in;          // triangles of the level below (levels > 0)
    double *out;
    int in_stride, out_stride; // triangles per (pair, matrix) in `in` / `out`
    int nodes_f, nodes_g;      // tiles of this level per matrix
    int prev_f, prev_g;        // triangles of the level below per matrix
    int level;
};

// Thread t owns column t / Q of the tile, rows t % Q, t % Q + Q, ... (RPQ
// of them) in registers.  Step k: the Q owners of column k form the
// reflector H = I - tau v v^H (v_k = 1) with H^H x = (beta, 0, ..., 0),
// beta real (for real data the transpose and a real tau), and publish v and
// tau in LDS (two buffers, so one barrier per step); the owners of the
// columns right of k apply H^H = I - conj(tau) v v^H to their rows.  Sums
// over a column use a fixed reduction order: four interleaved partial sums
// per thread (two for complex), then the Q threads' sums by DPP.  Complex elements are
// interleaved (CX).
template <int W2, bool CX>
__global__ __launch_bounds__(256) void k_qr_tile(QRLevel a)
{
    constexpr int CH = 2 * W2;          // tile rows
    constexpr int NT = 256;
    constexpr int Q = NT / W2;          // threads per column
    constexpr int RPQ = CH / Q;         // rows per thread
    constexpr int NP = CX ? 2 : 1;      // planes (real, imaginary)
    static_assert(Q >= 1 && (64 % Q) == 0 && RPQ % 2 == 0, "bad QR tile geometry");
    __shared__ double s_v[2][NP][CH];
    __shared__ double s_tau[2][NP];
    const int mt = blockIdx.z, l = blockIdx.y, c = blockIdx.x;
    if (c >= (mt ? a.nodes_g : a.nodes_f)) return;   // uniform: the grid covers the larger
    const int tid = threadIdx.x;
    const int jc = tid / Q, q = tid % Q;
    double x[NP][RPQ];
    if (a.level == 0) {
        const double *__restrict__ Y = mt ? a.Gw : a.Fw;
        const int64_t m = mt ? a.mgw : a.mfw;
        const int W = W2 / 2;
        const int p = a.pairs[2 * l], qq = a.pairs[2 * l + 1];
        const int64_t gc = (jc < W) ? (int64_t)p * W + jc : (int64_t)qq * W + (jc - W);
        const double *col = Y + NP * gc * m;
#pragma unroll
        for (int i = 0; i < RPQ; ++i) {
            const int64_t gr = (int64_t)c * CH + q + Q * i;
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) x[pl][i] = (gr < m) ? col[NP * gr + pl] : 0.0;
        }
    } else {
        const int prev = mt ? a.prev_g : a.prev_f;
        const double *__restrict__ ra =
            a.in + NP * (((size_t)l * 2 + mt) * a.in_stride + 2 * (size_t)c) * (W2 * W2);
        const bool second = 2 * c + 1 < prev;
#pragma unroll
        for (int i = 0; i < RPQ; ++i) {
            const int r = q + Q * i;
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) {
                double v = 0.0;
                if (r < W2) v = ra[NP * (jc * W2 + r) + pl];
                else if (second) v = ra[NP * (W2 * W2 + jc * W2 + (r - W2)) + pl];
                x[pl][i] = v;
            }
        }
    }
    for (int k = 0; k < W2; ++k) {
        const int par = k & 1;
        if (jc == k) {
            double s4[4] = {0.0, 0.0, 0.0, 0.0}, al[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) al[pl] = 0.0;
#pragma unroll
            for (int i = 0; i < RPQ; ++i) {
                const int r = q + Q * i;
                if (r > k) {
#pragma unroll
                    for (int pl = 0; pl < NP; ++pl) s4[i & 3] = fma(x[pl][i], x[pl][i], s4[i & 3]);
                }
                if (r == k) {
#pragma unroll
                    for (int pl = 0; pl < NP; ++pl) al[pl] = x[pl][i];
                }
            }
            // the Q owners of the column are Q consecutive lanes
            const double sq = dpp_group_sum<Q>((s4[0] + s4[1]) + (s4[2] + s4[3]));
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) al[pl] = dpp_group_sum<Q>(al[pl]);   // exact: one term
            const double ali = CX ? al[NP - 1] : 0.0;
            double beta = al[0], tau[NP], scale[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) tau[pl] = scale[pl] = 0.0;
            if (sq > 0.0 || ali != 0.0) {
                beta = -copysign(sqrt(fma(al[0], al[0], fma(ali, ali, sq))), al[0]);
                tau[0] = (beta - al[0]) / beta;
                if constexpr (CX) {
                    tau[NP - 1] = -ali / beta;
                    // 1 / (alpha - beta)
                    const double dr = al[0] - beta, di = ali;
                    const double den = fma(dr, dr, di * di);
                    scale[0] = dr / den;
                    scale[NP - 1] = -di / den;
                } else {
                    scale[0] = 1.0 / (al[0] - beta);
                }
            }
#pragma unroll
            for (int i = 0; i < RPQ; ++i) {
                const int r = q + Q * i;
                if constexpr (CX) {
                    double vr = 0.0, vi = 0.0;
                    if (r == k) vr = 1.0;
                    else if (r > k) {
                        vr = x[0][i] * scale[0] - x[NP - 1][i] * scale[NP - 1];
                        vi = x[0][i] * scale[NP - 1] + x[NP - 1][i] * scale[0];
                    }
                    s_v[par][0][r] = vr;
                    s_v[par][NP - 1][r] = vi;
                    if (r == k) {
                        x[0][i] = beta;
                        x[NP - 1][i] = 0.0;
                    }
                } else {
                    s_v[par][0][r] = (r == k) ? 1.0 : ((r > k) ? x[0][i] * scale[0] : 0.0);
                    if (r == k) x[0][i] = beta;
                }
            }
            if (q == 0) {
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) s_tau[par][pl] = tau[pl];
            }
        }
        __syncthreads();
        const double tr = s_tau[par][0], ti = CX ? s_tau[par][NP - 1] : 0.0;
        if ((tr != 0.0 || ti != 0.0) && jc > k) {
            if constexpr (CX) {
                // w = v^H a_j, then a_j -= conj(tau) w v
                double wr0 = 0.0, wr1 = 0.0, wi0 = 0.0, wi1 = 0.0;
#pragma unroll
                for (int i = 0; i < RPQ; i += 2) {
                    const int r = q + Q * i, r1 = q + Q * (i + 1);
                    const double v0r = s_v[par][0][r], v0i = s_v[par][NP - 1][r];
                    const double v1r = s_v[par][0][r1], v1i = s_v[par][NP - 1][r1];
                    wr0 = fma(v0r, x[0][i], fma(v0i, x[NP - 1][i], wr0));
                    wi0 = fma(v0r, x[NP - 1][i], fma(-v0i, x[0][i], wi0));
                    wr1 = fma(v1r, x[0][i + 1], fma(v1i, x[NP - 1][i + 1], wr1));
                    wi1 = fma(v1r, x[NP - 1][i + 1], fma(-v1i, x[0][i + 1], wi1));
                }
                const double wr = dpp_group_sum<Q>(wr0 + wr1), wi = dpp_group_sum<Q>(wi0 + wi1);
                const double cr = tr * wr + ti * wi, ci = tr * wi - ti * wr;   // conj(tau) w
#pragma unroll
                for (int i = 0; i < RPQ; ++i) {
                    const int r = q + Q * i;
                    const double vr = s_v[par][0][r], vi = s_v[par][NP - 1][r];
                    x[0][i] -= cr * vr - ci * vi;
                    x[NP - 1][i] -= cr * vi + ci * vr;
                }
            } else {
                double w4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int i = 0; i < RPQ; ++i) w4[i & 3] = fma(s_v[par][0][q + Q * i], x[0][i], w4[i & 3]);
                const double w = dpp_group_sum<Q>((w4[0] + w4[1]) + (w4[2] + w4[3]));
                const double tw = tr * w;
#pragma unroll
                for (int i = 0; i < RPQ; ++i) x[0][i] = fma(-tw, s_v[par][0][q + Q * i], x[0][i]);
            }
        }
    }
    double *__restrict__ R = a.out + NP * (((size_t)l * 2 + mt) * a.out_stride + c) * (W2 * W2);
#pragma unroll
    for (int i = 0; i < RPQ; ++i) {
        const int r = q + Q * i;
        if (r < W2) {
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) R[NP * (jc * W2 + r) + pl] = (r <= jc) ? x[pl][i] : 0.0;
        }
    }
}

// Sum over the 64 lanes of a wave in a fixed order (16-lane rows by DPP,
// then the four row sums as (r0 + r1) + (r2 + r3)); every lane gets it.
__device__ __forceinline__ double wave_total(double v)
{
    v = dpp_group_sum<16>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// The same tree for real pivot blocks of order 64 with wider nodes: a
// workgroup of 16 waves factors 512 rows (level 0: rows [c * 512,
// (c + 1) * 512) of the block columns; a further level: the triangles
// 8c .. 8c + 7 of the level below stacked, missing ones zero), so 4096 rows
// take two levels.  Wave g owns columns 4g .. 4g + 3 and lane l rows
// l + 64 i (i < 8) of them: a column lies in one wave, so its norm and its
// products with the reflector are wave sums, and each reflector entry a
// lane reads from LDS serves four columns.  Step k: the wave owning column
// k forms the reflector (as in k_qr_tile) and publishes v and tau (two
// buffers, one barrier per step); every wave with columns right of k
// applies H = I - tau v v^T to them.  Per-thread partial sums go in four
// interleaved chains.
__global__ __launch_bounds__(1024) void k_qr_wide(QRLevel a)
{
    constexpr int W2 = 64, CH = 512, C = 4, R = CH / 64;
    __shared__ double s_v[2][CH];
    __shared__ double s_tau[2];
    const int mt = blockIdx.z, l = blockIdx.y, c = blockIdx.x;
    if (c >= (mt ? a.nodes_g : a.nodes_f)) return;   // uniform: the grid covers the larger
    const int tid = threadIdx.x, lane = tid & 63, cg = tid >> 6;
    double x[C][R];
    if (a.level == 0) {
        const double *__restrict__ Y = mt ? a.Gw : a.Fw;
        const int64_t m = mt ? a.mgw : a.mfw;
        const int W = W2 / 2;
        const int p = a.pairs[2 * l], qq = a.pairs[2 * l + 1];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int jc = C * cg + j;
            const int64_t gc = (jc < W) ? (int64_t)p * W + jc : (int64_t)qq * W + (jc - W);
            const double *col = Y + gc * m;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int64_t gr = (int64_t)c * CH + lane + 64 * i;
                x[j][i] = (gr < m) ? col[gr] : 0.0;
            }
        }
    } else {
        const int prev = mt ? a.prev_g : a.prev_f;
        const double *__restrict__ ra = a.in + (((size_t)l * 2 + mt) * a.in_stride) * (W2 * W2);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int node = R * c + i;
#pragma unroll
            for (int j = 0; j < C; ++j)
                x[j][i] = (node < prev) ? ra[(size_t)node * (W2 * W2) + (C * cg + j) * W2 + lane] : 0.0;
        }
    }
    for (int k = 0; k < W2; ++k) {
        const int par = k & 1;
#pragma unroll
        for (int kj = 0; kj < C; ++kj) {             // static register indices
            if (cg != (k >> 2) || kj != (k & 3)) continue;   // wave-uniform: owner of column k
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (i > 0 || lane > k) s4[i & 3] = fma(x[kj][i], x[kj][i], s4[i & 3]);
            const double sq = wave_total((s4[0] + s4[1]) + (s4[2] + s4[3]));
            const double al = readlane_d(x[kj][0], k);
            double beta = al, tau = 0.0, scale = 0.0;
            if (sq > 0.0) {
                beta = -copysign(sqrt(fma(al, al, sq)), al);
                tau = (beta - al) / beta;
                scale = 1.0 / (al - beta);
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const bool below = i > 0 || lane > k;
                s_v[par][lane + 64 * i] = (i == 0 && lane == k) ? 1.0 : (below ? x[kj][i] * scale : 0.0);
            }
            if (lane == k) x[kj][0] = beta;
            if (lane == 0) s_tau[par] = tau;
        }
        __syncthreads();
        const double tr = s_tau[par];
        if (tr != 0.0 && C * cg + C - 1 > k) {       // wave-uniform
            double v[R];
#pragma unroll
            for (int i = 0; i < R; ++i) v[i] = s_v[par][lane + 64 * i];
            double w[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int i = 0; i < R; ++i) d4[i & 3] = fma(v[i], x[j][i], d4[i & 3]);
                w[j] = (d4[0] + d4[1]) + (d4[2] + d4[3]);
            }
#pragma unroll
            for (int j = 0; j < C; ++j) w[j] = wave_total(w[j]);
#pragma unroll
            for (int j = 0; j < C; ++j) {
                if (C * cg + j > k) {
                    const double tw = tr * w[j];
#pragma unroll
                    for (int i = 0; i < R; ++i) x[j][i] = fma(-tw, v[i], x[j][i]);
                }
            }
        }
    }
    double *__restrict__ Rout = a.out + (((size_t)l * 2 + mt) * a.out_stride + c) * (W2 * W2);
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const int jc = C * cg + j;
        Rout[jc * W2 + lane] = (lane <= jc) ? x[j][0] : 0.0;
    }
}

static void pivot_qr_wide(const Plan &P, const Ptrs &W, int step, hipStream_t s)
{
    constexpr int64_t CH = 512;
    QRLevel a;
    a.Fw = W.Fw;
    a.Gw = W.Gw;
    a.mfw = P.mfw;
    a.mgw = P.mgw;
    a.pairs = W.otab + (size_t)step * P.npairs * 2;
    const int L0 = pivot_qr_tiles(P);               // the buffers hold this many per pair
    int nf = (int)((P.mfw + CH - 1) / CH), ng = (int)((P.mgw + CH - 1) / CH);
    int pf = 0, pg = 0, level = 0;
    const double *in = nullptr;
    for (;;) {
        const bool last = (nf == 1 && ng == 1);
        a.level = level;
        a.nodes_f = nf;
        a.nodes_g = ng;
        a.prev_f = pf;
        a.prev_g = pg;
        a.in = in;
        a.in_stride = L0;
        a.out = last ? W.gram : W.qr[level & 1];
        a.out_stride = last ? 1 : L0;
        hipLaunchKernelGGL(k_qr_wide, dim3((unsigned)(nf > ng ? nf : ng), P.npairs, 2),
                           dim3(1024), 0, s, a);
        if (last) break;
        in = a.out;
        pf = nf;
        pg = ng;
        nf = (nf + 7) / 8;
        ng = (ng + 7) / 8;
        ++level;
    }
}

int pivot_qr_tiles(const Plan &P)
{
    const int64_t ch = 2 * (int64_t)P.W2;
    const int64_t m = P.mfw > P.mgw ? P.mfw : P.mgw;
    return (int)((m + ch - 1) / ch);
}

template <int W2, bool CX>
static void pivot_qr_impl(const Plan &P, const Ptrs &W, int step, hipStream_t s)
{
    constexpr int64_t CH = 2 * W2;
    QRLevel a;
    a.Fw = W.Fw;
    a.Gw = W.Gw;
    a.mfw = P.mfw;
    a.mgw = P.mgw;
    a.pairs = W.otab + (size_t)step * P.npairs * 2;
    const int L0 = pivot_qr_tiles(P);
    int nf = (int)((P.mfw + CH - 1) / CH), ng = (int)((P.mgw + CH - 1) / CH);
    int pf = 0, pg = 0, level = 0;
    const double *in = nullptr;
    for (;;) {
        const bool last = (nf == 1 && ng == 1);
        a.level = level;
        a.nodes_f = nf;
        a.nodes_g = ng;
        a.prev_f = pf;
        a.prev_g = pg;
        a.in = in;
        a.in_stride = L0;
        a.out = last ? W.gram : W.qr[level & 1];
        a.out_stride = last ? 1 : L0;
        hipLaunchKernelGGL((k_qr_tile<W2, CX>), dim3((unsigned)(nf > ng ? nf : ng), P.npairs, 2),
                           dim3(256), 0, s, a);
        if (last) break;
        in = a.out;
        pf = nf;
        pg = ng;
        nf = (nf + 1) / 2;
        ng = (ng + 1) / 2;
        ++level;
    }
}

// The pivot factors of every block pair of one step into W.gram (per pair:
// R_F, then R_G, W2 x W2 upper triangular; interleaved complex for complex
// pairs, with a real diagonal).
void launch_pivot_qr(const Plan &P, const Ptrs &W, int step, hipStream_t s)
{
    if (P.is_complex) {
        if (P.W2 == 16) pivot_qr_impl<16, true>(P, W, step, s);
        else pivot_qr_impl<32, true>(P, W, step, s);
        return;
    }
    switch (P.W2) {
    case 16: pivot_qr_impl<16, false>(P, W, step, s); break;
    case 32: pivot_qr_impl<32, false>(P, W, step, s); break;
    default: pivot_qr_wide(P, W, step, s); break;
    }
}

}  // namespace hz
