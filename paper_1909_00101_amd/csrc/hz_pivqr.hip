// hz_pivqr.hip -- pivot factors from QR factorizations of the block-column
// pairs instead of Gram matrices and their Cholesky factorizations (paper,
// Section 2.3, and Appendix E: for ill-conditioned pairs the Grams of the
// block-column pairs can be numerically indefinite, and the pairs are then
// shortened by QR).  With R the triangular factor of [Y_p Y_q] = Q R,
// R^T R is the pivot Gram, so R takes the place of the Cholesky factor; Q
// is never formed.
//
// Tall-skinny QR as a reduction tree: every workgroup factors one node of
// 512 rows and W2 columns with Householder reflections (the node in
// registers, the reflectors through LDS) and writes its W2 x W2 triangle;
// the leaves are consecutive 512-row chunks of [Y_p Y_q], each further
// level factors up to eight stacked triangles of the level below, until one
// triangle per block pair and matrix is left (4096 rows: two levels).  All
// pivot pairs of a step, F and G, go in one launch per level.  The factor
// is not squared, so a block pair whose columns are independent to working
// accuracy gets a usable factor where its Gram would lose half the digits.
#include <math.h>

#include "hz_device.h"
#include "hz_internal.h"

namespace hz {

// One level of the tree.  Level 0 reads rows [c * 512, (c + 1) * 512) of
// the block columns p, q of Fw (matrix 0) or Gw (matrix 1); a further level
// reads the triangles 8c .. 8c + 7 of the level below (missing ones are
// zero).  Triangles are column-major W2 x W2 with zeros below the diagonal,
// at out + ((pair * 2 + matrix) * out_stride + node) * W2 * W2 (elements of
// two doubles, real and imaginary, for complex pairs).
struct QRLevel {
    const double *Fw, *Gw;
    int64_t mfw, mgw;
    const int *pairs;          // this step's (p, q) per pivot pair
    const double *in;          // triangles of the level below (levels > 0)
    double *out;
    int in_stride, out_stride; // triangles per (pair, matrix) in `in` / `out`
    int nodes_f, nodes_g;      // nodes of this level per matrix
    int prev_f, prev_g;        // triangles of the level below per matrix
    int level;
};

constexpr int QR_ROWS = 512;   // rows of a node
constexpr int QR_FAN = 8;      // triangles combined by a node of a further level

// v_permlane32_swap / v_permlane16_swap with one register as both
// operands: the two results summed give, in every lane, the sum of its own
// value and the one 32 lanes (or one 16-lane row) away, in the same operand
// order in both lanes of a pair.
__device__ __forceinline__ double swap_sum32(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double a = __builtin_bit_cast(double, ((long long)hi[0] << 32) | lo[0]);
    const double c = __builtin_bit_cast(double, ((long long)hi[1] << 32) | lo[1]);
    return a + c;
}
__device__ __forceinline__ double swap_sum16(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double a = __builtin_bit_cast(double, ((long long)hi[0] << 32) | lo[0]);
    const double c = __builtin_bit_cast(double, ((long long)hi[1] << 32) | lo[1]);
    return a + c;
}

// Sum over the 64 lanes of a wave in a fixed order, every lane getting the
// same bits: the 16-lane rows by DPP (S0 .. S3), then (S0 + S2) + (S1 + S3)
// by the two lane swaps.
__device__ __forceinline__ double wave_total(double v)
{
    return swap_sum16(swap_sum32(dpp_group_sum<16>(v)));
}

// A workgroup of 16 waves factors one node.  Wave g owns the C = W2 / 16
// columns C g .. C g + C - 1 and lane l the rows l + 64 i (i < 8) of them:
// a column lies in one wave, so its norm and its products with a reflector
// are wave sums, and each reflector entry a lane reads from LDS serves C
// columns.  On a further level, triangle 8c + i takes rows 64 i ..
// 64 i + W2 - 1 of the node (the rows between are zero, which leaves the
// factorization unchanged).  Step k: the wave owning column k forms the
// reflector H = I - tau v v^H (v_k = 1) with H^H x = (beta, 0, ..., 0),
// beta real (for real data the transpose and a real tau), and publishes v
// and tau (two buffers, one barrier per step); every wave with columns
// right of k applies H^H = I - conj(tau) v v^H to them.  Per-thread partial
// sums go in four interleaved chains (complex: two per part).
template <int W2, bool CX>
__global__ __launch_bounds__(1024) void k_qr_node(QRLevel a)
{
    constexpr int CH = QR_ROWS, C = W2 / 16, R = CH / 64, NP = CX ? 2 : 1;
    static_assert(W2 == 16 || W2 == 32 || W2 == 64, "pivot block order 16, 32 or 64");
    __shared__ double s_v[2][NP][CH];
    __shared__ double s_tau[2][NP];
    const int mt = blockIdx.z, l = blockIdx.y, c = blockIdx.x;
    if (c >= (mt ? a.nodes_g : a.nodes_f)) return;   // uniform: the grid covers the larger
    const int tid = threadIdx.x, lane = tid & 63, cg = tid >> 6;
    double x[C][R][NP];
    if (a.level == 0) {
        const double *__restrict__ Y = mt ? a.Gw : a.Fw;
        const int64_t m = mt ? a.mgw : a.mfw;
        const int W = W2 / 2;
        const int p = a.pairs[2 * l], qq = a.pairs[2 * l + 1];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int jc = C * cg + j;
            const int64_t gc = (jc < W) ? (int64_t)p * W + jc : (int64_t)qq * W + (jc - W);
            const double *col = Y + NP * gc * m;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int64_t gr = (int64_t)c * CH + lane + 64 * i;
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) x[j][i][pl] = (gr < m) ? col[NP * gr + pl] : 0.0;
            }
        }
    } else {
        const int prev = mt ? a.prev_g : a.prev_f;
        const double *__restrict__ ra = a.in + NP * (((size_t)l * 2 + mt) * a.in_stride) * (W2 * W2);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int node = QR_FAN * c + i;
            const bool live = node < prev && lane < W2;
#pragma unroll
            for (int j = 0; j < C; ++j)
#pragma unroll
                for (int pl = 0; pl < NP; ++pl)
                    x[j][i][pl] = live ? ra[NP * ((size_t)node * (W2 * W2) + (C * cg + j) * W2 + lane) + pl]
                                       : 0.0;
        }
    }
    for (int k = 0; k < W2; ++k) {
        const int par = k & 1;
#pragma unroll
        for (int kj = 0; kj < C; ++kj) {             // static register indices
            if (cg != k / C || kj != k % C) continue;   // wave-uniform: owner of column k
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (i > 0 || lane > k) {
#pragma unroll
                    for (int pl = 0; pl < NP; ++pl) s4[i & 3] = fma(x[kj][i][pl], x[kj][i][pl], s4[i & 3]);
                }
            const double sq = wave_total((s4[0] + s4[1]) + (s4[2] + s4[3]));
            const double alr = readlane_d(x[kj][0][0], k);
            const double ali = CX ? readlane_d(x[kj][0][NP - 1], k) : 0.0;
            double beta = alr, tau[NP], scale[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) tau[pl] = scale[pl] = 0.0;
            if (sq > 0.0 || ali != 0.0) {
                beta = -copysign(sqrt(fma(alr, alr, fma(ali, ali, sq))), alr);
                tau[0] = (beta - alr) / beta;
                if constexpr (CX) {
                    tau[NP - 1] = -ali / beta;
                    // 1 / (alpha - beta)
                    const double dr = alr - beta, di = ali;
                    const double den = fma(dr, dr, di * di);
                    scale[0] = dr / den;
                    scale[NP - 1] = -di / den;
                } else {
                    scale[0] = 1.0 / (alr - beta);
                }
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const bool below = i > 0 || lane > k, diag = i == 0 && lane == k;
                const int r = lane + 64 * i;
                if constexpr (CX) {
                    const double xr = x[kj][i][0], xi = x[kj][i][NP - 1];
                    s_v[par][0][r] = diag ? 1.0 : (below ? xr * scale[0] - xi * scale[NP - 1] : 0.0);
                    s_v[par][NP - 1][r] = below ? xr * scale[NP - 1] + xi * scale[0] : 0.0;
                } else {
                    s_v[par][0][r] = diag ? 1.0 : (below ? x[kj][i][0] * scale[0] : 0.0);
                }
            }
            if (lane == k) {
                x[kj][0][0] = beta;
                if constexpr (CX) x[kj][0][NP - 1] = 0.0;
            }
            if (lane == 0) {
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) s_tau[par][pl] = tau[pl];
            }
        }
        __syncthreads();
        const double tr = s_tau[par][0], ti = CX ? s_tau[par][NP - 1] : 0.0;
        if ((tr != 0.0 || ti != 0.0) && C * cg + C - 1 > k) {   // wave-uniform
            double v[R][NP];
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) v[i][pl] = s_v[par][pl][lane + 64 * i];
            // w_j = v^H a_j
            double w[C][NP];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                if constexpr (CX) {
                    double r2[2] = {0.0, 0.0}, i2[2] = {0.0, 0.0};
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const double vr = v[i][0], vi = v[i][NP - 1];
                        const double xr = x[j][i][0], xi = x[j][i][NP - 1];
                        r2[i & 1] = fma(vr, xr, fma(vi, xi, r2[i & 1]));
                        i2[i & 1] = fma(vr, xi, fma(-vi, xr, i2[i & 1]));
                    }
                    w[j][0] = r2[0] + r2[1];
                    w[j][NP - 1] = i2[0] + i2[1];
                } else {
                    double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int i = 0; i < R; ++i) d4[i & 3] = fma(v[i][0], x[j][i][0], d4[i & 3]);
                    w[j][0] = (d4[0] + d4[1]) + (d4[2] + d4[3]);
                }
            }
#pragma unroll
            for (int j = 0; j < C; ++j)
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) w[j][pl] = wave_total(w[j][pl]);
#pragma unroll
            for (int j = 0; j < C; ++j) {
                if (C * cg + j <= k) continue;
                if constexpr (CX) {
                    // a_j -= conj(tau) w_j v
                    const double cr = tr * w[j][0] + ti * w[j][NP - 1];
                    const double ci = tr * w[j][NP - 1] - ti * w[j][0];
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const double vr = v[i][0], vi = v[i][NP - 1];
                        x[j][i][0] -= cr * vr - ci * vi;
                        x[j][i][NP - 1] -= cr * vi + ci * vr;
                    }
                } else {
                    const double tw = tr * w[j][0];
#pragma unroll
                    for (int i = 0; i < R; ++i) x[j][i][0] = fma(-tw, v[i][0], x[j][i][0]);
                }
            }
        }
    }
    if (lane < W2) {
        double *__restrict__ Rout = a.out + NP * (((size_t)l * 2 + mt) * a.out_stride + c) * (W2 * W2);
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int jc = C * cg + j;
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) Rout[NP * (jc * W2 + lane) + pl] = (lane <= jc) ? x[j][0][pl] : 0.0;
        }
    }
}

int pivot_qr_tiles(const Plan &P)
{
    const int64_t m = P.mfw > P.mgw ? P.mfw : P.mgw;
    return (int)((m + QR_ROWS - 1) / QR_ROWS);
}

template <int W2, bool CX>
static void pivot_qr_impl(const Plan &P, const Ptrs &W, int step, hipStream_t s)
{
    QRLevel a;
    a.Fw = W.Fw;
    a.Gw = W.Gw;
    a.mfw = P.mfw;
    a.mgw = P.mgw;
    a.pairs = W.otab + (size_t)step * P.npairs * 2;
    const int L0 = pivot_qr_tiles(P);
    int nf = (int)((P.mfw + QR_ROWS - 1) / QR_ROWS), ng = (int)((P.mgw + QR_ROWS - 1) / QR_ROWS);
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
        hipLaunchKernelGGL((k_qr_node<W2, CX>), dim3((unsigned)(nf > ng ? nf : ng), P.npairs, 2),
                           dim3(1024), 0, s, a);
        if (last) break;
        in = a.out;
        pf = nf;
        pg = ng;
        nf = (nf + QR_FAN - 1) / QR_FAN;
        ng = (ng + QR_FAN - 1) / QR_FAN;
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
    default: pivot_qr_impl<64, false>(P, W, step, s); break;
    }
}

}  // namespace hz
