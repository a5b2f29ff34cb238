// hz_pivqr.hip -- pivot factors from QR factorizations of the block-column
// pairs instead of Gram matrices and their Cholesky factorizations (paper,
// Section 2.3, and Appendix E: for ill-conditioned pairs the Grams of the
// block-column pairs can be numerically indefinite, and the pairs are then
// shortened by QR).  With R the triangular factor of [Y_p Y_q] = Q R,
// R^T R is the pivot Gram, so R takes the place of the Cholesky factor; Q
// is never formed.
//
// Tall-skinny QR as a reduction tree: every workgroup factors one tile of
// 2 * W2 rows and W2 columns with Householder reflections in LDS and writes
// its W2 x W2 triangle; the leaves are consecutive row chunks of [Y_p Y_q],
// each further level factors two stacked triangles of the level below,
// until one triangle per block pair and matrix is left.  All pivot pairs of
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

template <int W2>
__global__ __launch_bounds__(256) void k_qr_tile(QRLevel a)
{
    constexpr int CH = 2 * W2;          // tile rows
    constexpr int LDA = CH + 1;
    constexpr int NT = 256, NW = NT / 64;
    constexpr int Q = NT / W2;          // threads per column in the update
    constexpr int RPQ = CH / Q;         // rows per thread in the update
    static_assert(CH <= NT && Q >= 1 && (64 % Q) == 0, "bad QR tile geometry");
    __shared__ double A[W2 * LDA];      // column j at A + j * LDA
    __shared__ double s_v[CH];
    __shared__ double s_part[NW];
    const int mt = blockIdx.z, l = blockIdx.y, c = blockIdx.x;
    if (c >= (mt ? a.nodes_g : a.nodes_f)) return;   // uniform: the grid covers the larger
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    if (a.level == 0) {
        const double *__restrict__ Y = mt ? a.Gw : a.Fw;
        const int64_t m = mt ? a.mgw : a.mfw;
        const int W = W2 / 2;
        const int p = a.pairs[2 * l], q = a.pairs[2 * l + 1];
        for (int e = tid; e < W2 * CH; e += NT) {
            const int j = e / CH, r = e % CH;
            const int64_t gc = (j < W) ? (int64_t)p * W + j : (int64_t)q * W + (j - W);
            const int64_t gr = (int64_t)c * CH + r;
            A[j * LDA + r] = (gr < m) ? Y[gc * m + gr] : 0.0;
        }
    } else {
        const int prev = mt ? a.prev_g : a.prev_f;
        const double *__restrict__ ra =
            a.in + (((size_t)l * 2 + mt) * a.in_stride + 2 * (size_t)c) * (W2 * W2);
        const bool second = 2 * c + 1 < prev;
        for (int e = tid; e < W2 * CH; e += NT) {
            const int j = e / CH, r = e % CH;
            double v = 0.0;
            if (r < W2) v = ra[j * W2 + r];
            else if (second) v = ra[W2 * W2 + j * W2 + (r - W2)];
            A[j * LDA + r] = v;
        }
    }
    __syncthreads();

    const int jc = tid / Q, r0 = (tid % Q) * RPQ;   // update: column jc, rows r0 .. r0+RPQ-1
    for (int k = 0; k < W2; ++k) {
        // sum of squares below the diagonal of column k, in a fixed order
        double sq = 0.0;
        if (tid < CH && tid > k) {
            const double x = A[k * LDA + tid];
            sq = x * x;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off);
        if (lane == 0) s_part[wave] = sq;
        __syncthreads();
        double sigma = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sigma += s_part[w];
        const double alpha = A[k * LDA + k];
        // Householder reflector H = I - tau v v^T with v_k = 1 mapping
        // column k to (beta, 0, ..., 0); none when nothing is below the diagonal
        double beta = alpha, tau = 0.0, scale = 0.0;
        if (sigma > 0.0) {
            beta = -copysign(sqrt(fma(alpha, alpha, sigma)), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (tid < CH) s_v[tid] = (tid == k) ? 1.0 : ((tid > k) ? A[k * LDA + tid] * scale : 0.0);
        __syncthreads();
        if (tid == 0) A[k * LDA + k] = beta;
        if (tau != 0.0 && jc > k) {
            double w = 0.0;
#pragma unroll
            for (int i = 0; i < RPQ; ++i) {
                const int r = r0 + i;
                if (r >= k) w = fma(s_v[r], A[jc * LDA + r], w);
            }
#pragma unroll
            for (int off = Q / 2; off >= 1; off >>= 1) w += __shfl_xor(w, off);
            const double tw = tau * w;
#pragma unroll
            for (int i = 0; i < RPQ; ++i) {
                const int r = r0 + i;
                if (r >= k) A[jc * LDA + r] = fma(-tw, s_v[r], A[jc * LDA + r]);
            }
        }
        __syncthreads();
    }
    double *__restrict__ R = a.out + (((size_t)l * 2 + mt) * a.out_stride + c) * (W2 * W2);
    for (int e = tid; e < W2 * W2; e += NT) {
        const int j = e / W2, r = e % W2;
        R[j * W2 + r] = (r <= j) ? A[j * LDA + r] : 0.0;
    }
}

int pivot_qr_tiles(const Plan &P)
{
    const int64_t ch = 2 * (int64_t)P.W2;
    const int64_t m = P.mfw > P.mgw ? P.mfw : P.mgw;
    return (int)((m + ch - 1) / ch);
}

template <int W2>
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
        hipLaunchKernelGGL(k_qr_tile<W2>, dim3((unsigned)(nf > ng ? nf : ng), P.npairs, 2),
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
// R_F, then R_G, W2 x W2 upper triangular).
void launch_pivot_qr(const Plan &P, const Ptrs &W, int step, hipStream_t s)
{
    switch (P.W2) {
    case 16: pivot_qr_impl<16>(P, W, step, s); break;
    case 32: pivot_qr_impl<32>(P, W, step, s); break;
    default: pivot_qr_impl<64>(P, W, step, s); break;
    }
}

}  // namespace hz
