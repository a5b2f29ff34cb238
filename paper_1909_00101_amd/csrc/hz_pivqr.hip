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
// reflector H = I - tau v v^T (v_k = 1) that maps the column to
// (beta, 0, ..., 0) and publish v and tau in LDS (two buffers, so one
// barrier per step); the owners of the columns right of k apply H to their
// rows.  Sums over a column use a fixed reduction order.
template <int W2>
__global__ __launch_bounds__(256) void k_qr_tile(QRLevel a)
{
    constexpr int CH = 2 * W2;          // tile rows
    constexpr int NT = 256;
    constexpr int Q = NT / W2;          // threads per column
    constexpr int RPQ = CH / Q;         // rows per thread
    static_assert(Q >= 1 && (64 % Q) == 0 && RPQ % 2 == 0, "bad QR tile geometry");
    __shared__ double s_v[2][CH];
    __shared__ double s_tau[2];
    const int mt = blockIdx.z, l = blockIdx.y, c = blockIdx.x;
    if (c >= (mt ? a.nodes_g : a.nodes_f)) return;   // uniform: the grid covers the larger
    const int tid = threadIdx.x;
    const int jc = tid / Q, q = tid % Q;
    double x[RPQ];
    if (a.level == 0) {
        const double *__restrict__ Y = mt ? a.Gw : a.Fw;
        const int64_t m = mt ? a.mgw : a.mfw;
        const int W = W2 / 2;
        const int p = a.pairs[2 * l], qq = a.pairs[2 * l + 1];
        const int64_t gc = (jc < W) ? (int64_t)p * W + jc : (int64_t)qq * W + (jc - W);
        const double *col = Y + gc * m;
#pragma unroll
        for (int i = 0; i < RPQ; ++i) {
            const int64_t gr = (int64_t)c * CH + q + Q * i;
            x[i] = (gr < m) ? col[gr] : 0.0;
        }
    } else {
        const int prev = mt ? a.prev_g : a.prev_f;
        const double *__restrict__ ra =
            a.in + (((size_t)l * 2 + mt) * a.in_stride + 2 * (size_t)c) * (W2 * W2);
        const bool second = 2 * c + 1 < prev;
#pragma unroll
        for (int i = 0; i < RPQ; ++i) {
            const int r = q + Q * i;
            double v = 0.0;
            if (r < W2) v = ra[jc * W2 + r];
            else if (second) v = ra[W2 * W2 + jc * W2 + (r - W2)];
            x[i] = v;
        }
    }
    for (int k = 0; k < W2; ++k) {
        const int par = k & 1;
        if (jc == k) {
            double sq = 0.0, al = 0.0;
#pragma unroll
            for (int i = 0; i < RPQ; ++i) {
                const int r = q + Q * i;
                if (r > k) sq = fma(x[i], x[i], sq);
                if (r == k) al = x[i];
            }
#pragma unroll
            for (int off = Q / 2; off >= 1; off >>= 1) {
                sq += __shfl_xor(sq, off);
                al += __shfl_xor(al, off);       // one nonzero term: exact
            }
            double beta = al, tau = 0.0, scale = 0.0;
            if (sq > 0.0) {
                beta = -copysign(sqrt(fma(al, al, sq)), al);
                tau = (beta - al) / beta;
                scale = 1.0 / (al - beta);
            }
#pragma unroll
            for (int i = 0; i < RPQ; ++i) {
                const int r = q + Q * i;
                s_v[par][r] = (r == k) ? 1.0 : ((r > k) ? x[i] * scale : 0.0);
                if (r == k) x[i] = beta;
            }
            if (q == 0) s_tau[par] = tau;
        }
        __syncthreads();
        const double tau = s_tau[par];
        if (tau != 0.0 && jc > k) {
            double w0 = 0.0, w1 = 0.0;
#pragma unroll
            for (int i = 0; i < RPQ; i += 2) {
                w0 = fma(s_v[par][q + Q * i], x[i], w0);
                w1 = fma(s_v[par][q + Q * (i + 1)], x[i + 1], w1);
            }
            double w = w0 + w1;
#pragma unroll
            for (int off = Q / 2; off >= 1; off >>= 1) w += __shfl_xor(w, off);
            const double tw = tau * w;
#pragma unroll
            for (int i = 0; i < RPQ; ++i) x[i] = fma(-tw, s_v[par][q + Q * i], x[i]);
        }
    }
    double *__restrict__ R = a.out + (((size_t)l * 2 + mt) * a.out_stride + c) * (W2 * W2);
#pragma unroll
    for (int i = 0; i < RPQ; ++i) {
        const int r = q + Q * i;
        if (r < W2) R[jc * W2 + r] = (r <= jc) ? x[i] : 0.0;
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
