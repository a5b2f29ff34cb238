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
// over a column use a fixed reduction order.  Complex elements are
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
            double sq = 0.0, al[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) al[pl] = 0.0;
#pragma unroll
            for (int i = 0; i < RPQ; ++i) {
                const int r = q + Q * i;
                if (r > k) {
#pragma unroll
                    for (int pl = 0; pl < NP; ++pl) sq = fma(x[pl][i], x[pl][i], sq);
                }
                if (r == k) {
#pragma unroll
                    for (int pl = 0; pl < NP; ++pl) al[pl] = x[pl][i];
                }
            }
#pragma unroll
            for (int off = Q / 2; off >= 1; off >>= 1) {
                sq += __shfl_xor(sq, off);
#pragma unroll
                for (int pl = 0; pl < NP; ++pl) al[pl] += __shfl_xor(al[pl], off);   // exact
            }
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
                double wr = wr0 + wr1, wi = wi0 + wi1;
#pragma unroll
                for (int off = Q / 2; off >= 1; off >>= 1) {
                    wr += __shfl_xor(wr, off);
                    wi += __shfl_xor(wi, off);
                }
                const double cr = tr * wr + ti * wi, ci = tr * wi - ti * wr;   // conj(tau) w
#pragma unroll
                for (int i = 0; i < RPQ; ++i) {
                    const int r = q + Q * i;
                    const double vr = s_v[par][0][r], vi = s_v[par][NP - 1][r];
                    x[0][i] -= cr * vr - ci * vi;
                    x[NP - 1][i] -= cr * vi + ci * vr;
                }
            } else {
                double w0 = 0.0, w1 = 0.0;
#pragma unroll
                for (int i = 0; i < RPQ; i += 2) {
                    w0 = fma(s_v[par][0][q + Q * i], x[0][i], w0);
                    w1 = fma(s_v[par][0][q + Q * (i + 1)], x[0][i + 1], w1);
                }
                double w = w0 + w1;
#pragma unroll
                for (int off = Q / 2; off >= 1; off >>= 1) w += __shfl_xor(w, off);
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
    default: pivot_qr_impl<64, false>(P, W, step, s); break;
    }
}

}  // namespace hz
