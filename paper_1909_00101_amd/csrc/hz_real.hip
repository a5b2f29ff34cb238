// hz_real.hip -- FP64 kernels of the blocked one-sided implicit
// Hari-Zimmermann GSVD on gfx950 (CDNA4).
//
// Per solve:  prescale/copy-in  ->  sweeps of block steps
//             (Gram -> inner solve -> update)  ->  norms -> rank -> scatter.
// Every reduction has a fixed association order and no floating-point
// atomics are used, so reruns on the same input are bitwise identical.
#include "hz_device.h"
#include "hz_internal.h"
#include "hz_kernels_real.h"

namespace hz {

// ------------------------------------------------------------------------
// Prescale and copy-in (paper: Section 2, Z_0 = diag(1/||g_j||), and the
// initFGZ kernel of Section 3.3), fused with the bordering of Section 3.1.
// One wave per working column j < nw.  Columns j < n: d_j = 1/||g_j||,
// Fw(:,j) = d_j F(:,j), Gw(:,j) = d_j G(:,j), Zw(:,j) = d_j e_j.  Columns
// j >= n (bordering): unit entries at rows mf + (j-n) of Fw and mg + (j-n)
// of Gw, Zw(:,j) = e_j.  Rows beyond the data are zero.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prescale_copy(
    int64_t mf, int64_t mg, int64_t n, const double *__restrict__ F, int64_t ldf,
    const double *__restrict__ G, int64_t ldg, int64_t nw, int64_t mfw, int64_t mgw,
    int64_t nzw, double *__restrict__ Fw, double *__restrict__ Gw, double *__restrict__ Zw,
    int *__restrict__ status)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nw) return;
    double *fw = Fw + j * mfw, *gw = Gw + j * mgw, *zw = Zw + j * nzw;
    if (j < n) {
        const double *f = F + j * ldf, *g = G + j * ldg;
        double s = 0.0;
        for (int64_t r = lane; r < mg; r += 64) s = fma(g[r], g[r], s);
        s = wave_sum(s);
        const double d = 1.0 / sqrt(s);
        bool bad = !(s > 0.0) || !isfinite(s);
        for (int64_t r = lane; r < mfw; r += 64) {
            const double v = (r < mf) ? f[r] * d : 0.0;
            bad |= !isfinite(v);
            fw[r] = v;
        }
        for (int64_t r = lane; r < mgw; r += 64) gw[r] = (r < mg) ? g[r] * d : 0.0;
        for (int64_t r = lane; r < nzw; r += 64) zw[r] = (r == j) ? d : 0.0;
        if (bad) atomicOr(status + ST_FLAGS, FLAG_NONFINITE);
    } else {
        const int64_t k = j - n;
        for (int64_t r = lane; r < mfw; r += 64) fw[r] = (r == mf + k) ? 1.0 : 0.0;
        for (int64_t r = lane; r < mgw; r += 64) gw[r] = (r == mg + k) ? 1.0 : 0.0;
        for (int64_t r = lane; r < nzw; r += 64) zw[r] = (r == j) ? 1.0 : 0.0;
    }
}

// ------------------------------------------------------------------------
// Pivot Gram blocks (paper: Section 2.3, A_hat = [F_p F_q]^T [F_p F_q] and
// B_hat likewise).  FP64 MFMA 16x16x4.  Grid (splits, pairs, 2): each
// workgroup sums the rows of its split (64-row chunks loaded straight into
// the MFMA operand registers, two chunks in flight) into the lower-triangle
// 16x16 tiles of a W2 x W2 partial Gram (the inner solver reads only the
// lower triangle); each of the four waves takes a 16-row slab of every
// chunk, and their partials are summed as (w0 + w1) + (w2 + w3).  k_gram_sum then adds the split partials in split order:
// no floating-point atomics, so the result is reproducible bit for bit.
// ------------------------------------------------------------------------
template <int W2>
__global__ __launch_bounds__(256) void k_gram(const double *__restrict__ Fw,
                                              const double *__restrict__ Gw, int64_t mfw,
                                              int64_t mgw, const int *__restrict__ pairs,
                                              int splits, double *__restrict__ part)
{
    const int split = blockIdx.x, pr = blockIdx.y, mat = blockIdx.z;
    const int64_t m = mat ? mgw : mfw;
    const int64_t nch = m / 64;
    __shared__ __attribute__((aligned(16))) double tile[gram_lds<W2>()];
    gram_block<W2>(mat ? Gw : Fw, m, pairs[2 * pr], pairs[2 * pr + 1], nch * split / splits,
                   nch * (split + 1) / splits,
                   part + ((size_t)(pr * 2 + mat) * splits + split) * (W2 * W2), tile);
}

// Sum of the Gram split partials in split order (fixed association, so the
// result is reproducible bit for bit): grid (W2*W2/512, 2 * pairs), 256
// threads, two consecutive elements per thread, every split's load issued
// before the adds.
template <int W2>
__global__ __launch_bounds__(256) void k_gram_sum(const double *__restrict__ part, int splits,
                                                  double *__restrict__ gram)
{
    constexpr int MAXS = 16;
    const int pm = blockIdx.y;
    const int e = 2 * (blockIdx.x * 256 + threadIdx.x);
    if (e >= W2 * W2) return;
    if ((e % W2) / 16 < (e / W2) / 16) return;   // upper tiles: never read
    const double *src = part + (size_t)pm * splits * (W2 * W2) + e;
    d2 v[MAXS];
#pragma unroll
    for (int s = 0; s < MAXS; ++s)
        if (s < splits) v[s] = *(const d2 *)(src + (size_t)s * (W2 * W2));
    d2 acc = v[0];
#pragma unroll
    for (int s = 1; s < MAXS; ++s)
        if (s < splits) acc += v[s];
    *(d2 *)(gram + (size_t)pm * (W2 * W2) + e) = acc;
}

// ------------------------------------------------------------------------
// Inner solve of one pivot block pair (paper: Section 2.3 factorization,
// Section 2.1 pointwise method on the factors, Section 2.4 Theta rescale,
// Section 2.5 counters; Sections 3.5.2-3.5.3 for the shared-memory flow).
// One workgroup per block pair, NT = (W2/2) * LP threads: LP lanes per
// column pair of an inner step, RPL = W2/LP rows per lane.  Steps:
//  1. A_hat, B_hat = sum of the Gram partials (split order) into LDS.
//  2. Cholesky A_hat = F_hat^T F_hat, B_hat = G_hat^T G_hat (F_hat, G_hat
//     upper triangular), one wave per matrix: for 2w = 64 (and 2w = 32 with
//     two or more waves) in panels of 16 columns factored in registers
//     (lane = row, entries by readlane) with the trailing lower tiles
//     updated by FP64 MFMA; otherwise column by column, lane i keeping row
//     i, the new column of L broadcast through LDS (both matrices in one
//     wave); a non-positive pivot flags HZ_ECHOL.
//  3. Z_hat = diag(1/||g_hat_j||), F_hat, G_hat scaled by it.
//  4. Inner sweeps (<= inner_max, stop after a sweep without
//     transformations): per step, the LP lanes of a column pair form a_ii,
//     a_jj, a_ij, b_ij with DPP sums, then the skip test, the 2x2
//     transformation, criterion C1, the sorting swap, applied in LDS.
//  5. Z_tilde = Z_hat Theta, Theta_jj = (||f_hat_j||^2+||g_hat_j||^2)^-1/2.
// Counters per (step, pair): transformations, big ones, inner sweeps run.
// ------------------------------------------------------------------------
template <int W2, int LP, bool RING>
__global__ __launch_bounds__((W2 / 2) * LP) void k_inner(
    const double *__restrict__ gram, int nsplit, int npairs, int step,
    const int16_t *__restrict__ itab, int isteps, int inner_max, double tol, int sort, int variant,
    double *__restrict__ Zt, unsigned long long *__restrict__ cnt, int *__restrict__ status,
    unsigned long long *__restrict__ phase)
{
    const int pr = blockIdx.x;
    const int ns = nsplit > 0 ? nsplit : 1;   // nsplit 0: one triangular factor per matrix
    const double *pa = gram + (size_t)(pr * 2) * ns * (W2 * W2);
    __shared__ __attribute__((aligned(16))) double lds[inner_lds<W2>()];
    inner_solve<W2, LP, RING>(pa, pa + (size_t)ns * (W2 * W2), nsplit, W2 * W2, itab, isteps,
                        inner_max, tol, sort, variant,
                        Zt + (size_t)pr * (W2 * W2), cnt + ((size_t)step * npairs + pr) * 4,
                        status, step * 65536 + pr,
                        phase ? phase + ((size_t)step * npairs + pr) * 8 : nullptr, lds);
}

// ------------------------------------------------------------------------
// Block update (paper: Section 2.3, [F_p F_q] <- [F_p F_q] Z_tilde and the
// same for G and Z; Section 3.5.4 does it in place with one read and one
// write of the block columns).  FP64 MFMA 16x16x4 computing
// D' = Z_tilde^T X^T for 16-row tiles X of the block-column pair, so the
// loads of X and the stores of D' = (X Z_tilde)^T are both 128-byte column
// segments.  Z_tilde is staged once per workgroup in LDS (padded to avoid
// bank conflicts) and read as MFMA A-fragments per k-step, which keeps the
// register count low enough for several waves per SIMD.  A wave reads
// all W2 columns of its 16 rows before writing them: in place, no races.
// Grid (row ranges of the rows of Fw, Gw and Zw in sequence, pairs); each workgroup owns
// 4 * rows_per_wave consecutive rows, its waves taking 16-row tiles in turn.
// ------------------------------------------------------------------------
// A pair whose inner solve left Z_tilde = I (its counter word 3, written by
// the inner solver) is skipped (Section 2.5): every workgroup of the pair
// returns at once.
template <int W2>
__global__ __launch_bounds__(256) void k_update(double *__restrict__ Fw, double *__restrict__ Gw,
                                                double *__restrict__ Zw, int64_t mfw,
                                                int64_t mgw, int64_t nzw,
                                                const int *__restrict__ pairs,
                                                const double *__restrict__ Zt, int rows_per_wave,
                                                const unsigned long long *__restrict__ scnt)
{
    if (scnt[(size_t)blockIdx.y * 4 + 3]) return;
    // The rows of F, G and Z (each padded to a multiple of 64) are taken as
    // one sequence and cut into equal ranges of 4 * rows_per_wave; a range
    // that reaches the end of one matrix continues in the next (a 16-row
    // tile never straddles two), so the launch is one rounding of the
    // total, not three.
    const int pr = blockIdx.y;
    const int p = pairs[2 * pr], q = pairs[2 * pr + 1];
    const double *zt = Zt + (size_t)pr * (W2 * W2);
    const int64_t span = 4 * (int64_t)rows_per_wave;
    const int64_t vb = (int64_t)blockIdx.x * span;
    const int64_t total = mfw + mgw + nzw;
    const int64_t ve = (vb + span < total) ? vb + span : total;
    __shared__ double sz[update_lds<W2>()];
    update_row_seq<W2, 4>(
        [=](int64_t v, double *&y, int64_t &ld, int64_t &r) {
            if (v < mfw) {
                y = Fw;
                ld = mfw;
                r = v;
            } else if (v < mfw + mgw) {
                y = Gw;
                ld = mgw;
                r = v - mfw;
            } else {
                y = Zw;
                ld = nzw;
                r = v - mfw - mgw;
            }
        },
        p, q, vb, ve, zt, sz);
}

// ------------------------------------------------------------------------
// Final extraction (paper: Section 2.4 post-iterative phase and the rescale
// kernel of Section 3.4) and descending sort (Section 1).
// k_colnorms: one wave per working column: ||f_j||, ||g_j||, sigma_j =
//   ||f_j|| / ||g_j||, and whether the column is a bordering column (its Z
//   column is nonzero only in rows >= n).
// k_rank: stable descending rank of sigma among the non-bordering columns.
// k_scatter: U(:,rank) = f_j/||f_j||, V(:,rank) = g_j/||g_j||,
//   Z(:,rank) = theta_j z_j, Sigma_F = theta ||f_j||, Sigma_G = theta ||g_j||.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_colnorms(const double *__restrict__ Fw,
                                                  const double *__restrict__ Gw,
                                                  const double *__restrict__ Zw, int64_t mfw,
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
    const double *f = Fw + j * mfw, *g = Gw + j * mgw, *z = Zw + j * nzw;
    double a = 0.0, b = 0.0;
    for (int64_t r = lane; r < mfw; r += 64) a = fma(f[r], f[r], a);
    for (int64_t r = lane; r < mgw; r += 64) b = fma(g[r], g[r], b);
    int bz = 0;
    for (int64_t r = n + lane; r < nw; r += 64) bz |= (z[r] != 0.0);
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

__global__ __launch_bounds__(256) void k_rank(const double *__restrict__ sig,
                                              const int *__restrict__ border, int64_t nw,
                                              int *__restrict__ rank)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nw) return;
    if (border[j]) {
        rank[j] = -1;
        return;
    }
    const double s = sig[j];
    int64_t r = 0;
    for (int64_t k = 0; k < nw; ++k) {
        if (border[k]) continue;
        const double t = sig[k];
        r += (t > s) || (t == s && k < j);
    }
    rank[j] = (int)r;
}

__global__ __launch_bounds__(256) void k_scatter(
    const double *__restrict__ Fw, const double *__restrict__ Gw, const double *__restrict__ Zw,
    int64_t mfw, int64_t mgw, int64_t nzw, int64_t mf, int64_t mg, int64_t n, int64_t nw,
    const double *__restrict__ sf, const double *__restrict__ sg, const int *__restrict__ rank,
    double *__restrict__ U, int64_t ldu, double *__restrict__ V, int64_t ldv,
    double *__restrict__ Z, int64_t ldz, double *__restrict__ sigma,
    double *__restrict__ sigma_f, double *__restrict__ sigma_g)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nw) return;
    const int rk = rank[j];
    if (rk < 0 || rk >= n) return;
    const double x = sf[j], y = sg[j];
    const double th = 1.0 / sqrt(x * x + y * y);
    const double ix = 1.0 / x, iy = 1.0 / y;
    const double *f = Fw + j * mfw, *g = Gw + j * mgw, *z = Zw + j * nzw;
    double *u = U + (int64_t)rk * ldu, *v = V + (int64_t)rk * ldv, *zo = Z + (int64_t)rk * ldz;
    for (int64_t r = lane; r < mf; r += 64) u[r] = f[r] * ix;
    for (int64_t r = lane; r < mg; r += 64) v[r] = g[r] * iy;
    for (int64_t r = lane; r < n; r += 64) zo[r] = z[r] * th;
    if (lane == 0) {
        sigma[rk] = x / y;
        sigma_f[rk] = x * th;
        sigma_g[rk] = y * th;
    }
}

// n = 1 closed form (paper, Section 2).  One wave.
__global__ __launch_bounds__(64) void k_n1(int64_t mf, int64_t mg, double *__restrict__ F,
                                           double *__restrict__ G, double *__restrict__ Z,
                                           double *__restrict__ sigma,
                                           double *__restrict__ sigma_f,
                                           double *__restrict__ sigma_g,
                                           int *__restrict__ status)
{
    const int lane = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t r = lane; r < mf; r += 64) a = fma(F[r], F[r], a);
    for (int64_t r = lane; r < mg; r += 64) b = fma(G[r], G[r], b);
    a = wave_sum(a);
    b = wave_sum(b);
    const double nf = sqrt(a), ng = sqrt(b), rr = sqrt(a + b);
    for (int64_t r = lane; r < mf; r += 64) F[r] = F[r] / nf;
    for (int64_t r = lane; r < mg; r += 64) G[r] = G[r] / ng;
    if (lane == 0) {
        Z[0] = 1.0 / rr;
        sigma[0] = nf / ng;
        sigma_f[0] = nf / rr;
        sigma_g[0] = ng / rr;
        if (!(isfinite(nf / ng) && nf > 0.0 && ng > 0.0)) atomicOr(status + ST_FLAGS, FLAG_NONFINITE);
    }
}

// Diagnostic evaluation of hz_real_2x2_fast, one thread per pivot pair.
__global__ __launch_bounds__(256) void k_eval_2x2(int64_t count, const double *__restrict__ in,
                                                  double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    double z11, z21, z12, z22;
    bool c2small;
    hz_real_2x2_fast(in[4 * i], in[4 * i + 1], in[4 * i + 2], in[4 * i + 3], z11, z21, z12, z22,
                     c2small);
    out[4 * i] = z11;
    out[4 * i + 1] = z21;
    out[4 * i + 2] = z12;
    out[4 * i + 3] = z22;
}

// Diagnostic: the device's rounded-down product and its error term
// (Appendix A) on `count` operand pairs.
__global__ __launch_bounds__(256) void k_eval_mul_rd(int64_t count, const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ c, double *__restrict__ d)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    const double x = a[e], y = b[e];
    const double cd = mul_rd(x, y);
    c[e] = cd;
    d[e] = fma(x, y, -cd);
}

void launch_eval_mul_rd(int64_t count, const double *a, const double *b, double *c, double *d,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_eval_mul_rd, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       count, a, b, c, d);
}

void launch_eval_2x2(int64_t count, const double *in, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_eval_2x2, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count,
                       in, out);
}

// End-of-sweep summary (one workgroup): totals of the per-(step, pair)
// counters (integer sums: order-independent), the largest off-diagonal
// measure of the sweep when offd is given, and the status words, so the
// host reads SWEEP_TOT_N words per sweep.
__global__ __launch_bounds__(256) void k_sweep_totals(const unsigned long long *__restrict__ cnt,
                                                      int n, const double *__restrict__ offd,
                                                      int noffd, const int *__restrict__ status,
                                                      unsigned long long *__restrict__ tot)
{
    __shared__ unsigned long long s3[4][256];
    __shared__ double so[256];
    const int t = threadIdx.x;
    unsigned long long a = 0, b = 0, c = 0, d = 0;
    for (int i = t; i < n; i += 256) {
        a += cnt[4 * (size_t)i];
        b += cnt[4 * (size_t)i + 1];
        c += cnt[4 * (size_t)i + 2];
        d += cnt[4 * (size_t)i + 3];
    }
    double m = 0.0;
    if (offd)
        for (int i = t; i < noffd; i += 256) m = fmax(m, offd[i]);
    s3[0][t] = a;
    s3[1][t] = b;
    s3[2][t] = c;
    s3[3][t] = d;
    so[t] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            s3[0][t] += s3[0][t + h];
            s3[1][t] += s3[1][t + h];
            s3[2][t] += s3[2][t + h];
            s3[3][t] += s3[3][t + h];
            so[t] = fmax(so[t], so[t + h]);
        }
        __syncthreads();
    }
    if (t == 0) {
        tot[TOT_ALL] = s3[0][0];
        tot[TOT_BIG] = s3[1][0];
        tot[TOT_ISW] = s3[2][0];
        tot[TOT_OFFD] = __builtin_bit_cast(unsigned long long, so[0]);
        tot[TOT_FLAGS] = (unsigned long long)(unsigned)status[ST_FLAGS];
        tot[TOT_FAILPAIR] = (unsigned long long)(unsigned)status[ST_FAILPAIR];
        tot[TOT_SKIP] = s3[3][0];
    }
}

// ------------------------------------------------------------------ launchers

void launch_sweep_totals(const Plan &P, const Ptrs &W, hipStream_t s)
{
    hipLaunchKernelGGL(k_sweep_totals, dim3(1), dim3(256), 0, s, W.cnt, P.steps * P.npairs,
                       P.mixed ? W.offd : nullptr, P.steps * P.npairs * 2, W.status, W.tot);
}

void launch_prescale_real(const Plan &P, const Ptrs &W, const double *F, int64_t ldf,
                          const double *G, int64_t ldg, hipStream_t s)
{
    const unsigned nb = (unsigned)((P.nw + 3) / 4);
    hipLaunchKernelGGL(k_prescale_copy, dim3(nb), dim3(256), 0, s, P.mf, P.mg, P.n, F, ldf, G,
                       ldg, P.nw, P.mfw, P.mgw, P.nzw, W.Fw, W.Gw, W.Zw, W.status);
}

template <int W2, int LP, bool RING>
static void inner_launch(const Plan &P, const Ptrs &W, int step, const hz_params &prm,
                         double tol, const double *src, int ns, hipStream_t s)
{
    hipLaunchKernelGGL((k_inner<W2, LP, RING>), dim3(P.npairs), dim3((W2 / 2) * LP), 0, s, src,
                       ns, P.npairs, step, W.itab, P.isteps, prm.inner_max_sweeps, tol, prm.sort,
                       prm.variant, W.Zt, W.cnt, W.status, W.phase);
}

template <int W2>
static void inner_impl(const Plan &P, const Ptrs &W, int step, const hz_params &prm, double tol,
                       bool partials, hipStream_t s)
{
    const double *src = partials ? W.part : W.gram;
    const int ns = partials ? P.splits : (prm.pivot_qr ? 0 : 1);
    const bool ring = (prm.inner_ordering == HZ_ORD_RING);
    if constexpr (W2 == 16) {
        if (ring) inner_launch<W2, 8, true>(P, W, step, prm, tol, src, ns, s);
        else inner_launch<W2, 8, false>(P, W, step, prm, tol, src, ns, s);
    } else {
        if (P.inner_lp == 4) {
            if (ring) inner_launch<W2, 4, true>(P, W, step, prm, tol, src, ns, s);
            else inner_launch<W2, 4, false>(P, W, step, prm, tol, src, ns, s);
        } else if (P.inner_lp == 8) {
            if (ring) inner_launch<W2, 8, true>(P, W, step, prm, tol, src, ns, s);
            else inner_launch<W2, 8, false>(P, W, step, prm, tol, src, ns, s);
        } else {
            if (ring) inner_launch<W2, 16, true>(P, W, step, prm, tol, src, ns, s);
            else inner_launch<W2, 16, false>(P, W, step, prm, tol, src, ns, s);
        }
    }
}

void launch_inner_real(const Plan &P, const Ptrs &W, int step, const hz_params &prm, double tol,
                       bool partials, hipStream_t s)
{
    switch (P.W2) {
    case 16: inner_impl<16>(P, W, step, prm, tol, partials, s); break;
    case 32: inner_impl<32>(P, W, step, prm, tol, partials, s); break;
    default: inner_impl<64>(P, W, step, prm, tol, partials, s); break;
    }
}

void launch_gram_sum(const Plan &P, const Ptrs &W, hipStream_t s)
{
    const int W2 = P.W2;
    switch (W2) {
    case 16:
        hipLaunchKernelGGL(k_gram_sum<16>, dim3(1, 2 * P.npairs), dim3(256), 0, s, W.part,
                           P.splits, W.gram);
        break;
    case 32:
        hipLaunchKernelGGL(k_gram_sum<32>, dim3(2, 2 * P.npairs), dim3(256), 0, s, W.part,
                           P.splits, W.gram);
        break;
    default:
        hipLaunchKernelGGL(k_gram_sum<64>, dim3(8, 2 * P.npairs), dim3(256), 0, s, W.part,
                           P.splits, W.gram);
        break;
    }
}

template <int W2>
static void step_impl(const Plan &P, const Ptrs &W, int step, const hz_params &prm, double tol,
                      hipStream_t s)
{
    const int *pairs = W.otab + (size_t)step * P.npairs * 2;
    prof_mark(K_GRAM, true, s);
    if (prm.pivot_qr) {
        launch_pivot_qr(P, W, step, s);
    } else {
        hipLaunchKernelGGL(k_gram<W2>, dim3(P.splits, P.npairs, 2), dim3(256), 0, s, W.Fw, W.Gw,
                           P.mfw, P.mgw, pairs, P.splits, W.part);
        launch_gram_sum(P, W, s);
    }
    prof_mark(K_GRAM, false, s);
    prof_mark(K_INNER, true, s);
    inner_impl<W2>(P, W, step, prm, tol, false, s);
    prof_mark(K_INNER, false, s);
    const int64_t rpt = 4 * (int64_t)P.upd_rows;
    const int nt = (int)((P.mfw + P.mgw + P.nzw + rpt - 1) / rpt);
    prof_mark(K_UPDATE, true, s);
    hipLaunchKernelGGL(k_update<W2>, dim3(nt, P.npairs), dim3(256), 0, s, W.Fw, W.Gw, W.Zw,
                       P.mfw, P.mgw, P.nzw, pairs, W.Zt, P.upd_rows,
                       W.cnt + (size_t)step * P.npairs * 4);
    prof_mark(K_UPDATE, false, s);
}

void launch_step_real(const Plan &P, const Ptrs &W, int step, const hz_params &prm, double tol,
                      hipStream_t s)
{
    switch (P.W2) {
    case 16: step_impl<16>(P, W, step, prm, tol, s); break;
    case 32: step_impl<32>(P, W, step, prm, tol, s); break;
    default: step_impl<64>(P, W, step, prm, tol, s); break;
    }
}

void launch_rank(const Plan &P, const Ptrs &W, hipStream_t s)
{
    hipLaunchKernelGGL(k_rank, dim3((unsigned)((P.nw + 255) / 256)), dim3(256), 0, s, W.sig,
                       W.border, P.nw, W.rank);
}

void launch_finish_real(const Plan &P, const Ptrs &W, double *F, int64_t ldf, double *G,
                        int64_t ldg, double *Z, int64_t ldz, double *sigma, double *sigma_f,
                        double *sigma_g, hipStream_t s)
{
    const unsigned nb4 = (unsigned)((P.nw + 3) / 4);
    hipLaunchKernelGGL(k_colnorms, dim3(nb4), dim3(256), 0, s, W.Fw, W.Gw, W.Zw, P.mfw, P.mgw,
                       P.nzw, P.n, P.nw, W.sf, W.sg, W.sig, W.border, W.status);
    launch_rank(P, W, s);
    hipLaunchKernelGGL(k_scatter, dim3(nb4), dim3(256), 0, s, W.Fw, W.Gw, W.Zw, P.mfw, P.mgw,
                       P.nzw, P.mf, P.mg, P.n, P.nw, W.sf, W.sg, W.rank, F, ldf, G, ldg, Z, ldz,
                       sigma, sigma_f, sigma_g);
}

void launch_n1_real(int64_t mf, int64_t mg, double *F, double *G, double *Z, double *sigma,
                    double *sigma_f, double *sigma_g, int *status, hipStream_t s)
{
    hipLaunchKernelGGL(k_n1, dim3(1), dim3(64), 0, s, mf, mg, F, G, Z, sigma, sigma_f, sigma_g,
                       status);
}

}  // namespace hz
