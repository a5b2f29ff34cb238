// hz_shorten.hip -- QR shortening of a tall pair before the sweeps (paper,
// Section 2, the paragraph before the prescaling): F P1 = Q_F R_F and
// (G P1) P2 = Q_G R_G with column pivoting; the iteration then runs on the
// square pair F'' = R_F P2, G'' = R_G of order n, and the factors of (F, G)
// are recovered as Z = P1 P2 Z'', U = Q_F U'', V = Q_G V''.
//
// The column-pivoted QR of Y (m x n) is formed GPU-style, from dense
// products and n x n factorizations instead of a Householder panel loop
// over the tall matrix:
//   1. S = Y^T Y (FP64 MFMA);
//   2. Cholesky of S with diagonal pivoting, P^T S P = R1^T R1: at each step
//      the column with the largest remaining Schur-complement diagonal is
//      taken, which is the column of largest remaining norm -- the pivot
//      rule of column-pivoted QR, so in exact arithmetic P and R1 are that
//      factorization's;
//   3. Q1 = (Y P) R1^-1 (blocked triangular solve on the right, in place);
//   4. one refinement pass: R2^T R2 = Q1^T Q1 (Cholesky without pivoting),
//      Q = Q1 R2^-1, R = R2 R1 (Cholesky QR applied twice), which restores
//      the orthogonality of Q to rounding level while kappa(Y)^2 eps << 1.
// A non-positive or non-finite pivot sets FLAG_CHOL / FLAG_NONFINITE (the
// shortening needs F and G each of full column rank); the permutation stays
// a permutation in every case, so every later index is in range.
#include <float.h>
#include <math.h>
#include <string.h>

#include "hz_device.h"
#include "hz_internal.h"

namespace hz {

// ------------------------------------------------------------------ GEMM
// C (M x N) = alpha * op(A) * B + beta * C0, column-major.  op(A) = A
// (M x K, ld lda) or, with TA, A^T for A of K x M.  C0 may alias C (each
// workgroup reads its C0 tile only after its whole K loop, and writes the
// same tile); with beta == 0 C0 is not read.  A 64 x 64 tile of C per
// workgroup of four waves, each wave 32 x 32 (2 x 2 MFMA 16x16x4 blocks);
// K runs in chunks of 32 staged in LDS, the next chunk prefetched into
// registers while the current one is multiplied.
static constexpr int GK = 32, GLD = 66;

template <bool TA>
__global__ __launch_bounds__(256) void k_gemm(int64_t M, int64_t N, int64_t K, double alpha,
                                              const double *__restrict__ A, int64_t lda,
                                              const double *__restrict__ B, int64_t ldb,
                                              double beta, const double *C0, int64_t ldc0,
                                              double *C, int64_t ldc)
{
    __shared__ __attribute__((aligned(16))) double sA[GK * GLD];   // [k][i]
    __shared__ __attribute__((aligned(16))) double sB[GK * GLD];   // [k][j]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
    const int wr = 32 * (wave & 1), wc = 32 * (wave >> 1);
    const int i16 = lane & 15, k4 = lane >> 4;
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    // per-thread load coordinates: 8 elements of the A chunk, 8 of the B chunk
    double ra[8], rb[8];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = tid + 256 * t;
            int ii, kk;
            if (TA) { ii = e / GK; kk = e % GK; }      // A^T: k contiguous in memory
            else { ii = e % 64; kk = e / 64; }         // A: i contiguous in memory
            const int64_t gi = r0 + ii, gk = k0 + kk;
            ra[t] = (gi < M && gk < K) ? (TA ? A[gi * lda + gk] : A[gk * lda + gi]) : 0.0;
            const int jj = e / GK, kb = e % GK;
            const int64_t gj = c0 + jj, gkb = k0 + kb;
            rb[t] = (gj < N && gkb < K) ? B[gj * ldb + gkb] : 0.0;
        }
    };
    if (K > 0) load(0);
    for (int64_t k0 = 0; k0 < K; k0 += GK) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = tid + 256 * t;
            int ii, kk;
            if (TA) { ii = e / GK; kk = e % GK; }
            else { ii = e % 64; kk = e / 64; }
            sA[kk * GLD + ii] = ra[t];
            sB[(e % GK) * GLD + e / GK] = rb[t];
        }
        __syncthreads();
        if (k0 + GK < K) load(k0 + GK);
#pragma unroll
        for (int ks = 0; ks < GK / 4; ++ks) {
            const int kk = 4 * ks + k4;
            double fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = sA[kk * GLD + wr + 16 * a + i16];
#pragma unroll
            for (int b = 0; b < 2; ++b) fb[b] = sB[kk * GLD + wc + 16 * b + i16];
            // D' = B^T A^T: element r of lane l is C(i = l % 16, j = 4 r + l / 16)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(fb[b], fa[a], acc[a][b]);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = r0 + wr + 16 * a + i16;
                const int64_t gj = c0 + wc + 16 * b + 4 * r + k4;
                if (gi < M && gj < N) {
                    double v = alpha * acc[a][b][r];
                    if (beta != 0.0) v += beta * C0[gj * ldc0 + gi];
                    C[gj * ldc + gi] = v;
                }
            }
}

static void gemm(bool ta, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                 int64_t lda, const double *B, int64_t ldb, double beta, const double *C0,
                 int64_t ldc0, double *C, int64_t ldc, hipStream_t s)
{
    if (M <= 0 || N <= 0) return;
    const dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
    if (ta)
        hipLaunchKernelGGL(k_gemm<true>, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb,
                           beta, C0, ldc0, C, ldc);
    else
        hipLaunchKernelGGL(k_gemm<false>, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb,
                           beta, C0, ldc0, C, ldc);
}

// ------------------------------------------------------ pivoted Cholesky
// S (n x n, ld lds, both triangles) is the current Schur complement; Rt
// (n x n, ld ldr) receives R transposed and in the original column order:
// column j of Rt is row j of R, entry c of it belongs to original column c
// (zero once c has been pivoted at an earlier step).  d[c] is the current
// diagonal of S, done[c] marks pivoted columns, piv[j] the original column
// taken at step j.  One workgroup of PT threads runs the nb steps of the
// panel [j0, j0 + nb); thread t owns the columns t, t + PT, ... (CPT of
// them) and keeps their panel rows of R in registers.
static constexpr int PT = 1024;

template <int CPT, int NB>
__global__ __launch_bounds__(PT) void k_pchol_panel(int n, const double *__restrict__ S,
                                                    int64_t lds, double *__restrict__ Rt,
                                                    int64_t ldr, double *__restrict__ dg,
                                                    int *__restrict__ doneg, int *__restrict__ piv,
                                                    int j0, int nb, int pivoting,
                                                    int *__restrict__ status)
{
    __shared__ double s_bv[PT / 64];
    __shared__ int s_bi[PT / 64];
    __shared__ double s_rp[NB + 1];
    __shared__ int s_p;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int jn = (j0 + nb < n) ? j0 + nb : n;
    double dl[CPT];
    int dn[CPT];
    double rr[NB][CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int c = tid + PT * u;
        if (c < n) {
            dl[u] = (j0 == 0) ? S[(int64_t)c * lds + c] : dg[c];
            dn[u] = (j0 == 0) ? 0 : doneg[c];
        } else {
            dl[u] = 0.0;
            dn[u] = 1;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) rr[i][u] = 0.0;
    }
    for (int j = j0; j < jn; ++j) {
        const int t = j - j0;
        int p = j;
        if (pivoting) {
            // largest remaining diagonal (a NaN counts as +inf, so that it is
            // taken and reported); ties go to the smaller column index
            double bv = -INFINITY;
            int bi = INT_MAX;
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = tid + PT * u;
                const double key = (dl[u] != dl[u]) ? INFINITY : dl[u];
                if (!dn[u] && (key > bv || (key == bv && c < bi))) {
                    bv = key;
                    bi = c;
                }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int oi = __shfl_xor(bi, off);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            if (lane == 0) {
                s_bv[wv] = bv;
                s_bi[wv] = bi;
            }
            __syncthreads();
            if (tid == 0) {
                double b = s_bv[0];
                int ib = s_bi[0];
                for (int w = 1; w < PT / 64; ++w)
                    if (s_bv[w] > b || (s_bv[w] == b && s_bi[w] < ib)) {
                        b = s_bv[w];
                        ib = s_bi[w];
                    }
                s_p = ib;
            }
            __syncthreads();
            p = s_p;
        }
        // the owner of column p publishes its panel rows of R and d[p]
        if (tid == p % PT) {
            const int up = p / PT;
#pragma unroll
            for (int u = 0; u < CPT; ++u)
                if (u == up) {
#pragma unroll
                    for (int i = 0; i < NB; ++i)
                        if (i < t) s_rp[i] = rr[i][u];
                    s_rp[NB] = dl[u];
                    dn[u] = 1;
                }
        }
        __syncthreads();
        const double dp = s_rp[NB];
        const bool nonfinite = !(fabs(dp) <= DBL_MAX);
        const bool bad = nonfinite || !(dp > 0.0);
        const double r = bad ? 1.0 : sqrt(dp);
        if (bad && tid == 0) atomicOr(&status[ST_FLAGS], nonfinite ? FLAG_NONFINITE : FLAG_CHOL);
        const double *srow = S + (int64_t)p * lds;   // column p = row p (symmetric)
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = tid + PT * u;
            double v = 0.0;
            if (c < n && !dn[u]) {
                double sv = srow[c];
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    if (i < t) sv -= s_rp[i] * rr[i][u];
                v = sv / r;
                dl[u] -= v * v;
            } else if (c == p) {
                v = r;
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (i == t) rr[i][u] = v;
            if (c < n) Rt[(int64_t)j * ldr + c] = v;
        }
        if (tid == 0) piv[j] = p;
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int c = tid + PT * u;
        if (c < n) {
            dg[c] = dl[u];
            doneg[c] = dn[u];
        }
    }
}

// Trailing update after a panel: S -= Rt(:, j0:j0+nb) Rt(:, j0:j0+nb)^T over
// all of S (entries of pivoted columns are never read again).
__global__ __launch_bounds__(256) void k_pchol_update(int n, double *__restrict__ S, int64_t lds,
                                                      const double *__restrict__ Rt, int64_t ldr,
                                                      int j0, int nb)
{
    __shared__ double a[16][64], b[16][64];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    for (int e = tid; e < 16 * 64; e += 256) {
        const int i = e / 64, x = e % 64;
        const bool ok = i < nb;
        a[i][x] = (ok && r0 + x < n) ? Rt[(int64_t)(j0 + i) * ldr + r0 + x] : 0.0;
        b[i][x] = (ok && c0 + x < n) ? Rt[(int64_t)(j0 + i) * ldr + c0 + x] : 0.0;
    }
    __syncthreads();
    const int r = tid & 63;
    if (r0 + r >= n) return;
    for (int q = tid >> 6; q < 64; q += 4) {
        if (c0 + q >= n) break;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc += a[i][r] * b[i][q];
        S[(int64_t)(c0 + q) * lds + r0 + r] -= acc;
    }
}

// ------------------------------------------------- triangular pieces
// Inverses of the 64 x 64 diagonal blocks of the upper triangular R (n x n,
// ld ldr): block J is written to X + 4096 J (column-major 64 x 64), the
// trailing partial block padded with the identity.  Each wave solves
// R_JJ x = e_j for its columns by column-oriented back substitution, one
// row per lane.
__global__ __launch_bounds__(256) void k_trinv_diag(int n, const double *__restrict__ R,
                                                    int64_t ldr, double *__restrict__ X)
{
    __shared__ double sR[64 * 65];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b0 = blockIdx.x * 64;
    const int bs = (n - b0 < 64) ? n - b0 : 64;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e % 64, c = e / 64;
        double v = (r == c) ? 1.0 : 0.0;
        if (r < bs && c < bs && r <= c) v = R[(int64_t)(b0 + c) * ldr + b0 + r];
        sR[c * 65 + r] = v;
    }
    __syncthreads();
    for (int jj = 0; jj < 16; ++jj) {
        const int j = wave + 4 * jj;
        double x = (lane == j) ? 1.0 : 0.0;
        for (int k = j; k >= 0; --k) {
            const double xk = __shfl(x, k) / sR[k * 65 + k];
            if (lane == k) x = xk;
            else if (lane < k) x -= xk * sR[k * 65 + lane];
        }
        X[(int64_t)blockIdx.x * 4096 + j * 64 + lane] = x;
    }
}

// dst(0:m, j) = src(0:m, idx[j]) for j < ncol
__global__ __launch_bounds__(256) void k_gather_cols(int64_t m, int ncol, const int *__restrict__ idx,
                                                     const double *__restrict__ src, int64_t lds,
                                                     double *__restrict__ dst, int64_t ldd)
{
    const int j = blockIdx.y;
    const double *s = src + (int64_t)idx[j] * lds;
    double *d = dst + (int64_t)j * ldd;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
        d[i] = s[i];
}

// R(i, k) = Rt(idx[k], i) for i, k < n: the upper triangular factor in the
// pivoted column order (idx = piv), or the plain transpose (idx = null).
__global__ __launch_bounds__(256) void k_gather_rt(int n, const int *__restrict__ idx,
                                                   const double *__restrict__ Rt, int64_t ldr,
                                                   double *__restrict__ R, int64_t ldo)
{
    __shared__ double tile[32][33];
    const int i0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    // read Rt(idx[k], i): for fixed i (a column of Rt) the rows idx[k]
    for (int y = ty; y < 32; y += 8) {
        const int i = i0 + y, k = k0 + tx;
        double v = 0.0;
        if (i < n && k < n) v = Rt[(int64_t)i * ldr + (idx ? idx[k] : k)];
        tile[y][tx] = v;
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int k = k0 + y, i = i0 + tx;
        if (i < n && k < n) R[(int64_t)k * ldo + i] = tile[tx][y];
    }
}

// Z(q[j], :) = Z2(j, :): rows of the square pair's Z back in the original
// column order of (F, G).
__global__ __launch_bounds__(256) void k_scatter_rows(int n, const int *__restrict__ q,
                                                      const double *__restrict__ Z2, int64_t ld2,
                                                      double *__restrict__ Z, int64_t ldz)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int j = (int)(e % n), c = (int)(e / n);
    Z[(int64_t)c * ldz + q[j]] = Z2[(int64_t)c * ld2 + j];
}

// inv[p[j]] = j, and q2[j] = inv1[q[j]] when inv1 is given (the slot of
// q[j] in the order p of the first factorization).
__global__ __launch_bounds__(256) void k_perm_inverse(int n, const int *__restrict__ p,
                                                      int *__restrict__ inv)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) inv[p[j]] = j;
}

__global__ __launch_bounds__(256) void k_perm_compose(int n, const int *__restrict__ inv1,
                                                      const int *__restrict__ q,
                                                      int *__restrict__ q2)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) q2[j] = inv1[q[j]];
}

// ------------------------------------------------------------------ host

static int panel_width(int cpt) { return cpt <= 2 ? 16 : (cpt == 4 ? 8 : 4); }

int shorten_cpt(int64_t n)
{
    if (n <= PT) return 1;
    if (n <= 2 * PT) return 2;
    if (n <= 4 * PT) return 4;
    if (n <= 8 * PT) return 8;
    return 0;
}

bool make_splan(int64_t mf, int64_t mg, int64_t n, size_t solve_bytes, SPlan &S)
{
    S = SPlan();
    S.cpt = shorten_cpt(n);
    if (!S.cpt || n < 2) return false;
    S.mf = mf;
    S.mg = mg;
    S.n = n;
    S.nb = panel_width(S.cpt);
    S.ldqf = (mf + 7) / 8 * 8;
    S.ldqg = (mg + 7) / 8 * 8;
    S.ldn = (n + 7) / 8 * 8;
    S.nblk = (int)((n + 63) / 64);
    const int64_t mt = S.ldqf > S.ldqg ? S.ldqf : S.ldqg;
    const size_t nn = 8 * (size_t)S.ldn * n;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    S.o_qf = o; o = al(o + 8 * (size_t)S.ldqf * n);
    S.o_qg = o; o = al(o + 8 * (size_t)S.ldqg * n);
    S.o_s = o; o = al(o + nn);
    S.o_rt = o; o = al(o + nn);
    S.o_r1f = o; o = al(o + nn);
    S.o_r1g = o; o = al(o + nn);
    S.o_r2 = o; o = al(o + nn);
    S.o_f2 = o; o = al(o + nn);
    S.o_g2 = o; o = al(o + nn);
    S.o_z2 = o; o = al(o + nn);
    S.o_t = o; o = al(o + 8 * (size_t)mt * 64);
    S.o_xd = o; o = al(o + 8 * (size_t)S.nblk * 4096);
    S.o_d = o; o = al(o + 8 * (size_t)n);
    S.o_done = o; o = al(o + 4 * (size_t)n);
    S.o_p1 = o; o = al(o + 4 * (size_t)n);
    S.o_q = o; o = al(o + 4 * (size_t)n);
    S.o_inv1 = o; o = al(o + 4 * (size_t)n);
    S.o_p2 = o; o = al(o + 4 * (size_t)n);
    S.o_id = o; o = al(o + 4 * (size_t)n);
    S.o_status = o; o = al(o + 4 * ST_NSLOTS);
    S.o_solve = o; o = al(o + solve_bytes);
    S.total = o;
    return true;
}

// Cholesky of S (ld S.ldn) into Rt, with diagonal pivoting or without.
static void pchol(const SPlan &P, double *S, double *Rt, double *d, int *done, int *piv,
                  bool pivoting, int *status, hipStream_t s)
{
    const int n = (int)P.n, nb = P.nb;
    const unsigned gt = (unsigned)((n + 63) / 64);
    for (int j0 = 0; j0 < n; j0 += nb) {
        switch (P.cpt) {
        case 1:
            hipLaunchKernelGGL((k_pchol_panel<1, 16>), dim3(1), dim3(PT), 0, s, n, S, P.ldn, Rt,
                               P.ldn, d, done, piv, j0, nb, pivoting ? 1 : 0, status);
            break;
        case 2:
            hipLaunchKernelGGL((k_pchol_panel<2, 16>), dim3(1), dim3(PT), 0, s, n, S, P.ldn, Rt,
                               P.ldn, d, done, piv, j0, nb, pivoting ? 1 : 0, status);
            break;
        case 4:
            hipLaunchKernelGGL((k_pchol_panel<4, 8>), dim3(1), dim3(PT), 0, s, n, S, P.ldn, Rt,
                               P.ldn, d, done, piv, j0, nb, pivoting ? 1 : 0, status);
            break;
        default:
            hipLaunchKernelGGL((k_pchol_panel<8, 4>), dim3(1), dim3(PT), 0, s, n, S, P.ldn, Rt,
                               P.ldn, d, done, piv, j0, nb, pivoting ? 1 : 0, status);
            break;
        }
        if (j0 + nb < n)
            hipLaunchKernelGGL(k_pchol_update, dim3(gt, gt), dim3(256), 0, s, n, S, P.ldn, Rt,
                               P.ldn, j0, nb);
    }
}

// In place Y (m x n, ld ldy) <- Y R^-1 for the upper triangular R (ld ldn),
// by 64-column blocks: T = Y_J - Y_{<J} R_{<J,J}, then Y_J = T inv(R_JJ).
static void trsm_right(const SPlan &P, int64_t m, double *Y, int64_t ldy, const double *R,
                       double *T, double *Xd, hipStream_t s)
{
    const int n = (int)P.n;
    hipLaunchKernelGGL(k_trinv_diag, dim3((unsigned)P.nblk), dim3(256), 0, s, n, R, P.ldn, Xd);
    for (int J = 0; J < P.nblk; ++J) {
        const int64_t j0 = 64 * (int64_t)J, bs = (n - j0 < 64) ? n - j0 : 64;
        gemm(false, m, bs, j0, -1.0, Y, ldy, R + j0 * P.ldn, P.ldn, 1.0, Y + j0 * ldy, ldy, T,
             m, s);
        gemm(false, m, bs, bs, 1.0, T, m, Xd + 4096 * (int64_t)J, 64, 0.0, nullptr, 0,
             Y + j0 * ldy, ldy, s);
    }
}

// Given Q = Y P (m x n, ld ldq: Y's columns already in the pivot order) and
// R = R1 with R1^T R1 = P^T Y^T Y P (ld ldn), forms the orthonormal factor
// in place (Q <- Y P R1^-1, then one Cholesky-QR refinement) and R <- R2 R1,
// so that Y P = Q R.
static void cholqr2(const SPlan &P, int64_t m, double *Q, int64_t ldq, double *R, char *b,
                    hipStream_t s)
{
    const int n = (int)P.n;
    double *S = (double *)(b + P.o_s), *Rt = (double *)(b + P.o_rt);
    double *R2 = (double *)(b + P.o_r2), *T = (double *)(b + P.o_t), *Xd = (double *)(b + P.o_xd);
    double *d = (double *)(b + P.o_d);
    int *done = (int *)(b + P.o_done), *id = (int *)(b + P.o_id);
    int *status = (int *)(b + P.o_status);
    trsm_right(P, m, Q, ldq, R, T, Xd, s);
    gemm(true, n, n, m, 1.0, Q, ldq, Q, ldq, 0.0, nullptr, 0, S, P.ldn, s);
    pchol(P, S, Rt, d, done, id, false, status, s);
    hipLaunchKernelGGL(k_gather_rt, dim3((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32)),
                       dim3(256), 0, s, n, (const int *)nullptr, Rt, P.ldn, R2, P.ldn);
    trsm_right(P, m, Q, ldq, R2, T, Xd, s);
    // R <- R2 R (both upper triangular); S is free again and takes the product
    gemm(false, n, n, n, 1.0, R2, P.ldn, R, P.ldn, 0.0, nullptr, 0, S, P.ldn, s);
    (void)hipMemcpyAsync(R, S, 8 * (size_t)P.ldn * n, hipMemcpyDeviceToDevice, s);
}

hipError_t launch_shorten(const SPlan &P, void *work, const double *F, int64_t ldf,
                          const double *G, int64_t ldg, hipStream_t s)
{
    char *b = (char *)work;
    const int n = (int)P.n;
    double *Qf = (double *)(b + P.o_qf), *Qg = (double *)(b + P.o_qg);
    double *S = (double *)(b + P.o_s), *Rt = (double *)(b + P.o_rt);
    double *R1f = (double *)(b + P.o_r1f), *R1g = (double *)(b + P.o_r1g);
    double *F2 = (double *)(b + P.o_f2), *G2 = (double *)(b + P.o_g2);
    double *d = (double *)(b + P.o_d);
    int *done = (int *)(b + P.o_done), *p1 = (int *)(b + P.o_p1), *q = (int *)(b + P.o_q);
    int *inv1 = (int *)(b + P.o_inv1), *p2 = (int *)(b + P.o_p2);
    int *status = (int *)(b + P.o_status);
    const unsigned g1 = (unsigned)((n + 255) / 256);
    const dim3 gtr((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32));
    hipError_t e = hipMemsetAsync(status, 0, 4 * ST_NSLOTS, s);
    if (e != hipSuccess) return e;
    // F P1 = Q_F R_F: pivots from the Gram of F
    gemm(true, n, n, P.mf, 1.0, F, ldf, F, ldf, 0.0, nullptr, 0, S, P.ldn, s);
    pchol(P, S, Rt, d, done, p1, true, status, s);
    hipLaunchKernelGGL(k_gather_rt, gtr, dim3(256), 0, s, n, (const int *)p1, Rt, P.ldn, R1f,
                       P.ldn);
    hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((P.mf + 255) / 256), (unsigned)n),
                       dim3(256), 0, s, P.mf, n, (const int *)p1, F, ldf, Qf, P.ldqf);
    cholqr2(P, P.mf, Qf, P.ldqf, R1f, b, s);
    // (G P1) P2 = Q_G R_G: the pivoted Cholesky of G^T G yields the combined
    // order q = P1 P2 directly; P2 is its position in the order P1
    gemm(true, n, n, P.mg, 1.0, G, ldg, G, ldg, 0.0, nullptr, 0, S, P.ldn, s);
    pchol(P, S, Rt, d, done, q, true, status, s);
    hipLaunchKernelGGL(k_gather_rt, gtr, dim3(256), 0, s, n, (const int *)q, Rt, P.ldn, R1g,
                       P.ldn);
    hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((P.mg + 255) / 256), (unsigned)n),
                       dim3(256), 0, s, P.mg, n, (const int *)q, G, ldg, Qg, P.ldqg);
    cholqr2(P, P.mg, Qg, P.ldqg, R1g, b, s);
    hipLaunchKernelGGL(k_perm_inverse, dim3(g1), dim3(256), 0, s, n, (const int *)p1, inv1);
    hipLaunchKernelGGL(k_perm_compose, dim3(g1), dim3(256), 0, s, n, (const int *)inv1,
                       (const int *)q, p2);
    // F'' = R_F P2, G'' = R_G
    hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256),
                       0, s, (int64_t)n, n, (const int *)p2, R1f, P.ldn, F2, P.ldn);
    e = hipMemcpyAsync(G2, R1g, 8 * (size_t)P.ldn * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_unshorten(const SPlan &P, void *work, double *U, int64_t ldu, double *V,
                            int64_t ldv, double *Z, int64_t ldz, hipStream_t s)
{
    char *b = (char *)work;
    const int n = (int)P.n;
    const double *Qf = (const double *)(b + P.o_qf), *Qg = (const double *)(b + P.o_qg);
    const double *U2 = (const double *)(b + P.o_f2), *V2 = (const double *)(b + P.o_g2);
    const double *Z2 = (const double *)(b + P.o_z2);
    const int *q = (const int *)(b + P.o_q);
    gemm(false, P.mf, n, n, 1.0, Qf, P.ldqf, U2, P.ldn, 0.0, nullptr, 0, U, ldu, s);
    gemm(false, P.mg, n, n, 1.0, Qg, P.ldqg, V2, P.ldn, 0.0, nullptr, 0, V, ldv, s);
    const int64_t nn = (int64_t)n * n;
    hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, n, q,
                       Z2, P.ldn, Z, ldz);
    return hipGetLastError();
}

}  // namespace hz
