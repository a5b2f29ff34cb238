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

// F and G are factored side by side: every kernel below takes the two
// problems in one launch (blockIdx.z, or blockIdx.x for the single-
// workgroup Cholesky panel), since each step is latency bound and the two
// factorizations are independent until the permutations are combined.
// Every kernel comes for real (CX false) and interleaved complex (CX true)
// elements; pointers are to doubles, indices and leading dimensions count
// elements.  In the complex case ^T reads as ^H and the pivoted Cholesky is
// the Hermitian one (real diagonal).

// ------------------------------------------------------------------ GEMM
// C (M x N) = alpha * op(A) * B + beta * C0, column-major, per problem z;
// alpha and beta real.  op(A) = A (M x K, ld lda) or, with TA, A^T (A^H when
// complex) for A of K x M.  C0 may alias C (each workgroup reads its C0
// tile only after its whole K loop, and writes the same tile); with
// beta == 0 C0 is not read.  A 64 x 64 tile of C per workgroup of four
// waves, each wave 32 x 32 (2 x 2 MFMA 16x16x4 blocks); K runs in chunks of
// 32 staged in LDS, the next chunk prefetched into registers while the
// current one is multiplied.  Complex products are four real MFMA products
// on the real and imaginary planes of the tiles.
struct GemmArgs {
    const double *A[2], *B[2], *C0[2];
    double *C[2];
    int64_t M[2], N[2], K[2], lda[2], ldb[2], ldc0[2], ldc[2];
    double alpha, beta;
};

static constexpr int GK = 32, GLD = 66;

template <bool TA, bool CX>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    constexpr int NP = CX ? 2 : 1;      // planes (real, imaginary)
    __shared__ __attribute__((aligned(16))) double sA[NP][GK * GLD];   // [k][i]
    __shared__ __attribute__((aligned(16))) double sB[NP][GK * GLD];   // [k][j]
    const int z = blockIdx.z;
    const int64_t M = g.M[z], N = g.N[z], K = g.K[z];
    const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
    if (r0 >= M || c0 >= N) return;   // the grid covers the larger problem
    const double *__restrict__ A = g.A[z];
    const double *__restrict__ B = g.B[z];
    const int64_t lda = g.lda[z], ldb = g.ldb[z];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = 32 * (wave & 1), wc = 32 * (wave >> 1);
    const int i16 = lane & 15, k4 = lane >> 4;
    d4 acc[NP][2][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[p][a][b] = d4{0.0, 0.0, 0.0, 0.0};

    // each thread moves 8 elements of the A chunk and 8 of the B chunk
    double ra[NP][8], rb[NP][8];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = tid + 256 * t;
            int ii, kk;
            if (TA) { ii = e / GK; kk = e % GK; }      // A^T: k contiguous in memory
            else { ii = e % 64; kk = e / 64; }         // A: i contiguous in memory
            const int64_t gi = r0 + ii, gk = k0 + kk;
            const bool oka = gi < M && gk < K;
            const int64_t ia = TA ? gi * lda + gk : gk * lda + gi;
            const int jj = e / GK, kb = e % GK;
            const int64_t gj = c0 + jj, gkb = k0 + kb;
            const bool okb = gj < N && gkb < K;
            const int64_t ib = gj * ldb + gkb;
            if constexpr (CX) {
                const d2 va = oka ? *(const d2 *)(A + 2 * ia) : d2{0.0, 0.0};
                const d2 vb = okb ? *(const d2 *)(B + 2 * ib) : d2{0.0, 0.0};
                ra[0][t] = va[0];
                ra[NP - 1][t] = va[1];
                rb[0][t] = vb[0];
                rb[NP - 1][t] = vb[1];
            } else {
                ra[0][t] = oka ? A[ia] : 0.0;
                rb[0][t] = okb ? B[ib] : 0.0;
            }
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
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                sA[p][kk * GLD + ii] = ra[p][t];
                sB[p][(e % GK) * GLD + e / GK] = rb[p][t];
            }
        }
        __syncthreads();
        if (k0 + GK < K) load(k0 + GK);
#pragma unroll
        for (int ks = 0; ks < GK / 4; ++ks) {
            const int kk = 4 * ks + k4;
            double fa[NP][2], fb[NP][2];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
#pragma unroll
                for (int a = 0; a < 2; ++a) fa[p][a] = sA[p][kk * GLD + wr + 16 * a + i16];
#pragma unroll
                for (int b = 0; b < 2; ++b) fb[p][b] = sB[p][kk * GLD + wc + 16 * b + i16];
            }
            // D' = B^T A^T: element r of lane l is C(i = l % 16, j = 4 r + l / 16)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    if constexpr (CX) {
                        // (a_r + i a_i) (b_r + i b_i), a conjugated for A^H
                        const double sg = TA ? 1.0 : -1.0;
                        acc[0][a][b] = mfma16(fb[0][b], fa[0][a], acc[0][a][b]);
                        acc[0][a][b] = mfma16(fb[NP - 1][b], sg * fa[NP - 1][a], acc[0][a][b]);
                        acc[NP - 1][a][b] = mfma16(fb[NP - 1][b], fa[0][a], acc[NP - 1][a][b]);
                        acc[NP - 1][a][b] = mfma16(fb[0][b], -sg * fa[NP - 1][a], acc[NP - 1][a][b]);
                    } else {
                        acc[0][a][b] = mfma16(fb[0][b], fa[0][a], acc[0][a][b]);
                    }
                }
        }
    }
    const double *C0 = g.C0[z];
    double *C = g.C[z];
    const int64_t ldc0 = g.ldc0[z], ldc = g.ldc[z];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = r0 + wr + 16 * a + i16;
                const int64_t gj = c0 + wc + 16 * b + 4 * r + k4;
                if (gi < M && gj < N) {
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        double v = g.alpha * acc[p][a][b][r];
                        if (g.beta != 0.0) v += g.beta * C0[NP * (gj * ldc0 + gi) + p];
                        C[NP * (gj * ldc + gi) + p] = v;
                    }
                }
            }
}

static void gemm(bool ta, bool cx, int nz, const GemmArgs &g, hipStream_t s)
{
    int64_t mx = 0, nx = 0;
    for (int z = 0; z < nz; ++z) {
        mx = g.M[z] > mx ? g.M[z] : mx;
        nx = g.N[z] > nx ? g.N[z] : nx;
    }
    if (mx <= 0 || nx <= 0) return;
    const dim3 grid((unsigned)((mx + 63) / 64), (unsigned)((nx + 63) / 64), (unsigned)nz);
    if (cx) {
        if (ta) hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, s, g);
        else hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, s, g);
    } else {
        if (ta) hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, s, g);
        else hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, s, g);
    }
}

// ------------------------------------------------------ pivoted Cholesky
// S (n x n, ld, both triangles) is the current Schur complement; Rt (n x n,
// ld) receives R transposed (not conjugated) and in the original column
// order: column j of Rt is row j of R, entry c of it belongs to original
// column c (zero once c has been pivoted at an earlier step).  d[c] is the
// current (real) diagonal of S, done[c] marks pivoted columns, piv[j] the
// original column taken at step j (piv[j] = j without pivoting).
struct PcholArgs {
    const double *S[2];
    double *Rt[2], *d[2];
    int *done[2], *piv[2];
};

static constexpr int PT = 1024;

// Workgroup barrier that orders LDS only: global stores of R and loads of
// S stay in flight across it (nothing in the panel kernel reads global
// memory written in the same launch).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One workgroup of PT threads per problem runs the steps [j0, j0 + NB) of
// a panel.  Thread t owns the columns t, t + PT, ... (CPT of them): their
// diagonal entries and panel rows of R stay in its registers, and the
// panel rows are also kept in LDS (row stride CPT * PT), where the pivot
// column's entries are read by all.  With pivoting (PIV) a step is one
// barrier: the waves' (largest diagonal, column) candidates meet in LDS and
// every wave reduces them itself, so the pivot and its diagonal entry are
// known to all threads without a broadcast; the row of S at the pivot is
// then read from memory.  Without pivoting the panel's NB rows of S are
// read at its start and the diagonal entry of the next column is handed
// over in LDS.  Entry c of the row at the pivot p is S(p, c), read as the
// conjugate of S(c, p) in column p.
template <int CPT, int NB, bool PIV, bool CX>
__global__ __launch_bounds__(PT) void k_pchol_panel(int n, int64_t ld, PcholArgs a, int j0,
                                                    int *__restrict__ status)
{
    constexpr int RS = CPT * PT;
    constexpr int NP = CX ? 2 : 1;
    __shared__ double Rp[NP][NB * RS];
    __shared__ double s_bv[2][PT / 64];
    __shared__ int s_bi[2][PT / 64];
    __shared__ double s_dn[2];
    const int z = blockIdx.x;
    const double *__restrict__ S = a.S[z];
    double *__restrict__ Rt = a.Rt[z];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int jn = (j0 + NB < n) ? j0 + NB : n;
    double dl[CPT];
    int dn[CPT];
    double rr[NP][NB][CPT];
    double srows[NP][PIV ? 1 : NB][CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int c = tid + PT * u;
        if (c < n) {
            dl[u] = (j0 == 0) ? S[NP * ((int64_t)c * ld + c)] : a.d[z][c];
            dn[u] = (j0 == 0) ? 0 : a.done[z][c];
        } else {
            dl[u] = 0.0;
            dn[u] = 1;
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < NB; ++i) rr[p][i][u] = 0.0;
    }
    if (!PIV) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = tid + PT * u;
            if (c == j0) s_dn[0] = dl[u];
#pragma unroll
            for (int i = 0; i < (PIV ? 1 : NB); ++i) {
                const bool ok = j0 + i < n && c < n;
                const int64_t e = (int64_t)(j0 + i) * ld + c;
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    const double v = ok ? S[NP * e + p] : 0.0;
                    srows[p][i][u] = p ? -v : v;
                }
            }
        }
    }
    for (int j = j0; j < jn; ++j) {
        const int t = j - j0, par = t & 1;
        int p;
        double dp;
        double sv[NP][CPT];
        if (PIV) {
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
                s_bv[par][wv] = bv;
                s_bi[par][wv] = bi;
            }
            lds_barrier();
            bv = (lane < PT / 64) ? s_bv[par][lane] : -INFINITY;
            bi = (lane < PT / 64) ? s_bi[par][lane] : INT_MAX;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int oi = __shfl_xor(bi, off);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            p = __builtin_amdgcn_readfirstlane(bi);
            dp = bv;
            const double *srow = S + NP * (int64_t)p * ld;   // column p
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int c = tid + PT * u;
                const bool ok = c < n && !dn[u] && c != p;
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    const double v = ok ? srow[NP * c + q] : 0.0;
                    sv[q][u] = q ? -v : v;
                }
            }
        } else {
            lds_barrier();
            p = j;
            dp = s_dn[par];
#pragma unroll
            for (int u = 0; u < CPT; ++u)
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    sv[q][u] = 0.0;
#pragma unroll
                    for (int i = 0; i < (PIV ? 1 : NB); ++i)
                        if (i == t) sv[q][u] = srows[q][i][u];
                }
        }
#pragma unroll
        for (int u = 0; u < CPT; ++u)
            if (tid + PT * u == p) dn[u] = 1;
        const bool nonfinite = !(fabs(dp) <= DBL_MAX);
        const bool bad = nonfinite || !(dp > 0.0);
        const double r = bad ? 1.0 : sqrt(dp);
        if (bad && tid == 0) atomicOr(&status[ST_FLAGS], nonfinite ? FLAG_NONFINITE : FLAG_CHOL);
        double rp[NP][NB];
#pragma unroll
        for (int q = 0; q < NP; ++q)
#pragma unroll
            for (int i = 0; i < NB; ++i) rp[q][i] = (i < t) ? Rp[q][i * RS + p] : 0.0;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int c = tid + PT * u;
            double v[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) v[q] = 0.0;
            if (c < n && !dn[u]) {
                if constexpr (CX) {
                    // S(p, c) - sum_i conj(R(i, p)) R(i, c)
                    double xr = sv[0][u], xi = sv[NP - 1][u];
#pragma unroll
                    for (int i = 0; i < NB; ++i)
                        if (i < t) {
                            xr -= rp[0][i] * rr[0][i][u] + rp[NP - 1][i] * rr[NP - 1][i][u];
                            xi -= rp[0][i] * rr[NP - 1][i][u] - rp[NP - 1][i] * rr[0][i][u];
                        }
                    v[0] = xr / r;
                    v[NP - 1] = xi / r;
                    dl[u] -= v[0] * v[0] + v[NP - 1] * v[NP - 1];
                } else {
                    double x = sv[0][u];
#pragma unroll
                    for (int i = 0; i < NB; ++i)
                        if (i < t) x -= rp[0][i] * rr[0][i][u];
                    v[0] = x / r;
                    dl[u] -= v[0] * v[0];
                }
            } else if (c == p) {
                v[0] = r;
            }
#pragma unroll
            for (int q = 0; q < NP; ++q) {
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    if (i == t) rr[q][i][u] = v[q];
                if (c < n) {
                    Rp[q][t * RS + c] = v[q];
                    Rt[NP * ((int64_t)j * ld + c) + q] = v[q];
                }
            }
            if (!PIV && c == j + 1) s_dn[par ^ 1] = dl[u];
        }
        if (tid == 0) a.piv[z][j] = p;
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int c = tid + PT * u;
        if (c < n) {
            a.d[z][c] = dl[u];
            a.done[z][c] = dn[u];
        }
    }
}

// Trailing update after a panel: S -= R(j0:j0+nb, :)^H R(j0:j0+nb, :) over
// all of S (entries of pivoted columns are never read again); nb <= 16.
template <bool CX>
__global__ __launch_bounds__(256) void k_pchol_update(int n, int64_t ld, PcholArgs g, int j0,
                                                      int nb)
{
    constexpr int NP = CX ? 2 : 1;
    __shared__ double a[NP][16][64], b[NP][16][64];
    const int z = blockIdx.z;
    double *__restrict__ S = (double *)g.S[z];
    const double *__restrict__ Rt = g.Rt[z];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    for (int e = tid; e < 16 * 64; e += 256) {
        const int i = e / 64, x = e % 64;
        const bool ok = i < nb;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            a[p][i][x] = (ok && r0 + x < n) ? Rt[NP * ((int64_t)(j0 + i) * ld + r0 + x) + p] : 0.0;
            b[p][i][x] = (ok && c0 + x < n) ? Rt[NP * ((int64_t)(j0 + i) * ld + c0 + x) + p] : 0.0;
        }
    }
    __syncthreads();
    const int r = tid & 63;
    if (r0 + r >= n) return;
    for (int q = tid >> 6; q < 64; q += 4) {
        if (c0 + q >= n) break;
        double *s = S + NP * ((int64_t)(c0 + q) * ld + r0 + r);
        if constexpr (CX) {
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                ar += a[0][i][r] * b[0][i][q] + a[NP - 1][i][r] * b[NP - 1][i][q];
                ai += a[0][i][r] * b[NP - 1][i][q] - a[NP - 1][i][r] * b[0][i][q];
            }
            s[0] -= ar;
            s[NP - 1] -= ai;
        } else {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) acc += a[0][i][r] * b[0][i][q];
            s[0] -= acc;
        }
    }
}

// ------------------------------------------------- triangular pieces
// Inverses of the 64 x 64 diagonal blocks of the upper triangular R[z]
// (n x n, ld, real diagonal): block J goes to X[z] + 4096 J elements
// (column-major 64 x 64), the trailing partial block padded with the
// identity.  Each of the 16 waves solves R_JJ x = e_j for 4 columns j by
// column-oriented back substitution, one row per lane, with the diagonal's
// reciprocals formed once.
template <bool CX>
__global__ __launch_bounds__(1024) void k_trinv_diag(int n, int64_t ld, const double *R0,
                                                     const double *R1, double *X0, double *X1)
{
    constexpr int NP = CX ? 2 : 1;
    __shared__ double sR[NP][64 * 65];
    __shared__ double sI[64];
    const double *__restrict__ R = blockIdx.y ? R1 : R0;
    double *__restrict__ X = blockIdx.y ? X1 : X0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b0 = blockIdx.x * 64;
    const int bs = (n - b0 < 64) ? n - b0 : 64;
    for (int e = tid; e < 64 * 64; e += 1024) {
        const int r = e % 64, c = e / 64;
        const bool in = r < bs && c < bs && r <= c;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            double v = (r == c && p == 0) ? 1.0 : 0.0;
            if (in) v = R[NP * ((int64_t)(b0 + c) * ld + b0 + r) + p];
            sR[p][c * 65 + r] = v;
        }
    }
    __syncthreads();
    if (tid < 64) sI[tid] = 1.0 / sR[0][tid * 65 + tid];
    __syncthreads();
    for (int jj = 0; jj < 4; ++jj) {
        const int j = wave + 16 * jj;
        double xr = (lane == j) ? 1.0 : 0.0, xi = 0.0;
        for (int k = j; k >= 0; --k) {
            const double kr = __shfl(xr, k) * sI[k];
            if constexpr (CX) {
                const double ki = __shfl(xi, k) * sI[k];
                if (lane == k) {
                    xr = kr;
                    xi = ki;
                } else if (lane < k) {
                    const double rr = sR[0][k * 65 + lane], ri = sR[NP - 1][k * 65 + lane];
                    xr -= kr * rr - ki * ri;
                    xi -= kr * ri + ki * rr;
                }
            } else {
                if (lane == k) xr = kr;
                else if (lane < k) xr -= kr * sR[0][k * 65 + lane];
            }
        }
        double *out = X + NP * ((int64_t)blockIdx.x * 4096 + j * 64 + lane);
        out[0] = xr;
        if (CX) out[NP - 1] = xi;
    }
}

// dst[z](0:m[z], j) = src[z](0:m[z], idx[z][j]) for j < ncol
struct GatherArgs {
    const int *idx[2];
    const double *src[2];
    double *dst[2];
    int64_t m[2], lds[2], ldd[2];
};

template <bool CX>
__global__ __launch_bounds__(256) void k_gather_cols(GatherArgs g)
{
    constexpr int NP = CX ? 2 : 1;
    const int z = blockIdx.z, j = blockIdx.y;
    const int64_t m = g.m[z];
    const double *s = g.src[z] + NP * (int64_t)g.idx[z][j] * g.lds[z];
    double *d = g.dst[z] + NP * (int64_t)j * g.ldd[z];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        if constexpr (CX) *(d2 *)(d + 2 * i) = *(const d2 *)(s + 2 * i);
        else d[i] = s[i];
    }
}

// R[z](i, k) = Rt[z](idx[z][k], i) for i, k < n: the upper triangular factor
// in the pivoted column order (idx = piv), or the plain transpose (idx[z]
// null); 32 x 32 tiles through LDS.
template <bool CX>
__global__ __launch_bounds__(256) void k_gather_rt(int n, int64_t ld, GatherArgs g)
{
    constexpr int NP = CX ? 2 : 1;
    __shared__ double tile[NP][32][33];
    const int z = blockIdx.z;
    const int *idx = g.idx[z];
    const double *__restrict__ Rt = g.src[z];
    double *__restrict__ R = g.dst[z];
    const int i0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int y = ty; y < 32; y += 8) {
        const int i = i0 + y, k = k0 + tx;
        const bool ok = i < n && k < n;
        const int64_t e = ok ? (int64_t)i * ld + (idx ? idx[k] : k) : 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) tile[p][y][tx] = ok ? Rt[NP * e + p] : 0.0;
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int k = k0 + y, i = i0 + tx;
        if (i < n && k < n) {
#pragma unroll
            for (int p = 0; p < NP; ++p) R[NP * ((int64_t)k * ld + i) + p] = tile[p][tx][y];
        }
    }
}

// Z(q[j], :) = Z2(j, :): rows of the square pair's Z back in the original
// column order of (F, G).
template <bool CX>
__global__ __launch_bounds__(256) void k_scatter_rows(int n, const int *__restrict__ q,
                                                      const double *__restrict__ Z2, int64_t ld2,
                                                      double *__restrict__ Z, int64_t ldz)
{
    constexpr int NP = CX ? 2 : 1;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int j = (int)(e % n), c = (int)(e / n);
#pragma unroll
    for (int p = 0; p < NP; ++p)
        Z[NP * ((int64_t)c * ldz + q[j]) + p] = Z2[NP * ((int64_t)c * ld2 + j) + p];
}

// p2[j] = slot of q[j] in the order p1 (inv1 = p1^-1 formed first).
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

// Panel widths: the LDS copy of the panel rows is NB * CPT * 1024 elements
// (128 KiB) for every n range, half as many rows for complex elements.
static int panel_width(int cpt, int cx) { return 16 / cpt / (cx ? 2 : 1); }

int shorten_cpt(int64_t n)
{
    if (n <= PT) return 1;
    if (n <= 2 * PT) return 2;
    if (n <= 4 * PT) return 4;
    if (n <= 8 * PT) return 8;
    return 0;
}

bool make_splan(int64_t mf, int64_t mg, int64_t n, size_t solve_bytes, SPlan &S, int cx)
{
    S = SPlan();
    S.cpt = shorten_cpt(n);
    if (!S.cpt || n < 2) return false;
    S.cx = cx ? 1 : 0;
    const size_t es = cx ? 16 : 8;
    S.mf = mf;
    S.mg = mg;
    S.n = n;
    S.nb = panel_width(S.cpt, S.cx);
    S.ldqf = (mf + 7) / 8 * 8;
    S.ldqg = (mg + 7) / 8 * 8;
    S.ldn = (n + 7) / 8 * 8;
    S.nblk = (int)((n + 63) / 64);
    const size_t nn = es * (size_t)S.ldn * n;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    S.o_qf = o; o = al(o + es * (size_t)S.ldqf * n);
    S.o_qg = o; o = al(o + es * (size_t)S.ldqg * n);
    S.o_r1f = o; o = al(o + nn);
    S.o_r1g = o; o = al(o + nn);
    S.o_f2 = o; o = al(o + nn);
    S.o_g2 = o; o = al(o + nn);
    S.o_z2 = o; o = al(o + nn);
    for (int z = 0; z < 2; ++z) {
        const int64_t m = z ? S.ldqg : S.ldqf;
        S.o_s[z] = o; o = al(o + nn);
        S.o_rt[z] = o; o = al(o + nn);
        S.o_r2[z] = o; o = al(o + nn);
        S.o_t[z] = o; o = al(o + es * (size_t)m * 64);
        S.o_xd[z] = o; o = al(o + es * (size_t)S.nblk * 4096);
        S.o_d[z] = o; o = al(o + 8 * (size_t)n);
        S.o_done[z] = o; o = al(o + 4 * (size_t)n);
        S.o_id[z] = o; o = al(o + 4 * (size_t)n);
    }
    S.o_p1 = o; o = al(o + 4 * (size_t)n);
    S.o_q = o; o = al(o + 4 * (size_t)n);
    S.o_inv1 = o; o = al(o + 4 * (size_t)n);
    S.o_p2 = o; o = al(o + 4 * (size_t)n);
    S.o_status = o; o = al(o + 4 * ST_NSLOTS);
    S.o_solve = o; o = al(o + solve_bytes);
    S.total = o;
    return true;
}

template <typename T> static T *at(char *b, size_t o) { return (T *)(b + o); }

// Cholesky of S[z] (ld ldn) into Rt[z] for both problems, with diagonal
// pivoting (piv[z] = pivot order) or without (piv[z] = identity).
template <bool CX>
static void pchol(const SPlan &P, char *b, int *const piv[2], bool pivoting, int *status,
                  hipStream_t s)
{
    const int n = (int)P.n, nb = P.nb;
    PcholArgs a;
    for (int z = 0; z < 2; ++z) {
        a.S[z] = at<double>(b, P.o_s[z]);
        a.Rt[z] = at<double>(b, P.o_rt[z]);
        a.d[z] = at<double>(b, P.o_d[z]);
        a.done[z] = at<int>(b, P.o_done[z]);
        a.piv[z] = piv[z];
    }
    const unsigned gt = (unsigned)((n + 63) / 64);
    constexpr int H = CX ? 2 : 1;
    for (int j0 = 0; j0 < n; j0 += nb) {
        const dim3 g2(2), bt(PT);
        switch (P.cpt * 2 + (pivoting ? 1 : 0)) {
        case 3: hipLaunchKernelGGL((k_pchol_panel<1, 16 / H, true, CX>), g2, bt, 0, s, n, P.ldn, a, j0, status); break;
        case 2: hipLaunchKernelGGL((k_pchol_panel<1, 16 / H, false, CX>), g2, bt, 0, s, n, P.ldn, a, j0, status); break;
        case 5: hipLaunchKernelGGL((k_pchol_panel<2, 8 / H, true, CX>), g2, bt, 0, s, n, P.ldn, a, j0, status); break;
        case 4: hipLaunchKernelGGL((k_pchol_panel<2, 8 / H, false, CX>), g2, bt, 0, s, n, P.ldn, a, j0, status); break;
        case 9: hipLaunchKernelGGL((k_pchol_panel<4, 4 / H, true, CX>), g2, bt, 0, s, n, P.ldn, a, j0, status); break;
        case 8: hipLaunchKernelGGL((k_pchol_panel<4, 4 / H, false, CX>), g2, bt, 0, s, n, P.ldn, a, j0, status); break;
        case 17: hipLaunchKernelGGL((k_pchol_panel<8, 2 / H, true, CX>), g2, bt, 0, s, n, P.ldn, a, j0, status); break;
        default: hipLaunchKernelGGL((k_pchol_panel<8, 2 / H, false, CX>), g2, bt, 0, s, n, P.ldn, a, j0, status); break;
        }
        if (j0 + nb < n)
            hipLaunchKernelGGL(k_pchol_update<CX>, dim3(gt, gt, 2), dim3(256), 0, s, n, P.ldn, a, j0,
                               nb);
    }
}

// In place Y[z] (m[z] x n, ld ldy[z]) <- Y[z] R[z]^-1 for upper triangular
// R[z] (ld ldn), by 64-column blocks: T = Y_J - Y_{<J} R_{<J,J}, then
// Y_J = T inv(R_JJ).
template <bool CX>
static void trsm_right(const SPlan &P, char *b, double *const Y[2], const int64_t ldy[2],
                       const double *const R[2], hipStream_t s)
{
    constexpr int NP = CX ? 2 : 1;
    const int n = (int)P.n;
    const int64_t m[2] = {P.mf, P.mg};
    double *T[2] = {at<double>(b, P.o_t[0]), at<double>(b, P.o_t[1])};
    double *X[2] = {at<double>(b, P.o_xd[0]), at<double>(b, P.o_xd[1])};
    hipLaunchKernelGGL(k_trinv_diag<CX>, dim3((unsigned)P.nblk, 2), dim3(1024), 0, s, n, P.ldn,
                       R[0], R[1], X[0], X[1]);
    for (int J = 0; J < P.nblk; ++J) {
        const int64_t j0 = 64 * (int64_t)J, bs = (n - j0 < 64) ? n - j0 : 64;
        GemmArgs g1, g2;
        for (int z = 0; z < 2; ++z) {
            g1.A[z] = Y[z]; g1.lda[z] = ldy[z];
            g1.B[z] = R[z] + NP * j0 * P.ldn; g1.ldb[z] = P.ldn;
            g1.C0[z] = Y[z] + NP * j0 * ldy[z]; g1.ldc0[z] = ldy[z];
            g1.C[z] = T[z]; g1.ldc[z] = m[z];
            g1.M[z] = m[z]; g1.N[z] = bs; g1.K[z] = j0;
            g2.A[z] = T[z]; g2.lda[z] = m[z];
            g2.B[z] = X[z] + NP * 4096 * (int64_t)J; g2.ldb[z] = 64;
            g2.C0[z] = nullptr; g2.ldc0[z] = 0;
            g2.C[z] = Y[z] + NP * j0 * ldy[z]; g2.ldc[z] = ldy[z];
            g2.M[z] = m[z]; g2.N[z] = bs; g2.K[z] = bs;
        }
        g1.alpha = -1.0; g1.beta = 1.0;
        g2.alpha = 1.0; g2.beta = 0.0;
        gemm(false, CX, 2, g1, s);
        gemm(false, CX, 2, g2, s);
    }
}

// S[z] = Y[z]^T Y[z] (^H for complex; n x n, ld ldn) for Y[z] of m[z] rows.
template <bool CX>
static void gram2(const SPlan &P, char *b, const double *const Y[2], const int64_t ldy[2],
                  hipStream_t s)
{
    GemmArgs g;
    const int64_t m[2] = {P.mf, P.mg};
    for (int z = 0; z < 2; ++z) {
        g.A[z] = Y[z]; g.lda[z] = ldy[z];
        g.B[z] = Y[z]; g.ldb[z] = ldy[z];
        g.C0[z] = nullptr; g.ldc0[z] = 0;
        g.C[z] = at<double>(b, P.o_s[z]); g.ldc[z] = P.ldn;
        g.M[z] = P.n; g.N[z] = P.n; g.K[z] = m[z];
    }
    g.alpha = 1.0; g.beta = 0.0;
    gemm(true, CX, 2, g, s);
}

template <bool CX>
static hipError_t shorten_impl(const SPlan &P, void *work, const double *F, int64_t ldf,
                               const double *G, int64_t ldg, hipStream_t s)
{
    char *b = (char *)work;
    const int n = (int)P.n;
    int *p1 = at<int>(b, P.o_p1), *q = at<int>(b, P.o_q);
    int *inv1 = at<int>(b, P.o_inv1), *p2 = at<int>(b, P.o_p2);
    int *status = at<int>(b, P.o_status);
    double *Q[2] = {at<double>(b, P.o_qf), at<double>(b, P.o_qg)};
    const int64_t ldq[2] = {P.ldqf, P.ldqg};
    double *R1[2] = {at<double>(b, P.o_r1f), at<double>(b, P.o_r1g)};
    const unsigned g1 = (unsigned)((n + 255) / 256);
    const unsigned gn = (unsigned)((n + 31) / 32);
    hipError_t e = hipMemsetAsync(status, 0, 4 * ST_NSLOTS, s);
    if (e != hipSuccess) return e;
    // 1. pivots and R1 from the Grams: F P1 = Q_F R_F, and (G P1) P2 = Q_G R_G
    //    through the pivoted Cholesky of G^T G, whose order is q = P1 P2 (the
    //    position of q in the order P1 is P2)
    const double *Y0[2] = {F, G};
    const int64_t ldy0[2] = {ldf, ldg};
    gram2<CX>(P, b, Y0, ldy0, s);
    int *const piv1[2] = {p1, q};
    pchol<CX>(P, b, piv1, true, status, s);
    GatherArgs gr;
    for (int z = 0; z < 2; ++z) {
        gr.idx[z] = piv1[z];
        gr.src[z] = at<double>(b, P.o_rt[z]);
        gr.dst[z] = R1[z];
        gr.m[z] = n; gr.lds[z] = P.ldn; gr.ldd[z] = P.ldn;
    }
    hipLaunchKernelGGL(k_gather_rt<CX>, dim3(gn, gn, 2), dim3(256), 0, s, n, P.ldn, gr);
    // 2. Q = Y P, in place Q <- Q R1^-1
    GatherArgs gc;
    for (int z = 0; z < 2; ++z) {
        gc.idx[z] = piv1[z];
        gc.src[z] = Y0[z]; gc.lds[z] = ldy0[z];
        gc.dst[z] = Q[z]; gc.ldd[z] = ldq[z];
    }
    gc.m[0] = P.mf;
    gc.m[1] = P.mg;
    const int64_t mmax = P.mf > P.mg ? P.mf : P.mg;
    hipLaunchKernelGGL(k_gather_cols<CX>, dim3((unsigned)((mmax + 255) / 256), (unsigned)n, 2),
                       dim3(256), 0, s, gc);
    const double *R1c[2] = {R1[0], R1[1]};
    trsm_right<CX>(P, b, Q, ldq, R1c, s);
    // 3. refinement: R2^H R2 = Q^H Q, Q <- Q R2^-1, R = R2 R1
    const double *Qc[2] = {Q[0], Q[1]};
    gram2<CX>(P, b, Qc, ldq, s);
    int *const pid[2] = {at<int>(b, P.o_id[0]), at<int>(b, P.o_id[1])};
    pchol<CX>(P, b, pid, false, status, s);
    double *R2[2] = {at<double>(b, P.o_r2[0]), at<double>(b, P.o_r2[1])};
    for (int z = 0; z < 2; ++z) {
        gr.idx[z] = nullptr;
        gr.dst[z] = R2[z];
    }
    hipLaunchKernelGGL(k_gather_rt<CX>, dim3(gn, gn, 2), dim3(256), 0, s, n, P.ldn, gr);
    const double *R2c[2] = {R2[0], R2[1]};
    trsm_right<CX>(P, b, Q, ldq, R2c, s);
    GemmArgs g;
    for (int z = 0; z < 2; ++z) {
        g.A[z] = R2[z]; g.lda[z] = P.ldn;
        g.B[z] = R1[z]; g.ldb[z] = P.ldn;
        g.C0[z] = nullptr; g.ldc0[z] = 0;
        g.C[z] = at<double>(b, P.o_s[z]); g.ldc[z] = P.ldn;   // S[z] <- R = R2 R1
        g.M[z] = P.n; g.N[z] = P.n; g.K[z] = P.n;
    }
    g.alpha = 1.0; g.beta = 0.0;
    gemm(false, CX, 2, g, s);
    // 4. F'' = R_F P2, G'' = R_G
    hipLaunchKernelGGL(k_perm_inverse, dim3(g1), dim3(256), 0, s, n, (const int *)p1, inv1);
    hipLaunchKernelGGL(k_perm_compose, dim3(g1), dim3(256), 0, s, n, (const int *)inv1,
                       (const int *)q, p2);
    for (int z = 0; z < 2; ++z) {
        gc.idx[z] = z ? pid[1] : p2;     // G'' keeps its order (pid[1] is the identity)
        gc.src[z] = at<double>(b, P.o_s[z]); gc.lds[z] = P.ldn;
        gc.dst[z] = at<double>(b, z ? P.o_g2 : P.o_f2); gc.ldd[z] = P.ldn;
        gc.m[z] = n;
    }
    hipLaunchKernelGGL(k_gather_cols<CX>, dim3(g1, (unsigned)n, 2), dim3(256), 0, s, gc);
    return hipGetLastError();
}

hipError_t launch_shorten(const SPlan &P, void *work, const double *F, int64_t ldf,
                          const double *G, int64_t ldg, hipStream_t s)
{
    return P.cx ? shorten_impl<true>(P, work, F, ldf, G, ldg, s)
                : shorten_impl<false>(P, work, F, ldf, G, ldg, s);
}

hipError_t launch_unshorten(const SPlan &P, void *work, double *U, int64_t ldu, double *V,
                            int64_t ldv, double *Z, int64_t ldz, hipStream_t s)
{
    char *b = (char *)work;
    const int n = (int)P.n;
    GemmArgs g;
    g.A[0] = at<double>(b, P.o_qf); g.lda[0] = P.ldqf;
    g.A[1] = at<double>(b, P.o_qg); g.lda[1] = P.ldqg;
    g.B[0] = at<double>(b, P.o_f2); g.B[1] = at<double>(b, P.o_g2);
    g.ldb[0] = g.ldb[1] = P.ldn;
    g.C0[0] = g.C0[1] = nullptr;
    g.ldc0[0] = g.ldc0[1] = 0;
    g.C[0] = U; g.ldc[0] = ldu;
    g.C[1] = V; g.ldc[1] = ldv;
    g.M[0] = P.mf; g.M[1] = P.mg;
    g.N[0] = g.N[1] = n;
    g.K[0] = g.K[1] = n;
    g.alpha = 1.0; g.beta = 0.0;
    gemm(false, P.cx != 0, 2, g, s);
    const int64_t nn = (int64_t)n * n;
    const dim3 grid((unsigned)((nn + 255) / 256));
    if (P.cx)
        hipLaunchKernelGGL(k_scatter_rows<true>, grid, dim3(256), 0, s, n, at<int>(b, P.o_q),
                           at<double>(b, P.o_z2), P.ldn, Z, ldz);
    else
        hipLaunchKernelGGL(k_scatter_rows<false>, grid, dim3(256), 0, s, n, at<int>(b, P.o_q),
                           at<double>(b, P.o_z2), P.ldn, Z, ldz);
    return hipGetLastError();
}

}  // namespace hz
