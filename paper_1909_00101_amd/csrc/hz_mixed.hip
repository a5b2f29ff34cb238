// hz_mixed.hip -- FP32 kernels of the mixed-precision form and its FP64
// restart.  Early sweeps run on FP32 copies of F, G, Z with FP32 MFMA Gram
// blocks (FP32 accumulation) and FP32 MFMA block updates; Cholesky, the
// inner solve, the counters and Theta stay in FP64 (the Gram partials are
// widened to FP64, Z_tilde is rounded to FP32 only for the update).  Once the
// off-diagonal measure is small the FP64 iteration restarts from the
// original pair in the basis found so far: F1 = F Z32, G1 = G Z32 (FP64
// MFMA), Z1 = Z32 -- valid because every iterate satisfies F_k = F Z_k
// (paper, Section 2.1: the transformations accumulate into Z).
#include "hz_device.h"
#include "hz_internal.h"

namespace hz {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

// v_mfma_f32_16x16x4_f32: A[i][k] lane i + 16k, B[k][j] lane j + 16k,
// C[i][j] lane j + 16*(i/4), element i%4 (checked on gfx950).
__device__ __forceinline__ f4 mfma16f(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Prescale (Section 2) into FP32 working copies, with bordering.
__global__ __launch_bounds__(256) void k_prescale_copy32(
    int64_t mf, int64_t mg, int64_t n, const double *__restrict__ F, int64_t ldf,
    const double *__restrict__ G, int64_t ldg, int64_t nw, int64_t mfw, int64_t mgw, int64_t nzw,
    float *__restrict__ Fs, float *__restrict__ Gs, float *__restrict__ Zs,
    int *__restrict__ status)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nw) return;
    float *fw = Fs + j * mfw, *gw = Gs + j * mgw, *zw = Zs + j * nzw;
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
            fw[r] = (float)v;
        }
        for (int64_t r = lane; r < mgw; r += 64) gw[r] = (r < mg) ? (float)(g[r] * d) : 0.0f;
        for (int64_t r = lane; r < nzw; r += 64) zw[r] = (r == j) ? (float)d : 0.0f;
        if (bad) atomicOr(status + ST_FLAGS, FLAG_NONFINITE);
    } else {
        const int64_t k = j - n;
        for (int64_t r = lane; r < mfw; r += 64) fw[r] = (r == mf + k) ? 1.0f : 0.0f;
        for (int64_t r = lane; r < mgw; r += 64) gw[r] = (r == mg + k) ? 1.0f : 0.0f;
        for (int64_t r = lane; r < nzw; r += 64) zw[r] = (r == j) ? 1.0f : 0.0f;
    }
}

// Pivot Gram blocks from FP32 data with FP32 MFMA and FP32 accumulation;
// lower tiles; the four waves' tiles are summed in FP64 (row stride W2 + 2
// in LDS, so the 16 lanes of a tile row fall in distinct banks) and the split
// partial is written widened to FP64 (summed in split order by k_gram_sum).
template <int W2>
__global__ __launch_bounds__(256) void k_gram32(const float *__restrict__ Fs,
                                                const float *__restrict__ Gs, int64_t mfw,
                                                int64_t mgw, const int *__restrict__ pairs,
                                                int splits, double *__restrict__ part)
{
    constexpr int W = W2 / 2, NB = W2 / 16, LDT = 68, NLD = W2 / 16, LDR = W2 + 2;
    constexpr int NT = NB * (NB + 1) / 2;
    __shared__ __attribute__((aligned(16))) float tile[W2 * LDT];
    __shared__ __attribute__((aligned(16))) double red[W2 * LDR];
    const int split = blockIdx.x, pr = blockIdx.y, mat = blockIdx.z;
    const float *Y = mat ? Gs : Fs;
    const int64_t m = mat ? mgw : mfw;
    const int p = pairs[2 * pr], q = pairs[2 * pr + 1];
    const int64_t nch = m / 64;
    const int64_t c0 = nch * split / splits, c1 = nch * (split + 1) / splits;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lrow = 4 * (tid & 15), lcol = tid >> 4;   // 16 columns x 64 rows per pass

    f4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    const float *colp[NLD];
#pragma unroll
    for (int t = 0; t < NLD; ++t) {
        const int cc = lcol + 16 * t;
        const int gc = (cc < W) ? p * W + cc : q * W + (cc - W);
        colp[t] = Y + (int64_t)gc * m + lrow;
    }
    f4 buf[NLD];
    if (c0 < c1) {
#pragma unroll
        for (int t = 0; t < NLD; ++t) buf[t] = *(const f4 *)(colp[t] + c0 * 64);
    }
    for (int64_t c = c0; c < c1; ++c) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NLD; ++t) *(f4 *)(tile + (lcol + 16 * t) * LDT + lrow) = buf[t];
        __syncthreads();
        if (c + 1 < c1) {
#pragma unroll
            for (int t = 0; t < NLD; ++t) buf[t] = *(const f4 *)(colp[t] + (c + 1) * 64);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int ks = wave + 4 * s;
            float fr[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b)
                fr[b] = tile[(16 * b + (lane & 15)) * LDT + 4 * ks + (lane >> 4)];
            int t = 0;
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b, ++t) acc[t] = mfma16f(fr[a], fr[b], acc[t]);
        }
    }
    for (int wv = 0; wv < 4; ++wv) {
        __syncthreads();
        if (wave == wv) {
            int t = 0;
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b, ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int gi = 16 * a + 4 * (lane >> 4) + r, gj = 16 * b + (lane & 15);
                        double *dst = red + gj * LDR + gi;
                        *dst = (wv == 0) ? (double)acc[t][r] : *dst + (double)acc[t][r];
                    }
        }
    }
    __syncthreads();
    double *out = part + ((size_t)(pr * 2 + mat) * splits + split) * (W2 * W2);
    for (int e = 2 * tid; e < W2 * W2; e += 512)
        *(d2 *)(out + e) = *(const d2 *)(red + (e / W2) * LDR + e % W2);
}

// Block update of the FP32 copies, [Y_p Y_q] <- [Y_p Y_q] fl32(Z_tilde), FP32
// MFMA with D' = Z^T X^T (see k_update).  Each wave takes 32 rows at a time
// as 16 row pairs: a lane loads (and stores) two consecutive rows of a
// column as one 8-byte access, and two MFMA chains handle the even and the
// odd rows.  Element r of an accumulator in lane l is output column
// 16jb + 4(l/16) + r of row 2(l%16) (even chain) or 2(l%16) + 1 (odd).
template <int W2>
__global__ __launch_bounds__(256) void k_update32(float *__restrict__ Fs, float *__restrict__ Gs,
                                                  float *__restrict__ Zs, int64_t mfw,
                                                  int64_t mgw, int64_t nzw,
                                                  const int *__restrict__ pairs,
                                                  const double *__restrict__ Zt,
                                                  int rows_per_wave,
                                                  const unsigned long long *__restrict__ scnt)
{
    constexpr int W = W2 / 2, NB = W2 / 16, KS = W2 / 4, LDZ = W2 + 1;
    __shared__ float sz[W2 * LDZ];
    const int pr = blockIdx.y;
    if (scnt[(size_t)pr * 4 + 3]) return;   // Z_tilde = I: nothing to update
    const int p = pairs[2 * pr], q = pairs[2 * pr + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double *zt = Zt + (size_t)pr * (W2 * W2);
    {
        // every load of a thread issued before the first store
        constexpr int NZ = (W2 * W2) / 256;
        static_assert(NZ * 256 == W2 * W2, "Z_tilde staging geometry");
        double zv[NZ];
#pragma unroll
        for (int it = 0; it < NZ; ++it) zv[it] = zt[tid + 256 * it];
#pragma unroll
        for (int it = 0; it < NZ; ++it) {
            const int e = tid + 256 * it;
            sz[(e / W2) * LDZ + (e % W2)] = (float)zv[it];
        }
    }
    // The rows of F, G and Z (each a multiple of 64) are taken as one
    // sequence cut into workgroup ranges of 4 * rows_per_wave rows (a
    // multiple of 64); a 32-row tile never straddles two matrices, and its
    // matrix is chosen per tile.
    const int64_t span = 4 * (int64_t)rows_per_wave;
    const int64_t vb = (int64_t)blockIdx.x * span, total = mfw + mgw + nzw;
    const int64_t ve = (vb + span < total) ? vb + span : total;
    __syncthreads();
    const int k4 = lane >> 4, i16 = lane & 15;
    for (int64_t v0 = vb + 32 * wave; v0 < ve; v0 += 128) {
        __asm__ volatile("" ::: "memory");
        float *Y;
        int64_t m, r0;
        if (v0 < mfw) {
            Y = Fs;
            m = mfw;
            r0 = v0;
        } else if (v0 < mfw + mgw) {
            Y = Gs;
            m = mgw;
            r0 = v0 - mfw;
        } else {
            Y = Zs;
            m = nzw;
            r0 = v0 - mfw - mgw;
        }
        float *bp = Y + ((int64_t)p * W + k4) * m + 2 * i16;
        float *bq = Y + ((int64_t)q * W + k4) * m + 2 * i16;
        f2 xb[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s)
            xb[s] = (4 * s < W) ? *(const f2 *)(bp + (int64_t)(4 * s) * m + r0)
                                : *(const f2 *)(bq + (int64_t)(4 * s - W) * m + r0);
        f4 ae[NB], ao[NB];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
            ae[jb] = f4{0.f, 0.f, 0.f, 0.f};
            ao[jb] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
                const float za = sz[(16 * jb + i16) * LDZ + 4 * s + k4];
                ae[jb] = mfma16f(za, xb[s][0], ae[jb]);
                ao[jb] = mfma16f(za, xb[s][1], ao[jb]);
            }
        // output column 16jb + 4*k4 + r, rows r0 + 2*i16 (+1): stored through
        // the base pointers (which already carry the k4 column offset)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c0 = 16 * jb + 3 * k4 + r;   // + k4 via the base pointer
                const int cabs = 16 * jb + 4 * k4 + r;
                float *dst = (cabs < W) ? bp + (int64_t)c0 * m + r0 : bq + (int64_t)(c0 - W) * m + r0;
                *(f2 *)dst = f2{ae[jb][r], ao[jb][r]};
            }
    }
}

// Off-diagonal measure of the FP32 phase (reading R20): for the Gram blocks
// of one step, max over pairs and off-diagonal entries of
// |A_ij| / sqrt(A_ii A_jj) and |B_ij| / sqrt(B_ii B_jj).  One workgroup per
// (pair, matrix); the result is written per (step, pair, matrix).
template <int W2>
__global__ __launch_bounds__(256) void k_offdiag(const double *__restrict__ gram, int step,
                                                 int npairs, double *__restrict__ offd)
{
    __shared__ double dg[W2];
    __shared__ double red[256];
    const int pm = blockIdx.x;
    const double *A = gram + (size_t)pm * (W2 * W2);
    const int tid = threadIdx.x;
    for (int i = tid; i < W2; i += 256) dg[i] = A[i * W2 + i];
    __syncthreads();
    double mx = 0.0;
    // every load of a thread issued before the first use (the upper
    // entries are loaded and left unused)
    constexpr int NIT = (W2 * W2) / 256;
    static_assert(NIT * 256 == W2 * W2, "off-diagonal geometry");
    double av[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) av[it] = A[tid + 256 * it];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = tid + 256 * it, col = e / W2, row = e % W2;
        if (row > col) {
            const double v = fabs(av[it]) / sqrt(dg[row] * dg[col]);
            mx = (v > mx) ? v : mx;
        }
    }
    red[tid] = mx;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] = (red[tid + h] > red[tid]) ? red[tid + h] : red[tid];
        __syncthreads();
    }
    if (tid == 0) offd[(size_t)step * npairs * 2 + pm] = red[0];
}

// FP64 restart GEMM C(rows, N) = A(rows, K) * B(K, N) with A FP64 (the
// caller's original F or G, rows >= m_a read as zero), B FP32 (Z32, widened
// exactly), C FP64 with leading dimension ldc.  FP64 MFMA: each workgroup
// computes a 64-row x 64-column tile, B staged in LDS per 64-deep K chunk,
// each wave 16 rows.
__global__ __launch_bounds__(256) void k_restart_gemm(const double *__restrict__ A, int64_t lda,
                                                      int64_t m_a, int64_t K,
                                                      const float *__restrict__ B, int64_t ldb,
                                                      int64_t N, double *__restrict__ C,
                                                      int64_t ldc, int64_t rows)
{
    constexpr int LDB = 65;
    __shared__ double sb[64 * LDB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + 16 * wave;
    const int64_t c0 = (int64_t)blockIdx.y * 64;
    const int k4 = lane >> 4, i16 = lane & 15;
    d4 acc[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) acc[jb] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t row = r0 + i16;
    const bool rowok = row < m_a;
    for (int64_t k0 = 0; k0 < K; k0 += 64) {
        __syncthreads();
        for (int e = tid; e < 64 * 64; e += 256) {
            const int kk = e % 64, cc = e / 64;
            sb[cc * LDB + kk] =
                (k0 + kk < K && c0 + cc < N) ? (double)B[(c0 + cc) * ldb + k0 + kk] : 0.0;
        }
        __syncthreads();
        double xa[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int64_t kk = k0 + 4 * s + k4;
            xa[s] = (rowok && kk < K) ? A[kk * lda + row] : 0.0;
        }
        // D' = B^T A^T: A' fragment = B[k][16jb + j], B' fragment = A[row][k]
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
                acc[jb] = mfma16(sb[(16 * jb + i16) * LDB + 4 * s + k4], xa[s], acc[jb]);
    }
    if (r0 >= rows) return;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t col = c0 + 16 * jb + 4 * r + k4;
            if (col < N) C[col * ldc + r0 + i16] = acc[jb][r];
        }
}

// Rows m_a .. ldc-1 of the restarted working matrix: the bordering rows
// take the bordering part of Z32 (row m_a + b of Fw is row n + b of Z32),
// padding rows are zero.
__global__ __launch_bounds__(256) void k_restart_border(int64_t m_a, int64_t n, int64_t nb,
                                                        int64_t ldc, int64_t N,
                                                        const float *__restrict__ Zs, int64_t ldz,
                                                        double *__restrict__ C)
{
    const int64_t extra = ldc - m_a;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= extra * N) return;
    const int64_t j = e / extra, b = e % extra;
    C[j * ldc + m_a + b] = (b < nb) ? (double)Zs[j * ldz + n + b] : 0.0;
}

__global__ __launch_bounds__(256) void k_widen(const float *__restrict__ src, double *__restrict__ dst,
                                               int64_t count)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < count) dst[e] = (double)src[e];
}

// ------------------------------------------------------------------ launchers

void launch_prescale_mixed(const Plan &P, const Ptrs &W, const double *F, int64_t ldf,
                           const double *G, int64_t ldg, hipStream_t s)
{
    const unsigned nb = (unsigned)((P.nw + 3) / 4);
    hipLaunchKernelGGL(k_prescale_copy32, dim3(nb), dim3(256), 0, s, P.mf, P.mg, P.n, F, ldf, G,
                       ldg, P.nw, P.mfw, P.mgw, P.nzw, W.Fs, W.Gs, W.Zs, W.status);
}

template <int W2>
static void step32_impl(const Plan &P, const Ptrs &W, int step, const hz_params &prm, double tol,
                        hipStream_t s)
{
    const int *pairs = W.otab + (size_t)step * P.npairs * 2;
    prof_mark(K_GRAM, true, s);
    hipLaunchKernelGGL(k_gram32<W2>, dim3(P.splits, P.npairs, 2), dim3(256), 0, s, W.Fs, W.Gs,
                       P.mfw, P.mgw, pairs, P.splits, W.part);
    launch_gram_sum(P, W, s);
    hipLaunchKernelGGL(k_offdiag<W2>, dim3(2 * P.npairs), dim3(256), 0, s, W.gram, step,
                       P.npairs, W.offd);
    prof_mark(K_GRAM, false, s);
    prof_mark(K_INNER, true, s);
    launch_inner_real(P, W, step, prm, tol, false, s);
    prof_mark(K_INNER, false, s);
    const int64_t rpt = 4 * (int64_t)P.upd_rows;
    const int nt = (int)((P.mfw + P.mgw + P.nzw + rpt - 1) / rpt);
    prof_mark(K_UPDATE, true, s);
    hipLaunchKernelGGL(k_update32<W2>, dim3(nt, P.npairs), dim3(256), 0, s, W.Fs, W.Gs, W.Zs,
                       P.mfw, P.mgw, P.nzw, pairs, W.Zt, P.upd_rows,
                       W.cnt + (size_t)step * P.npairs * 4);
    prof_mark(K_UPDATE, false, s);
}

void launch_step_mixed32(const Plan &P, const Ptrs &W, int step, const hz_params &prm,
                         double tol, hipStream_t s)
{
    switch (P.W2) {
    case 16: step32_impl<16>(P, W, step, prm, tol, s); break;
    case 32: step32_impl<32>(P, W, step, prm, tol, s); break;
    default: step32_impl<64>(P, W, step, prm, tol, s); break;
    }
}

void launch_restart_mixed(const Plan &P, const Ptrs &W, const double *F, int64_t ldf,
                          const double *G, int64_t ldg, hipStream_t s)
{
    const int64_t nb = P.nw - P.n;
    const dim3 gf((unsigned)((P.mfw + 63) / 64), (unsigned)(P.nw / 64 + (P.nw % 64 ? 1 : 0)));
    const dim3 gg((unsigned)((P.mgw + 63) / 64), gf.y);
    hipLaunchKernelGGL(k_restart_gemm, gf, dim3(256), 0, s, F, ldf, P.mf, P.n, W.Zs, P.nzw, P.nw,
                       W.Fw, P.mfw, P.mfw);
    hipLaunchKernelGGL(k_restart_gemm, gg, dim3(256), 0, s, G, ldg, P.mg, P.n, W.Zs, P.nzw, P.nw,
                       W.Gw, P.mgw, P.mgw);
    const int64_t ef = (P.mfw - P.mf) * P.nw, eg = (P.mgw - P.mg) * P.nw;
    if (ef > 0)
        hipLaunchKernelGGL(k_restart_border, dim3((unsigned)((ef + 255) / 256)), dim3(256), 0, s,
                           P.mf, P.n, nb, P.mfw, P.nw, W.Zs, P.nzw, W.Fw);
    if (eg > 0)
        hipLaunchKernelGGL(k_restart_border, dim3((unsigned)((eg + 255) / 256)), dim3(256), 0, s,
                           P.mg, P.n, nb, P.mgw, P.nw, W.Zs, P.nzw, W.Gw);
    const int64_t ez = P.nzw * P.nw;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)((ez + 255) / 256)), dim3(256), 0, s, W.Zs, W.Zw,
                       ez);
}

}  // namespace hz
