// hz_batched.hip -- batched real GSVD of many independent pairs of uneven
// sizes.  Every block step is one launch of each phase over the tasks of
// all pairs that still iterate (a pair with fewer steps per sweep, or one
// that has converged, simply has no tasks or exits at once), so hundreds
// of small problems fill the GPU together.  Per-pair convergence is
// decided on the device after every sweep (paper, Section 2.5 stopping
// rule per pair); the host replays one captured hipGraph per sweep and
// reads back a single count of still-active pairs.
#include "hz_device.h"
#include "hz_internal.h"
#include "hz_kernels_real.h"

namespace hz {

// Prescale and copy-in of every pair (grid (column blocks, pairs)).
__global__ __launch_bounds__(256) void kb_prescale(const BProb *__restrict__ probs,
                                                   int *__restrict__ pstatus)
{
    const BProb &P = probs[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= P.nw) return;
    double *fw = P.Fw + j * P.mfw, *gw = P.Gw + j * P.mgw, *zw = P.Zw + j * P.nzw;
    if (j < P.n) {
        const double *f = P.F + j * P.ldf, *g = P.G + j * P.ldg;
        double s = 0.0;
        for (int64_t r = lane; r < P.mg; r += 64) s = fma(g[r], g[r], s);
        s = wave_sum(s);
        const double d = 1.0 / sqrt(s);
        bool bad = !(s > 0.0) || !isfinite(s);
        for (int64_t r = lane; r < P.mfw; r += 64) {
            const double v = (r < P.mf) ? f[r] * d : 0.0;
            bad |= !isfinite(v);
            fw[r] = v;
        }
        for (int64_t r = lane; r < P.mgw; r += 64) gw[r] = (r < P.mg) ? g[r] * d : 0.0;
        for (int64_t r = lane; r < P.nzw; r += 64) zw[r] = (r == j) ? d : 0.0;
        if (bad) atomicOr(pstatus + (size_t)blockIdx.y * ST_NSLOTS + ST_FLAGS, FLAG_NONFINITE);
    } else {
        const int64_t k = j - P.n;
        for (int64_t r = lane; r < P.mfw; r += 64) fw[r] = (r == P.mf + k) ? 1.0 : 0.0;
        for (int64_t r = lane; r < P.mgw; r += 64) gw[r] = (r == P.mg + k) ? 1.0 : 0.0;
        for (int64_t r = lane; r < P.nzw; r += 64) zw[r] = (r == j) ? 1.0 : 0.0;
    }
}

// Gram blocks of step k: task t = (pair i, block pair l), blockIdx.y = matrix.
template <int W2>
__global__ __launch_bounds__(256) void kb_gram(const BProb *__restrict__ probs,
                                               const int2 *__restrict__ tasks,
                                               const int *__restrict__ active, int step)
{
    const int2 tk = tasks[blockIdx.x];
    if (!active[tk.x]) return;
    const BProb &P = probs[tk.x];
    const int mat = blockIdx.y;
    const int *pr = P.otab + ((size_t)step * P.npairs + tk.y) * 2;
    const int64_t m = mat ? P.mgw : P.mfw;
    __shared__ __attribute__((aligned(16))) double tile[gram_lds<W2>()];
    gram_block<W2>(mat ? P.Gw : P.Fw, m, pr[0], pr[1], 0, m / 64,
                   P.gram + ((size_t)tk.y * 2 + mat) * (W2 * W2), tile);
}

template <int W2, int LP, bool RING>
__global__ __launch_bounds__((W2 / 2) * LP) void kb_inner(
    const BProb *__restrict__ probs, const int2 *__restrict__ tasks, const int *__restrict__ active,
    int step, const int16_t *__restrict__ itab, int isteps, int inner_max, int sort, int variant,
    unsigned long long *__restrict__ pcnt, int *__restrict__ pstatus)
{
    __shared__ unsigned long long c[4];
    const int2 tk = tasks[blockIdx.x];
    if (!active[tk.x]) return;
    const BProb &P = probs[tk.x];
    const double *pa = P.gram + (size_t)tk.y * 2 * (W2 * W2);
    __shared__ __attribute__((aligned(16))) double lds[inner_lds<W2>()];
    inner_solve<W2, LP, RING>(pa, pa + W2 * W2, 1, 0, itab, isteps, inner_max, P.tol, sort, variant,
                        P.Zt + (size_t)tk.y * (W2 * W2), c,
                        pstatus + (size_t)tk.x * ST_NSLOTS, step * 65536 + tk.y, nullptr, lds);
    __syncthreads();
    if (threadIdx.x == 0) {
        // integer sums: the result does not depend on the order of arrival
        atomicAdd(pcnt + (size_t)tk.x * 4 + 0, c[0]);
        atomicAdd(pcnt + (size_t)tk.x * 4 + 1, c[1]);
        atomicAdd(pcnt + (size_t)tk.x * 4 + 2, c[2]);
    }
}

template <int W2>
__global__ __launch_bounds__(256) void kb_update(const BProb *__restrict__ probs,
                                                 const int2 *__restrict__ tasks,
                                                 const int *__restrict__ active, int step)
{
    const int2 tk = tasks[blockIdx.x];
    if (!active[tk.x]) return;
    const BProb &P = probs[tk.x];
    const int *pr = P.otab + ((size_t)step * P.npairs + tk.y) * 2;
    const int part = blockIdx.y;
    double *Y = part == 0 ? P.Fw : (part == 1 ? P.Gw : P.Zw);
    const int64_t m = part == 0 ? P.mfw : (part == 1 ? P.mgw : P.nzw);
    __shared__ double sz[update_lds<W2>()];
    update_rows<W2, 4>(Y, m, pr[0], pr[1], 0, m, P.Zt + (size_t)tk.y * (W2 * W2), sz);
}

// End of a sweep, one workgroup: per pair, add the sweep's counters to the
// totals, stop the pair after a sweep with no big transformation (converged),
// at the sweep cap, or on a failure flag; count the pairs still active.
__global__ __launch_bounds__(256) void kb_converge(int batch, int max_sweeps,
                                                   int *__restrict__ active,
                                                   unsigned long long *__restrict__ pcnt,
                                                   unsigned long long *__restrict__ ptot,
                                                   int *__restrict__ pinfo,
                                                   const int *__restrict__ pstatus,
                                                   int *__restrict__ nactive)
{
    __shared__ int red[256];
    int cntv = 0;
    for (int i = threadIdx.x; i < batch; i += 256) {
        if (active[i]) {
            unsigned long long *c = pcnt + (size_t)i * 4;
            ptot[(size_t)i * 4 + 0] += c[0];
            ptot[(size_t)i * 4 + 1] += c[1];
            ptot[(size_t)i * 4 + 2] += c[2];
            const int sw = ++pinfo[(size_t)i * 4 + 0];
            if (pstatus[(size_t)i * ST_NSLOTS + ST_FLAGS]) {
                active[i] = 0;
            } else if (c[1] == 0) {
                active[i] = 0;
                pinfo[(size_t)i * 4 + 1] = 1;   // converged
            } else if (sw >= max_sweeps) {
                active[i] = 0;
            }
            c[0] = c[1] = c[2] = 0;
        }
        cntv += active[i];
    }
    red[threadIdx.x] = cntv;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) nactive[0] = red[0];
}

// Extraction and sort per pair (grid (column blocks, pairs)).
__global__ __launch_bounds__(256) void kb_colnorms(const BProb *__restrict__ probs,
                                                   int *__restrict__ pstatus)
{
    const BProb &P = probs[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= P.nw) return;
    const double *f = P.Fw + j * P.mfw, *g = P.Gw + j * P.mgw, *z = P.Zw + j * P.nzw;
    double a = 0.0, b = 0.0;
    for (int64_t r = lane; r < P.mfw; r += 64) a = fma(f[r], f[r], a);
    for (int64_t r = lane; r < P.mgw; r += 64) b = fma(g[r], g[r], b);
    int bz = 0;
    for (int64_t r = P.n + lane; r < P.nw; r += 64) bz |= (z[r] != 0.0);
    a = wave_sum(a);
    b = wave_sum(b);
    const int isb = __any(bz) ? 1 : 0;
    if (lane == 0) {
        const double x = sqrt(a), y = sqrt(b);
        P.sf[j] = x;
        P.sg[j] = y;
        P.sig[j] = x / y;
        P.border[j] = isb;
        if (!isb && !(isfinite(x / y) && x > 0.0 && y > 0.0))
            atomicOr(pstatus + (size_t)blockIdx.y * ST_NSLOTS + ST_FLAGS, FLAG_NONFINITE);
    }
}

__global__ __launch_bounds__(256) void kb_rank(const BProb *__restrict__ probs)
{
    const BProb &P = probs[blockIdx.y];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= P.nw) return;
    if (P.border[j]) {
        P.rank[j] = -1;
        return;
    }
    const double s = P.sig[j];
    int64_t r = 0;
    for (int64_t k = 0; k < P.nw; ++k) {
        if (P.border[k]) continue;
        const double t = P.sig[k];
        r += (t > s) || (t == s && k < j);
    }
    P.rank[j] = (int)r;
}

__global__ __launch_bounds__(256) void kb_scatter(const BProb *__restrict__ probs)
{
    const BProb &P = probs[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= P.nw) return;
    const int rk = P.rank[j];
    if (rk < 0 || rk >= P.n) return;
    const double x = P.sf[j], y = P.sg[j];
    const double th = 1.0 / sqrt(x * x + y * y);
    const double ix = 1.0 / x, iy = 1.0 / y;
    const double *f = P.Fw + j * P.mfw, *g = P.Gw + j * P.mgw, *z = P.Zw + j * P.nzw;
    double *u = P.U + (int64_t)rk * P.ldf, *v = P.V + (int64_t)rk * P.ldg;
    double *zo = P.Zo + (int64_t)rk * P.ldz;
    for (int64_t r = lane; r < P.mf; r += 64) u[r] = f[r] * ix;
    for (int64_t r = lane; r < P.mg; r += 64) v[r] = g[r] * iy;
    for (int64_t r = lane; r < P.n; r += 64) zo[r] = z[r] * th;
    if (lane == 0) {
        P.sigma[rk] = x / y;
        P.sigma_f[rk] = x * th;
        P.sigma_g[rk] = y * th;
    }
}

// ------------------------------------------------------------ persistent
// One launch for all sweeps of all pairs.  A task is one block pair of one
// step of one pair: its Gram blocks, inner solve and block update, with the
// device bodies and the operation order of kb_gram, kb_inner and kb_update
// (so the results are bitwise those of the per-step schedule).  Workgroups
// claim tasks from a list ordered by the pair's round r = sweep * steps +
// step (largest pairs first within a round) with one atomic counter; a
// task of round r of pair i first waits until all tasks of the pair's
// earlier rounds are done (pdone[i] = r * npairs).  Only tasks that have
// been claimed are waited on, and a workgroup claims only while it runs, so
// every wait ends whether or not the whole grid is resident.  At the first
// step of a sweep the pair's previous sweep is complete: without a big
// transformation in it (Section 2.5), or with a failure flag, the pair is
// finished and its remaining tasks are skipped.  Data written by a task are
// published with a device-scope release before the counter is raised and
// read after a device-scope acquire.  A wait that exceeds spin_limit polls
// sets FLAG_STALL on the pair and skips, so the kernel always ends.
template <int W2, int LP, bool RING>
__global__ __launch_bounds__((W2 / 2) * LP) void kb_persist(
    const BProb *__restrict__ probs, const int2 *__restrict__ tasks, int ntasks,
    int *__restrict__ qhead, unsigned *__restrict__ pdone, int *__restrict__ pfin,
    unsigned long long *__restrict__ psw, int max_sweeps, const int16_t *__restrict__ itab,
    int isteps, int inner_max, int sort, int variant, int *__restrict__ pstatus,
    unsigned spin_limit)
{
    constexpr int NT = (W2 / 2) * LP;
    static_assert(NT >= 256 && NT % 64 == 0, "a persistent workgroup has at least four waves");
    constexpr int L1 = gram_lds<W2>(), L2 = inner_lds<W2>(), L3 = update_lds<W2>();
    constexpr int LDSN = (L1 > L2 ? (L1 > L3 ? L1 : L3) : (L2 > L3 ? L2 : L3));
    __shared__ __attribute__((aligned(16))) double lds[LDSN];
    __shared__ unsigned long long c[4];
    __shared__ int s_task, s_skip;
    const int tid = threadIdx.x, lane = tid & 63;
    // Claiming, waiting and deciding run on all lanes of wave 0 with every
    // value read made wave-uniform (readfirstlane), so that every branch of
    // the task loop is uniform: a loop exit taken by one lane alone would
    // let the compiler split the wave between loop levels.
    const bool claimer = __builtin_amdgcn_readfirstlane(tid >> 6) == 0;
    for (;;) {
        if (claimer) {
            int t = 0;
            if (lane == 0) t = atomicAdd(qhead, 1);
            t = __builtin_amdgcn_readfirstlane(t);
            int skip = 0;
            if (t < ntasks) {
                const int2 tk = tasks[t];
                const int i = __builtin_amdgcn_readfirstlane(tk.x);
                const int r = __builtin_amdgcn_readfirstlane(tk.y) >> 12;
                const BProb &P = probs[i];
                const int steps = __builtin_amdgcn_readfirstlane(P.steps);
                const unsigned need = (unsigned)r * (unsigned)__builtin_amdgcn_readfirstlane(P.npairs);
                const int sw = r / steps, k = r % steps;
                int *const st = pstatus + (size_t)i * ST_NSLOTS;
                unsigned spins = 0;
                for (;;) {
                    const int fin = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(pfin + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (fin) {
                        skip = 1;
                        break;
                    }
                    const unsigned d = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(pdone + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (d >= need) break;
                    if (++spins > spin_limit) {
                        if (lane == 0) {
                            atomicOr(st + ST_FLAGS, FLAG_STALL);
                            __hip_atomic_store(pfin + i, 1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        }
                        skip = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                if (!skip && k == 0 && sw > 0) {
                    // the pair's previous sweep is complete (Section 2.5 stopping rule)
                    const int big = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(psw + ((size_t)i * max_sweeps + sw - 1) * 3 + 1,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull
                            ? 1 : 0);
                    const int fl = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                        st + ST_FLAGS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (fl != 0 || big == 0) {
                        if (lane == 0)
                            __hip_atomic_store(pfin + i, 1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        skip = 1;
                    }
                }
            }
            if (lane == 0) {
                s_task = t;
                s_skip = skip;
            }
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_task);
        if (t >= ntasks) break;
        if (__builtin_amdgcn_readfirstlane(s_skip)) continue;
        const int2 tk = tasks[t];
        const int i = __builtin_amdgcn_readfirstlane(tk.x);
        const int r = __builtin_amdgcn_readfirstlane(tk.y) >> 12;
        const int l = __builtin_amdgcn_readfirstlane(tk.y) & 4095;
        const BProb &P = probs[i];
        const int steps = __builtin_amdgcn_readfirstlane(P.steps);
        const int sw = r / steps, k = r % steps;
        int *const st = pstatus + (size_t)i * ST_NSLOTS;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int *pr = P.otab + ((size_t)k * P.npairs + l) * 2;
        double *const gm = P.gram + (size_t)l * 2 * (W2 * W2);
        gram_block<W2>(P.Fw, P.mfw, pr[0], pr[1], 0, P.mfw / 64, gm, lds);
        __syncthreads();
        gram_block<W2>(P.Gw, P.mgw, pr[0], pr[1], 0, P.mgw / 64, gm + W2 * W2, lds);
        __syncthreads();
        double *const zt = P.Zt + (size_t)l * (W2 * W2);
        inner_solve<W2, LP, RING>(gm, gm + W2 * W2, 1, 0, itab, isteps, inner_max, P.tol, sort,
                                  variant, zt, c, st, k * 65536 + l, nullptr, lds);
        __syncthreads();
        const bool ident = __builtin_amdgcn_readfirstlane(c[3] != 0 ? 1 : 0) != 0;
        if (tid == 0) {
            unsigned long long *q = psw + ((size_t)i * max_sweeps + sw) * 3;
            atomicAdd(q + 0, c[0]);
            atomicAdd(q + 1, c[1]);
            atomicAdd(q + 2, c[2]);
        }
        if (!ident) {
            // Z_tilde = I leaves the block columns as they are (Section 2.5)
            update_rows<W2, NT / 64>(P.Fw, P.mfw, pr[0], pr[1], 0, P.mfw, zt, lds);
            __syncthreads();
            update_rows<W2, NT / 64>(P.Gw, P.mgw, pr[0], pr[1], 0, P.mgw, zt, lds);
            __syncthreads();
            update_rows<W2, NT / 64>(P.Zw, P.nzw, pr[0], pr[1], 0, P.nzw, zt, lds);
        }
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomicAdd(pdone + i, 1u);
        }
    }
}

// After the persistent launch: per pair the sweeps run (a sweep follows
// one with a big transformation and no failure flag, up to max_sweeps),
// whether the last one had no big transformation, and the counter totals
// over them -- what kb_converge records sweep by sweep.
__global__ __launch_bounds__(256) void kb_persist_totals(const BProb *__restrict__ probs,
                                                         int batch, int max_sweeps,
                                                         const unsigned long long *__restrict__ psw,
                                                         const int *__restrict__ pstatus,
                                                         int *__restrict__ pinfo,
                                                         unsigned long long *__restrict__ ptot)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= batch || probs[i].n < 2) return;
    const int fl = pstatus[(size_t)i * ST_NSLOTS + ST_FLAGS];
    unsigned long long a = 0, b = 0, q = 0;
    int sw = 0, conv = 0;
    while (sw < max_sweeps) {
        const unsigned long long *c = psw + ((size_t)i * max_sweeps + sw) * 3;
        a += c[0];
        b += c[1];
        q += c[2];
        ++sw;
        if (fl) break;
        if (c[1] == 0) {
            conv = 1;
            break;
        }
    }
    pinfo[(size_t)i * 4] = sw;
    pinfo[(size_t)i * 4 + 1] = conv;
    ptot[(size_t)i * 4] = a;
    ptot[(size_t)i * 4 + 1] = b;
    ptot[(size_t)i * 4 + 2] = q;
}

// ------------------------------------------------------------------ launchers

void launchb_prescale(const BPlan &B, hipStream_t s)
{
    hipLaunchKernelGGL(kb_prescale, dim3((unsigned)((B.max_nw + 3) / 4), B.batch), dim3(256), 0,
                       s, B.probs, B.pstatus);
}

template <int W2>
static void stepb_impl(const BPlan &B, int k, const hz_params &prm, hipStream_t s)
{
    const int nt = B.ntasks[k];
    if (nt == 0) return;
    const int2 *tasks = B.tasks + B.task_off[k];
    prof_mark(K_GRAM, true, s);
    hipLaunchKernelGGL(kb_gram<W2>, dim3(nt, 2), dim3(256), 0, s, B.probs, tasks, B.active, k);
    prof_mark(K_GRAM, false, s);
    prof_mark(K_INNER, true, s);
    const bool ring = (prm.inner_ordering == HZ_ORD_RING);
    const int lp = (W2 == 16) ? 8 : (B.inner_lp == 4 || B.inner_lp == 16 ? B.inner_lp : 8);
    auto go = [&](auto kern, int l) {
        hipLaunchKernelGGL(kern, dim3(nt), dim3((W2 / 2) * l), 0, s, B.probs, tasks, B.active, k,
                           B.itab, B.isteps, prm.inner_max_sweeps, prm.sort, prm.variant, B.pcnt,
                           B.pstatus);
    };
    if (lp == 4) {
        if constexpr (W2 != 16) {
            if (ring) go(kb_inner<W2, 4, true>, 4);
            else go(kb_inner<W2, 4, false>, 4);
        }
    } else if (lp == 16) {
        if constexpr (W2 != 16) {
            if (ring) go(kb_inner<W2, 16, true>, 16);
            else go(kb_inner<W2, 16, false>, 16);
        }
    } else {
        if (ring) go(kb_inner<W2, 8, true>, 8);
        else go(kb_inner<W2, 8, false>, 8);
    }
    prof_mark(K_INNER, false, s);
    prof_mark(K_UPDATE, true, s);
    hipLaunchKernelGGL(kb_update<W2>, dim3(nt, 3), dim3(256), 0, s, B.probs, tasks, B.active, k);
    prof_mark(K_UPDATE, false, s);
}

void launchb_sweep(const BPlan &B, const hz_params &prm, hipStream_t s)
{
    for (int k = 0; k < B.kmax; ++k) {
        switch (B.W2) {
        case 16: stepb_impl<16>(B, k, prm, s); break;
        case 32: stepb_impl<32>(B, k, prm, s); break;
        default: stepb_impl<64>(B, k, prm, s); break;
        }
    }
    hipLaunchKernelGGL(kb_converge, dim3(1), dim3(256), 0, s, B.batch, prm.max_sweeps, B.active,
                       B.pcnt, B.ptot, B.pinfo, B.pstatus, B.nactive);
}

template <int W2, int LP, bool RING>
static hipError_t persist_launch(const BPlan &B, const hz_params &prm, hipStream_t s)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kb_persist<W2, LP, RING>,
                                                         (W2 / 2) * LP, 0);
    if (e != hipSuccess) return e;
    const int grid = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
    hipLaunchKernelGGL((kb_persist<W2, LP, RING>), dim3(grid), dim3((W2 / 2) * LP), 0, s,
                       B.probs, B.ptask, B.nptask, B.qhead, B.pdone, B.pfin, B.psw,
                       prm.max_sweeps, B.itab, B.isteps, prm.inner_max_sweeps, prm.sort,
                       prm.variant, B.pstatus, 1u << 22);
    return hipGetLastError();
}

// The persistent schedule: all sweeps in one launch, then the counter totals.
hipError_t launchb_persistent(const BPlan &B, const hz_params &prm, hipStream_t s)
{
    const bool ring = (prm.inner_ordering == HZ_ORD_RING);
    hipError_t e = hipErrorInvalidValue;
    if (B.W2 == 64 && B.inner_lp == 16)
        e = ring ? persist_launch<64, 16, true>(B, prm, s) : persist_launch<64, 16, false>(B, prm, s);
    else if (B.W2 == 64 && B.inner_lp == 8)
        e = ring ? persist_launch<64, 8, true>(B, prm, s) : persist_launch<64, 8, false>(B, prm, s);
    else if (B.W2 == 32 && B.inner_lp == 16)
        e = ring ? persist_launch<32, 16, true>(B, prm, s) : persist_launch<32, 16, false>(B, prm, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kb_persist_totals, dim3((B.batch + 255) / 256), dim3(256), 0, s, B.probs,
                       B.batch, prm.max_sweeps, B.psw, B.pstatus, B.pinfo, B.ptot);
    return hipGetLastError();
}

void launchb_finish(const BPlan &B, hipStream_t s)
{
    const dim3 g4((unsigned)((B.max_nw + 3) / 4), B.batch);
    hipLaunchKernelGGL(kb_colnorms, g4, dim3(256), 0, s, B.probs, B.pstatus);
    hipLaunchKernelGGL(kb_rank, dim3((unsigned)((B.max_nw + 255) / 256), B.batch), dim3(256), 0,
                       s, B.probs);
    hipLaunchKernelGGL(kb_scatter, g4, dim3(256), 0, s, B.probs);
}

}  // namespace hz
