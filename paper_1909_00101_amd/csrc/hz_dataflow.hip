// hz_dataflow.hip -- one persistent launch per outer sweep of the real FP64
// solver (pivot blocks of order 64).
//
// The block steps of a sweep (paper: Algorithm 1) are split into tasks:
//   GRAM(k, l, mat, s)   rows of split s of the pivot Gram block of pair l of
//                        step k, for F (mat 0) or G (mat 1) -> a partial
//   INNER(k, l)          the split partials added in split order, Cholesky,
//                        inner sweeps, Theta -> Z_tilde(k, l) and counters
//   UPDATE(k, l, t)      row tile t of [Y_p Y_q] <- [Y_p Y_q] Z_tilde(k, l) for
//                        the rows of F, then G, then Z
// with the dependencies the mathematics imposes: GRAM(k, l) needs every
// update tile of the two step-(k-1) pairs that held its block columns,
// INNER(k, l) needs its 2S partials, UPDATE(k, l) needs INNER(k, l).  Every
// (k, l) has its own partial and Z_tilde buffers, so no task overwrites data
// another still reads.
//
// The host lists the tasks in an order where each task comes after all it
// depends on, and interleaves the steps so that a pair of step k can start
// as soon as its two parents are updated, while the other pairs of step
// k-1 are still being solved or updated; the inner solves (latency bound,
// on a few dedicated workgroups) then overlap the bandwidth-bound Gram and
// update tasks on the remaining compute units.  Each workgroup runs its own
// ascending sub-list of that order and waits (bounded spin) until a task's
// inputs are complete; a wait that exceeds the spin limit sets an error
// word and gives up, so every workgroup exits.
//
// Completion is published with an agent-scope release fence by every
// thread before the workgroup barrier and a relaxed atomic increment; the
// waiting wave reads the counter with an agent-scope load and every thread
// follows the barrier with an agent-scope acquire fence, so data written on
// another XCD (and its L2) is seen.  The arithmetic of every task is fixed
// by (k, l, mat, s, t) alone -- not by which workgroup runs it or when --
// so the results are bitwise those of the per-step kernels.
#include "hz_device.h"
#include "hz_internal.h"
#include "hz_kernels_real.h"

namespace hz {

static constexpr int DF_W2 = 64, DF_LP = 16, DF_NT = 512;

__device__ __forceinline__ bool df_wait(const unsigned *p, unsigned target, unsigned limit,
                                        int *err)
{
    // executed by a whole wave: every lane reads the same word, and the
    // value steering the loop is taken from the first lane (uniform)
    unsigned it = 0;
    for (;;) {
        const unsigned v = (unsigned)__builtin_amdgcn_readfirstlane(
            (int)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (v >= target) return true;
        __builtin_amdgcn_s_sleep(4);
        // after one stalled wait every later wait gives up at once, so the
        // grid drains quickly
        const int e = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (++it > limit || (e & FLAG_STALL)) {
            atomicOr(err, FLAG_STALL);
            return false;
        }
    }
}

__global__ __launch_bounds__(DF_NT) void k_sweep_df(DFArgs A)
{
    constexpr int W2 = DF_W2;
    constexpr int LDS = inner_lds<W2>() > gram_lds<W2>()
                            ? (inner_lds<W2>() > update_lds<W2>() ? inner_lds<W2>() : update_lds<W2>())
                            : (gram_lds<W2>() > update_lds<W2>() ? gram_lds<W2>() : update_lds<W2>());
    __shared__ __attribute__((aligned(16))) double lds[LDS];
    const int tid = threadIdx.x;
    const size_t W2SQ = (size_t)W2 * W2;
    const int S = A.splits, NP = A.npairs;
    unsigned *const gram_done = A.dep;
    unsigned *const inner_done = A.dep + (size_t)A.steps * NP;
    unsigned *const upd_done = A.dep + 2 * (size_t)A.steps * NP;

    // Every workgroup walks its own list of task indices (ascending); the
    // list order is the dependency order, and the host assigns the inner
    // tasks to a few dedicated workgroups and the Gram and update tasks
    // round-robin to the rest.  A task only waits for tasks with smaller
    // indices; the smallest unfinished one belongs to a workgroup that has
    // finished all its earlier tasks, so it can run, and the grid drains --
    // given that every workgroup is resident, which the cooperative launch
    // guarantees.  All control flow here is wave-uniform: the waits and the
    // completion signal run in wave 0 as a whole (the other lanes add 0) and
    // every value a branch depends on is read through readfirstlane, so the
    // compiler cannot split lanes of a wave across the barriers.
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const unsigned one = (tid & 63) == 0 ? 1u : 0u;
    const int lb = __builtin_amdgcn_readfirstlane(A.wg_off[blockIdx.x]);
    const int le = __builtin_amdgcn_readfirstlane(A.wg_off[blockIdx.x + 1]);
    for (int li = lb; li < le; ++li) {
        const int t = __builtin_amdgcn_readfirstlane(A.wg_list[li]);
        const int4 Tv = A.tasks[t];
        const int kind = __builtin_amdgcn_readfirstlane(Tv.x);
        const int k = __builtin_amdgcn_readfirstlane(Tv.y);
        const int l = __builtin_amdgcn_readfirstlane(Tv.z);
        const int sub = __builtin_amdgcn_readfirstlane(Tv.w);
        const size_t kl = (size_t)k * NP + l;
        // wait until the task's inputs are complete
        if (wv == 0) {
            if (kind == DF_GRAM) {
                if (k > 0) {
                    const int pa = __builtin_amdgcn_readfirstlane(A.parents[kl].x);
                    const int pb = __builtin_amdgcn_readfirstlane(A.parents[kl].y);
                    const size_t base = (size_t)(k - 1) * NP;
                    df_wait(upd_done + base + pa, A.tiles, A.spin_limit, A.err);
                    df_wait(upd_done + base + pb, A.tiles, A.spin_limit, A.err);
                }
            } else if (kind == DF_INNER) {
                df_wait(gram_done + kl, 2u * S, A.spin_limit, A.err);
            } else {
                df_wait(inner_done + kl, 1u, A.spin_limit, A.err);
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

        const int *pr = A.otab + kl * 2;
        unsigned *sig;
        if (kind == DF_GRAM) {
            const int mat = sub / S, sp = sub % S;
            const int64_t m = mat ? A.mgw : A.mfw;
            const int64_t nch = m / 64;
            gram_block<W2>(mat ? A.Gw : A.Fw, m, pr[0], pr[1], nch * sp / S,
                              nch * (sp + 1) / S,
                              A.part + ((kl * 2 + mat) * S + sp) * W2SQ, lds);
            sig = gram_done + kl;
        } else if (kind == DF_INNER) {
            const double *pa = A.part + kl * 2 * S * W2SQ;
            inner_solve<W2, DF_LP>(pa, pa + S * W2SQ, S, W2SQ, A.itab, A.isteps, A.inner_max,
                                   A.tol, A.sort, A.variant, A.Zt + kl * W2SQ, A.cnt + kl * 4,
                                   A.status,
                                   k * 65536 + l, nullptr, lds);
            sig = inner_done + kl;
        } else {
            int64_t tt = sub;
            double *Y;
            int64_t m;
            if (tt < A.tiles_f) {
                Y = A.Fw;
                m = A.mfw;
            } else if (tt < A.tiles_f + A.tiles_g) {
                Y = A.Gw;
                m = A.mgw;
                tt -= A.tiles_f;
            } else {
                Y = A.Zw;
                m = A.nzw;
                tt -= A.tiles_f + A.tiles_g;
            }
            const int64_t rb = tt * A.tile_rows;
            const int64_t re = (rb + A.tile_rows < m) ? rb + A.tile_rows : m;
            // Z_tilde = I (counter word 3 of the inner task): nothing to update
            if (__builtin_amdgcn_readfirstlane((int)A.cnt[kl * 4 + 3]) == 0)
                update_rows<W2, 8>(Y, m, pr[0], pr[1], rb, re, A.Zt + kl * W2SQ, lds);
            sig = upd_done + kl;
        }
        // publish: every thread's stores reach the agent scope, then one
        // increment of the task's completion counter
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (wv == 0) __hip_atomic_fetch_add(sig, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Clears the dependency counters and the queue head of a sweep (a kernel,
// not a memset, so that it can sit in a captured graph).
__global__ __launch_bounds__(256) void k_df_clear(unsigned *__restrict__ dep, int n,
                                                  unsigned *__restrict__ head)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) dep[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) head[0] = 0u;
}

hipError_t df_occupancy(int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void *)k_sweep_df, DF_NT, 0);
}

hipError_t launch_sweep_df(const DFArgs &A, int nwg, hipStream_t s)
{
    const int n = 3 * A.steps * A.npairs;
    hipLaunchKernelGGL(k_df_clear, dim3((n + 255) / 256 < 64 ? (n + 255) / 256 : 64), dim3(256),
                       0, s, A.dep, n, A.head);
    DFArgs a = A;
    void *args[] = {&a};
    return hipLaunchCooperativeKernel((const void *)k_sweep_df, dim3(nwg), dim3(DF_NT), args, 0, s);
}

}  // namespace hz
