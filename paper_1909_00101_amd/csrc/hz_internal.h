// hz_internal.h -- host-side plan and kernel-launch interface of libhzgsvd.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/hzgsvd.h"

namespace hz {

// Geometry and workspace layout of one solve.  The working copies Fw, Gw,
// Zw are column-major with leading dimension equal to their (64-padded) row
// count; columns n .. nw-1 are the bordering columns of the paper's data
// layout (Section 3.1): a unit in a fresh row of F and of G, zeros elsewhere.
struct Plan {
    int64_t mf, mg, n;        // caller shape
    int64_t nw;               // columns after bordering, multiple of 2w
    int64_t mfw, mgw, nzw;    // padded row counts of Fw, Gw, Zw (multiples of 64)
    int w, W2;                // block width and pivot block order 2w
    int nblk;                 // N = nw / w block columns
    int npairs;               // N / 2 block pairs per step
    int steps;                // outer steps per sweep
    int isteps;               // inner steps per inner sweep
    int splits;               // row splits of the Gram kernel
    int upd_rows;             // rows per wave in the update kernel
    int inner_lp;             // lanes per column pair in the inner solver (8 or 16)
    int is_complex;
    size_t esz;               // bytes per matrix element (8 or 16)
    // workspace offsets (bytes)
    size_t o_fw, o_gw, o_zw, o_part, o_gram, o_zt, o_otab, o_itab, o_cnt, o_status, o_tot;
    size_t o_sf, o_sg, o_sig, o_rank, o_border;
    size_t o_fs, o_gs, o_zs, o_offd;   // mixed form only (FP32 copies, off-diagonal measure)
    size_t o_qr[2];                    // pivot_qr only: triangles of the QR tree, two levels
    int dataflow;                      // one persistent launch per sweep (hz_dataflow.hip)
    int df_tiles_f, df_tiles_g, df_tiles_z, df_ntasks;
    int64_t df_tile_rows;
    size_t o_dpart, o_dzt, o_dtask, o_dpar, o_ddep, o_dwg;
    int df_nwg, df_inner_wg;
    int mixed;
    size_t total;
};

struct Ptrs {
    char *base;
    double *Fw, *Gw, *Zw, *part, *gram, *Zt;
    unsigned long long *phase;   // optional per-(step, pair) phase clocks, or null
    int *otab;
    int16_t *itab;
    unsigned long long *cnt;
    int *status;
    double *sf, *sg, *sig;
    int *rank, *border;
    float *Fs, *Gs, *Zs;         // mixed form: FP32 working copies
    double *offd;                // mixed form: per (step, pair, matrix) off-diagonal measure
    double *qr[2];               // pivot_qr: QR tree levels (ping-pong)
    unsigned long long *tot;   // per-sweep summary (SWEEP_TOT_N words)
};

// One pair of a batched solve, as the batched kernels see it.
struct BProb {
    const double *F, *G;        // caller input (device)
    double *U, *V, *Zo;         // caller outputs (U aliases F, V aliases G)
    double *sigma, *sigma_f, *sigma_g;
    int64_t mf, mg, n, ldf, ldg, ldz;
    double *Fw, *Gw, *Zw;       // working copies (bordered, 64-row padded)
    int64_t mfw, mgw, nzw, nw;
    double *gram, *Zt;          // per block pair: Gram blocks, Z_tilde
    double *sf, *sg, *sig;
    int *rank, *border;
    const int *otab;            // this pair's block ordering (steps x npairs x 2)
    int nblk, npairs, steps, pad;
    double tol;
};

// Host-side plan of a batched solve (device pointers into one workspace).
struct BPlan {
    int batch, w, W2, inner_lp, isteps, kmax;
    int64_t max_nw;
    BProb *probs;
    int2 *tasks;                        // per step: (pair, block pair), largest pairs first
    std::vector<int> ntasks, task_off;  // per step
    int16_t *itab;
    int *active, *pinfo, *pstatus, *nactive;
    unsigned long long *pcnt, *ptot;
    // persistent schedule: task list (pair, round << 12 | block pair), queue
    // head, per pair tasks done and finished flag, per (pair, sweep) counters
    int2 *ptask;
    int nptask;
    int *qhead, *pfin;
    unsigned *pdone;
    unsigned long long *psw;
    size_t total;
};

// status[] slots written by kernels (integer atomics only)
// Ring ordering inside a pivot block (HZ_ORD_RING), shared by the inner
// solver and the host-side table of hz_ring_ordering.  At the level of
// blocks of size 2h, group u of a block keeps its column u and meets column
// h + ring_col(...) of the block in sub-step t of phase p, where the second
// half is cut into nset = max(h / gw, 1) sets of ssz = min(h, gw) columns
// (gw = lane groups per wave), wave ow = u / ssz of the block takes set
// (ow + p) mod nset and group gi = u mod ssz of it column gi xor t of the
// set.  h, gw, ssz and nset are powers of two.
__host__ __device__ inline int ring_col(int ssz, int nset, int ow, int gi, int p, int t)
{
    return ssz * ((ow + p) & (nset - 1)) + (gi ^ t);
}

enum { ST_FLAGS = 0, ST_FAILPAIR = 1, ST_NSLOTS = 4 };
enum { FLAG_NONFINITE = 1, FLAG_CHOL = 2, FLAG_STALL = 4 };

// Kernel kinds timed by the optional per-launch profiler.
enum { K_GRAM = 0, K_INNER = 1, K_UPDATE = 2, K_OTHER = 3, K_NKINDS = 4 };

// Per-launch event hook: called before (begin=true) and after each timed
// launch on stream s when profiling is enabled; no-op otherwise.
void prof_mark(int kind, bool begin, hipStream_t s);

// launchers (real FP64), hz_real.hip
void launch_prescale_real(const Plan &P, const Ptrs &W, const double *F, int64_t ldf,
                          const double *G, int64_t ldg, hipStream_t s);
void launch_step_real(const Plan &P, const Ptrs &W, int step, const hz_params &prm, double tol,
                      hipStream_t s);
void launch_finish_real(const Plan &P, const Ptrs &W, double *F, int64_t ldf, double *G,
                        int64_t ldg, double *Z, int64_t ldz, double *sigma, double *sigma_f,
                        double *sigma_g, hipStream_t s);
void launch_eval_2x2(int64_t count, const double *in, double *out, hipStream_t s);
void launch_eval_mul_rd(int64_t count, const double *a, const double *b, double *c, double *d,
                        hipStream_t s);
void launch_rank(const Plan &P, const Ptrs &W, hipStream_t s);
void launch_gram_sum(const Plan &P, const Ptrs &W, hipStream_t s);

// QR factors of the block-column pairs as pivot factors (hz_pivqr.hip): the
// tree levels of one step, ending in W.gram (per pair R_F, R_G, W2 x W2 upper).
void launch_pivot_qr(const Plan &P, const Ptrs &W, int step, hipStream_t s);
int pivot_qr_tiles(const Plan &P);   // leaf tiles of the taller matrix
void launch_inner_real(const Plan &P, const Ptrs &W, int step, const hz_params &prm, double tol,
                       bool partials, hipStream_t s);

// Per-sweep summary written by k_sweep_totals: sums of the per-(step, pair)
// counters, the largest off-diagonal measure (mixed form, as bits of a
// double), the status words and the number of block updates skipped.
enum { TOT_ALL = 0, TOT_BIG = 1, TOT_ISW = 2, TOT_OFFD = 3, TOT_FLAGS = 4, TOT_FAILPAIR = 5,
       TOT_SKIP = 6, SWEEP_TOT_N = 8 };
void launch_sweep_totals(const Plan &P, const Ptrs &W, hipStream_t s);

// Persistent dataflow sweep (hz_dataflow.hip), real FP64, pivot blocks of 64.
enum { DF_GRAM = 0, DF_INNER = 1, DF_UPDATE = 2 };
struct DFArgs {
    double *Fw, *Gw, *Zw;
    int64_t mfw, mgw, nzw;
    const int *otab;             // steps x npairs x 2
    int npairs, steps, splits;   // splits: Gram row splits per matrix
    int tiles_f, tiles_g, tiles_z, tiles;
    int64_t tile_rows;
    double *part;                // steps x npairs x 2 x splits x 64 x 64
    double *Zt;                  // steps x npairs x 64 x 64
    const int16_t *itab;
    int isteps, inner_max, sort, variant;
    double tol;
    unsigned long long *cnt;     // steps x npairs x 4 (as the per-step kernels)
    int *status;
    const int4 *tasks;           // (kind, step, pair, sub) in dependency order
    int ntasks;
    const int *wg_off;           // per workgroup: its task indices (into tasks), ascending,
    const int *wg_list;          //   wg_list[wg_off[w] .. wg_off[w + 1])
    const int2 *parents;         // per (step, pair): the two step-1 pairs holding its blocks
    unsigned *dep;               // 3 x steps x npairs completion counters
    unsigned *head;              // (unused with static assignment)
    unsigned spin_limit;
    int *err;
};
hipError_t launch_sweep_df(const DFArgs &A, int nwg, hipStream_t s);
hipError_t df_occupancy(int *per_cu);   // resident sweep workgroups per compute unit

// launchers (batched), hz_batched.hip
void launchb_prescale(const BPlan &B, hipStream_t s);
void launchb_sweep(const BPlan &B, const hz_params &prm, hipStream_t s);
void launchb_finish(const BPlan &B, hipStream_t s);
hipError_t launchb_persistent(const BPlan &B, const hz_params &prm, hipStream_t s);

// launchers (mixed precision), hz_mixed.hip
void launch_prescale_mixed(const Plan &P, const Ptrs &W, const double *F, int64_t ldf,
                           const double *G, int64_t ldg, hipStream_t s);
void launch_step_mixed32(const Plan &P, const Ptrs &W, int step, const hz_params &prm,
                         double tol, hipStream_t s);
void launch_restart_mixed(const Plan &P, const Ptrs &W, const double *F, int64_t ldf,
                          const double *G, int64_t ldg, hipStream_t s);

// launchers (complex128), hz_cplx.hip; matrices are interleaved complex
void launch_prescale_cplx(const Plan &P, const Ptrs &W, const double *F, int64_t ldf,
                          const double *G, int64_t ldg, hipStream_t s);
void launch_step_cplx(const Plan &P, const Ptrs &W, int step, const hz_params &prm, double tol,
                      hipStream_t s);
void launch_finish_cplx(const Plan &P, const Ptrs &W, double *F, int64_t ldf, double *G,
                        int64_t ldg, double *Z, int64_t ldz, double *sigma, double *sigma_f,
                        double *sigma_g, hipStream_t s);
void launch_n1_cplx(int64_t mf, int64_t mg, double *F, double *G, double *Z, double *sigma,
                    double *sigma_f, double *sigma_g, int *status, hipStream_t s);
void launch_eval_2x2_cplx(int64_t count, const double *in, double *out, hipStream_t s);
void launch_n1_real(int64_t mf, int64_t mg, double *F, double *G, double *Z, double *sigma,
                    double *sigma_f, double *sigma_g, int *status, hipStream_t s);

// QR shortening of a tall pair, real or complex (hz_shorten.hip).  Workspace offsets
// (bytes) of Q_F, Q_G (ld ldqf, ldqg), the n x n buffers (ld ldn) R1 of F
// and G, the square pair F'', G'' (overwritten by U'', V'') and Z''; per
// factored matrix the Gram / Schur complement S (later R), R transposed Rt,
// the refinement factor R2, a column-block temporary T, the inverted
// diagonal blocks Xd and the pivoting state; the permutations p1 (F), q (G,
// = P1 P2), inv1, p2; then the square solve's own workspace.
struct SPlan {
    int64_t mf, mg, n, ldqf, ldqg, ldn;
    int cpt, nb, nblk;
    int cx;                      // complex (interleaved) elements
    size_t o_qf, o_qg, o_r1f, o_r1g, o_f2, o_g2, o_z2;
    size_t o_s[2], o_rt[2], o_r2[2], o_t[2], o_xd[2], o_d[2], o_done[2], o_id[2];  // per F, G
    size_t o_p1, o_q, o_inv1, o_p2, o_status, o_solve;
    size_t total;
};
int shorten_cpt(int64_t n);   // 0 if n is beyond the shortening's limit (8192)
bool make_splan(int64_t mf, int64_t mg, int64_t n, size_t solve_bytes, SPlan &S, int cx);
hipError_t launch_shorten(const SPlan &P, void *work, const double *F, int64_t ldf,
                          const double *G, int64_t ldg, hipStream_t s);
hipError_t launch_unshorten(const SPlan &P, void *work, double *U, int64_t ldu, double *V,
                            int64_t ldv, double *Z, int64_t ldz, hipStream_t s);

}  // namespace hz
