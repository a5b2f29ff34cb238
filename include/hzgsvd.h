/*
 * hzgsvd.h -- C ABI of the MI355X (gfx950) one-sided, blocked, implicit
 * Hari-Zimmermann GSVD library (libhzgsvd.so).
 *
 * Problem (paper, Section 1 and the start of Section 2): for F (m_F x n) and
 * G (m_G x n) of full column rank with min(m_F, m_G) >= n, compute
 *     F Z = U Sigma_F,   G Z = V Sigma_G,   U^* U = V^* V = I,
 *     Sigma_F^2 + Sigma_G^2 = I,   Sigma = Sigma_G^{-1} Sigma_F,
 * with Z square and nonsingular and the generalized singular values sorted
 * descendingly by a symmetric permutation of the columns of U, V, Z.
 * U overwrites F and V overwrites G (Section 3.1.1: U in place of F, V in
 * place of G).  Sigma, Sigma_F and Sigma_G are real (double) vectors of
 * length n, also for complex input (Section 3.1.1).
 *
 * Method (Sections 2.1-2.5, 3.3-3.6): prescale by Z_0 = diag(1/||g_j||);
 * sweeps of parallel block steps; in each step every pivot block-column pair
 * (width w each) forms its 2w x 2w Gram blocks F_b^*F_b and G_b^*G_b,
 * Cholesky-factors them, runs the pointwise implicit Hari-Zimmermann method
 * on the factors (at most inner_max_sweeps inner sweeps: 30 = "full block",
 * 1 = "block oriented"), rescales the accumulated transformation by Theta
 * (Section 2.4) and postmultiplies the pivot block columns of F, G, Z by it.
 * The solve stops after an outer sweep with no "big" transformation
 * (criterion C1, Section 2.5) or after max_sweeps sweeps.
 *
 * Layout: every matrix is column-major (Fortran order) with a leading
 * dimension in elements; complex matrices are interleaved (re, im) double
 * pairs (C99 double complex / numpy complex128).
 *
 * Memory and ownership: F, G, Z, sigma, sigma_f, sigma_g and work are
 * caller-owned DEVICE pointers (HIP device memory of the current device).
 * info is a caller-owned HOST pointer (may be NULL).  The library keeps no
 * pointer after a call returns.  If work is NULL the library allocates the
 * workspace itself for the duration of the call, stream-ordered on `stream`
 * (hipMallocAsync / hipFreeAsync); otherwise work must hold at
 * least hz_*_work_size(...) bytes, 256-byte aligned.  Inputs are read once
 * into the workspace, so F and G may be any device buffers of the stated
 * shape.  stream is a hipStream_t (NULL = the default stream); every call is
 * synchronous with respect to the host: it returns after its work on
 * stream has completed (the sweep loop reads the convergence counters back
 * once per sweep, as in the paper's host algorithm, Algorithm 1).
 *
 * Errors (return value):
 *    0            success, converged
 *   -i            argument i (1-based, in the order of the prototype) is
 *                 invalid; nothing was launched
 *   HZ_ENOCONV    max_sweeps reached; outputs are valid but not converged
 *   HZ_ECHOL      a pivot Gram block was not numerically positive definite
 *                 (input not of full column rank, or too ill-conditioned for
 *                 Gram + Cholesky): a Cholesky pivot of the 2w x 2w block was
 *                 not above 2w * DBL_EPSILON times that column's diagonal
 *                 entry; info->failed_pair names the block pair; outputs are
 *                 not meaningful
 *   HZ_ENONFINITE a NaN or infinity was found in the input or arose; outputs
 *                 are not meaningful
 *   HZ_EHIP       a HIP runtime call failed
 *   HZ_ENOSCRATCH (hz_dgsvd_noalloc only) the solve needs more workspace
 *                 than its static scratch; nothing was launched
 */
#ifndef HZGSVD_H
#define HZGSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HZ_OK 0
#define HZ_ENOCONV 1
#define HZ_ECHOL 2
#define HZ_ENONFINITE 3
#define HZ_EHIP 4
#define HZ_ENOSCRATCH 5   /* hz_dgsvd_noalloc only: workspace beyond its static scratch */

/* Size of the static device scratch of hz_dgsvd_noalloc, per device. */
#define HZ_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* Parallel orderings (Section 2.2).  HZ_ORD_MM: modified modulus,
 * quasi-cyclic with s = N steps per sweep (step k pairs p < q with
 * p + q = k mod N, and the two fixed points of even k with each other).
 * HZ_ORD_RR: round robin, cyclic with s = N - 1 steps. */
#define HZ_ORD_MM 1
#define HZ_ORD_RR 2
/* HZ_ORD_RING (inner_ordering only): a cyclic ordering
 * of the 2w columns of a pivot block built for the inner solver's data
 * movement, level by level.  The columns form blocks of size 2h (h = w,
 * w/2, ..., 1); in a block, column u of the first half meets every column
 * of the second half once, keeping its place while the others come to it
 * (h steps).  Level by level that is w + w/2 + ... + 1 = 2w - 1 steps of w
 * disjoint pairs, every pair once (Section 2.2's conditions on a parallel
 * ordering).  The order of the second half's columns within a level follows
 * the solver's lane groups (sets of min(h, 64/inner_lanes) columns visited
 * by the groups of one wave in xor order), so it depends on inner_lanes. */
#define HZ_ORD_RING 3

/* hz_params.schedule */
#define HZ_SCHED_STEPS 1
#define HZ_SCHED_DATAFLOW 2
#define HZ_SCHED_PERSISTENT 3

typedef struct hz_params {
    int variant;          /* Table 1, prescaled: 0 = small transformations by criterion
                             C1 (scaled cosines equal 1), 4 = by criterion C2 (unscaled
                             cosines equal 1), Section 2.5, both with ordinary dot
                             products; 1 and 5 = 0 and 4 with the enhanced dot products
                             of Appendix A for the pointwise pivot entries of the inner
                             solver: real pairs a_ii, a_jj, a_ij, b_ij (products rounded
                             toward -infinity and their non-negative errors summed apart),
                             complex pairs the squared norms a_ii, a_jj by the appendix's
                             simpler procedure (a_ij, b_ij ordinary) */
    int ordering;         /* outer block ordering, HZ_ORD_MM (default) or HZ_ORD_RR */
    int inner_ordering;   /* pointwise ordering inside a block pair: HZ_ORD_RR (default),
                             HZ_ORD_MM or HZ_ORD_RING (not with the dataflow schedule) */
    int w;                /* block-column width: 0 = default, else 8, 16 or 32 */
    int inner_max_sweeps; /* inner sweeps per block step: 30 = FB (default), 1 = BO */
    int max_sweeps;       /* outer sweep cap (default 30, Algorithm 1) */
    double tol;           /* relative-orthogonality threshold; <= 0 selects
                             sqrt(n)*DBL_EPSILON (Section 2.1) */
    int sort;             /* 1 = per-step column sorting heuristic (default), 0 = none */
    double mixed_switch;  /* mixed form: switch to FP64 when the largest scaled
                             off-diagonal Gram entry of an FP32 sweep falls below
                             this (default 1e-5) */
    int max_fp32_sweeps;  /* mixed form: cap on FP32 sweeps (default 20) */
    /* kernel tunables (0 = built-in choice); they change rounding order, so a
       fixed setting gives bitwise-reproducible results */
    int inner_lanes;      /* lanes per column pair in the inner solver: 4, 8 or 16 (0 = 16 for
                             2w = 64, else 8; 2w = 16 always uses 8; the complex solver
                             runs 4 as 8) */
    int gram_splits;      /* row splits of the Gram kernel (1..16) */
    int update_rows;      /* rows per wave in the update kernel (multiple of 16) */
    int schedule;         /* real FP64 path: 0 = default, HZ_SCHED_STEPS = one launch per
                             phase and block step, HZ_SCHED_DATAFLOW = one persistent
                             launch per sweep whose workgroups take Gram, inner-solve and
                             update tasks from a dependency-ordered queue (w = 32 only).
                             hz_dgsvd_batched: 0 = HZ_SCHED_PERSISTENT where it applies
                             (w = 16 or 32), else HZ_SCHED_STEPS; HZ_SCHED_PERSISTENT =
                             one launch for all sweeps of all pairs, whose workgroups take
                             whole block-pair tasks (Gram, inner solve, update) from a
                             queue ordered by the pairs' steps, each pair deciding its own
                             convergence on the device (inner_lanes is then 16 for w = 16,
                             8 or 16 for w = 32); HZ_SCHED_STEPS = launches per block step
                             and a host check after every sweep */
    int qr_shorten;       /* hz_dgsvd, hz_zgsvd, hz_dgsvd_mixed: 1 = shorten the pair first
                             (Section 2, before the prescaling): F P1 = Q_F R_F and
                             (G P1) P2 = Q_G R_G with column pivoting, the sweeps run on the
                             n x n pair (R_F P2, R_G), and Z = P1 P2 Z'', U = Q_F U'',
                             V = Q_G V''.  The factorizations are formed from the Grams F^H F,
                             G^H G by Cholesky with diagonal pivoting (the pivot rule of
                             column-pivoted QR) and one Cholesky-QR refinement, so F and G
                             must each have full column rank with kappa^2 * eps well below 1,
                             else HZ_ECHOL (failed_pair = -1); n <= 8192.
                             0 (default) = no shortening */
    int pivot_qr;         /* hz_dgsvd, hz_zgsvd, per-step schedule: 1 = the pivot factors of every
                             block pair come from QR factorizations of the block-column
                             pairs [F_p F_q], [G_p G_q] (Section 2.3, Appendix E; a tree of
                             Householder factorizations of row tiles) instead of Cholesky
                             factorizations of their Grams, for pairs whose block columns are
                             too ill-conditioned for the Grams; 0 (default) = Grams */
    int timing;           /* 1 = fill hz_info.t_gram, t_inner, t_update, t_other for this call:
                             HIP events bracket every Gram, inner-solve and update launch and
                             the sweeps are launched directly instead of replayed from a
                             captured graph (a few per cent slower); 0 (default) = no timing */
} hz_params;

typedef struct hz_info {
    int sweeps;           /* outer sweeps executed (FP64 sweeps in the mixed form) */
    int sweeps_fp32;      /* FP32 sweeps (mixed form only) */
    int converged;        /* 1 if the last sweep had no big transformation */
    int w;                /* block width used */
    int64_t failed_pair;  /* HZ_ECHOL: step * 65536 + pair of the first failing block */
    uint64_t rot_total;   /* transformations applied (inner level, all sweeps) */
    uint64_t rot_big;     /* big transformations among them */
    double last_offdiag;  /* mixed form: off-diagonal measure of the last FP32 sweep */
    uint64_t inner_sweeps;/* inner sweeps run, summed over all block steps */
    int status;           /* this solve's status code (per pair in the batched form) */
    int n_offdiag;        /* mixed form: FP32 sweeps recorded in fp32_offdiag */
    double fp32_offdiag[32]; /* mixed form: the off-diagonal measure (largest scaled
                             off-diagonal pivot Gram entry) of each FP32 sweep, first 32 */
    double t_gram, t_inner, t_update, t_other; /* with hz_params.timing = 1: milliseconds
                             spent in the Gram (with their split sums or QR pivot factors),
                             inner-solve and update launches of this call, and the rest of
                             the call's wall time (prescale, extraction, host syncs) */
    uint64_t updates_skipped; /* block updates skipped because the inner solve applied no
                             transformation and no swap, so Z_tilde = I (Section 2.5) */
    int fp32_chol_restarts; /* mixed form: 1 if an FP32 pivot Gram was not numerically
                             positive definite and the FP32 phase ended early; the FP64
                             restart and sweeps then ran as usual */
} hz_info;

/* Fill *p with the defaults listed above. */
void hz_default_params(hz_params *p);

/* Workspace bytes needed by hz_dgsvd / hz_zgsvd for the given shape (0 if
 * the shape or the parameters are invalid). */
size_t hz_dgsvd_work_size(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n);
size_t hz_zgsvd_work_size(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n);
size_t hz_dgsvd_mixed_work_size(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n);

/* Real FP64 GSVD (variants 0 and 4, Sections 2-3).  Arguments in order:
 *  1 p (host, may be NULL = defaults), 2 m_f, 3 m_g, 4 n,
 *  5 F (device, m_f x n, overwritten by U), 6 ldf (>= m_f),
 *  7 G (device, m_g x n, overwritten by V), 8 ldg (>= m_g),
 *  9 Z (device, n x n, output), 10 ldz (>= n),
 * 11 sigma, 12 sigma_f, 13 sigma_g (device, n doubles each, output),
 * 14 work (device or NULL), 15 work_bytes, 16 info (host or NULL),
 * 17 stream (hipStream_t or NULL). */
int hz_dgsvd(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n,
             double *F, int64_t ldf, double *G, int64_t ldg, double *Z, int64_t ldz,
             double *sigma, double *sigma_f, double *sigma_g,
             void *work, size_t work_bytes, hz_info *info, void *stream);

/* hz_dgsvd without allocations, for callers that cannot allocate device
 * memory (code being captured into a graph, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments 1-13 and status codes as hz_dgsvd;
 * 14 info (host or NULL), 15 stream.  The workspace is a static device
 * array of HZ_NOALLOC_SCRATCH_BYTES that every GPU the library runs on
 * holds until the process ends: a solve whose hz_dgsvd_work_size exceeds it
 * returns HZ_ENOSCRATCH before launching anything.  The call allocates
 * nothing (no hipMalloc, pinned host buffer, event or graph): its sweeps are
 * launched directly, not replayed from a captured graph, and per-kernel
 * timing (p->timing, hz_profile_enable) is not collected; p->qr_shorten and
 * the dataflow schedule, which need their own buffers, return -1.  Every
 * call on one GPU shares that GPU's array and leaves its contents behind:
 * calls of one process are serialised by a lock, and calls that overlap on
 * one GPU from elsewhere (another process's copy is its own) would race.
 * Results are bitwise those of hz_dgsvd with the same parameters. */
int hz_dgsvd_noalloc(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n,
                     double *F, int64_t ldf, double *G, int64_t ldg, double *Z, int64_t ldz,
                     double *sigma, double *sigma_f, double *sigma_g, hz_info *info,
                     void *stream);

/* The block ordering the solver uses: fills table (host, steps * (N/2) * 2
 * ints, row k = the N/2 disjoint pairs (p, q), p < q, of step k) for kind
 * HZ_ORD_MM or HZ_ORD_RR on N (even, >= 2) block columns, and returns the
 * number of steps (N or N - 1), or -1 for a bad kind or N.  table may be
 * NULL to query the step count. */
int hz_ordering(int kind, int N, int *table);

/* The ring ordering (HZ_ORD_RING) of the inner solver on a pivot block of
 * N = 2w columns (4 <= N <= 64, a power of two) with `lanes` lanes per
 * column pair (4, 8 or 16; N/2 * lanes >= 64): fills table (host,
 * (N-1) * (N/2) * 2 ints, row k = the pair (i, j), i < j, that lane group g
 * of the solver takes in step k, for g = 0 .. N/2-1; lane groups 64/lanes
 * at a time form one wave) and sync (host, N-1 ints: 1 where the solver
 * synchronises its whole workgroup after step k, 0 where only the wave's
 * own program order separates step k from step k+1).  Either may be NULL.
 * Returns N - 1, or -1 for bad arguments. */
int hz_ring_ordering(int N, int lanes, int *table, int *sync);

/* Diagnostic: the task list of one sweep of the dataflow schedule
 * (HZ_SCHED_DATAFLOW) for these sizes and parameters (w must be 32).
 * Returns the number of tasks, or -1 if the schedule does not apply.
 * tasks (host, 4 ints per task: kind 0 = Gram / 1 = inner / 2 = update,
 * step, pair, sub-index), parents (host, 2 ints per (step, pair): the pairs
 * of the previous step holding its two block columns) and info (host,
 * 4 ints: steps, pairs per step, Gram splits per matrix, update tiles per
 * pair) may each be NULL. */
int hz_dataflow_tasks(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n, int *tasks,
                      int *parents, int *info);

/* Diagnostic: evaluate the device's real 2x2 transformation (the one the
 * inner solver uses, Section 2.1.2) on `count` pivot pairs.  in (device,
 * 4*count doubles: a_ii, a_jj, a_ij, b_ij per pair, with |b_ij| < 1 and the
 * 2x2 A positive semidefinite), out (device, 4*count doubles: Z11, Z21, Z12,
 * Z22 of Z' per pair).  Returns 0 or HZ_EHIP. */
int hz_eval_2x2(int64_t count, const double *in, double *out, void *stream);

/* Diagnostic: the device's product rounded toward -infinity and its error
 * term, as the enhanced dot products of variants 1 and 5 form them
 * (Appendix A): for each of `count` pairs, c[i] = a[i]*b[i] rounded down and
 * d[i] = a[i]*b[i] - c[i] >= 0 (exact in the normal range).  a, b, c, d are
 * device arrays of count doubles.  Returns 0, -1 (bad arguments) or
 * HZ_EHIP. */
int hz_eval_mul_rd(int64_t count, const double *a, const double *b, double *c, double *d,
                   void *stream);

/* Diagnostic: the device's complex 2x2 transformation (Section 2.1.1) on
 * `count` pivot pairs.  in (device, 6*count doubles per pair: a_ii, a_jj,
 * Re a_ij, Im a_ij, Re b_ij, Im b_ij, with |b_ij| < 1), out (device,
 * 6*count doubles: Z11, Re Z21, Im Z21, Re Z12, Im Z12, Z22 of Z').
 * Returns 0 or HZ_EHIP. */
int hz_eval_2x2_z(int64_t count, const double *in, double *out, void *stream);

/* Per-kernel timing of later solves in this process, for measurement:
 * with enable = 1 (or 2, see below) every Gram, inner-solve and update
 * launch is bracketed by HIP events on the solve's stream (resolved at the
 * host syncs each sweep already makes), and the sums are cleared; enable =
 * 3 brackets only the inner-solve launches; enable = 0 stops collecting.
 * While collecting, sweeps are launched directly instead of replayed from
 * a captured hipGraph.  Not for concurrent solves. */
void hz_profile_enable(int enable);

/* With hz_profile_enable(2), the inner solver also stamps the device wall
 * clock at its phase boundaries; this returns the mean microseconds per
 * inner launch and pivot pair of phases 0 = load Gram blocks, 1 =
 * Cholesky, 2 = factor prescale, 3 = inner sweeps, 4 = Theta rescale and
 * store, in a host array of nphases (<= 5) entries. */
int hz_profile_read_phases(double *us, int nphases);

/* Copy the accumulated per-kind kernel time (milliseconds) and launch
 * counts for kinds 0 = Gram, 1 = inner solve, 2 = update, 3 = other into
 * host arrays of nkinds entries (either may be NULL); returns the number of
 * kinds written. */
int hz_profile_read(double *ms, int64_t *launches, int nkinds);

/* Complex128 GSVD (transformations of Section 2.1.1, Hermitian Gram blocks
 * and Cholesky).  F, G, Z are interleaved complex (re, im) device buffers,
 * 16-byte aligned; sigma, sigma_f, sigma_g stay real (Section 3.1.1).
 * Arguments and status codes as hz_dgsvd; w must be 0, 8 or 16 (pivot blocks
 * of order <= 32). */
int hz_zgsvd(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n,
             double *F, int64_t ldf, double *G, int64_t ldg, double *Z, int64_t ldz,
             double *sigma, double *sigma_f, double *sigma_g,
             void *work, size_t work_bytes, hz_info *info, void *stream);

/* Mixed-precision real GSVD.  Early sweeps run on FP32 copies of the
 * prescaled pair (FP32 MFMA Gram blocks with FP32 accumulation, widened to
 * FP64; FP32 MFMA block updates with Z_tilde rounded to FP32); Cholesky, the
 * inner Hari-Zimmermann solve, the convergence counters and Theta stay in
 * FP64.  After the FP32 sweep whose largest scaled off-diagonal Gram entry
 * |a_pq|/sqrt(a_pp a_qq) (over A_hat and B_hat) is below p->mixed_switch,
 * or one without big transformations, or after p->max_fp32_sweeps, the
 * iteration restarts in FP64 from F Z32, G Z32 (FP64 MFMA GEMMs with the
 * original F, G; every iterate satisfies F_k = F Z_k, Section 2.1) and
 * FP64 sweeps run to the FP64 stopping rule.  Arguments and status codes
 * as hz_dgsvd; F and G are read again for the restart and only overwritten
 * by U and V at the end; info->sweeps_fp32 and info->last_offdiag report
 * the FP32 phase. */
int hz_dgsvd_mixed(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n,
                   double *F, int64_t ldf, double *G, int64_t ldg, double *Z, int64_t ldz,
                   double *sigma, double *sigma_f, double *sigma_g,
                   void *work, size_t work_bytes, hz_info *info, void *stream);

/* Batched real FP64 GSVD of `batch` independent pairs of uneven sizes
 * (pair i: F_i m_f[i] x n[i], G_i m_g[i] x n[i]).  Every block step of the
 * sweep is one launch over the pivot block pairs of all pairs still
 * iterating, largest pairs first; each pair stops after its own sweep
 * without big transformations (Section 2.5 stopping rule, per pair),
 * decided on the device, so the host reads back one count per sweep.
 * One sweep is captured once as a hipGraph and replayed (direct launches
 * when the profiler is on).  All pairs share the block width w (0 = 8 if
 * every n <= 32, else 16).  Arguments in order:
 *  1 p (host, may be NULL),  2 batch (0..65535),
 *  3 m_f, 4 m_g, 5 n (host arrays of batch sizes, same rules as hz_dgsvd),
 *  6 F (host array of batch device pointers, overwritten by U_i), 7 ldf,
 *  8 G (likewise, overwritten by V_i), 9 ldg, 10 Z (device outputs), 11 ldz,
 * 12 sigma, 13 sigma_f, 14 sigma_g (host arrays of device outputs),
 * 15 work (device or NULL, 256-byte aligned), 16 work_bytes,
 * 17 infos (host array of batch hz_info or NULL; infos[i].status is pair
 *    i's own status), 18 stream.
 * Returns the most severe per-pair status (HZ_ENONFINITE, then HZ_ECHOL,
 * then HZ_ENOCONV), HZ_OK when every pair converged, or -(argument index)
 * for a bad argument (the first offending pair's). */
int hz_dgsvd_batched(const hz_params *p, int batch, const int64_t *m_f, const int64_t *m_g,
                     const int64_t *n, double *const *F, const int64_t *ldf,
                     double *const *G, const int64_t *ldg, double *const *Z,
                     const int64_t *ldz, double *const *sigma, double *const *sigma_f,
                     double *const *sigma_g, void *work, size_t work_bytes, hz_info *infos,
                     void *stream);

/* Workspace bytes hz_dgsvd_batched needs for these sizes (0 if invalid). */
size_t hz_dgsvd_batched_work_size(const hz_params *p, int batch, const int64_t *m_f,
                                  const int64_t *m_g, const int64_t *n);

/* Autotuner (the launch-parameter search the batched and single-pair
 * forms use).  Starting from p (NULL = defaults), the ordering inside a
 * block pair when p->inner_ordering is 0 (round robin or modified modulus),
 * the choice between one inner sweep and p->inner_max_sweeps (block-oriented
 * or full-block inner level, Section 3.5) and every tunable field that p
 * leaves at 0 -- w, gram_splits, update_rows, inner_lanes -- are varied in
 * turn, in that order, with the others held at the best so far, in passes until one
 * changes nothing (at most two); each candidate is timed as a complete
 * solve up to, not including, the final extraction, which reads F and G
 * (device, caller-owned, left unmodified) and writes only a scratch
 * workspace the tuner allocates; with p->qr_shorten = 1 the pair is
 * shortened once, untimed, and the candidates are timed on the square pair
 * the shortened solve iterates on.  Only candidates that converge count.
 * The fastest is written to *best (host) and its time in milliseconds to
 * *best_ms (host, may be NULL), and appended to the text file cache_path
 * (may be NULL) under a key of the sizes, the fixed parameters, the device
 * and the library version; a later call with the same key returns the
 * cached choice without timing, so the parameters -- and hence the
 * results, which depend on w and the Gram splits -- stay the same from run
 * to run.  Returns HZ_OK, HZ_ENOCONV (no candidate converged), HZ_EHIP, or
 * -(argument index): hz_dgsvd_tune 1 p, 2 m_f, 3 m_g, 4 n, 5 F, 6 ldf,
 * 7 G, 8 ldg, 9 cache_path, 10 best, 11 best_ms, 12 stream. */
int hz_dgsvd_tune(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n, const double *F,
                  int64_t ldf, const double *G, int64_t ldg, const char *cache_path,
                  hz_params *best, double *best_ms, void *stream);

/* Autotuner of the batched form: as hz_dgsvd_tune over w, inner_lanes and
 * the inner sweep cap, and over the outer ordering (modified modulus or
 * round robin) when p->ordering is 0, timing hz_dgsvd_batched without the
 * extraction; best->ordering is the chosen one.
 * Arguments: 1 p, 2 batch (1..65535), 3 m_f, 4 m_g, 5 n (host arrays),
 * 6 F, 7 ldf, 8 G, 9 ldg (host arrays; device matrices left unmodified),
 * 10 cache_path, 11 best, 12 best_ms, 13 stream. */
int hz_dgsvd_batched_tune(const hz_params *p, int batch, const int64_t *m_f, const int64_t *m_g,
                          const int64_t *n, const double *const *F, const int64_t *ldf,
                          const double *const *G, const int64_t *ldg, const char *cache_path,
                          hz_params *best, double *best_ms, void *stream);

/* Short English description of a status code. */
const char *hz_strerror(int status);

/* Library version string. */
const char *hz_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HZGSVD_H */
