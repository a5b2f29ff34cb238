// hz_api.hip -- C ABI, planning and the host sweep loop of libhzgsvd
// (paper: Algorithm 1 of Section 3.6 -- prescale once, then outer sweeps of
// block steps, the per-step counters read back once per sweep, stop after a
// sweep without big transformations, then the final rescale/extraction).
#include <float.h>
#include <limits.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "hz_internal.h"

namespace hz {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Largest persistent grid of the dataflow schedule.
static constexpr int DF_MAX_WG = 1024;
static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Parallel orderings of Section 2.2 on N (even) indices; table[k][l] = (p, q).
// Modified modulus (quasi-cyclic, N steps): step k takes every p < q with
// p + q = k (mod N) and, for even k, pairs the two fixed points k/2 and
// k/2 + N/2.  Round robin (cyclic, N - 1 steps): index N - 1 stays, the
// others rotate: (k, N-1) and ((k-i) mod (N-1), (k+i) mod (N-1)).
template <typename T>
static int build_ordering(int kind, int N, std::vector<T> &tab)
{
    const int half = N / 2;
    if (kind == HZ_ORD_MM) {
        tab.assign((size_t)N * half * 2, 0);
        for (int k = 0; k < N; ++k) {
            int c = 0;
            for (int p = 0; p < N; ++p) {
                const int q = ((k - p) % N + N) % N;
                if (p < q) {
                    tab[(size_t)(k * half + c) * 2] = (T)p;
                    tab[(size_t)(k * half + c) * 2 + 1] = (T)q;
                    ++c;
                }
            }
            if ((k & 1) == 0) {
                tab[(size_t)(k * half + c) * 2] = (T)(k / 2);
                tab[(size_t)(k * half + c) * 2 + 1] = (T)(k / 2 + half);
            }
        }
        return N;
    }
    const int M = N - 1;
    tab.assign((size_t)M * half * 2, 0);
    for (int k = 0; k < M; ++k) {
        tab[(size_t)(k * half) * 2] = (T)k;
        tab[(size_t)(k * half) * 2 + 1] = (T)M;
        for (int i = 1; i < half; ++i) {
            int p = ((k - i) % M + M) % M, q = (k + i) % M;
            if (p > q) { const int t = p; p = q; q = t; }
            tab[(size_t)(k * half + i) * 2] = (T)p;
            tab[(size_t)(k * half + i) * 2 + 1] = (T)q;
        }
    }
    return M;
}

static int params_ok(const hz_params &p)
{
    if (p.variant != 0 && p.variant != 1 && p.variant != 4 && p.variant != 5) return 0;
    if (p.schedule != 0 && p.schedule != HZ_SCHED_STEPS && p.schedule != HZ_SCHED_DATAFLOW &&
        p.schedule != HZ_SCHED_PERSISTENT)
        return 0;
    if (p.ordering != HZ_ORD_MM && p.ordering != HZ_ORD_RR) return 0;
    if (p.inner_ordering != HZ_ORD_MM && p.inner_ordering != HZ_ORD_RR &&
        p.inner_ordering != HZ_ORD_RING)
        return 0;
    if (p.inner_ordering == HZ_ORD_RING && p.schedule == HZ_SCHED_DATAFLOW) return 0;
    if (p.w != 0 && p.w != 8 && p.w != 16 && p.w != 32) return 0;
    if (p.inner_max_sweeps < 1 || p.max_sweeps < 1) return 0;
    if (p.inner_lanes != 0 && p.inner_lanes != 4 && p.inner_lanes != 8 && p.inner_lanes != 16)
        return 0;
    if (p.gram_splits < 0 || p.gram_splits > 16 || p.update_rows < 0 || (p.update_rows % 16) != 0) return 0;
    if (p.qr_shorten != 0 && p.qr_shorten != 1) return 0;
    if (p.pivot_qr != 0 && p.pivot_qr != 1) return 0;
    if (p.pivot_qr && p.schedule == HZ_SCHED_DATAFLOW) return 0;
    return 1;
}

static int default_w(int64_t n, int is_complex)
{
    (void)is_complex;
    if (n <= 16) return 8;
    return 16;
}

// Complex pivot blocks are kept at order 2w <= 32 (three interleaved
// complex 32x32 tiles in LDS).
static int w_ok_for(const hz_params &p, int is_complex)
{
    return !is_complex || p.w == 0 || p.w == 8 || p.w == 16;
}

// The table the inner solver reads for a table ordering (the ring ordering
// is generated inside the solver; a round-robin table fills its slot).
static int inner_table_kind(int inner_ordering)
{
    return inner_ordering == HZ_ORD_RING ? HZ_ORD_RR : inner_ordering;
}

static bool make_plan(const hz_params &prm, int64_t mf, int64_t mg, int64_t n, int is_complex,
                      Plan &P, int mixed = 0)
{
    if (n < 2) return false;
    memset(&P, 0, sizeof(P));
    P.mf = mf;
    P.mg = mg;
    P.n = n;
    P.is_complex = is_complex;
    P.esz = is_complex ? 16 : 8;
    P.w = prm.w ? prm.w : default_w(n, is_complex);
    P.W2 = 2 * P.w;
    P.nw = round_up(n, P.W2);
    const int64_t nb = P.nw - n;
    P.mfw = round_up(mf + nb, 64);
    P.mgw = round_up(mg + nb, 64);
    P.nzw = round_up(P.nw, 64);
    P.nblk = (int)(P.nw / P.w);
    P.npairs = P.nblk / 2;
    P.steps = (prm.ordering == HZ_ORD_MM) ? P.nblk : P.nblk - 1;
    P.isteps = (prm.inner_ordering == HZ_ORD_MM) ? P.W2 : P.W2 - 1;
    const int64_t maxch = (P.mfw > P.mgw ? P.mfw : P.mgw) / 64;
    int64_t sp = prm.gram_splits ? prm.gram_splits : (512 + 2 * P.npairs - 1) / (2 * P.npairs);
    if (sp > 16) sp = 16;
    if (sp > maxch) sp = maxch;
    if (sp < 1) sp = 1;
    P.splits = (int)sp;
    // rows per wave of the update (the rows of F, G and Z are cut as one
    // sequence): 48 gives the real FP64 update of the 4096x1024 pair three
    // workgroups per compute unit
    P.upd_rows = prm.update_rows ? prm.update_rows : 48;
    P.inner_lp = prm.inner_lanes ? prm.inner_lanes : ((P.W2 == 64) ? 16 : 8);
    if (P.W2 == 16) P.inner_lp = 8;       // 8 column pairs x 8 lanes: one wave
    const size_t es = P.esz;
    size_t o = 0;
    P.o_fw = o; o = align256(o + es * (size_t)P.mfw * P.nw);
    P.o_gw = o; o = align256(o + es * (size_t)P.mgw * P.nw);
    P.o_zw = o; o = align256(o + es * (size_t)P.nzw * P.nw);
    P.o_part = o; o = align256(o + es * (size_t)P.npairs * 2 * P.splits * P.W2 * P.W2);
    P.o_gram = o; o = align256(o + es * (size_t)P.npairs * 2 * P.W2 * P.W2);
    P.o_zt = o; o = align256(o + es * (size_t)P.npairs * P.W2 * P.W2);
    P.o_otab = o; o = align256(o + sizeof(int) * (size_t)P.steps * P.npairs * 2);
    P.o_itab = o; o = align256(o + sizeof(int16_t) * (size_t)P.isteps * P.w * 2);
    P.o_cnt = o; o = align256(o + sizeof(unsigned long long) * (size_t)P.steps * P.npairs * 4);
    P.o_status = o; o = align256(o + sizeof(int) * ST_NSLOTS);
    P.o_tot = o; o = align256(o + sizeof(unsigned long long) * SWEEP_TOT_N);
    P.o_sf = o; o = align256(o + sizeof(double) * (size_t)P.nw);
    P.o_sg = o; o = align256(o + sizeof(double) * (size_t)P.nw);
    P.o_sig = o; o = align256(o + sizeof(double) * (size_t)P.nw);
    P.o_rank = o; o = align256(o + sizeof(int) * (size_t)P.nw);
    P.o_border = o; o = align256(o + sizeof(int) * (size_t)P.nw);
    P.dataflow = !is_complex && !mixed && P.W2 == 64 && P.inner_lp == 16 &&
                 prm.schedule == HZ_SCHED_DATAFLOW;
    if (P.dataflow) {
        P.df_tile_rows = 4 * (int64_t)P.upd_rows;
        P.df_tiles_f = (int)((P.mfw + P.df_tile_rows - 1) / P.df_tile_rows);
        P.df_tiles_g = (int)((P.mgw + P.df_tile_rows - 1) / P.df_tile_rows);
        P.df_tiles_z = (int)((P.nzw + P.df_tile_rows - 1) / P.df_tile_rows);
        const size_t kl = (size_t)P.steps * P.npairs;
        P.df_ntasks = (int)(kl * (2 * P.splits + 1 + P.df_tiles_f + P.df_tiles_g + P.df_tiles_z));
        P.o_dpart = o; o = align256(o + 8 * kl * 2 * P.splits * P.W2 * P.W2);
        P.o_dzt = o; o = align256(o + 8 * kl * P.W2 * P.W2);
        P.o_dtask = o; o = align256(o + 16 * (size_t)P.df_ntasks);
        P.o_dpar = o; o = align256(o + 8 * kl);
        P.o_ddep = o; o = align256(o + 4 * (3 * kl + 4));
        P.o_dwg = o; o = align256(o + 4 * ((size_t)DF_MAX_WG + 1 + P.df_ntasks));
    }
    if (prm.pivot_qr && !mixed) {
        const size_t tri = P.esz * (size_t)P.npairs * 2 * pivot_qr_tiles(P) * P.W2 * P.W2;
        P.o_qr[0] = o; o = align256(o + tri);
        P.o_qr[1] = o; o = align256(o + tri);
    }
    P.mixed = mixed;
    if (mixed) {
        P.o_fs = o; o = align256(o + sizeof(float) * (size_t)P.mfw * P.nw);
        P.o_gs = o; o = align256(o + sizeof(float) * (size_t)P.mgw * P.nw);
        P.o_zs = o; o = align256(o + sizeof(float) * (size_t)P.nzw * P.nw);
        P.o_offd = o; o = align256(o + sizeof(double) * (size_t)P.steps * P.npairs * 2);
    }
    P.total = o;
    return true;
}

static Ptrs make_ptrs(const Plan &P, void *work)
{
    Ptrs W;
    char *b = (char *)work;
    W.base = b;
    W.Fw = (double *)(b + P.o_fw);
    W.Gw = (double *)(b + P.o_gw);
    W.Zw = (double *)(b + P.o_zw);
    W.part = (double *)(b + P.o_part);
    W.gram = (double *)(b + P.o_gram);
    W.phase = nullptr;
    W.Zt = (double *)(b + P.o_zt);
    W.otab = (int *)(b + P.o_otab);
    W.itab = (int16_t *)(b + P.o_itab);
    W.cnt = (unsigned long long *)(b + P.o_cnt);
    W.status = (int *)(b + P.o_status);
    W.tot = (unsigned long long *)(b + P.o_tot);
    W.sf = (double *)(b + P.o_sf);
    W.sg = (double *)(b + P.o_sg);
    W.sig = (double *)(b + P.o_sig);
    W.rank = (int *)(b + P.o_rank);
    W.border = (int *)(b + P.o_border);
    W.Fs = P.mixed ? (float *)(b + P.o_fs) : nullptr;
    W.Gs = P.mixed ? (float *)(b + P.o_gs) : nullptr;
    W.Zs = P.mixed ? (float *)(b + P.o_zs) : nullptr;
    W.offd = P.mixed ? (double *)(b + P.o_offd) : nullptr;
    W.qr[0] = P.o_qr[0] ? (double *)(b + P.o_qr[0]) : nullptr;
    W.qr[1] = P.o_qr[1] ? (double *)(b + P.o_qr[1]) : nullptr;
    return W;
}

#define HZ_CHECK(call)                                                                         \
    do {                                                                                       \
        if ((call) != hipSuccess) {                                                            \
            rc = HZ_EHIP;                                                                      \
            goto done;                                                                         \
        }                                                                                      \
    } while (0)

// Validation common to the entry points: returns 0 or -(argument index).
static int check_args(int64_t mf, int64_t mg, int64_t n, const void *F, int64_t ldf,
                      const void *G, int64_t ldg, const void *Z, int64_t ldz, const void *s,
                      const void *sf, const void *sg)
{
    if (mf < 1) return -2;
    if (mg < 1) return -3;
    if (n < 1 || n > mf || n > mg || n > (int64_t)INT_MAX / 2) return -4;
    if (!F || ((uintptr_t)F & 7)) return -5;
    if (ldf < mf) return -6;
    if (!G || ((uintptr_t)G & 7)) return -7;
    if (ldg < mg) return -8;
    if (!Z || ((uintptr_t)Z & 7)) return -9;
    if (ldz < n) return -10;
    if (!s || ((uintptr_t)s & 7)) return -11;
    if (!sf || ((uintptr_t)sf & 7)) return -12;
    if (!sg || ((uintptr_t)sg & 7)) return -13;
    return 0;
}

// ------------------------------------------------------------ profiler
// Event timer: every timed launch is bracketed by two HIP events on its
// stream; the pending pairs are resolved at the host syncs the sweep loop
// already makes (flush), so timing adds no synchronisation.  One instance
// serves the process-wide profiler (hz_profile_*), another a single call
// with hz_params.timing = 1 (thread-local while that call runs).
struct EvTimer {
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<int> kind;
    int only = -1;                 // >= 0: events around launches of this kind only
    double ms[K_NKINDS] = {0, 0, 0, 0};
    int64_t launches[K_NKINDS] = {0, 0, 0, 0};
    void mark(int k, bool begin, hipStream_t s)
    {
        if (only >= 0 && k != only) return;
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            pool.push_back(e);
        }
        if (begin) kind.push_back(k);
        (void)hipEventRecord(pool[used++], s);
    }
    // Resolve recorded pairs; the caller has synchronised the stream.
    void flush()
    {
        for (size_t i = 0; i + 1 < used; i += 2) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, pool[i], pool[i + 1]) == hipSuccess) {
                const int k = kind[i / 2];
                ms[k] += t;
                launches[k] += 1;
            }
        }
        used = 0;
        kind.clear();
    }
    void clear()
    {
        used = 0;
        kind.clear();
        for (int k = 0; k < K_NKINDS; ++k) {
            ms[k] = 0.0;
            launches[k] = 0;
        }
    }
    ~EvTimer()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

struct Prof {
    std::mutex mu;
    bool on = false;
    EvTimer t;
    bool phases = false;           // also time the inner solver's phases
    double phase_us[5] = {0, 0, 0, 0, 0};
    int64_t phase_n = 0;
};
static Prof g_prof;
static thread_local EvTimer *tl_timer = nullptr;   // the running call's own timer

static thread_local bool tl_noalloc = false;       // the running call may not allocate

void prof_mark(int kind, bool begin, hipStream_t s)
{
    if (tl_noalloc) return;                         // events would be created on demand
    if (g_prof.on) g_prof.t.mark(kind, begin, s);
    if (tl_timer) tl_timer->mark(kind, begin, s);
}

static void prof_flush()
{
    if (g_prof.on) g_prof.t.flush();
    if (tl_timer) tl_timer->flush();
}

// Pinned host words the sweep loop reads the per-sweep summary into: one
// buffer per thread, allocated on first use and kept (so a solve does not
// pay for a pinned allocation).
static unsigned long long *sweep_readback()
{
    static thread_local unsigned long long *buf = nullptr;
    if (!buf && hipHostMalloc((void **)&buf, 64 * sizeof(unsigned long long), 0) != hipSuccess)
        buf = nullptr;
    return buf;
}

// Captured sweep graphs, kept across calls.  A graph holds the workspace
// addresses, the plan and the kernel arguments of one sweep, so it is keyed
// by all of them (the ordering tables are data in the workspace, rewritten
// by every call before the graph runs); the least recently used entry is
// destroyed beyond GRAPH_CACHE_MAX.  Calls that share a workspace must not
// overlap (they would race on it anyway).
static constexpr size_t GRAPH_CACHE_MAX = 1024;
struct GraphEntry {
    std::string key;
    hipGraph_t g;
    hipGraphExec_t e;
};
static std::mutex g_graph_mu;
static std::list<GraphEntry> g_graphs;

template <class Enqueue>
static hipError_t cached_graph(const std::string &key, Enqueue enqueue, hipStream_t cs,
                               hipGraphExec_t &exec)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
        if (it->key == key) {
            g_graphs.splice(g_graphs.begin(), g_graphs, it);
            exec = it->e;
            return hipSuccess;
        }
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) return err;
    enqueue(cs);
    err = hipStreamEndCapture(cs, &g);
    if (err != hipSuccess) return err;
    err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        (void)hipGraphDestroy(g);
        return err;
    }
    g_graphs.push_front(GraphEntry{key, g, e});
    while (g_graphs.size() > GRAPH_CACHE_MAX) {
        (void)hipGraphExecDestroy(g_graphs.back().e);
        (void)hipGraphDestroy(g_graphs.back().g);
        g_graphs.pop_back();
    }
    exec = e;
    return hipSuccess;
}

template <class T>
static void key_add(std::string &k, const T &v)
{
    k.append((const char *)&v, sizeof(v));
}

// One private non-blocking stream per device to capture the sweep graphs on
// (the caller's stream may be the null stream, which cannot be captured).
static hipStream_t capture_stream()
{
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

// Task list of one dataflow sweep (hz_dataflow.hip), in dependency order.
// Step 0: every pair's Gram tasks then its inner task.  Step k > 0: the
// pairs ordered by the later of their two parents' inner tasks; before a
// pair's Gram tasks come the update tiles of any parent not yet listed.
// The last step's update tiles close the list.  parents[k][l] holds the
// step-(k-1) pairs that held the block columns of pair l of step k.
static void build_df_tasks(const Plan &P, const std::vector<int> &otab, std::vector<int4> &tasks,
                           std::vector<int2> &parents)
{
    const int NP = P.npairs, NS = P.steps, S = P.splits;
    const int T = P.df_tiles_f + P.df_tiles_g + P.df_tiles_z;
    tasks.clear();
    tasks.reserve(P.df_ntasks);
    parents.assign((size_t)NS * NP, make_int2(0, 0));
    std::vector<int> owner(P.nblk), inner_pos((size_t)NS * NP, 0);
    std::vector<char> upd_listed((size_t)NS * NP, 0);
    auto emit_pair = [&](int k, int l) {
        for (int sub = 0; sub < 2 * S; ++sub) tasks.push_back(make_int4(DF_GRAM, k, l, sub));
        inner_pos[(size_t)k * NP + l] = (int)tasks.size();
        tasks.push_back(make_int4(DF_INNER, k, l, 0));
    };
    auto emit_update = [&](int k, int l) {
        if (upd_listed[(size_t)k * NP + l]) return;
        upd_listed[(size_t)k * NP + l] = 1;
        for (int t = 0; t < T; ++t) tasks.push_back(make_int4(DF_UPDATE, k, l, t));
    };
    for (int l = 0; l < NP; ++l) emit_pair(0, l);
    for (int k = 1; k < NS; ++k) {
        for (int l = 0; l < NP; ++l) {
            owner[otab[((size_t)(k - 1) * NP + l) * 2]] = l;
            owner[otab[((size_t)(k - 1) * NP + l) * 2 + 1]] = l;
        }
        std::vector<int> order(NP);
        std::vector<int> key(NP);
        for (int l = 0; l < NP; ++l) {
            const int a = owner[otab[((size_t)k * NP + l) * 2]];
            const int b = owner[otab[((size_t)k * NP + l) * 2 + 1]];
            parents[(size_t)k * NP + l] = make_int2(a, b);
            const int pa = inner_pos[(size_t)(k - 1) * NP + a];
            const int pb = inner_pos[(size_t)(k - 1) * NP + b];
            key[l] = pa > pb ? pa : pb;
            order[l] = l;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key[x] < key[y]; });
        for (int l : order) {
            const int2 par = parents[(size_t)k * NP + l];
            const int pa = inner_pos[(size_t)(k - 1) * NP + par.x];
            const int pb = inner_pos[(size_t)(k - 1) * NP + par.y];
            if (pa <= pb) { emit_update(k - 1, par.x); emit_update(k - 1, par.y); }
            else { emit_update(k - 1, par.y); emit_update(k - 1, par.x); }
            emit_pair(k, l);
        }
    }
    std::vector<int> last(NP);
    for (int l = 0; l < NP; ++l) last[l] = l;
    std::stable_sort(last.begin(), last.end(), [&](int x, int y) {
        return inner_pos[(size_t)(NS - 1) * NP + x] < inner_pos[(size_t)(NS - 1) * NP + y];
    });
    for (int l : last) emit_update(NS - 1, l);
    for (int k = 0; k + 1 < NS; ++k)
        for (int l = 0; l < NP; ++l) emit_update(k, l);   // pairs that parent nothing (none in MM)
}

enum { KIND_REAL = 0, KIND_COMPLEX = 1, KIND_MIXED = 2 };

// The host sweep loop shared by the real, complex and mixed solvers.
static int run_solve(const hz_params &prm, const Plan &P, void *work, size_t work_bytes,
                     hz_info *info, hipStream_t st, int kind, const void *F, int64_t ldf,
                     const void *G, int64_t ldg, void *U, void *V, void *Z, int64_t ldz,
                     double *sigma, double *sigma_f, double *sigma_g, bool finish = true,
                     bool noalloc = false);

// The QR-shortened real solve (qr_shorten = 1).
static int run_shortened(const hz_params &prm, const Plan &P, const SPlan &S, void *work,
                         hz_info *info, hipStream_t st, int kind, double *F, int64_t ldf,
                         double *G, int64_t ldg, double *Z, int64_t ldz, double *sigma,
                         double *sigma_f, double *sigma_g);

}  // namespace hz

using namespace hz;

extern "C" {

void hz_default_params(hz_params *p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->variant = 0;
    p->ordering = HZ_ORD_MM;
    p->inner_ordering = HZ_ORD_RR;
    p->w = 0;
    p->inner_max_sweeps = 30;
    p->max_sweeps = 30;
    p->tol = 0.0;
    p->sort = 1;
    p->mixed_switch = 1e-5;
    p->max_fp32_sweeps = 20;
}

const char *hz_strerror(int status)
{
    switch (status) {
    case HZ_OK: return "success";
    case HZ_ENOCONV: return "not converged within max_sweeps";
    case HZ_ECHOL: return "pivot Gram block not positive definite (rank-deficient or too ill-conditioned input)";
    case HZ_ENONFINITE: return "NaN or infinity in the input or the iteration";
    case HZ_EHIP: return "HIP runtime error";
    case HZ_ENOSCRATCH: return "the solve needs more workspace than the static scratch of hz_dgsvd_noalloc holds";
    default: return status < 0 ? "invalid argument" : "unknown status";
    }
}

const char *hz_version(void) { return "hzgsvd 0.2 (gfx950)"; }

int hz_eval_2x2(int64_t count, const double *in, double *out, void *stream)
{
    if (count < 0 || (count > 0 && (!in || !out))) return -1;
    if (count == 0) return 0;
    launch_eval_2x2(count, in, out, (hipStream_t)stream);
    if (hipGetLastError() != hipSuccess) return HZ_EHIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return HZ_EHIP;
    return 0;
}

int hz_eval_mul_rd(int64_t count, const double *a, const double *b, double *c, double *d,
                   void *stream)
{
    if (count < 0 || (count > 0 && (!a || !b || !c || !d))) return -1;
    if (count == 0) return 0;
    launch_eval_mul_rd(count, a, b, c, d, (hipStream_t)stream);
    if (hipGetLastError() != hipSuccess) return HZ_EHIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return HZ_EHIP;
    return 0;
}

int hz_ordering(int kind, int N, int *table)
{
    if ((kind != HZ_ORD_MM && kind != HZ_ORD_RR) || N < 2 || (N & 1) || N > (1 << 15)) return -1;
    std::vector<int> t;
    const int steps = build_ordering<int>(kind, N, t);
    if (table) memcpy(table, t.data(), t.size() * sizeof(int));
    return steps;
}

int hz_ring_ordering(int N, int lanes, int *table, int *sync)
{
    if (N < 4 || N > 64 || (N & (N - 1)) || (lanes != 4 && lanes != 8 && lanes != 16)) return -1;
    const int W = N / 2, gw = 64 / lanes, steps = N - 1;
    if (W * lanes < 64) return -1;               // the solver's workgroup is at least one wave
    if (!table && !sync) return steps;
    int st = 0;
    for (int h = W; h >= 1; h >>= 1) {
        const int nset = h >= gw ? h / gw : 1, ssz = h >= gw ? gw : h;
        for (int p = 0; p < nset; ++p)
            for (int t = 0; t < ssz; ++t, ++st) {
                for (int g = 0; g < W; ++g) {
                    const int blk = g / h, u = g % h;
                    if (table) {
                        table[((size_t)st * W + g) * 2] = blk * 2 * h + u;
                        table[((size_t)st * W + g) * 2 + 1] =
                            blk * 2 * h + h + ring_col(ssz, nset, u / ssz, u % ssz, p, t);
                    }
                }
                if (sync) sync[st] = (t + 1 == ssz) ? 1 : 0;
            }
    }
    return steps;
}

int hz_dataflow_tasks(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n, int *tasks,
                      int *parents, int *info)
{
    hz_params prm;
    if (p) prm = *p; else hz_default_params(&prm);
    prm.schedule = HZ_SCHED_DATAFLOW;
    if (!params_ok(prm) || prm.qr_shorten || m_f < n || m_g < n || n < 2) return -1;
    Plan P;
    if (!make_plan(prm, m_f, m_g, n, 0, P) || !P.dataflow) return -1;
    if (info) {
        info[0] = P.steps;
        info[1] = P.npairs;
        info[2] = P.splits;
        info[3] = P.df_tiles_f + P.df_tiles_g + P.df_tiles_z;
    }
    if (tasks || parents) {
        std::vector<int> otab;
        build_ordering<int>(prm.ordering, P.nblk, otab);
        std::vector<int4> t;
        std::vector<int2> par;
        build_df_tasks(P, otab, t, par);
        if (tasks) memcpy(tasks, t.data(), t.size() * sizeof(int4));
        if (parents) memcpy(parents, par.data(), par.size() * sizeof(int2));
    }
    return P.df_ntasks;
}

void hz_profile_enable(int enable)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = enable != 0;
    g_prof.phases = enable == 2;
    g_prof.t.only = (enable >= 4 && enable < 4 + K_NKINDS) ? enable - 4 : -1;
    for (int k = 0; k < 5; ++k) g_prof.phase_us[k] = 0.0;
    g_prof.phase_n = 0;
    g_prof.t.clear();
}

int hz_profile_read_phases(double *us, int nphases)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    const int n = nphases < 5 ? nphases : 5;
    for (int k = 0; k < n; ++k)
        us[k] = g_prof.phase_n ? g_prof.phase_us[k] / (double)g_prof.phase_n : 0.0;
    return n;
}

int hz_profile_read(double *ms, int64_t *launches, int nkinds)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    const int n = nkinds < K_NKINDS ? nkinds : K_NKINDS;
    for (int k = 0; k < n; ++k) {
        if (ms) ms[k] = g_prof.t.ms[k];
        if (launches) launches[k] = g_prof.t.launches[k];
    }
    return n;
}

size_t hz_dgsvd_work_size(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n);


static int solve_entry(int kind, const hz_params *p, int64_t m_f, int64_t m_g, int64_t n,
                       double *F, int64_t ldf, double *G, int64_t ldg, double *Z, int64_t ldz,
                       double *sigma, double *sigma_f, double *sigma_g, void *work,
                       size_t work_bytes, hz_info *info, void *stream)
{
    const int is_complex = (kind == KIND_COMPLEX);
    hz_params prm;
    if (p) prm = *p; else hz_default_params(&prm);
    if (!params_ok(prm) || !w_ok_for(prm, is_complex)) return -1;
    if (prm.schedule == HZ_SCHED_PERSISTENT) return -1;   // the batched form's schedule
    if (kind == KIND_MIXED && (prm.max_fp32_sweeps < 0 || !(prm.mixed_switch >= 0.0))) return -1;
    if (prm.qr_shorten && n > 1 && !shorten_cpt(n)) return -1;
    if (prm.pivot_qr && kind == KIND_MIXED) return -1;
    const int a = check_args(m_f, m_g, n, F, ldf, G, ldg, Z, ldz, sigma, sigma_f, sigma_g);
    if (a) return a;
    if (is_complex && (((uintptr_t)F | (uintptr_t)G | (uintptr_t)Z) & 15))
        return ((uintptr_t)F & 15) ? -5 : (((uintptr_t)G & 15) ? -7 : -9);
    if (work && ((uintptr_t)work & 255)) return -14;
    hipStream_t st = (hipStream_t)stream;
    if (info) memset(info, 0, sizeof(*info));
    if (n == 1) {
        int rc = HZ_OK;
        int *status = nullptr;
        int hs[ST_NSLOTS] = {0};
        bool own = false;
        if (work && work_bytes >= 256) status = (int *)work;
        else { if (hipMallocAsync((void **)&status, 256, st) != hipSuccess) return HZ_EHIP; own = true; }
        HZ_CHECK(hipMemsetAsync(status, 0, sizeof(int) * ST_NSLOTS, st));
        if (is_complex) launch_n1_cplx(m_f, m_g, F, G, Z, sigma, sigma_f, sigma_g, status, st);
        else launch_n1_real(m_f, m_g, F, G, Z, sigma, sigma_f, sigma_g, status, st);
        HZ_CHECK(hipGetLastError());
        HZ_CHECK(hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, st));
        HZ_CHECK(hipStreamSynchronize(st));
        if (hs[ST_FLAGS] & FLAG_NONFINITE) rc = HZ_ENONFINITE;
        if (info) { info->converged = 1; info->w = 1; info->status = rc; }
    done:
        if (own) (void)hipFreeAsync(status, st);
        return rc;
    }
    Plan P;
    if (prm.qr_shorten) {
        if (!make_plan(prm, n, n, n, is_complex, P, kind == KIND_MIXED)) return -4;
        SPlan S;
        if (!make_splan(m_f, m_g, n, P.total, S, is_complex)) return -4;
        if (work && work_bytes < S.total) return -15;
        return run_shortened(prm, P, S, work, info, st, kind, F, ldf, G, ldg, Z, ldz, sigma,
                             sigma_f, sigma_g);
    }
    if (!make_plan(prm, m_f, m_g, n, is_complex, P, kind == KIND_MIXED)) return -4;
    if (work && work_bytes < P.total) return -15;
    return run_solve(prm, P, work, work_bytes, info, st, kind, F, ldf, G, ldg, F, G, Z, ldz,
                     sigma, sigma_f, sigma_g);
}

static size_t work_size_entry(int kind, const hz_params *p, int64_t m_f, int64_t m_g,
                              int64_t n)
{
    const int is_complex = (kind == KIND_COMPLEX);
    hz_params prm;
    if (p) prm = *p; else hz_default_params(&prm);
    if (!params_ok(prm) || !w_ok_for(prm, is_complex) || m_f < n || m_g < n || n < 1) return 0;
    if (prm.qr_shorten && n > 1 && !shorten_cpt(n)) return 0;
    if (prm.pivot_qr && kind == KIND_MIXED) return 0;
    if (n == 1) return 256;
    Plan P;
    if (prm.qr_shorten) {
        SPlan S;
        if (!make_plan(prm, n, n, n, is_complex, P, kind == KIND_MIXED) ||
            !make_splan(m_f, m_g, n, P.total, S, is_complex))
            return 0;
        return S.total;
    }
    if (!make_plan(prm, m_f, m_g, n, is_complex, P, kind == KIND_MIXED)) return 0;
    return P.total;
}

int hz_dgsvd(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n, double *F, int64_t ldf,
             double *G, int64_t ldg, double *Z, int64_t ldz, double *sigma, double *sigma_f,
             double *sigma_g, void *work, size_t work_bytes, hz_info *info, void *stream)
{
    return solve_entry(KIND_REAL, p, m_f, m_g, n, F, ldf, G, ldg, Z, ldz, sigma, sigma_f,
                       sigma_g, work, work_bytes, info, stream);
}

int hz_dgsvd_mixed(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n, double *F,
                   int64_t ldf, double *G, int64_t ldg, double *Z, int64_t ldz, double *sigma,
                   double *sigma_f, double *sigma_g, void *work, size_t work_bytes, hz_info *info,
                   void *stream)
{
    return solve_entry(KIND_MIXED, p, m_f, m_g, n, F, ldf, G, ldg, Z, ldz, sigma, sigma_f,
                       sigma_g, work, work_bytes, info, stream);
}

int hz_zgsvd(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n, double *F, int64_t ldf,
             double *G, int64_t ldg, double *Z, int64_t ldz, double *sigma, double *sigma_f,
             double *sigma_g, void *work, size_t work_bytes, hz_info *info, void *stream)
{
    return solve_entry(KIND_COMPLEX, p, m_f, m_g, n, F, ldf, G, ldg, Z, ldz, sigma, sigma_f,
                       sigma_g, work, work_bytes, info, stream);
}

size_t hz_zgsvd_work_size(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n)
{
    return work_size_entry(KIND_COMPLEX, p, m_f, m_g, n);
}

}  // extern "C"

// Workspace of hz_dgsvd_noalloc: one static array per device, resolved to
// its device address once per device (the array's name is only a host-side
// stand-in).  g_scratch_mu also serialises the calls of this process that
// use the array, which would otherwise race on it.
static __device__ __align__(256) unsigned char scratch[HZ_NOALLOC_SCRATCH_BYTES];
static constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SCRATCH_MAX_DEVICES];

// The calling device's scratch address (g_scratch_mu held), or nullptr.
static void *scratch_ptr()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_MAX_DEVICES) return nullptr;
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

extern "C" {

int hz_dgsvd_noalloc(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n, double *F,
                     int64_t ldf, double *G, int64_t ldg, double *Z, int64_t ldz, double *sigma,
                     double *sigma_f, double *sigma_g, hz_info *info, void *stream)
{
    hz_params prm;
    if (p) prm = *p; else hz_default_params(&prm);
    if (!params_ok(prm) || !w_ok_for(prm, 0)) return -1;
    if (prm.qr_shorten || prm.timing || prm.schedule == HZ_SCHED_DATAFLOW) return -1;
    const int a = check_args(m_f, m_g, n, F, ldf, G, ldg, Z, ldz, sigma, sigma_f, sigma_g);
    if (a) return a;
    Plan P;
    const bool planned = (n == 1) || make_plan(prm, m_f, m_g, n, 0, P, false);
    if (!planned) return -4;
    if (n > 1 && P.dataflow) return -1;
    const size_t need = (n == 1) ? 256 : P.total;
    if (need > HZ_NOALLOC_SCRATCH_BYTES) return HZ_ENOSCRATCH;
    hipStream_t st = (hipStream_t)stream;
    if (info) memset(info, 0, sizeof(*info));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    void *work = scratch_ptr();
    if (!work) return HZ_EHIP;
    tl_noalloc = true;
    int rc = HZ_OK;
    if (n == 1) {
        int hs[ST_NSLOTS] = {0};
        int *status = (int *)work;
        if (hipMemcpyAsync(status, hs, sizeof(hs), hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = HZ_EHIP;
        } else {
            launch_n1_real(m_f, m_g, F, G, Z, sigma, sigma_f, sigma_g, status, st);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = HZ_EHIP;
            else if (hs[ST_FLAGS] & FLAG_NONFINITE)
                rc = HZ_ENONFINITE;
        }
        if (info) { info->converged = 1; info->w = 1; info->status = rc; }
    } else {
        rc = run_solve(prm, P, work, HZ_NOALLOC_SCRATCH_BYTES, info, st, KIND_REAL, F, ldf, G,
                       ldg, F, G, Z, ldz, sigma, sigma_f, sigma_g, true, true);
    }
    tl_noalloc = false;
    return rc;
}

size_t hz_dgsvd_mixed_work_size(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n)
{
    return work_size_entry(KIND_MIXED, p, m_f, m_g, n);
}

size_t hz_dgsvd_work_size(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n)
{
    return work_size_entry(KIND_REAL, p, m_f, m_g, n);
}

int hz_eval_2x2_z(int64_t count, const double *in, double *out, void *stream)
{
    if (count < 0 || (count > 0 && (!in || !out))) return -1;
    if (count == 0) return 0;
    launch_eval_2x2_cplx(count, in, out, (hipStream_t)stream);
    if (hipGetLastError() != hipSuccess) return HZ_EHIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return HZ_EHIP;
    return 0;
}

}  // extern "C"

namespace hz {

static int run_solve(const hz_params &prm, const Plan &P, void *work, size_t work_bytes,
                     hz_info *info, hipStream_t st, int kind, const void *F, int64_t ldf,
                     const void *G, int64_t ldg, void *U, void *V, void *Z, int64_t ldz,
                     double *sigma, double *sigma_f, double *sigma_g, bool finish,
                     bool noalloc)
{
    (void)work_bytes;
    const auto t_start = std::chrono::steady_clock::now();
    int rc = HZ_OK;
    bool own = false;
    hipGraph_t own_graph[2] = {nullptr, nullptr};      // uncached (library-owned workspace)
    hipGraphExec_t own_exec[2] = {nullptr, nullptr};
    hipGraphExec_t execs[2] = {nullptr, nullptr};
    // Without allocations (hz_dgsvd_noalloc) the per-sweep summary is read
    // into host stack memory instead of the thread's pinned buffer (whose
    // first use allocates it).
    unsigned long long hstack[64];
    unsigned long long *hpin = noalloc ? hstack : sweep_readback();
    unsigned long long *dphase = nullptr;
    if (!hpin) return HZ_EHIP;
    EvTimer call_timer;
    EvTimer *const prev_timer = tl_timer;
    if (prm.timing) tl_timer = &call_timer;
    if (!work) {
        if (hipMallocAsync(&work, P.total, st) != hipSuccess) {
            tl_timer = prev_timer;
            return HZ_EHIP;
        }
        own = true;
    }
    {
        Ptrs W = make_ptrs(P, work);
        std::vector<unsigned long long> hph;
        double clk_khz = 0.0;
        if (!noalloc && g_prof.on && g_prof.phases) {
            const size_t nph = (size_t)P.steps * P.npairs * 8;
            if (hipMalloc(&dphase, nph * sizeof(unsigned long long)) == hipSuccess) {
                W.phase = dphase;
                hph.resize(nph);
                int dev = 0, rate = 0;
                (void)hipGetDevice(&dev);
                (void)hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev);
                clk_khz = rate;
            }
        }
        const double tol = (prm.tol > 0.0) ? prm.tol : sqrt((double)P.n) * DBL_EPSILON;
        std::vector<int> otab;
        std::vector<int16_t> itab;
        build_ordering<int>(prm.ordering, P.nblk, otab);
        build_ordering<int16_t>(inner_table_kind(prm.inner_ordering), P.W2, itab);
        const int hs0[ST_NSLOTS] = {0, INT_MAX, 0, 0};
        int hs[ST_NSLOTS] = {0, INT_MAX, 0, 0};
        uint64_t tot_all = 0, tot_big = 0, tot_isw = 0, tot_skip = 0;
        int sweeps = 0, sweeps32 = 0, converged = 0, chol32 = 0;
        int n_off = 0;
        double offs[32];
        double last_off = 0.0;
        HZ_CHECK(hipMemcpyAsync(W.otab, otab.data(), otab.size() * sizeof(int),
                                hipMemcpyHostToDevice, st));
        HZ_CHECK(hipMemcpyAsync(W.itab, itab.data(), itab.size() * sizeof(int16_t),
                                hipMemcpyHostToDevice, st));
        HZ_CHECK(hipMemcpyAsync(W.status, hs0, sizeof(hs0), hipMemcpyHostToDevice, st));
        DFArgs dfa;
        int df_wg = 0;
        std::vector<int4> dtasks;
        std::vector<int2> dpar;
        std::vector<int> dwl;
        hipError_t df_err = hipSuccess;
        if (P.dataflow) {
            build_df_tasks(P, otab, dtasks, dpar);
            char *b = (char *)work;
            HZ_CHECK(hipMemcpyAsync(b + P.o_dtask, dtasks.data(), dtasks.size() * sizeof(int4),
                                    hipMemcpyHostToDevice, st));
            HZ_CHECK(hipMemcpyAsync(b + P.o_dpar, dpar.data(), dpar.size() * sizeof(int2),
                                    hipMemcpyHostToDevice, st));
            memset(&dfa, 0, sizeof(dfa));
            dfa.Fw = W.Fw;
            dfa.Gw = W.Gw;
            dfa.Zw = W.Zw;
            dfa.mfw = P.mfw;
            dfa.mgw = P.mgw;
            dfa.nzw = P.nzw;
            dfa.otab = W.otab;
            dfa.npairs = P.npairs;
            dfa.steps = P.steps;
            dfa.splits = P.splits;
            dfa.tiles_f = P.df_tiles_f;
            dfa.tiles_g = P.df_tiles_g;
            dfa.tiles_z = P.df_tiles_z;
            dfa.tiles = P.df_tiles_f + P.df_tiles_g + P.df_tiles_z;
            dfa.tile_rows = P.df_tile_rows;
            dfa.part = (double *)(b + P.o_dpart);
            dfa.Zt = (double *)(b + P.o_dzt);
            dfa.itab = W.itab;
            dfa.isteps = P.isteps;
            dfa.inner_max = prm.inner_max_sweeps;
            dfa.sort = prm.sort;
            dfa.variant = prm.variant;
            dfa.tol = tol;
            dfa.cnt = W.cnt;
            dfa.status = W.status;
            dfa.tasks = (const int4 *)(b + P.o_dtask);
            dfa.ntasks = P.df_ntasks;
            dfa.parents = (const int2 *)(b + P.o_dpar);
            dfa.dep = (unsigned *)(b + P.o_ddep);
            dfa.head = dfa.dep + 3 * (size_t)P.steps * P.npairs;
            dfa.spin_limit = 1u << 20;
            dfa.err = W.status + ST_FLAGS;
            int dev = 0, per_cu = 0;
            HZ_CHECK(hipGetDevice(&dev));
            HZ_CHECK(hipDeviceGetAttribute(&df_wg, hipDeviceAttributeMultiprocessorCount, dev));
            HZ_CHECK(df_occupancy(&per_cu));
            df_wg = df_wg * (per_cu > 0 ? per_cu : 1);
            if (df_wg > DF_MAX_WG) df_wg = DF_MAX_WG;
            // per-workgroup task lists: inner tasks round-robin over the
            // first NI workgroups, Gram and update tasks over the others,
            // each list in ascending (dependency) order
            const int NI = df_wg < 8 ? 0 : (P.npairs < df_wg / 4 ? P.npairs : df_wg / 4);
            std::vector<std::vector<int>> per((size_t)df_wg);
            int ci = 0, cm = 0;
            for (int i = 0; i < P.df_ntasks; ++i) {
                if (NI > 0 && dtasks[i].x == DF_INNER) per[(size_t)(ci++ % NI)].push_back(i);
                else per[(size_t)(NI + cm++ % (df_wg - NI))].push_back(i);
            }
            std::vector<int> wl((size_t)df_wg + 1 + P.df_ntasks);
            int o = 0;
            for (int w = 0; w < df_wg; ++w) {
                wl[w] = o;
                for (int i : per[w]) wl[(size_t)df_wg + 1 + o++] = i;
            }
            wl[df_wg] = o;
            dwl.swap(wl);
            int *dw = (int *)(b + P.o_dwg);
            HZ_CHECK(hipMemcpyAsync(dw, dwl.data(), dwl.size() * sizeof(int), hipMemcpyHostToDevice,
                                    st));
            dfa.wg_off = dw;
            dfa.wg_list = dw + df_wg + 1;
        }
        if (kind == KIND_COMPLEX)
            launch_prescale_cplx(P, W, (const double *)F, ldf, (const double *)G, ldg, st);
        else if (kind == KIND_MIXED)
            launch_prescale_mixed(P, W, (const double *)F, ldf, (const double *)G, ldg, st);
        else
            launch_prescale_real(P, W, (const double *)F, ldf, (const double *)G, ldg, st);
        HZ_CHECK(hipGetLastError());

        // One outer sweep: all block steps and the end-of-sweep summary,
        // then SWEEP_TOT_N words read back once (Algorithm 1).  Without
        // timing the sweep is replayed from a captured hipGraph (per
        // precision), cached across calls that reuse the workspace; the
        // dataflow sweep is a cooperative launch, which is not captured.
        const bool use_graph = !g_prof.on && !prm.timing && !P.dataflow && !noalloc;
        auto enqueue = [&](bool fp32, hipStream_t s) {
            if (P.dataflow && !fp32) {
                df_err = launch_sweep_df(dfa, df_wg, s);
                if (df_err == hipSuccess) launch_sweep_totals(P, W, s);
                return;
            }
            for (int k = 0; k < P.steps; ++k) {
                if (fp32) launch_step_mixed32(P, W, k, prm, tol, s);
                else if (kind == KIND_COMPLEX) launch_step_cplx(P, W, k, prm, tol, s);
                else launch_step_real(P, W, k, prm, tol, s);
            }
            launch_sweep_totals(P, W, s);
        };
        auto get_graph = [&](bool fp32) -> hipError_t {
            const int g = fp32 ? 1 : 0;
            if (execs[g]) return hipSuccess;
            hipStream_t cs = capture_stream();
            if (!cs) return hipErrorInvalidValue;
            auto enq = [&](hipStream_t s) { enqueue(fp32, s); };
            if (own) {
                // a workspace of this call only: capture, use once, destroy
                hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) return e;
                enq(cs);
                e = hipStreamEndCapture(cs, &own_graph[g]);
                if (e != hipSuccess) return e;
                e = hipGraphInstantiate(&own_exec[g], own_graph[g], nullptr, nullptr, 0);
                execs[g] = own_exec[g];
                return e;
            }
            int dev = 0;
            (void)hipGetDevice(&dev);
            std::string key;
            key_add(key, dev);
            key_add(key, kind);
            key_add(key, g);
            key_add(key, work);
            key_add(key, tol);
            key_add(key, P);
            key_add(key, prm.variant);
            key_add(key, prm.inner_ordering);   // the ring and round-robin plans are alike
            key_add(key, prm.inner_max_sweeps);
            key_add(key, prm.sort);
            key_add(key, prm.pivot_qr);
            return cached_graph(key, enq, cs, execs[g]);
        };
        auto sweep = [&](bool fp32, uint64_t &s_all, uint64_t &s_big) -> hipError_t {
            hipError_t e = hipSuccess;
            const int g = fp32 ? 1 : 0;
            if (use_graph) {
                e = get_graph(fp32);
                if (e != hipSuccess) return e;
                e = hipGraphLaunch(execs[g], st);
            } else {
                enqueue(fp32, st);
            }
            if (e != hipSuccess) return e;
            if (df_err != hipSuccess) return df_err;
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            e = hipMemcpyAsync(hpin, W.tot, SWEEP_TOT_N * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) return e;
            if (dphase) {
                e = hipMemcpyAsync(hph.data(), dphase, hph.size() * 8, hipMemcpyDeviceToHost, st);
                if (e != hipSuccess) return e;
            }
            e = hipStreamSynchronize(st);
            if (e != hipSuccess) return e;
            prof_flush();
            if (dphase && clk_khz > 0) {
                for (size_t i = 0; i < hph.size(); i += 8) {
                    for (int q = 0; q < 5; ++q)
                        g_prof.phase_us[q] += (double)(hph[i + q + 1] - hph[i + q]) / clk_khz * 1e3;
                    g_prof.phase_n += 1;
                }
            }
            s_all = hpin[TOT_ALL];
            s_big = hpin[TOT_BIG];
            tot_isw += hpin[TOT_ISW];
            tot_skip += hpin[TOT_SKIP];
            hs[ST_FLAGS] = (int)hpin[TOT_FLAGS];
            hs[ST_FAILPAIR] = (int)hpin[TOT_FAILPAIR];
            if (fp32) {
                last_off = __builtin_bit_cast(double, hpin[TOT_OFFD]);
                if (n_off < 32) offs[n_off++] = last_off;
            }
            tot_all += s_all;
            tot_big += s_big;
            return hipSuccess;
        };

        if (kind == KIND_MIXED) {
            // FP32 sweeps until the largest scaled off-diagonal Gram entry of a
            // sweep is below mixed_switch, a sweep has no big transformation, or
            // max_fp32_sweeps have run; then restart in FP64 from F Z32, G Z32.
            for (int sw = 0; sw < prm.max_fp32_sweeps; ++sw) {
                uint64_t s_all, s_big;
                HZ_CHECK(sweep(true, s_all, s_big));
                ++sweeps32;
                if (hs[ST_FLAGS]) break;
                if (s_big == 0 || last_off < prm.mixed_switch) break;
            }
            if (hs[ST_FLAGS]) {
                // An FP32 pivot Gram that is not numerically positive
                // definite ends the FP32 phase early: the failing block kept
                // Z_tilde = I and every other block's transformation was
                // applied, so Z32 is still a product of congruences and the
                // FP64 restart from F Z32, G Z32 is valid.  A non-finite
                // value in the FP32 iterates (e.g. an input beyond FP32
                // range) leaves nothing to restart from: the FP64 phase then
                // starts from the prescaled input, as the plain solver does
                // (and flags an input that is non-finite itself again).
                const bool nonfinite = (hs[ST_FLAGS] & FLAG_NONFINITE) != 0;
                chol32 = (hs[ST_FLAGS] & FLAG_CHOL) ? 1 : 0;
                memcpy(hs, hs0, sizeof(hs));
                HZ_CHECK(hipMemcpyAsync(W.status, hs0, sizeof(hs0), hipMemcpyHostToDevice, st));
                if (nonfinite)
                    launch_prescale_real(P, W, (const double *)F, ldf, (const double *)G, ldg, st);
                else
                    launch_restart_mixed(P, W, (const double *)F, ldf, (const double *)G, ldg, st);
            } else {
                launch_restart_mixed(P, W, (const double *)F, ldf, (const double *)G, ldg, st);
            }
            HZ_CHECK(hipGetLastError());
        }
        for (int sw = 0; sw < prm.max_sweeps; ++sw) {
            uint64_t s_all, s_big;
            HZ_CHECK(sweep(false, s_all, s_big));
            ++sweeps;
            if (hs[ST_FLAGS]) break;
            if (s_big == 0) {
                converged = 1;
                break;
            }
        }
        if (finish && !(hs[ST_FLAGS] & FLAG_CHOL)) {
            if (kind == KIND_COMPLEX)
                launch_finish_cplx(P, W, (double *)U, ldf, (double *)V, ldg, (double *)Z, ldz,
                                   sigma, sigma_f, sigma_g, st);
            else
                launch_finish_real(P, W, (double *)U, ldf, (double *)V, ldg, (double *)Z, ldz,
                                   sigma, sigma_f, sigma_g, st);
            HZ_CHECK(hipGetLastError());
            HZ_CHECK(hipMemcpyAsync(hs, W.status, sizeof(hs), hipMemcpyDeviceToHost, st));
        }
        HZ_CHECK(hipStreamSynchronize(st));
        if (hs[ST_FLAGS] & FLAG_STALL) rc = HZ_EHIP;
        else if (hs[ST_FLAGS] & FLAG_NONFINITE) rc = HZ_ENONFINITE;
        else if (hs[ST_FLAGS] & FLAG_CHOL) rc = HZ_ECHOL;
        else if (!converged) rc = HZ_ENOCONV;
        if (info) {
            info->sweeps = sweeps;
            info->sweeps_fp32 = sweeps32;
            info->converged = converged;
            info->w = P.w;
            info->failed_pair = (hs[ST_FLAGS] & FLAG_CHOL) ? hs[ST_FAILPAIR] : -1;
            info->rot_total = tot_all;
            info->rot_big = tot_big;
            info->inner_sweeps = tot_isw;
            info->last_offdiag = last_off;
            info->n_offdiag = n_off;
            for (int i = 0; i < n_off; ++i) info->fp32_offdiag[i] = offs[i];
            info->updates_skipped = tot_skip;
            info->fp32_chol_restarts = chol32;
            info->status = rc;
        }
    }
done:
    (void)hipStreamSynchronize(st);
    for (int g = 0; g < 2; ++g) {
        if (own_exec[g]) (void)hipGraphExecDestroy(own_exec[g]);
        if (own_graph[g]) (void)hipGraphDestroy(own_graph[g]);
    }
    if (dphase) (void)hipFree(dphase);
    if (own) {
        (void)hipFreeAsync(work, st);
        (void)hipStreamSynchronize(st);
    }
    tl_timer = prev_timer;
    if (prm.timing && info) {
        call_timer.flush();
        const double wall =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
                .count();
        info->t_gram = call_timer.ms[K_GRAM];
        info->t_inner = call_timer.ms[K_INNER];
        info->t_update = call_timer.ms[K_UPDATE];
        const double other = wall - info->t_gram - info->t_inner - info->t_update;
        info->t_other = other > 0.0 ? other : 0.0;
    }
    return rc;
}

// Shortening (hz_shorten.hip), a host sync to read its status, the square
// solve in the tail of the workspace (its final extraction writes U'', V''
// over F'', G'', and Z''), then U = Q_F U'', V = Q_G V'', Z = P1 P2 Z''.
// A failed factorization returns before the sweeps with info->failed_pair
// = -1.
static int run_shortened(const hz_params &prm, const Plan &P, const SPlan &S, void *work,
                         hz_info *info, hipStream_t st, int kind, double *F, int64_t ldf,
                         double *G, int64_t ldg, double *Z, int64_t ldz, double *sigma,
                         double *sigma_f, double *sigma_g)
{
    bool own = false;
    if (!work) {
        if (hipMallocAsync(&work, S.total, st) != hipSuccess) return HZ_EHIP;
        own = true;
    }
    char *b = (char *)work;
    int rc = HZ_OK;
    int hs[ST_NSLOTS] = {0, 0, 0, 0};
    if (launch_shorten(S, work, F, ldf, G, ldg, st) != hipSuccess ||
        hipMemcpyAsync(hs, b + S.o_status, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        rc = HZ_EHIP;
    else if (hs[ST_FLAGS] & FLAG_NONFINITE)
        rc = HZ_ENONFINITE;
    else if (hs[ST_FLAGS] & FLAG_CHOL)
        rc = HZ_ECHOL;
    if (rc != HZ_OK) {
        if (info) {
            memset(info, 0, sizeof(*info));
            info->w = P.w;
            info->failed_pair = -1;
            info->status = rc;
        }
    } else {
        double *F2 = (double *)(b + S.o_f2), *G2 = (double *)(b + S.o_g2);
        double *Z2 = (double *)(b + S.o_z2);
        // the mixed form reads F'', G'' again for its FP64 restart; its final
        // extraction, the only writer of U'', V'' over them, comes after
        rc = run_solve(prm, P, b + S.o_solve, S.total - S.o_solve, info, st, kind, F2, S.ldn,
                       G2, S.ldn, F2, G2, Z2, S.ldn, sigma, sigma_f, sigma_g, true);
        if (rc == HZ_OK || rc == HZ_ENOCONV) {
            if (launch_unshorten(S, work, F, ldf, G, ldg, Z, ldz, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = HZ_EHIP;
            if (info) info->status = rc;
        }
    }
    if (own) (void)hipFreeAsync(work, st);
    return rc;
}

}  // namespace hz

// ------------------------------------------------------------ batched form
namespace hz {

// Workspace layout of a batched solve.  The metadata region at the front
// (pair descriptors, per-step task lists, ordering tables, flags and
// counters) is staged on the host and copied in once; the per-pair working
// arrays follow, each 256-byte aligned.
struct BLayout {
    int w = 0, W2 = 0, isteps = 0, inner_lp = 0, kmax = 0;
    int persistent = 0;                  // one launch for all sweeps (kb_persist)
    int64_t max_nw = 0, nptask = 0;
    size_t o_probs = 0, o_tasks = 0, o_itab = 0, o_active = 0, o_pinfo = 0, o_pstatus = 0,
           o_nactive = 0, o_pcnt = 0, o_ptot = 0, meta = 0, total = 0;
    size_t o_ptask = 0, o_qhead = 0, o_pdone = 0, o_pfin = 0, o_psw = 0;
    std::vector<Plan> plan;              // per pair (n >= 2)
    std::vector<size_t> pair_off;        // per pair: start of its arrays
    std::vector<int> order;              // pairs by decreasing work
    std::vector<int> ntasks, task_off;   // per step
    std::vector<int> otab_nblk;          // distinct block counts
    std::vector<size_t> otab_off;
};

static size_t pair_bytes(const Plan &P)
{
    size_t o = 0;
    o = align256(o + 8 * (size_t)P.mfw * P.nw);
    o = align256(o + 8 * (size_t)P.mgw * P.nw);
    o = align256(o + 8 * (size_t)P.nzw * P.nw);
    o = align256(o + 8 * (size_t)P.npairs * 2 * P.W2 * P.W2);
    o = align256(o + 8 * (size_t)P.npairs * P.W2 * P.W2);
    o = align256(o + 3 * 8 * (size_t)P.nw);
    o = align256(o + 2 * 4 * (size_t)P.nw);
    return o;
}

static bool plan_batched(const hz_params &prm, int batch, const int64_t *mf, const int64_t *mg,
                         const int64_t *n, BLayout &L)
{
    int64_t nmax = 1;
    for (int i = 0; i < batch; ++i) nmax = n[i] > nmax ? n[i] : nmax;
    hz_params q = prm;
    L.w = prm.w ? prm.w : (nmax <= 32 ? 8 : 16);
    q.w = L.w;
    L.W2 = 2 * L.w;
    L.isteps = (prm.inner_ordering == HZ_ORD_MM) ? L.W2 : L.W2 - 1;
    L.inner_lp = prm.inner_lanes ? prm.inner_lanes : (L.W2 == 64 ? 16 : 8);
    if (L.W2 == 16) L.inner_lp = 8;
    // The persistent schedule (default where it applies) runs a task's
    // inner solve with the whole workgroup of at least four waves: 2w = 64
    // with 8 or 16 lanes per column pair, 2w = 32 with 16.
    const bool can_persist = L.W2 == 64 || L.W2 == 32;
    if (prm.schedule == HZ_SCHED_PERSISTENT && !can_persist) return false;
    L.persistent = can_persist && (prm.schedule == 0 || prm.schedule == HZ_SCHED_PERSISTENT);
    if (L.persistent) L.inner_lp = (L.W2 == 32) ? 16 : (L.inner_lp == 16 ? 16 : 8);
    L.plan.assign(batch, Plan{});
    std::vector<int64_t> work(batch, 0);
    for (int i = 0; i < batch; ++i) {
        if (n[i] < 2) continue;
        if (!make_plan(q, mf[i], mg[i], n[i], 0, L.plan[i])) return false;
        const Plan &P = L.plan[i];
        L.kmax = P.steps > L.kmax ? P.steps : L.kmax;
        L.max_nw = P.nw > L.max_nw ? P.nw : L.max_nw;
        work[i] = (P.mfw + P.mgw + P.nzw) * P.nw * P.nw;
        bool seen = false;
        for (int b : L.otab_nblk) seen |= (b == P.nblk);
        if (!seen) L.otab_nblk.push_back(P.nblk);
    }
    if (L.max_nw == 0) L.max_nw = 1;
    L.order.resize(batch);
    for (int i = 0; i < batch; ++i) L.order[i] = i;
    std::stable_sort(L.order.begin(), L.order.end(),
                     [&](int a, int b) { return work[a] > work[b]; });
    L.ntasks.assign(L.kmax, 0);
    L.task_off.assign(L.kmax, 0);
    int tot = 0;
    for (int k = 0; k < L.kmax; ++k) {
        L.task_off[k] = tot;
        for (int i : L.order)
            if (n[i] >= 2 && k < L.plan[i].steps) L.ntasks[k] += L.plan[i].npairs;
        tot += L.ntasks[k];
    }
    size_t o = 0;
    L.o_probs = o; o = align256(o + sizeof(BProb) * (size_t)batch);
    L.o_tasks = o; o = align256(o + sizeof(int2) * (size_t)(tot > 0 ? tot : 1));
    L.o_itab = o; o = align256(o + sizeof(int16_t) * (size_t)L.isteps * L.w * 2);
    L.otab_off.clear();
    for (int b : L.otab_nblk) {
        L.otab_off.push_back(o);
        const int steps = (prm.ordering == HZ_ORD_MM) ? b : b - 1;
        o = align256(o + sizeof(int) * (size_t)steps * (b / 2) * 2);
    }
    L.o_active = o; o = align256(o + sizeof(int) * (size_t)batch);
    L.o_pinfo = o; o = align256(o + sizeof(int) * 4 * (size_t)batch);
    L.o_pstatus = o; o = align256(o + sizeof(int) * ST_NSLOTS * (size_t)batch);
    L.o_nactive = o; o = align256(o + sizeof(int) * 4);
    L.o_pcnt = o; o = align256(o + sizeof(unsigned long long) * 4 * (size_t)batch);
    L.o_ptot = o; o = align256(o + sizeof(unsigned long long) * 4 * (size_t)batch);
    if (L.persistent) {
        // tasks of every round of every pair up to the sweep cap; the
        // packing holds rounds below 2^19 and block pairs below 4096
        int64_t nt = 0;
        for (int i = 0; i < batch; ++i) {
            if (n[i] < 2) continue;
            const Plan &P = L.plan[i];
            if (P.npairs > 4095 || (int64_t)prm.max_sweeps * P.steps >= (1 << 19)) return false;
            nt += (int64_t)prm.max_sweeps * P.steps * P.npairs;
        }
        if (nt > (1 << 26)) return false;
        L.nptask = nt;
        L.o_ptask = o; o = align256(o + sizeof(int2) * (size_t)(nt > 0 ? nt : 1));
        L.o_qhead = o; o = align256(o + sizeof(int) * 4);
        L.o_pdone = o; o = align256(o + sizeof(unsigned) * (size_t)batch);
        L.o_pfin = o; o = align256(o + sizeof(int) * (size_t)batch);
        L.o_psw = o; o = align256(o + sizeof(unsigned long long) * 3 * (size_t)batch * prm.max_sweeps);
    }
    L.meta = o;
    L.pair_off.assign(batch, 0);
    for (int i = 0; i < batch; ++i) {
        if (n[i] < 2) continue;
        L.pair_off[i] = o;
        o += pair_bytes(L.plan[i]);
    }
    L.total = o;
    return true;
}

// Validation of the batched arguments: 0 or -(argument index).
static int check_batched(int batch, const int64_t *mf, const int64_t *mg, const int64_t *n,
                         double *const *F, const int64_t *ldf, double *const *G,
                         const int64_t *ldg, double *const *Z, const int64_t *ldz,
                         double *const *s, double *const *sf, double *const *sg)
{
    if (batch < 0 || batch > 65535) return -2;
    if (batch == 0) return 0;
    if (!mf) return -3;
    if (!mg) return -4;
    if (!n) return -5;
    if (!F) return -6;
    if (!ldf) return -7;
    if (!G) return -8;
    if (!ldg) return -9;
    if (!Z) return -10;
    if (!ldz) return -11;
    if (!s) return -12;
    if (!sf) return -13;
    if (!sg) return -14;
    for (int i = 0; i < batch; ++i) {
        const int a = check_args(mf[i], mg[i], n[i], F[i], ldf[i], G[i], ldg[i], Z[i], ldz[i],
                                 s[i], sf[i], sg[i]);
        if (a) return a - 1;
    }
    return 0;
}

static int run_batched(const hz_params &prm, int batch, const int64_t *mf, const int64_t *mg,
                       const int64_t *n, double *const *F, const int64_t *ldf, double *const *G,
                       const int64_t *ldg, double *const *Z, const int64_t *ldz,
                       double *const *sigma, double *const *sigma_f, double *const *sigma_g,
                       const BLayout &L, void *work, hz_info *infos, hipStream_t st,
                       bool finish = true)
{
    int rc = HZ_OK;
    bool own = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<char> meta(L.meta, 0);
    std::vector<int> hinfo((size_t)batch * 4), hstat((size_t)batch * ST_NSLOTS);
    std::vector<unsigned long long> htot((size_t)batch * 4);
    int nact = 0, sweeps = 0;
    if (!work) {
        if (hipMallocAsync(&work, L.total, st) != hipSuccess) return HZ_EHIP;
        own = true;
    }
    {
        char *base = (char *)work;
        BPlan B;
        B.batch = batch;
        B.w = L.w;
        B.W2 = L.W2;
        B.inner_lp = L.inner_lp;
        B.isteps = L.isteps;
        B.kmax = L.kmax;
        B.max_nw = L.max_nw;
        B.probs = (BProb *)(base + L.o_probs);
        B.tasks = (int2 *)(base + L.o_tasks);
        B.ntasks = L.ntasks;
        B.task_off = L.task_off;
        B.itab = (int16_t *)(base + L.o_itab);
        B.active = (int *)(base + L.o_active);
        B.pinfo = (int *)(base + L.o_pinfo);
        B.pstatus = (int *)(base + L.o_pstatus);
        B.nactive = (int *)(base + L.o_nactive);
        B.pcnt = (unsigned long long *)(base + L.o_pcnt);
        B.ptot = (unsigned long long *)(base + L.o_ptot);
        B.ptask = (int2 *)(base + L.o_ptask);
        B.nptask = (int)L.nptask;
        B.qhead = (int *)(base + L.o_qhead);
        B.pdone = (unsigned *)(base + L.o_pdone);
        B.pfin = (int *)(base + L.o_pfin);
        B.psw = (unsigned long long *)(base + L.o_psw);
        B.total = L.total;

        // host staging of the metadata region
        char *hm = meta.data();
        BProb *hp = (BProb *)(hm + L.o_probs);
        int2 *ht = (int2 *)(hm + L.o_tasks);
        int *hact = (int *)(hm + L.o_active);
        int *hst = (int *)(hm + L.o_pstatus);
        {
            std::vector<int16_t> it;
            build_ordering<int16_t>(inner_table_kind(prm.inner_ordering), L.W2, it);
            memcpy(hm + L.o_itab, it.data(), it.size() * sizeof(int16_t));
            for (size_t t = 0; t < L.otab_nblk.size(); ++t) {
                std::vector<int> ot;
                build_ordering<int>(prm.ordering, L.otab_nblk[t], ot);
                memcpy(hm + L.otab_off[t], ot.data(), ot.size() * sizeof(int));
            }
        }
        for (int i = 0; i < batch; ++i) {
            hst[(size_t)i * ST_NSLOTS + ST_FAILPAIR] = INT_MAX;
            BProb &q = hp[i];
            memset(&q, 0, sizeof(q));
            q.F = F[i];
            q.G = G[i];
            q.U = F[i];
            q.V = G[i];
            q.Zo = Z[i];
            q.sigma = sigma[i];
            q.sigma_f = sigma_f[i];
            q.sigma_g = sigma_g[i];
            q.mf = mf[i];
            q.mg = mg[i];
            q.n = n[i];
            q.ldf = ldf[i];
            q.ldg = ldg[i];
            q.ldz = ldz[i];
            if (n[i] < 2) continue;
            const Plan &P = L.plan[i];
            hact[i] = 1;
            q.mfw = P.mfw;
            q.mgw = P.mgw;
            q.nzw = P.nzw;
            q.nw = P.nw;
            q.nblk = P.nblk;
            q.npairs = P.npairs;
            q.steps = P.steps;
            q.tol = (prm.tol > 0.0) ? prm.tol : sqrt((double)n[i]) * DBL_EPSILON;
            for (size_t t = 0; t < L.otab_nblk.size(); ++t)
                if (L.otab_nblk[t] == P.nblk) q.otab = (const int *)(base + L.otab_off[t]);
            size_t o = L.pair_off[i];
            q.Fw = (double *)(base + o); o = align256(o + 8 * (size_t)P.mfw * P.nw);
            q.Gw = (double *)(base + o); o = align256(o + 8 * (size_t)P.mgw * P.nw);
            q.Zw = (double *)(base + o); o = align256(o + 8 * (size_t)P.nzw * P.nw);
            q.gram = (double *)(base + o); o = align256(o + 8 * (size_t)P.npairs * 2 * P.W2 * P.W2);
            q.Zt = (double *)(base + o); o = align256(o + 8 * (size_t)P.npairs * P.W2 * P.W2);
            q.sf = (double *)(base + o);
            q.sg = q.sf + P.nw;
            q.sig = q.sg + P.nw;
            o = align256(o + 3 * 8 * (size_t)P.nw);
            q.rank = (int *)(base + o);
            q.border = q.rank + P.nw;
        }
        for (int k = 0; k < L.kmax; ++k) {
            int c = L.task_off[k];
            for (int i : L.order) {
                if (n[i] < 2 || k >= L.plan[i].steps) continue;
                for (int l = 0; l < L.plan[i].npairs; ++l) ht[c++] = make_int2(i, l);
            }
        }
        if (L.persistent) {
            // rounds r = sweep * steps + step of every pair, round by round,
            // largest pairs first within a round
            int2 *pt = (int2 *)(hm + L.o_ptask);
            int64_t c = 0, rmax = 0;
            for (int i = 0; i < batch; ++i)
                if (n[i] >= 2) rmax = std::max<int64_t>(rmax, (int64_t)prm.max_sweeps * L.plan[i].steps);
            for (int64_t r = 0; r < rmax; ++r)
                for (int i : L.order) {
                    if (n[i] < 2 || r >= (int64_t)prm.max_sweeps * L.plan[i].steps) continue;
                    for (int l = 0; l < L.plan[i].npairs; ++l)
                        pt[c++] = make_int2(i, (int)((r << 12) | l));
                }
        }
        HZ_CHECK(hipMemcpyAsync(base, hm, L.meta, hipMemcpyHostToDevice, st));
        for (int i = 0; i < batch && finish; ++i) {
            if (n[i] != 1) continue;
            launch_n1_real(mf[i], mg[i], F[i], G[i], Z[i], sigma[i], sigma_f[i], sigma_g[i],
                           B.pstatus + (size_t)i * ST_NSLOTS, st);
        }
        launchb_prescale(B, st);
        HZ_CHECK(hipGetLastError());

        const bool use_graph = !g_prof.on;
        if (L.persistent && L.kmax > 0) {
            // one launch for all sweeps (captured and replayed once, like a
            // sweep of the per-step schedule), then the counter totals
            if (use_graph) {
                hipStream_t cs = capture_stream();
                if (!cs) { rc = HZ_EHIP; goto done; }
                HZ_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                const hipError_t le = launchb_persistent(B, prm, cs);
                hipGraph_t g = nullptr;
                const hipError_t ce = hipStreamEndCapture(cs, &g);
                graph = g;
                HZ_CHECK(le);
                HZ_CHECK(ce);
                HZ_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
                HZ_CHECK(hipGraphLaunch(exec, st));
            } else {
                prof_mark(K_OTHER, true, st);
                HZ_CHECK(launchb_persistent(B, prm, st));
                prof_mark(K_OTHER, false, st);
            }
            sweeps = prm.max_sweeps;
        }
        if (use_graph && L.kmax > 0 && !L.persistent) {
            hipStream_t cs = capture_stream();
            if (!cs) { rc = HZ_EHIP; goto done; }
            HZ_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            launchb_sweep(B, prm, cs);
            HZ_CHECK(hipStreamEndCapture(cs, &graph));
            HZ_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        }
        for (int sw = 0; sw < prm.max_sweeps && L.kmax > 0 && !L.persistent; ++sw) {
            if (use_graph) HZ_CHECK(hipGraphLaunch(exec, st));
            else launchb_sweep(B, prm, st);
            HZ_CHECK(hipGetLastError());
            HZ_CHECK(hipMemcpyAsync(&nact, B.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
            HZ_CHECK(hipStreamSynchronize(st));
            prof_flush();
            ++sweeps;
            if (nact == 0) break;
        }
        if (finish) launchb_finish(B, st);
        HZ_CHECK(hipGetLastError());
        HZ_CHECK(hipMemcpyAsync(hinfo.data(), B.pinfo, hinfo.size() * sizeof(int),
                                hipMemcpyDeviceToHost, st));
        HZ_CHECK(hipMemcpyAsync(hstat.data(), B.pstatus, hstat.size() * sizeof(int),
                                hipMemcpyDeviceToHost, st));
        HZ_CHECK(hipMemcpyAsync(htot.data(), B.ptot, htot.size() * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, st));
        HZ_CHECK(hipStreamSynchronize(st));
        int worst = 0;   // 3 nonfinite, 2 chol, 1 noconv
        for (int i = 0; i < batch; ++i) {
            const int fl = hstat[(size_t)i * ST_NSLOTS + ST_FLAGS];
            const bool conv = (n[i] == 1) || hinfo[(size_t)i * 4 + 1];
            int prc = HZ_OK, sev = 0;
            if (fl & FLAG_STALL) { prc = HZ_EHIP; sev = 4; }
            else if (fl & FLAG_NONFINITE) { prc = HZ_ENONFINITE; sev = 3; }
            else if (fl & FLAG_CHOL) { prc = HZ_ECHOL; sev = 2; }
            else if (!conv) { prc = HZ_ENOCONV; sev = 1; }
            worst = sev > worst ? sev : worst;
            if (infos) {
                hz_info &f = infos[i];
                memset(&f, 0, sizeof(f));
                f.sweeps = hinfo[(size_t)i * 4];
                f.converged = conv ? 1 : 0;
                f.w = (n[i] == 1) ? 1 : L.w;
                f.failed_pair = (fl & FLAG_CHOL) ? hstat[(size_t)i * ST_NSLOTS + ST_FAILPAIR] : -1;
                f.rot_total = htot[(size_t)i * 4];
                f.rot_big = htot[(size_t)i * 4 + 1];
                f.inner_sweeps = htot[(size_t)i * 4 + 2];
                f.status = prc;
            }
        }
        rc = worst == 4 ? HZ_EHIP : worst == 3 ? HZ_ENONFINITE : worst == 2 ? HZ_ECHOL
           : worst == 1 ? HZ_ENOCONV : HZ_OK;
    }
done:
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (own) (void)hipFreeAsync(work, st);
    (void)sweeps;
    return rc;
}

}  // namespace hz

extern "C" {

size_t hz_dgsvd_batched_work_size(const hz_params *p, int batch, const int64_t *m_f,
                                  const int64_t *m_g, const int64_t *n)
{
    hz_params prm;
    if (p) prm = *p; else hz_default_params(&prm);
    if (!params_ok(prm) || prm.qr_shorten || prm.pivot_qr || batch < 0 || batch > 65535) return 0;
    if (batch == 0) return 256;
    if (!m_f || !m_g || !n) return 0;
    for (int i = 0; i < batch; ++i)
        if (n[i] < 1 || m_f[i] < n[i] || m_g[i] < n[i] || n[i] > (int64_t)INT_MAX / 2) return 0;
    BLayout L;
    if (!plan_batched(prm, batch, m_f, m_g, n, L)) return 0;
    return L.total;
}

int hz_dgsvd_batched(const hz_params *p, int batch, const int64_t *m_f, const int64_t *m_g,
                     const int64_t *n, double *const *F, const int64_t *ldf,
                     double *const *G, const int64_t *ldg, double *const *Z,
                     const int64_t *ldz, double *const *sigma, double *const *sigma_f,
                     double *const *sigma_g, void *work, size_t work_bytes, hz_info *infos,
                     void *stream)
{
    hz_params prm;
    if (p) prm = *p; else hz_default_params(&prm);
    if (!params_ok(prm) || prm.qr_shorten || prm.pivot_qr || prm.schedule == HZ_SCHED_DATAFLOW)
        return -1;
    const int a = check_batched(batch, m_f, m_g, n, F, ldf, G, ldg, Z, ldz, sigma, sigma_f,
                                sigma_g);
    if (a) return a;
    if (batch == 0) return HZ_OK;
    if (work && ((uintptr_t)work & 255)) return -15;
    BLayout L;
    if (!plan_batched(prm, batch, m_f, m_g, n, L)) return -5;
    if (work && work_bytes < L.total) return -16;
    return run_batched(prm, batch, m_f, m_g, n, F, ldf, G, ldg, Z, ldz, sigma, sigma_f, sigma_g,
                       L, work, infos, (hipStream_t)stream);
}

}  // extern "C"

// ------------------------------------------------------------ autotuner
// Chooses launch parameters by timing complete solves without the final
// extraction (prescale and sweeps to convergence read F and G and write
// only the workspace, so the caller's data are left as they were).  The
// choice is appended to a plain-text cache file keyed by the problem
// sizes, the fixed parameters and the device, so later runs -- and with
// them the results, which depend on the block width and the reduction
// splits -- are reproducible without timing again.
namespace hz {

static uint64_t fnv(uint64_t h, const void *p, size_t n)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

static uint64_t tune_key(const char *kind, const hz_params &p, int batch, const int64_t *mf,
                         const int64_t *mg, const int64_t *n)
{
    uint64_t h = 14695981039346656037ull;
    h = fnv(h, kind, strlen(kind));
    const int fixed[] = {p.variant, p.ordering, p.inner_ordering, p.w, p.max_sweeps, p.sort,
                         p.inner_lanes, p.gram_splits, p.update_rows};
    h = fnv(h, fixed, sizeof(fixed));
    h = fnv(h, &p.tol, sizeof(p.tol));
    if (p.qr_shorten) h = fnv(h, "qr_shorten", 10);   // keys without it are unchanged
    if (p.pivot_qr) h = fnv(h, "pivot_qr", 8);
    h = fnv(h, &batch, sizeof(batch));
    h = fnv(h, mf, sizeof(int64_t) * batch);
    h = fnv(h, mg, sizeof(int64_t) * batch);
    h = fnv(h, n, sizeof(int64_t) * batch);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        h = fnv(h, prop.gcnArchName, strlen(prop.gcnArchName));
        h = fnv(h, &prop.multiProcessorCount, sizeof(int));
    }
    const char *ver = hz_version();
    return fnv(h, ver, strlen(ver));
}

static std::mutex g_tune_mu;

// Cache line: "<key hex> w inner_max_sweeps inner_lanes gram_splits update_rows ms
// ordering inner_ordering" (a line without the orderings leaves them as given).
static bool cache_lookup(const char *path, uint64_t key, hz_params &p, double &ms)
{
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool hit = false;
    while (fgets(line, sizeof(line), f)) {
        unsigned long long k;
        int w, ims, lp, gs, ur, ord = 0, iord = 0;
        double t;
        const int got = sscanf(line, "%llx %d %d %d %d %d %lf %d %d", &k, &w, &ims, &lp, &gs,
                               &ur, &t, &ord, &iord);
        if (got >= 7 && k == key) {
            p.w = w;
            p.inner_max_sweeps = ims;
            p.inner_lanes = lp;
            p.gram_splits = gs;
            p.update_rows = ur;
            if (got >= 8 && ord) p.ordering = ord;
            if (got >= 9 && iord) p.inner_ordering = iord;
            ms = t;
            hit = true;     // the last matching line wins
        }
    }
    fclose(f);
    return hit && params_ok(p);
}

static void cache_store(const char *path, uint64_t key, const hz_params &p, double ms)
{
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%016llx %d %d %d %d %d %.6f %d %d\n", (unsigned long long)key, p.w,
            p.inner_max_sweeps, p.inner_lanes, p.gram_splits, p.update_rows, ms, p.ordering,
            p.inner_ordering);
    fclose(f);
}

static double now_ms()
{
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Coordinate search: each tunable that the caller left at 0 is varied in
// turn with the others held at the best values so far; a candidate counts
// only if it converges.  Returns the best time (ms) or a negative status.
template <typename Solve>
static double coordinate_search(hz_params &best, const std::vector<std::vector<int>> &axes,
                                const std::vector<int *> &fields, Solve solve)
{
    double best_ms = -1.0;
    {
        const double t = solve(best);
        if (t >= 0.0) best_ms = t;
    }
    // passes over the axes until one changes nothing (at most two): the best
    // value on an axis can depend on the ones chosen after it
    for (int pass = 0; pass < 2; ++pass) {
        bool changed = false;
        for (size_t a = 0; a < axes.size(); ++a) {
            const int keep = *fields[a];
            int arg = keep;
            for (int v : axes[a]) {
                if (v == keep) continue;
                hz_params c = best;
                // the field pointers address `best`; write into the copy instead
                *(int *)((char *)&c + ((char *)fields[a] - (char *)&best)) = v;
                if (!params_ok(c)) continue;
                const double t = solve(c);
                if (t >= 0.0 && (best_ms < 0.0 || t < best_ms)) {
                    best_ms = t;
                    arg = v;
                }
            }
            if (arg != keep) changed = true;
            *fields[a] = arg;
        }
        if (!changed) break;
    }
    return best_ms;
}

}  // namespace hz

extern "C" {

int hz_dgsvd_tune(const hz_params *p, int64_t m_f, int64_t m_g, int64_t n, const double *F,
                  int64_t ldf, const double *G, int64_t ldg, const char *cache_path,
                  hz_params *best, double *best_ms, void *stream)
{
    hz_params base;
    if (p) base = *p; else hz_default_params(&base);
    // inner_ordering 0 asks the tuner to choose the ordering inside a block pair
    const bool tune_iord = (base.inner_ordering == 0);
    if (tune_iord) base.inner_ordering = HZ_ORD_RR;
    if (!params_ok(base) || (base.qr_shorten && n > 1 && !shorten_cpt(n))) return -1;
    const double dummy = 0.0;
    const int a = check_args(m_f, m_g, n, F, ldf, G, ldg, &dummy, n, &dummy, &dummy, &dummy);
    if (a) return a;
    if (!best) return -10;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t key = tune_key(tune_iord ? "dgsvd_iord3" : "dgsvd", base, 1, &m_f, &m_g, &n);
    hz_params cur = base;
    double ms = 0.0;
    if (cache_lookup(cache_path, key, cur, ms)) {
        *best = cur;
        if (best_ms) *best_ms = ms;
        return HZ_OK;
    }
    if (n < 2) {
        *best = base;
        if (best_ms) *best_ms = 0.0;
        return HZ_OK;
    }
    int herr = 0;
    // With qr_shorten the pair is shortened once, untimed, and the candidates
    // are timed on the square pair (F'', G'') the sweeps then run on.
    const double *Ft = F, *Gt = G;
    int64_t mft = m_f, mgt = m_g, ldft = ldf, ldgt = ldg;
    void *swork = nullptr;
    if (base.qr_shorten) {
        SPlan S;
        int hs[ST_NSLOTS] = {0, 0, 0, 0};
        if (!make_splan(m_f, m_g, n, 0, S, 0)) return -4;
        if (hipMallocAsync(&swork, S.total, st) != hipSuccess) return HZ_EHIP;
        if (launch_shorten(S, swork, F, ldf, G, ldg, st) != hipSuccess ||
            hipMemcpyAsync(hs, (char *)swork + S.o_status, sizeof(hs), hipMemcpyDeviceToHost,
                           st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            (void)hipFreeAsync(swork, st);
            return HZ_EHIP;
        }
        if (hs[ST_FLAGS] & (FLAG_NONFINITE | FLAG_CHOL)) {
            (void)hipFreeAsync(swork, st);
            return (hs[ST_FLAGS] & FLAG_NONFINITE) ? HZ_ENONFINITE : HZ_ECHOL;
        }
        Ft = (const double *)((char *)swork + S.o_f2);
        Gt = (const double *)((char *)swork + S.o_g2);
        mft = mgt = n;
        ldft = ldgt = S.ldn;
    }
    auto solve = [&](const hz_params &c) -> double {
        Plan P;
        if (!make_plan(c, mft, mgt, n, 0, P)) return -1.0;
        void *work = nullptr;
        if (hipMallocAsync(&work, P.total, st) != hipSuccess) { herr = 1; return -1.0; }
        hz_info info;
        memset(&info, 0, sizeof(info));
        (void)hipStreamSynchronize(st);
        const double t0 = now_ms();
        const int rc = run_solve(c, P, work, P.total, &info, st, KIND_REAL, Ft, ldft, Gt, ldgt,
                                 nullptr, nullptr, nullptr, n, nullptr, nullptr, nullptr, false);
        const double t = now_ms() - t0;
        (void)hipFreeAsync(work, st);
        if (rc == HZ_EHIP) herr = 1;
        return rc == HZ_OK ? t : -1.0;
    };
    if (!base.w) cur.w = default_w(n, 0);
    if (!base.gram_splits) cur.gram_splits = 8;
    if (!base.update_rows) cur.update_rows = 48;
    if (!base.inner_lanes) cur.inner_lanes = 0;
    std::vector<std::vector<int>> axes;
    std::vector<int *> fields;
    if (tune_iord) {
        axes.push_back({HZ_ORD_RR, HZ_ORD_MM, HZ_ORD_RING});
        fields.push_back(&cur.inner_ordering);
    }
    axes.push_back({1, base.inner_max_sweeps});
    fields.push_back(&cur.inner_max_sweeps);
    if (!base.w) { axes.push_back({8, 16, 32}); fields.push_back(&cur.w); }
    if (!base.gram_splits) { axes.push_back({4, 8, 16}); fields.push_back(&cur.gram_splits); }
    if (!base.update_rows) { axes.push_back({16, 32, 48, 64, 80, 128}); fields.push_back(&cur.update_rows); }
    if (!base.inner_lanes) { axes.push_back({4, 8, 16}); fields.push_back(&cur.inner_lanes); }
    ms = coordinate_search(cur, axes, fields, solve);
    if (swork) (void)hipFreeAsync(swork, st);
    if (herr) return HZ_EHIP;
    if (ms < 0.0) return HZ_ENOCONV;
    *best = cur;
    if (best_ms) *best_ms = ms;
    cache_store(cache_path, key, cur, ms);
    return HZ_OK;
}

int hz_dgsvd_batched_tune(const hz_params *p, int batch, const int64_t *m_f, const int64_t *m_g,
                          const int64_t *n, const double *const *F, const int64_t *ldf,
                          const double *const *G, const int64_t *ldg, const char *cache_path,
                          hz_params *best, double *best_ms, void *stream)
{
    hz_params base;
    if (p) base = *p; else hz_default_params(&base);
    // ordering 0 asks the tuner to choose between modified modulus and round robin,
    // inner_ordering 0 the ordering inside a block pair
    const bool tune_ord = (base.ordering == 0);
    if (tune_ord) base.ordering = HZ_ORD_MM;
    const bool tune_iord = (base.inner_ordering == 0);
    if (tune_iord) base.inner_ordering = HZ_ORD_RR;
    if (!params_ok(base) || base.qr_shorten || base.pivot_qr) return -1;
    if (batch < 1 || batch > 65535) return -2;
    if (!m_f) return -3;
    if (!m_g) return -4;
    if (!n) return -5;
    if (!F) return -6;
    if (!ldf) return -7;
    if (!G) return -8;
    if (!ldg) return -9;
    const double dummy = 0.0;
    for (int i = 0; i < batch; ++i) {
        const int a = check_args(m_f[i], m_g[i], n[i], F[i], ldf[i], G[i], ldg[i], &dummy, n[i],
                                 &dummy, &dummy, &dummy);
        if (a) return a - 1;
    }
    if (!best) return -11;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t key = tune_key(tune_iord ? (tune_ord ? "dgsvd_batched_ord_iord3_persist"
                                                        : "dgsvd_batched_iord3_persist")
                                            : (tune_ord ? "dgsvd_batched_ord_persist"
                                                        : "dgsvd_batched_persist"),
                                  base, batch, m_f, m_g, n);
    hz_params cur = base;
    double ms = 0.0;
    if (cache_lookup(cache_path, key, cur, ms)) {
        *best = cur;
        if (best_ms) *best_ms = ms;
        return HZ_OK;
    }
    std::vector<double *> nul((size_t)batch, nullptr);
    std::vector<int64_t> ldz(n, n + batch);
    int herr = 0;
    auto solve = [&](const hz_params &c) -> double {
        BLayout L;
        if (!plan_batched(c, batch, m_f, m_g, n, L)) return -1.0;
        void *work = nullptr;
        if (hipMallocAsync(&work, L.total, st) != hipSuccess) { herr = 1; return -1.0; }
        std::vector<hz_info> infos((size_t)batch);
        (void)hipStreamSynchronize(st);
        const double t0 = now_ms();
        const int rc = run_batched(c, batch, m_f, m_g, n, (double *const *)F, ldf,
                                   (double *const *)G, ldg, nul.data(), ldz.data(), nul.data(),
                                   nul.data(), nul.data(), L, work, infos.data(), st, false);
        const double t = now_ms() - t0;
        (void)hipFreeAsync(work, st);
        if (rc == HZ_EHIP) herr = 1;
        return rc == HZ_OK ? t : -1.0;
    };
    int64_t nmax = 1;
    for (int i = 0; i < batch; ++i) nmax = n[i] > nmax ? n[i] : nmax;
    if (!base.w) cur.w = nmax <= 32 ? 8 : 16;
    std::vector<std::vector<int>> axes;
    std::vector<int *> fields;
    axes.push_back({1, base.inner_max_sweeps});
    fields.push_back(&cur.inner_max_sweeps);
    if (!base.w) { axes.push_back({8, 16, 32}); fields.push_back(&cur.w); }
    if (!base.inner_lanes) { axes.push_back({4, 8, 16}); fields.push_back(&cur.inner_lanes); }
    if (tune_ord) { axes.push_back({HZ_ORD_MM, HZ_ORD_RR}); fields.push_back(&cur.ordering); }
    if (tune_iord) {
        axes.push_back({HZ_ORD_RR, HZ_ORD_MM, HZ_ORD_RING});
        fields.push_back(&cur.inner_ordering);
    }
    ms = coordinate_search(cur, axes, fields, solve);
    if (herr) return HZ_EHIP;
    if (ms < 0.0) return HZ_ENOCONV;
    *best = cur;
    if (best_ms) *best_ms = ms;
    cache_store(cache_path, key, cur, ms);
    return HZ_OK;
}

}  // extern "C"
