// lexbfs.hip -- kernels and C ABI of the gfx950 chordality library.
//
// Path per graph (Lupinska, "A Parallel Algorithm to Test Chordality of
// Graphs"): LexBFS order (Section 6.1) -> parent-based perfect-elimination
// sweep (Section 6.2) -> witness and chordless-cycle certificate.
// The device-side state machine of LexBFS is described in lexbfs_device.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lexbfs.h"
#include "lexbfs_device.h"

using namespace lxd;

namespace {

constexpr int kAbiVersion = 1;
constexpr size_t kAlign = 256;
constexpr int kSweepThreads = 256;
constexpr int kFinishThreads = 256;
constexpr int kBatchThreads = 256;
// Internal plan flag (never accepted from callers): LexBFS order, rank and
// parent only, without the test's verdict, witness and certificate.
constexpr uint32_t kFlagOrderOnly = 0x80000000u;

// Description of the last failure on this thread (lexbfs_last_error).
thread_local char t_last_error[256] = "";

int fail_hip(hipError_t e, const char *where)
{
    snprintf(t_last_error, sizeof t_last_error, "%s: %s", where, hipGetErrorString(e));
    return LEXBFS_EHIP;
}

int fail_code(int code, const char *what)
{
    snprintf(t_last_error, sizeof t_last_error, "%s", what);
    return code;
}

#define LX_CHECK_LAUNCH(where)                                  \
    do {                                                        \
        const hipError_t e_ = hipGetLastError();                \
        if (e_ != hipSuccess) return fail_hip(e_, where);       \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel timing: while enabled, every launch is bracketed by a pair of HIP
// events on its stream (events are created when timing is switched on, so
// the launch path itself creates nothing).
// ---------------------------------------------------------------------------
constexpr int kKinds = LEXBFS_KERNEL_KINDS;
constexpr int kProfPairs = 8192;

struct Profiler {
    std::mutex mu;
    bool on = false;
    bool created = false;
    hipEvent_t ev[2 * kProfPairs];
    int kind[kProfPairs];
    int used = 0;
    int dropped = 0;
};
Profiler g_prof;

struct ProfScope {
    int slot = -1;
    hipStream_t s;
    ProfScope(int k, hipStream_t st) : s(st)
    {
        if (!g_prof.on) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!g_prof.on) return;
        if (g_prof.used >= kProfPairs) {
            ++g_prof.dropped;
            return;
        }
        slot = g_prof.used++;
        g_prof.kind[slot] = k;
        (void)hipEventRecord(g_prof.ev[2 * slot], s);
    }
    ~ProfScope()
    {
        if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot + 1], s);
    }
};

// Everything a kernel needs about one graph (device copy for batches).
struct GDesc {
    int32_t n;
    int32_t wn;        // ceil(n / 64)
    int64_t W;         // row stride in words
    const int32_t *rp;
    const int32_t *ci;
    const uint64_t *bits;
    int32_t *order;
    int32_t *rank;
    int32_t *parent;
    int32_t *cycle;
    int32_t *level;    // certificate scratch [n]
    int32_t *q0;       // [n]
    int32_t *q1;       // [n]
    int32_t *lnbuf;    // [n]
    uint32_t *failkey; // [1]
    uint32_t *gtab;    // [2n] class tables in global memory (large n), else null
    lexbfs_result_t *res;
    int64_t nnz;       // CSR entries (read only by the input check)
};

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t cas_agent(int32_t *p, int32_t expected, int32_t desired)
{
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return expected;
}

__device__ __forceinline__ bool test_bit(const uint64_t *row, int u) { return (row[u >> 6] >> (u & 63)) & 1ull; }

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// LDS of the certificate search of one team: a few shared integers, then
// three bitsets of wn words.
//   sc[0] frontier size, sc[1] predecessor, sc[2 .. 2+NW) reduction words,
//   sc[2+NW .. 2+2NW) per-wave counts
struct FinishLds {
    int32_t *sc;
    uint64_t *amask, *vis, *nxt;
};

__host__ __device__ inline size_t finish_head_bytes(int nwaves) { return align_up(4 * (2 + 2 * (size_t)nwaves), 16); }

__host__ __device__ inline size_t finish_lds_bytes(int wn, int nwaves)
{
    return finish_head_bytes(nwaves) + 3 * 8 * (size_t)(wn > 0 ? wn : 1);
}

__device__ __forceinline__ FinishLds carve_finish(void *base, int wn, int nwaves)
{
    FinishLds F;
    F.sc = (int32_t *)base;
    F.amask = (uint64_t *)((char *)base + finish_head_bytes(nwaves));
    F.vis = F.amask + (wn > 0 ? wn : 1);
    F.nxt = F.vis + (wn > 0 ? wn : 1);
    return F;
}

// ---------------------------------------------------------------------------
// Certificate search: layered BFS from src inside A = (V \ N[c]) + {src, dst},
// stopped after the layer that reaches dst; then back from dst, taking the
// smallest-id neighbour of the previous layer each time. Writes
// path[0] = src .. path[d] = dst and returns d + 1, or 0 if unreachable.
// Every lane of the team calls it with the same arguments.
//
// Layers are bitsets: a layer's successor is the OR of its vertices' rows,
// masked by A and by the visited set. The team's waves split the frontier
// (four rows in flight per wave), lanes split the words of a row, and the
// partial layers meet in LDS through atomic ORs. Each newly reached vertex
// gets level[u] = stamp << 16 | depth; stamps keep successive searches of
// one call apart without clearing level[] between them.
// ---------------------------------------------------------------------------
template <class Team>
__device__ int bfs_path(const Team &tm, const GDesc &g, int c, int src, int dst, int32_t *path, const FinishLds &F,
                        uint32_t stamp)
{
    constexpr int T = Team::kSize;
    constexpr int NW = Team::kWaves;
    LX_GLOBAL const uint64_t *bits = as_global(g.bits);
    LX_GLOBAL const int32_t *rp = as_global(g.rp);
    LX_GLOBAL const int32_t *ci = as_global(g.ci);
    LX_GLOBAL int32_t *level = as_global(g.level);
    LX_GLOBAL int32_t *q = as_global(g.q0);
    uint64_t *amask = F.amask, *vis = F.vis, *nxt = F.nxt;
    int32_t *s_nf = F.sc, *s_pred = F.sc + 1;
    const int tid = tm.tid, lane = tid & 63, wave = tid >> 6;
    const int wn = g.wn;
    const uint64_t tail = (g.n & 63) ? ((1ull << (g.n & 63)) - 1ull) : ~0ull;
    LX_GLOBAL const uint64_t *rowc = bits + (int64_t)c * g.W;
    for (int w = tid; w < wn; w += T) {
        uint64_t a = ~rowc[w];
        if (w == wn - 1) a &= tail;
        if (w == (c >> 6)) a &= ~(1ull << (c & 63));
        if (w == (src >> 6)) a |= 1ull << (src & 63);
        if (w == (dst >> 6)) a |= 1ull << (dst & 63);
        amask[w] = a;
        vis[w] = w == (src >> 6) ? (1ull << (src & 63)) : 0ull;
        nxt[w] = vis[w];
    }
    if (tid == 0) level[src] = (int32_t)(stamp << 16);
    tm.sync();
    int d = 0;
    for (;;) {
        // The frontier (nxt) as a list of ids in q.
        if (tid == 0) *s_nf = 0;
        tm.sync();
        for (int w = tid; w < wn; w += T) {
            uint64_t f = nxt[w];
            if (!f) continue;
            int p = atomicAdd(s_nf, __popcll(f));
            for (; f; f &= f - 1) q[p++] = (w << 6) + ctz64(f);
        }
        tm.sync_mem();
        const int nf = *s_nf;
        if (nf == 0) return 0;  // dst unreachable
        for (int w = tid; w < wn; w += T) nxt[w] = 0ull;
        tm.sync();
        // Next layer: OR of the frontier's rows, masked.
        for (int f0 = wave; f0 < nf; f0 += 4 * NW) {
            const int u0 = q[f0];
            const int u1 = f0 + NW < nf ? q[f0 + NW] : -1;
            const int u2 = f0 + 2 * NW < nf ? q[f0 + 2 * NW] : -1;
            const int u3 = f0 + 3 * NW < nf ? q[f0 + 3 * NW] : -1;
            for (int w = lane; w < wn; w += kWave) {
                uint64_t acc = bits[(int64_t)u0 * g.W + w];
                if (u1 >= 0) acc |= bits[(int64_t)u1 * g.W + w];
                if (u2 >= 0) acc |= bits[(int64_t)u2 * g.W + w];
                if (u3 >= 0) acc |= bits[(int64_t)u3 * g.W + w];
                acc &= amask[w] & ~vis[w];
                if (acc) atomicOr((unsigned long long *)&nxt[w], acc);
            }
        }
        tm.sync();
        ++d;
        bool found = false;
        for (int w = tid; w < wn; w += T) {
            const uint64_t nw = nxt[w];
            if (!nw) continue;
            vis[w] |= nw;
            for (uint64_t m = nw; m; m &= m - 1) {
                const int u = (w << 6) + ctz64(m);
                level[u] = (int32_t)((stamp << 16) | (uint32_t)d);
                found |= u == dst;
            }
        }
        if (tm.any_all(found)) break;
    }
    tm.sync_mem();  // levels visible to every lane
    if (tid == 0) path[d] = dst;
    int y = dst;
    for (int l = d; l >= 1; --l) {
        if (tid == 0) *s_pred = INT_MAX;
        tm.sync();
        const int32_t want = (int32_t)((stamp << 16) | (uint32_t)(l - 1));
        const int e = rp[y + 1];
        for (int j = rp[y] + tid; j < e; j += T) {  // rows ascend: first hit per lane is its minimum
            const int u = ci[j];
            if ((unsigned)u < (unsigned)g.n && level[u] == want) {
                atomicMin(s_pred, u);
                break;
            }
        }
        tm.sync();
        y = *s_pred;
        tm.sync();
        if (y == INT_MAX) return 0;  // only with a non-symmetric CSR
        if (tid == 0) path[l - 1] = y;
    }
    return d + 1;
}

__device__ __forceinline__ void write_result(lexbfs_result_t *out, int chordal, int v, int p, int z, int len, int fb)
{
    lexbfs_result_t r;
    r.chordal = chordal;
    r.witness_v = v;
    r.witness_p = p;
    r.witness_z = z;
    r.cycle_len = len;
    r.fallback = fb;
    r.reserved[0] = r.reserved[1] = 0;
    *out = r;
}

// Witness and certificate for one graph; every lane of the team calls it
// after the failing rank (failkey), order, rank and parent are visible.
template <class Team>
__device__ void finish_graph(const Team &tm, const GDesc &g, uint32_t flags, const FinishLds &F)
{
    constexpr int T = Team::kSize;
    constexpr int NW = Team::kWaves;
    uint32_t *s_red = (uint32_t *)(F.sc + 2);
    int32_t *s_wcnt = F.sc + 2 + NW;
    uint32_t stamp = 0;
    const int tid = tm.tid;
    const uint32_t fk = g.n > 0 ? g_load(g.failkey) : kNoFail;
    if (fk == kNoFail) {
        if (tid == 0) write_result(g.res, 1, -1, -1, -1, 0, 0);
        return;
    }
    const int v = g.order[fk];
    const int x = g.parent[v];
    const int rx = g.rank[x];
    const uint64_t *rowv = g.bits + (int64_t)v * g.W;
    const uint64_t *rowx = g.bits + (int64_t)x * g.W;
    const uint64_t tail = (g.n & 63) ? ((1ull << (g.n & 63)) - 1ull) : ~0ull;
    uint32_t best = UINT_MAX;
    for (int w = tid; w < g.wn; w += T) {
        for (uint64_t X = rowv[w] & ~rowx[w] & (w == g.wn - 1 ? tail : ~0ull); X; X &= X - 1) {
            const int z = (w << 6) + ctz64(X);
            const uint32_t rz = (uint32_t)g.rank[z];
            if ((int)rz < rx) best = min(best, rz);
        }
    }
    best = tm.min_all(best, s_red);
    if (best >= (uint32_t)g.n) {
        // Only reachable when the input breaks its contract (e.g. an
        // asymmetric bitset): report the failure without a certificate.
        if (tid == 0) write_result(g.res, 0, v, x, -1, 0, 0);
        return;
    }
    const int z = g.order[best];

    for (int u = tid; u < g.n; u += T) g.level[u] = 0;  // stamp 0: never matches a search
    tm.sync_mem();
    int len = 0, fb = 0;
    if (!(flags & LEXBFS_FLAG_FORCE_FALLBACK)) {
        len = bfs_path(tm, g, v, x, z, g.cycle + 1, F, ++stamp);
        if (len > 0) {
            if (tid == 0) g.cycle[0] = v;
            len += 1;
        }
    }
    if (len == 0) {
        fb = 1;
        // Fallback: vertices by ascending rank, pairs of non-adjacent earlier
        // neighbours by ascending (rank a, rank b).
        const int wave = tid >> 6, lane = tid & 63;
        for (int rv = 0; rv < g.n && len == 0; ++rv) {
            const int v2 = g.order[rv];
            const uint64_t *row2 = g.bits + (int64_t)v2 * g.W;
            int k = 0;
            for (int base = 0; base < rv; base += T) {  // LN(v2) in rank order
                const int r = base + tid;
                const bool in = r < rv && test_bit(row2, g.order[r]);
                const uint64_t bal = __ballot(in);
                if (lane == 0) s_wcnt[wave] = __popcll(bal);
                tm.sync();
                int off = k, total = 0;
                for (int w = 0; w < NW; ++w) {
                    if (w < wave) off += s_wcnt[w];
                    total += s_wcnt[w];
                }
                if (in) g_store_i(&g.lnbuf[off + __popcll(bal & lanemask_lt(lane))], g.order[r]);
                k += total;
                tm.sync();
            }
            tm.sync_mem();
            for (int ia = 0; ia < k && len == 0; ++ia) {
                const int a = g_load_i(&g.lnbuf[ia]);
                const uint64_t *rowa = g.bits + (int64_t)a * g.W;
                for (int ib = ia + 1; ib < k && len == 0; ++ib) {
                    const int b = g_load_i(&g.lnbuf[ib]);
                    if (test_bit(rowa, b)) continue;
                    if (stamp == 0xFFFFu) {  // stamps exhausted: clear the levels, start over
                        for (int u = tid; u < g.n; u += T) g.level[u] = 0;
                        tm.sync_mem();
                        stamp = 0;
                    }
                    len = bfs_path(tm, g, v2, b, a, g.cycle + 1, F, ++stamp);
                    if (len > 0) {
                        if (tid == 0) g.cycle[0] = v2;
                        len += 1;
                    }
                }
            }
        }
    }
    if (tid == 0) write_result(g.res, 0, v, x, z, len, fb);
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// State placement of a single-graph LexBFS launch, most capable first.
enum : int { kModeLds = 1, kModeCompact = 2, kModeGlobal = 3 };

// kIlv: ties by the interleaved rank (the renamed graphs of LexBFS+ sweeps);
// never used with the compact form.
template <int T, int kMode, bool kIlv = false>
__global__ __launch_bounds__(T) void k_lexbfs_single(GDesc g)
{
    extern __shared__ uint64_t lds[];
    vgpr_headroom<T>();
    if (threadIdx.x == 0 && g.failkey) *g.failkey = kNoFail;
    if (kMode == kModeCompact) {
        BlockTeam<T, false> tm{(int)threadIdx.x};
        lexbfs_team_compact(tm, g.n, g.bits, g.W, g.order, g.rank, g.parent, carve_compact(lds, g.n, T));
    } else if (kMode == kModeGlobal) {
        LdsLayoutG L = carve_lds_g(lds, g.n, T);
        GlobalTables tab(g.gtab, g.gtab + g.n);
        BlockTeam<T, true> tm{(int)threadIdx.x};
        lexbfs_team<BlockTeam<T, true>, GlobalTables, false, kIlv>(tm, g.n, g.bits, g.W, g.rp, g.order, g.rank,
                                                                  g.parent, L.starts, L.cls, tab, L.red);
    } else {
        LdsLayout L = carve_lds(lds, g.n, T);
        BlockTeam<T, false> tm{(int)threadIdx.x};
        if constexpr (T >= 512) {
            // Graphs of 4,097 to about 20,000 vertices (positions below 2^15):
            // the recorded-member form. Smaller teams match 16 ids or fewer
            // per lane, which costs less than its extra slot read and decode.
            LdsTablesSole tab;
            tab.clast = L.tab.clast;
            tab.cnt = L.tab.cnt;
            lexbfs_team<BlockTeam<T, false>, LdsTablesSole, false, kIlv, 32>(tm, g.n, g.bits, g.W, g.rp, g.order,
                                                                             g.rank, g.parent, L.starts, L.cls, tab,
                                                                             L.red);
        } else {
            lexbfs_team<BlockTeam<T, false>, LdsTables, false, kIlv, 32>(tm, g.n, g.bits, g.W, g.rp, g.order, g.rank,
                                                                         g.parent, L.starts, L.cls, L.tab, L.red);
        }
    }
}

// Parents of a finished order (the global-table LexBFS does not write them
// during its steps): one wavefront per vertex, grid-stride.
__global__ __launch_bounds__(256) void k_parents(GDesc g)
{
    const int waves = gridDim.x * (256 / kWave);
    const int first = blockIdx.x * (256 / kWave) + (int)(threadIdx.x >> 6);
    derive_parents(g.rp, g.ci, g.order, g.rank, g.parent, g.n, first, waves);
}

// Maximum Cardinality Search order of one graph (Section 5.1); the same
// sweep and certificate kernels then test it.
template <int T>
__global__ __launch_bounds__(T) void k_mcs_single(GDesc g)
{
    extern __shared__ uint64_t lds[];
    vgpr_headroom<T>();
    if (threadIdx.x == 0 && g.failkey) *g.failkey = kNoFail;
    BlockTeam<T, false> tm{(int)threadIdx.x};
    mcs_team(tm, g.n, g.bits, g.W, g.order, g.rank, g.parent, carve_mcs(lds, g.n, T, false, nullptr));
}

__global__ __launch_bounds__(kSweepThreads) void k_sweep_single(GDesc g, int rows_per_block, int G, int lg)
{
    const int r0 = blockIdx.x * rows_per_block;
    const int r1 = min(g.n, r0 + rows_per_block);
    sweep_rows<true>(g.bits, g.W, g.wn, g.rank, g.parent, g.n, r0, r1, G, lg, g.failkey);
}

// Verdict, witness and certificate of one graph on a T-lane workgroup
// (1,024 lanes for graphs with rows over 64 words: the certificate's BFS
// scans rows word-parallel).
template <int T>
__global__ __launch_bounds__(T) void k_finish_single(GDesc g, uint32_t flags)
{
    extern __shared__ uint64_t lds[];
    vgpr_headroom<T>();
    BlockTeam<T, false> tm{(int)threadIdx.x};
    finish_graph(tm, g, flags, carve_finish(lds, g.wn, T / kWave));
}

// ---------------------------------------------------------------------------
// LexBFS with one round of launches per step (the host loop of Section 6.1:
// a fixed sequence of kernels per step, one thread per vertex, every table
// in global memory). Kept as the comparison form for the persistent kernel.
// Same class naming as the persistent kernel: a class is the position range
// [c, clast[c]] named by its start; the pivot's neighbours in c move to the
// top cnt[c] positions (Observation 6.2), so the top class is the largest
// class id and the pivot is the unnumbered vertex of largest
// (class, -id) key, kept as (class << 32 | 0xFFFFFFFF - id) in a 64-bit max.
//   count:  number the pivot, shrink its class, count neighbours per class
//   assign: neighbours take their class's new upper part
//   close:  the first-counted neighbour of each class shrinks the old class;
//           every unnumbered vertex offers its key for the next pivot
// ---------------------------------------------------------------------------
struct StepTabs {
    uint32_t *cls;            // class of each vertex
    uint32_t *clast;          // last position of each live class
    uint32_t *cnt;            // neighbours of the pivot per class
    int32_t *lead;            // class counted first by this vertex, or -1
    unsigned long long *key;  // [2]: pivot key of this step and the next
};

constexpr int kStepThreads = 256;

__device__ __forceinline__ int step_pivot(const StepTabs &st, int i)
{
    return (int)(0xFFFFFFFFu - (uint32_t)st.key[i & 1]);  // written by the previous launch
}

__device__ __forceinline__ bool adjacent_bit(const GDesc &g, int x, int v)
{
    return (g.bits[(size_t)x * (size_t)g.W + (size_t)(v >> 6)] >> (v & 63)) & 1ull;
}

__global__ __launch_bounds__(kStepThreads) void k_step_init(GDesc g, StepTabs st)
{
    const int v = blockIdx.x * kStepThreads + threadIdx.x;
    if (v < g.n) {
        st.cls[v] = 0;
        st.cnt[v] = 0;
        st.lead[v] = -1;
        g.rank[v] = -1;
        g.parent[v] = -1;
    }
    if (v == 0) {
        st.clast[0] = (uint32_t)(g.n - 1);
        st.key[0] = 0xFFFFFFFFull;  // class 0, vertex 0
        st.key[1] = 0;
        if (g.failkey) *g.failkey = kNoFail;
    }
}

__global__ __launch_bounds__(kStepThreads) void k_step_count(GDesc g, StepTabs st, int i)
{
    const int x = step_pivot(st, i);
    const int v = blockIdx.x * kStepThreads + threadIdx.x;
    if (v == 0) {
        g.order[i] = x;
        g.rank[x] = i;
        st.key[(i + 1) & 1] = 0;
        const uint32_t top = (uint32_t)(g.n - 1 - i);  // the pivot's class ends here
        const uint32_t c = st.cls[x];
        if (c < top) st.clast[c] = top - 1;
    }
    if (v >= g.n || v == x || g.rank[v] >= 0 || !adjacent_bit(g, x, v)) return;
    const uint32_t c = st.cls[v];
    const uint32_t before = atomicAdd(&st.cnt[c], 1u);
    st.lead[v] = before == 0 ? (int32_t)c : -1;
    g.parent[v] = x;
}

__global__ __launch_bounds__(kStepThreads) void k_step_assign(GDesc g, StepTabs st, int i)
{
    const int x = step_pivot(st, i);
    const int v = blockIdx.x * kStepThreads + threadIdx.x;
    if (v >= g.n || v == x || g.rank[v] >= 0 || !adjacent_bit(g, x, v)) return;
    const uint32_t c = st.cls[v];
    const uint32_t last = st.clast[c];
    const uint32_t nw = last + 1 - st.cnt[c];
    if (nw != c) {
        st.cls[v] = nw;
        // Positions above c inside its range are no live class's start, so
        // no thread of this launch reads clast[nw].
        if (st.lead[v] >= 0) st.clast[nw] = last;
    }
}

__global__ __launch_bounds__(kStepThreads) void k_step_close(GDesc g, StepTabs st, int i)
{
    __shared__ unsigned long long red[kStepThreads / kWave];
    const int v = blockIdx.x * kStepThreads + threadIdx.x;
    unsigned long long k = 0;
    if (v < g.n) {
        const int32_t c = st.lead[v];
        if (c >= 0) {
            st.lead[v] = -1;
            const uint32_t nw = st.cls[v];
            if (nw != (uint32_t)c) st.clast[c] = nw - 1;
            st.cnt[c] = 0;
        }
        if (g.rank[v] < 0) k = ((unsigned long long)st.cls[v] << 32) | (0xFFFFFFFFu - (uint32_t)v);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(k, o, kWave);
        k = y > k ? y : k;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = k;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kStepThreads / kWave; ++w) k = red[w] > k ? red[w] : k;
        if (k) atomicMax(&st.key[(i + 1) & 1], k);
    }
}

// One graph of a batch on one team, start to finish: LexBFS with the fused
// elimination test, then (for a failing graph) the witness and certificate,
// reusing the team's LDS region.
template <class Team, bool kMcs, bool kIlv = false>
__device__ void batch_graph(const Team &tm, const GDesc &g, void *region, uint32_t flags)
{
    if (kMcs) {
        mcs_team<Team, true, 2>(tm, g.n, g.bits, g.W, g.order, g.rank, g.parent,
                                carve_mcs(region, g.n, Team::kSize, true, g.failkey));
    } else {
        BatchLayout B = carve_batch(region, g.n, Team::kSize, g.failkey);
        lexbfs_team<Team, LdsTables, true, kIlv, 16, 2>(tm, g.n, g.bits, g.W, g.rp, g.order, g.rank, g.parent,
                                                         B.L.starts, B.L.cls, B.L.tab, B.L.red, B.fp);
    }
    tm.sync_mem();  // order, rank, parent and the failing rank visible to the team
    if (!(flags & kFlagOrderOnly)) finish_graph(tm, g, flags, carve_finish(region, g.wn, Team::kWaves));
    tm.sync();        // the region is reused by the team's next graph
}

// ---------------------------------------------------------------------------
// Device-side ingestion: the packed adjacency bitset from the CSR (the
// paper's Adj matrix, Section 6.3, built on the device instead of copied).
// One wavefront per row: it clears its row's words in LDS, ORs in the bits
// of the row's CSR entries (read 64 at a time, coalesced), and writes the
// row back with coalesced 16-byte stores (64-bit ones where a row's words
// are not whole 16-byte pairs on 16-byte boundaries), padding words included.
// ---------------------------------------------------------------------------
constexpr int kBuildThreads = 256;

// Rows first, first + stride, ... of one graph, one wavefront at a time;
// `row` is this wavefront's LDS buffer of W words.
__device__ __forceinline__ void build_rows(int n, const int32_t *rp_, const int32_t *ci_, uint64_t *bits_, int64_t W,
                                           uint64_t *row, int first, int stride)
{
    LX_GLOBAL const int32_t *rp = as_global(rp_);
    LX_GLOBAL const int32_t *ci = as_global(ci_);
    LX_GLOBAL uint64_t *bits = as_global(bits_);
    const int lane = threadIdx.x & 63;
    const int64_t lim = W << 6;  // ids beyond the row's words are ignored
    const bool wide = !(W & 1) && !((uintptr_t)bits_ & 15) && !((uintptr_t)row & 15);
    for (int v = first; v < n; v += stride) {
        for (int64_t w = lane; w < W; w += kWave) row[w] = 0ull;
        __builtin_amdgcn_wave_barrier();
        const int b = rp[v], e = rp[v + 1];
        for (int j = b + lane; j < e; j += kWave) {
            const int u = ci[j];
            if ((unsigned)u < (uint64_t)lim) atomicOr((unsigned long long *)&row[u >> 6], 1ull << (u & 63));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        LX_GLOBAL uint64_t *out = bits + (int64_t)v * W;
        if (wide) {
            // Whole 16-byte pairs on 16-byte boundaries in LDS and in the
            // bitset: one 16-byte store per lane (0.175 against 0.180 ms for
            // the 512 MiB bitset of a 65,536-vertex graph).
            const u64x2 *row2 = (const u64x2 *)row;
            LX_GLOBAL u64x2 *out2 = (LX_GLOBAL u64x2 *)out;
            for (int64_t q = lane; q < (W >> 1); q += kWave) out2[q] = row2[q];
        } else {
            for (int64_t w = lane; w < W; w += kWave) out[w] = row[w];
        }
        __builtin_amdgcn_wave_barrier();  // the row buffer is cleared again only after every lane read it
    }
}

__global__ __launch_bounds__(kBuildThreads) void k_build_bitset(int n, const int32_t *__restrict__ rp,
                                                                const int32_t *__restrict__ ci, uint64_t *bits,
                                                                int64_t W)
{
    extern __shared__ uint64_t lds[];
    const int wave = threadIdx.x >> 6;
    build_rows(n, rp, ci, bits, W, lds + (int64_t)wave * W, blockIdx.x * (kBuildThreads / kWave) + wave,
               gridDim.x * (kBuildThreads / kWave));
}

// ---------------------------------------------------------------------------
// Input contract check (LEXBFS_FLAG_VALIDATE, lexbfs_validate). Section 3.1
// works with simple graphs: N(v) never holds v, adjacency is symmetric, and
// the CSR and the bitset must describe the same N(v). One wavefront per row;
// every read stays inside the arrays the contract sizes: row_ptr[0..n],
// col_idx[j] only for j inside [0, nnz) once the row's bounds are checked,
// bitset rows only for ids already checked to lie in 0..n-1.
//   CSR row v: ascending strictly (so no duplicates), ids in 0..n-1, no v;
//   every entry u has bit u in row v and bit v in row u; the number of set
//   bits in row v (bits >= n of the last word included) equals deg(v).
// With every CSR entry present in the bitset and the counts equal, the two
// agree exactly; with the reverse bits present the graph is symmetric.
// ---------------------------------------------------------------------------
enum : uint32_t {
    kBadRowPtr = 1u,   // row pointers not non-decreasing from 0 to nnz
    kBadId = 2u,       // a column index outside 0..n-1
    kSelfLoop = 4u,    // v in its own row
    kUnsorted = 8u,    // a row not strictly ascending (unsorted or duplicate)
    kNotInBits = 16u,  // a CSR entry whose bit is clear
    kAsym = 32u,       // u in N(v) but v not in N(u)
    kExtraBits = 64u,  // bits set that the CSR row does not hold
};

constexpr int kValidateThreads = 256;

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v |= (uint32_t)__shfl_xor((int)v, off, kWave);
    return v;
}

// Rows first, first + stride, ... of graph g; ORs the error bits found into
// *status (one atomic per wavefront, only when something is wrong).
__device__ void validate_rows(const GDesc &g, int first, int stride, uint32_t *status)
{
    LX_GLOBAL const int32_t *rp = as_global(g.rp);
    LX_GLOBAL const int32_t *ci = as_global(g.ci);
    LX_GLOBAL const uint64_t *bits = as_global(g.bits);
    const int lane = threadIdx.x & 63;
    const int n = g.n;
    const int64_t nnz = g.nnz;
    const int wn = (n + 63) >> 6;
    const uint64_t tailmask = (n & 63) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
    uint32_t bad = 0;
    for (int v = first; v < n; v += stride) {
        const int64_t b = rp[v], e = rp[v + 1];
        if (v == 0 && b != 0) bad |= kBadRowPtr;
        if (v == n - 1 && e != nnz) bad |= kBadRowPtr;
        if (b < 0 || e < b || e > nnz) {
            bad |= kBadRowPtr;
            continue;  // col_idx of this row is not known to be in bounds
        }
        for (int64_t j = b + lane; j < e; j += kWave) {
            const int u = ci[j];
            if (j > b && ci[j - 1] >= u) bad |= kUnsorted;
            if (u < 0 || u >= n) {
                bad |= kBadId;
                continue;
            }
            if (u == v) bad |= kSelfLoop;
            if (!((bits[(int64_t)v * g.W + (u >> 6)] >> (u & 63)) & 1ull)) bad |= kNotInBits;
            if (!((bits[(int64_t)u * g.W + (v >> 6)] >> (v & 63)) & 1ull)) bad |= kAsym;
        }
        uint32_t cnt = 0;
        for (int w = lane; w < wn; w += kWave) {
            const uint64_t x = bits[(int64_t)v * g.W + w];
            cnt += (uint32_t)__popcll(x);
            if (w == wn - 1 && (x & ~tailmask)) bad |= kExtraBits;  // bits >= n
        }
        cnt = wave_sum_dpp(cnt);
        if ((int64_t)cnt != e - b) bad |= kExtraBits;
    }
    bad = wave_or_u32(bad);
    if (lane == 0 && bad) atomicOr(status, bad);
}

__global__ __launch_bounds__(kValidateThreads) void k_validate_one(GDesc g, uint32_t *status)
{
    constexpr int wpb = kValidateThreads / kWave;
    validate_rows(g, blockIdx.x * wpb + (int)(threadIdx.x >> 6), gridDim.x * wpb, status);
}

// bpg blocks per graph; status[i] for graph i.
__global__ __launch_bounds__(kValidateThreads) void k_validate_batch(const GDesc *__restrict__ gds, int count, int bpg,
                                                                     uint32_t *status)
{
    constexpr int wpb = kValidateThreads / kWave;
    const int gi = blockIdx.x / bpg;
    if (gi >= count) return;
    const int bl = blockIdx.x - gi * bpg;
    validate_rows(gds[gi], bl * wpb + (int)(threadIdx.x >> 6), bpg * wpb, status + gi);
}

__global__ void k_fill_u32(uint32_t *p, int count, uint32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Batch: every block first takes large graphs (whole block per graph) from a
// longest-first queue; once those run out every wave takes small graphs.
template <int BT, bool kMcs, bool kIlv = false>
__global__ __launch_bounds__(BT) void k_batch(const GDesc *__restrict__ gds, const int32_t *__restrict__ sorted,
                                              int nbig, int count, uint32_t *qctr, int wave_region_bytes,
                                              uint32_t flags)
{
    extern __shared__ uint64_t lds[];
    __shared__ int s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int)atomicAdd(&qctr[0], 1u);
        __syncthreads();
        const int k = s_idx;
        __syncthreads();
        if (k >= nbig) break;
        BlockTeam<BT, false> tm{(int)threadIdx.x};
        batch_graph<BlockTeam<BT, false>, kMcs, kIlv>(tm, gds[sorted[k]], lds, flags);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    void *region = (char *)lds + (size_t)wave * wave_region_bytes;
    const int nsmall = count - nbig;
    for (;;) {
        int k = 0;
        if (lane == 0) k = (int)atomicAdd(&qctr[1], 1u);
        k = __shfl(k, 0, kWave);
        if (k >= nsmall) break;
        WaveTeam tm{lane};
        batch_graph<WaveTeam, kMcs, kIlv>(tm, gds[sorted[nbig + k]], region, flags);
    }
}

__global__ void k_batch_init(const GDesc *__restrict__ gds, int count, uint32_t *qctr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) *gds[i].failkey = kNoFail;
    if (i == 0) {
        qctr[0] = 0;
        qctr[1] = 0;
    }
}

// Batch graphs too large for a 256-lane team: one workgroup per graph with
// the team size and state of a single-graph call -- 512 lanes up to
// kLargeMidMaxN vertices, 1,024 above; class tables in LDS when they fit
// `lds_limit`, else the compact LDS layout, else class tables in global
// memory -- then the graph's sweep and certificate on the same workgroup.
constexpr int kLargeThreads = 1024;
constexpr int kLargeMidThreads = 512;
constexpr int kLargeMidMaxN = 32768;

template <int T, bool kMcs>
__global__ __launch_bounds__(T) void k_batch_large(const GDesc *__restrict__ gds, const int32_t *__restrict__ which,
                                                   uint32_t flags, int lds_limit)
{
    extern __shared__ uint64_t lds[];
    vgpr_headroom<T>();
    const GDesc g = gds[which[blockIdx.x]];
    if (kMcs) {
        BlockTeam<T, false> tm{(int)threadIdx.x};
        mcs_team(tm, g.n, g.bits, g.W, g.order, g.rank, g.parent, carve_mcs(lds, g.n, T, false, nullptr));
    } else if (lds_bytes_lds_tables(g.n, T) <= (size_t)lds_limit) {
        LdsLayout L = carve_lds(lds, g.n, T);
        BlockTeam<T, false> tm{(int)threadIdx.x};
        lexbfs_team<BlockTeam<T, false>, LdsTables, false, false, 32>(tm, g.n, g.bits, g.W, g.rp, g.order, g.rank,
                                                                     g.parent, L.starts, L.cls, L.tab, L.red);
    } else if (lds_bytes_compact(g.n, T) <= (size_t)lds_limit) {
        BlockTeam<T, false> tm{(int)threadIdx.x};
        lexbfs_team_compact(tm, g.n, g.bits, g.W, g.order, g.rank, g.parent, carve_compact(lds, g.n, T));
    } else {
        LdsLayoutG L = carve_lds_g(lds, g.n, T);
        GlobalTables tab(g.gtab, g.gtab + g.n);
        BlockTeam<T, true> tm{(int)threadIdx.x};
        lexbfs_team(tm, g.n, g.bits, g.W, g.rp, g.order, g.rank, g.parent, L.starts, L.cls, tab, L.red);
        tm.sync_mem();  // order and rank visible to every wave
        derive_parents(g.rp, g.ci, g.order, g.rank, g.parent, g.n, (int)(threadIdx.x >> 6), T / kWave);
    }
    BlockTeam<T, false> tm{(int)threadIdx.x};
    tm.sync_mem();  // rank and parent of every vertex visible to the sweep
    if (flags & kFlagOrderOnly) return;
    int G = 1, lg = 0;
    while (G < g.wn && G < kWave) {
        G <<= 1;
        ++lg;
    }
    sweep_rows<false>(g.bits, g.W, g.wn, g.rank, g.parent, g.n, 0, g.n, G, lg, g.failkey);
    tm.sync_mem();  // the failing rank visible to the certificate
    finish_graph(tm, g, flags, carve_finish(lds, g.wn, T / kWave));
}

// ---------------------------------------------------------------------------
// Multi-sweep LexBFS and the unit interval test. Section 3.2 surveys LexBFS
// as a building block of interval recognition and Section 8 leaves parallel
// interval testing open; the three-sweep test here is Corneil's
// (LexBFS, then LexBFS+ twice, then a check that every closed neighbourhood
// is consecutive in the last order; Corneil, Discrete Applied Mathematics
// 138 (2004)).
//
// A LexBFS+ sweep breaks ties between equal labels in favour of the vertex
// that comes last in a previous order prev. Renaming v to n-1-pos(v), with
// pos(v) the position of v in prev, makes that vertex the one of smallest
// new id, so a sweep is: rename the graph on the device (CSR, then bitset),
// run the LexBFS kernel unchanged, and rename its order back. New id a is
// old vertex prev[n-1-a], so only neighbour ids need pos. Renamed rows keep
// the order of their original entries (they are not ascending): the LexBFS
// kernel reads a CSR row only for its length and the parent pass only for a
// maximum over it, and neither depends on the order of the entries.
// ---------------------------------------------------------------------------
constexpr int kPlusThreads = 256;
constexpr int kPlusScanThreads = 1024;
constexpr int kPlusPerLane = LEXBFS_MAX_N / kPlusScanThreads;  // rows summed by one lane of the scan

// New ids of a renamed graph against tie ranks (the previous order
// reversed): equal when K = 0, else the interleaved order of a team with K
// vertices per lane (ilv_rank / ilv_id).
struct IlvMap {
    uint32_t K, lgK, tl, cl;
    __device__ IlvMap(int n, int k) : K((uint32_t)k), lgK(0), tl(0), cl(0)
    {
        if (K) {
            while ((1u << lgK) < K) ++lgK;
            tl = (uint32_t)(n - 1) >> lgK;
            cl = (uint32_t)n - (tl << lgK);
        }
    }
    __device__ __forceinline__ uint32_t rank_of(uint32_t a) const
    {
        return K ? ilv_rank(a & (K - 1), a >> lgK, tl, cl) : a;
    }
    __device__ __forceinline__ uint32_t id_of(uint32_t r) const { return K ? ilv_id(r, tl, cl, K) : r; }
};

// pos[v] = -1 for every v, flag = 0, and (when given) the interval key to
// "no failure".
__global__ __launch_bounds__(kPlusThreads) void k_plus_init(int n, int32_t *pos, int32_t *flag, uint32_t *key)
{
    const int i = blockIdx.x * kPlusThreads + threadIdx.x;
    if (i < n) pos[i] = -1;
    if (i == 0) {
        *flag = 0;
        if (key) *key = kNoFail;
    }
}

// pos[prev[i]] = i. flag becomes 1 unless prev is a permutation of 0..n-1
// (an id out of range, or an id seen twice).
__global__ __launch_bounds__(kPlusThreads) void k_plus_inverse(int n, const int32_t *__restrict__ prev,
                                                               int32_t *pos, int32_t *flag)
{
    const int i = blockIdx.x * kPlusThreads + threadIdx.x;
    if (i >= n) return;
    const int v = prev[i];
    if ((unsigned)v >= (unsigned)n || atomicExch(&pos[v], i) != -1) atomicOr(flag, 1);
}

// deg[a] = degree of old vertex prev[n-1-a] for a < n, 0 up to npad (a
// multiple of kPlusPerLane); all 0 when prev is not a permutation, which
// turns the renamed graph into an edgeless one.
__global__ __launch_bounds__(kPlusThreads) void k_plus_degree(int n, int npad, const int32_t *__restrict__ prev,
                                                              const int32_t *__restrict__ rp,
                                                              const int32_t *__restrict__ flag, int32_t *deg, int ik)
{
    const int a = blockIdx.x * kPlusThreads + threadIdx.x;
    if (a >= npad) return;
    int d = 0;
    if (a < n && *flag == 0) {
        const IlvMap map(n, ik);
        const int v = prev[n - 1 - (int)map.rank_of((uint32_t)a)];
        d = rp[v + 1] - rp[v];
    }
    deg[a] = d;
}

// rp2 = exclusive prefix sum of deg (n+1 entries). One workgroup: lane t
// loads its kPlusPerLane consecutive degrees with 16-byte loads, the team
// scans the lane totals, and each lane writes its run of row pointers.
__global__ __launch_bounds__(kPlusScanThreads) void k_plus_scan(int n, const int32_t *__restrict__ deg_,
                                                                int32_t *rp2)
{
    __shared__ uint32_t red[kPlusScanThreads / kWave];
    const int t = threadIdx.x;
    const int a0 = t * kPlusPerLane;
    const int4 *deg = (const int4 *)deg_;
    int4 x[kPlusPerLane / 4];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kPlusPerLane / 4; ++k) {
        x[k] = a0 < n ? deg[a0 / 4 + k] : make_int4(0, 0, 0, 0);
        s += (uint32_t)(x[k].x + x[k].y + x[k].z + x[k].w);
    }
    BlockTeam<kPlusScanThreads, false> tm{t};
    uint32_t off = tm.exclusive_scan(s, red);
    if (t == 0) rp2[0] = 0;
    if (a0 >= n) return;
#pragma unroll
    for (int k = 0; k < kPlusPerLane / 4; ++k) {
        const int a = a0 + 4 * k;
        const int d[4] = {x[k].x, x[k].y, x[k].z, x[k].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            off += (uint32_t)d[q];
            if (a + q < n) rp2[a + q + 1] = (int32_t)off;
        }
    }
}

// Lanes per renamed row (log2): rows of up to 64 words get the smallest
// power of two >= W2, at most 16, so a wavefront works on at least four
// rows at once (four dependent loads per row make each row latency-bound);
// longer rows get the whole wavefront.
__host__ __device__ __forceinline__ int rename_group_log2(int W2)
{
    if (W2 > kWave) return 6;
    int lg = 0;
    while ((1 << lg) < W2 && lg < 4) ++lg;
    return lg;
}

// LDS words of one wavefront's row buffers: (64 / G) rows of W2 words.
__host__ __device__ __forceinline__ int rename_buffer_words(int W2) { return W2 > kWave ? W2 : 4 * kWave; }

// Renamed rows of one graph, wavefront slots first, first + stride, ...,
// each slot taking 64 / G consecutive rows (G lanes per row): row a is the
// row of old vertex prev[n-1-rank(a)] with every neighbour u renamed to
// id(n-1-pos[u]) (rank and id of IlvMap, identities when ik = 0), written
// to the renamed CSR (entries past nnz, from a row_ptr
// that disagrees with nnz, are dropped) and, through the wavefront's LDS
// buffer `buf` (rename_buffer_words(W2) words), to row a of the renamed
// bitset. With `bad` (prev not a permutation) every row is empty.
__device__ __forceinline__ void rename_rows(int n, int64_t nnz, const int32_t *prev_, const int32_t *pos_,
                                            const int32_t *rp_, const int32_t *ci_, const int32_t *rp2_,
                                            int32_t *ci2_, uint64_t *bits2_, int W2, bool bad, uint64_t *buf,
                                            int first, int stride, int ik = 0)
{
    const IlvMap map(n, ik);
    LX_GLOBAL const int32_t *prev = as_global(prev_);
    LX_GLOBAL const int32_t *pos = as_global(pos_);
    LX_GLOBAL const int32_t *rp = as_global(rp_);
    LX_GLOBAL const int32_t *ci = as_global(ci_);
    LX_GLOBAL const int32_t *rp2 = as_global(rp2_);
    LX_GLOBAL int32_t *ci2 = as_global(ci2_);
    LX_GLOBAL uint64_t *bits2 = as_global(bits2_);
    const int lane = threadIdx.x & 63;
    const int lg = rename_group_log2(W2), G = 1 << lg, R = kWave >> lg;
    const int sub = lane >> lg, gl = lane & (G - 1);
    uint64_t *row = buf + sub * W2;  // R * W2 <= rename_buffer_words(W2)
    for (int base = first * R; base < n; base += stride * R) {
        const int a = base + sub;
        for (int w = gl; w < W2; w += G) row[w] = 0ull;
        __builtin_amdgcn_wave_barrier();
        if (a < n && !bad) {
            const int v = prev[n - 1 - (int)map.rank_of((uint32_t)a)];
            const int b = rp[v], e = rp[v + 1], o = rp2[a];
            for (int j = b + gl; j < e; j += G) {
                const int u = ci[j];
                const int u2 = (unsigned)u < (unsigned)n ? (int)map.id_of((uint32_t)(n - 1 - pos[u])) : u;
                const int64_t q = (int64_t)o + (j - b);
                if (q < nnz) ci2[q] = u2;
                if ((unsigned)u2 < (unsigned)n) atomicOr((unsigned long long *)&row[u2 >> 6], 1ull << (u2 & 63));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (a < n) {
            LX_GLOBAL uint64_t *out = bits2 + (int64_t)a * W2;
            for (int w = gl; w < W2; w += G) out[w] = row[w];
        }
        __builtin_amdgcn_wave_barrier();  // the row buffers are cleared again only after every lane read them
    }
}

// Renamed CSR rows and bitset of one graph.
__global__ __launch_bounds__(kPlusThreads) void k_plus_rows(int n, int64_t nnz, const int32_t *__restrict__ prev,
                                                            const int32_t *__restrict__ pos,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const int32_t *__restrict__ flag,
                                                            const int32_t *__restrict__ rp2, int32_t *ci2,
                                                            uint64_t *bits2, int ik)
{
    extern __shared__ uint64_t lds[];
    const int W2 = (n + 63) / 64;
    const int wave = threadIdx.x >> 6;
    rename_rows(n, nnz, prev, pos, rp, ci, rp2, ci2, bits2, W2, *flag != 0,
                lds + (int64_t)wave * rename_buffer_words(W2), blockIdx.x * (kPlusThreads / kWave) + wave,
                gridDim.x * (kPlusThreads / kWave), ik);
}

// The renamed sweep's outputs in old ids: order[i] = prev[n-1-order2[i]],
// rank its inverse, parent[v] = the old id of the renamed parent. All -1
// when prev is not a permutation.
__global__ __launch_bounds__(kPlusThreads) void k_plus_map(int n, const int32_t *__restrict__ prev,
                                                           const int32_t *__restrict__ order2,
                                                           const int32_t *__restrict__ parent2,
                                                           const int32_t *__restrict__ flag, int32_t *order,
                                                           int32_t *rank, int32_t *parent, int ik)
{
    const int i = blockIdx.x * kPlusThreads + threadIdx.x;
    if (i >= n) return;
    const int a = order2[i];
    if (*flag != 0 || (unsigned)a >= (unsigned)n) {
        order[i] = -1;
        if (rank) rank[i] = -1;
        if (parent) parent[i] = -1;
        return;
    }
    const IlvMap map(n, ik);
    const int v = prev[n - 1 - (int)map.rank_of((uint32_t)a)];
    order[i] = v;
    if (rank) rank[v] = i;
    if (parent) {
        const int p = parent2[a];
        parent[v] = (unsigned)p < (unsigned)n ? prev[n - 1 - (int)map.rank_of((uint32_t)p)] : -1;
    }
}

// Unit interval check of an order: the closed neighbourhood of every vertex
// must occupy consecutive positions. With rows free of repeats and
// self-loops, N[v] of the vertex at position i is consecutive iff the span of
// its positions (i included) is deg(v). One wavefront per position; key =
// smallest failing position.
__global__ __launch_bounds__(kPlusThreads) void k_ui_check(int n, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const int32_t *__restrict__ order,
                                                           const int32_t *__restrict__ rank, uint32_t *key)
{
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * (kPlusThreads / kWave);
    for (int i = blockIdx.x * (kPlusThreads / kWave) + (threadIdx.x >> 6); i < n; i += stride) {
        const int v = order[i];
        if ((unsigned)v >= (unsigned)n) {  // no order (the previous one was not a permutation)
            if (lane == 0) atomicMin(key, (uint32_t)i);
            continue;
        }
        const int b = rp[v], e = rp[v + 1];
        uint32_t lo = (uint32_t)i, hi = (uint32_t)i;
        for (int j = b + lane; j < e; j += kWave) {
            const int u = ci[j];
            const uint32_t r = (unsigned)u < (unsigned)n ? (uint32_t)rank[u] : (uint32_t)n;
            lo = min(lo, r);
            hi = max(hi, r);  // an id out of range counts as position n
        }
        lo = wave_min_u32(lo);
        hi = wave_max_u32(hi);
        if (lane == 0 && hi - lo != (uint32_t)(e - b)) atomicMin(key, (uint32_t)i);
    }
}

// Verdict and witness of one graph on one workgroup, `i` the smallest
// failing position (kNoFail if none). For the failing vertex v at position
// i, with [lo, hi] the span of N[v]: b is the earliest vertex in the span
// that is not in N[v], and the triple is (order[lo], b, v) when b comes
// before v, else (v, b, order[hi]): its first and last vertices are
// adjacent, the middle one is not adjacent to both.
template <int T>
__device__ void ui_witness_block(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const uint64_t *__restrict__ bits, int64_t W, const int32_t *__restrict__ order,
                                 const int32_t *__restrict__ rank, uint32_t i, lexbfs_interval_result_t *res,
                                 uint32_t *red)
{
    const int t = threadIdx.x;
    if (i == kNoFail) {
        if (t == 0) {
            res->unit_interval = 1;
            res->witness[0] = res->witness[1] = res->witness[2] = -1;
            for (int k = 0; k < 4; ++k) res->reserved[k] = 0;
        }
        return;
    }
    BlockTeam<T, false> tm{t};
    const int v = order[i];
    if ((unsigned)v >= (unsigned)n) {
        if (t == 0) {
            res->unit_interval = 0;
            res->witness[0] = res->witness[1] = res->witness[2] = -1;
            for (int k = 0; k < 4; ++k) res->reserved[k] = 0;
        }
        return;
    }
    const int b = rp[v], e = rp[v + 1];
    uint32_t lo = i, hi = i;
    for (int j = b + t; j < e; j += T) {
        const int u = ci[j];
        const uint32_t r = (unsigned)u < (unsigned)n ? (uint32_t)rank[u] : (uint32_t)n;
        lo = min(lo, r);
        hi = max(hi, r);
    }
    lo = tm.min_all(lo, red);
    hi = min(~tm.min_all(~hi, red), (uint32_t)n - 1);  // positions stay inside the order
    const uint64_t *row = bits + (int64_t)v * W;
    uint32_t cand = kNoFail;  // the first position of this lane's stride that is outside N[v]
    for (uint32_t p = lo + t; p <= hi; p += T)
        if (p != i && !test_bit(row, order[p])) {
            cand = p;
            break;
        }
    const uint32_t bp = tm.min_all(cand, red);
    if (t == 0) {
        res->unit_interval = 0;
        if (bp == kNoFail) {  // cannot happen for a graph that meets the input contract
            res->witness[0] = res->witness[1] = res->witness[2] = -1;
        } else if (bp < i) {
            res->witness[0] = order[lo];
            res->witness[1] = order[bp];
            res->witness[2] = v;
        } else {
            res->witness[0] = v;
            res->witness[1] = order[bp];
            res->witness[2] = order[hi];
        }
        for (int k = 0; k < 4; ++k) res->reserved[k] = 0;
    }
}

__global__ __launch_bounds__(kFinishThreads) void k_ui_witness(int n, const int32_t *__restrict__ rp,
                                                               const int32_t *__restrict__ ci,
                                                               const uint64_t *__restrict__ bits, int64_t W,
                                                               const int32_t *__restrict__ order,
                                                               const int32_t *__restrict__ rank,
                                                               const uint32_t *__restrict__ key,
                                                               lexbfs_interval_result_t *res)
{
    __shared__ uint32_t red[kFinishThreads / kWave];
    ui_witness_block<kFinishThreads>(n, rp, ci, bits, W, order, rank, *key, res, red);
}

// ---------------------------------------------------------------------------
// Batched unit interval test: the same steps for many graphs, each kernel
// covering the whole batch (a workgroup, or a row of workgroups, per graph);
// the three LexBFS passes are batch plans over the original and the renamed
// graphs.
// ---------------------------------------------------------------------------
struct IDesc {
    int32_t n;
    int32_t wn;         // ceil(n / 64): row stride of the renamed bitset
    int64_t nnz;
    int64_t W;          // row stride of the input bitset
    const int32_t *rp;
    const int32_t *ci;
    const uint64_t *bits;
    int32_t *rp2;       // renamed CSR [n+1], [nnz] and bitset [n * wn]
    int32_t *ci2;
    uint64_t *bits2;
    int32_t *pos;       // [n] position in the previous order
    int32_t *s1;        // the three orders [n] and the ranks of the third
    int32_t *s2;
    int32_t *s3;
    int32_t *rank3;
    int32_t *flag;      // [1] previous order not a permutation
    uint32_t *key;      // [1] smallest failing position of the third order
    lexbfs_interval_result_t *res;
    int32_t ik;         // K of the renamed graph's interleaved tie order, 0 = ids in rank order
};

constexpr int kIbThreads = 256;

// Renaming of one graph per workgroup after prev = s1 (sel 1) or s2 (sel 2):
// inverse and validity, renamed row lengths and their prefix sum -- the
// single-graph kernels' steps, ordered by workgroup barriers.
__global__ __launch_bounds__(kIbThreads) void k_ib_rename(const IDesc *__restrict__ ds, int sel)
{
    __shared__ int s_bad;
    __shared__ uint32_t red[kIbThreads / kWave];
    const IDesc d = ds[blockIdx.x];
    const int n = d.n;
    if (n == 0) return;
    const int32_t *prev = sel == 2 ? d.s2 : d.s1;
    const int t = threadIdx.x;
    if (t == 0) s_bad = 0;
    for (int v = t; v < n; v += kIbThreads) d.pos[v] = -1;
    __syncthreads();
    for (int i = t; i < n; i += kIbThreads) {
        const int v = prev[i];
        if ((unsigned)v >= (unsigned)n || atomicExch(&d.pos[v], i) != -1) atomicOr(&s_bad, 1);
    }
    __syncthreads();
    const bool bad = s_bad != 0;
    if (t == 0) *d.flag = bad ? 1 : 0;
    const IlvMap map(n, d.ik);
    for (int a = t; a < n; a += kIbThreads) {
        int deg = 0;
        if (!bad) {
            const int v = prev[n - 1 - (int)map.rank_of((uint32_t)a)];
            deg = d.rp[v + 1] - d.rp[v];
        }
        d.rp2[a + 1] = deg;
    }
    __syncthreads();
    const int per = (n + kIbThreads - 1) / kIbThreads;
    const int a0 = min(n, t * per), a1 = min(n, a0 + per);
    uint32_t sum = 0;
    for (int a = a0; a < a1; ++a) sum += (uint32_t)d.rp2[a + 1];
    BlockTeam<kIbThreads, false> tm{t};
    uint32_t off = tm.exclusive_scan(sum, red);
    for (int a = a0; a < a1; ++a) {
        off += (uint32_t)d.rp2[a + 1];
        d.rp2[a + 1] = (int32_t)off;
    }
    if (t == 0) d.rp2[0] = 0;
}

// Renamed CSR rows and bitsets: graph blockIdx.x, rows spread over the
// gridDim.y workgroups of its grid row; `bufw` LDS words per wavefront, the
// largest rename_buffer_words over the batch's graphs (not that of the widest
// row: graphs of up to 64-word rows buffer four rows per wavefront).
__global__ __launch_bounds__(kBuildThreads) void k_ib_rows(const IDesc *__restrict__ ds, int sel, int bufw)
{
    extern __shared__ uint64_t lds[];
    const IDesc d = ds[blockIdx.x];
    const int wave = threadIdx.x >> 6;
    rename_rows(d.n, d.nnz, sel == 2 ? d.s2 : d.s1, d.pos, d.rp, d.ci, d.rp2, d.ci2, d.bits2, d.wn, *d.flag != 0,
                lds + (int64_t)wave * bufw, blockIdx.y * (kBuildThreads / kWave) + wave,
                gridDim.y * (kBuildThreads / kWave), d.ik);
}

// The renamed pass's order in old ids: s2 from s1 (sel 2) or s3 and its
// ranks from s2 (sel 3, which also resets the failure key).
__global__ __launch_bounds__(kIbThreads) void k_ib_map(const IDesc *__restrict__ ds, const GDesc *__restrict__ renamed,
                                                       int sel)
{
    const IDesc d = ds[blockIdx.x];
    const int n = d.n;
    if (sel == 3 && threadIdx.x == 0) *d.key = kNoFail;
    if (n == 0) return;
    const int32_t *prev = sel == 2 ? d.s1 : d.s2;
    int32_t *out = sel == 2 ? d.s2 : d.s3;
    int32_t *rank = sel == 3 ? d.rank3 : nullptr;
    const int32_t *order2 = renamed[blockIdx.x].order;
    const bool bad = *d.flag != 0;
    const IlvMap map(n, d.ik);
    for (int i = threadIdx.x; i < n; i += kIbThreads) {
        const int a = order2[i];
        if (bad || (unsigned)a >= (unsigned)n) {
            out[i] = -1;
            if (rank) rank[i] = -1;
            continue;
        }
        const int v = prev[n - 1 - (int)map.rank_of((uint32_t)a)];
        out[i] = v;
        if (rank) rank[v] = i;
    }
}

// Consecutive-neighbourhood check: graph blockIdx.x, one lane per position,
// positions spread over the gridDim.y workgroups of the grid row.
__global__ __launch_bounds__(kIbThreads) void k_ib_check(const IDesc *__restrict__ ds)
{
    const IDesc d = ds[blockIdx.x];
    const int n = d.n;
    for (int i = blockIdx.y * kIbThreads + threadIdx.x; i < n; i += gridDim.y * kIbThreads) {
        const int v = d.s3[i];
        if ((unsigned)v >= (unsigned)n) {  // no order (the previous one was not a permutation)
            atomicMin(d.key, (uint32_t)i);
            continue;
        }
        const int b = d.rp[v], e = d.rp[v + 1];
        uint32_t lo = (uint32_t)i, hi = (uint32_t)i;
        for (int j = b; j < e; ++j) {
            const int u = d.ci[j];
            const uint32_t r = (unsigned)u < (unsigned)n ? (uint32_t)d.rank3[u] : (uint32_t)n;
            lo = min(lo, r);
            hi = max(hi, r);
        }
        if (hi - lo != (uint32_t)(e - b)) atomicMin(d.key, (uint32_t)i);
    }
}

__global__ __launch_bounds__(kIbThreads) void k_ib_witness(const IDesc *__restrict__ ds)
{
    __shared__ uint32_t red[kIbThreads / kWave];
    const IDesc d = ds[blockIdx.x];
    ui_witness_block<kIbThreads>(d.n, d.rp, d.ci, d.bits, d.W, d.s3, d.rank3, *d.key, d.res, red);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct DevInfo {
    int max_lds = 0;
    bool attrs_set = false;
};
std::mutex g_mu;
DevInfo g_dev[64];

int device_max_lds()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    DevInfo &d = g_dev[dev];
    if (d.max_lds == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return -1;
        d.max_lds = v;
    }
    return d.max_lds;
}

// Largest dynamic LDS a kernel may request: the device limit minus the
// kernel's static LDS. Raises the kernel's dynamic-LDS cap to that value
// once. Returns 0 on failure.
template <class K>
size_t dynamic_lds_limit(K kernel)
{
    // One entry per kernel (not per kernel signature): kernels of one
    // signature differ in their static LDS and each needs its attribute.
    static std::mutex mu;
    static std::vector<std::pair<const void *, size_t>> cache;
    const void *key = (const void *)kernel;
    std::lock_guard<std::mutex> lk(mu);
    for (const auto &e : cache)
        if (e.first == key) return e.second;
    const int maxl = device_max_lds();
    if (maxl <= 0) return 0;
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, key) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const size_t lim = (size_t)maxl - fa.sharedSizeBytes;
    if (hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    cache.emplace_back(key, lim);
    return lim;
}

// Team size for one graph on its own: K = ceil(n / T) vertices per lane.
int single_threads(int n)
{
    static int forced = -1;
    if (forced < 0) {
        const char *e = getenv("LEXBFS_SINGLE_THREADS");
        forced = e ? atoi(e) : 0;
    }
    int T;
    if (forced == 64 || forced == 128 || forced == 256 || forced == 512 || forced == 1024) T = forced;
    else if (n <= 512) T = 64;
    else if (n <= 1024) T = 128;   // measured: 3-4% fewer cycles per step than one wavefront
    else if (n <= 4096) T = 256;
    else if (n <= 32768) T = 512;  // measured: 1.3-2.0 us/step against 1.75-2.2 on 1024 lanes
    else T = 1024;
    while ((int64_t)T * 64 < n) T <<= 1;
    return T;
}

int validate_graph(const lexbfs_graph_t *g)
{
    if (!g) return LEXBFS_EINVAL;
    if (g->n < 0 || g->nnz < 0 || g->nnz >= (int64_t)1 << 31 || g->reserved != 0) return LEXBFS_EINVAL;
    if (g->n > LEXBFS_MAX_N) return LEXBFS_ETOOBIG;
    if (g->n == 0) return LEXBFS_OK;
    if (!g->row_ptr || !g->bits || (g->nnz > 0 && !g->col_idx)) return LEXBFS_EINVAL;
    if (g->words_per_row < (g->n + 63) / 64) return LEXBFS_EINVAL;
    return LEXBFS_OK;
}

// Workspace layout of a single-graph call.
struct SingleWs {
    size_t failkey, order, rank, parent, cycle, level, q0, q1, lnbuf, gtab, total;
};

constexpr SingleWs single_layout(int n)
{
    SingleWs L{};
    const size_t a = al((size_t)(n > 0 ? n : 1) * 4);
    size_t off = 0;
    L.failkey = off; off += kAlign;
    L.order = off; off += a;
    L.rank = off; off += a;
    L.parent = off; off += a;
    L.cycle = off; off += a;
    L.level = off; off += a;
    L.q0 = off; off += a;
    L.q1 = off; off += a;
    L.lnbuf = off; off += a;
    L.gtab = off; off += 2 * a;
    L.total = off;
    return L;
}

// Scratch of chordal_test_noalloc: a single-graph workspace for the largest
// supported n (about 2.5 MiB), one copy per device, held until the process
// ends. Host code never names the array itself (on the host it is a
// stand-in, not a device address); it uses the address hipGetSymbolAddress
// returns for the current device.
constexpr size_t kScratchBytes = single_layout(LEXBFS_MAX_N).total;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64];

// The device address of this device's scratch array, looked up once per
// device with that device current.
int scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "querying the current device");
    if (dev < 0 || dev >= 64) return fail_code(LEXBFS_EINVAL, "device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail_hip(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                   "looking up the scratch array's device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LEXBFS_OK;
}

// The LDS form the single-graph LexBFS kernel takes for n vertices on a
// T-lane team: the first of LDS tables, compact, global tables that fits.
template <int T>
int single_mode_T(int n, int &mode)
{
    const size_t lim_l = dynamic_lds_limit(k_lexbfs_single<T, kModeLds>);
    const size_t lim_c = dynamic_lds_limit(k_lexbfs_single<T, kModeCompact>);
    const size_t lim_g = dynamic_lds_limit(k_lexbfs_single<T, kModeGlobal>);
    if (!lim_l || !lim_c || !lim_g)
        return fail_code(LEXBFS_EHIP, "querying or raising the LexBFS kernel's LDS limit failed");
    if (n < 32768 && lds_bytes_lds_tables(n, T) <= lim_l) mode = kModeLds;  // positions below 2^15
    else if (lds_bytes_compact(n, T) <= lim_c) mode = kModeCompact;
    else if (lds_bytes_global_tables(n, T) <= lim_g) mode = kModeGlobal;
    else return fail_code(LEXBFS_ETOOBIG, "graph state does not fit the workgroup LDS");
    return LEXBFS_OK;
}

template <int T, int kMode>
int launch_single_mode(const GDesc &d, hipStream_t s, bool ilv, size_t lds)
{
    if (ilv) {
        if (dynamic_lds_limit(k_lexbfs_single<T, kMode, true>) < lds)
            return fail_code(LEXBFS_EHIP, "raising the LexBFS kernel's LDS limit failed");
        hipLaunchKernelGGL((k_lexbfs_single<T, kMode, true>), dim3(1), dim3(T), lds, s, d);
    } else {
        hipLaunchKernelGGL((k_lexbfs_single<T, kMode>), dim3(1), dim3(T), lds, s, d);
    }
    return LEXBFS_OK;
}

template <int T>
int launch_lexbfs_single_T(const GDesc &d, hipStream_t s, bool ilv)
{
    int mode = 0;
    int rc = single_mode_T<T>(d.n, mode);
    if (rc) return rc;
    ProfScope ps(0, s);
    if (mode == kModeLds) {
        rc = launch_single_mode<T, kModeLds>(d, s, ilv, lds_bytes_lds_tables(d.n, T));
    } else if (mode == kModeCompact) {
        hipLaunchKernelGGL((k_lexbfs_single<T, kModeCompact>), dim3(1), dim3(T), lds_bytes_compact(d.n, T), s, d);
    } else {
        rc = launch_single_mode<T, kModeGlobal>(d, s, ilv, lds_bytes_global_tables(d.n, T));
        if (rc) return rc;
        LX_CHECK_LAUNCH("LexBFS launch");
        const int blocks = std::min((d.n + 3) / 4, 2048);
        hipLaunchKernelGGL(k_parents, dim3(blocks), dim3(256), 0, s, d);
    }
    if (rc) return rc;
    LX_CHECK_LAUNCH("LexBFS launch");
    return LEXBFS_OK;
}

// ilv: ties by the interleaved rank; only for the forms other than compact
// (single_ilv_k says which).
int launch_lexbfs_single(const GDesc &d, hipStream_t s, bool ilv = false)
{
    switch (single_threads(d.n)) {
        case 64: return launch_lexbfs_single_T<64>(d, s, ilv);
        case 128: return launch_lexbfs_single_T<128>(d, s, ilv);
        case 256: return launch_lexbfs_single_T<256>(d, s, ilv);
        case 512: return launch_lexbfs_single_T<512>(d, s, ilv);
        default: return launch_lexbfs_single_T<1024>(d, s, ilv);
    }
}

// K of the interleaved tie order the single-graph kernel uses for n
// vertices, or 0 when its form (compact) keeps ids in rank order; < 0 on a
// failure.
int single_ilv_k(int n)
{
    const int T = single_threads(n);
    int mode = 0, rc = 0;
    switch (T) {
        case 64: rc = single_mode_T<64>(n, mode); break;
        case 128: rc = single_mode_T<128>(n, mode); break;
        case 256: rc = single_mode_T<256>(n, mode); break;
        case 512: rc = single_mode_T<512>(n, mode); break;
        default: rc = single_mode_T<1024>(n, mode); break;
    }
    if (rc) return rc;
    if (mode == kModeCompact) return 0;
    int K = 1;
    while (K * T < n) K <<= 1;
    return K;
}

template <int T>
int launch_mcs_single_T(const GDesc &d, hipStream_t s)
{
    const size_t lim = dynamic_lds_limit(k_mcs_single<T>);
    if (!lim) return fail_code(LEXBFS_EHIP, "querying or raising the MCS kernel's LDS limit failed");
    const size_t b = lds_bytes_mcs(d.n, T, false);
    if (b > lim) return fail_code(LEXBFS_ETOOBIG, "MCS state does not fit the workgroup LDS");
    ProfScope ps(0, s);
    hipLaunchKernelGGL(k_mcs_single<T>, dim3(1), dim3(T), b, s, d);
    LX_CHECK_LAUNCH("MCS launch");
    return LEXBFS_OK;
}

int launch_mcs_single(const GDesc &d, hipStream_t s)
{
    switch (single_threads(d.n)) {
        case 64: return launch_mcs_single_T<64>(d, s);
        case 128: return launch_mcs_single_T<128>(d, s);
        case 256: return launch_mcs_single_T<256>(d, s);
        case 512: return launch_mcs_single_T<512>(d, s);
        default: return launch_mcs_single_T<1024>(d, s);
    }
}

// The per-step form: three launches per step over ceil(n / 256) blocks.
// Its tables live in the certificate's scratch arrays (not yet in use) and
// the global class-table area of the workspace.
int launch_lexbfs_per_step(const GDesc &d, hipStream_t s)
{
    StepTabs st;
    st.cls = (uint32_t *)d.q0;
    st.lead = d.q1;
    st.clast = d.gtab;
    st.cnt = d.gtab + d.n;
    st.key = (unsigned long long *)d.lnbuf;  // 2 x 8 bytes of a >= 256-byte array
    const dim3 grid((d.n + kStepThreads - 1) / kStepThreads), block(kStepThreads);
    ProfScope ps(0, s);
    hipLaunchKernelGGL(k_step_init, grid, block, 0, s, d, st);
    LX_CHECK_LAUNCH("per-step LexBFS init launch");
    for (int i = 0; i < d.n; ++i) {
        hipLaunchKernelGGL(k_step_count, grid, block, 0, s, d, st, i);
        if (i + 1 == d.n) break;  // nothing left to split or choose
        hipLaunchKernelGGL(k_step_assign, grid, block, 0, s, d, st, i);
        hipLaunchKernelGGL(k_step_close, grid, block, 0, s, d, st, i);
    }
    LX_CHECK_LAUNCH("per-step LexBFS launches");
    return LEXBFS_OK;
}

void sweep_shape(int wn, int &G, int &lg)
{
    G = 1;
    lg = 0;
    while (G < wn && G < kWave) {
        G <<= 1;
        ++lg;
    }
}

// Rows per sweep block: one per group of G lanes (measured: many short
// blocks stream best, 0.121 ms per 512 MiB against 0.134 with four rows per
// group and 0.256 with sixteen).
int sweep_rows_per_block(int G) { return (kSweepThreads / kWave) * (kWave / G); }

// Dynamic LDS of the certificate kernel: three bitsets of wn words.
size_t finish_lds(int wn) { return finish_lds_bytes(wn, kFinishThreads / kWave); }

// LDS of one batch team: its LexBFS state, later reused by the certificate.
size_t batch_region_bytes(int n, int team)
{
    return align_up(std::max(lds_bytes_batch(n, team), finish_lds_bytes((n + 63) / 64, team / kWave)), 16);
}

GDesc make_desc(const lexbfs_graph_t *g, char *ws, const SingleWs &L, int32_t *order, int32_t *rank,
                int32_t *parent, int32_t *cycle, lexbfs_result_t *res)
{
    GDesc d;
    d.n = g->n;
    d.wn = (g->n + 63) / 64;
    d.W = g->words_per_row;
    d.rp = g->row_ptr;
    d.ci = g->col_idx;
    d.bits = g->bits;
    d.order = order ? order : (int32_t *)(ws + L.order);
    d.rank = rank ? rank : (int32_t *)(ws + L.rank);
    d.parent = parent ? parent : (int32_t *)(ws + L.parent);
    d.cycle = cycle ? cycle : (int32_t *)(ws + L.cycle);
    d.level = (int32_t *)(ws + L.level);
    d.q0 = (int32_t *)(ws + L.q0);
    d.q1 = (int32_t *)(ws + L.q1);
    d.lnbuf = (int32_t *)(ws + L.lnbuf);
    d.failkey = (uint32_t *)(ws + L.failkey);
    d.gtab = (uint32_t *)(ws + L.gtab);
    d.res = res;
    d.nnz = g->nnz;
    return d;
}

// Text of the first error bit of the input check.
const char *egraph_text(uint32_t bad)
{
    if (bad & kBadRowPtr) return "row pointers are not non-decreasing from 0 to nnz";
    if (bad & kBadId) return "a column index lies outside 0..n-1";
    if (bad & kSelfLoop) return "a vertex is listed in its own row (self-loop)";
    if (bad & kUnsorted) return "a CSR row is not strictly ascending (unsorted or duplicate entry)";
    if (bad & kNotInBits) return "a CSR entry is missing from the bitset";
    if (bad & kAsym) return "the adjacency is not symmetric";
    if (bad & kExtraBits) return "the bitset holds entries the CSR lacks (or bits at or above n)";
    return "graph violates the input contract";
}

// The input check of one graph, run to completion before returning (the
// verdict is needed on the host): LEXBFS_OK or LEXBFS_EGRAPH. `status` is
// one device word of the caller's workspace.
int check_graph_single(const GDesc &d, uint32_t *status, hipStream_t s)
{
    if (d.n <= 0) return LEXBFS_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, status, 1, 0u);
    const int blocks = std::max(1, std::min((d.n + 3) / 4, 2048));
    hipLaunchKernelGGL(k_validate_one, dim3(blocks), dim3(kValidateThreads), 0, s, d, status);
    LX_CHECK_LAUNCH("input check launch");
    uint32_t h = 0;
    hipError_t e = hipMemcpyAsync(&h, status, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "reading the input check");
    if (h) return fail_code(LEXBFS_EGRAPH, egraph_text(h));
    return LEXBFS_OK;
}

// Batch plan kept in the workspace.
struct BatchWs {
    size_t qctr, gds, sorted, failkeys, status, arrays, total;
};

// Largest n of the 256-lane tier (state in one workgroup's LDS).
int batch_tier_max_n(size_t lim)
{
    int lo = 0, hi = 64 * kBatchThreads;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (batch_region_bytes(mid, kBatchThreads) <= lim) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Per-graph arrays: order, rank, parent, cycle, level, q0, q1, lnbuf, and
// for graphs too large for any 256-lane team two more for class tables in
// global memory (used when even the compact LDS layout does not fit).
int batch_arrays(int n) { return n > 64 * kBatchThreads ? 10 : 8; }

BatchWs batch_layout(const lexbfs_graph_t *gs, int32_t count)
{
    BatchWs L;
    size_t off = 0;
    size_t arrays = 0;
    for (int i = 0; i < count; ++i) {
        const int n = gs[i].n;
        arrays += (size_t)batch_arrays(n) * al((size_t)(n > 0 ? n : 1) * 4);
    }
    L.qctr = off; off += kAlign;
    L.gds = off; off += al(sizeof(GDesc) * (size_t)count);
    L.sorted = off; off += al(4 * (size_t)count);
    L.failkeys = off; off += al(4 * (size_t)count);
    L.status = off; off += al(4 * (size_t)count);
    L.arrays = off; off += arrays;
    L.total = off;
    return L;
}

// Launch of the bitset builder over n rows of W words each.
int launch_build_bitset(int n, const int32_t *rp, const int32_t *ci, uint64_t *bits, int64_t W, hipStream_t s)
{
    const size_t lds = (size_t)(kBuildThreads / kWave) * 8 * (size_t)W;
    const size_t lim = dynamic_lds_limit(k_build_bitset);
    if (!lim) return fail_code(LEXBFS_EHIP, "querying or raising the bitset builder's LDS limit failed");
    if (lds > lim) return fail_code(LEXBFS_ETOOBIG, "bitset row buffers do not fit the workgroup LDS");
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int per_block = kBuildThreads / kWave;
    const int blocks = std::max(1, std::min((n + per_block - 1) / per_block, cus * 8));
    hipLaunchKernelGGL(k_build_bitset, dim3(blocks), dim3(kBuildThreads), lds, s, n, rp, ci, bits, W);
    LX_CHECK_LAUNCH("bitset builder launch");
    return LEXBFS_OK;
}

// Workspace of one LexBFS+ sweep: validity flag, pos, padded degrees, the
// renamed CSR and bitset, then a single-graph LexBFS workspace (which also
// holds the renamed order and parents).
struct PlusWs {
    size_t flag, pos, deg, rp2, ci2, bits2, lex, total;
};

int plus_pad(int n) { return (std::max(n, 1) + kPlusPerLane - 1) / kPlusPerLane * kPlusPerLane; }

PlusWs plus_layout(int n, int64_t nnz)
{
    PlusWs P;
    const size_t m = (size_t)std::max(n, 1);
    const size_t wn = (m + 63) / 64;
    size_t off = 0;
    P.flag = off; off += kAlign;
    P.pos = off; off += al(m * 4);
    P.deg = off; off += al((size_t)plus_pad(n) * 4);
    P.rp2 = off; off += al((m + 1) * 4);
    P.ci2 = off; off += al((size_t)std::max<int64_t>(nnz, 1) * 4);
    P.bits2 = off; off += al(m * wn * 8);
    P.lex = off; off += single_layout(n).total;
    P.total = off;
    return P;
}

// Workspace of the unit interval test: the first two orders, the third
// order (when the caller keeps none) and its ranks, the failure key, then
// a LexBFS+ sweep workspace (its LexBFS part also serves the first sweep).
struct UiWs {
    size_t key, s1, s2, s3, rank3, plus, total;
};

UiWs ui_layout(int n, int64_t nnz)
{
    UiWs U;
    const size_t a = al((size_t)std::max(n, 1) * 4);
    size_t off = 0;
    U.key = off; off += kAlign;
    U.s1 = off; off += a;
    U.s2 = off; off += a;
    U.s3 = off; off += a;
    U.rank3 = off; off += a;
    U.plus = off; off += plus_layout(n, nnz).total;
    U.total = off;
    return U;
}

// One LexBFS+ sweep of g after the order prev (all device pointers; rank
// and parent may be null). The interval key, when given, is reset with the
// sweep's other state.
int plus_sweep(const lexbfs_graph_t *g, const int32_t *prev, int32_t *order, int32_t *rank, int32_t *parent,
               char *ws, uint32_t *key, hipStream_t s)
{
    const int n = g->n;
    const PlusWs P = plus_layout(n, g->nnz);
    int32_t *flag = (int32_t *)(ws + P.flag);
    int32_t *pos = (int32_t *)(ws + P.pos);
    int32_t *deg = (int32_t *)(ws + P.deg);
    int32_t *rp2 = (int32_t *)(ws + P.rp2);
    int32_t *ci2 = (int32_t *)(ws + P.ci2);
    uint64_t *bits2 = (uint64_t *)(ws + P.bits2);
    const int blocks = (n + kPlusThreads - 1) / kPlusThreads;
    const int npad = plus_pad(n);
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    // The renamed graph's ids follow the kernel's interleaved tie order where
    // its LDS form supports one, so that a pivot's neighbours (close together
    // in the previous order) do not all land on one lane.
    const int ik = single_ilv_k(n);
    if (ik < 0) return ik;
    {
        ProfScope ps(3, s);
        hipLaunchKernelGGL(k_plus_init, dim3(blocks), dim3(kPlusThreads), 0, s, n, pos, flag, key);
        hipLaunchKernelGGL(k_plus_inverse, dim3(blocks), dim3(kPlusThreads), 0, s, n, prev, pos, flag);
        hipLaunchKernelGGL(k_plus_degree, dim3((npad + kPlusThreads - 1) / kPlusThreads), dim3(kPlusThreads), 0, s,
                           n, npad, prev, g->row_ptr, (const int32_t *)flag, deg, ik);
        hipLaunchKernelGGL(k_plus_scan, dim3(1), dim3(kPlusScanThreads), 0, s, n, (const int32_t *)deg, rp2);
        const int rblocks = std::max(1, std::min((n + 3) / 4, cus * 8));
        const size_t rlds = (size_t)(kPlusThreads / kWave) * 8 * (size_t)rename_buffer_words((n + 63) / 64);
        hipLaunchKernelGGL(k_plus_rows, dim3(rblocks), dim3(kPlusThreads), rlds, s, n, g->nnz, prev,
                           (const int32_t *)pos, g->row_ptr, g->col_idx, (const int32_t *)flag, (const int32_t *)rp2,
                           ci2, bits2, ik);
        LX_CHECK_LAUNCH("LexBFS+ renaming launches");
    }
    lexbfs_graph_t g2;
    g2.n = n;
    g2.reserved = 0;
    g2.nnz = g->nnz;
    g2.row_ptr = rp2;
    g2.col_idx = ci2;
    g2.bits = bits2;
    g2.words_per_row = (n + 63) / 64;
    const GDesc d = make_desc(&g2, ws + P.lex, single_layout(n), nullptr, nullptr, nullptr, nullptr, nullptr);
    int rc = launch_lexbfs_single(d, s, ik > 0);
    if (rc) return rc;
    {
        ProfScope ps(3, s);
        hipLaunchKernelGGL(k_plus_map, dim3(blocks), dim3(kPlusThreads), 0, s, n, prev, (const int32_t *)d.order,
                           (const int32_t *)d.parent, (const int32_t *)flag, order, rank, parent, ik);
    }
    LX_CHECK_LAUNCH("LexBFS+ order launch");
    return LEXBFS_OK;
}

}  // namespace

// A prepared batch: the descriptor table lives in the workspace; the host
// keeps the launch shape.
struct lexbfs_batch_plan {
    int count = 0;
    uint32_t flags = 0;
    char *ws = nullptr;
    BatchWs L{};
    std::vector<char> table;
    int nbig = 0;    // graphs on 256-lane workgroup teams
    int nsmall = 0;  // graphs on wavefront teams
    int nlarge = 0;  // graphs on the large tier (side streams): 1024-lane workgroups first, then 512-lane ones
    int nlarge_mid = 0;  // of which on 512-lane workgroups
    std::vector<int32_t> ilv_k;  // per graph: K of its team when its ties use the interleaved order, else 0
    bool interleaved = false;    // launch the interleaved-tie batch kernel
    size_t lds = 0;
    size_t lds_large = 0;      // dynamic LDS of the 1024-lane kernel
    size_t lds_large_mid = 0;  // and of the 512-lane kernel
    int region = 0;
    int blocks = 1;
    hipStream_t side = nullptr, side2 = nullptr;  // side2: the 512-lane kernel when both sizes run
    hipEvent_t fork = nullptr, join = nullptr, join2 = nullptr;
    ~lexbfs_batch_plan()
    {
        if (side) (void)hipStreamSynchronize(side);
        if (side2) (void)hipStreamSynchronize(side2);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (join2) (void)hipEventDestroy(join2);
        if (side) (void)hipStreamDestroy(side);
        if (side2) (void)hipStreamDestroy(side2);
    }
};

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int lexbfs_abi_version(void) { return kAbiVersion; }

const char *lexbfs_last_error(void) { return t_last_error; }

int lexbfs_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (on && !g_prof.created) {
        for (int i = 0; i < 2 * kProfPairs; ++i) {
            const hipError_t e = hipEventCreate(&g_prof.ev[i]);
            if (e != hipSuccess) return fail_hip(e, "creating timing events");
        }
        g_prof.created = true;
    }
    g_prof.on = on != 0;
    return LEXBFS_OK;
}

int lexbfs_profile_collect(int32_t *counts, double *ms)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (int k = 0; k < kKinds; ++k) {
        if (counts) counts[k] = 0;
        if (ms) ms[k] = 0.0;
    }
    for (int i = 0; i < g_prof.used; ++i) {
        hipError_t e = hipEventSynchronize(g_prof.ev[2 * i + 1]);
        if (e != hipSuccess) return fail_hip(e, "waiting for a timing event");
        float t = 0.f;
        e = hipEventElapsedTime(&t, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]);
        if (e != hipSuccess) return fail_hip(e, "reading a timing event");
        const int k = g_prof.kind[i];
        if (counts) counts[k] += 1;
        if (ms) ms[k] += t;
    }
    const int dropped = g_prof.dropped;
    g_prof.used = 0;
    g_prof.dropped = 0;
    return dropped;
}

const char *lexbfs_strerror(int code)
{
    switch (code) {
        case LEXBFS_OK: return "ok";
        case LEXBFS_EINVAL: return "invalid argument";
        case LEXBFS_ENOWS: return "workspace missing or too small";
        case LEXBFS_EHIP: return "HIP runtime or launch failure";
        case LEXBFS_EGRAPH: return "graph violates the input contract";
        case LEXBFS_ETOOBIG: return "graph too large for this device or library";
        default: return "unknown error";
    }
}

size_t lexbfs_workspace_bytes(int32_t n) { return single_layout(n < 0 ? 0 : n).total; }

int lexbfs_order(const lexbfs_graph_t *g, int32_t *order, int32_t *rank, int32_t *parent, void *ws,
                 size_t ws_bytes, void *stream)
{
    int rc = validate_graph(g);
    if (rc) return rc;
    if (!order && g->n > 0) return LEXBFS_EINVAL;
    const SingleWs L = single_layout(g->n);
    if (!ws || ws_bytes < L.total) return LEXBFS_ENOWS;
    if (g->n == 0) return LEXBFS_OK;
    const GDesc d = make_desc(g, (char *)ws, L, order, rank, parent, nullptr, nullptr);
    return launch_lexbfs_single(d, (hipStream_t)stream);
}

int lexbfs_validate(const lexbfs_graph_t *g, void *ws, size_t ws_bytes, void *stream)
{
    const int rc = validate_graph(g);
    if (rc) return rc;
    if (g->n == 0) return LEXBFS_OK;
    if (!ws || ws_bytes < kAlign) return LEXBFS_ENOWS;
    const GDesc d = make_desc(g, (char *)ws, single_layout(g->n), nullptr, nullptr, nullptr, nullptr, nullptr);
    return check_graph_single(d, (uint32_t *)ws, (hipStream_t)stream);
}

int chordal_test(const lexbfs_graph_t *g, lexbfs_result_t *res, const lexbfs_outputs_t *out, void *ws,
                 size_t ws_bytes, uint32_t flags, void *stream)
{
    int rc = validate_graph(g);
    if (rc) return rc;
    if (!res) return LEXBFS_EINVAL;
    const SingleWs L = single_layout(g->n);
    if (!ws || ws_bytes < L.total) return LEXBFS_ENOWS;
    hipStream_t s = (hipStream_t)stream;
    const GDesc d = make_desc(g, (char *)ws, L, out ? out->order : nullptr, out ? out->rank : nullptr,
                              out ? out->parent : nullptr, out ? out->cycle : nullptr, res);
    if ((flags & LEXBFS_FLAG_PER_STEP) && (flags & LEXBFS_FLAG_MCS))
        return fail_code(LEXBFS_EINVAL, "the per-step form exists for LexBFS only");
    if (flags & LEXBFS_FLAG_VALIDATE) {
        rc = check_graph_single(d, (uint32_t *)((char *)ws + L.failkey + 64), s);
        if (rc) return rc;
    }
    if (g->n > 0) {
        rc = (flags & LEXBFS_FLAG_MCS)        ? launch_mcs_single(d, s)
             : (flags & LEXBFS_FLAG_PER_STEP) ? launch_lexbfs_per_step(d, s)
                                              : launch_lexbfs_single(d, s);
        if (rc) return rc;
        int G, lg;
        sweep_shape(d.wn, G, lg);
        const int rpb = sweep_rows_per_block(G);
        {
            ProfScope ps(1, s);
            hipLaunchKernelGGL(k_sweep_single, dim3((d.n + rpb - 1) / rpb), dim3(kSweepThreads), 0, s, d, rpb, G, lg);
        }
        LX_CHECK_LAUNCH("sweep launch");
    }
    {
        ProfScope ps(2, s);
        if (d.wn > kWave)
            hipLaunchKernelGGL(k_finish_single<kLargeThreads>, dim3(1), dim3(kLargeThreads),
                               finish_lds_bytes(d.wn, kLargeThreads / kWave), s, d, flags);
        else
            hipLaunchKernelGGL(k_finish_single<kFinishThreads>, dim3(1), dim3(kFinishThreads), finish_lds(d.wn), s, d,
                               flags);
    }
    LX_CHECK_LAUNCH("certificate launch");
    return LEXBFS_OK;
}

size_t lexbfs_batch_workspace_bytes(const lexbfs_graph_t *gs, int32_t count)
{
    if (!gs || count <= 0) return kAlign;
    return batch_layout(gs, count).total;
}

namespace {
// The input check of every graph of a batch (descriptors already staged at
// dg), run to completion: LEXBFS_OK or LEXBFS_EGRAPH naming the first bad
// graph.
int check_graphs_batch(const lexbfs_graph_t *gs, int32_t count, const GDesc *dg, uint32_t *status, hipStream_t s)
{
    int maxn = 0;
    for (int i = 0; i < count; ++i) maxn = std::max(maxn, gs[i].n);
    if (maxn == 0) return LEXBFS_OK;
    const int bpg = std::max(1, std::min((maxn + 63) / 64, 16));  // blocks per graph
    hipLaunchKernelGGL(k_fill_u32, dim3((count + 255) / 256), dim3(256), 0, s, status, count, 0u);
    hipLaunchKernelGGL(k_validate_batch, dim3((unsigned)count * (unsigned)bpg), dim3(kValidateThreads), 0, s, dg,
                       count, bpg, status);
    LX_CHECK_LAUNCH("batch input check launch");
    std::vector<uint32_t> h((size_t)count);
    hipError_t e = hipMemcpyAsync(h.data(), status, 4 * (size_t)count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "reading the batch input check");
    for (int i = 0; i < count; ++i)
        if (h[i]) {
            snprintf(t_last_error, sizeof t_last_error, "graph %d: %s", i, egraph_text(h[i]));
            return LEXBFS_EGRAPH;
        }
    return LEXBFS_OK;
}

// interleave: graphs on wavefront and 256-lane teams break ties by the
// interleaved rank (ilv_rank) instead of the id; plan->ilv_k records their K.
int plan_create(const lexbfs_graph_t *gs, int32_t count, const lexbfs_outputs_t *outs, lexbfs_result_t *res,
                const lexbfs_tuning_t *tuning, void *ws, size_t ws_bytes, uint32_t flags, void *stream,
                bool side_stream, lexbfs_batch_plan_t **plan_out, bool interleave = false)
{
    if (!plan_out) return LEXBFS_EINVAL;
    *plan_out = nullptr;
    if (count < 0 || (count > 0 && (!gs || !res))) return LEXBFS_EINVAL;
    constexpr int BT = kBatchThreads;
    int wave_max_n = 1024;
    if (tuning) {
        if (tuning->block_threads != 0 && tuning->block_threads != BT) return LEXBFS_EINVAL;
        if (tuning->wave_max_n > 0) wave_max_n = tuning->wave_max_n;
        if (tuning->wave_max_n < 0) wave_max_n = 0;  // every graph on a workgroup
    }
    for (int i = 0; i < count; ++i) {
        const int rc = validate_graph(&gs[i]);
        if (rc) return rc;
    }
    const BatchWs L = batch_layout(gs, count);
    if (!ws || ws_bytes < L.total) return LEXBFS_ENOWS;
    if (count == 0) {
        lexbfs_batch_plan_t *P = new (std::nothrow) lexbfs_batch_plan_t();
        if (!P) return fail_code(LEXBFS_EINVAL, "out of host memory for the batch plan");
        *plan_out = P;
        return LEXBFS_OK;
    }
    const bool mcs = (flags & LEXBFS_FLAG_MCS) != 0;
    const size_t maxl = mcs ? dynamic_lds_limit(k_batch<BT, true>) : dynamic_lds_limit(k_batch<BT, false>);
    const size_t maxl_large = mcs ? dynamic_lds_limit(k_batch_large<kLargeThreads, true>)
                                  : dynamic_lds_limit(k_batch_large<kLargeThreads, false>);
    const size_t maxl_mid = mcs ? dynamic_lds_limit(k_batch_large<kLargeMidThreads, true>)
                                : dynamic_lds_limit(k_batch_large<kLargeMidThreads, false>);
    if (!maxl || !maxl_large || !maxl_mid)
        return fail_code(LEXBFS_EHIP, "querying or raising the batch kernels' LDS limits failed");
    const int tier_max = batch_tier_max_n(maxl);
    wave_max_n = std::min(wave_max_n, 64 * kWave);  // one lane owns at most 64 vertices
    // Every wave of a workgroup needs its own region: keep the wave
    // threshold where four regions fit the LDS of one workgroup.
    while (wave_max_n > 64 && (size_t)(BT / kWave) * batch_region_bytes(wave_max_n, kWave) > maxl) wave_max_n -= 64;
    int maxn_block = 0, maxn_wave = 0;
    for (int i = 0; i < count; ++i) {
        const int n = gs[i].n;
        if (n > tier_max) {
            const int T = n <= kLargeMidMaxN ? kLargeMidThreads : kLargeThreads;
            const size_t lim = n <= kLargeMidMaxN ? maxl_mid : maxl_large;
            if (!mcs && lds_bytes_lds_tables(n, T) > lim && lds_bytes_compact(n, T) > lim &&
                lds_bytes_global_tables(n, T) > lim)
                return fail_code(LEXBFS_ETOOBIG, "a batch graph's state does not fit the workgroup LDS");
            if (mcs && lds_bytes_mcs(n, T, false) > lim)
                return fail_code(LEXBFS_ETOOBIG, "a batch graph's MCS state does not fit the workgroup LDS");
        } else if (n > wave_max_n) {
            maxn_block = std::max(maxn_block, n);
        } else {
            maxn_wave = std::max(maxn_wave, n);
        }
    }
    const size_t region = maxn_wave > 0 ? batch_region_bytes(maxn_wave, kWave) : 0;
    size_t lds = std::max(batch_region_bytes(std::max(maxn_block, 1), BT), region * (BT / kWave));
    if (tuning && tuning->lds_bytes > 0) lds = std::max(lds, (size_t)tuning->lds_bytes);
    if (lds > maxl) return fail_code(LEXBFS_ETOOBIG, "batch graph state does not fit the workgroup LDS");
    lexbfs_batch_plan_t *P = new (std::nothrow) lexbfs_batch_plan_t();
    if (!P) return fail_code(LEXBFS_EINVAL, "out of host memory for the batch plan");
    P->count = count;
    P->flags = flags & ~kFlagOrderOnly;
    P->ws = (char *)ws;
    P->L = L;
    char *w = (char *)ws;

    // Host plan: descriptors; the order is workgroup-team graphs, then
    // wavefront-team graphs, then graphs of the 1024-lane tier, each part
    // longest first.
    P->table.resize(L.failkeys - L.gds);
    GDesc *hd = (GDesc *)P->table.data();
    int32_t *hsorted = (int32_t *)(P->table.data() + (L.sorted - L.gds));
    size_t aoff = L.arrays;
    for (int i = 0; i < count; ++i) {
        const lexbfs_graph_t &g = gs[i];
        const size_t a = al((size_t)(g.n > 0 ? g.n : 1) * 4);
        GDesc &d = hd[i];
        d.n = g.n;
        d.wn = (g.n + 63) / 64;
        d.W = g.words_per_row;
        d.rp = g.row_ptr;
        d.ci = g.col_idx;
        d.bits = g.bits;
        const lexbfs_outputs_t *o = outs ? &outs[i] : nullptr;
        d.order = (o && o->order) ? o->order : (int32_t *)(w + aoff);
        aoff += a;
        d.rank = (o && o->rank) ? o->rank : (int32_t *)(w + aoff);
        aoff += a;
        d.parent = (o && o->parent) ? o->parent : (int32_t *)(w + aoff);
        aoff += a;
        d.cycle = (o && o->cycle) ? o->cycle : (int32_t *)(w + aoff);
        aoff += a;
        d.level = (int32_t *)(w + aoff);
        aoff += a;
        d.q0 = (int32_t *)(w + aoff);
        aoff += a;
        d.q1 = (int32_t *)(w + aoff);
        aoff += a;
        d.lnbuf = (int32_t *)(w + aoff);
        aoff += a;
        d.gtab = nullptr;
        if (batch_arrays(g.n) == 10) {
            d.gtab = (uint32_t *)(w + aoff);
            aoff += 2 * a;
        }
        d.failkey = (uint32_t *)(w + L.failkeys) + i;
        d.res = res + i;
        d.nnz = g.nnz;
        hsorted[i] = i;
    }
    auto tier = [&](int i) { return gs[i].n > tier_max ? 2 : gs[i].n > wave_max_n ? 0 : 1; };
    std::stable_sort(hsorted, hsorted + count, [&](int a, int b) {
        const int ta = tier(a), tb = tier(b);
        return ta != tb ? ta < tb : gs[a].n > gs[b].n;
    });
    int nbig = 0, nsmall = 0;
    for (int k = 0; k < count; ++k) {
        const int t = tier(hsorted[k]);
        nbig += t == 0;
        nsmall += t == 1;
    }
    P->ilv_k.assign(count, 0);
    P->interleaved = interleave;
    if (interleave)
        for (int i = 0; i < count; ++i) {
            const int t = tier(i);
            if (t == 2 || gs[i].n == 0) continue;
            const int T = t == 0 ? BT : kWave;
            int K = 1;
            while (K * T < gs[i].n) K <<= 1;  // the team's vertices per lane, as lexbfs_team computes it
            P->ilv_k[i] = K;
        }
    P->nbig = nbig;
    P->nsmall = nsmall;
    P->nlarge = count - nbig - nsmall;
    for (int k = nbig + nsmall; k < count; ++k) P->nlarge_mid += gs[hsorted[k]].n <= kLargeMidMaxN;
    P->lds = lds;
    P->lds_large = maxl_large;
    P->lds_large_mid = maxl_mid;
    P->region = (int)region;
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int per_cu = std::max(1, (int)((size_t)device_max_lds() / lds));
    P->blocks = std::max(1, std::min(cus * per_cu, std::max(nbig, (nsmall + 3) / 4)));
    const bool both_large = P->nlarge_mid > 0 && P->nlarge_mid < P->nlarge;
    if (P->nlarge > 0 && (nbig + nsmall > 0 || both_large) && side_stream) {
        // The large tier runs on streams of the plan (one per team size),
        // forked from and joined back into the caller's stream at every
        // launch.
        if (hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&P->fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&P->join, hipEventDisableTiming) != hipSuccess ||
            (both_large && (hipStreamCreateWithFlags(&P->side2, hipStreamNonBlocking) != hipSuccess ||
                            hipEventCreateWithFlags(&P->join2, hipEventDisableTiming) != hipSuccess))) {
            delete P;
            return fail_code(LEXBFS_EHIP, "creating the batch plan's streams and events");
        }
    }
    const hipError_t e =
        hipMemcpyAsync(w + L.gds, P->table.data(), P->table.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) {
        delete P;
        return fail_hip(e, "staging the batch plan");
    }
    if (flags & LEXBFS_FLAG_VALIDATE) {
        const int rc = check_graphs_batch(gs, count, (const GDesc *)(w + L.gds), (uint32_t *)(w + L.status),
                                          (hipStream_t)stream);
        if (rc) {
            delete P;
            return rc;
        }
    }
    *plan_out = P;
    return LEXBFS_OK;
}
// Workspace of a batched unit interval test: two batch plans (original and
// renamed graphs, same sizes), scratch verdicts of the plans, the interval
// descriptors, then per graph its three orders, ranks, pos, renamed CSR and
// bitset, flag and key.
struct UiBatchWs {
    BatchWs plan;
    size_t planA, planB, pres, idesc, total;
    std::vector<size_t> graph;
};

size_t ui_graph_bytes(int n, int64_t nnz)
{
    const size_t m = (size_t)std::max(n, 1);
    return 5 * al(m * 4) + al((m + 1) * 4) + al((size_t)std::max<int64_t>(nnz, 1) * 4) + al(m * ((m + 63) / 64) * 8) +
           kAlign;
}

// (Fills U rather than returning it: this part of the file has C linkage.)
void ui_batch_layout(const lexbfs_graph_t *gs, int32_t count, UiBatchWs &U)
{
    U.plan = batch_layout(gs, count);
    size_t off = 0;
    U.planA = off; off += U.plan.total;
    U.planB = off; off += U.plan.total;
    U.pres = off; off += al(sizeof(lexbfs_result_t) * (size_t)count);
    U.idesc = off; off += al(sizeof(IDesc) * (size_t)count);
    U.graph.resize(count);
    for (int i = 0; i < count; ++i) {
        U.graph[i] = off;
        off += ui_graph_bytes(gs[i].n, gs[i].nnz);
    }
    U.total = off;
}

// Owns the two plans of one batched call.
struct PlanPair {
    lexbfs_batch_plan_t *a = nullptr, *b = nullptr;
    ~PlanPair()
    {
        delete a;
        delete b;
    }
};

int ui_batch_run(const lexbfs_graph_t *gs, int32_t count, lexbfs_interval_result_t *res, int32_t *const *orders,
                 char *w, const UiBatchWs &U, hipStream_t s)
{
    std::vector<IDesc> hd(count);
    std::vector<lexbfs_graph_t> g2(count);
    std::vector<lexbfs_outputs_t> oa(count);
    int maxn = 0, bufw = 1;
    for (int i = 0; i < count; ++i) {
        const lexbfs_graph_t &g = gs[i];
        const size_t m = (size_t)std::max(g.n, 1);
        const size_t a = al(m * 4);
        char *p = w + U.graph[i];
        IDesc &d = hd[i];
        d.n = g.n;
        d.wn = (g.n + 63) / 64;
        d.nnz = g.nnz;
        d.W = g.words_per_row;
        d.rp = g.row_ptr;
        d.ci = g.col_idx;
        d.bits = g.bits;
        d.s1 = (int32_t *)p; p += a;
        d.s2 = (int32_t *)p; p += a;
        d.s3 = (orders && orders[i]) ? orders[i] : (int32_t *)p; p += a;
        d.rank3 = (int32_t *)p; p += a;
        d.pos = (int32_t *)p; p += a;
        d.rp2 = (int32_t *)p; p += al((m + 1) * 4);
        d.ci2 = (int32_t *)p; p += al((size_t)std::max<int64_t>(g.nnz, 1) * 4);
        d.bits2 = (uint64_t *)p; p += al(m * ((m + 63) / 64) * 8);
        d.flag = (int32_t *)p;
        d.key = (uint32_t *)(p + 4);
        d.res = res + i;
        lexbfs_graph_t &r = g2[i];
        r.n = g.n;
        r.reserved = 0;
        r.nnz = g.nnz;
        r.row_ptr = d.rp2;
        r.col_idx = d.ci2;
        r.bits = d.bits2;
        r.words_per_row = std::max(d.wn, 1);
        oa[i].order = d.s1;
        oa[i].rank = oa[i].parent = oa[i].cycle = nullptr;
        maxn = std::max(maxn, g.n);
        bufw = std::max(bufw, rename_buffer_words(std::max(d.wn, 1)));
    }
    lexbfs_result_t *pres = (lexbfs_result_t *)(w + U.pres);
    PlanPair pp;
    int rc = plan_create(gs, count, oa.data(), pres, nullptr, w + U.planA, U.plan.total, 0, s, false, &pp.a);
    if (rc) return rc;
    // The renamed graphs' ties go to the interleaved rank: the renaming below
    // gives rank order to the previous order reversed, and consecutive ranks
    // land on different lanes (ids in that order would put a pivot's
    // neighbours, which are close in it, on one lane).
    rc = plan_create(g2.data(), count, nullptr, pres, nullptr, w + U.planB, U.plan.total, 0, s, false, &pp.b, true);
    if (rc) return rc;
    pp.a->flags |= kFlagOrderOnly;
    pp.b->flags |= kFlagOrderOnly;
    for (int i = 0; i < count; ++i) hd[i].ik = pp.b->ilv_k[i];
    // The interleaved-tie batch kernel has the same LDS layout; raise its limit.
    if (dynamic_lds_limit(k_batch<kBatchThreads, false, true>) < pp.b->lds)
        return fail_code(LEXBFS_EHIP, "raising the interleaved batch kernel's LDS limit failed");
    const IDesc *dd = (const IDesc *)(w + U.idesc);
    const hipError_t e = hipMemcpyAsync(w + U.idesc, hd.data(), sizeof(IDesc) * (size_t)count, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail_hip(e, "staging the interval descriptors");
    const GDesc *renamed = (const GDesc *)(w + U.planB + U.plan.gds);
    const int spread = std::max(1, 65536 / count);  // workgroups per graph for the row-parallel kernels
    const int ybits = std::max(1, std::min((maxn + 63) / 64, spread));
    const int ycheck = std::max(1, std::min((maxn + kIbThreads - 1) / kIbThreads, spread));
    rc = lexbfs_batch_plan_launch(pp.a, s);
    if (rc) return rc;
    for (int sel = 1; sel <= 2; ++sel) {
        {
            ProfScope ps(3, s);
            hipLaunchKernelGGL(k_ib_rename, dim3(count), dim3(kIbThreads), 0, s, dd, sel);
            hipLaunchKernelGGL(k_ib_rows, dim3(count, ybits), dim3(kBuildThreads),
                               (size_t)(kBuildThreads / kWave) * 8 * (size_t)bufw, s, dd, sel, bufw);
        }
        LX_CHECK_LAUNCH("batched LexBFS+ renaming launches");
        rc = lexbfs_batch_plan_launch(pp.b, s);
        if (rc) return rc;
        {
            ProfScope ps(3, s);
            hipLaunchKernelGGL(k_ib_map, dim3(count), dim3(kIbThreads), 0, s, dd, renamed, sel + 1);
        }
        LX_CHECK_LAUNCH("batched LexBFS+ order launch");
    }
    {
        ProfScope ps(1, s);
        hipLaunchKernelGGL(k_ib_check, dim3(count, ycheck), dim3(kIbThreads), 0, s, dd);
    }
    {
        ProfScope ps(2, s);
        hipLaunchKernelGGL(k_ib_witness, dim3(count), dim3(kIbThreads), 0, s, dd);
    }
    LX_CHECK_LAUNCH("batched interval check launches");
    return LEXBFS_OK;
}

}  // namespace

int lexbfs_batch_plan_create(const lexbfs_graph_t *gs, int32_t count, const lexbfs_outputs_t *outs,
                             lexbfs_result_t *res, const lexbfs_tuning_t *tuning, void *ws, size_t ws_bytes,
                             uint32_t flags, void *stream, lexbfs_batch_plan_t **plan_out)
{
    return plan_create(gs, count, outs, res, tuning, ws, ws_bytes, flags, stream, true, plan_out);
}

int lexbfs_batch_plan_launch(const lexbfs_batch_plan_t *P, void *stream)
{
    if (!P) return LEXBFS_EINVAL;
    if (P->count == 0) return LEXBFS_OK;
    constexpr int BT = kBatchThreads;
    hipStream_t s = (hipStream_t)stream;
    char *w = P->ws;
    const GDesc *dg = (const GDesc *)(w + P->L.gds);
    const int32_t *sorted = (const int32_t *)(w + P->L.sorted);
    uint32_t *qctr = (uint32_t *)(w + P->L.qctr);
    {
        ProfScope ps(3, s);
        hipLaunchKernelGGL(k_batch_init, dim3((P->count + 255) / 256), dim3(256), 0, s, dg, P->count, qctr);
    }
    LX_CHECK_LAUNCH("batch init launch");
    if (P->nlarge > 0) {
        // 1024-lane graphs (n above kLargeMidMaxN) come first in `sorted`,
        // then 512-lane ones; each size has its own kernel and, when both
        // run, its own stream.
        const int nl_big = P->nlarge - P->nlarge_mid;
        const int32_t *first = sorted + P->nbig + P->nsmall;
        hipStream_t ls = s, ls_mid = s;
        if (P->side) {
            hipError_t e = hipEventRecord(P->fork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(P->side, P->fork, 0);
            if (e == hipSuccess && P->side2) e = hipStreamWaitEvent(P->side2, P->fork, 0);
            if (e != hipSuccess) return fail_hip(e, "forking the large-graph streams");
            ls = P->side;
            ls_mid = P->side2 ? P->side2 : P->side;
        }
        const bool mcs = (P->flags & LEXBFS_FLAG_MCS) != 0;
        if (nl_big > 0) {
            ProfScope ps(0, ls);
            if (mcs)
                hipLaunchKernelGGL((k_batch_large<kLargeThreads, true>), dim3(nl_big), dim3(kLargeThreads),
                                   P->lds_large, ls, dg, first, P->flags, (int)P->lds_large);
            else
                hipLaunchKernelGGL((k_batch_large<kLargeThreads, false>), dim3(nl_big), dim3(kLargeThreads),
                                   P->lds_large, ls, dg, first, P->flags, (int)P->lds_large);
        }
        if (P->nlarge_mid > 0) {
            ProfScope ps(0, ls_mid);
            if (mcs)
                hipLaunchKernelGGL((k_batch_large<kLargeMidThreads, true>), dim3(P->nlarge_mid),
                                   dim3(kLargeMidThreads), P->lds_large_mid, ls_mid, dg, first + nl_big, P->flags,
                                   (int)P->lds_large_mid);
            else
                hipLaunchKernelGGL((k_batch_large<kLargeMidThreads, false>), dim3(P->nlarge_mid),
                                   dim3(kLargeMidThreads), P->lds_large_mid, ls_mid, dg, first + nl_big, P->flags,
                                   (int)P->lds_large_mid);
        }
        LX_CHECK_LAUNCH("batch large-graph launch");
        if (P->side) {
            hipError_t e = hipEventRecord(P->join, P->side);
            if (e == hipSuccess && P->side2) e = hipEventRecord(P->join2, P->side2);
            if (e != hipSuccess) return fail_hip(e, "recording the large-graph joins");
        }
    }
    if (P->nbig + P->nsmall > 0) {
        ProfScope ps(0, s);
        if (P->flags & LEXBFS_FLAG_MCS)
            hipLaunchKernelGGL((k_batch<BT, true>), dim3(P->blocks), dim3(BT), P->lds, s, dg, sorted, P->nbig,
                               P->nbig + P->nsmall, qctr, P->region, P->flags);
        else if (P->interleaved)
            hipLaunchKernelGGL((k_batch<BT, false, true>), dim3(P->blocks), dim3(BT), P->lds, s, dg, sorted,
                               P->nbig, P->nbig + P->nsmall, qctr, P->region, P->flags);
        else
            hipLaunchKernelGGL((k_batch<BT, false>), dim3(P->blocks), dim3(BT), P->lds, s, dg, sorted, P->nbig,
                               P->nbig + P->nsmall, qctr, P->region, P->flags);
    }
    LX_CHECK_LAUNCH("batch launch");
    if (P->nlarge > 0 && P->side) {
        hipError_t e = hipStreamWaitEvent(s, P->join, 0);
        if (e == hipSuccess && P->side2) e = hipStreamWaitEvent(s, P->join2, 0);
        if (e != hipSuccess) return fail_hip(e, "joining the large-graph streams");
    }
    return LEXBFS_OK;
}

void lexbfs_batch_plan_destroy(lexbfs_batch_plan_t *plan) { delete plan; }

int lexbfs_build_bitset(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, uint64_t *bits,
                        int64_t words_per_row, void *stream)
{
    if (n < 0 || n > LEXBFS_MAX_N) return n < 0 ? LEXBFS_EINVAL : LEXBFS_ETOOBIG;
    if (n == 0) return LEXBFS_OK;
    if (!row_ptr || !bits || words_per_row < (n + 63) / 64 || words_per_row > (int64_t)(LEXBFS_MAX_N / 64))
        return LEXBFS_EINVAL;
    return launch_build_bitset(n, row_ptr, col_idx, bits, words_per_row, (hipStream_t)stream);
}

size_t lexbfs_plus_workspace_bytes(int32_t n, int64_t nnz)
{
    return plus_layout(std::max(n, 0), std::max<int64_t>(nnz, 0)).total;
}

int lexbfs_plus_order(const lexbfs_graph_t *g, const int32_t *prev_order, int32_t *order, int32_t *rank,
                      int32_t *parent, void *ws, size_t ws_bytes, void *stream)
{
    if (!g) return LEXBFS_EINVAL;
    if (g->n < 0 || g->nnz < 0 || g->nnz >= (int64_t)1 << 31 || g->reserved != 0) return LEXBFS_EINVAL;
    if (g->n > LEXBFS_MAX_N) return LEXBFS_ETOOBIG;
    if (g->n == 0) return LEXBFS_OK;
    if (!g->row_ptr || (g->nnz > 0 && !g->col_idx) || !prev_order || !order) return LEXBFS_EINVAL;
    if (!ws || ws_bytes < plus_layout(g->n, g->nnz).total) return LEXBFS_ENOWS;
    return plus_sweep(g, prev_order, order, rank, parent, (char *)ws, nullptr, (hipStream_t)stream);
}

size_t unit_interval_workspace_bytes(int32_t n, int64_t nnz)
{
    return ui_layout(std::max(n, 0), std::max<int64_t>(nnz, 0)).total;
}

int unit_interval_test(const lexbfs_graph_t *g, lexbfs_interval_result_t *res, int32_t *order, void *ws,
                       size_t ws_bytes, void *stream)
{
    int rc = validate_graph(g);
    if (rc) return rc;
    if (!res) return LEXBFS_EINVAL;
    const int n = g->n;
    const UiWs U = ui_layout(n, g->nnz);
    if (!ws || ws_bytes < U.total) return LEXBFS_ENOWS;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    uint32_t *key = (uint32_t *)(w + U.key);
    int32_t *s1 = (int32_t *)(w + U.s1), *s2 = (int32_t *)(w + U.s2);
    int32_t *s3 = order ? order : (int32_t *)(w + U.s3);
    int32_t *rank3 = (int32_t *)(w + U.rank3);
    char *pw = w + U.plus;
    if (n == 0) {
        ProfScope ps(3, s);
        hipLaunchKernelGGL(k_plus_init, dim3(1), dim3(kPlusThreads), 0, s, 0, (int32_t *)nullptr,
                           (int32_t *)(pw + plus_layout(0, 0).flag), key);
        LX_CHECK_LAUNCH("interval key launch");
    } else {
        // Sweep 1: plain LexBFS, in the LexBFS part of the sweep workspace.
        const PlusWs P = plus_layout(n, g->nnz);
        const GDesc d1 = make_desc(g, pw + P.lex, single_layout(n), s1, nullptr, nullptr, nullptr, nullptr);
        rc = launch_lexbfs_single(d1, s);
        if (rc) return rc;
        rc = plus_sweep(g, s1, s2, nullptr, nullptr, pw, nullptr, s);
        if (rc) return rc;
        rc = plus_sweep(g, s2, s3, rank3, nullptr, pw, key, s);
        if (rc) return rc;
        int cus = 256, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        ProfScope ps(1, s);
        const int cblocks = std::max(1, std::min((n + 3) / 4, cus * 8));
        hipLaunchKernelGGL(k_ui_check, dim3(cblocks), dim3(kPlusThreads), 0, s, n, g->row_ptr, g->col_idx,
                           (const int32_t *)s3, (const int32_t *)rank3, key);
        LX_CHECK_LAUNCH("interval check launch");
    }
    {
        ProfScope ps(2, s);
        hipLaunchKernelGGL(k_ui_witness, dim3(1), dim3(kFinishThreads), 0, s, n, g->row_ptr, g->col_idx, g->bits,
                           g->words_per_row, (const int32_t *)s3, (const int32_t *)rank3, (const uint32_t *)key, res);
    }
    LX_CHECK_LAUNCH("interval witness launch");
    return LEXBFS_OK;
}

size_t unit_interval_batch_workspace_bytes(const lexbfs_graph_t *gs, int32_t count)
{
    if (!gs || count <= 0) return kAlign;
    UiBatchWs U;
    ui_batch_layout(gs, count, U);
    return U.total;
}

int unit_interval_test_batch(const lexbfs_graph_t *gs, int32_t count, lexbfs_interval_result_t *res,
                             int32_t *const *orders, void *ws, size_t ws_bytes, void *stream)
{
    if (count < 0 || (count > 0 && (!gs || !res))) return LEXBFS_EINVAL;
    if (count == 0) return LEXBFS_OK;
    for (int i = 0; i < count; ++i) {
        const int rc = validate_graph(&gs[i]);
        if (rc) return rc;
    }
    UiBatchWs U;
    ui_batch_layout(gs, count, U);
    if (!ws || ws_bytes < U.total) return LEXBFS_ENOWS;
    return ui_batch_run(gs, count, res, orders, (char *)ws, U, (hipStream_t)stream);
}

int32_t lexbfs_batch_max_n(void)
{
    const size_t lim = dynamic_lds_limit(k_batch<kBatchThreads, false>);
    if (!lim) return fail_code(LEXBFS_EHIP, "querying or raising the batch kernel's LDS limit failed");
    return batch_tier_max_n(lim);
}

size_t chordal_test_noalloc_max_bytes(void) { return kScratchBytes; }

int chordal_test_noalloc(const lexbfs_graph_t *g, lexbfs_result_t *res, const lexbfs_outputs_t *out, uint32_t flags,
                         void *stream)
{
    int rc = validate_graph(g);
    if (rc) return rc;
    if (!res) return LEXBFS_EINVAL;
    if (flags & LEXBFS_FLAG_VALIDATE)
        return fail_code(LEXBFS_EINVAL, "chordal_test_noalloc does not take LEXBFS_FLAG_VALIDATE (it waits on the host)");
    const size_t need = single_layout(g->n).total;
    if (need > kScratchBytes) return fail_code(LEXBFS_ETOOBIG, "graph needs more scratch than the fixed array holds");
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    // Every kernel of chordal_test sets the scratch it reads (failure key,
    // tables, queues) before reading it, so nothing is cleared here.
    return chordal_test(g, res, out, ws, kScratchBytes, flags, stream);
}

int chordal_test_batch(const lexbfs_graph_t *gs, int32_t count, const lexbfs_outputs_t *outs,
                       lexbfs_result_t *res, const lexbfs_tuning_t *tuning, void *ws, size_t ws_bytes,
                       uint32_t flags, void *stream)
{
    if (count == 0 && count >= 0) return LEXBFS_OK;
    lexbfs_batch_plan_t *P = nullptr;
    int rc = plan_create(gs, count, outs, res, tuning, ws, ws_bytes, flags, stream, false, &P);
    if (rc) return rc;
    rc = lexbfs_batch_plan_launch(P, stream);
    lexbfs_batch_plan_destroy(P);
    return rc;
}

}  // extern "C"
