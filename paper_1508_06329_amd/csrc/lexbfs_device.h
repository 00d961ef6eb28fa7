// lexbfs_device.h -- device code for the gfx950 chordality library.
//
// Three kernels make up the path (Lupinska, "A Parallel Algorithm to Test
// Chordality of Graphs"):
//
//   LexBFS   (Section 6.1, here a single persistent launch)
//   sweep    (Section 6.2 "testing": the parent-based perfect-elimination test)
//   finish   (witness and chordless-cycle certificate for failing graphs)
//
// ---------------------------------------------------------------------------
// LexBFS state: order-preserving class ids instead of a linked list of sets
// ---------------------------------------------------------------------------
// The paper keeps the sets of equal labels as a linked list ordered by label
// and inserts the set of a split directly after its parent set (Lemma 6.1,
// Observation 6.2); label strings are never compared (Section 6.3). Here the
// U unnumbered vertices occupy virtual positions [0, U); every class of
// equal labels is a contiguous position range [s, last], ranges are ordered
// by label (higher positions = larger labels), and a class is named by its
// first position s. Per vertex we keep only cls[v] = s; per class the last
// position clast[s] and a split counter cnt[s].
//
//   * Pivot: the unnumbered vertex with the largest (cls, -id) -- the
//     largest label, smallest id on ties. One max-reduction over a packed
//     32-bit key (cls << 16 | 0xFFFF - v).
//   * Removing the pivot from the top class [s, U) shrinks it to [s, U-1).
//   * Appending the step number to the labels of the pivot's unnumbered
//     neighbours splits each class C = [s, last] hit by c neighbours into
//     C \ N(x) = [s, last - c] and C & N(x) = [last - c + 1, last]: the
//     neighbours get the new id last - c + 1, directly above the remainder,
//     exactly where Observation 6.2 places the new set. If all of C is
//     adjacent (c = |C|) nothing changes. At most one new class per old
//     class (the paper's argument after Observation 6.2).
//   * Empty classes cannot occur except at the top, so the paper's
//     empty-set removal pass (Lemma 6.3) has no counterpart.
//   * Every id stays below U <= n <= 65536, so classes fit in 16 bits.
//
// The last pivot adjacent to y before y is numbered is y's latest earlier
// neighbour, so parent[y] (p(y) of Section 5.2) is recorded during the
// splits at no extra cost.
//
// Threads own vertex chunks: with a team of T lanes and chunk size K (a
// power of two, K*T >= n, K <= 64), lane t owns vertices [t*K, t*K + K).
// Each step a lane reads its K bits of the pivot's bitset row, handles its
// own neighbours, and reduces the key over its own unnumbered vertices.
//
// A team is either one 64-lane wavefront (batched small graphs) or a whole
// workgroup (large graphs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lxd {

constexpr int kWave = 64;
constexpr uint32_t kNoFail = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Wave reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, kWave));
    return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off, kWave));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off, kWave);
    return v;
}

__device__ __forceinline__ int ctz64(uint64_t x) { return __builtin_ctzll(x); }

// ---------------------------------------------------------------------------
// Agent-scope accessors for scratch tables in global memory. Waves of one
// workgroup share a CU but global atomics complete in L2, so plain loads
// could see a stale L1 line; every access goes to L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t g_load(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_store(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t g_load_i(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_store_i(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Teams
// ---------------------------------------------------------------------------
struct WaveTeam {
    int tid;  // lane
    static constexpr int kSize = kWave;
    __device__ __forceinline__ void sync() const
    {
        // LDS operations of one wave complete in issue order; this only has to
        // stop the compiler from moving memory operations across the point.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __device__ __forceinline__ uint32_t max_all(uint32_t v, uint32_t *) const { return wave_max_u32(v); }
    __device__ __forceinline__ void step_end() const { sync(); }
};

template <int T, bool kGlobalTables>
struct BlockTeam {
    int tid;
    static constexpr int kSize = T;
    __device__ __forceinline__ void sync() const
    {
        if (kGlobalTables) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (kGlobalTables) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    // Max over the team; every lane gets the result. red: T/64 LDS words.
    __device__ __forceinline__ uint32_t max_all(uint32_t v, uint32_t *red) const
    {
        v = wave_max_u32(v);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        sync();
        uint32_t r = red[0];
#pragma unroll
        for (int k = 1; k < T / kWave; ++k) r = max(r, red[k]);
        return r;
    }
    // The barrier inside max_all already separates consecutive steps.
    __device__ __forceinline__ void step_end() const {}
};

// ---------------------------------------------------------------------------
// Class tables (clast, cnt): in LDS when they fit, else in global scratch.
// ---------------------------------------------------------------------------
struct LdsTables {
    uint16_t *clast;
    uint32_t *cnt;
    __device__ __forceinline__ uint32_t last(uint32_t c) const { return clast[c]; }
    __device__ __forceinline__ void set_last(uint32_t c, uint32_t v) const { clast[c] = (uint16_t)v; }
    __device__ __forceinline__ uint32_t count(uint32_t c) const { return cnt[c]; }
    __device__ __forceinline__ void set_count(uint32_t c, uint32_t v) const { cnt[c] = v; }
    __device__ __forceinline__ uint32_t add(uint32_t c, uint32_t v) const { return atomicAdd(&cnt[c], v); }
};

struct GlobalTables {
    uint32_t *clast;
    uint32_t *cnt;
    __device__ __forceinline__ uint32_t last(uint32_t c) const { return g_load(&clast[c]); }
    __device__ __forceinline__ void set_last(uint32_t c, uint32_t v) const { g_store(&clast[c], v); }
    __device__ __forceinline__ uint32_t count(uint32_t c) const { return g_load(&cnt[c]); }
    __device__ __forceinline__ void set_count(uint32_t c, uint32_t v) const { g_store(&cnt[c], v); }
    __device__ __forceinline__ uint32_t add(uint32_t c, uint32_t v) const
    {
        return __hip_atomic_fetch_add(&cnt[c], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// LDS bytes of the LexBFS state for n vertices.
__host__ __device__ constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline size_t lds_bytes_lds_tables(int n, int team)
{
    const size_t wn = (size_t)(n + 63) / 64;
    return align_up(8 * wn + 4 * (size_t)(team / kWave > 0 ? team / kWave : 1) + 4 * (size_t)n + 2 * align_up(n, 2) * 2, 16);
}

__host__ __device__ inline size_t lds_bytes_global_tables(int n, int team)
{
    const size_t wn = (size_t)(n + 63) / 64;
    return align_up(8 * wn + 4 * (size_t)(team / kWave > 0 ? team / kWave : 1) + 2 * align_up(n, 2), 16);
}

// Carve the LDS region of one graph (tables in LDS).
struct LdsLayout {
    uint64_t *unm;
    uint32_t *red;
    uint16_t *cls;
    LdsTables tab;
};

__device__ __forceinline__ LdsLayout carve_lds(void *base, int n, int team)
{
    const int wn = (n + 63) >> 6;
    LdsLayout L;
    L.unm = (uint64_t *)base;
    L.red = (uint32_t *)(L.unm + wn);
    const int nred = team / kWave > 0 ? team / kWave : 1;
    L.tab.cnt = L.red + nred;
    L.cls = (uint16_t *)(L.tab.cnt + n);
    L.tab.clast = L.cls + ((n + 1) & ~1);
    return L;
}

struct LdsLayoutG {
    uint64_t *unm;
    uint32_t *red;
    uint16_t *cls;
};

__device__ __forceinline__ LdsLayoutG carve_lds_g(void *base, int n, int team)
{
    const int wn = (n + 63) >> 6;
    LdsLayoutG L;
    L.unm = (uint64_t *)base;
    L.red = (uint32_t *)(L.unm + wn);
    const int nred = team / kWave > 0 ? team / kWave : 1;
    L.cls = (uint16_t *)(L.red + nred);
    return L;
}

// ---------------------------------------------------------------------------
// LexBFS on one graph by one team.
// ---------------------------------------------------------------------------
template <class Team, class Tabs>
__device__ void lexbfs_team(const Team &tm, int n, const uint64_t *__restrict__ bits, int64_t W,
                            int32_t *__restrict__ order, int32_t *__restrict__ rank, int32_t *__restrict__ parent,
                            uint64_t *unm, uint16_t *cls, const Tabs &tab, uint32_t *red)
{
    constexpr int T = Team::kSize;
    const int t = tm.tid;
    if (n <= 0) return;
    const int wn = (n + 63) >> 6;
    int K = 1;
    while (K * T < n) K <<= 1;
    const int vbase = t * K;
    const int wi = vbase >> 6;
    const int sh = vbase & 63;
    const uint64_t cmask = (K == 64) ? ~0ull : (((1ull << K) - 1ull) << sh);
    const bool owner = vbase < n;

    for (int v = t; v < n; v += T) {
        cls[v] = 0;
        tab.set_count(v, 0);
    }
    // parent[v] is later written only by v's owner lane; the same lane clears it.
    if (owner)
        for (int v = vbase; v < min(vbase + K, n); ++v) parent[v] = -1;
    for (int w = t; w < wn; w += T) unm[w] = (w == wn - 1 && (n & 63)) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
    if (t == 0) tab.set_last(0, (uint32_t)(n - 1));
    tm.sync();

    uint32_t x = 0;     // pivot: vertex 0 first (smallest id, all labels empty)
    uint32_t stop = 0;  // its class
    int U = n;
    const uint64_t *rowbase = bits + wi;
    for (int i = 0; i < n; ++i) {
        U -= 1;
        if (t == 0) {
            order[i] = (int32_t)x;
            rank[x] = i;
            if ((int)stop < U) tab.set_last(stop, (uint32_t)(U - 1));
            atomicAnd((unsigned long long *)&unm[x >> 6], ~(1ull << (x & 63)));
        }
        uint64_t nb = 0;
        if (owner) nb = rowbase[(int64_t)x * W] & unm[wi] & cmask;

        // Phase A: count the neighbours of every hit class; record the parent.
        uint64_t lead = 0;
        for (uint64_t m = nb; m; m &= m - 1) {
            const int b = ctz64(m);
            const int y = (wi << 6) + b;
            const uint32_t C = cls[y];
            parent[y] = (int32_t)x;
            if (tab.add(C, 1) == 0) lead |= 1ull << b;
        }
        tm.sync();

        // Phase B: move the neighbours to the upper part of their class.
        uint64_t split = 0;
        for (uint64_t m = nb; m; m &= m - 1) {
            const int b = ctz64(m);
            const int y = (wi << 6) + b;
            const uint32_t C = cls[y];
            const uint32_t c = tab.count(C);
            const uint32_t last = tab.last(C);
            if (c < last - C + 1) {
                const uint32_t nw = last + 1 - c;
                cls[y] = (uint16_t)nw;
                if ((lead >> b) & 1ull) {
                    tab.set_last(nw, last);
                    tab.set_count(nw, C);  // remember the old class for phase C
                    split |= 1ull << b;
                }
            }
        }
        tm.sync();

        // Phase C: the leader of each hit class closes it; then pick the pivot.
        for (uint64_t m = lead; m; m &= m - 1) {
            const int b = ctz64(m);
            const int y = (wi << 6) + b;
            const uint32_t nw = cls[y];
            if ((split >> b) & 1ull) {
                const uint32_t C = tab.count(nw);
                tab.set_last(C, nw - 1);
                tab.set_count(C, 0);
                tab.set_count(nw, 0);
            } else {
                tab.set_count(nw, 0);
            }
        }
        if (i + 1 == n) break;
        uint32_t best = 0;
        if (owner) {
            for (uint64_t m = unm[wi] & cmask; m; m &= m - 1) {
                const uint32_t v = (uint32_t)((wi << 6) + ctz64(m));
                const uint32_t key = ((uint32_t)cls[v] << 16) | (0xFFFFu - v);
                best = max(best, key);
            }
        }
        best = tm.max_all(best, red);
        x = 0xFFFFu - (best & 0xFFFFu);
        stop = best >> 16;
        tm.step_end();
    }
}

// ---------------------------------------------------------------------------
// Perfect-elimination sweep (Section 6.2 "testing"): v fails iff some
// z in LN(v) \ {p(v)} is not adjacent to p(v). Every such z lies before
// p(v) in the order, and every neighbour of v before p(v) is in LN(v), so
//   fail(v) <=> exists z in N(v) \ N(p) with rank z < rank p
// (p itself is in N(v) \ N(p) but fails rank p < rank p). The words of
// row v and row p are swept together; only set bits of row_v & ~row_p need
// a rank lookup. The smallest failing rank is kept with atomicMin.
// A group of G lanes (a power of two <= 64) handles one row.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sweep_rows(const uint64_t *__restrict__ bits, int64_t W, int wn,
                                           const int32_t *__restrict__ rank, const int32_t *__restrict__ parent,
                                           int n, int r0, int r1, int G, int lg, uint32_t *failkey)
{
    const uint64_t tail = (n & 63) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
    const int lane = threadIdx.x & 63;
    const int gid = lane >> lg;
    const int gl = lane & (G - 1);
    const int gpw = kWave >> lg;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (gid * G));
    for (int vb = r0 + wave * gpw; vb < r1; vb += nwaves * gpw) {
        const int v = vb + gid;
        bool fail = false;
        int rv = 0;
        if (v < r1) {
            const int p = parent[v];
            if (p >= 0) {
                rv = rank[v];
                const int rp = rank[p];
                const uint64_t *a = bits + (int64_t)v * W;
                const uint64_t *b = bits + (int64_t)p * W;
                for (int w = gl; w < wn && !fail; w += G) {
                    uint64_t X = __builtin_nontemporal_load(a + w) & ~b[w];
                    if (w == wn - 1) X &= tail;  // ids >= n never index rank[]
                    while (X) {
                        const int z = (w << 6) + ctz64(X);
                        X &= X - 1;
                        if (rank[z] < rp) { fail = true; break; }
                    }
                }
            }
        }
        const uint64_t bal = __ballot(fail);
        if ((bal & gmask) && gl == 0) atomicMin(failkey, (uint32_t)rv);
    }
}

}  // namespace lxd
