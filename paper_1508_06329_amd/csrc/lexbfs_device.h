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
// Next pivot without a scan. After step i the largest label belongs to the
// highest pre-split class C_top among the unnumbered vertices, narrowed to
// C_top & N(x_i) when that is not empty (the split puts that part directly
// above the rest of C_top; every other class stays below C_top). Every lane
// keeps, as a bitmask over its own vertices, the members of the current top
// class. Then with T' = top \ {x_i}:
//   T' & N(x_i) not empty -> x_{i+1} = its smallest id, top = T' & N(x_i);
//   else T' not empty     -> x_{i+1} = smallest id of T', top = T';
//   else                  -> the top class is exhausted: its successor C_1
//                            is the class holding position U - 1, the
//                            highest class start at or below it (a bitmap
//                            of class starts is kept in LDS), each lane
//                            matches its vertices against C_1, and the rule
//                            above is applied to C_1.
// Whether x_i empties the top class is known before any reduction: the top
// class is [s, U] with s the pivot's class, so it empties iff s = U. Every
// step therefore takes one team reduction, of the selection key (max) and
// of the candidate class's neighbour count c (sum); the pivot's class for
// the next step follows without a read: the adjacent part of the candidate
// class [s', U - 1] moves to [U - c, U - 1]. Only the third case touches
// every vertex of a lane. All of this uses pre-split information only, so
// x_{i+1} is known as soon as x_i's row is in, and the load of x_{i+1}'s row
// is issued before the splits of step i run.
//
// A pivot none of whose neighbours is still unnumbered causes no split. The
// selection's reduction also sums the pivot's unnumbered neighbours over the
// team, so every lane knows it before the split phase and the team skips
// the barrier after that (empty) phase.
//
// Closing a split class without a third barrier: every neighbour of class C
// reads C's neighbour count and clast[C], then counts itself as moved with
// an atomic add; the one that moves last -- after every other neighbour has
// read -- writes the shrunken clast[C], marks the new class start and
// clears the counters for the next step.
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

// One DPP step of a 64-bit max scan: every lane takes the max of its value
// and the value DPP control CTRL routes to it (0 where nothing is routed).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp_max64_step(uint64_t v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROW_MASK, 0xF, true);
    const uint64_t o = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    return o > v ? o : v;
}

// Max over the 64 lanes (all lanes must be active); the result is uniform.
// Row shifts 1, 2, 4, 8 leave each 16-lane row's maximum in its lane 15;
// the row broadcasts 15 and 31 then carry it to lane 63.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
    v = dpp_max64_step<0x111, 0xF>(v);  // row_shr:1
    v = dpp_max64_step<0x112, 0xF>(v);  // row_shr:2
    v = dpp_max64_step<0x114, 0xF>(v);  // row_shr:4
    v = dpp_max64_step<0x118, 0xF>(v);  // row_shr:8
    v = dpp_max64_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_max64_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int ctz64(uint64_t x) { return __builtin_ctzll(x); }

// Pointers read from memory (batch descriptors) are generic to the compiler,
// which then emits flat instructions; those count against the LDS counter as
// well, so every LDS wait would also wait for outstanding row loads and
// stores. All graph and output arrays live in global memory: say so.
#define LX_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ LX_GLOBAL T *as_global(T *p)
{
    return (LX_GLOBAL T *)p;
}

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
// Register headroom of the kernels that run one 512- or 1,024-lane team per
// workgroup (LexBFS, MCS, the large batch tier, the single-graph finish): an empty asm that clobbers v95 at entry raises the kernel's VGPR
// allocation to at least 96 and emits no instruction. A build of the
// 1,024-lane LexBFS kernel with an allocation of exactly 88 VGPRs and live
// values in v84-v87 returned wrong orders on gfx950, on graphs whose pivots
// have thousands of neighbours; the identical machine code with a 96-register
// allocation returned the right ones, as do the builds below 84 registers.
// At 4 (or 2) waves per SIMD the larger allocation costs no occupancy.
template <int T>
__device__ __forceinline__ void vgpr_headroom()
{
    if constexpr (T >= 512) __asm__ volatile("" ::: "v95");
}

// Max of a 32-bit value over the 64 lanes with DPP (all lanes active); the
// result is uniform.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_max32_step(uint32_t v)
{
    const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, true);
    return o > v ? o : v;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_add32_step(uint32_t v)
{
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, true);
}

// Sum over the 64 lanes with DPP (all lanes active); the result is uniform.
__device__ __forceinline__ uint32_t wave_sum_dpp(uint32_t v)
{
    v = dpp_add32_step<0x111, 0xF>(v);  // row_shr:1
    v = dpp_add32_step<0x112, 0xF>(v);  // row_shr:2
    v = dpp_add32_step<0x114, 0xF>(v);  // row_shr:4
    v = dpp_add32_step<0x118, 0xF>(v);  // row_shr:8
    v = dpp_add32_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add32_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Inclusive prefix sum over the 64 lanes (lane order).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
    const int lane = (int)__lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_max_dpp(uint32_t v)
{
    v = dpp_max32_step<0x111, 0xF>(v);  // row_shr:1
    v = dpp_max32_step<0x112, 0xF>(v);  // row_shr:2
    v = dpp_max32_step<0x114, 0xF>(v);  // row_shr:4
    v = dpp_max32_step<0x118, 0xF>(v);  // row_shr:8
    v = dpp_max32_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_max32_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

struct WaveTeam {
    int tid;  // lane
    static constexpr int kSize = kWave;
    static constexpr int kWaves = 1;
    __device__ __forceinline__ void sync() const
    {
        // LDS operations of one wave complete in issue order; this only has to
        // stop the compiler from moving memory operations across the point.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __device__ __forceinline__ uint32_t max_all(uint32_t v, uint32_t *) const
    {
        v = wave_max_dpp(v);
        sync();
        return v;
    }
    __device__ __forceinline__ uint32_t max_all_lds(uint32_t v, uint32_t *red) const { return max_all(v, red); }
    // Max of v and sum of s over the team at once; the sum is returned in s.
    __device__ __forceinline__ uint32_t max_sum_all(uint32_t v, uint32_t &s, uint32_t *) const
    {
        v = wave_max_dpp(v);
        s = wave_sum_dpp(s);
        sync();
        return v;
    }
    // Barrier that also orders the team's global memory accesses. A team
    // is one wavefront (or one workgroup, below) on one CU, and everything
    // it shares through global memory is written and read inside the team,
    // so workgroup scope is the right one. Agent scope would compile to an
    // L2 write-back and invalidate on this multi-XCD part.
    __device__ __forceinline__ void sync_mem() const
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    __device__ __forceinline__ uint32_t min_all(uint32_t v, uint32_t *) const
    {
        v = wave_min_u32(v);
        sync();
        return v;
    }
    __device__ __forceinline__ bool any_all(bool p) const { return __ballot(p) != 0ull; }
    // Exclusive prefix sum over the lanes (lane order = vertex order).
    __device__ __forceinline__ uint32_t exclusive_scan(uint32_t v, uint32_t *) const
    {
        return wave_inclusive_scan(v) - v;
    }
};

// On gfx950 a workgroup barrier waits for LDS traffic only; global loads in
// flight (the prefetched pivot row) stay in flight across it. With the class
// tables in global memory (kGlobalTables) every table access is an L2
// atomic, load or store of this workgroup; the barrier's workgroup-scope
// release and acquire order them (the waves share one CU's memory path).
template <int T, bool kGlobalTables>
struct BlockTeam {
    int tid;
    static constexpr int kSize = T;
    static constexpr int kWaves = T / kWave;
    __device__ __forceinline__ void sync() const
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    // Max over the team (one barrier); every lane gets the result.
    // red: T/64 LDS words, not reused before the next barrier.
    __device__ __forceinline__ uint32_t max_all(uint32_t v, uint32_t *red) const
    {
        v = wave_max_dpp(v);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        sync();
        uint32_t r = red[0];
#pragma unroll
        for (int k = 1; k < kWaves; ++k) r = max(r, red[k]);
        return r;
    }
    // max_all with a barrier that orders LDS only (no global tables in use).
    __device__ __forceinline__ uint32_t max_all_lds(uint32_t v, uint32_t *red) const
    {
        v = wave_max_dpp(v);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        uint32_t r = red[0];
#pragma unroll
        for (int k = 1; k < kWaves; ++k) r = max(r, red[k]);
        return r;
    }
    // Max of v and sum of s (returned in s); red: 2 * T/64 LDS words.
    __device__ __forceinline__ uint32_t max_sum_all(uint32_t v, uint32_t &s, uint32_t *red) const
    {
        v = wave_max_dpp(v);
        s = wave_sum_dpp(s);
        if ((tid & 63) == 0) {
            red[tid >> 6] = v;
            red[kWaves + (tid >> 6)] = s;
        }
        sync();
        uint32_t r = red[0], q = red[kWaves];
#pragma unroll
        for (int k = 1; k < kWaves; ++k) {
            r = max(r, red[k]);
            q += red[kWaves + k];
        }
        s = q;
        return r;
    }
    // Barrier that also orders the workgroup's global memory accesses
    // (see WaveTeam::sync_mem for the scope).
    __device__ __forceinline__ void sync_mem() const
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    // Min over the team; red: T/64 LDS words, free again after return.
    __device__ __forceinline__ uint32_t min_all(uint32_t v, uint32_t *red) const
    {
        v = wave_min_u32(v);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        uint32_t r = red[0];
#pragma unroll
        for (int k = 1; k < kWaves; ++k) r = min(r, red[k]);
        __syncthreads();
        return r;
    }
    __device__ __forceinline__ bool any_all(bool p) const { return __syncthreads_or(p) != 0; }
    // Exclusive prefix sum over the team's lanes in lane order; red: T/64
    // LDS words, free again after return.
    __device__ __forceinline__ uint32_t exclusive_scan(uint32_t v, uint32_t *red) const
    {
        const uint32_t inc = wave_inclusive_scan(v);
        if ((tid & 63) == 63) red[tid >> 6] = inc;
        __syncthreads();
        uint32_t off = 0;
        for (int k = 0; k < (tid >> 6); ++k) off += red[k];
        __syncthreads();
        return off + inc - v;
    }
};

// ---------------------------------------------------------------------------
// Class tables. Per class c: clast[c], the last position of the class, and
// a 32-bit split word whose low half counts the pivot's neighbours in c
// (phase A) and whose high half counts those that have already moved
// (phase B). The low half is final and stable throughout phase B; the
// neighbour that moves last (high half reaching the count) closes the class
// and clears the word for the next step.
// LDS form: clast 16-bit; global form (large n): 32-bit entries in L2.
// ---------------------------------------------------------------------------
struct LdsTables {
    uint16_t *clast;
    uint32_t *cnt;
    static constexpr bool kInLds = true;
    static constexpr bool kSole = false;  // see LdsTablesSole
    __device__ __forceinline__ uint32_t last(uint32_t c) const { return clast[c]; }
    __device__ __forceinline__ void set_last(uint32_t c, uint32_t v) const { clast[c] = (uint16_t)v; }
    __device__ __forceinline__ uint32_t word(uint32_t c) const { return cnt[c]; }
    __device__ __forceinline__ void clear(uint32_t c) const { cnt[c] = 0u; }
    __device__ __forceinline__ void inc(uint32_t c) const { atomicAdd(&cnt[c], 1u); }
    __device__ __forceinline__ void add(uint32_t c, uint32_t k) const { atomicAdd(&cnt[c], k); }
    // Count one neighbour as moved; returns the word before.
    __device__ __forceinline__ uint32_t moved(uint32_t c) const { return atomicAdd(&cnt[c], 0x10000u); }
    __device__ __forceinline__ uint32_t moved_by(uint32_t c, uint32_t k) const { return atomicAdd(&cnt[c], k << 16); }
};

// LDS tables that also record the member of a one-vertex class created by a
// split, in the class's clast slot with flag bit 15 (positions stay below
// 2^15 where this form is used; such a class ends where it starts). The
// member never moves again (a one-position class cannot split) and the
// position is not reused once it is numbered, so a recorded member stays
// valid while its class lives. When the pivot empties the top class and the
// candidate class below is such a class, its member is the next pivot's only
// candidate and the selection skips matching class ids.
struct LdsTablesSole : LdsTables {
    static constexpr bool kSole = true;
    static constexpr uint32_t kFlag = 0x8000u;
    __device__ __forceinline__ uint32_t last(uint32_t c) const
    {
        const uint32_t r = clast[c];
        return (r & kFlag) ? c : r;
    }
    __device__ __forceinline__ void set_sole(uint32_t c, uint32_t v) const { clast[c] = (uint16_t)(kFlag | v); }
    __device__ __forceinline__ uint32_t slot(uint32_t c) const { return clast[c]; }
};

// The global form is read and written by one workgroup only (its team), so
// every access has workgroup scope: atomics complete in the L2 of the CU's
// own die and loads may be served by the CU's L1, which the same CU's
// atomics and stores keep current. (Agent scope would have to make each
// access coherent across the dies of the device.)
struct GlobalTables {
    LX_GLOBAL uint32_t *clast;
    LX_GLOBAL uint32_t *cnt;
    static constexpr bool kInLds = false;
    static constexpr bool kSole = false;
    static constexpr int kScope = __HIP_MEMORY_SCOPE_WORKGROUP;
    __device__ GlobalTables(uint32_t *cl, uint32_t *ct) : clast(as_global(cl)), cnt(as_global(ct)) {}
    __device__ __forceinline__ uint32_t last(uint32_t c) const
    {
        return __hip_atomic_load(clast + c, __ATOMIC_RELAXED, kScope);
    }
    __device__ __forceinline__ void set_last(uint32_t c, uint32_t v) const
    {
        __hip_atomic_store(clast + c, v, __ATOMIC_RELAXED, kScope);
    }
    __device__ __forceinline__ uint32_t word(uint32_t c) const { return __hip_atomic_load(cnt + c, __ATOMIC_RELAXED, kScope); }
    __device__ __forceinline__ void clear(uint32_t c) const { __hip_atomic_store(cnt + c, 0u, __ATOMIC_RELAXED, kScope); }
    __device__ __forceinline__ void inc(uint32_t c) const { __hip_atomic_fetch_add(cnt + c, 1u, __ATOMIC_RELAXED, kScope); }
    __device__ __forceinline__ void add(uint32_t c, uint32_t k) const
    {
        __hip_atomic_fetch_add(cnt + c, k, __ATOMIC_RELAXED, kScope);
    }
    __device__ __forceinline__ uint32_t moved(uint32_t c) const
    {
        return __hip_atomic_fetch_add(cnt + c, 0x10000u, __ATOMIC_RELAXED, kScope);
    }
    __device__ __forceinline__ uint32_t moved_by(uint32_t c, uint32_t k) const
    {
        return __hip_atomic_fetch_add(cnt + c, k << 16, __ATOMIC_RELAXED, kScope);
    }
};

// Optional parts of the LexBFS state for the fused elimination test: the
// parent of every vertex in LDS (16 bits, kNoParent = none) and one word
// for the smallest failing rank.
struct FusedPeo {
    uint16_t *par;     // [n] in LDS
    uint32_t *fk;      // one LDS word
    uint32_t *failkey; // global result word of the graph
};
constexpr uint16_t kNoParent = 0xFFFFu;

__host__ __device__ constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// LDS of one graph's state. Tables in LDS:
//   starts u64[wn] | red u32[2 waves] | cls u16[n] | clast u16[n] | cnt u32[n]
// Tables in global memory:
//   starts u64[wn] | red u32[2 waves] | cls u16[n]
// Every array starts on a 16-byte boundary (cls is read 16 bytes at a time).
__host__ __device__ inline size_t lds_bytes_lds_tables(int n, int team)
{
    const size_t wn = (size_t)(n + 63) / 64;
    const size_t nred = (size_t)(team / kWave > 0 ? team / kWave : 1);
    const size_t a = align_up(2 * (size_t)n, 16);
    return align_up(8 * wn, 16) + align_up(16 * nred, 16) + 2 * a + align_up(4 * (size_t)n, 16);
}

__host__ __device__ inline size_t lds_bytes_global_tables(int n, int team)
{
    const size_t wn = (size_t)(n + 63) / 64;
    const size_t nred = (size_t)(team / kWave > 0 ? team / kWave : 1);
    return align_up(8 * wn, 16) + align_up(16 * nred, 16) + align_up(2 * (size_t)n, 16);
}

struct LdsLayout {
    uint64_t *starts;
    uint32_t *red;
    uint16_t *cls;
    LdsTables tab;
};

__device__ __forceinline__ LdsLayout carve_lds(void *base, int n, int team)
{
    const size_t wn = (size_t)(n + 63) / 64;
    const size_t nred = (size_t)(team / kWave > 0 ? team / kWave : 1);
    const size_t a = align_up(2 * (size_t)n, 16);
    char *p = (char *)base;
    LdsLayout L;
    L.starts = (uint64_t *)p;
    p += align_up(8 * wn, 16);
    L.red = (uint32_t *)p;
    p += align_up(16 * nred, 16);
    L.cls = (uint16_t *)p;
    L.tab.clast = (uint16_t *)(p + a);
    L.tab.cnt = (uint32_t *)(p + 2 * a);
    return L;
}

// Batch graph state: the LDS tables, then the parents and the failing-rank
// word of the fused elimination test.
__host__ __device__ inline size_t lds_bytes_batch(int n, int team)
{
    return lds_bytes_lds_tables(n, team) + align_up(2 * (size_t)n, 16) + 16;
}

struct BatchLayout {
    LdsLayout L;
    FusedPeo fp;
};

__device__ __forceinline__ BatchLayout carve_batch(void *base, int n, int team, uint32_t *failkey)
{
    BatchLayout B;
    B.L = carve_lds(base, n, team);
    char *p = (char *)base + lds_bytes_lds_tables(n, team);
    B.fp.par = (uint16_t *)p;
    B.fp.fk = (uint32_t *)(p + align_up(2 * (size_t)n, 16));
    B.fp.failkey = failkey;
    return B;
}

struct LdsLayoutG {
    uint64_t *starts;
    uint32_t *red;
    uint16_t *cls;
};

__device__ __forceinline__ LdsLayoutG carve_lds_g(void *base, int n, int team)
{
    const size_t wn = (size_t)(n + 63) / 64;
    const size_t nred = (size_t)(team / kWave > 0 ? team / kWave : 1);
    char *p = (char *)base;
    LdsLayoutG L;
    L.starts = (uint64_t *)p;
    p += align_up(8 * wn, 16);
    L.red = (uint32_t *)p;
    p += align_up(16 * nred, 16);
    L.cls = (uint16_t *)p;
    return L;
}

// Class-id matching on packed 16-bit halves: after xor with the pattern,
// one v_pk_min_u16 against (1, 1) leaves 0 in a half that matched and 1 in
// one that did not, two ids per instruction.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// (1, 1) in a register whose value the compiler does not see: with the
// constant in view it turns min(x, 1) back into a compare and a select per
// half.
__device__ __forceinline__ uint32_t pk_ones()
{
    uint32_t r;
    __asm__("s_mov_b32 %0, 0x10001" : "=s"(r));
    return r;
}

// 8 class ids (one 16-byte LDS read) against pat = c | c << 16: bit 2k is
// set iff the low id of word k differs from c, bit 16 + 2k iff its high id
// does.
__device__ __forceinline__ uint32_t diff8(uint4 q, uint32_t pat, uint32_t ones)
{
    auto nz = [ones](uint32_t x) {
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, x),
                                                                      __builtin_bit_cast(u16x2, ones)));
    };
    return nz(q.x ^ pat) | nz(q.y ^ pat) << 2 | nz(q.z ^ pat) << 4 | nz(q.w ^ pat) << 6;
}

// Which of 8 consecutive 16-bit class ids equal c: bit j for entry j.
__device__ __forceinline__ uint32_t match8(uint4 q, uint32_t c)
{
    const uint32_t w = diff8(q, c | (c << 16), pk_ones());
    return ~(w | (w >> 15)) & 0xFFu;  // high-id flags 16 + 2k move to 2k + 1
}

// The same for 16 consecutive ids in two groups: bit j for entry j.
__device__ __forceinline__ uint32_t match16(uint4 a, uint4 b, uint32_t c)
{
    const uint32_t pat = c | (c << 16), ones = pk_ones();
    const uint32_t w = diff8(a, pat, ones) | diff8(b, pat, ones) << 8;
    return ~(w | (w >> 15)) & 0xFFFFu;
}

// Bits of my unnumbered vertices `um` (word positions) whose class is c.
// The needed 16-byte groups of ids are requested kG at a time, each batch
// before any of it is used: one LDS round trip per kG groups, not one per
// group. kG is the most a team's chunks need (chunks of up to 8 kG ids take
// one round trip; larger ones stay correct) and bounds the registers held.
template <int kG = 8>
__device__ __forceinline__ uint64_t chunk_match(const uint16_t *cls, uint64_t um, uint32_t c, int vbase, int sh, int K)
{
    if (!um) return 0;
    uint64_t res = 0;
    if (K >= 8) {
        const uint4 *p = (const uint4 *)(cls + vbase);
        const uint32_t nc = ~(c | (c << 16));  // matches no id
        for (int j0 = 0; j0 < K; j0 += 8 * kG) {
            uint4 q[kG];
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int b = j0 + 8 * j;
                q[j] = make_uint4(nc, nc, nc, nc);
                if (b < K && ((um >> (sh + b)) & 0xFFull)) q[j] = p[b >> 3];
            }
#pragma unroll
            for (int j = 0; j < kG; j += 2) {
                const int b = j0 + 8 * j;
                if (b >= K) break;
                // A second group past K holds no matches (filled above).
                const uint32_t m = j + 1 < kG ? match16(q[j], q[j + 1 < kG ? j + 1 : j], c) : match8(q[j], c);
                res |= (uint64_t)m << (sh + b);
            }
        }
        return res & um;
    }
    const int wbase = (vbase >> 6) << 6;
    for (uint64_t m = um; m; m &= m - 1) {
        const int b = ctz64(m);
        if (cls[wbase + b] == c) res |= 1ull << b;
    }
    return res;
}

// Selection key: case 2 (pivot-adjacent part of the top class) above case 1
// (rest of the top class), then the smallest id.
__device__ __forceinline__ uint32_t pick_key(uint64_t top, uint64_t nb, uint32_t wbase)
{
    const uint64_t a = top & nb;
    if (a) return 0x20000u | (0xFFFFu - (wbase + (uint32_t)ctz64(a)));
    if (top) return 0x10000u | (0xFFFFu - (wbase + (uint32_t)ctz64(top)));
    return 0u;
}

// Interleaved tie-break order. Lane t of a team owns ids t*K + j (slot j,
// 0 <= j < K; the last owner, lane tl = (n-1)/K, holds the cl = n - tl*K
// lowest slots). Ranks are dealt slot by slot across the owners: slot 0 of
// lanes 0..tl, then slot 1, ... -- rank(t, j) = j*tl + min(j, cl) + t. The
// smallest rank wins a tie instead of the smallest id. Within one lane the
// rank grows with the slot, as the id does, so a lane's best candidate is
// still its lowest set bit. A caller that names vertices by rank (a graph
// renamed so that rank order is the wanted tie order) gets consecutive ranks
// on different lanes: neighbours of a pivot then spread over the team
// instead of queueing on one lane.
__device__ __forceinline__ uint32_t ilv_rank(uint32_t j, uint32_t t, uint32_t tl, uint32_t cl)
{
    return j * tl + min(j, cl) + t;
}

__host__ __device__ __forceinline__ uint32_t ilv_id(uint32_t r, uint32_t tl, uint32_t cl, uint32_t K)
{
    const uint32_t A = tl + 1;  // owners of each slot below cl
    uint32_t j, t;
    if (r < cl * A) {
        j = r / A;
        t = r - j * A;
    } else {  // tl >= 1 here: slots cl.. have tl owners
        const uint32_t r2 = r - cl * A;
        j = cl + r2 / tl;
        t = r2 - (j - cl) * tl;
    }
    return t * K + j;
}

__device__ __forceinline__ uint32_t pick_key_ilv(uint64_t top, uint64_t nb, int sh, uint32_t t, uint32_t tl,
                                                 uint32_t cl)
{
    const uint64_t a = top & nb;
    if (a) return 0x20000u | (0xFFFFu - ilv_rank((uint32_t)(ctz64(a) - sh), t, tl, cl));
    if (top) return 0x10000u | (0xFFFFu - ilv_rank((uint32_t)(ctz64(top) - sh), t, tl, cl));
    return 0u;
}


// ---------------------------------------------------------------------------
// LexBFS on one graph by one team.
//   row_ptr: only row_ptr[n] (twice the edge count) is read, by single graphs.
//   red: 2 * waves LDS words (alternating between consecutive reductions).
//
// kPeo fuses the perfect-elimination test of Section 5.2 into the steps:
// when v = x_i is numbered, its earlier neighbours LN_v are exactly its
// numbered neighbours and its parent p(v) is the last pivot adjacent to it,
// so v fails iff (row_v & numbered & ~row_p) \ {p} is not empty. The team
// loads row_p together with row_v (the parent is known, from LDS, as soon as
// v is chosen) and keeps the smallest failing rank; parents are collected in
// LDS and written out at the end. Needs n < 65536 (16-bit parents).
// ---------------------------------------------------------------------------
// kIlv: ties go to the smallest interleaved rank (ilv_rank) instead of the
// smallest id. kPre: the largest K whose class ids the gone case loads
// early (8, 16 or 32; wider K matches from LDS), a register budget.
// kMatchG: 16-byte groups of class ids a chunk match requests per LDS round
// trip (8 covers K = 64 at once; batch teams, K <= 16, use 2), also a
// register budget.
template <class Team, class Tabs, bool kPeo = false, bool kIlv = false, int kPre = 16, int kMatchG = 8>
__device__ __forceinline__ void lexbfs_team(const Team &tm, int n, const uint64_t *bits_, int64_t W, const int32_t *row_ptr_,
                            int32_t *order_, int32_t *rank_, int32_t *parent_, uint64_t *starts, uint16_t *cls,
                            const Tabs &tab, uint32_t *red, const FusedPeo &fp = FusedPeo{})
{
    LX_GLOBAL const uint64_t *__restrict__ bits = as_global(bits_);
    LX_GLOBAL const int32_t *__restrict__ row_ptr = as_global(row_ptr_);
    LX_GLOBAL int32_t *__restrict__ order = as_global(order_);
    LX_GLOBAL int32_t *__restrict__ rank = as_global(rank_);
    LX_GLOBAL int32_t *__restrict__ parent = as_global(parent_);
    constexpr int T = Team::kSize;
    constexpr int NW = Team::kWaves;
    // Class tables in L2: each lane handles its neighbours class by class,
    // one atomic round trip per class instead of one per neighbour, and the
    // parents are not written during the steps (a lane may own 64 neighbours
    // of one pivot); derive_parents computes them from the finished order.
    constexpr bool kGroup = !Tabs::kInLds;
    const int t = tm.tid;
    if (n <= 0) return;
    const int wn = (n + 63) >> 6;
    int K = 1;
    while (K * T < n) K <<= 1;
    const uint32_t tl = (uint32_t)((n - 1) / K);      // last lane owning vertices (interleaved order)
    const uint32_t cl = (uint32_t)n - tl * (uint32_t)K; // its number of vertices
    const int vbase = t * K;
    const int wi = vbase >> 6;
    const int sh = vbase & 63;
    const uint32_t wbase = (uint32_t)wi << 6;
    uint64_t cmask = (K == 64) ? ~0ull : (((1ull << K) - 1ull) << sh);
    if (wi == wn - 1 && (n & 63)) cmask &= (1ull << (n & 63)) - 1ull;
    const bool owner = vbase < n;
    // Lanes past the last vertex read a word of the row as well (the last
    // one), so that every row load is issued by every lane: a load skipped
    // by part of the team would leave the compiler unsure how many loads are
    // in flight, and every later wait would then wait for all of them.
    LX_GLOBAL const uint64_t *rowbase = bits + min(wi, wn - 1);
    const uint64_t omask = owner ? cmask : 0ull;  // my vertices (none past the last)

    for (int v = t; v < n; v += T) {
        cls[v] = 0;
        tab.clear(v);
        if (kPeo) fp.par[v] = kNoParent;
    }
    for (int w = t; w < wn; w += T) starts[w] = w == 0 ? 1ull : 0ull;  // one class, starting at 0
    // parent[v] is later written only by v's owner lane; the same lane clears it.
    if (!kPeo && !kGroup && owner)
        for (int v = vbase; v < min(vbase + K, n); ++v) parent[v] = -1;
    if (t == 0) {
        tab.set_last(0, (uint32_t)(n - 1));
        if (kPeo) *fp.fk = kNoFail;
    }
    tm.sync();

    uint64_t um = owner ? cmask : 0ull;  // my unnumbered vertices (word positions)
    uint64_t top = um;                   // my members of the top class
    uint32_t x = 0;                      // first pivot: vertex 0 (smallest id, all labels empty)
    uint64_t rw = rowbase[0];            // my chunk's word of the pivot's row
    uint32_t xp = kNoParent;             // the pivot's parent (kPeo)
    uint64_t rp = 0ull;                  // my chunk's word of the parent's row (kPeo)
    uint32_t xcls = 0;        // the pivot's (post-split) class, derived at selection
    int par = 0;
    int U = n;
    // Single graphs: edges with both ends unnumbered. Once none is left, no
    // later pivot has an unnumbered neighbour, so nothing splits any more and
    // the team finishes in the tail loop below.
    // (Not with interleaved ties: the tail ranks a class's members in id
    // order.)
    uint32_t eu = (kPeo || kIlv) ? 1u : (uint32_t)(row_ptr[n] >> 1);
    bool tail = false;
    int i = 0;
    for (; i < n; ++i) {
        U -= 1;
        const uint32_t stop = Tabs::kInLds ? xcls : (uint32_t)cls[x];
        const bool gone = (int)stop == U;  // x was the last member of the top class
        // What the gone case reads, loaded now, in the shadow of the pivot
        // row: the two class-start words at and below position U - 1 and the
        // class ids of my chunk (K = 8, 16 or 32: one 16-byte read per 8 ids).
        // Nothing changes them before the case uses them: phase A writes
        // neither, and the class start cleared below is U, above U - 1.
        constexpr int kQ = kPre / 8;
        uint64_t s_hi = 0ull, s_lo = 0ull;
        uint32_t sole = 0u;  // recorded-member form: the clast slot of position U - 1
        uint4 cc[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) cc[q] = make_uint4(0u, 0u, 0u, 0u);
        if (gone && U > 0) {
            const int pw = (U - 1) >> 6;
            s_hi = starts[pw];
            if (pw > 0) s_lo = starts[pw - 1];
            if constexpr (Tabs::kSole) sole = tab.slot((uint32_t)(U - 1));
            if (K >= 8 && K <= kPre && owner) {
                const uint4 *p = (const uint4 *)(cls + vbase);
#pragma unroll
                for (int q = 0; q < kQ; ++q)
                    if (8 * q < K && vbase + 8 * q < n) cc[q] = p[q];  // only ids below n
            }
        }
        if (owner && (x >> 6) == (uint32_t)wi) {
            um &= ~(1ull << (x & 63));
            top &= ~(1ull << (x & 63));
        }
        uint64_t nb = rw & um;
        // Earlier neighbours of x in my chunk outside N(p(x)), p(x) itself
        // excluded (kPeo): x fails if there is one.
        uint64_t bad = 0ull;
        if (kPeo && xp != kNoParent) {
            bad = rw & ~um & omask & ~rp;
            if ((xp >> 6) == (uint32_t)wi) bad &= ~(1ull << (xp & 63));
        }
        // Global stores only after the row word is in: on gfx9 the memory
        // counter covers stores too, so a store issued between the row load
        // and its use would hold up the use until the store completes. The
        // empty asm pins the use of the row here, ahead of the stores.
        __asm__ volatile("" : "+v"(nb), "+v"(bad)::"memory");
        if (kPeo && bad) atomicMin(fp.fk, (uint32_t)i);
        if (t == 0) {
            if (!gone) tab.set_last(stop, (uint32_t)(U - 1));
            else atomicAnd((unsigned long long *)&starts[stop >> 6], ~(1ull << (stop & 63)));  // class gone
            if (kPeo) {
                cls[x] = (uint16_t)i;  // numbered: its class id slot now keeps its rank
            } else {
                order[i] = (int32_t)x;
                rank[x] = i;
            }
        }

        // Phase A: count the neighbours of every hit class; record the parent.
        uint32_t C0 = 0;     // class of my first neighbour, reused in phase B
        uint64_t sing = 0;   // my neighbours alone in their class (kGroup)
        // kGroup: my neighbours in their first class, whether that class
        // needs the tables, and the wave's shared handling of it (below).
        uint64_t gf = 0ull, act = 0ull;
        bool lf = false, agg = false;
        uint32_t cw = 0u, wtot = 0u;
        if (kGroup) {
            // A class of one position cannot split: its neighbour stays put
            // and the class tables are not touched (no round trip to L2).
            // The class-start bitmap does not change during phase A.
            // Each lane's first class is handled by its wave at once: when
            // the lanes whose first class needs the tables all have the same
            // one (a pivot adjacent to a run of ids, as in a clique), a
            // single atomic adds the wave's count, instead of one per lane on
            // one address -- those serialise in L2 and hold up the memory
            // path of the CU for every wave.
            // A one-position class holds only the neighbour that named it,
            // so its members need no match over the chunk.
            uint32_t Cf = 0u;
            if (nb) {
                Cf = cls[(int)wbase + ctz64(nb)];
                const uint32_t nx = Cf + 1u;
                if (nx >= (uint32_t)U || ((starts[nx >> 6] >> (nx & 63)) & 1ull)) {
                    gf = nb & (0ull - nb);
                    sing |= gf;
                } else {
                    gf = chunk_match<kMatchG>(cls, nb, Cf, vbase, sh, K);
                    lf = true;
                }
            }
            act = __ballot(lf);
            cw = act ? (uint32_t)__shfl((int)Cf, ctz64(act), kWave) : 0u;
            agg = act != 0ull && __ballot(lf && Cf == cw) == act;
            const uint32_t cf = lf ? (uint32_t)__popcll(gf) : 0u;
            if (agg) {
                wtot = wave_sum_dpp(cf);
                if ((uint32_t)(t & 63) == (uint32_t)ctz64(act)) tab.add(cw, wtot);
            } else if (lf) {
                tab.add(Cf, cf);
            }
            for (uint64_t m = nb & ~gf; m;) {
                const uint32_t C = cls[(int)wbase + ctz64(m)];
                const uint32_t nx = C + 1u;
                uint64_t g = m & (0ull - m);
                if (nx >= (uint32_t)U || ((starts[nx >> 6] >> (nx & 63)) & 1ull)) {
                    sing |= g;
                } else {
                    g = chunk_match<kMatchG>(cls, m, C, vbase, sh, K);  // my neighbours in C
                    tab.add(C, (uint32_t)__popcll(g));  // parents: derive_parents after the order
                }
                m &= ~g;
            }
        } else {
            for (uint64_t m = nb; m; m &= m - 1) {
                const int y = (int)wbase + ctz64(m);
                const uint32_t C = cls[y];
                if (m == nb) C0 = C;
                if (kPeo) fp.par[y] = (uint16_t)x;
                else parent[y] = (int32_t)x;
                tab.inc(C);
            }
        }
        if (i + 1 == n) break;

        // Next pivot (see the header comment). The candidate class is the top
        // class, or -- when x emptied it -- the class directly below, i.e.
        // the one holding position U - 1: the highest class start at or
        // below U - 1, looked up in at most two bitmap words by every lane
        // alike (almost always enough), else by the whole team.
        uint32_t cand = stop;
        if (gone) {
            const uint32_t pos = (uint32_t)(U - 1);
            int w = (int)(pos >> 6);
            uint64_t sw = s_hi & (~0ull >> (63 - (pos & 63)));
            if (!sw && w > 0) {
                sw = s_lo;
                --w;
            }
            if (sw) {
                cand = ((uint32_t)w << 6) | (uint32_t)(63 - __builtin_clzll(sw));
            } else {
                uint32_t hi = 0;
                for (int w2 = t; w2 < w; w2 += T) {
                    const uint64_t s2 = starts[w2];
                    if (s2) hi = max(hi, (uint32_t)((w2 << 6) | (63 - __builtin_clzll(s2))) + 1u);
                }
                cand = tm.max_all(hi, red + par * 2 * NW) - 1u;
                par ^= 1;
            }
            if (Tabs::kSole && cand == (uint32_t)(U - 1) && (sole & 0x8000u)) {
                // a one-vertex class with its member recorded: only the
                // member's owner lane has a candidate
                const uint32_t v = sole & 0x7FFFu;
                top = (v >= (uint32_t)vbase && v < (uint32_t)(vbase + K)) ? (1ull << (v & 63)) & um : 0ull;
            } else if (K >= 8 && K <= kPre) {
                uint64_t mm = 0ull;
#pragma unroll
                for (int q = 0; q < kQ; q += 2)  // ids past the chunk: masked by um
                    if (8 * q < K)
                        mm |= (uint64_t)(q + 1 < kQ ? match16(cc[q], cc[q + 1 < kQ ? q + 1 : q], cand)
                                                    : match8(cc[q], cand)) << (8 * q);
                top = (mm << sh) & um;
            } else {
                top = chunk_match<kMatchG>(cls, um, cand, vbase, sh, K);
            }
        }
        // One reduction: the selection key (max) and two 16-bit sums packed
        // in one word -- the candidate class's neighbour count and x's
        // unnumbered-neighbour count (each at most n - 1 < 2^16).
        uint32_t sums = (uint32_t)__popcll(top & nb) | ((uint32_t)__popcll(nb) << 16);
        const uint32_t key = kIlv ? pick_key_ilv(top, nb, sh, (uint32_t)t, tl, cl) : pick_key(top, nb, wbase);
        const uint32_t k = tm.max_sum_all(key, sums, red + par * 2 * NW);
        par ^= 1;
        const uint32_t c_adj = sums & 0xFFFFu;
        const bool xrem = (sums >> 16) != 0u;  // x has unnumbered neighbours: phase B has work
        if (!kPeo && !kIlv) {
            eu -= sums >> 16;
            tail = eu == 0u;
        }
        const uint32_t xn = kIlv ? ilv_id(0xFFFFu - (k & 0xFFFFu), tl, cl, (uint32_t)K) : 0xFFFFu - (k & 0xFFFFu);
        const bool adj = (k >> 16) == 2;
        if (adj) top &= nb;  // narrowed to the pivot's neighbours
        // The candidate class spans [cand, U - 1]; its c_adj members adjacent
        // to x move to [U - c_adj, U - 1] and hold the next pivot.
        xcls = adj ? (uint32_t)U - c_adj : cand;
        // The next pivot's row first: the latency that bounds the step.
        const uint64_t rwn = rowbase[(int64_t)xn * W];  // past the last vertex: masked by um
        const uint32_t pn = kPeo ? (uint32_t)fp.par[xn] : kNoParent;
        const uint64_t rpn = kPeo ? rowbase[(int64_t)(pn != kNoParent ? pn : xn) * W] : 0ull;  // used if p exists

        // Phase B: move the neighbours to the upper part of their class; the
        // last neighbour of a class to leave closes it.
        if (kGroup) {
            if (agg) {  // the wave's shared first class (phase A)
                const uint32_t C = cw;
                const uint32_t c = tab.word(C) & 0xFFFFu;
                const uint32_t last = tab.last(C);
                const bool split = c < last - C + 1;
                const uint32_t nw = last + 1 - c;
                if (split && lf)
                    for (uint64_t q = gf; q; q &= q - 1) cls[(int)wbase + ctz64(q)] = (uint16_t)nw;
                if ((uint32_t)(t & 63) == (uint32_t)ctz64(act)) {
                    if (split) tab.set_last(nw, last);
                    if ((tab.moved_by(C, wtot) >> 16) + wtot == c) {  // the last group out closes C
                        tab.clear(C);
                        if (split) {
                            tab.set_last(C, nw - 1);
                            atomicOr((unsigned long long *)&starts[nw >> 6], 1ull << (nw & 63));
                        }
                    }
                }
            }
            for (uint64_t m = nb & ~sing & (agg ? ~gf : ~0ull); m;) {
                const uint32_t C = cls[(int)wbase + ctz64(m)];
                const uint64_t g = chunk_match<kMatchG>(cls, m, C, vbase, sh, K);
                const uint32_t cg = (uint32_t)__popcll(g);
                const uint32_t c = tab.word(C) & 0xFFFFu;
                const uint32_t last = tab.last(C);
                const bool split = c < last - C + 1;
                const uint32_t nw = last + 1 - c;
                if (split) {
                    for (uint64_t q = g; q; q &= q - 1) cls[(int)wbase + ctz64(q)] = (uint16_t)nw;
                    tab.set_last(nw, last);
                }
                if ((tab.moved_by(C, cg) >> 16) + cg == c) {  // the last group out closes C
                    tab.clear(C);
                    if (split) {
                        tab.set_last(C, nw - 1);
                        atomicOr((unsigned long long *)&starts[nw >> 6], 1ull << (nw & 63));
                    }
                }
                m &= ~g;
            }
        } else {
            for (uint64_t m = nb; m; m &= m - 1) {
                const int y = (int)wbase + ctz64(m);
                const uint32_t C = m == nb ? C0 : (uint32_t)cls[y];
                const uint32_t c = tab.word(C) & 0xFFFFu;  // final neighbour count of C
                const uint32_t last = tab.last(C);
                const bool split = c < last - C + 1;
                const uint32_t nw = last + 1 - c;
                if (split) {
                    cls[y] = (uint16_t)nw;
                    tab.set_last(nw, last);
                }
                if ((tab.moved(C) >> 16) == c - 1) {  // the last one out closes C
                    tab.clear(C);
                    if (split) {
                        tab.set_last(C, nw - 1);
                        atomicOr((unsigned long long *)&starts[nw >> 6], 1ull << (nw & 63));
                        if constexpr (Tabs::kSole)
                            if (c == 1) tab.set_sole(nw, (uint32_t)y);  // y alone in its new class
                    }
                }
            }
        }
        if (xrem) tm.sync();  // barrier B: nothing to order when the pivot split nothing
        x = xn;
        rw = rwn;
        rp = rpn;
        xp = pn;
        if (tail) {
            ++i;
            break;
        }
    }
    if (!kPeo && !kIlv && tail) {
        // Tail: no unnumbered vertex has an unnumbered neighbour, so nothing
        // splits any more and the remaining steps only walk down the classes,
        // smallest id first within a class. With U0 = n - i unnumbered
        // vertices on positions [0, U0), class C = [C, E - 1] (E the next
        // class start above C, or U0) is numbered from step i + U0 - E on.
        // A one-vertex class (E = C + 1) fixes its vertex's rank at once;
        // every other class is ranked by one team prefix sum over its
        // members. This is the outcome of the remaining steps, computed
        // without taking them one by one.
        const uint32_t U0 = (uint32_t)(n - i);
        const uint32_t i0 = (uint32_t)i;
        auto is_start = [&](uint32_t p) { return (starts[p >> 6] >> (p & 63)) & 1ull; };
        for (uint64_t m = um; m; m &= m - 1) {
            const int v = (int)wbase + ctz64(m);
            const uint32_t C = cls[v];
            if (C + 1u == U0 || is_start(C + 1u)) {
                const uint32_t r = i0 + U0 - 1u - C;
                rank[v] = (int32_t)r;
                order[r] = v;
            }
        }
        uint32_t E = U0;  // start of the class above the words still to come
        for (int w = (int)((U0 - 1u) >> 6); w >= 0; --w) {
            uint64_t sw = starts[w];
            if ((uint32_t)w == ((U0 - 1u) >> 6)) sw &= ~0ull >> (63 - ((U0 - 1u) & 63));
            // A start p heads a one-position class iff p + 1 is a start or
            // is U0 (a virtual start; inside this word, or the next word's
            // first position as the carry).
            const uint64_t carry = E == ((uint32_t)(w + 1) << 6) ? (1ull << 63) : 0ull;
            const uint64_t virt = sw | ((uint32_t)w == (U0 >> 6) ? (1ull << (U0 & 63)) : 0ull);
            uint64_t multi = sw & ~((virt >> 1) | carry);  // classes of two or more positions
            while (multi) {
                const int b = 63 - __builtin_clzll(multi);
                multi &= ~(1ull << b);
                const uint32_t C = ((uint32_t)w << 6) | (uint32_t)b;
                const uint64_t above = b == 63 ? 0ull : sw & (~0ull << (b + 1));
                const uint32_t Ec = above ? (((uint32_t)w << 6) | (uint32_t)ctz64(above)) : E;
                const uint64_t mine = chunk_match<kMatchG>(cls, um, C, vbase, sh, K);
                const uint32_t cnt_l = (uint32_t)__popcll(mine);
                uint32_t r = i0 + (U0 - Ec) + tm.exclusive_scan(cnt_l, red + par * 2 * NW);
                for (uint64_t q = mine; q; q &= q - 1) {
                    const int v = (int)wbase + ctz64(q);
                    rank[v] = (int32_t)r;
                    order[r] = v;
                    ++r;
                }
            }
            if (sw) E = ((uint32_t)w << 6) | (uint32_t)ctz64(sw);
        }
    }
    if (kPeo) {
        tm.sync();
        // Outputs once per graph, from LDS: parents, and ranks from the class
        // id slots of the numbered vertices.
        for (int v = t; v < n; v += T) {
            const uint32_t p = fp.par[v];
            parent[v] = p == kNoParent ? -1 : (int32_t)p;
            const int32_t r = (int32_t)cls[v];
            rank[v] = r;
            order[r] = (int32_t)v;
        }
        if (t == 0) g_store(fp.failkey, *fp.fk);
    }
}

// ---------------------------------------------------------------------------
// Compact LexBFS state for large n (4 bytes + 1/8 byte per vertex in LDS).
// No class-end table: the last position of class c is the start of the next
// live class above it minus one (or U - 1 for the top class), found in a
// two-level bitmap of class starts (level 1 marks the non-zero words of
// level 0). Split counters are 16 bits; the first neighbour of a class to
// count itself leads it, and the classes are closed in a third phase after
// a barrier (no "moved" counter, no rem).
//   starts u64[wn] | sum u64[wn/64] | red u32[4 waves] | cls u16[n] | cnt u16[n]
// ---------------------------------------------------------------------------
__host__ __device__ inline size_t lds_bytes_compact(int n, int team)
{
    const size_t wn = (size_t)(n + 63) / 64;
    const size_t ws = (wn + 63) / 64;
    const size_t nred = (size_t)(team / kWave > 0 ? team / kWave : 1);
    return align_up(8 * wn, 16) + align_up(8 * ws, 16) + align_up(16 * nred, 16) + 2 * align_up(2 * (size_t)n, 16);
}

struct CompactLayout {
    uint64_t *starts;
    uint64_t *sum;
    uint32_t *red;
    uint16_t *cls;
    uint16_t *cnt;
};

__device__ __forceinline__ CompactLayout carve_compact(void *base, int n, int team)
{
    const size_t wn = (size_t)(n + 63) / 64;
    const size_t ws = (wn + 63) / 64;
    const size_t nred = (size_t)(team / kWave > 0 ? team / kWave : 1);
    const size_t a = align_up(2 * (size_t)n, 16);
    char *p = (char *)base;
    CompactLayout L;
    L.starts = (uint64_t *)p;
    p += align_up(8 * wn, 16);
    L.sum = (uint64_t *)p;
    p += align_up(8 * ws, 16);
    L.red = (uint32_t *)p;
    p += align_up(16 * nred, 16);
    L.cls = (uint16_t *)p;
    L.cnt = (uint16_t *)(p + a);
    return L;
}

// Start of the first live class above position c, or U if there is none.
__device__ __forceinline__ uint32_t next_start(const uint64_t *starts, const uint64_t *sum, int nsum, uint32_t c,
                                               uint32_t U)
{
    const uint32_t w = c >> 6;
    const uint32_t b = c & 63u;
    const uint64_t m = b == 63u ? 0ull : starts[w] & (~0ull << (b + 1u));
    if (m) return min(U, (w << 6) + (uint32_t)ctz64(m));
    const uint32_t w1 = w + 1u;
    for (int s1 = (int)(w1 >> 6); s1 < nsum; ++s1) {
        uint64_t mm = sum[s1];
        if (s1 == (int)(w1 >> 6)) mm &= ~0ull << (w1 & 63u);
        if (mm) {
            const uint32_t ww = ((uint32_t)s1 << 6) + (uint32_t)ctz64(mm);
            return min(U, (ww << 6) + (uint32_t)ctz64(starts[ww]));
        }
    }
    return U;
}

// The highest class start at or below position pos (position 0 always
// starts a class). Words above pos >> 6 are never consulted in the summary,
// so a concurrent clear of a start above pos does not disturb the lookup.
__device__ __forceinline__ uint32_t prev_start(const uint64_t *starts, const uint64_t *sum, uint32_t pos)
{
    const uint32_t w = pos >> 6;
    const uint64_t m = starts[w] & (~0ull >> (63u - (pos & 63u)));
    if (m) return (w << 6) | (uint32_t)(63 - __builtin_clzll(m));
    if (w == 0) return 0;
    const uint32_t w1 = w - 1u;
    for (int s1 = (int)(w1 >> 6); s1 >= 0; --s1) {
        uint64_t mm = sum[s1];
        if (s1 == (int)(w1 >> 6)) mm &= ~0ull >> (63u - (w1 & 63u));
        if (mm) {
            const uint32_t ww = ((uint32_t)s1 << 6) | (uint32_t)(63 - __builtin_clzll(mm));
            return (ww << 6) | (uint32_t)(63 - __builtin_clzll(starts[ww]));
        }
    }
    return 0;
}

template <class Team>
__device__ __forceinline__ void lexbfs_team_compact(const Team &tm, int n, const uint64_t *bits_, int64_t W, int32_t *order_,
                                    int32_t *rank_, int32_t *parent_, const CompactLayout &L)
{
    LX_GLOBAL const uint64_t *__restrict__ bits = as_global(bits_);
    LX_GLOBAL int32_t *__restrict__ order = as_global(order_);
    LX_GLOBAL int32_t *__restrict__ rank = as_global(rank_);
    LX_GLOBAL int32_t *__restrict__ parent = as_global(parent_);
    constexpr int T = Team::kSize;
    constexpr int NW = Team::kWaves;
    uint64_t *starts = L.starts, *sum = L.sum;
    uint16_t *cls = L.cls, *cnt = L.cnt;
    uint32_t *red = L.red;
    const int t = tm.tid;
    if (n <= 0) return;
    const int wn = (n + 63) >> 6;
    const int nsum = (wn + 63) >> 6;
    int K = 1;
    while (K * T < n) K <<= 1;
    const int vbase = t * K;
    const int wi = vbase >> 6;
    const int sh = vbase & 63;
    const uint32_t wbase = (uint32_t)wi << 6;
    uint64_t cmask = (K == 64) ? ~0ull : (((1ull << K) - 1ull) << sh);
    if (wi == wn - 1 && (n & 63)) cmask &= (1ull << (n & 63)) - 1ull;
    const bool owner = vbase < n;
    LX_GLOBAL const uint64_t *rowbase = bits + wi;
    auto cnt_inc = [&](uint32_t c) -> uint32_t {
        const uint32_t s = (c & 1u) * 16u;
        return (atomicAdd((uint32_t *)cnt + (c >> 1), 1u << s) >> s) & 0xFFFFu;
    };

    for (int v = t; v < n; v += T) {
        cls[v] = 0;
        cnt[v] = 0;
    }
    for (int w = t; w < wn; w += T) starts[w] = w == 0 ? 1ull : 0ull;
    for (int w = t; w < nsum; w += T) sum[w] = w == 0 ? 1ull : 0ull;
    if (owner)
        for (int v = vbase; v < min(vbase + K, n); ++v) parent[v] = -1;
    tm.sync();

    uint64_t um = owner ? cmask : 0ull;
    uint64_t top = um;
    uint32_t x = 0;
    uint64_t rw = owner ? rowbase[0] : 0ull;
    int par = 0;
    int U = n;
    for (int i = 0; i < n; ++i) {
        U -= 1;
        const uint32_t stop = cls[x];
        if (owner && (x >> 6) == (uint32_t)wi) {
            um &= ~(1ull << (x & 63));
            top &= ~(1ull << (x & 63));
        }
        uint64_t nb = rw & um;
        __asm__ volatile("" : "+v"(nb)::"memory");
        if (t == 0) {
            if ((int)stop >= U) {  // the top class is gone
                const uint64_t left =
                    atomicAnd((unsigned long long *)&starts[stop >> 6], ~(1ull << (stop & 63))) & ~(1ull << (stop & 63));
                if (!left) atomicAnd((unsigned long long *)&sum[stop >> 12], ~(1ull << ((stop >> 6) & 63)));
            }
            order[i] = (int32_t)x;
            rank[x] = i;
        }
        // Phase A: count neighbours per class; the first one leads the class.
        uint64_t lead = 0;
        for (uint64_t m = nb; m; m &= m - 1) {
            const int b = ctz64(m);
            const int y = (int)wbase + b;
            const uint32_t C = cls[y];
            parent[y] = (int32_t)x;
            if (cnt_inc(C) == 0) lead |= 1ull << b;
        }
        if (i + 1 == n) break;
        if ((int)stop >= U) {
            // x emptied the top class: the candidate is the class holding
            // position U - 1, found by every lane alike from the class-start
            // bitmap and its summary (no team scan and no extra reduction).
            top = chunk_match(cls, um, prev_start(starts, sum, (uint32_t)(U - 1)), vbase, sh, K);
        }
        const uint32_t k = tm.max_all(pick_key(top, nb, wbase), red + par * 2 * NW);
        par ^= 1;
        const uint32_t xn = 0xFFFFu - (k & 0xFFFFu);
        if ((k >> 16) == 2) top &= nb;
        const uint64_t rwn = owner ? rowbase[(int64_t)xn * W] : 0ull;

        // Phase B: move the neighbours up; leaders remember the old class.
        uint64_t split = 0;
        for (uint64_t m = nb; m; m &= m - 1) {
            const int b = ctz64(m);
            const int y = (int)wbase + b;
            const uint32_t C = cls[y];
            const uint32_t c = cnt[C];
            const uint32_t last = next_start(starts, sum, nsum, C, (uint32_t)U) - 1u;
            if (c < last - C + 1) {
                const uint32_t nw = last + 1 - c;
                cls[y] = (uint16_t)nw;
                if ((lead >> b) & 1ull) {
                    cnt[nw] = (uint16_t)C;
                    split |= 1ull << b;
                }
            }
        }
        tm.sync();
        // Phase C: leaders close their classes and publish the new starts.
        for (uint64_t m = lead; m; m &= m - 1) {
            const int b = ctz64(m);
            const uint32_t nw = cls[(int)wbase + b];
            if ((split >> b) & 1ull) {
                cnt[cnt[nw]] = 0;
                cnt[nw] = 0;
                atomicOr((unsigned long long *)&starts[nw >> 6], 1ull << (nw & 63));
                atomicOr((unsigned long long *)&sum[nw >> 12], 1ull << ((nw >> 6) & 63));
            } else {
                cnt[nw] = 0;
            }
        }
        tm.sync();
        x = xn;
        rw = rwn;
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
// p(v) from a finished order: the neighbour of largest rank below rank(v)
// (the latest earlier neighbour of Section 5.2), or -1. One wavefront per
// vertex: its lanes split v's CSR row and a wave max picks the rank.
// Vertices v = first, first + stride, ...
__device__ __forceinline__ void derive_parents(const int32_t *row_ptr_, const int32_t *col_idx_, const int32_t *order_,
                                               const int32_t *rank_, int32_t *parent_, int n, int first, int stride)
{
    LX_GLOBAL const int32_t *rp = as_global(row_ptr_);
    LX_GLOBAL const int32_t *ci = as_global(col_idx_);
    LX_GLOBAL const int32_t *order = as_global(order_);
    LX_GLOBAL const int32_t *rank = as_global(rank_);
    LX_GLOBAL int32_t *parent = as_global(parent_);
    const int lane = threadIdx.x & 63;
    for (int v = first; v < n; v += stride) {
        const int rv = rank[v];
        uint32_t best = 0;  // rank + 1 of the latest earlier neighbour so far
        for (int j = rp[v] + lane; j < rp[v + 1]; j += kWave) {
            const int ru = rank[ci[j]];
            if (ru < rv) best = max(best, (uint32_t)ru + 1u);
        }
        best = wave_max_u32(best);
        if (lane == 0) parent[v] = best ? order[best - 1] : -1;
    }
}

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

template <bool kWide>
__device__ __forceinline__ void sweep_rows(const uint64_t *bits_, int64_t W, int wn, const int32_t *rank_,
                                           const int32_t *parent_, int n, int r0, int r1, int G, int lg,
                                           uint32_t *failkey_)
{
    LX_GLOBAL const uint64_t *__restrict__ bits = as_global(bits_);
    LX_GLOBAL const int32_t *__restrict__ rank = as_global(rank_);
    LX_GLOBAL const int32_t *__restrict__ parent = as_global(parent_);
    LX_GLOBAL uint32_t *failkey = as_global(failkey_);
    const uint64_t tail = (n & 63) ? ((1ull << (n & 63)) - 1ull) : ~0ull;
    const int lane = threadIdx.x & 63;
    const int gid = lane >> lg;
    const int gl = lane & (G - 1);
    const int gpw = kWave >> lg;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (gid * G));
    const bool wide = kWide && G == kWave && !(W & 1) && !(wn & 1) && !((uintptr_t)bits_ & 15);
    uint32_t best = kNoFail;  // smallest failing rank among this lane group's rows
    for (int vb = r0 + wave * gpw; vb < r1; vb += nwaves * gpw) {
        const int v = vb + gid;
        bool fail = false;
        int rv = 0;
        if (wide) {
            // Rows of whole 16-byte pairs on 16-byte boundaries, one row per
            // wavefront (so v < r1 on every lane): 16-byte loads, four pairs
            // of each row per lane in flight, and the first round of row v
            // requested before v's parent id is in (its address needs only
            // v). No load sits under a branch, which would make the compiler
            // sink the row loads behind the wait for the parent id; a vertex
            // without a parent tests its row against itself, leaving no bit
            // to look up. 0.103 ms per 512 MiB bitset, against 0.108 with the
            // row requested after the parent id and 0.121 with 8-byte loads.
            const int np = wn >> 1;
            const int vr = min(v, r1 - 1);
            LX_GLOBAL const u64x2 *a2 = (LX_GLOBAL const u64x2 *)(bits + (int64_t)vr * W);
            u64x2 A[4], B[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) A[u] = __builtin_nontemporal_load(a2 + min(gl + u * G, np - 1));
            const int p = parent[vr];
            const int pr = p >= 0 ? p : vr;
            rv = rank[vr];
            const int rp = rank[pr];
            LX_GLOBAL const u64x2 *b2 = (LX_GLOBAL const u64x2 *)(bits + (int64_t)pr * W);
            for (int q0 = gl;;) {
#pragma unroll
                for (int u = 0; u < 4; ++u) B[u] = b2[min(q0 + u * G, np - 1)];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + u * G;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int w = 2 * q + h;
                        uint64_t X = q < np ? A[u][h] & ~B[u][h] : 0ull;
                        if (w == wn - 1) X &= tail;  // ids >= n never index rank[]
                        while (X && !fail) {
                            const int z = (w << 6) + ctz64(X);
                            X &= X - 1;
                            if (rank[z] < rp) fail = true;
                        }
                    }
                }
                q0 += 4 * G;
                if (q0 >= np || fail) break;
#pragma unroll
                for (int u = 0; u < 4; ++u) A[u] = __builtin_nontemporal_load(a2 + min(q0 + u * G, np - 1));
            }
        } else if (v < r1) {
            const int p = parent[v];
            if (p >= 0) {
                rv = rank[v];
                const int rp = rank[p];
                LX_GLOBAL const uint64_t *a = bits + (int64_t)v * W;
                LX_GLOBAL const uint64_t *b = bits + (int64_t)p * W;
                // Eight words of both rows per lane in flight before any is
                // tested (the early exit would otherwise serialise the loads).
                for (int w0 = gl; w0 < wn && !fail; w0 += 8 * G) {
                    // Addresses clamped to the last word rather than loads
                    // made conditional: conditional loads compile to branches
                    // that each wait for the loads before them.
                    uint64_t A[8], B[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int w = min(w0 + u * G, wn - 1);
                        A[u] = __builtin_nontemporal_load(a + w);
                        B[u] = b[w];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int w = w0 + u * G;
                        uint64_t X = w < wn ? A[u] & ~B[u] : 0ull;
                        if (w == wn - 1) X &= tail;  // ids >= n never index rank[]
                        while (X && !fail) {
                            const int z = (w << 6) + ctz64(X);
                            X &= X - 1;
                            if (rank[z] < rp) fail = true;
                        }
                    }
                }
            }
        }
        const uint64_t bal = __ballot(fail);
        if (bal & gmask) best = min(best, (uint32_t)rv);
    }
    // At most one atomic per wavefront, and only when it would lower the
    // current minimum: in a graph where most rows fail, an atomic per failing
    // row (or even per wavefront) queues thousands of them on one L2 word.
    best = wave_min_u32(best);
    if (lane == 0 && best != kNoFail &&
        best < __hip_atomic_load(failkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        __hip_atomic_fetch_min(failkey, best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Maximum Cardinality Search (Section 5.1): the label of a vertex is the
// number of its numbered neighbours; each step numbers an unnumbered vertex
// of largest label, smallest id first (the same tie-break as LexBFS).
//
// State: cnt[v] (16 bits, LDS), written only by v's owner lane, so the
// steps need no class tables and no second barrier. Every lane keeps, as a
// bitmask over its own vertices, the members of the top bucket (label =
// cmax, uniform). When x is numbered its unnumbered neighbours gain one:
//   A = top & N(x) now have cmax + 1  -> the next pivot is min(A) if any;
//   B = (top \ N(x)) + the neighbours that reach cmax
//                                     -> else min(B), the top stays cmax;
//   else no label cmax or cmax + 1 is left: every lane offers its best
//   (label, -id) and a second reduction finds the new cmax and pivot.
// One reduction per step (prioritised keys A over B); the parent of y is
// the last pivot adjacent to y, recorded when its count rises.
// ---------------------------------------------------------------------------
__host__ __device__ inline size_t lds_bytes_mcs(int n, int team, bool with_par)
{
    const size_t nred = (size_t)(team / kWave > 0 ? team / kWave : 1);
    const size_t a = align_up(2 * (size_t)n, 16);
    return align_up(16 * nred, 16) + a + (with_par ? a + 16 : 0);
}

struct McsLayout {
    uint32_t *red;
    uint16_t *cnt;
    FusedPeo fp;
};

__device__ __forceinline__ McsLayout carve_mcs(void *base, int n, int team, bool with_par, uint32_t *failkey)
{
    const size_t nred = (size_t)(team / kWave > 0 ? team / kWave : 1);
    const size_t a = align_up(2 * (size_t)n, 16);
    char *p = (char *)base;
    McsLayout L;
    L.red = (uint32_t *)p;
    p += align_up(16 * nred, 16);
    L.cnt = (uint16_t *)p;
    p += a;
    L.fp.par = with_par ? (uint16_t *)p : nullptr;
    L.fp.fk = with_par ? (uint32_t *)(p + a) : nullptr;
    L.fp.failkey = failkey;
    return L;
}

// Best (label + 1, -id) key over my unnumbered vertices `um` (0 if none),
// and, for a given label c, the mask of those with that label.
__device__ __forceinline__ uint32_t mcs_lane_best(const uint16_t *cnt, uint64_t um, int vbase, int sh, int K)
{
    uint32_t best = 0;
    const int wbase = (vbase >> 6) << 6;
    for (uint64_t m = um; m; m &= m - 1) {
        const int v = wbase + ctz64(m);
        const uint32_t c = min((uint32_t)cnt[v] + 1u, 0xFFFFu);
        best = max(best, (c << 16) | (0xFFFFu - (uint32_t)v));
    }
    (void)sh;
    (void)K;
    return best;
}

template <int kG>
__device__ __forceinline__ uint64_t mcs_lane_match(const uint16_t *cnt, uint64_t um, uint32_t c, int vbase, int sh, int K)
{
    return chunk_match<kG>(cnt, um, c, vbase, sh, K);
}

// kMatchG: 16-byte groups of a chunk matched per LDS round trip (chunk_match).
template <class Team, bool kPeo = false, int kMatchG = 8>
__device__ __forceinline__ void mcs_team(const Team &tm, int n, const uint64_t *bits_, int64_t W, int32_t *order_, int32_t *rank_,
                         int32_t *parent_, const McsLayout &L)
{
    LX_GLOBAL const uint64_t *__restrict__ bits = as_global(bits_);
    LX_GLOBAL int32_t *__restrict__ order = as_global(order_);
    LX_GLOBAL int32_t *__restrict__ rank = as_global(rank_);
    LX_GLOBAL int32_t *__restrict__ parent = as_global(parent_);
    constexpr int T = Team::kSize;
    constexpr int NW = Team::kWaves;
    uint16_t *cnt = L.cnt;
    uint32_t *red = L.red;
    const FusedPeo &fp = L.fp;
    const int t = tm.tid;
    if (n <= 0) return;
    const int wn = (n + 63) >> 6;
    int K = 1;
    while (K * T < n) K <<= 1;
    const int vbase = t * K;
    const int wi = vbase >> 6;
    const int sh = vbase & 63;
    const uint32_t wbase = (uint32_t)wi << 6;
    uint64_t cmask = (K == 64) ? ~0ull : (((1ull << K) - 1ull) << sh);
    if (wi == wn - 1 && (n & 63)) cmask &= (1ull << (n & 63)) - 1ull;
    const bool owner = vbase < n;
    LX_GLOBAL const uint64_t *rowbase = bits + wi;

    if (owner)
        for (int v = vbase; v < min(vbase + K, n); ++v) {
            cnt[v] = 0;
            if (kPeo) fp.par[v] = kNoParent;
            else parent[v] = -1;
        }
    if (kPeo && t == 0) *fp.fk = kNoFail;
    tm.sync();

    uint64_t um = owner ? cmask : 0ull;  // my unnumbered vertices
    uint64_t top = um;                   // my vertices of label cmax
    uint32_t cmax = 0;
    uint32_t x = 0;
    uint64_t rw = owner ? rowbase[0] : 0ull;
    uint32_t xp = kNoParent;
    uint64_t rp = 0ull;
    int par = 0;
    for (int i = 0; i < n; ++i) {
        if (owner && (x >> 6) == (uint32_t)wi) {
            um &= ~(1ull << (x & 63));
            top &= ~(1ull << (x & 63));
        }
        uint64_t nb = rw & um;
        uint64_t bad = 0ull;
        if (kPeo && xp != kNoParent) {
            bad = rw & ~um & cmask & ~rp;
            if ((xp >> 6) == (uint32_t)wi) bad &= ~(1ull << (xp & 63));
        }
        __asm__ volatile("" : "+v"(nb), "+v"(bad)::"memory");
        if (kPeo && bad) atomicMin(fp.fk, (uint32_t)i);
        if (t == 0) {
            order[i] = (int32_t)x;
            rank[x] = i;
        }
        // Raise my neighbours' labels; those reaching cmax join the top.
        uint64_t prom = 0ull;
        for (uint64_t m = nb; m; m &= m - 1) {
            const int y = (int)wbase + ctz64(m);
            const uint32_t c = (uint32_t)cnt[y] + 1u;
            cnt[y] = (uint16_t)c;
            if (kPeo) fp.par[y] = (uint16_t)x;
            else parent[y] = (int32_t)x;
            if (c == cmax) prom |= m & (~m + 1);
        }
        if (i + 1 == n) break;
        const uint64_t A = top & nb;
        const uint64_t B = (top & ~nb) | prom;
        uint32_t key = 0;
        if (A) key = 0x20000u | (0xFFFFu - (wbase + (uint32_t)ctz64(A)));
        else if (B) key = 0x10000u | (0xFFFFu - (wbase + (uint32_t)ctz64(B)));
        uint32_t k = tm.max_all(key, red + par * 2 * NW);
        par ^= 1;
        if ((k >> 16) == 2) {
            cmax += 1;
            top = A;
        } else if ((k >> 16) == 1) {
            top = B;
        } else {
            k = tm.max_all(mcs_lane_best(cnt, um, vbase, sh, K), red + par * 2 * NW);
            par ^= 1;
            cmax = (k >> 16) - 1u;
            top = mcs_lane_match<kMatchG>(cnt, um, cmax, vbase, sh, K);
        }
        const uint32_t xn = 0xFFFFu - (k & 0xFFFFu);
        const uint32_t pn = kPeo ? (uint32_t)fp.par[xn] : kNoParent;
        const uint64_t rwn = owner ? rowbase[(int64_t)xn * W] : 0ull;
        const uint64_t rpn = (kPeo && owner && pn != kNoParent) ? rowbase[(int64_t)pn * W] : 0ull;
        x = xn;
        rw = rwn;
        rp = rpn;
        xp = pn;
    }
    if (kPeo) {
        tm.sync();
        if (owner)
            for (int v = vbase; v < min(vbase + K, n); ++v) {
                const uint32_t p = fp.par[v];
                parent[v] = p == kNoParent ? -1 : (int32_t)p;
            }
        if (t == 0) g_store(fp.failkey, *fp.fk);
    }
}

}  // namespace lxd
