/*
 * graphgen.c -- seeded synthetic graph generators.
 *
 * This module produces inputs only. It holds none of the chordality method's
 * arithmetic (no ordering, no elimination test); both the CPU oracle and the
 * GPU library receive the arrays it writes.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood 2014) seeds xoshiro256**
 * (Blackman and Vigna 2018). Both are written here from their published
 * definitions.
 *
 * Graph layout written by every generator: an N x N adjacency bitset, row v
 * at bits + v*W, bit u of row v is word u>>6, bit u&63 (LSB first). The
 * caller allocates the rows zero-filled; generators only set bits, always
 * symmetrically and never on the diagonal. gg_bits_to_csr derives a sorted
 * int32 CSR from the bitset.
 *
 * Build: gcc -O2 -shared -fPIC graphgen.c -o libgraphgen.so -lm
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* Random numbers                                                            */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t s[4]; } gg_rng;

/* SplitMix64: advance the state by the golden-ratio increment, then apply
 * the two xor-shift-multiply rounds and a final xor-shift. */
static uint64_t splitmix64(uint64_t *state)
{
    uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

/* xoshiro256**: output rotl(s1 * 5, 7) * 9, then the linear state update. */
static uint64_t rng_next(gg_rng *r)
{
    uint64_t *s = r->s;
    const uint64_t out = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return out;
}

static void rng_seed(gg_rng *r, uint64_t seed)
{
    uint64_t st = seed;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&st);
}

/* Uniform integer in [0, k) by the 128-bit multiply-high map. */
static inline uint64_t rng_below(gg_rng *r, uint64_t k)
{
    return (uint64_t)(((unsigned __int128)rng_next(r) * k) >> 64);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double rng_unit(gg_rng *r)
{
    return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

/* Per-graph seed: SplitMix64 applied to (config_seed, index). */
uint64_t gg_graph_seed(uint64_t config_seed, uint64_t index)
{
    uint64_t st = config_seed ^ (index * 0xd1b54a32d192ed03ULL);
    splitmix64(&st);
    return splitmix64(&st);
}

/* Exposed for tests: n draws of xoshiro256** seeded through SplitMix64. */
void gg_rng_stream(uint64_t seed, int64_t n, uint64_t *out)
{
    gg_rng r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < n; i++) out[i] = rng_next(&r);
}

/* Exposed for tests: n raw SplitMix64 outputs from the given state. */
void gg_splitmix_stream(uint64_t state, int64_t n, uint64_t *out)
{
    for (int64_t i = 0; i < n; i++) out[i] = splitmix64(&state);
}

/* ------------------------------------------------------------------------ */
/* Bitset helpers                                                            */
/* ------------------------------------------------------------------------ */

static inline void set_edge(uint64_t *bits, int64_t W, int64_t u, int64_t v)
{
    bits[u * W + (v >> 6)] |= 1ULL << (v & 63);
    bits[v * W + (u >> 6)] |= 1ULL << (u & 63);
}

static inline int has_edge(const uint64_t *bits, int64_t W, int64_t u, int64_t v)
{
    return (int)((bits[u * W + (v >> 6)] >> (v & 63)) & 1ULL);
}

/* ------------------------------------------------------------------------ */
/* SUBTREE(n, T, smax): intersection graph of subtrees of a random tree.     */
/* Host tree: uniform labelled tree on T nodes decoded from a uniform Pruefer */
/* sequence. Vertex v: uniform root, size s uniform in [1, smax], BFS from    */
/* the root that shuffles the tree neighbours of each dequeued node, keeping  */
/* the first min(s, T) nodes reached. u ~ w iff their node sets intersect.    */
/* Writes vertices [0, n) into a bitset whose row stride W may exceed n/64.   */
/* ------------------------------------------------------------------------ */

static int prufer_tree(int T, gg_rng *r, int *eu, int *ev)
{
    /* Returns T-1 edges (eu[i], ev[i]). */
    if (T <= 1) return 0;
    if (T == 2) { eu[0] = 0; ev[0] = 1; return 1; }
    int m = T - 2;
    int *seq = (int *)malloc(sizeof(int) * (size_t)m);
    int *deg = (int *)malloc(sizeof(int) * (size_t)T);
    if (!seq || !deg) { free(seq); free(deg); return -1; }
    for (int i = 0; i < T; i++) deg[i] = 1;
    for (int i = 0; i < m; i++) { seq[i] = (int)rng_below(r, (uint64_t)T); deg[seq[i]]++; }
    /* Linear-time decoding: walk a pointer over leaves in increasing label. */
    int ptr = 0;
    while (deg[ptr] != 1) ptr++;
    int leaf = ptr, k = 0;
    for (int i = 0; i < m; i++) {
        int s = seq[i];
        eu[k] = leaf; ev[k] = s; k++;
        deg[leaf]--;
        deg[s]--;
        if (deg[s] == 1 && s < ptr) {
            leaf = s;
        } else {
            ptr++;
            while (deg[ptr] != 1) ptr++;
            leaf = ptr;
        }
    }
    /* The last two nodes of degree 1. */
    int a = -1, b = -1;
    for (int i = 0; i < T; i++) if (deg[i] == 1) { if (a < 0) a = i; else if (b < 0) b = i; }
    eu[k] = a; ev[k] = b; k++;
    free(seq); free(deg);
    return k;
}

int gg_subtree(int n, int T, int smax, uint64_t seed, uint64_t *bits, int64_t W)
{
    if (n < 0 || T < 1 || smax < 1 || (int64_t)n > W * 64) return -1;
    gg_rng r;
    rng_seed(&r, seed);
    int *eu = (int *)malloc(sizeof(int) * (size_t)(T > 1 ? T - 1 : 1));
    int *ev = (int *)malloc(sizeof(int) * (size_t)(T > 1 ? T - 1 : 1));
    int ne = prufer_tree(T, &r, eu, ev);
    if (ne < 0) { free(eu); free(ev); return -1; }
    /* Tree adjacency as CSR. */
    int *tptr = (int *)calloc((size_t)T + 1, sizeof(int));
    int *tadj = (int *)malloc(sizeof(int) * (size_t)(2 * ne + 1));
    for (int i = 0; i < ne; i++) { tptr[eu[i] + 1]++; tptr[ev[i] + 1]++; }
    for (int i = 0; i < T; i++) tptr[i + 1] += tptr[i];
    int *fill = (int *)malloc(sizeof(int) * (size_t)T);
    memcpy(fill, tptr, sizeof(int) * (size_t)T);
    for (int i = 0; i < ne; i++) { tadj[fill[eu[i]]++] = ev[i]; tadj[fill[ev[i]]++] = eu[i]; }
    free(fill); free(eu); free(ev);

    /* Grow every vertex's subtree; record (node, vertex) memberships. */
    int64_t cap = (int64_t)n * (smax < T ? smax : T);
    int *mem_node = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
    int *mem_vert = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
    int *queue = (int *)malloc(sizeof(int) * (size_t)T);
    int *stamp = (int *)malloc(sizeof(int) * (size_t)T);
    int *nbuf = (int *)malloc(sizeof(int) * (size_t)T);
    for (int i = 0; i < T; i++) stamp[i] = -1;
    int64_t nm = 0;
    for (int v = 0; v < n; v++) {
        int root = (int)rng_below(&r, (uint64_t)T);
        int s = 1 + (int)rng_below(&r, (uint64_t)smax);
        if (s > T) s = T;
        int head = 0, tail = 0, kept = 0;
        queue[tail++] = root; stamp[root] = v;
        mem_node[nm] = root; mem_vert[nm] = v; nm++; kept++;
        while (head < tail && kept < s) {
            int u = queue[head++];
            int deg = tptr[u + 1] - tptr[u];
            for (int j = 0; j < deg; j++) nbuf[j] = tadj[tptr[u] + j];
            for (int j = deg - 1; j > 0; j--) {           /* Fisher-Yates */
                int k2 = (int)rng_below(&r, (uint64_t)(j + 1));
                int t = nbuf[j]; nbuf[j] = nbuf[k2]; nbuf[k2] = t;
            }
            for (int j = 0; j < deg && kept < s; j++) {
                int w = nbuf[j];
                if (stamp[w] == v) continue;
                stamp[w] = v;
                queue[tail++] = w;
                mem_node[nm] = w; mem_vert[nm] = v; nm++; kept++;
            }
        }
    }
    free(queue); free(stamp); free(nbuf); free(tptr); free(tadj);

    /* Bucket memberships by tree node, then connect all pairs per node. */
    int *bptr = (int *)calloc((size_t)T + 1, sizeof(int));
    for (int64_t i = 0; i < nm; i++) bptr[mem_node[i] + 1]++;
    for (int i = 0; i < T; i++) bptr[i + 1] += bptr[i];
    int *bfill = (int *)malloc(sizeof(int) * (size_t)T);
    memcpy(bfill, bptr, sizeof(int) * (size_t)T);
    int *bv = (int *)malloc(sizeof(int) * (size_t)(nm > 0 ? nm : 1));
    for (int64_t i = 0; i < nm; i++) bv[bfill[mem_node[i]]++] = mem_vert[i];
    for (int t = 0; t < T; t++)
        for (int a = bptr[t]; a < bptr[t + 1]; a++)
            for (int b = a + 1; b < bptr[t + 1]; b++)
                if (bv[a] != bv[b]) set_edge(bits, W, bv[a], bv[b]);
    free(bptr); free(bfill); free(bv); free(mem_node); free(mem_vert);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* GNP(n, p): each pair independently with probability p, by geometric       */
/* skipping over the lexicographic list of pairs (u < v).                    */
/* ------------------------------------------------------------------------ */
int gg_gnp(int n, double p, uint64_t seed, uint64_t *bits, int64_t W)
{
    if (n < 0 || (int64_t)n > W * 64 || !(p >= 0.0) || p > 1.0) return -1;
    if (n < 2 || p == 0.0) return 0;
    gg_rng r;
    rng_seed(&r, seed);
    if (p == 1.0) {
        for (int u = 0; u < n; u++) for (int v = u + 1; v < n; v++) set_edge(bits, W, u, v);
        return 0;
    }
    const double lq = log1p(-p);
    int64_t v = 1, w = -1;           /* current pair is (w, v) with w < v */
    for (;;) {
        double ru = rng_unit(&r);
        int64_t skip = (int64_t)floor(log1p(-ru) / lq);
        w += 1 + skip;
        while (w >= v && v < n) { w -= v; v++; }
        if (v >= n) break;
        set_edge(bits, W, w, v);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* SPLIT(K, I, a): clique on ids [0, K); each id in [K, K+I) is joined to a   */
/* uniform a-subset of the clique chosen by Floyd's sampling.                */
/* ------------------------------------------------------------------------ */
int gg_split(int K, int I, int a, uint64_t seed, uint64_t *bits, int64_t W)
{
    if (K < 0 || I < 0 || a < 0 || a > K || (int64_t)(K + I) > W * 64) return -1;
    gg_rng r;
    rng_seed(&r, seed);
    for (int u = 0; u < K; u++) for (int v = u + 1; v < K; v++) set_edge(bits, W, u, v);
    for (int i = 0; i < I; i++) {
        int64_t x = (int64_t)K + i;
        /* Floyd: for j = K-a .. K-1 pick t in [0, j]; take t unless taken, else j. */
        for (int j = K - a; j < K; j++) {
            int t = (int)rng_below(&r, (uint64_t)(j + 1));
            if (has_edge(bits, W, x, t)) t = j;
            set_edge(bits, W, x, t);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* PLANT(L): add the cycle on ids [n0, n0+L) and one bridge from n0 to a     */
/* uniform existing vertex in [0, n0). Needs n0 >= 1 for the bridge.         */
/* ------------------------------------------------------------------------ */
int gg_plant(int n0, int L, uint64_t seed, uint64_t *bits, int64_t W)
{
    if (n0 < 0 || L < 3 || (int64_t)(n0 + L) > W * 64) return -1;
    gg_rng r;
    rng_seed(&r, seed);
    for (int i = 0; i < L; i++) set_edge(bits, W, n0 + i, n0 + (i + 1) % L);
    if (n0 >= 1) set_edge(bits, W, n0, (int64_t)rng_below(&r, (uint64_t)n0));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Format helpers                                                            */
/* ------------------------------------------------------------------------ */

/* Number of set bits in rows [0, n) over the first ceil(n/64) words. */
int64_t gg_bits_nnz(int n, const uint64_t *bits, int64_t W)
{
    int64_t wn = ((int64_t)n + 63) >> 6, total = 0;
    for (int64_t v = 0; v < n; v++)
        for (int64_t w = 0; w < wn; w++) total += __builtin_popcountll(bits[v * W + w]);
    return total;
}

/* Sorted CSR from the bitset. row_ptr has n+1 entries, col_idx gg_bits_nnz. */
int gg_bits_to_csr(int n, const uint64_t *bits, int64_t W, int32_t *row_ptr, int32_t *col_idx)
{
    int64_t wn = ((int64_t)n + 63) >> 6, k = 0;
    row_ptr[0] = 0;
    for (int64_t v = 0; v < n; v++) {
        for (int64_t w = 0; w < wn; w++) {
            uint64_t x = bits[v * W + w];
            while (x) {
                int b = __builtin_ctzll(x);
                x &= x - 1;
                col_idx[k++] = (int32_t)(w * 64 + b);
            }
        }
        if (k > 0x7fffffffLL) return -1;
        row_ptr[v + 1] = (int32_t)k;
    }
    return 0;
}

/* Bitset from a list of undirected edges (test helper). */
int gg_edges_to_bits(int n, int64_t m, const int32_t *eu, const int32_t *ev, uint64_t *bits, int64_t W)
{
    for (int64_t i = 0; i < m; i++) {
        if (eu[i] < 0 || ev[i] < 0 || eu[i] >= n || ev[i] >= n || eu[i] == ev[i]) return -1;
        set_edge(bits, W, eu[i], ev[i]);
    }
    return 0;
}

/* Uniform random permutation of [0, n) (test helper for relabelling). */
void gg_permutation(int n, uint64_t seed, int32_t *perm)
{
    gg_rng r;
    rng_seed(&r, seed);
    for (int i = 0; i < n; i++) perm[i] = i;
    for (int i = n - 1; i > 0; i--) {
        int j = (int)rng_below(&r, (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/* Draws for the batch and serving mixes, consumed in this order per graph:
 * log-uniform N on [lo, hi], the planted cycle length L in [4, 12], and one
 * exponential inter-arrival gap with unit mean. */
void gg_mix_draws(uint64_t seed, int64_t count, double lo, double hi,
                  int32_t *n_out, int32_t *L_out, double *gap_out)
{
    gg_rng r;
    rng_seed(&r, seed);
    const double a = log(lo), b = log(hi);
    for (int64_t i = 0; i < count; i++) {
        double u = rng_unit(&r);
        double x = exp(a + (b - a) * u);
        int32_t nn = (int32_t)floor(x);
        if (nn < (int32_t)lo) nn = (int32_t)lo;
        if (nn > (int32_t)hi - 1 && hi > lo + 1) nn = (int32_t)hi - 1;
        n_out[i] = nn;
        L_out[i] = 4 + (int32_t)rng_below(&r, 9);
        gap_out[i] = -log1p(-rng_unit(&r));
    }
}

/* Shuffled type list for the 50/25/25 mix: 0 = SUBTREE, 1 = GNP, 2 = planted. */
void gg_mix_types(uint64_t seed, int64_t count, int32_t *types)
{
    gg_rng r;
    rng_seed(&r, seed);
    int64_t half = count / 2, quarter = count / 4;
    for (int64_t i = 0; i < count; i++)
        types[i] = i < half ? 0 : (i < half + quarter ? 1 : 2);
    for (int64_t i = count - 1; i > 0; i--) {
        int64_t j = (int64_t)rng_below(&r, (uint64_t)(i + 1));
        int32_t t = types[i]; types[i] = types[j]; types[j] = t;
    }
}
