/*
 * oracle.c -- plain sequential CPU oracle for LexBFS + perfect-elimination
 * test (Lupinska, "A Parallel Algorithm to Test Chordality of Graphs").
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library. It shares no code with the GPU
 * library: no headers, no helpers, no tables.
 *
 * Graph input: n vertices, int32 CSR (row_ptr[n+1], col_idx[nnz]); every row
 * ascending, symmetric, no self-loops, no duplicates. Vertex ids are 0-based;
 * order[i] is the vertex numbered at step i (the paper's pi(i+1)) and
 * rank = order^-1.
 *
 * Functions and the passages they follow:
 *   oracle_lexbfs       Section 4.2, partition-refinement LexBFS box, with the
 *                       label semantics of the Section 4.1 LexBFS box (the
 *                       appended number goes to the neighbour's label) and
 *                       the placement rule of Lemma 6.1 / Observation 6.2
 *                       (the part adjacent to the pivot goes directly before
 *                       its old class, i.e. it gets the larger label).
 *   oracle_peo          Section 5.2 box "Test if a LexBFS order is a perfect
 *                       elimination order", with the outer loop over x that
 *                       the box omits, "no parent" as -1, and every failing
 *                       vertex recorded (the box stops at the first).
 *   oracle_mcs          Section 5.1, Maximum Cardinality Search box: the
 *                       label of a vertex is the number of its numbered
 *                       neighbours (the box's "label_x = label_x + 1" is
 *                       read as the neighbour's label, the same reading as
 *                       for LexBFS), the largest label is taken next, ties
 *                       to the smallest id; parent = last adjacent pivot.
 *   oracle_certificate  A chordless cycle for a failing graph. The paper has
 *                       no certificate; the rule is a project definition
 *                       (shortest path in G[(V \ N[v*]) + {x*, z*}] with
 *                       smallest-id predecessors, plus a total fallback).
 *                       Parity of the certificate is pinned by its invariants
 *                       (a chordless cycle of length >= 4) and by brute force
 *                       on small graphs, not by the paper.
 *
 * Build: gcc -O2 -shared -fPIC oracle.c -o liboracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* LexBFS by partition refinement                                            */
/* ------------------------------------------------------------------------ */
/*
 * The unnumbered vertices are kept as an ordered list of classes; every class
 * holds vertices with equal labels, and the first class has the largest
 * label. Inside a class the vertices form a doubly-linked list in ascending
 * id order, so the head of the first class is the smallest id among the
 * vertices with the largest label (the tie-break used throughout).
 *
 * Step i: x = head of the first class; number it. Scan N(x) in ascending id
 * order; every unnumbered y leaves its class C for the class C' placed
 * directly before C (created at C's first hit in this step) and is appended
 * at the tail of C'. Scanning in ascending order keeps every class sorted.
 * Classes left empty are removed. The last pivot adjacent to y before y is
 * numbered is recorded as parent[y]: it is the latest-ordered earlier
 * neighbour p(y) of Section 5.2.
 */
typedef struct {
    int head, tail;        /* vertex list of the class */
    int prev, next;        /* neighbours in the class list (-1 = none) */
    int stamp;             /* step in which this class was last split */
    int child;             /* class created before it in that step */
    int size;
} klass;

int oracle_lexbfs(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                  int32_t *order, int32_t *rank, int32_t *parent)
{
    if (n < 0) return -1;
    if (n == 0) return 0;
    /* A step can hold every old class (some emptied, awaiting removal) next
     * to one new class per emptied one: at most 2n records are live. */
    const int cap = 2 * n + 2;
    klass *K = (klass *)malloc(sizeof(klass) * (size_t)cap);
    int *freelist = (int *)malloc(sizeof(int) * (size_t)cap);
    int *cls = (int *)malloc(sizeof(int) * (size_t)n);
    int *vprev = (int *)malloc(sizeof(int) * (size_t)n);
    int *vnext = (int *)malloc(sizeof(int) * (size_t)n);
    int *touched = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    if (!K || !freelist || !cls || !vprev || !vnext || !touched) {
        free(K); free(freelist); free(cls); free(vprev); free(vnext); free(touched);
        return -2;
    }
    int nfree = 0;
    for (int c = cap - 1; c >= 1; c--) freelist[nfree++] = c;

    /* One class (id 0) with every vertex, ascending, empty label. */
    K[0].head = 0; K[0].tail = n - 1; K[0].prev = -1; K[0].next = -1;
    K[0].stamp = -1; K[0].child = -1; K[0].size = n;
    for (int v = 0; v < n; v++) {
        cls[v] = 0; vprev[v] = v - 1; vnext[v] = (v + 1 < n) ? v + 1 : -1;
        rank[v] = -1; parent[v] = -1;
    }
    int first = 0;

    for (int i = 0; i < n; i++) {
        /* Pivot: first element of the first class. */
        int c0 = first;
        int x = K[c0].head;
        /* Remove x from its class. */
        K[c0].head = vnext[x];
        if (vnext[x] >= 0) vprev[vnext[x]] = -1; else K[c0].tail = -1;
        K[c0].size--;
        if (K[c0].size == 0) {
            first = K[c0].next;
            if (first >= 0) K[first].prev = -1;
            freelist[nfree++] = c0;
        }
        order[i] = x;
        rank[x] = i;

        /* Refine every class by N(x). */
        int ntouched = 0;
        for (int j = row_ptr[x]; j < row_ptr[x + 1]; j++) {
            int y = col_idx[j];
            if (rank[y] >= 0) continue;
            int C = cls[y];
            if (K[C].stamp != i) {
                /* New class directly before C: larger label than C, smaller
                 * than the class that preceded C. */
                int Cp = freelist[--nfree];
                K[Cp].head = -1; K[Cp].tail = -1; K[Cp].size = 0;
                K[Cp].stamp = -1; K[Cp].child = -1;
                K[Cp].next = C;
                K[Cp].prev = K[C].prev;
                if (K[C].prev >= 0) K[K[C].prev].next = Cp; else first = Cp;
                K[C].prev = Cp;
                K[C].stamp = i;
                K[C].child = Cp;
                touched[ntouched++] = C;
            }
            int Cp = K[C].child;
            /* Unlink y from C. */
            if (vprev[y] >= 0) vnext[vprev[y]] = vnext[y]; else K[C].head = vnext[y];
            if (vnext[y] >= 0) vprev[vnext[y]] = vprev[y]; else K[C].tail = vprev[y];
            K[C].size--;
            /* Append y to the tail of C'. */
            vprev[y] = K[Cp].tail;
            vnext[y] = -1;
            if (K[Cp].tail >= 0) vnext[K[Cp].tail] = y; else K[Cp].head = y;
            K[Cp].tail = y;
            K[Cp].size++;
            cls[y] = Cp;
            parent[y] = x;
        }
        /* Drop classes emptied by the refinement. */
        for (int t = 0; t < ntouched; t++) {
            int C = touched[t];
            if (K[C].size != 0) continue;
            if (K[C].prev >= 0) K[K[C].prev].next = K[C].next; else first = K[C].next;
            if (K[C].next >= 0) K[K[C].next].prev = K[C].prev;
            freelist[nfree++] = C;
        }
    }
    free(K); free(freelist); free(cls); free(vprev); free(vnext); free(touched);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Perfect-elimination test on a given order                                 */
/* ------------------------------------------------------------------------ */
/*
 * p[x] = the neighbour of x with the largest rank below rank[x] (-1 if x has
 * no earlier neighbour). For every x, mark N(x); for every neighbour y with
 * p[y] == x, each z in LN(y) other than x must be marked (LN(y) \ {p(y)} is a
 * subset of N(p(y)); restricting to earlier vertices makes N(x) and LN(x)
 * interchangeable here since every such z precedes x). A vertex y failing
 * this is recorded in fail[y].
 *
 * witness[0..2] = (v*, x*, z*): v* the failing vertex of smallest rank,
 * x* = p(v*), z* the smallest-rank vertex of LN(v*) \ {x*} not adjacent to
 * x*. All -1 when no vertex fails. Returns 1 if the order is a perfect
 * elimination order, 0 if not, < 0 on error.
 */
int oracle_peo(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *rank,
               int32_t *p, uint8_t *fail, int32_t *witness)
{
    if (n < 0) return -1;
    witness[0] = witness[1] = witness[2] = -1;
    if (n == 0) return 1;
    int *mark = (int *)malloc(sizeof(int) * (size_t)n);
    if (!mark) return -2;
    for (int x = 0; x < n; x++) {
        mark[x] = -1;
        fail[x] = 0;
        int best = -1;
        for (int j = row_ptr[x]; j < row_ptr[x + 1]; j++) {
            int y = col_idx[j];
            if (rank[y] < rank[x] && (best < 0 || rank[y] > rank[best])) best = y;
        }
        p[x] = best;
    }
    for (int x = 0; x < n; x++) {
        for (int j = row_ptr[x]; j < row_ptr[x + 1]; j++) mark[col_idx[j]] = x;
        for (int j = row_ptr[x]; j < row_ptr[x + 1]; j++) {
            int y = col_idx[j];
            if (p[y] != x) continue;
            for (int k = row_ptr[y]; k < row_ptr[y + 1]; k++) {
                int z = col_idx[k];
                if (rank[z] < rank[y] && z != x && mark[z] != x) { fail[y] = 1; break; }
            }
        }
    }
    int vstar = -1;
    for (int v = 0; v < n; v++)
        if (fail[v] && (vstar < 0 || rank[v] < rank[vstar])) vstar = v;
    free(mark);
    if (vstar < 0) return 1;
    int xs = p[vstar], zs = -1;
    for (int j = row_ptr[vstar]; j < row_ptr[vstar + 1]; j++) {
        int z = col_idx[j];
        if (rank[z] >= rank[vstar] || z == xs) continue;
        /* z adjacent to x*? binary search in the sorted row of x*. */
        int lo = row_ptr[xs], hi = row_ptr[xs + 1] - 1, found = 0;
        while (lo <= hi) {
            int mid = lo + (hi - lo) / 2;
            if (col_idx[mid] == z) { found = 1; break; }
            if (col_idx[mid] < z) lo = mid + 1; else hi = mid - 1;
        }
        if (!found && (zs < 0 || rank[z] < rank[zs])) zs = z;
    }
    witness[0] = vstar; witness[1] = xs; witness[2] = zs;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Chordless-cycle certificate                                               */
/* ------------------------------------------------------------------------ */

static int adjacent(const int32_t *row_ptr, const int32_t *col_idx, int u, int v)
{
    int lo = row_ptr[u], hi = row_ptr[u + 1] - 1;
    while (lo <= hi) {
        int mid = lo + (hi - lo) / 2;
        if (col_idx[mid] == v) return 1;
        if (col_idx[mid] < v) lo = mid + 1; else hi = mid - 1;
    }
    return 0;
}

/*
 * Layered BFS from src inside the vertex set A = (V \ N[c]) + {src, dst}:
 * L0 = {src}, L(j+1) = unvisited neighbours of L(j) inside A; stops after the
 * layer that reaches dst. Then walks back from dst, taking at each layer the
 * smallest-id neighbour in the previous layer. Writes path[0] = src ..
 * path[d] = dst and returns d + 1, or 0 if dst is unreachable.
 */
static int layered_path(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                        int c, int src, int dst, int *level, int *queue, int *inA, int32_t *path)
{
    for (int u = 0; u < n; u++) { inA[u] = 1; level[u] = -1; }
    inA[c] = 0;
    for (int j = row_ptr[c]; j < row_ptr[c + 1]; j++) inA[col_idx[j]] = 0;
    inA[src] = 1; inA[dst] = 1;
    int head = 0, tail = 0;
    queue[tail++] = src; level[src] = 0;
    int layer_end = tail, d = 0;
    while (head < tail && level[dst] < 0) {
        /* Expand one whole layer. */
        while (head < layer_end) {
            int u = queue[head++];
            for (int j = row_ptr[u]; j < row_ptr[u + 1]; j++) {
                int y = col_idx[j];
                if (!inA[y] || level[y] >= 0) continue;
                level[y] = d + 1;
                queue[tail++] = y;
            }
        }
        layer_end = tail;
        d++;
    }
    if (level[dst] < 0) return 0;
    int len = level[dst];
    int y = dst;
    path[len] = dst;
    for (int l = len; l >= 1; l--) {
        int pred = -1;
        for (int j = row_ptr[y]; j < row_ptr[y + 1]; j++) {    /* ascending ids */
            int u = col_idx[j];
            if (level[u] == l - 1) { pred = u; break; }
        }
        path[l - 1] = pred;
        y = pred;
    }
    return len + 1;
}

/*
 * Primary rule: cycle = [v*, x*, ..., z*] with the path from x* to z* given
 * by layered_path avoiding N[v*]. Fallback (keeps the rule total when z* is
 * not reachable): the first triple (v, a, b) with v by ascending rank and
 * a, b in LN(v), ab not an edge, rank a < rank b, by ascending
 * (rank a, rank b), such that a is reachable from b avoiding N[v]; the cycle
 * is [v, b, ..., a]. Writes the cycle length to *len_out and whether the
 * fallback was used to *fallback_out. Returns 0, or < 0 on error / when no
 * cycle exists (the graph is chordal).
 */
int oracle_certificate(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *order,
                       const int32_t *rank, int32_t vstar, int32_t xstar, int32_t zstar, int32_t force_fallback,
                       int32_t *cycle, int32_t *len_out, int32_t *fallback_out)
{
    *len_out = 0; *fallback_out = 0;
    if (n <= 0) return -1;
    int *level = (int *)malloc(sizeof(int) * (size_t)n);
    int *queue = (int *)malloc(sizeof(int) * (size_t)n);
    int *inA = (int *)malloc(sizeof(int) * (size_t)n);
    int *ln = (int *)malloc(sizeof(int) * (size_t)n);
    int ret = -3;
    if (!level || !queue || !inA || !ln) { ret = -2; goto done; }
    if (!force_fallback && vstar >= 0) {
        int len = layered_path(n, row_ptr, col_idx, vstar, xstar, zstar, level, queue, inA, cycle + 1);
        if (len > 0) {
            cycle[0] = vstar;
            *len_out = len + 1;
            ret = 0;
            goto done;
        }
    }
    *fallback_out = 1;
    for (int rv = 0; rv < n; rv++) {
        int v = order[rv];
        /* LN(v) in rank order. */
        int k = 0;
        for (int r = 0; r < rv; r++) if (adjacent(row_ptr, col_idx, v, order[r])) ln[k++] = order[r];
        for (int ia = 0; ia < k; ia++) {
            for (int ib = ia + 1; ib < k; ib++) {
                int a = ln[ia], b = ln[ib];
                if (adjacent(row_ptr, col_idx, a, b)) continue;
                int len = layered_path(n, row_ptr, col_idx, v, b, a, level, queue, inA, cycle + 1);
                if (len > 0) {
                    cycle[0] = v;
                    *len_out = len + 1;
                    ret = 0;
                    goto done;
                }
            }
        }
    }
done:
    free(level); free(queue); free(inA); free(ln);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* Whole test for one graph                                                  */
/* ------------------------------------------------------------------------ */
/* Maximum Cardinality Search                                                */
/* ------------------------------------------------------------------------ */
/*
 * A binary max-heap of (label, id) entries ordered by larger label, then
 * smaller id. Raising a label pushes a new entry; entries of numbered
 * vertices or with an outdated label are dropped when they surface. The
 * heap top is therefore always the unnumbered vertex of largest label and,
 * among those, smallest id.
 */
typedef struct {
    int32_t label, id;
} mcs_entry;

static int mcs_before(mcs_entry a, mcs_entry b)
{
    return a.label > b.label || (a.label == b.label && a.id < b.id);
}

static void mcs_push(mcs_entry *h, int64_t *len, mcs_entry e)
{
    int64_t i = (*len)++;
    h[i] = e;
    while (i > 0) {
        int64_t up = (i - 1) / 2;
        if (!mcs_before(h[i], h[up])) break;
        mcs_entry t = h[i]; h[i] = h[up]; h[up] = t;
        i = up;
    }
}

static mcs_entry mcs_pop(mcs_entry *h, int64_t *len)
{
    mcs_entry top = h[0];
    h[0] = h[--(*len)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, best = i;
        if (l < *len && mcs_before(h[l], h[best])) best = l;
        if (r < *len && mcs_before(h[r], h[best])) best = r;
        if (best == i) break;
        mcs_entry t = h[i]; h[i] = h[best]; h[best] = t;
        i = best;
    }
    return top;
}

int oracle_mcs(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
               int32_t *order, int32_t *rank, int32_t *parent)
{
    if (n < 0) return -1;
    if (n == 0) return 0;
    const int64_t cap = (int64_t)n + (int64_t)row_ptr[n] + 1;
    mcs_entry *h = (mcs_entry *)malloc(sizeof(mcs_entry) * (size_t)cap);
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!h || !label) { free(h); free(label); return -2; }
    int64_t len = 0;
    for (int v = 0; v < n; v++) {
        label[v] = 0; rank[v] = -1; parent[v] = -1;
        mcs_entry e = {0, v};
        mcs_push(h, &len, e);
    }
    for (int i = 0; i < n; i++) {
        int x = -1;
        while (len > 0) {
            mcs_entry e = mcs_pop(h, &len);
            if (rank[e.id] < 0 && label[e.id] == e.label) { x = e.id; break; }
        }
        if (x < 0) { free(h); free(label); return -3; }  /* cannot happen */
        order[i] = x;
        rank[x] = i;
        for (int j = row_ptr[x]; j < row_ptr[x + 1]; j++) {
            int y = col_idx[j];
            if (rank[y] >= 0) continue;
            label[y] += 1;
            parent[y] = x;
            mcs_entry e = {label[y], y};
            mcs_push(h, &len, e);
        }
    }
    free(h); free(label);
    return 0;
}

/* ------------------------------------------------------------------------ */
/*
 * result[0] = chordal (1/0), result[1..3] = witness (v*, x*, z*),
 * result[4] = cycle length (0 if chordal), result[5] = fallback used.
 * order/rank/parent: [n]; cycle: [n] (written only if not chordal).
 */
static int chordal_test_with(int mcs, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             int32_t *order, int32_t *rank, int32_t *parent, int32_t *cycle, int32_t *result)
{
    for (int i = 0; i < 6; i++) result[i] = 0;
    result[0] = 1; result[1] = result[2] = result[3] = -1;
    if (n < 0) return -1;
    if (n == 0) return 0;
    int rc = mcs ? oracle_mcs(n, row_ptr, col_idx, order, rank, parent)
                 : oracle_lexbfs(n, row_ptr, col_idx, order, rank, parent);
    if (rc) return rc;
    int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *fail = (uint8_t *)malloc((size_t)n);
    int32_t w[3];
    if (!p || !fail) { free(p); free(fail); return -2; }
    int ok = oracle_peo(n, row_ptr, col_idx, rank, p, fail, w);
    free(p); free(fail);
    if (ok < 0) return ok;
    if (ok == 1) return 0;
    result[0] = 0; result[1] = w[0]; result[2] = w[1]; result[3] = w[2];
    int32_t len = 0, fb = 0;
    rc = oracle_certificate(n, row_ptr, col_idx, order, rank, w[0], w[1], w[2], 0, cycle, &len, &fb);
    if (rc) return rc;
    result[4] = len; result[5] = fb;
    return 0;
}

int oracle_chordal_test(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                        int32_t *order, int32_t *rank, int32_t *parent, int32_t *cycle, int32_t *result)
{
    return chordal_test_with(0, n, row_ptr, col_idx, order, rank, parent, cycle, result);
}

/* The same test on the Maximum Cardinality Search order (Theorem 5.2). */
int oracle_chordal_test_mcs(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                            int32_t *order, int32_t *rank, int32_t *parent, int32_t *cycle, int32_t *result)
{
    return chordal_test_with(1, n, row_ptr, col_idx, order, rank, parent, cycle, result);
}
