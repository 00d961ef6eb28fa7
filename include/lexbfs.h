/*
 * lexbfs.h -- C ABI of the MI355X (gfx950) chordality library.
 *
 * The library computes, on the GPU, the two steps of the chordality test of
 * Lupinska, "A Parallel Algorithm to Test Chordality of Graphs":
 *   1. a Lexicographic BFS order (Section 4.1 definition: every step numbers
 *      the unnumbered vertex with the lexicographically largest label and
 *      appends a strictly decreasing number to the labels of its unnumbered
 *      neighbours; the parallel form is Section 6.1), and
 *   2. the perfect-elimination test of that order (Section 5.2, parallel form
 *      Section 6.2): with p(v) the latest-ordered earlier neighbour of v, the
 *      graph is chordal iff LN(v) \ {p(v)} is a subset of N(p(v)) for every v
 *      (Theorem 5.1 and the argument of Section 5.3).
 *
 * Conventions shared by every entry point
 *   - Vertex ids are 0-based. order[i] is the vertex numbered at step i (the
 *     paper's pi(i+1)); rank[v] is its inverse; parent[v] = p(v) or -1.
 *   - Ties between equal labels go to the smallest vertex id, at every step
 *     (so the first vertex is 0, the paper's vertex 1). The paper leaves the
 *     choice open ("we cannot predict which one", Section 6.1); fixing it
 *     makes every output unique and reproducible.
 *   - A graph is given twice, in the same vertex ids: an int32 CSR (rows
 *     strictly ascending, symmetric, no self-loops) and an n x n adjacency
 *     bitset (row v at bits + v*words_per_row, bit u in word u>>6 at position
 *     u&63, LSB first; zero diagonal; bits >= n in the last word are zero).
 *     The paper keeps the graph as an n x n boolean matrix (Section 6.3); the
 *     bitset is that matrix packed 64 entries per word.
 *   - Unless stated otherwise every pointer is DEVICE memory owned by the
 *     caller. Inputs are never written. Nothing is allocated on the calls'
 *     path: scratch lives in the caller's workspace `ws` (device memory,
 *     256-byte aligned, size from the matching *_workspace_bytes function).
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream); outputs are valid once the stream has reached the call. The
 *     return value only reports argument errors and launch failures.
 *   - Calls are re-entrant as long as concurrent calls use distinct
 *     workspaces and outputs.
 */
#ifndef LEXBFS_H
#define LEXBFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define LEXBFS_OK 0
#define LEXBFS_EINVAL (-1)  /* null required pointer, n < 0, words_per_row < ceil(n/64), nnz outside [0, 2^31) */
#define LEXBFS_ENOWS (-2)   /* workspace pointer null or smaller than required */
#define LEXBFS_EHIP (-3)    /* a HIP runtime call or kernel launch failed */
#define LEXBFS_EGRAPH (-4)  /* input contract violated (only from lexbfs_validate or LEXBFS_FLAG_VALIDATE) */
#define LEXBFS_ETOOBIG (-5) /* n above LEXBFS_MAX_N or above what the device's LDS supports */

/* Largest supported vertex count: class ids and vertex ids are kept in 16 bits. */
#define LEXBFS_MAX_N 65536

/* Flags for chordal_test / chordal_test_batch. */
#define LEXBFS_FLAG_FORCE_FALLBACK 0x1u /* build the certificate with the fallback rule only (test hook) */
/* chordal_test only: run LexBFS as one round of three launches per step
 * (the host loop of Section 6.1, one thread per vertex, tables in global
 * memory) instead of the persistent kernel. Same results; a comparison form,
 * slower by the per-launch cost times 3n. Ignored by chordal_test_batch. */
#define LEXBFS_FLAG_PER_STEP 0x2u
/* chordal_test and chordal_test_batch: order the vertices by Maximum
 * Cardinality Search (Section 5.1 box: the label of a vertex is the number
 * of its numbered neighbours, the largest label is numbered next, smallest
 * id first) instead of LexBFS, then run the same perfect-elimination test,
 * witness and certificate on that order (Theorem 5.2: the graph is chordal
 * iff its MCS order is a perfect elimination order). Outputs order, rank and
 * parent are those of the MCS order. Not combinable with
 * LEXBFS_FLAG_PER_STEP (LEXBFS_EINVAL). */
#define LEXBFS_FLAG_MCS 0x4u
/* chordal_test, chordal_test_batch and lexbfs_batch_plan_create: check the
 * input contract on the device (as lexbfs_validate does) before any other
 * kernel runs, and return LEXBFS_EGRAPH without running the test if a
 * graph breaks it. The check's verdict is needed on the host, so with this
 * flag the call waits for `stream` to drain the check (not capturable into
 * a hipGraph); a plan is checked once, at creation. */
#define LEXBFS_FLAG_VALIDATE 0x8u

/* One graph. All pointers are device memory. */
typedef struct lexbfs_graph {
    int32_t n;                /* number of vertices, 0 <= n <= LEXBFS_MAX_N */
    int32_t reserved;         /* must be 0 */
    int64_t nnz;              /* CSR entries = 2|E|, 0 <= nnz < 2^31 */
    const int32_t *row_ptr;   /* [n+1] */
    const int32_t *col_idx;   /* [nnz], strictly ascending within each row */
    const uint64_t *bits;     /* [n * words_per_row] */
    int64_t words_per_row;    /* row stride in 64-bit words, >= ceil(n/64) */
} lexbfs_graph_t;

/* Verdict for one graph, written to device memory (32 bytes).
 * chordal = 1: the LexBFS order is a perfect elimination order (Theorem 5.1);
 *   witness_* = -1, cycle_len = 0.
 * chordal = 0: witness_v = v*, the failing vertex of smallest rank (also the
 *   first vertex whose left neighbourhood is not a clique, Section 5.3);
 *   witness_p = x* = p(v*); witness_z = z*, the smallest-rank vertex of
 *   LN(v*) \ {x*} not adjacent to x*. cycle_len >= 4 is the length of the
 *   chordless cycle written to the cycle output (see chordal_test).
 * fallback = 1 when the certificate came from the fallback rule. */
typedef struct lexbfs_result {
    int32_t chordal;
    int32_t witness_v;
    int32_t witness_p;
    int32_t witness_z;
    int32_t cycle_len;
    int32_t fallback;
    int32_t reserved[2];
} lexbfs_result_t;

/* Optional per-graph outputs, device pointers each of [n] int32, or NULL to
 * keep them in the workspace. */
typedef struct lexbfs_outputs {
    int32_t *order;
    int32_t *rank;
    int32_t *parent;
    int32_t *cycle;
} lexbfs_outputs_t;

/* Workspace bytes for lexbfs_order / chordal_test on a graph of n vertices. */
size_t lexbfs_workspace_bytes(int32_t n);

/*
 * lexbfs_validate -- check that g is what every other entry point assumes
 * (Section 3.1 works with simple graphs: N(v) never holds v and adjacency
 * is symmetric; the CSR and the bitset of lexbfs_graph_t must describe the
 * same N(v)). On the device, reading only inside the arrays the contract
 * sizes: row_ptr non-decreasing from row_ptr[0] = 0 to row_ptr[n] = nnz;
 * every column index in 0..n-1; every row strictly ascending (no
 * duplicates); no self-loop; every CSR entry (v, u) set in bitset row v and
 * its reverse set in row u; and no other bit set in a row's first
 * ceil(n/64) words (bits >= n included). The other entry points do not
 * check this themselves (it costs a pass over the CSR and the bitset):
 * given a graph that breaks it they may return wrong results or read out of
 * bounds.
 *   ws   device memory of at least 256 bytes (any workspace of this
 *        library's *_workspace_bytes size will do); one word is written
 * Waits for `stream` to finish the check. Returns LEXBFS_OK, LEXBFS_EGRAPH
 * (lexbfs_last_error names the first violated rule), LEXBFS_EINVAL,
 * LEXBFS_ENOWS, LEXBFS_ETOOBIG or LEXBFS_EHIP.
 */
int lexbfs_validate(const lexbfs_graph_t *g, void *ws, size_t ws_bytes, void *stream);

/*
 * lexbfs_order -- the LexBFS order (Section 4.1 definition; Section 6.1
 * parallel algorithm, here one persistent kernel instead of four launches
 * per step) together with its inverse and the parent p(v) of Section 5.2.
 *   g       graph (device pointers inside a host struct)
 *   order   [n] out, required
 *   rank    [n] out or NULL
 *   parent  [n] out or NULL
 * Errors: LEXBFS_EINVAL, LEXBFS_ENOWS, LEXBFS_ETOOBIG, LEXBFS_EHIP.
 */
int lexbfs_order(const lexbfs_graph_t *g, int32_t *order, int32_t *rank, int32_t *parent,
                 void *ws, size_t ws_bytes, void *stream);

/*
 * chordal_test -- LexBFS order, then the parent-based perfect-elimination
 * test (Section 6.2), then for a non-chordal graph the witness and a
 * chordless cycle of length >= 4 (not in the paper; defined as follows).
 * With A = (V \ N[v*]) + {x*, z*}: a breadth-first search inside A from x*
 * reaches z* at distance d; walking back from z*, each vertex's predecessor
 * is the smallest-id vertex of the previous layer adjacent to it. The cycle
 * is [v*, x*, ..., z*]. If z* is unreachable (or FORCE_FALLBACK is set), the
 * first triple (v, a, b) with v by ascending rank, a, b in LN(v) not
 * adjacent, rank a < rank b, ordered by (rank a, rank b), whose b reaches a
 * inside (V \ N[v]) + {a, b} gives [v, b, ..., a] by the same rule.
 *   res  [1] out, required
 *   out  host struct of optional device outputs, or NULL
 * Errors: as lexbfs_order.
 */
int chordal_test(const lexbfs_graph_t *g, lexbfs_result_t *res, const lexbfs_outputs_t *out,
                 void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/*
 * chordal_test_noalloc -- chordal_test for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the scratch lives in a fixed device
 * array of the library instead of a caller workspace. Same arguments (minus
 * ws), results and outputs as chordal_test. The caller still passes g, res
 * and the optional outputs.
 *   - The array holds chordal_test_noalloc_max_bytes() bytes (about
 *     2.5 MiB), enough for every n up to LEXBFS_MAX_N. Each device the
 *     library runs on holds its own copy until the process ends; the first
 *     call on a device looks up that copy's address (a runtime query with
 *     that device current, no allocation).
 *   - All calls on one device share that device's array, which keeps the
 *     last call's contents (each call writes what it reads before reading
 *     it). Calls that overlap on one device (other streams or threads) race:
 *     the caller serialises them.
 *   - Allocates nothing and calls no allocating routine.
 * Errors: as chordal_test, without LEXBFS_ENOWS; LEXBFS_ETOOBIG when the
 * graph would need more scratch than the array holds; LEXBFS_EINVAL with
 * LEXBFS_FLAG_VALIDATE (that check waits on the host: run lexbfs_validate,
 * with a workspace, beforehand).
 */
size_t chordal_test_noalloc_max_bytes(void);
int chordal_test_noalloc(const lexbfs_graph_t *g, lexbfs_result_t *res, const lexbfs_outputs_t *out,
                         uint32_t flags, void *stream);

/* Schedule for chordal_test_batch. A graph with n <= wave_max_n is run by
 * one 64-lane wavefront; a larger one by a whole workgroup of
 * block_threads lanes. wave_max_n = 0 takes the built-in threshold (1024),
 * a negative value puts every graph on a workgroup; the threshold is
 * lowered, in steps of 64, until four wavefront states fit the LDS of one
 * workgroup. lds_bytes is the dynamic LDS per workgroup (0 = derived from
 * the largest graph). */
typedef struct lexbfs_tuning {
    int32_t wave_max_n;
    int32_t block_threads;   /* 0 or 256 (the workgroup size); others: LEXBFS_EINVAL */
    int32_t lds_bytes;
    int32_t reserved;        /* must be 0 */
} lexbfs_tuning_t;

/* Workspace bytes for chordal_test_batch over these graphs (host array). */
size_t lexbfs_batch_workspace_bytes(const lexbfs_graph_t *gs, int32_t count);

/*
 * chordal_test_batch -- chordal_test on `count` independent graphs in one
 * pass: one persistent LexBFS launch over a longest-first work queue (a
 * graph per wavefront or per workgroup as the tuning says), one sweep
 * launch, one certificate launch.
 *   gs      HOST array [count] of graph descriptors (device pointers)
 *   outs    HOST array [count] of optional outputs, or NULL
 *   res     DEVICE array [count] of results
 *   tuning  HOST pointer or NULL for the built-in schedule
 * Equivalent to lexbfs_batch_plan_create + lexbfs_batch_plan_launch +
 * lexbfs_batch_plan_destroy: the per-graph descriptor table is staged into
 * the workspace with a host-to-device copy on `stream`; the calling thread
 * returns once the table has been staged. Every graph needs
 * n <= LEXBFS_MAX_N. A graph with n <= lexbfs_batch_max_n() runs start to
 * finish on one team (a wavefront or a 256-lane workgroup): LexBFS with the
 * perfect-elimination test of Section 5.2 folded into its steps, then the
 * witness and certificate. A larger one runs on its own 1024-lane
 * workgroup: LexBFS, sweep and certificate as in chordal_test (on `stream`,
 * before the other graphs, in this one-shot call). Results match
 * chordal_test in every case.
 * Errors: as chordal_test; LEXBFS_ETOOBIG names a graph beyond the limit.
 */
int chordal_test_batch(const lexbfs_graph_t *gs, int32_t count, const lexbfs_outputs_t *outs,
                       lexbfs_result_t *res, const lexbfs_tuning_t *tuning,
                       void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/*
 * Prepared batches. lexbfs_batch_plan_create validates the graphs, fixes the
 * schedule (longest-first queue, team per graph) and stages the descriptor
 * table into `ws` with a host-to-device copy on `stream` (the call returns
 * once the table has been staged). lexbfs_batch_plan_launch then only
 * launches kernels (no copies, no memsets), so it may be called many times
 * (the graphs' contents may change between launches, their sizes and
 * addresses may not) and may be captured into a hipGraph. If the batch mixes
 * graphs above lexbfs_batch_max_n() with smaller ones, the plan owns a
 * stream and two events (created here): each launch forks that stream from
 * `stream`, runs the larger graphs on it concurrently with the rest, and
 * joins it back into `stream`.
 * Results of a launch are valid once `stream` reaches it. The plan is host
 * memory owned by the caller until lexbfs_batch_plan_destroy, which waits for
 * the plan's own stream; the workspace must stay allocated while the plan is
 * used and must not be shared by two plans whose launches overlap.
 * Arguments and errors as chordal_test_batch.
 */
typedef struct lexbfs_batch_plan lexbfs_batch_plan_t;
int lexbfs_batch_plan_create(const lexbfs_graph_t *gs, int32_t count, const lexbfs_outputs_t *outs,
                             lexbfs_result_t *res, const lexbfs_tuning_t *tuning, void *ws, size_t ws_bytes,
                             uint32_t flags, void *stream, lexbfs_batch_plan_t **plan);
int lexbfs_batch_plan_launch(const lexbfs_batch_plan_t *plan, void *stream);
void lexbfs_batch_plan_destroy(lexbfs_batch_plan_t *plan);

/* Short English description of a return code (static storage). */
const char *lexbfs_strerror(int code);

/* Description of the most recent failure on the calling thread: the HIP
 * call and its error string after LEXBFS_EHIP, or the limit that was hit
 * after LEXBFS_ETOOBIG (static thread-local storage, "" if none). */
const char *lexbfs_last_error(void);

/* Kernel timing (a tracing aid). While enabled, every kernel launch of the
 * library is bracketed by a pair of HIP events recorded on the launch's
 * stream; the events are created by the enabling call, never on the launch
 * path. lexbfs_profile_collect waits for the recorded events, writes per
 * kernel kind (index below) the number of launches and their summed
 * duration in milliseconds since the previous collect, and returns the
 * number of launches that found the event pool (8192 pairs) full, or < 0 on
 * a HIP failure. counts/ms: host arrays of LEXBFS_KERNEL_KINDS entries. */
#define LEXBFS_KERNEL_KINDS 4 /* 0 LexBFS, 1 elimination sweep, 2 witness and certificate, 3 batch setup */
int lexbfs_profile_enable(int on);
int lexbfs_profile_collect(int32_t *counts, double *ms);

/*
 * Device-side ingestion (the step before the path: the paper builds its
 * N x N Adj matrix on the host and copies it, Section 6.3, and reports input
 * and allocation as most of its total time, Section 7). Builds the packed
 * bitset of lexbfs_graph_t from the CSR on `stream`: bit u of row v is set
 * iff u appears in v's CSR row; every word of every row is written,
 * padding words (beyond ceil(n/64)) as zero.
 *   row_ptr  DEVICE [n+1], col_idx DEVICE [row_ptr[n]] (ids >= 64 *
 *            words_per_row are ignored; the CSR contract of lexbfs_graph_t
 *            makes the result symmetric with a zero diagonal)
 *   bits     DEVICE [n * words_per_row], written
 * Errors: LEXBFS_EINVAL (n < 0, null pointer, words_per_row < ceil(n/64) or
 * > LEXBFS_MAX_N/64), LEXBFS_ETOOBIG (n > LEXBFS_MAX_N), LEXBFS_EHIP.
 */
int lexbfs_build_bitset(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, uint64_t *bits,
                        int64_t words_per_row, void *stream);

/* Largest n a batch graph may have to run on a wavefront or 256-lane team
 * on the current device (its state, about 12 bytes per vertex, must fit one
 * workgroup's LDS); larger graphs, up to LEXBFS_MAX_N, run on 1024-lane
 * workgroups. Negative LEXBFS_E* code on a HIP failure. */
int32_t lexbfs_batch_max_n(void);

/*
 * Multi-sweep LexBFS. Section 3.2 surveys LexBFS as the core of interval
 * graph recognition and Section 8 leaves a parallel interval test as future
 * work; these entry points are the first step of that direction.
 *
 * lexbfs_plus_order -- one LexBFS+ sweep: the LexBFS of Section 4.1 with
 * ties between equal labels going to the vertex that comes LAST in
 * prev_order (instead of the smallest id). Computed by renaming every vertex
 * v to n-1-(position of v in prev_order) on the device -- the tie rule then
 * picks the smallest new id -- building the renamed CSR and bitset in the
 * workspace, running the LexBFS kernel of lexbfs_order, and renaming the
 * result back.
 *   g           CSR part only (g->bits is not read; it may be NULL)
 *   prev_order  DEVICE [n], a permutation of 0..n-1
 *   order       DEVICE [n], written (required)
 *   rank,parent DEVICE [n] or NULL, as for lexbfs_order (parent = latest
 *               earlier neighbour in this order)
 *   ws          lexbfs_plus_workspace_bytes(n, nnz) bytes (about
 *               n*ceil(n/64)*8 for the renamed bitset + 4*nnz + 52*n)
 * If prev_order is not a permutation (detected on the device) order, rank
 * and parent are filled with -1. Errors: as lexbfs_order.
 */
size_t lexbfs_plus_workspace_bytes(int32_t n, int64_t nnz);
int lexbfs_plus_order(const lexbfs_graph_t *g, const int32_t *prev_order, int32_t *order, int32_t *rank,
                      int32_t *parent, void *ws, size_t ws_bytes, void *stream);

/* Verdict of unit_interval_test, written to device memory (32 bytes).
 * unit_interval = 1: the third order puts every closed neighbourhood on
 *   consecutive positions (a unit interval ordering); witness = -1.
 * unit_interval = 0: witness = (a, b, c) with a before b before c in the
 *   third order, ac an edge and b not adjacent to both a and c. With v the
 *   earliest vertex whose closed neighbourhood N[v] is not consecutive,
 *   [lo, hi] the positions N[v] spans and b the earliest vertex of the span
 *   outside N[v]: (vertex at lo, b, v) if b comes before v, else
 *   (v, b, vertex at hi). */
typedef struct lexbfs_interval_result {
    int32_t unit_interval;
    int32_t witness[3];
    int32_t reserved[4];
} lexbfs_interval_result_t;

/*
 * unit_interval_test -- Corneil's three-sweep unit interval recognition
 * (Discrete Applied Mathematics 138 (2004)): sigma1 = LexBFS (lexbfs_order's
 * order), sigma2 = LexBFS+ after sigma1, sigma3 = LexBFS+ after sigma2; the
 * graph is a unit interval graph iff every closed neighbourhood is
 * consecutive in sigma3. All steps run on `stream`.
 *   g      full graph (CSR and bitset)
 *   res    DEVICE lexbfs_interval_result_t, written (required)
 *   order  DEVICE [n] or NULL: sigma3
 *   ws     unit_interval_workspace_bytes(n, nnz) bytes
 * Errors: as chordal_test.
 */
size_t unit_interval_workspace_bytes(int32_t n, int64_t nnz);
int unit_interval_test(const lexbfs_graph_t *g, lexbfs_interval_result_t *res, int32_t *order, void *ws,
                       size_t ws_bytes, void *stream);

/*
 * unit_interval_test_batch -- unit_interval_test on `count` graphs with one
 * launch per step for the whole batch: the three sweeps are batch passes of
 * the chordal_test_batch kernels (order only), and renaming, bitset build,
 * mapping back and the check each cover every graph in one launch.
 * Results are those of unit_interval_test on each graph.
 *   gs      HOST array of `count` graphs (device pointers inside)
 *   res     DEVICE array of `count` lexbfs_interval_result_t, written
 *   orders  HOST array of `count` DEVICE pointers ([n_i] int32, sigma3 of
 *           graph i) or NULL entries; or NULL
 *   ws      unit_interval_batch_workspace_bytes(gs, count) bytes
 * Host-side preparation (two batch plans) happens inside the call.
 * Errors: as chordal_test_batch.
 */
size_t unit_interval_batch_workspace_bytes(const lexbfs_graph_t *gs, int32_t count);
int unit_interval_test_batch(const lexbfs_graph_t *gs, int32_t count, lexbfs_interval_result_t *res,
                             int32_t *const *orders, void *ws, size_t ws_bytes, void *stream);

/* Library ABI version (incremented on incompatible changes). */
int lexbfs_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LEXBFS_H */
