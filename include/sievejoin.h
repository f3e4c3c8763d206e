/*
 * sievejoin.h -- C ABI of the MI355X (gfx950) SieveJoin hot path.
 *
 * Method: arXiv 2308.16370, "SieveJoin: Boosting Multi-Way Joins with Reusable
 * Bloom Filters". A multi-way equi-join over integer key columns (the query
 * R join_b S join_c T of Section 2.2, generalised to chain, star and cyclic join
 * graphs) is answered in two phases:
 *   pruning     -- a Bloom filter is built on each relation's join attribute and the
 *                  filters are pushed from the right-most relation toward the root,
 *                  each relation being sieved by the filters of the relations after
 *                  it before it builds its own (Section 2.2, Fig. 2); cyclic queries
 *                  add a filter for the closing condition (Section 2.3) and an
 *                  optional forward pass sieves the relations on the right again
 *                  (the dotted arrow of Fig. 2);
 *   enumeration -- a binary hash-join plan over the sieved relations produces the
 *                  exact result (Section 2.2).
 * The result is exact: filters have no false negatives and every final match is
 * an equality test.
 *
 * Conventions
 *   - Every call returns an sj_status; SJ_OK is 0, errors are negative. No C++
 *     exception crosses this boundary. sj_last_error() describes the last error
 *     of a context.
 *   - All pointers named *_dev are device (HBM) pointers; everything else is host.
 *     Input columns and result buffers must be 16-byte aligned, the workspace
 *     256-byte aligned.
 *   - Inputs are borrowed: the caller keeps columns and workspace alive and
 *     unmodified until sj_plan_destroy(). The library never allocates device
 *     memory; the caller passes one workspace buffer (sj_bind_workspace).
 *   - Work is enqueued on the context's stream (caller-owned hipStream_t).
 *     Only sj_join() and calls given host output pointers wait for the stream.
 *   - A plan is not thread-safe. Distinct plans may run on distinct streams.
 *   - Keys are any int32 (no reserved value). Row ids are uint32 (a relation has
 *     fewer than 2^31 rows); counts are uint64; the checksum is uint64 modulo 2^64.
 *
 * Result definition (the exact multiset the plan returns):
 *   result   = { (rid_0, ..., rid_{n-1}) : every relation's predicate holds and
 *                 R_a[col_a][rid_a] == R_b[col_b][rid_b] for every edge }
 *   checksum = sum over result tuples of prod_i (mix64((i << 32) | rid_i) | 1),
 *              modulo 2^64, with mix64 the SplitMix64 output function.
 *   Tuples are written row-major, one int32 row id per relation in relation-index
 *   order, sorted lexicographically in the plan's enumeration order (relations in
 *   depth-first preorder from the root; for chains and stars listed root first,
 *   that is relation-index order). Exception: 3-cycles and 4-cliques counted by
 *   intersection (see sj_join) are written in the walk's order, the same in every
 *   run but not sorted.
 */
#ifndef SIEVEJOIN_H
#define SIEVEJOIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sj_status;

#define SJ_OK 0
#define SJ_ERR_INVALID (-1)     /* bad argument, NULL pointer, out-of-range option */
#define SJ_ERR_GRAPH (-2)       /* bad column/relation index, self-edge, disconnected graph */
#define SJ_ERR_NOMEM (-3)       /* workspace smaller than sj_plan() asked for */
#define SJ_ERR_CAPACITY (-4)    /* result buffer smaller than the result; nothing written */
#define SJ_ERR_STATE (-5)       /* call out of order (e.g. sj_join before sj_sieve) */
#define SJ_ERR_DEVICE (-6)      /* a HIP runtime call failed */
#define SJ_ERR_UNSUPPORTED (-7) /* valid query outside what this build executes */

#define SJ_MAX_RELS 16
#define SJ_MAX_COLS 64
#define SJ_MAX_EDGES 32

typedef struct sj_ctx sj_ctx;
typedef struct sj_plan_s sj_plan_t;

/* One relation instance. The same device columns may back several instances
 * (self-joins). Row r takes part iff pred_col < 0 or
 * pred_lo <= cols[pred_col][r] < pred_hi. */
typedef struct {
    int64_t nrows;                 /* 0 <= nrows < 2^31 */
    int32_t ncols;                 /* 1 <= ncols <= SJ_MAX_COLS */
    const int32_t *const *cols;    /* host array of ncols device pointers, nrows int32 each */
    int32_t pred_col;              /* -1: no predicate */
    int32_t pred_lo, pred_hi;
} sj_rel;

/* Equi-join condition R_{rel_a}[col_a] == R_{rel_b}[col_b]. Edges not on the
 * spanning tree found from the root are closing edges (cyclic queries). */
typedef struct {
    int32_t rel_a, col_a, rel_b, col_b;
} sj_edge;

/* Filter and schedule options. A zero field takes the default in brackets. */
typedef struct {
    uint32_t bits_per_key; /* [8] filter bits per key inserted into the filter */
    uint32_t k;            /* [6] bits set per key, 1..12 */
    uint32_t block_bits;   /* [512] filter block size: 256, 512 or 1024 bits */
    uint32_t passes;       /* [2] 1: the paper's backward pass only; 2: plus the forward pass */
    uint64_t seed;         /* filter hash seed (0 is a valid seed) */
    int32_t root;          /* -1: relation 0 (the left-most relation) */
    uint32_t flags;        /* SJ_FLAG_* bits; other bits must be 0 */
    /* Launch shape of the sieve steps (tuning only: results do not depend on them). */
    uint32_t probe_grid;   /* [256] workgroups of each probe and compaction launch
                              (1024 threads each, a contiguous share of the rows per
                              workgroup): a power of two, 64..1024 */
    uint32_t probe_lds;    /* [0] LDS a probe sets aside for one filter (the smallest it
                              reads whose size, known on the device only, fits):
                              0: as much as its filters could need, up to 108 KiB;
                              1: none, every filter is read through L2 (more
                              workgroups then fit per compute unit);
                              2: only when one of its filters fits at its largest
                              possible size (so the LDS is always used) */
} sj_opts;

/* Record a HIP event pair around every launch group on the context's stream
 * (costs a few microseconds per group); read with sj_profile_*(). Implies
 * SJ_FLAG_EAGER. */
#define SJ_FLAG_PROFILE 1u
/* Launch every kernel of sj_build_filters, sj_sieve and sj_join one by one. By
 * default the first call of each of these on a plan records its launches into a
 * HIP graph (on a private stream of the plan) and every call replays that graph on
 * the context's stream; the launches and their arguments are the same either way,
 * and so are the results. sj_bind_workspace drops the recorded graphs. */
#define SJ_FLAG_EAGER 2u
/* Count and write 3-cycle and 4-clique queries with the binary plan, which expands the
 * spanning tree and then checks the closing edges, instead of the default intersection
 * walk (see sj_join). The result is the same; for comparisons. */
#define SJ_FLAG_BINARY_CYCLES 4u
/* Failure injection, for tests of error handling: the named phase fails with
 * SJ_ERR_DEVICE, as a failed HIP call would, before it enqueues anything (no device
 * fault is involved). FILTERS: sj_build_filters; SIEVE: sj_sieve; JOIN: sj_join and
 * sj_join_async; RESULT: sj_result and sj_result_async. A server query submitted with
 * one of these fails alone, with that status, while the others finish. */
#define SJ_FLAG_FAULT_FILTERS 8u
#define SJ_FLAG_FAULT_SIEVE 16u
#define SJ_FLAG_FAULT_JOIN 32u
#define SJ_FLAG_FAULT_RESULT 64u
/* Run each sieve step that writes a survivor list as two launches (probe, then the
 * list from the probe's per-row bits and per-workgroup counts) instead of one launch
 * whose workgroups learn their output offsets by a look-back over the workgroups
 * before them. The survivor lists are the same; for comparisons. */
#define SJ_FLAG_SIEVE_TWO_LAUNCHES 128u

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream). The stream stays caller-owned. */
sj_status sj_ctx_create(int32_t device, void *hip_stream, sj_ctx **out);
sj_status sj_ctx_set_stream(sj_ctx *ctx, void *hip_stream);
/* Release the caller's context. Plans made on it keep it alive: it is freed when the
 * caller has destroyed it and its last plan is destroyed, in either order (plans and
 * contexts may be released by a garbage collector in any order). The caller must not
 * use the handle after this call. Plans enqueue on the context's stream only inside
 * their own calls: once the caller has destroyed that stream, a plan made on the context
 * may still be destroyed (also one attached to a filter catalogue), but not used. */
sj_status sj_ctx_destroy(sj_ctx *ctx);
/* Text of the context's last error ("" if none); valid until the next call on ctx. */
const char *sj_last_error(const sj_ctx *ctx);

/* Validate the join graph (Section 2.2: relations with join attributes joined by
 * equalities) and build the execution plan: the root and depth-first spanning
 * tree, the closing edges, the backward/closing/forward filter schedule, and the
 * workspace for every filter, survivor list, hash table and scan buffer. A filter
 * gets ceil(bits_per_key * n / block_bits) blocks for the n keys inserted into it
 * (the sizing of Bloomjoin, Section 2.1: bits per inserted tuple), computed on the
 * device once n is known. Host-only; launches nothing.
 * *workspace_bytes receives the device workspace the plan needs (worst case: every
 * row survives). `opts` may be NULL (all defaults). */
sj_status sj_plan(sj_ctx *ctx, const sj_rel *rels, int32_t nrels, const sj_edge *edges,
                  int32_t nedges, const sj_opts *opts, sj_plan_t **out, uint64_t *workspace_bytes);

/* Give the plan its device workspace (256-byte aligned, >= workspace_bytes). */
sj_status sj_bind_workspace(sj_plan_t *plan, void *workspace_dev, uint64_t bytes);

/* For callers that cannot allocate device memory (code under graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bind the plan to the library's
 * static workspace instead of a caller buffer. It is one array of SJ_STATIC_WORKSPACE_BYTES
 * per GPU, held by the library until the process ends; this call allocates nothing
 * (no hipMalloc, no library allocation). Fails with SJ_ERR_NOMEM, binding nothing, if
 * the plan's workspace_bytes exceed it. Every plan bound to it on one GPU shares it:
 * plans bound to it must not run at the same time (their phases would race on it),
 * and a plan's filters, survivors and count hold only until another plan bound to it
 * runs a phase (each phase clears what it needs zeroed, so no clearing is needed
 * between plans). The caller still passes the input columns and the result buffer. */
#define SJ_STATIC_WORKSPACE_BYTES (64ull << 20)
sj_status sj_bind_static_workspace(sj_plan_t *plan);

/* Pruning phase, backward pass (Section 2.2 step 1): for every non-root relation
 * from the leaves toward the root, scan its rows, keep those whose child-edge keys
 * all pass the children's filters, and insert the survivors' parent-edge keys into
 * the relation's own blocked Bloom filter. Asynchronous. */
sj_status sj_build_filters(sj_plan_t *plan);

/* Root sieve, closing-edge filters (Section 2.3) and, with passes = 2, the forward
 * pass; every relation ends as an ascending list of surviving row ids. With
 * survivors != NULL the call waits and writes each relation's survivor count to
 * survivors[0..nrels). */
sj_status sj_sieve(sj_plan_t *plan, uint64_t *survivors);

/* Enumeration phase, count pass (Section 2.2 step 2): hash tables on the sieved
 * relations, exact result size and checksum. Waits for the stream; count and
 * checksum are host pointers (either may be NULL). Acyclic graphs, and cyclic graphs
 * of at most 8 relations and 4 closing edges (Section 2.3), are executed; larger
 * cyclic graphs return SJ_ERR_UNSUPPORTED. A cyclic graph runs the binary plan: the
 * spanning tree without the last relation L of the preorder (a leaf) is enumerated,
 * and each prefix is matched with L's rows below its parent that satisfy every
 * closing edge. Two shapes are counted by intersection instead (the multi-way join
 * that Section 3.1.3 pairs with the sieve), with their tuples written by the same
 * walk (in walk order, not sorted):
 *   3-cycle root - P - L - root: for each root survivor the smaller of P's rows
 *     joining it and L's rows closing on it is walked, and each one's partner key is
 *     looked up in a hash of the other relation's (key, key) pairs;
 *   4-clique (six relations, one per pair of four variables a, b, c, d; the root's
 *     two join columns are a and b): for each root row (a, b) the values c come from
 *     the smaller of ac(a) and bc(b), and for each c the values d from the smallest of
 *     ad(a), bd(b) and cd(c), each checked in the other relations' pair hashes.
 * SJ_FLAG_BINARY_CYCLES selects the binary plan for these shapes too. */
sj_status sj_join(sj_plan_t *plan, uint64_t *count, uint64_t *checksum);

/* What sj_result writes per result tuple (Section 2.2: the join result itself; the
 * paper reports results or their count, Section 3.1):
 *   SJ_RIDS    one int32 row id per relation, in relation-index order (width nrels);
 *   SJ_VALUES  the tuple's values: output column q is column c_q of relation r_q at the
 *              tuple's row of r_q, for the projection (r_q, c_q) set by
 *              sj_plan_set_projection (width = its length). The default projection is
 *              every column of every relation, relations in index order.
 * Value tuples are the row-id tuples with each row id replaced by the row's values, in
 * the same order. */
#define SJ_RIDS 0
#define SJ_VALUES 1
#define SJ_MAX_PROJ 32

/* Materialise the result: count tuples, row-major, `width` int32 words each (see
 * SJ_RIDS / SJ_VALUES), into out_dev (room for capacity_tuples tuples). Fails with
 * SJ_ERR_CAPACITY, writing nothing, if capacity_tuples < count; SJ_ERR_UNSUPPORTED if
 * the value projection has more than SJ_MAX_PROJ columns. Asynchronous. */
sj_status sj_result(sj_plan_t *plan, int32_t *out_dev, uint64_t capacity_tuples, int32_t mode);

/* Set the columns SJ_VALUES writes: n (relation, column) pairs in rel_col[0 .. 2n), host
 * memory, copied (0 <= n <= SJ_MAX_PROJ; n = 0 restores the default). SJ_ERR_GRAPH for a
 * relation or column that does not exist. */
sj_status sj_plan_set_projection(sj_plan_t *plan, const int32_t *rel_col, int32_t n);

/* Device memory a query needs, for admission by footprint (batching and serving):
 * *workspace_bytes the plan's workspace (known after sj_plan); *width the int32 words per
 * result tuple in `mode`; *result_bytes the result's size in `mode`, known once the count
 * is on the host (after sj_join or sj_join_wait; else SJ_ERR_STATE). Any output pointer
 * may be NULL. Host-only. */
sj_status sj_plan_footprint(const sj_plan_t *plan, int32_t mode, uint64_t *workspace_bytes, uint64_t *result_bytes,
                            int32_t *width);

/* Asynchronous variant of the enumeration (Section 2.2 step 2), for callers that do
 * not need the count on the host before the tuples (a whole query then runs without
 * a host round trip; every phase is replayed as a recorded graph). sj_join_async takes
 * acyclic plans and the 3-cycles and 4-cliques counted by intersection; sj_result_async
 * acyclic plans only. Other cyclic plans return SJ_ERR_UNSUPPORTED (their count needs
 * a host step).
 *   sj_join_async    enqueues the count pass; the count stays on the device.
 *   sj_result_async  enqueues the materialisation into out_dev (room for
 *                    capacity_tuples tuples, in `mode` as for sj_result): the kernels
 *                    read the count on the device and write nothing if it exceeds the
 *                    capacity.
 *   sj_join_wait     waits for the stream and returns count and checksum; with
 *                    result_status != NULL, also SJ_ERR_CAPACITY if the last
 *                    sj_result_async found its buffer too small (nothing was written),
 *                    else SJ_OK.
 * After sj_join_async, sj_result (the synchronous call) needs sj_join_wait first. */
sj_status sj_join_async(sj_plan_t *plan);
sj_status sj_result_async(sj_plan_t *plan, int32_t *out_dev, uint64_t capacity_tuples, int32_t mode);
sj_status sj_join_wait(sj_plan_t *plan, uint64_t *count, uint64_t *checksum, sj_status *result_status);

sj_status sj_plan_destroy(sj_plan_t *plan);

/* ---- introspection (filters and survivors; used to check the pruning phase) ---- */

#define SJ_FILTER_BACKWARD 0 /* built on relation `rel` (its parent-edge column) in the backward pass */
#define SJ_FILTER_FORWARD 1  /* built on the parent of `rel` toward `rel` in the forward pass */
#define SJ_FILTER_CLOSING 2  /* built on the earlier end of closing edge `index` */

/* Number of filters the plan builds. */
sj_status sj_filter_count(const sj_plan_t *plan, int32_t *nfilters);
/* Identity of filter f: kind (SJ_FILTER_*), the relation it belongs to (rel for
 * backward/forward, the closing edge's ordinal among closing edges for closing),
 * the relation and column its keys come from, and its size in blocks. Reading
 * nblocks waits for the stream (the size of a filter on a relation with a
 * predicate is computed on the device). */
sj_status sj_filter_desc(sj_plan_t *plan, int32_t f, int32_t *kind, int32_t *index, int32_t *src_rel,
                         int32_t *src_col, uint32_t *nblocks);
/* Device-to-device copy of filter f's words (nblocks * block_bits / 32 uint32)
 * into dst_dev (room for capacity_words). Asynchronous. */
sj_status sj_filter_copy(sj_plan_t *plan, int32_t f, uint32_t *dst_dev, uint64_t capacity_words);
/* Inserts into a built filter (Section 2.4: a tuple inserted into a relation changes
 * the relation's filter only when the filter does not contain its key yet).
 * sj_filter_probe writes contained_dev[i] = 1 if filter f reports keys_dev[i] present,
 * else 0 (n bytes, caller-provided); *missing (host, may be NULL) receives how many
 * were not contained. sj_filter_insert does the same against the filter as it is
 * before the call and then sets the bits of every key found missing, in place: the
 * filter keeps its block count (its false-positive rate rises with the keys added) and
 * from then on contains every inserted key. Those missing keys are the ones whose
 * tuples may now join and must be propagated to the adjacent relations' filters (a
 * parent's rows with a matching key can now pass, and their keys go into the parent's
 * filter the same way). Backward filters can be updated after sj_build_filters,
 * forward and closing filters after sj_sieve; the next sj_build_filters or sj_sieve
 * rebuilds a filter from the relations and drops its inserts. A filter held in a
 * filter catalogue is shared and cannot be inserted into (SJ_ERR_STATE). Both calls
 * are asynchronous unless missing / inserted is non-NULL. */
sj_status sj_filter_probe(sj_plan_t *plan, int32_t f, const int32_t *keys_dev, uint64_t n, uint8_t *contained_dev,
                          uint64_t *missing);
sj_status sj_filter_insert(sj_plan_t *plan, int32_t f, const int32_t *keys_dev, uint64_t n, uint8_t *contained_dev,
                           uint64_t *inserted);
/* Propagation of inserted tuples (Section 2.4: a tuple inserted into relation R_i
 * changes R_i's filter only if the filter does not contain its key yet; otherwise the
 * search continues from R_i to its adjacent relations). `cols` is a host array of the
 * relation's ncols device pointers holding n new rows. The new rows that pass rel's
 * predicate and its children's backward filters insert their key toward rel's parent
 * into rel's backward filter (probe first, as sj_filter_insert); the keys it did not
 * hold select the parent's rows (its borrowed columns) whose key toward rel is one of
 * them and that pass the parent's predicate and its other children's filters; those
 * insert their key into the parent's backward filter, and so on up to the root's
 * children. inserted[i] (host, nrels entries, may be NULL) receives how many keys
 * (with multiplicity) relation i's filter did not hold. The maintained filters have
 * no false negatives for the grown relations; rel's filter equals a rebuild, an
 * ancestor's holds a subset of a rebuild's bits (keys that newly pass only through a
 * false positive are not followed). Needs sj_build_filters first; waits for the stream;
 * scratch (256-byte aligned, caller-owned) of sj_filter_propagate_scratch bytes. A
 * filter held in a filter catalogue is refused (SJ_ERR_STATE). */
sj_status sj_filter_propagate_scratch(const sj_plan_t *plan, int32_t rel, uint64_t n, uint64_t *bytes);
sj_status sj_filter_propagate(sj_plan_t *plan, int32_t rel, const int32_t *const *cols, uint64_t n, void *scratch_dev,
                              uint64_t scratch_bytes, uint64_t *inserted);

/* Counting filters (Section 2.4: counting Bloom filters, a counter per position, make
 * deletions possible). sj_plan_cfilter builds the counting twin of the plan's filter f:
 * one 4-bit counter per bit position (the same blocks, k, seed and bit pattern), counting
 * every key the filter's build inserted, with multiplicity; a bit of the plain filter is
 * set iff its counter is nonzero. counts_dev (caller-owned, 256-byte aligned) holds
 * nblocks * block_bits / 2 bytes of counters plus 256 bytes of bookkeeping. Counters
 * saturate at 15 and are then never decremented, so a deletion never clears a bit that a
 * remaining key needs. sj_cfilter_update adds (sign +1) or removes (sign -1) n keys;
 * sj_cfilter_probe answers contains(key) as sj_filter_probe does (waits only if missing
 * is non-NULL); sj_cfilter_export writes the plain filter's words; sj_cfilter_apply
 * writes them over filter f of a plan with the same shape (until the plan's next build
 * of f). After inserting and deleting keys without saturation, the exported filter
 * equals the filter built from the keys that remain. All calls but sj_plan_cfilter
 * (which reads the filter's block count) are asynchronous on the plan's stream. */
typedef struct sj_cfilter sj_cfilter;
sj_status sj_plan_cfilter(sj_plan_t *plan, int32_t f, void *counts_dev, uint64_t bytes, sj_cfilter **out);
sj_status sj_cfilter_update(sj_cfilter *cf, const int32_t *keys_dev, uint64_t n, int32_t sign);
sj_status sj_cfilter_probe(sj_cfilter *cf, const int32_t *keys_dev, uint64_t n, uint8_t *contained_dev,
                           uint64_t *missing);
sj_status sj_cfilter_export(sj_cfilter *cf, uint32_t *words_dev, uint64_t capacity_words);
sj_status sj_cfilter_apply(sj_cfilter *cf, sj_plan_t *plan, int32_t f);
sj_status sj_cfilter_destroy(sj_cfilter *cf);

/* Copy relation rel's final survivor row ids (ascending) into dst_dev (room for
 * capacity); *n receives the count. dst_dev may be NULL to query the count only.
 * Waits for the stream. */
sj_status sj_survivors_copy(sj_plan_t *plan, int32_t rel, uint32_t *dst_dev, uint64_t capacity,
                            uint64_t *n);

/* ---- profiling (plans created with SJ_FLAG_PROFILE) ---- */

/* Wait for the stream and add the elapsed time of every launch group recorded since
 * the last collect to its label's total. Without SJ_FLAG_PROFILE this does nothing. */
sj_status sj_profile_collect(sj_plan_t *plan);
/* Number of distinct launch-group labels seen so far. */
sj_status sj_profile_count(const sj_plan_t *plan, int32_t *n);
/* Label i (valid until the plan is destroyed), its total milliseconds and launch
 * count, and the algorithmic bytes of its last launch (0 where not modelled). Labels
 * name one kernel each where a byte model exists:
 *   "probe:..."         a sieve step: probed columns (and the predicate column of a
 *                       full scan) read, each probed filter read once; each survivor's
 *                       columns (and the row id of a survivor-list source) read, its row
 *                       id and columns written. With SJ_FLAG_SIEVE_TWO_LAUNCHES (or for
 *                       a step that writes no list) the probe launch alone: the probe's
 *                       reads and one survivor bit per row written;
 *   "compact:..."       (SJ_FLAG_SIEVE_TWO_LAUNCHES) survivor bits read, each survivor's
 *                       columns (and row id of a list source) read, its row id and
 *                       columns written;
 *   "bfb_hist:..."      filter build, region counts: the inserted keys (and the
 *                       predicate column of a full scan) read;
 *   "bfb_scatter:..."   the keys read again, each kept key staged (4 bytes);
 *   "bfb_region:..."    the staged keys read, the filter written once;
 *   "buckets:R<j>"      per sieved entry of relation j: an 8-byte (key, index) pair read
 *                       and written per active radix pass, the row id and join columns
 *                       gathered into bucket order (read and written), the key read for
 *                       the directory; 16 bytes per distinct key (directory entry, slot);
 *   "dp:R<j>"           per entry: its row id read; per child its key, the child's bucket
 *                       bounds and prefix weights at them read (32 bytes), the bounds
 *                       written (8 bytes); its own two prefix weights written (16 bytes);
 *   "materialize"       the result tuples written. */
sj_status sj_profile_entry(const sj_plan_t *plan, int32_t i, const char **label, double *total_ms,
                           uint64_t *launches, uint64_t *alg_bytes);
/* Collect, then zero every total. */
sj_status sj_profile_reset(sj_plan_t *plan);

/* ---- batches: many queries recorded into one graph (extension) ----
 *
 * A batch holds up to SJ_MAX_BATCH bound plans made on one context. sj_batch_submit
 * enqueues the whole query of every plan (sj_build_filters, sj_sieve, sj_join_async and,
 * for plans given an output, sj_result_async in `mode`) as one HIP graph in which the
 * plans run side by side, and replays it on the context's stream; the graph is
 * recorded on the first submit and again when the outputs, capacities or mode change.
 * Each plan's count, checksum and result status then come from sj_join_wait, and are
 * those of the plan run alone (the launches and their arguments are the same). Plans
 * must be acyclic or 3-cycles (count only: give them no output), not profiled and not
 * attached to a filter catalogue; they must stay alive and bound until the batch is
 * destroyed, and must not be used on their own while a submit of the batch is running.
 * out_dev may be NULL (counts only) or hold NULL entries.
 *
 * In this build sj_batch_submit is switched off and returns SJ_ERR_UNSUPPORTED: recording
 * a batch crashed the host process on MI355X with no cause found in this library's code.
 * sj_batch_create still validates plans. */

#define SJ_MAX_BATCH 256
typedef struct sj_batch sj_batch;
sj_status sj_batch_create(sj_ctx *ctx, sj_plan_t *const *plans, int32_t n, sj_batch **out);
sj_status sj_batch_submit(sj_batch *batch, int32_t *const *out_dev, const uint64_t *capacity_tuples, int32_t mode);
sj_status sj_batch_destroy(sj_batch *batch);

/* ---- serving: continuous admission of join queries (extension) ----
 *
 * A server runs many queries of the kind sj_plan accepts on one GPU at once. It owns
 * a caller-provided device arena (borrowed, 256-byte aligned, untouched by anyone
 * else while the server lives) and `slots` worker threads, each with its own HIP
 * stream (default priority). A query is admitted when a slot is free and its
 * workspace fits in the free arena; the oldest queued query that fits goes first, so
 * a later one may pass a query that does not fit yet. Once the exact count is known
 * the result's bytes are taken from the arena (SJ_ERR_CAPACITY if they can never fit
 * beside the workspace, SJ_ERR_NOMEM if no memory frees up within 2 s). While a running
 * query waits for its result's memory, no query is admitted; if every running query
 * waits (their workspaces fill the arena), the one admitted last frees its workspace and
 * goes back to the head of the queue, so the others can finish (it runs again later,
 * with the same result). The workspace
 * is freed when the query finishes; the result stays until sj_server_release. When no
 * query is running and no queued query fits for 2 s (the arena is held by results not
 * yet released), the oldest queued query fails with SJ_ERR_NOMEM, so every query
 * finishes or fails: callers release results as they consume them. Queries
 * on different slots overlap on the device. Each query's count, checksum and tuples
 * equal those of running it alone through sj_plan (same options): the kernels, inputs
 * and schedule are the same. The relations' device columns are borrowed until the
 * query is released. All server calls are thread-safe. */

#define SJ_MAX_SLOTS 16

#define SJ_QUERY_QUEUED 0
#define SJ_QUERY_RUNNING 1
#define SJ_QUERY_DONE 2
#define SJ_QUERY_FAILED 3

#define SJ_RESULT_TUPLES 0 /* materialise the row-id tuples into the arena (SJ_RIDS) */
#define SJ_RESULT_COUNT 1  /* count and checksum only */
#define SJ_RESULT_VALUES 2 /* materialise the value tuples (SJ_VALUES, default projection) */

typedef struct sj_server sj_server;

typedef struct {
    int32_t state;           /* SJ_QUERY_* */
    sj_status status;        /* SJ_OK, or the error that failed the query */
    uint64_t count, checksum;
    uint64_t result_offset;  /* byte offset of the count * width int32 words in the arena (DONE, tuples) */
    uint64_t workspace_bytes;
    int64_t t_submit_ns, t_admit_ns, t_done_ns; /* steady clock; 0 until reached */
    int32_t slot;            /* worker that ran it, -1 before admission */
    int32_t requeues;        /* times it gave its workspace back (see below) and was queued again */
    char error[160];         /* why the query failed ("" otherwise) */
} sj_query_info;

/* Start a server on HIP device `device` over arena [arena_dev, arena_dev + arena_bytes)
 * with 1..SJ_MAX_SLOTS workers. */
sj_status sj_server_create(int32_t device, void *arena_dev, uint64_t arena_bytes, int32_t slots, sj_server **out);
/* Validate and queue a query (same arguments as sj_plan; `opts` may be NULL). A graph
 * error or a workspace larger than the whole arena is returned here, and no ticket is
 * issued; sj_server_last_error describes it. */
sj_status sj_server_submit(sj_server *server, const sj_rel *rels, int32_t nrels, const sj_edge *edges,
                           int32_t nedges, const sj_opts *opts, int32_t result_mode, uint64_t *ticket);
/* State of a query; with wait != 0, block until it is DONE or FAILED. */
sj_status sj_server_query(sj_server *server, uint64_t ticket, int32_t wait, sj_query_info *info);
/* Forget a finished query and free its result (SJ_ERR_STATE while it is queued or running). */
sj_status sj_server_release(sj_server *server, uint64_t ticket);
/* Arena bytes in use and the peak so far, queries waiting for admission and running. */
sj_status sj_server_stats(sj_server *server, uint64_t *arena_used, uint64_t *arena_peak, int32_t *queued,
                          int32_t *running);
/* Text of the last submit error. */
const char *sj_server_last_error(const sj_server *server);
/* Fail the queued queries, wait for the running ones and stop the workers. */
sj_status sj_server_destroy(sj_server *server);

/* ---- filter catalogue: backward filters reused across queries (Section 2.3,
 *      "Reuse of Bloom Filters") ----
 *
 * A backward filter depends only on its relation's sub-tree of the join tree: the
 * relation's rows and predicate, the column it is built on, the columns its
 * children's filters are probed with, those filters (recursively) and the filter
 * options (bits_per_key, k, block_bits, seed, passes). A catalogue keeps such
 * filters resident in a caller-provided device arena (borrowed, 256-byte aligned,
 * used by no one else while the catalogue lives), keyed by a canonical signature of
 * exactly those inputs, in which relations are identified by their device column
 * pointers, row counts and predicate bounds. A plan attached to a catalogue reuses
 * every backward filter whose signature is resident: its build is dropped from the
 * pruning phase and the resident words are probed in place. A query that contains a
 * sub-join already answered (the paper's template Q1 inside an ad-hoc query Q2)
 * therefore skips those filter builds. Forward and closing-condition filters depend
 * on the whole query and are always built (for a cyclic query only the closing
 * filter is regenerated, as Section 2.3 describes). Survivor lists, counts, checksums
 * and tuples are identical with and without a catalogue: a reused filter holds the
 * same bits the plan would build.
 *
 * A filter the plan has to build is built straight into a catalogue entry reserved at
 * attach and is published once its build has been enqueued (later plans on other
 * streams wait for it with a HIP event). When the arena is full, unreferenced entries
 * are evicted least recently used first; a filter that still does not fit is built in
 * the plan's own workspace as usual. Entries referenced by a plan are never evicted.
 *
 * The catalogue cannot see writes to the columns: after changing a column's contents
 * in place, call sj_fcache_invalidate with its pointer (or sj_fcache_clear) and attach
 * new plans; a plan already attached keeps the entries it holds. All catalogue calls
 * are thread-safe; plans on different threads may share one catalogue. */

typedef struct sj_fcache sj_fcache;

typedef struct {
    uint64_t capacity_bytes, used_bytes;
    uint64_t entries;    /* resident (published) filters */
    uint64_t pinned;     /* entries held by at least one plan */
    uint64_t hits;       /* filters reused by an attaching plan */
    uint64_t misses;     /* filters an attaching plan builds into a new entry */
    uint64_t uncached;   /* misses with no room even after eviction (built in the workspace) */
    uint64_t evictions;
} sj_fcache_info;

/* Create a catalogue on HIP device `device` over [arena_dev, arena_dev + arena_bytes). */
sj_status sj_fcache_create(int32_t device, void *arena_dev, uint64_t arena_bytes, sj_fcache **out);
/* Attach `plan` to `cache` (NULL detaches). Resolves every backward filter of the plan
 * against the catalogue. A plan past sj_bind_workspace goes back to the bound state:
 * call sj_build_filters again. The plan keeps its entries until it is detached,
 * attached elsewhere or destroyed; the catalogue must outlive the attachment. */
sj_status sj_plan_use_filter_cache(sj_plan_t *plan, sj_fcache *cache);
/* How filter f of an attached plan is held: 0 in the plan's workspace, 1 reused from
 * the catalogue, 2 built by this plan into a catalogue entry. */
sj_status sj_plan_filter_cached(const sj_plan_t *plan, int32_t f, int32_t *how);
/* Drop every entry built from a column at `column_dev` (any column the filter's
 * sub-tree reads). Entries still held by plans leave the catalogue now and free their
 * memory when the last plan lets go. */
sj_status sj_fcache_invalidate(sj_fcache *cache, const void *column_dev);
/* Drop every entry (held ones as in sj_fcache_invalidate). */
sj_status sj_fcache_clear(sj_fcache *cache);
sj_status sj_fcache_stats(sj_fcache *cache, sj_fcache_info *info);
/* Destroy an empty-of-plans catalogue (SJ_ERR_STATE while a plan holds an entry).
 * Waits for the device work that used its entries. */
sj_status sj_fcache_destroy(sj_fcache *cache);
/* Attach every query the server runs from now on to `cache` (NULL: none). */
sj_status sj_server_use_filter_cache(sj_server *server, sj_fcache *cache);

#ifdef __cplusplus
}
#endif

#endif /* SIEVEJOIN_H */
