/*
 * gsmat: sparse-matrix BGP join on MI355X (gfx950) -- C ABI.
 *
 * Method (gSMat, arXiv 1807.07691):
 *   - An RDF dataset is a SET of (subject, predicate, object) triples
 *     (Sec. 3.1).  Vertices are caller-encoded int32 ids in [0, n_vertices),
 *     predicates int32 ids in [0, n_predicates) (the integer codes of the
 *     RDF cube, Sec. 5.1-5.2).
 *   - Each predicate h owns a boolean sparse matrix M_h of (s, o) pairs
 *     (Sec. 5.3), reached through a predicate-indexed table.  The library keeps
 *     every M_h twice: row-compressed by subject and column-compressed by
 *     object, each with the non-empty row ids, row offsets and member lists of
 *     the auxiliary arrays Row/Num/Rpos (Sec. 6.3).
 *   - A basic graph pattern (BGP) is a set of triple patterns (TPs) with a
 *     constant predicate (Sec. 3.2, Sec. 6.3).  Its answer is the final
 *     relation over all its variables obtained by joining the TP relations
 *     (Sec. 6, "Initializing / Joining / Returning"); with set semantics it is
 *     the set of assignments mu with (mu(s_i), p_i, mu(o_i)) in D for every i.
 *   - The plan orders TPs by statistics, keeping every new TP connected to the
 *     bound variables (Sec. 6.2, "connected minimal upper bound").
 *   - Every join step counts its output per input row, prefix-sums the counts
 *     and writes each row's output at its offset (Sec. 7.2.2, Algorithm
 *     "Pre-allocating result matrix space").
 *
 * Conventions for every entry point:
 *   - Return value: a gsmat_status; GSMAT_OK on success.  On error nothing is
 *     returned through output pointers (except the batch entry points, which
 *     hand back every query that succeeded and a status per query) and
 *     gsmat_last_error() describes the failure (thread-local).  No entry
 *     point throws or aborts.
 *   - Argument validation happens before any device work.
 *   - Handles (store, plan, result) are owned by the caller and released with
 *     the matching *_free.  A plan or result must not outlive its store.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a call is enqueued on that stream; calls return after
 *     the work they need on the host side has completed.
 *   - Device memory comes from the library's caching block allocator (blocks
 *     from hipMalloc, reused per stream, cross-stream reuse ordered by events)
 *     unless an allocator is given to gsmat_load_triples.
 *   - The store's index is immutable after gsmat_build_index; concurrent
 *     gsmat_join calls on different streams (and different results) are
 *     allowed.  gsmat_set_sparse_expand, gsmat_set_batch_tuning and
 *     gsmat_autotune_batch change tuning settings of the store and must not
 *     overlap other calls on it.
 *   - A result's (and a server's) memory is returned to the allocator on the
 *     stream it was made on: that stream must outlive them.
 *   - A gsmat_server_step whose round fails (device allocation, HIP error)
 *     returns that status; the queries the round carried finish as failed
 *     with it (reported by gsmat_server_poll) and the server stays usable.
 */
#ifndef GSMAT_H
#define GSMAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gsmat_status;
enum {
  GSMAT_OK = 0,
  GSMAT_EINVAL = 1,       /* bad pointer, size or id; malformed BGP */
  GSMAT_ENOMEM = 2,       /* device allocation failed, or budget below one row */
  GSMAT_EHIP = 3,         /* HIP runtime error (no device, launch failure, ...) */
  GSMAT_ESTATE = 4,       /* call out of order (e.g. join before build_index) */
  GSMAT_EUNSUPPORTED = 5, /* variable predicate, or ids too wide to pack */
  GSMAT_ETOOBIG = 6       /* result rows exceed the caller's max_rows */
};

typedef struct gsmat_store gsmat_store;   /* device CSR/CSC of every predicate */
typedef struct gsmat_query_plan gsmat_query_plan; /* host-only ordered step list */
typedef struct gsmat_result gsmat_result; /* device binding table, possibly in segments */
typedef struct gsmat_server gsmat_server; /* request loop over one store (continuous batching) */
typedef struct gsmat_dict gsmat_dict;     /* host string dictionary (h_p, h_so) */

/* Optional device allocator.  alloc returns NULL on failure.  free receives
 * the pointer and size that alloc returned.  Both are called on the host
 * thread of the gsmat call, with the stream the memory is used on. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, size_t bytes, void* stream, void* ctx);
  void* ctx;
} gsmat_allocator;

/* One triple pattern.  s and o: >= 0 is a vertex constant, < 0 is the
 * variable number -(x+1).  p: a predicate constant (>= 0); a negative p
 * (a variable predicate) is GSMAT_EUNSUPPORTED (Sec. 6.3 assumes it is known).
 * The variables of a BGP must be numbered densely 0..n_vars-1. */
typedef struct {
  int32_t s, p, o;
} gsmat_pattern;

/* Step kinds reported by gsmat_plan_info. */
enum {
  GSMAT_STEP_SCAN = 0,      /* materialise one TP's relation (first step) */
  GSMAT_STEP_INTERSECT = 1, /* star centre: intersect row/column id lists */
  GSMAT_STEP_EXPAND = 2,    /* one endpoint bound: append the other's neighbours */
  GSMAT_STEP_FILTER = 3,    /* both endpoints bound/constant: membership test */
  GSMAT_STEP_CARTESIAN = 4  /* no shared variable: cross product */
};

/* Plan modes. */
enum {
  GSMAT_PLAN_PAPER = 0,   /* statistic = pair count of the predicate; pure
                             connected-minimal-upper-bound order (Sec. 6.2.1) */
  GSMAT_PLAN_DEFAULT = 1,  /* statistic = triples the TP matches on its own;
                              constant-only TPs first; star centre intersection
                              as first step; filters before expansions */
  GSMAT_PLAN_ADAPTIVE = 2  /* GSMAT_PLAN_DEFAULT's first steps; afterwards the
                              join picks, at every step, a connected TP whose
                              endpoints are bound (filter) if any, else the
                              expansion with the smallest output estimated from
                              a sample of the bound rows; gsmat_plan_info then
                              reports the static order, not the executed one */
};

typedef struct {
  int32_t kind;        /* GSMAT_STEP_* */
  int32_t tp;          /* the TP this step evaluates (INTERSECT: first member) */
  int32_t orient;      /* EXPAND: 0 = from bound subject (row-compressed),
                          1 = from bound object (column-compressed); else -1 */
  int32_t var;         /* variable this step binds (INTERSECT: the centre; SCAN:
                          the subject variable or the object variable if the
                          subject is constant); -1 if none */
  uint32_t members;    /* INTERSECT: bit i set if TP i is in the star */
  int32_t pad;
  int64_t est_rows;    /* upper bound on the rows after this step (saturated) */
} gsmat_step_info;

/* ---- storage (Sec. 5) ---------------------------------------------------- */

/* Copies n host triples (s[i], p[i], o[i]) to the device.  Duplicates are
 * allowed and removed by gsmat_build_index (D is a set).  EINVAL if any id is
 * out of range, n < 0, or a pointer is NULL while n > 0; EUNSUPPORTED if
 * bits(n_predicates-1) + 2*bits(n_vertices-1) > 64 or n >= 2^32 (the device
 * sort ranks keys with 32-bit positions).  `alloc` may be NULL. */
gsmat_status gsmat_load_triples(const int32_t* s, const int32_t* p, const int32_t* o, int64_t n,
                                int32_t n_vertices, int32_t n_predicates,
                                const gsmat_allocator* alloc, void* stream, gsmat_store** out);

/* Builds, on the device, the per-predicate matrices: sort, deduplicate, split
 * by predicate, compress by subject and by object, and record statistics
 * (pair count, non-empty rows, non-empty columns) -- Sec. 5.3.  Predicates
 * whose non-empty rows reach n_vertices/dense_div also get a dense row
 * pointer (dense_div <= 0: default 32).  Idempotent. */
gsmat_status gsmat_build_index(gsmat_store* st, int32_t dense_div, void* stream);

/* Whole-store statistics: distinct triples, predicate count, device bytes
 * held by the index.  ESTATE before build. */
gsmat_status gsmat_store_stats(const gsmat_store* st, int64_t* n_triples, int32_t* n_predicates,
                               int64_t* device_bytes);

/* Hub bitmaps (an index option, Sec. 5.3 storage): in each orientation the
 * longest rows with at least min_len members (longest first, while their
 * bitmaps fit in max_bytes) also get a bitmap over all vertex ids, so a
 * membership test against such a row (a filter, or an intersection with a
 * constant's row) reads one bit instead of searching the row.  Results do not
 * change.  Off by default (min_len 16384, max_bytes 0); min_len <= 0 or
 * max_bytes <= 0 disables them.  Must precede gsmat_build_index (ESTATE
 * after). */
gsmat_status gsmat_set_hub_options(gsmat_store* st, int64_t min_len, int64_t max_bytes);

/* Statistics of one predicate: pairs, distinct subjects, distinct objects. */
gsmat_status gsmat_pred_stats(const gsmat_store* st, int32_t pred, int64_t* nnz, int64_t* n_rows,
                              int64_t* n_cols);

/* Copies one predicate's compressed matrix to host buffers: orient 0 = by
 * subject, 1 = by object.  keys[n_rows] (non-empty row ids ascending),
 * ptr[n_rows+1] (0-based offsets; ptr[0] = 0), nbr[nnz] (members ascending
 * within a row).  Sizes from gsmat_pred_stats (n_cols rows for orient 1). */
gsmat_status gsmat_export_matrix(const gsmat_store* st, int32_t pred, int32_t orient,
                                 int32_t* keys, int32_t* ptr, int32_t* nbr, void* stream);

void gsmat_store_free(gsmat_store* st);

/* ---- planning (Sec. 6.2) ------------------------------------------------- */

/* Orders the n_pats TPs and classifies each step.  Statistics come from the
 * store (mode GSMAT_PLAN_DEFAULT looks up the degrees of constants on the
 * device).  EINVAL on malformed patterns or non-dense variable numbers,
 * EUNSUPPORTED on a variable predicate or n_pats > 32. */
gsmat_status gsmat_plan(const gsmat_store* st, const gsmat_pattern* pats, int32_t n_pats,
                        int32_t mode, void* stream, gsmat_query_plan** out);

/* Host-only planning from caller-supplied per-TP statistics (the sort keys,
 * stat[i] >= 0) and per-TP "list sizes" for star intersection estimates
 * (may be NULL: stat is used).  Same rules as gsmat_plan. */
gsmat_status gsmat_plan_from_stats(const gsmat_pattern* pats, int32_t n_pats, int32_t mode,
                                   const int64_t* stat, gsmat_query_plan** out);

/* Number of steps and variables; steps[] receives up to `cap` entries. */
gsmat_status gsmat_plan_info(const gsmat_query_plan* pl, int32_t* n_steps, int32_t* n_vars,
                             gsmat_step_info* steps, int32_t cap);

void gsmat_plan_free(gsmat_query_plan* pl);

/* Plans n_queries BGPs at once: query i has the n_pats[i] patterns that
 * follow those of queries 0..i-1 in pats.  Same plans as gsmat_plan per
 * query; the device lookups of every query's constants go out as one batch
 * (one stream synchronisation for the whole call).  out[i] receives query
 * i's plan, or NULL when its patterns are rejected; status[i] (may be NULL)
 * its status.  Returns OK when every query was planned, else the status of
 * the first failed query (the other plans are still returned and must be
 * freed). */
gsmat_status gsmat_plan_batch(const gsmat_store* st, const gsmat_pattern* pats,
                              const int32_t* n_pats, int32_t n_queries, int32_t mode,
                              void* stream, gsmat_query_plan** out, gsmat_status* status);

/* ---- execution (Sec. 6.3, Sec. 7.2) --------------------------------------- */

/* Evaluates the plan on the device.  budget_bytes bounds each step's output
 * buffer; a larger step is cut into output ranges that are carried through
 * the remaining steps one at a time (chunked expansion, Sec. 7.3 "block
 * transmission"); budget_bytes <= 0 means no limit.  max_rows < 0 means no
 * limit; otherwise a result with more rows fails with ETOOBIG.  ENOMEM when an
 * allocation fails or the budget cannot hold a single output row. */
gsmat_status gsmat_join(gsmat_store* st, const gsmat_query_plan* pl, int64_t budget_bytes,
                        int64_t max_rows, void* stream, gsmat_result** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * evaluation of gsmat_join (no step budget, no max_rows), with every
 * intermediate table and every step's scratch kept in a fixed 64 MiB device
 * array of the library (one per GPU, held until the process ends), and the
 * result copied into the caller's device buffer: variable v's column at
 * out + v * out_stride, rows [0, *n_rows), in the row order gsmat_join gives.
 * No device memory is allocated or freed.  *n_rows always receives the row
 * count when it is known.  EINVAL for a NULL store, plan or n_rows, a NULL
 * out with out_cap > 0, out_cap < 0 or out_stride < out_cap; ENOMEM (message
 * names the limit) when the intermediates and the result do not fit the
 * 64 MiB array; ETOOBIG when the result has more than out_cap rows.  Calls on
 * one GPU share its array: they are serialised by a lock, and each call's
 * device work has ended when it returns. */
gsmat_status gsmat_join_noalloc(gsmat_store* st, const gsmat_query_plan* pl, int32_t* out,
                                int64_t out_stride, int64_t out_cap, int64_t* n_rows,
                                void* stream);

/* Evaluates n_plans plans together (Sec. 7.2's count, prefix sum, exact
 * allocation and write, run as one launch per phase for every query in the
 * batch).  Each query takes the same steps as under gsmat_join and yields
 * the same rows in the same order.  A query whose next step would need a
 * Cartesian product, a (?x p ?x) pattern, or a step output above
 * budget_bytes (or the batch's outputs of one step above budget_bytes in
 * total) is finished alone, as gsmat_join would.  budget_bytes and
 * max_rows apply per query as in gsmat_join.  out[i] receives query i's
 * result, or NULL if it failed; status[i] (may be NULL) its status.  Returns
 * OK when every query succeeded, else the status of the first failed query
 * (the other results are still returned and must be freed); a failure of
 * the batch itself (HIP error, device allocation) returns no results. */
gsmat_status gsmat_join_batch(gsmat_store* st, const gsmat_query_plan* const* plans,
                              int32_t n_plans, int64_t budget_bytes, int64_t max_rows,
                              void* stream, gsmat_result** out, gsmat_status* status);

/* How gsmat_join_batch runs its rounds (the rows and their order are the
 * same either way):
 *   1 (default) device-driven: every query's state stays in device memory; a
 *     round is a fixed sequence of launches that choose each query's step,
 *     count, scan, allocate (bump allocation from an output slab and a
 *     scratch region) and write, with sizes read on the device, so the host
 *     enqueues as many rounds as the longest plan needs and waits once.  A
 *     task that does not fit the regions waits a round; at the wait the host
 *     adds larger regions and runs the remaining rounds.  The batch's
 *     intermediate tables stay in device memory until its results are freed.
 *   0 host-driven: the host builds every round's tasks and allocations from
 *     sizes read back twice per round (the serving loop always runs so).
 * EINVAL for another value. */
gsmat_status gsmat_set_batch_engine(gsmat_store* st, int32_t engine);

/* Starting sizes, in bytes, of the device-driven batch's output slab and
 * scratch region for the next gsmat_join_batch on the store (0: 256 MiB and
 * 128 MiB).  After every batch the store keeps the sizes that batch needed
 * (plus an eighth) as the next starting sizes.  Small regions only cost
 * extra rounds; the rows do not change.  EINVAL for a negative size. */
gsmat_status gsmat_set_batch_regions(gsmat_store* st, int64_t out_bytes, int64_t scratch_bytes);

/* gsmat_plan_batch and gsmat_join_batch in one call, with the device-driven
 * rounds (the plan of Sec. 6.2 and the join of Sec. 6-7): the queries'
 * patterns as for gsmat_plan_batch (pats holds the n_pats[i] patterns of
 * query i after those of queries 0..i-1), planned in mode on the host and
 * packed straight into the batch's upload, with no plan objects.  Every query
 * yields exactly the rows, in the same order, and the per-step counters it
 * yields through gsmat_plan_batch + gsmat_join_batch.  out[i] and status[i]
 * as for gsmat_join_batch; a query that fails planning has its planning
 * status and no result.  EINVAL (nothing run) for a NULL store, array or
 * out, a negative count or an unknown mode; the store's batch engine setting
 * is not consulted. */
gsmat_status gsmat_join_batch_bgp(gsmat_store* st, const gsmat_pattern* pats,
                                  const int32_t* n_pats, int32_t n_queries, int32_t mode,
                                  int64_t budget_bytes, int64_t max_rows, void* stream,
                                  gsmat_result** out, gsmat_status* status);

/* Frees n plans (NULL entries are skipped) and sets every entry to NULL. *//* Frees n plans (NULL entries are skipped) and sets every entry to NULL. */
void gsmat_plan_free_many(gsmat_query_plan** plans, int32_t n);

/* Frees n results (NULL entries are skipped) and sets every entry to NULL. */
void gsmat_result_free_many(gsmat_result** results, int32_t n);

/* rows[i] = row count of results[i], or -1 for a NULL entry. */
gsmat_status gsmat_result_rows_many(const gsmat_result* const* results, int32_t n, int64_t* rows);

/* Sparse expansions in the batched join: an expansion of at least min_rows
 * input rows of which fewer than the fraction theta have any output first
 * compacts its rows with output (in order, with their output offsets) and
 * then walks only those in the merge-path write; the rows written and their
 * order do not change.  theta in [0, 1], 0 never; defaults 0.5 and 4096. */
gsmat_status gsmat_set_sparse_expand(gsmat_store* st, double theta, int64_t min_rows);

/* Count-phase tile shape and intersection strategy of the device-driven
 * batched join (engine 1).  Every count tile covers 2048 input rows;
 * count_items rows per thread (4, 8 or 16) sets its workgroup to 512, 256
 * or 128 threads.  Sorted-list intersections (a star centre bound from
 * several patterns with constant other endpoints, Sec. 6.3's first step)
 * take one of:
 *   GSMAT_ISECT_SEARCH (0, default): each driver id binary-searches every
 *     other list in device memory;
 *   GSMAT_ISECT_WINDOW (1): the ids a tile of the sorted driver can meet
 *     form one window of each list; a window of up to 2048 ids is staged in
 *     LDS (the paper keeps small operands in shared memory, Sec. 7.3) and
 *     searched there, a longer one is searched in memory within its bounds;
 *   GSMAT_ISECT_MERGE (2): a staged window is merged with the tile's driver
 *     ids along the merge path (equal shares of the two sorted sequences
 *     per thread); a longer one is searched as with WINDOW.
 * Lists with a hub bitmap (gsmat_build_index's hub option) are tested one
 * bit at a time and lists of row keys by row lookups under every strategy.
 * The rows and their order do not depend on either setting; the single-query
 * join and the host-driven rounds always search with 8 rows per thread.
 * Defaults 8 and SEARCH; EINVAL for other values. */
#define GSMAT_ISECT_SEARCH 0
#define GSMAT_ISECT_WINDOW 1
#define GSMAT_ISECT_MERGE 2
gsmat_status gsmat_set_batch_tuning(gsmat_store* st, int32_t count_items, int32_t intersect);

/* The store's batch tuning settings (any pointer may be NULL). */
gsmat_status gsmat_get_batch_tuning(const gsmat_store* st, double* theta, int64_t* min_rows,
                                    int32_t* count_items, int32_t* intersect);

/* The write strategy the batched join takes for an expansion of n_in input
 * rows of which n_nonempty have output, under the setting (theta, min_rows):
 * 1 = sparse (compacted rows with output), 0 = merge path over every row.
 * The compacted row list holds 32-bit row indices, so an expansion of 2^31
 * or more input rows always takes the merge path over every row.  Host
 * only, no device work. */
int32_t gsmat_expand_strategy(double theta, int64_t min_rows, int64_t n_in, int64_t n_nonempty);

/* What gsmat_autotune_batch chose and timed.  A candidate's time is the
 * fastest of three gsmat_join_batch runs in milliseconds (host wall time,
 * results discarded); -1 where a setting was not tuned. */
typedef struct gsmat_tune_report {
  double theta;            /* chosen sparse-expansion threshold */
  int32_t count_items;     /* chosen count rows per thread */
  int32_t intersect;       /* chosen GSMAT_ISECT_* */
  double theta_ms[5];      /* theta 0, 0.25, 0.5, 0.75, 1 */
  double items_ms[3];      /* count_items 4, 8, 16 */
  double intersect_ms[3];  /* SEARCH, WINDOW, MERGE */
} gsmat_tune_report;

/* Autotuner over the batched join's settings, one at a time in the order
 * theta, count_items, intersect: runs gsmat_join_batch on the plans once
 * untimed, then times each candidate of the setting with the others fixed
 * and keeps the fastest (the store's current value stays unless another is
 * faster by more than 3 %) before tuning the next.  With the host-driven
 * engine only theta is tuned.  The rows of any later join do not depend on
 * the choices.  rep may be NULL. */
gsmat_status gsmat_autotune_batch(gsmat_store* st, const gsmat_query_plan* const* plans,
                                  int32_t n_plans, int64_t budget_bytes, void* stream,
                                  gsmat_tune_report* rep);

/* Result shape; per-step rows in/out (arrays of n_steps entries, may be NULL)
 * are summed over chunks. */
gsmat_status gsmat_result_info(const gsmat_result* r, int64_t* n_rows, int32_t* n_vars,
                               int32_t* n_steps, int64_t* step_rows_in, int64_t* step_rows_out);

/* Copies rows [row_offset, row_offset + max_rows) (clipped to the result) to
 * host_rows, row-major [rows][n_vars], column j = variable j.  Row order is
 * unspecified but fixed for a given result.  *n_written = rows copied. */
gsmat_status gsmat_fetch_bindings(const gsmat_result* r, int64_t row_offset, int64_t max_rows,
                                  int32_t* host_rows, int64_t* n_written, void* stream);

void gsmat_result_free(gsmat_result* r);

/* ---- OPTIONAL, UNION and FILTER (Sec. 9) ---------------------------------
 *
 * The paper names these operators as future work without defining them.
 * Here they take the SPARQL algebra's meaning over bags of solution mappings,
 * and every BGP inside a query runs on the sparse-matrix join (Sec. 6-7).
 *
 * A query is the bag union of its branches, in ascending branch id.  A
 * branch has three parts:
 *   - its required BGP (the patterns of group 0; with none, the bag holding
 *     one mapping that binds nothing);
 *   - its OPTIONAL BGPs (groups 1, 2, ...), left-joined in ascending group id;
 *   - the conjunction of its FILTER conditions, applied last.
 * LeftJoin(A, B) keeps every merge of a row of A with a compatible row of B
 * (equal on every variable bound in both).  A row of A that has no such row
 * in B is kept alone.
 *
 * Patterns must be well designed: a variable that an OPTIONAL group shares
 * with any other group of its branch must occur in the branch's required
 * BGP.  Otherwise the call returns GSMAT_EUNSUPPORTED.  The required rows are
 * numbered, B's patterns run from the required table itself (the adaptive
 * step choice expands and filters off its bound columns), and the rows no
 * match kept are compacted and returned with B's variables unbound.
 *
 * FILTER conditions compare term ids: a variable or a constant id on each
 * side.  A comparison with an unbound operand is an error, and the row is
 * dropped (for != as well).  BOUND and NOT_BOUND take a variable in a.
 */
typedef struct {
  int32_t s, p, o;  /* as in gsmat_pattern; variables 0..n_vars-1 */
  int32_t branch;   /* union branch (>= 0) */
  int32_t group;    /* 0 required, > 0 an OPTIONAL group */
} gsmat_ext_pattern;

#define GSMAT_F_EQ 0
#define GSMAT_F_NE 1
#define GSMAT_F_LT 2
#define GSMAT_F_LE 3
#define GSMAT_F_GT 4
#define GSMAT_F_GE 5
#define GSMAT_F_BOUND 6
#define GSMAT_F_NOT_BOUND 7
typedef struct {
  int32_t op;      /* GSMAT_F_* */
  int32_t a, b;    /* terms: >= 0 an id, < 0 the variable -(x+1); b unused by BOUND ops */
  int32_t branch;  /* the branch it filters (a branch may consist of filters only) */
} gsmat_filter;

/* Evaluates the query.  n_vars (0..31) is the number of result columns: each
 * variable a term names must be below it, and a variable a row does not bind
 * is fetched as -1.  Rows come in branch order.  Within a branch their order
 * is unspecified but fixed for given inputs.  budget_bytes and max_rows act
 * as in gsmat_join: the budget chunks each BGP step, and max_rows bounds the
 * final row count (GSMAT_ETOOBIG).  The result has no per-step counters
 * (n_steps 0).
 * Errors:
 *   - The query is checked before the store and before any device work.
 *   - EINVAL: an empty query, a variable at or above n_vars, a negative branch
 *     or group, an unknown op, or BOUND on a constant.
 *   - EUNSUPPORTED: a variable predicate, a BGP of more than 32 patterns, more
 *     than 16 conditions in a branch, n_vars above 31, a pattern that is not
 *     well designed, or an OPTIONAL whose left side has 2^31 rows or more. */
gsmat_status gsmat_join_ext(gsmat_store* st, const gsmat_ext_pattern* pats, int32_t n_pats,
                            const gsmat_filter* filters, int32_t n_filters, int32_t n_vars,
                            int64_t budget_bytes, int64_t max_rows, void* stream,
                            gsmat_result** out);

/* ---- text boundary: dictionary and BGP parser (Sec. 5.2, Sec. 6.3) -------- */

/* A host dictionary: the bijections h_p (predicates) and h_so (subjects and
 * objects together), each assigning codes by order of occurrence (Sec. 5.2).
 * Codes are 0-based (the paper's codes minus one).  Host only; no device
 * work; not thread-safe. */
gsmat_status gsmat_dict_new(gsmat_dict** out);
void gsmat_dict_free(gsmat_dict* d);

/* Parses text triples, one per line, each ended by '.' or the line break:
 * terms are <iri>, "literal" (optional @lang or ^^<iri>), _:blank or any
 * other token without white space; '#' starts a comment.  Terms are coded in
 * order of occurrence (subject, predicate, object of each triple in turn),
 * continuing the dictionary's earlier codes.  The triples' codes are kept
 * for gsmat_dict_triples (replacing the previous text's).  EINVAL on a
 * syntax error (message names the line); the dictionary is then unchanged. */
gsmat_status gsmat_dict_load_text(gsmat_dict* d, const char* text, size_t len,
                                  int64_t* n_triples);

/* Copies the last loaded text's triple codes: s, p, o each [n_triples]. */
gsmat_status gsmat_dict_triples(const gsmat_dict* d, int32_t* s, int32_t* p, int32_t* o);

/* Number of subject/object terms and of predicates coded so far (the
 * n_vertices and n_predicates to load the triples with). */
gsmat_status gsmat_dict_sizes(const gsmat_dict* d, int32_t* n_terms, int32_t* n_predicates);

/* Code of one term (is_predicate selects h_p or h_so), -1 if absent. */
gsmat_status gsmat_dict_lookup(const gsmat_dict* d, const char* term, size_t len,
                               int32_t is_predicate, int32_t* code);

/* The term of a code (the decoding of results, Sec. 6.3): *len = its length;
 * with buf, copies it NUL-terminated (ETOOBIG if cap is too small).  EINVAL
 * for a code the dictionary does not have. */
gsmat_status gsmat_dict_term(const gsmat_dict* d, int32_t code, int32_t is_predicate, char* buf,
                             size_t cap, size_t* len);

/* Parses a BGP: either "SELECT ... WHERE { patterns }" or the bare pattern
 * list, patterns separated by '.'.  ?name and $name are variables, numbered
 * 0.. by first appearance (every variable is returned; a projection list is
 * not used); other terms are constants coded with the dictionary, a term it
 * has not seen getting one past its last code (it matches nothing).
 * Writes *n_pats (ETOOBIG with *n_pats set when it exceeds cap) and
 * *n_vars; var_names (may be NULL) receives the variable names without
 * their sigil, NUL-separated, in variable order.  EUNSUPPORTED on a
 * variable predicate. */
gsmat_status gsmat_parse_bgp(const gsmat_dict* d, const char* text, size_t len,
                             gsmat_pattern* pats, int32_t cap, int32_t* n_pats, int32_t* n_vars,
                             char* var_names, size_t names_cap);

/* ---- serving (continuous batching) ---------------------------------------- */

/* A request loop over one built store, on one stream.  Submitted plans wait
 * in arrival order until admitted: a query is admitted when a slot is free
 * (at most max_active admitted) and the bytes the admitted queries hold or
 * are estimated to need, plus its own estimate, stay within
 * mem_budget_bytes (a query is always admitted when none is).  The estimate
 * is the plan's largest table: the first step's relation size from the
 * planning lookups, each later expansion multiplying it by the mean row
 * length of its predicate, capped by the Theorem 1 bound (Sec. 6.2).  Each
 * gsmat_server_step admits what fits and runs one step of every admitted
 * query as one batched round (as in gsmat_join_batch with host-driven
 * rounds), so queries that arrive while others run join them at the next
 * round; when the server holds at most two queries, none started and none
 * waiting, the step instead runs the oldest to completion with the
 * single-query executor (the other waits for the next step; later arrivals
 * are admitted at the next step).  A round whose
 * outputs would exceed mem_budget_bytes defers the later queries' steps to
 * the next round (the first always runs).  step_budget_bytes and max_rows
 * apply per query as in gsmat_join (a step above step_budget_bytes finishes
 * alone, chunked).  Every query yields the rows, in the same order, that
 * gsmat_join gives it.  The store must outlive the server; plans must stay
 * alive until their result is polled.  Not thread-safe: one caller thread. */
gsmat_status gsmat_server_new(gsmat_store* st, int64_t mem_budget_bytes,
                              int64_t step_budget_bytes, int64_t max_rows, int32_t max_active,
                              void* stream, gsmat_server** out);

/* Queues a plan with the caller's tag (no device work). */
gsmat_status gsmat_server_submit(gsmat_server* sv, const gsmat_query_plan* pl, int64_t tag);

/* Admits waiting queries and runs one round.  Outputs (may be NULL): queries
 * admitted and unfinished, waiting, and finished but not yet polled. */
gsmat_status gsmat_server_step(gsmat_server* sv, int32_t* n_active, int32_t* n_waiting,
                               int32_t* n_done);

/* Hands over up to cap finished queries in completion order: tags[i],
 * results[i] (owned by the caller, NULL when the query failed) and
 * status[i].  *n_out = entries written.  Synchronises the stream first, so
 * the results are complete. */
gsmat_status gsmat_server_poll(gsmat_server* sv, int32_t cap, int64_t* tags,
                               gsmat_result** results, gsmat_status* status, int32_t* n_out);

/* Frees the server, its waiting queue and unpolled results. */
void gsmat_server_free(gsmat_server* sv);

/* Thread-local message for the last non-OK status of this thread. */
const char* gsmat_last_error(void);

/* Waits for the device and returns the unused blocks cached by the library's
 * allocator to the driver (the allocator stays usable).  Meant for process
 * shutdown after every handle is freed, and for callers that need the memory
 * back for other allocators. */
gsmat_status gsmat_release_pools(void);

/* ---- instrumentation ----------------------------------------------------- */

/* Rounds of the store's last device-driven gsmat_join_batch (at most 64
 * recorded): *n_rounds receives their number and out[8 * i + f] (for i <
 * cap) round i's f-th figure: tasks counted, count tiles, post tiles
 * (row offsets, compacted rows, filter and intersection compactions), write
 * tiles, split entries, output bytes allocated, candidate expansions
 * sampled, tasks deferred for lack of memory.  Host only. */
gsmat_status gsmat_batch_round_stats(const gsmat_store* st, int64_t* out, int32_t cap,
                                     int32_t* n_rounds);

/* Kernel classes timed when profiling is on. */
enum {
  GSMAT_K_COUNT = 0,    /* per-row output counts (+ tile sums) */
  GSMAT_K_SCAN = 1,     /* prefix sums */
  GSMAT_K_WRITE = 2,    /* expansion write (merge-path) */
  GSMAT_K_COMPACT = 3,  /* ordered compaction for filters / intersections */
  GSMAT_K_OTHER = 4,
  GSMAT_K_NCLASS = 5
};

/* Bit c of class_mask set: record a HIP event pair around every launch of
 * kernel class c, on the launch's stream (adds a little host work per launch);
 * 0 stops recording.  Resets the counters. */
void gsmat_prof_enable(int32_t class_mask);

/* Per class: launches, summed kernel milliseconds, algorithmic bytes.  Waits
 * for the recorded events.  Arrays of GSMAT_K_NCLASS entries. */
gsmat_status gsmat_prof_read(int64_t* launches, double* ms, double* bytes);

/* Host-side counters since the last gsmat_prof_enable: out5[0] ms inside
 * device allocations, [1] allocation count, [2] ms inside frees, [3] ms
 * waiting for streams, [4] number of waits. */
gsmat_status gsmat_prof_host(double* out5);

#ifdef __cplusplus
}
#endif

#endif /* GSMAT_H */
