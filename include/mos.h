/* mos.h -- exact multi-objective shortest paths on one AMD Instinct MI355X (gfx950).
 *
 * ABI version 1.  C interface; every id is 0-based; objectives are int32 and
 * non-negative.
 *
 * The problem (paper, Section 3): a directed graph G = (V, E, c) whose arcs
 * carry non-negative cost vectors c(e) of length D; given a start node v_s and
 * a goal node v_g, find the cost-unique set of Pareto-optimal v_s -> v_g path
 * costs (no returned vector is dominated by, or equal to, the cost of another
 * v_s -> v_g path) and one witness path per cost.  a dominates b when
 * a[k] <= b[k] for every k and a[k] < b[k] for some k.
 *
 * The search is the paper's ordered label-setting method (Algorithm 1,
 * NAMOA*, run in batches as in Algorithm 2, OPMOS): each step pops the B
 * lexicographically smallest open labels (ordered by F = g + h), expands their
 * out-arcs, filters the candidates against the goal front and against each
 * target node's frontier, prunes the frontier labels they dominate, resolves
 * dominance among candidates of the same step, and inserts the survivors.  The
 * heuristic h_k(v) is the exact shortest v -> v_g distance under objective k
 * (Section 4), computed on the GPU.  Only the expansion order depends on B;
 * the returned cost set does not.
 *
 * Memory: every array argument is HOST memory.  mos_graph_create copies the
 * graph to device memory; results are copied back to host memory and owned by
 * the mos_result handle.  Every destroy function accepts NULL.
 *
 * Errors: no call aborts.  Every call that can fail returns a mos_status;
 * out-parameters are written only on MOS_OK (and, for the calls that return
 * a result, on MOS_E_STEP_LIMIT, whose result is an exact prefix).  Argument validation happens
 * before any device call.  mos_last_error() gives a thread-local message for
 * the last failing call on the calling thread.
 */
#ifndef MOS_H_
#define MOS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOS_ABI_VERSION 1
#define MOS_MAX_OBJECTIVES 12 /* largest D accepted by mos_graph_create */

typedef struct mos_graph mos_graph;
typedef struct mos_result mos_result;
typedef struct mos_server mos_server;

typedef enum {
  MOS_OK = 0,
  MOS_E_INVALID_ARG = 1,   /* bad id, size, pointer or option */
  MOS_E_NEGATIVE_COST = 2, /* an arc cost is < 0 */
  MOS_E_OVERFLOW_RISK = 3, /* 2*sum_e c_k(e) + max_e c_k(e) >= INT32_MAX for some k */
  MOS_E_NO_DEVICE = 4,     /* no visible HIP device */
  MOS_E_DEVICE = 5,        /* a HIP runtime call failed */
  MOS_E_OUT_OF_MEMORY = 6, /* device or host allocation failed */
  MOS_E_LABEL_LIMIT = 7,   /* the search outgrew label_limit / the memory budget;
                              no partial front is ever reported as complete */
  MOS_E_CANCELLED = 8,     /* a served query was cancelled */
  MOS_E_NOT_READY = 9,     /* a served query has not finished yet */
  MOS_E_STEP_LIMIT = 10    /* the query reached options.step_budget: its result holds
                              only the exact part of the front below
                              stats.open_min_f1 (see step_budget) */
} mos_status;

/* Order in which OPEN is processed (mos_options.pop_order).  Any order gives
 * the same front (the search removes only dominated labels); the order decides
 * the work.  LEXICOGRAPHIC: each step pops the B lexicographically smallest F
 * (Algorithm 1's priority queue, batched as in Algorithm 2).  GENERATION: a
 * relaxed order, each step pops the B oldest labels by the step that generated
 * them (ties by F_2..F_d, then label id) -- a first-in first-out queue of
 * generations, the FIFO alternative to the priority queue that Section 7.1
 * measures. */
#define MOS_POP_LEXICOGRAPHIC 0
#define MOS_POP_GENERATION 1

/* Options for one solve.  Zero-initialise, set struct_size = sizeof(mos_options),
 * then override fields.  NULL options means all defaults. */
typedef struct {
  uint32_t struct_size;
  int32_t n_objectives; /* 0 = all D; else objectives 0..n-1 in stored order
                           (the paper's convention for its objective subsets, Table 1) */
  int32_t batch_width;  /* B, labels popped per step (paper: NUM_POP), 1..32768; 0 = default */
  int32_t max_slots;    /* mos_solve_batch: queries resident at once; 0 = auto */
  int64_t label_limit;  /* per query; 0 = bounded only by mem_budget */
  int64_t mem_budget;   /* bytes of device memory for search state; 0 = auto */
  void* stream;         /* hipStream_t to run on, or NULL for the library's own */
  int32_t costs_only;   /* 0 (default) = also reconstruct witness paths; 1 = costs only */
  int32_t steps_per_poll; /* device steps between host status polls; 0 = default */
  int32_t profile_kernels; /* sessions only: bit i set = time kernel i of every step with
                              HIP events (-1 = every kernel); the kernels are then
                              launched one by one instead of from a captured graph */
  int32_t heuristic_radius; /* heuristic (Section 4's reverse SSSP per objective): the
                              reverse search is cut at r * h_k(start) for r > 0, nodes
                              beyond the cut get the admissible lower bound cut + 1;
                              0 = default (r = 4); negative = exact on the whole graph.
                              The front does not depend on it, only the work does. */
  int64_t step_budget;      /* 0 = none; else a query still running after this many
                              label steps (counted at the next host poll) stops and
                              returns MOS_E_STEP_LIMIT together with a result: its
                              goal front so far cut to the entries whose first
                              objective is below stats.open_min_f1, the smallest
                              F_1 = g_1 + h_1 left in OPEN.  Every label that could
                              still reach the goal has F_1 >= that bound (h is a
                              lower bound of the remaining cost), so these entries are
                              exactly the final front's entries in that range.  For
                              mos_solve and mos_server_poll the result is written to
                              *out with this status; mos_solve_batch reports it per
                              query. */
  int32_t pop_order;        /* MOS_POP_LEXICOGRAPHIC (0, default) or MOS_POP_GENERATION */
  int32_t epsilon_ppm;      /* 0 (default) = the exact front.  e > 0: approximate front
                              (Sections 2 and 8 name epsilon-dominance for trading
                              exactness for work): every test against the goal front
                              uses p <= (1 + eps) x with eps = e / 10^6, tests against a
                              node's own labels stay exact.  The result is a set of
                              real path costs (with their paths), mutually
                              non-dominated, and every exact front vector y has an
                              entry a with a <= (1 + eps) y in every component.  A goal
                              label that is strictly below a front entry is always kept
                              (it replaces that entry), so the factor does not compound.
                              0 .. 10^9. */
  int32_t eager_goal;       /* 0 (default): a label at the goal joins the goal front when
                              OPEN pops it (Algorithm 1).  1: it joins the goal front
                              in the next step's goal step, straight after the step
                              that accepted it, without waiting for its turn in OPEN;
                              the front then prunes the search sooner.  The result is
                              the same front. */
  int32_t pipelined;        /* 0 (default): each step ends with the goal-front filter of
                              the labels it inserted.  1: that filter runs at the start
                              of the next step, on a second stream beside the next
                              step's pop, so the extraction of the next batch overlaps
                              the current batch's last stage (the current/next bags of
                              Section 5.1, Algorithm 2).  A label the filter has not yet
                              removed when it is popped is dropped by the pop-time
                              goal-front check instead.  The result is the same front;
                              with a step budget, the prefix is still exact.  The
                              engine of a batch or server call runs all its queries in
                              the mode of that call. */
  int32_t persistent_query; /* 0 (default): every step of every resident query is the
                              fixed sequence of grid-wide kernels.  1 (mos_solve,
                              mos_solve_batch, the server): each query runs its steps
                              inside one workgroup of its own, many steps per launch
                              with workgroup barriers between the phases of a step
                              (the batch is every OPEN label below an F1 bound; a
                              label reaching the goal joins the goal front at once).
                              For short queries, whose steps cannot fill the GPU.  The
                              result is the same front; the witness path of a front
                              vector reached by several equal-cost paths may differ
                              from mode 0's.  Ignored (mode 0) with a step budget, the
                              generation order, epsilon_ppm > 0 or a graph with an
                              out-degree above 1024; a query with one node holding
                              more labels of the smallest F1 than one batch is moved
                              to mode 0 and run again.  Slower than mode 0 on every
                              workload measured (one compute unit per query). */
} mos_options;

/* Counters of one query (paper, Section 6: label extractions, candidate
 * labels explored, solutions found; plus the dominance-check work).  A
 * "pair" is one (candidate vector, stored vector) comparison the method has to
 * make: against the goal front P, against another candidate of the same step
 * and target node, or against a live label of the target node's frontier. */
typedef struct {
  int64_t pops;            /* labels taken from OPEN and processed (expanded or merged
                              into the goal front) */
  int64_t goal_pops;       /* of which at the goal */
  int64_t candidates;      /* arcs expanded (candidate labels generated) */
  int64_t p_pairs;         /* candidate x goal-front pairs */
  int64_t group_pairs;     /* candidate x same-group candidate pairs */
  int64_t frontier_pairs;  /* candidate x frontier-label pairs */
  int64_t inserted;        /* labels inserted (incl. the start label) */
  int64_t pruned;          /* frontier labels removed by a dominating candidate */
  int64_t steps;           /* batched label steps run */
  int64_t front;           /* size of the returned front */
  int64_t frontier_bytes;  /* algorithmic bytes of frontier reads: 4*d per frontier pair-row */
  int64_t killed;          /* labels dropped when popped: the goal front dominates their F
                              (the paper's PruneOPEN, applied lazily) */
  int64_t frontier_bytes_onepass; /* part of frontier_bytes from groups checked by one
                                     wave in a single pass */
  int64_t pairs_onepass;   /* frontier + same-group pairs of those groups */
  int64_t near_scanned;    /* OPEN entries (near tier) scanned to select the batches */
  int64_t far_scanned;     /* OPEN entries (far tier) scanned to refill the near tier */
  int64_t tie_entries;     /* entries of the threshold F1 value ordered by full key */
  int64_t front_reads;     /* goal-front entries read by the goal-front updates */
  double search_ms;        /* device time of the label steps */
  double heuristic_ms;     /* device time of the heuristic (reverse SSSP) */
  int64_t open_min_f1;     /* INT32_MAX for a complete front; for a step-limited or
                              so-far result, the bound below which its first objective
                              makes the entries final (see step_budget) */
} mos_stats;

/* Graph: n_nodes nodes, n_arcs arcs in CSR form.  row_ptr[n_nodes+1] (int64,
 * non-decreasing, row_ptr[0] = 0, row_ptr[n] = n_arcs), col[n_arcs] (arc
 * targets), cost[n_arcs * D] arc-major (cost[e*D + k] = objective k of arc e),
 * 1 <= D <= MOS_MAX_OBJECTIVES.  Parallel arcs, self-loops and zero costs are
 * allowed.  Fails with MOS_E_NEGATIVE_COST for a negative cost and with
 * MOS_E_OVERFLOW_RISK when int32 sums could reach INT32_MAX (every accepted
 * label is a simple path, so g_k <= sum of c_k and F_k <= 2*sum + max; INT32_MAX
 * itself is kept free as a sentinel above every cost).  The arrays are
 * copied; the caller keeps ownership.  The graph is immutable afterwards and
 * may be shared by several threads and streams. */
mos_status mos_graph_create(int32_t n_nodes, int64_t n_arcs, int32_t D, const int64_t* row_ptr,
                            const int32_t* col, const int32_t* cost, mos_graph** out);
void mos_graph_destroy(mos_graph* g);

/* Exact front for one start/goal pair.  An unreachable goal gives MOS_OK with
 * an empty front; start == goal gives the single all-zero vector and an empty
 * path.  On success *out owns the result. */
mos_status mos_solve(const mos_graph* g, int32_t start, int32_t goal, const mos_options* opt,
                     mos_result** out);

/* nq queries solved together: queries are admitted into device-resident slots
 * as memory allows and all resident queries advance in the same fused step
 * launches.  n_objectives may be NULL (then opt->n_objectives applies to all).
 * out[i] and st[i] receive each query's result and status; a query's result
 * (paths included) does not depend on the other queries.  Returns MOS_OK if
 * every query succeeded, else the first failing status. */
mos_status mos_solve_batch(const mos_graph* g, int32_t nq, const int32_t* starts,
                           const int32_t* goals, const int32_t* n_objectives,
                           const mos_options* opt, mos_result** out, mos_status* st);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops or harnesses that forbid hipMalloc): mos_solve with costs only,
 * no device allocation and no allocating library call.  All device state comes
 * from one library-owned array of 256 MiB per GPU (made when the library is
 * loaded, held until the process ends), so the query's search state -- per-node
 * arrays of the whole graph plus its labels -- must fit into it:
 * MOS_E_INVALID_ARG names a graph whose per-node state alone does not fit,
 * MOS_E_LABEL_LIMIT a search that outgrows the rest.  costs is HOST memory of
 * cap * d int32 (d = the query's objective count); on MOS_OK it receives the
 * front, lexicographically ascending, and *size its entry count; a front larger
 * than cap gives MOS_E_INVALID_ARG (nothing written).  stats may be NULL.
 * Options as for mos_solve (costs_only, profile_kernels and max_slots are
 * ignored; mem_budget does not apply); the steps run on opt->stream (NULL = the
 * null stream), kernels launched one by one.  Calls on one GPU share its array
 * and would race: the library serialises them per device; the array's contents
 * do not carry from one call to the next. */
mos_status mos_solve_noalloc(const mos_graph* g, int32_t start, int32_t goal,
                             const mos_options* opt, int32_t* costs, int64_t cap, int64_t* size,
                             mos_stats* stats);

int64_t mos_result_size(const mos_result* r); /* number of front entries (0 for NULL) */
int32_t mos_result_dim(const mos_result* r);  /* d (0 for NULL) */
/* out[size*d]: the front, lexicographically ascending. */
mos_status mos_result_costs(const mos_result* r, int32_t* out);
/* Arc ids of the witness path of entry i.  *len receives the length; at most
 * cap ids are written to arcs (arcs may be NULL when cap == 0). */
mos_status mos_result_path(const mos_result* r, int64_t i, int32_t* arcs, int64_t cap,
                           int64_t* len);
mos_status mos_result_stats(const mos_result* r, mos_stats* out);
void mos_result_destroy(mos_result* r);

/* Device memory hooks (e.g. a framework's caching allocator).  alloc returns
 * device memory of at least the given size or NULL; release frees it.  Pass
 * NULL functions to restore hipMalloc/hipFree.  Affects later allocations. */
mos_status mos_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                             void (*release)(void* ptr, void* ctx), void* ctx);

/* Continuous-batching server over one graph.  Requests are queued by
 * mos_server_submit and admitted into free slots when their search-state
 * reservation fits into mem_budget_bytes; admitted queries share every step
 * launch with the queries already on the device, and finished ones leave at
 * once.  A query that outgrows its reservation is re-admitted alone with a
 * larger one (or fails with MOS_E_LABEL_LIMIT); other queries are unaffected. */
mos_status mos_server_create(const mos_graph* g, int64_t mem_budget_bytes, int32_t max_slots,
                             mos_server** out);
/* The same with solve options applied to every served query: batch_width,
 * steps_per_poll, label_limit, costs_only, heuristic_radius and step_budget
 * (n_objectives is per request; other fields are ignored).  NULL = defaults. */
mos_status mos_server_create_ex(const mos_graph* g, int64_t mem_budget_bytes, int32_t max_slots,
                                const mos_options* opt, mos_server** out);
mos_status mos_server_submit(mos_server* s, int32_t start, int32_t goal, int32_t n_objectives,
                             uint64_t* ticket);
/* MOS_E_NOT_READY until the query is done; then MOS_OK and *out (owned by the
 * caller), or the query's error (MOS_E_STEP_LIMIT also writes *out: the exact
 * prefix).  A ticket can be collected once. */
mos_status mos_server_poll(mos_server* s, uint64_t ticket, mos_result** out);
/* Blocks until the ticket is done (or timeout_ms elapses: MOS_E_NOT_READY;
 * timeout_ms < 0 waits without limit).  If the server's loop stops on a device
 * error, every query it has not finished is reported with that error: wait
 * and poll then return it instead of MOS_E_NOT_READY, and submit fails. */
mos_status mos_server_wait(mos_server* s, uint64_t ticket, int64_t timeout_ms, mos_result** out);
mos_status mos_server_cancel(mos_server* s, uint64_t ticket);
/* Server counters: [0] submitted, [1] finished, [2] resident now, [3] queued now,
 * [4] ticks run, [5] re-admissions after overflow. */
mos_status mos_server_counters(mos_server* s, int64_t* out6);
void mos_server_destroy(mos_server* s);

/* Single-query session: the query's label state stays resident on the device
 * and the caller advances the search a number of batched label steps at a time
 * (the same steps mos_solve runs).  mos_session_create computes the heuristic
 * and seeds the start label; mos_session_step runs up to nsteps steps and sets
 * *done to 1 once OPEN is empty (steps after that do nothing);
 * mos_session_stats reports the counters so far (a partial search: the front
 * size is that of the goal front so far); mos_session_result runs the search
 * to completion and returns the exact front (MOS_E_LABEL_LIMIT if the
 * reservation is outgrown).  Kernel times are kept when
 * options.profile_kernels has bit i set: entry i of mos_session_kernel_times gives the
 * kernel's name, its summed duration in ms and its launch count; i ranges
 * over 0 .. mos_session_kernel_count()-1. */
typedef struct mos_session mos_session;
mos_status mos_session_create(const mos_graph* g, int32_t start, int32_t goal,
                              const mos_options* opt, mos_session** out);
mos_status mos_session_step(mos_session* s, int64_t nsteps, int32_t* done);
mos_status mos_session_stats(const mos_session* s, mos_stats* out);
mos_status mos_session_result(mos_session* s, mos_result** out);
/* The goal front found so far (sorted, with witness paths unless costs_only)
 * without ending the search, and in *open_min_f1 the smallest first objective
 * F_1 = g_1 + h_1 over the labels still in OPEN (INT32_MAX when OPEN is empty).
 * With OPEN processed in lexicographic order and a consistent heuristic (the
 * exact per-objective distance, Section 4), every label that could still
 * reach the goal has F_1 >= *open_min_f1, so the entries whose first
 * objective is below it are exactly the final front's entries in that range:
 * a prefix of the exact answer, available long before the search ends. */
mos_status mos_session_front(mos_session* s, int32_t* open_min_f1, mos_result** out);
int32_t mos_session_kernel_count(void);
/* Change which kernels are timed from the next step on (same mask as
 * options.profile_kernels; 0 = none, steps then replay a captured graph). */
mos_status mos_session_set_profile(mos_session* s, int32_t mask);
mos_status mos_session_kernel_times(const mos_session* s, int32_t i, const char** name, double* ms,
                                    int64_t* launches);
/* How the session's steps were launched so far: *graph_replays replays of a
 * captured graph of *steps_per_replay steps each (the form mos_solve uses),
 * and *direct_steps steps whose kernels were launched one by one (profile mode
 * and remainders). */
mos_status mos_session_launch_counts(const mos_session* s, int64_t* graph_replays,
                                     int64_t* steps_per_replay, int64_t* direct_steps);
void mos_session_destroy(mos_session* s);

const char* mos_status_string(mos_status s);
const char* mos_last_error(void);

/* Heuristic only (the search's prerequisite step): h[k*n + v] = shortest
 * v -> goal distance under objective k for k < n_objectives (0 = D), or
 * INT32_MAX when the goal cannot be reached from v.  h is host memory of
 * n_objectives * n_nodes int32. */
mos_status mos_heuristic(const mos_graph* g, int32_t goal, int32_t n_objectives, int32_t* h);

#ifdef __cplusplus
}
#endif
#endif /* MOS_H_ */
