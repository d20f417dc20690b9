/*
 * wcdl.h -- C ABI of the worst-case-optimal Datalog engine for AMD MI355X.
 *
 * The engine evaluates Datalog programs (Horn clauses, paper Sec. 2
 * "Datalog"; stratified negation, Tab. 1) to their least fixpoint, stratum
 * by stratum, by semi-naive evaluation (Sec. 2, the
 * differential form of the fixpoint), running every multi-way rule body as a
 * worst-case-optimal join over flat, sorted, columnar uint32 relations
 * (Sec. 2 "Join Processing", Sec. 4).  Each iteration follows the staged
 * pipeline of Sec. 4: Histogram, Count, Scan/allocate, Materialize, Compute
 * Delta, Build Index, Merge; work is balanced by the root-level histogram of
 * Sec. 5 (Alg. 1 and Alg. 2).  All of it runs in HIP kernels on one GPU.
 *
 * Calls follow the paper's statement of the problem: declare relations with
 * their arity, load input facts as columns, register rules, run to the
 * fixpoint, read back derived relations.
 *
 * Conventions (every entry point):
 *  - Return a wcdl_status: 0 on success, a negative WCDL_E_* code on error.
 *    No C++ exception crosses this boundary.  After an error,
 *    wcdl_last_error() returns a human-readable message, and the engine is
 *    still valid unless the code is WCDL_E_DEVICE.
 *  - One engine is used by one host thread at a time.
 *  - Calls are synchronous: when a call returns, the device work it issued
 *    has completed and caller buffers passed to it may be reused.
 *  - Values are uint32; every uint32 value is a valid datum (no sentinel).
 *    Comparisons in rules are unsigned 32-bit.
 *  - Row counts, sizes and offsets are uint64.
 *  - Relations are sets: loading deduplicates silently; results are always
 *    returned sorted lexicographically by column 0, 1, ..., arity-1, with no
 *    duplicate rows.
 */
#ifndef WCDL_H
#define WCDL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wcdl_status;

#define WCDL_OK 0
#define WCDL_E_INVALID (-1)       /* null pointer, bad size, bad flag */
#define WCDL_E_ARITY (-2)         /* atom arity differs from the declaration */
#define WCDL_E_UNKNOWN_REL (-3)   /* relation id or name not declared */
#define WCDL_E_UNSAFE_RULE (-4)   /* head/comparison variable not bound by a body atom */
#define WCDL_E_UNSUPPORTED (-5)   /* exceeds the engine's static limits below */
#define WCDL_E_STATE (-6)         /* call not allowed in the current state */
#define WCDL_E_NOMEM (-7)         /* device allocation failed */
#define WCDL_E_BUDGET (-8)        /* a count-pass bound exceeded mem_budget_bytes */
#define WCDL_E_DEVICE (-9)        /* HIP runtime error; the engine must be destroyed */
#define WCDL_E_PARSE (-10)        /* rule text does not parse */
#define WCDL_E_CHECK (-11)        /* checked mode (WCDL_F_CHECKED): a relation
                                     invariant failed; the engine must be destroyed */

/* Static limits of one rule (after the planner's rewrites). */
#define WCDL_MAX_ARITY 6
#define WCDL_MAX_BODY 8
#define WCDL_MAX_VARS 8
#define WCDL_MAX_CMPS 8
#define WCDL_MAX_NEG 4

/* Configuration flags (wcdl_config.flags). */
#define WCDL_F_BALANCE_OFF 0x1u  /* one root key per workgroup instead of the
                                    histogram-balanced split of [0,T) (the
                                    ablation baseline of Sec. 7.3) */
#define WCDL_F_STREAMS_OFF 0x2u  /* evaluate rule versions one after another on
                                    one stream (the sequential schedule of
                                    Sec. 7.4) instead of phase-aligned on
                                    several streams (Sec. 6) */
#define WCDL_F_XPROD_OFF 0x4u    /* disable the per-unit decode fast path for
                                    cross-product plans (Sec. 5, work-unit
                                    decode); use the general kernel instead */
#define WCDL_F_STAGE_OFF 0x8u    /* never stage rows during the count pass: the
                                    write pass always re-runs the traversal */
#define WCDL_F_HEAD_BODY_OFF 0x20u /* merge every round's delta straight into the
                                    full relation instead of into a small head
                                    run that is flushed into the body past a
                                    size ratio (Sec. 4, Merge) */
#define WCDL_F_RUN_BITMAPS_OFF 0x40u /* never build run bitmaps: leaf probes always
                                    search (bitmaps answer probes into runs of
                                    >= 512 rows of copies a batch does not write) */
#define WCDL_F_GROUPED_SORT_OFF 0x80u /* sort every head chunk with the radix sort,
                                    also where the join already emits it in order
                                    of all but its last column (Sec. 4, Compute
                                    Delta: the grouped sort orders and dedups
                                    such chunks one LDS tile of groups at a time) */
#define WCDL_F_TILE_DEDUP_OFF 0x800u /* sort large unordered candidate sets with
                                    the radix passes directly, without first
                                    dropping rows repeated inside tiles of
                                    2,048 consecutive rows (Sec. 4, Compute
                                    Delta) */
#define WCDL_F_CHECKED 0x200u    /* checked mode: after every merge the engine
                                    verifies on the device that each stored copy
                                    of the relation is sorted without repeats and
                                    that the delta held no row the relation
                                    already had (Sec. 2: deltas are the new facts
                                    of a round); a failure is WCDL_E_CHECK.
                                    Costs one pass over the relation per merge. */
#define WCDL_F_COST_PLANNER 0x400u /* choose each rule version's variable order
                                    by a cost model over per-column distinct
                                    counts of the body relations (the paper's
                                    future work on variable orders, Sec. 9):
                                    the structural heuristic's order (most
                                    shared variable first, delta-first) is
                                    replaced where the model predicts a lower
                                    total with under a quarter of its join
                                    work, and a join without a
                                    delta is rooted at its most selective
                                    source; rules with a user order, batched
                                    engines and serving keep theirs */
#define WCDL_F_BATCHED 0x10u     /* batched mode: the engine holds many independent
                                    instances of one program.  Every relation gets
                                    an implicit leading column, the instance id:
                                    wcdl_load_columns / wcdl_read_columns take and
                                    return arity + 1 columns, column 0 holding the
                                    instance id, and every rule is evaluated within
                                    each instance (an instance variable is added to
                                    its head and to every body atom).  One run
                                    evaluates all instances together.  Declared
                                    arities are then limited to WCDL_MAX_ARITY - 1
                                    and rules to WCDL_MAX_VARS - 1 variables. */

typedef struct wcdl_engine wcdl_engine;

/* Device memory provider.  alloc returns device memory of at least `bytes`
 * bytes usable on `stream` (a hipStream_t), or NULL on failure; free releases
 * a pointer that alloc returned, with the same byte count.  The engine
 * caches blocks it frees and returns them all at wcdl_destroy.  When alloc is
 * NULL the engine uses hipMalloc/hipFree. */
typedef struct {
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, size_t bytes, void* stream);
  void* ctx;
} wcdl_allocator;

typedef struct {
  int32_t device;            /* HIP device ordinal */
  uint32_t n_streams;        /* number of entries in `streams`; 0 = engine creates 4 */
  void* const* streams;      /* hipStream_t handles owned by the caller; stream 0 is
                                the main stream (all default priority) */
  wcdl_allocator alloc;      /* see above */
  uint64_t mem_budget_bytes; /* 0 = unlimited.  Otherwise a bound on the device
                                memory held by the relations (every stored copy:
                                loaded facts, the full relation, its other column
                                orders, deltas; rows x stored arity x 4 bytes)
                                together with one round's candidate rows.  After
                                a round's count pass (Alg. 1 Phase 2), if the
                                rows it counted (x head arity x 4 bytes, before
                                deduplication) do not fit beside the relations
                                within the bound, the run fails with
                                WCDL_E_BUDGET before anything of that round is
                                written: the relations keep the last completed
                                round and the engine stays usable.  The count
                                kernels stop as soon as the rows found so far
                                cross the bound, so a round far over it fails
                                quickly.  The count
                                pass's staging arena is also held within the
                                bound.  Kernel scratch (sort buffers, histograms,
                                root keys) is not counted. */
  uint32_t flags;            /* WCDL_F_* */
  uint32_t wg_per_cu;        /* work-partition oversubscription: p = 256 CUs x
                                wg_per_cu workgroups per join; 0 = default (32) */
  uint32_t stage_pct;        /* count-pass staging arena, in percent of the rows
                                a rule version produced per work unit last time
                                (0 = default 125).  Rows that do not fit are
                                recomputed by the write pass. */
  uint64_t instance_cap_bytes; /* serving (batched engines): 0 = none.  Else an
                                instance whose rows counted by one step's count
                                passes take more than this many bytes (rows x
                                stored head arity x 4) is rejected before the
                                step writes anything: its rows are dropped from
                                every relation and it is listed by
                                wcdl_serve_rejected (the per-request form of
                                WCDL_E_BUDGET). */
  uint64_t chunk_bytes;      /* candidate rows of one head relation written at
                                once (Alg. 1 Phase 3): larger outputs are written
                                in ranges of workgroups, each range deduplicated
                                and subtracted before the next is written (0 =
                                6 % of device memory).  Fails with WCDL_E_BUDGET
                                if one work unit alone produces more. */
  uint32_t head_ratio;       /* a relation's head run (Sec. 4, Merge) is merged
                                into its body once it holds more than
                                1/head_ratio of the body's rows (and 65,536
                                rows); 0 = default 8 */
  uint32_t bitmap_min_run;   /* shortest run (rows sharing all but the last
                                column) that gets a run bitmap for leaf probes;
                                0 = default 512, smaller values act as 512 */
} wcdl_config;

/* Fill `cfg` with defaults (device 0, own streams, hipMalloc, no budget). */
void wcdl_config_default(wcdl_config* cfg);

/* Create an engine on cfg->device.  *out receives the engine. */
wcdl_status wcdl_create(const wcdl_config* cfg, wcdl_engine** out);

/* Destroy an engine and free every device buffer it holds.  NULL is a no-op. */
void wcdl_destroy(wcdl_engine* e);

/* Message describing the last error on this engine (never NULL; "" if none).
 * Valid until the next call on the engine. */
const char* wcdl_last_error(const wcdl_engine* e);

/* Declare a relation (paper Sec. 2: input and derived relations are both
 * just relations).  name: [A-Za-z_][A-Za-z0-9_]*, unique; 1 <= arity <=
 * WCDL_MAX_ARITY.  *rel_id receives its id (dense, from 0). */
wcdl_status wcdl_declare_relation(wcdl_engine* e, const char* name, uint32_t arity,
                                  uint32_t* rel_id);

/* Look up a relation id by name. */
wcdl_status wcdl_relation_id(const wcdl_engine* e, const char* name, uint32_t* rel_id);

/* Add input facts to a relation (Sec. 4: relations are flat structure-of-
 * arrays columns).  cols[j] points to n_rows uint32 values of column j,
 * j < arity; on_device != 0 means the pointers are device memory on the
 * engine's device, else host memory.  The engine copies the data (the caller
 * keeps ownership) and merges it with facts loaded before; duplicates are
 * dropped.  Facts may be loaded into relations that rules also derive; they
 * join the first delta of their stratum.  Allowed before and between runs. */
wcdl_status wcdl_load_columns(wcdl_engine* e, uint32_t rel, const uint32_t* const* cols,
                              uint64_t n_rows, int on_device);

/* Remove every loaded fact of a relation (derived facts are recomputed by
 * the next run). */
wcdl_status wcdl_clear_relation(wcdl_engine* e, uint32_t rel);

/* ---- Rules as data ---------------------------------------------------- */

#define WCDL_VAR 0u
#define WCDL_CONST 1u
typedef struct {
  uint32_t kind;  /* WCDL_VAR: value is a variable id local to the rule;
                     WCDL_CONST: value is the constant */
  uint32_t value;
} wcdl_term;

typedef struct {
  uint32_t rel;
  uint32_t arity;
  const wcdl_term* terms;
} wcdl_atom;

#define WCDL_LT 0u /* lhs <  rhs */
#define WCDL_LE 1u /* lhs <= rhs */
#define WCDL_NE 2u /* lhs != rhs */
#define WCDL_GT 3u /* lhs >  rhs */
#define WCDL_GE 4u /* lhs >= rhs */
typedef struct {
  uint32_t op;
  wcdl_term lhs;
  wcdl_term rhs;
} wcdl_cmp;

/* Head(...) <- Body_1(...), ..., Body_n(...), comparisons, not Neg_1(...),
 * ..., not Neg_k(...) (Sec. 2; negation as in Tab. 1, stratified).  Every
 * head, comparison and negated-atom variable must occur in a (positive) body
 * atom (safety).  A negated atom's relation must not depend on the head's
 * relation (the program stays stratifiable); a binding of the body yields
 * the head only if no negated atom's tuple is in its relation, which is
 * complete when the rule runs (it belongs to a lower stratum).
 * var_order, if not NULL, fixes the join's variable order (n_vars entries,
 * each body variable exactly once); NULL lets the planner choose (delta
 * relation outermost, Sec. 7.3). */
typedef struct {
  wcdl_atom head;
  uint32_t n_body;
  const wcdl_atom* body;
  uint32_t n_cmp;
  const wcdl_cmp* cmp;
  uint32_t n_vars;
  const uint32_t* var_order;
  uint32_t n_neg;            /* negated atoms (at most WCDL_MAX_NEG) */
  const wcdl_atom* neg;
} wcdl_rule;

/* Register one rule; *rule_id receives its id.  Rejected with
 * WCDL_E_UNSAFE_RULE, WCDL_E_ARITY, WCDL_E_UNKNOWN_REL or
 * WCDL_E_UNSUPPORTED (limits above, or a negated atom whose relation
 * depends on the head's: the program would not be stratifiable). */
wcdl_status wcdl_add_rule(wcdl_engine* e, const wcdl_rule* rule, uint32_t* rule_id);

/* Register rules from text, e.g.
 *   "path(x,y) :- edge(x,y).  path(x,z) :- path(x,y), edge(y,z), x != z."
 * Identifiers in argument position are variables ("_" is anonymous),
 * decimal numbers are constants, comparisons are < <= > >= !=, a body item
 * "!rel(...)" is a negated atom, and '%' or
 * '//' starts a comment.  Relations must be declared first.  A ground clause
 * without a body adds a fact.  All-or-nothing: on error no rule is added. */
wcdl_status wcdl_add_rules_text(wcdl_engine* e, const char* text);

/* Number of registered rules (helper rules from wcdl_split_rule included). */
wcdl_status wcdl_rule_count(const wcdl_engine* e, uint32_t* n);

/* Helper-relation splitting (Sec. 5, the CallGraphEdge rewrite): factor the
 * body atoms atom_idx[0..n) of rule rule_id into a relation whose columns
 * are the variables those atoms share with the rest of the rule (other
 * atoms, head, comparisons), in order of first occurrence.  The rule becomes
 * head <- remaining atoms, helper(shared...) and a rule
 * helper(shared...) <- selected atoms is added, carrying the orders among
 * its columns that the rule's comparisons imply.  Indices refer to the body
 * as the rule was registered; a later split of the same rule may select
 * atoms that an earlier one already moved into a helper (a conjunction may
 * repeat atoms), but not only such atoms.  A helper whose definition equals
 * an earlier helper's up to variable names is that relation again, with no
 * new rule.  The least model of every previously declared relation is
 * unchanged.  *helper_rel receives the helper's relation id (new ones are
 * named "<head>__h<k>"). */
wcdl_status wcdl_split_rule(wcdl_engine* e, uint32_t rule_id, const uint32_t* atom_idx,
                            uint32_t n, uint32_t* helper_rel);

/* Binary-join plan, for comparison with the worst-case optimal plans (Sec.
 * 7.2, Tab. 3: a conventional engine evaluates a body of three or more atoms
 * as a chain of two-way joins and materialises each intermediate relation
 * every iteration).  Every rule with three or more body atoms becomes a
 * left-deep chain: atoms 0..k-2 are factored into a helper relation
 * (wcdl_split_rule), whose own rule is split the same way until every body
 * has at most two atoms.  The least model of every declared relation is
 * unchanged; helpers hold the intermediate results as relations of their
 * own.  Call before any wcdl_split_rule (else WCDL_E_STATE) and not while
 * serving.  All or nothing: on error no rule changes.  *n_helpers (may be
 * NULL) receives the number of helper relations made. */
wcdl_status wcdl_binary_plan(wcdl_engine* e, uint32_t* n_helpers);

/* ---- Evaluation ------------------------------------------------------- */

/* Phase indices of wcdl_run_stats.phase_ms (device time, summed over rounds). */
#define WCDL_PH_HISTOGRAM 0   /* root-key histogram and its prefix sum (Alg. 1 Ph. 1) */
#define WCDL_PH_COUNT 1       /* count kernels + offset scan (Alg. 1 Ph. 2) */
#define WCDL_PH_MATERIALIZE 2 /* materialize kernels (Alg. 1 Ph. 3) */
#define WCDL_PH_DELTA 3       /* sort, dedup, difference against the full relation */
#define WCDL_PH_INDEX 4       /* sorting the delta into extra column orders */
#define WCDL_PH_MERGE 5       /* merging the delta into the full relations */
#define WCDL_PH_LOAD 6        /* input sorting and index building at run start */
#define WCDL_PH_OTHER 7
#define WCDL_N_PHASES 8

typedef struct {
  uint64_t rounds;           /* semi-naive rounds over all recursive strata,
                                each stratum's last (empty) round included */
  uint64_t derived_rows;     /* sum of the final sizes of every relation that
                                is the head of some rule */
  uint64_t candidate_rows;   /* rows written by materialize kernels (before
                                dedup), summed over the run */
  uint64_t join_units;       /* sum of T (histogram work units) over all joins */
  double wall_ms;            /* host wall time of the run */
  double phase_ms[WCDL_N_PHASES];
  /* Device time of the join kernels, from HIP events recorded around each
   * launch on the stream that runs it: [0] count (Alg. 1 Phase 2),
   * [1] materialize (Phase 3, including the cross-product decode path),
   * [2] histogram (Phase 1). */
  double kernel_ms[4];
  uint64_t kernel_launches[4];
  uint64_t candidates_checked; /* candidate values tested by materialize
                                  kernels (one per element of the smallest
                                  list of every intersection) */
  uint64_t candidates_per_level[WCDL_MAX_VARS]; /* the same, by join level
                                  (level 0 = root keys), summed over rules */
} wcdl_run_stats;

/* Evaluate every stratum to its fixpoint (Sec. 2 stratification; the loop of
 * Sec. 4 stops when the deduplicated delta is empty).  Derived relations are
 * recomputed from the loaded facts on every call.  stats may be NULL.  On
 * WCDL_E_BUDGET (see wcdl_config.mem_budget_bytes) the relations hold the
 * state after the last completed round of the stratum that failed (earlier
 * strata complete, later ones as loaded), reads return that state, and the
 * engine stays usable: a later run recomputes from the loaded facts. */
wcdl_status wcdl_run(wcdl_engine* e, wcdl_run_stats* stats);

/* Rows currently held by a relation (after wcdl_run: its least-model size). */
wcdl_status wcdl_relation_size(const wcdl_engine* e, uint32_t rel, uint64_t* n_rows);

/* Copy a relation out, sorted and deduplicated.  cols_out[j] receives column
 * j (capacity uint32 values each); on_device selects device or host
 * destination pointers.  *n_written receives the number of rows copied
 * (min(size, capacity)); use wcdl_relation_size first. */
wcdl_status wcdl_read_columns(const wcdl_engine* e, uint32_t rel, uint32_t* const* cols_out,
                              uint64_t capacity, uint64_t* n_written, int on_device);

/* Rows of a relation whose column 0 equals `lead` (in batched mode: the rows
 * of one instance): they are the contiguous rows [*first, *first + *count)
 * of the sorted relation. */
wcdl_status wcdl_relation_range(const wcdl_engine* e, uint32_t rel, uint32_t lead,
                                uint64_t* first, uint64_t* count);

/* Copy rows [first, first + n) of the sorted relation (all stored columns,
 * the instance column included in batched mode) into cols_out[j] (n values
 * each; device or host pointers as on_device says).  Fails with
 * WCDL_E_INVALID if the range exceeds the relation. */
wcdl_status wcdl_read_rows(const wcdl_engine* e, uint32_t rel, uint64_t first, uint64_t n,
                           uint32_t* const* cols_out, int on_device);

/* Autotuner: run the program once per candidate work-partition granularity
 * (workgroups per CU, see wcdl_config.wg_per_cu), keep the fastest for later
 * runs and report it in *chosen (and its run time in *best_ms).  The relations
 * hold the last candidate's (identical) results afterwards. */
wcdl_status wcdl_autotune(wcdl_engine* e, const uint32_t* wg_per_cu, uint32_t n, uint32_t* chosen,
                          double* best_ms);

/* Return the device blocks the engine keeps cached for reuse (freed
 * scratch) to the allocator, so that other engines or the caller can use
 * that memory; relations are untouched.  Waits for the engine's streams.
 * *released (may be NULL) receives the bytes returned. */
wcdl_status wcdl_trim(wcdl_engine* e, uint64_t* released);

/* Strategy flags the configuration tuner may set or clear. */
#define WCDL_TUNE_FLAGS (WCDL_F_STREAMS_OFF | WCDL_F_XPROD_OFF | WCDL_F_STAGE_OFF | \
                         WCDL_F_HEAD_BODY_OFF | WCDL_F_RUN_BITMAPS_OFF |            \
                         WCDL_F_GROUPED_SORT_OFF | WCDL_F_COST_PLANNER |           \
                         WCDL_F_TILE_DEDUP_OFF)

/* One configuration for wcdl_autotune_points: the partition granularity, the
 * count-pass staging arena size (0 = default), the strategy flags (only bits
 * of WCDL_TUNE_FLAGS; the engine's other flags are kept), the head-run flush
 * ratio and the run-bitmap threshold. */
typedef struct {
  uint32_t wg_per_cu;
  uint32_t stage_pct;
  uint32_t flags;
  uint32_t head_ratio;       /* as in wcdl_config (0 = default) */
  uint32_t bitmap_min_run;   /* as in wcdl_config (0 = default) */
} wcdl_tune_point;

/* Configuration tuner: run the program once per point, keep the fastest
 * point's settings for later runs, report its index in *chosen and its run
 * time in *best_ms.  Choices are remembered for the process, keyed by the
 * program (rules up to variable names) and the size bucket of its loaded
 * facts (floor of log2 of their row count): a later call with the same key
 * and the same points applies the remembered choice without running (then
 * *best_ms is the time measured when it was chosen).  The relations hold
 * the results of the last run (identical for every point).  Fails with
 * WCDL_E_INVALID on an empty list, a zero wg_per_cu or flags outside
 * WCDL_TUNE_FLAGS. */
wcdl_status wcdl_autotune_points(wcdl_engine* e, const wcdl_tune_point* points, uint32_t n,
                                 uint32_t* chosen, double* best_ms);

/* ---- Continuous evaluation (serving), batched engines only -------------
 *
 * Programs with negation cannot be served (WCDL_E_UNSUPPORTED).
 * A positive program's least model is also reached by one semi-naive loop
 * over all rules in which every relation, input relations included, has a
 * delta (Sec. 2's differential form; stratification is only an evaluation
 * order for positive programs).  Serving runs that loop one round per
 * wcdl_serve_step; facts admitted between steps are the next round's delta of
 * their relations, so new instances join while others are in flight and
 * share every launch with them (Sec. 6's monotonicity argument: the order in
 * which facts arrive does not change any instance's least model). */

typedef struct {
  uint64_t candidate_rows;  /* rows counted by this step's count passes */
  uint64_t new_rows;        /* rows new to the relations after this step */
  uint64_t resident_rows;   /* rows held by all relations after this step */
  double wall_ms;
  uint64_t bound_bytes;     /* bytes of the rows this step's count passes
                               counted (rows x head arity x 4): the memory
                               bound of the step (Alg. 1 Phase 2) */
  uint64_t resident_bytes;  /* bytes held by every stored copy of every
                               relation after the step */
  uint64_t rejected;        /* instances rejected by this step
                               (wcdl_config.instance_cap_bytes) */
  double phase_ms[WCDL_N_PHASES]; /* time of the step by phase, indexed by
                                    WCDL_PH_* as in wcdl_run_stats */
} wcdl_step_stats;

/* Start serving: relations keep their loaded facts, derived relations are
 * reset to them, every delta is empty.  Requires WCDL_F_BATCHED. */
wcdl_status wcdl_serve_begin(wcdl_engine* e);

/* Queue facts (arity + 1 columns, instance id first) for the next step. */
wcdl_status wcdl_serve_admit(wcdl_engine* e, uint32_t rel, const uint32_t* const* cols,
                             uint64_t n_rows, int on_device);

/* One round for every instance with work.  stats may be NULL. */
wcdl_status wcdl_serve_step(wcdl_engine* e, wcdl_step_stats* stats);

/* Instances that still have work (rows in some delta or admitted facts not yet
 * stepped), ascending; writes min(count, cap) ids, *count receives the total.
 * An admitted instance absent from this list has reached its fixpoint. */
wcdl_status wcdl_serve_live(wcdl_engine* e, uint32_t* ids, uint64_t cap, uint64_t* count);

/* wcdl_serve_live without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops): its
 * kernels work in a fixed static device array of about 4.5 MB per GPU, held
 * until the process ends.  Limits: instance ids below 2^22 (else
 * WCDL_E_UNSUPPORTED) and at most 2^20 live instances (else
 * WCDL_E_UNSUPPORTED; *count is not written).  Results equal
 * wcdl_serve_live's.  All engines on one GPU share the array: calls that
 * overlap on one GPU (from several host threads) race. */
wcdl_status wcdl_serve_live_static(wcdl_engine* e, uint32_t* ids, uint64_t cap, uint64_t* count);

/* Drop every row of the listed instances from every relation (frees their
 * memory).  ids need not be sorted. */
wcdl_status wcdl_serve_release(wcdl_engine* e, const uint32_t* ids, uint64_t n);

/* Instances rejected since serving began (instance_cap_bytes), ascending;
 * writes min(count, cap) ids, *count receives the total. */
wcdl_status wcdl_serve_rejected(wcdl_engine* e, uint32_t* ids, uint64_t cap, uint64_t* count);

/* Stop serving (relations keep their contents). */
wcdl_status wcdl_serve_end(wcdl_engine* e);

/* ---- Instances (batched engines) --------------------------------------
 *
 * An engine created with WCDL_F_BATCHED holds one compiled program; an
 * instance is one set of input facts of it, with its own least model.  Each
 * instance's rows carry its id in the leading column of every relation, so
 * many instances run in the same launches of every phase and never mix (the
 * instance variable occurs in every atom of every rule). */

typedef struct wcdl_instance wcdl_instance;

/* A new, empty instance; ids are handed out from 0 up. */
wcdl_status wcdl_instance_create(wcdl_engine* e, wcdl_instance** out);

/* The instance's id (the value of its leading column); 0xffffffff for NULL. */
uint32_t wcdl_instance_id(const wcdl_instance* in);

/* Add facts to the instance: cols[j] (j < declared arity) points to n_rows
 * values of column j, host or device memory as on_device says (the engine
 * copies them and prepends the instance column).  Outside serving they join
 * the loaded facts (wcdl_load_columns); while serving they are admitted for
 * the next step (wcdl_serve_admit). */
wcdl_status wcdl_instance_load(wcdl_instance* in, uint32_t rel, const uint32_t* const* cols,
                               uint64_t n_rows, int on_device);

/* Rows the relation holds for this instance. */
wcdl_status wcdl_instance_size(const wcdl_instance* in, uint32_t rel, uint64_t* n_rows);

/* Copy this instance's rows of a relation out, sorted and deduplicated,
 * without the instance column: cols_out[j] (j < declared arity) receives
 * min(size, capacity) values. */
wcdl_status wcdl_instance_read(const wcdl_instance* in, uint32_t rel, uint32_t* const* cols_out,
                               uint64_t capacity, uint64_t* n_written, int on_device);

/* Drop every row of the instance from every relation and free the handle. */
void wcdl_instance_destroy(wcdl_instance* in);

/* Evaluate the program for the listed instances together (one run: every
 * phase of every round covers all of them at once).  Afterwards the derived
 * relations hold exactly these instances' least models (rows of other
 * instances are not derived; their loaded facts stay).  Not while serving. */
wcdl_status wcdl_run_batch(wcdl_engine* e, wcdl_instance* const* v, uint32_t n,
                           wcdl_run_stats* stats);

/* While serving: one semi-naive round for the listed instances (admitted
 * facts of theirs not yet known join the round's deltas first); the work of
 * every other instance waits for a later step.  done[i] (if not NULL)
 * receives 1 when active[i] has reached its fixpoint (no delta rows and no
 * admitted facts left).  *next_bound_bytes (if not NULL) receives the bytes
 * the relations hold after the step plus the bytes this step's count passes
 * counted: the memory bound of the next step for admission decisions. */
wcdl_status wcdl_step(wcdl_engine* e, wcdl_instance* const* active, uint32_t n, uint8_t* done,
                      uint64_t* next_bound_bytes);

/* Sizes of a relation's per-round deltas in its (recursive) stratum during
 * the last run: |delta_0|, |delta_1|, ..., ending with the empty one.
 * Writes min(count, cap) entries; *count receives the total. */
wcdl_status wcdl_delta_sizes(const wcdl_engine* e, uint32_t rel, uint64_t* out, uint64_t cap,
                             uint64_t* count);

/* ---- Host-side views of the work partition (Sec. 5, Alg. 2 and the
 * work-unit decode), exported so the partitioner can be checked without a
 * GPU; the kernels use the same functions. ------------------------------ */

/* Slice of workgroup b among p over T units: [*b_s, *b_e) with
 * b_s = b * ceil(T/p), b_e = min(b_s + ceil(T/p), T). */
void wcdl_work_slice(uint64_t T, uint64_t p, uint64_t b, uint64_t* b_s, uint64_t* b_e);

/* Owner of work unit g under the inclusive prefix sums C[0..K): the first
 * key k with C[k] > g (so key k owns [C[k-1], C[k]), C[-1] = 0). */
uint64_t wcdl_owner_key(const uint64_t* C, uint64_t K, uint64_t g);

/* Decode unit g of a two-level cross product into (key, i1, i2):
 * local = g - C[key-1], i1 = local / d2[key], i2 = local % d2[key]. */
void wcdl_decode_unit(const uint64_t* C, uint64_t K, const uint32_t* d2, uint64_t g,
                      uint64_t* key, uint64_t* i1, uint64_t* i2);

#ifdef __cplusplus
}
#endif

#endif /* WCDL_H */
