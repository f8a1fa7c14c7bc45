/*
 * fastlbp — loopy belief propagation on binary factor graphs with local-structure factors,
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: "FastLBP: GPU-Accelerated Belief Propagation for Program Analysis" (arXiv 2509.22337).
 *   - The factor graph and the messages are those of Section 3.1-3.2: variable-to-factor
 *     messages Eq.(1), factor-to-variable messages Eq.(2), marginals Eq.(3).
 *   - Factors have local structure (Section 3.3, Eq.(4)): every factor type below is evaluated in
 *     O(degree) instead of enumerating 2^degree assignments.
 *   - An update strategy is a preorder over the edges (Section 4.2.1, Definition 2), given here as
 *     an integer rank per edge: equal ranks form one class, lower ranks are updated first within
 *     an iteration. FLOODING is the all-parallel strategy (PARALL of Table 1), RANKED covers the
 *     fixed sequential order (SEQFIX: distinct ranks), topological orders (TOPO) and ordered
 *     groups. A dependency analysis (Algorithm 2, Section 4.2.3) splits the ranked strategy into
 *     levels that are updated in parallel (Theorem 2).
 *
 * Conventions
 *   Variables are binary. Factors are given in factor-major CSR: factor a owns edges
 *   [factor_offsets[a], factor_offsets[a+1]); the HEAD of a factor is its LAST edge and the edges
 *   before it are its inputs x_1..x_n.
 *   Factor types:
 *     FASTLBP_PRIOR     degree 1; f(1) = p, f(0) = 1-p with p = factor_params[a].
 *     FASTLBP_AND       degree >= 2; f = [y = x_1 & ... & x_n].
 *     FASTLBP_OR        degree >= 2; f = [y = x_1 | ... | x_n].
 *     FASTLBP_NOT       degree 2;    f = [y = !x_1].
 *     FASTLBP_IMPLIES   degree >= 2; probabilistic Horn rule p: x_1 & ... & x_n -> y (Section 1,
 *                       Section 2.2): f = p if all inputs are 1 and y = 1, 1-p if all inputs are 1
 *                       and y = 0, 1 otherwise. p = factor_params[a] (1 = hard implication;
 *                       factor_params == NULL means p = 1).
 *     FASTLBP_NOISY_OR  degree >= 2; P(y = 0 | x) = (1 - leak) * prod_{j: x_j = 1} (1 - p_j),
 *                       leak = factor_params[a] in [0,1), p_j = edge_params[e] of input edge e.
 *     FASTLBP_TERMS     degree 1..64, no head: a sum of 1..64 weighted terms (Section 3.3, Eq.(4)),
 *                       f(x) = sum_t w_t * prod_k [c_tk = -1 or x_k = c_tk], given to
 *                       fastlbp_graph_create_terms; messages as Eq.(4) (Algorithm 1's result).
 *   Readings where the paper is silent: messages start uniform; every stored message is
 *   normalised; a computed message whose two entries are both 0 is replaced by the uniform message
 *   and counted in fastlbp_run_stats.contradictions; damping mixes normalised old and new
 *   messages, stored = lambda*old + (1-lambda)*new; the residual of an iteration is the largest
 *   change of P(x=1) over the messages written in it; a run stops after the first iteration whose
 *   residual is below tol (tol = 0: run max_iters iterations).
 *
 * Ownership and threading
 *   The caller owns every input array; the library copies what it needs before returning, so the
 *   arrays may be freed afterwards. Output arrays are caller-allocated host memory. A graph handle
 *   is not thread-safe; distinct handles are independent. All device work of a handle runs on the
 *   stream given in fastlbp_options (or on a stream the library creates); calls that return host
 *   results synchronise that stream.
 *
 * Errors
 *   Every int-returning call returns FASTLBP_OK (0) or a negative FASTLBP_E_* code, and
 *   fastlbp_last_error() then describes the failure (thread-local, valid until the next call on
 *   the same thread). A failed call leaves the handle as it was. Non-convergence and
 *   contradictions are not errors; they are reported in fastlbp_run_stats.
 */
#ifndef FASTLBP_H
#define FASTLBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FASTLBP_OK = 0,
    FASTLBP_E_INVALID_ARG = -1, /* NULL pointer, bad enum value, bad size, bad damping/tol */
    FASTLBP_E_BAD_GRAPH = -2,   /* malformed CSR, variable id out of range, duplicate variable in a
                                   factor, wrong arity, parameter outside [0,1] or NaN */
    FASTLBP_E_BAD_SCHEDULE = -3,/* rank array missing for FASTLBP_SCHED_RANKED */
    FASTLBP_E_OOM = -4,         /* device allocation failed */
    FASTLBP_E_DEVICE = -5,      /* no usable gfx950 device, or a HIP call failed */
    FASTLBP_E_TOO_LARGE = -6,   /* graph exceeds a documented limit (edges >= 2^31, factor degree
                                   > FASTLBP_MAX_DEGREE) or a server's memory budget */
    FASTLBP_E_STATE = -7        /* call not valid in the handle's state (e.g. run before a schedule) */
};

enum { FASTLBP_PRIOR = 0, FASTLBP_AND = 1, FASTLBP_OR = 2, FASTLBP_NOT = 3, FASTLBP_IMPLIES = 4,
       FASTLBP_NOISY_OR = 5, FASTLBP_TERMS = 6 };

/* Message precision. FP64: messages stored as float64 log-likelihood ratios, factor algebra in
 * linear float64. FP32: messages stored as float32 log-likelihood ratios and the factor algebra in
 * the float32 log domain; beliefs, the convergence residual and marginals stay float64. */
enum { FASTLBP_FP64 = 0, FASTLBP_FP32 = 1 };

enum { FASTLBP_SCHED_FLOODING = 0, FASTLBP_SCHED_RANKED = 1 };

/* Executor. LEVELS: one kernel launch per level and phase over the whole GPU (wide levels,
 * flooding). PERSISTENT: one workgroup runs every level and iteration of the run in a single
 * launch with workgroup barriers between phases (narrow levels, small graphs). HYBRID: LEVELS for
 * the wide levels, and each run of consecutive narrow levels in one single-workgroup launch per
 * iteration (schedules that mix a few wide levels with many narrow ones). AUTO picks by the width
 * of the levels. All give the same messages up to floating-point rounding order. */
enum { FASTLBP_EXEC_AUTO = 0, FASTLBP_EXEC_LEVELS = 1, FASTLBP_EXEC_PERSISTENT = 2, FASTLBP_EXEC_HYBRID = 3 };

#define FASTLBP_MAX_DEGREE 16385 /* largest factor degree (inputs + head) */
#define FASTLBP_MAX_TERM_DEGREE 64 /* largest degree of a TERMS factor */
#define FASTLBP_MAX_TERMS 64       /* most terms of one TERMS factor */

typedef struct fastlbp_options {
    int32_t precision;  /* FASTLBP_FP64 or FASTLBP_FP32 */
    int32_t device;     /* HIP device ordinal */
    void *stream;       /* hipStream_t to enqueue on; NULL = the library creates one */
    int32_t executor;   /* FASTLBP_EXEC_* */
    int32_t use_graph;  /* 1 = replay iterations from a captured hipGraph, 0 = plain launches */
    /* Optional device allocator (e.g. a framework's caching allocator). Both NULL = hipMalloc /
     * hipFree. alloc returns NULL on failure. */
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *alloc_ctx;
} fastlbp_options;

/* Fills *o with defaults: FP64, device 0, library stream, AUTO executor, graphs on, hipMalloc. */
void fastlbp_options_default(fastlbp_options *o);

typedef struct fastlbp_run_stats {
    int32_t iterations;          /* iterations executed by the last fastlbp_run */
    int32_t converged;           /* 1 if the last iteration's residual was below tol */
    double residual;             /* residual of the last iteration */
    int64_t contradictions;      /* messages replaced by uniform during the run */
    int32_t levels;              /* levels per iteration (dependency analysis) */
    int32_t executor;            /* FASTLBP_EXEC_LEVELS, _PERSISTENT or _HYBRID */
    double method_bytes_per_iter; /* bytes one iteration of the method moves at minimum, with s-byte
                                    * messages (s = 4 FP32, 8 FP64): per edge of every factor a level
                                    * touches 4 + 3s (its variable-major position, the f->v gathered
                                    * for Eq.(1), the v->f written and read back), per written edge s
                                    * (2s when damping or tol > 0 need the old value), s per NOISY_OR
                                    * activation and per term weight, 2 bits per term indicator.
                                    * Flooding: 4 + 5s per edge */
    double impl_bytes_per_iter;   /* bytes this implementation's kernels read and write per
                                    * iteration when every access goes to memory once: task records,
                                    * structure, parameters, float64 beliefs per factor edge, messages */
    double device_ms;            /* device time of the run, HIP events on the handle's stream */
    int64_t message_updates;     /* factor-to-variable updates performed (edges x iterations) */
    /* launch choices of the run (the library's defaults, or fastlbp_autotune's) */
    int32_t thread_max_degree;   /* factors of degree <= this ran one per thread */
    int32_t wave_max_degree;     /* then one per wavefront up to this degree, then one per workgroup */
    int32_t var_thread_max_degree; /* variables of degree <= this ran one per thread, else per wavefront */
    int32_t graph_iters;         /* iterations per hipGraph replay (LEVELS, HYBRID; 0 = the rule) */
    int32_t persistent_threads;  /* workgroup size of the persistent executor (0 = the rule) */
    int32_t tuned;               /* 1 if fastlbp_autotune set the handle's choices */
} fastlbp_run_stats;

typedef struct fastlbp_graph *fastlbp_graph_t;

/* ------------------------------------------------------------------------------------------ */
/* Graph (Section 3.1; the Initialization stage of Section 4.1)                                 */
/* ------------------------------------------------------------------------------------------ */

/* Creates a graph: validates the CSR, builds the variable-major transpose, folds PRIOR factors
 * into per-variable potentials, buckets factors by degree and uploads everything to the device.
 *   num_vars, num_factors  sizes (>= 0)
 *   factor_offsets [F+1]   non-decreasing, factor_offsets[0] = 0, E = factor_offsets[F] < 2^31
 *   edge_vars [E]          variable of each edge, in [0, num_vars), no variable twice per factor
 *   factor_types [F]       FASTLBP_PRIOR .. FASTLBP_NOISY_OR (TERMS: fastlbp_graph_create_terms)
 *   factor_params [F]      per type as above; may be NULL (PRIOR then defaults to 0.5, IMPLIES to 1)
 *   edge_params [E]        NOISY_OR activation of each input edge; may be NULL (then 1)
 * The schedule starts as FLOODING with uniform messages and no evidence.
 * Errors: E_INVALID_ARG, E_BAD_GRAPH, E_TOO_LARGE, E_OOM, E_DEVICE. */
int fastlbp_graph_create(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                         const int32_t *edge_vars, const uint8_t *factor_types, const double *factor_params,
                         const double *edge_params, const fastlbp_options *opts, fastlbp_graph_t *out);

/* As fastlbp_graph_create, with factors of type FASTLBP_TERMS (Section 3.3): a factor given as a
 * sum of weighted terms, each term fixing some of the factor's variables to a value and leaving
 * the others free (the indicator representation of Algorithm 1).
 *   term_offsets [F+1]     term range of each factor: non-decreasing, term_offsets[0] = 0; empty
 *                          for every factor that is not TERMS, 1..FASTLBP_MAX_TERMS for TERMS
 *   term_weights [T]       weight of each term, finite and >= 0 (T = term_offsets[F])
 *   term_indicators        for the terms of each factor in order, one int8 per edge of that factor
 *                          (term-major): 0 or 1 = the edge's variable is fixed to that value in the
 *                          term, -1 = wildcard; sum over factors of (terms x degree) entries
 * The three arrays may be NULL when no factor is TERMS. A TERMS factor has degree
 * 1..FASTLBP_MAX_TERM_DEGREE and no head: each edge receives Eq.(4). Errors: as
 * fastlbp_graph_create; E_TOO_LARGE for a TERMS factor beyond the limits. */
int fastlbp_graph_create_terms(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                               const int32_t *edge_vars, const uint8_t *factor_types, const double *factor_params,
                               const double *edge_params, const int64_t *term_offsets, const double *term_weights,
                               const int8_t *term_indicators, const fastlbp_options *opts, fastlbp_graph_t *out);

void fastlbp_graph_destroy(fastlbp_graph_t g);

/* Sizes and device memory of a handle. state_bytes: its own device state when resident (messages,
 * beliefs, potentials, marginals, run state; what a server's memory budget counts); structure_bytes
 * and plan_bytes: the graph structure and the current schedule's plan (shared with clones). */
typedef struct fastlbp_graph_info {
    int32_t num_vars, num_factors;
    int64_t num_edges;
    int32_t precision;
    int32_t resident;          /* 1 while the device state is allocated, 0 while evicted by a server */
    size_t state_bytes, structure_bytes, plan_bytes;
    int32_t levels;            /* levels of the current schedule */
    int32_t executed_levels;   /* levels holding non-PRIOR edges */
} fastlbp_graph_info;
int fastlbp_graph_get_info(fastlbp_graph_t g, fastlbp_graph_info *out);

/* Creates a second handle on the same graph: it shares the device structure and the current
 * schedule with `src` (no copy) and has its own messages (uniform), evidence (none) and stream.
 * Used to run many queries of one graph side by side (fastlbp_run_batch). A later
 * fastlbp_schedule_set on either handle gives that handle its own plan. The structure is freed
 * with the last handle that uses it. Errors: E_INVALID_ARG, E_OOM, E_DEVICE. */
int fastlbp_graph_clone(fastlbp_graph_t src, fastlbp_graph_t *out);

/* ------------------------------------------------------------------------------------------ */
/* Update strategy and dependency analysis (Section 4.2, Definition 2, Algorithm 2)             */
/* ------------------------------------------------------------------------------------------ */

/* Sets the update strategy. kind = FASTLBP_SCHED_FLOODING ignores edge_rank; RANKED requires
 * edge_rank [E] (any int32 values; equal ranks = one equivalence class of the preorder). Runs the
 * dependency analysis: edges are ordered by (rank, edge id); a rank class joins the current level
 * unless one of its edges has a neighbour of Definition 1 in that level, in which case the class
 * starts a new level (Algorithm 2 with cuts only between classes, which coincides with the
 * printed algorithm on total orders). PRIOR edges take part in the analysis like any edge.
 * *num_levels_out (may be NULL) receives the number of levels. Errors: E_INVALID_ARG,
 * E_BAD_SCHEDULE, E_OOM, E_DEVICE. */
int fastlbp_schedule_set(fastlbp_graph_t g, int32_t kind, const int32_t *edge_rank, int32_t *num_levels_out);

/* Sets a general update strategy: a preorder on the edges given as equivalence classes and strict
 * precedences between classes (the Hasse diagram of Section 4.2, Algorithm 2's input, or any
 * relation whose transitive closure is the intended order).
 *   num_classes            1 .. 16384
 *   edge_class [E]         class of each edge, in [0, num_classes)
 *   arcs [2*num_arcs]      pairs (x, y): every edge of class x is updated strictly before every edge
 *                          of class y; may be NULL when num_arcs = 0
 * The preorder must satisfy Definition 2: an edge and every edge of its N_E (Definition 1) lie in
 * comparable classes (pairs involving a PRIOR edge are exempt, their messages being constant).
 * The classes are then ordered by a deterministic topological sort (smallest class first among
 * those ready) and the result equals fastlbp_schedule_set(RANKED) with those ranks; by Theorem 2
 * the messages do not depend on which topological order is taken. Errors: E_INVALID_ARG (ids out
 * of range), E_TOO_LARGE (too many classes), E_BAD_SCHEDULE (a cycle, a class before itself, or
 * incomparable dependent edges), E_OOM, E_DEVICE. */
int fastlbp_schedule_set_classes(fastlbp_graph_t g, int32_t num_classes, const int32_t *edge_class, int32_t num_arcs,
                                 const int32_t *arcs, int32_t *num_levels_out);

/* Host-only form of the above: writes the ranks [E] the preorder induces (its topological order),
 * or fails as above. factor_types may be NULL (then no edge is treated as PRIOR). */
int fastlbp_classes_to_ranks(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                             const int32_t *edge_vars, const uint8_t *factor_types, int32_t num_classes,
                             const int32_t *edge_class, int32_t num_arcs, const int32_t *arcs, int32_t *edge_rank);

/* Copies the level of every edge [E] (0-based) of the current schedule. */
int fastlbp_schedule_levels(fastlbp_graph_t g, int32_t *level_of_edge);

/* Host-only dependency analysis with no device and no graph handle, for callers that only need
 * the levels. Same inputs and result as fastlbp_graph_create + fastlbp_schedule_set(RANKED) +
 * fastlbp_schedule_levels. factor_types may be NULL. Errors: E_INVALID_ARG, E_BAD_GRAPH. */
int fastlbp_analyze_levels(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                           const int32_t *edge_vars, const int32_t *edge_rank, int32_t *level_of_edge,
                           int32_t *num_levels_out);

/* Host-only validation of a graph (the checks of fastlbp_graph_create, no device needed). */
int fastlbp_graph_validate(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                           const int32_t *edge_vars, const uint8_t *factor_types, const double *factor_params,
                           const double *edge_params);

/* ------------------------------------------------------------------------------------------ */
/* Autotuning of the launch choices                                                              */
/* ------------------------------------------------------------------------------------------ */

/* Launch choices for one graph shape, and how they were found. */
typedef struct fastlbp_tune_result {
    int32_t executor;              /* FASTLBP_EXEC_LEVELS, _PERSISTENT or _HYBRID */
    int32_t thread_max_degree;     /* factors of degree <= this: one thread each (1..8) */
    int32_t wave_max_degree;       /* then one wavefront each up to this degree (<= 257), then a workgroup */
    int32_t var_thread_max_degree; /* variables of degree <= this: one thread each (<= 64), else a wavefront */
    int32_t graph_iters;           /* iterations per hipGraph replay (LEVELS, HYBRID); 0 = the rule */
    int32_t persistent_threads;    /* persistent workgroup size, 512 or 1024; 0 = the rule */
    int32_t candidates;            /* configurations timed (0 when the choice came from the cache) */
    int32_t from_cache;            /* 1 when the choice came from the cache file */
    double best_ms_per_iter;       /* device time per iteration of the choice when it was timed */
    double default_ms_per_iter;    /* the same for the library's default choice */
    uint64_t key;                  /* shape key the choice is cached under */
} fastlbp_tune_result;

/* Picks the launch choices for the handle's graph and schedule. Small graphs lack parallelism and
 * large ones are bound by memory (Section 5.2), so no fixed setting suits every shape: the tuner
 * times a few candidates (executor; which factors run one per thread, per wavefront or per
 * workgroup; which variables one per thread or per wavefront; iterations per hipGraph replay; the
 * persistent workgroup size), each for probe_iters iterations with `damping` from the handle's
 * current messages (restored after every probe), and puts the handle on the fastest. The choice is
 * appended to the cache file (cache_path, or the environment variable FASTLBP_AUTOTUNE_CACHE; none:
 * no caching) under a key of the graph's shape (sizes, degree histograms, level widths), and a
 * later call for a handle of the same shape takes it from there without timing, so given the
 * cache the choice is deterministic. Every choice computes the same messages up to floating-point
 * rounding order. A later fastlbp_schedule_set keeps the bucket cut-offs; clones inherit the
 * choices. out may be NULL. Errors: E_INVALID_ARG (probe_iters < 1, bad damping, cache not
 * writable: the handle is tuned nevertheless), E_OOM, E_DEVICE (the handle is left as it was). */
int fastlbp_autotune(fastlbp_graph_t g, int32_t probe_iters, double damping, const char *cache_path,
                     fastlbp_tune_result *out);

/* Host-only access to a tuning cache file (cache_path or FASTLBP_AUTOTUNE_CACHE). get: returns
 * FASTLBP_OK and fills *out when the file has a valid line for key (the last one wins), 1 when not;
 * put: appends r (which must name a valid executor and cut-offs). Errors: E_INVALID_ARG. */
int fastlbp_autotune_cache_get(const char *cache_path, uint64_t key, fastlbp_tune_result *out);
int fastlbp_autotune_cache_put(const char *cache_path, const fastlbp_tune_result *r);

/* ------------------------------------------------------------------------------------------ */
/* Evidence (the feedback loop of Section 5.2.2) and messages                                   */
/* ------------------------------------------------------------------------------------------ */

/* Clamps (values 0/1) or releases (value -1) n variables. Messages are kept, so the next run
 * starts warm from the current state. Errors: E_INVALID_ARG. */
int fastlbp_evidence_set(fastlbp_graph_t g, int32_t n, const int32_t *vars, const int8_t *values);

/* Releases every clamp. */
int fastlbp_evidence_clear(fastlbp_graph_t g);

/* Runs belief propagation (Section 3.2, executed as in Section 4.3): at most max_iters iterations
 * of the current schedule from the current message state. One iteration updates every non-PRIOR
 * factor-to-variable message once: level by level in the order of the dependency analysis, each
 * level computing the variable-to-factor messages of Eq.(1) its factors read and then their
 * factor-to-variable messages of Eq.(2) in O(degree) per factor (Section 3.3). By Theorem 2 this
 * gives exactly the messages of the update rule Eq.(5) under the schedule's preorder; FLOODING is
 * the synchronous case, each message computed from the previous iteration's values. New messages
 * are normalised and, with damping lambda in [0,1), mixed with the old ones as
 * lambda * old + (1 - lambda) * new. The run stops after the first iteration whose residual (the
 * largest change of P(x=1) over the messages it wrote) is below tol (tol = 0: never) or after
 * max_iters iterations. Messages stay on the device: the next run starts from them (warm start).
 * stats may be NULL. Errors: E_INVALID_ARG, E_DEVICE. */
int fastlbp_run(fastlbp_graph_t g, int32_t max_iters, double tol, double damping, fastlbp_run_stats *stats);

/* Size of the fixed device area fastlbp_run_noalloc works in, one per device, held from the first
 * such call on a device until the process ends. */
#define FASTLBP_NOALLOC_SCRATCH_BYTES 16384

/* As fastlbp_run, for callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the call allocates no device or host memory.
 * The run's own state (iteration counters, convergence residual and contradiction partials) and
 * the persistent executor's launch descriptor live in a fixed library area of
 * FASTLBP_NOALLOC_SCRATCH_BYTES bytes per device, which one run always fits; the LEVELS and HYBRID
 * executors launch their kernels directly instead of replaying a captured hipGraph (whose
 * instantiation allocates). The handle's messages, beliefs and evidence are used and updated as
 * by fastlbp_run, and the results are the same. Every call on a device shares that device's area
 * and the area keeps the last call's contents (each call clears what it needs): calls that overlap
 * on one device, from several threads or on several streams, race and must be serialised by the
 * caller. Errors: E_INVALID_ARG, E_STATE (the handle's device state was evicted by a server:
 * restoring it would allocate), E_DEVICE (the area's address could not be obtained, or a HIP call
 * failed). */
int fastlbp_run_noalloc(fastlbp_graph_t g, int32_t max_iters, double tol, double damping, fastlbp_run_stats *stats);

/* Adaptive update strategies as rank generators (the randomized and residual-driven schedules of
 * related work, Section 6). The run proceeds in blocks of `every` iterations (the last block may be
 * shorter); before each block the generator gives every edge a rank, the dependency analysis splits
 * the ranks into levels (as fastlbp_schedule_set(RANKED)), and the block runs from the messages the
 * previous block left, as fastlbp_run with tol and damping; the run stops after a block that
 * converged or after max_iters iterations in total.
 *   FASTLBP_RANKS_RANDOM    random ordered groups: all edges of factor a get the rank
 *                           SplitMix64(seed; counter block * 2^32 + a) mod groups, where SplitMix64
 *                           is the published generator's output for that counter (the value mixed
 *                           from seed + (counter + 1) * 0x9E3779B97F4A7C15)
 *   FASTLBP_RANKS_RESIDUAL  residual-driven: block 0 is flooding; then each edge's rank comes from
 *                           the change r_e of its message's P(x=1) over the previous block:
 *                           rank = groups - 1 - min(groups - 1, floor(groups * r_e / max r)), so
 *                           the largest changes are updated first (all rank 0 when nothing moved)
 * The last block's schedule stays set. stats (may be NULL): iterations, updates, contradictions and
 * device time summed over the blocks; the other fields from the last block. Errors: E_INVALID_ARG,
 * E_OOM, E_DEVICE. */
enum { FASTLBP_RANKS_RANDOM = 0, FASTLBP_RANKS_RESIDUAL = 1 };
int fastlbp_run_adaptive(fastlbp_graph_t g, int32_t generator, int32_t groups, int32_t every, uint64_t seed,
                         int32_t max_iters, double tol, double damping, fastlbp_run_stats *stats);

/* The two generators on the host, for callers that drive their own loop (and for checking):
 * ranks_random writes the ranks of block `block` into edge_rank [E] (factor_offsets [F+1] as in
 * fastlbp_graph_create); ranks_residual the ranks from two message states p_before, p_after [E] of
 * P(x=1) in [0,1]. Errors: E_INVALID_ARG, E_BAD_GRAPH. */
int fastlbp_ranks_random(int32_t num_factors, const int64_t *factor_offsets, int32_t groups, uint64_t seed,
                         int32_t block, int32_t *edge_rank);
int fastlbp_ranks_residual(int64_t num_edges, const double *p_before, const double *p_after, int32_t groups,
                           int32_t *edge_rank);

/* Runs n handles side by side in one launch of the persistent executor (one workgroup per
 * handle): each handle runs from its own message state and evidence, exactly as fastlbp_run with
 * FASTLBP_EXEC_PERSISTENT would, with the same max_iters, tol and damping. The handles may belong
 * to different graphs but must share one device and one precision, and none may appear twice.
 * stats [n] may be NULL; device_ms is the time of the whole launch. Errors: E_INVALID_ARG,
 * E_OOM, E_DEVICE. */
int fastlbp_run_batch(int32_t n, fastlbp_graph_t *graphs, int32_t max_iters, double tol, double damping,
                      fastlbp_run_stats *stats);

/* Marginals P(X_v = 1) [V] of Eq.(3) from the current messages, evidence and priors (float64).
 * A variable whose incoming messages contradict (all products 0) gets 0.5. */
int fastlbp_marginals(fastlbp_graph_t g, double *p1);

/* Current factor-to-variable messages (the state Eq.(1)-(3) are computed from) as P(x_v = 1) [E]
 * (PRIOR edges report their prior). For checkpointing a query's state, moving it to another
 * handle, and checking one iteration against a reference from a known state. */
int fastlbp_messages_get(fastlbp_graph_t g, double *f2v_p1);

/* Sets the factor-to-variable messages from P(x_v = 1) [E] in [0,1] (PRIOR entries ignored): the
 * start state of the next run. For restoring a checkpoint, warm-starting from another handle's
 * state, and one-step checks from a known state (exact 0 and 1 are represented exactly). Errors:
 * E_INVALID_ARG. */
int fastlbp_messages_set(fastlbp_graph_t g, const double *f2v_p1);

/* Resets every message to uniform, the initial state of a run (a cold start). */
int fastlbp_messages_reset(fastlbp_graph_t g);

/* ------------------------------------------------------------------------------------------ */
/* Alarm ranking: BINGO's interactive loop (Section 5.2.2, Section 5.3)                         */
/* ------------------------------------------------------------------------------------------ */

typedef struct fastlbp_alarm_stats {
    int32_t rounds;           /* alarms inspected */
    int32_t true_found;       /* true alarms among them */
    int64_t iterations;       /* BP iterations over all rounds */
    int64_t message_updates;  /* factor-to-variable updates over all rounds */
    double device_ms;         /* device time of the BP runs and alarm picks (HIP events) */
    double wall_ms;           /* host wall time of the whole loop */
    double method_bytes;      /* method bytes of the BP runs (method_bytes_per_iter x iterations) */
} fastlbp_alarm_stats;

/* The user-feedback loop of BINGO with a simulated user who knows the answers: each round runs
 * belief propagation (as fastlbp_run with max_iters, tol, damping, the current schedule, warm from
 * the messages the previous round left), picks the uninspected alarm with the highest marginal
 * P(x = 1), the value fastlbp_marginals would report (ties: the lowest position in alarm_vars; a
 * device reduction over beliefs rebuilt from the messages), asks
 * the user (labels) and clamps the alarm's variable to the answer. The loop ends once every true
 * alarm has been inspected or after max_rounds rounds.
 *   alarm_vars [A]   variables of the alarms, distinct, in [0, V)
 *   labels [A]       the user's answer per alarm: 1 = true alarm, 0 = false alarm
 *   out_order [max_rounds]  receives the positions (in alarm_vars) in inspection order
 *   out_prob [max_rounds]   receives each picked alarm's marginal at the time of the pick (NULL ok)
 * The clamps stay on the handle's evidence afterwards (fastlbp_evidence_clear releases them), and
 * clamps set before the call stay too. stats may be NULL. Inversion count, Rank-100%-T and
 * Rank-90%-T follow from out_order and labels. Errors: E_INVALID_ARG (bad sizes, a variable out of
 * range or repeated, a label outside {0, 1}), E_OOM, E_DEVICE. */
int fastlbp_alarm_loop(fastlbp_graph_t g, int32_t num_alarms, const int32_t *alarm_vars, const int8_t *labels,
                       int32_t max_rounds, int32_t max_iters, double tol, double damping, int32_t *out_order,
                       double *out_prob, fastlbp_alarm_stats *stats);

/* ------------------------------------------------------------------------------------------ */
/* Serving: continuous batching of queries (the interactive loop of Section 5.2.2 at scale)      */
/* ------------------------------------------------------------------------------------------ */

typedef struct fastlbp_server *fastlbp_server_t;

typedef struct fastlbp_server_options {
    int32_t device;        /* HIP device ordinal; every submitted graph must live there */
    int32_t precision;     /* FASTLBP_FP32 or FASTLBP_FP64; every submitted graph must use it */
    int32_t max_active;    /* runs advanced side by side (one workgroup each), >= 1 */
    int32_t step_iters;    /* iterations per step; requests join or leave between steps, >= 1 */
    size_t memory_budget;  /* bytes of device state (messages, beliefs, potentials, marginals, run
                              state) the server keeps resident for the graphs submitted to it: idle
                              graphs are evicted to host memory to stay within it, evicted graphs
                              are restored when admitted; 0 = 80% of the device's free memory at
                              creation */
    int32_t step_levels;   /* > 0: a run advances per step by about this many levels (its iterations
                              per step = step_levels / levels per iteration, at least 1; wide runs
                              count kernel launches per iteration instead of levels), so a step costs
                              about the same for every run and small graphs finish in a few steps
                              instead of waiting out the steps of large ones; after a step during
                              which no request arrived (and none waits), the next step of the
                              narrow runs is 4 times longer, so runs left alone take fewer launches; 0: every run advances
                              by step_iters */
} fastlbp_server_options;

typedef struct fastlbp_server_stats {
    int64_t completed;        /* requests finished successfully */
    int64_t message_updates;  /* factor-to-variable updates of the finished requests */
    int64_t steps;            /* steps so far */
    double busy_ms;           /* wall time spent in steps */
    double kernel_ms;         /* device time of the steps (HIP events): per step, the longest of
                               * its persistent launch and the wide runs on their own streams */
    double method_bytes;      /* method bytes of the finished requests (method_bytes_per_iter x iterations) */
    double p50_ms, p99_ms;    /* latency (submit to marginals ready) of the finished requests */
    int32_t pending, active;  /* queue length and runs in flight right now */
    int64_t evictions;        /* idle graphs whose device state was moved to host memory */
    int64_t restores;         /* evicted graphs whose device state was allocated again at admission */
    size_t resident_bytes;    /* device state of the server's graphs resident now */
    size_t peak_resident_bytes; /* largest resident_bytes after an admission round */
    int64_t persistent_launches; /* launches of the persistent executor (one per step with narrow runs) */
    double persistent_ms;     /* their device time (HIP events on the server's stream) */
    double persistent_method_bytes; /* their method bytes: each run's method_bytes_per_iter times the
                               * iterations it advanced in the launch */
} fastlbp_server_stats;

/* Defaults: device 0, FP32, 256 active runs, 2 iterations per step (used when step_levels is 0),
 * budget 0 (80% of free), step_levels 2048. */
void fastlbp_server_options_default(fastlbp_server_options *o);

/* Starts a server with its own host thread and stream. Errors: E_INVALID_ARG, E_DEVICE. */
int fastlbp_server_create(const fastlbp_server_options *opts, fastlbp_server_t *out);

/* Queues a request: apply the n_ev clamps (values 0/1, -1 releases) to the graph's evidence, then
 * run max_iters iterations at most (tol, damping as in fastlbp_run) from the graph's current
 * messages (warm start). A run whose graph the AUTO rule assigns to the LEVELS executor (levels
 * too wide for one workgroup) is stepped with that executor on the handle's own stream, alongside
 * the persistent launch of the other runs. The handle belongs to the server until the request
 * completes: the caller must not use it meanwhile. Requests on one handle run one after another,
 * in order.
 * *ticket identifies the request. Errors: E_INVALID_ARG (device or precision mismatch),
 * E_TOO_LARGE (graph state above the memory budget), E_STATE (server shutting down). */
int fastlbp_server_submit(fastlbp_server_t s, fastlbp_graph_t g, int32_t n_ev, const int32_t *ev_vars,
                          const int8_t *ev_vals, int32_t max_iters, double tol, double damping, uint64_t *ticket);

/* Returns 1 while the request is pending. When it is done: returns 0, copies the marginals into
 * p1 [V] (may be NULL), its stats and its latency in ms (submit to marginals ready), and forgets
 * the ticket; a failed request returns its error code once. Errors: E_INVALID_ARG (unknown ticket). */
int fastlbp_server_poll(fastlbp_server_t s, uint64_t ticket, double *p1, fastlbp_run_stats *stats,
                        double *latency_ms);

/* As fastlbp_server_poll, but blocks until the request is done. */
int fastlbp_server_wait(fastlbp_server_t s, uint64_t ticket, double *p1, fastlbp_run_stats *stats,
                        double *latency_ms);

/* Aggregate statistics of the server so far. */
int fastlbp_server_get_stats(fastlbp_server_t s, fastlbp_server_stats *out);

/* Stops the server: waits for the runs in flight, fails the queued requests with E_STATE. */
void fastlbp_server_destroy(fastlbp_server_t s);

/* Description of the last failure on this thread ("" if none). */
const char *fastlbp_last_error(void);

/* Library version string. */
const char *fastlbp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTLBP_H */
