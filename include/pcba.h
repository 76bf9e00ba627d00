/*
 * pcba.h -- C ABI of the MI355X (gfx950) implementation of the Parallel
 * Constrained Bernstein Algorithm (PCBA): a branch-and-bound solver for
 * polynomial programs on a box.
 *
 * Problem (P), Sec. II-B of the paper:
 *     minimise p(x) over x in D = [lo_1,hi_1] x ... x [lo_l,hi_l]
 *     subject to g_i(x) <= 0 (i = 1..alpha) and h_j(x) = 0 (j = 1..beta).
 * Algorithm inputs (Alg. PCBA): optimality tolerance eps, step tolerance delta,
 * equality tolerance eps_eq, the maximum number of patches M and of
 * iterations N.  Outputs: the estimate p* and a box x* (Alg. PCBA, return step),
 * or "infeasible".
 *
 * Conventions for every entry point:
 *  - Return value: PCBA_OK (0) or a negative PCBA_E_* code.  No exception ever
 *    crosses this boundary.  pcba_last_error() gives a message for the calling
 *    thread's last failure.
 *  - Pointers named *_coef / *_deg / lo / hi are HOST pointers.  Their contents
 *    are copied during the call; the caller may free them on return.
 *  - Polynomial layout: for multi-degree (n_1..n_l) the coefficient of x^J sits
 *    at offset sum_k j_k * prod_{m>k}(n_m+1) (row-major, x_l fastest).  The alpha
 *    inequality tensors are concatenated in order i = 1..alpha, each at its own
 *    multi-degree given by ineq_deg[i*l .. i*l+l-1]; equalities likewise.
 *  - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *    library's own stream).  The library calls the HIP runtime directly.
 *  - A problem handle is not thread-safe; distinct handles are independent.
 *  - Solver outcomes (infeasible, memory limit, iteration cap, time limit) are
 *    results, not errors: they are reported in pcba_result_t.outcome.
 */
#ifndef PCBA_H
#define PCBA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCBA_MAX_DIM 8      /* largest dimension l accepted */
#define PCBA_MAX_DEGREE 15  /* largest degree per variable accepted */

/* arithmetic of the per-step subdivision */
enum {
    PCBA_FP64_PLAIN = 0,  /* FP64 patches, unwidened bounds (the paper's semantics) */
    PCBA_FP32 = 1         /* FP32 patches (offsets from a per-patch FP64 base),
                             split by the engine split_engine names; every bound
                             widened by a rigorous rounding-error bound carried
                             per patch; FP64 root, periodic FP64 re-derivation,
                             FP64 certification */
};

/* how PCBA_FP32 splits a patch (pcba_options.split_engine) */
enum {
    PCBA_SPLIT_VALU = 0,  /* de Casteljau at the subdivision parameter on the vector
                             ALUs, one fibre per lane (Sec. II-E) */
    PCBA_SPLIT_MFMA = 1   /* on the matrix cores: both children of a block of fibres
                             as one product with the stacked subdivision matrices
                             [S_L; S_R] of Sec. II-E (FP32 MFMA) */
};

/* outcomes (pcba_result_t.outcome) */
enum {
    PCBA_RUNNING = -1,
    PCBA_OPTIMAL = 0,       /* stopping criteria met (tolerance definition, Sec. III-C) */
    PCBA_INFEASIBLE = 1,    /* every box eliminated as infeasible */
    PCBA_MEMORY_LIMIT = 2,  /* memory test: 2*length(L) > M (2^l*length(L) with fused_round) */
    PCBA_MAX_ITER = 3,      /* iteration count reached N */
    PCBA_TIMEOUT = 4        /* options.time_limit_s elapsed */
};

/* error codes (return values) */
enum {
    PCBA_OK = 0,
    PCBA_E_ARG = -1,     /* NULL pointer, l outside 1..PCBA_MAX_DIM, lo >= hi,
                            non-finite bound or coefficient, degree outside
                            0..PCBA_MAX_DEGREE, eps/delta/eps_eq <= 0, M < 2, N < 1,
                            unknown precision */
    PCBA_E_NOMEM = -2,   /* device memory for the root item and its two children
                            (or a growth step) could not be allocated */
    PCBA_E_DEVICE = -3,  /* a HIP runtime call failed */
    PCBA_E_STATE = -4    /* call out of order (e.g. reading a list never solved) */
};

typedef struct {
    double eps;              /* optimality tolerance, absolute, cost units (Def. of tolerances) */
    double delta;            /* step tolerance: max box width in the coordinates of D */
    double eps_eq;           /* equality tolerance */
    int64_t max_boxes;       /* M of the memory test (Alg. PCBA) */
    int32_t max_iters;       /* N (Alg. PCBA) */
    int32_t precision;       /* PCBA_FP64_PLAIN or PCBA_FP32 */
    int32_t rederive_every;  /* PCBA_FP32: steps between FP64 re-derivations (0 = never) */
    int32_t stale_filter;    /* 1: skip writing children whose cost lower bound already
                                exceeds the previous solution estimate (results are
                                unchanged); 0: write every child */
    int32_t retire_satisfied;/* 1 (default): an inequality whose patch on a box has
                                max B <= 0 is satisfied on the whole box (Thm. of
                                enclosure), and, since subdivision forms convex
                                combinations, on every sub-box; the box's descendants
                                stop carrying that patch.  Feasibility and the lists
                                are unchanged: in FP64 plain mode the results are
                                identical to 0, in FP32 mode they remain rigorous.
                                0: every box carries every patch, as in Alg. PCBA */
    int32_t fused_round;     /* 0 (default): each pass of the main loop splits one direction,
                                as Alg. PCBA does.  1: each pass is a whole round: every box
                                is split along all l axes at once (for l = 2, the children
                                S_a P S_b^T, a, b in {L, R}, of the subdivision matrices of
                                Sec. II-E), then bounded and cut off once.  Children are
                                convex combinations of their parent's coefficients, so a
                                quarter of an infeasible or suboptimal half is itself
                                infeasible or suboptimal: the round ends keep the estimate
                                and list of the one-direction passes, except where those
                                would have stopped or hit the memory test mid-round.  The
                                memory test then asks 2^l length(L) <= M; `steps` counts
                                rounds.  Requires l <= 2 and retire_satisfied = 0
                                (PCBA_E_ARG otherwise). */
    double time_limit_s;     /* 0 = none */
    /* Launch shape of the subdivision kernel (speed only: FP64 results do not
     * depend on it, FP32 bounds stay rigorous).  0 = the library's default. */
    int32_t tile_coefs;      /* coefficients per tile (per child region): 0, or 256..3584
                                (FP64) / 256..7168 (PCBA_FP32), and with fused_round at most
                                2/2^l of that; a patch larger than this gets a tile of its own;
                                at most 256 patches to a tile, and at most 64 cost patches when
                                the problem has constraints */
    int32_t wg_per_cu;       /* workgroups per compute unit of the launch: 0 = as many as
                                fit, else at most this many */
    /* Subdivision variants of Sec. III-D and Sec. II-E. */
    int32_t direction_rule;  /* 0 (default): directions in the order 1..l (Sec. III-D);
                                1: maximum width, the axis along which the boxes are widest
                                (the widest box at the list's depth vector; ties to the lowest
                                axis).  All boxes of a step share the direction. */
    int32_t split_engine;    /* PCBA_FP32 only: PCBA_SPLIT_VALU (default) or PCBA_SPLIT_MFMA.
                                Both carry a rigorous bound for their own rounding; the
                                results differ only within it */
    double subdiv_lambda;    /* subdivision parameter in (0,1), default 1/2: a box [a,b] along
                                the split axis becomes [a, a + lambda (b-a)] and the rest.  Away
                                from 1/2 boxes are no longer congruent: the stopping test uses
                                the widest box, max over axes of (hi - lo) max(lambda,
                                1-lambda)^depth, and with PCBA_FP32 rederive_every must be 0.
                                Not with fused_round. */
    int32_t persistent_steps;/* 0 (default): one launch per kernel per step.  1: when every
                                problem of a batch asks for it, the batch is of one precision (at
                                most 256 problems, lists of at most 4,096 boxes, FP32 split on
                                the vector ALUs) and no FP32
                                re-derivation falls due, several whole steps (subdivision, cut)
                                run in one cooperative launch with grid barriers between the
                                phases.  Results are the same either way; on MI355X the barriers'
                                device-scope release and acquire (eight XCDs, each with its own
                                L2) cost more than the launches they save. */
} pcba_options;

typedef struct {
    int32_t outcome;            /* PCBA_OPTIMAL ... PCBA_TIMEOUT (PCBA_RUNNING if unsolved) */
    int32_t has_x;              /* 1 if a feasible box was ever found */
    double p_up;                /* solution estimate p* (+inf if no feasible box) */
    double p_lo;                /* least lower bound of the last step */
    double x_lo[PCBA_MAX_DIM];  /* x* in the coordinates of D */
    double x_hi[PCBA_MAX_DIM];
    int32_t x_depth[PCBA_MAX_DIM];   /* id of x*: depth per axis ... */
    uint32_t x_index[PCBA_MAX_DIM];  /* ... and index per axis */
    int32_t rounds;             /* n: completed passes over all directions, from 1 */
    int32_t steps;              /* passes performed: directional subdivisions (rounds with fused_round) */
    int64_t list_len;           /* length of the list L now */
    int64_t peak_len;           /* max length of L at a memory test */
    int32_t depth[PCBA_MAX_DIM];/* depth vector of the boxes in L */
    int32_t next_dir;           /* direction (0-based) of the next subdivision */
    int32_t certified;          /* 1: FP64 re-derivation of x* certifies every g_i <= 0
                                   and every h_j inside the eps_eq band with a rigorous
                                   FP64 error bound */
    double p_cert;              /* rigorous FP64 upper bound of p over x* */
    double cert_err;            /* the FP64 error bound used for the certificate */
    double err_max;             /* PCBA_FP32: largest error bound given to a patch by a
                                   subdivision since the last reset (0 in FP64 plain mode) */
    double seconds;             /* wall time of the last solve call */
    int64_t capacity;           /* items the device list can hold now */
} pcba_result_t;

typedef struct pcba_problem pcba_problem;

/* Fills *opt with defaults: eps 1e-3, delta 1e-4, eps_eq 1e-4, M 2^20, N 28,
 * FP64 plain, re-derivation every 16 steps, retiring on, stale filter off,
 * one direction per pass, no time limit. */
void pcba_default_options(pcba_options* opt);

/* Builds problem (P) and its root item: every polynomial is zero-padded to the
 * common multi-degree of its kind (the memory formula of Sec. IV-C stores each
 * kind at one multi-degree) and converted to Bernstein form over D in FP64 on
 * the device (InitPatches, Alg. PCBA).  opt may be NULL (defaults).
 * On success *out owns device memory until pcba_destroy_problem. */
int pcba_create_problem(int32_t l, const double* lo, const double* hi,
                        const int32_t* cost_deg, const double* cost_coef,
                        int32_t n_ineq, const int32_t* ineq_deg, const double* ineq_coef,
                        int32_t n_eq, const int32_t* eq_deg, const double* eq_coef,
                        const pcba_options* opt, pcba_problem** out);

/* Runs Alg. PCBA to an outcome (memory test, subdivision, bounds, cut-off test,
 * elimination, stopping tests, advance), then certifies x* in FP64.
 * Blocks until done.  A problem already solved is left unchanged. */
int pcba_solve(pcba_problem* prob, void* stream);

/* Advances the problem by at most n_steps passes of the main loop (fewer if an
 * outcome is reached).  Used to compare step traces; blocks until done. */
int pcba_step(pcba_problem* prob, int32_t n_steps, void* stream);

/* Solves n independent problems together: every batched step subdivides,
 * bounds and compacts the lists of all unfinished problems in one launch per
 * kernel.  Each result equals the result of pcba_solve on that problem alone. */
int pcba_solve_batch(pcba_problem* const* probs, int32_t n, void* stream);

/* Copies the outcome and statistics of the last solve into *out (host). */
int pcba_result(const pcba_problem* prob, pcba_result_t* out);
/* pcba_result for n problems at once: out[b] (host array of n records) gets
 * the result of probs[b].  Reads host-side state only (no device call).
 * Returns PCBA_E_ARG, with out untouched, if any pointer is NULL or n < 0. */
int pcba_result_batch(const pcba_problem* const* probs, int32_t n, pcba_result_t* out);

/* Current list: length, then ids (host, len*l uint32: index per axis) and the
 * patches converted to FP64 (host, len*words doubles; words = pcba_patch_words).
 * Patches are the cost patch, the inequality patches, then the equality patches,
 * each at its kind's common multi-degree.  With retire_satisfied, an inequality
 * the box no longer carries (certified satisfied on it or on an ancestor) reads
 * back as NaN.  ids or patches may be NULL. */
int pcba_list_size(const pcba_problem* prob, int64_t* len);
int pcba_read_list(const pcba_problem* prob, uint32_t* ids, double* patches, int64_t cap);
/* PCBA_FP32 only: per-item, per-polynomial error bounds (host, len*(1+alpha+beta)). */
int pcba_read_errors(const pcba_problem* prob, double* err, int64_t cap);
int64_t pcba_patch_words(const pcba_problem* prob);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the ids and
 * patches of pcba_read_list, with the same layout and meaning, read through a
 * static device staging array of PCBA_STATIC_SCRATCH_BYTES per device (held by
 * the library until the process ends) instead of the device buffers that
 * pcba_read_list allocates per call.  The call makes no device allocation.
 *  - A list whose staging needs more than the array (len*words*8 bytes, rounded
 *    up to 256, plus len*l*4 bytes) is rejected with PCBA_E_ARG; nothing is read.
 *  - Every call on a device shares that device's array: calls that overlap on
 *    one device (other threads, other streams) race; the caller serializes them.
 *  - stream: a hipStream_t as void* on which the staging kernel and copies run
 *    (NULL = the library's stream of the calling thread, created on its first
 *    use); the call synchronizes it before it returns.
 *  - ids or patches may be NULL; cap as for pcba_read_list. */
#define PCBA_STATIC_SCRATCH_BYTES (64ll << 20)
int pcba_read_list_noalloc(const pcba_problem* prob, uint32_t* ids, double* patches, int64_t cap,
                           void* stream);

/* The step before the solver in RTD (Sec. II-C): each sensed obstacle point x_i
 * becomes one inequality of the planning problem, w(x_i, q) + eps_q <= 0, where
 * w(x, q) (x: a point in the plane, q: the l = 2 plan parameters) is >= 0 on the
 * forward reachable set, and eps_q > 0 makes the open safe set closed.
 *  - w_xdeg[2], w_qdeg[2]: w's multi-degree in x and in q (0..PCBA_MAX_DEGREE).
 *  - w_coef (host): the coefficient of x1^a x2^b q1^c q2^d at offset
 *    ((a*(w_xdeg[1]+1) + b)*(w_qdeg[0]+1) + c)*(w_qdeg[1]+1) + d.
 *  - pts (host): n_pts points, x1 then x2 for each.
 *  - out (host, caller-owned): n_pts polynomials in q of multi-degree w_qdeg, each
 *    (w_qdeg[0]+1)*(w_qdeg[1]+1) doubles in the layout of pcba_create_problem's
 *    coefficients: pass out as ineq_coef with w_qdeg as every row of ineq_deg.
 * FP64 on the host; PCBA_E_ARG for NULL pointers, n_pts < 0, degrees out of
 * range, non-finite eps_q or points. */
int pcba_rtd_constraints(const int32_t* w_xdeg, const int32_t* w_qdeg, const double* w_coef, int32_t n_pts,
                         const double* pts, double eps_q, double* out);

/* FP64 root patches (host, words doubles) as computed on the device. */
int pcba_read_root(const pcba_problem* prob, double* patches);

/* Device bytes one list item occupies for this problem (patches, id, error terms). */
int64_t pcba_item_bytes(const pcba_problem* prob);

/* Returns the problem to its initial state (L = {root item}), recomputing the
 * root patches on the device from the monomial coefficients it keeps resident,
 * so a solve can be repeated with no host-to-device traffic. */
int pcba_reset(pcba_problem* prob, void* stream);
/* pcba_reset for n problems with one launch per kernel. */
int pcba_reset_batch(pcba_problem* const* probs, int32_t n, void* stream);

/* Per-step trace of the last solve (device ring of PCBA_MAX_TRACE records):
 * for step s < min(steps, cap): parents subdivided k_in[s], children kept
 * k_kept[s], and p_up[s], p_lo[s] after the cut-off test.  Any pointer may be
 * NULL.  Returns the number of records written, or a negative error. */
#define PCBA_MAX_TRACE 512
int pcba_read_trace(const pcba_problem* prob, int32_t* k_in, int32_t* k_kept, double* p_up,
                    double* p_lo, int32_t cap);
/* The same steps: inequality patches carried by the k_in parents (a_in[s]) and
 * by the k_kept kept children (a_kept[s]); without retire_satisfied these are
 * k_in[s] and k_kept[s] times the number of inequalities. */
int pcba_read_trace_patches(const pcba_problem* prob, int64_t* a_in, int64_t* a_kept, int32_t cap);

/* List buffers come from a device arena that keeps freed memory for reuse
 * (a growing list or a new problem takes it again without a device
 * allocation).  This returns the arena's fully free chunks to the device. */
void pcba_release_cached_memory(void);

/* Releases every resource of the problem.  NULL is accepted. */
void pcba_destroy_problem(pcba_problem* prob);

/* ---- continuous batching (serving) ------------------------------------------------
 * An engine advances a changing set of resident problems together.  Problems
 * are admitted while the sum of their device footprints stays within the
 * budget; each pcba_engine_run call performs up to n_steps batched steps over
 * every admitted, unfinished problem; finished problems are certified and
 * handed back by pcba_engine_poll, freeing their share of the budget. */
typedef struct pcba_engine pcba_engine;

/* budget_bytes <= 0 means unlimited.  Each admitted problem is charged the
 * footprint of max(its capacity, reserve_boxes) list items (pcba_footprint_bytes);
 * a list that must grow beyond its charge waits, paused, until the budget has
 * room, except the oldest admitted problem, which always grows (so the engine
 * always makes progress). */
int pcba_engine_create(int64_t budget_bytes, int64_t reserve_boxes, void* stream,
                       pcba_engine** out);
/* Admits prob (returns 1 in *admitted) if its charge fits the remaining budget
 * (or the engine is empty), else leaves it with the caller (0 in *admitted). */
int pcba_engine_submit(pcba_engine* eng, pcba_problem* prob, int32_t* admitted);
/* Runs up to n_steps batched steps; *n_active = unfinished admitted problems. */
int pcba_engine_run(pcba_engine* eng, int32_t n_steps, int32_t* n_active);
/* Moves up to cap finished problems into done[]; *n_done = how many. */
int pcba_engine_poll(pcba_engine* eng, pcba_problem** done, int32_t cap, int32_t* n_done);
int64_t pcba_engine_used_bytes(const pcba_engine* eng);
void pcba_engine_destroy(pcba_engine* eng);

/* ---- kernel timing (HIP events around every launch of the step kernels) ----------
 * Kernel ids: 0 subdivide+bound FP64, 1 subdivide+bound FP32, 2 FP32 re-derivation,
 * 3 cut-off+compaction, 4 plan/memory test.  Off by default; timing adds one
 * event pair per launch. */
#define PCBA_NUM_KERNELS 5
void pcba_profile_enable(int32_t on);
void pcba_profile_reset(void);
/* total milliseconds and launch counts per kernel id (arrays of PCBA_NUM_KERNELS) */
void pcba_profile_read(double* ms, int64_t* launches);

/* ---- launch policy of the cut-off test and compaction (Alg. CutOffTest, Eliminate) --
 * A problem's cut runs in one workgroup while the step has at most `children`
 * children (2K, or 2^l K in a round); above that it is split over workgroups of
 * `part` children each (four more launches: the parts' minima, the estimate and
 * each part's kept count, the order-preserving compaction at the parts' offsets,
 * the state's updates).  Results are the same either way.  Process-wide; default
 * 32,768 and 4,096; children 0 never splits.  PCBA_E_ARG if children < 0 or
 * part < 64.  Set it while no engine runs steps. */
int pcba_set_cut_split(int64_t children, int32_t part);

/* Footprint estimate used for admission: bytes of a list of `boxes` items. */
int64_t pcba_footprint_bytes(const pcba_problem* prob, int64_t boxes);

const char* pcba_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
