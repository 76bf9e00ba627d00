/*
 * pcba_ref.h -- plain FP64 CPU oracle of the Parallel Constrained Bernstein
 * Algorithm (PCBA).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP library:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the HIP library.
 *
 * It is written to be read against the paper, not to be fast: scalar loops,
 * FP64 throughout, one list, no blocking or fusion.
 *
 *   Problem (P), Sec. II-B: minimise p(x) over a box D subject to
 *   g_i(x) <= 0 (i = 1..alpha) and h_j(x) = 0 (j = 1..beta).
 *
 * Coefficient layout: a polynomial of multi-degree (n_1..n_l) is stored with the
 * coefficient of x^J at offset sum_k j_k * prod_{m>k}(n_m+1) (x_l fastest).
 * The alpha inequality polynomials are concatenated in order, each at its own
 * multi-degree; likewise the beta equalities.
 *
 * Box ids: all boxes alive in one step are congruent, so a box is its depth
 * vector d (shared by the whole list) and one unsigned index i_k per axis: the
 * box is prod_k [lo_k + w_k*i_k/2^d_k, lo_k + w_k*(i_k+1)/2^d_k].
 */
#ifndef PCBA_REF_H
#define PCBA_REF_H

#ifdef __cplusplus
extern "C" {
#endif

#define PCBA_REF_MAX_DIM 8

enum {
    PCBA_REF_RUNNING = -1,
    PCBA_REF_OPTIMAL = 0,       /* stopping criteria met (Def. of tolerances, Sec. III-C) */
    PCBA_REF_INFEASIBLE = 1,    /* no item survives the cut-off test */
    PCBA_REF_MEMORY_LIMIT = 2,  /* 2*length(L) > M at the memory test */
    PCBA_REF_MAX_ITER = 3       /* iteration count reached N */
};

typedef struct pcba_ref pcba_ref;

typedef struct {
    int outcome;                          /* PCBA_REF_* */
    int has_x;                            /* 1 if a feasible item was ever found */
    double p_up;                          /* solution estimate (+inf if none) */
    double p_lo;                          /* least lower bound of the last step */
    double x_lo[PCBA_REF_MAX_DIM];        /* x* in original coordinates */
    double x_hi[PCBA_REF_MAX_DIM];
    int x_depth[PCBA_REF_MAX_DIM];        /* id of x*: depth vector and index */
    unsigned x_index[PCBA_REF_MAX_DIM];
    int rounds;                           /* n: completed passes over all l directions, from 1 */
    int steps;                            /* directional subdivisions performed */
    long long list_len;                   /* current length of L */
    long long peak_len;                   /* max length of L seen at a memory test */
    int depth[PCBA_REF_MAX_DIM];          /* current depth vector of the list */
    int next_dir;                         /* direction (0-based) of the next split */
} pcba_ref_result;

/* ---- primitives (Sec. II-D, II-E) ------------------------------------------------ */

/* Bernstein coefficients over the box [lo,hi] of the polynomial with monomial
 * coefficients `mono` (multi-degree deg[0..l-1]); `bern` has the same layout.
 * Returns 0, or -1 on a bad argument. */
int pcba_ref_to_bernstein(int l, const int* deg, const double* lo, const double* hi,
                          const double* mono, double* bern);

/* Midpoint subdivision of one patch along axis r (0-based): left/right child
 * patches, each with the parent's layout.  Returns 0 or -1. */
int pcba_ref_split(int l, const int* deg, int r, const double* parent,
                   double* left, double* right);

/* Split along axis r at parameter lambda in (0,1): the box's extent [a,b] along
 * r becomes [a, a + lambda (b-a)] (left) and [a + lambda (b-a), b] (right)
 * (Sec. II-E allows any parameter in [0,1]; 1/2 is pcba_ref_split).
 * Returns 0 or -1. */
int pcba_ref_split_at(int l, const int* deg, int r, double lambda, const double* parent,
                      double* left, double* right);

/* Round split: the patch bisected along every axis in turn, axis 0 first
 * (each of Sec. II-E's constant-matrix products along one axis, applied l
 * times), giving the 2^l children of the sub-boxes in the order of their id
 * bits, axis 0 most significant: child c takes the right half along axis k iff
 * bit (l-1-k) of c is set.  `children` holds 2^l patches of the parent's
 * layout.  Returns 0 or -1. */
int pcba_ref_split_round(int l, const int* deg, const double* parent, double* children);

/* ---- the algorithm (Alg. PCBA and its subroutines, Sec. III) ---------------------- */

/* Copies every input.  Degrees: cost_deg[l], ineq_deg[n_ineq*l], eq_deg[n_eq*l].
 * eps, delta, eps_eq > 0; max_boxes = M >= 2; max_iters = N >= 1.
 * Returns NULL on a bad argument or allocation failure. */
pcba_ref* pcba_ref_create(int l, const double* lo, const double* hi,
                          const int* cost_deg, const double* cost_coef,
                          int n_ineq, const int* ineq_deg, const double* ineq_coef,
                          int n_eq, const int* eq_deg, const double* eq_coef,
                          double eps, double delta, double eps_eq,
                          long long max_boxes, int max_iters);

/* One pass of the main loop: memory test, subdivision in the current direction,
 * bounds, cut-off test, infeasibility and stopping tests, elimination, and the
 * advance of direction and iteration count.  Returns PCBA_REF_RUNNING or the
 * final outcome (further calls return it again). */
int pcba_ref_step(pcba_ref* h);

/* Round mode, chosen before the first pass: 0 (default) splits along one
 * direction per pass, as Alg. PCBA does; 1 makes every pass a whole round,
 * splitting each item along all l directions at once (pcba_ref_split_round):
 * the memory test then asks 2^l * length(L) <= M, the cut-off, elimination
 * and stopping tests run once per round, and the iteration count advances
 * every pass.  Returns 0, or -1 once the problem has stepped. */
int pcba_ref_set_fused(pcba_ref* h, int on);

/* Direction rule and subdivision parameter, chosen before the first pass:
 * rule 0 (default) splits along the axes in the order 1..l (Sec. III-D);
 * rule 1 splits along the axis of maximum width (the widest box at the list's
 * depth vector, ties to the lowest axis; all boxes share the direction).
 * lambda in (0,1) (default 1/2) splits each box at a + lambda (b - a); the
 * stopping test then uses the widest box's width, max over axes of
 * (hi - lo) max(lambda, 1-lambda)^depth.  The iteration count n advances
 * every l passes.  Not with round mode.  Returns 0, or -1 on a bad argument
 * or once the problem has stepped. */
int pcba_ref_set_split(pcba_ref* h, int rule, double lambda);

/* Steps until an outcome is reached; returns it. */
int pcba_ref_solve(pcba_ref* h);

void pcba_ref_result_get(const pcba_ref* h, pcba_ref_result* out);

/* Words per item's patches: Pi(P+1) + alpha*Pi(G+1) + beta*Pi(H+1). */
long long pcba_ref_patch_words(const pcba_ref* h);
/* The common multi-degree of a kind (0 cost, 1 inequalities, 2 equalities). */
void pcba_ref_kind_degree(const pcba_ref* h, int kind, int* deg);

/* Copies the current list: ids[len*l] (indices i_k) and patches[len*words]
 * (cost patch, then inequality patches, then equality patches, each at the
 * kind's common multi-degree).  Either pointer may be NULL. */
void pcba_ref_list(const pcba_ref* h, unsigned* ids, double* patches);

/* Patches of the box (depth, index) derived from the root by the same sequence
 * of splits the main loop applies (the directions of the rule in force, at its
 * parameter; each step keeps the child named by the next bit of the index,
 * most significant first).  depth must be a depth vector the loop reaches.
 * Returns 0 or -1. */
int pcba_ref_derive(const pcba_ref* h, const int* depth, const unsigned* index,
                    double* patches);

void pcba_ref_destroy(pcba_ref* h);

#ifdef __cplusplus
}
#endif
#endif
