/*
 * pcba_ref.c -- plain FP64 CPU oracle of PCBA (Kousik, Zhang, Zhao, Vasudevan).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Shares no code
 * with the HIP library.
 *
 * What it follows:
 *   - Bernstein form and range enclosure: Sec. II-D (Thm. on enclosure).
 *   - Midpoint subdivision with constant matrices: Sec. II-E; here written as
 *     the de Casteljau recurrence with parameter 1/2, whose left and right
 *     outputs are exactly those matrix products.
 *   - The main loop: Alg. PCBA (Sec. III) with Alg. Subdivision,
 *     Alg. FindBounds, Alg. CutOffTest and Alg. Eliminate.
 *   - Feasible / infeasible / undecided: Def. of feasibility (Sec. III-E);
 *     solution estimate and suboptimality: the two definitions after it.
 *
 * Readings where the paper is silent, garbled or inconsistent (each is listed
 * in the design notes of the repository):
 *   R1 direction update cycles r = 1..l (the printed update never leaves r=1
 *      when l=2); the order 1..l is the one Sec. III-D states.
 *   R2 the cut-off test uses the definitions, not the garbled printed test:
 *      p_up is the min over feasible items of max B_p; p_lo and the keep
 *      decision are over items that are not infeasible; keep also needs
 *      min B_p <= p_up.
 *   R3 feasibility needs every g_i (max B_gi <= 0) and every h_j in the band
 *      -eps_eq <= min B_hj <= 0 <= max B_hj <= eps_eq; infeasibility needs one
 *      g_i with min B_gi > 0 or one h_j with min B_hj > 0 or max B_hj < 0.
 *   R4 the stopping test is the tolerance definition: some feasible item
 *      attains p_up, p_up - p_lo <= eps and the max box width <= delta, with
 *      widths measured in the original coordinates of D.
 *   R5 order within a pass: memory test, subdivide, bounds, cut-off,
 *      infeasibility exit, elimination, stopping test, advance; n == N is
 *      checked after the advance.
 *   R6 p_up is carried as a running minimum over passes; x* is updated to the
 *      first feasible child (in list order) attaining the new p_up whenever the
 *      pass's min over feasible children is <= the carried p_up.
 *   R7 each kind of polynomial is stored at a common multi-degree (componentwise
 *      max over that kind), as the memory formula of Sec. IV-C does; lower
 *      degrees are zero-padded in the monomial basis before conversion.
 *   R8 list order: children replace their parent, left before right.  The
 *      paper's elimination reorders the list; no result here depends on order
 *      except the x* tie-break, which R6 fixes.
 *   R9 round mode (not in the paper, which splits one direction per pass): a
 *      pass splits every item along all l directions, axis 0 first.  A
 *      child's coefficients are convex combinations of its parent's, so the
 *      children of an infeasible or suboptimal half are themselves infeasible
 *      or suboptimal: at the end of each round the estimate, the kept list and
 *      x* are those of the one-direction passes, except where those would have
 *      stopped or hit the memory test mid-round.  The memory test asks
 *      2^l * length(L) <= M; `steps` counts passes (rounds).
 */
#include "pcba_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KINDS 3

struct pcba_ref {
    int l;
    double lo[PCBA_REF_MAX_DIM], hi[PCBA_REF_MAX_DIM];
    int deg[KINDS][PCBA_REF_MAX_DIM];   /* common multi-degree of each kind */
    long long size[KINDS];              /* coefficients per patch of each kind */
    int count[KINDS];                   /* 1, alpha, beta */
    long long W;                        /* patch words per item */
    double eps, delta, eps_eq;
    long long M;
    int N;

    double* root;                       /* W coefficients over D */
    long long K;                        /* length of L */
    unsigned* ids;                      /* K*l */
    double* pat;                        /* K*W */
    int depth[PCBA_REF_MAX_DIM];
    int r;                              /* next direction, 0-based */
    int n;                              /* iteration count, starts at 1 */
    int steps;
    int status;
    double p_up, p_lo;
    int has_x;
    unsigned x_index[PCBA_REF_MAX_DIM];
    int x_depth[PCBA_REF_MAX_DIM];
    long long peak;
    int fused;                          /* 1: every pass splits along all l axes */
    int rule;                           /* direction rule: 0 cyclic, 1 maximum width */
    double lam;                         /* subdivision parameter (1/2: midpoint) */
};

/* ---- small helpers ---------------------------------------------------------------- */

static long long patch_size(int l, const int* deg)
{
    long long s = 1;
    for (int k = 0; k < l; ++k) s *= (long long)(deg[k] + 1);
    return s;
}

/* binomial coefficient C(n,k) as a double (exact for the degrees used here) */
static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * (double)(n - k + i) / (double)i;
    return c;
}

/* Apply the (m x m) matrix A along axis r of a patch with multi-degree deg:
 * out[.., k, ..] = sum_{i} A[k][i] * in[.., i, ..], summed in increasing i. */
static void apply_along_axis(int l, const int* deg, int r, const double* A,
                             const double* in, double* out)
{
    long long m = deg[r] + 1, stride = 1, outer = 1;
    for (int k = r + 1; k < l; ++k) stride *= deg[k] + 1;
    for (int k = 0; k < r; ++k) outer *= deg[k] + 1;
    for (long long o = 0; o < outer; ++o)
        for (long long s = 0; s < stride; ++s) {
            long long base = o * m * stride + s;
            for (long long k = 0; k < m; ++k) {
                double acc = 0.0;
                for (long long i = 0; i < m; ++i)
                    acc += A[k * m + i] * in[base + i * stride];
                out[base + k * stride] = acc;
            }
        }
}

/* ---- primitives ------------------------------------------------------------------- */

/*
 * Monomial -> Bernstein over [lo,hi], one axis at a time (tensor product).
 * Per axis of degree n with x = lo + w*t, w = hi - lo:
 *   1. affine pre-map (substitution x = lo + w t):
 *        a'_i = w^i * sum_{j=i..n} C(j,i) lo^(j-i) a_j
 *   2. monomial -> Bernstein on [0,1] (the precomputed conversion matrix of
 *      Sec. II-D):  beta_k = sum_{i=0..k} C(k,i)/C(n,i) * a'_i
 */
int pcba_ref_to_bernstein(int l, const int* deg, const double* lo, const double* hi,
                          const double* mono, double* bern)
{
    if (l < 1 || l > PCBA_REF_MAX_DIM || !deg || !lo || !hi || !mono || !bern) return -1;
    for (int k = 0; k < l; ++k)
        if (deg[k] < 0 || !(hi[k] > lo[k])) return -1;
    long long S = patch_size(l, deg);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)S);
    if (!tmp) return -1;
    memcpy(bern, mono, sizeof(double) * (size_t)S);
    for (int r = 0; r < l; ++r) {
        int n = deg[r];
        long long m = n + 1;
        double w = hi[r] - lo[r];
        double* A = (double*)calloc((size_t)(m * m), sizeof(double));
        double* U = (double*)calloc((size_t)(m * m), sizeof(double));
        if (!A || !U) { free(A); free(U); free(tmp); return -1; }
        for (int i = 0; i <= n; ++i) {
            double wi = 1.0;
            for (int t = 0; t < i; ++t) wi *= w;
            for (int j = i; j <= n; ++j) {
                double lp = 1.0;
                for (int t = 0; t < j - i; ++t) lp *= lo[r];
                A[i * m + j] = wi * binom(j, i) * lp;
            }
        }
        for (int k = 0; k <= n; ++k)
            for (int i = 0; i <= k; ++i)
                U[k * m + i] = binom(k, i) / binom(n, i);
        apply_along_axis(l, deg, r, A, bern, tmp);
        apply_along_axis(l, deg, r, U, tmp, bern);
        free(A);
        free(U);
    }
    free(tmp);
    return 0;
}

/*
 * Midpoint split along axis r by de Casteljau with parameter 1/2:
 *   c^(0)_i = b_i,  c^(m)_i = (c^(m-1)_i + c^(m-1)_{i+1}) / 2,
 *   left_k = c^(k)_0,  right_k = c^(n-k)_k.
 * These are the constant-matrix products M_{r,L} B and M_{r,R} B of Sec. II-E.
 */
int pcba_ref_split(int l, const int* deg, int r, const double* parent,
                   double* left, double* right)
{
    if (l < 1 || l > PCBA_REF_MAX_DIM || r < 0 || r >= l || !deg || !parent || !left || !right)
        return -1;
    long long n = deg[r], stride = 1, outer = 1;
    for (int k = r + 1; k < l; ++k) stride *= deg[k] + 1;
    for (int k = 0; k < r; ++k) outer *= deg[k] + 1;
    double c[64];
    if (n + 1 > 64) return -1;
    for (long long o = 0; o < outer; ++o)
        for (long long s = 0; s < stride; ++s) {
            long long base = o * (n + 1) * stride + s;
            for (long long i = 0; i <= n; ++i) c[i] = parent[base + i * stride];
            left[base] = c[0];
            right[base + n * stride] = c[n];
            for (long long m = 1; m <= n; ++m) {
                for (long long i = 0; i + m <= n; ++i) c[i] = (c[i] + c[i + 1]) * 0.5;
                left[base + m * stride] = c[0];
                right[base + (n - m) * stride] = c[n - m];
            }
        }
    return 0;
}

/*
 * Split at parameter lambda along axis r (the box [a,b] along r becomes
 * [a, a + lambda (b-a)] and [a + lambda (b-a), b]) by de Casteljau's
 * recurrence with that parameter:
 *   c^(0)_i = b_i,  c^(m)_i = (1 - lambda) c^(m-1)_i + lambda c^(m-1)_{i+1},
 *   left_k = c^(k)_0,  right_k = c^(n-k)_k.
 * lambda = 1/2 is pcba_ref_split, whose halving form it reproduces exactly.
 */
int pcba_ref_split_at(int l, const int* deg, int r, double lambda, const double* parent,
                      double* left, double* right)
{
    if (!(lambda > 0.0 && lambda < 1.0)) return -1;
    if (lambda == 0.5) return pcba_ref_split(l, deg, r, parent, left, right);
    if (l < 1 || l > PCBA_REF_MAX_DIM || r < 0 || r >= l || !deg || !parent || !left || !right)
        return -1;
    long long n = deg[r], stride = 1, outer = 1;
    for (int k = r + 1; k < l; ++k) stride *= deg[k] + 1;
    for (int k = 0; k < r; ++k) outer *= deg[k] + 1;
    double c[64];
    if (n + 1 > 64) return -1;
    const double mu = 1.0 - lambda;
    for (long long o = 0; o < outer; ++o)
        for (long long s = 0; s < stride; ++s) {
            long long base = o * (n + 1) * stride + s;
            for (long long i = 0; i <= n; ++i) c[i] = parent[base + i * stride];
            left[base] = c[0];
            right[base + n * stride] = c[n];
            for (long long m = 1; m <= n; ++m) {
                for (long long i = 0; i + m <= n; ++i) c[i] = mu * c[i] + lambda * c[i + 1];
                left[base + m * stride] = c[0];
                right[base + (n - m) * stride] = c[n - m];
            }
        }
    return 0;
}

/*
 * Round split: bisect along axis 0, then each half along axis 1, and so on.
 * After the split along axis k the children are ordered with the new bit
 * least significant, so the final order has axis 0's bit most significant.
 */
int pcba_ref_split_round(int l, const int* deg, const double* parent, double* children)
{
    if (l < 1 || l > PCBA_REF_MAX_DIM || !deg || !parent || !children) return -1;
    long long S = patch_size(l, deg);
    long long nc = 1LL << l;
    double* a = (double*)malloc(sizeof(double) * (size_t)(S * nc));
    double* b = (double*)malloc(sizeof(double) * (size_t)(S * nc));
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, parent, sizeof(double) * (size_t)S);
    long long have = 1;
    for (int k = 0; k < l; ++k) {
        for (long long c = 0; c < have; ++c)
            if (pcba_ref_split(l, deg, k, a + c * S, b + (2 * c) * S, b + (2 * c + 1) * S) != 0) {
                free(a); free(b);
                return -1;
            }
        have *= 2;
        double* t = a; a = b; b = t;
    }
    memcpy(children, a, sizeof(double) * (size_t)(S * nc));
    free(a);
    free(b);
    return 0;
}

/* ---- creation ------------------------------------------------------------------- */

static long long kind_offset(const pcba_ref* h, int kind, int idx)
{
    long long off = 0;
    for (int t = 0; t < kind; ++t) off += h->count[t] * h->size[t];
    return off + (long long)idx * h->size[kind];
}

/* Width along axis k of the widest box at depth d: the splits at lambda keep
 * the larger share max(lambda, 1 - lambda) (exactly 2^-d at the midpoint). */
static double axis_width(const pcba_ref* h, int k, int d)
{
    const double w = h->hi[k] - h->lo[k];
    if (h->lam == 0.5) return ldexp(w, -d);
    const double mu = h->lam > 0.5 ? h->lam : 1.0 - h->lam;
    double x = w;
    for (int t = 0; t < d; ++t) x *= mu;
    return x;
}

/* The direction of the next split: the next axis in the order 1..l
 * (Sec. III-D), or under the maximum-width rule the axis along which the
 * boxes are widest (ties: the lowest axis). */
static int next_direction(const pcba_ref* h, const int* depth, int r_prev, int first)
{
    if (h->rule == 0) return first ? 0 : (r_prev + 1) % h->l;
    int best = 0;
    double bw = axis_width(h, 0, depth[0]);
    for (int k = 1; k < h->l; ++k) {
        const double wk = axis_width(h, k, depth[k]);
        if (wk > bw) { bw = wk; best = k; }
    }
    return best;
}

/* Interval along axis k of the box with depth d and index i: the splits
 * followed from [0,1] (the unit box the patches are expressed over), the
 * index's bits most significant first (0: the part [a, a + lambda (b-a)],
 * 1: the rest), then mapped to D. */
static void box_interval(const pcba_ref* h, int k, int d, unsigned i, double* a_out, double* b_out)
{
    const double w = h->hi[k] - h->lo[k];
    double a, b;
    if (h->lam == 0.5) {
        a = ldexp((double)i, -d);
        b = ldexp((double)i + 1.0, -d);
    } else {
        a = 0.0;
        b = 1.0;
        for (int t = d - 1; t >= 0; --t) {
            const double m = a + h->lam * (b - a);
            if ((i >> t) & 1u) a = m; else b = m;
        }
    }
    *a_out = h->lo[k] + w * a;
    *b_out = h->lo[k] + w * b;
}

/* zero-pad a monomial tensor of multi-degree d to multi-degree D (d <= D) */
static void pad_monomials(int l, const int* d, const int* D, const double* in, double* out)
{
    long long Sd = patch_size(l, d), SD = patch_size(l, D);
    for (long long t = 0; t < SD; ++t) out[t] = 0.0;
    for (long long t = 0; t < Sd; ++t) {
        long long rem = t, off = 0, mul = 1;
        for (int k = l - 1; k >= 0; --k) {
            long long jk = rem % (d[k] + 1);
            rem /= d[k] + 1;
            off += jk * mul;
            mul *= D[k] + 1;
        }
        out[off] = in[t];
    }
}

pcba_ref* pcba_ref_create(int l, const double* lo, const double* hi,
                          const int* cost_deg, const double* cost_coef,
                          int n_ineq, const int* ineq_deg, const double* ineq_coef,
                          int n_eq, const int* eq_deg, const double* eq_coef,
                          double eps, double delta, double eps_eq,
                          long long max_boxes, int max_iters)
{
    if (l < 1 || l > PCBA_REF_MAX_DIM || !lo || !hi || !cost_deg || !cost_coef) return NULL;
    if (n_ineq < 0 || n_eq < 0) return NULL;
    if (n_ineq > 0 && (!ineq_deg || !ineq_coef)) return NULL;
    if (n_eq > 0 && (!eq_deg || !eq_coef)) return NULL;
    if (!(eps > 0) || !(delta > 0) || !(eps_eq > 0) || max_boxes < 2 || max_iters < 1)
        return NULL;
    for (int k = 0; k < l; ++k)
        if (!isfinite(lo[k]) || !isfinite(hi[k]) || !(hi[k] > lo[k])) return NULL;

    pcba_ref* h = (pcba_ref*)calloc(1, sizeof(pcba_ref));
    if (!h) return NULL;
    h->l = l;
    for (int k = 0; k < l; ++k) { h->lo[k] = lo[k]; h->hi[k] = hi[k]; }
    h->count[0] = 1;
    h->count[1] = n_ineq;
    h->count[2] = n_eq;
    const int* degs[KINDS] = {cost_deg, ineq_deg, eq_deg};
    const double* coefs[KINDS] = {cost_coef, ineq_coef, eq_coef};
    for (int t = 0; t < KINDS; ++t) {
        for (int k = 0; k < l; ++k) h->deg[t][k] = 0;
        for (int i = 0; i < h->count[t]; ++i)
            for (int k = 0; k < l; ++k) {
                int dk = degs[t][i * l + k];
                if (dk < 0 || dk > 62) { free(h); return NULL; }
                if (dk > h->deg[t][k]) h->deg[t][k] = dk;
            }
        h->size[t] = h->count[t] ? patch_size(l, h->deg[t]) : 0;
    }
    h->W = 0;
    for (int t = 0; t < KINDS; ++t) h->W += h->count[t] * h->size[t];
    h->eps = eps;
    h->delta = delta;
    h->eps_eq = eps_eq;
    h->M = max_boxes;
    h->N = max_iters;

    h->root = (double*)malloc(sizeof(double) * (size_t)h->W);
    h->ids = (unsigned*)calloc((size_t)l, sizeof(unsigned));
    h->pat = (double*)malloc(sizeof(double) * (size_t)h->W);
    if (!h->root || !h->ids || !h->pat) { pcba_ref_destroy(h); return NULL; }

    /* InitPatches: every polynomial to Bernstein form over D (Alg. PCBA, first step). */
    for (int t = 0; t < KINDS; ++t) {
        long long in_off = 0;
        for (int i = 0; i < h->count[t]; ++i) {
            const int* d = degs[t] + i * l;
            long long sd = patch_size(l, d);
            for (long long q = 0; q < sd; ++q)
                if (!isfinite(coefs[t][in_off + q])) { pcba_ref_destroy(h); return NULL; }
            double* padded = (double*)malloc(sizeof(double) * (size_t)h->size[t]);
            if (!padded) { pcba_ref_destroy(h); return NULL; }
            pad_monomials(l, d, h->deg[t], coefs[t] + in_off, padded);
            pcba_ref_to_bernstein(l, h->deg[t], lo, hi, padded,
                                  h->root + kind_offset(h, t, i));
            free(padded);
            in_off += sd;
        }
    }
    memcpy(h->pat, h->root, sizeof(double) * (size_t)h->W);
    h->K = 1;                     /* L = {root item} */
    h->rule = 0;
    h->lam = 0.5;
    h->r = 0;
    h->n = 1;
    h->status = PCBA_REF_RUNNING;
    h->p_up = INFINITY;
    h->p_lo = INFINITY;
    return h;
}

void pcba_ref_destroy(pcba_ref* h)
{
    if (!h) return;
    free(h->root);
    free(h->ids);
    free(h->pat);
    free(h);
}

/* ---- one pass of the main loop ------------------------------------------------ */

typedef struct {
    double minP, maxP;
    int feasible, infeasible;
} bounds_t;

/* FindBounds for one item followed by the feasibility classification. */
static bounds_t classify(const pcba_ref* h, const double* item)
{
    bounds_t b;
    b.minP = INFINITY;
    b.maxP = -INFINITY;
    for (long long q = 0; q < h->size[0]; ++q) {
        if (item[q] < b.minP) b.minP = item[q];
        if (item[q] > b.maxP) b.maxP = item[q];
    }
    b.feasible = 1;
    b.infeasible = 0;
    for (int t = 1; t < KINDS; ++t)
        for (int i = 0; i < h->count[t]; ++i) {
            const double* P = item + kind_offset(h, t, i);
            double mn = INFINITY, mx = -INFINITY;
            for (long long q = 0; q < h->size[t]; ++q) {
                if (P[q] < mn) mn = P[q];
                if (P[q] > mx) mx = P[q];
            }
            if (t == 1) {                                   /* g_i <= 0 */
                if (!(mx <= 0.0)) b.feasible = 0;
                if (mn > 0.0) b.infeasible = 1;
            } else {                                        /* h_j = 0 */
                if (!(-h->eps_eq <= mn && mn <= 0.0 && 0.0 <= mx && mx <= h->eps_eq))
                    b.feasible = 0;
                if (mn > 0.0 || mx < 0.0) b.infeasible = 1;
            }
        }
    if (b.infeasible) b.feasible = 0;
    return b;
}

int pcba_ref_step(pcba_ref* h)
{
    if (!h) return PCBA_REF_RUNNING;
    if (h->status != PCBA_REF_RUNNING) return h->status;
    const int l = h->l, r = h->r;
    const long long K = h->K, W = h->W;

    /* children per item: 2, or 2^l when a pass is a whole round */
    const long long nc = h->fused ? (1LL << l) : 2;

    /* memory test */
    if (K > h->peak) h->peak = K;
    if (nc * K > h->M) { h->status = PCBA_REF_MEMORY_LIMIT; return h->status; }

    /* Subdivision (parallel in the paper): each item is replaced by its left
     * then right child along direction r, or in round mode by its 2^l
     * children, in the order of their id bits (axis 0 most significant). */
    const long long C = nc * K;
    unsigned* cids = (unsigned*)malloc(sizeof(unsigned) * (size_t)(C * l));
    double* cpat = (double*)malloc(sizeof(double) * (size_t)(C * W));
    bounds_t* bd = (bounds_t*)malloc(sizeof(bounds_t) * (size_t)C);
    char* keep = (char*)malloc((size_t)C);
    if (!cids || !cpat || !bd || !keep) {
        free(cids); free(cpat); free(bd); free(keep);
        h->status = PCBA_REF_MEMORY_LIMIT;
        return h->status;
    }
    long long maxS = 0;
    for (int t = 0; t < KINDS; ++t)
        if (h->size[t] > maxS) maxS = h->size[t];
    double* round_out = h->fused ? (double*)malloc(sizeof(double) * (size_t)(nc * (maxS ? maxS : 1))) : NULL;
    if (h->fused && !round_out) {
        free(cids); free(cpat); free(bd); free(keep);
        h->status = PCBA_REF_MEMORY_LIMIT;
        return h->status;
    }
    for (long long k = 0; k < K; ++k) {
        const double* parent = h->pat + k * W;
        if (!h->fused) {
            double* left = cpat + (2 * k) * W;
            double* right = cpat + (2 * k + 1) * W;
            for (int t = 0; t < KINDS; ++t)
                for (int i = 0; i < h->count[t]; ++i) {
                    long long off = kind_offset(h, t, i);
                    pcba_ref_split_at(l, h->deg[t], r, h->lam, parent + off, left + off, right + off);
                }
            for (int q = 0; q < l; ++q) {
                cids[(2 * k) * l + q] = h->ids[k * l + q];
                cids[(2 * k + 1) * l + q] = h->ids[k * l + q];
            }
            cids[(2 * k) * l + r] = 2u * h->ids[k * l + r];
            cids[(2 * k + 1) * l + r] = 2u * h->ids[k * l + r] + 1u;
            continue;
        }
        /* round mode: every patch to its 2^l children, scattered to the items */
        for (int t = 0; t < KINDS; ++t)
            for (int i = 0; i < h->count[t]; ++i) {
                long long off = kind_offset(h, t, i);
                pcba_ref_split_round(l, h->deg[t], parent + off, round_out);
                for (long long c = 0; c < nc; ++c)
                    memcpy(cpat + (nc * k + c) * W + off, round_out + c * h->size[t],
                           sizeof(double) * (size_t)h->size[t]);
            }
        for (long long c = 0; c < nc; ++c)
            for (int q = 0; q < l; ++q)
                cids[(nc * k + c) * l + q] = 2u * h->ids[k * l + q] + (unsigned)((c >> (l - 1 - q)) & 1);
    }
    free(round_out);
    if (h->fused)
        for (int q = 0; q < l; ++q) h->depth[q] += 1;
    else
        h->depth[r] += 1;
    h->steps += 1;

    /* FindBounds (parallel in the paper) */
    for (long long c = 0; c < C; ++c) bd[c] = classify(h, cpat + c * W);

    /* CutOffTest: solution estimate, least lower bound, keep decision */
    double m = INFINITY;
    long long arg = -1;
    for (long long c = 0; c < C; ++c)
        if (bd[c].feasible && (arg < 0 || bd[c].maxP < m)) { m = bd[c].maxP; arg = c; }
    if (arg >= 0 && m <= h->p_up) {
        h->p_up = m;
        h->has_x = 1;
        for (int q = 0; q < l; ++q) {
            h->x_index[q] = cids[arg * l + q];
            h->x_depth[q] = h->depth[q];
        }
    }
    double plo = INFINITY;
    long long kept = 0;
    for (long long c = 0; c < C; ++c) {
        if (!bd[c].infeasible && bd[c].minP < plo) plo = bd[c].minP;
        keep[c] = (char)(!bd[c].infeasible && bd[c].minP <= h->p_up);
        kept += keep[c];
    }
    h->p_lo = plo;

    /* Eliminate: keep the surviving children, in list order */
    unsigned* nids = (unsigned*)malloc(sizeof(unsigned) * (size_t)((kept ? kept : 1) * l));
    double* npat = (double*)malloc(sizeof(double) * (size_t)((kept ? kept : 1) * W));
    if (!nids || !npat) {
        free(nids); free(npat); free(cids); free(cpat); free(bd); free(keep);
        h->status = PCBA_REF_MEMORY_LIMIT;
        return h->status;
    }
    long long j = 0;
    for (long long c = 0; c < C; ++c)
        if (keep[c]) {
            memcpy(nids + j * l, cids + c * l, sizeof(unsigned) * (size_t)l);
            memcpy(npat + j * W, cpat + c * W, sizeof(double) * (size_t)W);
            ++j;
        }
    free(h->ids);
    free(h->pat);
    h->ids = nids;
    h->pat = npat;
    h->K = kept;
    free(cids); free(cpat); free(bd); free(keep);

    /* infeasibility exit */
    if (kept == 0) { h->status = PCBA_REF_INFEASIBLE; return h->status; }

    /* stopping criteria: tolerances met by the feasible item attaining p_up */
    double width = 0.0;
    for (int q = 0; q < l; ++q) {
        double wq = axis_width(h, q, h->depth[q]);
        if (wq > width) width = wq;
    }
    if (h->p_up < INFINITY && h->p_up - h->p_lo <= h->eps && width <= h->delta) {
        h->status = PCBA_REF_OPTIMAL;
        return h->status;
    }

    /* prepare the next iteration (a round-mode pass is a whole round) */
    h->r = h->fused ? 0 : next_direction(h, h->depth, r, 0);
    if (h->fused || h->steps % l == 0) h->n += 1;
    if (h->n == h->N) { h->status = PCBA_REF_MAX_ITER; return h->status; }
    return PCBA_REF_RUNNING;
}

int pcba_ref_set_fused(pcba_ref* h, int on)
{
    if (!h || h->steps > 0 || h->status != PCBA_REF_RUNNING) return -1;
    if (on && (h->rule != 0 || h->lam != 0.5)) return -1;
    h->fused = on ? 1 : 0;
    return 0;
}

int pcba_ref_set_split(pcba_ref* h, int rule, double lambda)
{
    if (!h || h->steps > 0 || h->status != PCBA_REF_RUNNING) return -1;
    if ((rule != 0 && rule != 1) || !(lambda > 0.0 && lambda < 1.0)) return -1;
    if (h->fused && (rule != 0 || lambda != 0.5)) return -1;
    h->rule = rule;
    h->lam = lambda;
    h->r = next_direction(h, h->depth, 0, 1);
    return 0;
}

int pcba_ref_solve(pcba_ref* h)
{
    int s;
    while ((s = pcba_ref_step(h)) == PCBA_REF_RUNNING) { }
    return s;
}

void pcba_ref_result_get(const pcba_ref* h, pcba_ref_result* out)
{
    memset(out, 0, sizeof(*out));
    out->outcome = h->status;
    out->has_x = h->has_x;
    out->p_up = h->p_up;
    out->p_lo = h->p_lo;
    for (int q = 0; q < h->l; ++q) {
        out->depth[q] = h->depth[q];
        if (h->has_x) {
            double w = h->hi[q] - h->lo[q];
            out->x_depth[q] = h->x_depth[q];
            out->x_index[q] = h->x_index[q];
            (void)w;
            box_interval(h, q, h->x_depth[q], h->x_index[q], &out->x_lo[q], &out->x_hi[q]);
        }
    }
    out->rounds = h->n;
    out->steps = h->steps;
    out->list_len = h->K;
    out->peak_len = h->peak;
    out->next_dir = h->r;
}

long long pcba_ref_patch_words(const pcba_ref* h) { return h->W; }

void pcba_ref_kind_degree(const pcba_ref* h, int kind, int* deg)
{
    for (int q = 0; q < h->l; ++q) deg[q] = (kind >= 0 && kind < KINDS) ? h->deg[kind][q] : 0;
}

void pcba_ref_list(const pcba_ref* h, unsigned* ids, double* patches)
{
    if (ids) memcpy(ids, h->ids, sizeof(unsigned) * (size_t)(h->K * h->l));
    if (patches) memcpy(patches, h->pat, sizeof(double) * (size_t)(h->K * h->W));
}

int pcba_ref_derive(const pcba_ref* h, const int* depth, const unsigned* index,
                    double* patches)
{
    const int l = h->l;
    int total = 0;
    for (int q = 0; q < l; ++q) {
        if (depth[q] < 0 || depth[q] > 32) return -1;
        total += depth[q];
    }
    double* cur = (double*)malloc(sizeof(double) * (size_t)h->W);
    double* other = (double*)malloc(sizeof(double) * (size_t)h->W);
    if (!cur || !other) { free(cur); free(other); return -1; }
    memcpy(cur, h->root, sizeof(double) * (size_t)h->W);
    int done[PCBA_REF_MAX_DIM] = {0};
    int r = next_direction(h, done, 0, 1);
    for (int s = 0; s < total; ++s) {
        if (s > 0) r = next_direction(h, done, r, 0);
        /* the loop's sequence of directions must reach the depth vector */
        if (done[r] >= depth[r]) { free(cur); free(other); return -1; }
        unsigned bit = (index[r] >> (depth[r] - 1 - done[r])) & 1u;
        for (int t = 0; t < KINDS; ++t)
            for (int i = 0; i < h->count[t]; ++i) {
                long long off = kind_offset(h, t, i);
                /* scratch for the unused half */
                double* dump = (double*)malloc(sizeof(double) * (size_t)h->size[t]);
                if (!dump) { free(cur); free(other); return -1; }
                if (bit == 0)
                    pcba_ref_split_at(l, h->deg[t], r, h->lam, cur + off, other + off, dump);
                else
                    pcba_ref_split_at(l, h->deg[t], r, h->lam, cur + off, dump, other + off);
                free(dump);
            }
        double* sw = cur; cur = other; other = sw;
        done[r] += 1;
    }
    memcpy(patches, cur, sizeof(double) * (size_t)h->W);
    free(cur);
    free(other);
    return 0;
}
