// pcba_internal.h -- device data model shared by the kernels and the host
// runtime of the PCBA library (not part of the public C ABI).
//
// List storage (per problem): two item buffers used in turn.  In a step the
// parents are the K items named by `live` in buffer `cur`; the children of
// parent j go to slots 2j (left) and 2j+1 (right) of buffer cur^1, the order
// the subdivision of Alg. Subdivision produces when each item is replaced by
// its two halves (in a round, which splits every axis, its 2^l children go to
// slots 2^l j + c, c's bits the halves per axis, axis 0 most significant).
// The cut-off test then writes the slots of the surviving children, in order,
// into `live`: elimination is a stream compaction of slot indices, and no
// patch is moved.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcba {

constexpr int KINDS = 3;      // 0 cost p, 1 inequalities g_i, 2 equalities h_j
constexpr int MAXL = 8;       // PCBA_MAX_DIM
constexpr int MAXM = 16;      // longest fibre: degree 15 + 1
constexpr int SUB_THREADS = 256;
constexpr int CERT_PPB = 16;    // polynomials per certification workgroup
constexpr int PLAN_FUSE_MAX = 256;  // batches up to this size form the plan inside k_sub (<= SUB_THREADS)
constexpr int CUT_THREADS = 1024;
constexpr int CUT_CACHE = 4;      // children per thread k_cut keeps in registers
constexpr int CUT_PART_DEFAULT = 4096;           // children per workgroup of a split cut
constexpr long long CUT_SPLIT_DEFAULT = 32768;   // children above which a problem's cut is split

// Per (problem, part) record of a cut split across workgroups.
struct CutPart {
    double m;            // least max B over the part's feasible children
    double plo;          // least min B over its live children
    int arg;             // first child attaining m
    int valid;           // the part belongs to a running problem whose cut is split
    int kept;            // its kept children
    int pad;
    long long units;     // their inequality units (retiring mode)
    long long patches;   // their carried inequality patches (retiring mode)
};
constexpr int REDERIVE_CHUNK = 256;  // patches per re-derivation chunk
constexpr int MAX_BATCH = 2048;   // problems per launch
constexpr int MAX_TILE64 = 3584;  // largest tile (coefficients) of an FP64 unit: 14 per lane
constexpr int MAX_TILE32 = 7168;  // largest tile of an FP32 unit: 28 per lane
constexpr int NCMAX = 4;          // children per parent: 2, or 2^l = 4 in a round (l <= 2)

// per-child feasibility flags (OR-ed by every tile of the child)
enum : uint32_t {
    F_INFEAS = 1u,   // some g_i has min B > 0, or some h_j has min B > 0 or max B < 0
    F_NOTFEAS = 2u   // some g_i has max B > 0, or some h_j leaves the eps_eq band
};

enum : int32_t {
    ST_RUNNING = -1,
    ST_OPTIMAL = 0,
    ST_INFEASIBLE = 1,
    ST_MEMLIMIT = 2,
    ST_MAXITER = 3,
    ST_TIMEOUT = 4,
    ST_GROW = 16     // paused: the next step needs more list capacity
};

// Device-resident solver state of one problem (written by the cut kernel).
struct InstState {
    // what a step's plan reads (every subdivision workgroup reads it for every
    // problem): kept within the first 128 bytes
    int32_t status;
    int32_t K;          // live parents
    int32_t r;          // direction of the next split (0-based)
    int32_t n;          // iteration count, starts at 1
    int32_t steps;
    int32_t cur;        // buffer holding the parents
    int32_t has_x;
    int32_t cert_ok;
    double p_up, p_lo;
    int64_t peak;
    uint32_t epoch;     // incremented by every reset: makes record stamps unique per solve
    uint32_t pad1;
    int64_t u1;         // retiring mode: inequality units of the next step (sum of tiles)
    int64_t a_live;     // inequality patches carried by the live parents
    int64_t htop[2];    // retiring mode: patches appended to each buffer's heap
    int32_t depth[MAXL];
    uint32_t x_index[MAXL];
    int32_t x_depth[MAXL];
    double p_cert, cert_err;
    double err_max;
};

// What the step kernels need of a problem's state, published by the plan
// kernel at the start of every step and read-only until the cut kernel.
struct StepInfo {
    int32_t K, cur, r, steps;
    double p_up;
    uint32_t stamp;
    int32_t A;          // inequality patches the parents carry (retiring mode)
};

// stamp of the child records written in the current step of a problem
__host__ __device__ inline uint32_t step_stamp(const InstState* st)
{
    return st->epoch * 65536u + (uint32_t)st->steps + 1u;
}

constexpr int MAX_TRACE = 512;   // PCBA_MAX_TRACE
constexpr int MAX_STEPS = 60000; // steps per solve must stay below 65536 (record stamps)

// One record per step, written by the cut kernel.
struct TraceRec {
    int32_t k_in, k_kept;
    double p_up, p_lo;
    int64_t a_in, a_kept;   // inequality patches carried by the parents / the kept children
};

// Read-only description of one problem for a launch.
struct DevInst {
    // what a step's plan reads, in the first 128 bytes (one cache line)
    int32_t l, n_polys, T, fp32;
    int32_t count[KINDS];          // 1, alpha, beta
    int32_t ptp[KINDS];            // patches per k_sub tile (tiles span parents)
    int32_t tile_start[KINDS + 1]; // first tile of each kind; tile_start[KINDS] = T
    int32_t M;                     // memory-test bound
    int32_t cap;                   // slots per buffer
    int32_t N;                     // iteration cap
    int32_t stale;                 // stale-estimate write filter on
    int32_t rederive;              // FP32: re-derive from the FP64 root every this many steps
    int32_t retire;                // retire inequalities certified satisfied on a box
    int32_t rows;                  // transform rows per child: sum over kinds and axes of m
    int32_t fused;                 // 1: every step is a whole round (all l axes split at
                                   // once, 2^l children per parent); 0: one direction
    int64_t hcap;                  // patches each heap holds
    InstState* st;
    int* hostflag;                 // engine's pinned host word: set when the problem stops running
    // the rest
    int32_t S[KINDS];              // coefficients per patch of each kind
    int32_t tile_polys[KINDS];     // patches per tile of an item (re-derivation units)
    int64_t off[KINDS];            // element offset of each kind inside an item (root layout)
    int64_t soff[KINDS];           // the same inside a list slot (retiring mode keeps the
                                   // inequalities out of the slots, in the heaps)
    int64_t stride;                // elements per item slot
    int32_t dims[KINDS][MAXL];     // fibre length (degree + 1) per axis and kind
    double eps, delta, eps_eq;
    double width0[MAXL];           // hi - lo of D
    double lam;                    // subdivision parameter (1/2: midpoint)
    int32_t rule;                  // direction rule: 0 the order 1..l, 1 maximum width
    int32_t mfma;                  // FP32: split on the matrix cores (else de Casteljau on the VALUs)
    void* buf[2];                  // item buffers (double or float), cap * stride each
    uint32_t* ids[2];              // cap * l box indices
    float2* err[2];                // FP32 mode: cap * n_polys pairs (error bound, pending
                                   // shift s): the next split works on the stored values
                                   // less s, relative to the base plus s
    double* base[2];               // FP32 mode: cap * n_polys FP64 bases; a patch's
                                   // coefficients are base + its stored FP32 values
    int32_t* live;                 // cap: slots of the live items, in list order
    double* minP;                  // child records, cap each
    double* maxP;
    uint32_t* flags;
    unsigned long long* stamp;     // cap: the step's stamp (high word) and the bits of an FP32
                                   // value at or below the child's cost lower bound (low
                                   // word), written together in one store (stale filter)
    // retiring mode: a box carries only the inequalities not yet certified
    // satisfied on it.  act[b][slot*count[1] + q], q < na[b][slot], are their
    // (index, heap patch) pairs, in any order; the patch itself is S[1]
    // coefficients at heap[b] + heap_patch * S[1].  Each step appends the
    // children's patches to the heap of buffer cur^1 (reserving with htop).
    int2* act[2];
    int32_t* na[2];
    void* heap[2];
    int64_t* upre;                 // cap + 1: first inequality unit of each live item, then the total
    int4* umap;                    // hcap entries: re-derivation inequality unit v of the step ->
                                   // (parent, its slot, tile of its carried list, carried count)
    int4* pmap;                    // hcap entries: carried inequality patch P of the step, in parent
                                   // order -> (parent, its slot, inequality, heap patch); both
                                   // written by k_cut for the next step
    double* tmat;                  // FP32 re-derivation: cap/2 parents x 2 children x tmw doubles
    int32_t tmw;                   // transform words per child: sum over kinds and axes of m^2
    int32_t tmk[KINDS];            // offset of each kind's transforms inside a child's block
    double* root;                  // FP64 root patches (item layout, W doubles), converted in
                                   // two stages per axis (pre-map, then basis change): a
                                   // readback copy, null after the problem's first reset
    double* racc;                  // the same patches converted in one stage per axis with
                                   // the combined matrices (an accurate root)
    double* root_err;              // rigorous bound on |racc - exact| per patch
    double* root_abs;              // max |racc| over each patch
    double* cert;                  // certification scratch: n_polys * 3 doubles
    TraceRec* trace;               // MAX_TRACE step records
    const double* mono;            // monomials, zero-padded, item layout (W doubles)
    const double* mats;            // per kind and axis: pre-map A then conversion U (m x m each)
    const double* macc;            // per kind and axis: combined matrix M then |terms| bound Mabs
    const int* matoff;             // KINDS * MAXL offsets into mats
    // padding to a multiple of 128 bytes: in a device array (256-byte aligned)
    // every problem's plan fields (the first 112 bytes) then share one cache line
    char pad_end[96];
};
static_assert(sizeof(DevInst) % 128 == 0, "DevInst: keep the size a multiple of 128 bytes");

// ---- box geometry of the subdivision variants (Sec. III-D, Sec. II-E) -----------------

// Width along one axis of the widest box at depth d: splits at lam keep at
// most the share max(lam, 1 - lam) (exactly w 2^-d at the midpoint).
__host__ __device__ inline double axis_width(double w, double lam, int d)
{
    if (lam == 0.5) return ldexp(w, -d);
    const double mu = lam > 0.5 ? lam : 1.0 - lam;
    double x = w;
    for (int t = 0; t < d; ++t) x *= mu;
    return x;
}

// The direction of the next split under the maximum-width rule: the axis
// along which the widest box is widest, ties to the lowest axis.
__host__ __device__ inline int widest_axis(const double* width0, double lam, const int* depth, int l)
{
    int best = 0;
    double bw = axis_width(width0[0], lam, depth[0]);
    for (int k = 1; k < l; ++k) {
        const double wk = axis_width(width0[k], lam, depth[k]);
        if (wk > bw) {
            bw = wk;
            best = k;
        }
    }
    return best;
}

// The part [a, b] of [0, 1] that the box with index i at depth d covers along
// an axis: the splits followed from [0, 1], the index's bits most significant
// first (0: [a, a + lam (b - a)], 1: the rest).
__host__ __device__ inline void unit_interval(double lam, int d, uint32_t i, double& a, double& b)
{
    if (lam == 0.5) {
        a = ldexp((double)i, -d);
        b = ldexp((double)i + 1.0, -d);
        return;
    }
    a = 0.0;
    b = 1.0;
    for (int t = d - 1; t >= 0; --t) {
        const double m = a + lam * (b - a);
        if ((i >> t) & 1u)
            a = m;
        else
            b = m;
    }
}

// ordered integer keys: key(a) < key(b) iff a < b (non-NaN), so min/max of
// floating values can use integer atomics
__device__ __forceinline__ unsigned long long fkey(double x)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double funkey(unsigned long long k)
{
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ unsigned int fkey(float x)
{
    unsigned int b = __float_as_uint(x);
    return (b >> 31) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float funkey(unsigned int k)
{
    unsigned int b = (k >> 31) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

template <typename T> struct KeyOf;
template <> struct KeyOf<double> { typedef unsigned long long type; };
template <> struct KeyOf<float> { typedef unsigned int type; };

}  // namespace pcba
