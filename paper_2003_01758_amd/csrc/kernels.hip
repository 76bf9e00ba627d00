// kernels.hip -- gfx950 kernels of the PCBA hot path.
//
//   k_root      InitPatches (Alg. PCBA): monomial -> Bernstein over D, FP64,
//               with an a-priori rounding bound per patch.
//   k_sub       Alg. Subdivision fused with Alg. FindBounds: midpoint split of
//               every live item along direction r (de Casteljau with parameter
//               1/2, Sec. II-E), per-patch min/max, per-child feasibility flags
//               (Def. of feasibility), children written to slots 2j / 2j+1.
//   k_rederive  FP32 mode, every few steps: the children of a step derived
//               directly from the FP64 root patches by box id instead of from
//               the FP32 parents, which resets the carried rounding bound.
//   k_cut       Alg. CutOffTest + the infeasibility / stopping tests + Alg.
//               Eliminate as an order-preserving stream compaction + the advance
//               of direction and iteration count, one workgroup per problem.
//   k_certify   FP64 re-derivation of x* with a rigorous error bound.
#include <hip/hip_ext.h>

#include "kernels.h"

#include <float.h>
#include <math.h>

#include <mutex>
#include <vector>

namespace pcba {

// ------------------------------------------------------------------ small helpers

// A device pointer taken from a descriptor is generic to the compiler, and its
// loads and stores become FLAT instructions, which count on the LDS counter
// as well: a later wait for an LDS read then also waits for them, and loads
// issued early to overlap LDS work would complete before it.  Accesses
// through this view of the pointer are plain global-memory instructions.
template <typename T>
using gmem_t = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gmem_t<T> as_global(T* p)
{
    return (gmem_t<T>)p;
}
// the HIP vector classes cannot be copied out of a global-memory lvalue: the
// clang vector types of the same layout stand in for them
typedef int vec2i __attribute__((ext_vector_type(2)));
typedef int vec4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// block-wide min over blockDim.x (multiple of 64) threads; `sh` holds >= 16 doubles
__device__ double block_min(double v, double* sh)
{
    v = wave_min(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = (threadIdx.x < (unsigned)nw) ? sh[threadIdx.x] : INFINITY;
    if (w == 0) r = wave_min(r);
    __syncthreads();
    if (threadIdx.x == 0) sh[0] = r;
    __syncthreads();
    r = sh[0];
    __syncthreads();
    return r;
}
__device__ int block_min_i(int v, int* sh)
{
    v = wave_min_i(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    int r = (threadIdx.x < (unsigned)nw) ? sh[threadIdx.x] : INT_MAX;
    if (w == 0) r = wave_min_i(r);
    __syncthreads();
    if (threadIdx.x == 0) sh[0] = r;
    __syncthreads();
    r = sh[0];
    __syncthreads();
    return r;
}

// Min over the workgroup with one barrier: each wave's min to sh[w], then
// every thread reduces the waves' values.  A call site needs its own sh (or a
// barrier before sh is written again).
__device__ __forceinline__ double block_min1(double v, double* sh)
{
    v = wave_min(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r = fmin(r, sh[q]);
    return r;
}
__device__ __forceinline__ int block_min1_i(int v, int* sh)
{
    v = wave_min_i(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = sh[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r = min(r, sh[q]);
    return r;
}

// Tells the host that a problem left the running state (finished, or paused
// for list growth): one word of pinned host memory per engine, written with a
// vector store at system scope (null outside an engine).
__device__ __forceinline__ void signal_host(const DevInst& I)
{
    if (I.hostflag) __hip_atomic_store(I.hostflag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Units of work of one step, per class of problem:
//   class 0: FP64 problems (k_sub<double>)
//   class 1: FP32 problems splitting their FP32 parents (k_sub<float>)
//   class 2: FP32 problems whose step re-derives the children from the root
//   class 3: the transform rows of those problems (k_tmat, one thread per row)
// plan[c*(n+1) + b] = first unit of problem b in class c; plan[c*(n+1) + n] = total.
// What a step's plan reads of a problem's state, loaded at once (the fields
// share the state's first cache line) through a global-memory view.
struct PlanState {
    int32_t status, K, steps, cur, r;
    uint32_t epoch;
    double p_up;
    int64_t peak, u1, a_live;
};
__device__ __forceinline__ PlanState load_plan_state(const InstState* st)
{
    const gmem_t<const InstState> g = as_global(st);
    PlanState ps;
    ps.status = g->status;
    ps.K = g->K;
    ps.steps = g->steps;
    ps.cur = g->cur;
    ps.r = g->r;
    ps.epoch = g->epoch;
    ps.p_up = g->p_up;
    ps.peak = g->peak;
    ps.u1 = g->u1;
    ps.a_live = g->a_live;
    return ps;
}

__device__ __forceinline__ int unit_class(const DevInst& I, const PlanState& st)
{
    if (!I.fp32) return 0;
    const bool due = I.rederive > 0 && ((st.steps + 1) % I.rederive) == 0;
    return due ? 2 : 1;
}

// Tiles of k_sub in one step of a problem: the cost patches, the equality
// patches, then the inequality patches of all parents (all of them, or in
// retiring mode the carried ones), each cut into tiles of ptp[kind] patches.
__device__ __forceinline__ long long step_tiles(const DevInst& I, const PlanState& st)
{
    const long long K = st.K;
    const long long A = I.retire ? st.a_live : K * I.count[1];
    return (K + I.ptp[0] - 1) / I.ptp[0] + (K * I.count[2] + I.ptp[2] - 1) / I.ptp[2] +
           (A + I.ptp[1] - 1) / I.ptp[1];
}

// Units of one FP32 re-derivation step of a problem: every parent has one cost
// tile and its equality tiles; its inequality tiles are all of them, or in
// retiring mode as many as the inequalities it still carries need (their sum
// is the state's u1).
__device__ __forceinline__ long long step_units(const DevInst& I, const PlanState& st)
{
    const int T1 = I.tile_start[2] - I.tile_start[1];
    return I.retire ? (long long)st.K * (I.T - T1) + st.u1 : (long long)st.K * I.T;
}

// One problem's share of a step's plan: its units per class (v) and the
// snapshot of its state that the step's kernels use (si).  The memory test of
// Alg. PCBA runs at the start of the iteration: 2 length(L) > M (in a round
// 2^l length(L), the children it makes) ends the
// solve; more than the device list holds pauses the problem until the host
// grows the list.  With `commit` the outcome and the peak list length are
// stored in the state; a caller without it reaches the same decision from the
// same state (a status already moved off RUNNING gives no units either).
__device__ __forceinline__ void plan_one(const DevInst& I, bool commit, long long (&v)[4], StepInfo& si)
{
    const PlanState ps = load_plan_state(I.st);
    const gmem_t<InstState> st = as_global(I.st);
    v[0] = v[1] = v[2] = v[3] = 0;
    const int K = ps.K;
    const long long nc = I.fused ? (1 << I.l) : 2;   // children per parent
    if (ps.status == ST_RUNNING) {
        if (commit && (int64_t)K > ps.peak) st->peak = K;
        if (nc * K > (int64_t)I.M) {
            if (commit) {
                st->status = ST_MEMLIMIT;
                signal_host(I);
            }
        } else if (nc * K > (int64_t)I.cap || (I.retire && 2 * ps.a_live > I.hcap)) {
            if (commit) {
                st->status = ST_GROW;
                signal_host(I);
            }
        } else {
            const int c = unit_class(I, ps);
            v[c] = c == 2 ? step_units(I, ps) : step_tiles(I, ps);
            if (c == 2) v[3] = (long long)K * nc * I.rows;
        }
    }
    si.K = K;
    si.cur = ps.cur;
    si.r = ps.r;
    si.steps = ps.steps;
    si.p_up = ps.p_up;
    si.stamp = ps.epoch * 65536u + (uint32_t)ps.steps + 1u;   // step_stamp of the state
    si.A = (int)ps.a_live;
}

__global__ __launch_bounds__(1024) void k_plan(const DevInst* __restrict__ insts, int n,
                                               long long* __restrict__ plan,
                                               StepInfo* __restrict__ info)
{
    __shared__ long long wtot[4][16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
    long long carry[4] = {0, 0, 0, 0};
    for (int b0 = 0; b0 < n; b0 += blockDim.x) {
        const int b = b0 + t;
        long long v[4] = {0, 0, 0, 0};
        if (b < n) {
            StepInfo si;
            plan_one(insts[b], true, v, si);
            info[b] = si;
        }
        for (int c = 0; c < 4; ++c) {
            long long x = v[c];
            for (int o = 1; o < 64; o <<= 1) {
                long long y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (lane == 63) wtot[c][w] = x;
            v[c] = x - v[c];  // exclusive within the wave
        }
        __syncthreads();
        for (int c = 0; c < 4; ++c) {
            long long before = carry[c];
            for (int q = 0; q < w; ++q) before += wtot[c][q];
            if (b < n) plan[c * (n + 1) + b] = before + v[c];
            long long tot = 0;
            for (int q = 0; q < nw; ++q) tot += wtot[c][q];
            carry[c] += tot;
        }
        __syncthreads();
    }
    if (t < 4) plan[t * (n + 1) + n] = carry[t];
}

__device__ __forceinline__ int find_inst(const long long* __restrict__ pre, int n, long long u)
{
    int lo = 0, hi = n;  // pre[lo] <= u < pre[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= u) lo = mid; else hi = mid;
    }
    return lo;
}
// the same for a unit shared by the whole workgroup: the result is made
// wave-uniform so that the problem's descriptor and state are read through
// scalar loads
__device__ __forceinline__ int find_inst_uniform(const long long* __restrict__ pre, int n, long long u)
{
    return __builtin_amdgcn_readfirstlane(find_inst(pre, n, u));
}

// geometry of a fibre along axis r inside a patch of dims[0..l-1]
struct FibreGeom {
    int m, stride, F;
};
__device__ __forceinline__ FibreGeom fibre_geom(const int* dims, int l, int r, int S)
{
    FibreGeom g;
    g.m = dims[r];
    int s = 1;
    for (int k = r + 1; k < l; ++k) s *= dims[k];
    g.stride = s;
    g.F = S / g.m;
    return g;
}
// element offset (inside its patch) of the first coefficient of fibre q
__device__ __forceinline__ int fibre_base(const FibreGeom& g, int q)
{
    const int outer = q / g.stride, inner = q - outer * g.stride;
    return outer * g.m * g.stride + inner;
}

// The fibre geometry of every axis of one kind, staged once in LDS (by one
// thread) by kernels that walk the axes many times: the descriptor fields
// would otherwise be dependent global loads inside their loops.
struct AxisGeo {
    int m, stride, F, pad;
};
__device__ __forceinline__ void stage_geo(AxisGeo* g, const int* dims, int l, int S)
{
    int st = 1;
    for (int r = l - 1; r >= 0; --r) {
        const int m = dims[r];
        g[r].m = m;
        g[r].stride = st;
        g[r].F = m > 0 ? S / m : 0;
        g[r].pad = 0;
        st *= m;
    }
}

// One fibre of fixed length M transformed in place: out_k = sum_i T[k][i] x_i,
// the sum taken over i in increasing order; T row-major in LDS.
template <int M>
__device__ __forceinline__ void transform_fibre(double* __restrict__ x, int base, int stride,
                                                const double* __restrict__ T)
{
    double c[M];
#pragma unroll
    for (int i = 0; i < M; ++i) c[i] = x[base + i * stride];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < M; ++i) acc += T[k * M + i] * c[i];
        x[base + k * stride] = acc;
    }
}

__device__ __forceinline__ void transform_fibre_m(int m, double* x, int base, int stride, const double* T)
{
    switch (m) {
#define PCBA_TF_CASE(MV) \
    case MV: transform_fibre<MV>(x, base, stride, T); break;
        PCBA_TF_CASE(1) PCBA_TF_CASE(2) PCBA_TF_CASE(3) PCBA_TF_CASE(4)
        PCBA_TF_CASE(5) PCBA_TF_CASE(6) PCBA_TF_CASE(7) PCBA_TF_CASE(8)
        PCBA_TF_CASE(9) PCBA_TF_CASE(10) PCBA_TF_CASE(11) PCBA_TF_CASE(12)
        PCBA_TF_CASE(13) PCBA_TF_CASE(14) PCBA_TF_CASE(15) PCBA_TF_CASE(16)
#undef PCBA_TF_CASE
    default: break;
    }
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// `items` fibres of length m, fibre `it` at addr(it) with the given stride,
// each replaced in place by T x (T: m x m, row-major in LDS, FP64), on the
// matrix cores: each wave takes blocks of 16 fibres and runs ceil(m/4) steps
// of the 16x16x4 FP64 MFMA.  Lane (c, q) (c = lane % 16, q = lane / 16)
// supplies row c, column 4s + q of T and row 4s + q of fibre c, and receives
// rows q, q + 4, q + 8, q + 12 of the transformed fibre c.  Rows and columns
// beyond m are zero, so each output is a sum of the m products of its row, in
// some order: at most m roundings on any term's path (gamma_m, whatever the
// order).  A wave reads a block's fibres before it writes them and no other
// wave touches them.
template <typename Addr>
__device__ __forceinline__ void mfma_fibres_f64(int items, int m, int stride, const double* T, Addr addr)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int ks = (m + 3) >> 2;
    double a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int i = 4 * s + kq;
        a[s] = (col < m && i < m) ? T[col * m + i] : 0.0;
    }
    const int nblk = (items + 15) >> 4;
    for (int blk = w; blk < nblk; blk += nw) {
        const int it = blk * 16 + col;
        const bool v = it < items;
        double* x = v ? addr(it) : nullptr;
        double b[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = 4 * s + kq;
            b[s] = (s < ks && v && i < m) ? x[i * stride] : 0.0;
        }
        f64x4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (s < ks)   // uniform over the wave
                d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], d, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * q + kq;
            if (v && k < m) x[k * stride] = d[q];
        }
    }
}

// One axis of a run of polynomials staged in LDS slots (polynomial q of the
// run at slot + q * slot_stride, a second chain at + chain_off when nchain is
// 2): every (chain, polynomial, fibre) of the run is one work item of the
// block, whatever its kind, so that all lanes stay busy.  The run [pb, pe)
// spans at most the three kinds, whose polynomial indices are contiguous
// (c0 cost, then c1 inequalities, then equalities).  Each item applies the
// matrix at mats + mo.first[kind], then the one at mats + mo.second[kind] if
// that offset is not negative, to its fibre in place.  The matrices are given
// as offsets from the LDS array itself (not as pointers kept in a per-thread
// array), so that every read of them compiles to an LDS instruction.
struct MatOffs {
    int first[KINDS], second[KINDS];
};
template <bool MFMA>
__device__ __forceinline__ void run_axis(double* slot, int slot_stride, int chain_off, int nchain, int pb,
                                         int pe, int c0, int c1, const AxisGeo (*geo)[MAXL], int r,
                                         const double* mats, const MatOffs& mo)
{
#pragma unroll
    for (int kind = 0; kind < KINDS; ++kind) {
        const int lo = kind == 0 ? 0 : (kind == 1 ? c0 : c0 + c1);
        const int hi = kind == 0 ? c0 : (kind == 1 ? c0 + c1 : INT_MAX);
        const int q0 = max(pb, lo), q1 = min(pe, hi);
        if (q1 <= q0) continue;
        const AxisGeo ag = geo[kind][r];
        FibreGeom g;
        g.m = ag.m;
        g.stride = ag.stride;
        g.F = ag.F;
        // selects rather than an indexed read, which would place mo in scratch
        const int o0 = kind == 0 ? mo.first[0] : (kind == 1 ? mo.first[1] : mo.first[2]);
        const int o1 = kind == 0 ? mo.second[0] : (kind == 1 ? mo.second[1] : mo.second[2]);
        const double* T0 = mats + o0;
        const double* T1 = mats + o1;
        const bool two = o1 >= 0;
        const int per = g.F * nchain;
        const int items = (q1 - q0) * per;
        if (MFMA) {
            // every (polynomial, chain, fibre) of the kind with one matrix; the
            // second matrix, if any, in a second pass
            auto addr = [&](int it) {
                const int q = it / per, rem = it - q * per;
                const int ch = rem / g.F, f = rem - ch * g.F;
                return slot + (q0 - pb + q) * slot_stride + ch * chain_off + fibre_base(g, f);
            };
            mfma_fibres_f64(items, g.m, g.stride, T0, addr);
            if (two) mfma_fibres_f64(items, g.m, g.stride, T1, addr);
            continue;
        }
        for (int it = threadIdx.x; it < items; it += blockDim.x) {
            const int q = it / per, rem = it - q * per;
            const int ch = rem / g.F, f = rem - ch * g.F;
            double* x = slot + (q0 - pb + q) * slot_stride + ch * chain_off;
            const int base = fibre_base(g, f);
            transform_fibre_m(g.m, x, base, g.stride, T0);
            if (two) transform_fibre_m(g.m, x, base, g.stride, T1);
        }
    }
}

// gamma_m = m u / (1 - m u) with u = 2^-23 (covers unknown internal rounding)
__device__ __forceinline__ double gamma32(int m)
{
    const double mu = (double)m * 0x1p-23;
    return mu / (1.0 - mu);
}
__device__ __forceinline__ double gamma64(int m)
{
    const double mu = (double)m * 0x1p-53;
    return mu / (1.0 - mu) * 1.0000001;
}
__device__ __forceinline__ float round_up_f(double x)
{
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

// ------------------------------------------------------------------ k_root

// The problem of workgroup u: the host appends each workgroup's problem after
// the prefix of workgroup counts (pre[n + 1 + u]), one load instead of a search.
__device__ __forceinline__ int find_block(const int* __restrict__ pre, int n, int u)
{
    return pre[n + 1 + u];
}

__device__ __forceinline__ void poly_kind(const DevInst& I, int poly, int& kind, int& idx)
{
    kind = 0;
    idx = poly;
    if (idx >= I.count[0]) {
        idx -= I.count[0];
        kind = 1;
        if (idx >= I.count[1]) { idx -= I.count[1]; kind = 2; }
    }
}

// InitPatches: one workgroup per (problem, run of ppb polynomials), blocks of
// problem b are [pre[b], pre[b+1]).  Per axis r, the pre-map matrix A (x = lo +
// w t substituted) then the conversion matrix U are applied; every output
// coefficient sums over i in increasing order.  The result is the list's root
// item in FP64 plain mode (slot 0 of buffer 0) and is kept in `root`.  In FP32
// mode the root item is formed from the accurate root racc instead: its
// midrange as the FP64 base, FP32 offsets from it, and the bound root_err plus
// the offsets' rounding.
//   The workgroup stages the matrices of every kind and axis and the monomials
// of its run in LDS (loads all in flight at once); then each wave takes one
// polynomial per round, each lane whole fibres.  LDS (doubles): mat_words of
// matrices (A then U per kind and axis, the layout of `mats`), then ppb slots
// of max_S.
__global__ __launch_bounds__(256) void k_root(const DevInst* __restrict__ insts, int n,
                                             const int* __restrict__ pre, int max_S, int ppb,
                                             int mat_words)
{
    extern __shared__ double sh[];
    __shared__ AxisGeo s_geo[KINDS][MAXL];
    __shared__ int s_mo[KINDS][MAXL];
    const int bi = find_block(pre, n, blockIdx.x);
    const DevInst& I = insts[bi];
    const int l = I.l, nw = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int pb = (blockIdx.x - pre[bi]) * ppb;
    const int pe = min(I.n_polys, pb + ppb);
    const int c0 = I.count[0], c1 = I.count[1];
    const int S0 = I.S[0], S1 = I.S[1], S2 = I.S[2];
    const int64_t o0 = I.off[0], o1 = I.off[1], o2 = I.off[2];
    double* mats = sh;
    double* slot = sh + mat_words;
    int nmat = 0;
    for (int t = 0; t < KINDS; ++t)
        for (int r = 0; r < l; ++r) nmat += 2 * I.dims[t][r] * I.dims[t][r];
    // matrices and monomials of the run into LDS, up to 8 loads in flight per thread
    {
        const int total = nmat + (pe - pb) * max_S;
        for (int e0 = threadIdx.x; e0 < total; e0 += 8 * blockDim.x) {
            double v[8];
            int dst[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = e0 + k * blockDim.x;
                dst[k] = -1;
                if (e < nmat) {
                    v[k] = as_global(I.mats)[e];
                    dst[k] = e;
                } else if (e < total) {
                    const int q = (e - nmat) / max_S, i = (e - nmat) - q * max_S;
                    int idx = pb + q, kind = 0;
                    if (idx >= c0) {
                        idx -= c0;
                        kind = 1;
                        if (idx >= c1) { idx -= c1; kind = 2; }
                    }
                    const int S = kind == 0 ? S0 : (kind == 1 ? S1 : S2);
                    if (i < S) {
                        v[k] = as_global(I.mono)[(kind == 0 ? o0 : (kind == 1 ? o1 : o2)) + (int64_t)idx * S + i];
                        dst[k] = mat_words + q * max_S + i;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (dst[k] >= 0) sh[dst[k]] = v[k];
        }
    }
    if (threadIdx.x < KINDS) {
        const int t = threadIdx.x;
        stage_geo(s_geo[t], I.dims[t], l, I.S[t]);
        int o = 0;
        for (int t2 = 0; t2 < t; ++t2)
            for (int r = 0; r < l; ++r) o += 2 * I.dims[t2][r] * I.dims[t2][r];
        for (int r = 0; r < l; ++r) {
            s_mo[t][r] = o;
            o += 2 * I.dims[t][r] * I.dims[t][r];
        }
    }
    __syncthreads();
    for (int r = 0; r < l; ++r) {
        MatOffs mo;
        for (int t = 0; t < KINDS; ++t) {
            mo.first[t] = s_mo[t][r];
            mo.second[t] = s_mo[t][r] + s_geo[t][r].m * s_geo[t][r].m;
        }
        run_axis<false>(slot, max_S, 0, 1, pb, pe, c0, c1, s_geo, r, mats, mo);
        __syncthreads();
    }
    for (int p0 = pb; p0 < pe; p0 += nw) {
        const int poly = p0 + w;
        const bool act = poly < pe;
        int kind = 0, idx = poly;
        if (idx >= c0) {
            idx -= c0;
            kind = 1;
            if (idx >= c1) { idx -= c1; kind = 2; }
        }
        const int S = kind == 0 ? S0 : (kind == 1 ? S1 : S2);
        const int64_t off = (kind == 0 ? o0 : (kind == 1 ? o1 : o2)) + (int64_t)idx * S;
        double* x = slot + (poly - pb) * max_S;
        if (!act) continue;
        // the root item: slot 0 of buffer 0, or in retiring mode for an
        // inequality its heap patch idx
        const bool inheap = I.retire && kind == 1;
        void* dbase = inheap ? I.heap[0] : I.buf[0];
        const int64_t doff = inheap ? (int64_t)idx * S : I.soff[kind] + (int64_t)idx * S;
        if (I.root)   // the readback copy, written by the problem's first reset only
            for (int e = lane; e < S; e += 64) as_global(I.root)[off + e] = x[e];
        if (!I.fp32) {
            for (int e = lane; e < S; e += 64) as_global((double*)dbase)[doff + e] = x[e];
            if (lane == 0 && inheap) {
                I.act[0][idx] = make_int2(idx, idx);
                I.pmap[idx] = make_int4(0, 0, idx, idx);
            }
            continue;
        }
        // FP32: offsets from the midrange of the accurate root patch
        const double* ra = I.racc + off;
        double mn = INFINITY, mx = -INFINITY;
        for (int e = lane; e < S; e += 64) {
            mn = fmin(mn, ra[e]);
            mx = fmax(mx, ra[e]);
        }
        for (int o = 32; o > 0; o >>= 1) {
            mn = fmin(mn, __shfl_xor(mn, o, 64));
            mx = fmax(mx, __shfl_xor(mx, o, 64));
        }
        const double pbase = 0.5 * mn + 0.5 * mx;
        double hr = 0.0;
        for (int e = lane; e < S; e += 64) {
            const float d = (float)(ra[e] - pbase);
            hr = fmax(hr, fabs((double)d));
            ((float*)dbase)[doff + e] = d;
        }
        for (int o = 32; o > 0; o >>= 1) hr = fmax(hr, __shfl_xor(hr, o, 64));
        if (lane == 0) {
            if (inheap) {
                I.act[0][idx] = make_int2(idx, idx);
                I.pmap[idx] = make_int4(0, 0, idx, idx);
            }
            // the accurate root's bound, the rounding of the offsets (the FP64
            // difference and the conversion, 2^-23 of the largest), underflow
            I.err[0][poly] = make_float2(round_up_f(I.root_err[poly] + hr * 0x1p-23 + 0x1p-126), 0.0f);
            I.base[0][poly] = pbase;
        }
    }
}

// The accurate root, once per problem: per axis r one product with the
// combined matrix M (Bernstein coefficients on [lo, hi] of each monomial,
// formed by the polar form: M[k][j] is the average of lo^(j-i) hi^i over the
// hypergeometric weights C(k,i) C(n-k,j-i) / C(n,j), so no entry suffers
// cancellation), then the same chain on |coefficients| with Mabs (the sums of
// the terms' magnitudes).  Each entry of M is within gamma_46 Mabs of the exact
// one (at most 31 roundings per term, 15 in the sum) and each product adds
// gamma_m, so root_err = gamma_q times the |.| chain, q summing 47 + m per axis
// plus a few, is a rigorous bound on |racc - exact|.
__global__ __launch_bounds__(256) void k_racc(const DevInst* __restrict__ insts, int n,
                                             const int* __restrict__ pre)
{
    extern __shared__ double sh[];
    __shared__ double red[8];
    const int bi = find_block(pre, n, blockIdx.x);
    const DevInst& I = insts[bi];
    const int poly = blockIdx.x - pre[bi];
    int kind, idx;
    poly_kind(I, poly, kind, idx);
    const int S = I.S[kind];
    const int64_t off = I.off[kind] + (int64_t)idx * S;
    double* x = sh;
    double* y = sh + S;
    int q = 4;
    double amax = 0.0, rmax = 0.0;
    for (int absp = 0; absp < 2; ++absp) {
        for (int e = threadIdx.x; e < S; e += blockDim.x) x[e] = absp ? fabs(I.mono[off + e]) : I.mono[off + e];
        __syncthreads();
        for (int r = 0; r < I.l; ++r) {
            FibreGeom g = fibre_geom(I.dims[kind], I.l, r, S);
            const double* Mx = I.macc + I.matoff[kind * MAXL + r] + (absp ? g.m * g.m : 0);
            if (absp) q += 47 + g.m;
            for (int o = threadIdx.x; o < S; o += blockDim.x) {
                const int k = (o / g.stride) % g.m;
                const int fb = o - k * g.stride;
                double acc = 0.0;
                for (int i = 0; i < g.m; ++i) acc += Mx[k * g.m + i] * x[fb + i * g.stride];
                y[o] = acc;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < S; e += blockDim.x) x[e] = y[e];
            __syncthreads();
        }
        for (int e = threadIdx.x; e < S; e += blockDim.x) {
            if (absp) amax = fmax(amax, x[e]);
            else {
                I.racc[off + e] = x[e];
                rmax = fmax(rmax, fabs(x[e]));
            }
        }
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) {
        amax = fmax(amax, __shfl_xor(amax, o, 64));
        rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = amax;
        red[4 + (threadIdx.x >> 6)] = rmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            amax = fmax(amax, red[w]);
            rmax = fmax(rmax, red[4 + w]);
        }
        // the |.| chain is itself rounded (below gamma_q relative): 1.01
        I.root_err[poly] = gamma64(q) * amax * 1.01;
        I.root_abs[poly] = rmax;
    }
}

// Initial solver state of every problem: L = {root item}, n = 1, r = first
// direction, p_up = p_lo = +inf.
__global__ void k_reset(const DevInst* __restrict__ insts, int n)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const DevInst& I = insts[b];
    InstState* st = I.st;
    st->status = ST_RUNNING;
    st->K = 1;
    {
        const int d0[MAXL] = {};
        st->r = I.rule == 1 ? widest_axis(I.width0, I.lam, d0, I.l) : 0;
    }
    st->n = 1;
    st->steps = 0;
    st->cur = 0;
    st->has_x = 0;
    st->cert_ok = 0;
    st->p_up = INFINITY;
    st->p_lo = INFINITY;
    for (int k = 0; k < MAXL; ++k) { st->depth[k] = 0; st->x_index[k] = 0; st->x_depth[k] = 0; }
    st->peak = 0;
    st->p_cert = INFINITY;
    st->cert_err = 0.0;
    st->err_max = 0.0;
    st->epoch = st->epoch + 1u;
    const int T1 = I.tile_start[2] - I.tile_start[1];
    st->u1 = T1;
    st->a_live = I.count[1];
    st->htop[0] = I.retire ? I.count[1] : 0;
    st->htop[1] = 0;
    if (I.retire) {
        I.na[0][0] = I.count[1];
        I.na[1][0] = 0;
        I.na[1][1] = 0;
        I.upre[0] = 0;
        I.upre[1] = T1;
        for (int q = 0; q < T1; ++q) I.umap[q] = make_int4(0, 0, q, I.count[1]);
    }
    I.live[0] = 0;
    for (int k = 0; k < I.l; ++k) I.ids[0][k] = 0;
    I.flags[0] = 0;
    I.flags[1] = 0;
}

// ------------------------------------------------------------------ k_sub
//
// Work units of k_sub are tiles of consecutive patches of one kind of one
// problem, taken from the patches of all its parents in parent order: the cost
// patches (one per parent), then the equality patches (beta per parent), then
// the inequality patches (alpha per parent, or in retiring mode each parent's
// carried ones).  A tile therefore spans several parents when their patches
// are few, which with retiring is the common case: units are full tiles
// instead of one short tile per parent.  Per patch the workgroup stages in LDS
// its parent j, the parent's slot, its index in its kind and where its
// coefficients are.

// One fibre of fixed length M: de Casteljau with parameter 1/2 in registers.
// After level lev, c[0] is the left child's coefficient lev and c[M-1-lev] the
// right child's coefficient M-1-lev.  The left child overwrites the parent in
// buffer a (every fibre belongs to one thread), the right child goes to b.
template <typename T, int M>
__device__ __forceinline__ void split_fibre(T* __restrict__ a, T* __restrict__ b, int base,
                                            int stride, T s0, T& mnL, T& mxL, T& mnR, T& mxR, T& amax)
{
    T c[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        c[i] = a[base + i * stride];
        if constexpr (sizeof(T) == 4) c[i] -= s0;   // FP32: less the pending shift
        amax = fmax(amax, fabs(c[i]));
    }
    mnL = mxL = c[0];
    mnR = mxR = c[M - 1];
    if constexpr (sizeof(T) == 4) a[base] = c[0];   // the left child's first coefficient, shifted
    b[base + (M - 1) * stride] = c[M - 1];
#pragma unroll
    for (int lev = 1; lev < M; ++lev) {
#pragma unroll
        for (int i = 0; i + lev < M; ++i) c[i] = (c[i] + c[i + 1]) * (T)0.5;
        a[base + lev * stride] = c[0];
        b[base + (M - 1 - lev) * stride] = c[M - 1 - lev];
        mnL = fmin(mnL, c[0]);
        mxL = fmax(mxL, c[0]);
        mnR = fmin(mnR, c[M - 1 - lev]);
        mxR = fmax(mxR, c[M - 1 - lev]);
    }
}

// The same fibre split at parameter lam (the box [a,b] becomes [a, a + lam (b-a)]
// and the rest): c_i <- (1 - lam) c_i + lam c_{i+1}, products and sum in the
// order the oracle takes them.
template <typename T, int M>
__device__ __forceinline__ void split_fibre_at(T* __restrict__ a, T* __restrict__ b, int base, int stride, T s0,
                                               T lam, T& mnL, T& mxL, T& mnR, T& mxR, T& amax)
{
    const T mu = (T)1 - lam;
    T c[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        c[i] = a[base + i * stride];
        if constexpr (sizeof(T) == 4) c[i] -= s0;   // FP32: less the pending shift
        amax = fmax(amax, fabs(c[i]));
    }
    mnL = mxL = c[0];
    mnR = mxR = c[M - 1];
    if constexpr (sizeof(T) == 4) a[base] = c[0];   // the left child's first coefficient, shifted
    b[base + (M - 1) * stride] = c[M - 1];
#pragma unroll
    for (int lev = 1; lev < M; ++lev) {
#pragma unroll
        for (int i = 0; i + lev < M; ++i) c[i] = mu * c[i] + lam * c[i + 1];
        a[base + lev * stride] = c[0];
        b[base + (M - 1 - lev) * stride] = c[M - 1 - lev];
        mnL = fmin(mnL, c[0]);
        mxL = fmax(mxL, c[0]);
        mnR = fmin(mnR, c[M - 1 - lev]);
        mxR = fmax(mxR, c[M - 1 - lev]);
    }
}

// Barrier for LDS data only: waits for this wave's LDS operations, not for its
// global stores, which stay in flight across the barrier.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// global -> LDS copy with LB independent loads in flight per thread
template <typename T, int LB = 12>
__device__ __forceinline__ void copy_to_lds(T* __restrict__ dst, const T* __restrict__ src, int n)
{
    for (int e0 = threadIdx.x; e0 < n; e0 += LB * blockDim.x) {
        T v[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = e0 + q * blockDim.x;
            if (e < n) v[q] = src[e];
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = e0 + q * blockDim.x;
            if (e < n) dst[e] = v[q];
        }
    }
}

// Splits the staged tile (np patches of S coefficients at a) along the fibres
// of geometry g: left child in place in a, right child in b, per-patch min/max
// of both children and max |parent| folded into key.  With sh (FP32), patch p
// is split as its values less sh[p].  Callers follow with lds_barrier().
template <typename T, int MM>
__device__ __forceinline__ void tile_split(int np, int S, const FibreGeom& g, T* a, T* b,
                                           typename KeyOf<T>::type* key, double lam, const T* sh)
{
    const bool mid = lam == 0.5;
    const int TF = np * g.F;
    // quotients by reciprocals, exact for dividends below 2^22 (see patch_of)
    const float invF = 1.0f / (float)g.F, invT = 1.0f / (float)g.stride;
    for (int f = threadIdx.x; f < TF; f += blockDim.x) {
        const int p = (int)(((float)f + 0.5f) * invF);
        const int q = f - p * g.F;
        const int outer = (int)(((float)q + 0.5f) * invT);
        const int base = p * S + outer * g.m * g.stride + (q - outer * g.stride);
        T mnL, mxL, mnR, mxR, amax = (T)0;
        const T s0 = sh ? sh[p] : (T)0;
        switch (g.m) {
#define PCBA_SPLIT_CASE(MV)                                                                          \
        case MV:                                                                                     \
            if (MV <= MM) {                                                                          \
                if (mid)                                                                             \
                    split_fibre<T, MV>(a, b, base, g.stride, s0, mnL, mxL, mnR, mxR, amax);          \
                else                                                                                 \
                    split_fibre_at<T, MV>(a, b, base, g.stride, s0, (T)lam, mnL, mxL, mnR, mxR, amax); \
            }                                                                                        \
            break;
            PCBA_SPLIT_CASE(1) PCBA_SPLIT_CASE(2) PCBA_SPLIT_CASE(3) PCBA_SPLIT_CASE(4)
            PCBA_SPLIT_CASE(5) PCBA_SPLIT_CASE(6) PCBA_SPLIT_CASE(7) PCBA_SPLIT_CASE(8)
            PCBA_SPLIT_CASE(9) PCBA_SPLIT_CASE(10) PCBA_SPLIT_CASE(11) PCBA_SPLIT_CASE(12)
            PCBA_SPLIT_CASE(13) PCBA_SPLIT_CASE(14) PCBA_SPLIT_CASE(15) PCBA_SPLIT_CASE(16)
#undef PCBA_SPLIT_CASE
        default: mnL = mxL = mnR = mxR = (T)0; break;
        }
        atomicMin(&key[5 * p + 0], fkey(mnL));
        atomicMax(&key[5 * p + 1], fkey(mxL));
        atomicMin(&key[5 * p + 2], fkey(mnR));
        atomicMax(&key[5 * p + 3], fkey(mxR));
        atomicMax(&key[5 * p + 4], fkey(amax));
    }
}

// C(n, k) in FP32, exact for n <= 15 (every partial product is an integer
// below 2^17 and every division is exact)
__device__ __forceinline__ float binom_f(int n, int k)
{
    if (k < 0 || k > n) return 0.0f;
    float c = 1.0f;
    for (int i = 1; i <= k; ++i) c = c * (float)(n - k + i) / (float)i;
    return c;
}

// Entries of the midpoint subdivision matrices of Sec. II-E for fibres of
// length m (degree n = m - 1), row k (child coefficient) and column i (parent
// coefficient): the left half's coefficient k is sum_{i <= k} C(k,i) 2^-k b_i,
// the right half's sum_{i >= k} C(n-k, i-k) 2^-(n-k) b_i.  The entries are
// dyadic with numerators below 2^13, so exact in FP32; rows are non-negative
// and sum to one.
__device__ __forceinline__ float split_left(int m, int k, int i)
{
    return (k < m && i <= k) ? ldexpf(binom_f(k, i), -k) : 0.0f;
}
__device__ __forceinline__ float split_right(int m, int k, int i)
{
    const int n = m - 1;
    return (k < m && i >= k && i < m) ? ldexpf(binom_f(n - k, i - k), -(n - k)) : 0.0f;
}
// At a subdivision parameter lam: left row k holds C(k,i) lam^i (1-lam)^(k-i),
// right row k holds C(n-k, i-k) lam^(i-k) (1-lam)^(n-i); formed in FP64 and
// rounded to FP32 (relative error below 2^-24 per entry).
__device__ __forceinline__ double pow_i(double x, int e)
{
    double r = 1.0;
    for (int t = 0; t < e; ++t) r *= x;
    return r;
}
__device__ __forceinline__ float split_left_at(int m, int k, int i, double lam)
{
    return (k < m && i <= k) ? (float)((double)binom_f(k, i) * pow_i(lam, i) * pow_i(1.0 - lam, k - i)) : 0.0f;
}
__device__ __forceinline__ float split_right_at(int m, int k, int i, double lam)
{
    const int n = m - 1;
    return (k < m && i >= k && i < m)
               ? (float)((double)binom_f(n - k, i - k) * pow_i(lam, i - k) * pow_i(1.0 - lam, n - i))
               : 0.0f;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// FP32 tiles: the split as a fixed-matrix contraction on the matrix cores.
// The fibres of the tile along direction r are the columns of X (m x TF); the
// children are S_L X and S_R X, computed together as one product with the
// stacked matrix [S_L; S_R] (rows 0..15 the left child's coefficients, rows
// 16..31 the right child's).  Each wave takes blocks of 32 fibres and runs
// ceil(m/2) steps of the 32x32x2 FP32 MFMA: lane (c, q) (c = lane % 32,
// q = lane / 32) supplies row c, column 2s + q of the stacked matrix and row
// 2s + q of fibre c, and receives rows 8h + 4q .. 8h + 4q + 3 (h = 0..3) of
// the product for fibre c, so the two lanes of a fibre hold all of its
// children's coefficients between them.  Rows and columns beyond m are zero,
// so every output sums exactly the m products of its row.  Results go back as
// tile_split leaves them (with sh, patch p's values less sh[p] are split): the
// left child in place in a, the right child in b,
// per-patch min/max of both children and max |parent| folded into key.  A wave
// reads a block's fibres before it writes them and no other wave touches
// them, so the in-place write is safe.
// Rounding: each output is a sum of m products with non-negative weights
// summing to one, evaluated in some order with at most m roundings on any
// term's path, so |c~ - c| <= gamma_m max |b| (with u = 2^-23, covering the
// unit's internal rounding) plus m 2^-126 for flushed subnormals: the bound
// the caller carries for the split.
__device__ __forceinline__ void tile_split_mfma(int np, int S, const FibreGeom& g, float* a, float* b,
                                                unsigned* key, double lam, const float* sh)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int col = lane & 31, kq = lane >> 5;
    const int m = g.m, ks = (m + 1) >> 1;
    // this lane's entries of the stacked matrix: row col, columns 2s + kq
    float aS[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int i = 2 * s + kq;
        const int row = col & 15;
        const bool right = col >= 16;
        aS[s] = lam == 0.5 ? (right ? split_right(m, row, i) : split_left(m, row, i))
                           : (right ? split_right_at(m, row, i, lam) : split_left_at(m, row, i, lam));
    }
    const int TF = np * g.F;
    const int nblk = (TF + 31) >> 5;
    const float invF = 1.0f / (float)g.F;
    for (int blk = w; blk < nblk; blk += nw) {
        const int f = blk * 32 + col;
        const bool fv = f < TF;
        int p = 0, base = 0;
        if (fv) {
            p = (int)(((float)f + 0.5f) * invF);   // f / F (exact: f < 2^22)
            base = p * S + fibre_base(g, f - p * g.F);
        }
        float x[8];
        float amax = 0.0f;
        const float s0 = (fv && sh) ? sh[p] : 0.0f;   // the patch's pending shift
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int i = 2 * s + kq;
            x[s] = (s < ks && fv && i < m) ? a[base + i * g.stride] - s0 : 0.0f;
            amax = fmaxf(amax, fabsf(x[s]));
        }
        f32x16 d = {};
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (s < ks)   // uniform over the wave
                d = __builtin_amdgcn_mfma_f32_32x32x2f32(aS[s], x[s], d, 0, 0, 0);
        float mnL = INFINITY, mxL = -INFINITY, mnR = INFINITY, mxR = -INFINITY;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int row = 8 * (q >> 2) + 4 * kq + (q & 3);
            const int k = row & 15;
            if (fv && k < m) {
                if (row < 16) {
                    a[base + k * g.stride] = d[q];
                    mnL = fminf(mnL, d[q]);
                    mxL = fmaxf(mxL, d[q]);
                } else {
                    b[base + k * g.stride] = d[q];
                    mnR = fminf(mnR, d[q]);
                    mxR = fmaxf(mxR, d[q]);
                }
            }
        }
        // the two lanes of a fibre (lane and lane ^ 32)
        mnL = fminf(mnL, __shfl_xor(mnL, 32, 64));
        mxL = fmaxf(mxL, __shfl_xor(mxL, 32, 64));
        mnR = fminf(mnR, __shfl_xor(mnR, 32, 64));
        mxR = fmaxf(mxR, __shfl_xor(mxR, 32, 64));
        amax = fmaxf(amax, __shfl_xor(amax, 32, 64));
        if (fv && kq == 0) {
            atomicMin(&key[5 * p + 0], fkey(mnL));
            atomicMax(&key[5 * p + 1], fkey(mxL));
            atomicMin(&key[5 * p + 2], fkey(mnR));
            atomicMax(&key[5 * p + 3], fkey(mxR));
            atomicMax(&key[5 * p + 4], fkey(amax));
        }
    }
}

__device__ __forceinline__ long long uniform64(long long x)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(x & 0xffffffffll));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)x >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Unit v of a problem with K parents: the K cost tiles first (so that the cost
// bounds of most children are recorded before their constraint tiles start),
// then the equality tiles parent by parent, then the inequality tiles parent by
// parent.  In retiring mode parent j owns inequality units [upre[j], upre[j+1]),
// and the unit map gives, per inequality unit, the parent, its slot and its
// carried count as well (slot and na; -1 where not known here).  t is the tile
// index in item terms: an inequality tile t covers positions
// (t - tile_start[1]) * tile_polys[1] ... of the parent's carried list.
__device__ __forceinline__ void unit_of(const DevInst& I, long long v, int K, int& j, int& t, int& slot,
                                        int& na)
{
    slot = -1;
    na = -1;
    const int T1 = I.tile_start[2] - I.tile_start[1];
    const int T2 = I.T - I.tile_start[2];
    if (v < K) {
        j = (int)v;
        t = 0;
        return;
    }
    v -= K;
    if (v < (long long)K * T2) {
        j = (int)(v / T2);
        t = I.tile_start[2] + (int)(v - (long long)j * T2);
        return;
    }
    v -= (long long)K * T2;
    if (!I.retire) {
        j = (int)(v / T1);
        t = I.tile_start[1] + (int)(v - (long long)j * T1);
        return;
    }
    // the unit map that k_cut wrote: parent, its slot, tile, carried count
    // (v is uniform over the workgroup, so is the entry)
    const int4 m = I.umap[v];
    j = __builtin_amdgcn_readfirstlane(m.x);
    t = I.tile_start[1] + __builtin_amdgcn_readfirstlane(m.z);
    slot = __builtin_amdgcn_readfirstlane(m.y);
    na = __builtin_amdgcn_readfirstlane(m.w);
}

// Patch index of element e of a tile of patches of S coefficients: e / S,
// exact for e + S < 2^22 (the float quotient of e + 1/2 stays within 1/(2S)
// of its integer part plus one half).
__device__ __forceinline__ int patch_of(int e, float invS)
{
    return (int)(((float)e + 0.5f) * invS);
}

// Bounds of one patch of a child in FP64.  FP64 plain mode (e == 0): the
// exact min and max.  FP32 mode: the patch is base + stored values, and the
// bounds are widened by the carried error e and by the rounding of the FP64
// sums (below 2^-53 relative each), then one ulp outward.
template <typename T>
__device__ __forceinline__ void child_bounds(T mn, T mx, double e, double base, double& lo, double& hi)
{
    if (e == 0.0) {
        lo = (double)mn;
        hi = (double)mx;
    } else {
        const double a = base + (double)mn, b = base + (double)mx;
        lo = nextafter(a - e - fabs(a) * 0x1p-52, -INFINITY);
        hi = nextafter(b + e + fabs(b) * 0x1p-52, INFINITY);
    }
}

// One tile of k_sub (all fields uniform over the workgroup).
struct PackUnit {
    int bi, kind, np, S, TE, cur, r, gath;
    int contig;       // the tile's patches are consecutive patches of one parent
    int nc;           // children per parent: 2, or 2^l = 4 when the step is a round
    long long P0;     // first patch of the tile in the problem's sequence of this kind
    float invS;
    double pprev;
    uint32_t stamp;
    FibreGeom g;      // fibres of the split (a round: of axis 0)
    FibreGeom g2;     // a round: fibres of axis 1
    long long u;      // the unit, and the end of its problem's units of this kind
    long long ukend;
    long long total;  // patches of this kind in the problem's step
    int ptp, cnt;     // patches per tile of the kind; patches of the kind per parent
};

// a / b for a >= 0 and 0 < b < 2^31: a 32-bit division when a fits (the usual
// case), the 64-bit one otherwise
__device__ __forceinline__ long long div_nn(long long a, int b)
{
    return a < 0x100000000ll ? (long long)((unsigned)a / (unsigned)b) : a / b;
}

// Resolves unit u: the problem (hint only moves forward, since a block's
// units increase), the kind and the tile's first patch.  Per problem the
// units are ceil(K / ptp0) cost tiles, ceil(K beta / ptp2) equality tiles,
// then ceil(A / ptp1) inequality tiles, A the patches the parents carry.
__device__ __forceinline__ void resolve_packed(const DevInst* __restrict__ insts, int n,
                                               const long long* pre, const StepInfo* info, long long u,
                                               int& hint, PackUnit& c)
{
    if (pre[hint + 1] <= u) {
        int lo = hint + 1, hi = n;  // pre[lo] <= u < pre[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= u) lo = mid; else hi = mid;
        }
        hint = lo;
    }
    hint = __builtin_amdgcn_readfirstlane(hint);
    const DevInst& I = insts[hint];
    const StepInfo si = info[hint];
    c.bi = hint;
    long long v = u - pre[hint];
    const long long K = si.K;
    long long total;
    const long long U0 = div_nn(K + I.ptp[0] - 1, I.ptp[0]);
    if (v < U0) {
        c.kind = 0;
        total = K;
    } else {
        v -= U0;
        const long long n2 = K * I.count[2];
        const long long U2 = div_nn(n2 + I.ptp[2] - 1, I.ptp[2]);
        if (v < U2) {
            c.kind = 2;
            total = n2;
        } else {
            v -= U2;
            c.kind = 1;
            total = I.retire ? (long long)si.A : K * I.count[1];
        }
    }
    // the end of this kind's units (the next unit of the same kind continues
    // from this one: resolve_next)
    {
        const long long U = div_nn(total + I.ptp[c.kind] - 1, I.ptp[c.kind]);
        c.ukend = uniform64(u - v + U);
    }
    c.u = u;
    c.total = total;
    c.ptp = I.ptp[c.kind];
    c.cnt = c.kind == 0 ? 1 : I.count[c.kind];
    c.P0 = uniform64(v * I.ptp[c.kind]);
    c.np = __builtin_amdgcn_readfirstlane((int)min((long long)I.ptp[c.kind], total - c.P0));
    c.cur = si.cur;
    c.r = si.r;
    c.pprev = si.p_up;
    c.stamp = si.stamp;
    c.S = I.S[c.kind];
    c.invS = 1.0f / (float)c.S;
    c.TE = c.np * c.S;
    c.gath = I.retire && c.kind == 1;
    // without the heap, a parent's patches of a kind are consecutive in its
    // slot: a tile within one parent is one run of coefficients
    c.contig = !c.gath && div_nn(c.P0, c.cnt) == div_nn(c.P0 + c.np - 1, c.cnt);
    c.nc = I.fused ? (1 << I.l) : 2;
    if (c.nc == 4) {
        c.g = fibre_geom(I.dims[c.kind], I.l, 0, c.S);
        c.g2 = fibre_geom(I.dims[c.kind], I.l, 1, c.S);
    } else {
        c.g = fibre_geom(I.dims[c.kind], I.l, I.fused ? 0 : c.r, c.S);
        c.g2 = c.g;
    }
}

// Unit u when it follows `prev` (u = prev.u + 1) in the same problem and kind
// (a workgroup's units are consecutive): the next tile of the same patch
// sequence, without resolving it again; otherwise resolve_packed.
__device__ __forceinline__ void resolve_next(const DevInst* __restrict__ insts, int n, const long long* pre,
                                             const StepInfo* info, long long u, int& hint, const PackUnit& prev,
                                             PackUnit& c)
{
    if (u == prev.u + 1 && u < prev.ukend) {
        c = prev;
        c.u = u;
        c.P0 = uniform64(prev.P0 + prev.ptp);
        c.np = __builtin_amdgcn_readfirstlane((int)min((long long)prev.ptp, prev.total - c.P0));
        c.TE = c.np * c.S;
        c.contig = !c.gath && div_nn(c.P0, c.cnt) == div_nn(c.P0 + c.np - 1, c.cnt);
        return;
    }
    resolve_packed(insts, n, pre, info, u, hint, c);
}

// Patch p of a tile: its parent j, the parent's slot, its index in its kind,
// and the element offset of its coefficients in the source (the slot buffer,
// or in retiring mode for inequalities the heap).  Lanes p < np only.
__device__ __forceinline__ void patch_info(const DevInst& I, const PackUnit& c, int p, int4& inf,
                                           long long& src)
{
    const long long P = c.P0 + p;
    if (c.gath) {
        const vec4i m = ((gmem_t<const vec4i>)I.pmap)[P];
        inf = make_int4(m.x, m.y, m.z, 0);
        src = (long long)m.w * c.S;
        return;
    }
    const int cnt = c.kind == 0 ? 1 : I.count[c.kind];
    const int j = (int)div_nn(P, cnt), id = (int)(P - (long long)j * cnt);
    const int slot = as_global(I.live)[j];
    inf = make_int4(j, slot, id, 0);
    src = (long long)slot * I.stride + I.soff[c.kind] + (long long)id * c.S;
}

// Issues the global loads of a tile into registers; the patches' source
// offsets come from LDS.  The offsets are read first and the loads then issued
// back to back; the buffer's address is made wave-uniform (it is), so no load
// waits on the one before it.
template <typename T, int LB>
__device__ __forceinline__ void issue_packed(const DevInst& I, const PackUnit& c, const long long* src,
                                             T (&v)[LB])
{
    const unsigned long long bu = (unsigned long long)(c.gath ? I.heap[c.cur] : I.buf[c.cur]);
    const unsigned blo = __builtin_amdgcn_readfirstlane((unsigned)bu);
    const unsigned bhi = __builtin_amdgcn_readfirstlane((unsigned)(bu >> 32));
    const gmem_t<const T> base = as_global((const T*)(((unsigned long long)bhi << 32) | blo));
    long long o[LB];
    if (c.contig) {
        const long long s0 = uniform64(src[0]);
#pragma unroll
        for (int q = 0; q < LB; ++q) o[q] = s0 + min((int)threadIdx.x + q * SUB_THREADS, max(c.TE - 1, 0));
    } else {
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = min((int)threadIdx.x + q * SUB_THREADS, max(c.TE - 1, 0));
            const int p = patch_of(e, c.invS);
            o[q] = src[p] + (e - p * c.S);
        }
    }
#pragma unroll
    for (int q = 0; q < LB; ++q)
        if ((int)threadIdx.x + q * SUB_THREADS < c.TE) v[q] = base[o[q]];
}

// Exclusive scans over the workgroup of three counts per thread at once;
// returns the totals.  sc: LDS of 3 * (waves) ints.  Every thread calls it.
__device__ __forceinline__ int3 block_scan3(int3 x, int3& excl, int* sc)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int a = x.x, b = x.y, d = x.z;
    for (int o = 1; o < 64; o <<= 1) {
        const int ya = __shfl_up(a, o, 64), yb = __shfl_up(b, o, 64), yd = __shfl_up(d, o, 64);
        if (lane >= o) { a += ya; b += yb; d += yd; }
    }
    if (lane == 63) { sc[3 * w] = a; sc[3 * w + 1] = b; sc[3 * w + 2] = d; }
    lds_barrier();
    int3 before = make_int3(0, 0, 0), tot = make_int3(0, 0, 0);
    for (int q = 0; q < nw; ++q) {
        if (q < w) { before.x += sc[3 * q]; before.y += sc[3 * q + 1]; before.z += sc[3 * q + 2]; }
        tot.x += sc[3 * q];
        tot.y += sc[3 * q + 1];
        tot.z += sc[3 * q + 2];
    }
    lds_barrier();
    excl = make_int3(before.x + a - x.x, before.y + b - x.y, before.z + d - x.z);
    return tot;
}

// k_sub: one tile per workgroup at a time, software-pipelined: while a tile is
// split in LDS, the next tile's patch table is loaded and then its
// coefficients are in flight in registers.  Dynamic LDS, for tiles of at most
// tem coefficients and tpm patches (tpm <= SUB_THREADS: patch p is thread p's):
// the tile and the right child (tem each), the keys (5 tpm), two patch tables
// (source offsets, then (j, slot, index)), the FP32 shifts (2 tpm), then per
// patch or segment: write masks, scan values, heap patches, flags, positions,
// segment starts.
//
// With FUSE (at most PLAN_FUSE_MAX problems) the step's plan is not read
// from k_plan's output but formed by every workgroup in LDS from the problems'
// states (one thread per problem); workgroup 0 alone commits the memory test's
// outcome and writes the plan and snapshots for the step's later kernels.
// Returns whether the step has units of this launch's class at all.
// MF: FP32 problems may split on the matrix cores (the matrix-core code is
// compiled in only then, so that the vector-ALU form keeps its registers).
template <typename T, int MM, int LB, bool FUSE, bool MF>
__device__ __forceinline__ bool sub_run(const DevInst* __restrict__ insts, int n_inst,
                                        long long* __restrict__ plan, StepInfo* __restrict__ info, int tem,
                                        int tpm, int nr)
{
    typedef typename KeyOf<T>::type K;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_pre[PLAN_FUSE_MAX + 1];
    __shared__ StepInfo s_info[PLAN_FUSE_MAX];
    __shared__ long long s_wt[4][SUB_THREADS / 64];
    __shared__ int s_sc[3 * (SUB_THREADS / 64)];
    __shared__ int s_nseg;
    __shared__ long long s_hb;

    const bool fp32 = sizeof(T) == 4;
    const int cls = fp32 ? 1 : 0;
    const long long* pre = plan + cls * (n_inst + 1);
    const StepInfo* sinfo = info;
    if (FUSE) {
        // one thread per problem: its share of the plan, then workgroup scans of
        // the four classes (wave scans, then the waves' totals through LDS)
        const int b = threadIdx.x, lane = b & 63, w = b >> 6;
        const bool commit = blockIdx.x == 0;
        long long v[4] = {0, 0, 0, 0};
        if (b < n_inst) {
            StepInfo si;
            plan_one(insts[b], commit, v, si);
            s_info[b] = si;
            if (commit) info[b] = si;
        }
        long long x[4];
        for (int c = 0; c < 4; ++c) {
            x[c] = v[c];
            // a workgroup that does not commit needs its own class's scan only
            if (!commit && c != cls) continue;
            for (int o = 1; o < 64; o <<= 1) {
                const long long y = __shfl_up(x[c], o, 64);
                if (lane >= o) x[c] += y;
            }
            if (lane == 63) s_wt[c][w] = x[c];
        }
        __syncthreads();
        for (int c = 0; c < 4; ++c) {
            if (!commit && c != cls) continue;
            long long before = 0, tot = 0;
            for (int q = 0; q < SUB_THREADS / 64; ++q) {
                if (q < w) before += s_wt[c][q];
                tot += s_wt[c][q];
            }
            const long long ex = before + x[c] - v[c];
            if (c == cls) {
                if (b < n_inst) s_pre[b] = ex;
                if (b == 0) s_pre[n_inst] = tot;
            }
            if (commit) {
                if (b < n_inst) plan[c * (n_inst + 1) + b] = ex;
                if (b == 0) plan[c * (n_inst + 1) + n_inst] = tot;
            }
        }
        __syncthreads();
        pre = s_pre;
        sinfo = s_info;
    }
    const long long total = pre[n_inst];
    // each workgroup takes a run of consecutive units, so that its successive
    // tiles mostly belong to one problem (its descriptor stays in the scalar
    // cache) and to one parent (consecutive coefficients)
    const long long chunk = (total + gridDim.x - 1) / gridDim.x;
    long long u = (long long)blockIdx.x * chunk;
    const long long uend = min(total, u + chunk);
    if (u >= uend) return total > 0;

    // LDS carve-up (16-byte aligned pieces)
    unsigned char* q8 = smem;
    auto carve = [&](size_t bytes) {
        unsigned char* r = q8;
        q8 += (bytes + 15) & ~(size_t)15;
        return r;
    };
    // the tile and its children: nr regions (2, or 4 when a problem of the
    // launch splits whole rounds), packed at the tile's own size TE: region q
    // at La + q TE
    T* La = (T*)carve((size_t)nr * tem * sizeof(T));
    // per patch: 5 keys of the split (min, max of both halves, max |parent|);
    // a round's second split adds 5 per half
    K* Lkey = (K*)carve((size_t)5 * tpm * (nr > 2 ? 3 : 1) * sizeof(K));
    // the two patch tables (current and next tile) are chosen by selects, not
    // by an indexed per-thread array, so that their accesses stay LDS ones
    long long* Lsrc0 = (long long*)carve((size_t)tpm * 8);
    long long* Lsrc1 = (long long*)carve((size_t)tpm * 8);
    long long* Lsrc2 = (long long*)carve((size_t)tpm * 8);
    T* Lpend = (T*)carve((size_t)tpm * sizeof(T));      // FP32: per patch, its pending shift
    float* Lcerr = (float*)carve((size_t)tpm * 4);      // FP32: per patch, its carried bound
    double* Lcbase = (double*)carve((size_t)tpm * 8);   // FP32: per patch, its FP64 base
    int* Ldead = (int*)carve((size_t)tpm * 4);          // per patch: children known dead (stale filter)
    int4* Linf0 = (int4*)carve((size_t)tpm * 16);
    int4* Linf1 = (int4*)carve((size_t)tpm * 16);
    int4* Linf2 = (int4*)carve((size_t)tpm * 16);
    int* Lwm = (int*)carve((size_t)tpm * 4);          // per patch: children to write (bit c)
    int* Lpre = (int*)carve((size_t)(2 * tpm + 2) * 4);  // per patch: scan of kept (child 0, child 1)
    int* Ldst = (int*)carve((size_t)2 * tpm * 4);     // per patch and child: heap patch or -1
    uint32_t* Lsfl = (uint32_t*)carve((size_t)nr * tpm * 4);  // per segment and child: flags
    int* Lpos = (int*)carve((size_t)2 * tpm * 4);     // per segment and child: list position
    int* Lseg = (int*)carve((size_t)(tpm + 1) * 4);   // per segment: first patch
    int64_t* Ldsto = (int64_t*)carve((size_t)tpm * 8);  // per patch: destination less its tile offset

    const int tid = threadIdx.x;
    int hint = 0;
    PackUnit c, cn, c2;   // this tile, the next, the one after
    T v[LB];
    // FP32: this thread's patch's carried error and pending shift (current, next
    // tile) and its FP64 base
    float2 ce = make_float2(0.0f, 0.0f), ne = make_float2(0.0f, 0.0f);
    double cb = 0.0, nb = 0.0;
    // Three patch tables in LDS, in turn: this tile's (tb), the next one's
    // (its coefficients are loaded while this tile is processed) and the one
    // after (its table is loaded during this tile).  Chosen by selects, not by
    // an indexed per-thread array, so that their accesses stay LDS ones.
    int tb = 0;
    auto inf_of = [&](int b) { return b == 0 ? Linf0 : (b == 1 ? Linf1 : Linf2); };
    auto src_of = [&](int b) { return b == 0 ? Lsrc0 : (b == 1 ? Lsrc1 : Lsrc2); };
    auto fp32_patch = [&](const PackUnit& pu, const int4 pinf, float2& e, double& b) {
        const DevInst& In = insts[pu.bi];
        const int poly = pu.kind == 0 ? 0 : In.count[0] + (pu.kind == 2 ? In.count[1] : 0) + pinf.z;
        const int64_t pi = (int64_t)pinf.y * In.n_polys + poly;
        const gmem_t<const float> ep = as_global((const float*)In.err[pu.cur]);
        e = make_float2(ep[2 * pi], ep[2 * pi + 1]);
        b = as_global(In.base[pu.cur])[pi];
    };

    // the first tile's table, the second's, then the first tile's coefficients in flight
    resolve_packed(insts, n_inst, pre, sinfo, u, hint, c);
    if (tid < c.np) {
        int4 pinf;
        long long psrc;
        patch_info(insts[c.bi], c, tid, pinf, psrc);
        Linf0[tid] = pinf;
        Lsrc0[tid] = psrc;
    }
    long long u1 = u + 1;
    bool more1 = u1 < uend;
    if (more1) {
        resolve_next(insts, n_inst, pre, sinfo, u1, hint, c, cn);
        if (tid < cn.np) {
            int4 pinf;
            long long psrc;
            patch_info(insts[cn.bi], cn, tid, pinf, psrc);
            Linf1[tid] = pinf;
            Lsrc1[tid] = psrc;
        }
    }
    __syncthreads();
    issue_packed<T, LB>(insts[c.bi], c, Lsrc0, v);
    if (fp32 && tid < c.np) fp32_patch(c, Linf0[tid], ce, cb);

    for (;;) {
        const DevInst& I = insts[c.bi];
        const int kind = c.kind, np = c.np, S = c.S, TE = c.TE, cur = c.cur, r = c.r, l = I.l, nc = c.nc;
        const int4* inf = inf_of(tb);
        const int tn = tb == 2 ? 0 : tb + 1, t2 = tn == 2 ? 0 : tn + 1;
        T* Lb = La + TE;          // the right half of the (first) split
        K* Lkey2 = Lkey + 5 * np;   // a round: keys of the second split, 5 per (half, patch)
        // current tile: registers -> LDS; keys and segment flags reset
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = tid + q * SUB_THREADS;
            if (e < TE) La[e] = v[q];
        }
        if (tid < np) {
            for (int h = 0; h < (nc == 4 ? 3 : 1); ++h) {
                // h = 0: the patch's first split; h = 1, 2: the second split of
                // its halves (keys at Lkey2 + 5 (half * np + patch))
                K* kk = Lkey + 5 * (h * np + tid);
                kk[0] = ~(K)0;
                kk[1] = 0;
                kk[2] = ~(K)0;
                kk[3] = 0;
                kk[4] = 0;
            }
            for (int ch = 0; ch < nr; ++ch) Lsfl[nr * tid + ch] = 0;
            if (fp32) {
                Lpend[tid] = (T)ce.y;
                Lcerr[tid] = ce.x;
                Lcbase[tid] = cb;
            }
            Ldead[tid] = 0;
        }
        // the next tile's coefficients (and FP32 error bounds and bases) in
        // flight for the whole of this tile
        if (more1) {
            issue_packed<T, LB>(insts[cn.bi], cn, src_of(tn), v);
            if (fp32 && tid < cn.np) fp32_patch(cn, inf_of(tn)[tid], ne, nb);
        }
        // the tile after: resolve it and start loading its patch table
        const long long u2 = u1 + 1;
        const bool more2 = more1 && u2 < uend;
        int4 ninf = make_int4(0, 0, 0, 0);
        long long nsrc = 0;
        if (more2) {
            resolve_next(insts, n_inst, pre, sinfo, u2, hint, cn, c2);
            if (tid < c2.np) patch_info(insts[c2.bi], c2, tid, ninf, nsrc);
        }
        lds_barrier();
        // the split: FP64 plain tiles by de Casteljau as the oracle does, FP32
        // tiles by de Casteljau too or (the problem's choice, uniform over the
        // workgroup) on the matrix cores.  A round splits along axis 0 (halves in
        // regions 0 and 1), then both halves along axis 1 (the right quarters to
        // regions 2 and 3): region b0 + 2 b1 holds the child with bit b0 on axis 0
        // and b1 on axis 1, the same sequence of operations as the oracle's.
        bool on_mfma = false;
        if constexpr (sizeof(T) == 4 && MF) on_mfma = I.mfma != 0;
        // (FP32: the first split takes each patch's values less its pending shift)
        if (on_mfma)
            tile_split_mfma(np, S, c.g, (float*)La, (float*)Lb, (unsigned*)Lkey, I.lam, (const float*)Lpend);
        else
            tile_split<T, MM>(np, S, c.g, La, Lb, Lkey, I.lam, fp32 ? Lpend : nullptr);
        if (nc == 4) {
            lds_barrier();
            if (on_mfma)
                tile_split_mfma(2 * np, S, c.g2, (float*)La, (float*)(La + 2 * TE), (unsigned*)Lkey2, I.lam,
                                nullptr);
            else
                tile_split<T, MM>(2 * np, S, c.g2, La, La + 2 * TE, Lkey2, I.lam, nullptr);
        }
        // the table of the tile after next to LDS (its loads had the split to arrive)
        if (more2 && tid < c2.np) {
            inf_of(t2)[tid] = ninf;
            src_of(t2)[tid] = nsrc;
        }
        lds_barrier();

        // per patch (thread p): bounds of every child (widened in FP32 mode),
        // records (cost) or flags (constraints).  A constraint tile inside one
        // parent with at most 64 patches takes one wave per child instead
        // (thread p + 64 ch bounds child ch of patch p), so the children are
        // bounded in parallel; the patch's FP32 figures then come from LDS.
        const bool split_b = kind != 0 && c.contig && np <= 64 && nc * 64 <= SUB_THREADS;
        const int p = split_b ? (tid & 63) : tid;
        const int chb = split_b ? (tid >> 6) : 0;
        const bool act = split_b ? (p < np && chb < nc) : tid < np;
        const int ch0 = split_b ? chb : 0, ch1 = split_b ? chb + 1 : nc;   // the children it bounds
        int j = 0, slot = 0, id = 0, poly = 0;
        uint32_t f2[NCMAX] = {0, 0, 0, 0};
        double lo[NCMAX] = {0.0, 0.0, 0.0, 0.0}, hi[NCMAX] = {0.0, 0.0, 0.0, 0.0};
        double emx = 0.0;   // FP32: the largest error bound given to a child here
        // stale filter, constraint tiles: children already known dead are not
        // written (bit ch): infeasible by another tile of this step, or with a
        // cost lower bound recorded this step above the previous estimate (the
        // new one can only be lower, so the cut drops them).  The loads go out
        // here and are used after the bounds.
        uint32_t known_dead = 0;
        if (act) {
            const int4 ip = inf[p];
            j = ip.x;
            slot = ip.y;
            id = ip.z;
            if (I.stale && kind != 0 && !c.gath) {
                for (int ch = ch0; ch < ch1; ++ch) {
                    const int64_t ci = (int64_t)nc * j + ch;
                    const uint32_t fl = __hip_atomic_load(&I.flags[ci], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const unsigned long long rec = __hip_atomic_load(&I.stamp[ci], __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT);
                    const bool above = (uint32_t)(rec >> 32) == c.stamp &&
                                       (double)__uint_as_float((uint32_t)rec) > c.pprev;
                    if ((fl & F_INFEAS) || above) known_dead |= 1u << ch;
                }
            }
            poly = kind == 0 ? 0 : I.count[0] + (kind == 2 ? I.count[1] : 0) + id;
            // FP32: the split's rounding bound over the parent's offsets (for a
            // round, the first split's; the second adds its own per half)
            // gamma_k here takes u = 2^-23, twice the unit roundoff.  At the
            // midpoint both engines stay within gamma_m: the products round at
            // most m times on any term's path, de Casteljau rounds one sum per
            // level (m - 1 roundings of 2^-24, the halving exact).  Away from
            // it the matrix entries are rounded to FP32 (|S~ - S| <= 2^-24 S:
            // less than two more roundings per term).  De Casteljau rounds two
            // products and a sum per level, two roundings of 2^-24 on a term's
            // path (m - 1 of u), and when fl(lam) or fl(1 - fl(lam)) is not
            // exact the two weights are off by at most 2^-23 together, at most
            // u max|c| more per level.  Should subnormal results be flushed,
            // each rounded operation on a term's path adds below 2^-126 (at
            // most two per level at the midpoint, three away from it).
            const bool w_exact = (double)(float)I.lam == I.lam && (double)(1.0f - (float)I.lam) == 1.0 - I.lam;
            const int mx_extra = I.lam == 0.5 ? 0 : (I.mfma ? 2 : (w_exact ? 0 : c.g.m));
            // The split took the parent's values less its pending shift s, so
            // the children are offsets from the base plus s (in FP64, rounded:
            // 2^-52 of it); the subtraction rounds below 2^-23 of the largest
            // shifted value (max |parent| of the split's keys), or flushes.
            const double amax = fp32 ? (double)funkey(Lkey[5 * p + 4]) : 0.0;
            float pe = ce.x, ps = ce.y;
            double pb = cb;
            if (fp32 && split_b) {
                pe = Lcerr[p];
                ps = (float)Lpend[p];
                pb = Lcbase[p];
            }
            const bool shifted = fp32 && ps != 0.0f;
            const double nbs = shifted ? pb + (double)ps : pb;
            const double e1 = fp32 ? (double)pe + gamma32(c.g.m + mx_extra) * amax + (double)(3 * c.g.m) * 0x1p-126 +
                                         (shifted ? amax * 0x1p-23 + 0x1p-126 + fabs(nbs) * 0x1p-52 : 0.0)
                                   : 0.0;
            for (int ch = ch0; ch < ch1; ++ch) {
                // the keys of child ch: one split, half ch; a round, half b0 of the
                // first split and then half b1 of the second
                const int b0 = nc == 4 ? (ch >> 1) : ch, b1 = ch & 1;
                const K* kk = nc == 4 ? Lkey2 + 5 * (b0 * np + p) + 2 * b1 : Lkey + 5 * p + 2 * b0;
                const T mn = funkey(kk[0]), mx = funkey(kk[1]);
                double e = 0.0, base = 0.0;
                if (fp32) {
                    // the stored values are offsets from an FP64 base, which
                    // subdivision keeps (rows sum to one); the split's error grows
                    // with the offsets.  Each child is re-centred lazily: its
                    // midrange offset mc is stored as its pending shift, and its
                    // own split will subtract it first, so that the offsets it
                    // splits shrink with the box.
                    base = nbs;
                    double ee = e1;
                    if (nc == 4)
                        ee += gamma32(c.g2.m) * (double)funkey(Lkey2[5 * (b0 * np + p) + 4]) +
                              (double)(2 * c.g2.m) * 0x1p-126;
                    e = (double)round_up_f(ee);
                    const float mc = 0.5f * (float)mn + 0.5f * (float)mx;
                    const int64_t ci = (int64_t)(nc * j + ch) * I.n_polys + poly;
                    const gmem_t<float> eo = as_global((float*)I.err[cur ^ 1]);
                    eo[2 * ci] = (float)e;
                    eo[2 * ci + 1] = mc;
                    as_global(I.base[cur ^ 1])[ci] = nbs;
                    emx = fmax(emx, e);
                }
                child_bounds<T>(mn, mx, e, base, lo[ch], hi[ch]);
            }
            if (kind == 0) {
                // cost records, child ids, and with the stale filter the record
                // that constraint tiles of this step read
                const gmem_t<const uint32_t> pid = as_global((const uint32_t*)I.ids[cur]) + (int64_t)slot * l;
                const gmem_t<uint32_t> cid = as_global(I.ids[cur ^ 1]) + (int64_t)(nc * j) * l;
                for (int ch = 0; ch < nc; ++ch) {
                    as_global(I.minP)[nc * j + ch] = lo[ch];
                    as_global(I.maxP)[nc * j + ch] = hi[ch];
                    for (int k = 0; k < l; ++k) {
                        const uint32_t vv = pid[k];
                        // a round halves every axis (bit l-1-k of ch is axis k's half)
                        const bool split = I.fused || k == r;
                        const uint32_t half = I.fused ? (uint32_t)((ch >> (l - 1 - k)) & 1) : (uint32_t)ch;
                        cid[ch * l + k] = split ? 2u * vv + half : vv;
                    }
                }
                if (I.stale)
                    for (int ch = 0; ch < nc; ++ch) {
                        // the stamp and a float at or below the cost lower bound, in
                        // one store, so that a reader needs no fence
                        float fl = (float)lo[ch];
                        if ((double)fl > lo[ch]) fl = nextafterf(fl, -INFINITY);
                        const unsigned long long rec = ((unsigned long long)c.stamp << 32) | __float_as_uint(fl);
                        __hip_atomic_store(&I.stamp[nc * j + ch], rec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
            } else {
                for (int ch = ch0; ch < ch1; ++ch) {
                    uint32_t f = 0;
                    if (kind == 1) {
                        if (lo[ch] > 0.0) f |= F_INFEAS;
                        if (!(hi[ch] <= 0.0)) f |= F_NOTFEAS;
                    } else {
                        if (lo[ch] > 0.0 || hi[ch] < 0.0) f |= F_INFEAS;
                        if (!(-I.eps_eq <= lo[ch] && lo[ch] <= 0.0 && 0.0 <= hi[ch] && hi[ch] <= I.eps_eq))
                            f |= F_NOTFEAS;
                    }
                    f2[ch] = f;
                }
            }
        }
        if (fp32) {
            // the largest bound of the solve so far (non-negative doubles order
            // as their bit patterns)
            for (int o = 32; o > 0; o >>= 1) emx = fmax(emx, __shfl_xor(emx, o, 64));
            if ((tid & 63) == 0 && emx > 0.0)
                atomicMax((unsigned long long*)&I.st->err_max, (unsigned long long)__double_as_longlong(emx));
        }
        // constraint tiles: segments (runs of patches of one parent) and, in
        // retiring mode, which children keep each patch (an inequality
        // certified satisfied on a child, max B <= 0, stays satisfied on all its
        // sub-boxes, and the child drops it), in one workgroup scan
        int seg = 0, k0 = 0, k1 = 0;
        int3 ex = make_int3(0, 0, 0), tot = make_int3(0, 0, 0);
        if (kind != 0 && c.contig) {
            // a tile inside one parent is one segment: no scan.  The children's
            // flags are ORed per wave by ballots, then across the waves in LDS
            for (int ch = 0; ch < nc; ++ch) {
                const uint32_t f = (__ballot(act && (f2[ch] & F_INFEAS)) ? F_INFEAS : 0u) |
                                   (__ballot(act && (f2[ch] & F_NOTFEAS)) ? F_NOTFEAS : 0u);
                if (f && (tid & 63) == 0) atomicOr(&Lsfl[ch], f);
            }
            // the children known dead, per patch (one wave per child bounds them)
            if (act && known_dead) atomicOr(&Ldead[p], (int)known_dead);
            if (tid == 0) {
                Lseg[0] = 0;
                Lseg[1] = np;
                s_nseg = 1;
            }
            lds_barrier();
            if (tid < nc) {
                const uint32_t f = Lsfl[tid];
                if (f) atomicOr(&I.flags[nc * inf[0].x + tid], f);
            }
        } else if (kind != 0) {
            const int start = act && (p == 0 || inf[p - 1].x != j);
            if (c.gath && act) {
                k0 = hi[0] > 0.0;
                k1 = hi[1] > 0.0;
            }
            tot = block_scan3(make_int3(start, k0, k1), ex, s_sc);
            seg = ex.x + start - 1;
            if (act) {
                if (start) Lseg[seg] = p;
                for (int ch = 0; ch < nc; ++ch)
                    if (f2[ch]) atomicOr(&Lsfl[nr * seg + ch], f2[ch]);
                Lpre[2 * p] = ex.y;
                Lpre[2 * p + 1] = ex.z;
            }
            if (tid == 0) {
                Lseg[tot.x] = np;
                s_nseg = tot.x;
                Lpre[2 * np] = tot.y;
                Lpre[2 * np + 1] = tot.z;
            }
            lds_barrier();
            // per segment and child: the flags to the child's record; in
            // retiring mode its kept patches' place in the child's carried list,
            // and the tile's heap patches, reserved together
            if (tid < s_nseg) {
                const int a0 = Lseg[tid], a1 = Lseg[tid + 1];
                const int js = inf[a0].x;
                for (int ch = 0; ch < nc; ++ch) {
                    const uint32_t f = Lsfl[nr * tid + ch];
                    if (f) atomicOr(&I.flags[nc * js + ch], f);
                    if (c.gath) {
                        const int cnt = Lpre[2 * a1 + ch] - Lpre[2 * a0 + ch];
                        Lpos[2 * tid + ch] = cnt ? atomicAdd(&I.na[cur ^ 1][2 * js + ch], cnt) : 0;
                    }
                }
            }
            if (c.gath && tid == SUB_THREADS - 1)
                s_hb = (tot.y + tot.z) ? (long long)atomicAdd((unsigned long long*)&I.st->htop[cur ^ 1],
                                                              (unsigned long long)(tot.y + tot.z))
                                       : 0;
        }
        if (!c.gath) {
            // children patches to the children's slots, not to a child already
            // condemned (infeasible from this tile, or with the stale filter a
            // cost bound above the previous solution estimate).  A constraint
            // tile of one segment without the stale filter writes child ch
            // unless the tile's flags condemn it, which every thread reads
            const bool one_seg = kind != 0 && s_nseg == 1;
            const bool by_flags = one_seg && !I.stale;
            if (!by_flags) {
                if (act && chb == 0) {
                    int wm = 0;
                    const uint32_t kd = split_b ? (uint32_t)Ldead[p] : known_dead;
                    for (int ch = 0; ch < nc; ++ch) {
                        const bool w = kind == 0 ? !(I.stale && lo[ch] > c.pprev)
                                                 : !(Lsfl[nr * seg + ch] & F_INFEAS) && !((kd >> ch) & 1u);
                        if (w) wm |= 1 << ch;
                    }
                    Lwm[p] = wm;
                }
                lds_barrier();
            }
            const gmem_t<T> dbuf = as_global((T*)I.buf[cur ^ 1]);
            constexpr int SB = 8;
            // child ch of a parent is region ch of the split, or for a round
            // region b0 + 2 b1 (its halves on axes 0 and 1); it goes to slot nc j + ch.
            // A run of patches of one parent (a segment) is contiguous in LDS and
            // in the child's slot.  A tile of one segment (the usual constraint
            // tile without retiring) is copied as one run per child; otherwise
            // each patch's destination, less its position in the tile, is
            // tabulated once (-1: not written) and each element adds its offset.
            for (int ch = 0; ch < nc; ++ch) {
                const T* src = La + (nc == 4 ? (ch >> 1) + 2 * (ch & 1) : ch) * TE;
                if (one_seg) {
                    // uniform: the whole tile's child
                    if (by_flags ? (Lsfl[ch] & F_INFEAS) != 0u : !((Lwm[0] >> ch) & 1)) continue;
                    const int4 ip = inf[0];
                    const int64_t d0 = (int64_t)(nc * ip.x + ch) * I.stride + I.soff[kind] + (int64_t)ip.z * S;
                    // 16-byte stores: the elements before the destination's
                    // first 16-byte boundary and after its last one singly
                    // (buffers are 256-byte aligned), whole vectors between
                    constexpr int VE = 16 / sizeof(T);
                    using V = T __attribute__((ext_vector_type(VE)));
                    const int h = min((int)((VE - (int)(d0 & (VE - 1))) & (VE - 1)), TE);
                    const int nv = (TE - h) / VE, t0 = h + nv * VE, nt = TE - t0;
                    if (tid < h) dbuf[d0 + tid] = src[tid];
                    if (tid >= SUB_THREADS - nt) {
                        const int e = t0 + tid - (SUB_THREADS - nt);
                        dbuf[d0 + e] = src[e];
                    }
                    const gmem_t<V> dv = (gmem_t<V>)(dbuf + d0 + h);
                    const T* sv = src + h;
                    constexpr int SV = 4;
                    for (int i0 = tid; i0 < nv; i0 += SV * SUB_THREADS) {
                        V va[SV];
#pragma unroll
                        for (int q = 0; q < SV; ++q) {
                            const int i = i0 + q * SUB_THREADS;
                            if (i < nv)
#pragma unroll
                                for (int k = 0; k < VE; ++k) va[q][k] = sv[i * VE + k];
                        }
#pragma unroll
                        for (int q = 0; q < SV; ++q) {
                            const int i = i0 + q * SUB_THREADS;
                            if (i < nv) dv[i] = va[q];
                        }
                    }
                    continue;
                }
                if (act) {
                    const int4 ip = inf[p];
                    Ldsto[p] = ((Lwm[p] >> ch) & 1) ? (int64_t)(nc * ip.x + ch) * I.stride + I.soff[kind] +
                                                          (int64_t)ip.z * S - (int64_t)p * S
                                                    : (int64_t)-1;
                }
                lds_barrier();
                for (int e0 = tid; e0 < TE; e0 += SB * SUB_THREADS) {
                    T va[SB];
                    int64_t dd[SB];
#pragma unroll
                    for (int q = 0; q < SB; ++q) {
                        const int e = e0 + q * SUB_THREADS;
                        dd[q] = -1;
                        if (e < TE) {
                            const int pq = patch_of(e, c.invS);
                            dd[q] = Ldsto[pq];
                            va[q] = src[e];
                        }
                    }
#pragma unroll
                    for (int q = 0; q < SB; ++q)
                        if (dd[q] >= 0) dbuf[dd[q] + e0 + q * SUB_THREADS] = va[q];
                }
                lds_barrier();
            }
        } else {
            // retiring mode: every kept (patch, child) gets its heap patch and
            // its entry in the child's carried list
            lds_barrier();
            if (act) {
                const long long hb = s_hb;
                const int sp = Lseg[seg];
                for (int ch = 0; ch < 2; ++ch) {
                    int d = -1;
                    if (ch ? k1 : k0) {
                        const int rank = Lpre[2 * p + ch] - Lpre[2 * sp + ch];
                        d = (int)(hb + (ch ? tot.y + ex.z : ex.y));
                        vec2i a;
                        a.x = id;
                        a.y = d;
                        ((gmem_t<vec2i>)I.act[cur ^ 1])[(int64_t)(2 * j + ch) * I.count[1] + Lpos[2 * seg + ch] +
                                                        rank] = a;
                    }
                    Ldst[ch * tpm + p] = d;
                }
            }
            lds_barrier();
            // each kept patch to its heap patch
            const gmem_t<T> hc = as_global((T*)I.heap[cur ^ 1]);
#pragma unroll 2
            for (int e = tid; e < TE; e += SUB_THREADS) {
                const int pq = patch_of(e, c.invS);
                const int dl = Ldst[pq], dr = Ldst[tpm + pq];
                const int rr = e - pq * S;
                if (dl >= 0) hc[(int64_t)dl * S + rr] = La[e];
                if (dr >= 0) hc[(int64_t)dr * S + rr] = Lb[e];
            }
        }
        lds_barrier();
        if (!more1) break;
        c = cn;
        cn = c2;
        u = u1;
        u1 = u2;
        more1 = more2;
        ce = ne;
        cb = nb;
        tb = tn;
    }
    return true;
}

// Two workgroups of four waves per compute unit (two waves per SIMD): the
// register budget is then 256 per lane, which the FP32 form, with its matrix
// accumulators, would otherwise exceed by a few and fall to one wave per SIMD.
template <typename T, int MM, int LB, bool FUSE, bool MF>
__global__ __launch_bounds__(SUB_THREADS, 2) void k_sub(const DevInst* __restrict__ insts, int n_inst,
                                                    long long* __restrict__ plan,
                                                    StepInfo* __restrict__ info, int tem, int tpm, int nr)
{
    sub_run<T, MM, LB, FUSE, MF>(insts, n_inst, plan, info, tem, tpm, nr);
}

// ------------------------------------------------------------------ k_rederive

// Applies tmat (one m x m matrix per axis) to np patches in LDS (FP64), axis
// by axis, in place, as FP64 matrix-core products (mfma_fibres_f64): every
// fibre of the chunk along axis r is a column of one product with the axis's
// transform.
__device__ void apply_tmats(double* x, const double* tm, const int* tmoff, const AxisGeo* geo, int l,
                            int S, int np)
{
    for (int r = 0; r < l; ++r) {
        const AxisGeo ag = geo[r];
        FibreGeom g;
        g.m = ag.m;
        g.stride = ag.stride;
        g.F = ag.F;
        const double* Tm = tm + tmoff[r];
        // quotients by reciprocals, exact for dividends below 2^22 (see patch_of)
        const float invF = 1.0f / (float)g.F, invT = 1.0f / (float)g.stride;
        mfma_fibres_f64(np * g.F, g.m, g.stride, Tm, [&](int f) {
            const int p = (int)(((float)f + 0.5f) * invF);
            const int q = f - p * g.F;
            const int outer = (int)(((float)q + 0.5f) * invT);
            return x + p * S + outer * g.m * g.stride + (q - outer * g.stride);
        });
        __syncthreads();
    }
}

// Sub-interval transforms of every child of every parent whose step re-derives
// from the root: one thread per matrix row.  Row k of the transform for [a,b]
// and degree n is T[k][j] = sum_s b^{n-k}_s(a) b^k_{j-s}(b); both basis rows come
// from the recurrence b^q_s(t) = (1-t) b^{q-1}_s(t) + t b^{q-1}_{s-1}(t), whose
// terms are all non-negative (relative error below gamma_{2q} per value), so
// |T~ - T| <= gamma_{5m} T entrywise.
__global__ __launch_bounds__(256) void k_tmat(const DevInst* __restrict__ insts, int n_inst,
                                             const long long* __restrict__ plan)
{
    const long long* pre = plan + 3 * (n_inst + 1);
    const long long total = pre[n_inst];
    for (long long u = blockIdx.x * (long long)blockDim.x + threadIdx.x; u < total;
         u += (long long)gridDim.x * blockDim.x) {
        const int bi = find_inst(pre, n_inst, u);
        const DevInst& I = insts[bi];
        const InstState* st = I.st;
        const long long v = u - pre[bi];
        const int nc = I.fused ? (1 << I.l) : 2;
        const int j = (int)(v / (nc * I.rows));
        int rem = (int)(v - (long long)j * nc * I.rows);
        const int c = rem / I.rows;
        rem -= c * I.rows;
        // locate (kind, axis, row) of this thread
        int kind = 0, k = 0, off = I.tmk[0];
        for (;;) {
            if (I.count[kind] == 0) { ++kind; k = 0; off = I.tmk[min(kind, KINDS - 1)]; continue; }
            const int m = I.dims[kind][k];
            if (rem < m) break;
            rem -= m;
            off += m * m;
            if (++k == I.l) { ++kind; k = 0; off = I.tmk[min(kind, KINDS - 1)]; }
        }
        const int m = I.dims[kind][k], n = m - 1, row = rem;
        const int r = st->r, cur = st->cur;
        const uint32_t pid = I.ids[cur][(int64_t)I.live[j] * I.l + k];
        // child c halves axis r (a round: every axis, bit l-1-k of c on axis k)
        const bool split = I.fused || k == r;
        const int d = st->depth[k] + (split ? 1 : 0);
        const uint32_t half = I.fused ? (uint32_t)((c >> (I.l - 1 - k)) & 1) : (uint32_t)c;
        const uint32_t idx = split ? 2u * pid + half : pid;
        const double a = ldexp((double)idx, -d), b = ldexp((double)idx + 1.0, -d);
        double Ba[MAXM], Bb[MAXM];
#pragma unroll
        for (int q = 0; q < MAXM; ++q) { Ba[q] = (q == 0) ? 1.0 : 0.0; Bb[q] = Ba[q]; }
#pragma unroll
        for (int q = 1; q < MAXM; ++q) {
#pragma unroll
            for (int s2 = MAXM - 1; s2 >= 1; --s2) {
                if (s2 <= q && q <= n - row) Ba[s2] = (1.0 - a) * Ba[s2] + a * Ba[s2 - 1];
                if (s2 <= q && q <= row) Bb[s2] = (1.0 - b) * Bb[s2] + b * Bb[s2 - 1];
            }
            if (q <= n - row) Ba[0] = (1.0 - a) * Ba[0];
            if (q <= row) Bb[0] = (1.0 - b) * Bb[0];
        }
        double* out = I.tmat + ((int64_t)j * nc + c) * I.tmw + off + row * m;
#pragma unroll
        for (int jj = 0; jj < MAXM; ++jj) {
            if (jj > n) break;
            double acc = 0.0;
#pragma unroll
            for (int s2 = 0; s2 < MAXM; ++s2)
                if (s2 <= n - row && jj - s2 >= 0 && jj - s2 <= row) acc += Ba[s2] * Bb[(jj - s2) & (MAXM - 1)];
            out[jj] = acc;
        }
    }
}

// FP32 re-derivation step: the children of every live parent derived from the
// FP64 root by box id (the transforms of k_tmat applied axis by axis in FP64),
// rounded to FP32 with a fresh error bound, then bounded and flagged like
// k_sub.  Units and their order are those of k_sub.
__global__ __launch_bounds__(SUB_THREADS) void k_rederive(const DevInst* __restrict__ insts, int n_inst,
                                                         const long long* __restrict__ plan,
                                                         const StepInfo* __restrict__ info)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_flag[NCMAX];
    __shared__ int s_tmoff[MAXL];
    __shared__ AxisGeo s_geo[MAXL];
    const long long* pre = plan + 2 * (n_inst + 1);
    const long long total = pre[n_inst];
    for (long long u = blockIdx.x; u < total; u += gridDim.x) {
        const int bi = find_inst_uniform(pre, n_inst, u);
        const DevInst& I = insts[bi];
        const StepInfo si = info[bi];
        int j, t, mslot, mna;
        unit_of(I, u - pre[bi], si.K, j, t, mslot, mna);
        const int cur = si.cur, r = si.r, l = I.l;
        const int nc = I.fused ? (1 << l) : 2;
        const int pslot = mslot >= 0 ? mslot : __builtin_amdgcn_readfirstlane(I.live[j]);
        const int kind = (t < I.tile_start[1]) ? 0 : ((t < I.tile_start[2]) ? 1 : 2);
        const int p0 = (t - I.tile_start[kind]) * I.tile_polys[kind];
        // retiring mode: an inequality tile covers positions p0.. of the parent's carried list
        const bool gath = I.retire && kind == 1;
        const int2* pact = gath ? I.act[cur] + (int64_t)pslot * I.count[1] : nullptr;
        const int navail = gath ? (mna >= 0 ? mna : __builtin_amdgcn_readfirstlane(I.na[cur][pslot]))
                                : I.count[kind];
        const int np = min(I.tile_polys[kind], navail - p0);
        const int S = I.S[kind];
        // the tile is processed in chunks of at most MAX_TILE64 coefficients
        // and REDERIVE_CHUNK patches
        const int cp = min(REDERIVE_CHUNK, max(1, MAX_TILE64 / S));
        int tmsz = 0;
        for (int k = 0; k < l; ++k) tmsz += I.dims[kind][k] * I.dims[kind][k];
        // dynamic LDS: the chunk, the transforms, then per patch of a chunk its
        // FP64 base, FP64 range (order keys), root bound, FP32 offsets' range,
        // whether the child carries it, its heap patch (retiring mode) and its
        // polynomial: 52 bytes
        const int npc = min(np, cp);
        double* x = (double*)smem;
        double* tm = x + npc * S;
        double* s_base = tm + tmsz;
        unsigned long long* s_kd = (unsigned long long*)(s_base + npc);
        double* s_rb = (double*)(s_kd + 2 * npc);
        unsigned int* s_kf = (unsigned int*)(s_rb + npc);
        int* s_keep = (int*)(s_kf + 2 * npc);
        int* s_dst = s_keep + npc;
        int* s_poly = s_dst + npc;
        if (threadIdx.x < NCMAX) s_flag[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            int o = 0;
            for (int k = 0; k < l; ++k) { s_tmoff[k] = o; o += I.dims[kind][k] * I.dims[kind][k]; }
            stage_geo(s_geo, I.dims[kind], l, S);
        }
        double g64 = 0.0;
        for (int k = 0; k < l; ++k) g64 += gamma64(6 * I.dims[kind][k] + 6);
        for (int cc = 0; cc < nc * ((np + cp - 1) / cp); ++cc) {
            const int c = cc % nc;
            const int q0 = (cc / nc) * cp;
            const int nq = min(cp, np - q0);
            const int TE = nq * S;
            // the chunk's patches in the root (root layout) and in a slot
            const int64_t roff = I.off[kind] + (gath ? 0 : (int64_t)(p0 + q0) * S);
            const int64_t soff = I.soff[kind] + (int64_t)(p0 + q0) * S;
            const double* tsrc = I.tmat + ((int64_t)j * nc + c) * I.tmw + I.tmk[kind];
            // per patch: its polynomial and root figures, and the range keys reset
            for (int p = threadIdx.x; p < nq; p += blockDim.x) {
                const int id = gath ? pact[p0 + q0 + p].x : p0 + q0 + p;
                const int poly = kind == 0 ? 0 : I.count[0] + (kind == 2 ? I.count[1] : 0) + id;
                s_poly[p] = poly;
                // root bound (rows of T sum to one) + transform rounding on
                // |T||root| <= max|root|
                s_rb[p] = I.root_err[poly] + g64 * I.root_abs[poly] * 1.01;
                s_kd[2 * p] = ~0ull;
                s_kd[2 * p + 1] = 0ull;
                s_kf[2 * p] = ~0u;
                s_kf[2 * p + 1] = 0u;
            }
            copy_to_lds<double>(tm, tsrc, tmsz);
            if (!gath) {
                copy_to_lds<double, MAX_TILE64 / SUB_THREADS>(x, I.racc + roff, TE);   // one round of loads
            } else {
                for (int e = threadIdx.x; e < TE; e += blockDim.x) {
                    const int p = e / S;
                    x[e] = I.racc[roff + (int64_t)pact[p0 + q0 + p].x * S + (e - p * S)];
                }
            }
            __syncthreads();
            apply_tmats(x, tm, s_tmoff, s_geo, l, S, nq);
            float* child = (float*)I.buf[cur ^ 1] + (int64_t)(nc * j + c) * I.stride;
            float* hc = (float*)I.heap[cur ^ 1];
            uint32_t fl = 0;
            const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
            // each patch: its FP64 range and base (the midrange), then the
            // FP32 offsets' range, each by nseg threads per patch (thread s
            // takes the patch's elements s, s + nseg, ...) and order keys in
            // LDS; then one thread per patch forms the error bound and the
            // child's bounds
            const int nseg = max(1, min(S, (int)blockDim.x / nq));
            const int ntask = nq * nseg;
            for (int k = threadIdx.x; k < ntask; k += blockDim.x) {
                const int p = k / nseg, sg = k - p * nseg;
                double vmn = INFINITY, vmx = -INFINITY;
                for (int e = sg; e < S; e += nseg) {
                    const double v = x[p * S + e];
                    vmn = fmin(vmn, v);
                    vmx = fmax(vmx, v);
                }
                atomicMin(&s_kd[2 * p], fkey(vmn));
                atomicMax(&s_kd[2 * p + 1], fkey(vmx));
            }
            __syncthreads();
            for (int p = threadIdx.x; p < nq; p += blockDim.x)
                s_base[p] = 0.5 * funkey(s_kd[2 * p]) + 0.5 * funkey(s_kd[2 * p + 1]);
            __syncthreads();
            for (int k = threadIdx.x; k < ntask; k += blockDim.x) {
                const int p = k / nseg, sg = k - p * nseg;
                const double b = s_base[p];
                float mn = INFINITY, mx = -INFINITY;
                for (int e = sg; e < S; e += nseg) {
                    const float d = (float)(x[p * S + e] - b);
                    mn = fminf(mn, d);
                    mx = fmaxf(mx, d);
                }
                atomicMin(&s_kf[2 * p], fkey(mn));
                atomicMax(&s_kf[2 * p + 1], fkey(mx));
            }
            __syncthreads();
            for (int p = threadIdx.x; p < nq; p += blockDim.x) {
                const int poly = s_poly[p];
                const double base = s_base[p];
                const float mn = funkey(s_kf[2 * p]), mx = funkey(s_kf[2 * p + 1]);
                // the root's part + rounding of the offsets (the FP64
                // difference and the FP32 conversion) + underflow
                const double amax = fmax(fabs((double)mn), fabs((double)mx));
                const double e = (double)round_up_f(s_rb[p] + amax * 0x1p-23 + 0x1p-126);
                double lo, hi;
                child_bounds<float>(mn, mx, e, base, lo, hi);
                // retiring mode: an inequality certified satisfied is not carried
                s_keep[p] = !(gath && hi <= 0.0);
                I.err[cur ^ 1][(int64_t)(nc * j + c) * I.n_polys + poly] = make_float2((float)e, 0.0f);
                I.base[cur ^ 1][(int64_t)(nc * j + c) * I.n_polys + poly] = base;
                if (kind == 0) {
                    I.minP[nc * j + c] = lo;
                    I.maxP[nc * j + c] = hi;
                } else if (kind == 1) {
                    if (lo > 0.0) fl |= F_INFEAS;
                    if (!(hi <= 0.0)) fl |= F_NOTFEAS;
                } else {
                    if (lo > 0.0 || hi < 0.0) fl |= F_INFEAS;
                    if (!(-I.eps_eq <= lo && lo <= 0.0 && 0.0 <= hi && hi <= I.eps_eq))
                        fl |= F_NOTFEAS;
                }
            }
            __syncthreads();
            // retiring mode: wave 0 reserves the kept patches of the chunk in
            // the child's carried list and in the heap (one reservation each),
            // ranks them by ballot and records each one's heap patch
            if (gath && wv == 0) {
                int cnt = 0;
                for (int q = 0; q < nq; q += 64) cnt += __popcll(__ballot(q + lane < nq && s_keep[q + lane]));
                int pos = 0;
                long long hb = 0;
                if (lane == 0 && cnt) {
                    pos = atomicAdd(&I.na[cur ^ 1][2 * j + c], cnt);
                    hb = (long long)atomicAdd((unsigned long long*)&I.st->htop[cur ^ 1], (unsigned long long)cnt);
                }
                pos = __shfl(pos, 0, 64);
                hb = __shfl(hb, 0, 64);
                const unsigned long long below = (1ull << lane) - 1ull;
                for (int q = 0; q < nq; q += 64) {
                    const int p = q + lane;
                    const bool k = p < nq && s_keep[p];
                    const unsigned long long bal = __ballot(k);
                    const int rank = __popcll(bal & below);
                    if (k) {
                        I.act[cur ^ 1][(int64_t)(2 * j + c) * I.count[1] + pos + rank] =
                            make_int2(pact[p0 + q0 + p].x, (int)(hb + rank));
                        s_dst[p] = (int)(hb + rank);
                    }
                    pos += __popcll(bal);
                    hb += __popcll(bal);
                }
            }
            __syncthreads();
            // the kept patches' FP32 offsets: to the child's slot, or its heap patch
            const float invS = 1.0f / (float)S;
            for (int e = threadIdx.x; e < TE; e += blockDim.x) {
                const int p = patch_of(e, invS);
                if (!s_keep[p]) continue;
                float* dp = gath ? hc + (int64_t)s_dst[p] * S : child + soff + (int64_t)p * S;
                dp[e - p * S] = (float)(x[e] - s_base[p]);
            }
            if (fl) atomicOr(&s_flag[c], fl);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            for (int c = 0; c < nc; ++c)
                if (s_flag[c]) atomicOr(&I.flags[nc * j + c], s_flag[c]);
            if (kind == 0) {
                const uint32_t* pid = I.ids[cur] + (int64_t)pslot * l;
                uint32_t* cid = I.ids[cur ^ 1] + (int64_t)(nc * j) * l;
                for (int c = 0; c < nc; ++c)
                    for (int k = 0; k < l; ++k) {
                        const uint32_t v = pid[k];
                        const bool split = I.fused || k == r;
                        const uint32_t half = I.fused ? (uint32_t)((c >> (l - 1 - k)) & 1) : (uint32_t)c;
                        cid[c * l + k] = split ? 2u * v + half : v;
                    }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ k_cut

// The cut of problem b by the calling workgroup (a multiple of 64 lanes, at
// most NT).  phase 0: the whole cut by one workgroup, unless the step has more
// than `split` children (then it returns: the cut is split).  A split cut runs
// in four launches over G workgroups per problem, workgroup g taking children
// [g part, (g+1) part) of the step's C (parts[b G + g] holds its
// figures; the step's K, r, cur, steps and previous estimate come from info,
// which the state's updates in phase 4 do not touch):
//   1: the least max B over its feasible children (and the first child
//      attaining it) and the least min B over its live children;
//   2: the estimate from all parts' minima, then its kept children, their
//      inequality units and carried patches;
//   3: the offsets of its kept children from the parts before it, then the
//      same order-preserving compaction as phase 0 over its children;
//   4: the flags of the next step's children cleared over its share, and
//      (g = 0) the state's updates as phase 0 makes them.
template <int NT>
__device__ __forceinline__ void cut_phase(const DevInst* __restrict__ insts, const StepInfo* __restrict__ info,
                                          int b, int phase, int g, int G, CutPart* __restrict__ parts,
                                          long long split, int part)
{
    __shared__ double shd[NT / 64];
    __shared__ int shi[NT / 64];
    __shared__ int wsum[NT / 64 + 1];
    __shared__ long long wun[NT / 64 + 1];
    __shared__ long long wap[NT / 64 + 1];
    __shared__ int s_kc[NT];   // retiring mode: a chunk's kept children's slots
    __shared__ int s_ka[NT];   // and the offsets of their carried patches
    __shared__ long long wact[NT / 64];
    __shared__ double s_plo[NT / 64];
    const DevInst& I = insts[b];
    InstState* st = I.st;
    const int nc = I.fused ? (1 << I.l) : 2;   // children per parent (a round splits every axis)
    int K, r, cur, steps0;
    double pprev;
    if (phase == 0) {
        if (st->status != ST_RUNNING) return;
        K = st->K;
        if ((long long)nc * K > split) return;   // a split cut takes it
        r = st->r;
        cur = st->cur;
        steps0 = st->steps;
        pprev = st->p_up;
    } else {
        const StepInfo si = info[b];
        K = si.K;
        r = si.r;
        cur = si.cur;
        steps0 = si.steps;
        pprev = si.p_up;
    }
    const int C = nc * K, l = I.l;
    const int Gb = (int)(((long long)C + part - 1) / part);   // parts of a split cut
    CutPart* pp = parts + (long long)b * G;
    if (phase == 1) {
        // this part of a running problem whose cut is split, or nothing (the
        // later phases read the mark)
        const bool mine = st->status == ST_RUNNING && (long long)C > split && g < Gb;
        __syncthreads();
        if (threadIdx.x == 0) pp[g].valid = mine ? 1 : 0;
        if (!mine) return;
    } else if (phase > 1) {
        if (!pp[g].valid) return;
    }
    const int TP1 = I.tile_polys[1];
    const bool fin = pprev < INFINITY;
    const int tid = threadIdx.x;
    // this workgroup's children
    const int cbeg = phase == 0 ? 0 : g * part;
    const int cend = phase == 0 ? C : min(C, cbeg + part);
    if (phase == 1) {
        double mm = INFINITY, pl = INFINITY;
        int ag = INT_MAX;
        for (int c = cbeg + tid; c < cend; c += blockDim.x) {
            const double mnp = as_global(I.minP)[c];
            const uint32_t fl = as_global(I.flags)[c];
            const bool dead = fin && mnp > pprev;
            if (dead || (fl & F_INFEAS)) continue;
            pl = fmin(pl, mnp);
            if (fl & F_NOTFEAS) continue;
            const double mx = as_global(I.maxP)[c];
            if (mx < mm) {
                mm = mx;
                ag = c;
            }
        }
        const double mb = block_min1(mm, shd);
        const int ab = block_min1_i(mm == mb ? ag : INT_MAX, shi);
        const double pb = block_min1(pl, s_plo);
        if (tid == 0) {
            pp[g].m = mb;
            pp[g].arg = ab;
            pp[g].plo = pb;
        }
        return;
    }
    // state the final updates need, read before the passes: the step count,
    // carried patches, iteration count, per axis (thread k) its depth, and the
    // children's width
    const int n0 = st->n;
    const long long alive0 = st->a_live;
    const int depth_k = tid < l ? st->depth[tid] + ((I.fused || tid == r) ? 1 : 0) : 0;
    // the children's depth vector, and the widest child's width
    int dnew[MAXL];
    double width = 0.0;
    for (int k = 0; k < l; ++k) {
        dnew[k] = st->depth[k] + ((I.fused || k == r) ? 1 : 0);
        width = fmax(width, axis_width(I.width0[k], I.lam, dnew[k]));
    }

    // the child records, read once: the first CUT_CACHE * blockDim children are
    // kept in registers for the three passes below, any further ones are read
    // again in each pass (phase 0)
    const bool ret = I.retire != 0;
    const int bd = blockDim.x;
    double cmn[CUT_CACHE], cmx[CUT_CACHE];
    uint32_t cfl[CUT_CACHE];
    int cna[CUT_CACHE];
#pragma unroll
    for (int q = 0; q < CUT_CACHE; ++q) {
        const int c = tid + q * bd;
        cmn[q] = INFINITY;
        cmx[q] = INFINITY;
        cfl[q] = F_INFEAS;
        cna[q] = 0;
        if (phase == 0 && c < C) {
            cmn[q] = as_global(I.minP)[c];
            cmx[q] = as_global(I.maxP)[c];
            cfl[q] = as_global(I.flags)[c];
            if (ret) cna[q] = as_global(I.na[cur ^ 1])[c];
        }
    }

    // solution estimate: least max B_p over feasible children (phases 2-4: the
    // least of the parts' minima, the first child attaining it)
    double m = INFINITY;
    int arg = INT_MAX;
    if (phase > 1) {
        for (int q = 0; q < Gb; ++q) {
            const double pm = pp[q].m;
            if (pm < m) {
                m = pm;
                arg = pp[q].arg;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < CUT_CACHE; ++q) {
        const bool dead = fin && cmn[q] > pprev;
        if (!dead && !(cfl[q] & (F_INFEAS | F_NOTFEAS))) m = fmin(m, cmx[q]);
    }
    for (int c = tid + CUT_CACHE * bd; phase == 0 && c < C; c += bd) {
        const double mnp = I.minP[c];
        const bool dead = fin && mnp > pprev;
        if (!dead && !(I.flags[c] & (F_INFEAS | F_NOTFEAS))) m = fmin(m, I.maxP[c]);
    }
    if (phase == 0) m = block_min1(m, shd);
    const bool update = (m < INFINITY) && (m <= pprev);
    if (phase == 0 && update) {
#pragma unroll
        for (int q = 0; q < CUT_CACHE; ++q) {
            const int c = tid + q * bd;
            const bool dead = fin && cmn[q] > pprev;
            if (c < C && !dead && !(cfl[q] & (F_INFEAS | F_NOTFEAS)) && cmx[q] == m) arg = min(arg, c);
        }
        for (int c = tid + CUT_CACHE * bd; c < C; c += bd) {
            const double mnp = I.minP[c];
            const bool dead = fin && mnp > pprev;
            if (!dead && !(I.flags[c] & (F_INFEAS | F_NOTFEAS)) && I.maxP[c] == m) arg = min(arg, c);
        }
        arg = block_min1_i(arg, shi);
    }
    const double p_up = update ? m : pprev;

    // least lower bound, keep mask, order-preserving compaction into live[];
    // in retiring mode also the prefix of the kept children's inequality units
    double plo = INFINITY;
    int base = 0;
    long long ubase = 0, abase = 0, asum = 0;
    const int lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
    if (phase == 2) {
        // this part's kept children, their units and carried patches
        long long kk = 0, uu = 0, aa = 0;
        for (int c = cbeg + tid; c < cend; c += bd) {
            const double mnp = as_global(I.minP)[c];
            const uint32_t fl = as_global(I.flags)[c];
            const bool dead = fin && mnp > pprev;
            if (dead || (fl & F_INFEAS) || !(mnp <= p_up)) continue;
            kk += 1;
            if (ret) {
                const int a = as_global(I.na[cur ^ 1])[c];
                uu += (a + TP1 - 1) / TP1;
                aa += a;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            kk += __shfl_xor(kk, o, 64);
            uu += __shfl_xor(uu, o, 64);
            aa += __shfl_xor(aa, o, 64);
        }
        if (lane == 0) {
            wact[w] = kk;
            wun[w] = uu;
            wap[w] = aa;
        }
        __syncthreads();
        if (tid == 0) {
            long long k2 = 0, u2 = 0, a2 = 0;
            for (int q = 0; q < nw; ++q) {
                k2 += wact[q];
                u2 += wun[q];
                a2 += wap[q];
            }
            pp[g].kept = (int)k2;
            pp[g].units = u2;
            pp[g].patches = a2;
        }
        return;
    }
    if (phase == 3) {
        // the kept children, units and patches of the parts before this one
        for (int q = 0; q < g; ++q) {
            base += pp[q].kept;
            ubase += pp[q].units;
            abase += pp[q].patches;
        }
    }
    // one chunk of blockDim children starting at c0 (uniform trip count: every
    // thread runs every chunk, so the barriers inside are reached by all)
    auto chunk = [&](int c0, double mnp, uint32_t fl, int a) {
        const int c = c0 + tid;
        bool keep = false;
        if (c < cend) {
            const bool dead = fin && mnp > pprev;
            if (!dead && !(fl & F_INFEAS)) {
                plo = fmin(plo, mnp);
                keep = mnp <= p_up;
            }
        }
        long long ti = 0;
        if (keep && ret) {
            ti = (a + TP1 - 1) / TP1;
            asum += a;
        }
        const long long ak = (keep && ret) ? a : 0;
        long long ui = ti, ai = ak;   // inclusive scans of the unit and patch counts within the wave
        for (int o = 1; o < 64; o <<= 1) {
            const long long y = __shfl_up(ui, o, 64), z = __shfl_up(ai, o, 64);
            if (lane >= o) { ui += y; ai += z; }
        }
        const unsigned long long bal = __ballot(keep);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[w] = __popcll(bal);
        if (lane == 63) { wun[w] = ui; wap[w] = ai; }
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            long long uacc = 0, aacc = 0;
            for (int q = 0; q < nw; ++q) {
                const int v = wsum[q];
                wsum[q] = acc;
                acc += v;
                const long long uv = wun[q];
                wun[q] = uacc;
                uacc += uv;
                const long long av = wap[q];
                wap[q] = aacc;
                aacc += av;
            }
            wsum[nw] = acc;
            wun[nw] = uacc;
            wap[nw] = aacc;
        }
        __syncthreads();
        const int jn = base + wsum[w] + before;
        const long long exl = ai - ak;   // this lane's patches before it in the wave
        if (keep) {
            as_global(I.live)[jn] = c;
            if (ret) {
                const long long u0 = ubase + wun[w] + ui - ti;
                as_global(I.upre)[jn] = u0;
                for (int q = 0; q < (int)ti; ++q) {
                    vec4i um;
                    um.x = jn;
                    um.y = c;
                    um.z = q;
                    um.w = a;
                    ((gmem_t<vec4i>)I.umap)[u0 + q] = um;
                }
            }
        }
        if (ret) {
            // the kept children's carried patches, in order, for the next step's
            // tiles: the chunk's kept children (their slots and patch offsets)
            // go to LDS, then every lane copies patches, finding each one's
            // child by a binary search over the offsets
            if (keep) {
                s_kc[jn - base] = c;
                s_ka[jn - base] = (int)(wap[w] + exl);
            }
            __syncthreads();
            const int kc = wsum[nw];
            const int ctot = (int)wap[nw];
            for (int e0 = tid; e0 < ctot; e0 += 4 * bd) {
                vec2i got[4];
                int dst[4], jk[4], ck[4];
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int e = e0 + h * bd;
                    dst[h] = -1;
                    if (e < ctot) {
                        int lo = 0, hi = kc - 1;   // last kept child starting at or before e
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (s_ka[mid] <= e) lo = mid; else hi = mid - 1;
                        }
                        ck[h] = s_kc[lo];
                        jk[h] = base + lo;
                        got[h] = ((gmem_t<const vec2i>)I.act[cur ^ 1])[(int64_t)ck[h] * I.count[1] +
                                                                        (e - s_ka[lo])];
                        dst[h] = e;
                    }
                }
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    if (dst[h] >= 0) {
                        vec4i pm;
                        pm.x = jk[h];
                        pm.y = ck[h];
                        pm.z = got[h].x;
                        pm.w = got[h].y;
                        ((gmem_t<vec4i>)I.pmap)[abase + dst[h]] = pm;
                    }
            }
        }
        base += wsum[nw];
        ubase += wun[nw];
        abase += wap[nw];
        __syncthreads();
    };
    if (phase == 0) {
#pragma unroll
        for (int q = 0; q < CUT_CACHE; ++q) {
            if (q * bd >= C) break;
            chunk(q * bd, cmn[q], cfl[q], cna[q]);
        }
    }
    if (phase != 4) {
        for (int c0 = cbeg + (phase == 0 ? CUT_CACHE * bd : 0); c0 < cend; c0 += bd) {
            const int c = c0 + tid;
            double mnp = INFINITY;
            uint32_t fl = F_INFEAS;
            int a = 0;
            if (c < cend) {
                mnp = as_global(I.minP)[c];
                fl = as_global(I.flags)[c];
                if (ret) a = as_global(I.na[cur ^ 1])[c];
            }
            chunk(c0, mnp, fl, a);
        }
    }
    if (phase == 3) return;
    if (phase == 4) {
        // the totals of all parts
        for (int q = 0; q < Gb; ++q) {
            base += pp[q].kept;
            ubase += pp[q].units;
            asum += pp[q].patches;
            plo = fmin(plo, pp[q].plo);
        }
    }
    // least lower bound and the inequality patches the kept children carry,
    // in one reduction
    // (phase 4 has the totals in every lane already)
    if (phase == 0) {
        plo = wave_min(plo);
        for (int o = 32; o > 0; o >>= 1) asum += __shfl_xor(asum, o, 64);
        if (lane == 0) {
            s_plo[w] = plo;
            wact[w] = asum;
        }
        __syncthreads();
        plo = s_plo[0];
        asum = 0;
        for (int q = 0; q < nw; ++q) {
            plo = fmin(plo, s_plo[q]);
            asum += wact[q];
        }
    }
    const int Kn = base;
    if (!I.retire) asum = (long long)Kn * I.count[1];

    // clear the flags of the next step's children, and in retiring mode their
    // carried counts (they go to the buffer of this step's parents); a split
    // cut clears them in Gb shares
    {
        const long long nclr = min((long long)nc * Kn, (long long)I.cap);
        const long long share = phase == 0 ? nclr : (nclr + Gb - 1) / Gb;
        const long long c1 = min(nclr, (phase == 0 ? 0 : (long long)g * share) + share);
        for (long long c = (phase == 0 ? 0 : (long long)g * share) + tid; c < c1; c += blockDim.x) {
            as_global(I.flags)[c] = 0;
            if (I.retire) as_global(I.na[cur])[c] = 0;
        }
    }
    if (g != 0) return;   // the state's updates: one workgroup

    // per axis (thread k): its depth, and x*'s box if the estimate moved
    const int nxt = cur ^ 1;
    if (tid < l) {
        if (I.fused || tid == r) st->depth[tid] = depth_k;
        if (update) {
            st->x_index[tid] = I.ids[nxt][(int64_t)arg * l + tid];
            st->x_depth[tid] = depth_k;
        }
    }
    if (tid == 0) {
        if (steps0 < MAX_TRACE) {
            TraceRec tr;
            tr.k_in = K;
            tr.k_kept = Kn;
            tr.p_up = p_up;
            tr.p_lo = plo;
            tr.a_in = alive0;
            tr.a_kept = asum;
            I.trace[steps0] = tr;
        }
        st->a_live = asum;
        if (I.retire) {
            I.upre[Kn] = ubase;
            st->u1 = ubase;
            st->htop[cur] = 0;   // this step's parents' heap takes the next children
        }
        st->steps = steps0 + 1;
        if (update) st->has_x = 1;
        st->p_up = p_up;
        st->p_lo = plo;
        st->K = Kn;
        st->cur = nxt;
        if (Kn == 0) {
            st->status = ST_INFEASIBLE;
            signal_host(I);
        } else if (p_up < INFINITY && p_up - plo <= I.eps && width <= I.delta) {
            st->status = ST_OPTIMAL;
            signal_host(I);
        } else {
            // the next direction: axis 0 again after a round, the next axis in the
            // order 1..l, or the widest axis; the iteration count advances every
            // l directional steps (every round)
            const int rn = I.fused ? 0 : (I.rule == 1 ? widest_axis(I.width0, I.lam, dnew, l) : (r + 1) % l);
            st->r = rn;
            const int nn = n0 + ((I.fused || (steps0 + 1) % l == 0) ? 1 : 0);
            st->n = nn;
            if (nn == I.N) {
                st->status = ST_MAXITER;
                signal_host(I);
            }
        }
    }
}

template <int NT>
__device__ __forceinline__ void cut_run(const DevInst* __restrict__ insts, int b)
{
    cut_phase<NT>(insts, nullptr, b, 0, 0, 1, nullptr, LLONG_MAX, 1);
}

// The cut, one workgroup per problem; with split > 0, problems with more than
// split children at this step are left to k_cut_split.
__global__ __launch_bounds__(CUT_THREADS) void k_cut(const DevInst* __restrict__ insts, int n_inst,
                                                     long long split)
{
    (void)n_inst;
    cut_phase<CUT_THREADS>(insts, nullptr, blockIdx.x, 0, 0, 1, nullptr, split, 1);
}

// One phase (1-4) of the split cut: workgroup (b, g) = (blockIdx / G, blockIdx % G).
__global__ __launch_bounds__(CUT_THREADS) void k_cut_split(const DevInst* __restrict__ insts,
                                                           const StepInfo* __restrict__ info, int phase, int G,
                                                           CutPart* __restrict__ parts, long long split,
                                                           int part)
{
    const int b = blockIdx.x / G, g = blockIdx.x - b * G;
    cut_phase<CUT_THREADS>(insts, info, b, phase, g, G, parts, split, part);
}

// ------------------------------------------------------------------ k_steps

// Waits until every workgroup of the grid has arrived at barrier number gen
// (bar[0] counts arrivals; the grid is co-resident, launched cooperatively).
// Every wait is bounded: after STEP_WAIT_TICKS of the 100 MHz clock the
// workgroup sets bar[1], reports it in the host word herr and returns false,
// and every workgroup returns false once bar[1] is set, so the kernel always
// ends.
constexpr unsigned long long STEP_WAIT_TICKS = 1000000000ull;   // 10 s
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned gen, int* herr)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();   // this workgroup's writes before its arrival
        atomicAdd(&bar[0], 1u);
        const unsigned target = gen * gridDim.x;
        const unsigned long long t0 = wall_clock64();
        int ok = 1;
        while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                wall_clock64() - t0 > STEP_WAIT_TICKS) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
        if (!ok) {
            atomicExch(&bar[1], 1u);
            __hip_atomic_store(herr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __threadfence();   // the other workgroups' writes after it
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Up to n_steps steps of a batch of one precision in one cooperative launch:
// per step the subdivision (plan formed in LDS, as k_sub with FUSE), a grid
// barrier, the cut (workgroup b takes problems b, b + grid, ...), a grid
// barrier.  The sequence of operations per step is that of the k_sub and
// k_cut launches.  Stops early once the plan of a step has no units (no
// problem of the batch is running).
template <typename T, int MM, int LB>
__global__ __launch_bounds__(SUB_THREADS, 2) void k_steps(const DevInst* __restrict__ insts, int n_inst,
                                                      long long* __restrict__ plan,
                                                      StepInfo* __restrict__ info, int tem, int tpm, int nr,
                                                      int n_steps, unsigned* __restrict__ bar, int* herr)
{
    unsigned gen = 0;
    for (int s = 0; s < n_steps; ++s) {
        const bool work = sub_run<T, MM, LB, true, false>(insts, n_inst, plan, info, tem, tpm, nr);
        if (!grid_barrier(bar, ++gen, herr)) return;
        if (!work) return;   // the same plan in every workgroup: all leave together
        for (int b = blockIdx.x; b < n_inst; b += gridDim.x) {
            cut_run<SUB_THREADS>(insts, b);
            __syncthreads();
        }
        if (!grid_barrier(bar, ++gen, herr)) return;
    }
}

// ------------------------------------------------------------------ certification

// Certification of x*, one workgroup per (problem, run of ppb polynomials): the
// FP64 patch of x* from the accurate root with the sub-interval transforms, its
// min / max and a rigorous error bound: the root's own bound (rows of T sum to
// one) plus, per axis, gamma_{6m+6} times the |T| |root| chain (transform
// entries within gamma_{5m} relative, one product more).
//   The workgroup first puts the root patches of its run into LDS (all loads in
// flight at once) while it builds the transforms of every kind and axis; then
// each wave takes one polynomial per round and each lane whole fibres, the
// signed chain and the |.| chain side by side.  The basis values come from
// b^q_s(t) = C(q,s) t^s (1-t)^(q-s): at the midpoint parameter 1 - t is exact
// (t is dyadic), so each carries at most q+1 roundings; with another
// subdivision parameter 1 - t carries one rounding more and each value at most
// 2q: within the gamma_{2q} that the bound on T assumes.  The box certified is
// the one whose interval the host reports (the same FP64 recurrence from the
// index bits).
// LDS (doubles): transforms, KINDS * l blocks of mm^2 (mm: the problem's longest
// fibre); basis tables, 2 KINDS l mm^2; then 2 ppb slots of max_S.
__global__ __launch_bounds__(256) void k_certify(const DevInst* __restrict__ insts, int n,
                                                const int* __restrict__ pre, int max_S, int ppb,
                                                int tm_words)
{
    extern __shared__ double shc[];
    __shared__ AxisGeo s_geo[KINDS][MAXL];
    __shared__ int s_S[KINDS], s_cnt[KINDS];
    __shared__ long long s_off[KINDS];
    const int bi = find_block(pre, n, blockIdx.x);
    const DevInst& I = insts[bi];
    const InstState* st = I.st;
    if (!st->has_x) return;
    const int l = I.l, nw = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int pb = (blockIdx.x - pre[bi]) * ppb;
    const int pe = min(I.n_polys, pb + ppb);
    const int c0 = I.count[0], c1 = I.count[1];
    double* tm = shc;
    double* tab = shc + tm_words;
    double* slot = tab + 2 * tm_words;   // polynomial q of the run: signed at 2q, |.| at 2q+1
    // root patches of the run into LDS, up to 8 loads in flight per thread
    {
        const int S0 = I.S[0], S1 = I.S[1], S2 = I.S[2];
        const int64_t o0 = I.off[0], o1 = I.off[1], o2 = I.off[2];
        const int total = (pe - pb) * max_S;
        for (int e0 = threadIdx.x; e0 < total; e0 += 8 * blockDim.x) {
            double v[8];
            int dst[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = e0 + k * blockDim.x;
                dst[k] = -1;
                if (e < total) {
                    const int q = e / max_S, i = e - q * max_S;
                    int poly = pb + q, kind = 0;
                    if (poly >= c0) {
                        poly -= c0;
                        kind = 1;
                        if (poly >= c1) { poly -= c1; kind = 2; }
                    }
                    const int S = kind == 0 ? S0 : (kind == 1 ? S1 : S2);
                    if (i < S) {
                        v[k] = as_global(I.racc)[(kind == 0 ? o0 : (kind == 1 ? o1 : o2)) + (int64_t)poly * S + i];
                        dst[k] = 2 * q * max_S + i;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (dst[k] >= 0) {
                    slot[dst[k]] = v[k];
                    slot[dst[k] + max_S] = fabs(v[k]);
                }
        }
    }
    if (threadIdx.x < KINDS) {
        const int kind = threadIdx.x;
        s_S[kind] = I.S[kind];
        s_cnt[kind] = I.count[kind];
        s_off[kind] = I.off[kind];
        stage_geo(s_geo[kind], I.dims[kind], l, I.S[kind]);
    }
    int mm = 1;
    for (int kind = 0; kind < KINDS; ++kind)
        if (I.count[kind] > 0)
            for (int k = 0; k < l; ++k) mm = max(mm, I.dims[kind][k]);
    const int mm2 = mm * mm;
    const int nb = KINDS * l;
    // basis tables: block 2 (kind * l + axis) + side holds b^q_s(t) at q * m + s,
    // t = a (side 0) or b (side 1) of axis k of x*
    for (int e = threadIdx.x; e < 2 * nb * mm2; e += blockDim.x) {
        const int bk = e / mm2, ka = bk >> 1, side = bk & 1, kind = ka / l, k = ka - kind * l;
        const int q2 = e - bk * mm2;
        if (I.count[kind] == 0) continue;
        const int m = I.dims[kind][k];
        const int q = q2 / m, s2 = q2 - q * m;
        if (q >= m || s2 > q) continue;
        double ta, tb;
        unit_interval(I.lam, st->x_depth[k], st->x_index[k], ta, tb);
        const double t = side ? tb : ta;
        const double u = 1.0 - t;
        double v = 1.0;
        for (int i = 0; i < s2; ++i) v *= t;
        double v2 = 1.0;
        for (int i = 0; i < q - s2; ++i) v2 *= u;
        // C(q, s2), exact in FP64 for q < 16
        double cq = 1.0;
        for (int i = 1; i <= s2; ++i) cq = cq * (double)(q - s2 + i) / (double)i;
        tab[e] = cq * v * v2;
    }
    __syncthreads();
    // T[k][j] = sum_s b^{n-k}_s(a) b^k_{j-s}(b), one entry per thread
    for (int e = threadIdx.x; e < nb * mm2; e += blockDim.x) {
        const int ka = e / mm2, kind = ka / l, k = ka - kind * l, q = e - ka * mm2;
        if (s_cnt[kind] == 0) continue;
        const int m = s_geo[kind][k].m, nd = m - 1;
        if (q >= m * m) continue;
        const int row = q / m, j = q - row * m;
        const double* Ba = tab + (2 * ka) * mm2;
        const double* Bb = Ba + mm2;
        const int s0 = max(0, j - row), s1 = min(nd - row, j);
        double acc = 0.0;
        for (int s2 = s0; s2 <= s1; ++s2) acc += Ba[(nd - row) * m + s2] * Bb[row * m + (j - s2)];
        tm[ka * mm2 + q] = acc;
    }
    __syncthreads();
    for (int r = 0; r < l; ++r) {
        MatOffs mo;
        for (int t = 0; t < KINDS; ++t) {
            mo.first[t] = (t * l + r) * mm2;
            mo.second[t] = -1;
        }
        run_axis<true>(slot, 2 * max_S, max_S, 2, pb, pe, c0, c1, s_geo, r, tm, mo);
        __syncthreads();
    }
    for (int p0 = pb; p0 < pe; p0 += nw) {
        const int poly = p0 + w;
        const bool act = poly < pe;
        int kind = 0, idx = poly;
        if (idx >= c0) {
            idx -= c0;
            kind = 1;
            if (idx >= c1) { idx -= c1; kind = 2; }
        }
        const int S = s_S[kind];
        double* x = slot + 2 * (poly - pb) * max_S;
        double* xa = x + max_S;
        double mn = INFINITY, mx = -INFINITY, am = 0.0;
        if (act)
            for (int e = lane; e < S; e += 64) {
                mn = fmin(mn, x[e]);
                mx = fmax(mx, x[e]);
                am = fmax(am, xa[e]);
            }
        for (int o = 32; o > 0; o >>= 1) {
            mn = fmin(mn, __shfl_xor(mn, o, 64));
            mx = fmax(mx, __shfl_xor(mx, o, 64));
            am = fmax(am, __shfl_xor(am, o, 64));
        }
        if (act && lane == 0) {
            double gsum = 0.0;
            for (int r = 0; r < l; ++r) gsum += gamma64(6 * s_geo[kind][r].m + 6);
            I.cert[3 * poly + 0] = mn;
            I.cert[3 * poly + 1] = mx;
            I.cert[3 * poly + 2] = I.root_err[poly] + gsum * am * 1.01;
        }
    }
}

// One workgroup per problem: every g_i certified <= 0, every h_j inside the
// band, p_cert = max B_p + e rounded up.
__global__ __launch_bounds__(256) void k_certify_final(const DevInst* __restrict__ insts, int n)
{
    __shared__ int s_bad;
    __shared__ double s_e[4];
    const DevInst& I = insts[blockIdx.x];
    InstState* st = I.st;
    if (!st->has_x) {
        if (threadIdx.x == 0) { st->cert_ok = 0; st->p_cert = INFINITY; st->cert_err = 0.0; }
        return;
    }
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    int bad = 0;
    double emax = 0.0;
    for (int p = threadIdx.x; p < I.n_polys; p += blockDim.x) {
        const double mn = I.cert[3 * p], mx = I.cert[3 * p + 1], e = I.cert[3 * p + 2];
        emax = fmax(emax, e);
        if (p < I.count[0]) continue;
        if (p < I.count[0] + I.count[1]) {
            if (!(mx + e <= 0.0)) bad = 1;
        } else if (!(-I.eps_eq <= mn - e && mn + e <= 0.0 && 0.0 <= mx - e && mx + e <= I.eps_eq)) {
            bad = 1;
        }
    }
    if (bad) atomicOr(&s_bad, 1);
    for (int o = 32; o > 0; o >>= 1) emax = fmax(emax, __shfl_xor(emax, o, 64));
    if ((threadIdx.x & 63) == 0) s_e[threadIdx.x >> 6] = emax;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) emax = fmax(emax, s_e[w]);
        st->cert_ok = s_bad ? 0 : 1;
        st->p_cert = nextafter(I.cert[1] + I.cert[2], INFINITY);
        st->cert_err = emax;
    }
}

// ------------------------------------------------------------------ list read-out

template <typename T>
__global__ void k_pack(DevInst I, double* __restrict__ out, uint32_t* __restrict__ ids_out,
                       double* __restrict__ err_out, int64_t W)
{
    const InstState* st = I.st;
    const int j = blockIdx.x;
    if (j >= st->K) return;
    const int slot = I.live[j];
    const int cur = st->cur;
    const T* src = (const T*)I.buf[cur] + (int64_t)slot * I.stride;
    double* o = out + (int64_t)j * W;
    // cost and equalities from the slot; the inequalities from the slot, or in
    // retiring mode NaN except the carried ones, which come from the heap
    // FP32 mode: a patch's coefficients are its FP64 base plus the stored values
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    const double* pb = I.fp32 ? I.base[cur] + (int64_t)slot * I.n_polys : nullptr;
    for (int kind = 0; kind < KINDS; ++kind) {
        const int64_t n = (int64_t)I.count[kind] * I.S[kind];
        const bool inheap = I.retire && kind == 1;
        const int p0 = kind == 0 ? 0 : I.count[0] + (kind == 2 ? I.count[1] : 0);
        for (int64_t e = threadIdx.x; e < n; e += blockDim.x)
            o[I.off[kind] + e] = inheap ? nan
                                        : (double)src[I.soff[kind] + e] + (pb ? pb[p0 + e / I.S[kind]] : 0.0);
    }
    if (I.retire) {
        __syncthreads();
        const int na = I.na[cur][slot];
        const int2* act = I.act[cur] + (int64_t)slot * I.count[1];
        const T* h = (const T*)I.heap[cur];
        const int64_t S = I.S[1];
        for (int64_t e = threadIdx.x; e < (int64_t)na * S; e += blockDim.x) {
            const int64_t q = e / S;
            const int2 a = act[q];
            o[I.off[1] + (int64_t)a.x * S + (e - q * S)] =
                (double)h[(int64_t)a.y * S + (e - q * S)] + (pb ? pb[I.count[0] + a.x] : 0.0);
        }
    }
    if (threadIdx.x < (unsigned)I.l)
        ids_out[(int64_t)j * I.l + threadIdx.x] = I.ids[st->cur][(int64_t)slot * I.l + threadIdx.x];
    if (I.fp32 && err_out)
        for (int p = threadIdx.x; p < I.n_polys; p += blockDim.x)
            err_out[(int64_t)j * I.n_polys + p] = (double)I.err[st->cur][(int64_t)slot * I.n_polys + p].x;
}

__global__ void k_gather(const DevInst* __restrict__ insts, int n, InstState* __restrict__ out)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n; b += gridDim.x * blockDim.x)
        out[b] = *insts[b].st;
}

// ------------------------------------------------------------------ host launchers

// Device properties the launchers need, cached per device (the current device
// of the calling thread) under a lock: distinct problem handles may be driven
// from distinct threads and devices.
constexpr int MAX_DEVICES = 64;
struct DevProps {
    bool ok = false;
    int cus = 0;
    size_t lds = 65536;
};
static std::mutex g_props_mu;
static DevProps g_props[MAX_DEVICES];

static int current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) dev = 0;
    return dev;
}

static DevProps device_props(int dev)
{
    std::lock_guard<std::mutex> lk(g_props_mu);
    DevProps& p = g_props[dev];
    if (!p.ok) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            p.lds = (size_t)v;
        v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            p.cus = v;
        p.ok = true;
    }
    return p;
}

// LDS bytes a workgroup may use on the current device
static size_t lds_per_block() { return device_props(current_device()).lds; }

// Resident workgroups per CU of `kernel` with `lds` dynamic LDS bytes on the
// current device, cached per (device, kernel, lds) under a lock; 0 if unknown.
static int occupancy_per_cu(const void* kernel, int threads, size_t lds)
{
    struct Entry {
        int dev;
        const void* k;
        int threads;
        size_t lds;
        int per_cu;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    const int dev = current_device();
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Entry& e : cache)
            if (e.dev == dev && e.k == kernel && e.threads == threads && e.lds == lds) return e.per_cu;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess) nb = 0;
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back(Entry{dev, kernel, threads, lds, nb});
    return nb;
}


int root_run_length(int max_S, int tm_words)
{
    // polynomials per workgroup: one slot each beside the matrices in the
    // workgroup's LDS, at most 16
    const long long room = (long long)(lds_per_block() / sizeof(double)) - 2LL * tm_words;
    return (int)std::max(0LL, std::min(16LL, room / std::max(1, max_S)));
}

hipError_t launch_reset_root(const DevInst* d_insts, int n, const int* d_pre, int total_blocks, int max_S,
                             int tm_words, int ppb, hipStream_t s)
{
    if (ppb < 1 || ppb > root_run_length(max_S, tm_words)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reset, dim3((n + 63) / 64), dim3(64), 0, s, d_insts, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int mat_words = 2 * tm_words;
    const size_t lds = ((size_t)mat_words + (size_t)ppb * max_S) * sizeof(double);
    hipLaunchKernelGGL(k_root, dim3(total_blocks), dim3(256), lds, s, d_insts, n, d_pre, max_S, ppb, mat_words);
    return hipGetLastError();
}

hipError_t launch_racc(const DevInst* d_insts, int n, const int* d_pre, int total_polys, int max_S,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_racc, dim3(total_polys), dim3(256), 2 * (size_t)max_S * sizeof(double), s,
                       d_insts, n, d_pre);
    return hipGetLastError();
}

hipError_t launch_plan(const DevInst* d_insts, int n, long long* plan, StepInfo* info, hipStream_t s)
{
    // one lane per problem (the kernel loops over larger batches)
    const int threads = std::min(1024, std::max(64, (n + 63) / 64 * 64));
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(threads), 0, s, d_insts, n, plan, info);
    return hipGetLastError();
}

// Dynamic LDS bytes of k_sub for tiles of at most tem coefficients and tpm
// patches (the carve-up at the kernel's start, 16-byte aligned pieces).
size_t sub_lds_bytes(int tem, int tpm, bool fp32, int nr)
{
    const size_t el = fp32 ? 4 : 8;
    auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
    return r16((size_t)nr * tem * el) + r16((size_t)5 * tpm * (nr > 2 ? 3 : 1) * el) + 3 * r16((size_t)tpm * 8) +
           r16((size_t)tpm * el) + r16((size_t)tpm * 4) + r16((size_t)tpm * 8) + r16((size_t)tpm * 4) +
           3 * r16((size_t)tpm * 16) + r16((size_t)tpm * 4) +
           r16((size_t)(2 * tpm + 2) * 4) + r16((size_t)2 * tpm * 4) + r16((size_t)nr * tpm * 4) +
           r16((size_t)2 * tpm * 4) + r16((size_t)(tpm + 1) * 4) + r16((size_t)tpm * 8);
}

// With ev0/ev1 the launch stamps them at the kernel's own start and end.
template <typename T, int MM, bool FUSE, bool MF>
static hipError_t launch_sub_t(const DevInst* d_insts, int n, long long* plan, StepInfo* info, int grid,
                               int tem, int tpm, int nr, int wg_cap, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    // registers per thread for a tile in flight: the largest tile / 256 lanes
    constexpr int LB = (sizeof(T) == 8 ? MAX_TILE64 : MAX_TILE32) / SUB_THREADS;
    if (tem > LB * SUB_THREADS || tpm < 1 || tpm > SUB_THREADS || (nr != 2 && nr != NCMAX))
        return hipErrorInvalidValue;
    const size_t lds = sub_lds_bytes(tem, tpm, sizeof(T) == 4, nr);
    // no more workgroups than fit on the device at once: the rest would only
    // queue, while resident ones walk the units with the next tile in flight
    const int cus = device_props(current_device()).cus;
    int per_cu = occupancy_per_cu((const void*)k_sub<T, MM, LB, FUSE, MF>, SUB_THREADS, lds);
    if (wg_cap > 0 && per_cu > 0) per_cu = std::min(per_cu, wg_cap);
    if (cus > 0 && per_cu > 0) grid = std::min(grid, cus * per_cu);
    if (ev0)
        hipExtLaunchKernelGGL((k_sub<T, MM, LB, FUSE, MF>), dim3(grid), dim3(SUB_THREADS), lds, s, ev0, ev1, 0,
                              d_insts, n, plan, info, tem, tpm, nr);
    else
        hipLaunchKernelGGL((k_sub<T, MM, LB, FUSE, MF>), dim3(grid), dim3(SUB_THREADS), lds, s, d_insts, n, plan,
                           info, tem, tpm, nr);
    return hipGetLastError();
}

template <typename T, int MM, bool MF>
static hipError_t launch_sub_f(const DevInst* d_insts, int n, long long* plan, StepInfo* info, bool fuse,
                               int grid, int tem, int tpm, int nr, int wg_cap, hipStream_t s, hipEvent_t ev0,
                               hipEvent_t ev1)
{
    if (fuse)
        return launch_sub_t<T, MM, true, MF>(d_insts, n, plan, info, grid, tem, tpm, nr, wg_cap, s, ev0, ev1);
    return launch_sub_t<T, MM, false, MF>(d_insts, n, plan, info, grid, tem, tpm, nr, wg_cap, s, ev0, ev1);
}

hipError_t launch_sub(const DevInst* d_insts, int n, long long* plan, StepInfo* info, bool fuse,
                      bool fp32, bool mfma, int maxm, int grid, int tem, int tpm, int nr, int wg_cap, hipStream_t s,
                      hipEvent_t ev0, hipEvent_t ev1)
{
    if (fuse && n > PLAN_FUSE_MAX) return hipErrorInvalidValue;
    if (grid <= 0) {
        if (!fuse) return hipSuccess;
        grid = 1;   // the plan is still formed and written
    }
    if (fp32 && mfma) {
        if (maxm <= 8)
            return launch_sub_f<float, 8, true>(d_insts, n, plan, info, fuse, grid, tem, tpm, nr, wg_cap, s, ev0, ev1);
        return launch_sub_f<float, 16, true>(d_insts, n, plan, info, fuse, grid, tem, tpm, nr, wg_cap, s, ev0, ev1);
    }
    if (fp32) {
        if (maxm <= 8)
            return launch_sub_f<float, 8, false>(d_insts, n, plan, info, fuse, grid, tem, tpm, nr, wg_cap, s, ev0, ev1);
        return launch_sub_f<float, 16, false>(d_insts, n, plan, info, fuse, grid, tem, tpm, nr, wg_cap, s, ev0, ev1);
    }
    if (maxm <= 8)
        return launch_sub_f<double, 8, false>(d_insts, n, plan, info, fuse, grid, tem, tpm, nr, wg_cap, s, ev0, ev1);
    return launch_sub_f<double, 16, false>(d_insts, n, plan, info, fuse, grid, tem, tpm, nr, wg_cap, s, ev0, ev1);
}

template <typename T, int MM>
static hipError_t launch_steps_t(const DevInst* d_insts, int n, long long* plan, StepInfo* info, int tem, int tpm,
                                 int nr, int wg_cap, int n_steps, unsigned* bar, int* herr, hipStream_t s)
{
    constexpr int LB = (sizeof(T) == 8 ? MAX_TILE64 : MAX_TILE32) / SUB_THREADS;
    if (tem > LB * SUB_THREADS || tpm < 1 || tpm > SUB_THREADS || (nr != 2 && nr != NCMAX))
        return hipErrorInvalidValue;
    const size_t lds = sub_lds_bytes(tem, tpm, sizeof(T) == 4, nr);
    const void* kern = (const void*)k_steps<T, MM, LB>;
    const int cus = device_props(current_device()).cus;
    int per_cu = occupancy_per_cu(kern, SUB_THREADS, lds);
    if (wg_cap > 0 && per_cu > 0) per_cu = std::min(per_cu, wg_cap);
    if (cus <= 0 || per_cu <= 0) return hipErrorInvalidConfiguration;
    // the barrier's counters start at zero (a fill kernel, as for the flags)
    hipError_t e = hipMemsetAsync(bar, 0, 2 * sizeof(unsigned), s);
    if (e != hipSuccess) return e;
    int grid = cus * per_cu;
    void* args[] = {(void*)&d_insts, (void*)&n, (void*)&plan, (void*)&info, (void*)&tem,
                    (void*)&tpm, (void*)&nr, (void*)&n_steps, (void*)&bar, (void*)&herr};
    // co-residency of the whole grid is what the grid barrier relies on: the
    // cooperative launch fails rather than start a grid that does not fit
    return hipLaunchCooperativeKernel(kern, dim3(grid), dim3(SUB_THREADS), args, (unsigned)lds, s);
}

hipError_t launch_steps(const DevInst* d_insts, int n, long long* plan, StepInfo* info, bool fp32, int maxm,
                        int tem, int tpm, int nr, int wg_cap, int n_steps, unsigned* bar, int* herr,
                        hipStream_t s)
{
    if (n > PLAN_FUSE_MAX || n_steps <= 0) return hipErrorInvalidValue;
    if (fp32) {
        if (maxm <= 8)
            return launch_steps_t<float, 8>(d_insts, n, plan, info, tem, tpm, nr, wg_cap, n_steps, bar, herr, s);
        return launch_steps_t<float, 16>(d_insts, n, plan, info, tem, tpm, nr, wg_cap, n_steps, bar, herr, s);
    }
    if (maxm <= 8)
        return launch_steps_t<double, 8>(d_insts, n, plan, info, tem, tpm, nr, wg_cap, n_steps, bar, herr, s);
    return launch_steps_t<double, 16>(d_insts, n, plan, info, tem, tpm, nr, wg_cap, n_steps, bar, herr, s);
}

hipError_t launch_rederive(const DevInst* d_insts, int n, const long long* plan, const StepInfo* info,
                           int grid, int tgrid, size_t lds, hipStream_t s)
{
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tmat, dim3(tgrid), dim3(256), 0, s, d_insts, n, plan);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rederive, dim3(grid), dim3(SUB_THREADS), lds, s, d_insts, n, plan, info);
    return hipGetLastError();
}

hipError_t launch_cut(const DevInst* d_insts, const StepInfo* info, int n, int64_t max_children,
                      long long split, int part, CutPart* parts, int64_t parts_cap, hipStream_t s)
{
    // short lists: four waves walk the children in a few passes with cheaper
    // barriers; longer ones take eight waves (fewer passes, the carried-patch
    // copy twice as wide), the longest the full workgroup
    const int threads = max_children <= 1024 ? 256 : (max_children <= 8192 ? 512 : CUT_THREADS);
    const bool splitting = split > 0 && max_children > split;
    if (splitting && part < 1) return hipErrorInvalidValue;
    const int G = splitting ? (int)((max_children + part - 1) / part) : 1;
    if (splitting && (int64_t)n * G > parts_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cut, dim3(n), dim3(threads), 0, s, d_insts, n, splitting ? split : LLONG_MAX);
    hipError_t e = hipGetLastError();
    // problems with more children than split: four launches over G workgroups each
    for (int phase = 1; splitting && phase <= 4 && e == hipSuccess; ++phase) {
        hipLaunchKernelGGL(k_cut_split, dim3(n * G), dim3(CUT_THREADS), 0, s, d_insts, info, phase, G, parts,
                           split, part);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_gather(const DevInst* d_insts, int n, InstState* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, s, d_insts, n, out);
    return hipGetLastError();
}

int certify_run_length(int max_S, int tm_words)
{
    // polynomials per workgroup: two slots each beside the transforms and the
    // basis tables in the workgroup's LDS, at most 16
    const long long room = (long long)(lds_per_block() / sizeof(double)) - 3LL * tm_words;
    return (int)std::max(0LL, std::min(16LL, room / (2LL * std::max(1, max_S))));
}

hipError_t launch_certify(const DevInst* d_insts, int n, const int* d_pre, int total_blocks,
                          int max_S, int tm_words, int ppb, hipStream_t s)
{
    if (ppb < 1 || ppb > certify_run_length(max_S, tm_words)) return hipErrorInvalidValue;
    const size_t lds = (3 * (size_t)tm_words + 2 * (size_t)ppb * max_S) * sizeof(double);
    hipLaunchKernelGGL(k_certify, dim3(total_blocks), dim3(256), lds, s, d_insts, n, d_pre, max_S, ppb,
                       tm_words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_certify_final, dim3(n), dim3(256), 0, s, d_insts, n);
    return hipGetLastError();
}

hipError_t launch_pack(const DevInst& I, int K, double* out, uint32_t* ids, double* err, int64_t W,
                       hipStream_t s)
{
    if (K <= 0) return hipSuccess;
    if (I.fp32)
        hipLaunchKernelGGL(k_pack<float>, dim3(K), dim3(256), 0, s, I, out, ids, err, W);
    else
        hipLaunchKernelGGL(k_pack<double>, dim3(K), dim3(256), 0, s, I, out, ids, err, W);
    return hipGetLastError();
}

}  // namespace pcba
