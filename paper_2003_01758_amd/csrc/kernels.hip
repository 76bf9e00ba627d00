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
#include "kernels.h"

#include <float.h>
#include <math.h>

namespace pcba {

// ------------------------------------------------------------------ small helpers

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

// Units of work of one step, per class of problem:
//   class 0: FP64 problems (k_sub<double>)
//   class 1: FP32 problems splitting their FP32 parents (k_sub<float>)
//   class 2: FP32 problems whose step re-derives the children from the root
// plan[c*(n+1) + b] = first unit of problem b in class c; plan[c*(n+1) + n] = total.
__device__ __forceinline__ int unit_class(const DevInst& I, const InstState* st)
{
    if (!I.fp32) return 0;
    const bool due = I.rederive > 0 && ((st->steps + 1) % I.rederive) == 0;
    return due ? 2 : 1;
}

__global__ __launch_bounds__(1024) void k_plan(const DevInst* __restrict__ insts, int n,
                                               long long* __restrict__ plan)
{
    __shared__ long long wtot[3][16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
    long long carry[3] = {0, 0, 0};
    for (int b0 = 0; b0 < n; b0 += blockDim.x) {
        const int b = b0 + t;
        long long v[3] = {0, 0, 0};
        if (b < n) {
            const DevInst& I = insts[b];
            InstState* st = I.st;
            if (st->status == ST_RUNNING) {
                // memory test of Alg. PCBA at the start of the iteration:
                // 2 length(L) > M ends the solve; more than the device list
                // holds pauses the problem until the host grows the list
                if ((int64_t)st->K > st->peak) st->peak = st->K;
                if (2LL * st->K > (int64_t)I.M) st->status = ST_MEMLIMIT;
                else if (2LL * st->K > (int64_t)I.cap) st->status = ST_GROW;
                else v[unit_class(I, st)] = (long long)st->K * I.T;
            }
        }
        for (int c = 0; c < 3; ++c) {
            long long x = v[c];
            for (int o = 1; o < 64; o <<= 1) {
                long long y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (lane == 63) wtot[c][w] = x;
            v[c] = x - v[c];  // exclusive within the wave
        }
        __syncthreads();
        for (int c = 0; c < 3; ++c) {
            long long before = carry[c];
            for (int q = 0; q < w; ++q) before += wtot[c][q];
            if (b < n) plan[c * (n + 1) + b] = before + v[c];
            long long tot = 0;
            for (int q = 0; q < nw; ++q) tot += wtot[c][q];
            carry[c] += tot;
        }
        __syncthreads();
    }
    if (t < 3) plan[t * (n + 1) + n] = carry[t];
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

// One workgroup per polynomial.  mats holds, per kind and axis, the pre-map
// matrix A (x = lo + w t substituted) followed by the conversion matrix U,
// each m x m row-major; matoff[kind*MAXL + r] is the offset of that pair.
__global__ __launch_bounds__(256) void k_root(DevInst I, const double* __restrict__ mono,
                                             const double* __restrict__ mats,
                                             const int* __restrict__ matoff,
                                             double* __restrict__ root,
                                             double* __restrict__ root_err)
{
    extern __shared__ double sh[];
    __shared__ double red[4];
    const int poly = blockIdx.x;
    int kind = 0, idx = poly;
    if (idx >= I.count[0]) { idx -= I.count[0]; kind = 1; if (idx >= I.count[1]) { idx -= I.count[1]; kind = 2; } }
    const int S = I.S[kind];
    const int64_t off = I.off[kind] + (int64_t)idx * S;
    double* x = sh;       // current values
    double* y = sh + S;   // scratch
    int q_total = 2;
    double amax = 0.0;
    // pass 0: the conversion itself; pass 1: the same chain on |coefficients|
    // with |matrices|, whose largest entry bounds the rounding error
    for (int absp = 0; absp < 2; ++absp) {
        for (int e = threadIdx.x; e < S; e += blockDim.x) x[e] = absp ? fabs(mono[off + e]) : mono[off + e];
        __syncthreads();
        for (int r = 0; r < I.l; ++r) {
            FibreGeom g = fibre_geom(I.dims[kind], I.l, r, S);
            const double* A = mats + matoff[kind * MAXL + r];
            const double* U = A + g.m * g.m;
            if (absp) q_total += 2 * (g.m + 4);
            for (int pass = 0; pass < 2; ++pass) {
                const double* Mx = pass ? U : A;
                double* src = pass ? y : x;
                double* dst = pass ? x : y;
                for (int f = threadIdx.x; f < g.F; f += blockDim.x) {
                    const int base = fibre_base(g, f);
                    for (int k = 0; k < g.m; ++k) {
                        double acc = 0.0;
                        for (int i = 0; i < g.m; ++i) {
                            const double mk = absp ? fabs(Mx[k * g.m + i]) : Mx[k * g.m + i];
                            acc += mk * src[base + i * g.stride];
                        }
                        dst[base + k * g.stride] = acc;
                    }
                }
                __syncthreads();
            }
        }
        for (int e = threadIdx.x; e < S; e += blockDim.x) {
            if (absp) amax = fmax(amax, x[e]);
            else root[off + e] = x[e];
        }
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
        root_err[poly] = gamma64(q_total) * m * 1.01;
    }
}

// Root item into slot 0 of buffer 0 (FP32 mode: rounded, with its error bound).
template <typename T>
__global__ void k_root_item(DevInst I, int64_t W)
{
    T* dst = (T*)I.buf[0];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < W;
         e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = (T)I.root[e];
    if (I.fp32 && blockIdx.x == 0) {
        // e0 = FP64 conversion bound + rounding to FP32 (half an ulp, taken as u = 2^-23 rel.)
        for (int p = threadIdx.x; p < I.n_polys; p += blockDim.x) {
            int kind = 0, idx = p;
            if (idx >= I.count[0]) { idx -= I.count[0]; kind = 1; if (idx >= I.count[1]) { idx -= I.count[1]; kind = 2; } }
            const int S = I.S[kind];
            const double* P = I.root + I.off[kind] + (int64_t)idx * S;
            double amax = 0.0;
            for (int e = 0; e < S; ++e) amax = fmax(amax, fabs(P[e]));
            I.err[0][p] = round_up_f(I.root_err[p] + amax * 0x1p-23 + 0x1p-126);
        }
    }
}

// ------------------------------------------------------------------ k_sub

template <typename T>
struct SubLds {
    // layout inside dynamic LDS
    T* a;        // parent tile, overwritten by the left child
    T* b;        // right child
    typename KeyOf<T>::type* key;  // per patch: minL, maxL, minR, maxR, maxabs(parent)
};

// One fibre of fixed length M: de Casteljau with parameter 1/2 in registers.
// After level lev, c[0] is the left child's coefficient lev and c[M-1-lev] the
// right child's coefficient M-1-lev.  The left child overwrites the parent in
// buffer a (every fibre belongs to one thread), the right child goes to b.
template <typename T, int M>
__device__ __forceinline__ void split_fibre(T* __restrict__ a, T* __restrict__ b, int base,
                                            int stride, T& mnL, T& mxL, T& mnR, T& mxR, T& amax)
{
    T c[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        c[i] = a[base + i * stride];
        amax = fmax(amax, fabs(c[i]));
    }
    mnL = mxL = c[0];
    mnR = mxR = c[M - 1];
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

// Splits np consecutive patches of one kind (parent tile at `src`) along axis
// r inside LDS, and reduces per-patch min/max of both children and the
// parent's max |coefficient|.  All threads of the block call it.
template <typename T, int MM>
__device__ void split_tile_lds(const T* __restrict__ src, int np, int S, const FibreGeom& g,
                               SubLds<T> L)
{
    typedef typename KeyOf<T>::type K;
    const int TE = np * S;
    for (int e = threadIdx.x; e < TE; e += blockDim.x) L.a[e] = src[e];
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        L.key[5 * p + 0] = ~(K)0;  // min left
        L.key[5 * p + 1] = 0;      // max left
        L.key[5 * p + 2] = ~(K)0;  // min right
        L.key[5 * p + 3] = 0;      // max right
        L.key[5 * p + 4] = 0;      // max |parent|
    }
    __syncthreads();
    const int TF = np * g.F;
    for (int f = threadIdx.x; f < TF; f += blockDim.x) {
        const int p = f / g.F;
        const int base = p * S + fibre_base(g, f - p * g.F);
        T mnL, mxL, mnR, mxR, amax = (T)0;
        switch (g.m) {
#define PCBA_SPLIT_CASE(MV) \
        case MV: if (MV <= MM) split_fibre<T, MV>(L.a, L.b, base, g.stride, mnL, mxL, mnR, mxR, amax); break;
            PCBA_SPLIT_CASE(1) PCBA_SPLIT_CASE(2) PCBA_SPLIT_CASE(3) PCBA_SPLIT_CASE(4)
            PCBA_SPLIT_CASE(5) PCBA_SPLIT_CASE(6) PCBA_SPLIT_CASE(7) PCBA_SPLIT_CASE(8)
            PCBA_SPLIT_CASE(9) PCBA_SPLIT_CASE(10) PCBA_SPLIT_CASE(11) PCBA_SPLIT_CASE(12)
            PCBA_SPLIT_CASE(13) PCBA_SPLIT_CASE(14) PCBA_SPLIT_CASE(15) PCBA_SPLIT_CASE(16)
#undef PCBA_SPLIT_CASE
        default: mnL = mxL = mnR = mxR = (T)0; break;
        }
        atomicMin(&L.key[5 * p + 0], fkey(mnL));
        atomicMax(&L.key[5 * p + 1], fkey(mxL));
        atomicMin(&L.key[5 * p + 2], fkey(mnR));
        atomicMax(&L.key[5 * p + 3], fkey(mxR));
        atomicMax(&L.key[5 * p + 4], fkey(amax));
    }
    __syncthreads();
}

// widened bound of one patch of a child: lo/hi in double
template <typename T>
__device__ __forceinline__ void child_bounds(T mn, T mx, double e, double& lo, double& hi)
{
    if (e == 0.0) {
        lo = (double)mn;
        hi = (double)mx;
    } else {
        lo = nextafter((double)mn - e, -INFINITY);
        hi = nextafter((double)mx + e, INFINITY);
    }
}

template <typename T, int MM>
__global__ __launch_bounds__(SUB_THREADS) void k_sub(const DevInst* __restrict__ insts, int n_inst,
                                                    const long long* __restrict__ plan)
{
    typedef typename KeyOf<T>::type K;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_flag[2];
    __shared__ int s_dead[2];
    __shared__ double s_cost[4];

    // units of this launch: every running problem of this class contributes K * T
    const bool fp32 = sizeof(T) == 4;
    const long long* pre = plan + (fp32 ? 1 : 0) * (n_inst + 1);
    const long long total = pre[n_inst];

    for (long long u = blockIdx.x; u < total; u += gridDim.x) {
        const int bi = find_inst(pre, n_inst, u);
        const DevInst& I = insts[bi];
        const InstState* st = I.st;
        const long long local = u - pre[bi];
        const int j = (int)(local / I.T);
        const int t = (int)(local - (long long)j * I.T);
        const int cur = st->cur, r = st->r, l = I.l;
        const double pprev = st->p_up;
        const int pslot = I.live[j];
        const T* parent = (const T*)I.buf[cur] + (int64_t)pslot * I.stride;
        T* childL = (T*)I.buf[cur ^ 1] + (int64_t)(2 * j) * I.stride;
        T* childR = childL + I.stride;
        const int kind = (t < I.tile_start[1]) ? 0 : ((t < I.tile_start[2]) ? 1 : 2);
        const int p0 = (t - I.tile_start[kind]) * I.tile_polys[kind];
        const int np = min(I.tile_polys[kind], I.count[kind] - p0);
        const int S = I.S[kind];

        // LDS carve-up: a | b | keys
        int TEmax = 0;
        {
            // the host sizes LDS for the largest tile over the launch; recompute
            // this unit's layout from its own tile (cost tile may be larger)
            TEmax = max(np * S, I.S[0]);
        }
        SubLds<T> L;
        L.a = (T*)smem;
        L.b = L.a + TEmax;
        L.key = (K*)(L.b + TEmax);

        if (threadIdx.x < 2) s_flag[threadIdx.x] = 0;
        if (threadIdx.x == 0) { s_dead[0] = 0; s_dead[1] = 0; }

        // ---- stale-estimate filter: cost lower bounds of both children ----
        const bool need_cost = (kind == 0) || (I.stale && pprev < INFINITY);
        double minPL = 0, minPR = 0;
        if (need_cost) {
            FibreGeom gc = fibre_geom(I.dims[0], l, r, I.S[0]);
            split_tile_lds<T, MM>(parent + I.off[0], 1, I.S[0], gc, L);
            if (threadIdx.x == 0) {
                double e = 0.0;
                if (fp32) {
                    const float ep = I.err[cur][(int64_t)pslot * I.n_polys];
                    e = (double)round_up_f((double)ep + gamma32(gc.m) * (double)funkey(L.key[4]) +
                                           (double)gc.m * 0x1p-126);
                    if (kind == 0) {
                        I.err[cur ^ 1][(int64_t)(2 * j) * I.n_polys] = (float)e;
                        I.err[cur ^ 1][(int64_t)(2 * j + 1) * I.n_polys] = (float)e;
                    }
                }
                double lo, hi;
                child_bounds<T>(funkey(L.key[0]), funkey(L.key[1]), e, lo, hi);
                s_cost[0] = lo; s_cost[1] = hi;
                child_bounds<T>(funkey(L.key[2]), funkey(L.key[3]), e, lo, hi);
                s_cost[2] = lo; s_cost[3] = hi;
                s_dead[0] = s_cost[0] > pprev;
                s_dead[1] = s_cost[2] > pprev;
                if (kind == 0) {
                    I.minP[2 * j] = s_cost[0];
                    I.maxP[2 * j] = s_cost[1];
                    I.minP[2 * j + 1] = s_cost[2];
                    I.maxP[2 * j + 1] = s_cost[3];
                    // child ids: index along r doubles, plus 1 for the right half
                    const uint32_t* pid = I.ids[cur] + (int64_t)pslot * l;
                    uint32_t* cid = I.ids[cur ^ 1] + (int64_t)(2 * j) * l;
                    for (int k = 0; k < l; ++k) {
                        const uint32_t v = pid[k];
                        cid[k] = (k == r) ? 2u * v : v;
                        cid[l + k] = (k == r) ? 2u * v + 1u : v;
                    }
                }
            }
            __syncthreads();
            minPL = s_cost[0];
            minPR = s_cost[2];
            (void)minPL; (void)minPR;
            if (kind == 0) {
                // write the cost children unless already known suboptimal
                const int TE = I.S[0];
                const bool wl = !s_dead[0], wr = !s_dead[1];
                for (int e = threadIdx.x; e < TE; e += blockDim.x) {
                    if (wl) childL[I.off[0] + e] = L.a[e];
                    if (wr) childR[I.off[0] + e] = L.b[e];
                }
                __syncthreads();
                continue;
            }
        }
        // skip children another tile already found infeasible
        if (threadIdx.x == 0) {
            const uint32_t fl = __atomic_load_n(&I.flags[2 * j], __ATOMIC_RELAXED);
            const uint32_t fr = __atomic_load_n(&I.flags[2 * j + 1], __ATOMIC_RELAXED);
            if (fl & F_INFEAS) s_dead[0] = 1;
            if (fr & F_INFEAS) s_dead[1] = 1;
        }
        __syncthreads();
        const bool deadL = s_dead[0], deadR = s_dead[1];
        __syncthreads();
        if (deadL && deadR) continue;

        // ---- the tile of constraint patches ----
        FibreGeom g = fibre_geom(I.dims[kind], l, r, S);
        const int64_t toff = I.off[kind] + (int64_t)p0 * S;
        split_tile_lds<T, MM>(parent + toff, np, S, g, L);

        // per-patch bounds -> feasibility flags of both children
        uint32_t fL = 0, fR = 0;
        for (int p = threadIdx.x; p < np; p += blockDim.x) {
            const int poly = I.count[0] + (kind == 2 ? I.count[1] : 0) + p0 + p;
            double e = 0.0;
            if (fp32) {
                const float ep = I.err[cur][(int64_t)pslot * I.n_polys + poly];
                e = (double)round_up_f((double)ep + gamma32(g.m) * (double)funkey(L.key[5 * p + 4]) +
                                       (double)g.m * 0x1p-126);
                I.err[cur ^ 1][(int64_t)(2 * j) * I.n_polys + poly] = (float)e;
                I.err[cur ^ 1][(int64_t)(2 * j + 1) * I.n_polys + poly] = (float)e;
            }
            for (int c = 0; c < 2; ++c) {
                double lo, hi;
                child_bounds<T>(funkey(L.key[5 * p + 2 * c]), funkey(L.key[5 * p + 2 * c + 1]), e, lo, hi);
                uint32_t f = 0;
                if (kind == 1) {
                    if (lo > 0.0) f |= F_INFEAS;
                    if (!(hi <= 0.0)) f |= F_NOTFEAS;
                } else {
                    if (lo > 0.0 || hi < 0.0) f |= F_INFEAS;
                    if (!(-I.eps_eq <= lo && lo <= 0.0 && 0.0 <= hi && hi <= I.eps_eq)) f |= F_NOTFEAS;
                }
                if (c == 0) fL |= f; else fR |= f;
            }
        }
        if (fL) atomicOr(&s_flag[0], fL);
        if (fR) atomicOr(&s_flag[1], fR);
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_flag[0]) atomicOr(&I.flags[2 * j], s_flag[0]);
            if (s_flag[1]) atomicOr(&I.flags[2 * j + 1], s_flag[1]);
        }
        // children patches (skipped when the child is already known dead)
        const bool wl = !deadL && !(s_flag[0] & F_INFEAS);
        const bool wr = !deadR && !(s_flag[1] & F_INFEAS);
        const int TE = np * S;
        for (int e = threadIdx.x; e < TE; e += blockDim.x) {
            if (wl) childL[toff + e] = L.a[e];
            if (wr) childR[toff + e] = L.b[e];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ k_rederive

// Bernstein sub-interval transform on [a,b] inside [0,1] for degree n:
// T[k][j] = sum_s b^{n-k}_s(a) b^k_{j-s}(b) (the polar form of b^n_j at
// (a,..,a, b,..,b)), rows non-negative and summing to one.
__device__ double bern_basis(int n, int i, double t)
{
    double c = 1.0;
    for (int q = 1; q <= i; ++q) c = c * (double)(n - i + q) / (double)q;
    double v = c;
    for (int q = 0; q < i; ++q) v *= t;
    for (int q = 0; q < n - i; ++q) v *= (1.0 - t);
    return v;
}
__device__ double tmat_entry(int n, int k, int j, double a, double b)
{
    double s = 0.0;
    const int s0 = max(0, j - k), s1 = min(n - k, j);
    for (int q = s0; q <= s1; ++q) s += bern_basis(n - k, q, a) * bern_basis(k, j - q, b);
    return s;
}

// Applies tmat (one m x m matrix per axis) to a patch in LDS (FP64), axis by
// axis; x and y are two LDS buffers of S doubles; the result ends in x.
__device__ void apply_tmats(double* x, double* y, const double* tm, const int* tmoff,
                            const int* dims, int l, int S, int np)
{
    for (int r = 0; r < l; ++r) {
        FibreGeom g = fibre_geom(dims, l, r, S);
        const double* Tm = tm + tmoff[r];
        const int TF = np * g.F;
        for (int f = threadIdx.x; f < TF; f += blockDim.x) {
            const int p = f / g.F;
            const int base = p * S + fibre_base(g, f - p * g.F);
            for (int k = 0; k < g.m; ++k) {
                double acc = 0.0;
                for (int i = 0; i < g.m; ++i) acc += Tm[k * g.m + i] * x[base + i * g.stride];
                y[base + k * g.stride] = acc;
            }
        }
        __syncthreads();
        const int TE = np * S;
        for (int e = threadIdx.x; e < TE; e += blockDim.x) x[e] = y[e];
        __syncthreads();
    }
}

// FP32 re-derivation step: children of every live parent derived from the
// FP64 root by box id, rounded to FP32 with a fresh error bound, then bounded
// and flagged exactly like k_sub.
__global__ __launch_bounds__(SUB_THREADS) void k_rederive(const DevInst* __restrict__ insts, int n_inst,
                                                         const long long* __restrict__ plan)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_flag[2];
    __shared__ int s_tmoff[MAXL];
    const long long* pre = plan + 2 * (n_inst + 1);
    const long long total = pre[n_inst];
    for (long long u = blockIdx.x; u < total; u += gridDim.x) {
        const int bi = find_inst(pre, n_inst, u);
        const DevInst& I = insts[bi];
        const InstState* st = I.st;
        const long long local = u - pre[bi];
        const int j = (int)(local / I.T);
        const int t = (int)(local - (long long)j * I.T);
        const int cur = st->cur, r = st->r, l = I.l;
        const int pslot = I.live[j];
        const uint32_t* pid = I.ids[cur] + (int64_t)pslot * l;
        const int kind = (t < I.tile_start[1]) ? 0 : ((t < I.tile_start[2]) ? 1 : 2);
        const int p0 = (t - I.tile_start[kind]) * I.tile_polys[kind];
        const int np = min(I.tile_polys[kind], I.count[kind] - p0);
        const int S = I.S[kind];
        const int TE = np * S;
        const int64_t toff = I.off[kind] + (int64_t)p0 * S;

        // LDS: x | y (TE doubles each) | tmats (l * m^2 doubles)
        double* x = (double*)smem;
        double* y = x + TE;
        double* tm = y + TE;
        if (threadIdx.x == 0) {
            int o = 0;
            for (int k = 0; k < l; ++k) { s_tmoff[k] = o; o += I.dims[kind][k] * I.dims[kind][k]; }
        }
        if (threadIdx.x < 2) s_flag[threadIdx.x] = 0;
        __syncthreads();
        for (int c = 0; c < 2; ++c) {
            // child box: depth after this step, index with the new bit along r
            for (int k = 0; k < l; ++k) {
                const int m = I.dims[kind][k];
                const int d = st->depth[k] + (k == r ? 1 : 0);
                const uint32_t idx = (k == r) ? 2u * pid[k] + (uint32_t)c : pid[k];
                const double a = ldexp((double)idx, -d), bb = ldexp((double)idx + 1.0, -d);
                for (int e = threadIdx.x; e < m * m; e += blockDim.x)
                    tm[s_tmoff[k] + e] = tmat_entry(m - 1, e / m, e % m, a, bb);
            }
            for (int e = threadIdx.x; e < TE; e += blockDim.x) x[e] = I.root[toff + e];
            __syncthreads();
            apply_tmats(x, y, tm, s_tmoff, I.dims[kind], l, S, np);
            // per patch: FP64 bound, round to FP32, min/max of the FP32 values
            float* child = (float*)I.buf[cur ^ 1] + (int64_t)(2 * j + c) * I.stride;
            uint32_t fl = 0;
            const int wv = threadIdx.x >> 6;
            for (int p = wv; p < np; p += blockDim.x >> 6) {
                const int poly = (kind == 0 ? 0 : I.count[0] + (kind == 2 ? I.count[1] : 0) + p0 + p);
                const double* rp = I.root + toff + (int64_t)p * S;
                float mn = INFINITY, mx = -INFINITY;
                double rmax = 0.0;
                for (int e = threadIdx.x & 63; e < S; e += 64) {
                    const float v = (float)x[p * S + e];
                    child[toff + (int64_t)p * S + e] = v;
                    mn = fminf(mn, v);
                    mx = fmaxf(mx, v);
                    rmax = fmax(rmax, fabs(rp[e]));
                }
                for (int o = 32; o > 0; o >>= 1) {
                    mn = fminf(mn, __shfl_xor(mn, o, 64));
                    mx = fmaxf(mx, __shfl_xor(mx, o, 64));
                    rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
                }
                if ((threadIdx.x & 63) == 0) {
                    double g64 = 0.0;
                    for (int k = 0; k < l; ++k) g64 += gamma64(4 * I.dims[kind][k] + 6);
                    const double amax = fmax(fabs((double)mn), fabs((double)mx));
                    const double e = (double)round_up_f(I.root_err[poly] + g64 * rmax * 1.01 +
                                                        amax * 0x1p-23 + 0x1p-126);
                    I.err[cur ^ 1][(int64_t)(2 * j + c) * I.n_polys + poly] = (float)e;
                    double lo, hi;
                    child_bounds<float>(mn, mx, e, lo, hi);
                    if (kind == 0) {
                        I.minP[2 * j + c] = lo;
                        I.maxP[2 * j + c] = hi;
                    } else if (kind == 1) {
                        if (lo > 0.0) fl |= F_INFEAS;
                        if (!(hi <= 0.0)) fl |= F_NOTFEAS;
                    } else {
                        if (lo > 0.0 || hi < 0.0) fl |= F_INFEAS;
                        if (!(-I.eps_eq <= lo && lo <= 0.0 && 0.0 <= hi && hi <= I.eps_eq)) fl |= F_NOTFEAS;
                    }
                }
            }
            if (fl) atomicOr(&s_flag[c], fl);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (s_flag[0]) atomicOr(&I.flags[2 * j], s_flag[0]);
            if (s_flag[1]) atomicOr(&I.flags[2 * j + 1], s_flag[1]);
            if (kind == 0) {
                uint32_t* cid = I.ids[cur ^ 1] + (int64_t)(2 * j) * l;
                for (int k = 0; k < l; ++k) {
                    const uint32_t v = pid[k];
                    cid[k] = (k == r) ? 2u * v : v;
                    cid[l + k] = (k == r) ? 2u * v + 1u : v;
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ k_cut

__global__ __launch_bounds__(CUT_THREADS) void k_cut(const DevInst* __restrict__ insts, int n_inst)
{
    __shared__ double shd[CUT_THREADS / 64];
    __shared__ int shi[CUT_THREADS / 64];
    __shared__ int wsum[CUT_THREADS / 64 + 1];
    const DevInst& I = insts[blockIdx.x];
    InstState* st = I.st;
    if (st->status != ST_RUNNING) return;
    const int K = st->K, C = 2 * K, r = st->r;
    const double pprev = st->p_up;
    const bool fin = pprev < INFINITY;
    const int tid = threadIdx.x;

    // solution estimate: least max B_p over feasible children
    double m = INFINITY;
    for (int c = tid; c < C; c += blockDim.x) {
        const double mnp = I.minP[c];
        const bool dead = fin && mnp > pprev;
        if (!dead && !(I.flags[c] & (F_INFEAS | F_NOTFEAS))) m = fmin(m, I.maxP[c]);
    }
    m = block_min(m, shd);
    const bool update = (m < INFINITY) && (m <= pprev);
    int arg = INT_MAX;
    if (update) {
        for (int c = tid; c < C; c += blockDim.x) {
            const double mnp = I.minP[c];
            const bool dead = fin && mnp > pprev;
            if (!dead && !(I.flags[c] & (F_INFEAS | F_NOTFEAS)) && I.maxP[c] == m) arg = min(arg, c);
        }
        arg = block_min_i(arg, shi);
    }
    const double p_up = update ? m : pprev;

    // least lower bound, keep mask, order-preserving compaction into live[]
    double plo = INFINITY;
    int base = 0;
    const int lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
    for (int c0 = 0; c0 < C; c0 += blockDim.x) {
        const int c = c0 + tid;
        bool keep = false;
        if (c < C) {
            const double mnp = I.minP[c];
            const bool dead = fin && mnp > pprev;
            if (!dead && !(I.flags[c] & F_INFEAS)) {
                plo = fmin(plo, mnp);
                keep = mnp <= p_up;
            }
        }
        const unsigned long long bal = __ballot(keep);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[w] = __popcll(bal);
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int q = 0; q < nw; ++q) { const int v = wsum[q]; wsum[q] = acc; acc += v; }
            wsum[nw] = acc;
        }
        __syncthreads();
        if (keep) I.live[base + wsum[w] + before] = c;
        base += wsum[nw];
        __syncthreads();
    }
    plo = block_min(plo, shd);
    const int Kn = base;

    // clear the flags of the next step's children
    for (int c = tid; c < 2 * Kn && c < I.cap; c += blockDim.x) I.flags[c] = 0;

    if (tid == 0) {
        if (st->steps < MAX_TRACE) {
            TraceRec tr;
            tr.k_in = K;
            tr.k_kept = Kn;
            tr.p_up = p_up;
            tr.p_lo = plo;
            I.trace[st->steps] = tr;
        }
        st->depth[r] += 1;
        st->steps += 1;
        const int nxt = st->cur ^ 1;
        if (update) {
            const uint32_t* cid = I.ids[nxt] + (int64_t)arg * I.l;
            for (int k = 0; k < I.l; ++k) {
                st->x_index[k] = cid[k];
                st->x_depth[k] = st->depth[k];
            }
            st->has_x = 1;
        }
        st->p_up = p_up;
        st->p_lo = plo;
        st->K = Kn;
        st->cur = nxt;
        if (Kn == 0) {
            st->status = ST_INFEASIBLE;
        } else {
            double width = 0.0;
            for (int k = 0; k < I.l; ++k) width = fmax(width, ldexp(I.width0[k], -st->depth[k]));
            if (p_up < INFINITY && p_up - plo <= I.eps && width <= I.delta) {
                st->status = ST_OPTIMAL;
            } else {
                int rn = (r + 1) % I.l;
                st->r = rn;
                if (rn == 0) st->n += 1;
                if (st->n == I.N) st->status = ST_MAXITER;
            }
        }
    }
}

// ------------------------------------------------------------------ certification

// One workgroup per polynomial: FP64 patch of x* from the root with the
// sub-interval transforms, its min / max and a rigorous error bound
// (|T~ - T| <= gamma_{3m+5} T entrywise, one more gamma_m per product,
// plus the root's own bound; all values taken as |T| |x| sums).
__global__ __launch_bounds__(256) void k_certify(DevInst I)
{
    extern __shared__ double shc[];
    const InstState* st = I.st;
    if (!st->has_x) return;
    const int poly = blockIdx.x;
    int kind = 0, idx = poly;
    if (idx >= I.count[0]) { idx -= I.count[0]; kind = 1; if (idx >= I.count[1]) { idx -= I.count[1]; kind = 2; } }
    const int S = I.S[kind], l = I.l;
    double* x = shc;
    double* y = x + S;
    double* tm = y + S;
    __shared__ int tmoff[MAXL];
    __shared__ double red[3 * 4];
    if (threadIdx.x == 0) {
        int o = 0;
        for (int k = 0; k < l; ++k) { tmoff[k] = o; o += I.dims[kind][k] * I.dims[kind][k]; }
    }
    __syncthreads();
    for (int k = 0; k < l; ++k) {
        const int m = I.dims[kind][k];
        const double a = ldexp((double)st->x_index[k], -st->x_depth[k]);
        const double b = ldexp((double)st->x_index[k] + 1.0, -st->x_depth[k]);
        for (int e = threadIdx.x; e < m * m; e += blockDim.x)
            tm[tmoff[k] + e] = tmat_entry(m - 1, e / m, e % m, a, b);
    }
    const double* rp = I.root + I.off[kind] + (int64_t)idx * S;
    double gsum = 0.0;
    for (int r = 0; r < l; ++r) gsum += gamma64(4 * I.dims[kind][r] + 6);
    double mn = INFINITY, mx = -INFINITY, am = 0.0;
    // pass 0: the patch of x*; pass 1: |T| applied to |root|, which bounds the error
    for (int absp = 0; absp < 2; ++absp) {
        for (int e = threadIdx.x; e < S; e += blockDim.x) x[e] = absp ? fabs(rp[e]) : rp[e];
        __syncthreads();
        apply_tmats(x, y, tm, tmoff, I.dims[kind], l, S, 1);
        for (int e = threadIdx.x; e < S; e += blockDim.x) {
            if (absp) am = fmax(am, x[e]);
            else { mn = fmin(mn, x[e]); mx = fmax(mx, x[e]); }
        }
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, o, 64));
        mx = fmax(mx, __shfl_xor(mx, o, 64));
        am = fmax(am, __shfl_xor(am, o, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[3 * w] = mn; red[3 * w + 1] = mx; red[3 * w + 2] = am; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
            mn = fmin(mn, red[3 * q]);
            mx = fmax(mx, red[3 * q + 1]);
            am = fmax(am, red[3 * q + 2]);
        }
        // e <= root bound (rows of T sum to one) + sum over axes of gamma * |T||x|
        const double e = I.root_err[poly] + gsum * am * 1.01;
        I.cert[3 * poly + 0] = mn;
        I.cert[3 * poly + 1] = mx;
        I.cert[3 * poly + 2] = e;
    }
}

__global__ void k_certify_final(DevInst I)
{
    InstState* st = I.st;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (!st->has_x) { st->cert_ok = 0; st->p_cert = INFINITY; st->cert_err = 0.0; return; }
    int ok = 1;
    double emax = 0.0;
    for (int p = 0; p < I.n_polys; ++p) {
        const double mn = I.cert[3 * p], mx = I.cert[3 * p + 1], e = I.cert[3 * p + 2];
        emax = fmax(emax, e);
        if (p < I.count[0]) continue;
        if (p < I.count[0] + I.count[1]) {
            if (!(mx + e <= 0.0)) ok = 0;
        } else {
            if (!(-I.eps_eq <= mn - e && mn + e <= 0.0 && 0.0 <= mx - e && mx + e <= I.eps_eq)) ok = 0;
        }
    }
    st->cert_ok = ok;
    st->p_cert = nextafter(I.cert[1] + I.cert[2], INFINITY);
    st->cert_err = emax;
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
    const T* src = (const T*)I.buf[st->cur] + (int64_t)slot * I.stride;
    for (int64_t e = threadIdx.x; e < W; e += blockDim.x) out[(int64_t)j * W + e] = (double)src[e];
    if (threadIdx.x < (unsigned)I.l)
        ids_out[(int64_t)j * I.l + threadIdx.x] = I.ids[st->cur][(int64_t)slot * I.l + threadIdx.x];
    if (I.fp32 && err_out)
        for (int p = threadIdx.x; p < I.n_polys; p += blockDim.x)
            err_out[(int64_t)j * I.n_polys + p] = (double)I.err[st->cur][(int64_t)slot * I.n_polys + p];
}

__global__ void k_gather(const DevInst* __restrict__ insts, int n, InstState* __restrict__ out)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n; b += gridDim.x * blockDim.x)
        out[b] = *insts[b].st;
}

// ------------------------------------------------------------------ host launchers

hipError_t launch_root(const DevInst& I, const double* mono, const double* mats, const int* matoff,
                       double* root, double* root_err, int64_t W, int max_S, hipStream_t s)
{
    const size_t lds = 2 * (size_t)max_S * sizeof(double);
    hipLaunchKernelGGL(k_root, dim3(I.n_polys), dim3(256), lds, s, I, mono, mats, matoff, root,
                       root_err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int blocks = (int)std::min<int64_t>(1024, (W + 255) / 256);
    if (I.fp32)
        hipLaunchKernelGGL(k_root_item<float>, dim3(blocks), dim3(256), 0, s, I, W);
    else
        hipLaunchKernelGGL(k_root_item<double>, dim3(blocks), dim3(256), 0, s, I, W);
    return hipGetLastError();
}

hipError_t launch_plan(const DevInst* d_insts, int n, long long* plan, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, d_insts, n, plan);
    return hipGetLastError();
}

template <typename T, int MM>
static hipError_t launch_sub_t(const DevInst* d_insts, int n, const long long* plan, int grid,
                               size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_sub<T, MM>), dim3(grid), dim3(SUB_THREADS), lds, s, d_insts, n, plan);
    return hipGetLastError();
}

hipError_t launch_sub(const DevInst* d_insts, int n, const long long* plan, bool fp32, int maxm,
                      int grid, size_t lds, hipStream_t s)
{
    if (grid <= 0) return hipSuccess;
    if (fp32) {
        if (maxm <= 8) return launch_sub_t<float, 8>(d_insts, n, plan, grid, lds, s);
        return launch_sub_t<float, 16>(d_insts, n, plan, grid, lds, s);
    }
    if (maxm <= 8) return launch_sub_t<double, 8>(d_insts, n, plan, grid, lds, s);
    return launch_sub_t<double, 16>(d_insts, n, plan, grid, lds, s);
}

hipError_t launch_rederive(const DevInst* d_insts, int n, const long long* plan, int grid,
                           size_t lds, hipStream_t s)
{
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rederive, dim3(grid), dim3(SUB_THREADS), lds, s, d_insts, n, plan);
    return hipGetLastError();
}

hipError_t launch_cut(const DevInst* d_insts, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cut, dim3(n), dim3(CUT_THREADS), 0, s, d_insts, n);
    return hipGetLastError();
}

hipError_t launch_gather(const DevInst* d_insts, int n, InstState* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, s, d_insts, n, out);
    return hipGetLastError();
}

hipError_t launch_certify(const DevInst& I, int max_S, int max_m, hipStream_t s)
{
    const size_t lds = (2 * (size_t)max_S + (size_t)MAXL * max_m * max_m) * sizeof(double);
    hipLaunchKernelGGL(k_certify, dim3(I.n_polys), dim3(256), lds, s, I);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_certify_final, dim3(1), dim3(64), 0, s, I);
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
