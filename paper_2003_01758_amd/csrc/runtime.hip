// runtime.hip -- host runtime behind include/pcba.h: problem creation (root
// conversion on the device), the batched step engine (plan, subdivide+bound,
// cut-off+compaction, growth of the device list), certification and read-out.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pcba.h"
#include "kernels.h"
#include "pool.h"

using namespace pcba;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(PCBA_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int GRID_MAX = 2048;
constexpr int STEPS_PER_SYNC = 8;
constexpr int CHECK_STEPS = 4;      // steps between looks at the kernels' stop flag
constexpr int MAX_STEPS_PER_SYNC = 64;
constexpr int TILE_ELEMS = 2816;   // target coefficients per FP64 tile (per LDS region)
constexpr int MAX_PATCH = 3584;    // largest patch (coefficients): LDS stays within 64 KB
constexpr int CAP0 = 64;           // initial list capacity (items per buffer)

// children above which a problem's cut is split across workgroups (0: never)
std::atomic<long long> g_cut_split{CUT_SPLIT_DEFAULT};
std::atomic<int> g_cut_part{CUT_PART_DEFAULT};   // children per workgroup of a split cut

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * (double)(n - k + i) / (double)i;
    return c;
}

// kernel timing: event pairs recorded around every launch while enabled
struct Profile {
    bool on = false;
    double ms[PCBA_NUM_KERNELS] = {};
    int64_t launches[PCBA_NUM_KERNELS] = {};
    std::vector<hipEvent_t> ev;      // pool: 2 events per record
    std::vector<int> kid;            // kernel id of each pending record
    size_t used = 0;
};
Profile g_prof;

hipError_t prof_begin(hipStream_t s)
{
    if (!g_prof.on) return hipSuccess;
    if (2 * (g_prof.used + 1) > g_prof.ev.size()) {
        for (int q = 0; q < 2; ++q) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            g_prof.ev.push_back(e);
        }
    }
    return hipEventRecord(g_prof.ev[2 * g_prof.used], s);
}
hipError_t prof_end(int kernel, hipStream_t s)
{
    if (!g_prof.on) return hipSuccess;
    hipError_t r = hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s);
    if ((size_t)g_prof.kid.size() <= g_prof.used) g_prof.kid.resize(g_prof.used + 1);
    g_prof.kid[g_prof.used] = kernel;
    g_prof.used += 1;
    return r;
}
// an event pair for a launch that stamps it itself (hipExtLaunchKernelGGL);
// nulls when profiling is off
hipError_t prof_pair(int kernel, hipEvent_t* ev0, hipEvent_t* ev1)
{
    *ev0 = *ev1 = nullptr;
    if (!g_prof.on) return hipSuccess;
    if (2 * (g_prof.used + 1) > g_prof.ev.size()) {
        for (int q = 0; q < 2; ++q) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            g_prof.ev.push_back(e);
        }
    }
    *ev0 = g_prof.ev[2 * g_prof.used];
    *ev1 = g_prof.ev[2 * g_prof.used + 1];
    if ((size_t)g_prof.kid.size() <= g_prof.used) g_prof.kid.resize(g_prof.used + 1);
    g_prof.kid[g_prof.used] = kernel;
    g_prof.used += 1;
    return hipSuccess;
}

// after the stream is synchronised: fold the pending records into the totals
void prof_collect()
{
    for (size_t i = 0; i < g_prof.used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) == hipSuccess) {
            g_prof.ms[g_prof.kid[i]] += ms;
            g_prof.launches[g_prof.kid[i]] += 1;
        }
    }
    g_prof.used = 0;
}

}  // namespace

struct pcba_problem {
    int l = 0;
    double lo[MAXL] = {}, hi[MAXL] = {};
    int deg[KINDS][MAXL] = {};
    int S[KINDS] = {};
    int count[KINDS] = {};
    int64_t off[KINDS] = {};
    int64_t soff[KINDS] = {};   // offsets inside a list slot
    int64_t W = 0;
    int n_polys = 0;
    pcba_options opt{};
    bool fp32 = false;
    int nc = 2;                 // children per parent: 2, or 2^l when each step is a round
    size_t elem = 8;
    int tile_polys[KINDS] = {};
    int ptp[KINDS] = {};       // patches per k_sub tile
    int tile_start[KINDS + 1] = {};
    int T = 0;
    int64_t stride = 0;
    int maxm = 1;
    int max_S = 1;
    int64_t M_eff = 0;

    // device
    double* d_root = nullptr;
    double* d_root_err = nullptr;
    double* d_racc = nullptr;     // accurate root (one combined matrix per axis)
    double* d_macc = nullptr;     // combined matrices M and Mabs per kind and axis
    double* d_cert = nullptr;
    void* d_buf[2] = {nullptr, nullptr};
    uint32_t* d_ids[2] = {nullptr, nullptr};
    float2* d_err[2] = {nullptr, nullptr};   // FP32 mode: per-patch (error bound, pending shift)
    double* d_base[2] = {nullptr, nullptr};   // FP32 mode: per-patch FP64 bases
    int32_t* d_live = nullptr;
    double* d_minP = nullptr;
    double* d_maxP = nullptr;
    uint32_t* d_flags = nullptr;
    unsigned long long* d_stamp = nullptr;
    int2* d_act[2] = {nullptr, nullptr};   // retiring mode: carried inequalities per slot
    int32_t* d_na[2] = {nullptr, nullptr};
    void* d_heap[2] = {nullptr, nullptr};  // retiring mode: the carried inequality patches
    int64_t hcap = 0;                      // patches per heap
    int64_t* d_upre = nullptr;
    int4* d_umap = nullptr;                // retiring mode: hcap entries
    int4* d_pmap = nullptr;                // retiring mode: hcap entries
    bool retire = false;
    double* d_tmat = nullptr;
    int tmw = 0, rows = 0, tmk[KINDS] = {};
    InstState* d_st = nullptr;
    TraceRec* d_trace = nullptr;
    double* d_mono = nullptr;     // monomials in item layout (kept for pcba_reset)
    double* d_mats = nullptr;     // pre-map and conversion matrices
    int* d_matoff = nullptr;
    int64_t cap = 0;

    InstState h_st{};
    bool certified_done = false;
    double seconds = 0.0;
    double t_start = 0.0;
    int64_t footprint = 0;   // bytes charged by an engine
    bool list_released = false;  // finished, and its list freed for other problems
    bool root_written = false;   // d_root holds the root patches (written by the first reset)
    int host_steps = 0;      // steps known on the host (for re-derivation planning)
};

// Per-step buffers of an engine (descriptors, plan, step snapshots, states and
// their pinned staging), sized for `cap` problems on `dev`.
struct EngineBufs {
    int dev = -1;
    int cap = 0;
    DevInst* d_insts = nullptr;
    long long* d_plan = nullptr;
    StepInfo* d_info = nullptr;
    InstState* h_states = nullptr;  // pinned, coherent: the gather kernel writes the states here
    InstState* d_states = nullptr;  // its device address (no device-to-host copy call: such a
                                    // small asynchronous copy has stalled the host for ms)
    DevInst* h_insts = nullptr;    // pinned staging of the descriptors (outlives the async copy)
    int* h_flag = nullptr;         // pinned word the kernels set when a problem stops running
    int* d_flag = nullptr;         // its device address
    int* h_berr = nullptr;         // pinned word set by a timed-out grid barrier wait (k_steps)
    int* d_berr = nullptr;         // its device address
    unsigned* d_bar = nullptr;     // k_steps: the grid barrier's arrival count and abort word
    CutPart* d_parts = nullptr;    // records of cuts split across workgroups
    int64_t parts_cap = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};   // ends of the last two chunks of steps
};

struct pcba_engine {
    hipStream_t stream = nullptr;
    int64_t budget = 0, used = 0;
    int64_t reserve = 0;      // list items charged to every admitted problem at least
    std::vector<pcba_problem*> active;
    std::vector<pcba_problem*> done;
    EngineBufs b;
    bool dirty = true;
};

// ------------------------------------------------------------------ helpers

// Device staging of pcba_read_list_noalloc, for callers that cannot allocate:
// one array per device for the life of the process.  Host code never passes
// `scratch` itself to the device (in host code it names a host-side stand-in);
// static_scratch looks up, once per device with that device current, the
// array's device address and hands that out.
static __device__ __align__(256) unsigned char scratch[PCBA_STATIC_SCRATCH_BYTES];

static int static_scratch(unsigned char** out)
{
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static unsigned char* ptr[kMaxDev] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PCBA_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDev) return fail(PCBA_E_DEVICE, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PCBA_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        ptr[dev] = (unsigned char*)p;
    }
    *out = ptr[dev];
    return PCBA_OK;
}

// The library's stream of the calling thread on the current device, created on
// first use and kept for the life of the process (default priority,
// non-blocking).
static hipError_t library_stream(hipStream_t* out)
{
    constexpr int kMaxDev = 64;
    thread_local hipStream_t streams[kMaxDev] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
    if (!streams[dev]) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) {
            streams[dev] = nullptr;
            return e;
        }
    }
    *out = streams[dev];
    return hipSuccess;
}

// Engine buffers are kept for reuse: a batch solve creates an engine per call,
// and the device and pinned allocations would otherwise cost more than the
// first steps.  A few sets are cached per process.
std::mutex g_bufs_mu;
std::vector<EngineBufs> g_bufs_cache;

static void bufs_free(EngineBufs& b)
{
    if (b.d_insts) (void)hipFree(b.d_insts);
    if (b.d_plan) (void)hipFree(b.d_plan);
    if (b.d_info) (void)hipFree(b.d_info);
    if (b.h_states) (void)hipHostFree(b.h_states);
    if (b.h_insts) (void)hipHostFree(b.h_insts);
    if (b.h_flag) (void)hipHostFree(b.h_flag);
    if (b.h_berr) (void)hipHostFree(b.h_berr);
    if (b.d_bar) (void)hipFree(b.d_bar);
    if (b.d_parts) (void)hipFree(b.d_parts);
    for (int k = 0; k < 2; ++k)
        if (b.ev[k]) (void)hipEventDestroy(b.ev[k]);
    b = EngineBufs();
}

// Gives a set back to the cache (the caller has synchronised every stream that
// used it); `b` is left empty.
static void bufs_put(EngineBufs& b)
{
    if (b.cap == 0) return;
    {
        std::lock_guard<std::mutex> lk(g_bufs_mu);
        if (g_bufs_cache.size() < 8) {
            g_bufs_cache.push_back(b);
            b = EngineBufs();
            return;
        }
    }
    bufs_free(b);
}

// A set for at least `cap` problems on the current device: a cached one if
// one is large enough, else a new one.
static hipError_t bufs_get(int cap, EngineBufs* out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lk(g_bufs_mu);
        for (size_t i = 0; i < g_bufs_cache.size(); ++i)
            if (g_bufs_cache[i].dev == dev && g_bufs_cache[i].cap >= cap) {
                *out = g_bufs_cache[i];
                g_bufs_cache.erase(g_bufs_cache.begin() + i);
                return hipSuccess;
            }
    }
    EngineBufs b;
    b.dev = dev;
    const int c = std::max(cap, 64);
    e = hipMalloc((void**)&b.d_insts, c * sizeof(DevInst));
    if (e == hipSuccess) e = hipMalloc((void**)&b.d_plan, 4 * (size_t)(c + 1) * sizeof(long long));
    if (e == hipSuccess) e = hipMalloc((void**)&b.d_info, (size_t)c * sizeof(StepInfo));
    if (e == hipSuccess) e = hipHostMalloc((void**)&b.h_states, c * sizeof(InstState), hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&b.d_states, b.h_states, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b.h_insts, c * sizeof(DevInst), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b.h_flag, sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&b.d_flag, b.h_flag, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b.h_berr, sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&b.d_berr, b.h_berr, 0);
    if (e == hipSuccess) e = hipMalloc((void**)&b.d_bar, 2 * sizeof(unsigned));
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&b.ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        bufs_free(b);
        return e;
    }
    b.cap = c;
    *out = b;
    return hipSuccess;
}

static DevInst make_dev(const pcba_problem* P)
{
    DevInst I;
    memset(&I, 0, sizeof(I));
    I.l = P->l;
    I.n_polys = P->n_polys;
    I.T = P->T;
    I.fp32 = P->fp32 ? 1 : 0;
    for (int t = 0; t < KINDS; ++t) {
        for (int k = 0; k < MAXL; ++k) I.dims[t][k] = (k < P->l) ? P->deg[t][k] + 1 : 1;
        I.S[t] = P->S[t];
        I.count[t] = P->count[t];
        I.tile_polys[t] = P->tile_polys[t];
        I.ptp[t] = P->ptp[t];
        I.tile_start[t] = P->tile_start[t];
        I.off[t] = P->off[t];
        I.soff[t] = P->soff[t];
    }
    I.tile_start[KINDS] = P->tile_start[KINDS];
    I.stride = P->stride;
    I.M = (int32_t)std::min<int64_t>(P->M_eff, INT32_MAX);
    I.cap = (int32_t)P->cap;
    I.N = P->opt.max_iters;
    I.stale = P->opt.stale_filter ? 1 : 0;
    I.rederive = P->fp32 ? P->opt.rederive_every : 0;
    I.retire = P->retire ? 1 : 0;
    I.eps = P->opt.eps;
    I.delta = P->opt.delta;
    I.eps_eq = P->opt.eps_eq;
    for (int k = 0; k < MAXL; ++k) I.width0[k] = (k < P->l) ? P->hi[k] - P->lo[k] : 0.0;
    for (int b = 0; b < 2; ++b) {
        I.buf[b] = P->d_buf[b];
        I.ids[b] = P->d_ids[b];
        I.err[b] = P->d_err[b];
        I.base[b] = P->d_base[b];
        I.act[b] = P->d_act[b];
        I.na[b] = P->d_na[b];
        I.heap[b] = P->d_heap[b];
    }
    I.hcap = P->hcap;
    I.umap = P->d_umap;
    I.pmap = P->d_pmap;
    I.upre = P->d_upre;
    I.live = P->d_live;
    I.minP = P->d_minP;
    I.maxP = P->d_maxP;
    I.flags = P->d_flags;
    I.stamp = P->d_stamp;
    I.tmat = P->d_tmat;
    I.tmw = P->tmw;
    I.rows = P->rows;
    I.fused = P->opt.fused_round ? 1 : 0;
    I.rule = P->opt.direction_rule;
    I.mfma = (P->opt.precision == PCBA_FP32 && P->opt.split_engine == PCBA_SPLIT_MFMA) ? 1 : 0;
    I.lam = P->opt.subdiv_lambda;
    for (int t = 0; t < KINDS; ++t) I.tmk[t] = P->tmk[t];
    I.root = P->root_written ? nullptr : P->d_root;
    I.root_err = P->d_root_err;
    I.root_abs = P->d_root_err + P->n_polys;
    I.racc = P->d_racc;
    I.macc = P->d_macc;
    I.cert = P->d_cert;
    I.trace = P->d_trace;
    I.mono = P->d_mono;
    I.mats = P->d_mats;
    I.matoff = P->d_matoff;
    I.st = P->d_st;
    return I;
}

static int64_t item_bytes(const pcba_problem* P)
{
    // slot, box ids, FP32 (error bound, shift) and base per patch, live index,
    // minP, maxP, flags, stale-filter record
    return P->stride * (int64_t)P->elem + (int64_t)P->l * 4 + (P->fp32 ? P->n_polys * 16 : 0) + 4 + 8 + 8 + 4 + 8 +
           (P->retire ? (int64_t)P->count[1] * 8 + 4 + 8 : 0);
}

// Device bytes of a problem with `boxes` slots per buffer and heaps of `hcap`
// patches: two buffers of slots, two heaps, the root and records.
static int64_t footprint_of(const pcba_problem* P, int64_t boxes, int64_t hcap)
{
    return 2 * boxes * item_bytes(P) +
           (P->retire ? 2 * hcap * P->S[1] * (int64_t)P->elem + 2 * hcap * (int64_t)sizeof(int4) : 0) +
           P->W * 8 + P->n_polys * 32 + (int64_t)sizeof(InstState);
}

// Heap patches of a fresh list: the root's inequalities, and room for both
// children of the root (and a little more) before the first growth.
static int64_t hcap0(const pcba_problem* P)
{
    if (!P->retire) return 0;
    // 4 alpha patches, or up to 16 alpha while one heap stays within 8 MiB
    const int64_t by_bytes = ((int64_t)8 << 20) / std::max<int64_t>(1, (int64_t)P->S[1] * (int64_t)P->elem);
    return std::max<int64_t>(2, std::max<int64_t>(4 * (int64_t)P->count[1],
                                                  std::min<int64_t>(16 * (int64_t)P->count[1], by_bytes)));
}

// Slots of a fresh list: CAP0, or up to 1024 while the two buffers stay within
// 16 MiB, so that most problems never pause to grow; never beyond M.
static int64_t cap0_of(const pcba_problem* P)
{
    const int64_t by_bytes = ((int64_t)16 << 20) / std::max<int64_t>(1, 2 * item_bytes(P));
    return std::max<int64_t>(P->nc, std::min<int64_t>(P->M_eff, std::max<int64_t>(CAP0, std::min<int64_t>(1024, by_bytes))));
}

static void free_list(pcba_problem* P)
{
    for (int b = 0; b < 2; ++b) {
        if (P->d_buf[b]) pool_free(P->d_buf[b]);
        if (P->d_ids[b]) pool_free(P->d_ids[b]);
        if (P->d_err[b]) pool_free(P->d_err[b]);
        if (P->d_base[b]) pool_free(P->d_base[b]);
        P->d_base[b] = nullptr;
        if (P->d_act[b]) pool_free(P->d_act[b]);
        if (P->d_na[b]) pool_free(P->d_na[b]);
        if (P->d_heap[b]) pool_free(P->d_heap[b]);
        P->d_heap[b] = nullptr;
        P->d_buf[b] = nullptr;
        P->d_ids[b] = nullptr;
        P->d_err[b] = nullptr;
        P->d_act[b] = nullptr;
        P->d_na[b] = nullptr;
    }
    if (P->d_upre) pool_free(P->d_upre);
    P->d_upre = nullptr;
    if (P->d_umap) pool_free(P->d_umap);
    P->d_umap = nullptr;
    if (P->d_pmap) pool_free(P->d_pmap);
    P->d_pmap = nullptr;
    if (P->d_live) pool_free(P->d_live);
    if (P->d_minP) pool_free(P->d_minP);
    if (P->d_maxP) pool_free(P->d_maxP);
    if (P->d_flags) pool_free(P->d_flags);
    if (P->d_stamp) pool_free(P->d_stamp);
    if (P->d_tmat) pool_free(P->d_tmat);
    P->d_live = nullptr;
    P->d_minP = P->d_maxP = nullptr;
    P->d_flags = nullptr;
    P->d_stamp = nullptr;
    P->d_tmat = nullptr;
}

// (Re)allocates the list for `ncap` slots per buffer and, in retiring mode,
// heaps of `nhcap` inequality patches, keeping the current parents: the slots
// [0, old cap) of the parent buffer, their ids, error terms, carried lists and
// heap patches, and the live list are copied; the flags are cleared.
static int alloc_list(pcba_problem* P, int64_t ncap, int64_t nhcap, hipStream_t s)
{
    if (P->retire && nhcap > INT32_MAX)
        return fail(PCBA_E_NOMEM, "an inequality heap would exceed 2^31 patches");
    void* nb[2] = {nullptr, nullptr};
    uint32_t* ni[2] = {nullptr, nullptr};
    float2* ne[2] = {nullptr, nullptr};
    double* nbs[2] = {nullptr, nullptr};
    int32_t* nlive = nullptr;
    double *nmin = nullptr, *nmax = nullptr;
    uint32_t* nfl = nullptr;
    unsigned long long* nst = nullptr;
    double* ntm = nullptr;
    int2* nact[2] = {nullptr, nullptr};
    int32_t* nna[2] = {nullptr, nullptr};
    void* nhp[2] = {nullptr, nullptr};
    int64_t* nup = nullptr;
    int4* num = nullptr;
    int4* npm = nullptr;
    const bool need_tm = P->fp32 && P->opt.rederive_every > 0;
    const int64_t n_up = ncap + 1;   // kept children (up to ncap) plus the end
    auto cleanup = [&]() {
        if (nst) pool_free(nst);
        if (ntm) pool_free(ntm);
        if (nup) pool_free(nup);
        if (num) pool_free(num);
        if (npm) pool_free(npm);
        for (int b = 0; b < 2; ++b) {
            if (nb[b]) pool_free(nb[b]);
            if (ni[b]) pool_free(ni[b]);
            if (ne[b]) pool_free(ne[b]);
            if (nbs[b]) pool_free(nbs[b]);
            if (nact[b]) pool_free(nact[b]);
            if (nna[b]) pool_free(nna[b]);
            if (nhp[b]) pool_free(nhp[b]);
        }
        if (nlive) pool_free(nlive);
        if (nmin) pool_free(nmin);
        if (nmax) pool_free(nmax);
        if (nfl) pool_free(nfl);
    };
    bool ok = true;
    for (int b = 0; b < 2 && ok; ++b) {
        ok = pool_alloc(&nb[b], (size_t)ncap * P->stride * P->elem) == hipSuccess &&
             pool_alloc((void**)&ni[b], (size_t)ncap * P->l * sizeof(uint32_t)) == hipSuccess;
        if (ok && P->fp32)
            ok = pool_alloc((void**)&ne[b], (size_t)ncap * P->n_polys * sizeof(float2)) == hipSuccess &&
                 pool_alloc((void**)&nbs[b], (size_t)ncap * P->n_polys * sizeof(double)) == hipSuccess;
        if (ok && P->retire)
            ok = pool_alloc((void**)&nact[b], (size_t)ncap * P->count[1] * sizeof(int2)) == hipSuccess &&
                 pool_alloc((void**)&nna[b], (size_t)ncap * sizeof(int32_t)) == hipSuccess &&
                 pool_alloc(&nhp[b], (size_t)nhcap * P->S[1] * P->elem) == hipSuccess;
    }
    if (ok && P->retire)
        ok = pool_alloc((void**)&nup, (size_t)n_up * sizeof(int64_t)) == hipSuccess &&
             pool_alloc((void**)&num, (size_t)nhcap * sizeof(int4)) == hipSuccess &&
             pool_alloc((void**)&npm, (size_t)nhcap * sizeof(int4)) == hipSuccess;
    ok = ok && pool_alloc((void**)&nlive, (size_t)ncap * sizeof(int32_t)) == hipSuccess &&
         pool_alloc((void**)&nmin, (size_t)ncap * sizeof(double)) == hipSuccess &&
         pool_alloc((void**)&nmax, (size_t)ncap * sizeof(double)) == hipSuccess &&
         pool_alloc((void**)&nfl, (size_t)ncap * sizeof(uint32_t)) == hipSuccess &&
         pool_alloc((void**)&nst, (size_t)ncap * sizeof(unsigned long long)) == hipSuccess;
    if (ok && need_tm)
        ok = pool_alloc((void**)&ntm, (size_t)(ncap / 2 + 1) * 2 * P->tmw * sizeof(double)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        cleanup();
        return fail(PCBA_E_NOMEM, "device list allocation failed");
    }
    hipError_t e = hipMemsetAsync(nfl, 0, (size_t)ncap * sizeof(uint32_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(nst, 0, (size_t)ncap * sizeof(unsigned long long), s);
    for (int b = 0; b < 2 && e == hipSuccess && P->retire; ++b)
        e = hipMemsetAsync(nna[b], 0, (size_t)ncap * sizeof(int32_t), s);
    if (e == hipSuccess && P->cap > 0) {
        const int cur = P->h_st.cur;
        const int64_t used = std::min<int64_t>(P->cap, ncap);
        e = hipMemcpyAsync(nb[cur], P->d_buf[cur], (size_t)used * P->stride * P->elem,
                           hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ni[cur], P->d_ids[cur], (size_t)used * P->l * sizeof(uint32_t),
                               hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && P->fp32)
            e = hipMemcpyAsync(ne[cur], P->d_err[cur], (size_t)used * P->n_polys * sizeof(float2),
                               hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && P->fp32)
            e = hipMemcpyAsync(nbs[cur], P->d_base[cur], (size_t)used * P->n_polys * sizeof(double),
                               hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(nlive, P->d_live, (size_t)used * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && P->retire) {
            e = hipMemcpyAsync(nact[cur], P->d_act[cur], (size_t)used * P->count[1] * sizeof(int2),
                               hipMemcpyDeviceToDevice, s);
            // the parents' heap patches: everything appended to that heap so far
            const int64_t hused = std::min<int64_t>(P->h_st.htop[cur], std::min(P->hcap, nhcap));
            if (e == hipSuccess && hused > 0)
                e = hipMemcpyAsync(nhp[cur], P->d_heap[cur], (size_t)hused * P->S[1] * P->elem,
                                   hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(nna[cur], P->d_na[cur], (size_t)used * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(nup, P->d_upre, (size_t)std::min<int64_t>(n_up, P->cap + 1) * sizeof(int64_t),
                                   hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(num, P->d_umap, (size_t)std::min(P->hcap, nhcap) * sizeof(int4),
                                   hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(npm, P->d_pmap, (size_t)std::min(P->hcap, nhcap) * sizeof(int4),
                                   hipMemcpyDeviceToDevice, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) {
        cleanup();
        return fail(PCBA_E_DEVICE, std::string("list growth: ") + hipGetErrorString(e));
    }
    free_list(P);
    for (int b = 0; b < 2; ++b) {
        P->d_buf[b] = nb[b];
        P->d_ids[b] = ni[b];
        P->d_err[b] = ne[b];
        P->d_base[b] = nbs[b];
        P->d_act[b] = nact[b];
        P->d_na[b] = nna[b];
        P->d_heap[b] = nhp[b];
    }
    P->hcap = P->retire ? nhcap : 0;
    P->d_upre = nup;
    P->d_umap = num;
    P->d_pmap = npm;
    P->d_live = nlive;
    P->d_minP = nmin;
    P->d_maxP = nmax;
    P->d_flags = nfl;
    P->d_stamp = nst;
    P->d_tmat = ntm;
    P->cap = ncap;
    return PCBA_OK;
}

// Per-thread device scratch for small per-call arrays (problem descriptors,
// prefix sums): distinct threads never share it.
struct Scratch {
    void* p = nullptr;    // device
    void* hp = nullptr;   // pinned host staging of the same size
    size_t cap = 0;
    ~Scratch()
    {
        if (p) (void)hipFree(p);
        if (hp) (void)hipHostFree(hp);
    }
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (p) (void)hipFree(p);
        if (hp) (void)hipHostFree(hp);
        p = hp = nullptr;
        cap = 0;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) e = hipHostMalloc(&hp, bytes, hipHostMallocDefault);
        if (e == hipSuccess) cap = bytes;
        return e;
    }
};
thread_local Scratch t_scratch;

// LDS words of the certification transforms of a problem: every kind and
// axis, in blocks of its longest fibre squared
static size_t tm_words(const pcba_problem* P)
{
    return (size_t)KINDS * P->l * P->maxm * P->maxm;
}

// Uploads the descriptors of probs and the prefix sum of their workgroup
// counts (one per `per` polynomials) into `sc`, followed by each workgroup's
// problem (pre[n + 1 + w]); returns the total in *total.
static int upload_descs(pcba_problem* const* probs, int n, Scratch& sc, hipStream_t s,
                        DevInst** d_insts, int** d_pre, int* total, int* max_S, int* tmw, int per = 1)
{
    std::vector<DevInst> h(n);
    std::vector<int> pre(n + 1, 0);
    *max_S = 1;
    *tmw = 1;
    for (int b = 0; b < n; ++b) {
        h[b] = make_dev(probs[b]);
        pre[b + 1] = pre[b] + (probs[b]->n_polys + per - 1) / per;
        *max_S = std::max(*max_S, probs[b]->max_S);
        *tmw = std::max(*tmw, (int)tm_words(probs[b]));
    }
    for (int b = 0; b < n; ++b)
        for (int w = pre[b]; w < pre[b + 1]; ++w) pre.push_back(b);
    const size_t bytes_i = n * sizeof(DevInst);
    const size_t off_pre = (bytes_i + 255) / 256 * 256;
    const size_t total_b = off_pre + pre.size() * sizeof(int);
    // the staging buffer may still feed an earlier copy on this stream
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(sc.ensure(total_b));
    memcpy(sc.hp, h.data(), bytes_i);
    memcpy((char*)sc.hp + off_pre, pre.data(), pre.size() * sizeof(int));
    HIP_TRY(hipMemcpyAsync(sc.p, sc.hp, total_b, hipMemcpyHostToDevice, s));
    *d_insts = (DevInst*)sc.p;
    *d_pre = (int*)((char*)sc.p + off_pre);
    *total = pre[n];
    return PCBA_OK;
}

// The accurate root and its error bound (once per problem: they depend only on
// the problem's data).
static int accurate_root(pcba_problem* P, hipStream_t s)
{
    DevInst* d_insts = nullptr;
    int* d_pre = nullptr;
    int total = 0, max_S = 1, tmw = 1;
    int rc = upload_descs(&P, 1, t_scratch, s, &d_insts, &d_pre, &total, &max_S, &tmw);
    if (rc != PCBA_OK) return rc;
    HIP_TRY(launch_racc(d_insts, 1, d_pre, total, max_S, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PCBA_OK;
}

// Initial state of every problem: L = {root item}, root patches recomputed on
// the device from the resident monomials (InitPatches), n = 1, p_up = +inf.
static int reset_batch(pcba_problem* const* probs, int n, hipStream_t s)
{
    if (n <= 0) return PCBA_OK;
    for (int b = 0; b < n; ++b) {
        pcba_problem* P = probs[b];
        if (!P->list_released) continue;
        int rc = alloc_list(P, cap0_of(P), hcap0(P), s);
        if (rc != PCBA_OK) return rc;
        P->list_released = false;
    }
    int max_S = 1, tmw = 1;
    for (int b = 0; b < n; ++b) {
        max_S = std::max(max_S, probs[b]->max_S);
        tmw = std::max(tmw, (int)tm_words(probs[b]));
    }
    const int ppb = root_run_length(max_S, tmw);
    if (ppb < 1) return fail(PCBA_E_DEVICE, "root patches exceed the workgroup's LDS");
    DevInst* d_insts = nullptr;
    int* d_pre = nullptr;
    int total = 0;
    int rc = upload_descs(probs, n, t_scratch, s, &d_insts, &d_pre, &total, &max_S, &tmw, ppb);
    if (rc != PCBA_OK) return rc;
    HIP_TRY(launch_reset_root(d_insts, n, d_pre, total, max_S, tmw, ppb, s));
    HIP_TRY(hipStreamSynchronize(s));   // the host descriptors above are pageable
    for (int b = 0; b < n; ++b) probs[b]->root_written = true;
    for (int b = 0; b < n; ++b) {
        pcba_problem* P = probs[b];
        InstState st0;
        memset(&st0, 0, sizeof(st0));
        st0.status = ST_RUNNING;
        st0.K = 1;
        st0.n = 1;
        if (P->opt.direction_rule == 1) {
            double w0[MAXL];
            int d0[MAXL] = {};
            for (int k = 0; k < P->l; ++k) w0[k] = P->hi[k] - P->lo[k];
            st0.r = widest_axis(w0, P->opt.subdiv_lambda, d0, P->l);
        }
        st0.p_up = INFINITY;
        st0.p_lo = INFINITY;
        st0.p_cert = INFINITY;
        P->h_st = st0;
        P->certified_done = false;
        P->seconds = 0.0;
        P->host_steps = 0;
    }
    return PCBA_OK;
}

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* pcba_last_error(void) { return g_last_error.c_str(); }

void pcba_default_options(pcba_options* o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->eps = 1e-3;
    o->delta = 1e-4;
    o->eps_eq = 1e-4;
    o->max_boxes = 1 << 20;
    o->max_iters = 28;
    o->precision = PCBA_FP64_PLAIN;
    o->rederive_every = 16;
    o->stale_filter = 0;
    o->retire_satisfied = 1;
    o->fused_round = 0;
    o->time_limit_s = 0.0;
    o->tile_coefs = 0;
    o->wg_per_cu = 0;
    o->direction_rule = 0;
    o->split_engine = PCBA_SPLIT_VALU;
    o->subdiv_lambda = 0.5;
    o->persistent_steps = 0;
}

int pcba_create_problem(int32_t l, const double* lo, const double* hi, const int32_t* cost_deg,
                        const double* cost_coef, int32_t n_ineq, const int32_t* ineq_deg,
                        const double* ineq_coef, int32_t n_eq, const int32_t* eq_deg,
                        const double* eq_coef, const pcba_options* opt, pcba_problem** out)
{
    if (!out) return fail(PCBA_E_ARG, "out is NULL");
    *out = nullptr;
    if (l < 1 || l > PCBA_MAX_DIM) return fail(PCBA_E_ARG, "l outside 1..PCBA_MAX_DIM");
    if (!lo || !hi || !cost_deg || !cost_coef) return fail(PCBA_E_ARG, "NULL box or cost");
    if (n_ineq < 0 || n_eq < 0) return fail(PCBA_E_ARG, "negative constraint count");
    if (n_ineq > 0 && (!ineq_deg || !ineq_coef)) return fail(PCBA_E_ARG, "NULL inequality arrays");
    if (n_eq > 0 && (!eq_deg || !eq_coef)) return fail(PCBA_E_ARG, "NULL equality arrays");
    pcba_options o;
    pcba_default_options(&o);
    if (opt) o = *opt;
    if (!(o.eps > 0) || !(o.delta > 0) || !(o.eps_eq > 0) || !std::isfinite(o.eps) ||
        !std::isfinite(o.eps_eq))
        return fail(PCBA_E_ARG, "eps, delta and eps_eq must be positive");
    if (o.max_boxes < 2) return fail(PCBA_E_ARG, "max_boxes (M) must be >= 2");
    if (o.max_iters < 1) return fail(PCBA_E_ARG, "max_iters (N) must be >= 1");
    if ((int64_t)o.max_iters * l >= MAX_STEPS) return fail(PCBA_E_ARG, "max_iters * l must stay below 60000");
    if (o.precision != PCBA_FP64_PLAIN && o.precision != PCBA_FP32)
        return fail(PCBA_E_ARG, "unknown precision");
    if (o.rederive_every < 0) return fail(PCBA_E_ARG, "rederive_every must be >= 0");
    if (o.retire_satisfied != 0 && o.retire_satisfied != 1)
        return fail(PCBA_E_ARG, "retire_satisfied must be 0 or 1");
    if (o.fused_round != 0 && o.fused_round != 1) return fail(PCBA_E_ARG, "fused_round must be 0 or 1");
    {
        const int tmax = o.precision == PCBA_FP32 ? MAX_TILE32 : MAX_TILE64;
        if (o.tile_coefs != 0 && (o.tile_coefs < 256 || o.tile_coefs > tmax))
            return fail(PCBA_E_ARG, "tile_coefs must be 0 or within 256.." + std::to_string(tmax));
        // a round keeps 2^l child regions of a tile in LDS: the regions together
        // stay within the two of a one-direction step
        if (o.fused_round && o.tile_coefs * (1 << l) > 2 * tmax)
            return fail(PCBA_E_ARG, "tile_coefs too large for fused_round (2^l regions in LDS)");
    }
    if (o.wg_per_cu < 0) return fail(PCBA_E_ARG, "wg_per_cu must be >= 0");
    if (o.direction_rule != 0 && o.direction_rule != 1) return fail(PCBA_E_ARG, "direction_rule must be 0 or 1");
    if (o.persistent_steps != 0 && o.persistent_steps != 1)
        return fail(PCBA_E_ARG, "persistent_steps must be 0 or 1");
    if (o.split_engine != PCBA_SPLIT_VALU && o.split_engine != PCBA_SPLIT_MFMA)
        return fail(PCBA_E_ARG, "split_engine must be PCBA_SPLIT_VALU or PCBA_SPLIT_MFMA");
    if (!(o.subdiv_lambda > 0.0 && o.subdiv_lambda < 1.0))
        return fail(PCBA_E_ARG, "subdiv_lambda must lie in (0,1)");
    if (o.fused_round && (o.direction_rule != 0 || o.subdiv_lambda != 0.5))
        return fail(PCBA_E_ARG, "fused_round needs direction_rule = 0 and subdiv_lambda = 1/2");
    if (o.precision == PCBA_FP32 && o.subdiv_lambda != 0.5 && o.rederive_every != 0)
        return fail(PCBA_E_ARG, "PCBA_FP32 with subdiv_lambda != 1/2 needs rederive_every = 0");
    if (o.fused_round && l > 2) return fail(PCBA_E_ARG, "fused_round needs l <= 2");
    if (o.fused_round && o.retire_satisfied && n_ineq > 0)
        return fail(PCBA_E_ARG, "fused_round needs retire_satisfied = 0");
    for (int k = 0; k < l; ++k)
        if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) || !(hi[k] > lo[k]))
            return fail(PCBA_E_ARG, "box bounds must be finite with lo < hi");

    pcba_problem* P = new pcba_problem();
    P->l = l;
    for (int k = 0; k < l; ++k) { P->lo[k] = lo[k]; P->hi[k] = hi[k]; }
    P->opt = o;
    P->fp32 = o.precision == PCBA_FP32;
    P->nc = o.fused_round ? (1 << l) : 2;
    P->retire = o.retire_satisfied == 1 && n_ineq > 0;
    P->elem = P->fp32 ? 4 : 8;
    P->count[0] = 1;
    P->count[1] = n_ineq;
    P->count[2] = n_eq;
    const int32_t* degs[KINDS] = {cost_deg, ineq_deg, eq_deg};
    const double* coefs[KINDS] = {cost_coef, ineq_coef, eq_coef};
    for (int t = 0; t < KINDS; ++t) {
        for (int i = 0; i < P->count[t]; ++i)
            for (int k = 0; k < l; ++k) {
                const int d = degs[t][i * l + k];
                if (d < 0 || d > PCBA_MAX_DEGREE) {
                    delete P;
                    return fail(PCBA_E_ARG, "degree outside 0..PCBA_MAX_DEGREE");
                }
                P->deg[t][k] = std::max(P->deg[t][k], d);
            }
        int64_t S = 1;
        for (int k = 0; k < l; ++k) S *= P->deg[t][k] + 1;
        if (S > MAX_PATCH) {
            delete P;
            return fail(PCBA_E_ARG, "a patch exceeds 3584 coefficients");
        }
        P->S[t] = P->count[t] ? (int)S : 0;
        for (int k = 0; k < l; ++k) P->maxm = std::max(P->maxm, P->deg[t][k] + 1);
    }
    P->off[0] = 0;
    P->off[1] = P->S[0];
    P->off[2] = P->off[1] + (int64_t)P->count[1] * P->S[1];
    P->W = P->off[2] + (int64_t)P->count[2] * P->S[2];
    P->n_polys = 1 + n_ineq + n_eq;
    P->max_S = std::max(P->S[0], std::max(P->S[1], P->S[2]));
    // a list slot holds the item in the same layout, except in retiring mode,
    // where the inequalities live in the heaps and a slot is the cost, then
    // the equalities
    for (int t = 0; t < KINDS; ++t) P->soff[t] = P->off[t];
    int64_t slot_words = P->W;
    if (P->retire) {
        P->soff[1] = P->S[0];
        P->soff[2] = P->S[0];
        slot_words = P->S[0] + (int64_t)P->count[2] * P->S[2];
    }
    const int64_t align = P->fp32 ? 64 : 32;  // 256-byte item slots
    P->stride = (slot_words + align - 1) / align * align;
    // tiles: the cost alone, then runs of constraint patches of ~TILE_ELEMS coefficients
    P->tile_polys[0] = 1;
    P->tile_start[0] = 0;
    int T = 1;
    for (int t = 1; t < KINDS; ++t) {
        P->tile_start[t] = T;
        if (P->count[t] == 0) { P->tile_polys[t] = 1; continue; }
        // FP32 tiles hold twice the coefficients: the same bytes per unit
        const int target = P->fp32 ? 2 * TILE_ELEMS : TILE_ELEMS;
        P->tile_polys[t] = std::max(1, std::min(P->count[t], target / std::max(1, P->S[t])));
        T += (P->count[t] + P->tile_polys[t] - 1) / P->tile_polys[t];
    }
    P->tile_start[KINDS] = T;
    P->T = T;
    // k_sub tiles: runs of ~TILE_ELEMS coefficients of one kind across parents,
    // at most one patch per lane (a round keeps 2^l children of the tile in LDS:
    // its tiles are 2 / 2^l as large)
    // The LDS of a tile is sized for the largest tile of any kind and for the
    // most patches of any kind; with constraints, the cost patches (one per
    // parent, a small share of the work) go 64 to a tile, so that their count
    // does not set the per-patch tables of every tile.
    for (int t = 0; t < KINDS; ++t) {
        const int target = o.tile_coefs > 0 ? o.tile_coefs : (P->fp32 ? 2 * TILE_ELEMS : TILE_ELEMS) * 2 / P->nc;
        int cap = SUB_THREADS;
        if (t == 0 && P->count[1] + P->count[2] > 0) cap = 64;
        P->ptp[t] = P->count[t] ? std::max(1, std::min(cap, target / std::max(1, P->S[t]))) : 1;
    }
    // sub-interval transforms per child (FP32 re-derivation): m^2 words and m rows per kind and axis
    for (int t = 0; t < KINDS; ++t) {
        P->tmk[t] = P->tmw;
        if (P->count[t] == 0) continue;
        for (int k = 0; k < l; ++k) {
            P->tmw += (P->deg[t][k] + 1) * (P->deg[t][k] + 1);
            P->rows += P->deg[t][k] + 1;
        }
    }

    // monomials, zero-padded to each kind's common multi-degree, in item layout
    std::vector<double> mono(P->W, 0.0);
    for (int t = 0; t < KINDS; ++t) {
        int64_t in_off = 0;
        for (int i = 0; i < P->count[t]; ++i) {
            const int32_t* d = degs[t] + i * l;
            int64_t sd = 1;
            for (int k = 0; k < l; ++k) sd *= d[k] + 1;
            for (int64_t q = 0; q < sd; ++q) {
                const double v = coefs[t][in_off + q];
                if (!std::isfinite(v)) {
                    delete P;
                    return fail(PCBA_E_ARG, "non-finite coefficient");
                }
                int64_t rem = q, o2 = 0, mul = 1;
                for (int k = l - 1; k >= 0; --k) {
                    const int64_t jk = rem % (d[k] + 1);
                    rem /= d[k] + 1;
                    o2 += jk * mul;
                    mul *= P->deg[t][k] + 1;
                }
                mono[P->off[t] + (int64_t)i * P->S[t] + o2] = v;
            }
            in_off += sd;
        }
    }
    // per kind and axis: pre-map matrix A (x = lo + w t) and conversion matrix U
    std::vector<double> mats, macc;
    std::vector<int> matoff(KINDS * MAXL, 0);
    for (int t = 0; t < KINDS; ++t)
        for (int r = 0; r < l; ++r) {
            const int n = P->deg[t][r], m = n + 1;
            const double w = hi[r] - lo[r];
            matoff[t * MAXL + r] = (int)mats.size();
            std::vector<double> A(m * m, 0.0), U(m * m, 0.0);
            for (int i = 0; i <= n; ++i) {
                double wi = 1.0;
                for (int q = 0; q < i; ++q) wi *= w;
                for (int j = i; j <= n; ++j) {
                    double lp = 1.0;
                    for (int q = 0; q < j - i; ++q) lp *= lo[r];
                    A[i * m + j] = wi * binom(j, i) * lp;
                }
            }
            for (int k = 0; k <= n; ++k)
                for (int i = 0; i <= k; ++i) U[k * m + i] = binom(k, i) / binom(n, i);
            mats.insert(mats.end(), A.begin(), A.end());
            mats.insert(mats.end(), U.begin(), U.end());
            // combined matrix M = U A by the polar form of x^j at (lo x (n-k), hi x k):
            // a hypergeometric average of lo^(j-i) hi^i, and Mabs, the sum of the
            // terms' magnitudes (same offsets as A and U)
            std::vector<double> M(m * m, 0.0), Ma(m * m, 0.0);
            for (int k = 0; k <= n; ++k)
                for (int j = 0; j <= n; ++j) {
                    double sum = 0.0, sabs = 0.0;
                    for (int i = std::max(0, j - (n - k)); i <= std::min(j, k); ++i) {
                        double t = binom(k, i) * binom(n - k, j - i) / binom(n, j);
                        for (int q = 0; q < j - i; ++q) t *= lo[r];
                        for (int q = 0; q < i; ++q) t *= hi[r];
                        sum += t;
                        sabs += std::fabs(t);
                    }
                    M[k * m + j] = sum;
                    Ma[k * m + j] = sabs;
                }
            macc.insert(macc.end(), M.begin(), M.end());
            macc.insert(macc.end(), Ma.begin(), Ma.end());
        }

    // memory-test bound: M, and no more than the device can hold for two buffers
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        delete P;
        return fail(PCBA_E_DEVICE, "hipMemGetInfo failed (no device?)");
    }
    const int64_t per_item = 2 * item_bytes(P);
    const double avail = (double)free_b + (double)pool_cached_bytes();   // cached blocks are reusable
    const int64_t hbm_items = (int64_t)(avail * 0.85) / std::max<int64_t>(1, per_item);
    P->M_eff = std::min<int64_t>(o.max_boxes, std::max<int64_t>(2, hbm_items));
    if (P->M_eff < 2) {
        delete P;
        return fail(PCBA_E_NOMEM, "not enough device memory for the root item and two children");
    }

    hipStream_t s = nullptr;
    bool ok = library_stream(&s) == hipSuccess &&
              hipMalloc((void**)&P->d_root, P->W * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&P->d_root_err, 2 * P->n_polys * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&P->d_racc, P->W * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&P->d_macc, std::max<size_t>(1, macc.size()) * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&P->d_cert, 3 * P->n_polys * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&P->d_st, sizeof(InstState)) == hipSuccess &&
              hipMalloc((void**)&P->d_trace, MAX_TRACE * sizeof(TraceRec)) == hipSuccess &&
              hipMalloc((void**)&P->d_mono, P->W * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&P->d_mats, std::max<size_t>(1, mats.size()) * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&P->d_matoff, matoff.size() * sizeof(int)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        pcba_destroy_problem(P);
        return fail(PCBA_E_NOMEM, "device allocation failed");
    }
    const int64_t cap0 = cap0_of(P);
    int rc = alloc_list(P, std::max<int64_t>(2, cap0), hcap0(P), s);
    if (rc != PCBA_OK) {
        std::string m = g_last_error;
        pcba_destroy_problem(P);
        return fail(rc, m);
    }
    hipError_t e = hipMemcpyAsync(P->d_mono, mono.data(), P->W * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !mats.empty())
        e = hipMemcpyAsync(P->d_mats, mats.data(), mats.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !macc.empty())
        e = hipMemcpyAsync(P->d_macc, macc.data(), macc.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(P->d_matoff, matoff.data(), matoff.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) rc = accurate_root(P, s);
    if (e == hipSuccess && rc == PCBA_OK) rc = reset_batch(&P, 1, s);
    if (e != hipSuccess || rc != PCBA_OK) {
        std::string m = e != hipSuccess ? std::string(hipGetErrorString(e)) : g_last_error;
        pcba_destroy_problem(P);
        return fail(PCBA_E_DEVICE, std::string("root conversion: ") + m);
    }
    *out = P;
    return PCBA_OK;
}

int pcba_reset(pcba_problem* P, void* stream)
{
    if (!P) return fail(PCBA_E_ARG, "NULL problem");
    return reset_batch(&P, 1, (hipStream_t)stream);
}

int pcba_reset_batch(pcba_problem* const* probs, int32_t n, void* stream)
{
    if (n < 0 || (n > 0 && !probs)) return fail(PCBA_E_ARG, "bad batch");
    for (int b = 0; b < n; ++b)
        if (!probs[b]) return fail(PCBA_E_ARG, "NULL problem in batch");
    return reset_batch(probs, n, (hipStream_t)stream);
}

int pcba_read_trace(const pcba_problem* P, int32_t* k_in, int32_t* k_kept, double* p_up,
                    double* p_lo, int32_t cap)
{
    if (!P || cap < 0) return fail(PCBA_E_ARG, "bad arguments");
    const int n = std::min<int>(std::min<int>(P->h_st.steps, MAX_TRACE), cap);
    if (n <= 0) return 0;
    std::vector<TraceRec> h(n);
    HIP_TRY(hipMemcpy(h.data(), P->d_trace, n * sizeof(TraceRec), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
        if (k_in) k_in[i] = h[i].k_in;
        if (k_kept) k_kept[i] = h[i].k_kept;
        if (p_up) p_up[i] = h[i].p_up;
        if (p_lo) p_lo[i] = h[i].p_lo;
    }
    return n;
}

int pcba_read_trace_patches(const pcba_problem* P, int64_t* a_in, int64_t* a_kept, int32_t cap)
{
    if (!P || cap < 0) return fail(PCBA_E_ARG, "bad arguments");
    const int n = std::min<int>(std::min<int>(P->h_st.steps, MAX_TRACE), cap);
    if (n <= 0) return 0;
    std::vector<TraceRec> h(n);
    HIP_TRY(hipMemcpy(h.data(), P->d_trace, n * sizeof(TraceRec), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
        if (a_in) a_in[i] = h[i].a_in;
        if (a_kept) a_kept[i] = h[i].a_kept;
    }
    return n;
}

void pcba_release_cached_memory(void) { pool_trim(); }

void pcba_profile_enable(int32_t on) { g_prof.on = on != 0; }
void pcba_profile_reset(void)
{
    for (int k = 0; k < PCBA_NUM_KERNELS; ++k) { g_prof.ms[k] = 0.0; g_prof.launches[k] = 0; }
    g_prof.used = 0;
}
void pcba_profile_read(double* ms, int64_t* launches)
{
    for (int k = 0; k < PCBA_NUM_KERNELS; ++k) {
        if (ms) ms[k] = g_prof.ms[k];
        if (launches) launches[k] = g_prof.launches[k];
    }
}

void pcba_destroy_problem(pcba_problem* P)
{
    if (!P) return;
    free_list(P);
    if (P->d_root) (void)hipFree(P->d_root);
    if (P->d_root_err) (void)hipFree(P->d_root_err);
    if (P->d_racc) (void)hipFree(P->d_racc);
    if (P->d_macc) (void)hipFree(P->d_macc);
    if (P->d_cert) (void)hipFree(P->d_cert);
    if (P->d_st) (void)hipFree(P->d_st);
    if (P->d_trace) (void)hipFree(P->d_trace);
    if (P->d_mono) (void)hipFree(P->d_mono);
    if (P->d_mats) (void)hipFree(P->d_mats);
    if (P->d_matoff) (void)hipFree(P->d_matoff);
    delete P;
}

int64_t pcba_patch_words(const pcba_problem* P) { return P ? P->W : 0; }
int64_t pcba_item_bytes(const pcba_problem* P) { return P ? item_bytes(P) : 0; }

int64_t pcba_footprint_bytes(const pcba_problem* P, int64_t boxes)
{
    if (!P) return 0;
    return footprint_of(P, boxes, P->hcap);
}

// ---------------------------------------------------------------- engine

int pcba_engine_create(int64_t budget_bytes, int64_t reserve_boxes, void* stream, pcba_engine** out)
{
    if (!out || reserve_boxes < 0) return fail(PCBA_E_ARG, "bad engine arguments");
    hipStream_t s = (hipStream_t)stream;
    if (!s && library_stream(&s) != hipSuccess) return fail(PCBA_E_DEVICE, "stream creation failed");
    pcba_engine* E = new pcba_engine();
    E->budget = budget_bytes > 0 ? budget_bytes : INT64_MAX;
    E->reserve = reserve_boxes;
    E->stream = s;
    *out = E;
    return PCBA_OK;
}

void pcba_engine_destroy(pcba_engine* E)
{
    if (!E) return;
    if (E->stream) (void)hipStreamSynchronize(E->stream);
    bufs_put(E->b);
    delete E;
}

int64_t pcba_engine_used_bytes(const pcba_engine* E) { return E ? E->used : 0; }

int pcba_engine_submit(pcba_engine* E, pcba_problem* P, int32_t* admitted)
{
    if (!E || !P || !admitted) return fail(PCBA_E_ARG, "NULL argument");
    *admitted = 0;
    if (E->active.size() >= (size_t)MAX_BATCH) return PCBA_OK;
    const int64_t fp = pcba_footprint_bytes(P, std::max(P->cap, E->reserve));
    if (!E->active.empty() && E->used + fp > E->budget) return PCBA_OK;
    P->footprint = fp;
    E->used += fp;
    P->t_start = now_s();
    P->host_steps = P->h_st.steps;
    E->active.push_back(P);
    E->dirty = true;
    *admitted = 1;
    return PCBA_OK;
}

static int engine_upload(pcba_engine* E)
{
    const int n = (int)E->active.size();
    if (n > E->b.cap) {
        bufs_put(E->b);
        HIP_TRY(bufs_get(std::max(n, 2 * E->b.cap), &E->b));
    }
    // every earlier use of the staging buffer has completed: the engine
    // synchronises its stream at the end of each batch of steps
    for (int b = 0; b < n; ++b) {
        E->b.h_insts[b] = make_dev(E->active[b]);
        E->b.h_insts[b].hostflag = E->b.d_flag;
    }
    if (n) HIP_TRY(hipMemcpyAsync(E->b.d_insts, E->b.h_insts, n * sizeof(DevInst), hipMemcpyHostToDevice, E->stream));
    E->dirty = false;
    return PCBA_OK;
}

// The largest k_sub tile of a problem: coefficients and patches
static void sub_tile(const pcba_problem* P, int* tem, int* tpm)
{
    for (int t = 0; t < KINDS; ++t)
        if (t == 0 || P->count[t]) {
            *tem = std::max(*tem, P->ptp[t] * P->S[t]);
            *tpm = std::max(*tpm, P->ptp[t]);
        }
}
static size_t rederive_lds(const pcba_problem* P)
{
    // the largest chunk, transforms and per-patch records (52 bytes) of any kind
    int TE = P->S[0], npc = 1;
    for (int t = 1; t < KINDS; ++t)
        if (P->count[t]) {
            const int cp = std::min(REDERIVE_CHUNK, std::max(1, MAX_TILE64 / P->S[t]));
            TE = std::max(TE, std::min(P->tile_polys[t], cp) * P->S[t]);
            npc = std::max(npc, std::min(P->tile_polys[t], cp));
        }
    return ((size_t)TE + (size_t)P->l * P->maxm * P->maxm) * 8 + (size_t)npc * 52 + 16;
}

// FP64 certification of every finished problem in one launch, then their states.
static int certify_batch(pcba_engine* E, std::vector<pcba_problem*>& fin)
{
    const int n = (int)fin.size();
    if (n == 0) return PCBA_OK;
    int max_S = 1, tmw = 1;
    for (auto* P : fin) {
        max_S = std::max(max_S, P->max_S);
        tmw = std::max(tmw, (int)tm_words(P));
    }
    const int ppb = certify_run_length(max_S, tmw);
    if (ppb < 1) return fail(PCBA_E_DEVICE, "certification patches exceed the workgroup's LDS");
    DevInst* d_insts = nullptr;
    int* d_pre = nullptr;
    int total = 0;
    int rc = upload_descs(fin.data(), n, t_scratch, E->stream, &d_insts, &d_pre, &total, &max_S, &tmw, ppb);
    if (rc != PCBA_OK) return rc;
    HIP_TRY(launch_certify(d_insts, n, d_pre, total, max_S, tmw, ppb, E->stream));
    HIP_TRY(launch_gather(d_insts, n, E->b.d_states, E->stream));   // into host memory
    HIP_TRY(hipStreamSynchronize(E->stream));
    const double t = now_s();
    for (int b = 0; b < n; ++b) {
        fin[b]->h_st = E->b.h_states[b];
        fin[b]->certified_done = true;
        fin[b]->seconds = t - fin[b]->t_start;
    }
    return PCBA_OK;
}

// Frees the lists of the finished problems the engine still holds (their
// results stay readable; pcba_reset allocates a list again).  Returns the count.
static int release_done_lists(pcba_engine* E)
{
    int k = 0;
    (void)hipStreamSynchronize(E->stream);
    for (auto* P : E->done) {
        if (P->list_released || P->cap == 0) continue;
        free_list(P);
        P->cap = 0;
        P->list_released = true;
        k += 1;
    }
    return k;
}

// One batch of up to n_steps steps over the active problems, then a sync.
static int engine_steps(pcba_engine* E, int n_steps)
{
    if (E->active.empty()) return PCBA_OK;
    if (E->dirty) {
        int rc = engine_upload(E);
        if (rc != PCBA_OK) return rc;
    }
    const int n = (int)E->active.size();
    bool any64 = false, any32 = false, anyrd = false, mf32 = false;
    int maxm64 = 1, maxm32 = 1, nr64 = 2, nr32 = 2, wg64 = 0, wg32 = 0;
    size_t ldsrd = 0;
    int tem64 = 1, tpm64 = 1, tem32 = 1, tpm32 = 1;
    for (auto* P : E->active) {
        if (P->fp32) {
            any32 = true;
            if (P->opt.split_engine == PCBA_SPLIT_MFMA) mf32 = true;
            maxm32 = std::max(maxm32, P->maxm);
            nr32 = std::max(nr32, P->nc);
            wg32 = std::max(wg32, P->opt.wg_per_cu);
            sub_tile(P, &tem32, &tpm32);
            if (P->opt.rederive_every > 0) {
                anyrd = true;
                ldsrd = std::max(ldsrd, rederive_lds(P));
            }
        } else {
            any64 = true;
            maxm64 = std::max(maxm64, P->maxm);
            nr64 = std::max(nr64, P->nc);
            wg64 = std::max(wg64, P->opt.wg_per_cu);
            sub_tile(P, &tem64, &tpm64);
        }
    }
    // The steps go out in chunks of CHECK_STEPS; after each chunk the host
    // waits for the end of the chunk before it (the newest one keeps the GPU
    // busy) and stops early when a kernel has flagged a problem that finished
    // or paused for growth.
    __atomic_store_n(E->b.h_flag, 0, __ATOMIC_RELEASE);
    // Whole steps in one cooperative launch (k_steps) when the batch allows it:
    // one precision, at most PLAN_FUSE_MAX problems, every problem asking for it,
    // short lists (its cut runs on the subdivision's 256 lanes), kernel timing
    // off (the timed launches are per kernel), and for the steps in which no
    // FP32 re-derivation falls due.
    bool persist = !g_prof.on && n <= PLAN_FUSE_MAX && any64 != any32 && !mf32;
    for (auto* P : E->active)
        if (!P->opt.persistent_steps || P->cap > 4096) persist = false;
    if (persist) {
        int coop = 0;
        persist = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, E->b.dev) == hipSuccess && coop;
    }
    auto rd_due = [&](int s) {
        for (auto* P : E->active) {
            if (!P->fp32 || P->opt.rederive_every <= 0 || P->h_st.status != ST_RUNNING) continue;
            if ((P->host_steps + s + 1) % P->opt.rederive_every == 0) return true;
        }
        return false;
    };
    bool used_steps = false;
    if (persist) *E->b.h_berr = 0;
    for (int s = 0; s < n_steps; ++s) {
        if (s > 0 && s % CHECK_STEPS == 0) {
            const int k = (s / CHECK_STEPS) & 1;
            HIP_TRY(hipEventRecord(E->b.ev[k], E->stream));
            if (s >= 2 * CHECK_STEPS) {
                HIP_TRY(hipEventSynchronize(E->b.ev[k ^ 1]));
                if (__atomic_load_n(E->b.h_flag, __ATOMIC_ACQUIRE)) break;
            }
        }
        if (persist) {
            // the rest of this check interval, up to a step with a re-derivation
            const int lim = std::min(CHECK_STEPS - s % CHECK_STEPS, n_steps - s);
            int kk = 0;
            while (kk < lim && !rd_due(s + kk)) ++kk;
            if (kk > 0) {
                const bool f32 = any32;
                HIP_TRY(launch_steps(E->b.d_insts, n, E->b.d_plan, E->b.d_info, f32, f32 ? maxm32 : maxm64,
                                     f32 ? tem32 : tem64, f32 ? tpm32 : tpm64, f32 ? nr32 : nr64,
                                     f32 ? wg32 : wg64, kk, E->b.d_bar, E->b.d_berr, E->stream));
                used_steps = true;
                s += kk - 1;
                continue;
            }
        }
        // upper bound of this step's units: K at most multiplies by the
        // children per parent each step, and a problem never holds more than
        // cap / nc parents
        int64_t ub64 = 0, ub32 = 0, ubrd = 0, ubrows = 0, maxc = 0;
        for (auto* P : E->active) {
            if (P->h_st.status != ST_RUNNING) continue;
            const int64_t k = std::min<int64_t>(P->cap / P->nc, (int64_t)P->h_st.K << std::min(s * (P->nc / 2), 30));
            maxc = std::max(maxc, P->nc * k);
            const int64_t u = k * P->T;
            if (!P->fp32) ub64 += u;
            else {
                const int st = P->host_steps + s;
                const bool due = P->opt.rederive_every > 0 && ((st + 1) % P->opt.rederive_every) == 0;
                if (due) { ubrd += u; ubrows += k * P->nc * P->rows; } else ub32 += u;
            }
        }
        // the plan of the step: formed inside the first subdivision launch for
        // small batches, else by its own launch
        const bool l64 = any64 && ub64 > 0, l32 = any32 && ub32 > 0;
        bool planned = false;
        if (n > PLAN_FUSE_MAX || !(l64 || l32)) {
            HIP_TRY(prof_begin(E->stream));
            HIP_TRY(launch_plan(E->b.d_insts, n, E->b.d_plan, E->b.d_info, E->stream));
            HIP_TRY(prof_end(4, E->stream));
            planned = true;
        }
        if (l64) {
            hipEvent_t e0, e1;
            HIP_TRY(prof_pair(0, &e0, &e1));
            HIP_TRY(launch_sub(E->b.d_insts, n, E->b.d_plan, E->b.d_info, !planned, false, false, maxm64,
                               (int)std::min<int64_t>(GRID_MAX, ub64), tem64, tpm64, nr64, wg64, E->stream, e0, e1));
            planned = true;
        }
        if (l32) {
            hipEvent_t e0, e1;
            HIP_TRY(prof_pair(1, &e0, &e1));
            HIP_TRY(launch_sub(E->b.d_insts, n, E->b.d_plan, E->b.d_info, !planned, true, mf32, maxm32,
                               (int)std::min<int64_t>(GRID_MAX, ub32), tem32, tpm32, nr32, wg32, E->stream, e0, e1));
            planned = true;
        }
        if (anyrd && ubrd > 0) {
            HIP_TRY(prof_begin(E->stream));
            HIP_TRY(launch_rederive(E->b.d_insts, n, E->b.d_plan, E->b.d_info, (int)std::min<int64_t>(GRID_MAX, ubrd),
                                    (int)std::min<int64_t>(4096, (ubrows + 255) / 256), ldsrd, E->stream));
            HIP_TRY(prof_end(2, E->stream));
        }
        HIP_TRY(prof_begin(E->stream));
        const long long split = g_cut_split.load(std::memory_order_relaxed);
        const int part = g_cut_part.load(std::memory_order_relaxed);
        if (split > 0 && maxc > split) {
            // room for the split cut's records (grown between steps: the stream
            // is drained before the old buffer goes)
            const int64_t need = (int64_t)n * ((maxc + part - 1) / part);
            if (need > E->b.parts_cap) {
                HIP_TRY(hipStreamSynchronize(E->stream));
                if (E->b.d_parts) HIP_TRY(hipFree(E->b.d_parts));
                E->b.d_parts = nullptr;
                E->b.parts_cap = 0;
                HIP_TRY(hipMalloc((void**)&E->b.d_parts, (size_t)need * sizeof(CutPart)));
                E->b.parts_cap = need;
            }
        }
        HIP_TRY(launch_cut(E->b.d_insts, E->b.d_info, n, maxc, split, part, E->b.d_parts, E->b.parts_cap,
                           E->stream));
        HIP_TRY(prof_end(3, E->stream));
    }
    HIP_TRY(launch_gather(E->b.d_insts, n, E->b.d_states, E->stream));   // into host memory
    HIP_TRY(hipStreamSynchronize(E->stream));
    prof_collect();
    if (used_steps && __atomic_load_n(E->b.h_berr, __ATOMIC_ACQUIRE))
        return fail(PCBA_E_DEVICE, "a grid barrier of the step kernel timed out");

    // growth, time limits, finished problems
    const double t = now_s();
    std::vector<pcba_problem*> still, fin;
    // some problem will step again, or finish, without growing
    bool progress = false;
    for (int b = 0; b < n; ++b)
        if (E->b.h_states[b].status != ST_GROW) progress = true;
    for (int b = 0; b < n; ++b) {
        pcba_problem* P = E->active[b];
        P->h_st = E->b.h_states[b];
        P->host_steps = P->h_st.steps;
        if (P->h_st.status == ST_GROW) {
            // room for this step's children with a quarter to spare, and at least
            // half again the current capacity (bounded by M); in retiring mode the
            // same for the heap, whose children take at most twice the carried
            // patches of the parents
            const int64_t need = (int64_t)P->nc * P->h_st.K;
            int64_t want = P->cap, hwant = P->hcap;
            if (need > P->cap)
                want = std::min<int64_t>(P->M_eff, std::max<int64_t>(need + need / 4, P->cap + P->cap / 2));
            const int64_t hneed = 2 * P->h_st.a_live;
            if (P->retire && hneed > P->hcap) hwant = std::max<int64_t>(hneed + hneed / 4, P->hcap + P->hcap / 2);
            const int64_t extra = footprint_of(P, std::max(want, E->reserve), hwant) - P->footprint;
            if (b > 0 && extra > 0 && E->used + extra > E->budget) {
                still.push_back(P);   // stays paused until the budget has room
                continue;
            }
            // try only what can fit: the new list comes on top of the old one
            // for the copy; finished problems give their lists back first
            const int64_t nbytes = footprint_of(P, want, hwant);
            int rc = PCBA_E_NOMEM;
            if ((int64_t)pool_available_bytes() < nbytes) release_done_lists(E);
            if ((int64_t)pool_available_bytes() >= nbytes) {
                rc = alloc_list(P, want, hwant, E->stream);
                if (rc != PCBA_OK && release_done_lists(E) > 0) rc = alloc_list(P, want, hwant, E->stream);
            }
            InstState& st = P->h_st;
            if (rc == PCBA_OK) {
                st.status = ST_RUNNING;
            } else if (progress) {
                // the device is full: wait, paused, until other problems finish
                still.push_back(P);
                continue;
            } else {
                // nothing else can free memory: the memory test fires, and the
                // list this problem releases lets the others continue
                P->M_eff = P->cap;
                st.status = ST_MEMLIMIT;
                progress = true;
            }
            HIP_TRY(hipMemcpyAsync(P->d_st, &st, sizeof(st), hipMemcpyHostToDevice, E->stream));
            HIP_TRY(hipStreamSynchronize(E->stream));
            E->dirty = true;
            const int64_t fp = pcba_footprint_bytes(P, std::max(P->cap, E->reserve));
            E->used += fp - P->footprint;
            P->footprint = fp;
            if (st.status == ST_RUNNING) progress = true;
        }
        if (P->h_st.status == ST_RUNNING && P->opt.time_limit_s > 0 &&
            t - P->t_start > P->opt.time_limit_s) {
            P->h_st.status = ST_TIMEOUT;
            HIP_TRY(hipMemcpyAsync(P->d_st, &P->h_st, sizeof(InstState), hipMemcpyHostToDevice, E->stream));
        }
        if (P->h_st.status == ST_RUNNING) {
            still.push_back(P);
        } else {
            fin.push_back(P);
        }
    }
    if (!fin.empty()) {
        int rc = certify_batch(E, fin);
        if (rc != PCBA_OK) return rc;
        for (auto* P : fin) {
            E->used -= P->footprint;
            P->footprint = 0;
            E->done.push_back(P);
        }
        E->dirty = true;
    }
    if (still.size() != E->active.size()) {
        E->active.swap(still);
        E->dirty = true;
    }
    return PCBA_OK;
}

int pcba_engine_run(pcba_engine* E, int32_t n_steps, int32_t* n_active)
{
    if (!E || n_steps < 0) return fail(PCBA_E_ARG, "bad engine arguments");
    int rc = engine_steps(E, n_steps);
    if (n_active) *n_active = (int32_t)E->active.size();
    return rc;
}

int pcba_engine_poll(pcba_engine* E, pcba_problem** done, int32_t cap, int32_t* n_done)
{
    if (!E || !n_done || (cap > 0 && !done)) return fail(PCBA_E_ARG, "NULL argument");
    int k = 0;
    while (k < cap && !E->done.empty()) {
        done[k++] = E->done.front();
        E->done.erase(E->done.begin());
    }
    *n_done = k;
    return PCBA_OK;
}

// ---------------------------------------------------------------- solve

int pcba_solve_batch(pcba_problem* const* probs, int32_t n, void* stream)
{
    if (n < 0 || (n > 0 && !probs)) return fail(PCBA_E_ARG, "bad batch");
    pcba_engine* E = nullptr;
    int rc = pcba_engine_create(0, 0, stream, &E);
    if (rc != PCBA_OK) return rc;
    const double t0 = now_s();
    for (int i = 0; i < n; ++i) {
        if (!probs[i]) { pcba_engine_destroy(E); return fail(PCBA_E_ARG, "NULL problem in batch"); }
        if (probs[i]->h_st.status != ST_RUNNING) continue;
        int32_t adm = 0;
        rc = pcba_engine_submit(E, probs[i], &adm);
        if (rc != PCBA_OK || !adm) {
            pcba_engine_destroy(E);
            return rc != PCBA_OK ? rc : fail(PCBA_E_ARG, "batch larger than one engine launch");
        }
        probs[i]->t_start = t0;
    }
    // lists then grow within 85% of the HBM still free: a problem whose growth
    // does not fit waits for others to finish instead of failing, so a result
    // does not depend on what else is in the batch (the oldest always grows)
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
        E->budget = E->used + (int64_t)(0.85 * ((double)free_b + (double)pool_cached_bytes()));
    // between host checks the steps run until a kernel flags a problem that
    // stopped or paused (at most MAX_STEPS_PER_SYNC), or STEPS_PER_SYNC when a
    // time limit needs watching
    bool timed = false;
    for (auto* P : E->active) timed = timed || P->opt.time_limit_s > 0;
    while (!E->active.empty()) {
        rc = engine_steps(E, timed ? STEPS_PER_SYNC : MAX_STEPS_PER_SYNC);
        if (rc != PCBA_OK) break;
    }
    pcba_engine_destroy(E);
    return rc;
}

int pcba_solve(pcba_problem* P, void* stream)
{
    if (!P) return fail(PCBA_E_ARG, "NULL problem");
    pcba_problem* arr[1] = {P};
    return pcba_solve_batch(arr, 1, stream);
}

int pcba_step(pcba_problem* P, int32_t n_steps, void* stream)
{
    if (!P || n_steps < 0) return fail(PCBA_E_ARG, "bad arguments");
    if (P->h_st.status != ST_RUNNING) return PCBA_OK;
    pcba_engine* E = nullptr;
    int rc = pcba_engine_create(0, 0, stream, &E);
    if (rc != PCBA_OK) return rc;
    int32_t adm = 0;
    rc = pcba_engine_submit(E, P, &adm);
    const int target = P->h_st.steps + n_steps;
    while (rc == PCBA_OK && !E->active.empty() && P->h_st.steps < target) {
        rc = engine_steps(E, std::min(STEPS_PER_SYNC, target - P->h_st.steps));
    }
    if (!E->active.empty()) { E->used = 0; E->active.clear(); }
    pcba_engine_destroy(E);
    return rc;
}

int pcba_result(const pcba_problem* P, pcba_result_t* out)
{
    if (!P || !out) return fail(PCBA_E_ARG, "NULL argument");
    memset(out, 0, sizeof(*out));
    const InstState& st = P->h_st;
    out->outcome = (st.status == ST_GROW) ? PCBA_RUNNING : st.status;
    out->has_x = st.has_x;
    out->p_up = st.p_up;
    out->p_lo = st.p_lo;
    for (int k = 0; k < P->l; ++k) {
        out->depth[k] = st.depth[k];
        if (st.has_x) {
            const double w = P->hi[k] - P->lo[k];
            out->x_depth[k] = st.x_depth[k];
            out->x_index[k] = st.x_index[k];
            double ta, tb;
            unit_interval(P->opt.subdiv_lambda, st.x_depth[k], st.x_index[k], ta, tb);
            out->x_lo[k] = P->lo[k] + w * ta;
            out->x_hi[k] = P->lo[k] + w * tb;
        }
    }
    out->rounds = st.n;
    out->steps = st.steps;
    out->list_len = st.K;
    out->peak_len = st.peak;
    out->next_dir = st.r;
    out->certified = P->certified_done ? st.cert_ok : 0;
    out->p_cert = P->certified_done ? st.p_cert : INFINITY;
    out->cert_err = st.cert_err;
    out->err_max = st.err_max;
    out->seconds = P->seconds;
    out->capacity = P->cap;
    return PCBA_OK;
}

int pcba_result_batch(const pcba_problem* const* probs, int32_t n, pcba_result_t* out)
{
    if (n < 0 || (n > 0 && (!probs || !out))) return fail(PCBA_E_ARG, "NULL argument or n < 0");
    for (int32_t b = 0; b < n; ++b)
        if (!probs[b]) return fail(PCBA_E_ARG, "NULL problem in the batch");
    for (int32_t b = 0; b < n; ++b) {
        const int rc = pcba_result(probs[b], &out[b]);
        if (rc != PCBA_OK) return rc;
    }
    return PCBA_OK;
}

int pcba_list_size(const pcba_problem* P, int64_t* len)
{
    if (!P || !len) return fail(PCBA_E_ARG, "NULL argument");
    *len = P->h_st.K;
    return PCBA_OK;
}

static int read_list_impl(const pcba_problem* P, uint32_t* ids, double* patches, double* err,
                          int64_t cap)
{
    const int K = P->h_st.K;
    if (P->list_released) return fail(PCBA_E_STATE, "the list was released to make room for other problems");
    if (cap < K) return fail(PCBA_E_ARG, "capacity smaller than the list");
    if (K == 0) return PCBA_OK;
    hipStream_t s = nullptr;
    HIP_TRY(library_stream(&s));
    double* d_out = nullptr;
    uint32_t* d_ids = nullptr;
    double* d_err = nullptr;
    hipError_t e = hipMalloc((void**)&d_out, (size_t)K * P->W * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&d_ids, (size_t)K * P->l * sizeof(uint32_t));
    if (e == hipSuccess && P->fp32) e = hipMalloc((void**)&d_err, (size_t)K * P->n_polys * sizeof(double));
    if (e == hipSuccess) e = launch_pack(make_dev(P), K, d_out, d_ids, d_err, P->W, s);
    if (e == hipSuccess && patches)
        e = hipMemcpyAsync(patches, d_out, (size_t)K * P->W * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && ids)
        e = hipMemcpyAsync(ids, d_ids, (size_t)K * P->l * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && err && P->fp32)
        e = hipMemcpyAsync(err, d_err, (size_t)K * P->n_polys * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (d_out) (void)hipFree(d_out);
    if (d_ids) (void)hipFree(d_ids);
    if (d_err) (void)hipFree(d_err);
    if (e != hipSuccess) return fail(PCBA_E_DEVICE, std::string("read list: ") + hipGetErrorString(e));
    return PCBA_OK;
}

int pcba_read_list(const pcba_problem* P, uint32_t* ids, double* patches, int64_t cap)
{
    if (!P) return fail(PCBA_E_ARG, "NULL problem");
    return read_list_impl(P, ids, patches, nullptr, cap);
}

int pcba_read_errors(const pcba_problem* P, double* err, int64_t cap)
{
    if (!P || !err) return fail(PCBA_E_ARG, "NULL argument");
    if (!P->fp32) return fail(PCBA_E_STATE, "error bounds exist only in PCBA_FP32 mode");
    return read_list_impl(P, nullptr, nullptr, err, cap);
}

int pcba_read_list_noalloc(const pcba_problem* P, uint32_t* ids, double* patches, int64_t cap, void* stream)
{
    if (!P) return fail(PCBA_E_ARG, "NULL problem");
    const int64_t K = P->h_st.K;
    if (P->list_released) return fail(PCBA_E_STATE, "the list was released to make room for other problems");
    if (cap < K) return fail(PCBA_E_ARG, "capacity smaller than the list");
    // staging: the packed patches, then (256-byte aligned) the ids
    const int64_t pat_bytes = K * P->W * (int64_t)sizeof(double);
    const int64_t ids_off = (pat_bytes + 255) / 256 * 256;
    const int64_t need = ids_off + K * P->l * (int64_t)sizeof(uint32_t);
    if (need > PCBA_STATIC_SCRATCH_BYTES)
        return fail(PCBA_E_ARG, "the list needs " + std::to_string(need) +
                                    " bytes of staging, above the static scratch of " +
                                    std::to_string((long long)PCBA_STATIC_SCRATCH_BYTES) +
                                    " bytes (pcba_read_list has no such limit)");
    if (K == 0) return PCBA_OK;
    unsigned char* base = nullptr;
    int rc = static_scratch(&base);
    if (rc != PCBA_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (!s) HIP_TRY(library_stream(&s));
    double* d_out = (double*)base;
    uint32_t* d_ids = (uint32_t*)(base + ids_off);
    // an earlier call's staging may still be read by its copies
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(launch_pack(make_dev(P), (int)K, d_out, d_ids, nullptr, P->W, s));
    if (patches)
        HIP_TRY(hipMemcpyAsync(patches, d_out, (size_t)pat_bytes, hipMemcpyDeviceToHost, s));
    if (ids) HIP_TRY(hipMemcpyAsync(ids, d_ids, (size_t)K * P->l * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PCBA_OK;
}

int pcba_set_cut_split(int64_t children, int32_t part)
{
    if (children < 0) return fail(PCBA_E_ARG, "children must be >= 0");
    if (part < 64) return fail(PCBA_E_ARG, "part must be >= 64");
    g_cut_split.store(children, std::memory_order_relaxed);
    g_cut_part.store(part, std::memory_order_relaxed);
    return PCBA_OK;
}

int pcba_rtd_constraints(const int32_t* w_xdeg, const int32_t* w_qdeg, const double* w_coef, int32_t n_pts,
                         const double* pts, double eps_q, double* out)
{
    if (!w_xdeg || !w_qdeg || !w_coef || n_pts < 0 || (n_pts > 0 && (!pts || !out)))
        return fail(PCBA_E_ARG, "NULL argument or n_pts < 0");
    for (int k = 0; k < 2; ++k)
        if (w_xdeg[k] < 0 || w_qdeg[k] < 0 || w_xdeg[k] > PCBA_MAX_DEGREE || w_qdeg[k] > PCBA_MAX_DEGREE)
            return fail(PCBA_E_ARG, "degree outside 0..PCBA_MAX_DEGREE");
    if (!std::isfinite(eps_q)) return fail(PCBA_E_ARG, "eps_q must be finite");
    const int na = w_xdeg[0] + 1, nb = w_xdeg[1] + 1;
    const int64_t nq = (int64_t)(w_qdeg[0] + 1) * (w_qdeg[1] + 1);
    for (int32_t i = 0; i < n_pts; ++i) {
        const double x1 = pts[2 * i], x2 = pts[2 * i + 1];
        if (!std::isfinite(x1) || !std::isfinite(x2)) return fail(PCBA_E_ARG, "non-finite obstacle point");
        double* g = out + (int64_t)i * nq;
        for (int64_t e = 0; e < nq; ++e) g[e] = 0.0;
        // w(x_i, q): the coefficient of q1^c q2^d is sum_{a,b} w[a,b,c,d] x1^a x2^b
        double pa = 1.0;
        for (int a = 0; a < na; ++a) {
            double pb = pa;
            for (int b = 0; b < nb; ++b) {
                const double* wab = w_coef + ((int64_t)a * nb + b) * nq;
                for (int64_t e = 0; e < nq; ++e) g[e] += wab[e] * pb;
                pb *= x2;
            }
            pa *= x1;
        }
        g[0] += eps_q;
    }
    return PCBA_OK;
}

int pcba_read_root(const pcba_problem* P, double* patches)
{
    if (!P || !patches) return fail(PCBA_E_ARG, "NULL argument");
    HIP_TRY(hipMemcpy(patches, P->d_root, P->W * sizeof(double), hipMemcpyDeviceToHost));
    return PCBA_OK;
}

}  // extern "C"
