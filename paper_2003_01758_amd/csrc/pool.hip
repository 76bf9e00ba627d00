// pool.hip -- device memory arena for the list buffers.
//
// A list grows by allocating larger buffers, copying the parents and freeing
// the old ones, and finished problems give their lists back.  A list holds a
// dozen arrays, most of them small; with many problems resident and the device
// nearly full, each hipMalloc can take tens of milliseconds, far more than the
// kernels of a step.  Blocks under 1 GiB therefore come from an arena: chunks
// of 4 GiB taken from the device, 256-byte aligned blocks handed out best fit
// by size, freed blocks merged with their free neighbours inside the same
// chunk, and fully free chunks given back when room is needed (or on
// pool_trim).  Larger blocks are allocated from the device one by one and
// freed at once, so that the device's own address mapping, not the arena,
// deals with their fragmentation; those calls are few, and one is made only
// when the device reports room for it.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "pool.h"

namespace pcba {

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kHeadroom = (size_t)256 << 20;  // left free for the runtime and small buffers
constexpr size_t kChunk = (size_t)4 << 30;
constexpr size_t kLarge = (size_t)1 << 30;   // blocks at least this big bypass the arena

struct Block {
    size_t len;
    int chunk;
};

struct DeviceArena {
    std::vector<std::pair<char*, size_t>> chunks;   // base, size (base null once released)
    std::map<char*, Block> free_by_addr;
    std::multimap<size_t, char*> free_by_size;
    std::unordered_map<void*, Block> live;
    std::unordered_map<void*, size_t> large;   // blocks allocated on their own
    size_t free_bytes = 0;
};

std::mutex g_mu;
std::map<int, DeviceArena> g_arenas;

DeviceArena& arena_of_current()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    return g_arenas[dev];
}

void insert_free(DeviceArena& A, char* p, Block b)
{
    A.free_by_addr[p] = b;
    A.free_by_size.emplace(b.len, p);
    A.free_bytes += b.len;
}

void erase_free(DeviceArena& A, std::map<char*, Block>::iterator it)
{
    auto range = A.free_by_size.equal_range(it->second.len);
    for (auto s = range.first; s != range.second; ++s)
        if (s->second == it->first) {
            A.free_by_size.erase(s);
            break;
        }
    A.free_bytes -= it->second.len;
    A.free_by_addr.erase(it);
}

// Releases every chunk that is one free block.
size_t trim_locked(DeviceArena& A)
{
    size_t released = 0;
    for (int c = 0; c < (int)A.chunks.size(); ++c) {
        char* base = A.chunks[c].first;
        if (!base) continue;
        auto it = A.free_by_addr.find(base);
        if (it == A.free_by_addr.end() || it->second.chunk != c || it->second.len != A.chunks[c].second) continue;
        erase_free(A, it);
        (void)hipFree(base);
        released += A.chunks[c].second;
        A.chunks[c].first = nullptr;
        A.chunks[c].second = 0;
    }
    return released;
}

size_t device_free()
{
    size_t fr = 0, tot = 0;
    return hipMemGetInfo(&fr, &tot) == hipSuccess ? fr : 0;
}

// A new chunk able to hold `len`: kChunk bytes if the device has room for
// them, else exactly `len`.
bool add_chunk(DeviceArena& A, size_t len)
{
    size_t want = std::max(len, kChunk);
    size_t fr = device_free();
    if (fr < want + kHeadroom) {
        want = len;
        if (fr < want + kHeadroom && trim_locked(A) > 0) fr = device_free();
        if (fr < want + kHeadroom) return false;
    }
    char* base = nullptr;
    if (hipMalloc((void**)&base, want) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const int c = (int)A.chunks.size();
    A.chunks.emplace_back(base, want);
    insert_free(A, base, Block{want, c});
    return true;
}

}  // namespace

hipError_t pool_alloc(void** out, size_t bytes)
{
    *out = nullptr;
    const size_t len = (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceArena& A = arena_of_current();
    if (len >= kLarge) {
        size_t fr = device_free();
        if (fr < len + kHeadroom && trim_locked(A) > 0) fr = device_free();
        if (fr < len + kHeadroom) return hipErrorOutOfMemory;
        void* p = nullptr;
        if (hipMalloc(&p, len) != hipSuccess) {
            (void)hipGetLastError();
            return hipErrorOutOfMemory;
        }
        A.large[p] = len;
        *out = p;
        return hipSuccess;
    }
    auto fit = A.free_by_size.lower_bound(len);
    if (fit == A.free_by_size.end()) {
        if (!add_chunk(A, len)) return hipErrorOutOfMemory;
        fit = A.free_by_size.lower_bound(len);
        if (fit == A.free_by_size.end()) return hipErrorOutOfMemory;
    }
    char* p = fit->second;
    auto it = A.free_by_addr.find(p);
    const Block b = it->second;
    erase_free(A, it);
    if (b.len > len) insert_free(A, p + len, Block{b.len - len, b.chunk});
    A.live[p] = Block{len, b.chunk};
    *out = p;
    return hipSuccess;
}

void pool_free(void* vp)
{
    if (!vp) return;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceArena& A = arena_of_current();
    auto lg = A.large.find(vp);
    if (lg != A.large.end()) {
        A.large.erase(lg);
        (void)hipFree(vp);
        return;
    }
    auto lv = A.live.find(vp);
    if (lv == A.live.end()) {
        (void)hipFree(vp);   // not from the arena
        return;
    }
    char* p = (char*)vp;
    Block b = lv->second;
    A.live.erase(lv);
    // merge with the free neighbours of the same chunk
    auto next = A.free_by_addr.lower_bound(p);
    if (next != A.free_by_addr.end() && next->first == p + b.len && next->second.chunk == b.chunk) {
        b.len += next->second.len;
        erase_free(A, next);
    }
    auto prev = A.free_by_addr.lower_bound(p);
    if (prev != A.free_by_addr.begin()) {
        --prev;
        if (prev->first + prev->second.len == p && prev->second.chunk == b.chunk) {
            char* q = prev->first;
            b.len += prev->second.len;
            erase_free(A, prev);
            p = q;
        }
    }
    insert_free(A, p, b);
}

void pool_trim()
{
    std::lock_guard<std::mutex> lk(g_mu);
    trim_locked(arena_of_current());
}

size_t pool_available_bytes()
{
    const size_t fr = device_free();
    std::lock_guard<std::mutex> lk(g_mu);
    const size_t a = fr + arena_of_current().free_bytes;
    return a > kHeadroom ? a - kHeadroom : 0;
}

size_t pool_cached_bytes()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return arena_of_current().free_bytes;
}

}  // namespace pcba
