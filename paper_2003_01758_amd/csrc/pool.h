// pool.h -- device memory arena for the list buffers (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pcba {

// A 256-byte aligned block of at least `bytes` on the current device, carved
// from the arena (or, from 1 GiB up, allocated on its own); device memory is
// taken only when the device reports room for it (fully free chunks are
// returned first when that makes the room).  hipErrorOutOfMemory otherwise.
hipError_t pool_alloc(void** out, size_t bytes);
// Returns a block to the arena of the current device (NULL is ignored).  The
// caller guarantees no pending work still uses it.
void pool_free(void* p);
// Returns every fully free chunk of the current device to the device.
void pool_trim();
// Bytes held by the arena in free blocks.
size_t pool_cached_bytes();
// Device memory a new allocation could use now: free device memory plus the
// arena's free blocks, less a small headroom kept for the runtime.
size_t pool_available_bytes();

}  // namespace pcba
