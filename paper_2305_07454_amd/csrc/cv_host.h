// cv_host.h -- host-side helpers shared by the C-ABI entry points: argument
// checks, workspace carving, launch checks and the optional per-kernel timing.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "cvetl.h"

namespace cvh {

constexpr size_t WS_ALIGN = 256;

inline size_t align_up(size_t x, size_t a = WS_ALIGN) { return (x + a - 1) / a * a; }

inline uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Carves aligned sub-buffers out of a workspace; with base == nullptr it only
// measures, so the same code computes the size query and the layout.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T>
    T* take(uint64_t count)
    {
        off = align_up(off);
        T* p = base ? (T*)(base + off) : nullptr;
        off += (size_t)count * sizeof(T);
        return p;
    }
    size_t size() const { return align_up(off); }
};

inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Launch bookkeeping for the optional timing of kernel families.
struct TimedScope {
    const char* family;
    hipStream_t stream;
    void* token;
    TimedScope(const char* fam, hipStream_t s);
    ~TimedScope();
};

cv_status last_launch_status();

// fills `n` 32-bit words with `v` on `s` (a kernel, never hipMemsetAsync, so
// the sequence stays valid inside captured graphs)
void fill_u32(void* p, uint32_t v, uint64_t n, hipStream_t s);
void fill_u64(void* p, uint64_t v, uint64_t n, hipStream_t s);

// Checking build (CVETL_DEBUG): checker kernels after the sort and after the
// rows of a summary or grid call; nothing in the release build.
void debug_sort(const void* K0, const void* K1, const uint32_t* passes, const uint32_t* err0, const uint32_t* err1,
                uint64_t n, const uint32_t* perm, const uint64_t* soff, uint32_t S, hipStream_t s);
void debug_rows(const int64_t* keys, const uint32_t* cnt, const uint32_t* nj, const cv_result* res, uint64_t cap,
                const uint64_t* off, uint32_t S, uint32_t bit, hipStream_t s);

inline int grid_for(uint64_t n, int block, int cap = 1 << 30)
{
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (uint64_t)cap) g = cap;
    return (int)g;
}

}  // namespace cvh
