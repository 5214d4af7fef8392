// cv_debug.hip -- the checking build (CVETL_DEBUG, libcvetl_debug.so).
//
// After each stage, small checker kernels test what the stage guarantees and
// set bits of a per-device flag word (never a trap): the sort's final words
// strictly ascending (each word is (key bits) << index_bits | record index, so
// this is the order and its stability at once), the permutation's entries
// inside their shard, each shard's journey ids strictly ascending, and each
// shard's group keys strictly ascending with 1 <= distinct journeys <= count.
// In the release build the hooks compile to nothing and the two entry points
// return CV_ERR_UNSUPPORTED.
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_host.h"

using namespace cv;

#ifdef CVETL_DEBUG
namespace {

__device__ u32 g_dbg;  // the flag word of this device

__device__ __forceinline__ void dbg_raise(bool bad, u32 bit)
{
    if (__ballot(bad) && lane_id() == 0) atomicOr(&g_dbg, bit);
}

// a caller's array strictly ascending
__global__ void k_dbg_check(const u64* a, u64 n, u32 bit)
{
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        dbg_raise(i + 1 < n && !(a[i] < a[i + 1]), bit);
}

__global__ void k_dbg_words(const u64* K0, const u64* K1, const u32* passes, const u32* err0, const u32* err1, u64 n,
                            u32 bit)
{
    if (*err0 || *err1) return;  // a range or capacity error is reported by the sort itself
    const u64* a = (*passes & 1) ? K1 : K0;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        dbg_raise(i + 1 < n && !(a[i] < a[i + 1]), bit);
}

__global__ void k_dbg_perm(const u32* perm, u64 n, const u64* soff, u32 S, u32 bit)
{
    for (u64 k = (u64)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (u64)gridDim.x * blockDim.x) {
        u64 size = n;
        if (S > 1) {
            const u32 sh = shard_of(soff, S, k);
            size = soff[sh + 1] - soff[sh];
        }
        dbg_raise(perm[k] >= size, bit);
    }
}

// rows [0, count) of a result, per shard ([off[s], off[s+1]) when off is
// given): keys strictly ascending inside each shard; with cnt and nj, also
// 1 <= nj <= cnt
__global__ void k_dbg_rows(const i64* keys, const u32* cnt, const u32* nj, const cv_result* res, u64 cap,
                           const u64* off, u32 S, u32 bit)
{
    if (res->status != CV_OK) return;
    const u64 rows = res->count < cap ? res->count : cap;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (u64)gridDim.x * blockDim.x) {
        bool bad = false;
        if (i + 1 < rows) {
            bool same_shard = true;
            if (off && S > 1) {
                // i + 1 starts a shard when some off[s] equals it
                u32 lo = 0, hi = S;
                while (lo < hi) {
                    const u32 mid = (lo + hi) >> 1;
                    if (off[mid] < i + 1) lo = mid + 1;
                    else hi = mid;
                }
                same_shard = !(lo <= S && off[lo] == i + 1);
            }
            if (same_shard && !(keys[i] < keys[i + 1])) bad = true;
        }
        if (cnt && nj && (nj[i] < 1 || nj[i] > cnt[i])) bad = true;
        dbg_raise(bad, bit);
    }
}

}  // namespace
#endif

namespace cvh {

void debug_sort(const void* K0, const void* K1, const uint32_t* passes, const uint32_t* err0, const uint32_t* err1,
                uint64_t n, const uint32_t* perm, const uint64_t* soff, uint32_t S, hipStream_t s)
{
#ifdef CVETL_DEBUG
    const unsigned g = (unsigned)grid_for(n, 256, 4096);
    hipLaunchKernelGGL(k_dbg_words, dim3(g), dim3(256), 0, s, (const u64*)K0, (const u64*)K1, passes, err0, err1, n,
                       (u32)CV_DEBUG_SORT_ORDER);
    if (perm)
        hipLaunchKernelGGL(k_dbg_perm, dim3(g), dim3(256), 0, s, perm, n, soff, S, (u32)CV_DEBUG_PERM_RANGE);
#else
    (void)K0, (void)K1, (void)passes, (void)err0, (void)err1, (void)n, (void)perm, (void)soff, (void)S, (void)s;
#endif
}

void debug_rows(const int64_t* keys, const uint32_t* cnt, const uint32_t* nj, const cv_result* res, uint64_t cap,
                const uint64_t* off, uint32_t S, uint32_t bit, hipStream_t s)
{
#ifdef CVETL_DEBUG
    if (!res || !keys || cap == 0) return;
    hipLaunchKernelGGL(k_dbg_rows, dim3((unsigned)grid_for(cap, 256, 4096)), dim3(256), 0, s, keys, cnt, nj, res, cap,
                       off, S, bit);
#else
    (void)keys, (void)cnt, (void)nj, (void)res, (void)cap, (void)off, (void)S, (void)bit, (void)s;
#endif
}

}  // namespace cvh

extern "C" {

cv_status cv_debug_flags(uint32_t* flags, int reset)
{
#ifdef CVETL_DEBUG
    if (!flags) return CV_ERR_INVALID_ARGUMENT;
    if (hipDeviceSynchronize() != hipSuccess) return CV_ERR_DEVICE;
    if (hipMemcpyFromSymbol(flags, HIP_SYMBOL(g_dbg), sizeof(u32)) != hipSuccess) return CV_ERR_DEVICE;
    if (reset) {
        const u32 z = 0;
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_dbg), &z, sizeof(u32)) != hipSuccess) return CV_ERR_DEVICE;
    }
    return CV_OK;
#else
    (void)flags, (void)reset;
    return CV_ERR_UNSUPPORTED;
#endif
}

cv_status cv_debug_check_ascending(const uint64_t* a, uint64_t n, void* stream)
{
#ifdef CVETL_DEBUG
    if (n >= (1ull << 32) || (n > 0 && !a)) return CV_ERR_INVALID_ARGUMENT;
    if (n < 2) return CV_OK;
    hipLaunchKernelGGL(k_dbg_check, dim3((unsigned)cvh::grid_for(n, 256, 4096)), dim3(256), 0, (hipStream_t)stream,
                       (const u64*)a, n, (u32)CV_DEBUG_CHECK);
    return cvh::last_launch_status();
#else
    (void)a, (void)n, (void)stream;
    return CV_ERR_UNSUPPORTED;
#endif
}

}  // extern "C"
