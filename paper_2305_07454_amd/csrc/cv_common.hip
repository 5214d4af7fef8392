// cv_common.hip -- ABI version, error strings, fill kernels and the optional
// per-kernel-family timing used by the benchmark.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "cv_host.h"

namespace {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t v, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

struct Pending {
    hipEvent_t a, b;
};
struct Family {
    double total_ms = 0.0;
    uint64_t launches = 0;
    std::vector<Pending> pending;
};

std::mutex g_mu;
bool g_on = false;
std::unordered_map<std::string, Family> g_fam;
std::vector<hipEvent_t> g_free;

hipEvent_t get_event()
{
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drain(Family& f)
{
    for (auto& p : f.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            f.total_ms += ms;
            f.launches += 1;
        }
        g_free.push_back(p.a);
        g_free.push_back(p.b);
    }
    f.pending.clear();
}

}  // namespace

namespace cvh {

void fill_u32(void* p, uint32_t v, uint64_t n, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, (uint32_t*)p, v, n);
}

void fill_u64(void* p, uint64_t v, uint64_t n, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, (uint64_t*)p, v, n);
}

cv_status last_launch_status()
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CV_OK : CV_ERR_DEVICE;
}

TimedScope::TimedScope(const char* fam, hipStream_t s) : family(fam), stream(s), token(nullptr)
{
    if (!fam) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    hipEvent_t a = get_event();
    if (!a) return;
    if (hipEventRecord(a, s) != hipSuccess) {
        g_free.push_back(a);
        return;
    }
    token = (void*)a;
}

TimedScope::~TimedScope()
{
    if (!token) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t a = (hipEvent_t)token;
    hipEvent_t b = get_event();
    if (!b || hipEventRecord(b, stream) != hipSuccess) {
        // no closing event: this launch goes untimed
        g_free.push_back(a);
        if (b) g_free.push_back(b);
        return;
    }
    g_fam[family].pending.push_back(Pending{a, b});
}

}  // namespace cvh

extern "C" {

uint32_t cv_abi_version(void) { return CV_ABI_VERSION; }

const char* cv_strerror(cv_status s)
{
    // C callers may pass any int; read it as one rather than as the enum,
    // whose C++ value range ends at the largest enumerator's bit width.
    int v;
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
    case CV_OK: return "ok";
    case CV_ERR_INVALID_ARGUMENT: return "invalid argument";
    case CV_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case CV_ERR_CAPACITY: return "output capacity exceeded";
    case CV_ERR_RANGE: return "packed key range exceeds 64 bits";
    case CV_ERR_DEVICE: return "HIP device error";
    case CV_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

cv_status cv_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return CV_OK;
}

cv_status cv_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_fam) {
        drain(kv.second);
        kv.second.total_ms = 0.0;
        kv.second.launches = 0;
    }
    return CV_OK;
}

cv_status cv_timing_read(const char* family, double* total_ms, uint64_t* launches)
{
    if (!family || !total_ms || !launches) return CV_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_fam.find(family);
    if (it == g_fam.end()) {
        *total_ms = 0.0;
        *launches = 0;
        return CV_OK;
    }
    drain(it->second);
    *total_ms = it->second.total_ms;
    *launches = it->second.launches;
    return CV_OK;
}

}  // extern "C"
