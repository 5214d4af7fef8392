// cv_lattice.hip -- the dense spatio-temporal lattice built from a group
// table, its per-channel min-max normalisation, and a filter over groups
// (Methods steps (4)-(6); Table 2's speed / volume normalisation and volume
// filter rows; the transformed-data output's speed and volume channels per
// direction and time bin).
//
//   k_lat_fill     zero the lattice (16-byte stores)
//   k_lat_scatter  one thread per group: mean speed and distinct journeys
//                  into the cell of its time bin and direction
//   k_lat_minmax   per channel, min and max over the occupied cells
//   k_lat_norm     one thread per (cell, direction): both channels rescaled
//   k_filt_*       order-preserving compaction of group indices
#include <hip/hip_runtime.h>

#include <cmath>

#include "cv_device.h"
#include "cv_host.h"

using namespace cv;

namespace {

constexpr int LB = 256;
constexpr int FT = LB * 8;  // groups per filter tile

__global__ void __launch_bounds__(LB) k_lat_fill(float4* __restrict__ p, u64 n4)
{
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (u64 i = (u64)blockIdx.x * LB + threadIdx.x; i < n4; i += (u64)gridDim.x * LB) p[i] = z;
}

__global__ void __launch_bounds__(LB) k_lat_fill_tail(float* __restrict__ p, u64 from, u64 n)
{
    const u64 i = from + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// Group g's key = (td * n_lat + ilat) * n_lon + ilon with td = tbin, or
// tbin * D + sector when the lattice has D = n_dir + 1 direction sectors.
// Channels of a time bin: 2 d (mean speed of sector d) and 2 d + 1 (its
// distinct journeys).
__global__ void __launch_bounds__(LB) k_lat_scatter(const i64* __restrict__ key, const u32* __restrict__ count,
                                                     const u32* __restrict__ nj, const double* __restrict__ sum,
                                                     u64 G, i64 cells, u32 D, i64 t_first, i64 n_t,
                                                     float* __restrict__ out)
{
    for (u64 g = (u64)blockIdx.x * LB + threadIdx.x; g < G; g += (u64)gridDim.x * LB) {
        const i64 k = key[g];
        if (k < 0) continue;
        const i64 td = k / cells, cell = k % cells;
        const i64 tb = td / (i64)D, d = td % (i64)D;
        const i64 t = tb - t_first;
        if (t < 0 || t >= n_t) continue;
        const u32 c = count[g];
        const u64 base = ((u64)t * 2 * D + 2 * (u64)d) * (u64)cells + (u64)cell;
        out[base] = c ? (float)(sum[g] / (double)c) : 0.f;
        out[base + (u64)cells] = (float)nj[g];
    }
}

// Per channel, min and max over occupied cells (volume > 0), as ordered
// integer images.  Block b takes cells [CH * (b % cpi), +CH) of (time bin,
// sector) image b / cpi (each thread CH / LB of them) and writes its four
// partials (speed min / max, volume min / max) to part[4 b ..]; one block per
// sector then reduces them into mm[4 d ..] (no atomics on shared addresses).
constexpr int CH = LB * 16;

__global__ void __launch_bounds__(LB) k_lat_minmax(const float* __restrict__ lat, u32 D, u64 cells, u64 cpi,
                                                    u32* __restrict__ part)
{
    __shared__ u32 s_mm[4];
    const u64 img = blockIdx.x / cpi;
    const u64 c0 = (blockIdx.x % cpi) * CH;
    const u32 d = (u32)(img % D);
    const float* sp = lat + (img / D * 2 * D + 2 * d) * cells;
    const float* vo = sp + cells;
    u32 smin = ~0u, smax = 0u, vmin = ~0u, vmax = 0u;
#pragma unroll 4
    for (int k = 0; k < CH / LB; ++k) {
        const u64 i = c0 + (u64)k * LB + threadIdx.x;
        if (i < cells) {
            const float v = vo[i];
            if (v > 0.f) {
                const u32 a = ord_f32(sp[i]), b = ord_f32(v);
                smin = a < smin ? a : smin;
                smax = a > smax ? a : smax;
                vmin = b < vmin ? b : vmin;
                vmax = b > vmax ? b : vmax;
            }
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const u32 a = __shfl_xor(smin, o, WAVE), b = __shfl_xor(smax, o, WAVE);
        const u32 c = __shfl_xor(vmin, o, WAVE), e = __shfl_xor(vmax, o, WAVE);
        smin = a < smin ? a : smin;
        smax = b > smax ? b : smax;
        vmin = c < vmin ? c : vmin;
        vmax = e > vmax ? e : vmax;
    }
    if (threadIdx.x == 0) {
        s_mm[0] = ~0u;
        s_mm[1] = 0u;
        s_mm[2] = ~0u;
        s_mm[3] = 0u;
    }
    __syncthreads();
    if (lane_id() == 0 && smin != ~0u) {
        atomicMin(&s_mm[0], smin);
        atomicMax(&s_mm[1], smax);
        atomicMin(&s_mm[2], vmin);
        atomicMax(&s_mm[3], vmax);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u32* o = part + 4 * (u64)blockIdx.x;
        o[0] = s_mm[0];
        o[1] = s_mm[1];
        o[2] = s_mm[2];
        o[3] = s_mm[3];
    }
}

// sector d = blockIdx.x: the partials of its images t * D + d, all chunks
__global__ void __launch_bounds__(LB) k_lat_mm_reduce(const u32* __restrict__ part, u64 n_t, u32 D, u64 cpi,
                                                       u32* __restrict__ mm)
{
    __shared__ u32 s_mm[4];
    const u32 d = blockIdx.x;
    u32 a0 = ~0u, a1 = 0u, a2 = ~0u, a3 = 0u;
    const u64 per = n_t * cpi;
    for (u64 i = threadIdx.x; i < per; i += LB) {
        const u64 b = ((i / cpi) * D + d) * cpi + i % cpi;
        const u32* p = part + 4 * b;
        a0 = p[0] < a0 ? p[0] : a0;
        a1 = p[1] > a1 ? p[1] : a1;
        a2 = p[2] < a2 ? p[2] : a2;
        a3 = p[3] > a3 ? p[3] : a3;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const u32 x0 = __shfl_xor(a0, o, WAVE), x1 = __shfl_xor(a1, o, WAVE);
        const u32 x2 = __shfl_xor(a2, o, WAVE), x3 = __shfl_xor(a3, o, WAVE);
        a0 = x0 < a0 ? x0 : a0;
        a1 = x1 > a1 ? x1 : a1;
        a2 = x2 < a2 ? x2 : a2;
        a3 = x3 > a3 ? x3 : a3;
    }
    if (threadIdx.x == 0) {
        s_mm[0] = ~0u;
        s_mm[1] = 0u;
        s_mm[2] = ~0u;
        s_mm[3] = 0u;
    }
    __syncthreads();
    if (lane_id() == 0) {
        atomicMin(&s_mm[0], a0);
        atomicMax(&s_mm[1], a1);
        atomicMin(&s_mm[2], a2);
        atomicMax(&s_mm[3], a3);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mm[4 * d + 0] = s_mm[0];
        mm[4 * d + 1] = s_mm[1];
        mm[4 * d + 2] = s_mm[2];
        mm[4 * d + 3] = s_mm[3];
    }
}

// occupied cell: (x - min) / (max - min) of its channel in double, rounded to
// float (0 when max == min); an empty cell stays 0
__device__ __forceinline__ float rescale(float x, float mn, float mx)
{
    if (!(mx > mn)) return 0.f;
    return (float)(((double)x - (double)mn) / ((double)mx - (double)mn));
}

__global__ void __launch_bounds__(LB) k_lat_norm(float* __restrict__ lat, u32 D, u64 cells, u64 cpi,
                                                  const u32* __restrict__ mm)
{
    const u64 img = blockIdx.x / cpi;
    const u64 c0 = (blockIdx.x % cpi) * CH;
    const u32 d = (u32)(img % D);
    float* sp = lat + (img / D * 2 * D + 2 * d) * cells;
    float* vo = sp + cells;
    const float smn = unord_f32(mm[4 * d + 0]), smx = unord_f32(mm[4 * d + 1]);
    const float vmn = unord_f32(mm[4 * d + 2]), vmx = unord_f32(mm[4 * d + 3]);
#pragma unroll 4
    for (int k = 0; k < CH / LB; ++k) {
        const u64 i = c0 + (u64)k * LB + threadIdx.x;
        if (i < cells) {
            const float v = vo[i];
            if (v > 0.f) {
                sp[i] = rescale(sp[i], smn, smx);
                vo[i] = rescale(v, vmn, vmx);
            }
        }
    }
}

// the channels' min and max as floats (NaN for a channel with no occupied cell)
__global__ void k_lat_mm_out(const u32* __restrict__ mm, float* __restrict__ out, u32 C)
{
    const u32 i = threadIdx.x;
    if (i < 2 * C) {
        const u32 lo = mm[i & ~1u];
        out[i] = lo == ~0u ? __builtin_nanf("") : unord_f32(mm[i]);
    }
}

// filter predicate of group g
__device__ __forceinline__ bool keep(const u32* count, const u32* nj, const double* sum, u64 g, double vmin,
                                     double slo, double shi)
{
    const u32 c = count[g];
    if (c == 0 || (double)nj[g] < vmin) return false;
    const double m = sum[g] / (double)c;
    return m >= slo && m <= shi;
}

__global__ void __launch_bounds__(LB) k_filt_count(const u32* __restrict__ count, const u32* __restrict__ nj,
                                                    const double* __restrict__ sum, u64 G, double vmin, double slo,
                                                    double shi, u32* __restrict__ tcnt)
{
    __shared__ u32 s_w[LB / WAVE];
    const u64 t0 = (u64)blockIdx.x * FT;
    u32 c = 0;
    for (int i = 0; i < FT / LB; ++i) {
        const u64 g = t0 + (u64)i * LB + threadIdx.x;
        c += (u32)__popcll(__ballot(g < G && keep(count, nj, sum, g, vmin, slo, shi)));
    }
    if (lane_id() == 0) s_w[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 t = 0;
        for (int w = 0; w < LB / WAVE; ++w) t += s_w[w];
        tcnt[blockIdx.x] = t;
    }
}

// exclusive prefix of the tile counts (one block); tcnt[tiles] = total
__global__ void __launch_bounds__(1024) k_filt_scan(u32* __restrict__ tcnt, u64 tiles)
{
    __shared__ u32 s_tmp[1024 / WAVE];
    u32 carry = 0;
    for (u64 b = 0; b < tiles; b += 1024) {
        const u64 i = b + threadIdx.x;
        const u32 v = i < tiles ? tcnt[i] : 0u;
        u32 tot;
        const u32 ex = block_exclusive_sum<1024>(v, s_tmp, tot);
        if (i < tiles) tcnt[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) tcnt[tiles] = carry;
}

__global__ void __launch_bounds__(LB) k_filt_write(const u32* __restrict__ count, const u32* __restrict__ nj,
                                                    const double* __restrict__ sum, u64 G, double vmin, double slo,
                                                    double shi, const u32* __restrict__ tpre, u32* __restrict__ index,
                                                    u64 cap)
{
    __shared__ u32 s_w[LB / WAVE];
    __shared__ u32 s_base;
    const u64 t0 = (u64)blockIdx.x * FT;
    const int w = threadIdx.x / WAVE;
    if (threadIdx.x == 0) s_base = tpre[blockIdx.x];
    for (int i = 0; i < FT / LB; ++i) {
        const u64 g = t0 + (u64)i * LB + threadIdx.x;
        const bool k = g < G && keep(count, nj, sum, g, vmin, slo, shi);
        const u64 m = __ballot(k);
        if (lane_id() == 0) s_w[w] = (u32)__popcll(m);
        __syncthreads();
        u32 before = s_base;
        for (int x = 0; x < w; ++x) before += s_w[x];
        const u32 at = before + popc_below(m);
        if (k && at < cap) index[at] = (u32)g;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int x = 0; x < LB / WAVE; ++x) s_base += s_w[x];
        __syncthreads();
    }
}

__global__ void k_filt_result(const u32* __restrict__ tcnt, u64 tiles, u64 cap, cv_result* res)
{
    if (threadIdx.x != 0) return;
    cv_result r = {};
    const u64 total = tcnt[tiles];
    r.status = total > cap ? CV_ERR_CAPACITY : CV_OK;
    r.count = total;
    r.required = total > cap ? total : 0;
    *res = r;
}

bool lattice_dims(const cv_grid_spec* g, uint32_t n_dir, i64& cells, u32& D)
{
    if (!g || g->n_lat <= 0 || g->n_lon <= 0 || g->n_lat > (1ll << 31) || g->n_lon > (1ll << 31) || n_dir > 64)
        return false;
    cells = g->n_lat * g->n_lon;
    D = n_dir ? n_dir + 1 : 1;
    return true;
}

}  // namespace

extern "C" {

cv_status cv_lattice_dense(const cv_groups* groups, uint64_t n_groups, const cv_grid_spec* grid, uint32_t n_dir,
                           int64_t t_first, uint64_t n_t, float* lattice, void* stream)
{
    i64 cells;
    u32 D;
    if (!lattice_dims(grid, n_dir, cells, D) || n_t == 0 || !lattice) return CV_ERR_INVALID_ARGUMENT;
    if ((unsigned __int128)n_t * 2 * D * (u64)cells >= ((unsigned __int128)1 << 62)) return CV_ERR_RANGE;
    if (n_groups && (!groups || !groups->key || !groups->count || !groups->n_journeys || !groups->sum_speed))
        return CV_ERR_INVALID_ARGUMENT;
    if (!cvh::aligned(lattice, 4)) return CV_ERR_INVALID_ARGUMENT;
    hipStream_t s = (hipStream_t)stream;
    cvh::TimedScope ts_("lattice_dense", s);
    const u64 total = n_t * 2 * D * (u64)cells;
    // 16-byte stores from the first 16-byte boundary; the few floats around it singly
    const u64 head = (u64)((16 - ((uintptr_t)lattice & 15)) & 15) / 4;
    const u64 h = head < total ? head : total;
    if (h) hipLaunchKernelGGL(k_lat_fill_tail, dim3(1), dim3(LB), 0, s, lattice, (u64)0, h);
    const u64 n4 = (total - h) / 4;
    if (n4)
        hipLaunchKernelGGL(k_lat_fill, dim3(cvh::grid_for(n4, LB, 8192)), dim3(LB), 0, s,
                           (float4*)(lattice + h), n4);
    const u64 done = h + 4 * n4;
    if (done < total) hipLaunchKernelGGL(k_lat_fill_tail, dim3(1), dim3(LB), 0, s, lattice, done, total);
    if (n_groups)
        hipLaunchKernelGGL(k_lat_scatter, dim3(cvh::grid_for(n_groups, LB, 8192)), dim3(LB), 0, s, groups->key,
                           groups->count, groups->n_journeys, groups->sum_speed, (u64)n_groups, cells, D, t_first,
                           (i64)n_t, lattice);
    return cvh::last_launch_status();
}

cv_status cv_lattice_normalize_workspace_size(uint64_t n_t, const cv_grid_spec* grid, uint32_t n_dir, size_t* bytes)
{
    i64 cells;
    u32 D;
    if (!bytes || !lattice_dims(grid, n_dir, cells, D) || n_t == 0) return CV_ERR_INVALID_ARGUMENT;
    const u64 cpi = ((u64)cells + CH - 1) / CH;
    if ((unsigned __int128)n_t * D * cpi >= ((unsigned __int128)1 << 31)) return CV_ERR_RANGE;
    *bytes = cvh::align_up(n_t * D * cpi * 4 * sizeof(u32));
    return CV_OK;
}

cv_status cv_lattice_normalize(float* lattice, uint64_t n_t, const cv_grid_spec* grid, uint32_t n_dir,
                               float* channel_min_max, void* ws, size_t ws_bytes, void* stream)
{
    i64 cells;
    u32 D;
    if (!lattice_dims(grid, n_dir, cells, D) || n_t == 0 || !lattice || !channel_min_max ||
        !cvh::aligned(channel_min_max, 4))
        return CV_ERR_INVALID_ARGUMENT;
    if ((unsigned __int128)n_t * 2 * D * (u64)cells >= ((unsigned __int128)1 << 62)) return CV_ERR_RANGE;
    size_t need = 0;
    const cv_status e = cv_lattice_normalize_workspace_size(n_t, grid, n_dir, &need);
    if (e != CV_OK) return e;
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need) return CV_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    cvh::TimedScope ts_("lattice_norm", s);
    const u32 C = 2 * D;
    u32* mm = reinterpret_cast<u32*>(channel_min_max);  // ordered images until the last step
    const u64 cpi = ((u64)cells + CH - 1) / CH;          // blocks per image
    const u64 blocks = n_t * D * cpi;
    u32* part = (u32*)ws;
    hipLaunchKernelGGL(k_lat_minmax, dim3((unsigned)blocks), dim3(LB), 0, s, lattice, D, (u64)cells, cpi, part);
    hipLaunchKernelGGL(k_lat_mm_reduce, dim3(D), dim3(LB), 0, s, part, (u64)n_t, D, cpi, mm);
    hipLaunchKernelGGL(k_lat_norm, dim3((unsigned)blocks), dim3(LB), 0, s, lattice, D, (u64)cells, cpi, mm);
    hipLaunchKernelGGL(k_lat_mm_out, dim3(1), dim3(256), 0, s, mm, channel_min_max, C);
    return cvh::last_launch_status();
}

cv_status cv_groups_filter_workspace_size(uint64_t n_groups, size_t* bytes)
{
    if (!bytes || n_groups >= (1ull << 32)) return CV_ERR_INVALID_ARGUMENT;
    *bytes = cvh::align_up(((n_groups + FT - 1) / FT + 1) * sizeof(u32));
    return CV_OK;
}

cv_status cv_groups_filter(const cv_groups* groups, uint64_t n_groups, double min_volume, double speed_lo,
                           double speed_hi, uint32_t* index, uint64_t capacity, cv_result* res, void* ws,
                           size_t ws_bytes, void* stream)
{
    if (n_groups >= (1ull << 32) || !res || std::isnan(min_volume) || std::isnan(speed_lo) || std::isnan(speed_hi))
        return CV_ERR_INVALID_ARGUMENT;
    if (n_groups && (!groups || !groups->count || !groups->n_journeys || !groups->sum_speed))
        return CV_ERR_INVALID_ARGUMENT;
    if (capacity && !index) return CV_ERR_INVALID_ARGUMENT;
    size_t need = 0;
    cv_groups_filter_workspace_size(n_groups, &need);
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need) return CV_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    cvh::TimedScope ts_("groups_filter", s);
    const u64 tiles = (n_groups + FT - 1) / FT;
    u32* tcnt = (u32*)ws;
    if (tiles) {
        hipLaunchKernelGGL(k_filt_count, dim3((unsigned)tiles), dim3(LB), 0, s, groups->count, groups->n_journeys,
                           groups->sum_speed, (u64)n_groups, min_volume, speed_lo, speed_hi, tcnt);
    }
    hipLaunchKernelGGL(k_filt_scan, dim3(1), dim3(1024), 0, s, tcnt, tiles);
    if (tiles) {
        hipLaunchKernelGGL(k_filt_write, dim3((unsigned)tiles), dim3(LB), 0, s, groups->count, groups->n_journeys,
                           groups->sum_speed, (u64)n_groups, min_volume, speed_lo, speed_hi, tcnt, index,
                           (u64)capacity);
    }
    hipLaunchKernelGGL(k_filt_result, dim3(1), dim3(64), 0, s, tcnt, tiles, (u64)capacity, res);
    return cvh::last_launch_status();
}

}  // extern "C"
