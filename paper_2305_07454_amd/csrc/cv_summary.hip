// cv_summary.hip -- cv_journey_summary: one row per journey of sorted records.
//
// Journeys are maximal runs of equal journey id.  Tiles of ST records:
//   k_sum_count   heads per tile;
//   k_tile_scan   exclusive scan of the tile counts (one block) -> journey index
//                 of each tile's first head, J;
//   k_sum_init    identity values in the accumulator rows of the J journeys;
//   k_sum_reduce  each thread folds its SI consecutive records sequentially in
//                 exact fixed point; partials that span threads merge in LDS
//                 slots owned by the thread holding the journey's head; a
//                 journey fully inside the tile is written out directly, one
//                 that crosses a tile edge is added with integer atomics into
//                 its accumulator row (order-independent, hence deterministic);
//   k_sum_finalize accumulator rows -> output rows (exact sums rounded once).
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_host.h"

using namespace cv;

namespace {

constexpr int SB = 256;
constexpr int SI = 16;
constexpr int ST = SB * SI;
constexpr int FX_DIST = 128;  // distance: 2^-128 m resolution (exact for steps >= 2^-75 m)
constexpr int FX_SPD = 149;   // speed: exact for every float32

struct JAcc {
    u64 dist[3];
    u64 spd[3];
    u64 maxd;
    u64 latmin, latmax, lonmin, lonmax;
    u32 count, ndtz, maxs, touched;
};

struct SumMeta {
    u32 J;
};

__device__ __forceinline__ bool is_head(const i64* jid, u64 r) { return r == 0 || jid[r] != jid[r - 1]; }

__global__ void __launch_bounds__(SB) k_sum_count(const i64* __restrict__ jid, u32 n, u32* __restrict__ tile_cnt)
{
    __shared__ u32 tmp[SB / WAVE];
    const u64 base = (u64)blockIdx.x * ST;
    u32 c = 0;
    for (int i = threadIdx.x; i < ST; i += SB) {
        u64 r = base + i;
        if (r < n && is_head(jid, r)) ++c;
    }
    u32 total;
    block_exclusive_sum<SB>(c, tmp, total);
    if (threadIdx.x == 0) tile_cnt[blockIdx.x] = total;
}

// single block: exclusive scan of `tiles` counts in place; meta->J = total
__global__ void __launch_bounds__(256) k_tile_scan(u32* __restrict__ cnt, u32 tiles, SumMeta* meta)
{
    __shared__ u32 tmp[256 / WAVE];
    __shared__ u32 carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (u32 b = 0; b < tiles; b += 256) {
        u32 i = b + threadIdx.x;
        u32 v = i < tiles ? cnt[i] : 0u;
        u32 total;
        u32 e = block_exclusive_sum<256>(v, tmp, total);
        if (i < tiles) cnt[i] = carry + e;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) meta->J = carry;
}

__device__ __forceinline__ void jacc_identity(JAcc& a)
{
    a.dist[0] = a.dist[1] = a.dist[2] = 0;
    a.spd[0] = a.spd[1] = a.spd[2] = 0;
    a.maxd = ord_f64(0.0);
    a.latmin = ord_f64(__builtin_inf());
    a.latmax = ord_f64(-__builtin_inf());
    a.lonmin = ord_f64(__builtin_inf());
    a.lonmax = ord_f64(-__builtin_inf());
    a.count = 0;
    a.ndtz = 0;
    a.maxs = 0;
    a.touched = 0;
}

__global__ void __launch_bounds__(256) k_sum_init(JAcc* __restrict__ acc, const SumMeta* meta, u32 cap)
{
    u32 J = meta->J;
    u32 m = J < cap ? J : cap;
    for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        JAcc a;
        jacc_identity(a);
        acc[j] = a;
    }
}

// running partial of one journey inside one thread's chunk
struct Part {
    Fx192 dist, spd;
    u64 maxd, latmin, latmax, lonmin, lonmax;
    u32 count, ndtz, maxs;
};

__device__ __forceinline__ void part_reset(Part& p)
{
    fx_zero(p.dist);
    fx_zero(p.spd);
    p.maxd = ord_f64(0.0);
    p.latmin = ord_f64(__builtin_inf());
    p.latmax = ord_f64(-__builtin_inf());
    p.lonmin = ord_f64(__builtin_inf());
    p.lonmax = ord_f64(-__builtin_inf());
    p.count = 0;
    p.ndtz = 0;
    p.maxs = 0;
}

// LDS slot: carry-save sums so that merges are plain 64-bit adds
struct Slot {
    u64 dist[4];
    u64 spd[4];
    u64 maxd, latmin, latmax, lonmin, lonmax;
    u32 count, ndtz, maxs, pad;
};

__device__ __forceinline__ void slot_store(Slot& s, const Part& p)
{
    fx_to_cs(p.dist, s.dist);
    fx_to_cs(p.spd, s.spd);
    s.maxd = p.maxd;
    s.latmin = p.latmin;
    s.latmax = p.latmax;
    s.lonmin = p.lonmin;
    s.lonmax = p.lonmax;
    s.count = p.count;
    s.ndtz = p.ndtz;
    s.maxs = p.maxs;
}

__device__ __forceinline__ void slot_merge(Slot& s, const Part& p)
{
    u64 c[4];
    fx_to_cs(p.dist, c);
    for (int i = 0; i < 4; ++i)
        if (c[i]) atomicAdd((unsigned long long*)&s.dist[i], (unsigned long long)c[i]);
    fx_to_cs(p.spd, c);
    for (int i = 0; i < 4; ++i)
        if (c[i]) atomicAdd((unsigned long long*)&s.spd[i], (unsigned long long)c[i]);
    atomicMax((unsigned long long*)&s.maxd, (unsigned long long)p.maxd);
    atomicMin((unsigned long long*)&s.latmin, (unsigned long long)p.latmin);
    atomicMax((unsigned long long*)&s.latmax, (unsigned long long)p.latmax);
    atomicMin((unsigned long long*)&s.lonmin, (unsigned long long)p.lonmin);
    atomicMax((unsigned long long*)&s.lonmax, (unsigned long long)p.lonmax);
    atomicAdd(&s.count, p.count);
    atomicAdd(&s.ndtz, p.ndtz);
    atomicMax(&s.maxs, p.maxs);
}

struct Out {
    int64_t* jid;
    uint32_t* first;
    uint32_t* npts;
    int64_t* tstart;
    int64_t* tend;
    double* dist;
    double* sumspd;
    float* maxspd;
    double* maxdspd;
    uint32_t* ndtz;
    double *latmin, *latmax, *lonmin, *lonmax;
};

__device__ __forceinline__ void write_final(const Out& o, u32 j, u32 count, u32 ndtz, const Fx192& dist,
                                            const Fx192& spd, u32 maxs, u64 maxd, u64 la0, u64 la1, u64 lo0, u64 lo1)
{
    o.npts[j] = count;
    o.ndtz[j] = ndtz;
    o.dist[j] = fx_to_double<FX_DIST>(dist);
    o.sumspd[j] = fx_to_double<FX_SPD>(spd);
    o.maxspd[j] = unord_f32(maxs);
    o.maxdspd[j] = unord_f64(maxd);
    o.latmin[j] = unord_f64(la0);
    o.latmax[j] = unord_f64(la1);
    o.lonmin[j] = unord_f64(lo0);
    o.lonmax[j] = unord_f64(lo1);
}

__device__ __forceinline__ void part_final(const Out& o, u32 j, const Part& p)
{
    write_final(o, j, p.count, p.ndtz, p.dist, p.spd, p.maxs, p.maxd, p.latmin, p.latmax, p.lonmin, p.lonmax);
}

__device__ __forceinline__ void acc_merge_global(JAcc& a, u32 count, u32 ndtz, const Fx192& dist, const Fx192& spd,
                                                 u32 maxs, u64 maxd, u64 la0, u64 la1, u64 lo0, u64 lo1)
{
    atomic_add_fx(a.dist, dist);
    atomic_add_fx(a.spd, spd);
    atomicMax((unsigned long long*)&a.maxd, (unsigned long long)maxd);
    atomicMin((unsigned long long*)&a.latmin, (unsigned long long)la0);
    atomicMax((unsigned long long*)&a.latmax, (unsigned long long)la1);
    atomicMin((unsigned long long*)&a.lonmin, (unsigned long long)lo0);
    atomicMax((unsigned long long*)&a.lonmax, (unsigned long long)lo1);
    atomicAdd(&a.count, count);
    atomicAdd(&a.ndtz, ndtz);
    atomicMax(&a.maxs, maxs);
    atomicOr(&a.touched, 1u);
}

__global__ void __launch_bounds__(SB) k_sum_reduce(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                   const double* __restrict__ lat, const double* __restrict__ lon,
                                                   const float* __restrict__ spd, const double* __restrict__ step,
                                                   const double* __restrict__ dspd, const uint8_t* __restrict__ flags,
                                                   const u32* __restrict__ tile_prefix, u32 cap, Out o,
                                                   JAcc* __restrict__ acc)
{
    __shared__ Slot s_slot[SB + 1];  // s_slot[SB] is the journey continuing from the previous tile
    __shared__ u32 s_tmp[SB / WAVE];
    __shared__ int s_tmpi[SB / WAVE];
    __shared__ u32 s_hashead[SB];

    const int t = threadIdx.x;
    const u64 tile0 = (u64)blockIdx.x * ST;
    const u64 r0 = tile0 + (u64)t * SI;
    const u64 r1 = (r0 + SI < n) ? r0 + SI : (r0 < n ? (u64)n : r0);
    const u64 tile_end = (tile0 + ST < n) ? tile0 + ST : (u64)n;

    // heads in this thread's chunk
    u32 heads = 0;
    bool head0 = false;
    for (u64 r = r0; r < r1; ++r) {
        bool h = is_head(jid, r);
        heads += h;
        if (r == r0) head0 = h;
    }
    u32 tot;
    const u32 before = block_exclusive_sum<SB>(heads, s_tmp, tot);
    s_hashead[t] = heads ? 1u : 0u;
    // owner of the journey entering this chunk: last earlier thread with a head
    int mark = heads ? t : -1;
    {
        int w = t / WAVE;
        int inc = wave_inclusive_max(mark);
        if (lane_id() == WAVE - 1) s_tmpi[w] = inc;
        __syncthreads();
        int pre = -1;
        for (int i = 0; i < w; ++i) pre = s_tmpi[i] > pre ? s_tmpi[i] : pre;
        int incl = inc > pre ? inc : pre;
        // exclusive: drop this thread's own mark
        int excl_val = __shfl_up(incl, 1, WAVE);
        if (lane_id() == 0) excl_val = pre;
        mark = excl_val;  // owner for this thread's entering partial
    }
    const int owner = mark;
    // is there a thread after t in this tile holding a head?
    // (computed after the slot phase from s_hashead)

    const u32 tpre = tile_prefix[blockIdx.x];
    // journey index of record r0
    u32 j = tpre + before + (head0 ? 1u : 0u);
    j -= 1;  // index of the journey containing r0 (valid when r0 < n)

    if (t == 0) {
        Part z;
        part_reset(z);
        slot_store(s_slot[SB], z);
    }

    Part p;
    part_reset(p);
    bool p_from_head = head0;  // current partial started at a head inside this chunk
    bool entering_done = head0;  // the entering (pre) partial is empty when r0 is a head
    Part pre_part;
    part_reset(pre_part);
    bool have_pre = false;
    for (u64 r = r0; r < r1; ++r) {
        bool h = is_head(jid, r);
        if (h && r != r0) {
            // close current partial
            if (p_from_head) {
                if (j < cap) part_final(o, j, p);  // complete journey inside the chunk
            } else {
                pre_part = p;
                have_pre = true;
                entering_done = true;
            }
            ++j;
            part_reset(p);
            p_from_head = true;
        }
        if (h) {
            if (j < cap) {
                o.jid[j] = jid[r];
                o.first[j] = (u32)r;
                o.tstart[j] = ts[r];
            }
        }
        // last record of its journey?
        if (r + 1 >= n || jid[r + 1] != jid[r]) {
            if (j < cap) o.tend[j] = ts[r];
        }
        uint8_t f = flags[r];
        p.count += 1;
        p.ndtz += (f & CV_FLAG_DT_ZERO) ? 1u : 0u;
        Fx192 a = fx_from_double<FX_DIST>(step[r]);
        fx_add(p.dist, a);
        a = fx_from_double<FX_SPD>((double)spd[r]);
        fx_add(p.spd, a);
        u32 ms = ord_f32(spd[r]);
        p.maxs = ms > p.maxs ? ms : p.maxs;
        if (f & CV_FLAG_SPEED_OK) {
            u64 d = ord_f64(dspd[r]);
            p.maxd = d > p.maxd ? d : p.maxd;
        }
        double la = lat[r], lo = lon[r];
        if (isfinite(la) && isfinite(lo)) {
            u64 a0 = ord_f64(la), b0 = ord_f64(lo);
            p.latmin = a0 < p.latmin ? a0 : p.latmin;
            p.latmax = a0 > p.latmax ? a0 : p.latmax;
            p.lonmin = b0 < p.lonmin ? b0 : p.lonmin;
            p.lonmax = b0 > p.lonmax ? b0 : p.lonmax;
        }
    }
    // at chunk end: p is the suffix partial (from the last head) or, when the chunk
    // had no head, the whole chunk (an entering partial)
    if (!entering_done && r0 < r1) {
        pre_part = p;
        have_pre = true;
    }
    // phase 1: threads with a head own slot[t] = suffix partial
    if (heads) slot_store(s_slot[t], p);
    __syncthreads();
    // phase 2: entering partials merge into their owner's slot
    if (have_pre) slot_merge(s_slot[owner >= 0 ? owner : SB], pre_part);
    __syncthreads();
    // phase 3: flush slots
    const bool next_is_head = tile_end >= n || is_head(jid, tile_end);
    if (heads && r0 < r1) {
        // journey index of this thread's last head
        u32 jl = tpre + before + heads - 1;
        bool later = false;
        for (int u = t + 1; u < SB; ++u)
            if (s_hashead[u]) {
                later = true;
                break;
            }
        const Slot& s = s_slot[t];
        Fx192 dist = fx_from_cs(s.dist), sp = fx_from_cs(s.spd);
        if (later || next_is_head) {
            if (jl < cap) write_final(o, jl, s.count, s.ndtz, dist, sp, s.maxs, s.maxd, s.latmin, s.latmax, s.lonmin, s.lonmax);
        } else if (jl < cap) {
            acc_merge_global(acc[jl], s.count, s.ndtz, dist, sp, s.maxs, s.maxd, s.latmin, s.latmax, s.lonmin, s.lonmax);
        }
    }
    if (t == 0 && tpre > 0) {
        const Slot& s = s_slot[SB];
        if (s.count > 0) {
            u32 jp = tpre - 1;
            if (jp < cap) {
                Fx192 dist = fx_from_cs(s.dist), sp = fx_from_cs(s.spd);
                acc_merge_global(acc[jp], s.count, s.ndtz, dist, sp, s.maxs, s.maxd, s.latmin, s.latmax, s.lonmin,
                                 s.lonmax);
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_sum_finalize(const JAcc* __restrict__ acc, const SumMeta* meta, u32 cap,
                                                      Out o, cv_result* res)
{
    u32 J = meta->J;
    u32 m = J < cap ? J : cap;
    for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        const JAcc& a = acc[j];
        if (!a.touched) continue;
        Fx192 d, s;
        d.w[0] = a.dist[0];
        d.w[1] = a.dist[1];
        d.w[2] = a.dist[2];
        s.w[0] = a.spd[0];
        s.w[1] = a.spd[1];
        s.w[2] = a.spd[2];
        write_final(o, j, a.count, a.ndtz, d, s, a.maxs, a.maxd, a.latmin, a.latmax, a.lonmin, a.lonmax);
    }
    if (res && blockIdx.x == 0 && threadIdx.x == 0) {
        cv_result r = {};
        r.status = J > cap ? CV_ERR_CAPACITY : CV_OK;
        r.count = J;
        r.required = J > cap ? J : 0;
        *res = r;
    }
}

__global__ void k_sum_empty(cv_result* res)
{
    if (threadIdx.x == 0) {
        cv_result r = {};
        *res = r;
    }
}

struct SumLayout {
    SumMeta* meta;
    u32* tile_cnt;
    JAcc* acc;
    u64 tiles;
    size_t bytes;
    SumLayout(void* ws, u64 n, u64 cap)
    {
        cvh::Carver c(ws);
        tiles = (n + ST - 1) / ST;
        meta = c.take<SumMeta>(1);
        tile_cnt = c.take<u32>(tiles + 1);
        acc = c.take<JAcc>(cap < n ? cap : n);
        bytes = c.size();
    }
};

}  // namespace

extern "C" {

cv_status cv_summary_workspace_size(uint64_t n, uint64_t capacity, size_t* bytes)
{
    if (!bytes || n >= (1ull << 32)) return CV_ERR_INVALID_ARGUMENT;
    SumLayout L(nullptr, n, capacity);
    *bytes = L.bytes;
    return CV_OK;
}

cv_status cv_journey_summary(const cv_records* sorted, const cv_features* feat, const cv_journeys* out,
                             uint64_t capacity, cv_result* res, void* ws, size_t ws_bytes, void* stream)
{
    if (!sorted || !feat || !out || sorted->n >= (1ull << 32) || capacity >= (1ull << 32))
        return CV_ERR_INVALID_ARGUMENT;
    const u64 n = sorted->n;
    hipStream_t s = (hipStream_t)stream;
    SumLayout need(nullptr, n, capacity);
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need.bytes) return CV_ERR_WORKSPACE;
    if (n == 0) {
        if (res) hipLaunchKernelGGL(k_sum_empty, dim3(1), dim3(64), 0, s, res);
        return cvh::last_launch_status();
    }
    if (!sorted->journey_id || !sorted->ts_ms || !sorted->lat_deg || !sorted->lon_deg || !sorted->speed_mps ||
        !feat->step_m || !feat->speed_mps || !feat->flags)
        return CV_ERR_INVALID_ARGUMENT;
    if (capacity > 0 && (!out->journey_id || !out->first || !out->n_points || !out->t_start_ms || !out->t_end_ms ||
                         !out->distance_m || !out->sum_speed || !out->max_speed || !out->max_derived_speed ||
                         !out->n_dt_zero || !out->lat_min || !out->lat_max || !out->lon_min || !out->lon_max))
        return CV_ERR_INVALID_ARGUMENT;
    SumLayout L(ws, n, capacity);
    Out o{out->journey_id, out->first, out->n_points, out->t_start_ms, out->t_end_ms, out->distance_m,
          out->sum_speed, out->max_speed, out->max_derived_speed, out->n_dt_zero, out->lat_min, out->lat_max,
          out->lon_min, out->lon_max};
    const u32 cap = (u32)(capacity < n ? capacity : n);
    const u32 nn = (u32)n;
    cvh::TimedScope ts_("summary", s);
    hipLaunchKernelGGL(k_sum_count, dim3((unsigned)L.tiles), dim3(SB), 0, s, sorted->journey_id, nn, L.tile_cnt);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(256), 0, s, L.tile_cnt, (u32)L.tiles, L.meta);
    hipLaunchKernelGGL(k_sum_init, dim3(cvh::grid_for(cap, 256, 2048)), dim3(256), 0, s, L.acc, L.meta, cap);
    hipLaunchKernelGGL(k_sum_reduce, dim3((unsigned)L.tiles), dim3(SB), 0, s, nn, sorted->journey_id, sorted->ts_ms,
                       sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, feat->step_m, feat->speed_mps, feat->flags,
                       L.tile_cnt, cap, o, L.acc);
    hipLaunchKernelGGL(k_sum_finalize, dim3(cvh::grid_for(cap, 256, 2048)), dim3(256), 0, s, L.acc, L.meta, cap, o,
                       res);
    return cvh::last_launch_status();
}

}  // extern "C"
