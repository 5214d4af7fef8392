// cv_summary.hip -- cv_journey_summary: one row per journey of sorted records.
//
// Journeys are maximal runs of equal journey id.  Tiles of ST records:
//   k_sum_count   journey starts per tile;
//   k_tile_scan   exclusive scan of the tile counts (one block) -> journey index
//                 of each tile's first start, J;
//   k_sum_init    identity values in the accumulator rows of the J journeys;
//   k_sum_reduce  segmented reduction over journey boundaries: every wave walks
//                 its records in coalesced windows of 64, folding them in exact
//                 fixed point; a journey that starts and ends inside one wave's
//                 records is written out directly, the pieces of one that
//                 crosses a wave edge meet in its accumulator row through
//                 integer atomics (order-independent, hence deterministic);
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

__global__ void __launch_bounds__(SB) k_sum_count(const i64* __restrict__ jid, u32 n, u32* __restrict__ tile_cnt,
                                                  const u64* __restrict__ soff, u32 S)
{
    __shared__ u32 tmp[SB / WAVE];
    const u64 base = (u64)blockIdx.x * ST;
    u32 c = 0;
    for (int i = threadIdx.x; i < ST; i += SB) {
        u64 r = base + i;
        if (r < n && (is_head(jid, r) || (S > 1 && shard_start(soff, S, r)))) ++c;
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

// Partial aggregate of one journey (a lane's records, a wave's, or a tile's).
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

__device__ __forceinline__ void part_combine(Part& a, const Part& b)
{
    fx_add(a.dist, b.dist);
    fx_add(a.spd, b.spd);
    a.maxd = b.maxd > a.maxd ? b.maxd : a.maxd;
    a.latmin = b.latmin < a.latmin ? b.latmin : a.latmin;
    a.latmax = b.latmax > a.latmax ? b.latmax : a.latmax;
    a.lonmin = b.lonmin < a.lonmin ? b.lonmin : a.lonmin;
    a.lonmax = b.lonmax > a.lonmax ? b.lonmax : a.lonmax;
    a.count += b.count;
    a.ndtz += b.ndtz;
    a.maxs = b.maxs > a.maxs ? b.maxs : a.maxs;
}

template <typename F>
__device__ __forceinline__ void part_shuffle(Part& o, const Part& p, F&& sh)
{
    for (int i = 0; i < 3; ++i) {
        o.dist.w[i] = sh(p.dist.w[i]);
        o.spd.w[i] = sh(p.spd.w[i]);
    }
    o.maxd = sh(p.maxd);
    o.latmin = sh(p.latmin);
    o.latmax = sh(p.latmax);
    o.lonmin = sh(p.lonmin);
    o.lonmax = sh(p.lonmax);
    o.count = (u32)sh((u64)p.count);
    o.ndtz = (u32)sh((u64)p.ndtz);
    o.maxs = (u32)sh((u64)p.maxs);
}

// full wave reduction; every lane ends with the total
__device__ __forceinline__ void part_wave_reduce(Part& p)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        Part o;
        part_shuffle(o, p, [&](u64 v) { return (u64)__shfl_xor((unsigned long long)v, d, WAVE); });
        part_combine(p, o);
    }
}

// segmented inclusive scan across lanes; `head` starts a segment
__device__ __forceinline__ void part_seg_scan(Part& p, bool head)
{
    const int l = lane_id();
    bool f = head;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        Part o;
        part_shuffle(o, p, [&](u64 v) { return (u64)__shfl_up((unsigned long long)v, d, WAVE); });
        bool fo = __shfl_up(f, d, WAVE);
        if (l >= d) {
            if (!f) {
                part_combine(o, p);
                p = o;
            }
            f = f || fo;
        }
    }
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

__device__ __forceinline__ void flush_part(const Out& o, JAcc* acc, u32 cap, u32 j, const Part& p, bool whole)
{
    if (j >= cap || p.count == 0) return;
    if (whole) {
        write_final(o, j, p.count, p.ndtz, p.dist, p.spd, p.maxs, p.maxd, p.latmin, p.latmax, p.lonmin, p.lonmax);
        return;
    }
    JAcc& a = acc[j];
    atomic_add_fx(a.dist, p.dist);
    atomic_add_fx(a.spd, p.spd);
    atomicMax((unsigned long long*)&a.maxd, (unsigned long long)p.maxd);
    atomicMin((unsigned long long*)&a.latmin, (unsigned long long)p.latmin);
    atomicMax((unsigned long long*)&a.latmax, (unsigned long long)p.latmax);
    atomicMin((unsigned long long*)&a.lonmin, (unsigned long long)p.lonmin);
    atomicMax((unsigned long long*)&a.lonmax, (unsigned long long)p.lonmax);
    atomicAdd(&a.count, p.count);
    atomicAdd(&a.ndtz, p.ndtz);
    atomicMax(&a.maxs, p.maxs);
    atomicOr(&a.touched, 1u);
}

// Each wave owns WCH consecutive records and walks them in coalesced windows of
// 64.  Lanes fold their records into a private partial while the window holds
// no journey start; a window with starts closes the open journey (wave
// reduction), runs a segmented scan for journeys that begin in it, and hands
// the last one on as the new open journey.  A journey that begins and ends in
// the wave's records is written out directly; otherwise its pieces meet in the
// accumulator row through integer atomics.
constexpr int WI = SI;                  // windows per wave
constexpr int WCH = WAVE * WI;          // records per wave
static_assert(ST == (SB / WAVE) * WCH, "tile = waves x wave chunk");

__global__ void __launch_bounds__(SB) k_sum_reduce(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                   const double* __restrict__ lat, const double* __restrict__ lon,
                                                   const float* __restrict__ spd, const double* __restrict__ step,
                                                   const double* __restrict__ dspd, const uint8_t* __restrict__ flags,
                                                   const u32* __restrict__ tile_prefix, u32 cap, Out o,
                                                   JAcc* __restrict__ acc, const u64* __restrict__ soff, u32 S,
                                                   u64* __restrict__ jo)
{
    __shared__ u32 s_wh[SB / WAVE];
    const int w = threadIdx.x / WAVE;
    const int l = lane_id();
    const u64 cs = (u64)blockIdx.x * ST + (u64)w * WCH;  // wave chunk start
    const u64 ce = cs + WCH < n ? cs + WCH : (u64)n;      // wave chunk end (may be <= cs)

    // heads in this wave's chunk -> journey index of the wave's first head
    u32 hc = 0;
    for (int i = 0; i < WI; ++i) {
        u64 r = cs + (u64)i * WAVE + l;
        if (r < ce && (r == 0 || jid[r] != jid[r - 1] || (S > 1 && shard_start(soff, S, r)))) ++hc;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) hc += __shfl_xor(hc, d, WAVE);
    if (l == 0) s_wh[w] = hc;
    __syncthreads();
    u32 seen = tile_prefix[blockIdx.x];  // heads before the current position
    for (int k = 0; k < w; ++k) seen += s_wh[k];
    if (cs >= ce) return;

    Part p;
    part_reset(p);
    // open journey: the one containing the record before the next window
    u32 open_j = seen - 1;   // valid when the chunk starts mid-journey
    bool open_here = false;  // its first record lies in this chunk
    // window loads are issued one window ahead of their use
    struct Win {
        i64 j, jp, jn, t;
        double st, ds, la, lo;
        float sp;
        uint8_t f;
    };
    auto load = [&](int i, Win& x) {
        const u64 r = cs + (u64)i * WAVE + l;
        if (r < ce) {
            x.j = jid[r];
            x.jp = r > 0 ? jid[r - 1] : ~x.j;
            x.jn = r + 1 < n ? jid[r + 1] : ~x.j;
            if (S > 1) {
                // a shard start is a journey start even when the id continues
                if (shard_start(soff, S, r)) x.jp = ~x.j;
                if (r + 1 < n && shard_start(soff, S, r + 1)) x.jn = ~x.j;
            }
            x.t = ts[r];
            x.st = step[r];
            x.sp = spd[r];
            x.f = flags[r];
            x.ds = dspd[r];
            x.la = lat[r];
            x.lo = lon[r];
        }
    };
    Win cur, nxt;
    load(0, cur);
    for (int i = 0; i < WI; ++i) {
        if (i + 1 < WI) load(i + 1, nxt);
        const u64 r = cs + (u64)i * WAVE + l;
        const bool valid = r < ce;
        bool h = false, last = false;
        Part c;
        part_reset(c);
        if (valid) {
            h = (r == 0) || (cur.j != cur.jp);
            last = (r + 1 >= n) || (cur.jn != cur.j);
            c.count = 1;
            c.ndtz = (cur.f & CV_FLAG_DT_ZERO) ? 1u : 0u;
            c.dist = fx_from_double<FX_DIST>(cur.st);
            c.spd = fx_from_double<FX_SPD>((double)cur.sp);
            c.maxs = ord_f32(cur.sp);
            if (cur.f & CV_FLAG_SPEED_OK) c.maxd = ord_f64(cur.ds);
            if (isfinite(cur.la) && isfinite(cur.lo)) {
                c.latmin = c.latmax = ord_f64(cur.la);
                c.lonmin = c.lonmax = ord_f64(cur.lo);
            }
        }
        const u64 H = __ballot(h);
        // journey index of this lane's record
        const u32 jl = seen + popc_below(H) + (h ? 1u : 0u) - 1u;
        if (h && jl < cap) {
            o.jid[jl] = cur.j;
            o.first[jl] = (u32)r;
            o.tstart[jl] = cur.t;
        }
        if (h && S > 1 && jo) {
            // this record opens its shard's first journey: every shard starting
            // here (empty ones included) begins at journey jl
            const u32 sh = shard_of(soff, S, r);
            if (soff[sh] == r)
                for (int z = (int)sh; z >= 0 && soff[z] == r; --z) jo[z] = jl;
        }
        if (valid && last && jl < cap) o.tend[jl] = cur.t;
        if (H != 0) {
            const int f0 = __ffsll((long long)H) - 1;
            if (l < f0) part_combine(p, c);
            // close the journey that was open before the first start in this window
            part_wave_reduce(p);
            if (l == 0) flush_part(o, acc, cap, open_j, p, open_here);
            // journeys starting in this window
            Part s = c;
            part_seg_scan(s, h);
            // a segment that ends before lane 63 (next lane starts a journey) is a
            // whole journey: it began and ended inside this window
            const bool next_head = (l < WAVE - 1) && ((H >> (l + 1)) & 1ull);
            if (l >= f0 && next_head) flush_part(o, acc, cap, jl, s, true);
            // the last segment stays open; lane 63 holds its partial
            part_reset(p);
            if (l == WAVE - 1) p = s;
            seen += (u32)__popcll(H);
            open_j = seen - 1;
            open_here = true;
        } else {
            part_combine(p, c);
        }
        cur = nxt;
    }
    part_wave_reduce(p);
    if (l == 0) {
        const bool ends = (ce >= n) || (jid[ce] != jid[ce - 1]) || (S > 1 && shard_start(soff, S, ce));
        flush_part(o, acc, cap, open_j, p, open_here && ends);
    }
}

__global__ void __launch_bounds__(256) k_sum_finalize(const JAcc* __restrict__ acc, const SumMeta* meta, u32 cap,
                                                      Out o, cv_result* res, const u64* __restrict__ soff, u32 S,
                                                      u64* __restrict__ jo, u32 n)
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
    if (jo && blockIdx.x == 0 && threadIdx.x == 0) {
        // shards that start at the end of the records hold no journey
        jo[S] = J;
        for (int z = (int)S - 1; z >= 0 && soff[z] >= n; --z) jo[z] = J;
        if (S == 1) jo[0] = 0;
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

static cv_status summary_impl(const cv_records* sorted, const cv_features* feat, const u64* soff, u32 S,
                              const cv_journeys* out, uint64_t capacity, u64* jo, cv_result* res, void* ws,
                              size_t ws_bytes, void* stream)
{
    if (!sorted || !feat || !out || sorted->n >= (1ull << 32) || capacity >= (1ull << 32))
        return CV_ERR_INVALID_ARGUMENT;
    const u64 n = sorted->n;
    hipStream_t s = (hipStream_t)stream;
    SumLayout need(nullptr, n, capacity);
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need.bytes) return CV_ERR_WORKSPACE;
    if (n == 0) {
        if (res) hipLaunchKernelGGL(k_sum_empty, dim3(1), dim3(64), 0, s, res);
        if (jo) cvh::fill_u64(jo, 0, (u64)S + 1, s);
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
    hipLaunchKernelGGL(k_sum_count, dim3((unsigned)L.tiles), dim3(SB), 0, s, sorted->journey_id, nn, L.tile_cnt, soff, S);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(256), 0, s, L.tile_cnt, (u32)L.tiles, L.meta);
    hipLaunchKernelGGL(k_sum_init, dim3(cvh::grid_for(cap, 256, 2048)), dim3(256), 0, s, L.acc, L.meta, cap);
    hipLaunchKernelGGL(k_sum_reduce, dim3((unsigned)L.tiles), dim3(SB), 0, s, nn, sorted->journey_id, sorted->ts_ms,
                       sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, feat->step_m, feat->speed_mps, feat->flags,
                       L.tile_cnt, cap, o, L.acc, soff, S, jo);
    hipLaunchKernelGGL(k_sum_finalize, dim3(cvh::grid_for(cap, 256, 2048)), dim3(256), 0, s, L.acc, L.meta, cap, o,
                       res, soff, S, jo, nn);
    return cvh::last_launch_status();
}


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
    return summary_impl(sorted, feat, nullptr, 0, out, capacity, nullptr, res, ws, ws_bytes, stream);
}

cv_status cv_batch_journey_summary(const cv_records* sorted, const cv_features* feat, const uint64_t* shard_offsets,
                                   uint32_t n_shards, const cv_journeys* out, uint64_t capacity,
                                   uint64_t* journey_offsets, cv_result* res, void* ws, size_t ws_bytes, void* stream)
{
    if (n_shards == 0 || !shard_offsets || !journey_offsets || !cvh::aligned(shard_offsets, 8) ||
        !cvh::aligned(journey_offsets, 8))
        return CV_ERR_INVALID_ARGUMENT;
    return summary_impl(sorted, feat, shard_offsets, n_shards, out, capacity, journey_offsets, res, ws, ws_bytes,
                        stream);
}

}  // extern "C"
