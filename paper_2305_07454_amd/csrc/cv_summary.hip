// cv_summary.hip -- cv_journey_summary: one row per journey of sorted records.
//
// Journeys are maximal runs of equal journey id.  Tiles of ST records:
//   k_sum_count   journey starts per wave chunk (a tile holds NW chunks);
//   k_tile_scan   exclusive scan of the tile totals (one block) -> journey index
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

constexpr int NW = SB / WAVE;  // waves per block
constexpr int WI = SI;         // windows of 64 records per wave
constexpr int WCH = WAVE * WI; // records per wave
static_assert(ST == NW * WCH, "tile = waves x wave chunk");

// Journey starts among the records of window [a, a + 64) of a wave that walks
// consecutive windows: jprev is the id before the window (carried), sk the
// shard cursor.  Returns the lane mask of starts; jv is this lane's id.
__device__ __forceinline__ u64 window_heads(const i64* __restrict__ jid, u64 a, u64 end, i64& jprev, i64& jv,
                                            const u64* __restrict__ soff, u32 S, u32& sk, u64& smask, bool& s_end)
{
    const int l = lane_id();
    const u64 r = a + l;
    const bool valid = r < end;
    jv = valid ? jid[r] : 0;
    i64 jp = __shfl_up(jv, 1, WAVE);
    if (l == 0) jp = jprev;
    jprev = __shfl(jv, WAVE - 1, WAVE);
    smask = 0;
    s_end = false;
    if (S > 1) smask = shard_starts_in(soff, S, sk, a, s_end);
    return __ballot(valid && (r == 0 || jv != jp || ((smask >> l) & 1ull)));
}

// journey starts per wave chunk of WCH records: wcnt[tile * NW + wave]
__global__ void __launch_bounds__(SB) k_sum_count(const i64* __restrict__ jid, u32 n, u32* __restrict__ wcnt,
                                                  const u64* __restrict__ soff, u32 S)
{
    const int w = threadIdx.x / WAVE;
    const u64 cs = (u64)blockIdx.x * ST + (u64)w * WCH;
    const u64 ce = cs + WCH < n ? cs + WCH : (u64)n;
    u32 c = 0;
    if (cs < ce) {
        i64 jprev = cs > 0 ? jid[cs - 1] : 0;
        u32 sk = S > 1 ? shard_lower_bound(soff, S, cs) : 0u;
        for (u64 a = cs; a < ce; a += WAVE) {
            i64 jv;
            u64 sm;
            bool se;
            c += (u32)__popcll(window_heads(jid, a, ce, jprev, jv, soff, S, sk, sm, se));
        }
    }
    if (lane_id() == 0) wcnt[(u64)blockIdx.x * NW + w] = c;
}

// single block: tile_prefix[i] = journey starts before tile i; meta->J = total
__global__ void __launch_bounds__(256) k_tile_scan(const u32* __restrict__ wcnt, u32* __restrict__ tile_prefix,
                                                   u32 tiles, SumMeta* meta)
{
    __shared__ u32 tmp[256 / WAVE];
    __shared__ u32 carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (u32 b = 0; b < tiles; b += 256) {
        u32 i = b + threadIdx.x;
        u32 v = 0;
        if (i < tiles)
            for (int k = 0; k < NW; ++k) v += wcnt[(u64)i * NW + k];
        u32 total;
        u32 e = block_exclusive_sum<256>(v, tmp, total);
        if (i < tiles) tile_prefix[i] = carry + e;
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

// Cross-lane steps work one field at a time, so that only that field's
// shuffled copy is live next to the partial.
__device__ __forceinline__ u64 shfl_xor64(u64 v, int d) { return (u64)__shfl_xor((unsigned long long)v, d, WAVE); }
__device__ __forceinline__ u64 shfl_up64(u64 v, int d) { return (u64)__shfl_up((unsigned long long)v, d, WAVE); }

// full wave reduction; every lane ends with the total
__device__ __forceinline__ void part_wave_reduce(Part& p)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        Fx192 o;
        for (int i = 0; i < 3; ++i) o.w[i] = shfl_xor64(p.dist.w[i], d);
        fx_add(p.dist, o);
    }
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        Fx192 o;
        for (int i = 0; i < 3; ++i) o.w[i] = shfl_xor64(p.spd.w[i], d);
        fx_add(p.spd, o);
    }
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        u64 v;
        v = shfl_xor64(p.maxd, d);
        p.maxd = v > p.maxd ? v : p.maxd;
        v = shfl_xor64(p.latmin, d);
        p.latmin = v < p.latmin ? v : p.latmin;
        v = shfl_xor64(p.latmax, d);
        p.latmax = v > p.latmax ? v : p.latmax;
        v = shfl_xor64(p.lonmin, d);
        p.lonmin = v < p.lonmin ? v : p.lonmin;
        v = shfl_xor64(p.lonmax, d);
        p.lonmax = v > p.lonmax ? v : p.lonmax;
        u32 x;
        x = __shfl_xor(p.count, d, WAVE);
        p.count += x;
        x = __shfl_xor(p.ndtz, d, WAVE);
        p.ndtz += x;
        x = __shfl_xor(p.maxs, d, WAVE);
        p.maxs = x > p.maxs ? x : p.maxs;
    }
}

// segmented inclusive scan across lanes; `head` starts a segment.  Step k
// (distance 2^k) folds in the lane 2^k below when bit k of `take` is set.
__device__ __forceinline__ void part_seg_scan(Part& p, bool head)
{
    const int l = lane_id();
    u32 take = 0;
    bool f = head;
#pragma unroll
    for (int k = 0, d = 1; d < WAVE; ++k, d <<= 1) {
        const bool fo = __shfl_up(f, d, WAVE);
        if (l >= d) {
            if (!f) take |= 1u << k;
            f = f || fo;
        }
    }
#pragma unroll
    for (int k = 0, d = 1; d < WAVE; ++k, d <<= 1) {
        Fx192 o;
        for (int i = 0; i < 3; ++i) o.w[i] = shfl_up64(p.dist.w[i], d);
        if ((take >> k) & 1u) fx_add(p.dist, o);
    }
#pragma unroll
    for (int k = 0, d = 1; d < WAVE; ++k, d <<= 1) {
        Fx192 o;
        for (int i = 0; i < 3; ++i) o.w[i] = shfl_up64(p.spd.w[i], d);
        if ((take >> k) & 1u) fx_add(p.spd, o);
    }
#pragma unroll
    for (int k = 0, d = 1; d < WAVE; ++k, d <<= 1) {
        const bool t = (take >> k) & 1u;
        u64 v;
        v = shfl_up64(p.maxd, d);
        if (t && v > p.maxd) p.maxd = v;
        v = shfl_up64(p.latmin, d);
        if (t && v < p.latmin) p.latmin = v;
        v = shfl_up64(p.latmax, d);
        if (t && v > p.latmax) p.latmax = v;
        v = shfl_up64(p.lonmin, d);
        if (t && v < p.lonmin) p.lonmin = v;
        v = shfl_up64(p.lonmax, d);
        if (t && v > p.lonmax) p.lonmax = v;
        u32 x;
        x = __shfl_up(p.count, d, WAVE);
        if (t) p.count += x;
        x = __shfl_up(p.ndtz, d, WAVE);
        if (t) p.ndtz += x;
        x = __shfl_up(p.maxs, d, WAVE);
        if (t && x > p.maxs) p.maxs = x;
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

// A journey's partial into its accumulator row: a whole journey (all its
// records are in the partial) is stored, a piece is merged with integer atomics.
// The rows are turned into output rows by k_sum_finalize.
__device__ __forceinline__ void flush_part(JAcc* acc, u32 cap, u32 j, const Part& p, bool whole)
{
    if (j >= cap || p.count == 0) return;
    JAcc& a = acc[j];
    if (whole) {
        JAcc v;
        for (int i = 0; i < 3; ++i) {
            v.dist[i] = p.dist.w[i];
            v.spd[i] = p.spd.w[i];
        }
        v.maxd = p.maxd;
        v.latmin = p.latmin;
        v.latmax = p.latmax;
        v.lonmin = p.lonmin;
        v.lonmax = p.lonmax;
        v.count = p.count;
        v.ndtz = p.ndtz;
        v.maxs = p.maxs;
        v.touched = 1;
        a = v;
        return;
    }
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
// accumulator row through integer atomics.  Neighbouring ids come from lane
// shuffles; time stamps are read only at journey starts and ends.
__global__ void __launch_bounds__(SB) k_sum_reduce(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                   const double* __restrict__ lat, const double* __restrict__ lon,
                                                   const float* __restrict__ spd, const double* __restrict__ step,
                                                   const double* __restrict__ dspd, const uint8_t* __restrict__ flags,
                                                   const u32* __restrict__ tile_prefix, const u32* __restrict__ wcnt,
                                                   u32 cap, Out o, JAcc* __restrict__ acc,
                                                   const u64* __restrict__ soff, u32 S, u64* __restrict__ jo)
{
    const int w = threadIdx.x / WAVE;
    const int l = lane_id();
    const u64 cs = (u64)blockIdx.x * ST + (u64)w * WCH;  // wave chunk start
    const u64 ce = cs + WCH < n ? cs + WCH : (u64)n;      // wave chunk end (may be <= cs)
    if (cs >= ce) return;
    u32 seen = tile_prefix[blockIdx.x];  // journey starts before the current window
    for (int k = 0; k < w; ++k) seen += wcnt[(u64)blockIdx.x * NW + k];

    Part p;
    part_reset(p);
    // open journey: the one containing the record before the next window
    u32 open_j = seen - 1;   // valid when the chunk starts mid-journey
    bool open_here = false;  // its first record lies in this chunk
    i64 jprev = cs > 0 ? jid[cs - 1] : 0;
    u32 sk = S > 1 ? shard_lower_bound(soff, S, cs) : 0u;
    // value columns of a window, loaded one window ahead of their use
    struct Win {
        double st, ds, la, lo;
        float sp;
        uint8_t f;
    };
    auto load = [&](u64 a, Win& x) {
        const u64 r = a + l;
        if (r < ce) {
            x.st = step[r];
            x.sp = spd[r];
            x.f = flags[r];
            x.ds = dspd[r];
            x.la = lat[r];
            x.lo = lon[r];
        }
    };
    Win cur, nxt;
    load(cs, cur);
    for (int i = 0; i < WI; ++i) {
        const u64 a = cs + (u64)i * WAVE;
        if (a >= ce) break;
        if (i + 1 < WI) load(a + WAVE, nxt);
        const u64 r = a + l;
        const bool valid = r < ce;
        i64 jv;
        u64 smask;
        bool s_end;
        const u64 H = window_heads(jid, a, ce, jprev, jv, soff, S, sk, smask, s_end);
        const bool h = (H >> l) & 1ull;
        // last record of its journey: the next record starts one (or there is none)
        bool last = false;
        if (valid) {
            if (r + 1 >= n) last = true;
            else if (l < WAVE - 1) last = ((H >> (l + 1)) & 1ull) != 0;
            else last = jid[r + 1] != jv || s_end;
        }
        Part c;
        part_reset(c);
        if (valid) {
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
        // journey index of this lane's record
        const u32 jl = seen + popc_below(H) + (h ? 1u : 0u) - 1u;
        if (h && jl < cap) {
            // a journey's first record is indexed within its shard
            const u32 sh = S > 1 ? shard_of(soff, S, r) : 0u;
            o.jid[jl] = jv;
            o.first[jl] = (u32)(S > 1 ? r - soff[sh] : r);
            o.tstart[jl] = ts[r];
        }
        if (h && S > 1 && jo) {
            // this record opens its shard's first journey: every shard starting
            // here (empty ones included) begins at journey jl
            const u32 sh = shard_of(soff, S, r);
            if (soff[sh] == r)
                for (int z = (int)sh; z >= 0 && soff[z] == r; --z) jo[z] = jl;
        }
        if (last && jl < cap) o.tend[jl] = ts[r];
        if (H != 0) {
            const int f0 = __ffsll((long long)H) - 1;
            if (l < f0) part_combine(p, c);
            // close the journey that was open before the first start in this window
            part_wave_reduce(p);
            if (l == 0) flush_part(acc, cap, open_j, p, open_here);
            // journeys starting in this window
            Part s = c;
            part_seg_scan(s, h);
            // a segment that ends before lane 63 (next lane starts a journey) is a
            // whole journey: it began and ended inside this window
            const bool next_head = (l < WAVE - 1) && ((H >> (l + 1)) & 1ull);
            if (l >= f0 && next_head) flush_part(acc, cap, jl, s, true);
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
        flush_part(acc, cap, open_j, p, open_here && ends);
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
    u32* wcnt;
    u32* tile_prefix;
    JAcc* acc;
    u64 tiles;
    size_t bytes;
    SumLayout(void* ws, u64 n, u64 cap)
    {
        cvh::Carver c(ws);
        tiles = (n + ST - 1) / ST;
        meta = c.take<SumMeta>(1);
        wcnt = c.take<u32>(tiles * NW);
        tile_prefix = c.take<u32>(tiles + 1);
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
    hipLaunchKernelGGL(k_sum_count, dim3((unsigned)L.tiles), dim3(SB), 0, s, sorted->journey_id, nn, L.wcnt, soff, S);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(256), 0, s, L.wcnt, L.tile_prefix, (u32)L.tiles, L.meta);
    hipLaunchKernelGGL(k_sum_init, dim3(cvh::grid_for(cap, 256, 2048)), dim3(256), 0, s, L.acc, L.meta, cap);
    hipLaunchKernelGGL(k_sum_reduce, dim3((unsigned)L.tiles), dim3(SB), 0, s, nn, sorted->journey_id, sorted->ts_ms,
                       sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, feat->step_m, feat->speed_mps, feat->flags,
                       L.tile_prefix, L.wcnt, cap, o, L.acc, soff, S, jo);
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
