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

#include <mutex>
#include <type_traits>

#include "cv_device.h"
#include "cv_host.h"
#include "cv_sumtab.h"

using namespace cv;

namespace {

constexpr int SB = 256;
constexpr int SI = 64;
constexpr int ST = SB * SI;
constexpr int FX_DIST = SUM_FX_DIST;  // distance: 2^-128 m resolution (exact for steps >= 2^-75 m)
constexpr int FX_SPD = SUM_FX_SPD;    // speed: exact for every float32

struct SumMeta {
    u32 J;
};

constexpr int NW = SB / WAVE;  // waves per block
constexpr int WI = SI;         // windows of 64 records per wave
constexpr int WCH = WAVE * WI; // records per wave
static_assert(ST == NW * WCH, "tile = waves x wave chunk");

// Journey starts among the records of window [a, a + 64) of a wave that walks
// consecutive windows, from this lane's id jv (already loaded): jprev is the
// id before the window (carried), sk the shard cursor.  Returns the lane mask
// of starts.
__device__ __forceinline__ u64 heads_of(i64 jv, u64 a, u64 end, i64& jprev, const u64* __restrict__ soff, u32 S,
                                        u32& sk, u64& smask, bool& s_end)
{
    const int l = lane_id();
    const u64 r = a + l;
    const bool valid = r < end;
    i64 jp = __shfl_up(jv, 1, WAVE);
    if (l == 0) jp = jprev;
    jprev = __shfl(jv, WAVE - 1, WAVE);
    smask = 0;
    s_end = false;
    if (S > 1) smask = shard_starts_in(soff, S, sk, a, s_end);
    return __ballot(valid && (r == 0 || jv != jp || ((smask >> l) & 1ull)));
}

// journey starts per wave chunk of WCH records: wcnt[tile * NW + wave], and
// per tile: tcnt[tile]
__global__ void __launch_bounds__(SB) k_sum_count(const i64* __restrict__ jid, u32 n, u32* __restrict__ wcnt,
                                                  u32* __restrict__ tcnt, const u64* __restrict__ soff, u32 S)
{
    __shared__ u32 s_w[NW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);  // wave-uniform
    const u64 cs = (u64)blockIdx.x * ST + (u64)w * WCH;
    const u64 ce = cs + WCH < n ? cs + WCH : (u64)n;
    u32 c = 0;
    if (cs < ce) {
        i64 jprev = cs > 0 ? jid[cs - 1] : 0;
        u32 sk = S > 1 ? shard_lower_bound(soff, S, cs) : 0u;
        i64 jn = cs + lane_id() < ce ? jid[cs + lane_id()] : 0;
        for (u64 a = cs; a < ce; a += WAVE) {
            const i64 jv = jn;
            if (a + WAVE + lane_id() < ce) jn = jid[a + WAVE + lane_id()];  // next window, loaded ahead
            u64 sm;
            bool se;
            c += (u32)__popcll(heads_of(jv, a, ce, jprev, soff, S, sk, sm, se));
        }
    }
    if (lane_id() == 0) {
        wcnt[(u64)blockIdx.x * NW + w] = c;
        s_w[w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 t = 0;
        for (int k = 0; k < NW; ++k) t += s_w[k];
        tcnt[blockIdx.x] = t;
    }
}

// The same counts from the features' FIRST flags (set exactly at journey and
// shard starts): one byte per record instead of an id and its predecessor.
__global__ void __launch_bounds__(SB) k_sum_count_flags(const uint8_t* __restrict__ flags, u32 n,
                                                        u32* __restrict__ wcnt, u32* __restrict__ tcnt)
{
    __shared__ u32 s_w[NW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const u64 cs = (u64)blockIdx.x * ST + (u64)w * WCH;
    const u64 ce = cs + WCH < n ? cs + WCH : (u64)n;
    constexpr int FB = WCH / WAVE;  // flag bytes per lane
    static_assert(FB % 16 == 0 && CV_FLAG_FIRST == 1u, "whole 16-byte loads per lane; FIRST is bit 0");
    u32 c = 0;
    if (cs < ce) {
        // lane l counts the chunk's bytes [FB l, FB l + FB): 16-byte loads
        // when the chunk is whole and the column 16-byte aligned
        const u64 b0 = cs + (u64)lane_id() * FB;
        if (ce - cs == (u64)WCH && ((uintptr_t)flags & 15u) == 0) {
#pragma unroll
            for (int q = 0; q < FB / 16; ++q) {
                const uint4 v = *reinterpret_cast<const uint4*>(flags + b0 + 16 * q);
                c += (u32)(__popc(v.x & 0x01010101u) + __popc(v.y & 0x01010101u) + __popc(v.z & 0x01010101u) +
                           __popc(v.w & 0x01010101u));
            }
        } else {
            for (int k = 0; k < FB; ++k)
                if (b0 + k < ce) c += flags[b0 + k] & CV_FLAG_FIRST;
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) c += (u32)__shfl_xor((int)c, d, WAVE);
    }
    if (lane_id() == 0) {
        wcnt[(u64)blockIdx.x * NW + w] = c;
        s_w[w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 t = 0;
        for (int k = 0; k < NW; ++k) t += s_w[k];
        tcnt[blockIdx.x] = t;
    }
}

// single block: tile_prefix[i] = journey starts before tile i; meta->J = total.
// Each thread sums a contiguous run of tiles, one block scan joins the runs.
constexpr int SCAN_B = 1024;
__global__ void __launch_bounds__(SCAN_B) k_tile_scan(const u32* __restrict__ tcnt, u32* __restrict__ tile_prefix,
                                                      u32 tiles, SumMeta* meta)
{
    __shared__ u32 tmp[SCAN_B / WAVE];
    const u32 per = (tiles + SCAN_B - 1) / SCAN_B;
    const u32 a = threadIdx.x * per;
    const u32 b = a + per < tiles ? a + per : tiles;
    u32 sum = 0;
#pragma unroll 8
    for (u32 i = a; i < b; ++i) sum += tcnt[i];
    u32 total;
    u32 e = block_exclusive_sum<SCAN_B>(sum, tmp, total);
    for (u32 i = a; i < b; ++i) {
        tile_prefix[i] = e;
        e += tcnt[i];
    }
    if (threadIdx.x == 0) meta->J = total;
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
    a.gfirst = 0;
}

__global__ void __launch_bounds__(256) k_sum_init(JAcc* __restrict__ acc, AccX* __restrict__ accx, const SumMeta* meta,
                                                 u32 cap)
{
    u32 J = meta->J;
    u32 m = J < cap ? J : cap;
    for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        JAcc a;
        jacc_identity(a);
        acc[j] = a;
        AccX x = {};
        accx[j] = x;
    }
}

// Partial aggregates of one journey (a lane's records, a wave's, or a tile's),
// in two field groups reduced by two launches of the same kernel: the record
// count with the bounding box, and the exact sums with the zero-dt count and
// the maxima.  Each launch keeps only its group live, which keeps its
// register use (and so the waves in flight per SIMD) in bounds.
struct PartBox {
    u64 latmin, latmax, lonmin, lonmax;
    u32 count;
};
// The sums are 128-bit two's-complement integers: distance in units of 2^-72
// m, exact for steps of at least 2^-20 m (and zero); speed in units of 2^-53,
// exact for float32 speeds v with 2^-30 <= |v| < 2^10 (and zeros).  Any other
// value is added on its own, in the full 192-bit format, to the journey's
// side row (AccX).
struct PartSum {
    u64 dlo, dhi, slo, shi;
    u64 maxd;
    u32 ndtz, maxs, n;  // n: records folded in (empty partials are not flushed)
};

__device__ __forceinline__ void add128(u64& lo, u64& hi, u64 blo, u64 bhi)
{
    const u64 s = lo + blo;
    hi += bhi + (s < lo ? 1ull : 0ull);
    lo = s;
}

// v * 2^72 as a 128-bit integer when 2^-20 <= |v| < 2^40 or v = +-0
__device__ __forceinline__ bool dist_fix72(double v, u64& lo, u64& hi)
{
    const u64 b = (u64)__double_as_longlong(v);
    const u32 e = (u32)((b >> 52) & 0x7FFu);
    const u64 m = b & ((1ull << 52) - 1);
    lo = 0;
    hi = 0;
    if (e == 0) return m == 0;
    if (e < 1003 || e > 1062) return false;
    const u64 M = m | (1ull << 52);
    const u32 sft = e - 1003;  // 0 .. 59
    lo = M << sft;
    hi = sft ? (M >> (64 - sft)) : 0ull;
    if (b >> 63) {
        lo = ~lo + 1;
        hi = ~hi + (lo == 0 ? 1ull : 0ull);
    }
    return true;
}

// v * 2^53 as a signed integer when 2^-30 <= |v| < 2^10 or v = +-0
__device__ __forceinline__ bool spd_fix53(float v, i64& x)
{
    const u32 b = __float_as_uint(v);
    const u32 e = (b >> 23) & 0xFFu;
    const u32 m = b & 0x7FFFFFu;
    x = 0;
    if (e == 0) return m == 0;
    if (e < 97 || e > 136) return false;
    const i64 mag = (i64)((u64)(m | 0x800000u) << (e - 97));
    x = (b >> 31) ? -mag : mag;
    return true;
}

// the 128-bit sums in the 192-bit formats of the rows (2^-128 m, 2^-149)
__device__ __forceinline__ Fx192 dist192(u64 lo, u64 hi)
{
    Fx192 r;
    r.w[0] = lo << 56;
    r.w[1] = (lo >> 8) | (hi << 56);
    r.w[2] = (u64)((i64)hi >> 8);
    return r;
}
__device__ __forceinline__ Fx192 spd192(u64 lo, u64 hi)
{
    Fx192 r;
    r.w[0] = 0;
    r.w[1] = lo << 32;
    r.w[2] = (lo >> 32) | (hi << 32);
    return r;
}

__device__ __forceinline__ void part_reset(PartBox& p)
{
    p.latmin = ord_f64(__builtin_inf());
    p.latmax = ord_f64(-__builtin_inf());
    p.lonmin = ord_f64(__builtin_inf());
    p.lonmax = ord_f64(-__builtin_inf());
    p.count = 0;
}
__device__ __forceinline__ void part_reset(PartSum& p)
{
    p.dlo = p.dhi = p.slo = p.shi = 0;
    p.maxd = ord_f64(0.0);
    p.ndtz = 0;
    p.maxs = 0;
    p.n = 0;
}

__device__ __forceinline__ void part_combine(PartBox& a, const PartBox& b)
{
    a.latmin = b.latmin < a.latmin ? b.latmin : a.latmin;
    a.latmax = b.latmax > a.latmax ? b.latmax : a.latmax;
    a.lonmin = b.lonmin < a.lonmin ? b.lonmin : a.lonmin;
    a.lonmax = b.lonmax > a.lonmax ? b.lonmax : a.lonmax;
    a.count += b.count;
}
__device__ __forceinline__ void part_combine(PartSum& a, const PartSum& b)
{
    add128(a.dlo, a.dhi, b.dlo, b.dhi);
    add128(a.slo, a.shi, b.slo, b.shi);
    a.maxd = b.maxd > a.maxd ? b.maxd : a.maxd;
    a.ndtz += b.ndtz;
    a.maxs = b.maxs > a.maxs ? b.maxs : a.maxs;
    a.n += b.n;
}

// Cross-lane steps work one field at a time, so that only that field's
// shuffled copy is live next to the partial.  A step of distance d takes the
// lane d away (xor for the full reduction, below for the segmented scan);
// `take` says whether the step folds it in.
__device__ __forceinline__ u64 shfl64(u64 v, int d, bool up)
{
    return up ? (u64)__shfl_up((unsigned long long)v, d, WAVE) : (u64)__shfl_xor((unsigned long long)v, d, WAVE);
}
__device__ __forceinline__ u32 shfl32(u32 v, int d, bool up)
{
    return up ? (u32)__shfl_up(v, d, WAVE) : (u32)__shfl_xor(v, d, WAVE);
}

__device__ __forceinline__ void part_step(PartBox& p, int d, bool up, bool take)
{
    u64 v;
    v = shfl64(p.latmin, d, up);
    if (take && v < p.latmin) p.latmin = v;
    v = shfl64(p.latmax, d, up);
    if (take && v > p.latmax) p.latmax = v;
    v = shfl64(p.lonmin, d, up);
    if (take && v < p.lonmin) p.lonmin = v;
    v = shfl64(p.lonmax, d, up);
    if (take && v > p.lonmax) p.lonmax = v;
    const u32 x = shfl32(p.count, d, up);
    if (take) p.count += x;
}
__device__ __forceinline__ void part_step(PartSum& p, int d, bool up, bool take)
{
    const u64 dlo = shfl64(p.dlo, d, up), dhi = shfl64(p.dhi, d, up);
    if (take) add128(p.dlo, p.dhi, dlo, dhi);
    const u64 slo = shfl64(p.slo, d, up), shi = shfl64(p.shi, d, up);
    if (take) add128(p.slo, p.shi, slo, shi);
    const u64 v = shfl64(p.maxd, d, up);
    if (take && v > p.maxd) p.maxd = v;
    u32 x;
    x = shfl32(p.ndtz, d, up);
    if (take) p.ndtz += x;
    x = shfl32(p.maxs, d, up);
    if (take && x > p.maxs) p.maxs = x;
    x = shfl32(p.n, d, up);
    if (take) p.n += x;
}

// full wave reduction; every lane ends with the total
template <class P>
__device__ __forceinline__ void part_wave_reduce(P& p)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) part_step(p, d, false, true);
}

// segmented inclusive scan across lanes; `head` starts a segment
template <class P>
__device__ __forceinline__ void part_seg_scan(P& p, bool head)
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
    for (int k = 0, d = 1; d < WAVE; ++k, d <<= 1) part_step(p, d, true, ((take >> k) & 1u) != 0);
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
__device__ __forceinline__ void flush_part(JAcc* acc, u32 cap, u32 j, const PartBox& p, bool whole)
{
    if (j >= cap || p.count == 0) return;
    JAcc& a = acc[j];
    if (whole) {
        a.latmin = p.latmin;
        a.latmax = p.latmax;
        a.lonmin = p.lonmin;
        a.lonmax = p.lonmax;
        a.count = p.count;
        return;
    }
    atomicMin((unsigned long long*)&a.latmin, (unsigned long long)p.latmin);
    atomicMax((unsigned long long*)&a.latmax, (unsigned long long)p.latmax);
    atomicMin((unsigned long long*)&a.lonmin, (unsigned long long)p.lonmin);
    atomicMax((unsigned long long*)&a.lonmax, (unsigned long long)p.lonmax);
    atomicAdd(&a.count, p.count);
}
__device__ __forceinline__ void flush_part(JAcc* acc, u32 cap, u32 j, const PartSum& p, bool whole)
{
    if (j >= cap || p.n == 0) return;
    JAcc& a = acc[j];
    const Fx192 d = dist192(p.dlo, p.dhi), sp = spd192(p.slo, p.shi);
    if (whole) {
        for (int i = 0; i < 3; ++i) {
            a.dist[i] = d.w[i];
            a.spd[i] = sp.w[i];
        }
        a.maxd = p.maxd;
        a.ndtz = p.ndtz;
        a.maxs = p.maxs;
        return;
    }
    atomic_add_fx(a.dist, d);
    atomic_add_fx(a.spd, sp);
    atomicMax((unsigned long long*)&a.maxd, (unsigned long long)p.maxd);
    atomicAdd(&a.ndtz, p.ndtz);
    atomicMax(&a.maxs, p.maxs);
}

// Each wave owns WCH consecutive records and walks them in coalesced windows of
// 64, loaded a group of windows at a time.  Lanes fold their records into a private partial while the window holds
// no journey start; a window with starts closes the open journey (wave
// reduction), runs a segmented scan for journeys that begin in it, and hands
// the last one on as the new open journey.  A journey that begins and ends in
// the wave's records is stored directly; otherwise its pieces meet in the
// accumulator row through integer atomics.  Neighbouring ids come from lane
// shuffles.  BOX = true reduces PartBox and also writes each journey's id,
// first record; BOX = false reduces PartSum.  SHARDS = false compiles the
// plain form without the shard branches, whose loads would otherwise make
// every window wait for all loads in flight, prefetch included.
// FL = true: journey starts are read from the features' FIRST flags instead
// of comparing ids (the box pass then loads an id only at a journey start,
// to write it out).
template <bool BOX, bool SHARDS, bool FL = false>
__global__ void __launch_bounds__(SB) k_sum_reduce(u32 n, const i64* __restrict__ jid, const double* __restrict__ lat,
                                                   const double* __restrict__ lon, const float* __restrict__ spd, const double* __restrict__ step,
                                                   const double* __restrict__ dspd, const uint8_t* __restrict__ flags,
                                                   const u32* __restrict__ tile_prefix, const u32* __restrict__ wcnt,
                                                   u32 cap, Out o, JAcc* __restrict__ acc, AccX* __restrict__ accx,
                                                   const u64* __restrict__ soff, u32 S, u64* __restrict__ jo)
{
    using P = typename std::conditional<BOX, PartBox, PartSum>::type;
    if (!SHARDS) S = 0;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);  // wave-uniform
    const int l = lane_id();
    const u64 cs = (u64)blockIdx.x * ST + (u64)w * WCH;  // wave chunk start
    const u64 ce = cs + WCH < n ? cs + WCH : (u64)n;      // wave chunk end (may be <= cs)
    if (cs >= ce) return;
    u32 seen = tile_prefix[blockIdx.x];  // journey starts before the current window
    for (int k = 0; k < w; ++k) seen += wcnt[(u64)blockIdx.x * NW + k];

    P p;
    part_reset(p);
    // open journey: the one containing the record before the next window
    u32 open_j = seen - 1;   // valid when the chunk starts mid-journey
    bool open_here = false;  // its first record lies in this chunk
    i64 jprev = (!FL && cs > 0) ? jid[cs - 1] : 0;
    u32 sk = (SHARDS && !FL) ? shard_lower_bound(soff, S, cs) : 0u;
    // the shard holding the chunk's first record: a journey head's shard is
    // walked forward from it (a chunk spans few shards) instead of searched
    const u32 shc = (SHARDS && FL && S > 1) ? shard_of(soff, S, cs) : 0u;
    // the id after the chunk (its last record may end a journey)
    const i64 jend = (!FL && ce < n) ? jid[ce] : 0;
    // Windows are taken in groups of WG: the columns of a group (ids included)
    // are loaded together, from addresses clamped into the chunk, so that all
    // of a group's loads are in flight at once.
    constexpr int WG = 4;
    static_assert(WI % WG == 0, "whole groups");
    for (int g0 = 0; g0 < WI; g0 += WG) {
        if (cs + (u64)g0 * WAVE >= ce) break;
        i64 gj[WG];
        double gx0[WG], gx1[WG];
        float gsp[WG];
        uint8_t gf[WG];
#pragma unroll
        for (int k = 0; k < WG; ++k) {
            u64 r = cs + (u64)(g0 + k) * WAVE + l;
            r = r < ce ? r : ce - 1;
            gj[k] = FL ? 0 : jid[r];
            if constexpr (BOX) {
                gx0[k] = lat[r];
                gx1[k] = lon[r];
                if (FL) gf[k] = flags[r];
            } else {
                gx0[k] = step[r];
                gx1[k] = dspd[r];
                gsp[k] = spd[r];
                gf[k] = flags[r];
            }
        }
#pragma unroll
        for (int k = 0; k < WG; ++k) {
            const u64 a = cs + (u64)(g0 + k) * WAVE;
            if (a >= ce) break;
            const u64 r = a + l;
            const bool valid = r < ce;
            const i64 jv = gj[k];
            u64 smask;
            bool s_end;
            u64 H;
            if constexpr (FL) {
                H = __ballot(valid && (gf[k] & CV_FLAG_FIRST) != 0);
                smask = 0;
                s_end = false;
            } else {
                H = heads_of(jv, a, ce, jprev, soff, S, sk, smask, s_end);
            }
            const bool h = (H >> l) & 1ull;
            // journey index of this lane's record
            const u32 jl = seen + popc_below(H) + (h ? 1u : 0u) - 1u;
            P c;
            part_reset(c);
            if (valid) {
                if constexpr (BOX) {
                    c.count = 1;
                    if (isfinite(gx0[k]) && isfinite(gx1[k])) {
                        c.latmin = c.latmax = ord_f64(gx0[k]);
                        c.lonmin = c.lonmax = ord_f64(gx1[k]);
                    }
                } else {
                    c.n = 1;
                    c.ndtz = (gf[k] & CV_FLAG_DT_ZERO) ? 1u : 0u;
                    if (!dist_fix72(gx0[k], c.dlo, c.dhi) && jl < cap)
                        atomic_add_fx(accx[jl].dist, fx_from_double<FX_DIST>(gx0[k]));
                    i64 x;
                    if (spd_fix53(gsp[k], x)) {
                        c.slo = (u64)x;
                        c.shi = (u64)(x >> 63);
                    } else if (jl < cap) {
                        atomic_add_fx(accx[jl].spd, fx_from_double<FX_SPD>((double)gsp[k]));
                    }
                    c.maxs = ord_f32(gsp[k]);
                    if (gf[k] & CV_FLAG_SPEED_OK) c.maxd = ord_f64(gx1[k]);
                }
            }
            if constexpr (BOX) {
                const u32 sh = (h && S > 1) ? (FL ? shard_from(soff, S, shc, r) : shard_of(soff, S, r)) : 0u;
                if (h && jl < cap) {
                    // a journey's first record is indexed within its shard
                    if (o.jid) o.jid[jl] = FL ? jid[r] : jv;
                    if (o.first) o.first[jl] = (u32)(S > 1 ? r - soff[sh] : r);
                    acc[jl].gfirst = (u32)r;
                }
                if (h && S > 1 && jo) {
                    // this record opens its shard's first journey: every shard
                    // starting here (empty ones included) begins at journey jl
                    if (soff[sh] == r)
                        for (int z = (int)sh; z >= 0 && soff[z] == r; --z) jo[z] = jl;
                }
            }
            if (H != 0) {
                const int f0 = __ffsll((long long)H) - 1;
                if (l < f0) part_combine(p, c);
                // close the journey that was open before the first start in this window
                part_wave_reduce(p);
                if (l == 0) flush_part(acc, cap, open_j, p, open_here);
                // journeys starting in this window
                P sc = c;
                part_seg_scan(sc, h);
                // a segment that ends before lane 63 (next lane starts a journey)
                // is a whole journey: it began and ended inside this window
                const bool next_head = (l < WAVE - 1) && ((H >> (l + 1)) & 1ull);
                if (l >= f0 && next_head) flush_part(acc, cap, jl, sc, true);
                // the last segment stays open; lane 63 holds its partial
                part_reset(p);
                if (l == WAVE - 1) p = sc;
                seen += (u32)__popcll(H);
                open_j = seen - 1;
                open_here = true;
            } else {
                part_combine(p, c);
            }
        }
    }
    part_wave_reduce(p);
    if (l == 0) {
        const bool ends = FL ? ((ce >= n) || (flags[ce] & CV_FLAG_FIRST) != 0)
                             : ((ce >= n) || (jend != jprev) || (S > 1 && shard_start(soff, S, ce)));
        flush_part(acc, cap, open_j, p, open_here && ends);
    }
}

__global__ void __launch_bounds__(256) k_sum_finalize(const JAcc* __restrict__ acc, const AccX* __restrict__ accx,
                                                      const SumMeta* meta, u32 cap,
                                                      Out o, const i64* __restrict__ ts, cv_result* res,
                                                      const u64* __restrict__ soff, u32 S, u64* __restrict__ jo,
                                                      u32 n)
{
    u32 J = meta->J;
    u32 m = J < cap ? J : cap;
    for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        const JAcc& a = acc[j];
        Fx192 d, s;
        d.w[0] = a.dist[0];
        d.w[1] = a.dist[1];
        d.w[2] = a.dist[2];
        s.w[0] = a.spd[0];
        s.w[1] = a.spd[1];
        s.w[2] = a.spd[2];
        // values outside the 128-bit formats, added on their own
        const AccX& x = accx[j];
        Fx192 xd, xs;
        for (int i = 0; i < 3; ++i) {
            xd.w[i] = x.dist[i];
            xs.w[i] = x.spd[i];
        }
        fx_add(d, xd);
        fx_add(s, xs);
        write_final(o, j, a.count, a.ndtz, d, s, a.maxs, a.maxd, a.latmin, a.latmax, a.lonmin, a.lonmax);
        // a journey's records are consecutive: its time span is read at both ends
        o.tstart[j] = ts[a.gfirst];
        o.tend[j] = ts[a.gfirst + a.count - 1];
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
    u32* tcnt;
    u32* tile_prefix;
    JAcc* acc;
    AccX* accx;
    u64 tiles;
    size_t bytes;
    SumLayout(void* ws, u64 n, u64 cap)
    {
        cvh::Carver c(ws);
        tiles = (n + ST - 1) / ST;
        meta = c.take<SumMeta>(1);
        wcnt = c.take<u32>(tiles * NW);
        tcnt = c.take<u32>(tiles + 1);
        tile_prefix = c.take<u32>(tiles + 1);
        acc = c.take<JAcc>(cap < n ? cap : n);
        accx = c.take<AccX>(cap < n ? cap : n);
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
    // journey starts come from the features' FIRST flags here (the features
    // of these records mark exactly the journey and shard starts)
    hipLaunchKernelGGL(k_sum_count_flags, dim3((unsigned)L.tiles), dim3(SB), 0, s, feat->flags, nn, L.wcnt, L.tcnt);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(SCAN_B), 0, s, L.tcnt, L.tile_prefix, (u32)L.tiles, L.meta);
    hipLaunchKernelGGL(k_sum_init, dim3(cvh::grid_for(cap, 256, 2048)), dim3(256), 0, s, L.acc, L.accx, L.meta, cap);
    for (const bool box : {true, false}) {
        auto kern = box ? (S > 1 ? k_sum_reduce<true, true, true> : k_sum_reduce<true, false, true>)
                        : (S > 1 ? k_sum_reduce<false, true, true> : k_sum_reduce<false, false, true>);
        hipLaunchKernelGGL(kern, dim3((unsigned)L.tiles), dim3(SB), 0, s, nn, sorted->journey_id, sorted->lat_deg,
                           sorted->lon_deg, sorted->speed_mps, feat->step_m, feat->speed_mps, feat->flags,
                           L.tile_prefix, L.wcnt, cap, o, L.acc, L.accx, soff, S, jo);
    }
    hipLaunchKernelGGL(k_sum_finalize, dim3(cvh::grid_for(cap, 256, 2048)), dim3(256), 0, s, L.acc, L.accx, L.meta, cap, o,
                       sorted->ts_ms, res, soff, S, jo, nn);
    cvh::debug_rows(out->journey_id, nullptr, nullptr, res, cap, jo, S, CV_DEBUG_JOURNEY_ORDER, s);
    return cvh::last_launch_status();
}

// Workspace of the allocation-free entry point: one copy of this array per GPU
// (the code object's static device data), held until the process ends.  Host
// code reaches it only through the device address taken below; the array's
// name is not a device address on the host.
static __device__ __align__(256) unsigned char scratch[CV_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// the array's address on the current device, taken once per device
void* noalloc_scratch()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        if (!cvh::aligned(p, cvh::WS_ALIGN)) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

namespace cv {

size_t sum_partials_bytes(u64 n)
{
    SumLayout L(nullptr, n, 0);
    return L.bytes;
}

cv_status sum_partials(const cv_records* sorted, const cv_features* feat, u32 rows, JAcc* acc, AccX* accx, void* ws,
                       hipStream_t s)
{
    const u64 n = sorted->n;
    if (n == 0) return CV_OK;
    SumLayout L(ws, n, 0);
    Out o{};
    const u32 nn = (u32)n;
    hipLaunchKernelGGL(k_sum_count, dim3((unsigned)L.tiles), dim3(SB), 0, s, sorted->journey_id, nn, L.wcnt, L.tcnt,
                       nullptr, 0u);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(SCAN_B), 0, s, L.tcnt, L.tile_prefix, (u32)L.tiles, L.meta);
    hipLaunchKernelGGL(k_sum_init, dim3(cvh::grid_for(rows, 256, 2048)), dim3(256), 0, s, acc, accx, L.meta, rows);
    hipLaunchKernelGGL((k_sum_reduce<true, false>), dim3((unsigned)L.tiles), dim3(SB), 0, s, nn, sorted->journey_id,
                       sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, feat->step_m, feat->speed_mps,
                       feat->flags, L.tile_prefix, L.wcnt, rows, o, acc, accx, nullptr, 0u, nullptr);
    hipLaunchKernelGGL((k_sum_reduce<false, false>), dim3((unsigned)L.tiles), dim3(SB), 0, s, nn, sorted->journey_id,
                       sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, feat->step_m, feat->speed_mps,
                       feat->flags, L.tile_prefix, L.wcnt, rows, o, acc, accx, nullptr, 0u, nullptr);
    return cvh::last_launch_status();
}

}  // namespace cv

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

cv_status cv_journey_summary_noalloc(const cv_records* sorted, const cv_features* feat, const cv_journeys* out,
                                     uint64_t capacity, cv_result* res, void* stream)
{
    if (!sorted || sorted->n >= (1ull << 32) || capacity >= (1ull << 32)) return CV_ERR_INVALID_ARGUMENT;
    SumLayout need(nullptr, sorted->n, capacity);
    if (need.bytes > (size_t)CV_NOALLOC_SCRATCH_BYTES) return CV_ERR_WORKSPACE;
    void* ws = noalloc_scratch();
    if (!ws) return CV_ERR_DEVICE;
    return summary_impl(sorted, feat, nullptr, 0, out, capacity, nullptr, res, ws, (size_t)CV_NOALLOC_SCRATCH_BYTES,
                        stream);
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
