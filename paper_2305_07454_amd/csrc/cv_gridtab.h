// cv_gridtab.h -- pieces of the grid aggregate shared by the plain, batched
// and streaming forms:
//   * the binning of Algorithm 2 (grid_key) and (journey, time-bin) segment
//     starts;
//   * the HBM group table: one 64-byte entry per (time bin, cell) key with
//     count, distinct journeys, an exact speed sum in carry-save 40-bit chunks
//     and min / max speed as ordered integers, updated with integer atomics
//     only, so its content does not depend on the order of the updates;
//   * the tail of that table (the serving form's flush): occupied entries
//     compacted, radix-sorted by key, emitted in ascending key (kernels with
//     internal linkage, one copy per user);
//   * the partial row of a tile (GPart), which the plain and batched forms
//     merge by a key sort instead of a table (cv_gridpart.h writes them).
#pragma once
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_radix.h"
#include "cvetl.h"

namespace cv {
namespace {

constexpr int FX_SPD = 149;
constexpr int CS40 = 5;  // carry-save chunks of 40 bits: 2^24 adds per entry without overflow
constexpr u64 GEMPTY = ~0ull;

// one 64-byte line per group
struct GEntry {
    u64 key;
    u64 cs[CS40];
    u32 count, nj, mn, mx;
};
static_assert(sizeof(GEntry) == 64, "entry layout");

__device__ __forceinline__ void fx_to_cs40(const Fx192& a, u64 c[CS40])
{
    const u64 M = (1ull << 40) - 1;
    c[0] = a.w[0] & M;
    c[1] = ((a.w[0] >> 40) | (a.w[1] << 24)) & M;
    c[2] = (a.w[1] >> 16) & M;
    c[3] = ((a.w[1] >> 56) | (a.w[2] << 8)) & M;
    c[4] = a.w[2] >> 32;
}

__device__ __forceinline__ Fx192 fx_from_cs40(const u64 c[CS40])
{
    Fx192 r;
    fx_zero(r);
#pragma unroll
    for (int i = 0; i < CS40; ++i) {
        Fx192 t = fx_place(c[i], 40 * i);  // c[i] < 2^64: the part beyond bit 191 wraps away
        fx_add(r, t);
    }
    return r;
}

// A partial group row of one tile (plain and batched forms): the tile's
// records of one (journey, key), merged with the other partials of that key
// after a key sort.  32 bytes, one aligned sector.  The speed sum is a 96-bit
// two's complement integer in 2^-53 units (s[0] lowest; a tile's sum stays
// below 2^74 in magnitude), or (cn bit 31) s[0] holds the one speed of a
// record outside that format as float bits.
struct GPart {
    i64 jid;
    u32 s[3];
    u32 cn;      // records; bit 31: s[0] is a float's bits
    u32 mn, mx;  // ordered-integer min / max speed
};
static_assert(sizeof(GPart) == 32, "partial layout");

struct GridMeta {
    u32 groups;     // groups after the merge of the partials
    u32 overflow;   // HBM table full
    u64 n_out;      // records outside the grid
    u64 max_key;    // largest key seen
    u32 key_bits;
    u32 passes;
    u32 compact_n;
    u32 chunks;     // chunks of sorted partial pairs (the partial-row merge)
    u32 tickets[MAX_PASSES];
};

struct Spec {
    double lat0, lon0, dlat, dlon;
    i64 n_lat, n_lon, t0, bin_ms, tmax;
    double tinv;      // 1 / bin_ms, rounded (the time bin's quotient estimate)
    const u64* soff;  // shard offsets (batched form) or nullptr
    u32 S;            // number of shards (0 or 1: one problem)
    u32 kb;           // bits of the cell key; the shard index sits above them
    // direction dimension (nd sectors plus one for records without a
    // direction; nd = 0: none): a sensor heading per sorted record, else the
    // derived bearing with its flags
    u32 nd;
    double dstep, doff;  // sector width 360 / nd and offset, degrees
    const float* hdg;
    const double* brg;
    const uint8_t* bfl;
    u64* sout;  // batched form, nullable: records outside the grid per shard
};

// floor(a / b) for b > 0: a double estimate corrected by one integer step
// (exact for |a| < 2^52); wider operands take the integer division.
__device__ __forceinline__ i64 floor_div64(i64 a, i64 b)
{
    if (a > -(1ll << 52) && a < (1ll << 52)) {
        i64 q = (i64)floor((double)a / (double)b);
        i64 r = a - q * b;
        if (r < 0) q -= 1;
        else if (r >= b) q += 1;
        return q;
    }
    i64 q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

// The time bin floor((ts - t0) / bin_ms).  The quotient is estimated by a
// multiply with the rounded reciprocal of bin_ms; for |ts - t0| < 2^52 the
// estimate is within one of the quotient, so its floor is off by at most one
// and one integer step corrects it.  Offsets and widths below 2^30 (any time
// within twelve days of t0) take the step in 32-bit arithmetic, where no
// product overflows; wider offsets take it in 64 bits, and offsets beyond
// 2^52 the integer division.
__device__ __forceinline__ i64 time_bin(const Spec& g, i64 ts)
{
    const i64 a = ts - g.t0;
    if (g.bin_ms < (1ll << 30) && a >= -(1ll << 30) && a < (1ll << 30)) {
        const u32 a32 = (u32)a, b32 = (u32)g.bin_ms;
        int q = (int)floor((double)(int)a32 * g.tinv);
        const int r = (int)(a32 - (u32)q * b32);  // |r| < 2 bin_ms: exact through the wrap
        q += r < 0 ? -1 : (r >= (int)b32 ? 1 : 0);
        return (i64)q;
    }
    if (a > -(1ll << 52) && a < (1ll << 52)) {
        i64 q = (i64)floor((double)a * g.tinv);
        const i64 r = a - q * g.bin_ms;
        if (r < 0) q -= 1;
        else if (r >= g.bin_ms) q += 1;
        return q;
    }
    return floor_div64(a, g.bin_ms);
}

// Direction sector of a heading h in degrees (Algorithm 2 bins it by floor
// division with a sector width): floor((h + doff) / dstep) mod nd for h in
// [0, 360); nd for a missing direction (no valid heading or bearing).
__device__ __forceinline__ u32 dir_sector(const Spec& g, double h, bool ok)
{
    if (!ok || !(h >= 0.0 && h < 360.0)) return g.nd;
    const u32 s = (u32)floor((h + g.doff) / g.dstep);
    return s % g.nd;
}

// the sector of sorted record r: KD = 1 sensor heading, 2 derived bearing
template <int KD>
__device__ __forceinline__ u32 dir_at(const Spec& g, u64 r)
{
    if constexpr (KD == 1) return dir_sector(g, (double)g.hdg[r], true);
    else if constexpr (KD == 2) return dir_sector(g, g.brg[r], (g.bfl[r] & CV_FLAG_BEARING_OK) != 0);
    else return 0u;
}

// key (or -1) and time bin of a record of shard sh; floor of the IEEE
// quotient.  In the batched form the shard index is placed above the cell key;
// with directions, the sector sits between the time bin and the cell.
__device__ __forceinline__ i64 grid_key_in(const Spec& g, u32 sh, i64 ts, double la, double lo, i64& tb,
                                           u32 dir = 0)
{
    tb = time_bin(g, ts);
    if (!isfinite(la) || !isfinite(lo)) return -1;
    double fy = floor((la - g.lat0) / g.dlat);
    double fx = floor((lo - g.lon0) / g.dlon);
    if (!(fy >= 0.0 && fy < (double)g.n_lat && fx >= 0.0 && fx < (double)g.n_lon && tb >= 0 && tb < g.tmax)) return -1;
    const i64 td = g.nd ? tb * (i64)(g.nd + 1) + (i64)dir : tb;
    i64 k = (td * g.n_lat + (i64)fy) * g.n_lon + (i64)fx;
    if (g.S > 1) k |= (i64)((u64)sh << g.kb);
    return k;
}

// the same for record r (its shard found by binary search)
__device__ __forceinline__ i64 grid_key(const Spec& g, u64 r, i64 ts, double la, double lo, i64& tb, u32 dir = 0)
{
    return grid_key_in(g, g.S > 1 ? shard_of(g.soff, g.S, r) : 0u, ts, la, lo, tb, dir);
}

// first record of a (journey, time-bin) segment (shard starts included)
__device__ __forceinline__ bool seg_start(const Spec& g, const i64* jid, const i64* ts, u64 r, i64 tb)
{
    if (r == 0) return true;
    if (jid[r] != jid[r - 1]) return true;
    if (tb != time_bin(g, ts[r - 1])) return true;
    return g.S > 1 && shard_start(g.soff, g.S, r);
}

__global__ void __launch_bounds__(256) k_grid_clear(GEntry* __restrict__ tab, u64 slots, GridMeta* meta)
{
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < slots; i += (u64)gridDim.x * blockDim.x) {
        GEntry e;
        e.key = GEMPTY;
        for (int c = 0; c < CS40; ++c) e.cs[c] = 0;
        e.count = 0;
        e.nj = 0;
        e.mn = ~0u;
        e.mx = 0;
        tab[i] = e;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        GridMeta z = {};
        *meta = z;
    }
}

__device__ __forceinline__ void g_merge(GEntry& e, u32 count, u32 nj, const Fx192& sum, u32 mn, u32 mx)
{
    u64 c[CS40];
    fx_to_cs40(sum, c);
    for (int i = 0; i < CS40; ++i)
        if (c[i]) __hip_atomic_fetch_add(&e.cs[i], c[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // count and distinct journeys are adjacent words: one 64-bit add carries
    // both (a count stays below 2^32, so nothing crosses into nj)
    static_assert(offsetof(GEntry, nj) == offsetof(GEntry, count) + 4 && offsetof(GEntry, count) % 8 == 0,
                  "count and nj form one aligned 64-bit word");
    __hip_atomic_fetch_add(reinterpret_cast<u64*>(&e.count), (u64)count | ((u64)nj << 32), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_min(&e.mn, mn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_max(&e.mx, mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Probe limit of the HBM table.  Tables are sized to at most half full, where
// linear-probing runs are a few slots long; a table that is (nearly) full
// reports overflow after this many probes instead of scanning all its slots.
constexpr u64 G_PROBES = 4096;

__device__ __forceinline__ void g_insert(GEntry* tab, u64 mask, GridMeta* meta, u64 key, u32 count, u32 nj,
                                         const Fx192& sum, u32 mn, u32 mx)
{
    u64 h = mix64(key) & mask;
    for (u64 probe = 0; probe <= mask && probe < G_PROBES; ++probe) {
        u64 cur = tab[h].key;
        if (cur == key) {
            g_merge(tab[h], count, nj, sum, mn, mx);
            return;
        }
        if (cur == GEMPTY) {
            u64 prev = atomicCAS((unsigned long long*)&tab[h].key, (unsigned long long)GEMPTY, (unsigned long long)key);
            if (prev == GEMPTY || prev == key) {
                g_merge(tab[h], count, nj, sum, mn, mx);
                return;
            }
        }
        h = (h + 1) & mask;
    }
    atomicOr(&meta->overflow, 1u);
}

// each block compacts CSLOTS consecutive slots with one global atomic for its
// base; the order of the pairs is irrelevant (they are sorted by key next)
constexpr int CPT = 16;
constexpr int CSLOTS = 256 * CPT;

__global__ void __launch_bounds__(256) k_grid_compact(const GEntry* __restrict__ tab, u64 slots, GridMeta* meta,
                                                      u64* __restrict__ ckeys, u32* __restrict__ cvals)
{
    __shared__ u32 s_tmp[256 / WAVE];
    __shared__ u64 s_kmax[256 / WAVE];
    __shared__ u32 s_base;
    const u64 s0 = (u64)blockIdx.x * CSLOTS + (u64)threadIdx.x * CPT;
    u64 k[CPT];
    u32 c = 0;
    u64 kmax = 0;
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const u64 s = s0 + i;
        k[i] = s < slots ? tab[s].key : GEMPTY;
        c += k[i] != GEMPTY;
        if (k[i] != GEMPTY && k[i] > kmax) kmax = k[i];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const u64 o = __shfl_xor(kmax, d, WAVE);
        kmax = o > kmax ? o : kmax;
    }
    if (lane_id() == 0) s_kmax[threadIdx.x / WAVE] = kmax;
    u32 tot;
    const u32 e = block_exclusive_sum<256>(c, s_tmp, tot);
    if (threadIdx.x == 0) {
        s_base = tot ? atomicAdd(&meta->compact_n, tot) : 0u;
        u64 m = 0;
        for (int w = 0; w < 256 / WAVE; ++w) m = s_kmax[w] > m ? s_kmax[w] : m;
        if (m) atomicMax((unsigned long long*)&meta->max_key, (unsigned long long)m);
    }
    __syncthreads();
    u32 pos = s_base + e;
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        if (k[i] != GEMPTY) {
            ckeys[pos] = k[i];
            cvals[pos] = (u32)(s0 + i);
            ++pos;
        }
    }
}

__global__ void k_grid_bits(GridMeta* meta)
{
    if (threadIdx.x != 0) return;
    u64 mk = meta->max_key;
    u32 b = mk ? 64u - (u32)__clzll((long long)mk) : 0u;
    meta->key_bits = b;
    meta->passes = (b + RADIX_BITS - 1) / RADIX_BITS;
}

__global__ void __launch_bounds__(256) k_grid_emit(const GEntry* __restrict__ tab, const GridMeta* meta,
                                                   const u64* __restrict__ K0, const u64* __restrict__ K1,
                                                   const u32* __restrict__ V0, const u32* __restrict__ V1, u32 cap,
                                                   i64* __restrict__ o_key, u32* __restrict__ o_cnt,
                                                   u32* __restrict__ o_nj, double* __restrict__ o_sum,
                                                   float* __restrict__ o_min, float* __restrict__ o_max,
                                                   cv_result* res, u64 kmask)
{
    const u32 G = meta->compact_n;
    const u32 np = meta->passes;
    const u32* V = np == 0 ? V0 : ((np & 1) ? V1 : V0);
    const u64* K = np == 0 ? K0 : ((np & 1) ? K1 : K0);
    (void)K;
    const u32 m = G < cap ? G : cap;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const GEntry& e = tab[V[i]];
        o_key[i] = (i64)(e.key & kmask);
        o_cnt[i] = e.count;
        o_nj[i] = e.nj;
        o_sum[i] = fx_to_double<FX_SPD>(fx_from_cs40(e.cs));
        o_min[i] = unord_f32(e.mn);
        o_max[i] = unord_f32(e.mx);
    }
    if (res && blockIdx.x == 0 && threadIdx.x == 0) {
        cv_result r = {};
        const bool full = meta->overflow != 0;  // HBM table full: G is only a lower bound
        const bool over = full || G > cap;
        r.status = over ? CV_ERR_CAPACITY : CV_OK;
        r.count = G;
        if (full) r.required = ((u64)G + 1 > 2ull * cap) ? (u64)G + 1 : 2ull * cap;  // G: a lower bound
        else if (over) r.required = G;
        r.n_out_of_grid = meta->n_out;
        r.key_bits = meta->key_bits;
        *res = r;
    }
}

__attribute__((unused)) __global__ void k_grid_empty(cv_result* res)
{
    if (threadIdx.x == 0) {
        cv_result r = {};
        *res = r;
    }
}

// identity-permutation fill used when the group keys need no radix pass
__global__ void __launch_bounds__(256) k_iota_if_nopass(const GridMeta* meta, const u32* __restrict__ cvals,
                                                        u32* __restrict__ V0, u32 slots)
{
    if (meta->passes != 0) return;
    u32 G = meta->compact_n;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < G && i < slots; i += gridDim.x * blockDim.x)
        V0[i] = cvals[i];
}


}  // namespace
}  // namespace cv
