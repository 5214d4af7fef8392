// cv_sort.hip -- cv_sort_records: stable order of raw records by
// (journey id, timestamp), the paper's unique index over all journeys
// (Methods, step (2)).
//
// Pipeline (all stream-ordered, no host synchronisation):
//   1. k_dict_insert  min/max timestamp; whether time never decreases within a
//                     shard in input order (then the key needs no time bits);
//                     the time offsets' common factor 2^a 5^b; distinct
//                     journey ids into an open-addressing hash set
//                     (run-deduplicated), batched: each id's slot tagged with
//                     its shard, an id met in two shards flagged;
//   2. k_dict_compact distinct ids -> list; radix sort of the list (signed order);
//   3. k_dict_meta    journey count J, rank bits, time bits, key bits, passes;
//   4. k_dict_rank    dense order-preserving rank of each distinct id; batched:
//                     k_dict_shardkey + a stable sort by shard + k_dict_final,
//                     ranks in (shard, id) order (the shard then needs no
//                     bits of its own in the key unless an id spans shards);
//   5. k_pack_hist / k_pack_il
//                     key = rank << t_bits | (ts - t_min) / factor (or the
//                     rank alone for time-ordered input) and the digit
//                     histograms of every radix pass in the same read; for
//                     interleaved input k_pack_il also regroups each tile by
//                     journey and packs the payload per record;
//   6. radix passes   ceil(key_bits / 8) stable scatter passes, one less with a
//                     9-bit first digit for a key of 8k + 1 bits (skipped on device);
//   7. k_gather / k_gather_feat
//                     perm, journey id from the dictionary, ts from the key
//                     when it survives packing, lat/lon/speed through perm or
//                     from the packed payload; k_gather_feat adds the
//                     kinematics.
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_host.h"
#include "cv_kin.h"
#include "cv_radix.h"

using namespace cv;

namespace {

constexpr u64 EMPTY = 0x8000000000000000ull;  // INT64_MIN marks an empty slot
constexpr u64 SIGN = 0x8000000000000000ull;

struct SortMeta {
    u64 tmin_ord;
    u64 tmax_ord;
    u32 n_distinct;
    u32 has_min;
    u32 overflow;
    u32 J;
    u32 list_count;
    u32 dict_n;
    u32 rank_bits;
    u32 t_bits;
    u32 key_bits;
    u32 passes;
    u32 range_err;
    u32 shard_bits;
    u32 ib;   // index bits of a packed key word
    u32 p0;   // first pass whose input words are packed (ib and p0 adjacent: the radix passes read both)
    u32 w0;   // bits of the first radix digit: 9 where that saves a pass (a key of 8k + 1 bits), else 8
    u32 n_runs;  // runs of equal ids in input order (counted by the dictionary insert)
    u32 unordered;  // a timestamp below its predecessor's (same shard) in input order
    u32 ts_dropped; // key = (shard, rank) only: the input is time-ordered within every shard
    u32 multi_shard; // batched: an id in more than one shard (ranks then in id order, shard bits in the key)
    u32 t_nd5;       // bit b: some time offset is not a multiple of 5^(b+1) (b < 3)
    u64 t_or;        // OR of every |ts - ts[0]|: its trailing zeros are the offsets' common power of two
    u32 t_sh;        // the key's time offset is (ts - t_min) / (2^t_sh * t_p5): the offsets'
    u32 t_p5;        //   common factor of the form 2^a 5^b (b <= 3), e.g. 1000 for 1 Hz in ms
    u32 tickets[3 * MAX_PASSES];
};

__device__ __forceinline__ u32 bit_width64(u64 x) { return x ? 64u - (u32)__clzll((long long)x) : 0u; }

__global__ void k_sort_init(SortMeta* m)
{
    if (threadIdx.x == 0) {
        SortMeta z = {};
        z.tmin_ord = ~0ull;
        z.tmax_ord = 0;
        *m = z;
    }
}

// The dictionary is an open-addressing table of 16-byte slots {id, rank}:
// the id word is claimed by CAS (EMPTY when free) and the rank word is filled
// in once the distinct ids are sorted, so that one 16-byte load per probe
// returns both.  An insert probes linearly from mix64(id); the caller reads the
// first slot (so that the first probes of many records are in flight
// together) and this continues from it.
__device__ __forceinline__ bool dict_insert_from(u64* table, u64 mask, u64 key, u64 h, u64 cur)
{
    for (u64 probe = 0; probe <= mask; ++probe) {
        if (cur == key) return true;
        if (cur == EMPTY) {
            u64 prev =
                atomicCAS((unsigned long long*)&table[2 * h], (unsigned long long)EMPTY, (unsigned long long)key);
            if (prev == EMPTY || prev == key) return true;
        }
        h = (h + 1) & mask;
        cur = table[2 * h];
    }
    return false;
}

// Batched form: the insert of `key` for shard `sh`, continuing a probe at slot
// h whose entry e was read, also tags the slot's second word with the shard.
// A slot tagged with another shard means the id lies in two shards (multi).
// Both the inserter and a reader that finds the slot untagged tag it by
// compare-and-swap, so exactly one shard wins and any other sees it.
// Returns false when the table is full.
__device__ __forceinline__ bool dict_insert_tag(u64* table, u64 mask, u64 key, u64 h, ulonglong2 e, u64 sh,
                                                bool& multi)
{
    const ulonglong2* t2 = (const ulonglong2*)table;
    for (u64 probe = 0; probe <= mask; ++probe) {
        bool mine = e.x == key;
        if (!mine && e.x == EMPTY) {
            const u64 prev =
                atomicCAS((unsigned long long*)&table[2 * h], (unsigned long long)EMPTY, (unsigned long long)key);
            mine = prev == EMPTY || prev == key;
            e.y = EMPTY;  // (re)tag below by compare-and-swap
        }
        if (mine) {
            if (e.y != sh) {
                const u64 old = atomicCAS((unsigned long long*)&table[2 * h + 1], (unsigned long long)EMPTY,
                                          (unsigned long long)sh);
                if (old != EMPTY && old != sh) multi = true;
            }
            return true;
        }
        h = (h + 1) & mask;
        e = t2[h];
    }
    return false;
}

// slot of `key`, or ~0 when absent
__device__ __forceinline__ u64 dict_find(const u64* table, u64 mask, u64 key)
{
    u64 h = mix64(key) & mask;
    for (u64 probe = 0; probe <= mask; ++probe) {
        u64 cur = table[2 * h];
        if (cur == key) return h;
        if (cur == EMPTY) return ~0ull;
        h = (h + 1) & mask;
    }
    return ~0ull;
}

// rank of `key` (0 when absent), one 16-byte load per probe
__device__ __forceinline__ u32 dict_rank_of(const u64* table, u64 mask, u64 key)
{
    const ulonglong2* t2 = (const ulonglong2*)table;
    u64 h = mix64(key) & mask;
    for (u64 probe = 0; probe <= mask; ++probe) {
        const ulonglong2 e = t2[h];
        if (e.x == key) return (u32)e.y;
        if (e.x == EMPTY) return 0u;
        h = (h + 1) & mask;
    }
    return 0u;
}

// Each wave of the dictionary kernels walks its own contiguous range of
// windows of 64 records and keeps the ids it met last in a small LDS cache
// (direct-mapped, DC slots per wave): in time-ordered input, where many
// journeys interleave, a window's ids mostly appeared in the windows just
// before, and the cache spares those records the probe of the global table.
// A slot is written by one lane only (the lanes that miss on a slot elect
// one through the owner word), so an entry is never a mix of two writes.
constexpr int DC = 512;   // slots per wave in the insert (24 KB of LDS per workgroup; 256: 0.3 ms slower on
                          // the interleaved batched feed)
constexpr int DCH = 128;  // slots per wave in the key packing for input in long runs (16 KB with the histograms)
constexpr int DCP = 256;  // slots per wave in the interleaved key packing (its 1 024-thread workgroups are
                          // one per CU at their register count, whatever the LDS)
constexpr int DPW = 4;  // windows whose ids and times are loaded together (plain form: 90 VGPRs, 5 waves per SIMD)

__device__ __forceinline__ void wave_range(u32 n, u64& wbeg, u64& wend)
{
    const u64 nw = (u64)gridDim.x * (blockDim.x / WAVE);
    const u64 nwin = ((u64)n + WAVE - 1) / WAVE;
    const u64 per = (nwin + nw - 1) / nw;
    wbeg = ((u64)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE) * per;
    wend = wbeg + per < nwin ? wbeg + per : nwin;
}

template <int C>
__device__ __forceinline__ u32 dict_cache_slot(u64 key)
{
    static_assert((C & (C - 1)) == 0 && C <= 4096, "power of two");
    return (u32)(mix64(key) >> (64 - __builtin_ctz(C)));  // the hash's top bits
}

// bits 0..2: |d| not a multiple of 5, 25, 125
__device__ __forceinline__ u32 not_div5(u64 ad)
{
    if ((ad >> 32) == 0) {
        const u32 x = (u32)ad;
        return (x % 5u ? 1u : 0u) | (x % 25u ? 2u : 0u) | (x % 125u ? 4u : 0u);
    }
    return (ad % 5ull ? 1u : 0u) | (ad % 25ull ? 2u : 0u) | (ad % 125ull ? 4u : 0u);
}

// the key's time offset: (ts - t_min) divided by the offsets' common factor
// 2^sh 5^b (exact: every offset is a multiple of it)
__device__ __forceinline__ u64 time_offset(u64 toff, u32 sh, u32 p5)
{
    u64 q = toff >> sh;
    if (p5 == 5) q /= 5ull;
    else if (p5 == 25) q /= 25ull;
    else if (p5 == 125) q /= 125ull;
    return q;
}

// Also checks whether the timestamps never decrease within a shard in input
// order: then every journey's records already come in time order, and a
// stable sort by (shard, journey) alone gives the (journey, time) order.
// SHARDS (the batched form) also tags every id's slot with its shard and
// flags an id met in two shards; a run of equal ids then ends at a shard
// start, and a round of windows that meets a shard start or a shard other
// than the one its wave's cache was filled in bypasses the cache (whose
// entries would skip the shard check) and empties it.
template <bool SHARDS>
__global__ void __launch_bounds__(256) k_dict_insert(const i64* __restrict__ jid, const i64* __restrict__ ts, u32 n,
                                                     u64* __restrict__ table, u64 mask, SortMeta* m,
                                                     const u64* __restrict__ soff, u32 S)
{
    // (the batched form's 16-byte probes and shard checks take it to 4 waves
    // per SIMD, with 3 windows per round as with 4)
    constexpr int DP = DPW;
    __shared__ u64 s_min[4], s_max[4];
    __shared__ u64 c_key[4][DC];
    __shared__ u32 c_own[4][DC];
    const int w = threadIdx.x / WAVE;
    const int l = lane_id();
    for (int i = l; i < DC; i += WAVE) c_key[w][i] = EMPTY;  // EMPTY is never looked up
    u64 lo = ~0ull, hi = 0;
    bool has_min = false, full = false, multi = false;
    u64 wbeg, wend;
    wave_range(n, wbeg, wend);
    i64 prevj = 0;  // last id of the previous window
    bool hp = false;
    u32 runs = 0;   // records that start a run of equal ids (wave-uniform)
    // time of the record before the range (ordered form), then of each window's last
    u64 prevt = (wbeg < wend && wbeg > 0) ? ord_i64(ts[wbeg * WAVE - 1]) : 0ull;
    bool down = false;
    u32 shk = (S > 1 && wbeg < wend) ? shard_lower_bound(soff, S, wbeg * WAVE) : 0u;
    u32 csh = ~0u;  // the shard the wave's cache entries were met in (SHARDS)
    // the time offsets' common factor: every |ts - ts[0]| ORed together (its
    // trailing zeros) and which powers of five fail to divide one
    const u64 t0r = n ? ord_i64(ts[0]) : 0ull;
    u64 tor = 0;
    u32 nd5 = 0;
    for (u64 w0 = wbeg; w0 < wend; w0 += DP) {
        i64 jv[DP];
        u64 tv[DP];
#pragma unroll
        for (int k = 0; k < DP; ++k) {
            u64 i = (w0 + k) * WAVE + l;
            i = i < n ? i : (u64)n - 1;  // past the end: a valid record, not used
            jv[k] = jid[i];
            tv[k] = ord_i64(ts[i]);
        }
        // shard starts of each window (lane masks) and the window's shard
        // when none starts inside it (~0 otherwise); wave-uniform
        u64 starts[DP];
        u32 wsh[DP];
        bool byp = false;
#pragma unroll
        for (int k = 0; k < DP; ++k) {
            starts[k] = 0;
            wsh[k] = 0;
            if (S > 1 && w0 + k < wend) {
                const u32 k0 = __builtin_amdgcn_readfirstlane(shk);
                bool at_end = false;
                starts[k] = shard_starts_in(soff, S, shk, (w0 + k) * WAVE, at_end);
                wsh[k] = starts[k] ? ~0u : k0 - 1;
                if (SHARDS) byp |= wsh[k] != csh || wsh[k] == ~0u;
            }
        }
        if (SHARDS && byp) {
            for (int i = l; i < DC; i += WAVE) c_key[w][i] = EMPTY;
            __builtin_amdgcn_wave_barrier();
        }
        // first the run starts of every window and, for each that misses the
        // cache, the first probe, issued together; then the inserts in order
        bool miss[DP];
        u64 ph[DP];
        ulonglong2 pe[DP];
#pragma unroll
        for (int k = 0; k < DP; ++k) {
            miss[k] = false;
            if (w0 + k >= wend) continue;
            const u64 i = (w0 + k) * WAVE + l;
            const bool valid = i < n;
            const i64 j = jv[k];
            if (valid) {
                lo = tv[k] < lo ? tv[k] : lo;
                hi = tv[k] > hi ? tv[k] : hi;
                const u64 d = tv[k] - t0r;  // ts - ts[0] modulo 2^64 (the order map adds the same 2^63)
                const u64 ad = (i64)d < 0 ? 0ull - d : d;
                tor |= ad;
                if (nd5 != 7u) nd5 |= not_div5(ad);
            }
            const bool sstart = (starts[k] >> l) & 1ull;
            {
                // time order against the record before (none before record 0
                // and before a shard's first record)
                const u64 tp = __shfl_up(tv[k], 1, WAVE);
                const u64 tq = l == 0 ? prevt : tp;
                if (valid && i > 0 && !sstart && tv[k] < tq) down = true;
                prevt = __shfl(tv[k], WAVE - 1, WAVE);
            }
            // a record repeating the id before it adds nothing (in the
            // batched form, unless a shard starts at it)
            const i64 jp = __shfl_up(j, 1, WAVE);
            const bool dup = (l == 0 ? (hp && j == prevj) : j == jp) && !(SHARDS && sstart);
            prevj = __shfl(j, WAVE - 1, WAVE);
            hp = true;
            bool need = valid && !dup;
            runs += (u32)__popcll(__ballot(need));
            if (need && (u64)j == EMPTY) {
                has_min = true;
                need = false;
            }
            const u32 cs = dict_cache_slot<DC>((u64)j);
            miss[k] = need && ((SHARDS && byp) || c_key[w][cs] != (u64)j);
            ph[k] = mix64((u64)j) & mask;
            if (SHARDS) {
                if (miss[k]) pe[k] = ((const ulonglong2*)table)[ph[k]];
            } else if (miss[k]) {
                pe[k].x = table[2 * ph[k]];
            }
        }
#pragma unroll
        for (int k = 0; k < DP; ++k) {
            if (w0 + k >= wend) break;
            const u64 j = (u64)jv[k];
            const u32 cs = dict_cache_slot<DC>(j);
            if (SHARDS) {
                if (miss[k]) {
                    // the record's shard: the window's, or searched where a shard starts inside it
                    const u64 i = (w0 + k) * WAVE + l;
                    const u32 sh = wsh[k] != ~0u ? wsh[k] : shard_of(soff, S, i < n ? i : (u64)n - 1);
                    if (!dict_insert_tag(table, mask, j, ph[k], pe[k], (u64)sh, multi)) full = true;
                }
            } else if (miss[k] && !dict_insert_from(table, mask, j, ph[k], pe[k].x)) {
                full = true;
            }
            if (miss[k]) c_own[w][cs] = (u32)l;
            __builtin_amdgcn_wave_barrier();
            if (miss[k] && c_own[w][cs] == (u32)l) c_key[w][cs] = j;
            __builtin_amdgcn_wave_barrier();
        }
        if (SHARDS && byp) {
            // the entries just cached may come from several shards: start over
            // in the shard of the round's last window (none when a shard
            // starts inside it)
            for (int i = l; i < DC; i += WAVE) c_key[w][i] = EMPTY;
            __builtin_amdgcn_wave_barrier();
            u32 last = ~0u;
#pragma unroll
            for (int k = 0; k < DP; ++k)
                if (w0 + k < wend) last = wsh[k];
            csh = last;
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        u64 a = __shfl_xor(lo, d, WAVE), b = __shfl_xor(hi, d, WAVE);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if (l == 0) {
        s_min[w] = lo;
        s_max[w] = hi;
    }
    if (has_min) atomicOr(&m->has_min, 1u);
    if (full) atomicOr(&m->overflow, 1u);
    if (SHARDS && __ballot(multi) && l == 0) atomicOr(&m->multi_shard, 1u);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        tor |= __shfl_xor(tor, d, WAVE);
        nd5 |= __shfl_xor(nd5, d, WAVE);
    }
    if (l == 0) {
        if (tor) atomicOr((unsigned long long*)&m->t_or, (unsigned long long)tor);
        if (nd5) atomicOr(&m->t_nd5, nd5);
    }
    if (__ballot(down) && l == 0) atomicOr(&m->unordered, 1u);
    if (runs && l == 0) atomicAdd(&m->n_runs, runs);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x / WAVE); ++k) {
            lo = s_min[k] < lo ? s_min[k] : lo;
            hi = s_max[k] > hi ? s_max[k] : hi;
        }
        if (lo != ~0ull) atomicMin((unsigned long long*)&m->tmin_ord, (unsigned long long)lo);
        if (hi != 0) atomicMax((unsigned long long*)&m->tmax_ord, (unsigned long long)hi);
    }
}

__global__ void __launch_bounds__(256) k_dict_compact(const u64* __restrict__ table, u64 slots, u32 max_j,
                                                      SortMeta* m, u64* __restrict__ list)
{
    // one counter claim per workgroup and round (the list is sorted afterwards,
    // so the order of the claims does not matter)
    __shared__ u32 s_wc[256 / WAVE];
    __shared__ u32 s_base;
    u32 hm = m->has_min;
    if (blockIdx.x == 0 && threadIdx.x == 0 && hm && max_j > 0) list[0] = EMPTY ^ SIGN;
    const int w = threadIdx.x / WAVE;
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 b = (u64)blockIdx.x * blockDim.x; b < slots; b += stride) {
        const u64 s = b + threadIdx.x;
        const u64 k = s < slots ? table[2 * s] : EMPTY;
        const bool occ = k != EMPTY;
        const u64 msk = __ballot(occ);
        if (lane_id() == 0) s_wc[w] = (u32)__popcll(msk);
        __syncthreads();
        if (threadIdx.x == 0) {
            u32 t = 0;
            for (int x = 0; x < 256 / WAVE; ++x) t += s_wc[x];
            s_base = t ? atomicAdd(&m->list_count, t) : 0u;
        }
        __syncthreads();
        u32 base = s_base;
        for (int x = 0; x < w; ++x) base += s_wc[x];
        if (occ) {
            const u32 pos = base + popc_below(msk) + hm;
            if (pos < max_j) list[pos] = k ^ SIGN;
        }
        __syncthreads();
    }
}

__global__ void k_dict_meta(SortMeta* m, u32 max_j, u32 n, u32 n_shards, u32 allow_wide)
{
    if (threadIdx.x != 0) return;
    u32 J = m->list_count + m->has_min;  // distinct ids counted by the compaction
    m->J = J;
    if (J > max_j) m->overflow = 1;
    m->dict_n = J < max_j ? J : max_j;
    u32 rb = J > 1 ? bit_width64((u64)J - 1) : 0;
    u64 span = n ? (unord_i64(m->tmax_ord) - (u64)unord_i64(m->tmin_ord)) : 0;
    // the offsets' common factor 2^a 5^b (1 when the time stamps are all equal)
    u32 a = m->t_or ? (u32)__ffsll((long long)m->t_or) - 1u : 0u;
    u32 p5 = (m->t_nd5 & 1u) ? 1u : (m->t_nd5 & 2u) ? 5u : (m->t_nd5 & 4u) ? 25u : 125u;
    if (!m->t_or) p5 = 1;
    m->t_sh = a;
    m->t_p5 = p5;
    span = (span >> a) / p5;
    // time-ordered input needs no time bits in the key (see the insert)
    m->ts_dropped = m->unordered ? 0u : 1u;
    u32 tb = m->ts_dropped ? 0u : bit_width64(span);
    // batched: when every id lies in one shard, ranks follow (shard, id) order
    // and already keep the shards apart; otherwise the shard goes above them
    // (the INT64_MIN id, which is never in the table, counts as such a case)
    if (n_shards > 1 && m->has_min) m->multi_shard = 1;
    const u32 sb = (n_shards > 1 && m->multi_shard) ? bit_width64((u64)n_shards - 1) : 0;
    m->rank_bits = rb;
    m->t_bits = tb;
    m->shard_bits = sb;
    u32 kb = sb + rb + tb;
    if (kb > 64) {
        m->range_err = 1;
        kb = 0;
    }
    m->key_bits = kb;
    // Packed words (key >> 8 p0) << ib | index replace the (key, index) pairs
    // from pass p0 on; p0 is the first digit boundary from which the rest of
    // the key and the index fit one word.  p0 < passes whenever p0 > 0.
    const u32 ib = n > 1 ? bit_width64((u64)n - 1) : 1u;
    m->ib = ib;
    const u32 p0 = kb + ib > 64 ? (kb + ib - 64 + RADIX_BITS - 1) / RADIX_BITS : 0u;
    m->p0 = p0;
    // a key of 8k + 1 bits, packed from the first pass, takes a 9-bit first
    // digit and k passes instead of k + 1
    const u32 w0 = (allow_wide && p0 == 0 && kb > RADIX_BITS && kb % RADIX_BITS == 1) ? RADIX_BITS + 1 : RADIX_BITS;
    m->w0 = w0;
    m->passes = kb == 0 ? 0u : (kb <= w0 ? 1u : 1u + (kb - w0 + RADIX_BITS - 1) / RADIX_BITS);
}

// Batched form, after the distinct ids are sorted: each id's shard (its slot's
// tag) as the key of a stable sort that brings the list into (shard, id)
// order; 0 for every id when an id lies in several shards, so that the list
// keeps id order.
__global__ void __launch_bounds__(256) k_dict_shardkey(const u64* __restrict__ sorted_list, const SortMeta* m,
                                                       const u64* __restrict__ table, u64 mask, u64* __restrict__ skey)
{
    const u32 dn = m->dict_n;
    const bool multi = m->multi_shard != 0;
    for (u32 r = blockIdx.x * blockDim.x + threadIdx.x; r < dn; r += gridDim.x * blockDim.x) {
        const u64 k = sorted_list[r] ^ SIGN;
        u64 sh = 0;
        if (!multi && k != EMPTY) {
            const u64 slot = dict_find(table, mask, k);
            sh = slot != ~0ull ? table[2 * slot + 1] : 0ull;
        }
        skey[r] = sh;
    }
}

// Batched form: the list in (shard, id) order (perm: the stable sort's order of
// the id-sorted list) and each id's rank, its position in that order.
__global__ void __launch_bounds__(256) k_dict_final(const u64* __restrict__ sorted_list, const u32* __restrict__ perm,
                                                    const SortMeta* m, u64* __restrict__ table, u64 mask,
                                                    u64* __restrict__ final_list)
{
    const u32 dn = m->dict_n;
    for (u32 r = blockIdx.x * blockDim.x + threadIdx.x; r < dn; r += gridDim.x * blockDim.x) {
        const u64 v = sorted_list[perm[r]];
        final_list[r] = v;
        const u64 k = v ^ SIGN;
        if (k == EMPTY) continue;
        const u64 slot = dict_find(table, mask, k);
        if (slot != ~0ull) table[2 * slot + 1] = r;
    }
}

__global__ void __launch_bounds__(256) k_dict_rank(const u64* __restrict__ sorted_list, const SortMeta* m,
                                                   u64* __restrict__ table, u64 mask)
{
    u32 dn = m->dict_n;
    for (u32 r = blockIdx.x * blockDim.x + threadIdx.x; r < dn; r += gridDim.x * blockDim.x) {
        u64 k = sorted_list[r] ^ SIGN;
        if (k == EMPTY) continue;
        u64 s = dict_find(table, mask, k);
        if (s != ~0ull) table[2 * s + 1] = r;
    }
}

// Waves walk contiguous windows of 64 records, so the journey-rank digits of a
// window are usually equal in every lane: such a digit is counted with one LDS
// add instead of 64 colliding ones.
// Each wave walks its own contiguous range of windows of 64 records, PW
// windows per round with their ids and times loaded together; the (id, rank)
// of a window's last record carries into the next window, so the dictionary
// is probed only where a run of equal ids starts, and the shard (batched form)
// is followed forward from the range's first one.  SHARDS = false compiles the
// plain form without the shard search.
// One input record's payload, packed (the gather's form for interleaved input).
struct __attribute__((aligned(32))) PayRec {
    i64 ts;
    double lat, lon;
    float spd;
    u32 pad;
};

// Input whose runs of equal journey ids are short (journeys interleaved, as in
// a time-ordered feed) sends the gather through the sort's index to a separate
// memory segment per record and column; for such input the payload columns
// are first packed per record, so that the gather reads one 32-byte record.
constexpr u64 PAY_MIN_RUN = 8;  // mean run length below which the packed form is used
__device__ __forceinline__ bool pay_packed(const SortMeta* m, u32 n) { return (u64)m->n_runs * PAY_MIN_RUN > n; }

// rank of `key` continuing a probe sequence at slot h, whose entry e was read
__device__ __forceinline__ u32 dict_rank_from(const u64* table, u64 mask, u64 key, u64 h, ulonglong2 e)
{
    const ulonglong2* t2 = (const ulonglong2*)table;
    for (u64 probe = 0; probe <= mask; ++probe) {
        if (e.x == key) return (u32)e.y;
        if (e.x == EMPTY) return 0u;
        h = (h + 1) & mask;
        e = t2[h];
    }
    return 0u;
}

constexpr int PW = 8;
// Keys of every record with the digit histograms of every pass, for input in
// long runs of equal ids: each wave walks its own contiguous range of windows
// of 64 records, PW windows per round with their ids and times loaded
// together; the (id, rank) of a window's last record carries into the next
// window, so the dictionary is probed only where a run of equal ids starts
// (through the wave's cache), and the shard (batched form) is followed
// forward from the range's first one.  Returns at once for interleaved input
// (k_pack_il takes it).
template <bool SHARDS>
__global__ void __launch_bounds__(256) k_pack_hist(const i64* __restrict__ jid, const i64* __restrict__ ts, u32 n,
                                                   const u64* __restrict__ table, u64 mask, SortMeta* m,
                                                   u64* __restrict__ keys, u32* __restrict__ hist,
                                                   const u64* __restrict__ soff, u32 S)
{
    __shared__ u32 s_h[HIST_WIDE_WORDS];  // digit counts, wide layout (first digit w0 bits)
    // per-wave cache of (id, rank) pairs, as in the dictionary insert
    __shared__ u64 c_key[4][DCH];
    __shared__ u32 c_rank[4][DCH], c_own[4][DCH];
    if (pay_packed(m, n)) return;
    for (int i = threadIdx.x; i < HIST_WIDE_WORDS; i += blockDim.x) s_h[i] = 0;
    for (int i = threadIdx.x; i < 4 * DCH; i += blockDim.x) (&c_key[0][0])[i] = EMPTY;
    __syncthreads();
    const int wv_ = threadIdx.x / WAVE;
    const u32 tb = m->t_bits;
    const bool tdrop = m->ts_dropped != 0;
    const u32 np = m->passes;
    const u32 fdb = m->w0 == RADIX_BITS + 1 ? RADIX_BITS + 1 : RADIX_BITS;  // first digit bits
    const bool bad = m->range_err != 0;
    const u32 ib = m->ib;
    const bool packed = m->p0 == 0;
    const u64 tmin = (u64)unord_i64(m->tmin_ord);
    const u32 tsh = m->t_sh, tp5 = m->t_p5;
    const int l = lane_id();
    const u64 nw = (u64)gridDim.x * (blockDim.x / WAVE);
    const u64 nwin = ((u64)n + WAVE - 1) / WAVE;
    const u64 per = ((nwin + nw - 1) / nw + PW - 1) / PW * PW;  // windows per wave, whole rounds
    const u64 wbeg = ((u64)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE) * per;
    const u64 wend = wbeg + per < nwin ? wbeg + per : nwin;
    // id and rank of the previous window's last record
    bool hc = false;
    u64 cj = 0;
    u32 cr = 0;
    // shard of the current window's first record (batched form; wave-uniform)
    u32 shw = (SHARDS && wbeg < wend) ? shard_of(soff, S, wbeg * WAVE) : 0u;
    for (u64 w0 = wbeg; w0 < wend; w0 += PW) {
        u64 jv[PW], tv[PW];
#pragma unroll
        for (int k = 0; k < PW; ++k) {
            u64 i = (w0 + k) * WAVE + l;
            i = i < n ? i : (u64)n - 1;  // past the end: a valid record, not used
            jv[k] = (u64)jid[i];
            tv[k] = (u64)ts[i];
        }
#pragma unroll
        for (int k = 0; k < PW; ++k) {
            const u64 wi = w0 + k;
            if (wi >= wend) break;
            const u64 i = wi * WAVE + l;
            const bool valid = i < n;
            // only the first lane of each run of equal ids probes the dictionary;
            // the others take its rank (lane 0 continues the carried run)
            const u64 j = valid ? jv[k] : EMPTY;
            const u64 jp = __shfl_up(j, 1, WAVE);
            const bool runhead = l == 0 ? !(hc && j == cj) : j != jp;
            u32 r = 0;
            const bool look = valid && runhead && j != EMPTY;
            const u32 cs = dict_cache_slot<DCH>(j);
            bool miss = false;
            if (look) {
                if (c_key[wv_][cs] == j) {
                    r = c_rank[wv_][cs];
                } else {
                    r = dict_rank_of(table, mask, j);
                    miss = true;
                }
            }
            if (miss) c_own[wv_][cs] = (u32)l;
            __builtin_amdgcn_wave_barrier();
            if (miss && c_own[wv_][cs] == (u32)l) {
                c_key[wv_][cs] = j;
                c_rank[wv_][cs] = r;
            }
            __builtin_amdgcn_wave_barrier();
            const u64 heads = __ballot(runhead);
            const u64 upto = heads & (~0ull >> (63 - l));  // run starts at or below this lane
            const u32 rh = __shfl(r, upto ? 63 - __clzll((long long)upto) : 0, WAVE);
            r = upto ? rh : cr;
            cj = __shfl(j, WAVE - 1, WAVE);
            cr = __shfl(r, WAVE - 1, WAVE);
            hc = true;
            u64 key = 0;
            if (valid) {
                if (!bad) {
                    key = tdrop ? (u64)r : ((tb >= 64 ? 0ull : ((u64)r << tb)) | time_offset(tv[k] - tmin, tsh, tp5));
                    if (SHARDS && m->shard_bits) {
                        // the window's first shard, then forward to this record's
                        shw = __builtin_amdgcn_readfirstlane(shard_from(soff, S, shw, wi * WAVE));
                        const u32 sh = shard_from(soff, S, shw, i);
                        key |= (u64)sh << (m->rank_bits + tb);
                    }
                }
                keys[i] = packed ? ((key << ib) | i) : key;
            }
            const u64 vm = __ballot(valid);
            const int lead = __ffsll((long long)vm) - 1;
            for (u32 p = 0; p < np; ++p) {
                const u32 lo = p ? fdb + (p - 1) * RADIX_BITS : 0u;
                const u32 d = (u32)(key >> lo) & ((p ? RADIX : 1u << fdb) - 1u);
                u32* hp = s_h + hist_wide_off((int)p);
                const u32 d0 = __shfl(d, lead, WAVE);
                if (__ballot(valid && d != d0) == 0) {
                    if (l == lead) atomicAdd(&hp[d0], (u32)__popcll(vm));
                } else if (valid) {
                    atomicAdd(&hp[d], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (u32 i = threadIdx.x; i < (u32)HIST_WIDE_WORDS; i += blockDim.x)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// Keys and digit histograms for interleaved input (short runs of equal ids, as
// in a time-ordered feed), where nearly every record probes the dictionary:
// every block takes a contiguous range of tiles of PT records, and each
// record's first probe is issued with the tile's others before any is used.
// With `pay` (the fused gather), the tile's records are also regrouped
// by the low byte of their journey rank (a stable local multisplit, so equal
// keys keep their input order): the key words and the packed payloads go to
// the regrouped positions, and each payload carries its input index.  After
// the sort, consecutive records of a journey then read consecutive payloads
// of each tile instead of one cache line per record.
constexpr int PT_B = 1024;               // threads per block (tiles of 4 096 records: half the per-tile scans and barriers of 2 048)
constexpr int PT_I = 4;                  // records per thread
constexpr int PT = PT_B * PT_I;          // records per tile
template <bool SHARDS>
__global__ void __launch_bounds__(PT_B) k_pack_il(const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                 const double* __restrict__ lat, const double* __restrict__ lon,
                                                 const float* __restrict__ spd, PayRec* __restrict__ pay, u32 n,
                                                 const u64* __restrict__ table, u64 mask, SortMeta* m,
                                                 u64* __restrict__ keys, u32* __restrict__ hist,
                                                 const u64* __restrict__ soff, u32 S)
{
    constexpr int NW = PT_B / WAVE;
    __shared__ u32 s_h[HIST_WIDE_WORDS];  // digit counts, wide layout (first digit w0 bits)
    __shared__ u64 c_key[NW][DCP];
    __shared__ u32 c_rank[NW][DCP], c_own[NW][DCP];
    __shared__ uint16_t s_whist[NW][RADIX];  // per-wave digit counts, then offsets
    __shared__ u32 s_start[RADIX];
    __shared__ u32 s_tmp[NW];
    if (!pay_packed(m, n)) return;
    for (int i = threadIdx.x; i < HIST_WIDE_WORDS; i += blockDim.x) s_h[i] = 0;
    for (int i = threadIdx.x; i < NW * DCP; i += blockDim.x) (&c_key[0][0])[i] = EMPTY;
    const int w = threadIdx.x / WAVE;
    const int l = lane_id();
    const u32 tb = m->t_bits;
    const bool tdrop = m->ts_dropped != 0;
    const u32 np = m->passes;
    const u32 fdb = m->w0 == RADIX_BITS + 1 ? RADIX_BITS + 1 : RADIX_BITS;  // first digit bits
    const bool bad = m->range_err != 0;
    const u32 ib = m->ib;
    const bool packed = m->p0 == 0;
    const bool group = pay != nullptr;
    const u32 rbits = m->rank_bits;
    const u32 sbits = m->shard_bits;  // 0: the ranks keep the shards apart
    // without time bits the first digit of a key is the low byte of its rank,
    // which the regrouping counts per tile: that pass's histogram is added
    // from those counts, one add per digit and tile
    const u32 p_first = (group && tdrop && !bad && rbits >= (u32)RADIX_BITS && np > 0 && fdb == RADIX_BITS) ? 1u : 0u;
    const u64 tmin = (u64)unord_i64(m->tmin_ord);
    const u32 tsh = m->t_sh, tp5 = m->t_p5;
    const ulonglong2* t2 = (const ulonglong2*)table;
    const u64 tiles = ((u64)n + PT - 1) / PT;
    const u64 per = (tiles + gridDim.x - 1) / gridDim.x;
    const u64 tb0 = (u64)blockIdx.x * per;
    const u64 tb1 = tb0 + per < tiles ? tb0 + per : tiles;
    u32 shw = (SHARDS && tb0 < tb1) ? shard_of(soff, S, tb0 * PT) : 0u;
    for (u64 tile = tb0; tile < tb1; ++tile) {
        const u64 base = tile * PT + (u64)w * (PT_I * WAVE);  // this wave's 512 records
        for (int i = l; i < RADIX; i += WAVE) s_whist[w][i] = 0;
        __syncthreads();
        u64 jv[PT_I], tv[PT_I];
        double la[PT_I], lo[PT_I];
        float sp[PT_I];
#pragma unroll
        for (int k = 0; k < PT_I; ++k) {
            u64 i = base + (u64)k * WAVE + l;
            i = i < n ? i : (u64)n - 1;  // past the end: a valid record, not used
            jv[k] = (u64)jid[i];
            tv[k] = (u64)ts[i];
            if (group) {
                la[k] = lat[i];
                lo[k] = lon[i];
                sp[k] = spd[i];
            }
        }
        // ranks: the wave's cache, else the first probe of every miss issued together
        u32 rk[PT_I];
        bool miss[PT_I];
        u64 ph[PT_I];
        ulonglong2 pe[PT_I];
#pragma unroll
        for (int k = 0; k < PT_I; ++k) {
            const u64 i = base + (u64)k * WAVE + l;
            const u64 j = jv[k];
            const bool look = i < n && j != EMPTY;  // the INT64_MIN id has rank 0
            const u32 cs = dict_cache_slot<DCP>(j);
            rk[k] = 0;
            miss[k] = false;
            if (look) {
                if (c_key[w][cs] == j) rk[k] = c_rank[w][cs];
                else miss[k] = true;
            }
            ph[k] = mix64(j) & mask;
            if (miss[k]) pe[k] = t2[ph[k]];
        }
#pragma unroll
        for (int k = 0; k < PT_I; ++k) {
            const u64 j = jv[k];
            const u32 cs = dict_cache_slot<DCP>(j);
            if (miss[k]) {
                rk[k] = dict_rank_from(table, mask, j, ph[k], pe[k]);
                c_own[w][cs] = (u32)l;
            }
            __builtin_amdgcn_wave_barrier();
            if (miss[k] && c_own[w][cs] == (u32)l) {
                c_key[w][cs] = j;
                c_rank[w][cs] = rk[k];
            }
            __builtin_amdgcn_wave_barrier();
        }
        // keys, histograms and the local multisplit by the rank's low byte
        u64 key[PT_I];
        u32 rnk[PT_I];
#pragma unroll
        for (int k = 0; k < PT_I; ++k) {
            const u64 i = base + (u64)k * WAVE + l;
            const bool valid = i < n;
            key[k] = 0;
            if (valid && !bad) {
                key[k] = tdrop ? (u64)rk[k] : ((tb >= 64 ? 0ull : ((u64)rk[k] << tb)) | time_offset(tv[k] - tmin, tsh, tp5));
                if (SHARDS && sbits) {
                    shw = __builtin_amdgcn_readfirstlane(shard_from(soff, S, shw, base + (u64)k * WAVE));
                    const u32 sh = shard_from(soff, S, shw, i);
                    key[k] |= (u64)sh << (rbits + tb);
                }
            }
            const u64 vm = __ballot(valid);
            const int lead = vm ? __ffsll((long long)vm) - 1 : 0;
            for (u32 p = p_first; p < np; ++p) {
                const u32 dlo = p ? fdb + (p - 1) * RADIX_BITS : 0u;
                const u32 d = (u32)(key[k] >> dlo) & ((p ? RADIX : 1u << fdb) - 1u);
                u32* hp = s_h + hist_wide_off((int)p);
                const u32 d0 = __shfl(d, lead, WAVE);
                if (__ballot(valid && d != d0) == 0) {
                    if (l == lead && vm) atomicAdd(&hp[d0], (u32)__popcll(vm));
                } else if (valid) {
                    atomicAdd(&hp[d], 1u);
                }
            }
            rnk[k] = 0;
            if (group) {
                const u32 d = rk[k] & (RADIX - 1);
                const u64 peers = wave_peers<RADIX_BITS>(d, vm);
                const u32 below = popc_below(peers);
                const u32 cnt = (u32)__popcll(peers);
                const u32 before = valid ? (u32)s_whist[w][d] : 0u;
                rnk[k] = before + below;
                __builtin_amdgcn_wave_barrier();
                if (valid && below == cnt - 1) s_whist[w][d] = (uint16_t)(before + cnt);
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (group) {
            __syncthreads();
            // per digit: offsets of the waves, and the tile's digit starts
            u32 tcount = 0;
            if (threadIdx.x < RADIX) {
                const int d = threadIdx.x;
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) {
                    const u32 c = s_whist[ww][d];
                    s_whist[ww][d] = (uint16_t)tcount;
                    tcount += c;
                }
            }
            if (p_first && threadIdx.x < RADIX && tcount) s_h[threadIdx.x] += tcount;
            u32 total;
            const u32 st = block_exclusive_sum<PT_B>(threadIdx.x < RADIX ? tcount : 0u, s_tmp, total);
            if (threadIdx.x < RADIX) s_start[threadIdx.x] = st;
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < PT_I; ++k) {
            const u64 i = base + (u64)k * WAVE + l;
            if (i >= n) continue;
            u64 at = i;
            if (group) {
                const u32 d = rk[k] & (RADIX - 1);
                at = tile * PT + s_start[d] + s_whist[w][d] + rnk[k];
                ulonglong2* q = (ulonglong2*)(pay + at);
                q[0] = make_ulonglong2(tv[k], (u64)__double_as_longlong(la[k]));
                q[1] = make_ulonglong2((u64)__double_as_longlong(lo[k]), (u64)__float_as_uint(sp[k]) | (i << 32));
            }
            keys[at] = packed ? ((key[k] << ib) | at) : key[k];
        }
        __syncthreads();
    }
    __syncthreads();
    for (u32 i = threadIdx.x; i < (u32)HIST_WIDE_WORDS; i += blockDim.x)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// The final words are packed: (key >> 8 p0) << ib | source index.  Every
// thread takes GU records a grid stride apart per round, their loads issued
// together.  SHARDS = false compiles the plain form without the shard search;
// FULL = true is the form for callers that want every sorted column.
constexpr int GU = 4;
template <bool SHARDS, bool FULL>
__global__ void __launch_bounds__(256) k_gather(u32 n, const SortMeta* m, const u64* __restrict__ K0,
                                                const u64* __restrict__ K1, const u64* __restrict__ dict_sorted,
                                                const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                const double* __restrict__ lat, const double* __restrict__ lon,
                                                const float* __restrict__ spd, u32* __restrict__ perm,
                                                i64* __restrict__ o_jid, i64* __restrict__ o_ts,
                                                double* __restrict__ o_lat, double* __restrict__ o_lon,
                                                float* __restrict__ o_spd, const u64* __restrict__ soff, u32 S)
{
    const u32 np = m->passes;
    const u32 tb = m->t_bits;
    const u32 rb = m->rank_bits;
    const u32 ib = m->ib;
    const u32 drop = m->p0 * RADIX_BITS;
    const u64 rmask = rb >= 64 ? ~0ull : ((1ull << rb) - 1);
    const u64 imask = (1ull << ib) - 1;
    const u32 dn = m->dict_n;
    const bool exact = (m->range_err == 0) && (m->overflow == 0);
    // the journey rank survives packing when its bits lie above the dropped digits
    const bool rank_in_key = exact && drop <= tb;
    const u32 rshift = ib + tb - drop;
    // the time offset survives only when nothing was dropped (and the key had it)
    const bool ts_in_key = exact && drop == 0 && !m->ts_dropped;
    const u64 tmin = (u64)unord_i64(m->tmin_ord);
    const u64 tmask = tb >= 64 ? ~0ull : ((1ull << tb) - 1);
    const u64 tdiv = ((u64)m->t_p5) << m->t_sh;  // the time offset's unit
    const u64* K = (np & 1) ? K1 : K0;
    const u32 stride = gridDim.x * blockDim.x;
    for (u32 k0 = blockIdx.x * blockDim.x + threadIdx.x; k0 < n; k0 += GU * stride) {
        u64 wv[GU];
        u32 vv[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const u32 k = k0 + u * stride;
            wv[u] = K[k < n ? k : n - 1];  // past the end: a valid word, not stored
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) vv[u] = (u32)(wv[u] & imask);
        if constexpr (FULL) {
            // every column requested: all gathers issued before the first store
            double ola[GU], olo[GU];
            float osp[GU];
            i64 oj[GU], ot[GU];
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                ola[u] = lat[vv[u]];
                olo[u] = lon[vv[u]];
                osp[u] = spd[vv[u]];
            }
            if (rank_in_key) {
#pragma unroll
                for (int u = 0; u < GU; ++u) {
                    u64 r = rshift >= 64 ? 0ull : ((wv[u] >> rshift) & rmask);
                    r = r < dn ? r : dn - 1;
                    oj[u] = (i64)(dict_sorted[r] ^ SIGN);
                }
            } else {
#pragma unroll
                for (int u = 0; u < GU; ++u) oj[u] = jid[vv[u]];
            }
            if (ts_in_key) {
#pragma unroll
                for (int u = 0; u < GU; ++u) ot[u] = (i64)(tmin + ((wv[u] >> ib) & tmask) * tdiv);
            } else {
#pragma unroll
                for (int u = 0; u < GU; ++u) ot[u] = ts[vv[u]];
            }
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const u32 k = k0 + u * stride;
                if (k >= n) break;
                u32 pv = vv[u];
                if (SHARDS) {
                    // a shard keeps its records: the output position and its source share the shard
                    u32 sh = shard_of(soff, S, k - threadIdx.x);  // the block row's first shard, then forward
                    while (sh + 1 < S && soff[sh + 1] <= k) ++sh;
                    pv -= (u32)soff[sh];
                }
                perm[k] = pv;
                o_jid[k] = oj[u];
                o_ts[k] = ot[u];
                o_lat[k] = ola[u];
                o_lon[k] = olo[u];
                o_spd[k] = osp[u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const u32 k = k0 + u * stride;
                if (k >= n) break;
                const u64 w = wv[u];
                const u32 v = vv[u];
                u32 pv = v;
                if (SHARDS) {
                    u32 sh = shard_of(soff, S, k - threadIdx.x);
                    while (sh + 1 < S && soff[sh + 1] <= k) ++sh;
                    pv = v - (u32)soff[sh];
                }
                perm[k] = pv;
                if (o_jid) {
                    const u64 r = rshift >= 64 ? 0ull : ((w >> rshift) & rmask);
                    o_jid[k] = (rank_in_key && r < dn) ? (i64)(dict_sorted[r] ^ SIGN) : jid[v];
                }
                if (o_ts) o_ts[k] = ts_in_key ? (i64)(tmin + ((w >> ib) & tmask) * tdiv) : ts[v];
                if (o_lat) o_lat[k] = lat[v];
                if (o_lon) o_lon[k] = lon[v];
                if (o_spd) o_spd[k] = spd[v];
            }
        }
    }
}

__global__ void k_sort_finish(const SortMeta* m, cv_result* res)
{
    if (threadIdx.x != 0) return;
    cv_result r = {};
    r.status = m->range_err ? CV_ERR_RANGE : (m->overflow ? CV_ERR_CAPACITY : CV_OK);
    r.count = m->J;
    r.required = m->overflow ? m->J : 0;
    r.key_bits = m->key_bits;
    r.packed_pass = m->p0;
    r.flags = m->w0;  // bits of the first radix digit
    *res = r;
}

__global__ void k_empty_result(cv_result* res)
{
    if (threadIdx.x == 0) {
        cv_result r = {};
        *res = r;
    }
}

struct SortLayout {
    SortMeta* meta;
    u64* table;  // slots x {id, rank}
    u64* dl0;
    u64* dl1;
    u32* dv0;
    u32* dv1;
    u64* dsk0;  // batched: shard keys of the sorted distinct ids (ping-pong)
    u64* dsk1;
    u64* dlf;   // batched: the distinct ids in (shard, id) order
    u32* shist;
    u64* sstatus;
    u32* soffs;
    u32* zero_begin;  // start of the region cleared to zero
    u32* hist;
    u32* dhist;
    u64* status;
    u64* dstatus;
    size_t zero_bytes;
    u32* offs;
    u32* doffs;
    u64* K0;
    u64* K1;
    PayRec* pay;  // packed payload (interleaved input, fused gather)
    u32* V0;
    u32* V1;
    u64 slots;
    u64 tiles, dtiles;
    size_t bytes;

    SortLayout(void* ws, u64 n, u64 max_j)
    {
        cvh::Carver c(ws);
        slots = cvh::next_pow2(2 * max_j < 1024 ? 1024 : 2 * max_j);
        tiles = (n + sort_min_tile() - 1) / sort_min_tile();
        dtiles = (max_j + sort_min_tile() - 1) / sort_min_tile();
        meta = c.take<SortMeta>(1);
        table = c.take<u64>(2 * slots);
        dl0 = c.take<u64>(max_j);
        dl1 = c.take<u64>(max_j);
        dv0 = c.take<u32>(max_j);
        dv1 = c.take<u32>(max_j);
        dsk0 = c.take<u64>(max_j);
        dsk1 = c.take<u64>(max_j);
        dlf = c.take<u64>(max_j);
        size_t z0 = cvh::align_up(c.off);
        hist = c.take<u32>(HIST_WIDE_WORDS);  // record sort: wide layout
        dhist = c.take<u32>(MAX_PASSES * RADIX);
        shist = c.take<u32>(MAX_PASSES * RADIX);
        dstatus = c.take<u64>(dtiles * RADIX + 1);
        sstatus = c.take<u64>(dtiles * RADIX + 1);
        // last in the cleared range: room for 512 words per tile of the
        // smallest tile (a 9-bit first digit); a call clears what its shape uses
        status = c.take<u64>(tiles * 2 * RADIX + 1);
        size_t z1 = cvh::align_up(c.off);
        zero_begin = (u32*)(c.base ? c.base + z0 : nullptr);
        zero_bytes = z1 - z0;
        if (c.base) {
            const u64 st = (u64)(sort_block(sort_shape()) >= 2 * RADIX ? 2 * RADIX : RADIX);
            const u64 used = ((n + sort_tile(sort_shape()) - 1) / sort_tile(sort_shape())) * st + 1;
            const size_t zu = cvh::align_up((size_t)((char*)(status + used) - (char*)c.base));
            zero_bytes = (zu < z1 ? zu : z1) - z0;
        }
        offs = c.take<u32>(HIST_WIDE_WORDS);
        doffs = c.take<u32>(MAX_PASSES * RADIX);
        soffs = c.take<u32>(MAX_PASSES * RADIX);
        K0 = c.take<u64>(n);
        K1 = c.take<u64>(n);
        pay = c.take<PayRec>(n);
        V0 = c.take<u32>(n);
        V1 = c.take<u32>(n);
        bytes = c.size();
    }
};

bool valid_ptr8(const void* p) { return p == nullptr || cvh::aligned(p, 8); }

u32 bit_width_host(u64 x)
{
    u32 b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

}  // namespace

namespace {

// The gather fused with the per-point kinematics of the sorted records: every
// block writes a contiguous tile of GFT sorted records and evaluates the same
// stencil as the features kernel (cv_kin.h) on them, so that the sorted
// columns are not read back from memory.  Record t0 + 64 g + l of the tile is
// lane l of group g = u * 4 + wave (u = 0, 1): its predecessor is lane l - 1
// of the same group (a lane shuffle), or for lane 0 the last lane of group
// g - 1, which leaves it in a small LDS edge array.  Edge slot 0 holds record
// t0 - 2 and slot 1 record t0 - 1 (the tile's predecessor, whose own step
// thread 0 evaluates); group g's last record goes to slot g + 2.
constexpr int GFT = 512;
template <bool SHARDS>
__global__ void __launch_bounds__(256) k_gather_feat(u32 n, const SortMeta* m, const u64* __restrict__ K0,
                                                     const u64* __restrict__ K1, const u64* __restrict__ dict_sorted,
                                                     const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                     const double* __restrict__ lat, const double* __restrict__ lon,
                                                     const float* __restrict__ spd, u32* __restrict__ perm,
                                                     cv_records_out so, cv_features fo, const u64* __restrict__ soff,
                                                     u32 S, const PayRec* __restrict__ pay)
{
    constexpr int GFI = GFT / 256;
    constexpr int NWB = 256 / WAVE;
    constexpr int NE = GFI * NWB + 2;
    __shared__ i64 e_jid[NE], e_ts[NE];
    __shared__ double e_lat[NE], e_lon[NE], e_sphi[NE], e_cphi[NE], e_v[NE], e_b[NE];
    __shared__ u32 e_f[NE];
    __shared__ u32 s_sh0;  // shard of record t0 - 2 (batched form)
    const u32 tb = m->t_bits;
    const u32 rb = m->rank_bits;
    const u32 ib = m->ib;
    const u32 drop = m->p0 * RADIX_BITS;
    const u64 rmask = rb >= 64 ? ~0ull : ((1ull << rb) - 1);
    const u64 imask = (1ull << ib) - 1;
    const u32 dn = m->dict_n;
    const bool exact = (m->range_err == 0) && (m->overflow == 0);
    const bool rank_in_key = exact && drop <= tb;
    const u32 rshift = ib + tb - drop;
    const bool ts_in_key = exact && drop == 0 && !m->ts_dropped;
    const u64 tmin = (u64)unord_i64(m->tmin_ord);
    const u64 tmask = tb >= 64 ? ~0ull : ((1ull << tb) - 1);
    const u64 tdiv = ((u64)m->t_p5) << m->t_sh;  // the time offset's unit
    const u64* K = (m->passes & 1) ? K1 : K0;
    const int t = threadIdx.x;
    const int w = t / WAVE;
    const int l = lane_id();
    const long t0 = (long)blockIdx.x * GFT;
    // slots 0 .. GFI - 1: the tile's records; slot GFI: threads 0 and 1 fetch
    // records t0 - 2 and t0 - 1 (the others repeat their first record)
    constexpr int NS = GFI + 1;
    long kk[NS];
#pragma unroll
    for (int u = 0; u < GFI; ++u) kk[u] = t0 + (long)(u * NWB + w) * WAVE + l;
    kk[GFI] = t < 2 ? t0 - 2 + t : kk[0];
    if (SHARDS && t == 0) s_sh0 = shard_of(soff, S, (u64)(t0 >= 2 ? t0 - 2 : 0));
    // the sorted words, their source indices and columns; every load from a
    // clamped index, all issued before any is used
    u64 wv[NS];
    u32 vv[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const long k = kk[u] < 0 ? 0 : (kk[u] < (long)n ? kk[u] : (long)n - 1);
        wv[u] = K[k];
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) vv[u] = (u32)(wv[u] & imask);
    double ola[NS], olo[NS];
    float osp[NS];
    i64 oj[NS], ot[NS];
    i64 pts[NS];  // time stamps read with the packed payload
    // the input index of each sorted record: the sort's value, or, with the
    // packed payload (whose positions the key packing regrouped), the index
    // the payload carries
    u32 src[NS];
    const bool packed = pay_packed(m, n);
    if (packed) {
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const ulonglong2* q = (const ulonglong2*)(pay + vv[u]);
            const ulonglong2 a = q[0], b = q[1];
            pts[u] = (i64)a.x;
            ola[u] = __longlong_as_double((long long)a.y);
            olo[u] = __longlong_as_double((long long)b.x);
            osp[u] = __uint_as_float((u32)b.y);
            src[u] = (u32)(b.y >> 32);
        }
    } else {
#pragma unroll
        for (int u = 0; u < NS; ++u) src[u] = vv[u];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            ola[u] = lat[vv[u]];
            olo[u] = lon[vv[u]];
            osp[u] = spd[vv[u]];
        }
    }
    if (rank_in_key) {
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            u64 r = rshift >= 64 ? 0ull : ((wv[u] >> rshift) & rmask);
            r = r < dn ? r : dn - 1;
            oj[u] = (i64)(dict_sorted[r] ^ SIGN);
        }
    } else {
#pragma unroll
        for (int u = 0; u < NS; ++u) oj[u] = jid[src[u]];
    }
    if (ts_in_key) {
#pragma unroll
        for (int u = 0; u < NS; ++u) ot[u] = (i64)(tmin + ((wv[u] >> ib) & tmask) * tdiv);
    } else if (packed) {
#pragma unroll
        for (int u = 0; u < NS; ++u) ot[u] = pts[u];
    } else {
#pragma unroll
        for (int u = 0; u < NS; ++u) ot[u] = ts[vv[u]];
    }
    // sin and cos of each latitude, once per point
    double osph[NS], ocph[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        osph[u] = 0.0;
        ocph[u] = 0.0;
        if (isfinite(ola[u]) && isfinite(olo[u])) sincos(ola[u] * KIN_DEG2RAD, &osph[u], &ocph[u]);
    }
#pragma unroll
    for (int u = 0; u < GFI; ++u) {
        const long k = kk[u];
        if (k < (long)n) {
            if (!SHARDS) perm[k] = src[u];
            so.journey_id[k] = oj[u];
            so.ts_ms[k] = ot[u];
            so.lat_deg[k] = ola[u];
            so.lon_deg[k] = olo[u];
            so.speed_mps[k] = osp[u];
        }
        if (l == WAVE - 1) {
            const int e = u * NWB + w + 2;
            e_jid[e] = oj[u];
            e_ts[e] = ot[u];
            e_lat[e] = ola[u];
            e_lon[e] = olo[u];
            e_sphi[e] = osph[u];
            e_cphi[e] = ocph[u];
        }
    }
    if (t < 2) {
        e_jid[t] = oj[GFI];
        e_ts[t] = ot[GFI];
        e_lat[t] = ola[GFI];
        e_lon[t] = olo[GFI];
        e_sphi[t] = osph[GFI];
        e_cphi[t] = ocph[GFI];
    }
    __syncthreads();
    // shard of each record (batched form), walked forward from the tile's
    // first one: journey heads at shard starts, shard-relative source indices
    // (records before the next shard's start need no load: the block's first
    // shard and the start of the shard after it are read once)
    u32 shs[GFI];
    u64 sst[GFI];  // start of each record's shard
    {
        const u32 sh0 = SHARDS ? s_sh0 : 0u;
        const u64 st0 = SHARDS ? soff[sh0] : 0ull;
        const u64 nx0 = (SHARDS && sh0 + 1 < S) ? soff[sh0 + 1] : ~0ull;
#pragma unroll
        for (int u = 0; u < GFI; ++u) {
            shs[u] = 0;
            sst[u] = 0;
            if (SHARDS && kk[u] < (long)n) {
                const bool same = (u64)kk[u] < nx0;
                shs[u] = same ? sh0 : shard_from(soff, S, sh0, (u64)kk[u]);
                sst[u] = same ? st0 : soff[shs[u]];
                perm[kk[u]] = src[u] - (u32)sst[u];
            }
        }
    }
    // steps (k - 1 -> k) of the tile's records; thread 0 also takes the step
    // of record t0 - 1 (the first record's predecessor)
    KinStep ks[GFI];
#pragma unroll
    for (int u = 0; u < GFI; ++u) {
        const long k = kk[u];
        const int g = u * NWB + w;
        i64 pj = __shfl_up(oj[u], 1, WAVE), pt = __shfl_up(ot[u], 1, WAVE);
        double pla = __shfl_up(ola[u], 1, WAVE), plo = __shfl_up(olo[u], 1, WAVE);
        double psph = __shfl_up(osph[u], 1, WAVE), pcph = __shfl_up(ocph[u], 1, WAVE);
        if (l == 0) {
            pj = e_jid[g + 1];
            pt = e_ts[g + 1];
            pla = e_lat[g + 1];
            plo = e_lon[g + 1];
            psph = e_sphi[g + 1];
            pcph = e_cphi[g + 1];
        }
        bool head = k == 0 || pj != oj[u];
        if (SHARDS && !head && k < (long)n) head = sst[u] == (u64)k;
        ks[u] = kin_step(head, isfinite(ola[u]) && isfinite(olo[u]), ot[u], ola[u], olo[u], ocph[u],
                         isfinite(pla) && isfinite(plo), pt, pla, plo, pcph, psph);
        if (l == WAVE - 1) {
            const int e = g + 2;
            e_f[e] = ks[u].f;
            e_v[e] = ks[u].v;
            e_b[e] = ks[u].b;
        }
    }
    if (t == 0) {
        const long kr = t0 - 1;
        KinStep hs = KinStep{0.0, 0.0, 0.0, 0.0, 0u};
        if (kr >= 0) {
            bool head = kr == 0 || e_jid[0] != e_jid[1];
            if (SHARDS && !head) head = soff[shard_from(soff, S, s_sh0, (u64)kr)] == (u64)kr;
            const double la = e_lat[1], lo = e_lon[1], lap = e_lat[0], lop = e_lon[0];
            hs = kin_step(head, isfinite(la) && isfinite(lo), e_ts[1], la, lo, e_cphi[1], isfinite(lap) && isfinite(lop),
                          e_ts[0], lap, lop, e_cphi[0], e_sphi[0]);
        }
        e_f[1] = hs.f;
        e_v[1] = hs.v;
        e_b[1] = hs.b;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < GFI; ++u) {
        const long k = kk[u];
        const int g = u * NWB + w;
        u32 pf = (u32)__shfl_up((int)ks[u].f, 1, WAVE);
        double pv = __shfl_up(ks[u].v, 1, WAVE), pb = __shfl_up(ks[u].b, 1, WAVE);
        if (l == 0) {
            pf = e_f[g + 1];
            pv = e_v[g + 1];
            pb = e_b[g + 1];
        }
        if (k >= (long)n) continue;
        u32 f = ks[u].f;
        double acc, dh;
        kin_final(f, ks[u].v, ks[u].b, ks[u].dts, pf, pv, pb, acc, dh);
        fo.step_m[k] = ks[u].step;
        fo.dt_s[k] = ks[u].dts;
        fo.speed_mps[k] = ks[u].v;
        fo.accel_mps2[k] = acc;
        fo.bearing_deg[k] = ks[u].b;
        fo.dheading_deg[k] = dh;
        fo.flags[k] = (uint8_t)f;
    }
}

}  // namespace

static cv_status sort_impl(const cv_records* in, const uint64_t* soff, uint32_t S, uint64_t max_journeys, uint32_t* perm,
                           const cv_records_out* sorted, cv_result* res, void* ws, size_t ws_bytes, void* stream,
                           const cv_features* feat = nullptr)
{
    if (!in || in->n >= (1ull << 32) || max_journeys >= (1ull << 31)) return CV_ERR_INVALID_ARGUMENT;
    const u64 n = in->n;
    if (max_journeys == 0) max_journeys = 1;
    hipStream_t s = (hipStream_t)stream;
    cv_records_out so = {};
    if (sorted) so = *sorted;
    if (n > 0) {
        if (!in->journey_id || !in->ts_ms || !perm) return CV_ERR_INVALID_ARGUMENT;
        if ((so.lat_deg && !in->lat_deg) || (so.lon_deg && !in->lon_deg) || (so.speed_mps && !in->speed_mps))
            return CV_ERR_INVALID_ARGUMENT;
        if (!valid_ptr8(in->journey_id) || !valid_ptr8(in->ts_ms) || !valid_ptr8(in->lat_deg) ||
            !valid_ptr8(in->lon_deg) || !valid_ptr8(so.journey_id) || !valid_ptr8(so.ts_ms) ||
            !valid_ptr8(so.lat_deg) || !valid_ptr8(so.lon_deg) || !cvh::aligned(perm, 4))
            return CV_ERR_INVALID_ARGUMENT;
    }
    SortLayout need(nullptr, n, max_journeys);
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need.bytes) return CV_ERR_WORKSPACE;
    if (n == 0) {
        if (res) hipLaunchKernelGGL(k_empty_result, dim3(1), dim3(64), 0, s, res);
        return cvh::last_launch_status();
    }
    SortLayout L(ws, n, max_journeys);
    const u32 nn = (u32)n;
    const u32 mj = (u32)max_journeys;
    const u64 mask = L.slots - 1;
    const int gs = cvh::grid_for(n, 256, 2048);
    {
        cvh::TimedScope ts_("sort_prep", s);
        hipLaunchKernelGGL(k_sort_init, dim3(1), dim3(64), 0, s, L.meta);
        cvh::fill_u64(L.table, EMPTY, 2 * L.slots, s);
        cvh::fill_u32(L.zero_begin, 0u, L.zero_bytes / 4, s);
        hipLaunchKernelGGL(S > 1 ? k_dict_insert<true> : k_dict_insert<false>, dim3(gs), dim3(256), 0, s,
                           in->journey_id, in->ts_ms, nn, L.table, mask, L.meta, soff, S);
        hipLaunchKernelGGL(k_dict_compact, dim3(cvh::grid_for(L.slots, 256, 2048)), dim3(256), 0, s, L.table,
                           L.slots, mj, L.meta, L.dl0);
        hipLaunchKernelGGL(k_dict_meta, dim3(1), dim3(64), 0, s, L.meta, mj, nn, S, sort_wide_first() ? 1u : 0u);
        // sort the distinct ids (64-bit, signed order via the flipped sign bit)
        const u32* dn = &L.meta->dict_n;
        radix_hist(L.dl0, mj, dn, MAX_PASSES, nullptr, L.dhist, cvh::grid_for(max_journeys, 256, 512), s);
        radix_scan(L.dhist, L.doffs, MAX_PASSES, s);
        radix_passes(L.dl0, L.dl1, nullptr, L.dv0, L.dv1, mj, dn, nullptr, MAX_PASSES, L.doffs, L.dstatus,
                     L.meta->tickets + MAX_PASSES, s);
        if (S > 1) {
            // the id-sorted list, stably by shard: (shard, id) order, and ranks in it
            const int sp = (int)((bit_width_host((u64)S - 1) + RADIX_BITS - 1) / RADIX_BITS);
            const int dg = cvh::grid_for(max_journeys, 256, 1024);
            hipLaunchKernelGGL(k_dict_shardkey, dim3(dg), dim3(256), 0, s, L.dl0, L.meta, L.table, mask, L.dsk0);
            radix_hist(L.dsk0, mj, dn, sp, nullptr, L.shist, cvh::grid_for(max_journeys, 256, 512), s);
            radix_scan(L.shist, L.soffs, sp, s);
            radix_passes(L.dsk0, L.dsk1, nullptr, L.dv0, L.dv1, mj, dn, nullptr, sp, L.soffs, L.sstatus,
                         L.meta->tickets + 2 * MAX_PASSES, s);
            hipLaunchKernelGGL(k_dict_final, dim3(dg), dim3(256), 0, s, L.dl0, (sp & 1) ? L.dv1 : L.dv0, L.meta,
                               L.table, mask, L.dlf);
        } else {
            hipLaunchKernelGGL(k_dict_rank, dim3(cvh::grid_for(max_journeys, 256, 1024)), dim3(256), 0, s, L.dl0,
                               L.meta, L.table, mask);
        }
        // interleaved input (short runs of equal ids): the payload packed per
        // record for the fused gather, in the same pass
        hipLaunchKernelGGL(S > 1 ? k_pack_hist<true> : k_pack_hist<false>, dim3(gs), dim3(256), 0, s, in->journey_id,
                           in->ts_ms, nn, L.table, mask, L.meta, L.K0, L.hist, soff, S);
        hipLaunchKernelGGL(S > 1 ? k_pack_il<true> : k_pack_il<false>, dim3(cvh::grid_for(n, PT, 2048)), dim3(PT_B), 0,
                           s, in->journey_id,
                           in->ts_ms, in->lat_deg, in->lon_deg, in->speed_mps, feat ? L.pay : nullptr, nn, L.table,
                           mask, L.meta, L.K0, L.hist, soff, S);
        radix_scan(L.hist, L.offs, MAX_PASSES, s, &L.meta->w0);
    }
    radix_passes(L.K0, L.K1, nullptr, L.V0, L.V1, nn, nullptr, &L.meta->key_bits, MAX_PASSES, L.offs, L.status,
                 L.meta->tickets, s, /*timed=*/true, &L.meta->ib, &L.meta->w0);
    const u64* dict_ids = S > 1 ? L.dlf : L.dl0;  // journey ids by rank
    if (feat) {
        cvh::TimedScope ts_("gather_features", s);
        auto gk = S > 1 ? k_gather_feat<true> : k_gather_feat<false>;
        hipLaunchKernelGGL(gk, dim3((unsigned)((n + GFT - 1) / GFT)), dim3(256), 0, s, nn, L.meta, L.K0, L.K1, dict_ids,
                           in->journey_id, in->ts_ms, in->lat_deg, in->lon_deg, in->speed_mps, perm, so, *feat, soff,
                           S, L.pay);
    } else {
        cvh::TimedScope ts_("gather", s);
        const bool full = so.journey_id && so.ts_ms && so.lat_deg && so.lon_deg && so.speed_mps;
        auto gk = S > 1 ? (full ? k_gather<true, true> : k_gather<true, false>)
                        : (full ? k_gather<false, true> : k_gather<false, false>);
        hipLaunchKernelGGL(gk, dim3(cvh::grid_for(n, 256, 8192)), dim3(256), 0, s, nn, L.meta, L.K0, L.K1, dict_ids,
                           in->journey_id, in->ts_ms, in->lat_deg, in->lon_deg, in->speed_mps, perm,
                           so.journey_id, so.ts_ms, so.lat_deg, so.lon_deg, so.speed_mps, soff, S);
    }
    cvh::debug_sort(L.K0, L.K1, &L.meta->passes, &L.meta->range_err, &L.meta->overflow, n, perm, soff, S, s);
    if (res) hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(64), 0, s, L.meta, res);
    return cvh::last_launch_status();
}


namespace cv {
// the record sort for other translation units of the library (no shards)
cv_status sort_records_into(const cv_records* in, uint64_t max_journeys, uint32_t* perm, const cv_records_out* sorted,
                            cv_result* res, void* ws, size_t ws_bytes, hipStream_t stream)
{
    return sort_impl(in, nullptr, 0, max_journeys, perm, sorted, res, ws, ws_bytes, (void*)stream);
}
}  // namespace cv

extern "C" {

cv_status cv_sort_workspace_size(uint64_t n, uint64_t max_journeys, size_t* bytes)
{
    if (!bytes || n >= (1ull << 32) || max_journeys >= (1ull << 31)) return CV_ERR_INVALID_ARGUMENT;
    if (max_journeys == 0) max_journeys = 1;
    SortLayout L(nullptr, n, max_journeys);
    *bytes = L.bytes;
    return CV_OK;
}

cv_status cv_sort_records(const cv_records* in, uint64_t max_journeys, uint32_t* perm, const cv_records_out* sorted,
                          cv_result* res, void* ws, size_t ws_bytes, void* stream)
{
    return sort_impl(in, nullptr, 0, max_journeys, perm, sorted, res, ws, ws_bytes, stream);
}

cv_status cv_batch_sort_records(const cv_records* in, const uint64_t* shard_offsets, uint32_t n_shards,
                                uint64_t max_journeys, uint32_t* perm, const cv_records_out* sorted, cv_result* res,
                                void* ws, size_t ws_bytes, void* stream)
{
    if (n_shards == 0 || !shard_offsets || !cvh::aligned(shard_offsets, 8)) return CV_ERR_INVALID_ARGUMENT;
    return sort_impl(in, shard_offsets, n_shards, max_journeys, perm, sorted, res, ws, ws_bytes, stream);
}

static bool feat_complete(const cv_records_out* so, const cv_features* f)
{
    return so && f && so->journey_id && so->ts_ms && so->lat_deg && so->lon_deg && so->speed_mps && f->step_m &&
           f->dt_s && f->speed_mps && f->accel_mps2 && f->bearing_deg && f->dheading_deg && f->flags;
}

cv_status cv_sort_records_features(const cv_records* in, uint64_t max_journeys, uint32_t* perm,
                                   const cv_records_out* sorted, const cv_features* feat, cv_result* res, void* ws,
                                   size_t ws_bytes, void* stream)
{
    if (in && in->n && !feat_complete(sorted, feat)) return CV_ERR_INVALID_ARGUMENT;
    return sort_impl(in, nullptr, 0, max_journeys, perm, sorted, res, ws, ws_bytes, stream, feat);
}

cv_status cv_batch_sort_records_features(const cv_records* in, const uint64_t* shard_offsets, uint32_t n_shards,
                                         uint64_t max_journeys, uint32_t* perm, const cv_records_out* sorted,
                                         const cv_features* feat, cv_result* res, void* ws, size_t ws_bytes,
                                         void* stream)
{
    if (n_shards == 0 || !shard_offsets || !cvh::aligned(shard_offsets, 8)) return CV_ERR_INVALID_ARGUMENT;
    if (in && in->n && !feat_complete(sorted, feat)) return CV_ERR_INVALID_ARGUMENT;
    return sort_impl(in, shard_offsets, n_shards, max_journeys, perm, sorted, res, ws, ws_bytes, stream, feat);
}

}  // extern "C"
