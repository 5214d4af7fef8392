// cv_device.h -- device-side building blocks shared by the gfx950 kernels.
//
// * exact fixed-point accumulation of floating-point terms (192-bit two's
//   complement in three 64-bit limbs) and one round-to-nearest-even
//   conversion back to double, so every sum is independent of the order in
//   which tiles, waves or atomics add their terms;
// * order-preserving integer images of float/double/int64 for integer
//   atomicMin / atomicMax;
// * wave64 / block scans and the single-pass decoupled look-back that turns
//   per-tile counts into exclusive prefixes (Merrill & Garland, 2016).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cv {

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// 192-bit fixed point.  A finite double v is represented as trunc(v * 2^F):
// for F = 149 every float32 is exact; for F = 128 every double >= 2^-75 is.
// ---------------------------------------------------------------------------
struct Fx192 {
    u64 w[3];
};

__device__ __forceinline__ void fx_zero(Fx192& a) { a.w[0] = a.w[1] = a.w[2] = 0; }

__device__ __forceinline__ void fx_add(Fx192& a, const Fx192& b)
{
    u64 s0 = a.w[0] + b.w[0];
    u64 c0 = s0 < a.w[0];
    u64 s1 = a.w[1] + b.w[1];
    u64 c1 = s1 < a.w[1];
    u64 s1c = s1 + c0;
    c1 += s1c < s1;
    a.w[0] = s0;
    a.w[1] = s1c;
    a.w[2] = a.w[2] + b.w[2] + c1;
}

__device__ __forceinline__ void fx_neg(Fx192& a)
{
    a.w[0] = ~a.w[0];
    a.w[1] = ~a.w[1];
    a.w[2] = ~a.w[2];
    a.w[0] += 1;
    u64 c = a.w[0] == 0;
    a.w[1] += c;
    c = c & (a.w[1] == 0);
    a.w[2] += c;
}

// Place a 53-bit integer m at bit offset sh (0 <= sh < 192) of a 192-bit word
// without indexing the limbs at run time (a run-time index would force the
// limbs into scratch memory).
__device__ __forceinline__ Fx192 fx_place(u64 m, int sh)
{
    Fx192 r;
    const int wd = sh >> 6, bt = sh & 63;
    const u64 lo = m << bt;
    const u64 hi = bt ? (m >> (64 - bt)) : 0ull;
    r.w[0] = wd == 0 ? lo : 0ull;
    r.w[1] = wd == 1 ? lo : (wd == 0 ? hi : 0ull);
    r.w[2] = wd == 2 ? lo : (wd == 1 ? hi : 0ull);
    return r;
}

template <int F>
__device__ __forceinline__ Fx192 fx_from_double(double v)
{
    Fx192 r;
    fx_zero(r);
    u64 bits = (u64)__double_as_longlong(v);
    int e = (int)((bits >> 52) & 0x7FF);
    u64 m = bits & ((1ull << 52) - 1);
    if (e == 0) {
        if (m == 0) return r;
        e = 1;
    } else {
        m |= 1ull << 52;
    }
    const int sh = e - 1075 + F;  // v = m * 2^(e-1075); scaled: m * 2^sh
    if (sh <= -53) return r;
    if (sh < 0) r.w[0] = m >> (-sh);
    else if (sh < 192) r = fx_place(m, sh);
    if (bits >> 63) fx_neg(r);
    return r;
}

// bits [lo, lo + 64) of a 192-bit word (lo in [0, 192)), no run-time indexing
__device__ __forceinline__ u64 fx_extract64(const Fx192& a, int lo)
{
    const int wd = lo >> 6, bt = lo & 63;
    const u64 w0 = wd == 0 ? a.w[0] : (wd == 1 ? a.w[1] : a.w[2]);
    const u64 w1 = wd == 0 ? a.w[1] : (wd == 1 ? a.w[2] : 0ull);
    return bt ? ((w0 >> bt) | (w1 << (64 - bt))) : w0;
}

// true when any of the bits [0, k) is set (0 <= k <= 192)
__device__ __forceinline__ bool fx_any_below(const Fx192& a, int k)
{
    const u64 m0 = k >= 64 ? ~0ull : (k <= 0 ? 0ull : ((1ull << k) - 1));
    const int k1 = k - 64;
    const u64 m1 = k1 >= 64 ? ~0ull : (k1 <= 0 ? 0ull : ((1ull << k1) - 1));
    const int k2 = k - 128;
    const u64 m2 = k2 >= 64 ? ~0ull : (k2 <= 0 ? 0ull : ((1ull << k2) - 1));
    return ((a.w[0] & m0) | (a.w[1] & m1) | (a.w[2] & m2)) != 0;
}

// Round-to-nearest-even of the fixed-point value times 2^-F.
template <int F>
__device__ __forceinline__ double fx_to_double(Fx192 a)
{
    const bool neg = (a.w[2] >> 63) != 0;
    if (neg) fx_neg(a);
    int p;
    if (a.w[2]) p = 128 + 63 - __clzll((long long)a.w[2]);
    else if (a.w[1]) p = 64 + 63 - __clzll((long long)a.w[1]);
    else if (a.w[0]) p = 63 - __clzll((long long)a.w[0]);
    else return 0.0;
    double r;
    if (p <= 52) {
        r = ldexp((double)a.w[0], -F);
    } else {
        // mantissa = bits [p-52, p]; round bit p-53; sticky below it
        int lo = p - 52;
        u64 mant = fx_extract64(a, lo) & ((1ull << 53) - 1);
        const int rb = lo - 1;
        const u64 round = (fx_extract64(a, rb) & 1ull);
        const bool sticky = fx_any_below(a, rb);
        if (round && (sticky || (mant & 1))) {
            mant += 1;
            if (mant == (1ull << 53)) {
                mant >>= 1;
                lo += 1;
            }
        }
        r = ldexp((double)mant, lo - F);
    }
    return neg ? -r : r;
}

// 192-bit add into three global (or LDS) limbs with carries carried by the
// return values of the atomics: order-independent and exact.
__device__ __forceinline__ void atomic_add_fx(u64* L, const Fx192& a)
{
    u64 c0 = 0;
    if (a.w[0]) {
        u64 old0 = atomicAdd((unsigned long long*)&L[0], (unsigned long long)a.w[0]);
        c0 = (old0 + a.w[0]) < old0;
    }
    u64 a1 = a.w[1] + c0;
    u64 c1 = (a1 < c0) ? 1 : 0;
    if (a1) {
        u64 old1 = atomicAdd((unsigned long long*)&L[1], (unsigned long long)a1);
        c1 += (old1 + a1) < old1;
    }
    u64 a2 = a.w[2] + c1;
    if (a2) atomicAdd((unsigned long long*)&L[2], (unsigned long long)a2);
}

// Carry-save form for LDS accumulation: four 48-bit chunks held in 64-bit
// counters; up to 2^16 terms add without overflow, normalised once.
__device__ __forceinline__ void fx_to_cs(const Fx192& a, u64 c[4])
{
    const u64 M = (1ull << 48) - 1;
    c[0] = a.w[0] & M;
    c[1] = ((a.w[0] >> 48) | (a.w[1] << 16)) & M;
    c[2] = ((a.w[1] >> 32) | (a.w[2] << 32)) & M;
    c[3] = a.w[2] >> 16;
}

__device__ __forceinline__ Fx192 fx_from_cs(const u64 c[4])
{
    // sum_i c[i] * 2^(48 i) mod 2^192
    Fx192 r, t;
    fx_zero(r);
    t.w[0] = c[0];
    t.w[1] = 0;
    t.w[2] = 0;
    fx_add(r, t);
    t.w[0] = c[1] << 48;
    t.w[1] = c[1] >> 16;
    t.w[2] = 0;
    fx_add(r, t);
    t.w[0] = 0;
    t.w[1] = c[2] << 32;
    t.w[2] = c[2] >> 32;
    fx_add(r, t);
    t.w[0] = 0;
    t.w[1] = 0;
    t.w[2] = c[3] << 16;
    fx_add(r, t);
    return r;
}

// ---------------------------------------------------------------------------
// order-preserving images
// ---------------------------------------------------------------------------
__device__ __forceinline__ float canon0f(float v) { return v == 0.0f ? 0.0f : v; }
__device__ __forceinline__ double canon0d(double v) { return v == 0.0 ? 0.0 : v; }

__device__ __forceinline__ u32 ord_f32(float v)
{
    u32 b = __float_as_uint(canon0f(v));
    return (b >> 31) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(u32 u)
{
    u32 b = (u >> 31) ? (u & 0x7FFFFFFFu) : ~u;
    return __uint_as_float(b);
}
__device__ __forceinline__ u64 ord_f64(double v)
{
    u64 b = (u64)__double_as_longlong(canon0d(v));
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double unord_f64(u64 u)
{
    u64 b = (u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ u64 ord_i64(i64 v) { return (u64)v ^ 0x8000000000000000ull; }
__device__ __forceinline__ i64 unord_i64(u64 u) { return (i64)(u ^ 0x8000000000000000ull); }

__device__ __forceinline__ u64 mix64(u64 x)
{
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

// ---------------------------------------------------------------------------
// shards (independent problems laid out back to back): offsets[0..S] in
// records, offsets[0] = 0, non-decreasing; empty shards allowed
// ---------------------------------------------------------------------------
// the shard holding record r: the largest s with offsets[s] <= r
__device__ __forceinline__ u32 shard_of(const u64* __restrict__ off, u32 S, u64 r)
{
    u32 lo = 0, hi = S;
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (off[mid] <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}

// the same, walking forward from a shard s <= shard_of(r) (a shard holding an
// earlier record): a few steps, then a binary search for long walks
__device__ __forceinline__ u32 shard_from(const u64* __restrict__ off, u32 S, u32 s, u64 r)
{
#pragma unroll 1
    for (int i = 0; i < 4; ++i) {
        if (s + 1 >= S || off[s + 1] > r) return s;
        ++s;
    }
    return shard_of(off, S, r);
}

__device__ __forceinline__ bool shard_start(const u64* __restrict__ off, u32 S, u64 r)
{
    return S > 0 && off[shard_of(off, S, r)] == r;
}

// first k in [0, S] with off[k] >= a (S when none)
__device__ __forceinline__ u32 shard_lower_bound(const u64* __restrict__ off, u32 S, u64 a)
{
    u32 lo = 0, hi = S;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (off[mid] < a) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Shard starts among the records [a, a + 64) as a lane mask, for a wave that
// walks consecutive windows: k is the first shard whose start is >= a and moves
// past the window; at_end tells whether a shard starts at a + 64.  k and a are
// wave-uniform (the caller makes them so), which lets the offsets be read with
// scalar loads that do not hold up the wave's vector loads.
__device__ __forceinline__ u64 shard_starts_in(const u64* __restrict__ off, u32 S, u32& k, u64 a, bool& at_end)
{
    u64 m = 0;
    k = __builtin_amdgcn_readfirstlane(k);
    u64 nb = k < S ? off[k] : ~0ull;
    while (nb < a + 64) {
        m |= 1ull << (nb - a);
        ++k;
        nb = k < S ? off[k] : ~0ull;
    }
    at_end = nb == a + 64;
    return m;
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

// number of set bits of `mask` in lanes below this lane
__device__ __forceinline__ u32 popc_below(u64 mask)
{
    return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0));
}

// Lanes of `valid` whose digit d (the low BITS bits) equals this lane's: one
// ballot per bit; a lane differs from this one where a ballot differs from the
// lane's own bit, sign-extended to a 32-bit mask, and the differences of all
// bits are ORed per 32-lane half (about 5 vector instructions per bit).
template <int BITS>
__device__ __forceinline__ u64 wave_peers(u32 d, u64 valid)
{
    u32 dlo = 0, dhi = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const u32 s = (u32)(((int)(d << (31 - b))) >> 31);  // 0 or ~0
        const u64 bal = __ballot(s != 0u);
        dlo |= (u32)bal ^ s;
        dhi |= (u32)(bal >> 32) ^ s;
    }
    return valid & ~(((u64)dhi << 32) | dlo);
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v)
{
    int l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T o = __shfl_up(v, d, WAVE);
        if (l >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_max(T v)
{
    int l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T o = __shfl_up(v, d, WAVE);
        if (l >= d) v = v > o ? v : o;
    }
    return v;
}

// Block-wide exclusive sum of one value per thread.  `tmp` holds BLOCK/64
// entries of LDS.  Contains __syncthreads; call from every thread.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* tmp, T& total)
{
    constexpr int NW = BLOCK / WAVE;
    int w = threadIdx.x / WAVE, l = lane_id();
    T inc = wave_inclusive_sum(v);
    if (l == WAVE - 1) tmp[w] = inc;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        T x = tmp[i];
        if (i < w) base += x;
        tot += x;
    }
    total = tot;
    __syncthreads();
    return base + inc - v;
}

// ---------------------------------------------------------------------------
// Decoupled look-back.  A status word is [flag:2 | value:62]; flag 1 = the
// tile's own aggregate is published, 2 = its inclusive prefix is.  Tiles are
// numbered by an atomic ticket taken at block start, so every tile a block
// waits on has already been scheduled and publishes without waiting itself.
// ---------------------------------------------------------------------------
constexpr u64 LB_AGG = 1ull << 62;
constexpr u64 LB_PRE = 2ull << 62;
constexpr u64 LB_VAL = (1ull << 62) - 1;

__device__ __forceinline__ void lb_publish(u64* p, u64 v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 lb_peek(u64* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One thread: publish `agg` for `tile` and return the exclusive prefix.
__device__ __forceinline__ u64 lookback_exclusive(u64* status, u32 tile, u64 agg)
{
    if (tile == 0) {
        lb_publish(&status[0], LB_PRE | agg);
        return 0;
    }
    lb_publish(&status[tile], LB_AGG | agg);
    u64 excl = 0;
    int t = (int)tile - 1;
    while (t >= 0) {
        u64 w = lb_peek(&status[t]);
        u64 f = w & ~LB_VAL;
        if (f == 0) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += w & LB_VAL;
        if (f == LB_PRE) break;
        --t;
    }
    lb_publish(&status[tile], LB_PRE | (excl + agg));
    return excl;
}

// Wave-parallel variant: the whole wave (all 64 lanes, uniform control flow)
// inspects 64 predecessor tiles per step.  Returns the exclusive prefix in
// every lane.  Lane 0 publishes.
__device__ __forceinline__ u64 wave_lookback_exclusive(u64* status, u32 tile, u64 agg)
{
    int l = lane_id();
    if (tile == 0) {
        if (l == 0) lb_publish(&status[0], LB_PRE | agg);
        return 0;
    }
    if (l == 0) lb_publish(&status[tile], LB_AGG | agg);
    u64 excl = 0;
    int base = (int)tile - 1;  // lane l looks at tile base - l
    while (true) {
        int t = base - l;
        u64 w = (t >= 0) ? lb_peek(&status[t]) : LB_PRE;  // virtual inclusive 0 before tile 0
        u64 f = w & ~LB_VAL;
        // wait until every inspected tile has published something
        if (__ballot(f == 0) != 0) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        u64 pre = __ballot(f == LB_PRE);
        // first lane (nearest tile) holding an inclusive prefix
        int stop = pre ? __ffsll((long long)pre) - 1 : WAVE;
        u64 v = (l <= stop && t >= 0) ? (w & LB_VAL) : 0;
        // wave sum
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
        excl += v;
        if (pre) break;
        base -= WAVE;
    }
    if (l == 0) lb_publish(&status[tile], LB_PRE | (excl + agg));
    return excl;
}

}  // namespace cv
