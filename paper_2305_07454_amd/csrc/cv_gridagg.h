// cv_gridagg.h -- the tile kernel of the serving form's grid aggregate, which
// adds every tile's groups into a resident HBM table and so needs the
// distinct-journey flag of every run head inside the tile, and the run-piece
// arithmetic (exact 128-bit speed sums, cross-lane joins of run pieces) that
// the plain and batched tile kernel (cv_gridpart.h) shares.  A policy type
// supplies the serving form's rules: records flagged late (they count in their
// cells but never as a new distinct journey, and a change of that status
// starts a segment), cells a journey's open segment carried over from earlier
// pushes, and a hook that sees every record that counts its journey in a cell.
#pragma once
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_gridtab.h"

namespace cv {
namespace {

// the plain and batched forms: nothing is late or carried; kDir says where a
// direction sector comes from (0: no direction dimension, 1: a sensor heading
// column, 2: the derived bearing and its flags)
template <int KD>
struct GridPlainT {
    static constexpr bool kStream = false;
    static constexpr int kDir = KD;
    __device__ bool late(u64) const { return false; }
    __device__ bool carried(u64, u64) const { return false; }
    __device__ void first(u64, u64) const {}
};
using GridPlain = GridPlainT<0>;
using GridHeading = GridPlainT<1>;
using GridBearing = GridPlainT<2>;

constexpr int GB = 256;
constexpr int GI = 8;
constexpr int GT = GB * GI;
constexpr int HALO = 256;
static_assert(HALO % GB == 0, "whole halo rows");
constexpr int LHS_PROBES = 32;
struct LSlot {
    u64 cs[4];
    u32 count, nj, mn, mx;
};
static_assert(offsetof(LSlot, nj) == offsetof(LSlot, count) + 4 && offsetof(LSlot, count) % 8 == 0,
              "count and nj form one aligned 64-bit word");

constexpr uint8_t B_SEG = 1;   // first record of a (journey, time-bin) segment
constexpr uint8_t B_RUN = 2;   // first record of a run (segment start or key change)
constexpr uint8_t B_FIRST = 4; // run head whose key is new in its segment (counts its journey)
constexpr uint8_t B_LATE = 8;  // late record (serving form)
constexpr uint8_t B_PEND = 16; // run head left to the block-wide scan of its segment's earlier records

// Partial aggregate of one run (or piece of a run).  The speed sum is a
// 128-bit two's-complement integer in units of 2^-53, exact for every float32
// speed v with 2^-30 <= |v| < 2^10 (and for zeros).  A record with any other
// speed is a run of its own (the records on both sides of it start runs), so
// its piece holds that one speed: RUN_ODD is set and lo holds the float's
// bits, converted to the 192-bit format when the piece is inserted.  Count
// and distinct journeys share one word (count in bits 0-15, journeys in bits
// 16-30: a piece holds at most GT / 4 records); bit 31 is RUN_ODD.
constexpr u32 RUN_ODD = 0x80000000u;
struct RunPart {
    u64 lo, hi;
    u32 cn, mn, mx;
};

__device__ __forceinline__ void run_reset(RunPart& p)
{
    p.lo = 0;
    p.hi = 0;
    p.cn = 0;
    p.mn = ~0u;
    p.mx = 0;
}

__device__ __forceinline__ void add128(u64& lo, u64& hi, u64 blo, u64 bhi)
{
    const u64 s = lo + blo;
    hi += bhi + (s < lo ? 1ull : 0ull);
    lo = s;
}

__device__ __forceinline__ void run_combine(RunPart& a, const RunPart& b)
{
    add128(a.lo, a.hi, b.lo, b.hi);
    a.cn += b.cn;
    a.mn = b.mn < a.mn ? b.mn : a.mn;
    a.mx = b.mx > a.mx ? b.mx : a.mx;
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

// the 128-bit sum in the table's 192-bit format (2^-149 units)
__device__ __forceinline__ Fx192 run_sum192(const RunPart& p)
{
    Fx192 r;
    r.w[0] = 0;
    r.w[1] = p.lo << 32;
    r.w[2] = (p.lo >> 32) | (p.hi << 32);
    return r;
}

// one step of a cross-lane reduction or scan: fold in the partial d lanes away
// (xor: full reduction; up: the lane below) when `take`
__device__ __forceinline__ void run_step(RunPart& p, int d, bool up, bool take)
{
    const u64 lo = up ? (u64)__shfl_up((unsigned long long)p.lo, d, WAVE) : (u64)__shfl_xor((unsigned long long)p.lo, d, WAVE);
    const u64 hi = up ? (u64)__shfl_up((unsigned long long)p.hi, d, WAVE) : (u64)__shfl_xor((unsigned long long)p.hi, d, WAVE);
    const u32 cn = up ? (u32)__shfl_up(p.cn, d, WAVE) : (u32)__shfl_xor(p.cn, d, WAVE);
    const u32 mn = up ? (u32)__shfl_up(p.mn, d, WAVE) : (u32)__shfl_xor(p.mn, d, WAVE);
    const u32 mx = up ? (u32)__shfl_up(p.mx, d, WAVE) : (u32)__shfl_xor(p.mx, d, WAVE);
    if (take) {
        add128(p.lo, p.hi, lo, hi);
        p.cn += cn;
        p.mn = mn < p.mn ? mn : p.mn;
        p.mx = mx > p.mx ? mx : p.mx;
    }
}

__device__ __forceinline__ void run_wave_reduce(RunPart& p)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) run_step(p, d, false, true);
}

// segmented inclusive scan across lanes; `head` starts a segment
__device__ __forceinline__ void run_seg_scan(RunPart& p, bool head)
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
    for (int k = 0, d = 1; d < WAVE; ++k, d <<= 1) run_step(p, d, true, ((take >> k) & 1u) != 0);
}

// Where a tile's group contributions go: the serving form's resident HBM
// hash table (kept across pushes).
struct SinkTable {
    GEntry* tab;
    u64 mask;
    GridMeta* meta;
    __device__ void put(u64 key, u32 count, u32 nj, const Fx192& sum, u32 mn, u32 mx, u32*, u64*, u64) const
    {
        g_insert(tab, mask, meta, key, count, nj, sum, mn, mx);
    }
};

// one contribution to key's group in the tile's LDS table; no free slot within
// the probe limit hands it to the sink on its own
template <int LHS, class Sink>
__device__ __forceinline__ void slot_insert(u64* s_hkey, LSlot* s_h, const Sink& sk, u32* s_np, u64* s_kmax, u64 tile,
                                            u64 key, const Fx192& sum, u32 count, u32 nj, u32 mn, u32 mx)
{
    u64 h = mix64(key) & (LHS - 1);
    for (int probe = 0; probe < LHS_PROBES; ++probe) {
        u64 cur = s_hkey[h];
        if (cur == GEMPTY) {
            const u64 prev =
                atomicCAS((unsigned long long*)&s_hkey[h], (unsigned long long)GEMPTY, (unsigned long long)key);
            cur = prev == GEMPTY ? key : prev;
        }
        if (cur == key) {
            LSlot& sl = s_h[h];
            u64 c[4];
            fx_to_cs(sum, c);
            for (int i = 0; i < 4; ++i)
                if (c[i]) atomicAdd((unsigned long long*)&sl.cs[i], (unsigned long long)c[i]);
            // count and nj are adjacent: one 64-bit add (a tile's count stays below 2^32)
            if (count | nj) atomicAdd(reinterpret_cast<unsigned long long*>(&sl.count), (u64)count | ((u64)nj << 32));
            if (mn != ~0u) atomicMin(&sl.mn, mn);
            if (mx) atomicMax(&sl.mx, mx);
            return;
        }
        h = (h + 1) & (LHS - 1);
    }
    sk.put(key, count, nj, sum, mn, mx, s_np, s_kmax, tile);
}

template <int LHS, class Sink>
__device__ __forceinline__ void run_insert(u64* s_hkey, LSlot* s_h, const Sink& sk, u32* s_np, u64* s_kmax, u64 tile,
                                           u64 key, const RunPart& p)
{
    const Fx192 sum = (p.cn & RUN_ODD) ? fx_from_double<FX_SPD>((double)__uint_as_float((u32)p.lo)) : run_sum192(p);
    slot_insert<LHS>(s_hkey, s_h, sk, s_np, s_kmax, tile, key, sum, p.cn & 0xFFFFu, (p.cn >> 16) & 0x7FFFu, p.mn,
                     p.mx);
}

// a speed outside the 128-bit fast format (a run of its own)
__device__ __forceinline__ bool spd_odd(float v)
{
    i64 x;
    return !spd_fix53(v, x);
}

// three workgroups per CU fit the LDS of the 256-slot table: the register
// budget is set to match (the larger tables leave room for fewer)
template <int LHS, class Pol, class Sink>
__global__ void __launch_bounds__(GB) __attribute__((amdgpu_waves_per_eu(LHS <= 256 ? 3 : (LHS <= 512 ? 2 : 1))))
k_grid_agg(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts, const double* __restrict__ lat,
           const double* __restrict__ lon, const float* __restrict__ spd, Spec g, Sink sk, GridMeta* meta, Pol pol)
{
    constexpr int NQ = HALO + GT;
    __shared__ i64 s_key[NQ];       // keys per record; later the keys of the run-head list
    __shared__ __attribute__((aligned(16))) uint8_t s_bits[NQ];
    __shared__ uint16_t s_lpos[NQ];  // run-head list: q | segment start << 15
    __shared__ __attribute__((aligned(16))) float s_spd[GT];
    __shared__ u64 s_hkey[LHS];
    __shared__ LSlot s_h[LHS];
    constexpr int NWG = GB / WAVE;
    __shared__ i64 s_lj[HALO / GB + GI][NWG], s_ltb[HALO / GB + GI][NWG];  // wave row ends
    __shared__ i64 s_lk[HALO / GB + GI][NWG];                               // wave row ends: key
    __shared__ u32 s_cnt[(HALO / GB + GI) * NWG];                          // run heads per wave row
    __shared__ i64 s_ltbs[HALO / GB + GI][NWG];                             // wave row starts
    __shared__ uint8_t s_llt[HALO / GB + GI][NWG];                          // wave row ends: late
    __shared__ i64 s_pj, s_ptb;  // the record before the first row
    __shared__ uint8_t s_plt;
    __shared__ int s_lo;
    __shared__ u32 s_npend, s_pn, s_nfound;
    __shared__ unsigned long long s_r0[2];
    __shared__ u64 s_out[GB / WAVE];
    __shared__ uint8_t s_rodd[HALO / GB + GI][NWG];  // a speed outside the fast format in this wave row
    __shared__ u32 s_np;                             // partial rows this tile wrote (partial sink)
    __shared__ u64 s_kmax;                           // their largest key

    const int t = threadIdx.x;
    const u64 tile0 = (u64)blockIdx.x * GT;
    const u32 tvalid = (u32)((u64)n - tile0 < (u64)GT ? (u64)n - tile0 : (u64)GT);
    for (int i = t; i < LHS; i += GB) {
        s_hkey[i] = GEMPTY;
        LSlot z;
        z.cs[0] = z.cs[1] = z.cs[2] = z.cs[3] = 0;
        z.count = 0;
        z.nj = 0;
        z.mn = ~0u;
        z.mx = 0;
        s_h[i] = z;
    }
    // The tile's records and the HALO records before it (rows of GB, striped,
    // coalesced): every column is loaded first, so that all loads are in flight
    // together; then keys, speeds and segment-start bits.  A record's
    // predecessor is the lane below; lane 0 takes it from lane 63 of the wave
    // row before (through LDS), the first row's from memory.  Shards are found
    // from the first row's one forward.
    constexpr int HR = HALO / GB;  // halo rows
    constexpr int NR = HR + GI;    // rows loaded
    const int lane = lane_id();
    const int w = t / WAVE;
    const long base = (long)tile0 - HALO;  // record of LDS position 0
    i64 vj[NR], vt[NR];
    double vla[NR], vlo[NR];
    float vsp[GI];
    uint8_t vlt[NR];
    // direction inputs (only in the forms with a direction dimension)
    float vh[Pol::kDir == 1 ? NR : 1];
    double vb[Pol::kDir == 2 ? NR : 1];
    uint8_t vbf[Pol::kDir == 2 ? NR : 1];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        // positions outside [0, n) read a record in range (ignored below): no
        // branches between the loads
        long r = base + rr * GB + t;
        r = r < 0 ? 0 : (r < (long)n ? r : (long)n - 1);
        vj[rr] = jid[r];
        vt[rr] = ts[r];
        vla[rr] = lat[r];
        vlo[rr] = lon[r];
        if (rr >= HR) vsp[rr - HR] = spd[r];
        vlt[rr] = Pol::kStream ? (uint8_t)pol.late((u64)r) : (uint8_t)0;
        if constexpr (Pol::kDir == 1) vh[rr] = g.hdg[r];
        if constexpr (Pol::kDir == 2) {
            vb[rr] = g.brg[r];
            vbf[rr] = g.bfl[r];
        }
    }
    if (t == 0) {
        s_pj = base > 0 ? jid[base - 1] : 0;
        s_ptb = base > 0 ? time_bin(g, ts[base - 1]) : 0;
        s_plt = (Pol::kStream && base > 0) ? (uint8_t)pol.late((u64)(base - 1)) : (uint8_t)0;
        s_lo = -1;
        s_npend = 0;
        s_np = 0;
        s_kmax = 0;
    }
    u64 n_out = 0;
    const u32 sh0 = g.S > 1 ? shard_of(g.soff, g.S, (u64)(base > 0 ? base : 0)) : 0u;
    uint8_t seg_b[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        const int q = rr * GB + t;
        const long r = base + q;
        const bool in = r >= 0 && r < (long)n;
        i64 k = -1, tb = 0;
        u32 sh = sh0;
        if (in) {
            if (g.S > 1)
                while (sh + 1 < g.S && g.soff[sh + 1] <= (u64)r) ++sh;
            u32 dir = 0;
            if constexpr (Pol::kDir == 1) dir = dir_sector(g, (double)vh[rr], true);
            if constexpr (Pol::kDir == 2) dir = dir_sector(g, vb[rr], (vbf[rr] & CV_FLAG_BEARING_OK) != 0);
            k = grid_key_in(g, sh, vt[rr], vla[rr], vlo[rr], tb, dir);
            if (rr >= HR && k < 0) {
                ++n_out;
                if (g.sout) atomicAdd((unsigned long long*)&g.sout[sh], 1ull);
            }
        }
        const i64 jp = __shfl_up(vj[rr], 1, WAVE);
        const i64 tbp = __shfl_up(tb, 1, WAVE);
        const u32 ltp = Pol::kStream ? (u32)__shfl_up((u32)vlt[rr], 1, WAVE) : 0u;
        const i64 kp = __shfl_up(k, 1, WAVE);
        if (lane == WAVE - 1) {
            s_lj[rr][w] = vj[rr];
            s_ltb[rr][w] = tb;
            s_llt[rr][w] = vlt[rr];
            s_lk[rr][w] = k;
        }
        // lane 0's bit is completed below, once lane 63 of the row before is in LDS;
        // a change of the late status starts a segment too
        const bool seg = r == 0 || (lane > 0 && (vj[rr] != jp || tb != tbp || (u32)vlt[rr] != ltp)) ||
                         (g.S > 1 && g.soff[sh] == (u64)r);
        seg_b[rr] = ((!in || seg) ? B_SEG : 0) | (vlt[rr] ? B_LATE : 0) | ((lane > 0 && k != kp) ? B_RUN : 0);
        if (lane == 0) s_ltbs[rr][w] = tb;
        s_key[q] = k;
        if (rr >= HR) s_spd[q - HALO] = in ? vsp[rr - HR] : 0.f;
        if (rr >= HR) {
            const u64 om = __ballot(in && spd_odd(vsp[rr - HR]));
            if (lane == 0) s_rodd[rr][w] = om != 0;
        }
    }
    __syncthreads();
    // Segment and run starts of lane 0 (its predecessor is lane 63 of the wave
    // row before, through LDS), then the run-head list: the heads of the
    // loaded positions in position order, placed by per-row ballots and one
    // prefix over the (row, wave) counts.  Position 0 always opens the list.
    const int qend = HALO + (int)tvalid;
    int lo_cand = -1;
    u64 hm[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        const int q = rr * GB + t;
        const long r = base + q;
        uint8_t b = seg_b[rr];
        if (lane == 0 && r > 0 && r < (long)n && !(b & B_SEG)) {
            // predecessor: lane 63 of the previous wave row
            const bool first_row = w == 0 && rr == 0;
            const int pr = w > 0 ? rr : rr - 1;
            const int pw = w > 0 ? w - 1 : NWG - 1;
            const i64 pj = first_row ? s_pj : s_lj[pr][pw];
            const i64 ptb = first_row ? s_ptb : s_ltb[pr][pw];
            const uint8_t plt = first_row ? s_plt : s_llt[pr][pw];
            if (vj[rr] != pj || s_ltbs[rr][w] != ptb || (Pol::kStream && vlt[rr] != plt)) b |= B_SEG;
            else if (!first_row && s_key[q] != s_lk[pr][pw]) b |= B_RUN;
        }
        if ((b & B_SEG) || q == 0) b |= B_RUN;
        if (rr >= HR) {
            // a record whose speed is outside the fast format is a run of its
            // own: it and the record after it start runs (the tile's first
            // record starts a piece of the aggregation anyway)
            const int pr = w > 0 ? rr : rr - 1;
            const int pw = w > 0 ? w - 1 : NWG - 1;
            const bool chk = s_rodd[rr][w] || (lane == 0 && pr >= HR && s_rodd[pr][pw]);
            if (chk && r < (long)n) {
                const int qt = q - HALO;
                if (spd_odd(s_spd[qt]) || (qt > 0 && spd_odd(s_spd[qt - 1]))) b |= B_RUN;
            }
        }
        s_bits[q] = b;
        if ((b & B_SEG) && q <= HALO) lo_cand = q;
        hm[rr] = __ballot((b & B_RUN) && r < (long)n);
        if (lane == 0) s_cnt[rr * NWG + w] = (u32)__popcll(hm[rr]);
    }
    // the tile's first segment starts at the last segment start at or before
    // the tile's first record; none in the halo: it starts further back
    if (lo_cand >= 0) atomicMax(&s_lo, lo_cand);
    __syncthreads();
    const bool exhausted = s_lo < 0;
    int L;
    {
        static_assert(NR * NWG <= WAVE, "one count per lane");
        const u32 c = lane < NR * NWG ? s_cnt[lane] : 0u;
        const u32 inc = wave_inclusive_sum(c);
        L = (int)__shfl(inc, NR * NWG - 1, WAVE);
        const u64 below = (1ull << lane) - 1ull;
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            const int q = rr * GB + t;
            const u32 off = __shfl(inc - c, rr * NWG + w, WAVE);
            if ((hm[rr] >> lane) & 1ull)
                s_lpos[off + (u32)__popcll(hm[rr] & below)] = (uint16_t)(q | ((s_bits[q] & B_SEG) ? 0x8000 : 0));
        }
    }
    __syncthreads();

    // distinct-journey flag of every run head inside the tile: no earlier run
    // head of its segment has the same key (and, in the serving form, the key
    // is not among the cells the journey's open segment carried over)
    for (int e = t; e < L; e += GB) {
        const u32 pe = s_lpos[e];
        const int q = (int)(pe & 0x7FFFu);
        if (q < HALO) continue;
        const i64 k = s_key[q];
        if (k < 0 || (s_bits[q] & B_LATE)) continue;
        bool first = true;
        long r0 = base + q;  // the segment's first record
        if (!(pe & 0x8000u)) {
            // back over the earlier heads, four per round (their loads issued
            // together), until the same key or the segment's start
            int f = e - 1;
            bool closed = false;
            while (f >= 0) {
                u32 pf[4];
                i64 kf[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) pf[u] = s_lpos[f - u >= 0 ? f - u : 0];
#pragma unroll
                for (int u = 0; u < 4; ++u) kf[u] = s_key[pf[u] & 0x7FFFu];
                bool stop = false;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (stop) continue;
                    if (f - u < 0) {
                        stop = true;
                        f = -1;
                    } else if (kf[u] == k) {
                        first = false;
                        stop = true;
                    } else if (pf[u] & 0x8000u) {
                        closed = true;
                        r0 = base + (long)(pf[u] & 0x7FFFu);
                        stop = true;
                    }
                }
                if (stop) break;
                f -= 4;
            }
            if (first && f < 0 && !closed && exhausted) {
                // the segment starts before the loaded halo: left to the block-wide scan below
                s_bits[q] |= B_PEND;
                atomicAdd(&s_npend, 1u);
                continue;
            }
        }
        if (Pol::kStream && first && pol.carried((u64)r0, (u64)k)) first = false;
        if (first) {
            s_bits[q] |= B_FIRST;
            if (Pol::kStream) pol.first((u64)(base + q), (u64)k);
        }
    }
    __syncthreads();
    // Pending heads all lie in the tile's first segment, which starts before
    // the loaded halo.  The block reads that segment's earlier records
    // backwards, GB at a time (coalesced), until the chunk that holds the
    // segment's first record, and marks every pending key it meets.  The keys
    // sit in an open-addressing set in the LDS of the group table (not in use
    // yet), at most LHS / 2 of them per round.
    if (exhausted && s_npend > 0) {
        constexpr u32 PR = LHS / 2;
        u32* s_pfound = reinterpret_cast<u32*>(s_h);
        u32* s_pq = s_pfound + LHS;
        u32 left = s_npend;
        while (left > 0) {
            for (int i = t; i < LHS; i += GB) s_hkey[i] = GEMPTY;
            if (t == 0) {
                s_pn = 0;
                s_nfound = 0;
                s_r0[0] = 0;
                s_r0[1] = 0;
            }
            __syncthreads();
            for (int q = t; q < qend; q += GB) {
                if (!(s_bits[q] & B_PEND)) continue;
                if (atomicAdd(&s_pn, 1u) >= PR) continue;  // a later round
                s_bits[q] &= (uint8_t)~B_PEND;
                const u64 k = (u64)s_key[q];
                u32 h = (u32)mix64(k) & (LHS - 1);
                while (atomicCAS((unsigned long long*)&s_hkey[h], (unsigned long long)GEMPTY,
                                 (unsigned long long)k) != GEMPTY)
                    h = (h + 1) & (LHS - 1);  // pending keys are distinct and at most half the slots
                s_pq[h] = (u32)q;
                s_pfound[h] = 0;
            }
            __syncthreads();
            const u32 taken = s_pn < PR ? s_pn : PR;
            long top = base - 1;  // records [top - GB + 1, top] this chunk
            long r0 = -1;         // the segment's first record, once met
            for (int it = 0;; ++it) {
                const long r = top - t;
                long c = -1;  // the segment starts at c (when r belongs to a boundary)
                i64 k = -1;
                if (r >= 0) {
                    i64 tb;
                    k = grid_key(g, (u64)r, ts[r], lat[r], lon[r], tb, dir_at<Pol::kDir>(g, (u64)r));
                    if (Pol::kStream && pol.late((u64)r)) {
                        c = r + 1;  // late records are outside every segment of non-late ones
                        k = -1;
                    } else if (seg_start(g, jid, ts, (u64)r, tb) || (Pol::kStream && pol.late((u64)(r - 1)))) {
                        c = r;
                    }
                }
                if (c >= 0) atomicMax(&s_r0[it & 1], (unsigned long long)(c + 1));
                __syncthreads();
                const long rc = (long)s_r0[it & 1] - 1;  // -1: the segment goes on below this chunk
                if (t == 0) s_r0[(it + 1) & 1] = 0;
                if (k >= 0 && r >= rc) {
                    u32 h = (u32)mix64((u64)k) & (LHS - 1);
                    for (int pr = 0; pr < LHS; ++pr) {
                        const u64 cur = s_hkey[h];
                        if (cur == (u64)k) {
                            if (atomicExch(&s_pfound[h], 1u) == 0) atomicAdd(&s_nfound, 1u);
                            break;
                        }
                        if (cur == GEMPTY) break;
                        h = (h + 1) & (LHS - 1);
                    }
                }
                __syncthreads();
                if (rc >= 0) {
                    r0 = rc;
                    break;
                }
                if (s_nfound == taken) break;  // every pending key met: none counts its journey
                top -= GB;
            }
            for (int h = t; h < LHS; h += GB) {
                const u64 k = s_hkey[h];
                if (k == GEMPTY || s_pfound[h]) continue;
                const int q = (int)s_pq[h];
                if (Pol::kStream && pol.carried((u64)r0, k)) continue;
                s_bits[q] |= B_FIRST;
                if (Pol::kStream) pol.first((u64)(base + q), k);
            }
            __syncthreads();
            left -= taken;
        }
        // the LDS group table back to empty
        for (int i = t; i < LHS; i += GB) {
            s_hkey[i] = GEMPTY;
            LSlot z;
            z.cs[0] = z.cs[1] = z.cs[2] = z.cs[3] = 0;
            z.count = 0;
            z.nj = 0;
            z.mn = ~0u;
            z.mx = 0;
            s_h[i] = z;
        }
        __syncthreads();
    }
    // Aggregation: every wave takes GT/4 records of the tile, every lane PER
    // consecutive ones of them.  A lane folds its records serially into
    // pieces cut at run starts: a run that starts and ends inside the lane is
    // one LDS hash insert; the piece before the lane's first start continues
    // a run from the lanes below, and the piece after its last start goes on
    // into the lanes above.  One segmented scan over the lanes joins those
    // pieces, and the lane where a run ends inserts it.  A wave's first record
    // starts a piece of its own.  All aggregates add (or take min / max), so
    // where a run is cut into pieces changes nothing.  Flags are read 8 to a
    // word and speeds 4 to a word; keys only at run starts (a run has one key).
    {
        constexpr int WREC = GT / (GB / WAVE);
        constexpr int PER = WREC / WAVE;
        static_assert(PER == 8, "one 64-bit word of flags per lane");
        const int w = t / WAVE, l = lane_id();
        const int qa = HALO + w * WREC;
        const int q0 = qa + PER * l;
        const int nv = qend - q0 < 0 ? 0 : (qend - q0 > PER ? PER : qend - q0);
        const u64 bits8 = *reinterpret_cast<const u64*>(&s_bits[q0]);
        const float4 spa = *reinterpret_cast<const float4*>(&s_spd[q0 - HALO]);
        const float4 spb = *reinterpret_cast<const float4*>(&s_spd[q0 - HALO + 4]);
        const float sp8[PER] = {spa.x, spa.y, spa.z, spa.w, spb.x, spb.y, spb.z, spb.w};
        RunPart cur, pre;
        run_reset(cur);
        run_reset(pre);
        bool hh = false;  // the lane holds a run start
        i64 ck = nv > 0 ? s_key[q0] : -1;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            if (i >= nv) break;
            const uint8_t b = (uint8_t)(bits8 >> (8 * i));
            if ((b & B_RUN) || (i == 0 && l == 0)) {
                if (i > 0) {
                    if (!hh) pre = cur;
                    else if (ck >= 0 && cur.cn) run_insert<LHS>(s_hkey, s_h, sk, &s_np, &s_kmax, blockIdx.x, (u64)ck, cur);
                    run_reset(cur);
                    ck = s_key[q0 + i];
                }
                hh = true;
            }
            if (ck >= 0) {
                const float sp = sp8[i];
                i64 x;
                if (spd_fix53(sp, x)) {
                    add128(cur.lo, cur.hi, (u64)x, (u64)(x >> 63));
                } else {
                    // a speed outside the 128-bit range: the record is a piece of
                    // its own (both neighbours start runs), so cur was empty
                    cur.lo = (u64)__float_as_uint(sp);
                    cur.hi = 0;
                    cur.cn |= RUN_ODD;
                }
                cur.cn += 1u | ((b & B_FIRST) ? (1u << 16) : 0u);
                const u32 o = ord_f32(sp);
                cur.mn = o < cur.mn ? o : cur.mn;
                cur.mx = o > cur.mx ? o : cur.mx;
            }
        }
        // the piece that goes on into the lanes above (the whole lane when it
        // holds no start), joined across lanes
        RunPart out = cur;
        run_seg_scan(out, hh);
        // the run open below this lane: the scan's value of the lane below
        RunPart in;
        in.lo = (u64)__shfl_up((unsigned long long)out.lo, 1, WAVE);
        in.hi = (u64)__shfl_up((unsigned long long)out.hi, 1, WAVE);
        in.cn = (u32)__shfl_up(out.cn, 1, WAVE);
        in.mn = (u32)__shfl_up(out.mn, 1, WAVE);
        in.mx = (u32)__shfl_up(out.mx, 1, WAVE);
        if (l == 0) run_reset(in);
        if (hh && l > 0) {
            run_combine(in, pre);
            const i64 kb = s_key[q0 - 1];  // the run ends in this lane: its key is the record below's
            if (kb >= 0 && in.cn) run_insert<LHS>(s_hkey, s_h, sk, &s_np, &s_kmax, blockIdx.x, (u64)kb, in);
        }
        const int qlast = (qa + WREC < qend ? qa + WREC : qend) - 1;
        if (l == WAVE - 1 && qlast >= qa) {
            const i64 ke = s_key[qlast];  // the run open at the wave's end
            if (ke >= 0 && out.cn) run_insert<LHS>(s_hkey, s_h, sk, &s_np, &s_kmax, blockIdx.x, (u64)ke, out);
        }
    }
    // out-of-grid count (one global atomic per tile, only when non-zero)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) n_out += __shfl_xor(n_out, d, WAVE);
    if (lane_id() == 0) s_out[t / WAVE] = n_out;
    __syncthreads();
    if (t == 0) {
        u64 tot = 0;
        for (int w = 0; w < GB / WAVE; ++w) tot += s_out[w];
        if (tot) atomicAdd((unsigned long long*)&meta->n_out, (unsigned long long)tot);
    }
    // the LDS table to the sink
    for (int i = t; i < LHS; i += GB) {
        const u64 key = s_hkey[i];
        if (key == GEMPTY) continue;
        const LSlot& sl = s_h[i];
        const Fx192 sum = fx_from_cs(sl.cs);
        sk.put(key, sl.count, sl.nj, sum, sl.mn, sl.mx, &s_np, &s_kmax, blockIdx.x);
    }
}


}  // namespace
}  // namespace cv
