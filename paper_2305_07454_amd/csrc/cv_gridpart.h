// cv_gridpart.h -- the tile kernel of the plain and batched grid aggregate and
// of its direction forms (cv_grid.hip describes the whole call).
//
// Per tile of GT records in (journey, time) order it writes one partial row
// per (journey, key) that the tile holds, in record order.  A key carries its
// time bin, so the records of one (journey, key) all lie in one (journey,
// time-bin) segment; inside the tile a run of equal keys is tied to the
// earliest run of the same key in its segment (a bounded look back over the
// run heads), and the runs tied to one root add into one LDS accumulator.
// Distinct journeys are not counted here: the merge of the partials counts a
// journey once per key, because a key's partials reach it in record order,
// where the partials of one journey are adjacent.
#pragma once
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_gridagg.h"
#include "cv_gridtab.h"

namespace cv {
namespace {

// (journey, key) accumulators per tile in LDS: 320 keep the kernel's LDS at
// 40 KB, so that four workgroups share a CU (a tile of the batched workload's
// 0.001 deg x 1 min grid holds about 250 keys on average; a tile with more
// roots takes the path where runs without an accumulator write own rows)
constexpr int PR_MAX = 320;
constexpr int SCAN_BACK = 128;  // run heads a run head looks back over for its key
// what a run head's entry of s_root holds once the rows are numbered
constexpr uint16_t H_NONE = 0xFFFF;  // run outside the grid: dropped
constexpr uint16_t H_SELF = 0xFFFE;  // (before numbering) run with a speed outside the fast format
constexpr uint16_t H_ROW = 0x8000;   // the run writes its own row (index in the low bits)
constexpr uint16_t H_ACC = 0x4000;   // a root with an accumulator (its index in the low bits)
// other values: the head index of the run's root (which holds H_ACC)
constexpr uint16_t L_SEG = 0x8000;   // s_lpos: the head starts a (journey, time-bin) segment
constexpr uint16_t L_ODD = 0x4000;   // s_lpos: the head's record has a speed outside the fast format
constexpr uint8_t B_ODD = 32;        // record speed outside the 128-bit fast format
constexpr u32 PART_ODD = 0x80000000u;

// Where the partial rows go: a region of GT rows per tile, their count and
// their largest key per tile.
struct PartSink {
    u64* key;     // [tiles * GT]
    GPart* part;  // [tiles * GT]
    u32* count;   // [tiles]
    u64* kmax;    // [tiles]
};

// The 2^-53-unit 96-bit sum of a partial in the 192-bit 2^-149-unit format:
// the value times 2^96, taken modulo 2^192.
__device__ __forceinline__ Fx192 part_sum192(const GPart& p)
{
    Fx192 r;
    r.w[0] = 0;
    r.w[1] = (u64)p.s[0] << 32;
    r.w[2] = (u64)p.s[1] | ((u64)p.s[2] << 32);
    return r;
}

// a partial row from a 128-bit two's complement sum (its low 96 bits)
__device__ __forceinline__ GPart make_part(i64 jid, u64 lo, u64 hi, u32 cn, u32 mn, u32 mx)
{
    GPart p;
    p.jid = jid;
    p.s[0] = (u32)lo;
    p.s[1] = (u32)(lo >> 32);
    p.s[2] = (u32)hi;
    p.cn = cn;
    p.mn = mn;
    p.mx = mx;
    return p;
}

// Four waves per SIMD for the plain key (what the LDS allows); the direction
// forms carry a heading or bearing column too and keep three, which their
// registers need without spilling.
// FL: journey (and shard) starts come from the kinematics' FIRST flags, one
// byte per record, instead of comparing journey ids with the predecessor's;
// the ids are then read only for the partial rows.
template <int KD, bool FL = false>
__global__ void __launch_bounds__(GB) __attribute__((amdgpu_waves_per_eu(KD == 0 ? 4 : 3)))
k_grid_part(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts, const double* __restrict__ lat,
            const double* __restrict__ lon, const float* __restrict__ spd, Spec g, PartSink sk, GridMeta* meta,
            const uint8_t* __restrict__ first)
{
    constexpr int NWG = GB / WAVE;
    constexpr int WREC = GT / NWG;  // consecutive records per wave in the aggregation
    constexpr int PER = WREC / WAVE;
    constexpr int HPM = GT / GB;    // run heads per thread at most in the numbering
    static_assert(PER == 8, "one 64-bit word of flags per lane");
    static_assert(GI * NWG <= WAVE, "one row count per lane");
    static_assert(PR_MAX < H_ACC && GT <= 0x3FFF, "head and accumulator indices fit the tags");
    __shared__ i64 s_hkey[GT];       // run head -> its key
    __shared__ __attribute__((aligned(16))) uint8_t s_bits[GT];
    __shared__ uint16_t s_lpos[GT];  // run head -> position | L_SEG | L_ODD
    __shared__ uint16_t s_root[GT];  // run head -> its root head; then the H_* info
    __shared__ u64 s_c0[PR_MAX], s_c1[PR_MAX];  // sum: two carry-save 43-bit chunks (mod 2^86)
    __shared__ u32 s_cn[PR_MAX], s_mn[PR_MAX], s_mx[PR_MAX];
    __shared__ uint16_t s_orow[PR_MAX], s_opos[PR_MAX], s_ohead[PR_MAX];  // accumulator -> row, root position, head
    __shared__ i64 s_lj[GI][NWG], s_ltb[GI][NWG], s_lk[GI][NWG];  // lane 63 of every wave row
    __shared__ u32 s_cnt[GI * NWG];
    __shared__ uint8_t s_rodd[GI][NWG];
    __shared__ u64 s_tmp[GB / WAVE];
    __shared__ u32 s_tmp32[GB / WAVE];
    __shared__ u64 s_red[GB / WAVE];

    const int t = threadIdx.x;
    const int lane = lane_id();
    const int w = t / WAVE;
    const u64 tile0 = (u64)blockIdx.x * GT;
    const u32 tvalid = (u32)((u64)n - tile0 < (u64)GT ? (u64)n - tile0 : (u64)GT);

    // 1. the tile's records, rows of GB striped over the block (coalesced);
    //    every column is loaded first so that all loads are in flight together
    i64 vj[FL ? 1 : GI], vt[GI], vtb[GI], vk[GI];
    uint8_t vfl[FL ? GI : 1];
    double vla[GI], vlo[GI];
    float vsp[GI];
    float vh[KD == 1 ? GI : 1];
    double vb[KD == 2 ? GI : 1];
    uint8_t vbf[KD == 2 ? GI : 1];
#pragma unroll
    for (int rr = 0; rr < GI; ++rr) {
        u64 r = tile0 + (u64)(rr * GB + t);
        r = r < n ? r : (u64)n - 1;  // past the end: a record in range, not used
        if constexpr (FL) vfl[rr] = first[r];
        else vj[rr] = jid[r];
        vt[rr] = ts[r];
        vla[rr] = lat[r];
        vlo[rr] = lon[r];
        vsp[rr] = spd[r];
        if constexpr (KD == 1) vh[rr] = g.hdg[r];
        if constexpr (KD == 2) {
            vb[rr] = g.brg[r];
            vbf[rr] = g.bfl[r];
        }
    }
    // the tile's first shard, its start and the next shard's start (the same
    // addresses in every lane); a record before the next start needs no search
    u32 sh0 = 0;
    u64 s0start = ~0ull, nxt = ~0ull;
    if (g.S > 1) {
        sh0 = shard_of(g.soff, g.S, tile0);
        s0start = g.soff[sh0];
        nxt = sh0 + 1 < g.S ? g.soff[sh0 + 1] : ~0ull;
    }
    u64 n_out = 0;
    uint8_t bq[GI];
#pragma unroll
    for (int rr = 0; rr < GI; ++rr) {
        const int q = rr * GB + t;
        const u64 r = tile0 + (u64)q;
        const bool in = (u32)q < tvalid;
        i64 k = -1, tb = 0;
        bool sstart = false;
        if (in) {
            u32 sh = sh0;
            if (g.S > 1) {
                if (r < nxt) {
                    sstart = r == s0start;
                } else {
                    sh = shard_from(g.soff, g.S, sh0, r);
                    sstart = g.soff[sh] == r;
                }
            }
            u32 dir = 0;
            if constexpr (KD == 1) dir = dir_sector(g, (double)vh[rr], true);
            if constexpr (KD == 2) dir = dir_sector(g, vb[rr], (vbf[rr] & CV_FLAG_BEARING_OK) != 0);
            k = grid_key_in(g, sh, vt[rr], vla[rr], vlo[rr], tb, dir);
            if (k < 0) {
                ++n_out;
                if (g.sout) atomicAdd((unsigned long long*)&g.sout[sh], 1ull);
            }
        }
        vtb[rr] = tb;
        vk[rr] = k;
        const i64 tbp = __shfl_up(tb, 1, WAVE);
        const i64 kp = __shfl_up(k, 1, WAVE);
        if (lane == WAVE - 1) {
            if constexpr (!FL) s_lj[rr][w] = vj[rr];
            s_ltb[rr][w] = tb;
            s_lk[rr][w] = k;
        }
        // lane 0 compares with lane 63 of the wave row before, below
        bool seg;
        if constexpr (FL) {
            // FIRST marks every journey start, shard starts included
            seg = (in && (vfl[rr] & CV_FLAG_FIRST)) || (lane > 0 && tb != tbp);
        } else {
            const i64 jp = __shfl_up(vj[rr], 1, WAVE);
            seg = sstart || (lane > 0 && (vj[rr] != jp || tb != tbp));
        }
        const bool odd = in && spd_odd(vsp[rr]);
        // the tile's first record and the first record of every wave's share
        // of the aggregation start runs: no run is split between waves
        const bool run = seg || q % WREC == 0 || (lane > 0 && k != kp);
        bq[rr] = (seg ? B_SEG : 0) | (run ? B_RUN : 0) | (odd ? B_ODD : 0);
        const u64 om = __ballot(odd);
        if (lane == 0) s_rodd[rr][w] = om != 0;
    }
    __syncthreads();

    // 2. segment and run starts of lane 0, runs of one record around speeds
    //    outside the fast format, and the run heads of each wave row
    u64 hm[GI];
#pragma unroll
    for (int rr = 0; rr < GI; ++rr) {
        const int q = rr * GB + t;
        const bool in = (u32)q < tvalid;
        uint8_t b = bq[rr];
        const int pr = w > 0 ? rr : rr - 1;
        const int pw = w > 0 ? w - 1 : NWG - 1;
        if (lane == 0 && q > 0 && in && !(b & B_SEG)) {
            if ((!FL && vj[FL ? 0 : rr] != s_lj[pr][pw]) || vtb[rr] != s_ltb[pr][pw]) b |= B_SEG | B_RUN;
            else if (vk[rr] != s_lk[pr][pw]) b |= B_RUN;
        }
        const bool chk = s_rodd[rr][w] || (lane == 0 && q > 0 && s_rodd[pr][pw]);
        if (chk && in && ((b & B_ODD) || (q > 0 && spd_odd(spd[tile0 + (u64)q - 1])))) b |= B_RUN;
        bq[rr] = b;
        s_bits[q] = b;
        hm[rr] = __ballot((b & B_RUN) && in);
        if (lane == 0) s_cnt[rr * NWG + w] = (u32)__popcll(hm[rr]);
    }
    __syncthreads();

    // 3. the run-head list in position order (per-row ballots placed by one
    //    prefix over the (row, wave) counts), with each head's key
    int L;
    {
        const u32 c = lane < GI * NWG ? s_cnt[lane] : 0u;
        const u32 inc = wave_inclusive_sum(c);
        L = (int)__shfl(inc, GI * NWG - 1, WAVE);
        const u64 below = (1ull << lane) - 1ull;
#pragma unroll
        for (int rr = 0; rr < GI; ++rr) {
            const int q = rr * GB + t;
            const u32 off = __shfl(inc - c, rr * NWG + w, WAVE);
            if ((hm[rr] >> lane) & 1ull) {
                const u32 e = off + (u32)__popcll(hm[rr] & below);
                s_lpos[e] = (uint16_t)(q | ((bq[rr] & B_SEG) ? L_SEG : 0) | ((bq[rr] & B_ODD) ? L_ODD : 0));
                s_hkey[e] = vk[rr];
            }
        }
    }
    __syncthreads();

    // 4. the root of every run head: the earliest head of its segment with the
    //    same key (itself when there is none); a look back that stops at the
    //    window's end before the segment's start makes the head its own root.
    //    Several roots of one (journey, key) only cost extra partial rows.
    for (int e = t; e < L; e += GB) {
        const uint16_t pe = s_lpos[e];
        const i64 k = s_hkey[e];
        uint16_t root;
        if (k < 0) {
            root = H_NONE;
        } else if (pe & L_ODD) {
            root = H_SELF;
        } else {
            int rt = e;
            bool done = (pe & L_SEG) || e == 0;
            int f = e - 1;
            for (int steps = 0; !done && steps < SCAN_BACK; steps += 4) {
                uint16_t pf[4];
                i64 kf[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int x = f - u >= 0 ? f - u : 0;
                    pf[u] = s_lpos[x];
                    kf[u] = s_hkey[x];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (done) continue;
                    if (kf[u] == k && !(pf[u] & L_ODD)) rt = f - u;
                    if ((pf[u] & L_SEG) || f - u == 0) done = true;
                }
                f -= 4;
            }
            root = (uint16_t)(done ? rt : e);
        }
        s_root[e] = root;
    }
    // run heads before each lane's records in the aggregation layout
    const int qa = w * WREC;
    const int q0 = qa + PER * lane;
    const int nv = (int)tvalid - q0 < 0 ? 0 : ((int)tvalid - q0 > PER ? PER : (int)tvalid - q0);
    const u64 bits8 = *reinterpret_cast<const u64*>(&s_bits[q0]);
    u32 hc = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i)
        if (i < nv && ((bits8 >> (8 * i)) & B_RUN)) ++hc;
    __syncthreads();

    // 5. numbering, in list order: roots get accumulators (the first PR_MAX of
    //    them), rows follow position order (a root with an accumulator writes
    //    one; a run of its own writes one; beyond PR_MAX roots, every run of a
    //    root without an accumulator writes its own).  One packed scan gives
    //    the roots, the rows when no root lacks an accumulator, and the run
    //    heads before each aggregation lane.
    const int HP = (L + GB - 1) / GB;
    const int h0 = t * HP < L ? t * HP : L;
    const int h1 = h0 + HP < L ? h0 + HP : L;
    u32 nr = 0, nw = 0;
#pragma unroll
    for (int u = 0; u < HPM; ++u) {
        const int e = h0 + u;
        if (e >= h1) continue;
        const uint16_t v = s_root[e];
        nr += v == (uint16_t)e;
        nw += v == (uint16_t)e || v == H_SELF;
    }
    u64 tot;
    const u64 ex = block_exclusive_sum<GB>((u64)nr | ((u64)nw << 16) | ((u64)hc << 32), s_tmp, tot);
    const u32 R = (u32)(tot & 0xFFFF);
    const u32 hbase = (u32)(ex >> 32);
    u32 ROWS = (u32)((tot >> 16) & 0xFFFF);
    u64 kmax = 0;
    if (R <= (u32)PR_MAX) {
        u32 o = (u32)(ex & 0xFFFF), row = (u32)((ex >> 16) & 0xFFFF);
#pragma unroll
        for (int u = 0; u < HPM; ++u) {
            const int e = h0 + u;
            if (e >= h1) continue;
            const uint16_t v = s_root[e];
            if (v == (uint16_t)e) {
                const int q = s_lpos[e] & 0x07FF;
                s_orow[o] = (uint16_t)row++;
                s_opos[o] = (uint16_t)q;
                s_ohead[o] = (uint16_t)e;
                s_root[e] = (uint16_t)(H_ACC | o++);
            } else if (v == H_SELF) {
                s_root[e] = (uint16_t)(H_ROW | row++);
            } else {
                continue;  // members keep their root's head index; dropped runs stay H_NONE
            }
            const u64 k = (u64)s_hkey[e];
            kmax = k > kmax ? k : kmax;
        }
    } else {
        // more roots than accumulators: a second count of the rows, since the
        // runs tied to a root without one each write their own
        {
            u32 o = (u32)(ex & 0xFFFF);
#pragma unroll
            for (int u = 0; u < HPM; ++u) {
                const int e = h0 + u;
                if (e < h1 && s_root[e] == (uint16_t)e) s_root[e] = (uint16_t)(H_ACC | o++);
            }
        }
        __syncthreads();
        u32 nrow = 0;
#pragma unroll
        for (int u = 0; u < HPM; ++u) {
            const int e = h0 + u;
            if (e >= h1) continue;
            const uint16_t v = s_root[e];
            if (v == H_NONE) continue;
            if (v == H_SELF || (v & H_ACC)) ++nrow;
            else if ((s_root[v] & 0x3FFF) >= (u32)PR_MAX) ++nrow;
        }
        u32 rt;
        u32 row = block_exclusive_sum<GB>(nrow, s_tmp32, rt);
        ROWS = rt;
        uint16_t info[HPM];
#pragma unroll
        for (int u = 0; u < HPM; ++u) {
            const int e = h0 + u;
            info[u] = H_NONE;
            if (e >= h1) continue;
            const uint16_t v = s_root[e];
            uint16_t x = v;  // members of roots with an accumulator keep the root's index
            if (v == H_NONE) {
                continue;
            } else if (v == H_SELF) {
                x = (uint16_t)(H_ROW | row++);
            } else if (v & H_ACC) {
                const u32 o = v & 0x3FFF;
                if (o < (u32)PR_MAX) {
                    s_orow[o] = (uint16_t)row++;
                    s_opos[o] = (uint16_t)(s_lpos[e] & 0x07FF);
                    s_ohead[o] = (uint16_t)e;
                } else {
                    x = (uint16_t)(H_ROW | row++);
                }
            } else if ((s_root[v] & 0x3FFF) >= (u32)PR_MAX) {
                x = (uint16_t)(H_ROW | row++);
            }
            if (x & (H_ROW | H_ACC)) {
                const u64 k = (u64)s_hkey[e];
                kmax = k > kmax ? k : kmax;
            }
            info[u] = x;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < HPM; ++u)
            if (h0 + u < h1) s_root[h0 + u] = info[u];
    }
    const u32 RA = R < (u32)PR_MAX ? R : (u32)PR_MAX;
    for (u32 o = t; o < RA; o += GB) {
        s_c0[o] = 0;
        s_c1[o] = 0;
        s_cn[o] = 0;
        s_mn[o] = ~0u;
        s_mx[o] = 0;
    }
    __syncthreads();
    // the journey ids of the accumulator rows, fetched now, used at the end
    static_assert(PR_MAX <= 2 * GB, "two accumulator rows per thread");
    i64 rj0 = 0, rj1 = 0;
    if ((u32)t < RA) rj0 = jid[tile0 + s_opos[t]];
    if ((u32)(t + GB) < RA) rj1 = jid[tile0 + s_opos[t + GB]];

    // 6. every run reduced once (a lane folds its PER consecutive records into
    //    pieces cut at run starts; one segmented scan joins the pieces of runs
    //    that cross lanes) and added into its root's accumulator, or written
    //    as a row of its own
    auto put = [&](int e, const RunPart& p) {
        if (e < 0 || (p.cn & 0xFFFFu) == 0) return;
        uint16_t x = s_root[e];
        if (x == H_NONE) return;
        if (!(x & (H_ROW | H_ACC))) x = s_root[x];  // a member: its root's accumulator
        if (x & H_ROW) {
            const u32 row = x & 0x07FF;
            const int q = s_lpos[e] & 0x07FF;
            const u64 at = (u64)blockIdx.x * GT + row;
            sk.key[at] = (u64)s_hkey[e];
            sk.part[at] = make_part(jid[tile0 + (u64)q], p.lo, p.hi,
                                    (p.cn & 0xFFFFu) | ((p.cn & RUN_ODD) ? PART_ODD : 0u), p.mn, p.mx);
        } else {
            const u32 o = x & 0x3FFF;
            const u64 M43 = (1ull << 43) - 1;
            const u64 a0 = p.lo & M43;
            const u64 a1 = ((p.lo >> 43) | (p.hi << 21)) & M43;
            if (a0) atomicAdd((unsigned long long*)&s_c0[o], (unsigned long long)a0);
            if (a1) atomicAdd((unsigned long long*)&s_c1[o], (unsigned long long)a1);
            atomicAdd(&s_cn[o], p.cn & 0xFFFFu);
            atomicMin(&s_mn[o], p.mn);
            atomicMax(&s_mx[o], p.mx);
        }
    };
    {
        // the lane's speeds again from global memory (just read by the tile,
        // so from cache): staging them in LDS would cost the fourth workgroup
        float sp8[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) sp8[i] = spd[tile0 + (u64)(i < nv ? q0 + i : 0)];
        RunPart cur, pre;
        run_reset(cur);
        run_reset(pre);
        bool hh = false;          // the lane holds a run start
        int ec = (int)hbase - 1;  // head of the run the current piece belongs to
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            if (i >= nv) break;
            const uint8_t b = (uint8_t)(bits8 >> (8 * i));
            if (b & B_RUN) {
                if (i > 0) {
                    if (!hh) pre = cur;
                    else put(ec, cur);
                    run_reset(cur);
                }
                hh = true;
                ++ec;
            }
            const float sp = sp8[i];
            i64 x;
            if (spd_fix53(sp, x)) {
                add128(cur.lo, cur.hi, (u64)x, (u64)(x >> 63));
            } else {
                // a run of its own: cur was empty
                cur.lo = (u64)__float_as_uint(sp);
                cur.hi = 0;
                cur.cn |= RUN_ODD;
            }
            cur.cn += 1u;
            const u32 o = ord_f32(sp);
            cur.mn = o < cur.mn ? o : cur.mn;
            cur.mx = o > cur.mx ? o : cur.mx;
        }
        // the piece that goes on into the lanes above (the whole lane when it
        // holds no start), joined across lanes
        RunPart out = cur;
        run_seg_scan(out, hh);
        RunPart inr;
        inr.lo = (u64)__shfl_up((unsigned long long)out.lo, 1, WAVE);
        inr.hi = (u64)__shfl_up((unsigned long long)out.hi, 1, WAVE);
        inr.cn = (u32)__shfl_up(out.cn, 1, WAVE);
        inr.mn = (u32)__shfl_up(out.mn, 1, WAVE);
        inr.mx = (u32)__shfl_up(out.mx, 1, WAVE);
        if (lane == 0) run_reset(inr);
        if (hh && lane > 0) {
            // the run open below this lane ends here: its head is the last one before q0
            run_combine(inr, pre);
            put((int)hbase - 1, inr);
        }
        if (lane == WAVE - 1 && qa < (int)tvalid) put(ec, out);  // the run open at the wave's end
    }
    // out-of-grid count (one global atomic per tile, only when non-zero) and
    // the largest key of the tile's rows
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        n_out += __shfl_xor(n_out, d, WAVE);
        const u64 o = __shfl_xor(kmax, d, WAVE);
        kmax = o > kmax ? o : kmax;
    }
    if (lane == 0) {
        s_red[w] = kmax;
        s_tmp32[w] = (u32)n_out;
    }
    __syncthreads();

    // 7. the rows of the accumulators
    for (u32 o = t; o < RA; o += GB) {
        const u64 at = (u64)blockIdx.x * GT + s_orow[o];
        // the 128-bit sum from its two 43-bit carry-save chunks, mod 2^86 and
        // sign-extended (a tile's sum is below 2^74 in magnitude)
        const u64 c0 = s_c0[o], c1 = s_c1[o];
        u64 lo = c0 + (c1 << 43);
        u64 hi = (c1 >> 21) + (lo < c0 ? 1ull : 0ull);
        hi &= (1ull << 22) - 1;
        if (hi >> 21) hi |= ~((1ull << 22) - 1);
        sk.key[at] = (u64)s_hkey[s_ohead[o]];
        sk.part[at] = make_part(o < (u32)GB ? rj0 : rj1, lo, hi, s_cn[o], s_mn[o], s_mx[o]);
    }
    if (t == 0) {
        u64 km = 0, no = 0;
        for (int i = 0; i < NWG; ++i) {
            km = s_red[i] > km ? s_red[i] : km;
            no += s_tmp32[i];
        }
        sk.count[blockIdx.x] = ROWS;
        sk.kmax[blockIdx.x] = km;
        if (no) atomicAdd((unsigned long long*)&meta->n_out, (unsigned long long)no);
    }
}

}  // namespace
}  // namespace cv
