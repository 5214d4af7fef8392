// cv_grid.hip -- cv_grid_aggregate: the spatio-temporal lattice of the paper
// (Methods steps (3)-(5); Algorithm 2's floor((x - x_min) / x_step) bins; the
// count / sum / count-unique / mean reductions of Table 3), as a sparse,
// key-sorted group table over (journey, time)-sorted records.
//
//   k_grid_agg   per tile of GT records, staged in LDS with coalesced loads:
//     * key = (tbin * n_lat + ilat) * n_lon + ilon per record (-1 outside);
//     * runs: maximal stretches of one key inside one (journey, time-bin)
//       segment.  Records of one (journey, tbin) are contiguous after the sort,
//       so a run head counts its journey for the cell (distinct-journey flag)
//       iff no earlier run head of the same segment has the same key.  Run heads
//       are compacted into an LDS list and each one compares itself with the
//       earlier heads of its segment; segments entering the tile bring a halo
//       loaded on demand (global memory beyond it);
//     * each run is reduced by one thread (count, exact speed sum, min, max),
//       then inserted into an LDS open-addressing table; runs that find no LDS
//       slot spill straight to the HBM table; at tile end the LDS table is
//       merged into the HBM table with non-returning integer atomics (sums in
//       carry-save 40-bit chunks), so the result does not depend on the order;
//   k_grid_compact  occupied HBM slots -> (key, slot) pairs;
//   radix sort of the pairs by key (the same LSD sort as the record order);
//   k_grid_emit     rows in ascending key, sums rounded once to double.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cv_device.h"
#include "cv_host.h"
#include "cv_gridtab.h"
#include "cv_radix.h"

using namespace cv;

namespace {

constexpr int GB = 256;
constexpr int GI = 8;
constexpr int GT = GB * GI;
constexpr int HALO = 512;
constexpr int LHS_PROBES = 32;
struct LSlot {
    u64 cs[4];
    u32 count, nj, mn, mx;
};

constexpr uint8_t B_SEG = 1;   // first record of a (journey, time-bin) segment
constexpr uint8_t B_RUN = 2;   // first record of a run (segment start or key change)
constexpr uint8_t B_FIRST = 4; // run head whose key is new in its segment (counts its journey)

// partial aggregate of one run (or piece of a run)
struct RunPart {
    Fx192 sum;
    u32 count, nj, mn, mx;
};

__device__ __forceinline__ void run_reset(RunPart& p)
{
    fx_zero(p.sum);
    p.count = 0;
    p.nj = 0;
    p.mn = ~0u;
    p.mx = 0;
}

__device__ __forceinline__ void run_combine(RunPart& a, const RunPart& b)
{
    fx_add(a.sum, b.sum);
    a.count += b.count;
    a.nj += b.nj;
    a.mn = b.mn < a.mn ? b.mn : a.mn;
    a.mx = b.mx > a.mx ? b.mx : a.mx;
}

template <typename F>
__device__ __forceinline__ void run_shuffle(RunPart& o, const RunPart& p, F&& sh)
{
    o.sum.w[0] = sh(p.sum.w[0]);
    o.sum.w[1] = sh(p.sum.w[1]);
    o.sum.w[2] = sh(p.sum.w[2]);
    o.count = (u32)sh((u64)p.count);
    o.nj = (u32)sh((u64)p.nj);
    o.mn = (u32)sh((u64)p.mn);
    o.mx = (u32)sh((u64)p.mx);
}

__device__ __forceinline__ void run_wave_reduce(RunPart& p)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        RunPart o;
        run_shuffle(o, p, [&](u64 v) { return (u64)__shfl_xor((unsigned long long)v, d, WAVE); });
        run_combine(p, o);
    }
}

__device__ __forceinline__ void run_seg_scan(RunPart& p, bool head)
{
    const int l = lane_id();
    bool f = head;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        RunPart o;
        run_shuffle(o, p, [&](u64 v) { return (u64)__shfl_up((unsigned long long)v, d, WAVE); });
        const bool fo = __shfl_up(f, d, WAVE);
        if (l >= d) {
            if (!f) {
                run_combine(o, p);
                p = o;
            }
            f = f || fo;
        }
    }
}

// one run's partial into the tile's LDS table; no free slot within the probe
// limit spills it straight to the HBM table
template <int LHS>
__device__ __forceinline__ void run_insert(u64* s_hkey, LSlot* s_h, GEntry* tab, u64 gmask, GridMeta* meta, u64 key,
                                           const RunPart& p)
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
            fx_to_cs(p.sum, c);
            for (int i = 0; i < 4; ++i)
                if (c[i]) atomicAdd((unsigned long long*)&sl.cs[i], (unsigned long long)c[i]);
            atomicAdd(&sl.count, p.count);
            if (p.nj) atomicAdd(&sl.nj, p.nj);
            atomicMin(&sl.mn, p.mn);
            atomicMax(&sl.mx, p.mx);
            return;
        }
        h = (h + 1) & (LHS - 1);
    }
    g_insert(tab, gmask, meta, key, p.count, p.nj, p.sum, p.mn, p.mx);
}

template <int LHS>
__global__ void __launch_bounds__(GB)
k_grid_agg(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts, const double* __restrict__ lat,
           const double* __restrict__ lon, const float* __restrict__ spd, Spec g, GEntry* __restrict__ tab, u64 gmask,
           GridMeta* meta)
{
    constexpr int NQ = HALO + GT;
    __shared__ i64 s_key[NQ];       // keys per record; later the keys of the run-head list
    __shared__ uint8_t s_bits[NQ];
    __shared__ uint16_t s_lpos[NQ];  // run-head list: q | segment start << 15
    __shared__ float s_spd[GT];
    __shared__ u64 s_hkey[LHS];
    __shared__ LSlot s_h[LHS];
    __shared__ u32 s_tmp[GB / WAVE];
    __shared__ u32 s_flag;
    __shared__ u32 s_nlist;
    __shared__ u64 s_out[GB / WAVE];

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
    // tile records (striped, coalesced): key, segment-start bit, speed.  A
    // record's predecessor is the lane below (lane 0 reads its own); shards are
    // found from the tile's first one forward.
    u64 n_out = 0;
    const u32 sh0 = g.S > 1 ? shard_of(g.soff, g.S, tile0) : 0u;
    const int lane = lane_id();
#pragma unroll
    for (int ii = 0; ii < GI; ++ii) {
        const int i = ii * GB + t;
        const u64 r = tile0 + i;
        i64 k = -1, j = 0, tb = 0;
        float sp = 0.f;
        u32 sh = sh0;
        if (r < n) {
            if (g.S > 1)
                while (sh + 1 < g.S && g.soff[sh + 1] <= r) ++sh;
            j = jid[r];
            k = grid_key_in(g, sh, ts[r], lat[r], lon[r], tb);
            n_out += (k < 0);
            sp = spd[r];
        }
        i64 jp = __shfl_up(j, 1, WAVE);
        i64 tbp = __shfl_up(tb, 1, WAVE);
        if (lane == 0 && r < n && r > 0) {
            jp = jid[r - 1];
            tbp = floor_div64(ts[r - 1] - g.t0, g.bin_ms);
        }
        const bool seg = r == 0 || j != jp || tb != tbp || (g.S > 1 && g.soff[sh] == r);
        s_key[HALO + i] = k;
        s_bits[HALO + i] = (r >= n || seg) ? B_SEG : 0;
        s_spd[i] = sp;
    }
    if (t == 0) s_flag = 0;
    __syncthreads();
    // halo, loaded backwards in rows of GB until a segment start shows up
    int lo_bound = HALO;
    bool exhausted = false;
    if (!(s_bits[HALO] & B_SEG)) {
        while (true) {
            if (lo_bound - GB < 0) {
                exhausted = true;
                break;
            }
            const int q = lo_bound - GB + t;
            const long r = (long)tile0 - HALO + q;
            i64 k = -1;
            uint8_t b = B_SEG;
            if (r >= 0) {
                i64 tb;
                k = grid_key(g, (u64)r, ts[r], lat[r], lon[r], tb);
                b = seg_start(g, jid, ts, (u64)r, tb) ? B_SEG : 0;
            }
            s_key[q] = k;
            s_bits[q] = b;
            if (b) atomicOr(&s_flag, 1u);
            __syncthreads();
            const bool found = s_flag != 0;
            lo_bound -= GB;
            __syncthreads();
            if (found) break;
        }
    }
    // run-head bits over [lo_bound, HALO + tvalid)
    const int qend = HALO + (int)tvalid;
    for (int q = lo_bound + t; q < qend; q += GB) {
        uint8_t b = s_bits[q];
        if ((b & B_SEG) || q == lo_bound || s_key[q] != s_key[q - 1]) b |= B_RUN;
        s_bits[q] = b;
    }
    if (t == 0) s_nlist = 0;
    __syncthreads();
    // order-preserving compaction of run heads into a list of positions
    for (int base = lo_bound; base < qend; base += GB) {
        const int q = base + t;
        const bool rh = q < qend && (s_bits[q] & B_RUN);
        u32 tot;
        const u32 e = block_exclusive_sum<GB>(rh ? 1u : 0u, s_tmp, tot);
        const u32 at = s_nlist;
        if (rh) s_lpos[at + e] = (uint16_t)(q | ((s_bits[q] & B_SEG) ? 0x8000 : 0));
        __syncthreads();
        if (t == 0) s_nlist = at + tot;
        __syncthreads();
    }
    const int L = (int)s_nlist;
    // distinct-journey flag of every run head inside the tile: no earlier run
    // head of its segment has the same key
    for (int e = t; e < L; e += GB) {
        const u32 pe = s_lpos[e];
        const int q = (int)(pe & 0x7FFFu);
        if (q < HALO) continue;
        const i64 k = s_key[q];
        if (k < 0) continue;
        bool first = true;
        if (!(pe & 0x8000u)) {
            int f = e - 1;
            bool closed = false;
            for (; f >= 0; --f) {
                const u32 pf = s_lpos[f];
                if (s_key[pf & 0x7FFFu] == k) {
                    first = false;
                    break;
                }
                if (pf & 0x8000u) {
                    closed = true;
                    break;
                }
            }
            if (first && f < 0 && !closed && exhausted) {
                // the segment starts before the loaded halo: continue in global memory
                long rr = (long)tile0 - HALO + lo_bound - 1;
                while (rr >= 0) {
                    i64 tb;
                    const i64 kk = grid_key(g, (u64)rr, ts[rr], lat[rr], lon[rr], tb);
                    if (kk == k) {
                        first = false;
                        break;
                    }
                    if (seg_start(g, jid, ts, (u64)rr, tb)) break;
                    --rr;
                }
            }
        }
        if (first) s_bits[q] |= B_FIRST;
    }
    __syncthreads();
    // Aggregation: every wave walks its GT/4 records of the tile in windows of
    // 64.  Lanes fold records into a private partial while the window holds no
    // run start; a window with starts closes the open run (wave reduction) and
    // scans the runs that begin in it (segmented scan); each finished run is one
    // LDS hash insert.  A wave's first record starts a piece of its own.
    {
        constexpr int WREC = GT / (GB / WAVE);
        const int w = t / WAVE, l = lane_id();
        const int qa = HALO + w * WREC;
        RunPart p;
        run_reset(p);
        i64 open_key = -1;
        for (int i = 0; i < WREC / WAVE; ++i) {
            const int q = qa + i * WAVE + l;
            const bool valid = q < qend;
            const i64 k = valid ? s_key[q] : -1;
            const uint8_t b = valid ? s_bits[q] : 0;
            const bool head = valid && ((b & B_RUN) || (i == 0 && l == 0));
            RunPart c;
            run_reset(c);
            if (valid && k >= 0) {
                const float sp = s_spd[q - HALO];
                c.count = 1;
                c.nj = (b & B_FIRST) ? 1u : 0u;
                c.sum = fx_from_double<FX_SPD>((double)sp);
                c.mn = c.mx = ord_f32(sp);
            }
            const u64 H = __ballot(head);
            if (H == 0) {
                run_combine(p, c);
                continue;
            }
            const int f0 = __ffsll((long long)H) - 1;
            if (l < f0) run_combine(p, c);
            run_wave_reduce(p);
            if (l == 0 && open_key >= 0 && p.count) run_insert<LHS>(s_hkey, s_h, tab, gmask, meta, (u64)open_key, p);
            RunPart sc = c;
            run_seg_scan(sc, head);
            const bool next_head = (l < WAVE - 1) && ((H >> (l + 1)) & 1ull);
            // key of the run each lane belongs to: the key of its head lane
            if (l >= f0 && next_head && k >= 0 && sc.count) run_insert<LHS>(s_hkey, s_h, tab, gmask, meta, (u64)k, sc);
            const int lh = 63 - __clzll((long long)H);  // last head lane: the run left open
            open_key = __shfl(k, lh, WAVE);
            run_reset(p);
            if (l == WAVE - 1) p = sc;
        }
        run_wave_reduce(p);
        if (l == 0 && open_key >= 0 && p.count) run_insert<LHS>(s_hkey, s_h, tab, gmask, meta, (u64)open_key, p);
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
    // merge the LDS table into the HBM table
    for (int i = t; i < LHS; i += GB) {
        const u64 key = s_hkey[i];
        if (key == GEMPTY) continue;
        const LSlot& sl = s_h[i];
        const Fx192 sum = fx_from_cs(sl.cs);
        g_insert(tab, gmask, meta, key, sl.count, sl.nj, sum, sl.mn, sl.mx);
    }
}

struct GridLayout {
    GridMeta* meta;
    GEntry* tab;
    u64* K0;
    u64* K1;
    u32* C;  // compaction values (slot index), the sort's input values
    u32* V0;
    u32* V1;
    u32* zero_begin;
    size_t zero_bytes;
    u32* hist;
    u64* status;
    u32* offs;
    u64 slots, stiles, tiles;
    size_t bytes;
    GridLayout(void* ws, u64 n, u64 cap)
    {
        cvh::Carver c(ws);
        u64 want = 2 * (cap < 1 ? 1 : cap);
        slots = cvh::next_pow2(want < 4096 ? 4096 : want);
        stiles = (slots + sort_min_tile() - 1) / sort_min_tile();
        tiles = (n + GT - 1) / GT;
        meta = c.take<GridMeta>(1);
        tab = c.take<GEntry>(slots);
        K0 = c.take<u64>(slots);
        K1 = c.take<u64>(slots);
        C = c.take<u32>(slots);
        V0 = c.take<u32>(slots);
        V1 = c.take<u32>(slots);
        size_t z0 = cvh::align_up(c.off);
        hist = c.take<u32>(MAX_PASSES * RADIX);
        status = c.take<u64>(stiles * RADIX + 1);
        size_t z1 = cvh::align_up(c.off);
        zero_begin = (u32*)(c.base ? c.base + z0 : nullptr);
        zero_bytes = z1 - z0;
        offs = c.take<u32>(MAX_PASSES * RADIX);
        bytes = c.size();
    }
};

int g_lds_slots = 256;  // LDS hash slots per tile (tuning knob "grid_lds_slots")

bool spec_ok(const cv_grid_spec* g)
{
    if (!g) return false;
    if (!(g->dlat_deg > 0.0) || !(g->dlon_deg > 0.0)) return false;
    if (!std::isfinite(g->lat0_deg) || !std::isfinite(g->lon0_deg) || !std::isfinite(g->dlat_deg) ||
        !std::isfinite(g->dlon_deg))
        return false;
    if (g->n_lat <= 0 || g->n_lon <= 0 || g->bin_ms <= 0) return false;
    if (g->n_lat > (1ll << 31) || g->n_lon > (1ll << 31)) return false;
    __int128 cells = (__int128)g->n_lat * g->n_lon;
    if (g->n_t > 0 && cells * g->n_t >= ((__int128)1 << 63)) return false;
    return true;
}

}  // namespace

namespace cv {
bool set_grid_lds_slots(int v)
{
    if (v != 256 && v != 512 && v != 1024) return false;
    g_lds_slots = v;
    return true;
}
int grid_lds_slots() { return g_lds_slots; }
}  // namespace cv

static cv_status grid_impl(const cv_records* sorted, const u64* soff, u32 S, const cv_grid_spec* grid,
                           const cv_groups* out, uint64_t capacity, u64* go, cv_result* res, void* ws, size_t ws_bytes,
                           void* stream)
{
    if (!sorted || !out || sorted->n >= (1ull << 32) || capacity >= (1ull << 31) || !spec_ok(grid))
        return CV_ERR_INVALID_ARGUMENT;
    const u64 n = sorted->n;
    hipStream_t s = (hipStream_t)stream;
    GridLayout need(nullptr, n, capacity);
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need.bytes) return CV_ERR_WORKSPACE;
    if (n == 0) {
        if (res) hipLaunchKernelGGL(k_grid_empty, dim3(1), dim3(64), 0, s, res);
        if (go) cvh::fill_u64(go, 0, (u64)S + 1, s);
        return cvh::last_launch_status();
    }
    if (!sorted->journey_id || !sorted->ts_ms || !sorted->lat_deg || !sorted->lon_deg || !sorted->speed_mps)
        return CV_ERR_INVALID_ARGUMENT;
    if (capacity > 0 &&
        (!out->key || !out->count || !out->n_journeys || !out->sum_speed || !out->min_speed || !out->max_speed))
        return CV_ERR_INVALID_ARGUMENT;
    GridLayout L(ws, n, capacity);
    Spec g;
    g.lat0 = grid->lat0_deg;
    g.lon0 = grid->lon0_deg;
    g.dlat = grid->dlat_deg;
    g.dlon = grid->dlon_deg;
    g.n_lat = grid->n_lat;
    g.n_lon = grid->n_lon;
    g.t0 = grid->t0_ms;
    g.bin_ms = grid->bin_ms;
    g.tmax = grid->n_t > 0 ? grid->n_t : (INT64_MAX / (grid->n_lat * grid->n_lon));
    g.soff = soff;
    g.S = S;
    g.kb = 0;
    if (S > 1) {
        // cell keys < n_t * n_lat * n_lon; the shard index goes above them
        const unsigned __int128 cells = (unsigned __int128)grid->n_t * grid->n_lat * grid->n_lon;
        u32 kb = 0;
        while (kb < 63 && ((unsigned __int128)1 << kb) < cells) ++kb;
        u32 sb = 0;
        while (((u64)1 << sb) < S) ++sb;
        if (kb + sb > 63) return CV_ERR_RANGE;
        g.kb = kb;
    }
    const u64 kmask = S > 1 ? ((1ull << g.kb) - 1) : ~0ull;
    const u32 nn = (u32)n;
    const u32 slots = (u32)L.slots;
    {
        cvh::TimedScope ts_("grid_agg", s);
        hipLaunchKernelGGL(k_grid_clear, dim3(cvh::grid_for(L.slots, 256, 4096)), dim3(256), 0, s, L.tab, L.slots,
                           L.meta);
        cvh::fill_u32(L.zero_begin, 0u, L.zero_bytes / 4, s);
        const dim3 gg((unsigned)L.tiles), gb(GB);
        if (g_lds_slots >= 1024)
            hipLaunchKernelGGL((k_grid_agg<1024>), gg, gb, 0, s, nn, sorted->journey_id, sorted->ts_ms,
                               sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, g, L.tab, L.slots - 1, L.meta);
        else if (g_lds_slots >= 512)
            hipLaunchKernelGGL((k_grid_agg<512>), gg, gb, 0, s, nn, sorted->journey_id, sorted->ts_ms,
                               sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, g, L.tab, L.slots - 1, L.meta);
        else
            hipLaunchKernelGGL((k_grid_agg<256>), gg, gb, 0, s, nn, sorted->journey_id, sorted->ts_ms,
                               sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, g, L.tab, L.slots - 1, L.meta);
    }
    {
        cvh::TimedScope ts_("grid_tail", s);
        hipLaunchKernelGGL(k_grid_compact, dim3((unsigned)((L.slots + CSLOTS - 1) / CSLOTS)), dim3(256), 0, s, L.tab,
                           L.slots, L.meta, L.K0, L.C);
        hipLaunchKernelGGL(k_grid_bits, dim3(1), dim3(64), 0, s, L.meta);
        const u32* cnt = &L.meta->compact_n;
        const u32* bits = &L.meta->key_bits;
        radix_hist(L.K0, slots, cnt, MAX_PASSES, bits, L.hist, cvh::grid_for(L.slots, 256, 1024), s);
        radix_scan(L.hist, L.offs, MAX_PASSES, s);
        radix_passes(L.K0, L.K1, L.C, L.V0, L.V1, slots, cnt, bits, MAX_PASSES, L.offs, L.status, L.meta->tickets, s);
        hipLaunchKernelGGL(k_iota_if_nopass, dim3(cvh::grid_for(L.slots, 256, 1024)), dim3(256), 0, s, L.meta, L.C,
                           L.V0, slots);
        const u32 cap = (u32)capacity;
        hipLaunchKernelGGL(k_grid_emit, dim3(cvh::grid_for(capacity ? capacity : 1, 256, 4096)), dim3(256), 0, s,
                           L.tab, L.meta, L.K0, L.K1, L.V0, L.V1, cap, out->key, out->count, out->n_journeys,
                           out->sum_speed, out->min_speed, out->max_speed, res, kmask);
        if (go)
            hipLaunchKernelGGL(k_group_offsets, dim3(cvh::grid_for((u64)S + 1, 256, 64)), dim3(256), 0, s, L.meta,
                               L.K0, L.K1, S, g.kb, go);
    }
    return cvh::last_launch_status();
}


extern "C" {

cv_status cv_grid_workspace_size(uint64_t n, const cv_grid_spec* grid, uint64_t capacity, size_t* bytes)
{
    if (!bytes || n >= (1ull << 32) || capacity >= (1ull << 31) || !spec_ok(grid)) return CV_ERR_INVALID_ARGUMENT;
    GridLayout L(nullptr, n, capacity);
    *bytes = L.bytes;
    return CV_OK;
}

cv_status cv_grid_aggregate(const cv_records* sorted, const cv_grid_spec* grid, const cv_groups* out,
                            uint64_t capacity, cv_result* res, void* ws, size_t ws_bytes, void* stream)
{
    return grid_impl(sorted, nullptr, 0, grid, out, capacity, nullptr, res, ws, ws_bytes, stream);
}

cv_status cv_batch_grid_aggregate(const cv_records* sorted, const uint64_t* shard_offsets, uint32_t n_shards,
                                  const cv_grid_spec* grid, const cv_groups* out, uint64_t capacity,
                                  uint64_t* group_offsets, cv_result* res, void* ws, size_t ws_bytes, void* stream)
{
    if (n_shards == 0 || !shard_offsets || !group_offsets || !cvh::aligned(shard_offsets, 8) ||
        !cvh::aligned(group_offsets, 8) || !grid || grid->n_t <= 0)
        return CV_ERR_INVALID_ARGUMENT;
    return grid_impl(sorted, shard_offsets, n_shards, grid, out, capacity, group_offsets, res, ws, ws_bytes, stream);
}

}  // extern "C"
