// cv_grid.hip -- cv_grid_aggregate: the spatio-temporal lattice of the paper
// (Methods steps (3)-(5); Algorithm 2's floor((x - x_min) / x_step) bins; the
// count / sum / count-unique / mean reductions of Table 3), as a sparse,
// key-sorted group table over (journey, time)-sorted records.
//
//   k_grid_agg   per tile of GT records:
//     * key = (tbin * n_lat + ilat) * n_lon + ilon per record (-1 outside);
//     * distinct-journey flag: a record counts towards n_journeys iff no earlier
//       record of its (journey, time-bin) segment has the same key.  Records of
//       one (journey, tbin) are contiguous after the sort, so a backward scan
//       that stops at the segment start decides it; segments entering the tile
//       are covered by a halo loaded into LDS on demand (global memory beyond);
//     * runs of equal key inside a thread's records are pre-reduced, then
//       inserted into an LDS open-addressing table; entries that find no LDS
//       slot spill straight to the HBM table; at tile end the LDS table is
//       merged into the HBM table with integer atomics (exact sums, so the
//       result is independent of tile and atomic order);
//   k_grid_compact  occupied HBM slots -> (key, slot) pairs;
//   radix sort of the pairs by key (the same LSD sort as the record order);
//   k_grid_emit     rows in ascending key, sums rounded once to double.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cv_device.h"
#include "cv_host.h"
#include "cv_radix.h"

using namespace cv;

namespace {

constexpr int GB = 256;
constexpr int GI = 8;
constexpr int GT = GB * GI;
constexpr int HALO = 1024;
constexpr int LHS = 512;
constexpr int LHS_PROBES = 32;
constexpr int FX_SPD = 149;
constexpr u64 GEMPTY = ~0ull;

struct GEntry {
    u64 key;
    u64 sum[3];
    u32 count, nj, mn, mx;
};
static_assert(sizeof(GEntry) == 48, "entry layout");

struct GridMeta {
    u32 G;          // distinct keys inserted into the HBM table
    u32 overflow;   // HBM table full
    u64 n_out;      // records outside the grid
    u64 max_key;    // largest key seen
    u32 key_bits;
    u32 passes;
    u32 compact_n;
    u32 pad;
    u32 tickets[MAX_PASSES];
};

struct Spec {
    double lat0, lon0, dlat, dlon;
    i64 n_lat, n_lon, t0, bin_ms, tmax;
};

__device__ __forceinline__ i64 floor_div64(i64 a, i64 b)
{
    i64 q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

// key (or -1) and time bin of one record; floor of the IEEE quotient
__device__ __forceinline__ i64 grid_key(const Spec& g, i64 ts, double la, double lo, i64& tb)
{
    tb = floor_div64(ts - g.t0, g.bin_ms);
    if (!isfinite(la) || !isfinite(lo)) return -1;
    double fy = floor((la - g.lat0) / g.dlat);
    double fx = floor((lo - g.lon0) / g.dlon);
    if (!(fy >= 0.0 && fy < (double)g.n_lat && fx >= 0.0 && fx < (double)g.n_lon && tb >= 0 && tb < g.tmax)) return -1;
    return (tb * g.n_lat + (i64)fy) * g.n_lon + (i64)fx;
}

__global__ void __launch_bounds__(256) k_grid_clear(GEntry* __restrict__ tab, u64 slots, GridMeta* meta)
{
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < slots; i += (u64)gridDim.x * blockDim.x) {
        GEntry e;
        e.key = GEMPTY;
        e.sum[0] = e.sum[1] = e.sum[2] = 0;
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
    atomicAdd(&e.count, count);
    if (nj) atomicAdd(&e.nj, nj);
    atomic_add_fx(e.sum, sum);
    atomicMin(&e.mn, mn);
    atomicMax(&e.mx, mx);
}

__device__ __forceinline__ void g_insert(GEntry* tab, u64 mask, GridMeta* meta, u64 key, u32 count, u32 nj,
                                         const Fx192& sum, u32 mn, u32 mx)
{
    u64 h = mix64(key) & mask;
    for (u64 probe = 0; probe <= mask; ++probe) {
        u64 cur = tab[h].key;
        if (cur == key) {
            g_merge(tab[h], count, nj, sum, mn, mx);
            return;
        }
        if (cur == GEMPTY) {
            u64 prev = atomicCAS((unsigned long long*)&tab[h].key, (unsigned long long)GEMPTY, (unsigned long long)key);
            if (prev == GEMPTY) atomicAdd(&meta->G, 1u);
            if (prev == GEMPTY || prev == key) {
                g_merge(tab[h], count, nj, sum, mn, mx);
                return;
            }
        }
        h = (h + 1) & mask;
    }
    atomicOr(&meta->overflow, 1u);
}

struct LSlot {
    u64 cs[4];
    u32 count, nj, mn, mx;
};

__global__ void __launch_bounds__(GB, 2)
k_grid_agg(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts, const double* __restrict__ lat,
           const double* __restrict__ lon, const float* __restrict__ spd, Spec g, GEntry* __restrict__ tab, u64 gmask,
           GridMeta* meta)
{
    __shared__ i64 s_key[HALO + GT];
    __shared__ uint8_t s_seg[HALO + GT];  // 1: first record of a (journey, time-bin) segment
    __shared__ float s_spd[GT];
    __shared__ u64 s_hkey[LHS];
    __shared__ LSlot s_h[LHS];
    __shared__ u32 s_flag;
    __shared__ u64 s_out[GB / WAVE];

    const int t = threadIdx.x;
    const u64 tile0 = (u64)blockIdx.x * GT;
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
    // tile records: striped, coalesced loads; key, segment-start flag, speed
    u64 n_out = 0;
    for (int i = t; i < GT; i += GB) {
        u64 r = tile0 + i;
        i64 k = -1;
        uint8_t sg = 1;
        float sp = 0.f;
        if (r < n) {
            i64 tb;
            k = grid_key(g, ts[r], lat[r], lon[r], tb);
            n_out += (k < 0);
            sp = spd[r];
            if (r > 0) {
                i64 tbp = floor_div64(ts[r - 1] - g.t0, g.bin_ms);
                sg = (jid[r] != jid[r - 1]) || (tb != tbp);
            }
        }
        s_key[HALO + i] = k;
        s_seg[HALO + i] = sg;
        s_spd[i] = sp;
    }
    if (t == 0) s_flag = 0;
    __syncthreads();
    // halo: only when the first segment of the tile started before it
    int lo_bound = HALO;  // lowest valid LDS index
    bool need = s_seg[HALO] == 0;
    bool halo_exhausted = false;
    while (need) {
        if (lo_bound - GB < 0) {
            halo_exhausted = true;
            break;
        }
        int q = lo_bound - GB + t;
        long r = (long)tile0 - HALO + q;
        i64 k = -1;
        uint8_t sg = 1;
        if (r >= 0) {
            i64 tb;
            k = grid_key(g, ts[r], lat[r], lon[r], tb);
            if (r > 0) {
                i64 tbp = floor_div64(ts[r - 1] - g.t0, g.bin_ms);
                sg = (jid[r] != jid[r - 1]) || (tb != tbp);
            }
        }
        s_key[q] = k;
        s_seg[q] = sg;
        if (sg) atomicOr(&s_flag, 1u);
        __syncthreads();
        need = s_flag == 0;
        lo_bound -= GB;
        __syncthreads();
    }

    // per-thread runs over GI consecutive records
    const int q0 = HALO + t * GI;
    u64 kmax = 0;
    i64 rk = -1;
    u32 rc = 0, rnj = 0, rmn = ~0u, rmx = 0;
    Fx192 rsum;
    fx_zero(rsum);
    auto flush = [&]() {
        if (rc == 0) return;
        u64 key = (u64)rk;
        u64 h = mix64(key) & (LHS - 1);
        bool done = false;
        for (int probe = 0; probe < LHS_PROBES; ++probe) {
            u64 cur = s_hkey[h];
            if (cur == GEMPTY) {
                u64 prev = atomicCAS((unsigned long long*)&s_hkey[h], (unsigned long long)GEMPTY,
                                     (unsigned long long)key);
                cur = prev == GEMPTY ? key : prev;
            }
            if (cur == key) {
                LSlot& s = s_h[h];
                u64 c[4];
                fx_to_cs(rsum, c);
                for (int i = 0; i < 4; ++i)
                    if (c[i]) atomicAdd((unsigned long long*)&s.cs[i], (unsigned long long)c[i]);
                atomicAdd(&s.count, rc);
                if (rnj) atomicAdd(&s.nj, rnj);
                atomicMin(&s.mn, rmn);
                atomicMax(&s.mx, rmx);
                done = true;
                break;
            }
            h = (h + 1) & (LHS - 1);
        }
        if (!done) g_insert(tab, gmask, meta, key, rc, rnj, rsum, rmn, rmx);  // spill to HBM
        rc = 0;
        rnj = 0;
        rmn = ~0u;
        rmx = 0;
        fx_zero(rsum);
    };
    for (int i = 0; i < GI; ++i) {
        const int q = q0 + i;
        const u64 r = tile0 + (u64)(q - HALO);
        if (r >= n) break;
        const i64 k = s_key[q];
        if (k < 0) {
            flush();
            continue;
        }
        kmax = (u64)k > kmax ? (u64)k : kmax;
        // distinct-journey flag: earlier record of the same segment with this key?
        bool first = true;
        if (!s_seg[q]) {
            int p = q - 1;
            while (true) {
                if (p < lo_bound) {
                    // beyond the loaded halo: continue in global memory
                    long rr = (long)tile0 - HALO + p;
                    while (rr >= 0) {
                        i64 tb;
                        i64 kk = grid_key(g, ts[rr], lat[rr], lon[rr], tb);
                        if (kk == k) {
                            first = false;
                            break;
                        }
                        if (rr == 0) break;
                        i64 tbp = floor_div64(ts[rr - 1] - g.t0, g.bin_ms);
                        if (jid[rr] != jid[rr - 1] || tb != tbp) break;
                        --rr;
                    }
                    break;
                }
                if (s_key[p] == k) {
                    first = false;
                    break;
                }
                if (s_seg[p]) break;
                --p;
            }
        }
        const bool same_run = rc > 0 && rk == k && !s_seg[q];
        if (!same_run) {
            flush();
            rk = k;
        }
        float sp = s_spd[q - HALO];
        rc += 1;
        rnj += first ? 1u : 0u;
        Fx192 a = fx_from_double<FX_SPD>((double)sp);
        fx_add(rsum, a);
        u32 o = ord_f32(sp);
        rmn = o < rmn ? o : rmn;
        rmx = o > rmx ? o : rmx;
    }
    flush();
    (void)halo_exhausted;
    // out-of-grid count
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
        u64 key = s_hkey[i];
        if (key == GEMPTY) continue;
        const LSlot& s = s_h[i];
        Fx192 sum = fx_from_cs(s.cs);
        g_insert(tab, gmask, meta, key, s.count, s.nj, sum, s.mn, s.mx);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        u64 o = __shfl_xor(kmax, d, WAVE);
        kmax = o > kmax ? o : kmax;
    }
    if (lane_id() == 0 && kmax) atomicMax((unsigned long long*)&meta->max_key, (unsigned long long)kmax);
}

__global__ void __launch_bounds__(256) k_grid_compact(const GEntry* __restrict__ tab, u64 slots, GridMeta* meta,
                                                      u64* __restrict__ ckeys, u32* __restrict__ cvals)
{
    for (u64 s = (u64)blockIdx.x * blockDim.x + threadIdx.x; s < slots; s += (u64)gridDim.x * blockDim.x) {
        u64 k = tab[s].key;
        if (k != GEMPTY) {
            u32 pos = atomicAdd(&meta->compact_n, 1u);
            ckeys[pos] = k;
            cvals[pos] = (u32)s;
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
                                                   cv_result* res)
{
    const u32 G = meta->compact_n;
    const u32 np = meta->passes;
    const u32* V = np == 0 ? V0 : ((np & 1) ? V1 : V0);
    const u64* K = np == 0 ? K0 : ((np & 1) ? K1 : K0);
    (void)K;
    const u32 m = G < cap ? G : cap;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const GEntry& e = tab[V[i]];
        o_key[i] = (i64)e.key;
        o_cnt[i] = e.count;
        o_nj[i] = e.nj;
        Fx192 s;
        s.w[0] = e.sum[0];
        s.w[1] = e.sum[1];
        s.w[2] = e.sum[2];
        o_sum[i] = fx_to_double<FX_SPD>(s);
        o_min[i] = unord_f32(e.mn);
        o_max[i] = unord_f32(e.mx);
    }
    if (res && blockIdx.x == 0 && threadIdx.x == 0) {
        cv_result r = {};
        const bool full = meta->overflow != 0;  // HBM table full: G is only a lower bound
        const bool over = full || G > cap;
        r.status = over ? CV_ERR_CAPACITY : CV_OK;
        r.count = G;
        if (full) r.required = ((u64)G + 1 > 2ull * cap) ? (u64)G + 1 : 2ull * cap;
        else if (over) r.required = G;
        r.n_out_of_grid = meta->n_out;
        r.key_bits = meta->key_bits;
        *res = r;
    }
}

__global__ void k_grid_empty(cv_result* res)
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
        stiles = (slots + SORT_TILE - 1) / SORT_TILE;
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
    if (!sorted || !out || sorted->n >= (1ull << 32) || capacity >= (1ull << 31) || !spec_ok(grid))
        return CV_ERR_INVALID_ARGUMENT;
    const u64 n = sorted->n;
    hipStream_t s = (hipStream_t)stream;
    GridLayout need(nullptr, n, capacity);
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need.bytes) return CV_ERR_WORKSPACE;
    if (n == 0) {
        if (res) hipLaunchKernelGGL(k_grid_empty, dim3(1), dim3(64), 0, s, res);
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
    const u32 nn = (u32)n;
    const u32 slots = (u32)L.slots;
    {
        cvh::TimedScope ts_("grid_agg", s);
        hipLaunchKernelGGL(k_grid_clear, dim3(cvh::grid_for(L.slots, 256, 4096)), dim3(256), 0, s, L.tab, L.slots,
                           L.meta);
        cvh::fill_u32(L.zero_begin, 0u, L.zero_bytes / 4, s);
        hipLaunchKernelGGL(k_grid_agg, dim3((unsigned)L.tiles), dim3(GB), 0, s, nn, sorted->journey_id, sorted->ts_ms,
                           sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, g, L.tab, L.slots - 1, L.meta);
    }
    {
        cvh::TimedScope ts_("grid_tail", s);
        hipLaunchKernelGGL(k_grid_compact, dim3(cvh::grid_for(L.slots, 256, 4096)), dim3(256), 0, s, L.tab, L.slots,
                           L.meta, L.K0, L.C);
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
                           out->sum_speed, out->min_speed, out->max_speed, res);
    }
    return cvh::last_launch_status();
}

}  // extern "C"
