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
#include "cv_gridagg.h"
#include "cv_gridtab.h"
#include "cv_radix.h"

using namespace cv;

namespace {

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

// out[k] = in[perm[k]]: a payload column in the sort's order (GU per round,
// loads issued together)
template <class T>
__global__ void __launch_bounds__(256) k_gather_col(const T* __restrict__ in, const u32* __restrict__ perm,
                                                    T* __restrict__ out, u32 n)
{
    constexpr int GU = 4;
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 k0 = (u64)blockIdx.x * blockDim.x + threadIdx.x; k0 < n; k0 += GU * stride) {
        u32 p[GU];
        T v[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const u64 k = k0 + u * stride;
            p[u] = perm[k < n ? k : n - 1];
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) v[u] = in[p[u] < n ? p[u] : n - 1];  // a permutation of [0, n)
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const u64 k = k0 + u * stride;
            if (k < n) out[k] = v[u];
        }
    }
}

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

// the tile kernel for a table size and a direction source
template <class Pol>
static void launch_tiles(dim3 gg, hipStream_t s, u32 nn, const cv_records* sorted, const Spec& g, GEntry* tab,
                         u64 gmask, GridMeta* meta)
{
    const dim3 gb(GB);
    if (g_lds_slots >= 1024)
        hipLaunchKernelGGL((k_grid_agg<1024, Pol>), gg, gb, 0, s, nn, sorted->journey_id, sorted->ts_ms,
                           sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, g, tab, gmask, meta, Pol{});
    else if (g_lds_slots >= 512)
        hipLaunchKernelGGL((k_grid_agg<512, Pol>), gg, gb, 0, s, nn, sorted->journey_id, sorted->ts_ms,
                           sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, g, tab, gmask, meta, Pol{});
    else
        hipLaunchKernelGGL((k_grid_agg<256, Pol>), gg, gb, 0, s, nn, sorted->journey_id, sorted->ts_ms,
                           sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, g, tab, gmask, meta, Pol{});
}

// nd > 0: a direction dimension of nd sectors (plus one for records without a
// direction) from the sorted heading column hdg, else from feat's bearing
static cv_status grid_impl(const cv_records* sorted, const u64* soff, u32 S, const cv_grid_spec* grid,
                           const cv_groups* out, uint64_t capacity, u64* go, cv_result* res, void* ws, size_t ws_bytes,
                           void* stream, u32 nd = 0, double doff = 0.0, const float* hdg = nullptr,
                           const cv_features* feat = nullptr)
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
    g.tmax = grid->n_t > 0 ? grid->n_t : (INT64_MAX / (grid->n_lat * grid->n_lon * (i64)(nd + 1)));
    g.soff = soff;
    g.S = S;
    g.kb = 0;
    g.nd = nd;
    g.dstep = nd ? 360.0 / (double)nd : 0.0;
    g.doff = doff;
    g.hdg = hdg;
    g.brg = (nd && !hdg) ? feat->bearing_deg : nullptr;
    g.bfl = (nd && !hdg) ? feat->flags : nullptr;
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
        const dim3 gg((unsigned)L.tiles);
        if (nd == 0) launch_tiles<GridPlain>(gg, s, nn, sorted, g, L.tab, L.slots - 1, L.meta);
        else if (hdg) launch_tiles<GridHeading>(gg, s, nn, sorted, g, L.tab, L.slots - 1, L.meta);
        else launch_tiles<GridBearing>(gg, s, nn, sorted, g, L.tab, L.slots - 1, L.meta);
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

cv_status cv_grid_aggregate_dir(const cv_records* sorted, const float* heading_deg, const cv_features* feat,
                                const cv_grid_spec* grid, uint32_t n_dir, double dir_offset_deg, const cv_groups* out,
                                uint64_t capacity, cv_result* res, void* ws, size_t ws_bytes, void* stream)
{
    if (!grid || n_dir < 1 || n_dir > 64 || !(dir_offset_deg >= 0.0 && dir_offset_deg < 360.0))
        return CV_ERR_INVALID_ARGUMENT;
    if (!heading_deg && (!feat || !feat->bearing_deg || !feat->flags)) return CV_ERR_INVALID_ARGUMENT;
    if (grid->n_t > 0 && (__int128)grid->n_t * grid->n_lat * grid->n_lon * (n_dir + 1) >= ((__int128)1 << 63))
        return CV_ERR_RANGE;
    return grid_impl(sorted, nullptr, 0, grid, out, capacity, nullptr, res, ws, ws_bytes, stream, n_dir,
                     dir_offset_deg, heading_deg, feat);
}

cv_status cv_gather_column(const void* in, const uint32_t* perm, void* out, uint64_t n, uint32_t elem_bytes,
                           void* stream)
{
    if (n >= (1ull << 32) || (elem_bytes != 4 && elem_bytes != 8)) return CV_ERR_INVALID_ARGUMENT;
    if (n == 0) return CV_OK;
    if (!in || !perm || !out || !cvh::aligned(in, elem_bytes) || !cvh::aligned(out, elem_bytes))
        return CV_ERR_INVALID_ARGUMENT;
    hipStream_t s = (hipStream_t)stream;
    const unsigned blocks = (unsigned)cvh::grid_for(n, 256, 8192);
    if (elem_bytes == 4)
        hipLaunchKernelGGL((k_gather_col<uint32_t>), dim3(blocks), dim3(256), 0, s, (const uint32_t*)in, perm,
                           (uint32_t*)out, (u32)n);
    else
        hipLaunchKernelGGL((k_gather_col<u64>), dim3(blocks), dim3(256), 0, s, (const u64*)in, perm, (u64*)out,
                           (u32)n);
    return cvh::last_launch_status();
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
