// cv_grid.hip -- cv_grid_aggregate: the spatio-temporal lattice of the paper
// (Methods steps (3)-(5); Algorithm 2's floor((x - x_min) / x_step) bins; the
// count / sum / count-unique / mean reductions of Table 3), as a sparse,
// key-sorted group table over (journey, time)-sorted records.
//
//   k_grid_part  per tile of GT records, read with coalesced loads:
//     * key = (tbin * n_lat + ilat) * n_lon + ilon per record (-1 outside);
//     * runs: maximal stretches of one key inside one (journey, time-bin)
//       segment; each is reduced once (count, exact speed sum, min, max);
//     * the runs of one (journey, key) inside the tile add into one partial
//       row, and the tile writes its partial rows in record order into its
//       own region (at most GT rows: each holds >= 1 record);
//   partials of all tiles -> compacted (key, row) pairs (scan of the counts),
//     in tile order;
//   radix sort of the pairs by key (the same stable LSD sort as the record
//     order), so a key's partials stay in record order;
//   k_gpart_heads / k_gpart_emit: groups are runs of equal key in the sorted
//     pairs; each group's first pair sums its partials exactly (integer adds
//     and min / max, so the order of the partials changes nothing), counts a
//     journey once per run of equal journey ids among them (the partials of
//     one journey are adjacent in record order), and writes the row, in
//     ascending key.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cv_device.h"
#include "cv_host.h"
#include "cv_gridpart.h"
#include "cv_gridtab.h"
#include "cv_radix.h"

using namespace cv;

namespace {

// scans of per-tile / per-chunk counts: SCH counts per block
constexpr int SCB = 256;
constexpr int SCP = 8;
constexpr int SCH = SCB * SCP;
// sorted partial pairs per chunk of the head count and the emit
constexpr int ECB = 256;
constexpr int ECP = 4;  // (4: 118 VGPRs in the emit, 4 waves per SIMD)
constexpr int ECH = ECB * ECP;

struct GridLayout {
    GridMeta* meta;
    GPart* part;  // [pmax] partial rows, GT per tile
    u64* K0;      // [pmax] compacted keys; the sort's first key buffer
    u64* K1;      // [pmax] the tiles' partial keys; then the sort's second key buffer
    u32* V0;      // [pmax] compacted partial rows (the sort's pass-0 values); then its first value buffer
    u32* V1;      // [pmax]
    u32* tcnt;    // [tiles] partial rows per tile
    u32* toff;    // [tiles] their first compacted position
    u64* tmax;    // [tiles] largest key per tile
    u32* bsum;    // [nb] per-block sums of a scan
    u64* bmax;    // [nb]
    u32* hcnt;    // [chunks] group heads per chunk of sorted pairs, then their exclusive scan
    u32* zero_begin;
    size_t zero_bytes;
    u32* hist;
    u64* status;
    u32* offs;
    u64 pmax, stiles, tiles, chunks, nb;
    size_t bytes;
    GridLayout(void* ws, u64 n)
    {
        cvh::Carver c(ws);
        tiles = (n + GT - 1) / GT;
        pmax = tiles * GT;
        stiles = (pmax + sort_min_tile() - 1) / sort_min_tile();
        chunks = (pmax + ECH - 1) / ECH;
        const u64 big = tiles > chunks ? tiles : chunks;
        nb = (big + SCH - 1) / SCH;
        meta = c.take<GridMeta>(1);
        part = c.take<GPart>(pmax);
        K0 = c.take<u64>(pmax);
        K1 = c.take<u64>(pmax);
        V0 = c.take<u32>(pmax);
        V1 = c.take<u32>(pmax);
        tcnt = c.take<u32>(tiles);
        toff = c.take<u32>(tiles + 1);
        tmax = c.take<u64>(tiles);
        bsum = c.take<u32>(nb + 1);
        bmax = c.take<u64>(nb + 1);
        hcnt = c.take<u32>(chunks + 1);
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

__global__ void k_gmeta_init(GridMeta* meta)
{
    if (threadIdx.x == 0) {
        GridMeta z = {};
        *meta = z;
    }
}

// Block b of a scan: the sum of v[b * SCH, (b + 1) * SCH) (and the largest of
// vmax there when given), n = *n_dev when given, else n_max.
__global__ void __launch_bounds__(SCB) k_scan_up(const u32* __restrict__ v, u32 n_max, const u32* __restrict__ n_dev,
                                                 const u64* __restrict__ vmax, u32* __restrict__ bsum,
                                                 u64* __restrict__ bmax)
{
    __shared__ u32 s_t[SCB / WAVE];
    __shared__ u64 s_m[SCB / WAVE];
    const u32 n = n_dev ? *n_dev : n_max;
    const u64 i0 = (u64)blockIdx.x * SCH + (u64)threadIdx.x * SCP;
    u32 c = 0;
    u64 m = 0;
#pragma unroll
    for (int k = 0; k < SCP; ++k) {
        const u64 i = i0 + k;
        if (i < n) {
            c += v[i];
            if (vmax) m = vmax[i] > m ? vmax[i] : m;
        }
    }
    u32 tot;
    block_exclusive_sum<SCB>(c, s_t, tot);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const u64 o = __shfl_xor(m, d, WAVE);
        m = o > m ? o : m;
    }
    if (lane_id() == 0) s_m[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = tot;
        u64 mm = 0;
        for (int w = 0; w < SCB / WAVE; ++w) mm = s_m[w] > mm ? s_m[w] : mm;
        bmax[blockIdx.x] = mm;
    }
}

// One block: exclusive scan of the nb block sums in place.  mode 0 (the
// tiles' partial counts): total = partial rows, the largest key gives the
// sort's key width and passes, and the chunk count of the sorted pairs;
// mode 1 (group heads per chunk): total = groups.
__global__ void __launch_bounds__(SCB) k_scan_top(u32* __restrict__ bsum, u32 nb, const u64* __restrict__ bmax,
                                                  GridMeta* meta, int mode)
{
    __shared__ u32 s_t[SCB / WAVE];
    __shared__ u32 carry;
    __shared__ u64 s_m;
    if (threadIdx.x == 0) {
        carry = 0;
        s_m = 0;
    }
    __syncthreads();
    for (u32 b = 0; b < nb; b += SCB) {
        const u32 i = b + threadIdx.x;
        const u32 v = i < nb ? bsum[i] : 0u;
        if (mode == 0 && i < nb && bmax[i]) atomicMax((unsigned long long*)&s_m, (unsigned long long)bmax[i]);
        u32 tot;
        const u32 e = block_exclusive_sum<SCB>(v, s_t, tot);
        if (i < nb) bsum[i] = carry + e;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (mode == 0) {
            meta->compact_n = carry;
            meta->max_key = s_m;
            const u32 bits = s_m ? 64u - (u32)__clzll((long long)s_m) : 0u;
            meta->key_bits = bits;
            meta->passes = (bits + RADIX_BITS - 1) / RADIX_BITS;
            meta->chunks = (u32)(((u64)carry + ECH - 1) / ECH);
        } else {
            meta->groups = carry;
        }
    }
}

// Block b: exclusive offsets of v[b * SCH, (b + 1) * SCH) from bsum[b], into out.
__global__ void __launch_bounds__(SCB) k_scan_down(const u32* __restrict__ v, u32 n_max, const u32* __restrict__ n_dev,
                                                   const u32* __restrict__ bsum, u32* __restrict__ out)
{
    __shared__ u32 s_t[SCB / WAVE];
    const u32 n = n_dev ? *n_dev : n_max;
    const u64 i0 = (u64)blockIdx.x * SCH + (u64)threadIdx.x * SCP;
    u32 x[SCP];
    u32 c = 0;
#pragma unroll
    for (int k = 0; k < SCP; ++k) {
        const u64 i = i0 + k;
        x[k] = i < n ? v[i] : 0u;
        c += x[k];
    }
    u32 tot;
    u32 e = block_exclusive_sum<SCB>(c, s_t, tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCP; ++k) {
        const u64 i = i0 + k;
        if (i < n) out[i] = e;
        e += x[k];
    }
}

// One wave per tile: its partial keys to their compacted positions, with the
// partial's row (tile * GT + j) as the sort's value.
__global__ void __launch_bounds__(256) k_gpart_compact(const u64* __restrict__ pkey, const u32* __restrict__ tcnt,
                                                       const u32* __restrict__ toff, u32 tiles, u64* __restrict__ K0,
                                                       u32* __restrict__ V0)
{
    const u32 wv = (blockIdx.x * 256 + threadIdx.x) / WAVE;
    const u32 nw = gridDim.x * 256 / WAVE;
    const int l = lane_id();
    for (u32 t = wv; t < tiles; t += nw) {
        const u32 c = tcnt[t], o = toff[t];
        const u64 b = (u64)t * GT;
        for (u32 j = l; j < c; j += WAVE) {
            K0[o + j] = pkey[b + j];
            V0[o + j] = (u32)(b + j);
        }
    }
}

// the sorted pairs after meta->passes passes (ping-pong buffers)
__device__ __forceinline__ const u64* sorted_keys(const GridMeta* m, const u64* K0, const u64* K1)
{
    return (m->passes & 1) ? K1 : K0;
}
__device__ __forceinline__ const u32* sorted_vals(const GridMeta* m, const u32* V0, const u32* V1)
{
    return (m->passes & 1) ? V1 : V0;
}

// group heads (first pair of each key) per chunk of ECH sorted pairs
__global__ void __launch_bounds__(ECB) k_gpart_heads(const GridMeta* meta, const u64* __restrict__ K0,
                                                     const u64* __restrict__ K1, u32* __restrict__ hcnt)
{
    __shared__ u32 s_t[ECB / WAVE];
    const u32 P = meta->compact_n;
    const u32 chunks = meta->chunks;
    const u64* K = sorted_keys(meta, K0, K1);
    for (u32 c = blockIdx.x; c < chunks; c += gridDim.x) {
        const u64 i0 = (u64)c * ECH + (u64)threadIdx.x * ECP;
        u32 h = 0;
        u64 prev = (i0 > 0 && i0 < P) ? K[i0 - 1] : ~0ull;
#pragma unroll
        for (int k = 0; k < ECP; ++k) {
            const u64 i = i0 + k;
            if (i < P) {
                const u64 key = K[i];
                h += (i == 0 || key != prev) ? 1u : 0u;
                prev = key;
            }
        }
        u32 tot;
        block_exclusive_sum<ECB>(h, s_t, tot);
        if (threadIdx.x == 0) hcnt[c] = tot;
        __syncthreads();
    }
}

// Rows in ascending key: the first pair of each key sums the partials of its
// group (the pairs that follow with the same key) and writes the row.  In the
// batched form, group_offsets[s] = first row of shard s (keys carry the shard
// above bit kb).
__global__ void __launch_bounds__(ECB) k_gpart_emit(const GridMeta* meta, const u64* __restrict__ K0,
                                                    const u64* __restrict__ K1, const u32* __restrict__ V0,
                                                    const u32* __restrict__ V1, const GPart* __restrict__ part,
                                                    const u32* __restrict__ hoff, u32 cap, i64* __restrict__ o_key,
                                                    u32* __restrict__ o_cnt, u32* __restrict__ o_nj,
                                                    double* __restrict__ o_sum, float* __restrict__ o_min,
                                                    float* __restrict__ o_max, u64* __restrict__ go, u32 S, u32 kb,
                                                    u64 kmask, cv_result* res)
{
    const u32 P = meta->compact_n;
    const u32 G = meta->groups;
    const u32 chunks = meta->chunks;
    const u64* K = sorted_keys(meta, K0, K1);
    const u32* V = sorted_vals(meta, V0, V1);
    const bool sharded = go && S > 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (res) {
            cv_result r = {};
            r.status = meta->overflow ? CV_ERR_DEVICE : (G > cap ? CV_ERR_CAPACITY : CV_OK);
            r.count = G;
            r.required = G > cap ? G : 0;
            r.n_out_of_grid = meta->n_out;
            r.key_bits = meta->key_bits;
            *res = r;
        }
        if (go && (P == 0 || !sharded))  // no groups, or one problem: shard 0 holds every row
            for (u32 s = 0; s <= S; ++s) go[s] = s == 0 ? 0u : G;
    }
    // A chunk's ECH pairs are taken in ECP rows of ECB: thread t has pairs
    // c * ECH + k * ECB + t, so the heads of a row write consecutive output
    // rows (coalesced stores), and each thread still issues its ECP gathers
    // of first partials together.
    __shared__ u32 s_rw[ECP][ECB / WAVE];
    const int t = threadIdx.x, lane = lane_id(), w = t / WAVE;
    for (u32 c = blockIdx.x; c < chunks; c += gridDim.x) {
        const u64 ic = (u64)c * ECH;
        u64 key[ECP], kprev[ECP];
        u32 hb = 0;
#pragma unroll
        for (int k = 0; k < ECP; ++k) {
            const u64 i = ic + (u64)k * ECB + t;
            key[k] = i < P ? K[i] : 0ull;
            kprev[k] = (i > 0 && i < P) ? K[i - 1] : ~0ull;
        }
#pragma unroll
        for (int k = 0; k < ECP; ++k) {
            const u64 i = ic + (u64)k * ECB + t;
            const bool h = i < P && (i == 0 || key[k] != kprev[k]);
            if (h) hb |= 1u << k;
            const u64 bm = __ballot(h);
            if (lane == 0) s_rw[k][w] = (u32)__popcll(bm);
        }
        // every head's first partial, the gathers issued together
        u32 vv[ECP];
        GPart pf[ECP];
#pragma unroll
        for (int k = 0; k < ECP; ++k) vv[k] = ((hb >> k) & 1u) ? V[ic + (u64)k * ECB + t] : 0u;
#pragma unroll
        for (int k = 0; k < ECP; ++k)
            if ((hb >> k) & 1u) pf[k] = part[vv[k]];
        __syncthreads();
        u32 rbase = hoff[c];
#pragma unroll
        for (int k = 0; k < ECP; ++k) {
            const u64 i = ic + (u64)k * ECB + t;
            u32 before = 0, rowt = 0;
#pragma unroll
            for (int x = 0; x < ECB / WAVE; ++x) {
                const u32 v = s_rw[k][x];
                before += x < w ? v : 0u;
                rowt += v;
            }
            const u32 row = rbase + before + popc_below(__ballot((hb >> k) & 1u));
            rbase += rowt;
            if (!((hb >> k) & 1u)) continue;
            if (sharded) {
                const u32 sh = (u32)(key[k] >> kb);
                const long ps = i == 0 ? -1 : (long)(kprev[k] >> kb);
                for (long s2 = ps + 1; s2 <= (long)sh; ++s2) go[s2] = row;
            }
            if (row < cap) {
                GPart pr = pf[k];
                u64 cnt = 0;
                u32 nj = 0;
                Fx192 sum;
                fx_zero(sum);
                u32 mn = ~0u, mx = 0;
                i64 pj = pr.jid;
                u64 j = i;
                bool more = j + 1 < P && K[j + 1] == key[k];
                for (;;) {
                    cnt += pr.cn & ~PART_ODD;
                    nj += (j == i || pr.jid != pj) ? 1u : 0u;
                    pj = pr.jid;
                    const Fx192 tt = (pr.cn & PART_ODD) ? fx_from_double<FX_SPD>((double)__uint_as_float(pr.s[0]))
                                                        : part_sum192(pr);
                    fx_add(sum, tt);
                    mn = pr.mn < mn ? pr.mn : mn;
                    mx = pr.mx > mx ? pr.mx : mx;
                    if (!more) break;
                    ++j;
                    pr = part[V[j]];
                    more = j + 1 < P && K[j + 1] == key[k];
                }
                o_key[row] = (i64)(key[k] & kmask);
                o_cnt[row] = (u32)cnt;
                o_nj[row] = nj;
                o_sum[row] = fx_to_double<FX_SPD>(sum);
                o_min[row] = unord_f32(mn);
                o_max[row] = unord_f32(mx);
            }
        }
        if (sharded && P > 0 && (u64)P - 1 >= ic && (u64)P - 1 < ic + ECH && ((u64)P - 1 - ic) % ECB == (u64)t) {
            // the last pair: the shards after the last group's shard start at G
            const u32 sh = (u32)(K[P - 1] >> kb);
            for (u32 s2 = sh + 1; s2 <= S; ++s2) go[s2] = G;
        }
        __syncthreads();
    }
}

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

// the tile kernel for a direction source (0 none, 1 heading column, 2 bearing)
template <int KD, bool FL = false>
static void launch_parts(dim3 gg, hipStream_t s, u32 nn, const cv_records* sorted, const Spec& g, const PartSink& sk,
                         GridMeta* meta, const uint8_t* first = nullptr)
{
    hipLaunchKernelGGL((k_grid_part<KD, FL>), gg, dim3(GB), 0, s, nn, sorted->journey_id, sorted->ts_ms,
                       sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, g, sk, meta, first);
}

// exclusive scan of v[0, n) into out (n = *n_dev when given, at most n_max);
// mode as in k_scan_top
static void scan_counts(const u32* v, u32 n_max, const u32* n_dev, const u64* vmax, u32* out, const GridLayout& L,
                        int mode, hipStream_t s)
{
    const u32 nb = (u32)((n_max + SCH - 1) / SCH);
    const dim3 g(nb ? nb : 1);
    hipLaunchKernelGGL(k_scan_up, g, dim3(SCB), 0, s, v, n_max, n_dev, vmax, L.bsum, L.bmax);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCB), 0, s, L.bsum, nb, L.bmax, L.meta, mode);
    hipLaunchKernelGGL(k_scan_down, g, dim3(SCB), 0, s, v, n_max, n_dev, L.bsum, out);
}

// nd > 0: a direction dimension of nd sectors (plus one for records without a
// direction) from the sorted heading column hdg, else from feat's bearing
static cv_status grid_impl(const cv_records* sorted, const u64* soff, u32 S, const cv_grid_spec* grid,
                           const cv_groups* out, uint64_t capacity, u64* go, cv_result* res, void* ws, size_t ws_bytes,
                           void* stream, u32 nd = 0, double doff = 0.0, const float* hdg = nullptr,
                           const cv_features* feat = nullptr, u64* sout = nullptr, const uint8_t* first = nullptr)
{
    if (!sorted || !out || sorted->n >= (1ull << 32) || capacity >= (1ull << 32) || !spec_ok(grid))
        return CV_ERR_INVALID_ARGUMENT;
    const u64 n = sorted->n;
    hipStream_t s = (hipStream_t)stream;
    GridLayout need(nullptr, n);
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need.bytes) return CV_ERR_WORKSPACE;
    if (n == 0) {
        if (res) hipLaunchKernelGGL(k_grid_empty, dim3(1), dim3(64), 0, s, res);
        if (go) cvh::fill_u64(go, 0, (u64)S + 1, s);
        if (sout) cvh::fill_u64(sout, 0ull, S ? S : 1, s);
        return cvh::last_launch_status();
    }
    if (!sorted->journey_id || !sorted->ts_ms || !sorted->lat_deg || !sorted->lon_deg || !sorted->speed_mps)
        return CV_ERR_INVALID_ARGUMENT;
    if (capacity > 0 &&
        (!out->key || !out->count || !out->n_journeys || !out->sum_speed || !out->min_speed || !out->max_speed))
        return CV_ERR_INVALID_ARGUMENT;
    GridLayout L(ws, n);
    Spec g;
    g.lat0 = grid->lat0_deg;
    g.lon0 = grid->lon0_deg;
    g.dlat = grid->dlat_deg;
    g.dlon = grid->dlon_deg;
    g.n_lat = grid->n_lat;
    g.n_lon = grid->n_lon;
    g.t0 = grid->t0_ms;
    g.bin_ms = grid->bin_ms;
    g.tinv = 1.0 / (double)grid->bin_ms;
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
    g.sout = sout;
    u32 sb = 0;
    if (S > 1) {
        // cell keys < n_t * n_lat * n_lon; the shard index goes above them
        const unsigned __int128 cells = (unsigned __int128)grid->n_t * grid->n_lat * grid->n_lon;
        u32 kb = 0;
        while (kb < 63 && ((unsigned __int128)1 << kb) < cells) ++kb;
        while (((u64)1 << sb) < S) ++sb;
        if (kb + sb > 63) return CV_ERR_RANGE;
        g.kb = kb;
    }
    // passes the merge's key sort can need: every key lies below the grid's
    // count of (time bin, sector, cell) keys, with the shard index above kb
    // when sharded; the device's count of key bits skips the rest
    int mpasses = MAX_PASSES;
    {
        const unsigned __int128 keys = (unsigned __int128)g.tmax * (unsigned __int128)(nd + 1) *
                                       (unsigned __int128)grid->n_lat * (unsigned __int128)grid->n_lon;
        u32 b = 0;
        while (b < 64 && ((unsigned __int128)1 << b) < keys) ++b;
        if (S > 1) b = nd == 0 ? g.kb + sb : 64u;
        const int need = (int)((b + RADIX_BITS - 1) / RADIX_BITS);
        mpasses = need < MAX_PASSES ? need : MAX_PASSES;
    }
    const u64 kmask = S > 1 ? ((1ull << g.kb) - 1) : ~0ull;
    const u32 nn = (u32)n;
    const u32 tiles = (u32)L.tiles;
    const u32 pmax = (u32)(L.pmax - 1 < 0xFFFFFFFFull ? L.pmax : 0xFFFFFFFFull);
    {
        cvh::TimedScope ts_("grid_agg", s);
        hipLaunchKernelGGL(k_gmeta_init, dim3(1), dim3(64), 0, s, L.meta);
        if (sout) cvh::fill_u64(sout, 0ull, S ? S : 1, s);
        PartSink sk{L.K1, L.part, L.tcnt, L.tmax};
        const dim3 gg(tiles);
        if (nd == 0 && first) launch_parts<0, true>(gg, s, nn, sorted, g, sk, L.meta, first);
        else if (nd == 0) launch_parts<0>(gg, s, nn, sorted, g, sk, L.meta);
        else if (hdg) launch_parts<1>(gg, s, nn, sorted, g, sk, L.meta);
        else launch_parts<2>(gg, s, nn, sorted, g, sk, L.meta);
    }
    {
        cvh::TimedScope ts_("grid_tail", s);
        // partial rows -> compacted (key, row) pairs
        cvh::fill_u32(L.zero_begin, 0u, L.zero_bytes / 4, s);
        scan_counts(L.tcnt, tiles, nullptr, L.tmax, L.toff, L, 0, s);
        hipLaunchKernelGGL(k_gpart_compact, dim3(cvh::grid_for((u64)tiles * WAVE, 256, 8192)), dim3(256), 0, s,
                           L.K1, L.tcnt, L.toff, tiles, L.K0, L.V0);
        // key sort of the pairs
        const u32* cnt = &L.meta->compact_n;
        const u32* bits = &L.meta->key_bits;
        radix_hist(L.K0, pmax, cnt, mpasses, bits, L.hist, cvh::grid_for(L.pmax, 256, 1024), s);
        radix_scan(L.hist, L.offs, mpasses, s);
        radix_passes(L.K0, L.K1, L.V0, L.V0, L.V1, pmax, cnt, bits, mpasses, L.offs, L.status, L.meta->tickets, s);
        // groups: heads of equal-key runs, their rows, the merge
        const unsigned eg = (unsigned)cvh::grid_for(L.chunks, 1, 4096);
        hipLaunchKernelGGL(k_gpart_heads, dim3(eg), dim3(ECB), 0, s, L.meta, L.K0, L.K1, L.hcnt);
        scan_counts(L.hcnt, (u32)L.chunks, &L.meta->chunks, nullptr, L.hcnt, L, 1, s);
        hipLaunchKernelGGL(k_gpart_emit, dim3(eg), dim3(ECB), 0, s, L.meta, L.K0, L.K1, L.V0, L.V1, L.part, L.hcnt,
                           (u32)capacity, out->key, out->count, out->n_journeys, out->sum_speed, out->min_speed,
                           out->max_speed, go, S, g.kb, kmask, res);
        cvh::debug_rows(out->key, out->count, out->n_journeys, res, capacity, go, S, CV_DEBUG_GROUP_ORDER, s);
    }
    return cvh::last_launch_status();
}


extern "C" {

cv_status cv_grid_workspace_size(uint64_t n, const cv_grid_spec* grid, uint64_t capacity, size_t* bytes)
{
    if (!bytes || n >= (1ull << 32) || capacity >= (1ull << 32) || !spec_ok(grid)) return CV_ERR_INVALID_ARGUMENT;
    GridLayout L(nullptr, n);
    *bytes = L.bytes;
    return CV_OK;
}

cv_status cv_grid_aggregate(const cv_records* sorted, const cv_grid_spec* grid, const cv_groups* out,
                            uint64_t capacity, cv_result* res, void* ws, size_t ws_bytes, void* stream)
{
    return grid_impl(sorted, nullptr, 0, grid, out, capacity, nullptr, res, ws, ws_bytes, stream);
}

cv_status cv_grid_aggregate_flags(const cv_records* sorted, const uint8_t* flags, const cv_grid_spec* grid,
                                  const cv_groups* out, uint64_t capacity, cv_result* res, void* ws, size_t ws_bytes,
                                  void* stream)
{
    if (!flags && sorted && sorted->n > 0) return CV_ERR_INVALID_ARGUMENT;
    return grid_impl(sorted, nullptr, 0, grid, out, capacity, nullptr, res, ws, ws_bytes, stream, 0, 0.0, nullptr,
                     nullptr, nullptr, flags);
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

cv_status cv_batch_workspace_size(uint64_t n, uint32_t n_shards, uint64_t max_journeys, uint64_t journey_capacity,
                                  const cv_grid_spec* grid, uint64_t group_capacity, size_t* bytes)
{
    if (!bytes || n_shards == 0) return CV_ERR_INVALID_ARGUMENT;
    size_t a = 0, b = 0, c = 0;
    cv_status e = cv_sort_workspace_size(n, max_journeys, &a);
    if (e == CV_OK) e = cv_summary_workspace_size(n, journey_capacity, &b);
    if (e == CV_OK) e = cv_grid_workspace_size(n, grid, group_capacity, &c);
    if (e != CV_OK) return e;
    // the stages run one after the other on one stream: one region serves all three
    size_t m = a > b ? a : b;
    *bytes = m > c ? m : c;
    return CV_OK;
}

cv_status cv_batch_run(const cv_records* in, const uint64_t* shard_offsets, uint32_t n_shards,
                       const cv_grid_spec* grid, uint64_t max_journeys, uint32_t* perm, const cv_records_out* sorted,
                       const cv_features* feat, const cv_journeys* journeys, uint64_t journey_capacity,
                       uint64_t* journey_offsets, const cv_groups* groups, uint64_t group_capacity,
                       uint64_t* group_offsets, uint64_t* shard_n_out, cv_result* res, void* ws, size_t ws_bytes,
                       void* stream)
{
    if (!in || !sorted || !feat || !grid || n_shards == 0 || !shard_offsets || !journey_offsets ||
        !group_offsets || !res || grid->n_t <= 0)
        return CV_ERR_INVALID_ARGUMENT;
    if (!sorted->journey_id || !sorted->ts_ms || !sorted->lat_deg || !sorted->lon_deg || !sorted->speed_mps)
        return CV_ERR_INVALID_ARGUMENT;
    if (shard_n_out && !cvh::aligned(shard_n_out, 8)) return CV_ERR_INVALID_ARGUMENT;
    size_t need = 0;
    cv_status e = cv_batch_workspace_size(in->n, n_shards, max_journeys, journey_capacity, grid, group_capacity,
                                          &need);
    if (e != CV_OK) return e;
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need) return CV_ERR_WORKSPACE;
    e = cv_batch_sort_records_features(in, shard_offsets, n_shards, max_journeys, perm, sorted, feat, res, ws,
                                       ws_bytes, stream);
    if (e != CV_OK) return e;
    cv_records srt{};
    srt.journey_id = sorted->journey_id;
    srt.ts_ms = sorted->ts_ms;
    srt.lat_deg = sorted->lat_deg;
    srt.lon_deg = sorted->lon_deg;
    srt.speed_mps = sorted->speed_mps;
    srt.n = in->n;
    e = cv_batch_journey_summary(&srt, feat, shard_offsets, n_shards, journeys, journey_capacity, journey_offsets,
                                 res + 1, ws, ws_bytes, stream);
    if (e != CV_OK) return e;
    return grid_impl(&srt, shard_offsets, n_shards, grid, groups, group_capacity, group_offsets, res + 2, ws,
                     ws_bytes, stream, 0, 0.0, nullptr, nullptr, shard_n_out, feat->flags);
}

}  // extern "C"
