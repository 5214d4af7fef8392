// cv_hygiene.hip -- optional record hygiene on (journey, time)-sorted records:
// dropping exact duplicate records (Table 1 shows one) and splitting journeys
// into trips at time gaps.  Both are order-preserving passes over tiles of
// HT records: per-tile counts (wave ballots), one scan of the tile counts,
// then the write.
//
//   k_dup_count / k_dup_write    records kept: not an exact copy of an earlier
//                                record of the same (journey, time stamp)
//   k_trip_count / k_trip_write  trip starts: a journey's first record or a
//                                gap longer than gap_ms; dense trip numbers
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_host.h"

using namespace cv;

namespace {

constexpr int HB = 256;
constexpr int HT = HB * 8;  // records per tile

// true when sorted record k repeats an earlier record of its (journey, time
// stamp) run bit for bit in latitude, longitude and speed
__device__ __forceinline__ bool is_dup(const i64* jid, const i64* ts, const double* lat, const double* lon,
                                       const float* spd, u64 k)
{
    const i64 j = jid[k], t = ts[k];
    const u64 a = (u64)__double_as_longlong(lat[k]), b = (u64)__double_as_longlong(lon[k]);
    const u32 c = __float_as_uint(spd[k]);
    for (u64 p = k; p > 0;) {
        --p;
        if (jid[p] != j || ts[p] != t) break;
        if ((u64)__double_as_longlong(lat[p]) == a && (u64)__double_as_longlong(lon[p]) == b &&
            __float_as_uint(spd[p]) == c)
            return true;
    }
    return false;
}

__device__ __forceinline__ bool trip_start(const i64* jid, const i64* ts, u64 k, i64 gap)
{
    if (k == 0 || jid[k] != jid[k - 1]) return true;
    // ts is non-decreasing inside a journey: the difference is exact in u64
    return (u64)ts[k] - (u64)ts[k - 1] > (u64)gap;
}

template <class Pred>
__device__ __forceinline__ void tile_count(u64 n, u32* tcnt, Pred pred)
{
    __shared__ u32 s_w[HB / WAVE];
    const u64 t0 = (u64)blockIdx.x * HT;
    u32 c = 0;
    for (int i = 0; i < HT / HB; ++i) {
        const u64 k = t0 + (u64)i * HB + threadIdx.x;
        c += (u32)__popcll(__ballot(k < n && pred(k)));
    }
    if (lane_id() == 0) s_w[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 t = 0;
        for (int w = 0; w < HB / WAVE; ++w) t += s_w[w];
        tcnt[blockIdx.x] = t;
    }
}

// exclusive prefix of the tile counts (one block); tcnt[tiles] = total
__global__ void __launch_bounds__(1024) k_hyg_scan(u32* __restrict__ tcnt, u64 tiles)
{
    __shared__ u32 s_tmp[1024 / WAVE];
    u32 carry = 0;
    for (u64 b = 0; b < tiles; b += 1024) {
        const u64 i = b + threadIdx.x;
        const u32 v = i < tiles ? tcnt[i] : 0u;
        u32 tot;
        const u32 ex = block_exclusive_sum<1024>(v, s_tmp, tot);
        if (i < tiles) tcnt[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) tcnt[tiles] = carry;
}

__global__ void __launch_bounds__(HB) k_dup_count(const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                  const double* __restrict__ lat, const double* __restrict__ lon,
                                                  const float* __restrict__ spd, u64 n, u32* __restrict__ tcnt)
{
    tile_count(n, tcnt, [&](u64 k) { return !is_dup(jid, ts, lat, lon, spd, k); });
}

__global__ void __launch_bounds__(HB) k_dup_write(const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                  const double* __restrict__ lat, const double* __restrict__ lon,
                                                  const float* __restrict__ spd, const u32* __restrict__ perm, u64 n,
                                                  const u32* __restrict__ tpre, cv_records_out o,
                                                  u32* __restrict__ perm_out)
{
    __shared__ u32 s_w[HB / WAVE];
    __shared__ u32 s_base;
    const u64 t0 = (u64)blockIdx.x * HT;
    const int w = threadIdx.x / WAVE;
    if (threadIdx.x == 0) s_base = tpre[blockIdx.x];
    for (int i = 0; i < HT / HB; ++i) {
        const u64 k = t0 + (u64)i * HB + threadIdx.x;
        const bool keep = k < n && !is_dup(jid, ts, lat, lon, spd, k);
        const u64 m = __ballot(keep);
        if (lane_id() == 0) s_w[w] = (u32)__popcll(m);
        __syncthreads();
        u32 at = s_base + popc_below(m);
        for (int x = 0; x < w; ++x) at += s_w[x];
        if (keep) {
            o.journey_id[at] = jid[k];
            o.ts_ms[at] = ts[k];
            o.lat_deg[at] = lat[k];
            o.lon_deg[at] = lon[k];
            o.speed_mps[at] = spd[k];
            if (perm_out) perm_out[at] = perm[k];
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int x = 0; x < HB / WAVE; ++x) s_base += s_w[x];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(HB) k_trip_count(const i64* __restrict__ jid, const i64* __restrict__ ts, u64 n,
                                                   i64 gap, u32* __restrict__ tcnt)
{
    tile_count(n, tcnt, [&](u64 k) { return trip_start(jid, ts, k, gap); });
}

// trip_id[k] = number of trip starts at or before k, minus one; trip
// journeys[t] = the journey id of trip t's first record (t < cap)
__global__ void __launch_bounds__(HB) k_trip_write(const i64* __restrict__ jid, const i64* __restrict__ ts, u64 n,
                                                   i64 gap, const u32* __restrict__ tpre, i64* __restrict__ trip_id,
                                                   i64* __restrict__ trip_journey, u64 cap)
{
    __shared__ u32 s_w[HB / WAVE];
    __shared__ u32 s_base;
    const u64 t0 = (u64)blockIdx.x * HT;
    const int w = threadIdx.x / WAVE;
    if (threadIdx.x == 0) s_base = tpre[blockIdx.x];
    for (int i = 0; i < HT / HB; ++i) {
        const u64 k = t0 + (u64)i * HB + threadIdx.x;
        const bool st = k < n && trip_start(jid, ts, k, gap);
        const u64 m = __ballot(st);
        if (lane_id() == 0) s_w[w] = (u32)__popcll(m);
        __syncthreads();
        // starts up to and including this lane
        u32 upto = s_base + popc_below(m) + (st ? 1u : 0u);
        for (int x = 0; x < w; ++x) upto += s_w[x];
        if (k < n) {
            trip_id[k] = (i64)upto - 1;
            if (st && (u64)upto - 1 < cap && trip_journey) trip_journey[upto - 1] = jid[k];
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int x = 0; x < HB / WAVE; ++x) s_base += s_w[x];
        __syncthreads();
    }
}

__global__ void k_hyg_result(const u32* __restrict__ tcnt, u64 tiles, u64 cap, cv_result* res)
{
    if (threadIdx.x != 0 || !res) return;
    cv_result r = {};
    const u64 total = tcnt[tiles];
    r.status = total > cap ? CV_ERR_CAPACITY : CV_OK;
    r.count = total;
    r.required = total > cap ? total : 0;
    *res = r;
}

bool records_ok(const cv_records* r)
{
    return r && (r->n == 0 || (r->journey_id && r->ts_ms && r->lat_deg && r->lon_deg && r->speed_mps));
}

}  // namespace

extern "C" {

cv_status cv_hygiene_workspace_size(uint64_t n, size_t* bytes)
{
    if (!bytes || n >= (1ull << 32)) return CV_ERR_INVALID_ARGUMENT;
    *bytes = cvh::align_up(((n + HT - 1) / HT + 1) * sizeof(u32));
    return CV_OK;
}

cv_status cv_drop_duplicates(const cv_records* sorted, const uint32_t* perm, const cv_records_out* out,
                             uint32_t* perm_out, cv_result* res, void* ws, size_t ws_bytes, void* stream)
{
    if (!records_ok(sorted) || sorted->n >= (1ull << 32) || !out || !res) return CV_ERR_INVALID_ARGUMENT;
    const u64 n = sorted->n;
    if (n && (!out->journey_id || !out->ts_ms || !out->lat_deg || !out->lon_deg || !out->speed_mps))
        return CV_ERR_INVALID_ARGUMENT;
    if (perm_out && !perm) return CV_ERR_INVALID_ARGUMENT;
    size_t need = 0;
    cv_hygiene_workspace_size(n, &need);
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need) return CV_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    cvh::TimedScope ts_("drop_duplicates", s);
    const u64 tiles = (n + HT - 1) / HT;
    u32* tcnt = (u32*)ws;
    if (tiles)
        hipLaunchKernelGGL(k_dup_count, dim3((unsigned)tiles), dim3(HB), 0, s, sorted->journey_id, sorted->ts_ms,
                           sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, n, tcnt);
    hipLaunchKernelGGL(k_hyg_scan, dim3(1), dim3(1024), 0, s, tcnt, tiles);
    if (tiles)
        hipLaunchKernelGGL(k_dup_write, dim3((unsigned)tiles), dim3(HB), 0, s, sorted->journey_id, sorted->ts_ms,
                           sorted->lat_deg, sorted->lon_deg, sorted->speed_mps, perm, n, tcnt, *out, perm_out);
    hipLaunchKernelGGL(k_hyg_result, dim3(1), dim3(64), 0, s, tcnt, tiles, n, res);
    return cvh::last_launch_status();
}

cv_status cv_split_trips(const cv_records* sorted, int64_t gap_ms, int64_t* trip_id, int64_t* trip_journey,
                         uint64_t capacity, cv_result* res, void* ws, size_t ws_bytes, void* stream)
{
    if (!sorted || sorted->n >= (1ull << 32) || gap_ms < 0 || !res) return CV_ERR_INVALID_ARGUMENT;
    const u64 n = sorted->n;
    if (n && (!sorted->journey_id || !sorted->ts_ms || !trip_id)) return CV_ERR_INVALID_ARGUMENT;
    if (capacity && !trip_journey) return CV_ERR_INVALID_ARGUMENT;
    size_t need = 0;
    cv_hygiene_workspace_size(n, &need);
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need) return CV_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    cvh::TimedScope ts_("split_trips", s);
    const u64 tiles = (n + HT - 1) / HT;
    u32* tcnt = (u32*)ws;
    if (tiles)
        hipLaunchKernelGGL(k_trip_count, dim3((unsigned)tiles), dim3(HB), 0, s, sorted->journey_id, sorted->ts_ms, n,
                           (i64)gap_ms, tcnt);
    hipLaunchKernelGGL(k_hyg_scan, dim3(1), dim3(1024), 0, s, tcnt, tiles);
    if (tiles)
        hipLaunchKernelGGL(k_trip_write, dim3((unsigned)tiles), dim3(HB), 0, s, sorted->journey_id, sorted->ts_ms, n,
                           (i64)gap_ms, tcnt, trip_id, capacity ? trip_journey : nullptr, (u64)capacity);
    hipLaunchKernelGGL(k_hyg_result, dim3(1), dim3(64), 0, s, tcnt, tiles, (u64)capacity, res);
    return cvh::last_launch_status();
}

}  // extern "C"
