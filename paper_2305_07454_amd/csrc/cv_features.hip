// cv_features.hip -- cv_journey_features: per-point kinematics inside each
// journey of (journey, time)-sorted records.
//
// A block of FB threads owns FB consecutive points; consecutive blocks overlap
// by two points, so every phase is one pass of one item per thread:
//   thread t loads point base + t and computes sin(phi), cos(phi) once;
//   thread t >= 1 evaluates the step (t-1 -> t): distance, dt, speed, bearing;
//   thread t >= 2 writes record base + t, whose acceleration and heading change
//   take the speed and bearing of step t-1 from LDS.
// A block writes FB - 2 records.  Every expression is evaluated as
// parenthesised below with IEEE double division and no FMA contraction (this
// file is compiled with -ffp-contract=off).
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_host.h"
#include "cv_kin.h"

using namespace cv;

namespace {

constexpr int FB = 256;
constexpr int FOUT = FB - 2;  // records written per block

__global__ void __launch_bounds__(FB) k_features(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                 const double* __restrict__ lat, const double* __restrict__ lon,
                                                 double* __restrict__ o_step, double* __restrict__ o_dt,
                                                 double* __restrict__ o_spd, double* __restrict__ o_acc,
                                                 double* __restrict__ o_brg, double* __restrict__ o_dhd,
                                                 uint8_t* __restrict__ o_flags, const u64* __restrict__ soff,
                                                 u32 S)
{
    __shared__ i64 s_jid[FB];
    __shared__ i64 s_ts[FB];
    __shared__ double s_lat[FB];
    __shared__ double s_lon[FB];
    __shared__ double s_sphi[FB];
    __shared__ double s_cphi[FB];
    __shared__ double s_v[FB];
    __shared__ double s_b[FB];
    __shared__ u32 s_f[FB];

    const int t = threadIdx.x;
    const long r = (long)blockIdx.x * FOUT - 2 + t;  // this thread's point and step
    const bool in = r >= 0 && r < (long)n;
    i64 j = 0, tsr = 0;
    double la = 0.0, lo = 0.0, sphi = 0.0, cphi = 0.0;
    bool fin = false;
    if (in) {
        j = jid[r];
        tsr = ts[r];
        la = lat[r];
        lo = lon[r];
        fin = isfinite(la) && isfinite(lo);
        if (fin) sincos(la * KIN_DEG2RAD, &sphi, &cphi);
    }
    s_jid[t] = j;
    s_ts[t] = tsr;
    s_lat[t] = la;
    s_lon[t] = lo;
    s_sphi[t] = sphi;
    s_cphi[t] = cphi;
    __syncthreads();

    // step (t-1 -> t) of record r
    KinStep k{0.0, 0.0, 0.0, 0.0, 0u};
    if (in && t >= 1) {
        const int p = t - 1;
        bool head = (r == 0) || (s_jid[p] != j);
        if (S > 1 && !head) {
            // the block's first shard, then forward to this record's
            const long b0 = (long)blockIdx.x * FOUT - 2;
            u32 sh = shard_of(soff, S, (u64)(b0 > 0 ? b0 : 0));
            while (sh + 1 < S && soff[sh + 1] <= (u64)r) ++sh;
            head = soff[sh] == (u64)r;
        }
        const double lap = s_lat[p], lop = s_lon[p];
        k = kin_step(head, fin, tsr, la, lo, cphi, isfinite(lap) && isfinite(lop), s_ts[p], lap, lop, s_cphi[p],
                     s_sphi[p]);
    }
    s_v[t] = k.v;
    s_b[t] = k.b;
    s_f[t] = k.f;
    __syncthreads();
    if (!in || t < 2) return;
    const int p = t - 1;
    u32 f = k.f;
    double acc, dh;
    kin_final(f, k.v, k.b, k.dts, s_f[p], s_v[p], s_b[p], acc, dh);
    const double step = k.step, dts = k.dts, v = k.v, b = k.b;
    o_step[r] = step;
    o_dt[r] = dts;
    o_spd[r] = v;
    o_acc[r] = acc;
    o_brg[r] = b;
    o_dhd[r] = dh;
    o_flags[r] = (uint8_t)f;
}

}  // namespace

static cv_status features_impl(const cv_records* sorted, const u64* soff, u32 S, const cv_features* out, void* stream)
{
    if (!sorted || !out || sorted->n >= (1ull << 32)) return CV_ERR_INVALID_ARGUMENT;
    const u64 n = sorted->n;
    if (n == 0) return CV_OK;
    if (!sorted->journey_id || !sorted->ts_ms || !sorted->lat_deg || !sorted->lon_deg) return CV_ERR_INVALID_ARGUMENT;
    if (!out->step_m || !out->dt_s || !out->speed_mps || !out->accel_mps2 || !out->bearing_deg ||
        !out->dheading_deg || !out->flags)
        return CV_ERR_INVALID_ARGUMENT;
    hipStream_t s = (hipStream_t)stream;
    cvh::TimedScope ts_("features", s);
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n + FOUT - 1) / FOUT)), dim3(FB), 0, s, (u32)n, sorted->journey_id,
                       sorted->ts_ms, sorted->lat_deg, sorted->lon_deg, out->step_m, out->dt_s, out->speed_mps,
                       out->accel_mps2, out->bearing_deg, out->dheading_deg, out->flags, soff, S);
    return cvh::last_launch_status();
}

extern "C" cv_status cv_journey_features(const cv_records* sorted, const cv_features* out, void* stream)
{
    return features_impl(sorted, nullptr, 0, out, stream);
}

extern "C" cv_status cv_batch_journey_features(const cv_records* sorted, const uint64_t* shard_offsets,
                                               uint32_t n_shards, const cv_features* out, void* stream)
{
    if (n_shards == 0 || !shard_offsets || !cvh::aligned(shard_offsets, 8)) return CV_ERR_INVALID_ARGUMENT;
    return features_impl(sorted, shard_offsets, n_shards, out, stream);
}
