// cv_features.hip -- cv_journey_features: per-point kinematics inside each
// journey of (journey, time)-sorted records.
//
// A block owns FB consecutive records.  It stages FB + 2 points (two of halo
// before the tile) in LDS with sin(phi) and cos(phi) computed once per point,
// then evaluates FB + 1 steps (p -> k) so that acceleration and heading change
// of record k can use the speed and bearing of record k-1 from LDS.  Every
// expression is evaluated as parenthesised below with IEEE double division and
// no FMA contraction (this file is compiled with -ffp-contract=off).
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_host.h"

using namespace cv;

namespace {

constexpr int FB = 256;
constexpr double EARTH_R_M = 6371008.8;
constexpr double DEG2RAD = 3.14159265358979323846 / 180.0;
constexpr double RAD2DEG = 180.0 / 3.14159265358979323846;

__global__ void __launch_bounds__(FB) k_features(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                 const double* __restrict__ lat, const double* __restrict__ lon,
                                                 double* __restrict__ o_step, double* __restrict__ o_dt,
                                                 double* __restrict__ o_spd, double* __restrict__ o_acc,
                                                 double* __restrict__ o_brg, double* __restrict__ o_dhd,
                                                 uint8_t* __restrict__ o_flags, const u64* __restrict__ soff,
                                                 u32 S)
{
    __shared__ i64 s_jid[FB + 2];
    __shared__ i64 s_ts[FB + 2];
    __shared__ double s_lat[FB + 2];
    __shared__ double s_lon[FB + 2];
    __shared__ double s_sphi[FB + 2];
    __shared__ double s_cphi[FB + 2];
    __shared__ u32 s_fin[FB + 2];
    __shared__ double s_step[FB + 1];
    __shared__ double s_dt[FB + 1];
    __shared__ double s_v[FB + 1];
    __shared__ double s_b[FB + 1];
    __shared__ u32 s_f[FB + 1];

    const long s0 = (long)blockIdx.x * FB;
    // points q <-> record s0 - 2 + q
    for (int q = threadIdx.x; q < FB + 2; q += FB) {
        long r = s0 - 2 + q;
        if (r >= 0 && r < (long)n) {
            double la = lat[r], lo = lon[r];
            s_jid[q] = jid[r];
            s_ts[q] = ts[r];
            s_lat[q] = la;
            s_lon[q] = lo;
            bool fin = isfinite(la) && isfinite(lo);
            s_fin[q] = fin;
            double phi = la * DEG2RAD;
            s_sphi[q] = fin ? sin(phi) : 0.0;
            s_cphi[q] = fin ? cos(phi) : 0.0;
        }
    }
    __syncthreads();

    // step j <-> record k = s0 - 1 + j: predecessor point q = j, own point q = j + 1
    for (int j = threadIdx.x; j < FB + 1; j += FB) {
        long k = s0 - 1 + j;
        double step = 0.0, dts = 0.0, v = 0.0, b = 0.0;
        u32 f = 0;
        if (k >= 0 && k < (long)n) {
            const int qk = j + 1, qp = j;
            bool head = (k == 0) || (s_jid[qk] != s_jid[qp]) || (S > 1 && shard_start(soff, S, (u64)k));
            if (head) {
                f = CV_FLAG_FIRST | (s_fin[qk] ? 0u : CV_FLAG_BAD_COORD);
            } else {
                i64 dt_ms = s_ts[qk] - s_ts[qp];
                f = dt_ms == 0 ? CV_FLAG_DT_ZERO : 0u;
                if (!s_fin[qk] || !s_fin[qp]) {
                    f |= CV_FLAG_BAD_COORD;
                } else {
                    dts = (double)dt_ms / 1000.0;
                    double dphi = (s_lat[qk] - s_lat[qp]) * DEG2RAD;
                    double dlam = (s_lon[qk] - s_lon[qp]) * DEG2RAD;
                    double sp = sin(0.5 * dphi);
                    double sl = sin(0.5 * dlam);
                    double cphi1 = s_cphi[qp];
                    double cphi2 = s_cphi[qk];
                    double a = (sp * sp) + ((cphi1 * cphi2) * (sl * sl));
                    step = (2.0 * EARTH_R_M) * asin(fmin(1.0, sqrt(a)));
                    if (dt_ms > 0) {
                        v = step / dts;
                        f |= CV_FLAG_SPEED_OK;
                    }
                    if (step > 0.0) {
                        double y = sin(dlam) * cphi2;
                        double x = sin(dphi) + (((2.0 * s_sphi[qp]) * cphi2) * (sl * sl));
                        b = atan2(y, x) * RAD2DEG;
                        if (b < 0.0) b += 360.0;
                        if (b >= 360.0) b -= 360.0;
                        f |= CV_FLAG_BEARING_OK;
                    }
                }
            }
        }
        s_step[j] = step;
        s_dt[j] = dts;
        s_v[j] = v;
        s_b[j] = b;
        s_f[j] = f;
    }
    __syncthreads();

    // record k = s0 + t owns step j = t + 1; its predecessor's step is j - 1 = t
    const int t = threadIdx.x;
    const long k = s0 + t;
    if (k >= (long)n) return;
    const int j = t + 1;
    u32 f = s_f[j];
    const u32 fp = s_f[j - 1];
    const double v = s_v[j], b = s_b[j], dts = s_dt[j];
    double acc = 0.0, dh = 0.0;
    if ((f & CV_FLAG_SPEED_OK) && (fp & CV_FLAG_SPEED_OK)) {
        acc = (v - s_v[j - 1]) / dts;
        f |= CV_FLAG_ACCEL_OK;
    }
    if ((f & CV_FLAG_BEARING_OK) && (fp & CV_FLAG_BEARING_OK)) {
        double d = b - s_b[j - 1];
        if (d > 180.0) d -= 360.0;
        else if (d <= -180.0) d += 360.0;
        dh = d;
        f |= CV_FLAG_DHEAD_OK;
    }
    o_step[k] = s_step[j];
    o_dt[k] = dts;
    o_spd[k] = v;
    o_acc[k] = acc;
    o_brg[k] = b;
    o_dhd[k] = dh;
    o_flags[k] = (uint8_t)f;
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
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n + FB - 1) / FB)), dim3(FB), 0, s, (u32)n, sorted->journey_id,
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
