// cv_kin.h -- the per-point kinematics of (journey, time)-sorted records
// (haversine step on a sphere, dt, derived speed, initial bearing, then
// acceleration and heading change from the step before), shared by the
// features kernel and the fused gather-and-features kernel of the sort.
// Every expression is evaluated as parenthesised, with IEEE double division
// and no FMA contraction (files including this are compiled with
// -ffp-contract=off), so both kernels give the same bits.
#pragma once
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cvetl.h"

namespace cv {

constexpr double KIN_EARTH_R_M = 6371008.8;
constexpr double KIN_DEG2RAD = 3.14159265358979323846 / 180.0;
constexpr double KIN_RAD2DEG = 180.0 / 3.14159265358979323846;

struct KinStep {
    double step, dts, v, b;
    u32 f;
};

// the step (p -> k) of record k: p is its predecessor in the sorted order
// unless k heads a journey (or a shard); fin / pfin: finite coordinates;
// cphi, sphi: cos and sin of the latitudes (computed once per point)
__device__ __forceinline__ KinStep kin_step(bool head, bool fin, i64 ts, double la, double lo, double cphi2,
                                            bool pfin, i64 pts, double lap, double lop, double cphi1,
                                            double sphi1)
{
    KinStep o;
    o.step = 0.0;
    o.dts = 0.0;
    o.v = 0.0;
    o.b = 0.0;
    if (head) {
        o.f = CV_FLAG_FIRST | (fin ? 0u : CV_FLAG_BAD_COORD);
        return o;
    }
    const i64 dt_ms = ts - pts;
    u32 f = dt_ms == 0 ? CV_FLAG_DT_ZERO : 0u;
    if (!fin || !pfin) {
        o.f = f | CV_FLAG_BAD_COORD;
        return o;
    }
    o.dts = (double)dt_ms / 1000.0;
    const double dphi = (la - lap) * KIN_DEG2RAD;
    const double dlam = (lo - lop) * KIN_DEG2RAD;
    // half-angle sines and cosines; the full-angle sines of the bearing
    // follow from them (sin 2u = 2 sin u cos u)
    double sp, cp, sl, cl;
    sincos(0.5 * dphi, &sp, &cp);
    sincos(0.5 * dlam, &sl, &cl);
    const double a = (sp * sp) + ((cphi1 * cphi2) * (sl * sl));
    o.step = (2.0 * KIN_EARTH_R_M) * asin(fmin(1.0, sqrt(a)));
    if (dt_ms > 0) {
        o.v = o.step / o.dts;
        f |= CV_FLAG_SPEED_OK;
    }
    if (o.step > 0.0) {
        const double y = ((2.0 * sl) * cl) * cphi2;
        const double x = ((2.0 * sp) * cp) + (((2.0 * sphi1) * cphi2) * (sl * sl));
        double b = atan2(y, x) * KIN_RAD2DEG;
        if (b < 0.0) b += 360.0;
        if (b >= 360.0) b -= 360.0;
        o.b = b;
        f |= CV_FLAG_BEARING_OK;
    }
    o.f = f;
    return o;
}

// acceleration and heading change of a step from the step before (fp, vp,
// bp); f gains ACCEL_OK / DHEAD_OK
__device__ __forceinline__ void kin_final(u32& f, double v, double b, double dts, u32 fp, double vp, double bp,
                                          double& acc, double& dh)
{
    acc = 0.0;
    dh = 0.0;
    if ((f & CV_FLAG_SPEED_OK) && (fp & CV_FLAG_SPEED_OK)) {
        acc = (v - vp) / dts;
        f |= CV_FLAG_ACCEL_OK;
    }
    if ((f & CV_FLAG_BEARING_OK) && (fp & CV_FLAG_BEARING_OK)) {
        double d = b - bp;
        if (d > 180.0) d -= 360.0;
        else if (d <= -180.0) d += 360.0;
        dh = d;
        f |= CV_FLAG_DHEAD_OK;
    }
}

}  // namespace cv
