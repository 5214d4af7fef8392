// cv_sumtab.h -- the exact per-journey accumulator rows of the journey summary,
// shared with the serving form (which folds a batch's rows into its resident
// journeys).
#pragma once
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cvetl.h"

namespace cv {

constexpr int SUM_FX_DIST = 128;  // distance: 2^-128 m units
constexpr int SUM_FX_SPD = 149;   // speed: 2^-149 units (exact for every float32)

// One journey's exact partial aggregate.  Sums are 192-bit two's-complement
// limbs; maxima and the box are ordered integers; gfirst is the index of the
// journey's first record in the sorted array.
struct JAcc {
    u64 dist[3];
    u64 spd[3];
    u64 maxd;
    u64 latmin, latmax, lonmin, lonmax;
    u32 count, ndtz, maxs, gfirst;
};

// side row of a journey: sums of the values outside the 128-bit fast formats
struct AccX {
    u64 dist[3], spd[3];
};

// Exact partials of every journey of n sorted records into acc[0 .. rows) and
// accx[0 .. rows) (journeys are maximal runs of equal id, numbered in order;
// journeys past `rows` are dropped).  ws holds sum_partials_bytes(n) bytes.
size_t sum_partials_bytes(u64 n);
cv_status sum_partials(const cv_records* sorted, const cv_features* feat, u32 rows, JAcc* acc, AccX* accx, void* ws,
                       hipStream_t s);

}  // namespace cv
