/*
 * cv_oracle.c -- CPU oracle for the connected-vehicle ETL hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded,
 * obviously-correct definition of what the GPU path computes.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header or constant with the HIP library; neither includes or
 * links the other.
 *
 * Built with: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared ... -lm
 * (no fast-math, no FMA contraction: every floating-point expression below is
 * evaluated exactly as parenthesised, with glibc's libm for sin/cos/asin/atan2/
 * sqrt/floor).
 *
 * What the paper fixes and what is read into it
 * ---------------------------------------------
 * The paper (Methods, "Accelerated ETL Algorithm/Framework", steps (2)-(5),
 * and Algorithm 2) describes: a unique index over the records of all
 * journeys; discretised latitude, longitude and time bins obtained as
 * floor((x - x_min) / x_step); one unrolled global index per record built from
 * those bins; and per-cell reductions (count, sum, count-unique, mean; Table 3
 * "Reduction" rows).  It gives no ordering rule, no kinematics and no
 * per-journey summary; those are defined below as plain definitions (order by
 * (journey, time) with ties in input order; haversine on a sphere; exact
 * rounded sums).  Every function cites the passage or the reading it follows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Feature flag bits (per sorted record). */
#define F_FIRST      0x01u  /* first record of its journey                 */
#define F_DT_ZERO    0x02u  /* same timestamp as the predecessor           */
#define F_SPEED_OK   0x04u  /* derived speed defined (dt > 0)              */
#define F_ACCEL_OK   0x08u  /* acceleration defined                        */
#define F_BEARING_OK 0x10u  /* bearing defined (non-zero step)             */
#define F_DHEAD_OK   0x20u  /* heading change defined                      */
#define F_BAD_COORD  0x40u  /* non-finite coordinate at k or predecessor   */

/* Sphere radius (mean Earth radius, 6371.0088 km) and degree conversions. */
static const double EARTH_R_M = 6371008.8;
static const double DEG2RAD = 3.14159265358979323846 / 180.0;
static const double RAD2DEG = 180.0 / 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Exact rounded summation.                                                  */
/*                                                                           */
/* The sum of a list of doubles is defined as the exact real sum rounded to  */
/* nearest-even.  Computed with Shewchuk's non-overlapping partials (Adaptive */
/* Precision Floating-Point Arithmetic, 1997) followed by the half-way        */
/* correction used by Python's math.fsum; all inputs are finite.             */
/* ------------------------------------------------------------------------ */
typedef struct {
    double p[160];
    int n;
} xsum_t;

static void xsum_init(xsum_t* s) { s->n = 0; }

static void xsum_add(xsum_t* s, double x)
{
    int i = 0;
    for (int j = 0; j < s->n; ++j) {
        double y = s->p[j];
        if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
        double hi = x + y;
        double lo = y - (hi - x);
        if (lo != 0.0) s->p[i++] = lo;
        x = hi;
    }
    if (i >= 160) abort();
    s->p[i] = x;
    s->n = i + 1;
}

/* An exactly-zero sum is +0.0 (signed zeros count as +0.0 throughout). */
static double xsum_round_raw(const xsum_t* s);
static double xsum_round(const xsum_t* s) { return xsum_round_raw(s) + 0.0; }

static double xsum_round_raw(const xsum_t* s)
{
    int n = s->n;
    double hi = 0.0, lo = 0.0;
    if (n == 0) return 0.0;
    hi = s->p[--n];
    while (n > 0) {
        double x = hi;
        double y = s->p[--n];
        hi = x + y;
        double yr = hi - x;
        lo = y - yr;
        if (lo != 0.0) break;
    }
    if (n > 0 && ((lo < 0.0 && s->p[n - 1] < 0.0) || (lo > 0.0 && s->p[n - 1] > 0.0))) {
        double y = lo * 2.0;
        double x = hi + y;
        double yr = x - hi;
        if (y == yr) hi = x;
    }
    return hi;
}

double orc_fsum(int64_t n, const double* x)
{
    xsum_t s;
    xsum_init(&s);
    for (int64_t i = 0; i < n; ++i) xsum_add(&s, x[i]);
    return xsum_round(&s);
}

/* -0.0 counts as +0.0 in min/max of speeds. */
static float canon0(float v) { return v == 0.0f ? 0.0f : v; }

/* ------------------------------------------------------------------------ */
/* Order: the paper's "unique index" over all journeys (Methods, step (2)),   */
/* read as a stable sort of record indices by (journey id, timestamp), both   */
/* compared as signed 64-bit integers, ties kept in input order.  The sort is */
/* a plain top-down merge sort written out here, so that stability is a      */
/* property of this code (the merge takes from the left run on equal keys),  */
/* not of the C library's qsort.                                             */
/* ------------------------------------------------------------------------ */
static const int64_t* g_jid;
static const int64_t* g_ts;

/* 1 when record i's (journey, time) key is strictly below record j's */
static int key_less(uint32_t i, uint32_t j)
{
    if (g_jid[i] != g_jid[j]) return g_jid[i] < g_jid[j];
    return g_ts[i] < g_ts[j];
}

/* sort a[lo, hi) stably, tmp as scratch of the same length */
static void merge_sort(uint32_t* a, uint32_t* tmp, int64_t lo, int64_t hi)
{
    if (hi - lo < 2) return;
    int64_t mid = lo + (hi - lo) / 2;
    merge_sort(a, tmp, lo, mid);
    merge_sort(a, tmp, mid, hi);
    int64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) {
        /* the right element goes first only when strictly smaller */
        if (key_less(a[j], a[i])) tmp[k++] = a[j++];
        else tmp[k++] = a[i++];
    }
    while (i < mid) tmp[k++] = a[i++];
    while (j < hi) tmp[k++] = a[j++];
    for (k = lo; k < hi; ++k) a[k] = tmp[k];
}

void orc_sort(int64_t n, const int64_t* jid, const int64_t* ts, uint32_t* perm)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    uint32_t* tmp = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    if (!tmp) abort();
    g_jid = jid;
    g_ts = ts;
    merge_sort(perm, tmp, 0, n);
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Late records of a stream (the serving form's reading of the order when    */
/* records arrive in pushes).  The paper's pipeline is batch only; the       */
/* streamed result is defined as the plain result on the concatenation of    */
/* the pushes, provided no journey's time goes backwards across pushes.  A   */
/* record that does is late: its time is below the largest time of the       */
/* non-late records its journey had in earlier pushes.  Within one push the  */
/* records are ordered by the sort, so only earlier pushes can make a record */
/* late.  push_end[b] is the end (exclusive) of push b in arrival order;     */
/* late[i] receives 1 for a late record, else 0.  Returns the late count.    */
/* ------------------------------------------------------------------------ */
static int key_jid_arrival_less(uint32_t i, uint32_t j)
{
    if (g_jid[i] != g_jid[j]) return g_jid[i] < g_jid[j];
    return i < j;
}

static void merge_sort_by_journey(uint32_t* a, uint32_t* tmp, int64_t lo, int64_t hi)
{
    if (hi - lo < 2) return;
    int64_t mid = lo + (hi - lo) / 2;
    merge_sort_by_journey(a, tmp, lo, mid);
    merge_sort_by_journey(a, tmp, mid, hi);
    int64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) {
        if (key_jid_arrival_less(a[j], a[i])) tmp[k++] = a[j++];
        else tmp[k++] = a[i++];
    }
    while (i < mid) tmp[k++] = a[i++];
    while (j < hi) tmp[k++] = a[j++];
    for (k = lo; k < hi; ++k) a[k] = tmp[k];
}

int64_t orc_stream_late(int64_t n, const int64_t* jid, const int64_t* ts, int64_t n_push,
                        const int64_t* push_end, uint8_t* late)
{
    int64_t* push = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    uint32_t* idx = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    uint32_t* tmp = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    if (!push || !idx || !tmp) abort();
    /* the push of every record */
    int64_t b = 0;
    for (int64_t i = 0; i < n; ++i) {
        while (b < n_push && push_end[b] <= i) ++b;
        push[i] = b;
        idx[i] = (uint32_t)i;
        late[i] = 0;
    }
    /* each journey's records in arrival order */
    g_jid = jid;
    merge_sort_by_journey(idx, tmp, 0, n);
    int64_t n_late = 0;
    for (int64_t a = 0; a < n;) {
        int64_t e = a + 1;
        while (e < n && jid[idx[e]] == jid[idx[a]]) ++e;
        int have_last = 0, have_cur = 0;
        int64_t last = 0;     /* largest non-late time of earlier pushes */
        int64_t cur = 0;      /* largest non-late time of the current push */
        int64_t cur_push = -1;
        for (int64_t c = a; c < e; ++c) {
            uint32_t i = idx[c];
            if (push[i] != cur_push) {
                /* a new push: what the previous one held becomes history */
                if (have_cur && (!have_last || cur > last)) {
                    last = cur;
                    have_last = 1;
                }
                have_cur = 0;
                cur_push = push[i];
            }
            if (have_last && ts[i] < last) {
                late[i] = 1;
                ++n_late;
            } else if (!have_cur || ts[i] > cur) {
                cur = ts[i];
                have_cur = 1;
            }
        }
        a = e;
    }
    free(push);
    free(idx);
    free(tmp);
    return n_late;
}

/* ------------------------------------------------------------------------ */
/* Per-point kinematics over records sorted by (journey, time).              */
/*                                                                           */
/* The dataset carries GPS position, speed and heading per sample (Methods,  */
/* "Connected Vehicle Dataset"); the paper derives none of them, so the      */
/* definitions are: step = great-circle (haversine) distance on a sphere of  */
/* radius 6371008.8 m from the predecessor p = k-1 of the same journey; dt in */
/* seconds; speed = step / dt when dt > 0; acceleration = backward difference */
/* of that speed over dt when both speeds exist; bearing = initial            */
/* great-circle course from p to k, clockwise from north in [0, 360), defined */
/* when the step is non-zero; heading change = bearing(k) - bearing(p)        */
/* wrapped into (-180, 180].  The bearing's x term uses the identity          */
/* cos(a)sin(b) - sin(a)cos(b)cos(d) = sin(b-a) + 2 sin(a)cos(b)sin^2(d/2),   */
/* which avoids the cancellation of the textbook form for short steps.        */
/* ------------------------------------------------------------------------ */
void orc_features(int64_t n, const int64_t* jid, const int64_t* ts,
                  const double* lat, const double* lon,
                  double* step_m, double* dt_s, double* speed_mps, double* accel_mps2,
                  double* bearing_deg, double* dheading_deg, uint8_t* flags)
{
    for (int64_t k = 0; k < n; ++k) {
        int head = (k == 0) || (jid[k] != jid[k - 1]);
        step_m[k] = 0.0;
        dt_s[k] = 0.0;
        speed_mps[k] = 0.0;
        accel_mps2[k] = 0.0;
        bearing_deg[k] = 0.0;
        dheading_deg[k] = 0.0;
        int bad_k = !isfinite(lat[k]) || !isfinite(lon[k]);
        if (head) {
            flags[k] = (uint8_t)(F_FIRST | (bad_k ? F_BAD_COORD : 0u));
            continue;
        }
        int64_t p = k - 1;
        int64_t dt_ms = ts[k] - ts[p];
        unsigned f = (dt_ms == 0) ? F_DT_ZERO : 0u;
        if (bad_k || !isfinite(lat[p]) || !isfinite(lon[p])) {
            flags[k] = (uint8_t)(f | F_BAD_COORD);
            continue;
        }
        double dts = (double)dt_ms / 1000.0;
        double phi1 = lat[p] * DEG2RAD;
        double phi2 = lat[k] * DEG2RAD;
        double dphi = (lat[k] - lat[p]) * DEG2RAD;
        double dlam = (lon[k] - lon[p]) * DEG2RAD;
        double sp = sin(0.5 * dphi);
        double sl = sin(0.5 * dlam);
        double cphi1 = cos(phi1);
        double cphi2 = cos(phi2);
        double a = (sp * sp) + ((cphi1 * cphi2) * (sl * sl));
        double step = (2.0 * EARTH_R_M) * asin(fmin(1.0, sqrt(a)));
        double v = 0.0;
        if (dt_ms > 0) {
            v = step / dts;
            f |= F_SPEED_OK;
        }
        double acc = 0.0;
        if ((f & F_SPEED_OK) && (flags[p] & F_SPEED_OK)) {
            acc = (v - speed_mps[p]) / dts;
            f |= F_ACCEL_OK;
        }
        double b = 0.0;
        if (step > 0.0) {
            double y = sin(dlam) * cphi2;
            double x = sin(dphi) + (((2.0 * sin(phi1)) * cphi2) * (sl * sl));
            b = atan2(y, x) * RAD2DEG;
            if (b < 0.0) b += 360.0;
            if (b >= 360.0) b -= 360.0;
            f |= F_BEARING_OK;
        }
        double dh = 0.0;
        if ((f & F_BEARING_OK) && (flags[p] & F_BEARING_OK)) {
            double d = b - bearing_deg[p];
            if (d > 180.0) d -= 360.0;
            else if (d <= -180.0) d += 360.0;
            dh = d;
            f |= F_DHEAD_OK;
        }
        step_m[k] = step;
        dt_s[k] = dts;
        speed_mps[k] = v;
        accel_mps2[k] = acc;
        bearing_deg[k] = b;
        dheading_deg[k] = dh;
        flags[k] = (uint8_t)f;
    }
}

/* ------------------------------------------------------------------------ */
/* Per-journey summary (one row per journey, ascending journey id).           */
/* A journey is a maximal run of equal journey id in sorted order (the       */
/* paper's "unique journey identifier", Methods, dataset description).        */
/* Sums are exact-rounded; signed zeros count as +0.0; the bounding box       */
/* covers points whose latitude and longitude are both finite (+inf/-inf when */
/* there is none); max derived speed is over SPEED_OK points (0.0 if none).   */
/* Returns the number of journeys J; rows beyond `cap` are not written.      */
/* ------------------------------------------------------------------------ */
int64_t orc_summary(int64_t n, const int64_t* jid, const int64_t* ts,
                    const double* lat, const double* lon, const float* speed,
                    const double* step_m, const double* dspeed, const uint8_t* flags,
                    int64_t cap,
                    int64_t* o_jid, uint32_t* o_first, uint32_t* o_npts,
                    int64_t* o_tstart, int64_t* o_tend,
                    double* o_dist, double* o_sumspd, float* o_maxspd,
                    double* o_maxdspd, uint32_t* o_ndtz,
                    double* o_latmin, double* o_latmax, double* o_lonmin, double* o_lonmax)
{
    int64_t J = 0;
    int64_t k = 0;
    xsum_t sd, ss;
    while (k < n) {
        int64_t e = k + 1;
        while (e < n && jid[e] == jid[k]) ++e;
        if (J < cap) {
            xsum_init(&sd);
            xsum_init(&ss);
            float maxs = 0.0f;
            int have_s = 0;
            double maxd = 0.0;
            uint32_t ndz = 0;
            double la0 = INFINITY, la1 = -INFINITY, lo0 = INFINITY, lo1 = -INFINITY;
            for (int64_t i = k; i < e; ++i) {
                xsum_add(&sd, step_m[i]);
                xsum_add(&ss, (double)speed[i]);
                float s = canon0(speed[i]);
                if (!have_s || s > maxs) { maxs = s; have_s = 1; }
                if ((flags[i] & F_SPEED_OK) && dspeed[i] > maxd) maxd = dspeed[i];
                if (flags[i] & F_DT_ZERO) ++ndz;
                if (isfinite(lat[i]) && isfinite(lon[i])) {
                    double a = lat[i] + 0.0, o = lon[i] + 0.0;      /* -0.0 as +0.0 */
                    if (a < la0) la0 = a;
                    if (a > la1) la1 = a;
                    if (o < lo0) lo0 = o;
                    if (o > lo1) lo1 = o;
                }
            }
            o_jid[J] = jid[k];
            o_first[J] = (uint32_t)k;
            o_npts[J] = (uint32_t)(e - k);
            o_tstart[J] = ts[k];
            o_tend[J] = ts[e - 1];
            o_dist[J] = xsum_round(&sd);
            o_sumspd[J] = xsum_round(&ss);
            o_maxspd[J] = maxs;
            o_maxdspd[J] = maxd;
            o_ndtz[J] = ndz;
            o_latmin[J] = la0;
            o_latmax[J] = la1;
            o_lonmin[J] = lo0;
            o_lonmax[J] = lo1;
        }
        ++J;
        k = e;
    }
    return J;
}

/* ------------------------------------------------------------------------ */
/* Spatio-temporal grid aggregate.                                            */
/*                                                                           */
/* Algorithm 2: lat_bin = (lat - lat_min) // lat_step, likewise for           */
/* longitude, and the time bin from minutes // step.  Read here as            */
/* floor(fl(fl(x - x0) / step)) in IEEE double for the spatial bins and as    */
/* integer floor division of (ts - t0) by bin_ms for the time bin.  Methods   */
/* step (4): one unrolled global index per record, read as the time-major     */
/* key (tbin * n_lat + ilat) * n_lon + ilon.  Step (5): each lattice cell     */
/* holds the records with that index; Table 3's reductions give count, sum,   */
/* count-unique and the mean (= sum / count).  Per key: count, number of      */
/* distinct journey ids, exact-rounded sum of speed, min and max speed        */
/* (-0.0 as +0.0).  A record is in the grid iff both coordinates are finite,  */
/* 0 <= ilat < n_lat, 0 <= ilon < n_lon, tbin >= 0 and (n_t > 0 ? tbin < n_t  */
/* : the key fits in a signed 64-bit integer).  Rows come out in ascending   */
/* key.  Returns the number of groups G; rows beyond `cap` are not written.  */
/* ------------------------------------------------------------------------ */
static const int64_t* g_key;

static int cmp_key_jid_idx(const void* a, const void* b)
{
    uint32_t i = *(const uint32_t*)a, j = *(const uint32_t*)b;
    if (g_key[i] != g_key[j]) return g_key[i] < g_key[j] ? -1 : 1;
    if (g_jid[i] != g_jid[j]) return g_jid[i] < g_jid[j] ? -1 : 1;
    return (i > j) - (i < j);
}

static int64_t floor_div64(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

int64_t orc_grid_keys(int64_t n, const int64_t* ts, const double* lat, const double* lon,
                      double lat0, double lon0, double dlat, double dlon,
                      int64_t n_lat, int64_t n_lon, int64_t t0, int64_t bin_ms, int64_t n_t,
                      int64_t* key)
{
    int64_t n_out = 0;
    int64_t cells = n_lat * n_lon;
    int64_t tmax = (n_t > 0) ? n_t : (INT64_MAX / cells);
    for (int64_t i = 0; i < n; ++i) {
        key[i] = -1;
        if (!isfinite(lat[i]) || !isfinite(lon[i])) { ++n_out; continue; }
        double fy = floor((lat[i] - lat0) / dlat);
        double fx = floor((lon[i] - lon0) / dlon);
        int64_t tb = floor_div64(ts[i] - t0, bin_ms);
        if (!(fy >= 0.0 && fy < (double)n_lat && fx >= 0.0 && fx < (double)n_lon &&
              tb >= 0 && tb < tmax)) {
            ++n_out;
            continue;
        }
        key[i] = (tb * n_lat + (int64_t)fy) * n_lon + (int64_t)fx;
    }
    return n_out;
}

/* Groups of equal key among records with key >= 0: count, distinct journeys
 * (records sorted by (key, journey, index); a journey counts once per key),
 * exact speed sum rounded once, min and max speed; rows in ascending key.
 * Rows past cap are counted, not written.  key[] is freed here. */
static int64_t group_by_key(int64_t n, const int64_t* jid, const float* speed, int64_t* key, int64_t cap,
                            int64_t* o_key, uint32_t* o_count, uint32_t* o_nj, double* o_sum,
                            float* o_min, float* o_max)
{
    uint32_t* idx = (uint32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    if (!idx) abort();
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (key[i] >= 0) idx[m++] = (uint32_t)i;
    g_key = key;
    g_jid = jid;
    qsort(idx, (size_t)m, sizeof(uint32_t), cmp_key_jid_idx);
    int64_t G = 0;
    xsum_t s;
    for (int64_t a = 0; a < m;) {
        int64_t b = a + 1;
        while (b < m && key[idx[b]] == key[idx[a]]) ++b;
        if (G < cap) {
            uint32_t nj = 0;
            float mn = canon0(speed[idx[a]]), mx = mn;
            xsum_init(&s);
            for (int64_t c = a; c < b; ++c) {
                uint32_t i = idx[c];
                if (c == a || jid[i] != jid[idx[c - 1]]) ++nj;
                float v = canon0(speed[i]);
                if (v < mn) mn = v;
                if (v > mx) mx = v;
                xsum_add(&s, (double)speed[i]);
            }
            o_key[G] = key[idx[a]];
            o_count[G] = (uint32_t)(b - a);
            o_nj[G] = nj;
            o_sum[G] = xsum_round(&s);
            o_min[G] = mn;
            o_max[G] = mx;
        }
        ++G;
        a = b;
    }
    free(key);
    free(idx);
    return G;
}

int64_t orc_grid(int64_t n, const int64_t* jid, const int64_t* ts,
                 const double* lat, const double* lon, const float* speed,
                 double lat0, double lon0, double dlat, double dlon,
                 int64_t n_lat, int64_t n_lon, int64_t t0, int64_t bin_ms, int64_t n_t,
                 int64_t cap,
                 int64_t* o_key, uint32_t* o_count, uint32_t* o_nj, double* o_sum,
                 float* o_min, float* o_max, int64_t* o_nout)
{
    int64_t* key = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!key) abort();
    *o_nout = orc_grid_keys(n, ts, lat, lon, lat0, lon0, dlat, dlon, n_lat, n_lon, t0, bin_ms,
                            n_t, key);
    return group_by_key(n, jid, speed, key, cap, o_key, o_count, o_nj, o_sum, o_min, o_max);
}

/* Direction sector (Algorithm 2: the heading binned by floor division with a
 * sector width; the transformed-data output: speeds and volumes per cardinal
 * direction).  Reading: nd sectors of width 360/nd degrees, sector =
 * floor((h + off) / (360/nd)) mod nd for a heading h in [0, 360); off = 0 is
 * the literal floor division, off = 45 with nd = 4 centres N, E, S, W.  A
 * record without a direction (h outside [0, 360) or NaN; a derived bearing
 * that is not defined) falls in the extra sector nd, so that counts over all
 * sectors still sum to the records in the grid. */
int64_t orc_dir_sector(double h, int32_t ok, int64_t nd, double off)
{
    if (!ok || !(h >= 0.0 && h < 360.0)) return nd;
    double step = 360.0 / (double)nd;
    int64_t q = (int64_t)floor((h + off) / step);
    return q % nd;
}

/* The lattice with a direction dimension: key =
 * ((tbin * (nd + 1) + sector) * n_lat + ilat) * n_lon + ilon for records in
 * the grid (the same bins as orc_grid_keys).  The heading of record i is
 * heading[i] when heading is given, else bearing[i] when flags[i] has
 * F_BEARING_OK. */
int64_t orc_grid_dir(int64_t n, const int64_t* jid, const int64_t* ts,
                     const double* lat, const double* lon, const float* speed,
                     const float* heading, const double* bearing, const uint8_t* flags,
                     int64_t nd, double off,
                     double lat0, double lon0, double dlat, double dlon,
                     int64_t n_lat, int64_t n_lon, int64_t t0, int64_t bin_ms, int64_t n_t,
                     int64_t cap,
                     int64_t* o_key, uint32_t* o_count, uint32_t* o_nj, double* o_sum,
                     float* o_min, float* o_max, int64_t* o_nout)
{
    int64_t* key = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!key) abort();
    int64_t cells = n_lat * n_lon;
    int64_t tmax = (n_t > 0) ? n_t : (INT64_MAX / (cells * (nd + 1)));
    int64_t n_out = 0;
    for (int64_t i = 0; i < n; ++i) {
        key[i] = -1;
        if (!isfinite(lat[i]) || !isfinite(lon[i])) { ++n_out; continue; }
        double fy = floor((lat[i] - lat0) / dlat);
        double fx = floor((lon[i] - lon0) / dlon);
        int64_t tb = floor_div64(ts[i] - t0, bin_ms);
        if (!(fy >= 0.0 && fy < (double)n_lat && fx >= 0.0 && fx < (double)n_lon &&
              tb >= 0 && tb < tmax)) {
            ++n_out;
            continue;
        }
        int64_t sec = heading ? orc_dir_sector((double)heading[i], 1, nd, off)
                              : orc_dir_sector(bearing[i], (flags[i] & F_BEARING_OK) != 0, nd, off);
        key[i] = ((tb * (nd + 1) + sec) * n_lat + (int64_t)fy) * n_lon + (int64_t)fx;
    }
    *o_nout = n_out;
    return group_by_key(n, jid, speed, key, cap, o_key, o_count, o_nj, o_sum, o_min, o_max);
}
