// cv_stream.hip -- serving form of the ETL path: records arrive in chunks;
// the open journeys and the group table stay resident on the device.
//
// The result of any sequence of pushes equals the plain path applied to the
// concatenation of all pushed records in arrival order (ties in arrival
// order), provided every journey's timestamps do not go backwards across
// pushes.  A record older than its journey's last pushed record is "late": it
// gets the LATE flag and no kinematics, counts in its journey's totals and in
// the grid (never as a new distinct journey), and leaves the journey's state
// alone.
//
// One push over a batch of n records:
//   1. stable sort of the batch by (journey, time) (the record sort);
//   2. journey starts of the sorted batch -> batch journeys [boff[j], boff[j+1]);
//   3. each batch journey finds or claims its resident row (hash on the id);
//   4. kinematics per record; a journey's first record in the batch takes the
//      row's last point as its predecessor; written in the batch's input order;
//   5. one thread per batch journey folds its records into the row's running
//      summary (exact fixed point) and the resident group table, deciding the
//      distinct-journey flag from the cells seen in the journey's open
//      (journey, time-bin) segment, which the row carries across pushes: the
//      first KCELLS cells in the row, further ones in the row's own overflow
//      table (a page of a device-wide pool, taken the first time one of the
//      row's segments needs it and cleared when the next segment starts).
// Flush: journey rows in ascending id and the group table in ascending key.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "cv_device.h"
#include "cv_gridagg.h"
#include "cv_gridtab.h"
#include "cv_host.h"
#include "cv_radix.h"
#include "cv_sumtab.h"

using namespace cv;

namespace cv {
cv_status sort_records_into(const cv_records* in, uint64_t max_journeys, uint32_t* perm, const cv_records_out* sorted,
                            cv_result* res, void* ws, size_t ws_bytes, hipStream_t stream);
}

namespace {

constexpr int KCELLS = 16;  // distinct cells remembered in a journey's row for its open segment
constexpr u32 OVF_NONE = 0xFFFFFFFFu;   // the row has no overflow table yet
constexpr u32 OVF_FAIL = 0xFFFFFFFEu;   // the pool ran out for this row
constexpr int OVF_SLOTS = 512;          // open-addressing slots of one overflow table
constexpr u32 OVF_MAX = 384;            // cells one segment may keep there (75 % load)
constexpr u64 OVF_EMPTY = ~0ull;        // group keys are non-negative

constexpr u64 JEMPTY = 0x8000000000000000ull;
constexpr u32 FLAG_LATE = 0x80u;
constexpr u32 FLAG_PRED_CARRIED = 0x100u;  // internal: predecessor is the row's last point
constexpr int FX_DIST = 128;
constexpr int ST_TILE = 4096;
constexpr double EARTH_R_M = 6371008.8;
constexpr double DEG2RAD = 3.14159265358979323846 / 180.0;
constexpr double RAD2DEG = 180.0 / 3.14159265358979323846;

struct JRow {
    i64 last_ts;
    double last_lat, last_lon, last_v, last_b;
    u32 last_flags, has_last;
    u64 dist[3], spd[3];
    u64 maxd, latmin, latmax, lonmin, lonmax;
    u64 tmin_ord, tmax_ord;
    u32 count, ndtz, maxs, ncell;
    i64 seg_tbin;
    u64 cell[KCELLS];
    u32 ovf, novf;  // overflow table (page index) and the cells it holds for the open segment
};

struct StreamMeta {
    u32 Jb;             // journeys in the current batch
    u32 jt_full;        // journey table full (sticky)
    u32 cell_overflow;  // a segment outgrew its overflow table or the pool ran out:
                        // distinct-journey counts may be high (sticky)
    u32 ovf_next;       // overflow tables taken from the pool
    u32 ap_n;           // cells appended this push (records that counted their journey in a cell)
    u32 pad3;
    u64 batch_late, batch_out;
    u64 total_records, total_late, total_out;
    u32 jcount;         // flush: occupied journey rows
    u32 min_used;       // the reserved row of journey id INT64_MIN is taken
    GridMeta gm;        // group table bookkeeping (overflow, compaction, key bits)
    u32 jtickets[MAX_PASSES];
};

// Journey table: open addressing on the id, JEMPTY marking a free slot.  The
// one id equal to JEMPTY (INT64_MIN) cannot live in a slot; it has the
// reserved row mask + 1, taken through the min_used flag.
__device__ __forceinline__ u64 jt_find_or_insert(u64* keys, u64 mask, u64 key, bool& inserted, u32* min_used)
{
    inserted = false;
    if (key == JEMPTY) {
        inserted = atomicCAS(min_used, 0u, 1u) == 0u;
        return mask + 1;
    }
    u64 h = mix64(key) & mask;
    for (u64 probe = 0; probe <= mask && probe < G_PROBES; ++probe) {
        u64 cur = keys[h];
        if (cur == key) return h;
        if (cur == JEMPTY) {
            u64 prev = atomicCAS((unsigned long long*)&keys[h], (unsigned long long)JEMPTY, (unsigned long long)key);
            if (prev == JEMPTY) {
                inserted = true;
                return h;
            }
            if (prev == key) return h;
        }
        h = (h + 1) & mask;
    }
    return ~0ull;
}

__global__ void k_st_init_meta(StreamMeta* m)
{
    if (threadIdx.x == 0) {
        StreamMeta z = {};
        *m = z;
    }
}

__global__ void k_st_begin(StreamMeta* m)
{
    if (threadIdx.x == 0) {
        m->batch_late = 0;
        m->batch_out = m->gm.n_out;  // the count before this batch
        m->ap_n = 0;
        m->Jb = 0;
    }
}

// journey starts per tile of the sorted batch
__global__ void __launch_bounds__(256) k_st_count(const i64* __restrict__ jid, u32 n, u32* __restrict__ cnt)
{
    __shared__ u32 tmp[4];
    const u64 base = (u64)blockIdx.x * ST_TILE;
    u32 c = 0;
    for (int i = threadIdx.x; i < ST_TILE; i += 256) {
        const u64 r = base + i;
        if (r < n && (r == 0 || jid[r] != jid[r - 1])) ++c;
    }
    u32 tot;
    block_exclusive_sum<256>(c, tmp, tot);
    if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_st_scan(u32* __restrict__ cnt, u32 tiles, StreamMeta* m)
{
    __shared__ u32 tmp[4];
    __shared__ u32 carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (u32 b = 0; b < tiles; b += 256) {
        const u32 i = b + threadIdx.x;
        const u32 v = i < tiles ? cnt[i] : 0u;
        u32 tot;
        const u32 e = block_exclusive_sum<256>(v, tmp, tot);
        if (i < tiles) cnt[i] = carry + e;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) m->Jb = carry;
}

// boff[j] = sorted position of batch journey j's first record; boff[Jb] = n
__global__ void __launch_bounds__(256) k_st_heads(const i64* __restrict__ jid, u32 n, const u32* __restrict__ prefix,
                                                  const StreamMeta* m, u32* __restrict__ boff)
{
    __shared__ u32 tmp[4];
    const u64 base = (u64)blockIdx.x * ST_TILE;
    // each thread takes ST_TILE/256 consecutive records so positions stay ordered
    constexpr int PER = ST_TILE / 256;
    const u64 r0 = base + (u64)threadIdx.x * PER;
    u32 c = 0;
    for (int i = 0; i < PER; ++i) {
        const u64 r = r0 + i;
        if (r < n && (r == 0 || jid[r] != jid[r - 1])) ++c;
    }
    u32 tot;
    u32 e = block_exclusive_sum<256>(c, tmp, tot) + prefix[blockIdx.x];
    for (int i = 0; i < PER; ++i) {
        const u64 r = r0 + i;
        if (r < n && (r == 0 || jid[r] != jid[r - 1])) boff[e++] = (u32)r;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) boff[m->Jb] = n;
}

__global__ void __launch_bounds__(256) k_st_journeys(const i64* __restrict__ jid, const u32* __restrict__ boff,
                                                     StreamMeta* m, u64* __restrict__ jkeys, u64 jmask,
                                                     JRow* __restrict__ rows, u32* __restrict__ bslot)
{
    const u32 Jb = m->Jb;
    for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < Jb; j += gridDim.x * blockDim.x) {
        const u64 key = (u64)jid[boff[j]];
        bool ins;
        const u64 s = jt_find_or_insert(jkeys, jmask, key, ins, &m->min_used);
        if (s == ~0ull) {
            atomicOr(&m->jt_full, 1u);
            bslot[j] = ~0u;
            continue;
        }
        bslot[j] = (u32)s;
        if (ins) {
            JRow r = {};
            r.has_last = 0;
            r.maxd = ord_f64(0.0);
            r.latmin = ord_f64(__builtin_inf());
            r.latmax = ord_f64(-__builtin_inf());
            r.lonmin = ord_f64(__builtin_inf());
            r.lonmax = ord_f64(-__builtin_inf());
            r.tmin_ord = ~0ull;
            r.tmax_ord = 0;
            r.seg_tbin = INT64_MIN;
            r.ovf = OVF_NONE;
            rows[s] = r;
        }
    }
}

__device__ __forceinline__ u32 batch_journey_of(const u32* __restrict__ boff, u32 Jb, u32 k)
{
    u32 lo = 0, hi = Jb;  // boff[lo] <= k < boff[hi]
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (boff[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Kinematics of the sorted batch.  Same stencil as the plain kernel, with the
// resident last point standing in for the predecessor of a journey's first
// record in the batch; outputs land at the records' input positions.
constexpr int FB = 256;

__global__ void __launch_bounds__(FB) k_st_features(u32 n, const i64* __restrict__ jid, const i64* __restrict__ ts,
                                                    const double* __restrict__ lat, const double* __restrict__ lon,
                                                    const u32* __restrict__ perm, const u32* __restrict__ boff,
                                                    const StreamMeta* m, const u32* __restrict__ bslot,
                                                    const JRow* __restrict__ rows, cv_features o,
                                                    double* __restrict__ fs_step, double* __restrict__ fs_v,
                                                    double* __restrict__ fs_b, uint8_t* __restrict__ fs_flags)
{
    __shared__ i64 s_jid[FB + 2], s_ts[FB + 2];
    __shared__ double s_lat[FB + 2], s_lon[FB + 2], s_sphi[FB + 2], s_cphi[FB + 2];
    __shared__ u32 s_fin[FB + 2];
    __shared__ double s_step[FB + 1], s_dt[FB + 1], s_v[FB + 1], s_b[FB + 1], s_pv[FB + 1], s_pb[FB + 1];
    __shared__ u32 s_f[FB + 1], s_pf[FB + 1];
    __shared__ u32 s_jb[FB + 2], s_scan[FB / WAVE], s_jb0;
    const u32 Jb = m->Jb;
    const long s0 = (long)blockIdx.x * FB;
    for (int q = threadIdx.x; q < FB + 2; q += FB) {
        const long r = s0 - 2 + q;
        if (r >= 0 && r < (long)n) {
            const double la = lat[r], lo = lon[r];
            s_jid[q] = jid[r];
            s_ts[q] = ts[r];
            s_lat[q] = la;
            s_lon[q] = lo;
            const bool fin = isfinite(la) && isfinite(lo);
            s_fin[q] = fin;
            const double phi = la * DEG2RAD;
            s_sphi[q] = fin ? sin(phi) : 0.0;
            s_cphi[q] = fin ? cos(phi) : 0.0;
        }
    }
    // Batch journey of every record: one search for the block's first record
    // (LDS position qb), then a block scan of journey starts after it.
    const int qb = s0 == 0 ? 2 : 1;
    if (threadIdx.x == 0) s_jb0 = batch_journey_of(boff, Jb, (u32)(s0 - 2 + qb));
    __syncthreads();
    {
        const int q = threadIdx.x + 1;
        const long r = s0 - 2 + q;
        const u32 h = (q > qb && r < (long)n && s_jid[q] != s_jid[q - 1]) ? 1u : 0u;
        u32 tot;
        const u32 ex = block_exclusive_sum<FB>(h, s_scan, tot);
        s_jb[q] = s_jb0 + ex + h;
        if (threadIdx.x == 0) {
            const long rl = s0 + FB - 1;  // LDS position FB + 1
            s_jb[FB + 1] = s_jb0 + tot + ((rl < (long)n && s_jid[FB + 1] != s_jid[FB]) ? 1u : 0u);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < FB + 1; j += FB) {
        const long k = s0 - 1 + j;
        double step = 0.0, dts = 0.0, v = 0.0, b = 0.0, pv = 0.0, pb = 0.0;
        u32 f = 0, pf = 0;
        if (k >= 0 && k < (long)n) {
            const int qk = j + 1, qp = j;
            const u32 jb = s_jb[qk];
            const u32 slot = bslot[jb];
            const bool have_row = slot != ~0u;
            const JRow* row = have_row ? &rows[slot] : nullptr;
            const bool has_last = have_row && row->has_last;
            const i64 lts = has_last ? row->last_ts : 0;
            const bool late = has_last && s_ts[qk] < lts;
            const bool head_b = (u32)k == boff[jb];
            // predecessor: the batch record before (same journey, not late), else the resident last point
            int pred = 0;  // 0 none, 1 record k-1, 2 resident point
            if (!late) {
                if (!head_b && !(has_last && s_ts[qp] < lts)) pred = 1;
                else if (has_last) pred = 2;
            }
            if (late) {
                f = FLAG_LATE;
            } else if (pred == 0) {
                f = CV_FLAG_FIRST | (s_fin[qk] ? 0u : CV_FLAG_BAD_COORD);
            } else {
                const i64 pts = pred == 1 ? s_ts[qp] : lts;
                const double plat = pred == 1 ? s_lat[qp] : row->last_lat;
                const double plon = pred == 1 ? s_lon[qp] : row->last_lon;
                const bool pfin = pred == 1 ? (s_fin[qp] != 0) : (isfinite(plat) && isfinite(plon));
                const i64 dt_ms = s_ts[qk] - pts;
                f = dt_ms == 0 ? CV_FLAG_DT_ZERO : 0u;
                if (pred == 2) {
                    f |= FLAG_PRED_CARRIED;
                    pv = row->last_v;
                    pb = row->last_b;
                    pf = row->last_flags;
                }
                if (!s_fin[qk] || !pfin) {
                    f |= CV_FLAG_BAD_COORD;
                } else {
                    dts = (double)dt_ms / 1000.0;
                    const double dphi = (s_lat[qk] - plat) * DEG2RAD;
                    const double dlam = (s_lon[qk] - plon) * DEG2RAD;
                    // half-angle sines and cosines; the full-angle sines of the
                    // bearing follow from them (sin 2u = 2 sin u cos u)
                    double sp, cp, sl, cl;
                    sincos(0.5 * dphi, &sp, &cp);
                    sincos(0.5 * dlam, &sl, &cl);
                    const double phi1 = plat * DEG2RAD;
                    const double cphi1 = pred == 1 ? s_cphi[qp] : cos(phi1);
                    const double sphi1 = pred == 1 ? s_sphi[qp] : sin(phi1);
                    const double cphi2 = s_cphi[qk];
                    const double a = (sp * sp) + ((cphi1 * cphi2) * (sl * sl));
                    step = (2.0 * EARTH_R_M) * asin(fmin(1.0, sqrt(a)));
                    if (dt_ms > 0) {
                        v = step / dts;
                        f |= CV_FLAG_SPEED_OK;
                    }
                    if (step > 0.0) {
                        const double y = ((2.0 * sl) * cl) * cphi2;
                        const double x = ((2.0 * sp) * cp) + (((2.0 * sphi1) * cphi2) * (sl * sl));
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
        s_pv[j] = pv;
        s_pb[j] = pb;
        s_pf[j] = pf;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const long k = s0 + t;
    if (k >= (long)n) return;
    const int j = t + 1;
    u32 f = s_f[j];
    const bool carried = (f & FLAG_PRED_CARRIED) != 0;
    f &= ~FLAG_PRED_CARRIED;
    const u32 fp = carried ? s_pf[j] : s_f[j - 1];
    const double vp = carried ? s_pv[j] : s_v[j - 1];
    const double bp = carried ? s_pb[j] : s_b[j - 1];
    const double v = s_v[j], b = s_b[j], dts = s_dt[j];
    double acc = 0.0, dh = 0.0;
    if (!(f & (FLAG_LATE | CV_FLAG_FIRST))) {
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
    const u32 dst = perm[k];
    o.step_m[dst] = s_step[j];
    o.dt_s[dst] = dts;
    o.speed_mps[dst] = v;
    o.accel_mps2[dst] = acc;
    o.bearing_deg[dst] = b;
    o.dheading_deg[dst] = dh;
    o.flags[dst] = (uint8_t)f;
    fs_step[k] = s_step[j];
    fs_v[k] = v;
    fs_b[k] = b;
    fs_flags[k] = (uint8_t)f;
}

// a cell that counted its journey in this push: the row and the group key
struct Append {
    u64 key;
    u32 slot, pad;
};

// Membership of a cell in a row's overflow table (read side).
__device__ __forceinline__ bool ovf_contains(const u64* tab, u64 key)
{
    u32 h = (u32)mix64(key) & (OVF_SLOTS - 1);
    for (int probe = 0; probe < OVF_SLOTS; ++probe) {
        const u64 cur = tab[h];
        if (cur == key) return true;
        if (cur == OVF_EMPTY) return false;
        h = (h + 1) & (OVF_SLOTS - 1);
    }
    return false;
}

// Grid tile kernel policy of the serving form.  Late records count in their
// cells but never as a new distinct journey; a journey's first segment in the
// batch that continues the row's open segment (same time bin) also checks the
// cells the row carried over; every record that counts its journey in a cell
// is appended for the row update that follows the tile kernel.
struct GridStream {
    static constexpr bool kStream = true;
    static constexpr int kDir = 0;
    const i64* jid;          // sorted batch
    const uint8_t* flags;    // sorted batch features' flags
    const u32* boff;         // batch journey starts
    const StreamMeta* m;     // Jb
    const u32* bslot;        // resident row of each batch journey
    const JRow* rows;
    const u64* ovf_pool;
    i64 cells;               // n_lat * n_lon: a key's time bin is key / cells
    Append* ap;
    u32 apcap;
    u32* ap_n;

    __device__ bool late(u64 r) const { return (flags[r] & FLAG_LATE) != 0; }
    __device__ u32 slot_of(u64 r) const { return bslot[batch_journey_of(boff, m->Jb, (u32)r)]; }
    // r0: first record of a segment of non-late records; key: a cell of it
    __device__ bool carried(u64 r0, u64 key) const
    {
        if (r0 > 0 && jid[r0 - 1] == jid[r0] && !late(r0 - 1)) return false;  // begins inside the batch
        const u32 slot = slot_of(r0);
        if (slot == ~0u) return false;
        const JRow& R = rows[slot];
        if (R.seg_tbin != (i64)(key / (u64)cells)) return false;
        const u32 nc = R.ncell < (u32)KCELLS ? R.ncell : (u32)KCELLS;
        for (u32 c = 0; c < nc; ++c)
            if (R.cell[c] == key) return true;
        if (R.novf && R.ovf < OVF_FAIL) return ovf_contains(ovf_pool + (u64)R.ovf * OVF_SLOTS, key);
        return false;
    }
    __device__ void first(u64 r, u64 key) const
    {
        const u32 slot = slot_of(r);
        if (slot == ~0u) return;
        const u32 i = atomicAdd(ap_n, 1u);
        if (i < apcap) {
            ap[i].key = key;
            ap[i].slot = slot;
        }
    }
};

// One thread per batch journey: the batch's exact partial (JAcc / AccX row j)
// joins the resident row; the last non-late record becomes the row's last
// point; when the batch's last non-late record opens a new (journey, time-bin)
// segment, the row's cell set starts empty for it.
__global__ void __launch_bounds__(256) k_st_merge(const i64* __restrict__ ts, const double* __restrict__ lat,
                                                  const double* __restrict__ lon, const u32* __restrict__ boff,
                                                  StreamMeta* m, const u32* __restrict__ bslot,
                                                  JRow* __restrict__ rows, const JAcc* __restrict__ acc,
                                                  const AccX* __restrict__ accx, u32 arows,
                                                  const double* __restrict__ fs_v,
                                                  const double* __restrict__ fs_b,
                                                  const uint8_t* __restrict__ fs_flags, Spec g,
                                                  u64* __restrict__ ovf_pool)
{
    __shared__ u64 s_late[256 / WAVE];
    const u32 Jb = m->Jb;
    u64 late_n = 0;
    for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < Jb; j += gridDim.x * blockDim.x) {
        const u32 slot = bslot[j];
        if (slot == ~0u || j >= arows) continue;
        JRow& R = rows[slot];
        const u32 a = boff[j], e = boff[j + 1];
        const JAcc& A = acc[j];
        const AccX& X = accx[j];
        Fx192 d, sp, t;
        for (int i = 0; i < 3; ++i) {
            d.w[i] = R.dist[i];
            sp.w[i] = R.spd[i];
        }
        for (int i = 0; i < 3; ++i) t.w[i] = A.dist[i];
        fx_add(d, t);
        for (int i = 0; i < 3; ++i) t.w[i] = X.dist[i];
        fx_add(d, t);
        for (int i = 0; i < 3; ++i) t.w[i] = A.spd[i];
        fx_add(sp, t);
        for (int i = 0; i < 3; ++i) t.w[i] = X.spd[i];
        fx_add(sp, t);
        for (int i = 0; i < 3; ++i) {
            R.dist[i] = d.w[i];
            R.spd[i] = sp.w[i];
        }
        R.count += A.count;
        R.ndtz += A.ndtz;
        R.maxs = A.maxs > R.maxs ? A.maxs : R.maxs;
        R.maxd = A.maxd > R.maxd ? A.maxd : R.maxd;
        R.latmin = A.latmin < R.latmin ? A.latmin : R.latmin;
        R.latmax = A.latmax > R.latmax ? A.latmax : R.latmax;
        R.lonmin = A.lonmin < R.lonmin ? A.lonmin : R.lonmin;
        R.lonmax = A.lonmax > R.lonmax ? A.lonmax : R.lonmax;
        // the batch is in (journey, time) order: its time span is at both ends
        const u64 t0 = ord_i64(ts[a]), t1 = ord_i64(ts[e - 1]);
        R.tmin_ord = t0 < R.tmin_ord ? t0 : R.tmin_ord;
        R.tmax_ord = t1 > R.tmax_ord ? t1 : R.tmax_ord;
        // late records come first (older than the row's last point)
        u32 k = a;
        while (k < e && (fs_flags[k] & FLAG_LATE)) ++k;
        late_n += k - a;
        if (k < e) {
            const u32 lg = e - 1;  // the last record is the last non-late one
            R.last_ts = ts[lg];
            R.last_lat = lat[lg];
            R.last_lon = lon[lg];
            R.last_v = fs_v[lg];
            R.last_b = fs_b[lg];
            R.last_flags = fs_flags[lg];
            R.has_last = 1;
            const i64 tb = time_bin(g, ts[lg]);
            if (tb != R.seg_tbin) {
                R.seg_tbin = tb;
                R.ncell = 0;
                if (R.novf && R.ovf < OVF_FAIL) {
                    u64* pg = ovf_pool + (u64)R.ovf * OVF_SLOTS;
                    for (int c = 0; c < OVF_SLOTS; ++c) pg[c] = OVF_EMPTY;
                }
                R.novf = 0;
            }
        }
    }
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) late_n += __shfl_xor(late_n, dd, WAVE);
    if (lane_id() == 0) s_late[threadIdx.x / WAVE] = late_n;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 tl = 0;
        for (int w = 0; w < 256 / WAVE; ++w) tl += s_late[w];
        if (tl) atomicAdd((unsigned long long*)&m->batch_late, (unsigned long long)tl);
    }
}

// One thread per appended cell: cells of a row's open segment (after the
// merge) join the row's set, in the row while it has room.  Each cell takes a
// position in the set with one atomic; the cell at position KCELLS (one per
// row, ever at most one per push) takes the row's overflow table from the
// pool when the row has none, so a row holds at most one table.  Cells of
// earlier segments of the batch are dropped.  ap[i].pad keeps the position
// (or ~0u) for k_st_append_ovf.
__global__ void __launch_bounds__(256) k_st_append(Append* __restrict__ ap, StreamMeta* m, u32 apcap,
                                                   JRow* __restrict__ rows, u32 ovf_pages, i64 cells)
{
    const u32 na = m->ap_n < apcap ? m->ap_n : apcap;
    if (blockIdx.x == 0 && threadIdx.x == 0 && m->ap_n > apcap) atomicOr(&m->cell_overflow, 1u);
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += gridDim.x * blockDim.x) {
        const u64 key = ap[i].key;
        JRow& R = rows[ap[i].slot];
        u32 c = ~0u;
        if ((i64)(key / (u64)cells) == R.seg_tbin) {
            c = atomicAdd(&R.ncell, 1u);
            if (c < (u32)KCELLS) {
                R.cell[c] = key;
            } else if (c == (u32)KCELLS && R.ovf == OVF_NONE) {
                const u32 pg = atomicAdd(&m->ovf_next, 1u);
                R.ovf = pg < ovf_pages ? pg : OVF_FAIL;
            }
        }
        ap[i].pad = c;
    }
}

// One thread per appended cell past the row's KCELLS: the cell joins the
// row's overflow table (open addressing, bounded load).  A full table, or a
// row the pool had no table for, sets the sticky overflow flag.
__global__ void __launch_bounds__(256) k_st_append_ovf(const Append* __restrict__ ap, StreamMeta* m, u32 apcap,
                                                       JRow* __restrict__ rows, u64* __restrict__ ovf_pool)
{
    const u32 na = m->ap_n < apcap ? m->ap_n : apcap;
    bool full = false;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += gridDim.x * blockDim.x) {
        const u32 c = ap[i].pad;
        if (c == ~0u || c < (u32)KCELLS) continue;
        JRow& R = rows[ap[i].slot];
        const u32 pg = R.ovf;
        if (pg >= OVF_FAIL || atomicAdd(&R.novf, 1u) >= OVF_MAX) {
            full = true;
            continue;
        }
        const u64 key = ap[i].key;
        u64* tab = ovf_pool + (u64)pg * OVF_SLOTS;
        u32 h = (u32)mix64(key) & (OVF_SLOTS - 1);
        bool placed = false;
        for (int probe = 0; probe < OVF_SLOTS && !placed; ++probe) {
            const u64 prev = atomicCAS((unsigned long long*)&tab[h], (unsigned long long)OVF_EMPTY,
                                       (unsigned long long)key);
            placed = prev == OVF_EMPTY || prev == key;
            h = (h + 1) & (OVF_SLOTS - 1);
        }
        if (!placed) full = true;
    }
    if (full) atomicOr(&m->cell_overflow, 1u);
}

__global__ void k_st_finish(StreamMeta* m, const cv_result* sres, u32 n, cv_result* res)
{
    if (threadIdx.x != 0) return;
    m->batch_out = m->gm.n_out - m->batch_out;
    m->total_records += n;
    m->total_late += m->batch_late;
    m->total_out += m->batch_out;
    if (!res) return;
    cv_result r = {};
    u32 st = CV_OK;
    if (sres->status != CV_OK) st = sres->status;
    else if (m->jt_full || m->gm.overflow) st = CV_ERR_CAPACITY;
    r.status = st;
    r.flags = m->cell_overflow ? 1u : 0u;
    r.count = m->Jb;
    r.n_late = m->batch_late;
    r.n_out_of_grid = m->batch_out;
    r.key_bits = sres->key_bits;
    *res = r;
}

// ---- flush: journey rows in ascending id ----
__global__ void __launch_bounds__(256) k_st_jcompact(const u64* __restrict__ jkeys, u64 slots, StreamMeta* m,
                                                     u64* __restrict__ ck, u32* __restrict__ cv)
{
    for (u64 b = (u64)blockIdx.x * blockDim.x; b < slots; b += (u64)gridDim.x * blockDim.x) {
        const u64 s = b + threadIdx.x;
        const u64 k = s < slots ? jkeys[s] : JEMPTY;
        const bool occ = k != JEMPTY;
        const u64 msk = __ballot(occ);
        u32 base = 0;
        if (lane_id() == 0 && msk) base = atomicAdd(&m->jcount, (u32)__popcll(msk));
        base = __shfl(base, 0, WAVE);
        if (occ) {
            const u32 pos = base + popc_below(msk);
            ck[pos] = k ^ 0x8000000000000000ull;  // signed order
            cv[pos] = (u32)s;
        }
    }
    // the reserved row of journey id INT64_MIN (its key reads INT64_MIN: jkeys[slots] stays JEMPTY)
    if (blockIdx.x == 0 && threadIdx.x == 0 && m->min_used) {
        const u32 pos = atomicAdd(&m->jcount, 1u);
        ck[pos] = 0;
        cv[pos] = (u32)slots;
    }
}

// first = exclusive prefix of n_points in id order (one block)
__global__ void __launch_bounds__(256) k_st_jfirst(const JRow* __restrict__ rows, const u32* __restrict__ order,
                                                   const StreamMeta* m, u32* __restrict__ first, u32 cap)
{
    __shared__ u32 tmp[4];
    __shared__ u32 carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const u32 J = m->jcount;
    for (u32 b = 0; b < J; b += 256) {
        const u32 i = b + threadIdx.x;
        const u32 v = i < J ? rows[order[i]].count : 0u;
        u32 tot;
        const u32 e = block_exclusive_sum<256>(v, tmp, tot);
        if (i < J && i < cap) first[i] = carry + e;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_st_jemit(const JRow* __restrict__ rows, const u64* __restrict__ jkeys,
                                                  const u32* __restrict__ order, const StreamMeta* m, u32 cap,
                                                  cv_journeys o, cv_result* res)
{
    const u32 J = m->jcount;
    const u32 lim = J < cap ? J : cap;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < lim; i += gridDim.x * blockDim.x) {
        const u32 s = order[i];
        const JRow& R = rows[s];
        Fx192 d, sp;
        d.w[0] = R.dist[0];
        d.w[1] = R.dist[1];
        d.w[2] = R.dist[2];
        sp.w[0] = R.spd[0];
        sp.w[1] = R.spd[1];
        sp.w[2] = R.spd[2];
        o.journey_id[i] = (i64)jkeys[s];
        o.n_points[i] = R.count;
        o.t_start_ms[i] = unord_i64(R.tmin_ord);
        o.t_end_ms[i] = unord_i64(R.tmax_ord);
        o.distance_m[i] = fx_to_double<FX_DIST>(d);
        o.sum_speed[i] = fx_to_double<FX_SPD>(sp);
        o.max_speed[i] = unord_f32(R.maxs);
        o.max_derived_speed[i] = unord_f64(R.maxd);
        o.n_dt_zero[i] = R.ndtz;
        o.lat_min[i] = unord_f64(R.latmin);
        o.lat_max[i] = unord_f64(R.latmax);
        o.lon_min[i] = unord_f64(R.lonmin);
        o.lon_max[i] = unord_f64(R.lonmax);
    }
    if (res && blockIdx.x == 0 && threadIdx.x == 0) {
        cv_result r = {};
        r.status = (J > cap || m->jt_full) ? CV_ERR_CAPACITY : CV_OK;
        r.count = J;
        r.required = J > cap ? J : 0;
        r.n_late = m->total_late;
        r.n_out_of_grid = m->total_out;
        r.flags = m->cell_overflow ? 1u : 0u;
        *res = r;
    }
}

}  // namespace

// host-side stream object
struct cv_stream {
    Spec g;
    u64 jslots, gslots, max_batch;
    size_t resident_bytes;  // meta, journey table and rows, group table, overflow pool: the state a snapshot holds
    // resident state
    StreamMeta* meta;
    u64* jkeys;
    JRow* rows;
    GEntry* tab;
    u64* ovf_pool;
    // per-push scratch
    void* sort_ws;
    size_t sort_ws_bytes;
    u32* perm;
    i64 *s_jid, *s_ts;
    double *s_lat, *s_lon;
    float* s_spd;
    double *fs_step, *fs_v, *fs_b;
    uint8_t* fs_flags;
    u32 *tile_cnt, *boff, *bslot;
    cv_result* sres;
    cv::JAcc* acc;  // exact partial summaries of the batch's journeys
    cv::AccX* accx;
    u64 arows;      // rows of acc / accx
    void* sum_ws;
    Append* ap;     // cells that counted their journey in this push
    // flush scratch
    u64 *gK0, *gK1, *jK0, *jK1;
    u32 *gC, *gV0, *gV1, *jV0, *jV1, *jfirst;
    u32 *ghist, *goffs, *jhist, *joffs;
    u64 *gstatus, *jstatus;
    size_t zero_off, zero_bytes;  // region cleared at creation (tables) - informational
};

namespace {

// overflow tables in the pool: one per 32 journey slots (one per 64 journeys)
u32 ovf_pages(u64 jslots) { return (u32)(jslots / 32 < 64 ? 64 : jslots / 32); }

// a batch with more journeys than the table has slots overflows the table anyway
u64 acc_rows(u64 jslots, u64 mb) { return mb < jslots ? (mb ? mb : 1) : jslots; }

struct StreamLayout {
    size_t bytes;
    template <class F>
    static void carve(cvh::Carver& c, u64 jslots, u64 gslots, u64 mb, F&& f)
    {
        const u64 opages = ovf_pages(jslots);
        const u64 tiles = (mb + ST_TILE - 1) / ST_TILE;
        size_t sort_ws = 0;
        cv_sort_workspace_size(mb, mb ? mb : 1, &sort_ws);
        f("meta", c.take<StreamMeta>(1));
        f("jkeys", c.take<u64>(jslots + 1));
        f("rows", c.take<JRow>(jslots + 1));
        f("tab", c.take<GEntry>(gslots));
        f("ovf_pool", c.take<u64>(opages * OVF_SLOTS));
        // everything above persists across pushes; everything below is per-push or per-flush scratch
        f("sort_ws", c.take<char>(sort_ws));
        f("perm", c.take<u32>(mb));
        f("s_jid", c.take<i64>(mb));
        f("s_ts", c.take<i64>(mb));
        f("s_lat", c.take<double>(mb));
        f("s_lon", c.take<double>(mb));
        f("s_spd", c.take<float>(mb));
        f("fs_step", c.take<double>(mb));
        f("fs_v", c.take<double>(mb));
        f("fs_b", c.take<double>(mb));
        f("fs_flags", c.take<uint8_t>(mb));
        f("tile_cnt", c.take<u32>(tiles + 1));
        f("boff", c.take<u32>(mb + 1));
        f("bslot", c.take<u32>(mb + 1));
        f("sres", c.take<cv_result>(1));
        const u64 arows = acc_rows(jslots, mb);
        f("acc", c.take<cv::JAcc>(arows));
        f("accx", c.take<cv::AccX>(arows));
        f("sum_ws", c.take<char>(cv::sum_partials_bytes(mb)));
        f("ap", c.take<Append>(mb));
        const u64 gst = (gslots + sort_min_tile() - 1) / sort_min_tile();
        const u64 jst = (jslots + 1 + sort_min_tile() - 1) / sort_min_tile();
        f("gK0", c.take<u64>(gslots));
        f("gK1", c.take<u64>(gslots));
        f("gC", c.take<u32>(gslots));
        f("gV0", c.take<u32>(gslots));
        f("gV1", c.take<u32>(gslots));
        f("ghist", c.take<u32>(MAX_PASSES * RADIX));
        f("goffs", c.take<u32>(MAX_PASSES * RADIX));
        f("gstatus", c.take<u64>(gst * RADIX + 1));
        f("jK0", c.take<u64>(jslots + 1));
        f("jK1", c.take<u64>(jslots + 1));
        f("jV0", c.take<u32>(jslots + 1));
        f("jV1", c.take<u32>(jslots + 1));
        f("jfirst", c.take<u32>(jslots + 1));
        f("jhist", c.take<u32>(MAX_PASSES * RADIX));
        f("joffs", c.take<u32>(MAX_PASSES * RADIX));
        f("jstatus", c.take<u64>(jst * RADIX + 1));
    }
};

void slots_for(u64 max_journeys, u64 max_groups, u64& js, u64& gs)
{
    js = cvh::next_pow2(2 * (max_journeys < 512 ? 512 : max_journeys));
    gs = cvh::next_pow2(2 * (max_groups < 2048 ? 2048 : max_groups));
}

bool stream_spec_ok(const cv_grid_spec* g)
{
    if (!g) return false;
    if (!(g->dlat_deg > 0.0) || !(g->dlon_deg > 0.0) || !std::isfinite(g->lat0_deg) || !std::isfinite(g->lon0_deg))
        return false;
    if (g->n_lat <= 0 || g->n_lon <= 0 || g->bin_ms <= 0 || g->n_lat > (1ll << 31) || g->n_lon > (1ll << 31))
        return false;
    return true;
}

// Header of a snapshot: what must match between the stream that wrote it and
// the stream that restores it (the resident layout depends on the table sizes
// and the binning on the grid).
struct SnapHeader {
    u64 magic;
    u64 abi;
    u64 jslots, gslots, opages;
    u64 resident_bytes;
    double lat0, lon0, dlat, dlon;
    i64 n_lat, n_lon, t0, bin_ms, tmax;
};
constexpr u64 SNAP_MAGIC = 0x31706e7374657663ull;  // "cvetsnp1"
constexpr size_t SNAP_HDR = 256;
static_assert(sizeof(SnapHeader) <= SNAP_HDR, "snapshot header");

SnapHeader snap_header(const cv_stream* st)
{
    SnapHeader h;
    std::memset(&h, 0, sizeof(h));
    h.magic = SNAP_MAGIC;
    h.abi = CV_ABI_VERSION;
    h.jslots = st->jslots;
    h.gslots = st->gslots;
    h.opages = ovf_pages(st->jslots);
    h.resident_bytes = st->resident_bytes;
    h.lat0 = st->g.lat0;
    h.lon0 = st->g.lon0;
    h.dlat = st->g.dlat;
    h.dlon = st->g.dlon;
    h.n_lat = st->g.n_lat;
    h.n_lon = st->g.n_lon;
    h.t0 = st->g.t0;
    h.bin_ms = st->g.bin_ms;
    h.tmax = st->g.tmax;
    return h;
}

}  // namespace

extern "C" {

cv_status cv_stream_state_size(const cv_grid_spec* grid, uint64_t max_journeys, uint64_t max_groups,
                               uint64_t max_batch, size_t* bytes)
{
    if (!bytes || !stream_spec_ok(grid) || max_batch >= (1ull << 31) || max_journeys >= (1ull << 30) ||
        max_groups >= (1ull << 30))
        return CV_ERR_INVALID_ARGUMENT;
    u64 js, gs;
    slots_for(max_journeys, max_groups, js, gs);
    cvh::Carver c(nullptr);
    StreamLayout::carve(c, js, gs, max_batch, [](const char*, void*) {});
    *bytes = c.size();
    return CV_OK;
}

cv_status cv_stream_create(const cv_grid_spec* grid, uint64_t max_journeys, uint64_t max_groups, uint64_t max_batch,
                           void* state, size_t state_bytes, void* stream, cv_stream** out)
{
    if (!out || !stream_spec_ok(grid) || max_batch >= (1ull << 31) || max_journeys >= (1ull << 30) ||
        max_groups >= (1ull << 30))
        return CV_ERR_INVALID_ARGUMENT;
    size_t need = 0;
    cv_stream_state_size(grid, max_journeys, max_groups, max_batch, &need);
    if (!state || !cvh::aligned(state, cvh::WS_ALIGN) || state_bytes < need) return CV_ERR_WORKSPACE;
    cv_stream* st = new (std::nothrow) cv_stream();
    if (!st) return CV_ERR_DEVICE;
    slots_for(max_journeys, max_groups, st->jslots, st->gslots);
    st->max_batch = max_batch;
    Spec& g = st->g;
    g.lat0 = grid->lat0_deg;
    g.lon0 = grid->lon0_deg;
    g.dlat = grid->dlat_deg;
    g.dlon = grid->dlon_deg;
    g.n_lat = grid->n_lat;
    g.n_lon = grid->n_lon;
    g.t0 = grid->t0_ms;
    g.bin_ms = grid->bin_ms;
    g.tinv = 1.0 / (double)grid->bin_ms;
    g.tmax = grid->n_t > 0 ? grid->n_t : (INT64_MAX / (grid->n_lat * grid->n_lon));
    g.soff = nullptr;
    g.S = 0;
    g.kb = 0;
    g.nd = 0;
    g.dstep = g.doff = 0.0;
    g.hdg = nullptr;
    g.brg = nullptr;
    g.bfl = nullptr;
    g.sout = nullptr;
    cvh::Carver c(state);
    StreamLayout::carve(c, st->jslots, st->gslots, max_batch, [&](const char* name, void* p) {
        const std::string nm(name);
        if (nm == "meta") st->meta = (StreamMeta*)p;
        else if (nm == "jkeys") st->jkeys = (u64*)p;
        else if (nm == "rows") st->rows = (JRow*)p;
        else if (nm == "tab") st->tab = (GEntry*)p;
        else if (nm == "ovf_pool") st->ovf_pool = (u64*)p;
        else if (nm == "sort_ws") {
            st->sort_ws = p;
            st->resident_bytes = (size_t)((char*)p - (char*)state);
        }
        else if (nm == "perm") st->perm = (u32*)p;
        else if (nm == "s_jid") st->s_jid = (i64*)p;
        else if (nm == "s_ts") st->s_ts = (i64*)p;
        else if (nm == "s_lat") st->s_lat = (double*)p;
        else if (nm == "s_lon") st->s_lon = (double*)p;
        else if (nm == "s_spd") st->s_spd = (float*)p;
        else if (nm == "fs_step") st->fs_step = (double*)p;
        else if (nm == "fs_v") st->fs_v = (double*)p;
        else if (nm == "fs_b") st->fs_b = (double*)p;
        else if (nm == "fs_flags") st->fs_flags = (uint8_t*)p;
        else if (nm == "tile_cnt") st->tile_cnt = (u32*)p;
        else if (nm == "boff") st->boff = (u32*)p;
        else if (nm == "bslot") st->bslot = (u32*)p;
        else if (nm == "sres") st->sres = (cv_result*)p;
        else if (nm == "acc") st->acc = (cv::JAcc*)p;
        else if (nm == "accx") st->accx = (cv::AccX*)p;
        else if (nm == "sum_ws") st->sum_ws = p;
        else if (nm == "ap") st->ap = (Append*)p;
        else if (nm == "gK0") st->gK0 = (u64*)p;
        else if (nm == "gK1") st->gK1 = (u64*)p;
        else if (nm == "gC") st->gC = (u32*)p;
        else if (nm == "gV0") st->gV0 = (u32*)p;
        else if (nm == "gV1") st->gV1 = (u32*)p;
        else if (nm == "ghist") st->ghist = (u32*)p;
        else if (nm == "goffs") st->goffs = (u32*)p;
        else if (nm == "gstatus") st->gstatus = (u64*)p;
        else if (nm == "jK0") st->jK0 = (u64*)p;
        else if (nm == "jK1") st->jK1 = (u64*)p;
        else if (nm == "jV0") st->jV0 = (u32*)p;
        else if (nm == "jV1") st->jV1 = (u32*)p;
        else if (nm == "jfirst") st->jfirst = (u32*)p;
        else if (nm == "jhist") st->jhist = (u32*)p;
        else if (nm == "joffs") st->joffs = (u32*)p;
        else if (nm == "jstatus") st->jstatus = (u64*)p;
    });
    cv_sort_workspace_size(max_batch, max_batch ? max_batch : 1, &st->sort_ws_bytes);
    st->arows = acc_rows(st->jslots, max_batch);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_st_init_meta, dim3(1), dim3(64), 0, s, st->meta);
    cvh::fill_u64(st->jkeys, JEMPTY, st->jslots + 1, s);
    hipLaunchKernelGGL(k_grid_clear, dim3(cvh::grid_for(st->gslots, 256, 4096)), dim3(256), 0, s, st->tab, st->gslots,
                       &st->meta->gm);
    cvh::fill_u64(st->ovf_pool, OVF_EMPTY, (u64)ovf_pages(st->jslots) * OVF_SLOTS, s);
    cv_status e = cvh::last_launch_status();
    if (e != CV_OK) {
        delete st;
        return e;
    }
    *out = st;
    return CV_OK;
}

cv_status cv_stream_push(cv_stream* st, const cv_records* batch, const cv_features* feat, cv_result* res, void* stream)
{
    if (!st || !batch || !feat || batch->n > st->max_batch) return CV_ERR_INVALID_ARGUMENT;
    const u64 n = batch->n;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        hipLaunchKernelGGL(k_st_begin, dim3(1), dim3(64), 0, s, st->meta);
        if (res) {
            cvh::fill_u32(st->sres, 0u, sizeof(cv_result) / 4, s);
            hipLaunchKernelGGL(k_st_finish, dim3(1), dim3(64), 0, s, st->meta, st->sres, 0u, res);
        }
        return cvh::last_launch_status();
    }
    if (!batch->journey_id || !batch->ts_ms || !batch->lat_deg || !batch->lon_deg || !batch->speed_mps ||
        !feat->step_m || !feat->dt_s || !feat->speed_mps || !feat->accel_mps2 || !feat->bearing_deg ||
        !feat->dheading_deg || !feat->flags)
        return CV_ERR_INVALID_ARGUMENT;
    const u32 nn = (u32)n;
    cvh::TimedScope ts_("stream_push", s);
    hipLaunchKernelGGL(k_st_begin, dim3(1), dim3(64), 0, s, st->meta);
    cv_records_out so{st->s_jid, st->s_ts, st->s_lat, st->s_lon, st->s_spd};
    cv_status e = CV_OK;
    {
        cvh::TimedScope t1("stream_sort", s);
        // a batch holds at most n distinct journeys: the dictionary of its sort is
        // sized (and cleared) for n, within the workspace carved for max_batch
        e = cv::sort_records_into(batch, n, st->perm, &so, st->sres, st->sort_ws, st->sort_ws_bytes, s);
        if (e != CV_OK) return e;
    }
    const u32 tiles = (u32)((n + ST_TILE - 1) / ST_TILE);
    {
        cvh::TimedScope t2("stream_journeys", s);
        hipLaunchKernelGGL(k_st_count, dim3(tiles), dim3(256), 0, s, st->s_jid, nn, st->tile_cnt);
        hipLaunchKernelGGL(k_st_scan, dim3(1), dim3(256), 0, s, st->tile_cnt, tiles, st->meta);
        hipLaunchKernelGGL(k_st_heads, dim3(tiles), dim3(256), 0, s, st->s_jid, nn, st->tile_cnt, st->meta,
                           st->boff);
        hipLaunchKernelGGL(k_st_journeys, dim3(cvh::grid_for(n, 256, 2048)), dim3(256), 0, s, st->s_jid, st->boff,
                           st->meta, st->jkeys, st->jslots - 1, st->rows, st->bslot);
    }
    {
        cvh::TimedScope t3("stream_features", s);
        hipLaunchKernelGGL(k_st_features, dim3((unsigned)((n + FB - 1) / FB)), dim3(FB), 0, s, nn, st->s_jid,
                           st->s_ts, st->s_lat, st->s_lon, st->perm, st->boff, st->meta, st->bslot, st->rows, *feat,
                           st->fs_step, st->fs_v, st->fs_b, st->fs_flags);
    }
    {
        // summaries: the plain kernels' exact per-journey partials of the batch
        cvh::TimedScope t4("stream_summary", s);
        cv_records sb{};
        sb.journey_id = st->s_jid;
        sb.ts_ms = st->s_ts;
        sb.lat_deg = st->s_lat;
        sb.lon_deg = st->s_lon;
        sb.speed_mps = st->s_spd;
        sb.n = n;
        cv_features fb{};
        fb.step_m = st->fs_step;
        fb.speed_mps = st->fs_v;
        fb.flags = st->fs_flags;
        e = cv::sum_partials(&sb, &fb, (u32)st->arows, st->acc, st->accx, st->sum_ws, s);
        if (e != CV_OK) return e;
    }
    const i64 cells = st->g.n_lat * st->g.n_lon;
    {
        // groups: the grid tile kernel into the resident table
        cvh::TimedScope t5("stream_grid", s);
        GridStream pol{st->s_jid, st->fs_flags, st->boff, st->meta, st->bslot, st->rows, st->ovf_pool,
                       cells,     st->ap,       (u32)st->max_batch, &st->meta->ap_n};
        const SinkTable sk{st->tab, st->gslots - 1, &st->meta->gm};
        hipLaunchKernelGGL((k_grid_agg<256, GridStream, SinkTable>), dim3((unsigned)((n + GT - 1) / GT)), dim3(GB), 0,
                           s, nn, st->s_jid, st->s_ts, st->s_lat, st->s_lon, st->s_spd, st->g, sk, &st->meta->gm, pol);
    }
    {
        // resident rows: the partials, the last point, the open segment's cells
        cvh::TimedScope t6("stream_merge", s);
        hipLaunchKernelGGL(k_st_merge, dim3(cvh::grid_for(n, 256, 2048)), dim3(256), 0, s, st->s_ts, st->s_lat,
                           st->s_lon, st->boff, st->meta, st->bslot, st->rows, st->acc, st->accx, (u32)st->arows,
                           st->fs_v, st->fs_b, st->fs_flags, st->g, st->ovf_pool);
        hipLaunchKernelGGL(k_st_append, dim3(cvh::grid_for(n, 256, 2048)), dim3(256), 0, s, st->ap, st->meta,
                           (u32)st->max_batch, st->rows, ovf_pages(st->jslots), cells);
        hipLaunchKernelGGL(k_st_append_ovf, dim3(cvh::grid_for(n, 256, 2048)), dim3(256), 0, s, st->ap, st->meta,
                           (u32)st->max_batch, st->rows, st->ovf_pool);
    }
    hipLaunchKernelGGL(k_st_finish, dim3(1), dim3(64), 0, s, st->meta, st->sres, nn, res);
    return cvh::last_launch_status();
}

cv_status cv_stream_flush(cv_stream* st, const cv_journeys* journeys, uint64_t journey_capacity,
                          const cv_groups* groups, uint64_t group_capacity, cv_result* res, void* stream)
{
    if (!st || !journeys || !groups || journey_capacity >= (1ull << 32) || group_capacity >= (1ull << 32))
        return CV_ERR_INVALID_ARGUMENT;
    hipStream_t s = (hipStream_t)stream;
    const u32 jcap = (u32)journey_capacity, gcap = (u32)group_capacity;
    // journeys
    cvh::fill_u32(&st->meta->jcount, 0u, 1, s);
    cvh::fill_u32(st->jhist, 0u, MAX_PASSES * RADIX, s);
    const u64 jrows = st->jslots + 1;  // table slots and the reserved row
    const u64 jst = (jrows + sort_min_tile() - 1) / sort_min_tile();
    cvh::fill_u64(st->jstatus, 0ull, jst * RADIX + 1, s);
    cvh::fill_u32(st->meta->jtickets, 0u, MAX_PASSES, s);
    hipLaunchKernelGGL(k_st_jcompact, dim3(cvh::grid_for(st->jslots, 256, 4096)), dim3(256), 0, s, st->jkeys,
                       st->jslots, st->meta, st->jK0, st->jV0);
    const u32* jn = &st->meta->jcount;
    radix_hist(st->jK0, (u32)jrows, jn, MAX_PASSES, nullptr, st->jhist, cvh::grid_for(jrows, 256, 1024), s);
    radix_scan(st->jhist, st->joffs, MAX_PASSES, s);
    // 8 passes: the sorted pairs end in (jK0, jV0); pass 0 reads the slot values from jV0 via jfirst copy
    u32* vfirst = st->jfirst;
    if (hipMemcpyAsync(vfirst, st->jV0, jrows * sizeof(u32), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return CV_ERR_DEVICE;
    radix_passes(st->jK0, st->jK1, vfirst, st->jV0, st->jV1, (u32)jrows, jn, nullptr, MAX_PASSES, st->joffs,
                 st->jstatus, st->meta->jtickets, s);
    cv_status e = CV_OK;
    if (jcap > 0) {
        if (!journeys->journey_id || !journeys->first || !journeys->n_points || !journeys->t_start_ms ||
            !journeys->t_end_ms || !journeys->distance_m || !journeys->sum_speed || !journeys->max_speed ||
            !journeys->max_derived_speed || !journeys->n_dt_zero || !journeys->lat_min || !journeys->lat_max ||
            !journeys->lon_min || !journeys->lon_max)
            return CV_ERR_INVALID_ARGUMENT;
        hipLaunchKernelGGL(k_st_jfirst, dim3(1), dim3(256), 0, s, st->rows, st->jV0, st->meta, journeys->first, jcap);
    }
    hipLaunchKernelGGL(k_st_jemit, dim3(cvh::grid_for(jcap ? jcap : 1, 256, 4096)), dim3(256), 0, s, st->rows,
                       st->jkeys, st->jV0, st->meta, jcap, *journeys, res);
    // groups: compaction, key sort, emit (same tail as the plain grid)
    cvh::fill_u32(&st->meta->gm.compact_n, 0u, 1, s);
    cvh::fill_u64(&st->meta->gm.max_key, 0ull, 1, s);
    cvh::fill_u32(st->ghist, 0u, MAX_PASSES * RADIX, s);
    const u64 gst = (st->gslots + sort_min_tile() - 1) / sort_min_tile();
    cvh::fill_u64(st->gstatus, 0ull, gst * RADIX + 1, s);
    cvh::fill_u32(st->meta->gm.tickets, 0u, MAX_PASSES, s);
    hipLaunchKernelGGL(k_grid_compact, dim3((unsigned)((st->gslots + CSLOTS - 1) / CSLOTS)), dim3(256), 0, s, st->tab,
                       st->gslots, &st->meta->gm, st->gK0, st->gC);
    hipLaunchKernelGGL(k_grid_bits, dim3(1), dim3(64), 0, s, &st->meta->gm);
    const u32* cnt = &st->meta->gm.compact_n;
    const u32* bits = &st->meta->gm.key_bits;
    radix_hist(st->gK0, (u32)st->gslots, cnt, MAX_PASSES, bits, st->ghist, cvh::grid_for(st->gslots, 256, 1024), s);
    radix_scan(st->ghist, st->goffs, MAX_PASSES, s);
    radix_passes(st->gK0, st->gK1, st->gC, st->gV0, st->gV1, (u32)st->gslots, cnt, bits, MAX_PASSES, st->goffs,
                 st->gstatus, st->meta->gm.tickets, s);
    hipLaunchKernelGGL(k_iota_if_nopass, dim3(cvh::grid_for(st->gslots, 256, 1024)), dim3(256), 0, s, &st->meta->gm,
                       st->gC, st->gV0, (u32)st->gslots);
    if (gcap > 0 && (!groups->key || !groups->count || !groups->n_journeys || !groups->sum_speed ||
                     !groups->min_speed || !groups->max_speed))
        return CV_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(k_grid_emit, dim3(cvh::grid_for(gcap ? gcap : 1, 256, 4096)), dim3(256), 0, s, st->tab,
                       &st->meta->gm, st->gK0, st->gK1, st->gV0, st->gV1, gcap, groups->key, groups->count,
                       groups->n_journeys, groups->sum_speed, groups->min_speed, groups->max_speed,
                       res ? res + 1 : nullptr, ~0ull);
    e = cvh::last_launch_status();
    return e;
}

cv_status cv_stream_snapshot_size(const cv_stream* st, size_t* bytes)
{
    if (!st || !bytes) return CV_ERR_INVALID_ARGUMENT;
    *bytes = SNAP_HDR + st->resident_bytes;
    return CV_OK;
}

cv_status cv_stream_snapshot(cv_stream* st, void* host_buf, size_t bytes, void* stream)
{
    if (!st || !host_buf || bytes < SNAP_HDR + st->resident_bytes) return CV_ERR_INVALID_ARGUMENT;
    const SnapHeader h = snap_header(st);
    std::memset(host_buf, 0, SNAP_HDR);
    std::memcpy(host_buf, &h, sizeof(h));
    if (hipMemcpyAsync((char*)host_buf + SNAP_HDR, st->meta, st->resident_bytes, hipMemcpyDeviceToHost,
                       (hipStream_t)stream) != hipSuccess)
        return CV_ERR_DEVICE;
    return CV_OK;
}

cv_status cv_stream_restore(cv_stream* st, const void* host_buf, size_t bytes, void* stream)
{
    if (!st || !host_buf || bytes < SNAP_HDR) return CV_ERR_INVALID_ARGUMENT;
    SnapHeader h;
    std::memcpy(&h, host_buf, sizeof(h));
    const SnapHeader mine = snap_header(st);
    if (h.magic != SNAP_MAGIC || h.abi != CV_ABI_VERSION || bytes < SNAP_HDR + h.resident_bytes ||
        std::memcmp(&h, &mine, sizeof(h)) != 0)
        return CV_ERR_INVALID_ARGUMENT;
    if (hipMemcpyAsync(st->meta, (const char*)host_buf + SNAP_HDR, st->resident_bytes, hipMemcpyHostToDevice,
                       (hipStream_t)stream) != hipSuccess)
        return CV_ERR_DEVICE;
    return CV_OK;
}

cv_status cv_stream_destroy(cv_stream* st)
{
    delete st;
    return CV_OK;
}

}  // extern "C"
