// cv_csv.hip -- extraction of Table-1-shaped text rows (journey id,
// timestamp, latitude, longitude, postal code, speed, heading) into record
// columns on the device: the "E" of the ETL path ahead of the key prep.
//
//   k_csv_count   newlines per tile of CT bytes (16-byte loads)
//   k_csv_scan    exclusive prefix of the tile counts
//   k_csv_rows    row start offsets, in order
//   k_csv_parse   one thread per row: the fields of the row
#include <hip/hip_runtime.h>

#include "cv_device.h"
#include "cv_host.h"

using namespace cv;

namespace {

constexpr int CB = 256;          // threads per block
constexpr int CPT = 64;          // bytes per thread
constexpr int CT = CB * CPT;     // bytes per tile

// newline positions (relative to p) among the bytes of one thread's stretch
// [p, p + len), len <= CPT; bit i of the result marks byte i
__device__ __forceinline__ u64 newline_mask(const unsigned char* __restrict__ text, u64 p, u64 nbytes)
{
    u64 m = 0;
    if (p + CPT <= nbytes) {
        const uint4* q = reinterpret_cast<const uint4*>(text + p);
        uint4 v[CPT / 16];
#pragma unroll
        for (int i = 0; i < CPT / 16; ++i) v[i] = q[i];
#pragma unroll
        for (int i = 0; i < CPT / 16; ++i) {
            const u32 w[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (((w[j] >> (8 * b)) & 0xFFu) == 0x0Au) m |= 1ull << (16 * i + 4 * j + b);
        }
    } else {
        for (int i = 0; i < CPT && p + i < nbytes; ++i)
            if (text[p + i] == '\n') m |= 1ull << i;
    }
    return m;
}

__global__ void __launch_bounds__(CB) k_csv_count(const unsigned char* __restrict__ text, u64 nbytes,
                                                  u32* __restrict__ tcnt)
{
    __shared__ u32 s_w[CB / WAVE];
    const u64 p = (u64)blockIdx.x * CT + (u64)threadIdx.x * CPT;
    u32 c = p < nbytes ? (u32)__popcll(newline_mask(text, p, nbytes)) : 0u;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, WAVE);
    if (lane_id() == 0) s_w[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 t = 0;
        for (int w = 0; w < CB / WAVE; ++w) t += s_w[w];
        tcnt[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(1024) k_csv_scan(u32* __restrict__ tcnt, u64 tiles)
{
    __shared__ u32 s_tmp[1024 / WAVE];
    u64 carry = 0;
    for (u64 b = 0; b < tiles; b += 1024) {
        const u64 i = b + threadIdx.x;
        const u32 v = i < tiles ? tcnt[i] : 0u;
        u32 tot;
        const u32 ex = block_exclusive_sum<1024>(v, s_tmp, tot);
        if (i < tiles) tcnt[i] = (u32)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0) tcnt[tiles] = (u32)carry;
}

// Line starts: 0 and every byte after a newline, in order, into
// start[0 .. cap_lines]; a line ends at the next start (its newline
// included).  start[lines] = nbytes.
__global__ void __launch_bounds__(CB) k_csv_rows(const unsigned char* __restrict__ text, u64 nbytes,
                                                 const u32* __restrict__ tpre, u64* __restrict__ start, u64 cap_lines)
{
    __shared__ u32 s_tmp[CB / WAVE];
    const u64 p = (u64)blockIdx.x * CT + (u64)threadIdx.x * CPT;
    u64 m = p < nbytes ? newline_mask(text, p, nbytes) : 0ull;
    u32 tot;
    u32 at = tpre[blockIdx.x] + block_exclusive_sum<CB>((u32)__popcll(m), s_tmp, tot);
    if (blockIdx.x == 0 && threadIdx.x == 0) start[0] = 0;
    while (m) {
        const int b = __ffsll((long long)m) - 1;
        m &= m - 1;
        ++at;  // the line after this newline
        if (at <= cap_lines) start[at] = p + (u64)b + 1;
    }
}

// ------------------------------------------------------------------ fields

__device__ __forceinline__ bool is_digit(unsigned char c) { return c >= '0' && c <= '9'; }

// up to 8 bytes, packed big-endian (string order = integer order)
__device__ __forceinline__ bool parse_id(const unsigned char* s, int len, i64& out)
{
    if (len < 1 || len > 8) return false;
    u64 v = 0;
    for (int i = 0; i < 8; ++i) v = (v << 8) | (i < len ? (u64)s[i] : 0ull);
    out = (i64)v;
    return (v >> 63) == 0;  // bytes below 0x80
}

__device__ __forceinline__ int digits(const unsigned char* s, int n)
{
    int v = 0;
    for (int i = 0; i < n; ++i) {
        if (!is_digit(s[i])) return -1;
        v = v * 10 + (s[i] - '0');
    }
    return v;
}

// days since 1970-01-01 of a proleptic Gregorian date (civil-from-days
// inverse: eras of 400 years, March-based years)
__device__ __forceinline__ i64 days_from_civil(i64 y, int m, int d)
{
    y -= m <= 2;
    const i64 era = (y >= 0 ? y : y - 399) / 400;
    const i64 yoe = y - era * 400;
    const i64 doy = (153 * (m + (m > 2 ? -3 : 9)) + 2) / 5 + d - 1;
    const i64 doe = yoe * 365 + yoe / 4 - yoe / 100 + doy;
    return era * 146097 + doe - 719468;
}

// "YYYY-MM-DD HH:MM:SS" with an optional fraction of 1 to 3 digits: UTC ms
__device__ __forceinline__ bool parse_ts(const unsigned char* s, int len, i64& out)
{
    if (len < 19 || s[4] != '-' || s[7] != '-' || s[10] != ' ' || s[13] != ':' || s[16] != ':') return false;
    const int y = digits(s, 4), mo = digits(s + 5, 2), d = digits(s + 8, 2);
    const int h = digits(s + 11, 2), mi = digits(s + 14, 2), se = digits(s + 17, 2);
    if (y < 1 || mo < 1 || mo > 12 || d < 1 || h < 0 || h > 23 || mi < 0 || mi > 59 || se < 0 || se > 59) return false;
    const bool leap = (y % 4 == 0 && y % 100 != 0) || y % 400 == 0;
    const int mdays[12] = {31, 28, 31, 30, 31, 30, 31, 31, 30, 31, 30, 31};
    if (d > mdays[mo - 1] + ((mo == 2 && leap) ? 1 : 0)) return false;
    int ms = 0;
    if (len > 19) {
        const int f = len - 20;
        if (s[19] != '.' || f < 1 || f > 3) return false;
        const int v = digits(s + 20, f);
        if (v < 0) return false;
        ms = f == 1 ? v * 100 : (f == 2 ? v * 10 : v);
    }
    out = ((days_from_civil(y, mo, d) * 24 + h) * 60 + mi) * 60000 + (i64)se * 1000 + ms;
    return true;
}

// A plain decimal ([-+]digits[.digits]): the integer of its significant
// digits (below 2^53) and the count of fraction digits (at most 22) give
// the exact quotient rounded once (one IEEE division by an exact power of
// ten); other forms are refused.
__device__ __forceinline__ bool parse_decimal(const unsigned char* s, int len, double& out)
{
    constexpr double P10[23] = {1e0,  1e1,  1e2,  1e3,  1e4,  1e5,  1e6,  1e7,  1e8,  1e9,  1e10, 1e11,
                                1e12, 1e13, 1e14, 1e15, 1e16, 1e17, 1e18, 1e19, 1e20, 1e21, 1e22};
    int i = 0;
    bool neg = false;
    if (i < len && (s[i] == '-' || s[i] == '+')) neg = s[i++] == '-';
    u64 m = 0;
    int nd = 0, frac = 0;
    bool dot = false;
    for (; i < len; ++i) {
        const unsigned char c = s[i];
        if (c == '.') {
            if (dot) return false;
            dot = true;
            continue;
        }
        if (!is_digit(c)) return false;
        ++nd;
        if (m > (1ull << 53) / 10) return false;  // beyond the exact range
        m = m * 10 + (c - '0');
        if (dot) ++frac;
    }
    if (nd == 0 || m >= (1ull << 53) || frac > 22) return false;
    const double v = frac ? (double)m / P10[frac] : (double)m;
    out = neg ? -v : v;
    return true;
}

constexpr int SB = 32 * 1024;  // LDS bytes staged per block

struct Row {
    i64 jid, ts;
    double lat, lon, spd, hdg;
    bool ok;
};

// The fields of one row of rl bytes at s (its line end included).  Inlined
// into each caller, so that a row staged in LDS is read with LDS loads.
__device__ __forceinline__ Row parse_row(const unsigned char* s, u64 rl)
{
    Row w;
    if (rl && s[rl - 1] == '\n') --rl;
    if (rl && s[rl - 1] == '\r') --rl;
    const int len = (int)(rl < (u64)(1 << 20) ? rl : (u64)(1 << 20));
    // field boundaries: exactly six commas
    int cpos[6];
    int nc = 0;
    bool ok = rl < (u64)(1 << 20);
    for (int i = 0; i < len && ok; ++i) {
        if (s[i] == ',') {
            if (nc < 6) cpos[nc] = i;
            ++nc;
        } else if (s[i] == '"') {
            ok = false;
        }
    }
    ok = ok && nc == 6;
    w.jid = 0;
    w.ts = 0;
    w.lat = w.lon = w.spd = w.hdg = __builtin_nan("");
    if (ok) {
        ok = parse_id(s, cpos[0], w.jid) && parse_ts(s + cpos[0] + 1, cpos[1] - cpos[0] - 1, w.ts) &&
             parse_decimal(s + cpos[1] + 1, cpos[2] - cpos[1] - 1, w.lat) &&
             parse_decimal(s + cpos[2] + 1, cpos[3] - cpos[2] - 1, w.lon) &&
             parse_decimal(s + cpos[4] + 1, cpos[5] - cpos[4] - 1, w.spd);
        const int hl = len - cpos[5] - 1;
        if (ok && hl > 0 && !parse_decimal(s + cpos[5] + 1, hl, w.hdg)) ok = false;
    }
    if (!ok) {
        w.jid = 0;
        w.ts = 0;
        w.lat = w.lon = w.spd = w.hdg = __builtin_nan("");
    }
    w.ok = ok;
    return w;
}

// The rows that fit the capacity, after the header (meta: header lines
// skipped, rows to parse), CB per block, one per thread; malformed rows are
// counted in res->n_bad.  A block's rows are contiguous text: when they fit
// SB bytes they are staged in LDS with 16-byte loads and parsed from there.
__global__ void __launch_bounds__(CB) k_csv_parse(const unsigned char* __restrict__ text, u64 nbytes,
                                                  const u64* __restrict__ start, const u64* __restrict__ meta,
                                                  cv_records_out o, float* __restrict__ heading,
                                                  uint8_t* __restrict__ row_ok, cv_result* res)
{
    __shared__ __attribute__((aligned(16))) unsigned char s_txt[SB + 16];
    const u64 first = meta[0], rows = meta[1];
    const u64 r0 = (u64)blockIdx.x * CB;
    if (r0 >= rows) return;
    const u64 r1 = r0 + CB < rows ? r0 + CB : rows;
    const u64 B0 = start[first + r0], B1 = start[first + r1];
    const u64 A0 = B0 & ~15ull;
    const bool staged = B1 - A0 <= SB;
    if (staged) {
        for (u64 a = A0 + 16 * (u64)threadIdx.x; a < B1; a += 16 * CB) {
            if (a + 16 <= nbytes) {
                *reinterpret_cast<uint4*>(&s_txt[a - A0]) = *reinterpret_cast<const uint4*>(text + a);
            } else {
                for (u64 c = a; c < a + 16 && c < nbytes; ++c) s_txt[c - A0] = text[c];
            }
        }
    }
    __syncthreads();
    u64 bad = 0;
    const u64 r = r0 + threadIdx.x;
    if (r < r1) {
        const u64 b = start[first + r];
        const u64 rl = start[first + r + 1] - b;  // the row's bytes, its line end included
        const Row w = staged ? parse_row(s_txt + (b - A0), rl) : parse_row(text + b, rl);
        bad += w.ok ? 0 : 1;
        o.journey_id[r] = w.jid;
        o.ts_ms[r] = w.ts;
        o.lat_deg[r] = w.lat;
        o.lon_deg[r] = w.lon;
        o.speed_mps[r] = (float)w.spd;
        if (heading) heading[r] = (float)w.hdg;
        if (row_ok) row_ok[r] = w.ok ? 1 : 0;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) bad += __shfl_xor(bad, d, WAVE);
    if (lane_id() == 0 && bad) atomicAdd((unsigned long long*)&res->n_bad, (unsigned long long)bad);
}

// result: rows = lines (a last line without its newline counts) minus the header
__global__ void k_csv_begin(const u32* __restrict__ tcnt, u64 tiles, const unsigned char* __restrict__ text,
                            u64 nbytes, int header, u64 cap, u64* __restrict__ start, u64* __restrict__ meta,
                            cv_result* res)
{
    if (threadIdx.x != 0) return;
    const u64 nl = tcnt[tiles];
    const u64 lines = nl + ((nbytes && text[nbytes - 1] != '\n') ? 1 : 0);
    const u64 skip = (header && lines) ? 1 : 0;
    const u64 rows = lines - skip;
    // the end of the last line, when it lies within the offsets kept
    if (lines <= cap + skip) start[lines] = nbytes;
    meta[0] = skip;
    meta[1] = rows < cap ? rows : cap;
    cv_result r = {};
    r.status = rows > cap ? CV_ERR_CAPACITY : CV_OK;
    r.count = rows;
    r.required = rows > cap ? rows : 0;
    *res = r;
}

}  // namespace

extern "C" {

cv_status cv_csv_workspace_size(uint64_t nbytes, uint64_t capacity, size_t* bytes)
{
    if (!bytes || capacity >= (1ull << 32)) return CV_ERR_INVALID_ARGUMENT;
    const u64 tiles = (nbytes + CT - 1) / CT;
    if (tiles >= (1ull << 31)) return CV_ERR_INVALID_ARGUMENT;
    *bytes = cvh::align_up((tiles + 1) * sizeof(u32)) + cvh::align_up((capacity + 3) * sizeof(u64)) +
             cvh::align_up(2 * sizeof(u64));
    return CV_OK;
}

cv_status cv_csv_extract(const char* text, uint64_t nbytes, int32_t has_header, const cv_records_out* out,
                         float* heading_deg, uint8_t* row_ok, uint64_t capacity, cv_result* res, void* ws,
                         size_t ws_bytes, void* stream)
{
    if (!res || !out || capacity >= (1ull << 32) || (nbytes && !text) || !cvh::aligned(text, 16))
        return CV_ERR_INVALID_ARGUMENT;
    if (capacity && (!out->journey_id || !out->ts_ms || !out->lat_deg || !out->lon_deg || !out->speed_mps))
        return CV_ERR_INVALID_ARGUMENT;
    size_t need = 0;
    cv_status e = cv_csv_workspace_size(nbytes, capacity, &need);
    if (e != CV_OK) return e;
    if (!ws || !cvh::aligned(ws, cvh::WS_ALIGN) || ws_bytes < need) return CV_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    cvh::TimedScope ts_("csv_extract", s);
    const u64 tiles = (nbytes + CT - 1) / CT;
    cvh::Carver c(ws);
    u32* tcnt = c.take<u32>(tiles + 1);
    u64* start = c.take<u64>(capacity + 3);
    u64* meta = c.take<u64>(2);
    const unsigned char* t = (const unsigned char*)text;
    if (tiles) hipLaunchKernelGGL(k_csv_count, dim3((unsigned)tiles), dim3(CB), 0, s, t, (u64)nbytes, tcnt);
    hipLaunchKernelGGL(k_csv_scan, dim3(1), dim3(1024), 0, s, tcnt, tiles);
    // offsets of the first capacity + 1 (+ header) lines
    const u64 cap_lines = capacity + 2;
    if (tiles)
        hipLaunchKernelGGL(k_csv_rows, dim3((unsigned)tiles), dim3(CB), 0, s, t, (u64)nbytes, tcnt, start,
                           cap_lines);
    else
        cvh::fill_u64(start, 0ull, 1, s);
    hipLaunchKernelGGL(k_csv_begin, dim3(1), dim3(64), 0, s, tcnt, tiles, t, (u64)nbytes, has_header ? 1 : 0,
                       (u64)capacity, start, meta, res);
    if (capacity)
        hipLaunchKernelGGL(k_csv_parse, dim3((unsigned)((capacity + CB - 1) / CB)), dim3(CB), 0, s, t, (u64)nbytes,
                           start, meta, *out, heading_deg, row_ok, res);
    return cvh::last_launch_status();
}

}  // extern "C"
