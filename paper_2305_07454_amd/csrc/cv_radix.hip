// cv_radix.hip -- kernels and host launchers of the stable LSD radix sort
// described in cv_radix.h.
#include <hip/hip_runtime.h>

#include <string>

#include "cv_host.h"
#include "cv_radix.h"

namespace cv {

namespace {

// status word: [flag:2 | tag:6 | value:56]; the tag (pass + 1) lets all passes
// of one sort share one status array cleared once per sort.
__device__ __forceinline__ u64 rs_word(u64 flag, u32 tag, u64 v) { return (flag << 62) | ((u64)tag << 56) | v; }

// Histogram of all digits of all passes.  hist[p * RADIX + d].
__global__ void __launch_bounds__(256) k_radix_hist(const u64* __restrict__ keys, u32 n_max,
                                                    const u32* __restrict__ n_dev, int passes,
                                                    const u32* __restrict__ bits_dev, u32* __restrict__ hist)
{
    __shared__ u32 s_h[MAX_PASSES * RADIX];
    for (int i = threadIdx.x; i < MAX_PASSES * RADIX; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    u32 n = n_dev ? *n_dev : n_max;
    int np = passes;
    if (bits_dev) {
        int b = (int)*bits_dev;
        int need = (b + RADIX_BITS - 1) / RADIX_BITS;
        np = need < np ? need : np;
    }
    // the loop runs the same trips in every lane of a wave (whole waves per
    // stride); a digit shared by every valid lane adds once
    const u32 stride = gridDim.x * blockDim.x;
    const u32 first = blockIdx.x * blockDim.x + (threadIdx.x & ~(u32)(WAVE - 1));
    for (u32 b = first; b < n; b += stride) {
        const u32 i = b + (u32)lane_id();
        const bool ok = i < n;
        const u64 k = ok ? keys[i] : 0ull;
        const u64 vm = __ballot(ok);
        const int lead = __ffsll((long long)vm) - 1;
        for (int p = 0; p < np; ++p) {
            const u32 d = (u32)(k >> (p * RADIX_BITS)) & (RADIX - 1);
            const u32 d0 = __shfl(d, lead, WAVE);
            if (__ballot(ok && d != d0) == 0) {
                if (lane_id() == lead) atomicAdd(&s_h[p * RADIX + d0], (u32)__popcll(vm));
            } else if (ok) {
                atomicAdd(&s_h[p * RADIX + d], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np * RADIX; i += blockDim.x)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// Exclusive scan of each pass's digit counts (one block, a thread per digit).
// With w0 (device, nullable) the counts use the wide layout: the first digit
// has w0 bits (8 or 9) and 512 counters.
__global__ void __launch_bounds__(2 * RADIX) k_radix_scan(const u32* __restrict__ hist, u32* __restrict__ offs,
                                                          int passes, const u32* __restrict__ w0_dev)
{
    __shared__ u32 tmp[2 * RADIX / WAVE];
    const u32 w0 = first_digit_bits(w0_dev);
    for (int p = 0; p < passes; ++p) {
        const u32 bins = 1u << (p == 0 ? w0 : (u32)RADIX_BITS);
        const int base = w0_dev ? hist_wide_off(p) : p * RADIX;
        u32 total;
        const u32 v = threadIdx.x < bins ? hist[base + threadIdx.x] : 0u;
        const u32 e = block_exclusive_sum<2 * RADIX>(v, tmp, total);
        if (threadIdx.x < bins) offs[base + threadIdx.x] = e;
    }
}

// One stable scatter pass on digit `pass`: bits [8*pass, 8*pass+8), or, with
// a first digit of w0 = pack[2] bits (9): [0, w0) for pass 0 and
// [w0 + 8 (pass - 1), w0 + 8 pass) after it.  DB: bits of the digit this
// instantiation handles (8, or 9 for a wide first digit; a launch whose
// width is not the pass's leaves at once).
// vals_in == nullptr means the identity (input index).  LOOP: a block goes on
// taking tiles (a grid smaller than the tile count); otherwise it takes one.
template <int SORT_BLOCK, int SORT_ITEMS, bool LOOP, int DB = RADIX_BITS>
__global__ void __launch_bounds__(SORT_BLOCK)
k_radix_pass(const u64* __restrict__ keys_in, const u32* __restrict__ vals_in, u64* __restrict__ keys_out,
             u32* __restrict__ vals_out, u32 n_max, const u32* __restrict__ n_dev, int pass,
             const u32* __restrict__ bits_dev, const u32* __restrict__ digit_offs, u64* __restrict__ status,
             u32* __restrict__ ticket, const u32* __restrict__ pack)
{
    constexpr int NW = SORT_BLOCK / WAVE;
    constexpr int SORT_TILE = SORT_BLOCK * SORT_ITEMS;
    constexpr int RK = 1 << DB;  // digit values
    static_assert(SORT_BLOCK >= RK, "one thread per digit");
    static_assert(SORT_TILE <= 65535, "16-bit in-tile offsets");
    // per-wave digit counts, then in-tile offsets (< SORT_TILE, so 16 bits)
    __shared__ uint16_t s_whist[NW][RK];
    __shared__ u32 s_start[RK];
    __shared__ u32 s_gshift[RK];
    // staging: keys in digit order; then, in passes that carry index values,
    // the values in the same order (the buffer reused as 32-bit words)
    __shared__ u64 s_keys[SORT_TILE];
    __shared__ u32 s_tmp[NW];
    __shared__ u32 s_tile;

    // the launch's scalars from device memory, all loaded before any is used.
    // packing: from pass p0 on, a key word holds (key >> 8 p0) << ib | index
    // (a wide first digit only with p0 = 0)
    u32 ib = 0, w0r = RADIX_BITS;
    int p0 = 1 << 20;
    if (pack) {
        ib = pack[0];
        p0 = (int)pack[1];
        w0r = pack[2];
    }
    const u32 bits = bits_dev ? *bits_dev : ~0u;
    const u32 n = n_dev ? *n_dev : n_max;
    const int w0 = w0r == RADIX_BITS + 1 ? RADIX_BITS + 1 : RADIX_BITS;
    if ((pass == 0 ? w0 : RADIX_BITS) != DB) return;  // the other width's launch takes this pass
    const int lo = pass == 0 ? 0 : w0 + (pass - 1) * RADIX_BITS;  // the digit's lowest key bit
    if ((u32)lo >= bits) return;
    const bool pin = pass >= p0;           // input words are packed
    const bool pout = pass + 1 >= p0;      // output words are packed
    const int shift = pin ? (int)ib + lo - p0 * RADIX_BITS : lo;
    // this pass's global start of digit threadIdx.x, read before it is needed
    const u32 doff = threadIdx.x < RK ? digit_offs[threadIdx.x] : 0u;
    // Tiles are taken by ticket (with LOOP, until the tickets pass the last
    // tile, so a grid smaller than the tile count covers every tile); a tile
    // waits only on tiles whose tickets were taken before, by blocks already
    // running.
    // A block of a one-tile-per-block grid sized for n_max whose tile lies past
    // a count read on the device leaves before it takes a ticket: exactly the
    // first ceil(n / tile) blocks take the tickets 0 .. ceil(n / tile) - 1,
    // and the idle ones put no load on the ticket counter.
    if (!LOOP && (u64)blockIdx.x * SORT_TILE >= n) return;
    for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    for (int i = threadIdx.x; i < NW * RK; i += SORT_BLOCK) (&s_whist[0][0])[i] = 0;
    __syncthreads();
    const u32 tile = s_tile;
    const u64 tile_base = (u64)tile * SORT_TILE;
    if (tile_base >= n) return;

    const int w = threadIdx.x / WAVE;
    const int l = lane_id();
    u64 key[SORT_ITEMS];
    u32 val[SORT_ITEMS];
    u32 rnk[SORT_ITEMS];
    const u64 wbase = tile_base + (u64)w * (SORT_ITEMS * WAVE);
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
        u64 idx = wbase + (u64)i * WAVE + l;
        bool ok = idx < n;
        key[i] = ok ? keys_in[idx] : ~0ull;
        val[i] = (ok && !pin) ? (vals_in ? vals_in[idx] : (u32)idx) : 0u;
    }
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
        u64 idx = wbase + (u64)i * WAVE + l;
        bool ok = idx < n;
        u32 d = (u32)(key[i] >> shift) & (RK - 1);
        const u64 peers = wave_peers<DB>(d, __ballot(ok));
        u32 below = popc_below(peers);
        u32 cnt = __popcll(peers);
        u32 before = ok ? (u32)s_whist[w][d] : 0u;
        rnk[i] = before + below;
        __builtin_amdgcn_wave_barrier();
        if (ok && below == cnt - 1) s_whist[w][d] = (uint16_t)(before + cnt);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // per digit: exclusive offsets across waves, tile count
    u32 tcount = 0;
    if (threadIdx.x < RK) {
        const int d = threadIdx.x;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            u32 c = s_whist[ww][d];
            s_whist[ww][d] = (uint16_t)tcount;
            tcount += c;
        }
    }
    u32 total;
    u32 start = block_exclusive_sum<SORT_BLOCK>(threadIdx.x < RK ? tcount : 0u, s_tmp, total);
    const u32 tag = (u32)pass + 1;
    if (threadIdx.x < RK) {
        s_start[threadIdx.x] = start;
        // this tile's digit count, for the look-back of later tiles
        lb_publish(status + (u64)tile * RK + threadIdx.x, rs_word(tile == 0 ? 2 : 1, tag, tcount));
    }
    __syncthreads();

    // keys to LDS in digit order (stable); the look-back below overlaps with
    // the other threads' staging
    u32 pos[SORT_ITEMS];
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i) {
        u64 idx = wbase + (u64)i * WAVE + l;
        pos[i] = ~0u;
        if (idx < n) {
            u32 d = (u32)(key[i] >> shift) & (RK - 1);
            pos[i] = s_start[d] + s_whist[w][d] + rnk[i];
            s_keys[pos[i]] = key[i];
        }
    }
    if (threadIdx.x < RK) {
        const int d = threadIdx.x;
        // look-back for digit d over earlier tiles of this pass
        u64 excl = 0;
        if (tile != 0) {
            // LBW tiles at a time (their status words read together): take
            // aggregates in order up to the first inclusive prefix; stop early
            // at a tile that has not published yet and read again from it
            constexpr int LBW = 4;
            long t = (long)tile - 1;
            bool done = false;
            while (!done) {
                u64 wv[LBW];
#pragma unroll
                for (int j = 0; j < LBW; ++j)
                    wv[j] = t - j >= 0 ? lb_peek(status + (u64)(t - j) * RK + d) : 0ull;
                int used = 0;
#pragma unroll
                for (int j = 0; j < LBW; ++j) {
                    if (done || used < j) break;  // stopped earlier in this batch
                    const u32 hdr = (u32)(wv[j] >> 56);
                    if (t - j < 0 || (hdr & 63u) != tag) break;
                    excl += wv[j] & ((1ull << 56) - 1);
                    used = j + 1;
                    if ((hdr >> 6) == 2u) done = true;
                }
                t -= used;
                if (!done && used < LBW) __builtin_amdgcn_s_sleep(1);
            }
            lb_publish(status + (u64)tile * RK + d, rs_word(2, tag, excl + tcount));
        }
        s_gshift[d] = doff + (u32)excl - start;
    }
    __syncthreads();
    const u32 tvalid = (u32)((n - tile_base) < (u64)SORT_TILE ? (n - tile_base) : (u64)SORT_TILE);
    // read back the staged keys this thread writes out: positions t + k * SORT_BLOCK
    u64 kk[SORT_ITEMS];
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        const u32 j = threadIdx.x + (u32)k * SORT_BLOCK;
        kk[k] = j < tvalid ? s_keys[j] : 0ull;
    }
    if (pin) {
#pragma unroll
        for (int k = 0; k < SORT_ITEMS; ++k) {
            const u32 j = threadIdx.x + (u32)k * SORT_BLOCK;
            if (j < tvalid) keys_out[s_gshift[(u32)(kk[k] >> shift) & (RK - 1)] + j] = kk[k];
        }
        if constexpr (!LOOP) return;
        __syncthreads();  // LDS free for the next tile
        continue;
    }
    // the index values follow the keys through the same staging buffer
    __syncthreads();
    u32* s_vals = (u32*)s_keys;
#pragma unroll
    for (int i = 0; i < SORT_ITEMS; ++i)
        if (pos[i] != ~0u) s_vals[pos[i]] = val[i];
    __syncthreads();
    // the pass that starts packing packs on the way out
    const int drop = p0 * RADIX_BITS;
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        const u32 j = threadIdx.x + (u32)k * SORT_BLOCK;
        if (j < tvalid) {
            const u32 g = s_gshift[(u32)(kk[k] >> shift) & (RK - 1)] + j;
            const u32 v = s_vals[j];
            if (pout) {
                keys_out[g] = ((drop >= 64 ? 0ull : (kk[k] >> drop)) << ib) | (u64)v;
            } else {
                keys_out[g] = kk[k];
                vals_out[g] = v;
            }
        }
    }
    if constexpr (!LOOP) return;
    __syncthreads();  // LDS free for the next tile
    }
}


}  // namespace

void radix_hist(const u64* keys, u32 n_max, const u32* n_dev, int passes, const u32* bits_dev, u32* hist,
                int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_radix_hist, dim3(grid), dim3(256), 0, s, keys, n_max, n_dev, passes, bits_dev, hist);
}

void radix_scan(const u32* hist, u32* offs, int passes, hipStream_t s, const u32* w0_dev)
{
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(2 * RADIX), 0, s, hist, offs, passes, w0_dev);
}

namespace {

// A pass whose record count is read on the device launches one block per
// tile of n_max (the blocks past the count leave at once) up to
// DEVICE_COUNT_MAX_TILES tiles; beyond that, DEVICE_COUNT_GRID blocks that
// loop over tiles (a form that needs more registers, so fewer blocks per CU).
constexpr u64 DEVICE_COUNT_GRID = 2048;
constexpr u64 DEVICE_COUNT_MAX_TILES = 1ull << 17;

// tile shapes compiled into the library; the sort uses sort_shape()
struct Shape {
    int block, items;
};
// (every shape has at least one thread per digit)
constexpr Shape SHAPES[] = {{256, 16}, {256, 32}, {512, 8}, {512, 16}, {1024, 8}, {1024, 16}};
constexpr int N_SHAPES = sizeof(SHAPES) / sizeof(SHAPES[0]);
int g_shape = 0;
bool g_wide_first = true;  // tuning "radix_wide_first"

template <int B, int I, int DB = RADIX_BITS>
void launch_pass(u64 tiles, hipStream_t s, const u64* kin, const u32* vin, u64* kout, u32* vout, u32 n_max,
                 const u32* n_dev, int p, const u32* bits_dev, const u32* offs, u64* status, u32* ticket,
                 const u32* pack)
{
    // a count known only on the device and a very large bound: a grid that
    // fills the GPU, whose blocks take tiles until the count is covered
    if (n_dev && tiles > DEVICE_COUNT_MAX_TILES)
        hipLaunchKernelGGL((k_radix_pass<B, I, true, DB>), dim3((unsigned)DEVICE_COUNT_GRID), dim3(B), 0, s, kin,
                           vin, kout, vout, n_max, n_dev, p, bits_dev, offs, status, ticket, pack);
    else
        hipLaunchKernelGGL((k_radix_pass<B, I, false, DB>), dim3((unsigned)(tiles ? tiles : 1)), dim3(B), 0, s, kin,
                           vin, kout, vout, n_max, n_dev, p, bits_dev, offs, status, ticket, pack);
}

}  // namespace

int sort_shape_count() { return N_SHAPES; }
int sort_shape() { return g_shape; }
bool set_sort_shape(int i)
{
    if (i < 0 || i >= N_SHAPES) return false;
    g_shape = i;
    return true;
}
int sort_tile(int i) { return SHAPES[i].block * SHAPES[i].items; }
int sort_block(int i) { return SHAPES[i].block; }
bool sort_wide_first() { return g_wide_first && SHAPES[g_shape].block >= 2 * RADIX; }
int sort_min_tile()
{
    int m = sort_tile(0);
    for (int i = 1; i < N_SHAPES; ++i) m = sort_tile(i) < m ? sort_tile(i) : m;
    return m;
}

void radix_passes(u64* k0, u64* k1, const u32* v_first, u32* v0, u32* v1, u32 n_max, const u32* n_dev,
                  const u32* bits_dev, int passes, const u32* offs, u64* status, u32* tickets, hipStream_t s,
                  bool timed, const u32* pack, const u32* w0_dev)
{
    static const char* const names[MAX_PASSES] = {"sort_pass0", "sort_pass1", "sort_pass2", "sort_pass3",
                                                  "sort_pass4", "sort_pass5", "sort_pass6", "sort_pass7"};
    const int sh = g_shape;
    const u64 tile = (u64)sort_tile(sh);
    // the kernels read the first digit's width with the packing words
    if (w0_dev && w0_dev != pack + 2) return;  // (the record sort keeps them adjacent)
    const u64 tiles = ((u64)n_max + tile - 1) / tile;
    for (int p = 0; p < passes; ++p) {
        const u64* kin = (p & 1) ? k1 : k0;
        const u32* vin = p == 0 ? v_first : ((p & 1) ? v1 : v0);
        u64* kout = (p & 1) ? k0 : k1;
        u32* vout = (p & 1) ? v0 : v1;
        cvh::TimedScope ts_(timed ? names[p] : nullptr, s);
        const u32* o = offs + (w0_dev ? hist_wide_off(p) : p * RADIX);
        auto go = [&](auto launch) {
            launch(tiles, s, kin, vin, kout, vout, n_max, n_dev, p, bits_dev, o, status, tickets + p, pack);
        };
        // the first pass of a sort that may take a 9-bit first digit: both
        // widths are launched, and the one that is not the pass's leaves at once
        // (shapes below 512 threads have no 9-bit form; the sort then keeps 8)
        const bool wide = w0_dev && p == 0;
        switch (sh) {
        case 0: go(launch_pass<256, 16>); break;
        case 1: go(launch_pass<256, 32>); break;
        case 2:
            if (wide) go(launch_pass<512, 8, RADIX_BITS + 1>);
            go(launch_pass<512, 8>);
            break;
        case 3:
            if (wide) go(launch_pass<512, 16, RADIX_BITS + 1>);
            go(launch_pass<512, 16>);
            break;
        case 4:
            if (wide) go(launch_pass<1024, 8, RADIX_BITS + 1>);
            go(launch_pass<1024, 8>);
            break;
        default:
            if (wide) go(launch_pass<1024, 16, RADIX_BITS + 1>);
            go(launch_pass<1024, 16>);
            break;
        }
    }
}

}  // namespace cv

namespace cv {
}  // namespace cv

extern "C" {

cv_status cv_tuning_set(const char* name, int64_t value)
{
    if (!name) return CV_ERR_INVALID_ARGUMENT;
    const std::string n(name);
    // range-checked as int64 before the narrowing, so 2^32 + i is not shape i
    if (n == "sort_shape")
        return value >= 0 && value < cv::sort_shape_count() && cv::set_sort_shape((int)value)
                   ? CV_OK
                   : CV_ERR_INVALID_ARGUMENT;
    if (n == "radix_wide_first") {
        if (value != 0 && value != 1) return CV_ERR_INVALID_ARGUMENT;
        cv::g_wide_first = value != 0;
        return CV_OK;
    }
    return CV_ERR_INVALID_ARGUMENT;
}

cv_status cv_tuning_get(const char* name, int64_t* value)
{
    if (!name || !value) return CV_ERR_INVALID_ARGUMENT;
    const std::string n(name);
    if (n == "sort_shape") *value = cv::sort_shape();
    else if (n == "sort_shapes") *value = cv::sort_shape_count();
    else if (n == "sort_tile") *value = cv::sort_tile(cv::sort_shape());
    else if (n == "sort_block") *value = cv::sort_block(cv::sort_shape());
    else if (n == "radix_bits") *value = cv::RADIX_BITS;
    else if (n == "radix_wide_first") *value = cv::g_wide_first ? 1 : 0;
    else return CV_ERR_INVALID_ARGUMENT;
    return CV_OK;
}

}  // extern "C"
