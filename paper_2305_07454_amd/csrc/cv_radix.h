// cv_radix.h -- stable LSD radix sort of (u64 key, u32 value) pairs for gfx950.
//
// One up-front histogram pass computes the digit counts of every pass (the
// multiset of a key digit does not change under permutation).  Each scatter
// pass then reads a tile of keys once:
//   1. wave64 multisplit: per key, 8 ballots give the mask of lanes holding the
//      same 8-bit digit; the rank inside the wave is the popcount of that mask
//      below the lane plus the wave's running count of the digit (LDS);
//   2. per-digit exclusive offsets across the block's waves, and the tile's
//      digit histogram;
//   3. decoupled look-back over earlier tiles, one thread per digit, gives the
//      tile's global offset of every digit;
//   4. keys are staged in LDS in tile-sorted order and written out so that
//      consecutive threads write consecutive addresses of each digit run.
// Stability holds because every step orders by (wave, item, lane), which is
// the input order of the tile.  The record sort may take its first digit 9
// bits wide (9 ballots, 512 counters and look-back words) when that saves a
// pass; every other digit has 8 bits.
#pragma once
#include "cv_device.h"

namespace cv {

constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int MAX_PASSES = 8;

// A sort may take its first digit 9 bits wide where that saves a pass (a key
// of 8k + 1 bits).  Its digit counts then use the wide layout: the first
// digit's 512 counters, then 256 per later digit.
constexpr int HIST_WIDE_WORDS = (MAX_PASSES + 1) * RADIX;
__host__ __device__ constexpr int hist_wide_off(int p) { return p ? (p + 1) * RADIX : 0; }
// bits of the first digit: *w0 (device, nullable) when it is 9, else 8
__device__ __forceinline__ u32 first_digit_bits(const u32* w0) { return (w0 && *w0 == RADIX_BITS + 1) ? RADIX_BITS + 1 : RADIX_BITS; }

// Tile shapes (threads per block x keys per thread) compiled into the library.
// The sort launches the selected one; workspaces are sized for the smallest
// tile so any shape fits.
int sort_shape_count();
int sort_shape();
bool set_sort_shape(int i);
int sort_tile(int i);
int sort_block(int i);
int sort_min_tile();
// whether the selected shape has a 9-bit first-digit pass (512 threads or
// more) and the tuning allows it
bool sort_wide_first();

// Host launchers (defined in cv_radix.hip).
//   radix_hist : digit histograms of `passes` passes (limited on device by
//                ceil(*bits_dev / 8) when bits_dev is given) added into hist.
//   radix_scan : per-pass exclusive scan hist -> offs.
//   radix_passes: up to `passes` stable scatter passes, ping-pong k0 -> k1 -> k0
//                ...; pass p is skipped on device when 8p >= *bits_dev.  vals of
//                pass 0 come from v_first (nullptr = identity).  After p passes
//                the data sits in (k1, v1) when p is odd, in (k0, v0) when even.
void radix_hist(const u64* keys, u32 n_max, const u32* n_dev, int passes, const u32* bits_dev, u32* hist,
                int grid, hipStream_t s);
void radix_scan(const u32* hist, u32* offs, int passes, hipStream_t s, const u32* w0_dev = nullptr);
//                When `timed`, pass p is bracketed as timing family "sort_pass<p>".
//                pack [device, 3] (nullable): {ib, p0, w0}: from pass p0 on,
//                key words hold (key >> 8 p0) << ib | index and no value
//                arrays are used (p0 = 0: the input keys are packed
//                already); w0 is the first digit's width (8 or 9).
//                w0_dev [device] (nullable): bits of the first digit (8 or
//                9; 9 only with p0 = 0), the word after pack's two; offs then
//                use the wide layout and status holds 512 words per tile.
void radix_passes(u64* k0, u64* k1, const u32* v_first, u32* v0, u32* v1, u32 n_max, const u32* n_dev,
                  const u32* bits_dev, int passes, const u32* offs, u64* status, u32* tickets, hipStream_t s,
                  bool timed = false, const u32* pack = nullptr, const u32* w0_dev = nullptr);

}  // namespace cv
