/*
 * cvetl.h -- C ABI of the MI355X (gfx950) connected-vehicle ETL core.
 *
 * The paper this implements ("Accelerating Statewide Connected Vehicles Big
 * (Sensor Fusion) Data ETL Pipelines on GPUs", Methods: "Accelerated ETL
 * Algorithm/Framework for Spatio-Temporal CV Data", steps (2)-(6), and
 * Algorithm 2) turns raw per-vehicle sensor records into an index over unique
 * journeys and a spatio-temporal lattice of per-cell reductions.  This library
 * exposes that data-parallel core as four stream-ordered calls:
 *
 *   cv_sort_records      order records by (journey id, timestamp)  [step (2): unique index]
 *   cv_journey_features  per-point kinematics inside each journey  [sensor fields of the dataset]
 *   cv_journey_summary   one summary row per journey               [unique journeys, Abstract/Discussion]
 *   cv_grid_aggregate    (time bin x lat bin x lon bin) aggregates [steps (3)-(5), Algorithm 2, Table 3 reductions]
 *
 * Conventions for every call
 * --------------------------
 * - All array pointers are DEVICE pointers unless marked [host].  Structs passed
 *   by pointer (cv_records, cv_features, ...) live in host memory and are read
 *   before the call returns.
 * - Every call only enqueues kernels on `stream` (a hipStream_t; NULL = the
 *   default stream).  It never synchronises and never allocates: scratch
 *   memory comes from the caller's workspace `ws` of `ws_bytes` bytes, whose
 *   required size the matching *_workspace_size() call returns.  The
 *   workspace must be 256-byte aligned and must not be shared by calls that
 *   may run concurrently.
 * - The caller owns all memory.  Outputs must not alias inputs.
 * - Argument errors are returned synchronously as a cv_status and nothing is
 *   enqueued.  Conditions only the device can see (output capacity exceeded,
 *   key range too wide) are written to the caller's device-resident cv_result
 *   (`res`, may be NULL when the caller does not need it) by the last kernel
 *   of the call; read it after synchronising the stream.
 * - n == 0 is valid and produces empty outputs.  n must be < 2^32.
 * - Floating-point results are deterministic: every sum is accumulated exactly
 *   in fixed point (integer adds are order-independent) and rounded once.
 */
#ifndef CVETL_H
#define CVETL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CV_ABI_VERSION 1u

typedef enum {
    CV_OK = 0,
    CV_ERR_INVALID_ARGUMENT = 1, /* null pointer, bad size or bad grid spec           */
    CV_ERR_WORKSPACE = 2,        /* ws NULL, misaligned or smaller than required       */
    CV_ERR_CAPACITY = 3,         /* (device) output rows exceed capacity; see required */
    CV_ERR_RANGE = 4,            /* packed key or lattice index would overflow         */
    CV_ERR_DEVICE = 5,           /* a HIP launch or runtime call failed                */
    CV_ERR_UNSUPPORTED = 6       /* no gfx950 device / feature not available           */
} cv_status;

/* Raw sensor records, structure of arrays (Table 1's columns used by the path). */
typedef struct {
    const int64_t* journey_id; /* opaque journey id mapped to int64 by the caller      */
    const int64_t* ts_ms;      /* sample time, integer milliseconds                    */
    const double* lat_deg;     /* WGS84 latitude, degrees                              */
    const double* lon_deg;     /* WGS84 longitude, degrees                             */
    const float* speed_mps;    /* sensor speed; finite, |speed| < 1024                 */
    uint64_t n;                /* number of records, < 2^32                            */
} cv_records;

/* Output columns of the sort: the input columns permuted into sorted order. */
typedef struct {
    int64_t* journey_id;
    int64_t* ts_ms;
    double* lat_deg;
    double* lon_deg;
    float* speed_mps;
} cv_records_out;

/* Per-point kinematics; every array has n elements (one per sorted record). */
typedef struct {
    double* step_m;       /* haversine distance from the predecessor, metres       */
    double* dt_s;         /* time since the predecessor, seconds                   */
    double* speed_mps;    /* step_m / dt_s when dt > 0                             */
    double* accel_mps2;   /* backward difference of speed_mps over dt_s            */
    double* bearing_deg;  /* initial great-circle course, [0, 360)                 */
    double* dheading_deg; /* bearing change, (-180, 180]                           */
    uint8_t* flags;       /* CV_FLAG_* bits                                        */
} cv_features;

#define CV_FLAG_FIRST 0x01u      /* first record of its journey                 */
#define CV_FLAG_DT_ZERO 0x02u    /* same timestamp as the predecessor           */
#define CV_FLAG_SPEED_OK 0x04u   /* speed_mps defined                           */
#define CV_FLAG_ACCEL_OK 0x08u   /* accel_mps2 defined                          */
#define CV_FLAG_BEARING_OK 0x10u /* bearing_deg defined (non-zero step)         */
#define CV_FLAG_DHEAD_OK 0x20u   /* dheading_deg defined                        */
#define CV_FLAG_BAD_COORD 0x40u  /* non-finite coordinate here or predecessor   */

/* One row per journey, ascending journey id; each array has `capacity` rows. */
typedef struct {
    int64_t* journey_id;
    uint32_t* first;             /* index of the journey's first sorted record      */
    uint32_t* n_points;
    int64_t* t_start_ms;
    int64_t* t_end_ms;
    double* distance_m;          /* exact-rounded sum of step_m                     */
    double* sum_speed;           /* exact-rounded sum of the sensor speed           */
    float* max_speed;            /* max sensor speed (-0 as +0)                     */
    double* max_derived_speed;   /* max speed_mps over SPEED_OK points, else 0      */
    uint32_t* n_dt_zero;         /* number of DT_ZERO points                        */
    double* lat_min;             /* bounding box over points with finite lat & lon  */
    double* lat_max;             /*   (+inf / -inf when there is none)              */
    double* lon_min;
    double* lon_max;
} cv_journeys;

/* Binning parameters of Algorithm 2: lat_bin = floor((lat - lat0) / dlat) etc. */
typedef struct {
    double lat0_deg, lon0_deg; /* grid origin (south-west corner)                   */
    double dlat_deg, dlon_deg; /* cell size, > 0                                    */
    int64_t n_lat, n_lon;      /* cells per axis, > 0                               */
    int64_t t0_ms;             /* start of time bin 0                               */
    int64_t bin_ms;            /* time-bin width, > 0                               */
    int64_t n_t;               /* number of time bins; <= 0 means unbounded         */
} cv_grid_spec;

/* One row per occupied (time bin, cell) key, ascending key. */
typedef struct {
    int64_t* key;         /* (tbin * n_lat + ilat) * n_lon + ilon               */
    uint32_t* count;      /* records in the cell                                */
    uint32_t* n_journeys; /* distinct journey ids in the cell                   */
    double* sum_speed;    /* exact-rounded sum of speed (mean = sum / count)    */
    float* min_speed;     /* -0 as +0                                           */
    float* max_speed;
} cv_groups;

/* Device-resident result word written by the last kernel of a call. */
typedef struct {
    uint32_t status;        /* cv_status of the device-side checks              */
    uint32_t flags;         /* sort call: bits of the first radix digit (8, or
                               9 where a key of 8k + 1 bits saves a pass);
                               other calls: 0 unless documented there         */
    uint64_t count;         /* rows produced (journeys / groups)                */
    uint64_t required;      /* capacity needed when status == CV_ERR_CAPACITY   */
    uint64_t n_out_of_grid; /* records outside the grid (grid call)             */
    uint64_t n_late;        /* reserved for streaming, 0                        */
    uint64_t key_bits;      /* bits of the packed sort key (sort call)          */
    uint64_t packed_pass;   /* sort call: first radix pass that moves one word
                               (key high digits | record index) per record    */
    uint64_t n_bad;         /* csv call: malformed rows (else 0)                */
} cv_result;

uint32_t cv_abi_version(void);
const char* cv_strerror(cv_status s);

/* ------------------------------------------------------------------------
 * cv_sort_records -- stable order of the records by (journey_id, ts_ms), both
 * compared as signed 64-bit integers, ties in input order (the paper's unique
 * index over all journeys, Methods step (2)).
 *   in            [host struct] input columns (device arrays), n records.
 *   max_journeys  capacity of the journey dictionary (distinct journey ids);
 *                 more distinct ids set res->status = CV_ERR_CAPACITY and
 *                 res->required to a lower bound of the distinct count.
 *   perm          [device, n] out: perm[k] = input index of the k-th record.
 *   sorted        [host struct, nullable] out columns; any member may be NULL.
 *   res           [device, nullable] out: status, count = distinct journeys,
 *                 key_bits = bits of the packed (journey rank, time) key;
 *                 status CV_ERR_RANGE if that key would exceed 64 bits.
 *   ws, ws_bytes  workspace of at least cv_sort_workspace_size(n, max_journeys).
 * --------------------------------------------------------------------- */
cv_status cv_sort_workspace_size(uint64_t n, uint64_t max_journeys, size_t* bytes /*[host]*/);
cv_status cv_sort_records(const cv_records* in, uint64_t max_journeys, uint32_t* perm,
                          const cv_records_out* sorted, cv_result* res, void* ws, size_t ws_bytes,
                          void* stream);

/* ------------------------------------------------------------------------
 * cv_journey_features -- per-point kinematics of records already in
 * (journey, time) order.  For record k with predecessor p = k-1 in the same
 * journey: dt_s = (ts[k]-ts[p])/1000; step_m = haversine distance on a sphere
 * of radius 6371008.8 m; speed = step/dt when dt > 0; accel = (speed[k] -
 * speed[p]) / dt when both speeds are defined; bearing = initial course from p
 * to k when the step is non-zero; dheading = bearing[k] - bearing[p] wrapped
 * into (-180, 180] when both are defined.  The first record of a journey and
 * records with a non-finite coordinate at k or p get all-zero values and the
 * FIRST / BAD_COORD flags.  No workspace.
 * --------------------------------------------------------------------- */
cv_status cv_journey_features(const cv_records* sorted, const cv_features* out, void* stream);

/* ------------------------------------------------------------------------
 * cv_sort_records_features / cv_batch_sort_records_features -- the sort
 * (cv_sort_records / cv_batch_sort_records) and the kinematics of the sorted
 * records (cv_journey_features / cv_batch_journey_features) in one call:
 * the gather writes each tile of sorted records and evaluates their
 * kinematics from LDS, so the sorted columns are not read back.  Every
 * output is bit for bit that of the two calls.  `sorted` and `feat` must
 * name every column.  Workspace as cv_sort_workspace_size (which includes
 * room for the payload packed per record: when the input's runs of equal
 * journey ids are short, as in a time-ordered feed, time, lat, lon and speed
 * are first packed into one 32-byte record per input record, so the gather
 * reads one record instead of four scattered columns).
 * --------------------------------------------------------------------- */
cv_status cv_sort_records_features(const cv_records* in, uint64_t max_journeys, uint32_t* perm,
                                   const cv_records_out* sorted, const cv_features* feat, cv_result* res, void* ws,
                                   size_t ws_bytes, void* stream);
cv_status cv_batch_sort_records_features(const cv_records* in, const uint64_t* shard_offsets, uint32_t n_shards,
                                         uint64_t max_journeys, uint32_t* perm, const cv_records_out* sorted,
                                         const cv_features* feat, cv_result* res, void* ws, size_t ws_bytes,
                                         void* stream);

/* ------------------------------------------------------------------------
 * cv_journey_summary -- one row per journey (maximal run of equal journey_id)
 * of sorted records, in ascending journey id, from the records and their
 * features (step_m, speed_mps and flags are read; `feat` must be the features
 * of these records as cv_journey_features computes them: the FIRST flags
 * mark the journeys' first records, which delimit the sums).  Rows past `capacity` are
 * not written; then res->status = CV_ERR_CAPACITY, res->required = journeys.
 * res->count = number of journeys.
 * --------------------------------------------------------------------- */
cv_status cv_summary_workspace_size(uint64_t n, uint64_t capacity, size_t* bytes /*[host]*/);
cv_status cv_journey_summary(const cv_records* sorted, const cv_features* feat,
                             const cv_journeys* out, uint64_t capacity, cv_result* res, void* ws,
                             size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * cv_journey_summary_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): cv_journey_summary with the same arguments, outputs and device
 * result, minus the workspace.  The workspace is a library-owned device array
 * of CV_NOALLOC_SCRATCH_BYTES bytes; each GPU the library runs on holds its
 * own copy until the process ends.  The call allocates nothing.
 *   Limit: cv_summary_workspace_size(n, capacity) must not exceed
 *   CV_NOALLOC_SCRATCH_BYTES (about 152 bytes per row of min(n, capacity)
 *   plus a few bytes per 4096 records: some 200 000 journey rows), else
 *   CV_ERR_WORKSPACE and nothing is enqueued.
 *   The stream must belong to the current device.  CV_ERR_DEVICE when the
 *   array's device address cannot be obtained.
 *   Every call on one GPU uses that GPU's single array, and each call
 *   rewrites what it reads there (nothing carries over from an earlier call).
 *   Calls that may overlap on one GPU race: issue them on one stream, or
 *   serialise them.
 * --------------------------------------------------------------------- */
#define CV_NOALLOC_SCRATCH_BYTES (32u << 20)
cv_status cv_journey_summary_noalloc(const cv_records* sorted, const cv_features* feat, const cv_journeys* out,
                                     uint64_t capacity, cv_result* res, void* stream);

/* ------------------------------------------------------------------------
 * cv_grid_aggregate -- spatio-temporal lattice of Algorithm 2 and Methods
 * steps (3)-(5) over sorted records.  ilat = floor((lat - lat0)/dlat) and ilon
 * likewise (one IEEE subtraction, one IEEE division, floor), tbin =
 * floor((ts - t0)/bin_ms) in integers; a record is in the grid when both
 * coordinates are finite, 0 <= ilat < n_lat, 0 <= ilon < n_lon, tbin >= 0 and
 * tbin < n_t (n_t > 0) or the key fits in int64 (n_t <= 0).  Per key:
 * count, distinct journeys, exact-rounded speed sum, min and max speed; rows
 * in ascending key.  `capacity` bounds the rows written; more groups set
 * res->status = CV_ERR_CAPACITY with res->required = groups (the rows below
 * capacity are written either way).  res->count = groups, res->n_out_of_grid
 * = records outside the grid.  The workspace depends on n alone (about 64
 * bytes per record: each tile of sorted records leaves at most one partial
 * row per record, which a key sort merges into the group rows), so any
 * capacity < 2^32 fits it.
 * --------------------------------------------------------------------- */
cv_status cv_grid_workspace_size(uint64_t n, const cv_grid_spec* grid /*[host]*/, uint64_t capacity,
                                 size_t* bytes /*[host]*/);
cv_status cv_grid_aggregate(const cv_records* sorted, const cv_grid_spec* grid /*[host]*/,
                            const cv_groups* out, uint64_t capacity, cv_result* res, void* ws,
                            size_t ws_bytes, void* stream);
/* cv_grid_aggregate_flags -- the same call with the journey starts taken from
 *   flags [device, n]: the flags column of cv_journey_features for the same
 *   sorted records (CV_FLAG_FIRST marks each journey's first record).  The
 *   tile kernel then reads one byte per record instead of comparing each
 *   journey id with its predecessor's; outputs and workspace are those of
 *   cv_grid_aggregate.  flags NULL with n > 0: CV_ERR_INVALID_ARGUMENT. */
cv_status cv_grid_aggregate_flags(const cv_records* sorted, const uint8_t* flags, const cv_grid_spec* grid /*[host]*/,
                                  const cv_groups* out, uint64_t capacity, cv_result* res, void* ws, size_t ws_bytes,
                                  void* stream);

/* ------------------------------------------------------------------------
 * cv_grid_aggregate_dir -- the lattice with the direction dimension of
 * Algorithm 2 (a direction bin by floor division of the heading by a sector
 * width) and of the transformed-data output (speeds and volumes per
 * cardinal direction, 8 channels per time bin).  n_dir sectors (1..64) of
 * width 360/n_dir degrees; a record's sector is
 *   floor((h + dir_offset_deg) / (360 / n_dir)) mod n_dir   for h in [0, 360)
 * (dir_offset_deg in [0, 360): 0 bins the heading literally, 45 with n_dir 4
 * centres the sectors on N, E, S, W), and n_dir for a record without a
 * direction (NaN or a heading outside [0, 360), or a derived bearing without
 * CV_FLAG_BEARING_OK).  h is heading_deg[k] [device, float, sorted order;
 * see cv_gather_column] when given, else feat->bearing_deg with feat->flags
 * (cv_journey_features of the same sorted records).  Keys are
 *   ((tbin * (n_dir + 1) + sector) * n_lat + ilat) * n_lon + ilon
 * and everything else is as cv_grid_aggregate (same workspace size).
 * CV_ERR_RANGE when n_t * n_lat * n_lon * (n_dir + 1) does not fit in int64.
 * --------------------------------------------------------------------- */
cv_status cv_grid_aggregate_dir(const cv_records* sorted, const float* heading_deg, const cv_features* feat,
                                const cv_grid_spec* grid /*[host]*/, uint32_t n_dir, double dir_offset_deg,
                                const cv_groups* out, uint64_t capacity, cv_result* res, void* ws,
                                size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * cv_gather_column -- out[k] = in[perm[k]] for k < n: a payload column that
 * the sort does not carry (a sensor heading, say) brought into the sorted
 * order.  in, out [device], elem_bytes 4 or 8, aligned to it; perm [device]
 * is the permutation of [0, n) written by cv_sort_records for the same n
 * (an index >= n reads element n - 1).
 * --------------------------------------------------------------------- */
cv_status cv_gather_column(const void* in, const uint32_t* perm, void* out, uint64_t n, uint32_t elem_bytes,
                           void* stream);

/* ------------------------------------------------------------------------
 * Dense lattice, normalisation and filter (Methods steps (4)-(6); Table 2's
 * speed normalisation, volume normalisation and volume filter rows; the
 * transformed-data output's speed and volume channels per direction and
 * time bin).
 *
 * cv_lattice_dense -- scatter a group table (cv_grid_aggregate or
 *   cv_grid_aggregate_dir with the same grid and n_dir; n_dir = 0 for the
 *   lattice without directions) into lattice [device, float32]
 *   [n_t][C][n_lat][n_lon] for time bins t_first .. t_first + n_t - 1, with
 *   C = 2 D and D = n_dir + 1 (1 when n_dir = 0): channel 2 d is the mean
 *   sensor speed of sector d (sum_speed / count, in double, rounded to
 *   float), channel 2 d + 1 its distinct journeys (the volume).  Cells
 *   without a group are 0; groups of other time bins are skipped.  The whole
 *   tensor is written.
 * cv_lattice_normalize -- in place, per channel over all n_t time bins:
 *   an occupied cell (volume > 0) becomes (x - min) / (max - min) with min
 *   and max over the channel's occupied cells (in double, rounded to float;
 *   0 when max == min); empty cells stay 0.  channel_min_max [device,
 *   2 C floats] receives each channel's min and max (NaN for a channel with
 *   no occupied cell).  A workspace of cv_lattice_normalize_workspace_size
 *   bytes (256-byte aligned) holds per-block partials.
 * cv_groups_filter -- index [device, uint32] of the groups, in ascending
 *   order, whose distinct journeys are >= min_volume and whose mean speed
 *   (sum_speed / count) lies in [speed_lo, speed_hi]; res->count = groups
 *   kept; more than `capacity` sets CV_ERR_CAPACITY with res->required.  A
 *   workspace of cv_groups_filter_workspace_size bytes (256-byte aligned).
 * --------------------------------------------------------------------- */
cv_status cv_lattice_dense(const cv_groups* groups, uint64_t n_groups, const cv_grid_spec* grid /*[host]*/,
                           uint32_t n_dir, int64_t t_first, uint64_t n_t, float* lattice, void* stream);
cv_status cv_lattice_normalize_workspace_size(uint64_t n_t, const cv_grid_spec* grid /*[host]*/, uint32_t n_dir,
                                              size_t* bytes /*[host]*/);
cv_status cv_lattice_normalize(float* lattice, uint64_t n_t, const cv_grid_spec* grid /*[host]*/, uint32_t n_dir,
                               float* channel_min_max, void* ws, size_t ws_bytes, void* stream);
cv_status cv_groups_filter_workspace_size(uint64_t n_groups, size_t* bytes /*[host]*/);
cv_status cv_groups_filter(const cv_groups* groups, uint64_t n_groups, double min_volume, double speed_lo,
                           double speed_hi, uint32_t* index, uint64_t capacity, cv_result* res, void* ws,
                           size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Record hygiene (optional passes on sorted records; both change what the
 * later calls see, so they are opt-in).  Workspace: cv_hygiene_workspace_size
 * bytes (256-byte aligned).
 *
 * cv_drop_duplicates -- keep a sorted record unless an earlier record of the
 *   same (journey_id, ts_ms) has bit-identical lat_deg, lon_deg and
 *   speed_mps (an exact duplicate row, as Table 1's first and fourth rows):
 *   the kept records, in order, to `out` [device, capacity n]; perm_out
 *   [device, nullable] receives perm [device] of the kept ones (the input
 *   positions).  res->count = records kept.
 * cv_split_trips -- trips of sorted records: a trip starts at a journey's
 *   first record and at a record more than gap_ms (>= 0) after the one
 *   before.  trip_id [device, n] receives each record's trip number (0, 1,
 *   ... in record order, so it can serve as journey_id of the later calls);
 *   trip_journey [device, capacity] the journey id of each trip.
 *   res->count = trips; more than capacity sets CV_ERR_CAPACITY with
 *   res->required (trip_id is complete either way).
 * --------------------------------------------------------------------- */
cv_status cv_hygiene_workspace_size(uint64_t n, size_t* bytes /*[host]*/);
cv_status cv_drop_duplicates(const cv_records* sorted, const uint32_t* perm, const cv_records_out* out,
                             uint32_t* perm_out, cv_result* res, void* ws, size_t ws_bytes, void* stream);
cv_status cv_split_trips(const cv_records* sorted, int64_t gap_ms, int64_t* trip_id, int64_t* trip_journey,
                         uint64_t capacity, cv_result* res, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * cv_csv_extract -- the extraction ahead of the key prep: text rows shaped
 * as Table 1 (journey id, timestamp, latitude, longitude, postal code,
 * speed, heading; comma-separated, one row per line, LF or CRLF) into
 * record columns, in row order.  text [device, 16-byte aligned, nbytes];
 * has_header skips the first line.  Fields:
 *   journey id   1..8 bytes below 0x80, packed big-endian into int64 (so
 *                string order is integer order)
 *   timestamp    "YYYY-MM-DD HH:MM:SS" (proleptic Gregorian, UTC) with an
 *                optional fraction of 1-3 digits -> ms since 1970-01-01
 *   lat, lon     plain decimals ([-+]digits[.digits]) whose significant
 *                digits form an integer below 2^53 and with at most 22
 *                fraction digits -> the double nearest the decimal
 *   postal code  skipped
 *   speed        plain decimal as above -> double -> float32
 *   heading      empty (NaN) or a plain decimal -> float32 (heading_deg,
 *                [device, nullable])
 * A row with another shape (field count, quotes, an invalid date, a
 * decimal outside the forms above) is malformed: its columns are 0 / NaN,
 * row_ok[r] = 0 (nullable), and res->n_bad counts it.  res->count = rows
 * (header excluded); rows past `capacity` are counted, not written
 * (CV_ERR_CAPACITY with res->required).  Workspace:
 * cv_csv_workspace_size(nbytes, capacity) bytes, 256-byte aligned.
 * --------------------------------------------------------------------- */
cv_status cv_csv_workspace_size(uint64_t nbytes, uint64_t capacity, size_t* bytes /*[host]*/);
cv_status cv_csv_extract(const char* text, uint64_t nbytes, int32_t has_header, const cv_records_out* out,
                         float* heading_deg, uint8_t* row_ok, uint64_t capacity, cv_result* res, void* ws,
                         size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent problems ("shards", e.g. county-day files of
 * very uneven size) laid out back to back in one record array and processed
 * by the same launches as one batch.  shard_offsets [device, n_shards + 1]:
 * shard s holds records [offsets[s], offsets[s+1]); offsets[0] = 0,
 * offsets[n_shards] = n, non-decreasing (empty shards allowed); the caller
 * guarantees this layout.  Every result equals the plain call applied to each
 * shard on its own: a journey id present in two shards is two journeys,
 * perm and a journey's `first` are shard-relative (they index records within
 * their shard), and outputs are concatenated in shard order.
 *   journey_offsets [device, n_shards + 1] out: shard s owns journey rows
 *                   [journey_offsets[s], journey_offsets[s+1]).
 *   group_offsets   [device, n_shards + 1] out: likewise for group rows; the
 *                   batched grid needs a bounded time axis (n_t > 0) and
 *                   returns CV_ERR_RANGE when shard index and cell key do not
 *                   fit 63 bits together.
 * Workspace sizes are those of the plain calls for the total n.
 * --------------------------------------------------------------------- */
cv_status cv_batch_sort_records(const cv_records* in, const uint64_t* shard_offsets, uint32_t n_shards,
                                uint64_t max_journeys, uint32_t* perm, const cv_records_out* sorted,
                                cv_result* res, void* ws, size_t ws_bytes, void* stream);
cv_status cv_batch_journey_features(const cv_records* sorted, const uint64_t* shard_offsets, uint32_t n_shards,
                                    const cv_features* out, void* stream);
cv_status cv_batch_journey_summary(const cv_records* sorted, const cv_features* feat,
                                   const uint64_t* shard_offsets, uint32_t n_shards, const cv_journeys* out,
                                   uint64_t capacity, uint64_t* journey_offsets, cv_result* res, void* ws,
                                   size_t ws_bytes, void* stream);
cv_status cv_batch_grid_aggregate(const cv_records* sorted, const uint64_t* shard_offsets, uint32_t n_shards,
                                  const cv_grid_spec* grid /*[host]*/, const cv_groups* out, uint64_t capacity,
                                  uint64_t* group_offsets, cv_result* res, void* ws, size_t ws_bytes,
                                  void* stream);

/* ------------------------------------------------------------------------
 * cv_batch_run -- the whole batched path in one call: the sort with the
 * kinematics (cv_batch_sort_records_features), the journey summaries
 * (cv_batch_journey_summary) and the group table (cv_batch_grid_aggregate),
 * enqueued in that order on `stream`, every output as those calls define it.
 *   shard_n_out  [device, n_shards, nullable] out: records outside the grid
 *                per shard.
 *   res          [device, 3 results] out: the sort's, the summary's, the grid's.
 *   ws           one workspace of cv_batch_workspace_size bytes serves all
 *                three stages (they run one after the other).
 * --------------------------------------------------------------------- */
cv_status cv_batch_workspace_size(uint64_t n, uint32_t n_shards, uint64_t max_journeys, uint64_t journey_capacity,
                                  const cv_grid_spec* grid /*[host]*/, uint64_t group_capacity,
                                  size_t* bytes /*[host]*/);
cv_status cv_batch_run(const cv_records* in, const uint64_t* shard_offsets, uint32_t n_shards,
                       const cv_grid_spec* grid /*[host]*/, uint64_t max_journeys, uint32_t* perm,
                       const cv_records_out* sorted, const cv_features* feat, const cv_journeys* journeys,
                       uint64_t journey_capacity, uint64_t* journey_offsets, const cv_groups* groups,
                       uint64_t group_capacity, uint64_t* group_offsets, uint64_t* shard_n_out, cv_result* res,
                       void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Serving form: records arrive in chunks and are pushed in batches (one or
 * more chunks in arrival order); the open journeys (last point, running
 * summary, cells of the open time-bin segment) and the group table stay
 * resident in the caller's device `state` between pushes.
 *
 * Every result equals the plain calls applied to the concatenation of all
 * pushed records in push order (ties in arrival order), provided a journey's
 * timestamps never go backwards across pushes.  A record older than its
 * journey's last pushed record is late: flag CV_FLAG_LATE, all-zero
 * kinematics, counted in its journey's totals and in its cell (never as a new
 * distinct journey), journey state unchanged.  The distinct-journey flag
 * remembers the cells of each open (journey, time-bin) segment: 16 in the
 * journey's row, up to 384 more in an overflow table the row takes from a
 * pool (one table per 64 journeys of max_journeys).  A segment with more
 * cells, or a row that finds the pool empty, sets bit 0 of cv_result.flags
 * (its journey may then be counted more than once in a cell).
 *
 *   cv_stream_state_size  bytes of device state for the capacities (journeys
 *                         ever seen, groups ever seen, records per push).
 *   cv_stream_create      [host out] *out: a host handle over `state` (256-byte
 *                         aligned, caller-owned); initialises it on `stream`.
 *   cv_stream_push        one batch: features of every record written at the
 *                         record's position in the batch (input order); res:
 *                         status, count = journeys in the batch, n_late and
 *                         n_out_of_grid of the batch, flags.
 *   cv_stream_flush       journeys in ascending id (first = position in the
 *                         sorted concatenation) and groups in ascending key;
 *                         res points to two results: res[0] journeys (count,
 *                         totals of late and out-of-grid records), res[1] groups.
 *                         The stream stays usable (flush is a snapshot).
 *   cv_stream_destroy     frees the host handle (the state is the caller's).
 * Pushes and flushes of one stream must be ordered on one HIP stream.  Every
 * int64 journey id is valid, INT64_MIN included (it has a reserved row).
 *
 * Checkpoint / resume of a stream (the paper persists only its transformed
 * output; the resident serving state is this library's own):
 *   cv_stream_snapshot_size  [host out] bytes of a snapshot: a 256-byte header
 *                         plus the resident state (journey table and rows,
 *                         overflow pool, group table with its exact limbs, the
 *                         running totals); it depends on the capacities the
 *                         stream was created with, not on how full it is.
 *   cv_stream_snapshot    copies that state into host_buf [host, >= the size
 *                         above; pinned memory lets the copy run
 *                         asynchronously] in stream order after the pushes
 *                         before it; read host_buf only after synchronising
 *                         `stream`.
 *   cv_stream_restore     replaces the resident state of `st` with a snapshot;
 *                         `st` must have been created with the same grid,
 *                         max_journeys and max_groups (max_batch may differ),
 *                         else CV_ERR_INVALID_ARGUMENT and nothing is
 *                         enqueued.  host_buf must stay unchanged until
 *                         `stream` has passed the copy.  Pushes after a restore
 *                         continue exactly as after the snapshot.
 * --------------------------------------------------------------------- */
#define CV_FLAG_LATE 0x80u /* serving form: record older than its journey's state */
typedef struct cv_stream cv_stream;
cv_status cv_stream_state_size(const cv_grid_spec* grid /*[host]*/, uint64_t max_journeys, uint64_t max_groups,
                               uint64_t max_batch, size_t* bytes /*[host]*/);
cv_status cv_stream_create(const cv_grid_spec* grid /*[host]*/, uint64_t max_journeys, uint64_t max_groups,
                           uint64_t max_batch, void* state, size_t state_bytes, void* stream,
                           cv_stream** out /*[host]*/);
cv_status cv_stream_push(cv_stream* st, const cv_records* batch, const cv_features* feat, cv_result* res,
                         void* stream);
cv_status cv_stream_flush(cv_stream* st, const cv_journeys* journeys, uint64_t journey_capacity,
                          const cv_groups* groups, uint64_t group_capacity, cv_result* res, void* stream);
cv_status cv_stream_snapshot_size(const cv_stream* st, size_t* bytes /*[host]*/);
cv_status cv_stream_snapshot(cv_stream* st, void* host_buf /*[host]*/, size_t bytes, void* stream);
cv_status cv_stream_restore(cv_stream* st, const void* host_buf /*[host]*/, size_t bytes, void* stream);
cv_status cv_stream_destroy(cv_stream* st);

/* ------------------------------------------------------------------------
 * Tuning knobs (process-wide; set by an autotuner, read back by callers).
 *   "sort_shape"   index of the radix-pass tile shape (threads x keys per
 *                  thread) used by every sort; 0 .. "sort_shapes" - 1.
 *   "sort_shapes"  number of compiled shapes (read-only).
 *   "sort_tile"    keys per tile of the current shape (read-only).
 *   "sort_block"   threads per block of the current shape (read-only).
 *   "radix_bits"   bits per radix digit of every sort (read-only).
 *   "radix_wide_first" 1 (default): the record sort takes a 9-bit first
 *                  digit for a key of 8k + 1 bits packed from the first
 *                  pass (shapes of 512 threads or more), one pass fewer;
 *                  0: 8-bit digits only.
 * Unknown names or out-of-range values return CV_ERR_INVALID_ARGUMENT.
 * --------------------------------------------------------------------- */
cv_status cv_tuning_set(const char* name /*[host]*/, int64_t value);
cv_status cv_tuning_get(const char* name /*[host]*/, int64_t* value /*[host]*/);

/* ------------------------------------------------------------------------
 * Per-kernel timing (measurement support).  When enabled, the library brackets
 * every launch of the named kernel family with HIP events on the launch stream
 * and accumulates the elapsed time; cv_timing_read synchronises those events.
 * Families: "sort_prep", "sort_pass0" .. "sort_pass7" (one per radix digit
 * pass of the record sort; a pass whose digit lies above the packed key's
 * width exits at once on the device), "gather", "features", "summary",
 * "grid_agg", "grid_tail".
 * --------------------------------------------------------------------- */
cv_status cv_timing_enable(int on);
cv_status cv_timing_reset(void);
cv_status cv_timing_read(const char* family /*[host]*/, double* total_ms /*[host]*/,
                         uint64_t* launches /*[host]*/);

/* ------------------------------------------------------------------------
 * Checking build.  A library compiled with CVETL_DEBUG (libcvetl_debug.so)
 * runs small checker kernels after each stage; a failed check sets a bit of
 * a per-device flag word (no trap, no change to any output):
 *   CV_DEBUG_SORT_ORDER     the sort's final words are not strictly
 *                           ascending (each is its key bits above its record
 *                           index, so order and stability are both checked)
 *   CV_DEBUG_PERM_RANGE     a perm entry outside its shard (or [0, n))
 *   CV_DEBUG_JOURNEY_ORDER  a summary's journey ids not strictly ascending
 *                           within a shard
 *   CV_DEBUG_GROUP_ORDER    a group table's keys not strictly ascending within
 *                           a shard, or a row with distinct journeys outside
 *                           [1, count]
 *   CV_DEBUG_CHECK          set by cv_debug_check_ascending
 * Stage checks need the call's cv_result (res) to bound the rows.
 * cv_debug_flags -- synchronises the current device, copies its flag word to
 *   *flags [host] and clears it when reset != 0.
 * cv_debug_check_ascending -- enqueues the order check on a caller's device
 *   array of n uint64 values (n < 2^32) on stream (a test of the checker).
 * Both return CV_ERR_UNSUPPORTED in the release build.
 * --------------------------------------------------------------------- */
#define CV_DEBUG_SORT_ORDER 0x01u
#define CV_DEBUG_PERM_RANGE 0x02u
#define CV_DEBUG_JOURNEY_ORDER 0x04u
#define CV_DEBUG_GROUP_ORDER 0x08u
#define CV_DEBUG_CHECK 0x10u
cv_status cv_debug_flags(uint32_t* flags /*[host]*/, int reset);
cv_status cv_debug_check_ascending(const uint64_t* a, uint64_t n, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CVETL_H */
