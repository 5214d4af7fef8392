// The library's host-side argument checking and size arithmetic, built with
// the address and undefined-behaviour sanitizers (host code only; the device
// code is not compiled in).  Every call here must be answered on the host:
// extreme sizes, overflowing grids, non-finite cell sizes, null pointers,
// missing or short workspaces, unknown tuning and timing names.  No call
// reaches a kernel launch.  Exit 0 when every answer is the documented one.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <limits>

#include "cvetl.h"

static int failures = 0;
#define EXPECT(c)                                                          \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "line %d: expected %s\n", __LINE__, #c);  \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static const uint64_t U64MAX = std::numeric_limits<uint64_t>::max();
static const int64_t I64MAX = std::numeric_limits<int64_t>::max();
static const int64_t I64MIN = std::numeric_limits<int64_t>::min();

static cv_grid_spec good_grid()
{
    cv_grid_spec g;
    g.lat0_deg = 36.0;
    g.lon0_deg = -95.8;
    g.dlat_deg = 0.01;
    g.dlon_deg = 0.01;
    g.n_lat = 460;
    g.n_lon = 670;
    g.t0_ms = 1577836800000ll;
    g.bin_ms = 900000;
    g.n_t = 96;
    return g;
}

// A query either refuses the arguments (a bad spec, or keys or lattice indices
// that would overflow) or answers a size that did not wrap: at least `floor`
// bytes.
static void size_query(cv_status s, size_t bytes, double floor, int line)
{
    if (s == CV_OK && (double)bytes < floor) {
        std::fprintf(stderr, "line %d: size %zu below %.0f (wrapped?)\n", line, bytes, floor);
        ++failures;
    }
    if (s != CV_OK && s != CV_ERR_INVALID_ARGUMENT && s != CV_ERR_RANGE) {
        std::fprintf(stderr, "line %d: status %d\n", line, (int)s);
        ++failures;
    }
}
#define SIZE(call, floor) size_query((call), sz, (floor), __LINE__)

int main()
{
    size_t sz = 0;
    EXPECT(cv_abi_version() == CV_ABI_VERSION);
    for (int s = 0; s < 8; ++s) EXPECT(cv_strerror((cv_status)s) != nullptr);

    // --- workspace sizes at the edges of their domains
    const uint64_t ns[] = {0, 1, 2, 1u << 20, (1ull << 32) - 1, 1ull << 32, 1ull << 40, U64MAX};
    for (uint64_t n : ns) {
        for (uint64_t mj : {uint64_t(0), uint64_t(1), uint64_t(1) << 31, U64MAX}) {
            SIZE(cv_sort_workspace_size(n, mj, &sz), (double)n * 8.0 * (n < (1ull << 32)));
            SIZE(cv_summary_workspace_size(n, mj, &sz), 0);
            SIZE(cv_batch_workspace_size(n, 115, mj, mj, nullptr, 100, &sz), 0);
            cv_grid_spec g = good_grid();
            SIZE(cv_batch_workspace_size(n, 115, mj, mj, &g, mj, &sz), 0);
            SIZE(cv_batch_workspace_size(n, 0xFFFFFFFFu, mj, mj, &g, mj, &sz), 0);
            SIZE(cv_stream_state_size(&g, mj, mj, n, &sz), 0);
        }
        SIZE(cv_hygiene_workspace_size(n, &sz), 0);
        SIZE(cv_groups_filter_workspace_size(n, &sz), 0);
        SIZE(cv_csv_workspace_size(n, n, &sz), 0);
        SIZE(cv_csv_workspace_size(n, U64MAX, &sz), 0);
    }
    EXPECT(cv_sort_workspace_size(1ull << 32, 10, &sz) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_sort_workspace_size(1000, 10, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_summary_workspace_size(1000, 10, nullptr) == CV_ERR_INVALID_ARGUMENT);

    // --- grid specs: every field at its extremes
    const double dvals[] = {0.0, -0.01, 1e-300, 1e300, NAN, INFINITY, -INFINITY, 0.01};
    const int64_t ivals[] = {I64MIN, -1, 0, 1, 1 << 20, 1ll << 31, 1ll << 40, I64MAX};
    for (double d : dvals) {
        cv_grid_spec g = good_grid();
        g.dlat_deg = d;
        SIZE(cv_grid_workspace_size(1000, &g, 100, &sz), 0);
        g = good_grid();
        g.dlon_deg = d;
        SIZE(cv_grid_workspace_size(1000, &g, 100, &sz), 0);
        g = good_grid();
        g.lat0_deg = d;
        g.lon0_deg = d;
        SIZE(cv_grid_workspace_size(1000, &g, 100, &sz), 0);
        SIZE(cv_stream_state_size(&g, 10, 10, 10, &sz), 0);
    }
    for (int64_t a : ivals)
        for (int64_t b : ivals) {
            cv_grid_spec g = good_grid();
            g.n_lat = a;
            g.n_lon = b;
            SIZE(cv_grid_workspace_size(1000, &g, 100, &sz), 0);
            SIZE(cv_lattice_normalize_workspace_size(10, &g, 4, &sz), 0);
            g = good_grid();
            g.n_t = a;
            g.bin_ms = b;
            SIZE(cv_grid_workspace_size(1000, &g, 100, &sz), 0);
            SIZE(cv_batch_workspace_size(1000, 3, 10, 10, &g, 100, &sz), 0);
            SIZE(cv_stream_state_size(&g, 10, 10, 10, &sz), 0);
            g = good_grid();
            g.t0_ms = a;
            g.n_t = b;
            SIZE(cv_grid_workspace_size(1000, &g, 100, &sz), 0);
            for (uint64_t nt : {uint64_t(0), uint64_t(1), uint64_t(1) << 40, U64MAX})
                for (uint32_t nd : {0u, 1u, 8u, 0xFFFFFFFFu}) {
                    cv_grid_spec h = good_grid();
                    h.n_lat = a;
                    h.n_lon = b;
                    SIZE(cv_lattice_normalize_workspace_size(nt, &h, nd, &sz), 0);
                }
        }
    {
        cv_grid_spec g = good_grid();
        g.dlat_deg = 0.0;
        EXPECT(cv_grid_workspace_size(1000, &g, 100, &sz) == CV_ERR_INVALID_ARGUMENT);
        g = good_grid();
        g.bin_ms = 0;
        EXPECT(cv_grid_workspace_size(1000, &g, 100, &sz) == CV_ERR_INVALID_ARGUMENT);
        g = good_grid();
        g.dlon_deg = NAN;
        EXPECT(cv_grid_workspace_size(1000, &g, 100, &sz) == CV_ERR_INVALID_ARGUMENT);
        EXPECT(cv_grid_workspace_size(1000, nullptr, 100, &sz) == CV_ERR_INVALID_ARGUMENT);
    }

    // --- compute entry points: refused on the host before any launch
    int64_t dummy64 = 0;
    double dummyd = 0;
    float dummyf = 0;
    cv_records none{};
    none.n = 10;
    cv_records ok{&dummy64, &dummy64, &dummyd, &dummyd, &dummyf, 10};
    cv_records big = ok;
    big.n = 1ull << 32;
    cv_records many = ok;
    many.n = 1ull << 20;
    cv_features feat{};
    cv_journeys jr{};
    cv_groups gr{};
    cv_records_out rout{};
    uint32_t perm_dummy = 0;
    cv_grid_spec g = good_grid();
    char text[8] = "a,b\n";
    uint64_t offs[2] = {0, 10};
    EXPECT(cv_sort_records(nullptr, 10, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_sort_records(&none, 10, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_sort_records(&big, 10, &perm_dummy, nullptr, nullptr, nullptr, 0, nullptr) ==
           CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_sort_records(&ok, 10, &perm_dummy, nullptr, nullptr, nullptr, 0, nullptr) == CV_ERR_WORKSPACE);
    EXPECT(cv_sort_records(&ok, 10, &perm_dummy, &rout, nullptr, &dummy64, 1, nullptr) == CV_ERR_WORKSPACE);
    EXPECT(cv_journey_features(nullptr, nullptr, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_journey_features(&none, &feat, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_journey_features(&big, &feat, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_journey_summary(&ok, &feat, &jr, 10, nullptr, nullptr, 0, nullptr) == CV_ERR_WORKSPACE);
    EXPECT(cv_journey_summary(&big, &feat, &jr, 10, nullptr, nullptr, 0, nullptr) != CV_OK);
    EXPECT(cv_journey_summary(nullptr, &feat, &jr, 10, nullptr, nullptr, 0, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_journey_summary_noalloc(&many, &feat, &jr, 1 << 20, nullptr, nullptr) == CV_ERR_WORKSPACE);
    EXPECT(cv_journey_summary_noalloc(&big, &feat, &jr, 10, nullptr, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_journey_summary_noalloc(&ok, &feat, &jr, U64MAX, nullptr, nullptr) != CV_OK);
    EXPECT(cv_grid_aggregate(&ok, &g, &gr, 10, nullptr, nullptr, 0, nullptr) == CV_ERR_WORKSPACE);
    EXPECT(cv_grid_aggregate(&ok, nullptr, &gr, 10, nullptr, nullptr, 0, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_grid_aggregate(&big, &g, &gr, 10, nullptr, nullptr, 0, nullptr) != CV_OK);
    EXPECT(cv_grid_aggregate_dir(&ok, nullptr, nullptr, &g, 0, 0.0, &gr, 10, nullptr, nullptr, 0, nullptr) != CV_OK);
    EXPECT(cv_gather_column(nullptr, nullptr, nullptr, 10, 8, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_gather_column(&dummy64, &perm_dummy, &dummy64, 10, 3, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_gather_column(&dummy64, &perm_dummy, &dummy64, 1ull << 32, 8, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_lattice_dense(&gr, 10, nullptr, 0, 0, 10, nullptr, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_lattice_normalize(nullptr, 10, &g, 0, nullptr, nullptr, 0, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_groups_filter(&gr, 10, 1.0, 0.0, 1.0, nullptr, 10, nullptr, nullptr, 0, nullptr) != CV_OK);
    EXPECT(cv_drop_duplicates(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_csv_extract(nullptr, 10, 0, &rout, nullptr, nullptr, 10, nullptr, nullptr, 0, nullptr) ==
           CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_csv_extract(text, 4, 1, &rout, nullptr, nullptr, 10, nullptr, nullptr, 0, nullptr) != CV_OK);
    EXPECT(cv_batch_run(&ok, nullptr, 1, &g, 10, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0,
                        nullptr, nullptr, nullptr, nullptr, 0, nullptr) != CV_OK);
    EXPECT(cv_batch_run(&ok, offs, 1, &g, 10, &perm_dummy, &rout, &feat, &jr, 10, nullptr, &gr, 10, nullptr,
                        nullptr, nullptr, nullptr, 0, nullptr) != CV_OK);
    EXPECT(cv_batch_sort_records(&ok, offs, 0, 10, &perm_dummy, nullptr, nullptr, nullptr, 0, nullptr) != CV_OK);

    // --- serving state: creation refused without state memory; null handles
    cv_stream* st = nullptr;
    EXPECT(cv_stream_create(&g, 10, 10, 10, nullptr, 0, nullptr, &st) != CV_OK && st == nullptr);
    EXPECT(cv_stream_create(nullptr, 10, 10, 10, nullptr, 0, nullptr, &st) != CV_OK);
    EXPECT(cv_stream_push(nullptr, &ok, &feat, nullptr, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_stream_flush(nullptr, &jr, 10, &gr, 10, nullptr, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_stream_snapshot_size(nullptr, &sz) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_stream_snapshot(nullptr, nullptr, 0, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_stream_restore(nullptr, nullptr, 0, nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_stream_destroy(nullptr) != CV_ERR_DEVICE);

    // --- tuning and timing registries
    int64_t v = -1, shape0 = -1, shapes = -1;
    EXPECT(cv_tuning_get("sort_shape", &shape0) == CV_OK && shape0 >= 0);
    EXPECT(cv_tuning_get("sort_shapes", &shapes) == CV_OK && shapes > 0);
    EXPECT(cv_tuning_get("sort_tile", &v) == CV_OK && v > 0);
    EXPECT(cv_tuning_get("radix_bits", &v) == CV_OK && v > 0 && v <= 16);
    EXPECT(cv_tuning_get(nullptr, &v) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_tuning_get("sort_shape", nullptr) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_tuning_get("", &v) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_tuning_get("no such knob", &v) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_tuning_set(nullptr, 0) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_tuning_set("no such knob", 0) == CV_ERR_INVALID_ARGUMENT);
    for (int64_t x : {I64MIN, int64_t(-1), shapes, I64MAX})
        EXPECT(cv_tuning_set("sort_shape", x) == CV_ERR_INVALID_ARGUMENT);
    EXPECT(cv_tuning_set("sort_shapes", 1) == CV_ERR_INVALID_ARGUMENT);
    for (int64_t s = 0; s < shapes; ++s) EXPECT(cv_tuning_set("sort_shape", s) == CV_OK);
    EXPECT(cv_tuning_set("sort_shape", shape0) == CV_OK);
    EXPECT(cv_timing_enable(1) == CV_OK && cv_timing_enable(0) == CV_OK && cv_timing_reset() == CV_OK);
    double ms = -1;
    uint64_t launches = 7;
    EXPECT(cv_timing_read("sort_pass0", &ms, &launches) == CV_OK && ms == 0.0 && launches == 0);
    EXPECT(cv_timing_read("no such family", &ms, &launches) == CV_OK && launches == 0);
    EXPECT(cv_timing_read(nullptr, &ms, &launches) == CV_ERR_INVALID_ARGUMENT);

    std::printf("%s: %d failure(s)\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
