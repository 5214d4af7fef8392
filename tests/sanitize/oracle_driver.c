/* The oracle end to end on seeded adversarial inputs, built with the address
 * and undefined-behaviour sanitizers: ties, duplicate rows, the extreme ids,
 * non-finite coordinates, speeds outside every fast format, empty input.
 * Checks the invariants that need no second implementation (perm is a
 * permutation, the sort is ordered and stable, points and cell counts add up
 * to the records).  Usage: oracle_driver <n> <seed>; exit 0 when all hold. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double orc_fsum(int64_t n, const double* x);
void orc_sort(int64_t n, const int64_t* jid, const int64_t* ts, uint32_t* perm);
int64_t orc_stream_late(int64_t n, const int64_t* jid, const int64_t* ts, int64_t n_push, const int64_t* push_end,
                        uint8_t* late);
void orc_features(int64_t n, const int64_t* jid, const int64_t* ts, const double* lat, const double* lon,
                  double* step_m, double* dt_s, double* speed_mps, double* accel_mps2, double* bearing_deg,
                  double* dheading_deg, uint8_t* flags);
int64_t orc_summary(int64_t n, const int64_t* jid, const int64_t* ts, const double* lat, const double* lon,
                    const float* speed, const double* step_m, const double* dspeed, const uint8_t* flags,
                    int64_t cap, int64_t* o_jid, uint32_t* o_first, uint32_t* o_npts, int64_t* o_tstart,
                    int64_t* o_tend, double* o_dist, double* o_sumspd, float* o_maxspd, double* o_maxdspd,
                    uint32_t* o_ndtz, double* o_latmin, double* o_latmax, double* o_lonmin, double* o_lonmax);
int64_t orc_grid(int64_t n, const int64_t* jid, const int64_t* ts, const double* lat, const double* lon,
                 const float* speed, double lat0, double lon0, double dlat, double dlon, int64_t n_lat,
                 int64_t n_lon, int64_t t0, int64_t bin_ms, int64_t n_t, int64_t cap, int64_t* o_key,
                 uint32_t* o_count, uint32_t* o_nj, double* o_sum, float* o_min, float* o_max, int64_t* o_nout);
int64_t orc_grid_dir(int64_t n, const int64_t* jid, const int64_t* ts, const double* lat, const double* lon,
                     const float* speed, const float* heading, const double* bearing, const uint8_t* flags,
                     int64_t nd, double off, double lat0, double lon0, double dlat, double dlon, int64_t n_lat,
                     int64_t n_lon, int64_t t0, int64_t bin_ms, int64_t n_t, int64_t cap, int64_t* o_key,
                     uint32_t* o_count, uint32_t* o_nj, double* o_sum, float* o_min, float* o_max,
                     int64_t* o_nout);

static uint64_t rng_state;
static uint64_t next_u64(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double next_unit(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

#define NEW(T, k) ((T*)calloc((size_t)((k) > 0 ? (k) : 1), sizeof(T)))
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                               \
        }                                                           \
    } while (0)

int main(int argc, char** argv)
{
    const int64_t n = argc > 1 ? atoll(argv[1]) : 5000;
    rng_state = argc > 2 ? (uint64_t)atoll(argv[2]) : 1;
    const int64_t ids[] = {INT64_MIN, INT64_MAX, -1, 0, 1, 424242, -77};
    int64_t *jid = NEW(int64_t, n), *ts = NEW(int64_t, n);
    double *lat = NEW(double, n), *lon = NEW(double, n);
    float* spd = NEW(float, n);
    for (int64_t i = 0; i < n; ++i) {
        jid[i] = ids[next_u64() % 7];
        ts[i] = 1577836800000ll + (int64_t)(next_u64() % 64) * 30000 - 60000;  /* ties, some before t0 */
        lat[i] = 35.9 + 4.8 * next_unit();
        lon[i] = -95.9 + 6.9 * next_unit();
        spd[i] = (float)(40.0 * next_unit());
        const uint64_t r = next_u64() % 100;
        if (r == 0) lat[i] = NAN;
        if (r == 1) lon[i] = INFINITY;
        if (r == 2) spd[i] = -0.0f;
        if (r == 3) spd[i] = 1e-38f;     /* below every fast format */
        if (r == 4) spd[i] = 1.5e3f;     /* above the 2^10 fast bound */
        if (r == 5 && i > 0) {           /* an exact duplicate of the row before */
            jid[i] = jid[i - 1];
            ts[i] = ts[i - 1];
            lat[i] = lat[i - 1];
            lon[i] = lon[i - 1];
            spd[i] = spd[i - 1];
        }
    }
    uint32_t* perm = NEW(uint32_t, n);
    orc_sort(n, jid, ts, perm);
    uint8_t* seen = NEW(uint8_t, n);
    for (int64_t k = 0; k < n; ++k) {
        CHECK(perm[k] < (uint64_t)n && !seen[perm[k]]);
        seen[perm[k]] = 1;
    }
    int64_t *sj = NEW(int64_t, n), *st = NEW(int64_t, n);
    double *sla = NEW(double, n), *slo = NEW(double, n);
    float* ssp = NEW(float, n);
    for (int64_t k = 0; k < n; ++k) {
        const uint32_t p = perm[k];
        sj[k] = jid[p];
        st[k] = ts[p];
        sla[k] = lat[p];
        slo[k] = lon[p];
        ssp[k] = spd[p];
        if (k > 0) {
            CHECK(sj[k - 1] < sj[k] || (sj[k - 1] == sj[k] && st[k - 1] <= st[k]));
            if (sj[k - 1] == sj[k] && st[k - 1] == st[k]) CHECK(perm[k - 1] < perm[k]);
        }
    }
    double *step = NEW(double, n), *dt = NEW(double, n), *dsp = NEW(double, n), *acc = NEW(double, n),
           *brg = NEW(double, n), *dh = NEW(double, n);
    uint8_t* fl = NEW(uint8_t, n);
    orc_features(n, sj, st, sla, slo, step, dt, dsp, acc, brg, dh, fl);
    const int64_t cap = n;
    int64_t *oj = NEW(int64_t, cap), *ots = NEW(int64_t, cap), *ote = NEW(int64_t, cap);
    uint32_t *ofi = NEW(uint32_t, cap), *onp = NEW(uint32_t, cap), *onz = NEW(uint32_t, cap);
    double *odi = NEW(double, cap), *osu = NEW(double, cap), *omd = NEW(double, cap), *la0 = NEW(double, cap),
           *la1 = NEW(double, cap), *lo0 = NEW(double, cap), *lo1 = NEW(double, cap);
    float* oms = NEW(float, cap);
    const int64_t J = orc_summary(n, sj, st, sla, slo, ssp, step, dsp, fl, cap, oj, ofi, onp, ots, ote, odi, osu,
                                  oms, omd, onz, la0, la1, lo0, lo1);
    int64_t pts = 0;
    for (int64_t j = 0; j < J; ++j) pts += onp[j];
    CHECK(pts == n);
    int64_t *gk = NEW(int64_t, cap), nout = 0;
    uint32_t *gc = NEW(uint32_t, cap), *gn = NEW(uint32_t, cap);
    double* gs = NEW(double, cap);
    float *gmin = NEW(float, cap), *gmax = NEW(float, cap);
    const int64_t G = orc_grid(n, sj, st, sla, slo, ssp, 36.0, -95.8, 0.01, 0.01, 460, 670, 1577836800000ll,
                               900000, 96, cap, gk, gc, gn, gs, gmin, gmax, &nout);
    int64_t cnt = 0;
    for (int64_t g = 0; g < G; ++g) {
        cnt += gc[g];
        if (g > 0) CHECK(gk[g - 1] < gk[g]);
        CHECK(gn[g] >= 1 && gn[g] <= gc[g]);
    }
    CHECK(cnt + nout == n);
    float* hd = NEW(float, n);
    for (int64_t k = 0; k < n; ++k) hd[k] = (float)(400.0 * next_unit() - 20.0);
    int64_t nout2 = 0;
    const int64_t G2 = orc_grid_dir(n, sj, st, sla, slo, ssp, hd, NULL, NULL, 4, 45.0, 36.0, -95.8, 0.01, 0.01,
                                    460, 670, 1577836800000ll, 900000, 96, cap, gk, gc, gn, gs, gmin, gmax, &nout2);
    cnt = 0;
    for (int64_t g = 0; g < G2; ++g) cnt += gc[g];
    CHECK(cnt + nout2 == n);
    const int64_t G3 = orc_grid_dir(n, sj, st, sla, slo, ssp, NULL, brg, fl, 8, 0.0, 36.0, -95.8, 0.01, 0.01, 460,
                                    670, 1577836800000ll, 900000, 0, cap, gk, gc, gn, gs, gmin, gmax, &nout2);
    CHECK(G3 >= 0);
    int64_t ends[3] = {n / 3, (2 * n) / 3, n};
    uint8_t* late = NEW(uint8_t, n);
    const int64_t nl = orc_stream_late(n, jid, ts, 3, ends, late);
    CHECK(nl >= 0 && nl <= n);
    CHECK(isfinite(orc_fsum(n, step)));
    printf("ok n=%lld journeys=%lld groups=%lld late=%lld\n", (long long)n, (long long)J, (long long)G,
           (long long)nl);
    free(jid); free(ts); free(lat); free(lon); free(spd); free(perm); free(seen); free(sj); free(st); free(sla);
    free(slo); free(ssp); free(step); free(dt); free(dsp); free(acc); free(brg); free(dh); free(fl); free(oj);
    free(ots); free(ote); free(ofi); free(onp); free(onz); free(odi); free(osu); free(omd); free(la0); free(la1);
    free(lo0); free(lo1); free(oms); free(gk); free(gc); free(gn); free(gs); free(gmin); free(gmax); free(hd);
    free(late);
    return 0;
}
