/* Test driver for a sanitizer build of the oracle's C library (CPU only):
 * calls every exported function on small inputs of all three sample formats,
 * including the rejected-argument paths, and checks a few results against
 * each other (the direct grid against its own cells, the fold against a sum
 * of the wiped samples).  Exit status 0 = no mismatch; the sanitizers abort
 * on the first error they detect. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_ca_code(int prn, uint8_t *out);
int orc_code_replica(int prn, int64_t fs_hz, int64_t n0, int64_t count, int8_t *out);
void orc_lut(int16_t *cosL, int16_t *sinL);
double orc_bin_freq(double lo, double step, int k);
uint32_t orc_nco_step(double f_if, double f_bin, double fs);
int64_t orc_code_shift(int64_t b, int Tc, int64_t N, double f_bin);
int orc_wipe(const void *samples, int fmt, int64_t n_samples, uint32_t D, int64_t n0, int64_t count,
             int64_t *out);
int orc_wipe_fold(const void *samples, int fmt, int64_t n_samples, int64_t fs_hz, double f_if, double lo,
                  double step, int n_dopp, int Tc, int Nnc, int64_t *out);
int orc_grid_direct(const void *samples, int fmt, int64_t n_samples, int64_t fs_hz, double f_if,
                    const int32_t *prn_list, int n_prn, double lo, double step, int n_dopp, int Tc, int Nnc,
                    double *P, int nthreads, int code_doppler);
int orc_cells_direct(const void *samples, int fmt, int64_t n_samples, int64_t fs_hz, double f_if,
                     const int32_t *prn_list, int n_prn, double lo, double step, int n_dopp, int Tc, int Nnc,
                     const int32_t *cells, int64_t n_cells, double *out, int nthreads, int code_doppler);
int orc_track(const void *samples, int fmt, int64_t n_samples, int n_ch, const int32_t *prn, const uint32_t *D,
              const uint32_t *phi0, const int64_t *q0, const int64_t *R, const int64_t *dl, int64_t start,
              int64_t len, int n_epochs, int64_t *out, int nthreads);

static int fails = 0;
#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            fails++;                                                   \
        }                                                              \
    } while (0)

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)
{ /* xorshift64* */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 2685821657736338717ull) >> 32);
}

static size_t record_bytes(int fmt, int64_t n) { return fmt == 1 ? 2 * n : fmt == 0 ? n : (n + 3) / 4; }

static void run_format(int fmt)
{
    const int64_t fs = 2046000, N = 2046;
    const int Tc = 2, Nnc = 2, nd = 3, np = 2;
    const int64_t n = Tc * Nnc * N + 5;
    const size_t nb = record_bytes(fmt, n);
    uint8_t *x = malloc(nb);
    for (size_t i = 0; i < nb; ++i) x[i] = (uint8_t)rnd();
    if (fmt == 0)
        for (size_t i = 0; i < nb; ++i) x[i] = (uint8_t)(int8_t)((int)(rnd() % 4) * 2 - 3);
    const double f_if = fmt == 1 ? 0.0 : 511500.0, lo = -1000.0, step = 1000.0;
    const int32_t prns[2] = {3, 30};

    int64_t *fold = malloc(sizeof(int64_t) * nd * Nnc * N * 2);
    CHECK(orc_wipe_fold(x, fmt, n, fs, f_if, lo, step, nd, Tc, Nnc, fold) == 0);
    /* fold of bin 1, block 1 against the wiped samples summed by hand */
    int64_t *y = malloc(sizeof(int64_t) * Tc * N * 2);
    const uint32_t D = orc_nco_step(f_if, orc_bin_freq(lo, step, 1), (double)fs);
    CHECK(orc_wipe(x, fmt, n, D, Tc * N, Tc * N, y) == 0);
    for (int64_t m = 0; m < N; ++m) {
        int64_t re = 0, im = 0;
        for (int t = 0; t < Tc; ++t) {
            re += y[2 * (t * N + m)];
            im += y[2 * (t * N + m) + 1];
        }
        const int64_t *f = fold + ((1 * Nnc + 1) * N + m) * 2;
        CHECK(f[0] == re && f[1] == im);
    }

    for (int cd = 0; cd <= 1; ++cd) {
        double *P = malloc(sizeof(double) * np * nd * N);
        CHECK(orc_grid_direct(x, fmt, n, fs, f_if, prns, np, lo, step, nd, Tc, Nnc, P, 2, cd) == 0);
        int32_t cells[3 * 6];
        for (int i = 0; i < 6; ++i) {
            cells[3 * i] = i % np;
            cells[3 * i + 1] = i % nd;
            cells[3 * i + 2] = (int32_t)(rnd() % N);
        }
        double v[6];
        CHECK(orc_cells_direct(x, fmt, n, fs, f_if, prns, np, lo, step, nd, Tc, Nnc, cells, 6, v, 2, cd) == 0);
        for (int i = 0; i < 6; ++i)
            CHECK(v[i] == P[((int64_t)cells[3 * i] * nd + cells[3 * i + 1]) * N + cells[3 * i + 2]]);
        free(P);
    }

    /* tracking correlators: two channels, three epochs */
    const int32_t tp[2] = {3, 30};
    const uint32_t tD[2] = {D, D + 12345u}, phi0[2] = {0u, 1u << 30};
    const int64_t q0[2] = {0, 500LL << 32}, R[2] = {(1LL << 32) / 2, (1LL << 32) / 2};
    const int64_t dl[2] = {1LL << 31, 1LL << 31};
    int64_t out[2 * 3 * 6];
    CHECK(orc_track(x, fmt, n, 2, tp, tD, phi0, q0, R, dl, 7, 1000, 3, out, 2) == 0);

    /* rejected arguments */
    CHECK(orc_wipe_fold(x, fmt, 10, fs, f_if, lo, step, nd, Tc, Nnc, fold) != 0);
    CHECK(orc_wipe_fold(x, 9, n, fs, f_if, lo, step, nd, Tc, Nnc, fold) != 0);
    CHECK(orc_track(x, fmt, n, 2, tp, tD, phi0, q0, R, dl, n - 10, 1000, 3, out, 1) != 0);
    free(y);
    free(fold);
    free(x);
}

int main(void)
{
    uint8_t code[1023];
    for (int prn = 1; prn <= 37; ++prn) CHECK(orc_ca_code(prn, code) == 0);
    CHECK(orc_ca_code(0, code) != 0 && orc_ca_code(38, code) != 0);
    int8_t rep[5000];
    CHECK(orc_code_replica(7, 5000000, 3, 5000, rep) == 0);
    CHECK(orc_code_replica(7, 0, 0, 10, rep) != 0);
    int16_t c[1024], s[1024];
    orc_lut(c, s);
    CHECK(c[0] == 4096 && s[256] == 4096);
    CHECK(orc_code_shift(24, 4, 16368, 7500.0) == 7); /* 7.48 samples */
    for (int fmt = 0; fmt < 3; ++fmt) run_format(fmt);
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle sanitizer driver: all checks passed\n");
    return 0;
}
