/*
 * gnss_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU reference for GPS L1 C/A acquisition
 * (the acquisition channel of the paper's Fig. 2, Sec. 3: carrier and code
 * NCOs -> mixing -> correlation over all code shifts -> detection).
 * Integers are exact; floating point is IEEE double.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load this library; the
 * product (the HIP library) never does, and the two share no code, tables or
 * constant generators.
 *
 * Conventions (readings of the paper where it is silent, see the design notes):
 *  - C/A code from the GPS interface specification IS-GPS-200, Table 3-Ia,
 *    generated here with the G2 *tap-pair* form.  Logic 0 -> +1, 1 -> -1.
 *  - Code replica at sample rate fs (code NCO of Fig. 2):
 *        c[n] = 1 - 2*code[ floor(n*1023000/fs) mod 1023 ]   (64-bit integers)
 *  - Carrier NCO: 32-bit phase accumulator, step
 *        D_k = (uint32)(int64) llround( (f_if + f_k) * 2^32 / fs ),
 *        f_k = lo + k*step  (IEEE double, evaluated as written),
 *    phase of global sample n: phi_n = (uint32)(n * D_k), LUT index phi_n >> 22.
 *  - LUT: cosL[i] = lround(4096 cos(2 pi i/1024)), sinL[i] = lround(4096 sin(..)).
 *  - Mixing (first mixing stage of Fig. 2): y[n] = x[n] * (cosL[i] - j sinL[i]).
 *  - Coherent block b (block processing, Sec. 4) covers global samples
 *    [b*Tc*N, (b+1)*Tc*N), N = fs/1000.  For every lag tau in [0, N):
 *        R_b[tau] = sum_{n in block b} y[n] * c[(n - tau) mod N]
 *    (the "sample shift and multiply" correlation of Sec. 3, over all shifts).
 *  - P[p][k][tau] = sum_b |R_b[tau]|^2 * 2^-24, summed in double, b ascending.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* Sample formats (same meaning as the product's public header, restated). */
#define ORC_REAL_I8 0          /* one int8 per sample                          */
#define ORC_CPLX_I8 1          /* interleaved I, Q int8                        */
#define ORC_REAL_2BIT_PACKED 2 /* 4 samples/byte, LSB pair first;
                                  00:+1 01:+3 10:-1 11:-3                      */

/* IS-GPS-200 Table 3-Ia: G2 output tap pair (stage numbers 1..10) per PRN 1..37. */
static const int orc_taps[37][2] = {
    {2, 6}, {3, 7}, {4, 8}, {5, 9}, {1, 9}, {2, 10}, {1, 8}, {2, 9}, {3, 10},
    {2, 3}, {3, 4}, {5, 6}, {6, 7}, {7, 8}, {8, 9}, {9, 10}, {1, 4}, {2, 5},
    {3, 6}, {4, 7}, {5, 8}, {6, 9}, {1, 3}, {4, 6}, {5, 7}, {6, 8}, {7, 9},
    {8, 10}, {1, 6}, {2, 7}, {3, 8}, {4, 9}, {5, 10}, {4, 10}, {1, 7}, {2, 8},
    {4, 10}};

/* One C/A code period (1023 chips, values 0/1).  G1 = 1 + x^3 + x^10,
 * G2 = 1 + x^2 + x^3 + x^6 + x^8 + x^9 + x^10, both registers start all ones,
 * outputs are read before each shift. */
int orc_ca_code(int prn, uint8_t *out)
{
    if (prn < 1 || prn > 37 || !out) return ORC_EINVAL;
    int g1[11], g2[11];
    for (int i = 1; i <= 10; i++) { g1[i] = 1; g2[i] = 1; }
    const int t1 = orc_taps[prn - 1][0], t2 = orc_taps[prn - 1][1];
    for (int n = 0; n < 1023; n++) {
        out[n] = (uint8_t)(g1[10] ^ g2[t1] ^ g2[t2]);
        int fb1 = g1[3] ^ g1[10];
        int fb2 = g2[2] ^ g2[3] ^ g2[6] ^ g2[8] ^ g2[9] ^ g2[10];
        for (int i = 10; i > 1; i--) { g1[i] = g1[i - 1]; g2[i] = g2[i - 1]; }
        g1[1] = fb1;
        g2[1] = fb2;
    }
    return ORC_OK;
}

/* Code replica c[n0 .. n0+count) as +1/-1 int8 at sample rate fs_hz. */
int orc_code_replica(int prn, int64_t fs_hz, int64_t n0, int64_t count, int8_t *out)
{
    uint8_t code[1023];
    if (fs_hz <= 0 || n0 < 0 || count < 0 || !out) return ORC_EINVAL;
    int rc = orc_ca_code(prn, code);
    if (rc) return rc;
    for (int64_t i = 0; i < count; i++) {
        int64_t n = n0 + i;
        int64_t chip = (n * 1023000) / fs_hz;
        out[i] = (int8_t)(1 - 2 * code[chip % 1023]);
    }
    return ORC_OK;
}

void orc_lut(int16_t *cosL, int16_t *sinL)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int i = 0; i < 1024; i++) {
        cosL[i] = (int16_t)lround(4096.0 * cos(two_pi * (double)i / 1024.0));
        sinL[i] = (int16_t)lround(4096.0 * sin(two_pi * (double)i / 1024.0));
    }
}

double orc_bin_freq(double lo, double step, int k)
{
    return lo + (double)k * step;
}

uint32_t orc_nco_step(double f_if, double f_bin, double fs)
{
    double f = f_if + f_bin;
    return (uint32_t)(int64_t)llround(f * 4294967296.0 / fs);
}

/* Code-Doppler compensation of the non-coherent sum (an option).  The code
 * rate scales with the carrier Doppler (f_L1 = 1540 x the chip rate), so a
 * satellite's correlation peak at Doppler f moves by f / f_L1 samples per
 * sample.  Block b starts b*Tc*N samples into the record; its peak sits
 * delta_b = llround(b*Tc*N * f / 1575.42e6) samples earlier than block 0's,
 * and the compensated power is P[tau] = sum_b |R_b[(tau - delta_b) mod N]|^2. */
int64_t orc_code_shift(int64_t b, int Tc, int64_t N, double f_bin)
{
    double x = (double)(b * (int64_t)Tc * N) * f_bin / 1575420000.0;
    return (int64_t)llround(x);
}

/* Read sample n of the record as (re, im) integers. */
static void orc_sample(const void *samples, int fmt, int64_t n, int64_t *re, int64_t *im)
{
    if (fmt == ORC_REAL_I8) {
        *re = ((const int8_t *)samples)[n];
        *im = 0;
    } else if (fmt == ORC_CPLX_I8) {
        *re = ((const int8_t *)samples)[2 * n];
        *im = ((const int8_t *)samples)[2 * n + 1];
    } else {
        uint8_t byte = ((const uint8_t *)samples)[n / 4];
        int code = (byte >> (2 * (n % 4))) & 3;
        static const int val[4] = {1, 3, -1, -3};
        *re = val[code];
        *im = 0;
    }
}

/* Mixed (carrier-wiped) samples y[n0 .. n0+count) for one carrier step D,
 * with a caller-supplied LUT.  out is [count][2] int64. */
static void orc_wipe_lut(const void *samples, int fmt, uint32_t D, int64_t n0, int64_t count,
                         const int16_t *cosL, const int16_t *sinL, int64_t *out)
{
    for (int64_t i = 0; i < count; i++) {
        int64_t n = n0 + i;
        uint32_t phi = (uint32_t)((uint64_t)n * (uint64_t)D);
        int idx = (int)(phi >> 22);
        int64_t c = cosL[idx], s = sinL[idx];
        int64_t xr, xi;
        orc_sample(samples, fmt, n, &xr, &xi);
        /* (xr + j xi)(c - j s) */
        out[2 * i] = xr * c + xi * s;
        out[2 * i + 1] = xi * c - xr * s;
    }
}

int orc_wipe(const void *samples, int fmt, int64_t n_samples, uint32_t D,
             int64_t n0, int64_t count, int64_t *out)
{
    int16_t cosL[1024], sinL[1024];
    if (!samples || !out || fmt < 0 || fmt > 2 || n0 < 0 || count < 0 || n0 + count > n_samples)
        return ORC_EINVAL;
    orc_lut(cosL, sinL);
    orc_wipe_lut(samples, fmt, D, n0, count, cosL, sinL, out);
    return ORC_OK;
}

static int orc_check_common(const void *samples, int fmt, int64_t n_samples, int64_t fs_hz,
                            int n_dopp, int Tc, int Nnc, int64_t *N_out)
{
    if (!samples || fmt < 0 || fmt > 2 || fs_hz <= 0 || fs_hz % 1000 != 0) return ORC_EINVAL;
    if (n_dopp < 1 || Tc < 1 || Nnc < 1) return ORC_EINVAL;
    int64_t N = fs_hz / 1000;
    if ((int64_t)Tc * Nnc * N > n_samples) return ORC_EINVAL;
    *N_out = N;
    return ORC_OK;
}

/* Folded coherent blocks: f[k][b][m] = sum_{t<Tc} y_k[(b*Tc + t)*N + m].
 * out is [n_dopp][Nnc][N][2] int64. */
int orc_wipe_fold(const void *samples, int fmt, int64_t n_samples, int64_t fs_hz,
                  double f_if, double lo, double step, int n_dopp, int Tc, int Nnc,
                  int64_t *out)
{
    int64_t N;
    int rc = orc_check_common(samples, fmt, n_samples, fs_hz, n_dopp, Tc, Nnc, &N);
    if (rc) return rc;
    int64_t blk = (int64_t)Tc * N;
    int16_t cosL[1024], sinL[1024];
    orc_lut(cosL, sinL);
    int64_t *y = (int64_t *)malloc(sizeof(int64_t) * 2 * blk);
    if (!y) return ORC_ENOMEM;
    for (int k = 0; k < n_dopp; k++) {
        uint32_t D = orc_nco_step(f_if, orc_bin_freq(lo, step, k), (double)fs_hz);
        for (int b = 0; b < Nnc; b++) {
            orc_wipe_lut(samples, fmt, D, (int64_t)b * blk, blk, cosL, sinL, y);
            int64_t *f = out + (((int64_t)k * Nnc + b) * N) * 2;
            for (int64_t m = 0; m < N; m++) {
                int64_t re = 0, im = 0;
                for (int t = 0; t < Tc; t++) {
                    re += y[2 * ((int64_t)t * N + m)];
                    im += y[2 * ((int64_t)t * N + m) + 1];
                }
                f[2 * m] = re;
                f[2 * m + 1] = im;
            }
        }
    }
    free(y);
    return ORC_OK;
}

/* Direct time-domain correlation of one coherent block at one lag:
 * R = sum_{n in block} y[n] * c[(n - tau) mod N].  y holds the block's mixed
 * samples, n_first is the global index of y[0], c is one code period (N). */
static void orc_corr_block(const int64_t *y, int64_t blk, int64_t n_first, const int8_t *c,
                           int64_t N, int64_t tau, int64_t *Rre, int64_t *Rim)
{
    int64_t re = 0, im = 0;
    int64_t ci = (n_first - tau) % N; /* code index of the block's first sample */
    if (ci < 0) ci += N;
    for (int64_t i = 0; i < blk; i++) {
        re += y[2 * i] * c[ci];
        im += y[2 * i + 1] * c[ci];
        if (++ci == N) ci = 0;
    }
    *Rre = re;
    *Rim = im;
}

/* Full power grid by direct correlation.  P is [n_prn][n_dopp][N] doubles.
 * (PRN, Doppler) rows are independent tasks handed out dynamically to the
 * worker threads, as the paper's Listing 2 does for its channel tasks. */
int orc_grid_direct(const void *samples, int fmt, int64_t n_samples, int64_t fs_hz,
                    double f_if, const int32_t *prn_list, int n_prn, double lo, double step,
                    int n_dopp, int Tc, int Nnc, double *P, int nthreads, int code_doppler)
{
    int64_t N;
    int rc = orc_check_common(samples, fmt, n_samples, fs_hz, n_dopp, Tc, Nnc, &N);
    if (rc) return rc;
    if (!prn_list || n_prn < 1 || !P) return ORC_EINVAL;
    for (int i = 0; i < n_prn; i++)
        if (prn_list[i] < 1 || prn_list[i] > 37) return ORC_EINVAL;
    int64_t blk = (int64_t)Tc * N;
    int64_t used = blk * Nnc;
    int n_task = n_prn * n_dopp;
    int failed = 0;
    int16_t cosL[1024], sinL[1024];
    orc_lut(cosL, sinL);
    (void)nthreads;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        int64_t *y = (int64_t *)malloc(sizeof(int64_t) * 2 * used);
        int8_t *c = (int8_t *)malloc((size_t)N);
        if (!y || !c) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic)
        for (int task = 0; task < n_task; task++) {
            if (!y || !c) continue;
            int pi = task / n_dopp, k = task % n_dopp;
            uint32_t D = orc_nco_step(f_if, orc_bin_freq(lo, step, k), (double)fs_hz);
            orc_wipe_lut(samples, fmt, D, 0, used, cosL, sinL, y);
            orc_code_replica(prn_list[pi], fs_hz, 0, N, c);
            double *row = P + ((int64_t)pi * n_dopp + k) * N;
            for (int64_t tau = 0; tau < N; tau++) {
                double acc = 0.0;
                for (int b = 0; b < Nnc; b++) {
                    int64_t Rre, Rim;
                    int64_t t = tau;
                    if (code_doppler) {
                        t = (tau - orc_code_shift(b, Tc, N, orc_bin_freq(lo, step, k))) % N;
                        if (t < 0) t += N;
                    }
                    orc_corr_block(y + 2 * (int64_t)b * blk, blk, (int64_t)b * blk, c, N, t,
                                   &Rre, &Rim);
                    acc += ((double)Rre * (double)Rre + (double)Rim * (double)Rim) * 0x1p-24;
                }
                row[tau] = acc;
            }
        }
        free(y);
        free(c);
    }
    return failed ? ORC_ENOMEM : ORC_OK;
}

/* Selected cells by direct correlation.  cells is [n_cells][3] =
 * (index into prn_list, Doppler bin k, lag tau); out[i] = P of cell i. */
int orc_cells_direct(const void *samples, int fmt, int64_t n_samples, int64_t fs_hz,
                     double f_if, const int32_t *prn_list, int n_prn, double lo, double step,
                     int n_dopp, int Tc, int Nnc, const int32_t *cells, int64_t n_cells,
                     double *out, int nthreads, int code_doppler)
{
    int64_t N;
    int rc = orc_check_common(samples, fmt, n_samples, fs_hz, n_dopp, Tc, Nnc, &N);
    if (rc) return rc;
    if (!prn_list || n_prn < 1 || !cells || !out || n_cells < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n_cells; i++) {
        const int32_t *cl = cells + 3 * i;
        if (cl[0] < 0 || cl[0] >= n_prn || cl[1] < 0 || cl[1] >= n_dopp || cl[2] < 0 ||
            cl[2] >= N || prn_list[cl[0]] < 1 || prn_list[cl[0]] > 37)
            return ORC_EINVAL;
    }
    int64_t blk = (int64_t)Tc * N;
    int failed = 0;
    int16_t cosL[1024], sinL[1024];
    orc_lut(cosL, sinL);
    (void)nthreads;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        int64_t *y = (int64_t *)malloc(sizeof(int64_t) * 2 * blk);
        int8_t *c = (int8_t *)malloc((size_t)N);
        if (!y || !c) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic)
        for (int64_t i = 0; i < n_cells; i++) {
            if (!y || !c) continue;
            const int32_t *cl = cells + 3 * i;
            uint32_t D = orc_nco_step(f_if, orc_bin_freq(lo, step, cl[1]), (double)fs_hz);
            orc_code_replica(prn_list[cl[0]], fs_hz, 0, N, c);
            double acc = 0.0;
            for (int b = 0; b < Nnc; b++) {
                int64_t Rre, Rim;
                int64_t t = cl[2];
                if (code_doppler) {
                    t = (t - orc_code_shift(b, Tc, N, orc_bin_freq(lo, step, cl[1]))) % N;
                    if (t < 0) t += N;
                }
                orc_wipe_lut(samples, fmt, D, (int64_t)b * blk, blk, cosL, sinL, y);
                orc_corr_block(y, blk, (int64_t)b * blk, c, N, t, &Rre, &Rim);
                acc += ((double)Rre * (double)Rre + (double)Rim * (double)Rim) * 0x1p-24;
            }
            out[i] = acc;
        }
        free(y);
        free(c);
    }
    return failed ? ORC_ENOMEM : ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Tracking correlators (the tracking channel of Fig. 3: carrier and code NCOs,
 * the first mixing stage, then time-domain correlation with the code replica,
 * Sec. 3).  The paper shows the channel only as a figure; the reading here is
 * the usual early / prompt / late correlator set, with the NCOs in fixed point
 * so that every result is an exact integer:
 *
 *   channel c: PRN, carrier step D (uint32, cycles * 2^32 per sample) and
 *   initial phase phi0 (uint32, cycles * 2^32 at sample 0); code phase q0 and
 *   code step R (int64, chips * 2^32 at sample 0 and per sample); early-late
 *   offset dl (int64, chips * 2^32).
 *   For global sample n:
 *     phase(n) = (uint32)(phi0 + n * D),  y[n] = x[n] * (cosL - j sinL)[phase(n) >> 22]
 *     q(n) = q0 + n * R
 *     chip_X(n) = floor((q(n) + off_X) / 2^32) mod 1023 (mathematical mod),
 *       off_E = +dl (replica advanced), off_P = 0, off_L = -dl
 *     X_e = sum over n in epoch e of y[n] * (1 - 2 code[chip_X(n)])
 *   Epoch e covers samples [start + e*len, start + (e+1)*len).
 *   out[c][e][X][re, im], X = 0 early, 1 prompt, 2 late, int64.
 * With phi0 = 0 the carrier and mixing are those of the acquisition oracle.
 * ------------------------------------------------------------------------- */
int orc_track(const void *samples, int fmt, int64_t n_samples, int n_ch, const int32_t *prn,
              const uint32_t *D, const uint32_t *phi0, const int64_t *q0, const int64_t *R,
              const int64_t *dl, int64_t start, int64_t len, int n_epochs, int64_t *out,
              int nthreads)
{
    int16_t cosL[1024], sinL[1024];
    if (!samples || !prn || !D || !phi0 || !q0 || !R || !dl || !out) return ORC_EINVAL;
    if (fmt < 0 || fmt > 2 || n_ch < 1 || start < 0 || len < 1 || n_epochs < 1) return ORC_EINVAL;
    if (start + len * (int64_t)n_epochs > n_samples) return ORC_EINVAL;
    for (int c = 0; c < n_ch; c++)
        if (prn[c] < 1 || prn[c] > 37) return ORC_EINVAL;
    orc_lut(cosL, sinL);
    (void)nthreads;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t ce = 0; ce < (int64_t)n_ch * n_epochs; ce++) {
        const int c = (int)(ce / n_epochs), e = (int)(ce % n_epochs);
        uint8_t code[1023];
        orc_ca_code(prn[c], code);
        int64_t acc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        const int64_t off[3] = {dl[c], 0, -dl[c]};
        for (int64_t i = 0; i < len; i++) {
            const int64_t n = start + (int64_t)e * len + i;
            const uint32_t ph = (uint32_t)(phi0[c] + (uint32_t)((uint64_t)n * (uint64_t)D[c]));
            const int idx = (int)(ph >> 22);
            const int64_t cs = cosL[idx], sn = sinL[idx];
            int64_t xr, xi;
            orc_sample(samples, fmt, n, &xr, &xi);
            const int64_t yr = xr * cs + xi * sn, yi = xi * cs - xr * sn;
            const int64_t q = q0[c] + n * R[c];
            for (int x = 0; x < 3; x++) {
                int64_t v = q + off[x];
                int64_t chip = v >= 0 ? v / 4294967296LL : -((-v + 4294967295LL) / 4294967296LL);
                chip %= 1023;
                if (chip < 0) chip += 1023;
                const int64_t s = 1 - 2 * (int64_t)code[chip];
                acc[x][0] += s * yr;
                acc[x][1] += s * yi;
            }
        }
        int64_t *o = out + ce * 6;
        for (int x = 0; x < 3; x++) {
            o[2 * x] = acc[x][0];
            o[2 * x + 1] = acc[x][1];
        }
    }
    return ORC_OK;
}
