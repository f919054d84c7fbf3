/*
 * oracle.c -- plain CPU reference for the X-engine (TEST INFRASTRUCTURE ONLY).
 *
 * This file is the checker, not the product.  Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may load it.  It shares no code, header
 * or table with the GPU library.
 *
 * What it computes (Ord et al., "The Murchison Widefield Array Correlator"):
 *   - Sec. 2, eq. (3): an FX correlator forms the cross-power spectrum of two
 *     inputs as the product of their Fourier-transformed voltages.  The printed
 *     equation omits the conjugate on the second factor; the cross-power is read
 *     here as x_i * conj(x_j).
 *   - Sec. 1.1 / Sec. 3.4: per fine channel, the products of all input pairs are
 *     integrated (summed) over time on the device.
 *   - Appendix C, "GPU Output": the matrix is Hermitian, so only the lower
 *     triangle including the diagonal (autocorrelations) is kept.
 *   - Appendix A, data-format list: each sample is one byte, 4-bit real and
 *     4-bit imaginary two's complement, with the code 8 (i.e. -8) meaning
 *     invalid data.  Reading: real part in the high nibble; a sample with an
 *     invalid code in either nibble contributes nothing (decodes to 0 + 0j).
 *
 * For every channel f and 0 <= j <= i < N:
 *   Re V_f[i][j] = sum_t re_i re_j + im_i im_j
 *   Im V_f[i][j] = sum_t im_i re_j - re_i im_j
 * evaluated in int64, i.e. exactly.  Output layout: out[f][b][2] with
 * b = i*(i+1)/2 + j and [0] = Re, [1] = Im.
 *
 * Input layouts: 0 = (time, channel, input), byte offset (t*F + f)*N + i, the
 * paper's GPU input order of Appendix C ("GPU Input") with the sample packed;
 * 1 = (channel, time, input), byte offset (f*T + t)*N + i.
 *
 * Parallelism: OpenMP over channels only.  The inner loops are the plain
 * triple loop over (i, j, t).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Decode one packed sample.  Returns 1 for a valid sample, 0 for an invalid one
 * (either 4-bit code equal to 8), in which case both parts are set to 0. */
int oracle_decode(uint8_t b, int32_t *re, int32_t *im)
{
    int hi = (b >> 4) & 0xF;
    int lo = b & 0xF;
    if (hi == 8 || lo == 8) {
        *re = 0;
        *im = 0;
        return 0;
    }
    *re = hi >= 8 ? hi - 16 : hi;
    *im = lo >= 8 ? lo - 16 : lo;
    return 1;
}

static size_t in_offset(int layout, int n_inputs, int n_chan, int n_time, int f, int t, int i)
{
    if (layout == 0)
        return ((size_t)t * n_chan + f) * n_inputs + i;
    return ((size_t)f * n_time + t) * n_inputs + i;
}

/* Decode one channel into input-major arrays re[i*T + t], im[i*T + t]. */
static void decode_channel(const uint8_t *in, int layout, int n_inputs, int n_chan, int n_time,
                           int f, int32_t *re, int32_t *im)
{
    for (int t = 0; t < n_time; ++t)
        for (int i = 0; i < n_inputs; ++i)
            oracle_decode(in[in_offset(layout, n_inputs, n_chan, n_time, f, t, i)],
                          &re[(size_t)i * n_time + t], &im[(size_t)i * n_time + t]);
}

static int check_args(const void *in, int n_inputs, int n_chan, int n_time, int layout, const void *out)
{
    if (!in || !out || n_inputs < 1 || n_chan < 1 || n_time < 1 || (layout != 0 && layout != 1))
        return -1;
    return 0;
}

/* Lower triangle including the diagonal: out[f][i*(i+1)/2 + j][2], int64. */
int oracle_xmac(const uint8_t *in, int n_inputs, int n_chan, int n_time, int layout, int64_t *out)
{
    if (check_args(in, n_inputs, n_chan, n_time, layout, out))
        return -1;
    const size_t nb = (size_t)n_inputs * (n_inputs + 1) / 2;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int f = 0; f < n_chan; ++f) {
        int32_t *re = malloc(sizeof(int32_t) * (size_t)n_inputs * n_time);
        int32_t *im = malloc(sizeof(int32_t) * (size_t)n_inputs * n_time);
        if (!re || !im) {
            free(re);
            free(im);
#pragma omp atomic write
            err = -2;
            continue;
        }
        decode_channel(in, layout, n_inputs, n_chan, n_time, f, re, im);
        int64_t *o = out + (size_t)f * nb * 2;
        for (int i = 0; i < n_inputs; ++i) {
            const int32_t *ar = re + (size_t)i * n_time, *ai = im + (size_t)i * n_time;
            for (int j = 0; j <= i; ++j) {
                const int32_t *br = re + (size_t)j * n_time, *bi = im + (size_t)j * n_time;
                int64_t sr = 0, si = 0;
                for (int t = 0; t < n_time; ++t) {
                    sr += (int64_t)ar[t] * br[t] + (int64_t)ai[t] * bi[t];
                    si += (int64_t)ai[t] * br[t] - (int64_t)ar[t] * bi[t];
                }
                size_t b = (size_t)i * (i + 1) / 2 + j;
                o[2 * b] = sr;
                o[2 * b + 1] = si;
            }
        }
        free(re);
        free(im);
    }
    return err;
}

/* Every ordered pair (i, j), upper triangle included: out[f][i][j][2], int64.
 * Used to check Hermitian symmetry; the same definition, no triangle. */
int oracle_xmac_full(const uint8_t *in, int n_inputs, int n_chan, int n_time, int layout, int64_t *out)
{
    if (check_args(in, n_inputs, n_chan, n_time, layout, out))
        return -1;
    const size_t nn = (size_t)n_inputs * n_inputs;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int f = 0; f < n_chan; ++f) {
        int32_t *re = malloc(sizeof(int32_t) * (size_t)n_inputs * n_time);
        int32_t *im = malloc(sizeof(int32_t) * (size_t)n_inputs * n_time);
        if (!re || !im) {
            free(re);
            free(im);
#pragma omp atomic write
            err = -2;
            continue;
        }
        decode_channel(in, layout, n_inputs, n_chan, n_time, f, re, im);
        int64_t *o = out + (size_t)f * nn * 2;
        for (int i = 0; i < n_inputs; ++i)
            for (int j = 0; j < n_inputs; ++j) {
                int64_t sr = 0, si = 0;
                for (int t = 0; t < n_time; ++t) {
                    int64_t ar = re[(size_t)i * n_time + t], ai = im[(size_t)i * n_time + t];
                    int64_t br = re[(size_t)j * n_time + t], bi = im[(size_t)j * n_time + t];
                    sr += ar * br + ai * bi;
                    si += ai * br - ar * bi;
                }
                o[2 * ((size_t)i * n_inputs + j)] = sr;
                o[2 * ((size_t)i * n_inputs + j) + 1] = si;
            }
        free(re);
        free(im);
    }
    return err;
}

/* Incoherent beam (Sec. 3.4, other XMAC modes): per channel and time sample,
 * the total power sum_i |x_i(t)|^2.  out[f][t], int64. */
int oracle_incoherent_beam(const uint8_t *in, int n_inputs, int n_chan, int n_time, int layout, int64_t *out)
{
    if (check_args(in, n_inputs, n_chan, n_time, layout, out))
        return -1;
#pragma omp parallel for schedule(static)
    for (int f = 0; f < n_chan; ++f)
        for (int t = 0; t < n_time; ++t) {
            int64_t p = 0;
            for (int i = 0; i < n_inputs; ++i) {
                int32_t r, m;
                oracle_decode(in[in_offset(layout, n_inputs, n_chan, n_time, f, t, i)], &r, &m);
                p += (int64_t)r * r + (int64_t)m * m;
            }
            out[(size_t)f * n_time + t] = p;
        }
    return 0;
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
