/*
 * CPU oracle for the X-engine correlation -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU baseline
 * build, load or call this file.  It shares no code, header or table with
 * the GPU library and is deliberately the plain definition, written out:
 * no blocking, no packing tricks, int64 sums.
 *
 * What is computed (Sec. 2.2, "Computational Requirements"):
 *   - each sample is one byte, 4 bits of real and 4 bits of imaginary part;
 *     the part is stored offset-binary, value = nibble - 8, real part in the
 *     high nibble unless `re_low` asks for the other order;
 *   - for every pair of inputs 0 <= i <= j < N -- the N(N+1)/2 products per
 *     sample that the cost model eta = dnu * N(N+1)/2 counts, autocorrelations
 *     included -- the visibility
 *         V_ij = sum_t x_i(t) * conj(x_j(t))
 *              = sum_t (re_i re_j + im_i im_j) + j (im_i re_j - re_i im_j).
 *
 * Output: int64 (Re, Im) pairs.  Packed mode writes the upper triangle row
 * by row, pair (i, j) at index i*N - i*(i-1)/2 + (j - i); full mode writes
 * the whole N x N matrix (row i, column j) so that Hermitian symmetry can be
 * checked.
 */
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Decode one stored nibble into its signed value. */
static int nibble_value(unsigned nib) { return (int)nib - 8; }

/*
 * samples    : uint8, sample t of input i at samples[t * row_stride + i]
 * n_samples  : T >= 0
 * n_inputs   : N >= 1
 * row_stride : bytes between consecutive time samples, >= N
 * re_low     : 0 = real part in the high nibble, 1 = in the low nibble
 * full       : 0 = packed upper triangle [N(N+1)/2][2], 1 = full [N][N][2]
 * out        : int64 output, overwritten
 * returns 0, or -1 on bad arguments / allocation failure
 */
int xo_correlate(const uint8_t *samples, int64_t n_samples, int64_t n_inputs,
                 int64_t row_stride, int re_low, int full, int64_t *out)
{
    if (!samples || !out || n_samples < 0 || n_inputs < 1 || row_stride < n_inputs)
        return -1;
    const int64_t T = n_samples, N = n_inputs;

    /* Decode into per-input rows so the sum over t reads memory in order. */
    int8_t *re = (int8_t *)malloc((size_t)(N * (T > 0 ? T : 1)));
    int8_t *im = (int8_t *)malloc((size_t)(N * (T > 0 ? T : 1)));
    if (!re || !im) { free(re); free(im); return -1; }
    for (int64_t t = 0; t < T; ++t) {
        for (int64_t i = 0; i < N; ++i) {
            unsigned b = samples[t * row_stride + i];
            unsigned hi = b >> 4, lo = b & 15u;
            re[i * T + t] = (int8_t)nibble_value(re_low ? lo : hi);
            im[i * T + t] = (int8_t)nibble_value(re_low ? hi : lo);
        }
    }

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < N; ++i) {
        const int8_t *ri = re + i * T, *ii = im + i * T;
        for (int64_t j = (full ? 0 : i); j < N; ++j) {
            const int8_t *rj = re + j * T, *ij = im + j * T;
            int64_t vr = 0, vi = 0;
            for (int64_t t = 0; t < T; ++t) {
                /* x_i * conj(x_j) with x = re + j im */
                vr += (int64_t)ri[t] * rj[t] + (int64_t)ii[t] * ij[t];
                vi += (int64_t)ii[t] * rj[t] - (int64_t)ri[t] * ij[t];
            }
            int64_t k = full ? (i * N + j) : (i * N - i * (i - 1) / 2 + (j - i));
            out[2 * k] = vr;
            out[2 * k + 1] = vi;
        }
    }
    free(re);
    free(im);
    return 0;
}

/* Threads of later parallel regions (n >= 1; ignored without OpenMP). */
void xo_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of threads an OpenMP parallel region would use (0 without OpenMP). */
int xo_num_threads(void)
{
#ifdef _OPENMP
    int n = 0;
    #pragma omp parallel
    {
        #pragma omp single
        n = omp_get_num_threads();
    }
    return n;
#else
    return 1;
#endif
}
