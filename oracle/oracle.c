/*
 * FP64 CPU oracle for the 1-D complex discrete Fourier transform.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * What it computes (Hunt, Mullin, Rosenkrantz, Raynolds, "A
 * Transformation-Based Approach for the Design of Parallel/Distributed
 * Scientific Software: the FFT", Section 2.1, Fig. 2.1):
 *
 *     X[k] = sum_{j<n} x[j] * w_n^(sign*j*k),  w_n = exp(2*pi*i/n),
 *
 * for n = 2^t, t >= 1, with no scaling in either direction and the output in
 * natural order.  sign is a parameter: the paper's own loops use the +1
 * exponent (Section 3, Fig. 3.8 / 3.9 weights EXP(2*pi*i*row/L)); the usual
 * forward transform is sign = -1.
 *
 * Data layout: interleaved complex, x[2*j] = Re x_j, x[2*j+1] = Im x_j.
 *
 * Functions:
 *   oracle_dft        the definition written out, O(n^2).  The exponent j*k
 *                     is reduced modulo n in integers before one cos/sin per
 *                     term, so each term's weight carries one rounding.
 *   oracle_fft        Fig. 2.1 in recursive form: the input is split into its
 *                     even and odd subsequences (which, applied all the way
 *                     down, is the bit-reversal permutation P_n of line (1)),
 *                     and each level combines two half-length results with
 *                     the butterfly matrix B_L = [[I, Omega],[I, -Omega]],
 *                     Omega = diag(1, w_L, ..., w_L^(L/2-1)) (line (6)).  Each
 *                     weight is computed directly from its integer exponent
 *                     (no recurrence), as in Section 3.5, Fig. 3.8.
 *   oracle_fft_batch  oracle_fft over a contiguous batch, spread over POSIX
 *                     threads (one transform per task).
 *
 * Pins (tests that fix this file to something other than itself) live in
 * tests/test_oracle_pins.py: brute force against oracle_dft for n <= 256,
 * closed forms (delta -> all ones, pure tone -> n*delta, n = 2 and n = 4 by
 * hand), Parseval, linearity, shift theorem, round trip, Hermitian symmetry
 * of real input, a numpy.fft cross-check, and an independent numpy
 * restatement of the paper's staged radix-2 loop and its Section 4
 * block/cyclic plan (tests/paper_plan.py, written from the prose of
 * Sections 2-4, not a transcription of the printed loop nests).
 *
 * Build: gcc -O2 -std=c99 -fPIC -shared (no -ffast-math; IEEE round to
 * nearest even).
 */
#define _POSIX_C_SOURCE 200809L
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_OOM (-2)

static const double TWO_PI = 6.283185307179586476925286766559;

static int is_pow2_ge2(int64_t n) { return n >= 2 && (n & (n - 1)) == 0; }

/* The definition, term by term. */
int oracle_dft(const double *x, double *X, int64_t n, int sign)
{
    if (!x || !X || n < 1 || (sign != 1 && sign != -1)) return ORACLE_E_ARG;
    if (n > (int64_t)1 << 30) return ORACLE_E_ARG;
    for (int64_t k = 0; k < n; ++k) {
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            uint64_t e = ((uint64_t)j * (uint64_t)k) % (uint64_t)n;
            double a = TWO_PI * (double)e / (double)n;
            double wr = cos(a), wi = (double)sign * sin(a);
            double xr = x[2 * j], xi = x[2 * j + 1];
            re += xr * wr - xi * wi;
            im += xr * wi + xi * wr;
        }
        X[2 * k] = re;
        X[2 * k + 1] = im;
    }
    return ORACLE_OK;
}

/*
 * One level of Fig. 2.1 for a sub-transform of length L whose input is the
 * subsequence x[0], x[s], x[2s], ... (s = n/L after the even/odd splits).
 * out[0..L/2) receives the transform of the even-indexed half and
 * out[L/2..L) that of the odd-indexed half; then B_L combines them:
 *     out[r]       = even[r] + w_L^(sign*r) * odd[r]
 *     out[r + L/2] = even[r] - w_L^(sign*r) * odd[r]
 * The weight w_L^r equals w_n^(r*n/L): it is read from a table of w_n^e,
 * e < n/2, each entry computed directly with cos/sin.
 */
static void fft_level(const double *x, int64_t s, double *out, int64_t L,
                      const double *wtab, int64_t n)
{
    if (L == 1) {
        out[0] = x[0];
        out[1] = x[1];
        return;
    }
    int64_t h = L / 2;
    fft_level(x, 2 * s, out, h, wtab, n);
    fft_level(x + 2 * s, 2 * s, out + 2 * h, h, wtab, n);
    int64_t step = n / L;
    for (int64_t r = 0; r < h; ++r) {
        double wr = wtab[2 * (r * step)], wi = wtab[2 * (r * step) + 1];
        double er = out[2 * r], ei = out[2 * r + 1];
        double orr = out[2 * (r + h)], oi = out[2 * (r + h) + 1];
        double cr = wr * orr - wi * oi;
        double ci = wr * oi + wi * orr;
        out[2 * r] = er + cr;
        out[2 * r + 1] = ei + ci;
        out[2 * (r + h)] = er - cr;
        out[2 * (r + h) + 1] = ei - ci;
    }
}

/* Table of w_n^(sign*e) for e < n/2, each computed directly. */
static double *weight_table(int64_t n, int sign)
{
    int64_t h = n / 2;
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)(h > 0 ? h : 1));
    if (!w) return NULL;
    for (int64_t e = 0; e < h; ++e) {
        double a = TWO_PI * (double)e / (double)n;
        w[2 * e] = cos(a);
        w[2 * e + 1] = (double)sign * sin(a);
    }
    return w;
}

static int fft_one(const double *x, double *X, int64_t n, const double *wtab)
{
    fft_level(x, 1, X, n, wtab, n);
    return ORACLE_OK;
}

int oracle_fft(const double *x, double *X, int64_t n, int sign)
{
    if (!x || !X || !is_pow2_ge2(n) || (sign != 1 && sign != -1)) return ORACLE_E_ARG;
    if (x == X) return ORACLE_E_ARG; /* out of place only */
    double *w = weight_table(n, sign);
    if (!w) return ORACLE_E_OOM;
    int rc = fft_one(x, X, n, w);
    free(w);
    return rc;
}

typedef struct {
    const double *x;
    double *X;
    int64_t n, batch;
    const double *w;
    int64_t next;
    pthread_mutex_t mu;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *job = (batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->mu);
        int64_t b = job->next++;
        pthread_mutex_unlock(&job->mu);
        if (b >= job->batch) break;
        fft_one(job->x + 2 * b * job->n, job->X + 2 * b * job->n, job->n, job->w);
    }
    return NULL;
}

int oracle_fft_batch(const double *x, double *X, int64_t n, int64_t batch, int sign,
                     int nthreads)
{
    if (!x || !X || !is_pow2_ge2(n) || batch < 0 || (sign != 1 && sign != -1))
        return ORACLE_E_ARG;
    if (x == X) return ORACLE_E_ARG;
    if (batch == 0) return ORACLE_OK;
    double *w = weight_table(n, sign);
    if (!w) return ORACLE_E_OOM;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > batch) nthreads = (int)batch;
    batch_job job = {x, X, n, batch, w, 0, PTHREAD_MUTEX_INITIALIZER};
    pthread_t *tid = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!tid) {
        free(w);
        return ORACLE_E_OOM;
    }
    for (int i = 1; i < nthreads; ++i) {
        if (pthread_create(&tid[i], NULL, batch_worker, &job) != 0) {
            nthreads = i; /* run with the threads that did start */
            break;
        }
    }
    batch_worker(&job);
    for (int i = 1; i < nthreads; ++i) pthread_join(tid[i], NULL);
    free(tid);
    free(w);
    return ORACLE_OK;
}
