/*
 * Plain C oracle for exact 1-NN search over iSAX summaries.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark; never by the product library. It shares no code or headers with the GPU library.
 * Built with -O2 -ffp-contract=off so every float64 operation is rounded on its own, in the same
 * order as the numpy oracle (oracle/reference.py); the two are checked bit-for-bit.
 *
 *  - orc_summarise: PAA (Section 2.2: segment means; ascending float64 sum, then / L) and the
 *    8-bit iSAX symbol (count of Gaussian boundaries <= the mean; boundaries passed in).
 *  - orc_ed2 / orc_ed2_at: squared Euclidean distance (Section 2.1), float64, ascending j:
 *    d = q_j - x_j; t = d * d; acc = acc + t.
 *  - orc_nn_many: the 1-NN by definition (Section 2.1), ties to the lowest index, for many
 *    queries; queries are split over POSIX threads (each query's arithmetic is unchanged).
 *  - orc_lb2: squared iSAX lower bound (Section 3.3.1: ABOVE / BELOW / IN branches;
 *    L * sum_s delta_s^2, ascending s).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void orc_summarise(const float *x, int64_t N, int32_t n, int32_t w, const double *beta257,
                   double *paa_out, uint8_t *sym_out)
{
    const int32_t L = n / w;
    for (int64_t i = 0; i < N; ++i) {
        const float *row = x + i * (int64_t)n;
        for (int32_t s = 0; s < w; ++s) {
            double acc = 0.0;
            for (int32_t j = 0; j < L; ++j)
                acc = acc + (double)row[s * L + j];
            const double m = acc / (double)L;
            int c = 0;
            for (int k = 1; k <= 255; ++k)
                if (beta257[k] <= m) c = k;  /* boundaries ascend: last k with beta_k <= m */
            if (paa_out) paa_out[i * w + s] = m;
            if (sym_out) sym_out[i * w + s] = (uint8_t)c;
        }
    }
}

static double ed2_row(const float *q, const float *x, int32_t n)
{
    double acc = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        const double d = (double)q[j] - (double)x[j];
        const double t = d * d;
        acc = acc + t;
    }
    return acc;
}

void orc_ed2(const float *q, const float *X, int64_t N, int32_t n, double *out)
{
    for (int64_t i = 0; i < N; ++i) out[i] = ed2_row(q, X + i * (int64_t)n, n);
}

void orc_ed2_at(const float *q, const float *X, int32_t n, const int64_t *idx, int64_t K,
                double *out)
{
    for (int64_t k = 0; k < K; ++k) out[k] = ed2_row(q, X + idx[k] * (int64_t)n, n);
}

typedef struct {
    const float *Q, *X;
    int64_t M, N;
    int32_t n;
    int64_t *idx;
    double *d2;
    int64_t next;           /* next query to take; protected by mu */
    pthread_mutex_t mu;
} nn_job;

static void *nn_worker(void *arg)
{
    nn_job *J = (nn_job *)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        const int64_t m = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (m >= J->M) break;
        const float *q = J->Q + m * (int64_t)J->n;
        double best = INFINITY;
        int64_t bi = -1;
        for (int64_t i = 0; i < J->N; ++i) {
            const double d = ed2_row(q, J->X + i * (int64_t)J->n, J->n);
            if (d < best) { best = d; bi = i; }  /* strict: first (lowest) index keeps a tie */
        }
        J->idx[m] = bi;
        J->d2[m] = best;
    }
    return NULL;
}

int orc_nn_many(const float *Q, int64_t M, const float *X, int64_t N, int32_t n, int32_t threads,
                int64_t *idx, double *d2)
{
    nn_job J;
    J.Q = Q; J.X = X; J.M = M; J.N = N; J.n = n; J.idx = idx; J.d2 = d2; J.next = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (threads < 1) threads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    if (!th) return -1;
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&th[t], NULL, nn_worker, &J) == 0) ++started;
    if (started == 0) nn_worker(&J);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&J.mu);
    return started;
}

void orc_lb2(const double *qpaa, const uint8_t *sym, int64_t N, int32_t w, int32_t L,
             const double *beta257, double *out)
{
    for (int64_t i = 0; i < N; ++i) {
        double acc = 0.0;
        for (int32_t s = 0; s < w; ++s) {
            const int c = sym[i * w + s];
            const double lo = beta257[c], hi = beta257[c + 1], qv = qpaa[s];
            double d = 0.0;
            if (qv < lo) d = lo - qv;        /* BELOW the region */
            else if (qv > hi) d = qv - hi;   /* ABOVE the region */
            acc = acc + d * d;               /* IN: contributes 0 */
        }
        out[i] = (double)L * acc;
    }
}
