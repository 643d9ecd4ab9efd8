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
 *  - orc_nn_many_blocked: the same 1-NN by definition, eight queries per pass over the
 *    collection (the eight running sums of one series advance together; each pair's arithmetic
 *    and the tie rule are those of orc_nn_many, so the results are bit-identical). Used where
 *    tests check many queries against large collections.
 *  - orc_lb2: squared iSAX lower bound (Section 3.3.1: ABOVE / BELOW / IN branches;
 *    L * sum_s delta_s^2, ascending s).
 *  - orc_exact_search: serial twin of ParIS+ exact search (Section 3.3.3: ExactSearch with its
 *    LBC and RDC workers, run by one thread), step for step as the numpy twin
 *    oracle/reference.py:exact_search: the approximate search's members give the first
 *    best-so-far; every series gets its lower bound; those not above the best-so-far are sorted
 *    by (bound, index) and refined with early abandoning.
 */
#define _ISOC11_SOURCE
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

/* ---- eight queries per pass ------------------------------------------------------------ */
#define QB 8
typedef struct {
    const float *Q, *X;
    int64_t M, N;
    int32_t n;
    int64_t *idx;
    double *d2;
    int64_t next;           /* next group of QB queries; protected by mu */
    pthread_mutex_t mu;
} nnb_job;

/* The distances of one series to the QB queries of a group, each summed in ascending j with
   one rounding per operation: lane k of the vectors holds query k's running sum (vector
   subtract, multiply and add are the IEEE operations of the scalar loop, lane by lane). */
typedef double v4d __attribute__((vector_size(32)));
#define ROW_DISTANCES_BODY                                                           \
    v4d a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};                        \
    for (int32_t j = 0; j < n; ++j) {                                                \
        const double xv = (double)x[j];                                              \
        const v4d xj = {xv, xv, xv, xv};                                             \
        const v4d d0 = qd[2 * j] - xj, d1 = qd[2 * j + 1] - xj;                      \
        const v4d t0 = d0 * d0, t1 = d1 * d1;                                        \
        a0 = a0 + t0;                                                                \
        a1 = a1 + t1;                                                                \
    }                                                                                \
    for (int k = 0; k < 4; ++k) { out[k] = a0[k]; out[4 + k] = a1[k]; }

__attribute__((target("avx2"))) static void row_distances_avx2(const v4d *qd, const float *x, int32_t n,
                                                                 double *out)
{
    ROW_DISTANCES_BODY
}

static void row_distances_plain(const v4d *qd, const float *x, int32_t n, double *out)
{
    ROW_DISTANCES_BODY
}

static void *nnb_worker(void *arg)
{
    nnb_job *J = (nnb_job *)arg;
    const int32_t n = J->n;
    v4d *qd = (v4d *)aligned_alloc(32, sizeof(v4d) * 2 * (size_t)n);   /* exact float64 copies */
    if (!qd) return NULL;
    const int avx2 = __builtin_cpu_supports("avx2");
    for (;;) {
        pthread_mutex_lock(&J->mu);
        const int64_t m0 = J->next;
        J->next += QB;
        pthread_mutex_unlock(&J->mu);
        if (m0 >= J->M) break;
        const int64_t cnt = J->M - m0 < QB ? J->M - m0 : QB;
        for (int32_t j = 0; j < n; ++j)
            for (int k = 0; k < QB; ++k)
                qd[2 * j + k / 4][k % 4] = (double)J->Q[(m0 + (k < cnt ? k : 0)) * (int64_t)n + j];
        double best[QB];
        int64_t bi[QB];
        for (int k = 0; k < QB; ++k) { best[k] = INFINITY; bi[k] = -1; }
        for (int64_t i = 0; i < J->N; ++i) {
            const float *x = J->X + i * (int64_t)n;
            double a[QB];
            if (avx2) row_distances_avx2(qd, x, n, a);
            else row_distances_plain(qd, x, n, a);
            for (int k = 0; k < QB; ++k)
                if (a[k] < best[k]) { best[k] = a[k]; bi[k] = i; }
        }
        for (int k = 0; k < cnt; ++k) {
            J->idx[m0 + k] = bi[k];
            J->d2[m0 + k] = best[k];
        }
    }
    free(qd);
    return NULL;
}

int orc_nn_many_blocked(const float *Q, int64_t M, const float *X, int64_t N, int32_t n, int32_t threads,
                        int64_t *idx, double *d2)
{
    nnb_job J;
    J.Q = Q; J.X = X; J.M = M; J.N = N; J.n = n; J.idx = idx; J.d2 = d2; J.next = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (threads < 1) threads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    if (!th) return -1;
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&th[t], NULL, nnb_worker, &J) == 0) ++started;
    if (started == 0) nnb_worker(&J);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&J.mu);
    return started;
}

/* ---- serial exact-search twin ---------------------------------------------------------- */
typedef struct { double lb; int64_t i; } lb_entry;

static int lb_entry_cmp(const void *pa, const void *pb)
{
    const lb_entry *a = (const lb_entry *)pa, *b = (const lb_entry *)pb;
    if (a->lb < b->lb) return -1;
    if (a->lb > b->lb) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

/* Pruning test of the twin: a bound or a best-so-far comparison keeps the same slack as the
   numpy twin (relative 1e-9, absolute 1e-12), which covers the rounding of the PAA values. */
static int pruned(double v, double bsf) { return v > bsf * (1.0 + 1e-9) + 1e-12; }

/*
 * q            float32 [n] query; X float32 [N][n]; sym uint8 [N][w] iSAX words of X
 * members      series of the approximate search's leaf (n_members of them; may be 0)
 * qpaa         float64 [w] PAA of the query (the numpy oracle's paa())
 * beta257      region boundaries (index 0 = -inf, 256 = +inf)
 * out_idx/out_d2: the answer; counters (may be NULL): [0] seed index, [1] lb survivors,
 * [2] refined, [3] abandoned, [4] best-so-far updates. Returns 0, or -1 if out of memory.
 */
int orc_exact_search(const float *q, const float *X, int64_t N, int32_t n, const uint8_t *sym,
                     int32_t w, const int64_t *members, int64_t n_members, const double *qpaa,
                     const double *beta257, int64_t *out_idx, double *out_d2, int64_t *counters)
{
    const int32_t L = n / w;
    double bsf = INFINITY;
    int64_t bsf_i = -1;
    /* 1. approximate search: the smallest distance over the leaf's members, ties lowest index */
    for (int64_t k = 0; k < n_members; ++k) {
        const int64_t i = members[k];
        const double d = ed2_row(q, X + i * (int64_t)n, n);
        if (d < bsf || (d == bsf && i < bsf_i)) { bsf = d; bsf_i = i; }
    }
    const int64_t seed_i = bsf_i;
    /* 2. lower bound of every series; the ones not above the best-so-far are candidates */
    lb_entry *cand = (lb_entry *)malloc(sizeof(lb_entry) * (size_t)(N > 0 ? N : 1));
    if (!cand) return -1;
    int64_t nc = 0;
    for (int64_t i = 0; i < N; ++i) {
        double acc = 0.0;
        for (int32_t s = 0; s < w; ++s) {
            const int c = sym[i * w + s];
            const double lo = beta257[c], hi = beta257[c + 1], qv = qpaa[s];
            double d = 0.0;
            if (qv < lo) d = lo - qv;
            else if (qv > hi) d = qv - hi;
            acc = acc + d * d;
        }
        const double lb = (double)L * acc;
        if (!pruned(lb, bsf)) { cand[nc].lb = lb; cand[nc].i = i; ++nc; }
    }
    /* 3. candidates in ascending (bound, index) */
    qsort(cand, (size_t)nc, sizeof(lb_entry), lb_entry_cmp);
    /* 4. refinement: re-check against the current best-so-far, early-abandoning distance */
    int64_t refined = 0, abandoned = 0, updates = 0;
    for (int64_t k = 0; k < nc; ++k) {
        const int64_t i = cand[k].i;
        if (pruned(cand[k].lb, bsf)) continue;
        ++refined;
        const float *x = X + i * (int64_t)n;
        double acc = 0.0;
        int ab = 0;
        for (int32_t j = 0; j < n; ++j) {
            const double d = (double)q[j] - (double)x[j];
            const double t = d * d;
            acc = acc + t;
            if (acc > bsf) { ab = 1; break; }
        }
        if (ab) { ++abandoned; continue; }
        if (acc < bsf || (acc == bsf && i < bsf_i)) { bsf = acc; bsf_i = i; ++updates; }
    }
    free(cand);
    *out_idx = bsf_i;
    *out_d2 = bsf;
    if (counters) {
        counters[0] = seed_i;
        counters[1] = nc;
        counters[2] = refined;
        counters[3] = abandoned;
        counters[4] = updates;
    }
    return 0;
}
