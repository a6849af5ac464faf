/*
 * Exact K-nearest-neighbour search by definition -- oracle (test
 * infrastructure only; never linked into the product library).
 *
 * Section 2.1 (KNNS problem): delta(v, q) = sum over the D coordinates of
 * (v_i - q_i)^2.  Every float32 value is widened exactly to double and the
 * sum is accumulated in double, one coordinate after another.  The k
 * smallest (delta, row id) pairs are kept in ascending order by simple
 * insertion; rows beyond n are padded with id -1 and distance +inf.
 *
 * Parallelism: queries are independent; OpenMP splits the query loop.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* (da, ia) < (db, ib) in (distance, id) order */
static int pair_less(double da, int64_t ia, double db, int64_t ib) {
    return da < db || (da == db && ia < ib);
}

static void one_query(const float *x, int64_t n, int32_t d, const float *q, int32_t k,
                      int64_t *ids, double *dist) {
    for (int32_t j = 0; j < k; ++j) {
        ids[j] = -1;
        dist[j] = INFINITY;
    }
    for (int64_t v = 0; v < n; ++v) {
        const float *row = x + v * (int64_t)d;
        double s = 0.0;
        for (int32_t i = 0; i < d; ++i) {
            double t = (double)row[i] - (double)q[i];
            s += t * t;
        }
        /* insert (s, v) if it beats the current k-th pair */
        if (!pair_less(s, v, dist[k - 1], ids[k - 1]) && ids[k - 1] >= 0) continue;
        int32_t p = k - 1;
        while (p > 0 && (ids[p - 1] < 0 || pair_less(s, v, dist[p - 1], ids[p - 1]))) {
            dist[p] = dist[p - 1];
            ids[p] = ids[p - 1];
            --p;
        }
        dist[p] = s;
        ids[p] = v;
    }
}

int oracle_knn_fp64(const float *x, int64_t n, int32_t d, const float *queries, int64_t nq,
                    int32_t k, int64_t *out_ids, double *out_dist, int32_t threads) {
    if (!x || !queries || !out_ids || !out_dist || n < 0 || d < 1 || nq < 0 || k < 1) return -1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t qi = 0; qi < nq; ++qi)
        one_query(x, n, d, queries + qi * (int64_t)d, k, out_ids + qi * (int64_t)k,
                  out_dist + qi * (int64_t)k);
    return 0;
}
