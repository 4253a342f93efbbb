/*
 * Brute-force k-NN oracle (FP64) -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library.  It shares no code, header or constant with the HIP path.
 *
 * What it computes (the plain definition the paper's method reaches exactly):
 *   * P = (p_0 .. p_{n-1}) ordered by birth rank (Sec. 3, the prefix recurrence Eq. 2);
 *     the prefix P_{1:m} is the ranks r < m (Sec. 4.2, prefix-subset queries), minus
 *     ranks marked dead by a deletion (Sec. 4.3: after deleting p_i the structure must answer
 *     as if P \ {p_i} had been inserted in the original relative order).
 *   * D(r) = squared Euclidean distance (Sec. 2.2, Voronoi nearest neighbour), evaluated in
 *     float64 from float32 inputs with every operation rounded:
 *       dx = (double)q.x - (double)p.x  (likewise dy, dz);  D = (dx*dx + dy*dy) + dz*dz.
 *     This file must be compiled with -ffp-contract=off so that no FMA is formed.
 *   * The answer is the k candidates with the smallest key (D, r) in ascending order: ties
 *     in D go to the smaller (older) rank, as the strict comparison of the 1-NN descent in
 *     Alg. 1 keeps the older site.  Output distances are (float)sqrt(D).  When fewer than k
 *     live ranks exist below m, the row is padded with rank -1 and distance +inf.
 *
 * Implementation: for every query, one pass over the prefix keeps the k best keys in a
 * sorted array by insertion (no blocking, no reordering).  Queries are independent and
 * split across OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int key_less(double da, int32_t ra, double db, int32_t rb) {
    return da < db || (da == db && ra < rb);
}

static double sq_dist(const float *q, const float *p) {
    double dx = (double)q[0] - (double)p[0];
    double dy = (double)q[1] - (double)p[1];
    double dz = (double)q[2] - (double)p[2];
    double s = dx * dx;
    s = s + dy * dy;
    s = s + dz * dz;
    return s;
}

/* One query: fills idx[0..k-1], D[0..k-1] (sorted ascending by (D, rank)). */
static void knn_one(const float *pts, const uint8_t *live, const float *q, int32_t k,
                    int64_t m, int32_t *idx, double *D) {
    int32_t cnt = 0;
    for (int64_t r = 0; r < m; ++r) {
        if (live && !live[r]) continue;
        double d = sq_dist(q, pts + 3 * r);
        if (cnt == k && !key_less(d, (int32_t)r, D[k - 1], idx[k - 1])) continue;
        int32_t pos = cnt < k ? cnt : k - 1;
        while (pos > 0 && key_less(d, (int32_t)r, D[pos - 1], idx[pos - 1])) {
            D[pos] = D[pos - 1];
            idx[pos] = idx[pos - 1];
            --pos;
        }
        D[pos] = d;
        idx[pos] = (int32_t)r;
        if (cnt < k) ++cnt;
    }
    for (int32_t j = cnt; j < k; ++j) {
        idx[j] = -1;
        D[j] = INFINITY;
    }
}

/*
 * pts      float32 [n][3] by birth rank
 * live     uint8 [n] (1 = present) or NULL for all live
 * q        float32 [nq][3]
 * k_arr    int32 [nq] per-query k, or NULL to use k_scalar
 * m_arr    int32 [nq] per-query prefix, or NULL to use m_scalar
 * row_off  int64 [nq+1] output row offsets when k_arr is given (row i starts at row_off[i]);
 *          NULL means row i starts at i*k_scalar
 * out_idx  int32, out_dist float32, out_D float64 (out_D may be NULL)
 * Returns 0, or -1 on an invalid argument.
 */
int oracle_knn(const float *pts, int64_t n, const uint8_t *live, const float *q, int64_t nq,
               const int32_t *k_arr, int32_t k_scalar, const int32_t *m_arr, int64_t m_scalar,
               const int64_t *row_off, int32_t *out_idx, float *out_dist, double *out_D,
               int nthreads) {
    if (n < 1 || nq < 0 || !pts || (nq > 0 && (!q || !out_idx || !out_dist))) return -1;
    if (k_arr && !row_off) return -1;
    if (!k_arr && k_scalar < 1) return -1;
    int32_t kmax = k_scalar;
    if (k_arr) {
        kmax = 1;
        for (int64_t i = 0; i < nq; ++i) {
            if (k_arr[i] < 1) return -1;
            if (k_arr[i] > kmax) kmax = k_arr[i];
        }
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int bad = 0;
#pragma omp parallel
    {
        double *Dbuf = (double *)malloc(sizeof(double) * (size_t)kmax);
        int32_t *Ibuf = (int32_t *)malloc(sizeof(int32_t) * (size_t)kmax);
        if (!Dbuf || !Ibuf) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < nq; ++i) {
                int32_t k = k_arr ? k_arr[i] : k_scalar;
                int64_t m = m_arr ? (int64_t)m_arr[i] : m_scalar;
                if (m > n) m = n;
                if (m < 0) m = 0;
                int64_t off = row_off ? row_off[i] : i * (int64_t)k_scalar;
                knn_one(pts, live, q + 3 * i, k, m, Ibuf, Dbuf);
                for (int32_t j = 0; j < k; ++j) {
                    out_idx[off + j] = Ibuf[j];
                    out_dist[off + j] = Ibuf[j] < 0 ? INFINITY : (float)sqrt(Dbuf[j]);
                    if (out_D) out_D[off + j] = Dbuf[j];
                }
            }
        }
        free(Dbuf);
        free(Ibuf);
    }
    return bad ? -1 : 0;
}

/* Number of threads an OpenMP parallel region would use (for reporting). */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
