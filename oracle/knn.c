/*
 * Oracle for the smoothing lengths (Sec. 3.1) -- TEST INFRASTRUCTURE ONLY.
 *
 * The smoothing length of a particle is the radius that holds its N_sph
 * nearest neighbours: the distance to its k-th nearest other particle (the
 * particle itself excluded, coincident particles counted at distance 0), in
 * projection (2D) or in space (3D, which the paper finds better), and with
 * several species only among particles of its own species.  Written as the
 * definition: every squared distance dx^2 + dy^2 (+ dz^2), then the k-th
 * smallest by selection, then its square root.  O(n^2).
 */
#include <math.h>
#include <stdlib.h>

#include "oracle.h"

/* k-th smallest (1-based) of a[0..n-1] by quickselect (a is reordered). */
static double kth_smallest(double* a, int64_t n, int64_t k)
{
    int64_t lo = 0, hi = n - 1, want = k - 1;
    while (lo < hi) {
        const double pivot = a[lo + (hi - lo) / 2];
        int64_t i = lo, j = hi;
        while (i <= j) {
            while (a[i] < pivot) ++i;
            while (a[j] > pivot) --j;
            if (i <= j) {
                const double t = a[i];
                a[i] = a[j];
                a[j] = t;
                ++i;
                --j;
            }
        }
        if (want <= j) hi = j;
        else if (want >= i) lo = i;
        else return a[want];
    }
    return a[want];
}

int ora_knn(const double* x, const double* y, int64_t n, int k, double* s_out, int nthreads)
{
    return ora_knn_ex(x, y, NULL, NULL, n, k, NULL, n, s_out, nthreads);
}

int ora_knn_at(const double* x, const double* y, int64_t n, int k, const int64_t* queries, int64_t nq,
               double* s_out, int nthreads)
{
    return ora_knn_ex(x, y, NULL, NULL, n, k, queries, nq, s_out, nthreads);
}

int ora_knn_ex(const double* x, const double* y, const double* z, const int32_t* species, int64_t n, int k,
               const int64_t* queries, int64_t nq, double* s_out, int nthreads)
{
    if (n < 2 || k < 1 || k > n - 1) return -1;
    int bad = 0;
#pragma omp parallel num_threads(nthreads)
    {
        double* d2 = (double*)malloc(sizeof(double) * (size_t)(n - 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nq; ++t) {
            const int64_t i = queries ? queries[t] : t;
            int64_t m = 0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                if (species && species[j] != species[i]) continue;
                const double dx = x[i] - x[j], dy = y[i] - y[j];
                double r2 = dx * dx + dy * dy;
                if (z) {
                    const double dz = z[i] - z[j];
                    r2 = r2 + dz * dz;
                }
                d2[m++] = r2;
            }
            if (m < k) {
#pragma omp atomic write
                bad = 1;
                s_out[t] = NAN;
            } else {
                s_out[t] = sqrt(kth_smallest(d2, m, k));
            }
        }
        free(d2);
    }
    return bad ? -1 : 0;
}
