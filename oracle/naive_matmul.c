/*
 * FP64 naive matrix product, test infrastructure only (the oracle's side).
 *
 * This is the plain three-loop product of the paper's naive CPU method
 * (section 4.1): for every row i and column j, c[i][j] starts at zero and
 * accumulates a[i][k] * b[k][j] for k = 0 .. n-1 in ascending order.  All
 * matrices are n x n, row-major, float64.  Rows of c are independent, so
 * they may be spread over OpenMP threads without changing any result: every
 * c[i][j] is summed by one thread in the same k order.
 *
 * Nothing on the GPU side includes, links or calls this file.
 */
#include <stdint.h>

void oracle_naive_matmul_f64(const double *a, const double *b, double *c, int64_t n)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += a[i * n + k] * b[k * n + j];
            c[i * n + j] = acc;
        }
    }
}

/* Sets the OpenMP thread count for later calls (no effect without OpenMP). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Thread count OpenMP would use for the loop above (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
