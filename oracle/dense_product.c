/*
 * Oracle: matrix-free dense kernel product  y[i] += alpha * sum_j k(p_i, p_j) x[j].
 *
 * TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
 * baseline may load this library.  The product path never does.
 *
 * This is the dense matrix the hierarchical formats approximate (Sec. 2.1:
 * the model problem's matrix is dense and non-zero everywhere).  The point
 * kernels stand in for the paper's Galerkin integrals:
 *   0  Laplace      1 / (4 pi |x - y|)
 *   1  screened     exp(-|x - y|) / |x - y|
 *   2  constant     1
 *   3  identity     delta_ij
 *   4  rank one     (1 + x_1)(2 + y_2 y_3)
 * with k(p_i, p_i) := 0 for every kernel except the identity.
 * The sum over j runs in increasing j, one row per OpenMP iteration, float64.
 */
#include <math.h>
#include <stdint.h>

static double kval(int kernel, const double* a, const double* b) {
    if (kernel == 2) return 1.0;
    if (kernel == 4) return (1.0 + a[0]) * (2.0 + b[1] * b[2]);
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (kernel == 0) return 1.0 / (4.0 * M_PI * r);
    return exp(-r) / r;
}

/* rows: the row indices to evaluate (original order); y has length n. */
void oracle_dense_product(const double* pts, int64_t n, int kernel, double alpha,
                          const double* x, double* y, const int64_t* rows, int64_t nrows) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t i = rows[q];
        double acc = 0.0;
        if (kernel == 3) {
            acc = x[i];
        } else {
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                acc += kval(kernel, pts + 3 * i, pts + 3 * j) * x[j];
            }
        }
        y[i] += alpha * acc;
    }
}

/* squared Frobenius norm of the kernel matrix (diagonal excluded), float64 */
double oracle_kernel_fro2(const double* pts, int64_t n, int kernel) {
    double tot = 0.0;
    #pragma omp parallel for reduction(+:tot) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        if (kernel == 3) { acc = 1.0; }
        else {
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double v = kval(kernel, pts + 3 * i, pts + 3 * j);
                acc += v * v;
            }
        }
        tot += acc;
    }
    return tot;
}
