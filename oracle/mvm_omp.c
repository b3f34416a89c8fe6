/*
 * Oracle: the H, uniform-H and H^2 products y := alpha * M * x + y (eq. 4)
 * in plain C, float64, parallel over independent clusters with OpenMP.
 *
 * TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
 * baseline may load this library.  The product path never does.
 *
 * Every function evaluates the plain definition of the product of the
 * stored matrix (the sum over the block leaves b = (t, s) of M_b x|s added
 * to y|t), grouped so that no two threads write the same entry:
 *   - coefficient vectors are computed one cluster or block per iteration;
 *   - y is written per leaf cluster r of the cluster tree: every block whose
 *     row cluster t contains r adds the rows of r of its product.  The leaf
 *     clusters partition the index set (Def. 2.1), so every row of y is
 *     written by exactly one iteration.
 * H   (Sec. 2.2, 3.1): t_b = X_b^T x|s, then y|r += alpha W_b|r diag(sigma_b) t_b
 *     and y|r += alpha D_b|r x|s.
 * UH  (Sec. 2.3, 3.2): s_s = X_s^T x|s for every column cluster, the
 *     coupling sums t_t = sum_b S_b s_s over the block row of t (eq. 5), then
 *     y|r += alpha (sum over t containing r of W_t|r t_t + dense rows).
 * H^2 (Sec. 2.4, 3.3): s at the leaves from the leaf bases, then level by
 *     level towards the root s_v = sum over sons c of F_c^T s_c; coupling sums
 *     as for UH; level by level from the root t_c += E_c t_parent; finally
 *     y|r += alpha (W_r t_r + dense rows) at the leaves.
 * Vectors are in cluster order.  Matrices are column-major (leading
 * dimension = row count), one pointer per block or node as in the ABI's
 * value set.  Each entry point returns the number of threads that ran.
 * A host STREAM-style triad (a = b + q c) measures the host's memory
 * bandwidth for the same report.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nnodes;
    const int64_t* begin;
    const int64_t* end;
    const int32_t* level;
    const int32_t* parent;
    const int32_t* son0;
    const int32_t* son1;
    int64_t nblocks;
    const int32_t* tau;
    const int32_t* sigma;
    const int32_t* adm;
} tree_t;

/* out[i - r0] += sum_j A[i + j m] v[j] for rows r0 <= i < r1 of an m x k matrix */
static void rows_times(const double* A, int64_t m, int64_t k, int64_t r0, int64_t r1, const double* v,
                       double* out) {
    for (int64_t j = 0; j < k; ++j) {
        const double vj = v[j];
        const double* col = A + j * m;
        for (int64_t i = r0; i < r1; ++i) out[i - r0] += col[i] * vj;
    }
}

/* out[j] = sum_i A[i + j m] v[i] for an m x k matrix (A^T v) */
static void transposed_times(const double* A, int64_t m, int64_t k, const double* v, double* out) {
    for (int64_t j = 0; j < k; ++j) {
        double acc = 0.0;
        const double* col = A + j * m;
        for (int64_t i = 0; i < m; ++i) acc += col[i] * v[i];
        out[j] = acc;
    }
}

static int64_t size_of(const tree_t* T, int32_t v) { return T->end[v] - T->begin[v]; }

/* blocks grouped by row cluster: first[v] .. first[v+1] in list */
static void block_rows(const tree_t* T, int64_t* first, int64_t* list) {
    memset(first, 0, sizeof(int64_t) * (T->nnodes + 1));
    for (int64_t b = 0; b < T->nblocks; ++b) first[T->tau[b] + 1]++;
    for (int32_t v = 0; v < T->nnodes; ++v) first[v + 1] += first[v];
    int64_t* fill = malloc(sizeof(int64_t) * (T->nnodes + 1));
    memcpy(fill, first, sizeof(int64_t) * (T->nnodes + 1));
    for (int64_t b = 0; b < T->nblocks; ++b) list[fill[T->tau[b]]++] = b;
    free(fill);
}

static int32_t leaf_list(const tree_t* T, int32_t* leaves) {
    int32_t nl = 0;
    for (int32_t v = 0; v < T->nnodes; ++v)
        if (T->son0[v] < 0) leaves[nl++] = v;
    return nl;
}

/* rows of leaf r from the dense blocks of the block row of t (t contains r) */
static void dense_rows(const tree_t* T, const int64_t* first, const int64_t* list, int32_t t, int32_t r,
                       const double* const* dense, const double* x, double* acc) {
    const int64_t r0 = T->begin[r] - T->begin[t], r1 = T->end[r] - T->begin[t];
    for (int64_t q = first[t]; q < first[t + 1]; ++q) {
        const int64_t b = list[q];
        if (T->adm[b]) continue;
        const int32_t s = T->sigma[b];
        rows_times(dense[b], size_of(T, t), size_of(T, s), r0, r1, x + T->begin[s], acc);
    }
}

int oracle_h_mvm(const tree_t* T, const double* const* dense, const int32_t* rank, const double* const* W,
                 const double* const* sv, const double* const* X, double alpha, const double* x, double* y,
                 int nthreads) {
    int used = 1;
    int64_t* first = malloc(sizeof(int64_t) * (T->nnodes + 1));
    int64_t* list = malloc(sizeof(int64_t) * (T->nblocks > 0 ? T->nblocks : 1));
    int32_t* leaves = malloc(sizeof(int32_t) * T->nnodes);
    int64_t* toff = malloc(sizeof(int64_t) * (T->nblocks + 1));
    block_rows(T, first, list);
    const int32_t nl = leaf_list(T, leaves);
    toff[0] = 0;
    for (int64_t b = 0; b < T->nblocks; ++b) toff[b + 1] = toff[b] + (T->adm[b] ? rank[b] : 0);
    double* tb = malloc(sizeof(double) * (toff[T->nblocks] > 0 ? toff[T->nblocks] : 1));
#pragma omp parallel num_threads(nthreads)
    {
#pragma omp single
        used = omp_get_num_threads();
        /* t_b = diag(sigma_b) X_b^T x|s for every low-rank block */
#pragma omp for schedule(dynamic, 16)
        for (int64_t b = 0; b < T->nblocks; ++b) {
            if (!T->adm[b] || rank[b] == 0) continue;
            const int32_t s = T->sigma[b];
            transposed_times(X[b], size_of(T, s), rank[b], x + T->begin[s], tb + toff[b]);
            for (int32_t j = 0; j < rank[b]; ++j) tb[toff[b] + j] *= sv[b][j];
        }
        /* y|r for every leaf r: all blocks whose row cluster contains r */
#pragma omp for schedule(dynamic, 4)
        for (int32_t q = 0; q < nl; ++q) {
            const int32_t r = leaves[q];
            const int64_t nr = size_of(T, r);
            double* acc = calloc(nr, sizeof(double));
            for (int32_t t = r; t >= 0; t = T->parent[t]) {
                const int64_t r0 = T->begin[r] - T->begin[t], r1 = T->end[r] - T->begin[t];
                for (int64_t e = first[t]; e < first[t + 1]; ++e) {
                    const int64_t b = list[e];
                    if (T->adm[b] && rank[b] > 0) rows_times(W[b], size_of(T, t), rank[b], r0, r1, tb + toff[b], acc);
                }
                dense_rows(T, first, list, t, r, dense, x, acc);
            }
            for (int64_t i = 0; i < nr; ++i) y[T->begin[r] + i] += alpha * acc[i];
            free(acc);
        }
    }
    free(tb);
    free(toff);
    free(leaves);
    free(list);
    free(first);
    return used;
}

int oracle_uh_mvm(const tree_t* T, const double* const* dense, const int32_t* row_rank, const int32_t* col_rank,
                  const double* const* row_basis, const double* const* col_basis, const double* const* coupling,
                  double alpha, const double* x, double* y, int nthreads) {
    int used = 1;
    int64_t* first = malloc(sizeof(int64_t) * (T->nnodes + 1));
    int64_t* list = malloc(sizeof(int64_t) * (T->nblocks > 0 ? T->nblocks : 1));
    int32_t* leaves = malloc(sizeof(int32_t) * T->nnodes);
    int64_t* soff = malloc(sizeof(int64_t) * (T->nnodes + 1));
    int64_t* toff = malloc(sizeof(int64_t) * (T->nnodes + 1));
    block_rows(T, first, list);
    const int32_t nl = leaf_list(T, leaves);
    soff[0] = toff[0] = 0;
    for (int32_t v = 0; v < T->nnodes; ++v) {
        soff[v + 1] = soff[v] + col_rank[v];
        toff[v + 1] = toff[v] + row_rank[v];
    }
    double* s = malloc(sizeof(double) * (soff[T->nnodes] + 1));
    double* t = calloc(toff[T->nnodes] + 1, sizeof(double));
#pragma omp parallel num_threads(nthreads)
    {
#pragma omp single
        used = omp_get_num_threads();
        /* forward transformation s_v = X_v^T x|v */
#pragma omp for schedule(dynamic, 16)
        for (int32_t v = 0; v < T->nnodes; ++v)
            if (col_rank[v] > 0) transposed_times(col_basis[v], size_of(T, v), col_rank[v], x + T->begin[v], s + soff[v]);
        /* coupling sums t_t = sum_b S_b s_s over the low-rank blocks of t's block row (eq. 5) */
#pragma omp for schedule(dynamic, 16)
        for (int32_t v = 0; v < T->nnodes; ++v) {
            if (row_rank[v] == 0) continue;
            for (int64_t e = first[v]; e < first[v + 1]; ++e) {
                const int64_t b = list[e];
                const int32_t c = T->sigma[b];
                if (!T->adm[b] || col_rank[c] == 0) continue;
                rows_times(coupling[b], row_rank[v], col_rank[c], 0, row_rank[v], s + soff[c], t + toff[v]);
            }
        }
        /* backward transformation and dense blocks, per leaf row cluster */
#pragma omp for schedule(dynamic, 4)
        for (int32_t q = 0; q < nl; ++q) {
            const int32_t r = leaves[q];
            const int64_t nr = size_of(T, r);
            double* acc = calloc(nr, sizeof(double));
            for (int32_t v = r; v >= 0; v = T->parent[v]) {
                const int64_t r0 = T->begin[r] - T->begin[v], r1 = T->end[r] - T->begin[v];
                if (row_rank[v] > 0) rows_times(row_basis[v], size_of(T, v), row_rank[v], r0, r1, t + toff[v], acc);
                dense_rows(T, first, list, v, r, dense, x, acc);
            }
            for (int64_t i = 0; i < nr; ++i) y[T->begin[r] + i] += alpha * acc[i];
            free(acc);
        }
    }
    free(t);
    free(s);
    free(toff);
    free(soff);
    free(leaves);
    free(list);
    free(first);
    return used;
}

int oracle_h2_mvm(const tree_t* T, const double* const* dense, const int32_t* row_rank, const int32_t* col_rank,
                  const double* const* row_leaf_basis, const double* const* row_transfer,
                  const double* const* col_leaf_basis, const double* const* col_transfer,
                  const double* const* coupling, double alpha, const double* x, double* y, int nthreads) {
    int used = 1;
    int64_t* first = malloc(sizeof(int64_t) * (T->nnodes + 1));
    int64_t* list = malloc(sizeof(int64_t) * (T->nblocks > 0 ? T->nblocks : 1));
    int32_t* leaves = malloc(sizeof(int32_t) * T->nnodes);
    int64_t* soff = malloc(sizeof(int64_t) * (T->nnodes + 1));
    int64_t* toff = malloc(sizeof(int64_t) * (T->nnodes + 1));
    block_rows(T, first, list);
    const int32_t nl = leaf_list(T, leaves);
    int32_t depth = 0;
    for (int32_t v = 0; v < T->nnodes; ++v) depth = T->level[v] > depth ? T->level[v] : depth;
    /* nodes grouped by level */
    int64_t* lfirst = calloc(depth + 2, sizeof(int64_t));
    int32_t* lnodes = malloc(sizeof(int32_t) * T->nnodes);
    for (int32_t v = 0; v < T->nnodes; ++v) lfirst[T->level[v] + 1]++;
    for (int32_t l = 0; l <= depth; ++l) lfirst[l + 1] += lfirst[l];
    {
        int64_t* fill = malloc(sizeof(int64_t) * (depth + 2));
        memcpy(fill, lfirst, sizeof(int64_t) * (depth + 2));
        for (int32_t v = 0; v < T->nnodes; ++v) lnodes[fill[T->level[v]]++] = v;
        free(fill);
    }
    soff[0] = toff[0] = 0;
    for (int32_t v = 0; v < T->nnodes; ++v) {
        soff[v + 1] = soff[v] + col_rank[v];
        toff[v + 1] = toff[v] + row_rank[v];
    }
    double* s = calloc(soff[T->nnodes] + 1, sizeof(double));
    double* t = calloc(toff[T->nnodes] + 1, sizeof(double));
#pragma omp parallel num_threads(nthreads)
    {
#pragma omp single
        used = omp_get_num_threads();
        /* upward pass, deepest level first: leaf bases, then s_v = sum_c F_c^T s_c */
        for (int32_t l = depth; l >= 0; --l) {
#pragma omp for schedule(dynamic, 16)
            for (int64_t q = lfirst[l]; q < lfirst[l + 1]; ++q) {
                const int32_t v = lnodes[q];
                if (col_rank[v] == 0) continue;
                if (T->son0[v] < 0) {
                    transposed_times(col_leaf_basis[v], size_of(T, v), col_rank[v], x + T->begin[v], s + soff[v]);
                } else {
                    const int32_t sons[2] = {T->son0[v], T->son1[v]};
                    for (int u = 0; u < 2; ++u) {
                        const int32_t c = sons[u];
                        if (col_rank[c] == 0) continue;
                        double* tmp = malloc(sizeof(double) * col_rank[v]);
                        transposed_times(col_transfer[c], col_rank[c], col_rank[v], s + soff[c], tmp);
                        for (int32_t j = 0; j < col_rank[v]; ++j) s[soff[v] + j] += tmp[j];
                        free(tmp);
                    }
                }
            }
        }
        /* coupling sums (eq. 5) */
#pragma omp for schedule(dynamic, 16)
        for (int32_t v = 0; v < T->nnodes; ++v) {
            if (row_rank[v] == 0) continue;
            for (int64_t e = first[v]; e < first[v + 1]; ++e) {
                const int64_t b = list[e];
                const int32_t c = T->sigma[b];
                if (!T->adm[b] || col_rank[c] == 0) continue;
                rows_times(coupling[b], row_rank[v], col_rank[c], 0, row_rank[v], s + soff[c], t + toff[v]);
            }
        }
        /* downward pass from the root: t_c += E_c t_parent */
        for (int32_t l = 1; l <= depth; ++l) {
#pragma omp for schedule(dynamic, 16)
            for (int64_t q = lfirst[l]; q < lfirst[l + 1]; ++q) {
                const int32_t c = lnodes[q];
                const int32_t p = T->parent[c];
                if (row_rank[c] == 0 || row_rank[p] == 0) continue;
                rows_times(row_transfer[c], row_rank[c], row_rank[p], 0, row_rank[c], t + toff[p], t + toff[c]);
            }
        }
        /* leaves: W_r t_r plus the dense rows of every block row containing r */
#pragma omp for schedule(dynamic, 4)
        for (int32_t q = 0; q < nl; ++q) {
            const int32_t r = leaves[q];
            const int64_t nr = size_of(T, r);
            double* acc = calloc(nr, sizeof(double));
            if (row_rank[r] > 0) rows_times(row_leaf_basis[r], nr, row_rank[r], 0, nr, t + toff[r], acc);
            for (int32_t v = r; v >= 0; v = T->parent[v]) dense_rows(T, first, list, v, r, dense, x, acc);
            for (int64_t i = 0; i < nr; ++i) y[T->begin[r] + i] += alpha * acc[i];
            free(acc);
        }
    }
    free(t);
    free(s);
    free(lnodes);
    free(lfirst);
    free(toff);
    free(soff);
    free(leaves);
    free(list);
    free(first);
    return used;
}

/* a[i] = b[i] + q c[i]; returns the threads that ran */
int oracle_triad(double* a, const double* b, const double* c, double q, int64_t n, int nthreads) {
    int used = 1;
#pragma omp parallel num_threads(nthreads)
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) a[i] = b[i] + q * c[i];
    }
    return used;
}
