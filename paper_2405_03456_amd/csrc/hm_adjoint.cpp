// The adjoint M^T of a hierarchical matrix as a hierarchical matrix of the
// same form over the transposed block tree (the remark after Alg. 3: the
// adjoint product runs over block columns; all data is real, so the adjoint
// is the transpose).  Block b of the transposed layout is (sigma_b, tau_b):
//   dense     D_b^T (a transposed copy),
//   H         (W diag(sigma) X^T)^T = X diag(sigma) W^T: the factors swap,
//   UH        M_b^T = X_s S_b^T W_t^T: row and column bases (with their
//             ranks and weights) swap, couplings are transposed copies,
//   H2        as UH, and the row and column transfer matrices swap.
// The cluster tree is shared (M is square over one index set), so only the
// block list changes.
#include <new>
#include <vector>

#include "hm_pack.h"

namespace hm {

namespace {

// column-major m x k  ->  k x m
void transpose_into(const double* A, int64_t m, int64_t k, std::vector<double>& out) {
    out.resize((size_t)(m * k));
    for (int64_t j = 0; j < k; ++j)
        for (int64_t i = 0; i < m; ++i) out[(size_t)(j + i * k)] = A[i + j * m];
}

}  // namespace

hm_status transpose_matrix(const Layout& L, int32_t format, const hm_values* v, Transposed& T) {
    T = Transposed{};
    T.layout.L = L;
    T.layout.L.blk_tau = L.blk_sigma;
    T.layout.L.blk_sigma = L.blk_tau;
    const size_t nb = L.blk_tau.size(), nn = L.node_begin.size();
    T.store.reserve(nb);
    T.dense.assign(nb, nullptr);
    for (size_t b = 0; b < nb; ++b) {
        if (L.blk_adm[b] || !v->dense || !v->dense[b]) continue;
        T.store.emplace_back();
        transpose_into(v->dense[b], L.size(L.blk_tau[b]), L.size(L.blk_sigma[b]), T.store.back());
        T.dense[b] = T.store.back().data();
    }
    T.v.dense = T.dense.data();
    if (format == HM_FMT_H) {
        T.v.rank = v->rank;
        T.v.W = v->X;
        T.v.X = v->W;
        T.v.sigma = v->sigma;
    } else {
        T.v.row_rank = v->col_rank;
        T.v.col_rank = v->row_rank;
        T.v.row_basis = v->col_basis;
        T.v.col_basis = v->row_basis;
        T.v.row_sv = v->col_sv;
        T.v.col_sv = v->row_sv;
        T.v.row_transfer = v->col_transfer;
        T.v.col_transfer = v->row_transfer;
        T.coupling.assign(nb, nullptr);
        for (size_t b = 0; b < nb; ++b) {
            if (!L.blk_adm[b] || !v->coupling || !v->coupling[b]) continue;
            const int32_t kr = v->row_rank[L.blk_tau[b]], kc = v->col_rank[L.blk_sigma[b]];
            if ((int64_t)kr * kc == 0) continue;
            T.store.emplace_back();
            transpose_into(v->coupling[b], kr, kc, T.store.back());
            T.coupling[b] = T.store.back().data();
        }
        T.v.coupling = T.coupling.data();
    }
    (void)nn;
    return HM_OK;
}

}  // namespace hm
