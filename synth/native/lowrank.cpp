// Native part of the input generator: kernel blocks and eps-truncated
// low-rank factors for large problems.
//
// Low-rank blocks: adaptive cross approximation with partial pivoting
// (Bebendorf) builds M ~ U V^T from O(k) kernel rows and columns, stopping
// when the last cross ||u||*||v|| falls below eps/20 of the running
// Frobenius estimate twice in a row; then U = Q1 R1, V = Q2 R2 (Householder),
// R1 R2^T = A S B^T (one-sided Jacobi SVD), and the result is truncated with
// the Frobenius rule sqrt(sum_{i>=k} s_i^2) <= eps * ||s||_2, giving
// W = Q1 A_k, sigma = s_k, X = Q2 B_k.
//
// This only produces inputs; the achieved accuracy is measured against the
// dense kernel product, never assumed.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

struct Pts {
    const double* p;   // cluster order, n x 3
    int kernel;
};

inline double kval(const Pts& P, int64_t i, int64_t j) {
    if (i == j) return P.kernel == 3 ? 1.0 : 0.0;
    const double* a = P.p + 3 * i;
    const double* b = P.p + 3 * j;
    switch (P.kernel) {
        case 2: return 1.0;
        case 3: return 0.0;
        case 4: return (1.0 + a[0]) * (2.0 + b[1] * b[2]);
        default: break;
    }
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    double r = std::sqrt(dx * dx + dy * dy + dz * dz);
    if (P.kernel == 0) return 1.0 / (4.0 * M_PI * r);
    return std::exp(-r) / r;
}

// Householder QR of A (m x k, col-major, m >= k assumed or handled): returns
// Q (m x kk) explicit and R (kk x k), kk = min(m, k).
void qr(int64_t m, int64_t k, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& R) {
    const int64_t kk = std::min(m, k);
    std::vector<double> tau(kk, 0.0);
    for (int64_t j = 0; j < kk; ++j) {
        double* col = &A[j * m];
        double nrm = 0.0;
        for (int64_t i = j; i < m; ++i) nrm += col[i] * col[i];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) {
            tau[j] = 0.0;
            continue;
        }
        double alpha = col[j] >= 0 ? -nrm : nrm;
        double v0 = col[j] - alpha;
        // v = [1, col[j+1..]/v0], tau = -v0/alpha
        for (int64_t i = j + 1; i < m; ++i) col[i] /= v0;
        tau[j] = -v0 / alpha;
        col[j] = alpha;
        for (int64_t c = j + 1; c < k; ++c) {
            double* cc = &A[c * m];
            double s = cc[j];
            for (int64_t i = j + 1; i < m; ++i) s += col[i] * cc[i];
            s *= tau[j];
            cc[j] -= s;
            for (int64_t i = j + 1; i < m; ++i) cc[i] -= s * col[i];
        }
    }
    R.assign(kk * k, 0.0);
    for (int64_t c = 0; c < k; ++c)
        for (int64_t i = 0; i <= std::min(c, kk - 1); ++i) R[i + c * kk] = A[i + c * m];
    Q.assign(m * kk, 0.0);
    for (int64_t c = 0; c < kk; ++c) Q[c + c * m] = 1.0;
    for (int64_t j = kk - 1; j >= 0; --j) {
        if (tau[j] == 0.0) continue;
        const double* v = &A[j * m];
        for (int64_t c = j; c < kk; ++c) {
            double* q = &Q[c * m];
            double s = q[j];
            for (int64_t i = j + 1; i < m; ++i) s += v[i] * q[i];
            s *= tau[j];
            q[j] -= s;
            for (int64_t i = j + 1; i < m; ++i) q[i] -= s * v[i];
        }
    }
}

// One-sided Jacobi SVD of C (r x c col-major): C = U diag(s) V^T, s descending.
void jacobi_svd(int64_t r, int64_t c, std::vector<double> U, std::vector<double>& Uo, std::vector<double>& s,
                std::vector<double>& Vo) {
    std::vector<double> V(c * c, 0.0);
    for (int64_t i = 0; i < c; ++i) V[i + i * c] = 1.0;
    for (int sweep = 0; sweep < 80; ++sweep) {
        double off = 0.0;
        for (int64_t p = 0; p < c; ++p)
            for (int64_t q = p + 1; q < c; ++q) {
                double a = 0, b = 0, g = 0;
                double* up = &U[p * r];
                double* uq = &U[q * r];
                for (int64_t i = 0; i < r; ++i) {
                    a += up[i] * up[i];
                    b += uq[i] * uq[i];
                    g += up[i] * uq[i];
                }
                if (g == 0.0) continue;
                double rel = std::fabs(g) / std::sqrt(a * b);
                if (!(rel > 1e-15)) continue;
                off = std::max(off, rel);
                double zeta = (b - a) / (2.0 * g);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int64_t i = 0; i < r; ++i) {
                    double x = up[i], y = uq[i];
                    up[i] = cs * x - sn * y;
                    uq[i] = sn * x + cs * y;
                }
                double* vp = &V[p * c];
                double* vq = &V[q * c];
                for (int64_t i = 0; i < c; ++i) {
                    double x = vp[i], y = vq[i];
                    vp[i] = cs * x - sn * y;
                    vq[i] = sn * x + cs * y;
                }
            }
        if (off <= 1e-15) break;
    }
    std::vector<double> sv(c);
    for (int64_t j = 0; j < c; ++j) {
        double nrm = 0;
        for (int64_t i = 0; i < r; ++i) nrm += U[i + j * r] * U[i + j * r];
        sv[j] = std::sqrt(nrm);
    }
    std::vector<int64_t> ord(c);
    for (int64_t j = 0; j < c; ++j) ord[j] = j;
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return sv[a] > sv[b]; });
    Uo.assign(r * c, 0.0);
    Vo.assign(c * c, 0.0);
    s.assign(c, 0.0);
    for (int64_t jj = 0; jj < c; ++jj) {
        int64_t j = ord[jj];
        s[jj] = sv[j];
        for (int64_t i = 0; i < r; ++i) Uo[i + jj * r] = sv[j] > 0 ? U[i + j * r] / sv[j] : 0.0;
        for (int64_t i = 0; i < c; ++i) Vo[i + jj * c] = V[i + j * c];
    }
}

struct LR {
    int32_t k = 0;
    std::vector<double> W, S, X;
};

void aca_block(const Pts& P, int64_t r0, int64_t m, int64_t c0, int64_t n, double eps, LR& out) {
    const double eps_aca = eps / 20.0;
    std::vector<std::vector<double>> Us, Vs;
    std::vector<char> used(m, 0);
    std::vector<double> row(n), col(m);
    double norm2 = 0.0;
    int64_t i = 0;
    int ok_streak = 0;
    const int64_t kmax = std::min(m, n);
    int64_t zero_rows = 0;
    while ((int64_t)Us.size() < kmax) {
        used[i] = 1;
        for (int64_t j = 0; j < n; ++j) row[j] = kval(P, r0 + i, c0 + j);
        for (size_t l = 0; l < Us.size(); ++l) {
            const double ui = Us[l][i];
            const double* v = Vs[l].data();
            for (int64_t j = 0; j < n; ++j) row[j] -= ui * v[j];
        }
        int64_t jp = 0;
        double best = 0.0;
        for (int64_t j = 0; j < n; ++j)
            if (std::fabs(row[j]) > best) {
                best = std::fabs(row[j]);
                jp = j;
            }
        if (best == 0.0) {
            // an exactly zero residual row: try the next unused row
            ++zero_rows;
            int64_t nxt = -1;
            for (int64_t t = 0; t < m; ++t)
                if (!used[t]) {
                    nxt = t;
                    break;
                }
            if (nxt < 0 || zero_rows > 3) break;
            i = nxt;
            continue;
        }
        std::vector<double> v(n), u(m);
        const double piv = row[jp];
        for (int64_t j = 0; j < n; ++j) v[j] = row[j] / piv;
        for (int64_t t = 0; t < m; ++t) u[t] = kval(P, r0 + t, c0 + jp);
        for (size_t l = 0; l < Us.size(); ++l) {
            const double vj = Vs[l][jp];
            const double* uu = Us[l].data();
            for (int64_t t = 0; t < m; ++t) u[t] -= vj * uu[t];
        }
        double uu2 = 0, vv2 = 0;
        for (int64_t t = 0; t < m; ++t) uu2 += u[t] * u[t];
        for (int64_t j = 0; j < n; ++j) vv2 += v[j] * v[j];
        double cross = 0.0;
        for (size_t l = 0; l < Us.size(); ++l) {
            double a = 0, b = 0;
            for (int64_t t = 0; t < m; ++t) a += Us[l][t] * u[t];
            for (int64_t j = 0; j < n; ++j) b += Vs[l][j] * v[j];
            cross += a * b;
        }
        norm2 += 2.0 * cross + uu2 * vv2;
        Us.push_back(std::move(u));
        Vs.push_back(std::move(v));
        const double step = std::sqrt(uu2 * vv2);
        if (step <= eps_aca * std::sqrt(std::max(norm2, 0.0)))
            ++ok_streak;
        else
            ok_streak = 0;
        if (ok_streak >= 2) break;
        // next row: largest entry of the new column among unused rows
        int64_t nxt = -1;
        double bu = -1.0;
        const double* uu = Us.back().data();
        for (int64_t t = 0; t < m; ++t)
            if (!used[t] && std::fabs(uu[t]) > bu) {
                bu = std::fabs(uu[t]);
                nxt = t;
            }
        if (nxt < 0) break;
        i = nxt;
    }
    const int64_t k = (int64_t)Us.size();
    if (k == 0) {
        out.k = 0;
        return;
    }
    std::vector<double> U(m * k), V(n * k);
    for (int64_t l = 0; l < k; ++l) {
        std::memcpy(&U[l * m], Us[l].data(), m * sizeof(double));
        std::memcpy(&V[l * n], Vs[l].data(), n * sizeof(double));
    }
    std::vector<double> Q1, R1, Q2, R2;
    qr(m, k, U, Q1, R1);
    qr(n, k, V, Q2, R2);
    const int64_t k1 = std::min(m, k), k2 = std::min(n, k);
    // C = R1 R2^T  (k1 x k2)
    std::vector<double> C(k1 * k2, 0.0);
    for (int64_t a = 0; a < k1; ++a)
        for (int64_t b = 0; b < k2; ++b) {
            double sacc = 0;
            for (int64_t l = 0; l < k; ++l) sacc += R1[a + l * k1] * R2[b + l * k2];
            C[a + b * k1] = sacc;
        }
    std::vector<double> A, s, B;
    jacobi_svd(k1, k2, C, A, s, B);
    // truncation: smallest r with sqrt(sum_{i>=r} s_i^2) <= eps * ||s||
    double tot = 0;
    for (double v : s) tot += v * v;
    const double tol2 = eps * eps * tot;
    int64_t r = (int64_t)s.size();
    double tail = 0.0;
    while (r > 0 && tail + s[r - 1] * s[r - 1] <= tol2) {
        tail += s[r - 1] * s[r - 1];
        --r;
    }
    out.k = (int32_t)r;
    out.S.assign(s.begin(), s.begin() + r);
    out.W.assign(m * r, 0.0);
    out.X.assign(n * r, 0.0);
    for (int64_t c = 0; c < r; ++c) {
        for (int64_t l = 0; l < k1; ++l) {
            const double a = A[l + c * k1];
            if (a == 0.0) continue;
            for (int64_t t = 0; t < m; ++t) out.W[t + c * m] += Q1[t + l * m] * a;
        }
        for (int64_t l = 0; l < k2; ++l) {
            const double b = B[l + c * k2];
            if (b == 0.0) continue;
            for (int64_t t = 0; t < n; ++t) out.X[t + c * n] += Q2[t + l * n] * b;
        }
    }
}

template <class F>
void parallel_for(int64_t count, int nthreads, const std::vector<int64_t>& order, F f) {
    if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
    std::atomic<int64_t> next(0);
    auto work = [&]() {
        for (;;) {
            int64_t q = next.fetch_add(1);
            if (q >= count) break;
            f(order.empty() ? q : order[q]);
        }
    };
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) th.emplace_back(work);
    for (auto& t : th) t.join();
}

struct Handle {
    std::vector<LR> blocks;
};

}  // namespace

extern "C" {

void synth_dense_blocks(const double* pts_cluster, int kernel, const int64_t* blocks, int64_t nb,
                        double* const* outs, int nthreads) {
    Pts P{pts_cluster, kernel};
    std::vector<int64_t> none;
    parallel_for(nb, nthreads, none, [&](int64_t b) {
        const int64_t r0 = blocks[4 * b], m = blocks[4 * b + 1], c0 = blocks[4 * b + 2], n = blocks[4 * b + 3];
        double* o = outs[b];
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) o[i + j * m] = kval(P, r0 + i, c0 + j);
    });
}

void* synth_lowrank(const double* pts_cluster, int kernel, const int64_t* blocks, int64_t nb, double eps,
                    int nthreads) {
    Pts P{pts_cluster, kernel};
    Handle* h = new Handle();
    h->blocks.resize(nb);
    std::vector<int64_t> order(nb);
    for (int64_t b = 0; b < nb; ++b) order[b] = b;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        return blocks[4 * a + 1] + blocks[4 * a + 3] > blocks[4 * b + 1] + blocks[4 * b + 3];
    });
    parallel_for(nb, nthreads, order, [&](int64_t b) {
        aca_block(P, blocks[4 * b], blocks[4 * b + 1], blocks[4 * b + 2], blocks[4 * b + 3], eps, h->blocks[b]);
    });
    return h;
}

void synth_lowrank_ranks(void* hv, int32_t* ranks) {
    Handle* h = (Handle*)hv;
    for (size_t b = 0; b < h->blocks.size(); ++b) ranks[b] = h->blocks[b].k;
}

void synth_lowrank_copy(void* hv, double* const* W, double* const* S, double* const* X) {
    Handle* h = (Handle*)hv;
    for (size_t b = 0; b < h->blocks.size(); ++b) {
        const LR& lr = h->blocks[b];
        if (lr.k == 0) continue;
        std::memcpy(W[b], lr.W.data(), lr.W.size() * sizeof(double));
        std::memcpy(S[b], lr.S.data(), lr.S.size() * sizeof(double));
        std::memcpy(X[b], lr.X.data(), lr.X.size() * sizeof(double));
    }
}

void synth_lowrank_free(void* hv) { delete (Handle*)hv; }

}  // extern "C"
