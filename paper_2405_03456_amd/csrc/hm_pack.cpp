// Packing of a hierarchical matrix into row-owner streams.
//
// Phases per format (each is one pass of the owner kernel):
//   H  (Alg. 1/3):  h_vt   t_b = X_b^T x|s                 owner = low-rank block
//                   h_rows y|rho += a sum_{b: t_b >= rho} (D_b|rho x|s or U_b|rho t_b)
//                                                          owner = leaf cluster rho
//   UH (Alg. 4/5, eq. 5):
//                   uh_fwd  s_s = X_s^T x|s                owner = column cluster
//                   uh_coup t_t = sum_b S_b s_s            owner = row cluster
//                   uh_rows y|rho += a (sum_{t >= rho} W_t|rho t_t + dense)
//   H2 (Alg. 6/7):  h2_up_leaf s = X_s^T x|s at leaves
//                   h2_up_L  s_s = sum_{s'} F_s'^T s_s'    one phase per level, leaves to root
//                   h2_dn_L  t_t = E_t t_parent + sum_b S_b s_s   one phase per level, root down
//                   h2_rows y|rho += a (W_rho t_rho + dense)
// Each leaf cluster rho is owned by one set of tasks and y|rho is written
// once per product: clusters of one level are disjoint and the block rows of
// all ancestors are gathered into rho's stream, which is the race-freedom
// argument of Sec. 3.1 turned into a static schedule.
//
// Storage: a source matrix is quantised once (per-column scales, Sec. 4.1
// direct compression) and every owner reads its own row slice of it, so a
// block's data is split across the leaf streams of its row cluster without
// duplication.  Factors read along columns (X_b, X_s) are stored transposed
// so that every product is "one lane per output row".
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <thread>

#include "hm_pack.h"

namespace hm {

namespace {

struct Use {
    int64_t data_off;
    int64_t r0, nr;        // normal: rows [r0, r0+nr);  transposed: ignored (all rows)
    bool transposed;
};

struct Source {
    const double* A = nullptr;   // m x k column-major
    std::vector<double> own;     // storage if A is a host-made copy (transposes)
    int64_t m = 0, k = 0;
    int32_t dtype = HM_F64;
    const double* colfactor = nullptr;   // folded into the column scale (sigma of W_b)
    int32_t scale_off = -1;      // per-column scales c_j * f_j (shared by all uses)
    std::vector<Use> uses;
    int64_t cls = 0;             // stats class: 0 dense, 1 factor, 2 coupling, 3 transfer
};

// formats whose columns carry a range scale (narrow exponent range)
bool range_scaled(int32_t dt) { return dt == HM_F16 || dt == HM_FP8E4M3; }

struct Builder {
    const Layout& L;
    int32_t fmt;
    const hm_values* V;
    PackOptions opt;
    int32_t dense_dt, diag_dt, factor_dt, coup_dt;
    std::deque<Phase> phases;      // deque: owners keep references while they are built
    std::vector<Source> src;
    int64_t data_bytes = 0;
    int64_t nscales = 0;
    int64_t ws = 0;
    std::string err;

    Builder(const Layout& l, int32_t f, const hm_values* v, const PackOptions& o)
        : L(l), fmt(f), V(v), opt(o) {}

    int64_t alloc_data(int64_t bytes) {
        int64_t off = (data_bytes + 15) & ~int64_t(15);
        data_bytes = off + bytes;
        return off;
    }

    int32_t add_source(const double* A, int64_t m, int64_t k, int32_t dt, const double* colfactor,
                       int cls) {
        Source s;
        s.A = A;
        s.m = m;
        s.k = k;
        s.dtype = dt;
        s.colfactor = colfactor;
        s.cls = cls;
        if (range_scaled(dt) || colfactor) {
            s.scale_off = (int32_t)nscales;
            nscales += k;
        }
        src.push_back(std::move(s));
        return (int32_t)src.size() - 1;
    }

    // host transpose (for F^T), stored inside the source
    int32_t add_source_transposed(const double* A, int64_t m, int64_t k, int32_t dt, int cls) {
        int32_t id = add_source(nullptr, k, m, dt, nullptr, cls);
        Source& s = src[id];
        s.own.resize((size_t)(m * k));
        for (int64_t j = 0; j < k; ++j)
            for (int64_t i = 0; i < m; ++i) s.own[(size_t)(j + i * k)] = A[i + j * m];
        s.A = s.own.data();
        return id;
    }

    // ---- owner construction
    Phase* ph = nullptr;
    DOwner cur{};
    int32_t cur_cols = 0;

    Phase& new_phase(const char* name) {
        phases.emplace_back();
        phases.back().name = name;
        return phases.back();
    }

    void begin_owner(Phase& p, int32_t nrows, int32_t mode, int32_t out_off, int32_t rscale_off) {
        ph = &p;
        cur = DOwner{};
        cur.nrows = nrows;
        cur.item0 = (int32_t)p.items.size();
        cur.nitems = 0;
        cur.out_off = out_off;
        cur.mode = mode;
        cur.rscale_off = rscale_off;
        cur_cols = 0;
        if (nrows > p.max_rows) p.max_rows = nrows;
    }

    // item = rows [r0, r0+nr) of source s (all its columns), or the transpose
    void add_item(int32_t s, int64_t r0, bool transposed, int32_t vec_off) {
        Source& S = src[s];
        const int64_t nr = cur.nrows;
        const int64_t ncols = transposed ? S.m : S.k;
        if (ncols == 0 || nr == 0) return;
        const int64_t bytes = nr * ncols * dtype_bytes(S.dtype);
        DItem it{};
        it.data_off = alloc_data(bytes);
        it.col0 = cur_cols;
        it.ncols = (int32_t)ncols;
        it.vec_off = vec_off;
        it.scale_off = transposed ? -1 : S.scale_off;
        it.dtype = (int16_t)S.dtype;
        it.acc64 = S.dtype == HM_F64 ? 1 : 0;
        ph->items.push_back(it);
        ph->data_bytes += bytes;
        cur.nitems++;
        cur_cols += (int32_t)ncols;
        S.uses.push_back(Use{it.data_off, r0, nr, transposed});
    }

    void end_owner() {
        Phase& p = *ph;
        const int32_t owner_id = (int32_t)p.owners.size();
        // cut the owner's columns into tasks of about opt.task_bytes
        int32_t ntasks = 0;
        int32_t start_col = 0, start_item = cur.item0;
        int64_t acc = 0;
        for (int32_t i = 0; i < cur.nitems; ++i) {
            const DItem& it = p.items[cur.item0 + i];
            const int64_t bpc = (int64_t)cur.nrows * dtype_bytes(it.dtype);
            int32_t j = 0;
            while (j < it.ncols) {
                int64_t room = opt.task_bytes - acc;
                int64_t take = std::max<int64_t>(1, room / bpc);
                take = std::min<int64_t>(take, it.ncols - j);
                acc += take * bpc;
                j += (int32_t)take;
                if (acc >= opt.task_bytes) {
                    DTask t{};
                    t.owner = owner_id;
                    t.c0 = start_col;
                    t.c1 = it.col0 + j;
                    t.item_start = start_item;
                    t.local = ntasks++;
                    p.tasks.push_back(t);
                    start_col = t.c1;
                    start_item = (j == it.ncols) ? cur.item0 + i + 1 : cur.item0 + i;
                    acc = 0;
                }
            }
        }
        if (start_col < cur_cols || ntasks == 0) {
            DTask t{};
            t.owner = owner_id;
            t.c0 = start_col;
            t.c1 = cur_cols;
            t.item_start = std::min(start_item, cur.item0 + std::max(cur.nitems - 1, 0));
            t.local = ntasks++;
            p.tasks.push_back(t);
        }
        cur.ntasks = ntasks;
        if (ntasks > 1) {
            cur.part_off = (int32_t)p.part_elems;
            p.part_elems += (int64_t)ntasks * cur.nrows;
            p.reduce_owners.push_back(owner_id);
        } else {
            cur.part_off = 0;
        }
        p.owners.push_back(cur);
        ph = nullptr;
    }

    // ---- helpers
    std::vector<std::vector<int32_t>> row_blocks;   // per node: block ids with tau == node
    std::vector<int32_t> leaves;

    void index_blocks() {
        row_blocks.assign(L.node_begin.size(), {});
        for (size_t b = 0; b < L.blk_tau.size(); ++b) row_blocks[L.blk_tau[b]].push_back((int32_t)b);
        for (int32_t v = 0; v < (int32_t)L.node_begin.size(); ++v)
            if (L.leaf(v)) leaves.push_back(v);
        // leaves are in depth-first order, i.e. by cluster position
    }

    std::vector<int32_t> ancestors_root_first(int32_t v) const {
        std::vector<int32_t> a;
        for (int32_t u = v; u >= 0; u = L.node_parent[u]) a.push_back(u);
        std::reverse(a.begin(), a.end());
        return a;
    }

    int32_t dense_source(int32_t b) {
        const int32_t t = L.blk_tau[b], s = L.blk_sigma[b];
        const int32_t dt = (t == s) ? diag_dt : dense_dt;
        return add_source(V->dense[b], L.size(t), L.size(s), dt, nullptr, 0);
    }

    bool check(bool ok, const char* msg) {
        if (!ok && err.empty()) err = msg;
        return ok;
    }

    bool check_dense() {
        if (!V->dense) return check(false, "values.dense is required");
        for (size_t b = 0; b < L.blk_tau.size(); ++b)
            if (!L.blk_adm[b] && !V->dense[b]) return check(false, "missing dense block values");
        return true;
    }

    // --------------------------------------------------------------- H
    bool build_h() {
        if (!check_dense()) return false;
        if (!V->rank || !V->W || !V->sigma || !V->X) return check(false, "H needs rank, W, sigma, X");
        const int64_t nb = (int64_t)L.blk_tau.size();
        std::vector<int32_t> tb_off(nb, -1), usrc(nb, -1), dsrc(nb, -1);
        for (int64_t b = 0; b < nb; ++b) {
            if (!L.blk_adm[b]) continue;
            const int32_t k = V->rank[b];
            const int64_t mt = L.size(L.blk_tau[b]), ms = L.size(L.blk_sigma[b]);
            if (k < 0 || k > std::min(mt, ms)) return check(false, "rank out of range");
            if (k > 0 && (!V->W[b] || !V->sigma[b] || !V->X[b])) return check(false, "missing factor");
            if (k > 0) {
                tb_off[b] = (int32_t)ws;
                ws += k;
            }
        }
        Phase& pa = new_phase("h_vt");
        for (int64_t b = 0; b < nb; ++b) {
            if (!L.blk_adm[b] || V->rank[b] == 0) continue;
            const int32_t k = V->rank[b];
            const int32_t s = L.blk_sigma[b];
            int32_t xs = add_source(V->X[b], L.size(s), k, factor_dt, nullptr, 1);
            begin_owner(pa, k, 0, tb_off[b], src[xs].scale_off);
            add_item(xs, 0, true, (int32_t)L.node_begin[s]);
            end_owner();
            usrc[b] = add_source(V->W[b], L.size(L.blk_tau[b]), k, factor_dt, V->sigma[b], 1);
        }
        Phase& pb = new_phase("h_rows");
        for (int32_t rho : leaves) {
            begin_owner(pb, (int32_t)L.size(rho), 1, (int32_t)L.node_begin[rho], -1);
            for (int32_t t : ancestors_root_first(rho)) {
                const int64_t r0 = L.node_begin[rho] - L.node_begin[t];
                for (int32_t b : row_blocks[t]) {
                    const int32_t s = L.blk_sigma[b];
                    if (L.blk_adm[b]) {
                        if (V->rank[b] > 0) add_item(usrc[b], r0, false, tb_off[b]);
                    } else {
                        if (dsrc[b] < 0) dsrc[b] = dense_source(b);
                        add_item(dsrc[b], r0, false, (int32_t)L.node_begin[s]);
                    }
                }
            }
            end_owner();
        }
        return true;
    }

    // -------------------------------------------------------------- UH
    bool build_uh() {
        if (!check_dense()) return false;
        if (!V->row_rank || !V->col_rank || !V->row_basis || !V->col_basis || !V->coupling)
            return check(false, "UH needs row/col ranks, bases and couplings");
        const int32_t N = (int32_t)L.node_begin.size();
        const int64_t nb = (int64_t)L.blk_tau.size();
        std::vector<int32_t> s_off(N, -1), t_off(N, -1), wsrc(N, -1), dsrc(nb, -1);
        for (int32_t v = 0; v < N; ++v) {
            const int32_t kr = V->row_rank[v], kc = V->col_rank[v];
            if (kr < 0 || kc < 0 || kr > L.size(v) || kc > L.size(v)) return check(false, "basis rank out of range");
            if ((kr > 0 && !V->row_basis[v]) || (kc > 0 && !V->col_basis[v])) return check(false, "missing basis");
            if (kc > 0) { s_off[v] = (int32_t)ws; ws += kc; }
            if (kr > 0) { t_off[v] = (int32_t)ws; ws += kr; }
        }
        for (int64_t b = 0; b < nb; ++b)
            if (L.blk_adm[b]) {
                const int32_t kr = V->row_rank[L.blk_tau[b]], kc = V->col_rank[L.blk_sigma[b]];
                if (kr > 0 && kc > 0 && !V->coupling[b]) return check(false, "missing coupling");
            }
        Phase& pf = new_phase("uh_fwd");
        for (int32_t v = 0; v < N; ++v) {
            const int32_t kc = V->col_rank[v];
            if (kc == 0) continue;
            int32_t xs = add_source(V->col_basis[v], L.size(v), kc, factor_dt, nullptr, 1);
            begin_owner(pf, kc, 0, s_off[v], src[xs].scale_off);
            add_item(xs, 0, true, (int32_t)L.node_begin[v]);
            end_owner();
        }
        Phase& pc = new_phase("uh_coup");
        for (int32_t t = 0; t < N; ++t) {
            const int32_t kr = V->row_rank[t];
            if (kr == 0) continue;
            begin_owner(pc, kr, 0, t_off[t], -1);
            for (int32_t b : row_blocks[t]) {
                if (!L.blk_adm[b]) continue;
                const int32_t s = L.blk_sigma[b];
                const int32_t kc = V->col_rank[s];
                if (kc == 0) continue;
                int32_t cs = add_source(V->coupling[b], kr, kc, coup_dt, nullptr, 2);
                add_item(cs, 0, false, s_off[s]);
            }
            end_owner();
        }
        for (int32_t v = 0; v < N; ++v)
            if (V->row_rank[v] > 0) wsrc[v] = add_source(V->row_basis[v], L.size(v), V->row_rank[v], factor_dt, nullptr, 1);
        Phase& pr = new_phase("uh_rows");
        for (int32_t rho : leaves) {
            begin_owner(pr, (int32_t)L.size(rho), 1, (int32_t)L.node_begin[rho], -1);
            for (int32_t t : ancestors_root_first(rho)) {
                const int64_t r0 = L.node_begin[rho] - L.node_begin[t];
                if (wsrc[t] >= 0) add_item(wsrc[t], r0, false, t_off[t]);
                for (int32_t b : row_blocks[t]) {
                    if (L.blk_adm[b]) continue;
                    if (dsrc[b] < 0) dsrc[b] = dense_source(b);
                    add_item(dsrc[b], r0, false, (int32_t)L.node_begin[L.blk_sigma[b]]);
                }
            }
            end_owner();
        }
        return true;
    }

    // -------------------------------------------------------------- H2
    bool build_h2() {
        if (!check_dense()) return false;
        if (!V->row_rank || !V->col_rank || !V->row_basis || !V->col_basis || !V->coupling ||
            !V->row_transfer || !V->col_transfer)
            return check(false, "H2 needs ranks, leaf bases, transfers and couplings");
        const int32_t N = (int32_t)L.node_begin.size();
        const int64_t nb = (int64_t)L.blk_tau.size();
        std::vector<int32_t> s_off(N, -1), t_off(N, -1), dsrc(nb, -1);
        for (int32_t v = 0; v < N; ++v) {
            const int32_t kr = V->row_rank[v], kc = V->col_rank[v];
            if (kr < 0 || kc < 0) return check(false, "negative rank");
            if (L.leaf(v) && (kr > L.size(v) || kc > L.size(v))) return check(false, "leaf rank exceeds cluster size");
            if (L.leaf(v) && ((kr > 0 && !V->row_basis[v]) || (kc > 0 && !V->col_basis[v])))
                return check(false, "missing leaf basis");
            const int32_t p = L.node_parent[v];
            if (p >= 0) {
                if (kr > 0 && V->row_rank[p] > 0 && !V->row_transfer[v]) return check(false, "missing row transfer");
                if (kc > 0 && V->col_rank[p] > 0 && !V->col_transfer[v]) return check(false, "missing col transfer");
            }
            if (kc > 0) { s_off[v] = (int32_t)ws; ws += kc; }
            if (kr > 0) { t_off[v] = (int32_t)ws; ws += kr; }
        }
        Phase& pl = new_phase("h2_up_leaf");
        for (int32_t g : leaves) {
            const int32_t kc = V->col_rank[g];
            if (kc == 0) continue;
            int32_t xs = add_source(V->col_basis[g], L.size(g), kc, factor_dt, nullptr, 1);
            begin_owner(pl, kc, 0, s_off[g], src[xs].scale_off);
            add_item(xs, 0, true, (int32_t)L.node_begin[g]);
            end_owner();
        }
        std::vector<std::vector<int32_t>> by_level(L.depth + 1);
        for (int32_t v = 0; v < N; ++v) by_level[L.node_level[v]].push_back(v);
        for (int32_t lv = L.depth - 1; lv >= 0; --lv) {
            bool any = false;
            for (int32_t v : by_level[lv]) any |= (!L.leaf(v) && V->col_rank[v] > 0);
            if (!any) continue;
            Phase& pu = new_phase("h2_up");
            for (int32_t v : by_level[lv]) {
                const int32_t kc = V->col_rank[v];
                if (L.leaf(v) || kc == 0) continue;
                begin_owner(pu, kc, 0, s_off[v], -1);
                for (int32_t c : {L.node_son0[v], L.node_son1[v]}) {
                    const int32_t kcc = V->col_rank[c];
                    if (kcc == 0) continue;
                    // F_c is kcc x kc; F_c^T is kc x kcc, scaled per column of F_c^T
                    int32_t fs = add_source_transposed(V->col_transfer[c], kcc, kc, coup_dt, 3);
                    add_item(fs, 0, false, s_off[c]);
                }
                end_owner();
            }
        }
        for (int32_t lv = 0; lv <= L.depth; ++lv) {
            bool any = false;
            for (int32_t v : by_level[lv]) any |= V->row_rank[v] > 0;
            if (!any) continue;
            Phase& pd = new_phase("h2_down");
            for (int32_t t : by_level[lv]) {
                const int32_t kr = V->row_rank[t];
                if (kr == 0) continue;
                begin_owner(pd, kr, 0, t_off[t], -1);
                const int32_t p = L.node_parent[t];
                if (p >= 0 && V->row_rank[p] > 0) {
                    int32_t es = add_source(V->row_transfer[t], kr, V->row_rank[p], coup_dt, nullptr, 3);
                    add_item(es, 0, false, t_off[p]);
                }
                for (int32_t b : row_blocks[t]) {
                    if (!L.blk_adm[b]) continue;
                    const int32_t s = L.blk_sigma[b];
                    const int32_t kc = V->col_rank[s];
                    if (kc == 0) continue;
                    if (!V->coupling[b]) return check(false, "missing coupling");
                    int32_t cs = add_source(V->coupling[b], kr, kc, coup_dt, nullptr, 2);
                    add_item(cs, 0, false, s_off[s]);
                }
                end_owner();
            }
        }
        Phase& pr = new_phase("h2_rows");
        for (int32_t rho : leaves) {
            begin_owner(pr, (int32_t)L.size(rho), 1, (int32_t)L.node_begin[rho], -1);
            const int32_t kr = V->row_rank[rho];
            if (kr > 0) {
                int32_t ws_ = add_source(V->row_basis[rho], L.size(rho), kr, factor_dt, nullptr, 1);
                add_item(ws_, 0, false, t_off[rho]);
            }
            for (int32_t t : ancestors_root_first(rho)) {
                const int64_t r0 = L.node_begin[rho] - L.node_begin[t];
                for (int32_t b : row_blocks[t]) {
                    if (L.blk_adm[b]) continue;
                    if (dsrc[b] < 0) dsrc[b] = dense_source(b);
                    add_item(dsrc[b], r0, false, (int32_t)L.node_begin[L.blk_sigma[b]]);
                }
            }
            end_owner();
        }
        return true;
    }

    // ------------------------------------------------------------ fill
    // Quantise every source once and write its slices.  Sources are
    // independent, so this runs on several host threads.
    bool fill(std::vector<uint8_t>& data, std::vector<double>& scales, int64_t* per_dtype,
              int64_t* per_class) {
        data.assign((size_t)data_bytes, 0);
        scales.assign((size_t)nscales, 1.0);
        std::vector<int> bad(src.size(), 0);
        auto work = [&](size_t i0, size_t i1) {
            std::vector<double> codes;
            std::vector<double> c;
            for (size_t si = i0; si < i1; ++si) {
                Source& S = src[si];
                if (S.uses.empty()) continue;
                const int64_t m = S.m, k = S.k;
                codes.resize((size_t)(m * k));
                c.assign((size_t)k, 1.0);
                const double fmax = dtype_max(S.dtype);
                for (int64_t j = 0; j < k; ++j) {
                    const double* col = S.A + j * m;
                    double mx = 0.0;
                    for (int64_t i = 0; i < m; ++i) {
                        if (!std::isfinite(col[i])) bad[si] = 1;
                        double a = std::fabs(col[i]);
                        if (a > mx) mx = a;
                    }
                    double cj = 1.0;
                    if (range_scaled(S.dtype) && mx > 0.0) {
                        cj = (double)(float)(mx / fmax);
                        if (cj < 1.1754943508222875e-38) cj = 1.1754943508222875e-38;   // 2^-126
                    }
                    c[(size_t)j] = cj;
                    for (int64_t i = 0; i < m; ++i)
                        codes[(size_t)(i + j * m)] = round_to(S.dtype, cj == 1.0 ? col[i] : col[i] / cj);
                }
                if (S.scale_off >= 0)
                    for (int64_t j = 0; j < k; ++j)
                        scales[(size_t)(S.scale_off + j)] = c[(size_t)j] * (S.colfactor ? S.colfactor[j] : 1.0);
                const int eb = dtype_bytes(S.dtype);
                for (const Use& u : S.uses) {
                    uint8_t* dst = data.data() + u.data_off;
                    if (!u.transposed) {
                        for (int64_t j = 0; j < k; ++j)
                            for (int64_t i = 0; i < u.nr; ++i) {
                                uint64_t bits = encode(S.dtype, codes[(size_t)(u.r0 + i + j * m)]);
                                std::memcpy(dst + (size_t)((i + j * u.nr) * eb), &bits, (size_t)eb);
                            }
                    } else {
                        // slab = A^T (k x m), column stride k
                        for (int64_t i = 0; i < m; ++i)
                            for (int64_t j = 0; j < k; ++j) {
                                uint64_t bits = encode(S.dtype, codes[(size_t)(i + j * m)]);
                                std::memcpy(dst + (size_t)((j + i * k) * eb), &bits, (size_t)eb);
                            }
                    }
                }
            }
        };
        // transposed sources with per-row scales: scales of A's columns are the
        // owner's row scales; they are written above through scale_off.
        unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        size_t chunk = (src.size() + nt - 1) / nt;
        for (unsigned t = 0; t < nt; ++t) {
            size_t a = t * chunk, b = std::min(src.size(), a + chunk);
            if (a < b) th.emplace_back(work, a, b);
        }
        for (auto& t : th) t.join();
        for (size_t si = 0; si < src.size(); ++si)
            if (bad[si]) return check(false, "non-finite value in matrix data");
        for (const Source& S : src) {
            int64_t bytes = 0;
            for (const Use& u : S.uses)
                bytes += (u.transposed ? S.m * S.k : u.nr * S.k) * dtype_bytes(S.dtype);
            per_dtype[S.dtype] += bytes;
            per_class[S.cls] += bytes;
        }
        return true;
    }
};

// Every index a kernel will form from the tables must stay inside its
// buffer; checked on the host before anything is uploaded.
bool validate(const Packed& P, int64_t n, std::string& why) {
    const int64_t nsc = (int64_t)P.scales.size();
    const int64_t nd = (int64_t)P.data.size();
    for (const Phase& ph : P.phases) {
        const int64_t no = (int64_t)ph.owners.size(), ni = (int64_t)ph.items.size();
        for (int64_t o = 0; o < no; ++o) {
            const DOwner& ow = ph.owners[o];
            if (ow.nrows <= 0 || ow.nitems < 0 || ow.item0 < 0 || ow.item0 + ow.nitems > ni || ow.ntasks < 1) {
                why = "owner table";
                return false;
            }
            const int64_t lim = ow.mode == 0 ? P.ws_elems : n;
            if (ow.out_off < 0 || ow.out_off + ow.nrows > lim) { why = "owner output range"; return false; }
            if (ow.rscale_off >= 0 && ow.rscale_off + ow.nrows > nsc) { why = "row scales"; return false; }
            if (ow.ntasks > 1 && (ow.part_off < 0 || ow.part_off + (int64_t)ow.ntasks * ow.nrows > P.part_elems)) {
                why = "partial range";
                return false;
            }
            int32_t col = 0;
            for (int32_t i = 0; i < ow.nitems; ++i) {
                const DItem& it = ph.items[ow.item0 + i];
                const int eb = dtype_bytes(it.dtype);
                if (eb == 0 || it.col0 != col || it.ncols <= 0) { why = "item columns"; return false; }
                if (it.data_off < 0 || it.data_off + (int64_t)ow.nrows * it.ncols * eb > nd) { why = "item data"; return false; }
                if (it.vec_off < 0 || it.vec_off + (int64_t)it.ncols > P.ws_elems) { why = "item input"; return false; }
                if (it.scale_off >= 0 && it.scale_off + (int64_t)it.ncols > nsc) { why = "item scales"; return false; }
                col += it.ncols;
            }
        }
        std::vector<int32_t> seen(no, 0);
        for (const DTask& t : ph.tasks) {
            if (t.owner < 0 || t.owner >= no) { why = "task owner"; return false; }
            const DOwner& ow = ph.owners[t.owner];
            int32_t ncols = 0;
            if (ow.nitems) ncols = ph.items[ow.item0 + ow.nitems - 1].col0 + ph.items[ow.item0 + ow.nitems - 1].ncols;
            if (t.c0 < 0 || t.c0 > t.c1 || t.c1 > ncols || t.local != seen[t.owner]++) { why = "task columns"; return false; }
            if (t.c0 < t.c1) {
                if (t.item_start < ow.item0 || t.item_start >= ow.item0 + ow.nitems) { why = "task item"; return false; }
                const DItem& it = ph.items[t.item_start];
                if (t.c0 < it.col0 || t.c0 >= it.col0 + it.ncols) { why = "task first item"; return false; }
            }
        }
        for (int64_t o = 0; o < no; ++o)
            if (seen[o] != ph.owners[o].ntasks) { why = "task count"; return false; }
        for (int32_t r : ph.reduce_owners)
            if (r < 0 || r >= no || ph.owners[r].ntasks < 2) { why = "reduce list"; return false; }
    }
    return true;
}

}  // namespace

hm_status pack(const Layout& L, int32_t format, const hm_values* v, const hm_precision* p,
               const PackOptions& opt, Packed& out) {
    if (!v || !p) {
        set_error("hm_upload: null values or precision");
        return HM_EINVAL;
    }
    for (int32_t dt : {p->dense_dtype, p->diag_dtype, p->factor_dtype, p->coupling_dtype})
        if (dt < HM_F64 || dt > HM_FP8E4M3) {
            set_error("hm_upload: unsupported dtype");
            return HM_EINVAL;
        }
    if (p->accum < HM_ACC_AUTO || p->accum > HM_ACC_F64) {
        set_error("hm_upload: bad accumulation mode");
        return HM_EINVAL;
    }
    Builder B(L, format, v, opt);
    B.dense_dt = p->dense_dtype;
    B.diag_dt = p->diag_dtype;
    B.factor_dt = p->factor_dtype;
    B.coup_dt = p->coupling_dtype;
    B.ws = L.n;   // x in cluster order comes first
    B.index_blocks();
    bool ok = false;
    if (format == HM_FMT_H)
        ok = B.build_h();
    else if (format == HM_FMT_UH)
        ok = B.build_uh();
    else if (format == HM_FMT_H2)
        ok = B.build_h2();
    else {
        set_error("hm_upload: unknown format");
        return HM_EINVAL;
    }
    if (!ok) {
        set_error("hm_upload: " + B.err);
        return HM_ELAYOUT;
    }
    int64_t per_dtype[6] = {0, 0, 0, 0, 0, 0};
    int64_t per_class[4] = {0, 0, 0, 0};
    if (!B.fill(out.data, out.scales, per_dtype, per_class)) {
        set_error("hm_upload: " + B.err);
        return HM_EINVAL;
    }
    bool all64 = p->dense_dtype == HM_F64 && p->diag_dtype == HM_F64 && p->factor_dtype == HM_F64 &&
                 p->coupling_dtype == HM_F64;
    if (p->accum == HM_ACC_F64)
        out.acc64 = 1;
    else if (p->accum == HM_ACC_F32)
        out.acc64 = 0;
    else
        out.acc64 = (p->eps < 1e-7 || all64) ? 1 : 0;
    out.format = format;
    out.ws_elems = B.ws;
    out.part_elems = 0;
    for (auto& ph : B.phases) out.part_elems = std::max(out.part_elems, ph.part_elems);
    out.phases.assign(std::make_move_iterator(B.phases.begin()), std::make_move_iterator(B.phases.end()));
    hm_stats& s = out.stats;
    s = hm_stats{};
    s.n = L.n;
    s.nblocks = (int64_t)L.blk_tau.size();
    for (size_t b = 0; b < L.blk_tau.size(); ++b) (L.blk_adm[b] ? s.nlowrank : s.ndense)++;
    s.bytes_dense = per_class[0];
    s.bytes_factors = per_class[1];
    s.bytes_coupling = per_class[2];
    s.bytes_transfer = per_class[3];
    for (int d = 0; d < 5; ++d) s.bytes_per_dtype[d] = per_dtype[d];
    s.bytes_scales = (int64_t)out.scales.size() * 8;
    int64_t meta = 0;
    for (auto& ph : out.phases)
        meta += (int64_t)(ph.owners.size() * sizeof(DOwner) + ph.items.size() * sizeof(DItem) +
                          ph.tasks.size() * sizeof(DTask) + ph.reduce_owners.size() * 4);
    s.bytes_meta = meta + L.n * 8;   // + permutation
    s.bytes_workspace = (out.ws_elems + out.part_elems) * 8;
    if (format == HM_FMT_H) {
        for (size_t b = 0; b < L.blk_tau.size(); ++b)
            if (L.blk_adm[b]) {
                s.sum_rank += v->rank[b];
                s.max_rank = std::max(s.max_rank, v->rank[b]);
            }
    } else {
        for (size_t i = 0; i < L.node_begin.size(); ++i) {
            s.sum_rank += v->row_rank[i] + v->col_rank[i];
            s.max_rank = std::max(s.max_rank, std::max(v->row_rank[i], v->col_rank[i]));
        }
    }
    s.accum = out.acc64 ? HM_ACC_F64 : HM_ACC_F32;
    std::string why;
    if (!validate(out, L.n, why)) {
        set_error("hm_upload: internal plan check failed (" + why + ")");
        return HM_ELAYOUT;
    }
    return HM_OK;
}

}  // namespace hm
