// Host construction of the cluster tree and block tree (Def. 2.1, 2.2).
//
// Compiled with -ffp-contract=off: the box midpoint and the squared
// diameter/distance predicates are evaluated as written (one rounding per
// operation, sums over x, y, z in that order), so a layout is a
// deterministic function of the points.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "hm_internal.h"

namespace hm {

namespace {

struct Builder {
    const double* P;
    Layout& L;
    std::vector<int64_t> scratch;
    int64_t pos = 0;

    Builder(const double* p, Layout& l) : P(p), L(l) {}

    int32_t new_node(int32_t level, int32_t parent) {
        L.node_begin.push_back(0);
        L.node_end.push_back(0);
        L.node_level.push_back(level);
        L.node_parent.push_back(parent);
        L.node_son0.push_back(-1);
        L.node_son1.push_back(-1);
        for (int d = 0; d < 3; ++d) {
            L.node_lo.push_back(0.0);
            L.node_hi.push_back(0.0);
        }
        return (int32_t)L.node_begin.size() - 1;
    }

    // idx: the cluster's point indices (original order ids) in current order.
    // Creates the node for them in depth-first pre-order.
    void build(std::vector<int64_t>& idx, int32_t level, int32_t parent) {
        int32_t v = new_node(level, parent);
        const int64_t m = (int64_t)idx.size();
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = P[3 * idx[0] + d];
            hi[d] = lo[d];
        }
        for (int64_t i = 1; i < m; ++i)
            for (int d = 0; d < 3; ++d) {
                double c = P[3 * idx[i] + d];
                if (c < lo[d]) lo[d] = c;
                if (c > hi[d]) hi[d] = c;
            }
        for (int d = 0; d < 3; ++d) {
            L.node_lo[3 * v + d] = lo[d];
            L.node_hi[3 * v + d] = hi[d];
        }
        if (level > L.depth) L.depth = level;
        const bool balanced = L.partition != HM_PART_STANDARD;
        if (balanced ? (level >= L.blr_depth || m < 2) : m <= L.leaf_size) {
            L.node_begin[v] = pos;
            for (int64_t i = 0; i < m; ++i) L.perm[pos + i] = idx[i];
            pos += m;
            L.node_end[v] = pos;
            return;
        }
        int axis = 0;
        double best = hi[0] - lo[0];
        for (int d = 1; d < 3; ++d) {
            double e = hi[d] - lo[d];
            if (e > best) {
                best = e;
                axis = d;
            }
        }
        std::vector<int64_t> a, b;
        if (balanced) {
            // cardinality bisection: the points ordered by the axis
            // coordinate (stable), son 0 takes the first half (rounded down)
            const double* PP = P;
            std::stable_sort(idx.begin(), idx.end(),
                             [PP, axis](int64_t u, int64_t w) { return PP[3 * u + axis] < PP[3 * w + axis]; });
            a.assign(idx.begin(), idx.begin() + m / 2);
            b.assign(idx.begin() + m / 2, idx.end());
        } else {
            const double mid = 0.5 * (lo[axis] + hi[axis]);
            a.reserve(m);
            b.reserve(m);
            for (int64_t i = 0; i < m; ++i) {
                if (P[3 * idx[i] + axis] < mid)
                    a.push_back(idx[i]);
                else
                    b.push_back(idx[i]);
            }
            if (a.empty() || b.empty()) {
                a.assign(idx.begin(), idx.begin() + m / 2);
                b.assign(idx.begin() + m / 2, idx.end());
            }
        }
        std::vector<int64_t>().swap(idx);   // release before recursing
        int32_t s0 = (int32_t)L.node_begin.size();
        build(a, level + 1, v);
        int32_t s1 = (int32_t)L.node_begin.size();
        build(b, level + 1, v);
        L.node_son0[v] = s0;
        L.node_son1[v] = s1;
        L.node_begin[v] = L.node_begin[s0];
        L.node_end[v] = L.node_end[s1];
    }
};

bool admissible(const Layout& L, int32_t t, int32_t s) {
    const double* lt = &L.node_lo[3 * t];
    const double* ht = &L.node_hi[3 * t];
    const double* ls = &L.node_lo[3 * s];
    const double* hs = &L.node_hi[3 * s];
    double dt = 0.0, ds = 0.0, dd = 0.0;
    for (int d = 0; d < 3; ++d) {
        double et = ht[d] - lt[d];
        double es = hs[d] - ls[d];
        dt = dt + et * et;
        ds = ds + es * es;
        double g = 0.0;
        double a = ls[d] - ht[d];
        double b = lt[d] - hs[d];
        if (a > g) g = a;
        if (b > g) g = b;
        dd = dd + g * g;
    }
    double mn = dt < ds ? dt : ds;
    return mn <= (L.eta * L.eta) * dd && dd > 0.0;
}

// The admissibility of the chosen partition (Sec. 2.2 and its remark on
// BLR and HODLR): standard; off-diagonal (weak) for HODLR, every pair of
// distinct clusters; for BLR the standard condition between leaf clusters
// only, so the block tree reaches all pairs of leaves (one level).
bool block_admissible(const Layout& L, int32_t t, int32_t s) {
    if (L.partition == HM_PART_HODLR) return t != s;
    if (L.partition == HM_PART_BLR) return L.leaf(t) && L.leaf(s) && admissible(L, t, s);
    return admissible(L, t, s);
}

void block_tree(Layout& L) {
    std::vector<std::pair<int32_t, int32_t>> stack;
    stack.push_back({0, 0});
    while (!stack.empty()) {
        auto [t, s] = stack.back();
        stack.pop_back();
        if (block_admissible(L, t, s)) {
            L.blk_tau.push_back(t);
            L.blk_sigma.push_back(s);
            L.blk_adm.push_back(1);
        } else if (L.leaf(t) || L.leaf(s)) {
            L.blk_tau.push_back(t);
            L.blk_sigma.push_back(s);
            L.blk_adm.push_back(0);
        } else {
            int32_t t0 = L.node_son0[t], t1 = L.node_son1[t];
            int32_t s0 = L.node_son0[s], s1 = L.node_son1[s];
            // pushed in reverse so (t0,s0), (t0,s1), (t1,s0), (t1,s1) pop in order
            stack.push_back({t1, s1});
            stack.push_back({t1, s0});
            stack.push_back({t0, s1});
            stack.push_back({t0, s0});
        }
    }
}

}  // namespace

}  // namespace hm

extern "C" hm_status hm_build_layout(const double* points, int64_t n, const hm_layout_opts* opts,
                                     hm_layout** out) {
    if (!out || !points || n < 1) {
        hm::set_error("hm_build_layout: null argument or n < 1");
        return HM_EINVAL;
    }
    *out = nullptr;
    int32_t leaf = opts ? opts->leaf_size : 64;
    double eta = opts ? opts->eta : 2.0;
    const int32_t part = opts ? opts->partition : HM_PART_STANDARD;
    if (leaf < 1 || !(eta > 0.0) || !std::isfinite(eta) ||
        (part != HM_PART_STANDARD && part != HM_PART_HODLR && part != HM_PART_BLR)) {
        hm::set_error("hm_build_layout: leaf_size must be >= 1, eta > 0 and partition one of HM_PART_*");
        return HM_EINVAL;
    }
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(points[i])) {
            hm::set_error("hm_build_layout: non-finite point coordinate");
            return HM_EINVAL;
        }
    hm_layout* lay = new (std::nothrow) hm_layout();
    if (!lay) {
        hm::set_error("hm_build_layout: out of host memory");
        return HM_ENOMEM;
    }
    try {
        hm::Layout& L = lay->L;
        L.n = n;
        L.leaf_size = leaf;
        L.eta = eta;
        L.partition = part;
        // balanced trees: the smallest depth d with ceil(n / 2^d) <= leaf_size
        while (L.blr_depth < 62 && ((n + (int64_t(1) << L.blr_depth) - 1) >> L.blr_depth) > leaf) ++L.blr_depth;
        L.perm.assign(n, -1);
        std::vector<int64_t> idx(n);
        for (int64_t i = 0; i < n; ++i) idx[i] = i;
        hm::Builder b(points, L);
        b.build(idx, 0, -1);
        hm::block_tree(L);
    } catch (const std::bad_alloc&) {
        delete lay;
        hm::set_error("hm_build_layout: out of host memory");
        return HM_ENOMEM;
    }
    *out = lay;
    return HM_OK;
}

extern "C" hm_status hm_layout_export(const hm_layout* layout, hm_layout_view* v) {
    if (!layout || !v) {
        hm::set_error("hm_layout_export: null argument");
        return HM_EINVAL;
    }
    const hm::Layout& L = layout->L;
    v->n = L.n;
    v->nnodes = (int64_t)L.node_begin.size();
    v->nblocks = (int64_t)L.blk_tau.size();
    v->depth = L.depth;
    v->perm = L.perm.data();
    v->node_begin = L.node_begin.data();
    v->node_end = L.node_end.data();
    v->node_level = L.node_level.data();
    v->node_parent = L.node_parent.data();
    v->node_son0 = L.node_son0.data();
    v->node_son1 = L.node_son1.data();
    v->blk_tau = L.blk_tau.data();
    v->blk_sigma = L.blk_sigma.data();
    v->blk_adm = L.blk_adm.data();
    return HM_OK;
}

extern "C" void hm_layout_free(hm_layout* layout) { delete layout; }

extern "C" hm_status hm_layout_stats(const hm_layout* layout, hm_layout_info* info) {
    if (!layout || !info) {
        hm::set_error("hm_layout_stats: null argument");
        return HM_EINVAL;
    }
    const hm::Layout& L = layout->L;
    *info = hm_layout_info{};
    auto lv = [](int32_t l) { return l < HM_MAX_LEVELS - 1 ? l : HM_MAX_LEVELS - 1; };
    info->n = L.n;
    info->nnodes = (int64_t)L.node_begin.size();
    info->nblocks = (int64_t)L.blk_tau.size();
    info->depth = L.depth;
    info->min_leaf = INT32_MAX;
    for (int32_t v = 0; v < (int32_t)info->nnodes; ++v) {
        info->nodes_per_level[lv(L.node_level[v])]++;
        if (L.leaf(v)) {
            info->nleaves++;
            info->min_leaf = std::min<int32_t>(info->min_leaf, (int32_t)L.size(v));
            info->max_leaf = std::max<int32_t>(info->max_leaf, (int32_t)L.size(v));
        }
    }
    if (info->nleaves == 0) info->min_leaf = 0;
    for (size_t b = 0; b < L.blk_tau.size(); ++b) {
        const int32_t t = L.blk_tau[b], s = L.blk_sigma[b];
        const double area = (double)L.size(t) * (double)L.size(s);
        const int32_t l = lv(L.node_level[t]);
        if (L.blk_adm[b]) {
            info->nlowrank++;
            info->lowrank_per_level[l]++;
            info->lowrank_area += area;
            info->lowrank_area_per_level[l] += area;
        } else {
            info->ndense++;
            info->ndiag += t == s;
            info->dense_per_level[l]++;
            info->dense_area += area;
            info->dense_area_per_level[l] += area;
        }
    }
    return HM_OK;
}
