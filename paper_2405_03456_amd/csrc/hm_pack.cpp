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
#include <array>
#include <cstdlib>
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
    int32_t ebits = 0;           // AFLP exponent width (0 for the other formats)
    const double* colfactor = nullptr;   // folded into the column scale (sigma of W_b)
    int32_t scale_off = -1;      // per-column scales c_j * f_j (shared by all uses)
    std::vector<Use> uses;
    int64_t cls = 0;             // stats class: 0 dense, 1 factor, 2 coupling, 3 transfer
};

// Slabs are stored in 16-byte tiles: tile t of an item holds columns
// [t*V, t*V+V) of all its rows, row-major (one 16-byte chunk per row), with
// V = floor(16 / element size) (3-, 5-, 6- and 7-byte codecs leave the end
// of the chunk zero).  Missing columns of the last tile are zero.
int tile_cols(int32_t dt) { return 16 / dtype_bytes(dt); }
int64_t tile_count(int32_t dt, int64_t ncols) { return (ncols + tile_cols(dt) - 1) / tile_cols(dt); }

// formats whose columns carry a scale: narrow exponent range (FP16, FP8) or
// AFLP's power-of-two scale
bool range_scaled(int32_t dt) { return dt == HM_F16 || dt == HM_FP8E4M3 || is_aflp(dt); }

// Storage scale of one column (1 for FP64/FP32/BF16/FPX) and its codes.
double column_scale(const double* col, int64_t m, int32_t dt) {
    if (is_aflp(dt)) return std::ldexp(1.0, aflp_scale_exp(col, m));
    if (!range_scaled(dt)) return 1.0;
    double mx = 0.0;
    for (int64_t i = 0; i < m; ++i) mx = std::max(mx, std::fabs(col[i]));
    if (mx == 0.0) return 1.0;
    double c = (double)(float)(mx / dtype_max(dt));
    return c < 1.1754943508222875e-38 ? 1.1754943508222875e-38 : c;   // 2^-126
}

// VALR (Sec. 4.2): the cheapest format whose measured column error
// ||w - c*q||_2 (squares summed in row order, float64) is at most delta.
int32_t valr_choose(const double* col, int64_t m, double delta) {
    static const int32_t ladder[4] = {HM_FP8E4M3, HM_F16, HM_BF16, HM_F32};
    const double d2 = delta * delta;
    for (int32_t dt : ladder) {
        const double c = column_scale(col, m, dt);
        double e2 = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            const double q = round_to(dt, c == 1.0 ? col[i] : col[i] / c);
            const double d = col[i] - c * q;
            e2 = e2 + d * d;
        }
        if (e2 <= d2) return dt;
    }
    return HM_F64;
}

// VALR (Sec. 4.2) over the codecs of Sec. 4.1: the narrowest AFLP width
// (exponent width e of the factor) or the first FPX row whose measured
// column error is at most delta; FP64 otherwise.
int32_t valr_choose_aflp(const double* col, int64_t m, double delta, int e) {
    const double d2 = delta * delta;
    const int k = aflp_scale_exp(col, m);
    for (int B = 1; B <= 7; ++B) {
        if (!aflp_feasible(B, e)) continue;
        double e2 = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            double q;
            aflp_encode(col[i], k, e, B, &q);
            const double d = col[i] - q;
            e2 = e2 + d * d;
        }
        if (e2 <= d2) return aflp_dtype(B);
    }
    return HM_F64;
}

int32_t valr_choose_fpx(const double* col, int64_t m, double delta) {
    static const int32_t ladder[6] = {HM_BF16, HM_FPX24, HM_F32, HM_FPX40, HM_FPX48, HM_FPX56};
    const double d2 = delta * delta;
    for (int32_t dt : ladder) {
        double e2 = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            const double d = col[i] - round_to(dt, col[i]);
            e2 = e2 + d * d;
        }
        if (e2 <= d2) return dt;
    }
    return HM_F64;
}

// Per-column formats of one factor under an adaptive policy: the codec
// ladders (e: the factor's AFLP exponent width), or the hardware ladder
// (valr_formats).
std::vector<int32_t> valr_formats(const double* A, int64_t m, int64_t k, const std::vector<double>& deltas,
                                  bool promote);
std::vector<int32_t> column_formats(int32_t policy, const double* A, int64_t m, int64_t k,
                                    const std::vector<double>& deltas, bool promote, int e) {
    if (policy == HM_VALR_AUTO) return valr_formats(A, m, k, deltas, promote);
    std::vector<int32_t> dts((size_t)k);
    for (int64_t j = 0; j < k; ++j)
        dts[(size_t)j] = policy == HM_AFLP_AUTO ? valr_choose_aflp(A + j * m, m, deltas[(size_t)j], e)
                                                : valr_choose_fpx(A + j * m, m, deltas[(size_t)j]);
    return dts;
}

bool adaptive(int32_t dt) { return dt == HM_VALR_AUTO || dt == HM_AFLP_AUTO || dt == HM_FPX_AUTO; }
bool aflp_kind(int32_t dt) { return dt == HM_AFLP_AUTO || is_aflp(dt); }

// VALR formats of the k columns of one factor: each column's cheapest format
// (valr_choose, Sec. 4.2).  With `promote` (a storage choice of this
// library, off by default), a format used by fewer columns than one 16-byte
// tile holds is then promoted to the least precise more precise format the
// factor already uses, provided that costs that format at most the one tile
// the short run frees.  A promoted column is stored more precisely than its
// budget needs; short runs of cheap columns would otherwise cost a nearly
// empty padded tile and a separate item each.
std::vector<int32_t> valr_formats(const double* A, int64_t m, int64_t k, const std::vector<double>& deltas,
                                  bool promote) {
    std::vector<int32_t> dts((size_t)k);
    for (int64_t j = 0; j < k; ++j) dts[(size_t)j] = valr_choose(A + j * m, m, deltas[(size_t)j]);
    if (!promote) return dts;
    static const int32_t order[5] = {HM_FP8E4M3, HM_BF16, HM_F16, HM_F32, HM_F64};   // precision, ascending
    int64_t cnt[5] = {0, 0, 0, 0, 0};
    for (int32_t d : dts) cnt[d]++;
    auto tiles = [](int64_t c, int32_t d) { return (c + 16 / dtype_bytes(d) - 1) / (16 / dtype_bytes(d)); };
    for (int a = 0; a < 4; ++a) {
        const int32_t d = order[a];
        if (cnt[d] == 0 || cnt[d] >= 16 / dtype_bytes(d)) continue;
        for (int b = a + 1; b < 5; ++b) {
            const int32_t t = order[b];
            if (cnt[t] == 0) continue;
            if (tiles(cnt[t] + cnt[d], t) <= tiles(cnt[t], t) + 1) {
                for (int32_t& x : dts)
                    if (x == d) x = t;
                cnt[t] += cnt[d];
                cnt[d] = 0;
            }
            break;
        }
    }
    return dts;
}

// Direct compression (Sec. 4.1): cheapest format with unit roundoff <= eps.
int32_t direct_for_eps(double eps) {
    if (eps >= 0.0625) return HM_FP8E4M3;
    if (eps >= 0.00048828125) return HM_F16;
    if (eps >= 5.9604644775390625e-08) return HM_F32;
    return HM_F64;
}

// leaf clusters from which the dependent stages' default task size doubles
constexpr int64_t kChainDoubleLeaves = 2048;

struct Builder {
    const Layout& L;
    int32_t fmt;
    const hm_values* V;
    PackOptions opt;
    int32_t dense_dt, diag_dt, factor_dt, coup_dt;
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

    // dt may be a codec policy or a fixed AFLP width: resolved here from the
    // matrix (ebits > 0: the AFLP exponent width already fixed by the whole
    // factor this source is a run of)
    int32_t add_source(const double* A, int64_t m, int64_t k, int32_t dt, const double* colfactor,
                       int cls, int ebits = 0) {
        Source s;
        s.A = A;
        s.m = m;
        s.k = k;
        if (aflp_kind(dt)) {
            const int e = ebits > 0 ? ebits : (A ? aflp_matrix_ebits(A, m, k) : 1);
            int B = 0;
            if (dt == HM_AFLP_AUTO) {
                B = aflp_direct_width(e, eps);
            } else {
                B = aflp_width(dt);
                while (B <= 7 && !aflp_feasible(B, e)) ++B;
                if (B > 7) B = 0;
            }
            dt = B ? aflp_dtype(B) : HM_F64;
            s.ebits = B ? e : 0;
        } else if (dt == HM_FPX_AUTO) {
            dt = fpx_for_eps(eps);
        }
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

    double eps = 0.0;
    std::deque<std::vector<double>> pool;   // stable storage for host-made matrices

    // A factor (low-rank factor or cluster basis) stored as runs of columns
    // of one dtype: one run unless factor_dt is VALR_AUTO.
    struct Run {
        int32_t src, c0, k;
    };
    // deltas: per-column error budget delta_j of VALR (unused otherwise);
    // breaks (optional): brk[j] != 0 forces a run to start at column j
    // dts_in (optional): the formats, already chosen, of the k columns
    // es_in (optional): their AFLP exponent widths (else one for the factor)
    std::vector<Run> add_factor(const double* A, int64_t m, int64_t k, const double* colfactor, int cls,
                                const std::vector<double>& deltas, const std::vector<uint8_t>* brk = nullptr,
                                const std::vector<int32_t>* dts_in = nullptr,
                                const std::vector<int32_t>* es_in = nullptr) {
        std::vector<Run> runs;
        if (k == 0) return runs;
        // AFLP: one exponent width for the whole factor (every run of it)
        const int e = aflp_kind(factor_dt) && !es_in ? aflp_matrix_ebits(A, m, k) : 0;
        std::vector<int32_t> dts(k, factor_dt);
        if (adaptive(factor_dt))
            dts = dts_in ? *dts_in : column_formats(factor_dt, A, m, k, deltas, opt.valr_promote, e);
        std::vector<int32_t> es(k, e);
        if (es_in) es = *es_in;
        int64_t j0 = 0;
        for (int64_t j = 1; j <= k; ++j)
            if (j == k || dts[j] != dts[j0] || es[j] != es[j0] || (brk && (*brk)[(size_t)j])) {
                runs.push_back(Run{add_source(A + j0 * m, m, j - j0, dts[j0], colfactor ? colfactor + j0 : nullptr, cls,
                                              es[j0]),
                                   (int32_t)j0, (int32_t)(j - j0)});
                j0 = j;
            }
        return runs;
    }

    // scale index of column j of a factor (-1 = 1.0)
    int64_t run_scale(const std::vector<Run>& runs, int32_t j) const {
        for (const Run& r : runs)
            if (j < r.c0 + r.k) return src[r.src].scale_off >= 0 ? src[r.src].scale_off + (j - r.c0) : -1;
        return -1;
    }

    // element-wise scale products: scales[dst] = s(a) * s(b), s(-1) = 1
    std::vector<std::array<int64_t, 3>> efolds;
    int32_t fold_list(const std::vector<int64_t>& a, const std::vector<int64_t>& b) {
        bool any = false;
        for (size_t i = 0; i < a.size(); ++i) any |= a[i] >= 0 || b[i] >= 0;
        if (!any) return -1;
        const int32_t dst = (int32_t)nscales;
        nscales += (int64_t)a.size();
        for (size_t i = 0; i < a.size(); ++i) efolds.push_back({dst + (int64_t)i, a[i], b[i]});
        return dst;
    }

    // scales[dst + j] = scales[a + j] * scales[b + j] (a or b < 0: factor 1),
    // evaluated after every source has been quantised
    struct Fold {
        int64_t dst, a, b, k;
    };
    std::vector<Fold> folds;
    int32_t fold_scales(int32_t a, int32_t b, int64_t k) {
        if (a < 0 && b < 0) return -1;
        if (a < 0 || b < 0) return a < 0 ? b : a;
        int32_t dst = (int32_t)nscales;
        nscales += k;
        folds.push_back(Fold{dst, a, b, k});
        return dst;
    }

    // host transpose (for F^T), stored inside the source
    int32_t add_source_transposed(const double* A, int64_t m, int64_t k, int32_t dt, int cls) {
        std::vector<double> T((size_t)(m * k));
        for (int64_t j = 0; j < k; ++j)
            for (int64_t i = 0; i < m; ++i) T[(size_t)(j + i * k)] = A[i + j * m];
        int32_t id = add_source(T.data(), k, m, dt, nullptr, cls);
        Source& s = src[id];
        s.own = std::move(T);   // the buffer moves with its data
        s.A = s.own.data();
        return id;
    }

    // ---- owner construction
    // Owners and items go straight into the global tables.  Tasks go to the
    // stage the owner was begun in, except tasks made only of floating items
    // (dense leaves: they read nothing but x), which are kept aside and later
    // spread over all stages to fill each launch (see place_floating).
    std::vector<DOwner> owners;
    std::vector<DItem> items;
    std::vector<uint8_t> item_floating;
    std::vector<std::pair<int32_t, int32_t>> item_use;   // (source, index of its Use) per item
    std::vector<std::vector<DTask>> stage_tasks;
    std::vector<int64_t> stage_bytes;
    std::vector<std::string> stage_names;
    std::vector<std::pair<DTask, int64_t>> floating;   // (task, bytes)
    std::vector<int32_t> item_stage;                    // per item: its tasks' stage (-1: the owner's)
    int64_t part_elems = 0;
    int32_t cur_stage = -1;
    DOwner cur{};
    int32_t cur_cols = 0;
    int32_t cur_tiles = 0;

    int32_t new_stage(const char* name) {
        stage_tasks.emplace_back();
        stage_bytes.push_back(0);
        stage_names.push_back(name);
        return (int32_t)stage_tasks.size() - 1;
    }

    void begin_owner(int32_t stage, int32_t nrows, int32_t mode, int32_t out_off, int32_t rscale_off) {
        cur_stage = stage;
        cur = DOwner{};
        cur.nrows = nrows;
        cur.item0 = (int32_t)items.size();
        cur.nitems = 0;
        cur.out_off = out_off;
        cur.mode = mode;
        cur.rscale_off = rscale_off;
        cur_cols = 0;
        cur_tiles = 0;
    }

    // item = rows [r0, r0+nr) of source s (all its columns), or the transpose
    // unscaled: the source's column scales were folded into the producer of
    // the item's input vector (see fold_scales), so the item multiplies none.
    // stage >= 0: the item's tasks run in that (earlier) stage, not in the
    // stage the owner was begun in (see build_h2)
    void add_item(int32_t s, int64_t r0, bool transposed, int32_t vec_off, bool unscaled = false,
                  bool floats = false, int32_t stage = -1) {
        Source& S = src[s];
        const int64_t nr = cur.nrows;
        const int64_t ncols = transposed ? S.m : S.k;
        if (ncols == 0 || nr == 0) return;
        const int64_t bytes = tile_count(S.dtype, ncols) * nr * 16;
        DItem it{};
        it.data_off = alloc_data(bytes);
        it.tile0 = cur_tiles;
        cur_tiles += (int32_t)tile_count(S.dtype, ncols);
        it.col0 = cur_cols;
        it.ncols = (int32_t)ncols;
        it.vec_off = vec_off;
        it.scale_off = (transposed || unscaled) ? -1 : S.scale_off;
        it.dtype = (int16_t)S.dtype;
        it.ebits = (int16_t)S.ebits;
        items.push_back(it);
        item_floating.push_back(floats ? 1 : 0);
        item_stage.push_back(stage);
        item_use.emplace_back(s, (int32_t)S.uses.size());
        cur.nitems++;
        cur_cols += (int32_t)ncols;
        S.uses.push_back(Use{it.data_off, r0, nr, transposed});
    }

    // Order the owner's items by (floating, dtype, AFLP exponent width),
    // stably, so that each dtype is one run of columns and tasks (which hold
    // one dtype and one exponent width) are cut only at the few run boundaries; mixed-format factors would otherwise split an
    // owner at every format change.  Columns, tiles and data offsets are
    // reassigned in the new order (the items' data is one contiguous block).
    void group_items() {
        const int32_t n = cur.nitems, i0 = cur.item0;
        if (n < 2) return;
        std::vector<int32_t> order(n);
        for (int32_t i = 0; i < n; ++i) order[i] = i;
        auto key = [&](int32_t i) {
            return ((int64_t)(item_floating[i0 + i] * 32 + items[i0 + i].dtype) * 16 + items[i0 + i].ebits) *
                       (1 << 20) + (item_stage[i0 + i] + 1);
        };
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });
        bool same = true;
        for (int32_t i = 0; i < n; ++i) same &= order[i] == i;
        if (same) return;
        std::vector<DItem> it(n);
        std::vector<uint8_t> fl(n);
        std::vector<int32_t> sg(n);
        std::vector<std::pair<int32_t, int32_t>> us(n);
        int64_t off = items[i0].data_off;
        int32_t col = 0, tile = 0;
        for (int32_t k = 0; k < n; ++k) {
            const int32_t i = i0 + order[k];
            DItem d = items[i];
            const int64_t tiles = tile_count(d.dtype, d.ncols);
            d.data_off = off;
            d.col0 = col;
            d.tile0 = tile;
            off += tiles * cur.nrows * 16;
            col += d.ncols;
            tile += (int32_t)tiles;
            it[k] = d;
            fl[k] = item_floating[i];
            sg[k] = item_stage[i];
            us[k] = item_use[i];
            src[us[k].first].uses[us[k].second].data_off = d.data_off;
        }
        for (int32_t k = 0; k < n; ++k) {
            items[i0 + k] = it[k];
            item_floating[i0 + k] = fl[k];
            item_stage[i0 + k] = sg[k];
            item_use[i0 + k] = us[k];
        }
    }

    void end_owner() {
        group_items();
        const int32_t owner_id = (int32_t)owners.size();
        // cut the owner's columns into tasks of about opt.task_bytes, on tile
        // boundaries, never mixing floating and fixed items in one task
        std::vector<std::pair<DTask, int64_t>> made;
        int32_t start_col = 0, start_item = cur.item0;
        int64_t acc = 0;
        auto emit = [&](int32_t c1) {
            DTask t{};
            t.owner = owner_id;
            t.c0 = start_col;
            t.c1 = c1;
            t.item_start = start_item;
            t.local = (int32_t)made.size();
            made.push_back({t, acc});
            start_col = c1;
            acc = 0;
        };
        for (int32_t i = 0; i < cur.nitems; ++i) {
            const int32_t ii = cur.item0 + i;
            const DItem& it = items[ii];
            // a task never mixes floating and fixed items, nor two dtypes or
            // AFLP exponent widths
            if (i > 0 && start_col < it.col0 &&
                (item_floating[ii] != item_floating[ii - 1] || it.dtype != items[ii - 1].dtype ||
                 it.ebits != items[ii - 1].ebits || item_stage[ii] != item_stage[ii - 1])) {
                emit(it.col0);
                start_item = ii;
            }
            const int V = tile_cols(it.dtype);
            const int64_t bpt = (int64_t)cur.nrows * 16;     // bytes per tile
            // a task may stage its inputs in LDS (narrow owners always, wide
            // ones when they read unreduced sums): at most MAX_TASK_INPUTS
            // input values (tiles * V) per task
            const int64_t cap = (int64_t)(MAX_TASK_INPUTS / V) * bpt;
            // default task size by storage format (measured on the single-
            // vector product): 32 KiB of float64 tiles, 16 KiB of narrower
            // ones; the dependent stages of a matrix with at least
            // kChainDoubleLeaves leaf clusters take twice that (fewer tasks
            // and partial sums on the chain pay once its stages still have
            // enough tasks to fill the chip; on smaller matrices they cost
            // parallelism)
            const int64_t base = it.dtype == HM_F64 ? 32768 : 16384;
            const int64_t chain = (int64_t)leaves.size() >= kChainDoubleLeaves ? 2 * base : base;
            const int64_t tb = item_floating[ii] ? (opt.task_bytes ? opt.task_bytes : base)
                               : opt.chain_task_bytes ? opt.chain_task_bytes
                               : opt.task_bytes       ? opt.task_bytes
                                                      : chain;
            const int64_t target = std::min<int64_t>(tb, cap);
            int32_t j = 0;
            while (j < it.ncols) {
                int64_t room = target - acc;
                int64_t take = std::max<int64_t>(1, room / bpt) * V;   // whole tiles
                take = std::min<int64_t>(take, it.ncols - j);
                acc += ((take + V - 1) / V) * bpt;
                j += (int32_t)take;
                if (acc >= target) {
                    emit(it.col0 + j);
                    start_item = (j == it.ncols) ? ii + 1 : ii;
                }
            }
        }
        if (start_col < cur_cols || made.empty()) {
            start_item = std::min(start_item, cur.item0 + std::max(cur.nitems - 1, 0));
            emit(cur_cols);
        }
        cur.ntasks = (int32_t)made.size();
        cur.part_off = 0;
        if (cur.ntasks > 1) {
            cur.part_off = (int32_t)part_elems;
            part_elems += (int64_t)cur.ntasks * cur.nrows;
        }
        // column -> tile of the owner's stream (task bounds are tile aligned
        // inside an item; an item's end maps to its last tile + 1)
        auto tile_of = [&](int32_t c) -> int32_t {
            for (int32_t i = 0; i < cur.nitems; ++i) {
                const DItem& it = items[cur.item0 + i];
                if (c < it.col0 + it.ncols) return it.tile0 + (c - it.col0) / tile_cols(it.dtype);
            }
            return cur_tiles;
        };
        const int64_t stream = cur.nitems ? items[cur.item0].data_off : 0;
        for (auto& tb : made) {
            DTask& t = tb.first;
            t.k0 = tile_of(t.c0);
            t.k1 = tile_of(t.c1);
            t.stream = stream;
            t.nrows = cur.nrows;
            t.dtype = (int16_t)(t.c0 < t.c1 ? items[t.item_start].dtype : -1);
            // mode bits 8..11: the AFLP exponent width of the task's items
            t.mode = (int16_t)(cur.mode | (t.c0 < t.c1 ? items[t.item_start].ebits << 8 : 0));
            t.out_off = cur.out_off;
            t.ntasks = cur.ntasks;
            t.part_off = cur.part_off;
            t.rscale_off = cur.rscale_off;
            const bool fl = t.c0 < t.c1 && item_floating[t.item_start];
            if (fl) {
                floating.push_back(tb);
            } else {
                const int32_t si = t.c0 < t.c1 && item_stage[t.item_start] >= 0 ? item_stage[t.item_start] : cur_stage;
                stage_tasks[si].push_back(t);
                stage_bytes[si] += tb.second;
            }
        }
        owners.push_back(cur);
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

    // the dense leaves whose row cluster contains rho (floating items)
    void add_dense_items(int32_t rho, const std::vector<int32_t>& anc, std::vector<int32_t>& dsrc) {
        for (int32_t t : anc) {
            const int64_t r0 = L.node_begin[rho] - L.node_begin[t];
            for (int32_t b : row_blocks[t]) {
                if (L.blk_adm[b]) continue;
                if (dsrc[b] < 0) dsrc[b] = dense_source(b);
                add_item(dsrc[b], r0, false, (int32_t)L.node_begin[L.blk_sigma[b]], false, true);
            }
        }
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

    // VALR tolerances.  H block b = W diag(s) X^T: its columns w_j, x_j get
    // delta_j = delta / s_j with delta = eps ||s||_2 / (1 + 2k), so the bound
    // of eq. (6) stays at the truncation error eps ||s||_2.  Cluster bases
    // with weights s: delta = eps ||s||_2 / k (eq. 7).
    static double norm2(const double* w, int64_t k) {
        double t = 0.0;
        for (int64_t j = 0; j < k; ++j) t = t + w[j] * w[j];
        return std::sqrt(t);
    }
    // delta_j = delta / w_j (a zero weight gives an unlimited budget)
    static std::vector<double> deltas_for(const double* w, int64_t k, double delta) {
        std::vector<double> d((size_t)k);
        for (int64_t j = 0; j < k; ++j) d[(size_t)j] = w[j] > 0.0 ? delta / w[j] : HUGE_VAL;
        return d;
    }
    bool need_sv(const double* const* sv, int32_t v, int32_t k) {
        if (!adaptive(factor_dt) || k == 0) return true;
        return check(sv && sv[v], "VALR storage needs row_sv / col_sv basis weights");
    }
    std::vector<Run> basis_factor(const double* A, int64_t m, int64_t k, const double* const* sv, int32_t v) {
        std::vector<double> d;
        if (adaptive(factor_dt)) d = deltas_for(sv[v], k, eps * norm2(sv[v], k) / (double)k);
        return add_factor(A, m, k, nullptr, 1, d);
    }

    // Input-side bases under VALR (UH column bases, H2 leaf column bases):
    // the basis is a transposed owner whose rows are its columns, and an
    // owner's rows must share one format.  The columns are therefore reordered
    // so that equal formats are adjacent (stable), giving one owner per format
    // instead of one per run; perm[p] = original column at position p (empty:
    // unchanged).  Every consumer of the coefficient vector (coupling columns,
    // H2 transfer rows) is permuted the same way, so the product is unchanged.
    std::vector<Run> grouped_basis(const double* A, int64_t m, int64_t k, const double* const* sv, int32_t v,
                                   std::vector<int32_t>& perm) {
        perm.clear();
        if (!adaptive(factor_dt) || k == 0) return basis_factor(A, m, k, sv, v);
        std::vector<double> d = deltas_for(sv[v], k, eps * norm2(sv[v], k) / (double)k);
        const int e = aflp_kind(factor_dt) ? aflp_matrix_ebits(A, m, k) : 0;   // of the whole basis
        const std::vector<int32_t> dts = column_formats(factor_dt, A, m, k, d, opt.valr_promote, e);
        std::vector<int32_t> order((size_t)k);
        for (int64_t j = 0; j < k; ++j) order[(size_t)j] = (int32_t)j;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return dts[a] < dts[b]; });
        bool same = true;
        for (int64_t j = 0; j < k; ++j) same &= order[(size_t)j] == j;
        if (same) return add_factor(A, m, k, nullptr, 1, d, nullptr, &dts);
        pool.emplace_back((size_t)(m * k));
        std::vector<double>& P = pool.back();
        std::vector<double> dp((size_t)k);
        std::vector<int32_t> dtp((size_t)k);
        for (int64_t p = 0; p < k; ++p) {
            std::memcpy(P.data() + p * m, A + (int64_t)order[(size_t)p] * m, sizeof(double) * (size_t)m);
            dp[(size_t)p] = d[(size_t)order[(size_t)p]];
            dtp[(size_t)p] = dts[(size_t)order[(size_t)p]];
        }
        perm = order;
        return add_factor(P.data(), m, k, nullptr, 1, dp, nullptr, &dtp);
    }
    // columns of a (rows x cols) matrix in the order perm (empty: A itself)
    const double* permute_cols(const double* A, int64_t rows, int64_t cols, const std::vector<int32_t>& perm) {
        if (perm.empty()) return A;
        pool.emplace_back((size_t)(rows * cols));
        std::vector<double>& P = pool.back();
        for (int64_t p = 0; p < cols; ++p)
            std::memcpy(P.data() + p * rows, A + (int64_t)perm[(size_t)p] * rows, sizeof(double) * (size_t)rows);
        return P.data();
    }
    // rows of a (rows x cols) column-major matrix in the order perm
    const double* permute_rows(const double* A, int64_t rows, int64_t cols, const std::vector<int32_t>& perm) {
        if (perm.empty()) return A;
        pool.emplace_back((size_t)(rows * cols));
        std::vector<double>& P = pool.back();
        for (int64_t j = 0; j < cols; ++j)
            for (int64_t p = 0; p < rows; ++p) P[(size_t)(p + j * rows)] = A[perm[(size_t)p] + j * rows];
        return P.data();
    }

    // --------------------------------------------------------------- H
    bool build_h() {
        if (!check_dense()) return false;
        if (!V->rank || !V->W || !V->sigma || !V->X) return check(false, "H needs rank, W, sigma, X");
        const int64_t nb = (int64_t)L.blk_tau.size();
        std::vector<int32_t> dsrc(nb, -1);
        std::vector<std::vector<Run>> urun(nb);
        for (int64_t b = 0; b < nb; ++b) {
            if (!L.blk_adm[b]) continue;
            const int32_t k = V->rank[b];
            const int64_t mt = L.size(L.blk_tau[b]), ms = L.size(L.blk_sigma[b]);
            if (k < 0 || k > std::min(mt, ms)) return check(false, "rank out of range");
            if (k > 0 && (!V->W[b] || !V->sigma[b] || !V->X[b])) return check(false, "missing factor");
        }
        // t_b = X_b^T x|s for all low-rank blocks of one block column s at
        // once: the X_b^T are stacked into one owner (they read the same x|s),
        // and the t_b of a block column are laid out consecutively.
        std::vector<std::vector<int32_t>> col_lr(L.node_begin.size());
        for (int64_t b = 0; b < nb; ++b)
            if (L.blk_adm[b] && V->rank[b] > 0) col_lr[L.blk_sigma[b]].push_back((int32_t)b);
        // position of t_b[j] in the workspace; with VALR the stacked columns of
        // a block column are reordered by the format of X (stable), so X^T
        // gives one owner per format and t_b may be scattered in its block
        // column's range
        std::vector<std::vector<int32_t>> tpos(nb);
        const int32_t pa = new_stage("h_vt");
        for (int32_t s = 0; s < (int32_t)col_lr.size(); ++s) {
            if (col_lr[s].empty()) continue;
            const int64_t ms = L.size(s);
            int64_t K = 0;
            for (int32_t b : col_lr[s]) K += V->rank[b];
            // stacked X = [X_b1 X_b2 ...] (|s| x K) with per-column weights
            pool.emplace_back((size_t)(ms * K));
            std::vector<double>& Xs = pool.back();
            std::vector<double> Ds;              // VALR budgets of the stacked columns
            std::vector<int64_t> uscale;         // U-side scale index per stacked column
            int64_t c0 = 0;
            for (int32_t b : col_lr[s]) {
                const int32_t k = V->rank[b];
                std::memcpy(Xs.data() + c0 * ms, V->X[b], sizeof(double) * (size_t)(ms * k));
                std::vector<double> d((size_t)k, 0.0);
                if (adaptive(factor_dt))
                    d = deltas_for(V->sigma[b], k, eps * norm2(V->sigma[b], k) / (1.0 + 2.0 * k));
                Ds.insert(Ds.end(), d.begin(), d.end());
                c0 += k;
            }
            // order of the stacked columns: by X's format under VALR (and
            // AFLP exponent width: each X_b is its own stored matrix, with
            // its own e, though stacked)
            std::vector<int32_t> order((size_t)K), inv((size_t)K);
            for (int64_t o = 0; o < K; ++o) order[(size_t)o] = (int32_t)o;
            std::vector<int32_t> dtx((size_t)K, factor_dt);   // X's formats, chosen per block
            std::vector<int32_t> esx((size_t)K, 0);           // X's AFLP exponent widths
            if (adaptive(factor_dt) || aflp_kind(factor_dt)) {
                int64_t o0 = 0;
                for (int32_t b : col_lr[s]) {
                    const int32_t k = V->rank[b];
                    std::vector<double> d(Ds.begin() + o0, Ds.begin() + o0 + k);
                    const double* Xb = Xs.data() + o0 * ms;
                    const int e = aflp_kind(factor_dt) ? aflp_matrix_ebits(Xb, ms, k) : 0;
                    if (adaptive(factor_dt)) {
                        const std::vector<int32_t> f = column_formats(factor_dt, Xb, ms, k, d, opt.valr_promote, e);
                        std::copy(f.begin(), f.end(), dtx.begin() + o0);
                    }
                    std::fill(esx.begin() + o0, esx.begin() + o0 + k, e);
                    o0 += k;
                }
                std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
                    return dtx[a] != dtx[b] ? dtx[a] < dtx[b] : esx[a] < esx[b];
                });
            }
            for (int64_t p = 0; p < K; ++p) inv[(size_t)order[(size_t)p]] = (int32_t)p;
            const int32_t base = (int32_t)ws;
            ws += K;
            // U side: runs of W_b never cross a jump of t_b's positions
            c0 = 0;
            uscale.clear();
            for (int32_t b : col_lr[s]) {
                const int32_t k = V->rank[b];
                std::vector<uint8_t> brk((size_t)k, 0);
                tpos[b].resize((size_t)k);
                for (int32_t j = 0; j < k; ++j) {
                    tpos[b][(size_t)j] = base + inv[(size_t)(c0 + j)];
                    brk[(size_t)j] = j > 0 && tpos[b][(size_t)j] != tpos[b][(size_t)j - 1] + 1;
                }
                std::vector<double> d(Ds.begin() + c0, Ds.begin() + c0 + k);
                urun[b] = add_factor(V->W[b], L.size(L.blk_tau[b]), k, V->sigma[b], 1, d, &brk);
                for (int32_t j = 0; j < k; ++j) uscale.push_back(run_scale(urun[b], j));
                c0 += k;
            }
            const double* Xo = Xs.data();
            std::vector<double> Dp = Ds;
            std::vector<int32_t> dtp = dtx, esp = esx;
            bool same = true;
            for (int64_t p = 0; p < K; ++p) same &= order[(size_t)p] == p;
            if (!same) {
                pool.emplace_back((size_t)(ms * K));
                std::vector<double>& Xp = pool.back();
                for (int64_t p = 0; p < K; ++p) {
                    std::memcpy(Xp.data() + p * ms, Xs.data() + (int64_t)order[(size_t)p] * ms,
                                sizeof(double) * (size_t)ms);
                    Dp[(size_t)p] = Ds[(size_t)order[(size_t)p]];
                    dtp[(size_t)p] = dtx[(size_t)order[(size_t)p]];
                    esp[(size_t)p] = esx[(size_t)order[(size_t)p]];
                }
                Xo = Xp.data();
            }
            std::vector<Run> xr = add_factor(Xo, ms, K, nullptr, 1, Dp, nullptr, &dtp, &esp);
            for (const Run& r : xr) {
                // row scale: X's range scale times the U-side column scale
                // (sigma_j and W's range scale) of the same column
                std::vector<int64_t> a, bb;
                for (int32_t j = 0; j < r.k; ++j) {
                    a.push_back(src[r.src].scale_off >= 0 ? src[r.src].scale_off + j : -1);
                    bb.push_back(uscale[(size_t)order[(size_t)(r.c0 + j)]]);
                }
                begin_owner(pa, r.k, 0, base + r.c0, fold_list(a, bb));
                add_item(r.src, 0, true, (int32_t)L.node_begin[s]);
                end_owner();
            }
        }
        const int32_t pb = new_stage("h_rows");
        for (int32_t rho : leaves) {
            begin_owner(pb, (int32_t)L.size(rho), 1, (int32_t)L.node_begin[rho], -1);
            const std::vector<int32_t> anc = ancestors_root_first(rho);
            for (int32_t t : anc) {
                const int64_t r0 = L.node_begin[rho] - L.node_begin[t];
                for (int32_t b : row_blocks[t])
                    if (L.blk_adm[b] && V->rank[b] > 0)
                        for (const Run& r : urun[b]) add_item(r.src, r0, false, tpos[b][(size_t)r.c0], true);
            }
            add_dense_items(rho, anc, dsrc);
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
        std::vector<int32_t> s_off(N, -1), t_off(N, -1), dsrc(nb, -1);
        std::vector<std::vector<Run>> wrun(N);
        for (int32_t v = 0; v < N; ++v) {
            const int32_t kr = V->row_rank[v], kc = V->col_rank[v];
            if (kr < 0 || kc < 0 || kr > L.size(v) || kc > L.size(v)) return check(false, "basis rank out of range");
            if ((kr > 0 && !V->row_basis[v]) || (kc > 0 && !V->col_basis[v])) return check(false, "missing basis");
            if (!need_sv(V->row_sv, v, kr) || !need_sv(V->col_sv, v, kc)) return false;
            if (kc > 0) { s_off[v] = (int32_t)ws; ws += kc; }
            if (kr > 0) { t_off[v] = (int32_t)ws; ws += kr; }
        }
        for (int64_t b = 0; b < nb; ++b)
            if (L.blk_adm[b]) {
                const int32_t kr = V->row_rank[L.blk_tau[b]], kc = V->col_rank[L.blk_sigma[b]];
                if (kr > 0 && kc > 0 && !V->coupling[b]) return check(false, "missing coupling");
            }
        const int32_t pf = new_stage("uh_fwd");
        std::vector<std::vector<int32_t>> cperm(N);
        for (int32_t v = 0; v < N; ++v) {
            const int32_t kc = V->col_rank[v];
            if (kc == 0) continue;
            for (const Run& r : grouped_basis(V->col_basis[v], L.size(v), kc, V->col_sv, v, cperm[v])) {
                begin_owner(pf, r.k, 0, s_off[v] + r.c0, src[r.src].scale_off);
                add_item(r.src, 0, true, (int32_t)L.node_begin[v]);
                end_owner();
            }
        }
        for (int32_t v = 0; v < N; ++v)
            if (V->row_rank[v] > 0) wrun[v] = basis_factor(V->row_basis[v], L.size(v), V->row_rank[v], V->row_sv, v);
        const int32_t pc = new_stage("uh_coup");
        for (int32_t t = 0; t < N; ++t) {
            const int32_t kr = V->row_rank[t];
            if (kr == 0) continue;
            // t_t is produced times the column scales of W_t (its only consumer)
            std::vector<int64_t> a, none(kr, -1);
            for (int32_t j = 0; j < kr; ++j) a.push_back(run_scale(wrun[t], j));
            begin_owner(pc, kr, 0, t_off[t], fold_list(a, none));
            for (int32_t b : row_blocks[t]) {
                if (!L.blk_adm[b]) continue;
                const int32_t s = L.blk_sigma[b];
                const int32_t kc = V->col_rank[s];
                if (kc == 0) continue;
                int32_t cs = add_source(permute_cols(V->coupling[b], kr, kc, cperm[s]), kr, kc, coup_dt, nullptr, 2);
                add_item(cs, 0, false, s_off[s]);
            }
            end_owner();
        }
        const int32_t pr = new_stage("uh_rows");
        for (int32_t rho : leaves) {
            begin_owner(pr, (int32_t)L.size(rho), 1, (int32_t)L.node_begin[rho], -1);
            const std::vector<int32_t> anc = ancestors_root_first(rho);
            for (int32_t t : anc)
                for (const Run& r : wrun[t])
                    add_item(r.src, L.node_begin[rho] - L.node_begin[t], false, t_off[t] + r.c0, true);
            add_dense_items(rho, anc, dsrc);
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
            if (L.leaf(v) && (!need_sv(V->row_sv, v, kr) || !need_sv(V->col_sv, v, kc))) return false;
            const int32_t p = L.node_parent[v];
            if (p >= 0) {
                if (kr > 0 && V->row_rank[p] > 0 && !V->row_transfer[v]) return check(false, "missing row transfer");
                if (kc > 0 && V->col_rank[p] > 0 && !V->col_transfer[v]) return check(false, "missing col transfer");
            }
            if (kc > 0) { s_off[v] = (int32_t)ws; ws += kc; }
            if (kr > 0) { t_off[v] = (int32_t)ws; ws += kr; }
        }
        const int32_t pl = new_stage("h2_up_leaf");
        std::vector<std::vector<int32_t>> cperm(N);
        for (int32_t g : leaves) {
            const int32_t kc = V->col_rank[g];
            if (kc == 0) continue;
            for (const Run& r : grouped_basis(V->col_basis[g], L.size(g), kc, V->col_sv, g, cperm[g])) {
                begin_owner(pl, r.k, 0, s_off[g] + r.c0, src[r.src].scale_off);
                add_item(r.src, 0, true, (int32_t)L.node_begin[g]);
                end_owner();
            }
        }
        std::vector<std::vector<int32_t>> by_level(L.depth + 1);
        for (int32_t v = 0; v < N; ++v) by_level[L.node_level[v]].push_back(v);
        for (int32_t lv = L.depth - 1; lv >= 0; --lv) {
            bool any = false;
            for (int32_t v : by_level[lv]) any |= (!L.leaf(v) && V->col_rank[v] > 0);
            if (!any) continue;
            const int32_t pu = new_stage("h2_up");
            for (int32_t v : by_level[lv]) {
                const int32_t kc = V->col_rank[v];
                if (L.leaf(v) || kc == 0) continue;
                begin_owner(pu, kc, 0, s_off[v], -1);
                for (int32_t c : {L.node_son0[v], L.node_son1[v]}) {
                    const int32_t kcc = V->col_rank[c];
                    if (kcc == 0) continue;
                    // F_c is kcc x kc; F_c^T is kc x kcc, scaled per column of F_c^T
                    int32_t fs = add_source_transposed(permute_rows(V->col_transfer[c], kcc, kc, cperm[c]), kcc, kc,
                                                       coup_dt, 3);
                    add_item(fs, 0, false, s_off[c]);
                }
                end_owner();
            }
        }
        std::vector<std::vector<Run>> lrun(N);
        for (int32_t rho : leaves)
            if (V->row_rank[rho] > 0)
                lrun[rho] = basis_factor(V->row_basis[rho], L.size(rho), V->row_rank[rho], V->row_sv, rho);
        // The coupling products S_b s_s depend only on the upward pass, so
        // (by default) they run before the downward pass, as partial sums of
        // their row cluster's coefficient owner; the downward recursion
        // t_t = E_t t_parent + (those partial sums) then only adds the small
        // transfer products level by level (Alg. 7's recursion; each owner's
        // partial sums are added in a fixed task order, so the result is
        // deterministic).
        // All of them run in one launch right after the upward pass (measured
        // faster than running each in the upward launch after its input's:
        // the long coarse-level coupling tasks then set those launches'
        // tails, while in one launch they overlap the rest).
        const bool early = opt.coupling_first;
        const int32_t pc = early ? new_stage("h2_coup") : -1;
        for (int32_t lv = 0; lv <= L.depth; ++lv) {
            bool any = false;
            for (int32_t v : by_level[lv]) any |= V->row_rank[v] > 0;
            if (!any) continue;
            const int32_t pd = new_stage("h2_down");
            for (int32_t t : by_level[lv]) {
                const int32_t kr = V->row_rank[t];
                if (kr == 0) continue;
                // a leaf's coefficients feed only its own basis: fold its column scales
                int32_t rs = -1;
                if (L.leaf(t)) {
                    std::vector<int64_t> a, none(kr, -1);
                    for (int32_t j = 0; j < kr; ++j) a.push_back(run_scale(lrun[t], j));
                    rs = fold_list(a, none);
                }
                begin_owner(pd, kr, 0, t_off[t], rs);
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
                    int32_t cs = add_source(permute_cols(V->coupling[b], kr, kc, cperm[s]), kr, kc, coup_dt, nullptr, 2);
                    add_item(cs, 0, false, s_off[s], false, false,
                             early ? pc : -1);
                }
                end_owner();
            }
        }
        const int32_t pr = new_stage("h2_rows");
        for (int32_t rho : leaves) {
            begin_owner(pr, (int32_t)L.size(rho), 1, (int32_t)L.node_begin[rho], -1);
            for (const Run& r : lrun[rho]) add_item(r.src, 0, false, t_off[rho] + r.c0, true);
            add_dense_items(rho, ancestors_root_first(rho), dsrc);
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
            std::vector<uint64_t> codes;   // the stored bit pattern of every entry
            std::vector<double> c;
            for (size_t si = i0; si < i1; ++si) {
                Source& S = src[si];
                if (S.uses.empty()) continue;
                const int64_t m = S.m, k = S.k;
                codes.resize((size_t)(m * k));
                c.assign((size_t)k, 1.0);
                for (int64_t j = 0; j < k; ++j) {
                    const double* col = S.A + j * m;
                    for (int64_t i = 0; i < m; ++i)
                        if (!std::isfinite(col[i])) bad[si] = 1;
                    if (bad[si]) break;
                    const double cj = column_scale(col, m, S.dtype);
                    c[(size_t)j] = cj;
                    if (is_aflp(S.dtype)) {   // codes relative to the column's 2^k
                        const int kj = aflp_scale_exp(col, m);
                        double q;
                        for (int64_t i = 0; i < m; ++i)
                            codes[(size_t)(i + j * m)] = aflp_encode(col[i], kj, S.ebits, aflp_width(S.dtype), &q);
                        continue;
                    }
                    for (int64_t i = 0; i < m; ++i)
                        codes[(size_t)(i + j * m)] =
                            encode(S.dtype, round_to(S.dtype, cj == 1.0 ? col[i] : col[i] / cj));
                }
                if (bad[si]) continue;
                if (S.scale_off >= 0)
                    for (int64_t j = 0; j < k; ++j)
                        scales[(size_t)(S.scale_off + j)] = c[(size_t)j] * (S.colfactor ? S.colfactor[j] : 1.0);
                const int eb = dtype_bytes(S.dtype);
                const int V = tile_cols(S.dtype);
                // slab element (row a, column b) of an R-row slab, tiled: the
                // code's eb bytes, least significant first, at byte (b % V) * eb
                auto put = [&](uint8_t* dst, int64_t R, int64_t a, int64_t b, uint64_t bits) {
                    std::memcpy(dst + (size_t)(((b / V) * R + a) * 16 + (b % V) * eb), &bits, (size_t)eb);
                };
                for (const Use& u : S.uses) {
                    uint8_t* dst = data.data() + u.data_off;
                    if (!u.transposed) {
                        for (int64_t j = 0; j < k; ++j)
                            for (int64_t i = 0; i < u.nr; ++i) put(dst, u.nr, i, j, codes[(size_t)(u.r0 + i + j * m)]);
                    } else {
                        // slab = A^T (k rows, m columns)
                        for (int64_t i = 0; i < m; ++i)
                            for (int64_t j = 0; j < k; ++j) put(dst, k, j, i, codes[(size_t)(i + j * m)]);
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
        for (const Fold& f : folds)
            for (int64_t j = 0; j < f.k; ++j)
                scales[(size_t)(f.dst + j)] = (f.a >= 0 ? scales[(size_t)(f.a + j)] : 1.0) *
                                              (f.b >= 0 ? scales[(size_t)(f.b + j)] : 1.0);
        for (const auto& f : efolds)
            scales[(size_t)f[0]] = (f[1] >= 0 ? scales[(size_t)f[1]] : 1.0) * (f[2] >= 0 ? scales[(size_t)f[2]] : 1.0);
        for (const Source& S : src) {
            int64_t bytes = 0;
            for (const Use& u : S.uses)
                bytes += u.transposed ? tile_count(S.dtype, S.m) * S.k * 16 : tile_count(S.dtype, S.k) * u.nr * 16;
            per_dtype[S.dtype] += bytes;
            per_class[S.cls] += bytes;
        }
        return true;
    }
};

// Every index a kernel will form from the tables must stay inside its
// buffer; checked on the host before anything is uploaded.  Also checks the
// schedule: every owner's tasks are all placed, a split coefficient owner is
// reduced in the stage of its tasks, and every split y owner in the last.
bool validate(const Packed& P, int64_t n, std::string& why) {
    const int64_t nsc = (int64_t)P.scales.size();
    const int64_t nd = (int64_t)P.data.size();
    const int64_t no = (int64_t)P.owners.size(), ni = (int64_t)P.items.size();
    for (int64_t o = 0; o < no; ++o) {
        const DOwner& ow = P.owners[o];
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
        int32_t col = 0, tile = 0;
        for (int32_t i = 0; i < ow.nitems; ++i) {
            const DItem& it = P.items[ow.item0 + i];
            const int eb = dtype_bytes(it.dtype);
            if (eb == 0 || it.col0 != col || it.ncols <= 0) { why = "item columns"; return false; }
            if (it.tile0 != tile || it.data_off != P.items[ow.item0].data_off + (int64_t)tile * ow.nrows * 16) {
                why = "owner stream not contiguous";
                return false;
            }
            tile += (int32_t)tile_count(it.dtype, it.ncols);
            const int64_t padded = tile_count(it.dtype, it.ncols) * (16 / eb);
            if (it.data_off < 0 || (it.data_off & 15) ||
                it.data_off + (int64_t)ow.nrows * 16 * tile_count(it.dtype, it.ncols) > nd) {
                why = "item data";
                return false;
            }
            // the last tile's padding columns read inputs/scales past the item
            // (multiplied by zero data); buffers carry TILE_PAD extra entries
            if (it.vec_off < 0 || it.vec_off + padded > P.ws_elems + TILE_PAD) { why = "item input"; return false; }
            if (it.scale_off >= 0 && it.scale_off + padded > nsc + TILE_PAD) { why = "item scales"; return false; }
            col += it.ncols;
        }
    }
    // workspace entries left as partial sums in the single-vector product
    if ((int64_t)P.dsrc.size() != P.ws_elems + TILE_PAD || P.staged.size() != P.tasks.size()) {
        why = "deferred-sum tables";
        return false;
    }
    // an owner is deferred when its first entry is (then all of them are)
    std::vector<int32_t> deferred_owner(P.ws_elems + TILE_PAD, -1);
    std::vector<uint8_t> is_deferred(no, 0);
    for (int64_t o = 0; o < no; ++o) {
        const DOwner& ow = P.owners[o];
        const bool deferred = ow.mode == 0 && ow.ntasks > 1 && P.dsrc[ow.out_off] != 0;
        if (deferred && (ow.ntasks >= (1 << 16) || ow.nrows >= (1 << 15))) { why = "deferred-sum range"; return false; }
        is_deferred[o] = deferred;
        for (int32_t r = 0; r < ow.nrows && ow.mode == 0; ++r) {
            const int64_t d = P.dsrc[ow.out_off + r];
            const int64_t want = deferred ? deferred_sum(ow.part_off + r, ow.ntasks, ow.nrows) : 0;
            if (d != want) { why = "deferred-sum entry"; return false; }
            if (deferred) deferred_owner[ow.out_off + r] = (int32_t)o;
        }
    }
    for (int64_t e = 0; e < P.ws_elems + TILE_PAD; ++e)
        if (P.dsrc[e] != 0 && deferred_owner[e] < 0) { why = "deferred-sum entry without owner"; return false; }
    std::vector<int32_t> seen(no, 0), stage_of(no, -1), reduced(no, -1);
    const int32_t ns = (int32_t)P.stages.size();
    // last stage holding a task of each owner: a coefficient owner may have
    // tasks in several stages (the H2 couplings run before the transfers);
    // its entries are complete only after the last
    std::vector<int32_t> last_of(no, -1);
    for (int32_t si = 0; si < ns; ++si)
        for (int64_t k = P.stages[si].t0; k < P.stages[si].t1 && k < (int64_t)P.tasks.size(); ++k)
            if (P.tasks[k].owner >= 0 && P.tasks[k].owner < no) last_of[P.tasks[k].owner] = si;
    for (int32_t si = 0; si < ns; ++si) {
        const Stage& st = P.stages[si];
        if (st.t0 < 0 || st.t0 > st.t1 || st.t1 > (int64_t)P.tasks.size()) { why = "stage range"; return false; }
        for (int64_t k = st.t0; k < st.t1; ++k) {
            const DTask& t = P.tasks[k];
            if (t.owner < 0 || t.owner >= no) { why = "task owner"; return false; }
            const DOwner& ow = P.owners[t.owner];
            if (t.nrows != ow.nrows || (t.mode & 0xFF) != ow.mode || t.out_off != ow.out_off || t.ntasks != ow.ntasks ||
                t.part_off != ow.part_off || t.rscale_off != ow.rscale_off) {
                why = "task copy of owner fields";
                return false;
            }
            if (t.dtype != (t.c0 < t.c1 ? P.items[t.item_start].dtype : -1)) { why = "task dtype"; return false; }
            int32_t ncols = 0;
            if (ow.nitems) ncols = P.items[ow.item0 + ow.nitems - 1].col0 + P.items[ow.item0 + ow.nitems - 1].ncols;
            if (t.c0 < 0 || t.c0 > t.c1 || t.c1 > ncols || t.local < 0 || t.local >= ow.ntasks) {
                why = "task columns";
                return false;
            }
            int32_t otiles = 0;
            if (ow.nitems) {
                const DItem& last = P.items[ow.item0 + ow.nitems - 1];
                otiles = last.tile0 + (int32_t)tile_count(last.dtype, last.ncols);
            }
            if (t.k0 < 0 || t.k0 > t.k1 || t.k1 > otiles || (t.k0 < t.k1) != (t.c0 < t.c1) ||
                (ow.nitems && t.stream != P.items[ow.item0].data_off)) {
                why = "task tiles";
                return false;
            }
            if (t.c0 < t.c1) {
                if (t.item_start < ow.item0 || t.item_start >= ow.item0 + ow.nitems) { why = "task item"; return false; }
                const DItem& fi = P.items[t.item_start];
                if (t.k0 != fi.tile0 + (t.c0 - fi.col0) / (16 / dtype_bytes(fi.dtype))) { why = "task first tile"; return false; }
                if (((t.mode >> 8) & 15) != fi.ebits || (is_aflp(fi.dtype) && !aflp_feasible(aflp_width(fi.dtype), fi.ebits))) {
                    why = "task AFLP exponent width";
                    return false;
                }
                const DItem& it = P.items[t.item_start];
                if (t.c0 < it.col0 || t.c0 >= it.col0 + it.ncols) { why = "task first item"; return false; }
                if ((t.c0 - it.col0) % (16 / dtype_bytes(it.dtype))) { why = "task not tile aligned"; return false; }
                // one dtype per task; the inputs fit the LDS slice
                for (int32_t j = t.item_start; j < ow.item0 + ow.nitems && P.items[j].col0 < t.c1; ++j)
                    if (P.items[j].dtype != it.dtype || P.items[j].ebits != it.ebits) {
                        why = "task mixes dtypes";
                        return false;
                    }
                if ((int64_t)(t.k1 - t.k0) * (16 / dtype_bytes(it.dtype)) > MAX_TASK_INPUTS) {
                    why = "task inputs exceed LDS slice";
                    return false;
                }
                // inputs that are unreduced sums: the task stages them, and
                // their owner ran in an earlier stage of the dependent chain
                for (int32_t j = t.item_start; j < ow.item0 + ow.nitems && P.items[j].col0 < t.c1; ++j) {
                    const DItem& dj = P.items[j];
                    const int32_t jb = std::max(t.c0 - dj.col0, 0), je = std::min(dj.ncols, t.c1 - dj.col0);
                    for (int32_t c = jb; c < je; ++c) {
                        const int32_t src = deferred_owner[dj.vec_off + c];
                        if (src < 0) continue;
                        if (!P.staged[k]) { why = "unreduced input read without staging"; return false; }
                        if (st.aux || last_of[src] < 0 || last_of[src] >= si) {
                            why = "unreduced input not produced by an earlier stage";
                            return false;
                        }
                    }
                }
            }
            ++seen[t.owner];
            if (ow.mode == 0) {
                if (st.aux && last_of[t.owner] != si) { why = "coefficient owner spans the second stream"; return false; }
                stage_of[t.owner] = si;
            }
        }
        for (int32_t r : st.reduce) {
            if (r < 0 || r >= no || P.owners[r].ntasks < 2 || reduced[r] >= 0) { why = "reduce list"; return false; }
            reduced[r] = si;
            if (P.owners[r].mode == 0 ? stage_of[r] != si : si != ns - 1) { why = "reduce placement"; return false; }
        }
        // the single-vector product launches the reductions of the owners
        // that are not deferred (y owners, coefficient owners of stages with
        // a long owner), in the order of `reduce`
        size_t nl = 0;
        for (int32_t r : st.reduce) nl += !is_deferred[r];
        if (st.reduce_launch.size() != nl) { why = "reduce launch list"; return false; }
        for (size_t i = 0, j = 0; i < st.reduce.size(); ++i)
            if (!is_deferred[st.reduce[i]] && st.reduce_launch[j++] != st.reduce[i]) {
                why = "reduce launch list";
                return false;
            }
    }
    for (int64_t o = 0; o < no; ++o) {
        if (seen[o] != P.owners[o].ntasks) { why = "task count"; return false; }
        if (P.owners[o].ntasks > 1 && reduced[o] < 0) { why = "split owner never reduced"; return false; }
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
        if (!storage_dtype(dt) && !adaptive(dt)) {
            set_error("hm_upload: unsupported dtype");
            return HM_EINVAL;
        }
    const bool valr = adaptive(p->dense_dtype) || adaptive(p->diag_dtype) || adaptive(p->factor_dtype) ||
                      adaptive(p->coupling_dtype);
    if (valr && !(p->eps > 0.0 && std::isfinite(p->eps))) {
        set_error("hm_upload: VALR_AUTO / AFLP_AUTO / FPX_AUTO need eps > 0");
        return HM_EINVAL;
    }
    if (p->accum < HM_ACC_AUTO || p->accum > HM_ACC_F64) {
        set_error("hm_upload: bad accumulation mode");
        return HM_EINVAL;
    }
    Builder B(L, format, v, opt);
    // VALR_AUTO for dense, diagonal and coupling/transfer matrices means
    // direct compression in the cheapest format with unit roundoff <= eps
    // (the diagonal near-field blocks stay FP64)
    auto direct = [&](int32_t dt) { return dt == HM_VALR_AUTO ? direct_for_eps(p->eps) : dt; };
    B.dense_dt = direct(p->dense_dtype);
    B.diag_dt = p->diag_dtype == HM_VALR_AUTO ? HM_F64 : p->diag_dtype;
    B.factor_dt = p->factor_dtype;
    B.coup_dt = direct(p->coupling_dtype);
    B.eps = p->eps;
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
    int64_t per_dtype[HM_NDTYPES] = {};
    int64_t per_class[4] = {0, 0, 0, 0};
    if (!B.fill(out.data, out.scales, per_dtype, per_class)) {
        set_error("hm_upload: " + B.err);
        return HM_EINVAL;
    }
    bool all64 = B.dense_dt == HM_F64 && B.diag_dt == HM_F64 && B.factor_dt == HM_F64 && B.coup_dt == HM_F64;
    if (p->accum == HM_ACC_F64)
        out.acc64 = 1;
    else if (p->accum == HM_ACC_F32)
        out.acc64 = 0;
    else
        out.acc64 = (p->eps < 1e-7 || all64) ? 1 : 0;
    out.format = format;
    out.ws_elems = B.ws;
    out.part_elems = B.part_elems;
    // Water-fill the floating (dense) tasks into the stages, least-loaded
    // stage first, so every launch carries independent work behind its
    // dependent tasks; then lay the stages out as consecutive task ranges.
    {
        const int32_t ns = (int32_t)B.stage_tasks.size();
        if (ns == 0) {
            set_error("hm_upload: empty plan");
            return HM_ELAYOUT;
        }
        std::vector<int64_t> load = B.stage_bytes;
        int32_t dense_stage = -1;
        if (opt.concurrent_dense && !B.floating.empty()) {
            // the dense leaves read only x: one stage of their own, run on a
            // second stream next to the chain of dependent stages
            dense_stage = B.new_stage("dense");
            // by dtype, so that the stage can run as one launch per dtype
            // (aux_split_by_dtype); each owner's tasks keep their order
            std::stable_sort(B.floating.begin(), B.floating.end(),
                             [](const std::pair<DTask, int64_t>& a, const std::pair<DTask, int64_t>& b) {
                                 return a.first.dtype < b.first.dtype;
                             });
            for (auto& tb : B.floating) B.stage_tasks[dense_stage].push_back(tb.first);
        } else {
            for (auto& tb : B.floating) {
                int32_t best = 0;
                for (int32_t si = 1; si < ns; ++si)
                    if (load[si] < load[best]) best = si;
                B.stage_tasks[best].push_back(tb.first);
                load[best] += tb.second;
            }
        }
        const int32_t nst = (int32_t)B.stage_tasks.size();
        out.owners = std::move(B.owners);
        out.items = std::move(B.items);
        out.tasks.clear();
        out.stages.clear();
        for (int32_t si = 0; si < nst; ++si) {
            Stage st;
            st.name = B.stage_names[si];
            st.aux = si == dense_stage;
            st.t0 = (int64_t)out.tasks.size();
            out.tasks.insert(out.tasks.end(), B.stage_tasks[si].begin(), B.stage_tasks[si].end());
            st.t1 = (int64_t)out.tasks.size();
            out.stages.push_back(std::move(st));
        }
        // coefficient owners are reduced right after their stage, y owners at the end
        Stage fin;
        fin.name = "y_reduce";
        fin.t0 = fin.t1 = (int64_t)out.tasks.size();
        std::vector<int32_t> stage_of(out.owners.size(), -1);
        for (int32_t si = 0; si < nst; ++si)
            for (int64_t k = out.stages[si].t0; k < out.stages[si].t1; ++k) stage_of[out.tasks[k].owner] = si;
        for (int32_t o = 0; o < (int32_t)out.owners.size(); ++o) {
            if (out.owners[o].ntasks < 2) continue;
            if (out.owners[o].mode == 0)
                out.stages[stage_of[o]].reduce.push_back(o);
            else
                fin.reduce.push_back(o);
        }
        if (!fin.reduce.empty()) out.stages.push_back(std::move(fin));
        // Single-vector product: the split coefficient owners of a stage get
        // no reduction launch when none of them has more than
        // kMaxDeferredTasks tasks; each later task reading one of their
        // outputs adds the partial sums (in task order) while it stages its
        // inputs.  A stage with a longer owner keeps its launch (every
        // consumer re-adding hundreds of partials costs more than one
        // launch).  The reductions of y owners stay (the final stage).
        constexpr int32_t kMaxDeferredTasks = 16;
        out.dsrc.assign(out.ws_elems + TILE_PAD, 0);
        for (auto& st : out.stages) {
            int32_t longest = 0;
            for (int32_t o : st.reduce)
                if (out.owners[o].mode == 0) longest = std::max(longest, out.owners[o].ntasks);
            const bool defer = longest <= kMaxDeferredTasks;
            for (int32_t o : st.reduce) {
                const DOwner& ow = out.owners[o];
                if (ow.mode == 0 && defer)
                    for (int32_t r = 0; r < ow.nrows; ++r)
                        out.dsrc[ow.out_off + r] = deferred_sum(ow.part_off + r, ow.ntasks, ow.nrows);
                else
                    st.reduce_launch.push_back(o);
            }
        }
        {
            std::vector<int64_t> cnt(out.dsrc.size() + 1, 0);   // prefix count of deferred entries
            for (size_t e = 0; e < out.dsrc.size(); ++e) cnt[e + 1] = cnt[e] + (out.dsrc[e] != 0);
            out.staged.assign(out.tasks.size(), 0);
            for (size_t k = 0; k < out.tasks.size(); ++k) {
                const DTask& t = out.tasks[k];
                int32_t c = t.c0;
                for (int32_t it = t.item_start; c < t.c1; ++it) {
                    const DItem& item = out.items[it];
                    const int32_t jb = c - item.col0, je = std::min(item.ncols, t.c1 - item.col0);
                    if (cnt[item.vec_off + je] > cnt[item.vec_off + jb]) out.staged[k] = 1;
                    c = item.col0 + je;
                }
            }
        }
        for (auto& st : out.stages) {
            for (int64_t k = st.t0; k < st.t1; ++k) {
                const DTask& t = out.tasks[k];
                const DOwner& ow = out.owners[t.owner];
                // tiles of the task's column range
                int32_t c = t.c0;
                for (int32_t it = t.item_start; c < t.c1; ++it) {
                    const DItem& item = out.items[it];
                    const int V = tile_cols(item.dtype);
                    const int32_t jb = c - item.col0, je = std::min(item.ncols, t.c1 - item.col0);
                    st.data_bytes += (int64_t)((je + V - 1) / V - jb / V) * ow.nrows * 16;
                    st.data_entries += (int64_t)((je + V - 1) / V - jb / V) * ow.nrows * V;
                    st.method_bytes += (double)(je - jb) * ow.nrows * dtype_bytes(item.dtype);
                    st.dtype_mask |= 1 << item.dtype;
                    c = item.col0 + je;
                }
                const double outb = 8.0 * ow.nrows * (t.ntasks > 1 ? 1 : (ow.mode == 0 ? 2 : 3));
                st.alg_bytes += outb + sizeof(DTask);
                st.method_bytes += outb;
            }
            for (int32_t o : st.reduce) {
                const DOwner& ow = out.owners[o];
                st.alg_bytes += 8.0 * ow.nrows * (ow.ntasks + (ow.mode == 0 ? 2 : 3));
                st.method_bytes += 8.0 * ow.nrows * (ow.ntasks + (ow.mode == 0 ? 2 : 3));
            }
            st.alg_bytes += (double)st.data_bytes;
        }
    }
    hm_stats& s = out.stats;
    s = hm_stats{};
    s.n = L.n;
    s.nblocks = (int64_t)L.blk_tau.size();
    for (size_t b = 0; b < L.blk_tau.size(); ++b) (L.blk_adm[b] ? s.nlowrank : s.ndense)++;
    s.bytes_dense = per_class[0];
    s.bytes_factors = per_class[1];
    s.bytes_coupling = per_class[2];
    s.bytes_transfer = per_class[3];
    for (int d = 0; d < HM_NDTYPES; ++d) s.bytes_per_dtype[d] = per_dtype[d];
    s.bytes_scales = (int64_t)out.scales.size() * 8;
    int64_t meta = (int64_t)(out.owners.size() * sizeof(DOwner) + out.items.size() * sizeof(DItem) +
                             out.tasks.size() * sizeof(DTask));
    for (auto& st : out.stages) meta += (int64_t)st.reduce.size() * 4;
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
    for (const Source& S : B.src) s.entries_per_dtype[S.dtype] += S.m * S.k;
    s.nowners = (int64_t)out.owners.size();
    s.nitems = (int64_t)out.items.size();
    s.ntasks = (int64_t)out.tasks.size();
    s.nlaunch = 1;   // gather
    for (auto& st : out.stages) {
        s.nlaunch += (st.t1 > st.t0) + !st.reduce_launch.empty();
        if (st.aux && st.t1 > st.t0 && aux_split_by_dtype(st.dtype_mask))
            s.nlaunch += __builtin_popcount(st.dtype_mask) - 1;   // one launch per dtype
    }
    s.algorithmic_bytes = (double)(s.bytes_dense + s.bytes_factors + s.bytes_coupling + s.bytes_transfer +
                                   s.bytes_scales + s.bytes_meta) +
                          24.0 * L.n + 16.0 * (out.ws_elems - L.n);
    // the method's own bytes: every stored entry once at its element size, a
    // float32 scale per range-scaled column, x read, y read and written, and
    // every coefficient entry written and read once (float64)
    s.method_bytes = 24.0 * L.n + 16.0 * (out.ws_elems - L.n);
    for (const Source& S : B.src)
        s.method_bytes += (double)S.m * S.k * dtype_bytes(S.dtype) + (range_scaled(S.dtype) ? 4.0 * S.k : 0.0);
    std::string why;
    if (!validate(out, L.n, why)) {
        set_error("hm_upload: internal plan check failed (" + why + ")");
        return HM_ELAYOUT;
    }
    return HM_OK;
}

void build_mr_plan(const std::vector<DOwner>& owners, const std::vector<DItem>& items,
                   const std::vector<DTask>& tasks, const std::vector<Stage>& stages, int64_t target_bytes,
                   MrPlan& out) {
    out = MrPlan{};
    out.target_bytes = target_bytes;
    out.owners = owners;
    struct Chunk {
        DTask t;         // owner fields, c0/c1, item_start, k0/k1, stream
        int32_t stage;
    };
    std::vector<Chunk> chunks;
    std::vector<int32_t> nchunk(owners.size(), 0), last_stage(owners.size(), -1);
    const int32_t nst = (int32_t)stages.size();
    for (int32_t si = 0; si < nst; ++si) {
        const Stage& st = stages[si];
        int64_t acc = 0;
        for (int64_t k = st.t0; k < st.t1; ++k) {
            const DTask& t = tasks[k];
            const DOwner& ow = owners[t.owner];
            const int32_t dt = t.c0 < t.c1 ? items[t.item_start].dtype : -1;
            const int64_t bytes = (int64_t)(t.k1 - t.k0) * std::min(ow.nrows, 64) * 16;
            bool merge = false;
            if (!chunks.empty()) {
                const Chunk& c = chunks.back();
                const int32_t cdt = c.t.c0 < c.t.c1 ? items[c.t.item_start].dtype : -1;
                // one dtype and one AFLP exponent width (mode bits 8-11) per task
                merge = c.stage == si && c.t.owner == t.owner && c.t.c1 == t.c0 && cdt == dt && dt >= 0 &&
                        c.t.mode == t.mode && c.t.k1 == t.k0 && acc + bytes <= target_bytes;
            }
            if (merge) {
                chunks.back().t.c1 = t.c1;
                chunks.back().t.k1 = t.k1;
                acc += bytes;
            } else {
                chunks.push_back(Chunk{t, si});
                chunks.back().t.local = nchunk[t.owner]++;
                acc = bytes;
            }
            last_stage[t.owner] = std::max(last_stage[t.owner], si);
        }
    }
    for (size_t o = 0; o < owners.size(); ++o) {
        DOwner& ow = out.owners[o];
        ow.ntasks = std::max(nchunk[o], 1);
        ow.part_off = 0;
        if (ow.ntasks > 1) {
            ow.part_off = (int32_t)out.part_elems;
            out.part_elems += (int64_t)ow.ntasks * ow.nrows;
        }
    }
    // stages: the task stages of the plan (its final reduce-only stage is rebuilt)
    for (int32_t si = 0; si < nst; ++si) {
        const Stage& src = stages[si];
        if (src.t0 == src.t1 && !src.reduce.empty() && si == nst - 1) break;
        Stage st;
        st.name = src.name;
        st.aux = src.aux;
        st.t0 = (int64_t)out.tasks.size();
        for (const Chunk& c : chunks) {
            if (c.stage != si) continue;
            const DOwner& ow = out.owners[c.t.owner];
            for (int32_t r0 = 0; r0 < ow.nrows; r0 += 64) {
                DTask t = c.t;
                t.ntasks = ow.ntasks;
                t.part_off = ow.part_off;
                t.pad = r0;
                out.tasks.push_back(t);
                st.data_bytes += (int64_t)(t.k1 - t.k0) * std::min(64, ow.nrows - r0) * 16;
                if (t.c0 < t.c1)
                    st.data_entries += (int64_t)(t.k1 - t.k0) * std::min(64, ow.nrows - r0) *
                                       tile_cols(items[t.item_start].dtype);
            }
        }
        st.t1 = (int64_t)out.tasks.size();
        out.stages.push_back(std::move(st));
    }
    Stage fin;
    fin.name = "y_reduce";
    fin.t0 = fin.t1 = (int64_t)out.tasks.size();
    for (int32_t o = 0; o < (int32_t)owners.size(); ++o) {
        const DOwner& ow = out.owners[o];
        if (ow.ntasks < 2) continue;
        if (ow.mode == 0)
            out.stages[last_stage[o]].reduce.push_back(o);
        else
            fin.reduce.push_back(o);
    }
    if (!fin.reduce.empty()) out.stages.push_back(std::move(fin));
}

}  // namespace hm

namespace hm {

hm_status pack_options(const hm_upload_opts* o, PackOptions& opt) {
    opt = PackOptions{};
    if (!o) return HM_OK;
    if ((o->task_bytes != 0 && o->task_bytes < 1024) || (o->chain_task_bytes != 0 && o->chain_task_bytes < 1024)) {
        set_error("hm_upload: task_bytes and chain_task_bytes must be 0 (default) or at least 1024");
        return HM_EINVAL;
    }
    if (o->dense_grid < 0 || o->fork_after < 0 || (o->spread_dense & ~1) || (o->valr_promote & ~1) ||
        o->dense_after < 0 || o->spin_limit_us < 0 ||
        (o->schedule != HM_SCHED_PERSISTENT && o->schedule != HM_SCHED_STAGED)) {
        set_error("hm_upload: negative dense_grid / fork_after / dense_after / spin_limit_us, a flag other "
                  "than 0 / 1, or an unknown schedule");
        return HM_EINVAL;
    }
    if (o->tickets_per_grab < 0 || o->tickets_per_grab > 256) {
        set_error("hm_upload: tickets_per_grab must be in [0, 256]");
        return HM_EINVAL;
    }
    if (o->tickets_per_grab) opt.tickets_per_grab = o->tickets_per_grab;
    if (o->adjoint & ~1) {
        set_error("hm_upload: adjoint must be 0 or 1");
        return HM_EINVAL;
    }
    opt.adjoint = o->adjoint != 0;
    if (o->sync < HM_SYNC_OWNER || o->sync > HM_SYNC_PRIVATE ||
        (o->sync != HM_SYNC_OWNER && o->schedule == HM_SCHED_PERSISTENT)) {
        set_error("hm_upload: sync must be HM_SYNC_OWNER, HM_SYNC_ATOMIC or HM_SYNC_PRIVATE (the last two with "
                  "the staged schedule)");
        return HM_EINVAL;
    }
    opt.sync = o->sync;
    opt.schedule = o->schedule;
    opt.dense_after = o->dense_after;
    if (o->spin_limit_us) opt.spin_limit_us = o->spin_limit_us;
    if (o->task_bytes) opt.task_bytes = o->task_bytes;
    if (o->chain_task_bytes) opt.chain_task_bytes = o->chain_task_bytes;
    opt.concurrent_dense = o->spread_dense == 0;
    opt.valr_promote = o->valr_promote != 0;
    if (o->h2_levels & ~1) {
        set_error("hm_upload: h2_levels must be 0 or 1");
        return HM_EINVAL;
    }
    opt.coupling_first = o->h2_levels == 0;
    return HM_OK;
}

}  // namespace hm

extern "C" hm_status hm_plan_stats(const hm_layout* layout, int32_t format, const hm_values* values,
                                   const hm_precision* prec, const hm_upload_opts* opts, hm_stats* out) {
    if (!layout || !values || !prec || !out) {
        hm::set_error("hm_plan_stats: null argument");
        return HM_EINVAL;
    }
    hm::Packed P;
    hm::PackOptions opt;
    hm_status st = hm::pack_options(opts, opt);
    if (st != HM_OK) return st;
    try {
        st = hm::pack(layout->L, format, values, prec, opt, P);
        if (st == HM_OK && opt.schedule == HM_SCHED_PERSISTENT) {
            // the persistent queue is built and its progress rule checked as in hm_upload
            hm::Queue Q;
            std::vector<int32_t> order;
            st = hm::build_queue(P, layout->L.n, Q);
            if (st == HM_OK) st = hm::queue_order(P.owners, Q.tasks, Q, opt.dense_after, order);
            if (st == HM_OK) P.stats.nlaunch = 2;   // gather + the persistent launch
        }
    } catch (const std::bad_alloc&) {
        hm::set_error("hm_plan_stats: out of host memory while packing");
        return HM_ENOMEM;
    }
    if (st == HM_OK) *out = P.stats;
    return st;
}
