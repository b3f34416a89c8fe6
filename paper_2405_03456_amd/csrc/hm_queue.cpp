// Persistent schedule of the single-vector product: every task of the plan
// and every reduction of a split owner in one ticket queue, run by one
// launch (k_persistent).
//
// The order is a topological order of the product's data flow (Sec. 3: the
// forward transforms or upward pass before the couplings that read their
// coefficients, the downward pass level by level, the leaf rows last), taken
// from the stage order of the plan; the dense near-field tasks, which read
// only x, are spread between the dependent stages.  Instead of waiting for a
// whole stage, an item waits only for the owners whose outputs it reads:
//   - task k reads the coefficient entries of its columns; each entry was
//     written by one coefficient owner, which is complete once its counter
//     reaches target[o] (its tasks, plus its reduction if it has one);
//   - the reduction of owner o waits for the owner's own tasks.
// Every producer precedes its consumers in the queue, so a wave only ever
// waits for items with smaller tickets, which are held by running waves:
// the smallest unfinished ticket never waits, and the queue always drains.
#include <algorithm>
#include <string>
#include <vector>

#include "hm_pack.h"

namespace hm {

hm_status build_queue(const Packed& P, int64_t n, Queue& q) {
    q = Queue{};
    const int64_t no = (int64_t)P.owners.size(), nt = (int64_t)P.tasks.size();
    const int64_t nws = P.ws_elems + TILE_PAD;
    // producer owner of every workspace entry (x entries: none)
    std::vector<int32_t> prod((size_t)nws, -1);
    for (int64_t o = 0; o < no; ++o) {
        const DOwner& ow = P.owners[o];
        if (ow.mode != 0) continue;
        for (int32_t r = 0; r < ow.nrows; ++r) prod[(size_t)(ow.out_off + r)] = (int32_t)o;
    }
    std::vector<uint8_t> has_reduce((size_t)no, 0);
    for (const Stage& st : P.stages)
        for (int32_t o : st.reduce_launch) has_reduce[(size_t)o] = 1;
    q.target.resize((size_t)no);
    for (int64_t o = 0; o < no; ++o) q.target[(size_t)o] = P.owners[o].ntasks + has_reduce[(size_t)o];
    // dependencies of every task: the producers of the entries its columns read
    // (the zero-data padding columns of a last tile multiply whatever finite
    // value they read and need no producer)
    q.tasks = P.tasks;
    q.dep_first.assign((size_t)nt + 1, 0);
    std::vector<int32_t> tmp;
    for (int64_t k = 0; k < nt; ++k) {
        DTask& t = q.tasks[(size_t)k];
        const DOwner& ow = P.owners[t.owner];
        tmp.clear();
        int32_t c = t.c0;
        for (int32_t it = t.item_start; c < t.c1 && it < ow.item0 + ow.nitems; ++it) {
            const DItem& item = P.items[it];
            const int32_t jb = c - item.col0, je = std::min(item.ncols, t.c1 - item.col0);
            for (int32_t j = jb; j < je; ++j) {
                const int32_t p = prod[(size_t)(item.vec_off + j)];
                if (p >= 0) tmp.push_back(p);
            }
            c = item.col0 + je;
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        // a task that reads coefficients produced in the same launch stages
        // its inputs (coherent loads into LDS): mode bit 2
        if (!tmp.empty() || P.staged[(size_t)k]) t.mode = (int16_t)(t.mode | 4);
        q.deps.insert(q.deps.end(), tmp.begin(), tmp.end());
        q.dep_first[(size_t)k + 1] = (int32_t)q.deps.size();
        if (t.c0 < t.c1) q.dtype_mask |= 1 << t.dtype;
    }
    // chain stages in plan order, the dense tasks aside, the final reductions last
    for (const Stage& st : P.stages) {
        if (st.aux) {
            for (int64_t k = st.t0; k < st.t1; ++k) q.dense.push_back((int32_t)k);
            continue;
        }
        if (st.t1 == st.t0 && &st == &P.stages.back()) {
            for (int32_t o : st.reduce_launch) q.final_reduce.push_back(~o);
            continue;
        }
        std::vector<int32_t> part;
        for (int64_t k = st.t0; k < st.t1; ++k) part.push_back((int32_t)k);
        for (int32_t o : st.reduce_launch) part.push_back(~o);
        q.chain.push_back(std::move(part));
    }
    q.nchain = (int32_t)q.chain.size();
    (void)n;
    return HM_OK;
}

hm_status queue_order(const std::vector<DOwner>& owners, const std::vector<DTask>& tasks, const Queue& q,
                      int32_t dense_after, std::vector<int32_t>& order) {
    order.clear();
    const int32_t nc = q.nchain;
    const int32_t first = std::min(std::max(dense_after, 0), nc);   // positions first .. nc
    const int64_t nd = (int64_t)q.dense.size();
    const int64_t npos = nc - first + 1;
    int64_t di = 0;
    auto dense_until = [&](int32_t pos) {   // dense tasks due at boundary position pos
        const int64_t want = pos < first ? 0 : nd * (pos - first + 1) / npos;
        while (di < want) order.push_back(q.dense[(size_t)di++]);
    };
    for (int32_t s = 0; s < nc; ++s) {
        dense_until(s);
        order.insert(order.end(), q.chain[(size_t)s].begin(), q.chain[(size_t)s].end());
    }
    dense_until(nc);
    order.insert(order.end(), q.final_reduce.begin(), q.final_reduce.end());
    // progress check: every item's producers (and a reduction's own tasks)
    // come before it
    const int64_t no = (int64_t)owners.size();
    std::vector<int32_t> left((size_t)no);
    for (int64_t o = 0; o < no; ++o) left[(size_t)o] = q.target[(size_t)o];
    std::vector<int32_t> tasks_left((size_t)no);
    for (int64_t o = 0; o < no; ++o) tasks_left[(size_t)o] = owners[o].ntasks;
    size_t ntask_items = 0, nred = 0;
    for (int32_t it : order) {
        if (it >= 0) {
            for (int32_t d = q.dep_first[(size_t)it]; d < q.dep_first[(size_t)it + 1]; ++d)
                if (left[(size_t)q.deps[(size_t)d]] != 0) {
                    set_error("hm_upload: persistent queue: a task precedes one of its producers");
                    return HM_ELAYOUT;
                }
            const int32_t o = tasks[(size_t)it].owner;
            left[(size_t)o]--;
            tasks_left[(size_t)o]--;
            ++ntask_items;
        } else {
            const int32_t o = ~it;
            if (tasks_left[(size_t)o] != 0) {
                set_error("hm_upload: persistent queue: a reduction precedes its owner's tasks");
                return HM_ELAYOUT;
            }
            left[(size_t)o]--;
            ++nred;
        }
    }
    for (int64_t o = 0; o < no; ++o)
        if (left[(size_t)o] != 0) {
            set_error("hm_upload: persistent queue: owner " + std::to_string(o) + " (mode " +
                      std::to_string(owners[o].mode) + ", " + std::to_string(owners[o].ntasks) +
                      " tasks) is not complete at the end (" + std::to_string(left[(size_t)o]) + " left, " +
                      std::to_string(tasks_left[(size_t)o]) + " tasks left)");
            return HM_ELAYOUT;
        }
    if (ntask_items != tasks.size()) {
        set_error("hm_upload: persistent queue: task count");
        return HM_ELAYOUT;
    }
    (void)nred;
    return HM_OK;
}

}  // namespace hm
