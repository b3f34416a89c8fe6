// Host packing of an H / UH / H2 matrix into the execution plan.
#pragma once

#include "hm_internal.h"
#include "hm_plan.h"

namespace hm {

struct PackOptions {
    int64_t task_bytes = 0;       // target matrix bytes per task (one wavefront); 0 = by format
    int64_t chain_task_bytes = 0; // ... of the dependent stages' tasks (0 = task_bytes, else by format and size)
    bool concurrent_dense = true; // dense leaves as one independent stage (else spread over the stages)
    bool valr_promote = false;    // VALR: fill the 16-byte tiles of short format runs (see valr_formats)
    int32_t schedule = HM_SCHED_STAGED;
    int32_t dense_after = 0;      // persistent schedule: interleave point of the dense tasks
    int64_t spin_limit_us = 2000000;
    int32_t tickets_per_grab = 4;
    bool adjoint = false;         // also upload M^T for HM_ADJOINT products
    int32_t sync = HM_SYNC_OWNER; // how tasks sharing output rows combine them
    bool coupling_first = true;   // H2: every level's couplings in one launch after the up pass
};

// Validated PackOptions from the ABI's hm_upload_opts (NULL = defaults).
hm_status pack_options(const hm_upload_opts* o, PackOptions& opt);

struct Packed {
    int32_t format = 0;
    int32_t acc64 = 1;
    std::vector<DOwner> owners;
    std::vector<DItem> items;
    std::vector<DTask> tasks;      // stage after stage
    std::vector<Stage> stages;
    std::vector<uint8_t> data;     // quantised matrix data, column-major slabs
    std::vector<double> scales;    // per-column / per-row scales
    int64_t ws_elems = 0;          // x in cluster order + coefficient vectors
    int64_t part_elems = 0;        // partial sums, one region per split owner
    // Single-vector product only: per workspace entry (ws_elems + TILE_PAD),
    // 0 = read the workspace, else deferred_sum(...) of the partial sums
    // that make up the entry; per task, 1 = stage the inputs through it.
    std::vector<int64_t> dsrc;
    std::vector<uint8_t> staged;
    hm_stats stats{};
};

hm_status pack(const Layout& L, int32_t format, const hm_values* v, const hm_precision* p,
               const PackOptions& opt, Packed& out);

// Persistent schedule of the single-vector product (hm_queue.cpp): the
// plan's tasks and split-owner reductions as one ticket queue.  A queue
// entry e >= 0 is task e, e < 0 the reduction of owner ~e.
struct Queue {
    std::vector<DTask> tasks;          // the plan's tasks; mode bit 2 set where inputs are staged
    std::vector<int32_t> dep_first;    // per task: its producer owners are deps[dep_first[k] .. dep_first[k+1])
    std::vector<int32_t> deps;
    std::vector<int32_t> target;       // per owner: completion count once its outputs are final
    std::vector<std::vector<int32_t>> chain;   // queue entries of each dependent stage, in order
    std::vector<int32_t> dense;        // the independent (near-field) tasks
    std::vector<int32_t> final_reduce; // queue entries (~owner) of the reductions after everything
    int32_t nchain = 0;
    int32_t dtype_mask = 0;
};

hm_status build_queue(const Packed& P, int64_t n, Queue& q);

// The queue order with the dense tasks spread evenly over the boundaries
// between the dependent stages from boundary `dense_after` on (0 = before the
// first stage); checks that every item follows its producers.
hm_status queue_order(const std::vector<DOwner>& owners, const std::vector<DTask>& tasks, const Queue& q,
                      int32_t dense_after, std::vector<int32_t>& order);

// The adjoint M^T as a matrix of the same form over the transposed block
// tree (hm_adjoint.cpp): the layout with every block (t, s) turned into
// (s, t), and a value set whose pointers refer to the caller's arrays or to
// transposed copies held here.
struct Transposed {
    hm_layout layout;
    std::vector<std::vector<double>> store;
    std::vector<const double*> dense, coupling;
    hm_values v{};
};

hm_status transpose_matrix(const Layout& L, int32_t format, const hm_values* v, Transposed& T);

// Task table of the many-right-hand-side engine, derived from a packed plan.
// Consecutive tasks of one owner in one stage (same dtype, adjacent
// columns) are merged into column chunks of about `target_bytes` per 64-row
// group, and every chunk is split into row groups of at most 64 rows
// (DTask::pad = first row).  Owners split over several chunks get partial
// sums (ntasks / part_off of `owners`); coefficient owners are reduced after
// their stage, y owners in a final reduce stage.
struct MrPlan {
    std::vector<DTask> tasks;
    std::vector<DOwner> owners;
    std::vector<Stage> stages;
    int64_t part_elems = 0;
    int64_t target_bytes = 0;
};

void build_mr_plan(const std::vector<DOwner>& owners, const std::vector<DItem>& items,
                   const std::vector<DTask>& tasks, const std::vector<Stage>& stages, int64_t target_bytes,
                   MrPlan& out);

}  // namespace hm
