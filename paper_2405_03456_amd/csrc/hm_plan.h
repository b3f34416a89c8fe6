// Packed execution plan of one uploaded matrix: the device tables read by
// the kernels and the host-side description of the launch sequence.
//
// Every phase of every format is the same operation: a set of *owners*, each
// owning `nrows` consecutive outputs, computes
//     out[r] = rscale[r] * sum_items sum_j A_item[r, j] * (w[vec + j] * cscale[j])
// where A_item is a column-major slab (column stride = nrows) stored in one
// dtype.  The columns of an owner are cut into *tasks* of bounded size; one
// wavefront runs one task with one lane per output row.  Owners with one
// task write their result directly, the others leave per-task partial sums
// that a reduce pass adds in task order (deterministic, no atomics).
//
// Output modes: 0 = coefficient vector (ws[out + r] = v), 1 = y in original
// order (y[perm[out + r]] += alpha*v), 2 = y in cluster order.
#pragma once

#include <cstdint>
#include <vector>

namespace hm {

struct DItem {            // 32 bytes
    int64_t data_off;     // byte offset of element (0,0) in the data arena
    int32_t col0;         // first column within the owner's column range
    int32_t ncols;
    int32_t vec_off;      // workspace index of the input for column 0
    int32_t scale_off;    // index of column 0's scale, -1 = none
    int16_t dtype;
    int16_t acc64;        // accumulate in float64 even in float32 mode
    int32_t pad;
};

struct DOwner {           // 32 bytes
    int32_t nrows;
    int32_t item0;
    int32_t nitems;
    int32_t out_off;
    int32_t mode;
    int32_t ntasks;
    int32_t part_off;     // partial sums: part[part_off + local * nrows + r]
    int32_t rscale_off;   // per-row output scale, -1 = none
};

struct DTask {            // 32 bytes
    int32_t owner;
    int32_t c0, c1;       // owner columns [c0, c1)
    int32_t item_start;   // absolute index of the item holding column c0
    int32_t local;        // task index within its owner
    int32_t pad[3];
};

static_assert(sizeof(DItem) == 32, "DItem layout");
static_assert(sizeof(DOwner) == 32, "DOwner layout");
static_assert(sizeof(DTask) == 32, "DTask layout");

struct Phase {
    // host copies
    std::vector<DOwner> owners;
    std::vector<DItem> items;
    std::vector<DTask> tasks;
    std::vector<int32_t> reduce_owners;   // owners with ntasks > 1
    int64_t part_elems = 0;
    int32_t max_rows = 0;
    int64_t data_bytes = 0;               // matrix bytes this phase streams
    // device offsets (bytes) inside the metadata buffer
    int64_t d_owners = 0, d_items = 0, d_tasks = 0, d_reduce = 0;
    const char* name = "";
};

}  // namespace hm
