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
// that are added in task order (deterministic, no atomics): by a reduce pass
// for y owners, and for coefficient owners of the single-vector product by
// every later task that reads them (see deferred_sum).
//
// Output modes: 0 = coefficient vector (ws[out + r] = v), 1 = y in original
// order (y[perm[out + r]] += alpha*v), 2 = y in cluster order.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hm.h"

namespace hm {

struct DItem {            // 32 bytes
    int64_t data_off;     // byte offset of element (0,0) in the data arena
    int32_t col0;         // first column within the owner's column range
    int32_t ncols;
    int32_t vec_off;      // workspace index of the input for column 0
    int32_t scale_off;    // index of column 0's scale, -1 = none
    int16_t dtype;
    int16_t ebits;        // AFLP exponent width of the item's source (0 for other formats)
    int32_t tile0;        // first tile within the owner's tile stream
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

// The items of one owner are stored back to back and share its row count,
// so the owner's data is one stream of tiles of nrows*16 bytes; a task is
// the tile range [k0, k1) of that stream (columns [c0, c1)).
struct DTask {            // 64 bytes; carries its owner's fields so a wave
    int32_t owner;        // starts streaming after one descriptor load
    int32_t c0, c1;       // owner columns [c0, c1)
    int32_t item_start;   // absolute index of the item holding column c0
    int32_t local;        // task index within its owner
    int32_t nrows;
    int16_t mode;         // bits 0-1 output mode, 2 staged inputs, 3 atomic, 4 private y;
                          // bits 8-11 the AFLP exponent width of its items
    int16_t dtype;        // dtype of every item the task touches (-1: no columns)
    int32_t out_off, ntasks, part_off, rscale_off;
    int32_t k0, k1;       // owner tiles [k0, k1)
    int32_t pad;          // many-RHS plan: first row of the task's 64-row group
    int64_t stream;       // byte offset of the owner's tile 0 in the data arena
};

// Input vectors and scale arrays carry this many trailing entries so that
// the zero-padded columns of a last tile read in-bounds finite values.
constexpr int64_t TILE_PAD = 16;

// Owners with at most 32 rows stage a task's inputs in LDS; a task of such
// an owner reads at most this many input values (tiles * columns per tile).
constexpr int64_t MAX_TASK_INPUTS = 1024;

static_assert(sizeof(DItem) == 32, "DItem layout");
static_assert(sizeof(DOwner) == 32, "DOwner layout");
static_assert(sizeof(DTask) == 64, "DTask layout");

// One kernel launch of the product: tasks [t0, t1) of the global task table
// (all mutually independent), followed by the reduction of the split owners
// in `reduce` (owners whose every task ran in this or an earlier stage).
struct Stage {
    std::string name;
    int64_t t0 = 0, t1 = 0;
    std::vector<int32_t> reduce;
    int64_t data_bytes = 0;      // matrix bytes streamed by its tasks
    int64_t data_entries = 0;    // matrix entries streamed (tile padding included)
    double alg_bytes = 0;        // data + partial/output writes
    double method_bytes = 0;     // the same without tile padding and task descriptors
    int32_t dtype_mask = 0;      // dtypes of the items its tasks touch
    bool aux = false;            // independent of the other stages: runs on a second stream
    std::vector<int32_t> reduce_launch;   // the owners of `reduce` the single-vector product
                                          // reduces with a launch (y owners)
};

// The second-stream stage (the dense near field, independent tasks) runs as
// one launch per dtype when its tasks hold more than one codec: each launch
// then takes the task kernel compiled for that codec alone (fewer registers,
// more waves per SIMD than the kernel of the whole codec family).  Its tasks
// are sorted by dtype for that; results do not depend on the order.
inline bool aux_split_by_dtype(int32_t mask) {
    const int32_t codecs = mask >> HM_FPX24;
    return codecs != 0 && __builtin_popcount(mask & ~1) > 1;
}

// A workspace entry that the single-vector product leaves as the partial
// sums of its split owner: value = sum over l < count of part[base + l * stride],
// packed as base | count << 32 | stride << 48 (base < 2^32, count and stride < 2^16).
inline int64_t deferred_sum(int64_t base, int64_t count, int64_t stride) {
    return base | (count << 32) | (stride << 48);
}

}  // namespace hm
