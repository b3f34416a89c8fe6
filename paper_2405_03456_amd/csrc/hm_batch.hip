// Many right-hand sides: Y += alpha * M * X for R columns at once.
//
// The plan is the one of the single-vector product (owners, items, tasks,
// stages); only the inner operation changes.  With R columns a task is the
// dense contraction C[nrows x R] = A[nrows x K] * B[K x R], where A is the
// task's stored slab and B holds the inputs of its K columns (times their
// column scales).  It runs on the matrix cores with the 16x16x4 MFMA
// (float32, or float64 when the matrix accumulates in float64):
//
//   * lane l = 16*kq + rl loads the 16-byte tile row `rl` of tile kb + kq,
//     so one wave load brings in 4 tiles of 16 rows (1 KiB);
//   * element c of that tile row is the A operand A[rl][kq] of MFMA #c, the
//     matching input value W[col(kb + kq, c)][j0 + NRB*rl + b] the B operand
//     of right-hand-side block b, so the V MFMAs of a load step cover all
//     4*V columns of the 4 tiles;
//   * each wave owns up to 64 rows (4 row groups) and 16*NRB right-hand
//     sides, and keeps 4*NRB accumulator tiles in registers.  Output column
//     rl of block b is right-hand side j0 + NRB*rl + b: the NRB values one
//     lane needs are adjacent and come in one load.
//
// Vectors live in entry-major workspaces (value j of entry i at i*R + j), so
// the B operands of 16 lanes are 16*NRB consecutive values.  The input X is
// gathered into cluster order and the output accumulated into a cluster-
// order buffer; both are transposed through LDS to and from the caller's
// column-major X and Y.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "hm_device.h"

namespace hm {
namespace mr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t word(const uint4& q, int i) {
    return i == 0 ? q.x : i == 1 ? q.y : i == 2 ? q.z : q.w;
}

// element c (compile-time after unrolling) of a tile row, widened to T
// (e: the task's AFLP exponent width)
template <int DT, typename T>
__device__ __forceinline__ T elem(const uint4& q, int c, int e) {
    if constexpr (DT >= HM_FPX24) {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
        return (T)dev::Tile<DT>::elem(w, c, e);
    } else if constexpr (DT == HM_F64) {
        return (T)(c == 0 ? __hiloint2double((int)q.y, (int)q.x) : __hiloint2double((int)q.w, (int)q.z));
    } else if constexpr (DT == HM_F32) {
        return (T)__uint_as_float(word(q, c));
    } else if constexpr (DT == HM_BF16) {
        const uint32_t w = word(q, c >> 1);
        return (T)__uint_as_float((c & 1) ? (w & 0xffff0000u) : (w << 16));
    } else if constexpr (DT == HM_F16) {
        const uint32_t w = word(q, c >> 1);
        return (T)dev::f16_to_f32((uint16_t)((c & 1) ? (w >> 16) : (w & 0xffffu)));
    } else {
        return (T)dev::fp8_to_f32((uint8_t)(word(q, c >> 2) >> (8 * (c & 3))));
    }
}

// A[i][k] comes from lane i + 16k, B[k][j] from lane j + 16k.  Result
// element v of lane l = 16q + j is C[row(q, v)][j]: the float32 form holds
// four consecutive rows per lane, the float64 form every fourth row.
template <bool ACC64> struct Mfma;
template <> struct Mfma<false> {
    using T = float;
    using V = f32x4;
    __device__ static V step(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int q, int v) { return 4 * q + v; }
};
template <> struct Mfma<true> {
    using T = double;
    using V = f64x4;
    __device__ static V step(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int q, int v) { return q + 4 * v; }
};

struct ItemPos {
    int it, k0, k1, vec, sc, nc;
};

template <int V>
__device__ __forceinline__ ItemPos item_pos(const DItem* __restrict__ items, int it) {
    const DItem d = items[it];
    return ItemPos{it, d.tile0, d.tile0 + (d.ncols + V - 1) / V, d.vec_off, d.scale_off, d.ncols};
}

// Coefficient vectors (mode-0 outputs) are kept in one precision only: float64
// (wsm) when the matrix accumulates in float64, else float32 (wsm32).  Only
// the gathered x (entries below n) is held in both.
struct Outs {
    double* wsm;        // float64 entries, entry-major
    float* wsm32;       // float32 entries
    double* ym;         // y outputs (modes 1, 2) in cluster order, entry-major
    double* partm;      // partial sums of split owners
    const double* scales;
    int R;
    int64_t n;          // entries below n hold x (both precisions)
    bool mat64;         // the matrix accumulates in float64
};

__device__ __forceinline__ void put(const DTask& tk, const Outs& o, int row, int j, double v) {
    if (tk.rscale_off >= 0) v *= o.scales[tk.rscale_off + row];
    if (tk.ntasks > 1) {
        o.partm[((int64_t)tk.part_off + (int64_t)tk.local * tk.nrows + row) * o.R + j] = v;
    } else if ((tk.mode & 3) == 0) {
        const int64_t i = (int64_t)(tk.out_off + row) * o.R + j;
        if (o.mat64)
            o.wsm[i] = v;
        else
            o.wsm32[i] = (float)v;
    } else {
        o.ym[(int64_t)(tk.out_off + row) * o.R + j] += v;
    }
}

// One task: rows [r0, r0 + 64) (r0 = DTask::pad) against right-hand sides
// [j0, j0 + 16*NRB).  The wave walks 4 tiles per step; the item bookkeeping
// of those tiles is uniform (scalar loads), so only the tile data and the
// input values are vector loads, and the next step's loads are in flight
// while the current step's MFMAs run.
template <int DT, bool ACC64, int NRB>
__device__ __forceinline__ void task_rows(const DTask& tk, const DItem* __restrict__ items,
                                          const uint8_t* __restrict__ data, const double* __restrict__ wsm,
                                          const float* __restrict__ wsm32, int j0, int lane, const Outs& o) {
    using M = Mfma<ACC64>;
    using T = typename M::T;
    constexpr int V = dev::Tile<DT>::V;
    const int ebits = dev::task_ebits(tk.mode);
    const int rl = lane & 15, kq = lane >> 4;
    const int nrows = tk.nrows, r0 = tk.pad;
    const int nrg = min(4, (nrows - r0 + 15) / 16);
    const int64_t rt = (int64_t)nrows * 16;
    const uint8_t* base = data + tk.stream;
    const int k0 = tk.k0, k1 = tk.k1;
    const int R = o.R;
    int rows[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) rows[g] = min(r0 + g * 16 + rl, nrows - 1);
    typename M::V acc[4][NRB];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int b = 0; b < NRB; ++b) acc[g][b] = typename M::V{0, 0, 0, 0};

    struct Buf {
        uint4 q[4];
        T b[V][NRB];
    };
    ItemPos cur = item_pos<V>(items, tk.item_start);
    auto load = [&](Buf& f, int kb) {
        // uniform: the item of each of the 4 tiles of this step
        int vec[4], sc[4], t0[4], nc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = min(kb + u, k1 - 1);
            while (t >= cur.k1) cur = item_pos<V>(items, cur.it + 1);
            vec[u] = cur.vec;
            sc[u] = cur.sc;
            t0[u] = cur.k0;
            nc[u] = cur.nc;
        }
        const int tt = kb + kq;
        const bool valid = tt < k1;
        const int tc = valid ? tt : k1 - 1;
        const int myvec = kq == 0 ? vec[0] : kq == 1 ? vec[1] : kq == 2 ? vec[2] : vec[3];
        const int mysc = kq == 0 ? sc[0] : kq == 1 ? sc[1] : kq == 2 ? sc[2] : sc[3];
        const int myt0 = kq == 0 ? t0[0] : kq == 1 ? t0[1] : kq == 2 ? t0[2] : t0[3];
        const int mync = kq == 0 ? nc[0] : kq == 1 ? nc[1] : kq == 2 ? nc[2] : nc[3];
#pragma unroll
        for (int g = 0; g < 4; ++g)
            if (g < nrg) f.q[g] = *reinterpret_cast<const uint4*>(base + (int64_t)tc * rt + rows[g] * 16);
        const int cb = (tc - myt0) * V;
#pragma unroll
        for (int c = 0; c < V; ++c) {
            // the zero data past an item's last column takes the weight of
            // that last column (its own input and scale: finite), not the
            // neighbouring entry's, whose input times scale can overflow
            // float32 (zero times infinity is NaN); the index is clamped so
            // the loads stay unconditional
            const int cc = min(cb + c, mync - 1);
            const int64_t wi = (int64_t)(myvec + cc) * R + j0 + NRB * rl;
            T s = (T)1;
            if (mysc >= 0) s = (T)o.scales[mysc + cc];
            if (!valid) s = (T)0;
            // float64 products read float64 inputs where they exist: always
            // in a float64 matrix, only x in a float32 one
            const bool wide_in = ACC64 && (o.mat64 || myvec + cc < o.n);
            if constexpr (NRB == 2) {
                // R and j0 are multiples of 32: wi is even, the pair aligned
                if (wide_in) {
                    const double2 w = *reinterpret_cast<const double2*>(wsm + wi);
                    f.b[c][0] = (T)w.x * s;
                    f.b[c][1] = (T)w.y * s;
                } else {
                    const float2 w = *reinterpret_cast<const float2*>(wsm32 + wi);
                    f.b[c][0] = (T)w.x * s;
                    f.b[c][1] = (T)w.y * s;
                }
            } else {
#pragma unroll
                for (int b = 0; b < NRB; ++b)
                    f.b[c][b] = (wide_in ? (T)wsm[wi + b] : (T)wsm32[wi + b]) * s;
            }
        }
    };
    auto compute = [&](const Buf& f) {
#pragma unroll
        for (int c = 0; c < V; ++c)
#pragma unroll
            for (int g = 0; g < 4; ++g)
                if (g < nrg) {
                    const T a = elem<DT, T>(f.q[g], c, ebits);
#pragma unroll
                    for (int b = 0; b < NRB; ++b) acc[g][b] = M::step(a, f.b[c][b], acc[g][b]);
                }
    };
    // float32 accumulators are moved into float64 sums every kFlush tiles,
    // so a float32 accumulation chain never spans more than kFlush tiles
    constexpr int kFlush = 32;
    double sum[ACC64 ? 1 : 4][ACC64 ? 1 : NRB][ACC64 ? 1 : 4];
    if constexpr (!ACC64) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int b = 0; b < NRB; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) sum[g][b][i] = 0.0;
    }
    auto flush = [&]() {
        if constexpr (!ACC64) {
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int b = 0; b < NRB; ++b) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) sum[g][b][i] += (double)acc[g][b][i];
                    acc[g][b] = typename M::V{0, 0, 0, 0};
                }
        }
    };
    Buf fa, fb;
    load(fa, k0);
    for (int kb = k0; kb < k1; kb += 8) {
        load(fb, kb + 4);
        __builtin_amdgcn_sched_barrier(0);
        compute(fa);
        if (kb + 8 < k1) load(fa, kb + 8);
        __builtin_amdgcn_sched_barrier(0);
        if (kb + 4 < k1) compute(fb);
        if (!ACC64 && ((kb - k0 + 8) % kFlush) == 0) flush();
    }
    flush();
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if (g >= nrg) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = r0 + g * 16 + M::row(kq, i);
            if (row < nrows)
#pragma unroll
                for (int b = 0; b < NRB; ++b) {
                    double v;
                    if constexpr (ACC64)
                        v = acc[g][b][i];
                    else
                        v = sum[g][b][i];
                    put(tk, o, row, j0 + NRB * rl + b, v);
                }
        }
    }
}

// Wave w of a task list: task w / nblk against right-hand-side block w % nblk.
template <bool ACC64, int NRB, int MASK>
__device__ __forceinline__ void task_wave(const DTask* __restrict__ tasks, int64_t w, int nblk,
                                          const DItem* __restrict__ items, const uint8_t* __restrict__ data,
                                          const double* __restrict__ scales, double* wsm, float* wsm32,
                                          double* __restrict__ ym, double* __restrict__ partm, int R, int64_t n,
                                          int lane) {
    const int64_t t = w / nblk;
    const int j0 = (int)(w - t * nblk) * 16 * NRB;
    const DTask tk = tasks[t];
    const Outs o{wsm, wsm32, ym, partm, scales, R, n, ACC64};
    const int dt = tk.dtype;
    // MASK: the dtypes that may occur in the launched stage (one bit per
    // dtype); the other cases are not compiled, which keeps the register
    // budget of single-dtype stages low
    switch (dt) {
        case HM_F64:
            if constexpr ((MASK & (1 << HM_F64)) != 0)
                task_rows<HM_F64, true, NRB>(tk, items, data, wsm, wsm32, j0, lane, o);
            break;
        case HM_F32:
            if constexpr ((MASK & (1 << HM_F32)) != 0)
                task_rows<HM_F32, ACC64, NRB>(tk, items, data, wsm, wsm32, j0, lane, o);
            break;
        case HM_BF16:
            if constexpr ((MASK & (1 << HM_BF16)) != 0)
                task_rows<HM_BF16, ACC64, NRB>(tk, items, data, wsm, wsm32, j0, lane, o);
            break;
        case HM_F16:
            if constexpr ((MASK & (1 << HM_F16)) != 0)
                task_rows<HM_F16, ACC64, NRB>(tk, items, data, wsm, wsm32, j0, lane, o);
            break;
        case HM_FP8E4M3:
            if constexpr ((MASK & (1 << HM_FP8E4M3)) != 0)
                task_rows<HM_FP8E4M3, ACC64, NRB>(tk, items, data, wsm, wsm32, j0, lane, o);
            break;
#define HM_MR_CASE(D)                                                                                    \
    case D:                                                                                             \
        if constexpr ((MASK & (1 << D)) != 0)                                                           \
            task_rows<D, ACC64 || dev::kWide<D>, NRB>(tk, items, data, wsm, wsm32, j0, lane, o);         \
        break;
            HM_MR_CASE(HM_FPX24)
            HM_MR_CASE(HM_FPX40)
            HM_MR_CASE(HM_FPX48)
            HM_MR_CASE(HM_FPX56)
            HM_MR_CASE(HM_AFLP8)
            HM_MR_CASE(HM_AFLP16)
            HM_MR_CASE(HM_AFLP24)
            HM_MR_CASE(HM_AFLP32)
            HM_MR_CASE(HM_AFLP40)
            HM_MR_CASE(HM_AFLP48)
            HM_MR_CASE(HM_AFLP56)
#undef HM_MR_CASE
        default: {
            // a task without columns contributes zero
            for (int idx = lane; idx < 64 * 16 * NRB; idx += 64) {
                const int row = tk.pad + idx / (16 * NRB);
                if (row < tk.nrows) put(tk, o, row, j0 + idx % (16 * NRB), 0.0);
            }
        }
    }
}

// One wavefront per (task, block of 16*NRB right-hand sides); the blocks of
// one task are adjacent waves of one workgroup, so the task's slab is read
// from HBM about once.
template <bool ACC64, int NRB, int MASK>
__global__ __launch_bounds__(256) void k_tasks(const DTask* __restrict__ tasks, int ntasks, int nblk,
                                               const DItem* __restrict__ items, const uint8_t* __restrict__ data,
                                               const double* __restrict__ scales, double* wsm, float* wsm32,
                                               double* __restrict__ ym, double* __restrict__ partm, int R,
                                               int64_t n) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * 4 + wave;
    if (w >= (int64_t)ntasks * nblk) return;
    task_wave<ACC64, NRB, MASK>(tasks, w, nblk, items, data, scales, wsm, wsm32, ym, partm, R, n, threadIdx.x & 63);
}

// Several matrices in one launch: the stage tasks of up to kMaxJobs
// matrices, passed by value; wave w belongs to the last job whose first
// wave is <= w.
constexpr int kMaxJobs = 24;
struct Job {
    const DTask* tasks;
    const DItem* items;
    const uint8_t* data;
    const double* scales;
    double* wsm;
    float* wsm32;
    double* ym;
    double* partm;
    int64_t wave0;
    int64_t n;
    int32_t nblk, R;
};
struct Jobs {
    int32_t njobs;
    int64_t total;
    Job j[kMaxJobs];
};

template <bool ACC64, int NRB, int MASK>
__global__ __launch_bounds__(256) void k_tasks_multi(const Jobs J) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * 4 + wave;
    if (w >= J.total) return;
    int ji = 0;
    while (ji + 1 < J.njobs && w >= J.j[ji + 1].wave0) ++ji;
    const Job& jb = J.j[ji];
    task_wave<ACC64, NRB, MASK>(jb.tasks, w - jb.wave0, jb.nblk, jb.items, jb.data, jb.scales, jb.wsm, jb.wsm32,
                                jb.ym, jb.partm, jb.R, jb.n, threadIdx.x & 63);
}

// Sum the partial results of split owners in a fixed order.  Entries are
// independent: block (o, c) of the grid sums entries [256c, 256c + 256) of
// owner o of the list, one thread per entry, with eight independent sums
// (the loads of a pass are all in flight at once; missing ones read zero).
__device__ __forceinline__ void reduce_entry(const DOwner& ow, int64_t idx, const double* __restrict__ partm,
                                             double* wsm, float* wsm32, double* __restrict__ ym, int R,
                                             bool mat64) {
    const int64_t span = (int64_t)ow.nrows * R;
    if (idx >= span) return;
    const double* p = partm + (int64_t)ow.part_off * R + idx;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l = 0; l < ow.ntasks; l += 8) {
        double q[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) q[w] = l + w < ow.ntasks ? p[(int64_t)(l + w) * span] : 0.0;
#pragma unroll
        for (int w = 0; w < 8; ++w) acc[w] += q[w];
    }
    const double v = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    const int64_t e = (int64_t)ow.out_off * R + idx;
    if (ow.mode == 0) {
        if (mat64)
            wsm[e] = v;
        else
            wsm32[e] = (float)v;
    } else {
        ym[e] += v;
    }
}

__global__ __launch_bounds__(256) void k_reduce(const int32_t* __restrict__ list, const DOwner* __restrict__ owners,
                                                const double* __restrict__ partm, double* wsm, float* wsm32,
                                                double* __restrict__ ym, int R, int mat64) {
    reduce_entry(owners[list[blockIdx.x]], (int64_t)blockIdx.y * 256 + threadIdx.x, partm, wsm, wsm32, ym, R,
                 mat64 != 0);
}

struct RJob {
    const int32_t* list;
    const DOwner* owners;
    const double* partm;
    double* wsm;
    float* wsm32;
    double* ym;
    int64_t owner0;     // first global owner index of this job
    int32_t R, mat64;
};
struct RJobs {
    int32_t njobs;
    int64_t total;      // owners over all jobs
    RJob j[kMaxJobs];
};

__global__ __launch_bounds__(256) void k_reduce_multi(const RJobs J) {
    const int64_t i = blockIdx.x;
    int ji = 0;
    while (ji + 1 < J.njobs && i >= J.j[ji + 1].owner0) ++ji;
    const RJob& jb = J.j[ji];
    reduce_entry(jb.owners[jb.list[i - jb.owner0]], (int64_t)blockIdx.y * 256 + threadIdx.x, jb.partm, jb.wsm,
                 jb.wsm32, jb.ym, jb.R, jb.mat64 != 0);
}

// X (column-major, ldx, original order) -> wsm / wsm32 in cluster order,
// entry-major; padding columns j >= nrhs get zeros and ym is cleared.  A
// block moves a 64 (points) x 64 (columns) tile through LDS: it reads X with
// consecutive lanes on consecutive points and writes each point's row of
// values at its cluster position iperm[o] with consecutive lanes on
// consecutive columns (iperm = null: cluster order already).
template <typename XT>
__global__ __launch_bounds__(256) void k_gather(const XT* __restrict__ X, int64_t ldx, int nrhs,
                                                const int64_t* __restrict__ iperm, int64_t n, int R,
                                                double* __restrict__ wsm, float* __restrict__ wsm32,
                                                double* __restrict__ ym) {
    __shared__ double tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t o0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    const int64_t o = o0 + tx;
    for (int jj = ty; jj < 64; jj += 4) {
        const int j = j0 + jj;
        tile[jj][tx] = (o < n && j < nrhs) ? (double)X[o + (int64_t)j * ldx] : 0.0;
    }
    __syncthreads();
    for (int ii = ty; ii < 64; ii += 4) {
        const int64_t oo = o0 + ii;
        const int j = j0 + tx;
        if (oo < n && j < R) {
            const int64_t r = iperm ? iperm[oo] : oo;
            const double v = tile[tx][ii];
            wsm[r * R + j] = v;
            wsm32[r * R + j] = (float)v;
            ym[r * R + j] = 0.0;
        }
    }
}

// Y[o, j] += alpha * ym[iperm[o] * R + j]  (column-major Y, ldy), via LDS.
template <typename YT>
__global__ __launch_bounds__(256) void k_scatter(YT* __restrict__ Y, int64_t ldy, int nrhs,
                                                 const int64_t* __restrict__ iperm, int64_t n, int R,
                                                 const double* __restrict__ ym, double alpha) {
    __shared__ double tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t o0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    for (int ii = ty; ii < 64; ii += 4) {
        const int64_t oo = o0 + ii;
        const int j = j0 + tx;
        double v = 0.0;
        if (oo < n && j < R) v = ym[(iperm ? iperm[oo] : oo) * R + j];
        tile[ii][tx] = v;
    }
    __syncthreads();
    const int64_t o = o0 + tx;
    if (o < n) {
        for (int jj = ty; jj < 64; jj += 4) {
            const int j = j0 + jj;
            if (j < nrhs) {
                YT* p = Y + o + (int64_t)j * ldy;
                *p = (YT)((double)*p + alpha * tile[tx][jj]);
            }
        }
    }
}

using TaskKernel = void (*)(const DTask*, int, int, const DItem*, const uint8_t*, const double*, double*, float*,
                            double*, double*, int, int64_t);

// [acc64][NRB - 1][dtype of a single-dtype run of tasks; entry 5 = all
// hardware formats]
#define HM_MR_ROW(K, A, N)                                                                               \
    {                                                                                                   \
        &K<A, N, 1 << 0>, &K<A, N, 1 << 1>, &K<A, N, 1 << 2>, &K<A, N, 1 << 3>, &K<A, N, 1 << 4>,       \
            &K<A, N, 31>, &K<A, N, 1 << 6>, &K<A, N, 1 << 7>, &K<A, N, 1 << 8>, &K<A, N, 1 << 9>,        \
            &K<A, N, 1 << 10>, &K<A, N, 1 << 11>, &K<A, N, 1 << 12>, &K<A, N, 1 << 13>,                 \
            &K<A, N, 1 << 14>, &K<A, N, 1 << 15>, &K<A, N, 1 << 16>                                     \
    }
static const TaskKernel kTasks[2][2][HM_NDTYPES] = {
    {HM_MR_ROW(k_tasks, false, 1), HM_MR_ROW(k_tasks, false, 2)},
    {HM_MR_ROW(k_tasks, true, 1), HM_MR_ROW(k_tasks, true, 2)}};

using MultiKernel = void (*)(const Jobs);
static const MultiKernel kMulti[2][2][HM_NDTYPES] = {
    {HM_MR_ROW(k_tasks_multi, false, 1), HM_MR_ROW(k_tasks_multi, false, 2)},
    {HM_MR_ROW(k_tasks_multi, true, 1), HM_MR_ROW(k_tasks_multi, true, 2)}};
#undef HM_MR_ROW


}  // namespace mr

// Column-chunk size of the many-RHS plan (bytes per 64-row group) unless
// the tuner picked another one.
static constexpr int64_t kDefaultMrTarget = 256 * 1024;

// Build (or rebuild for another chunk size) the matrix's many-RHS plan and
// copy its tables to the device.
static hm_status ensure_mr_plan(hm_matrix* m, int64_t target) {
    if (m->mr_meta && m->mr_target == target) return HM_OK;
    MrPlan P;
    try {
        build_mr_plan(m->h_owners, m->h_items, m->h_tasks, m->h_stages, target, P);
    } catch (const std::bad_alloc&) {
        set_error("hm_mvm_batch: out of host memory");
        return HM_ENOMEM;
    }
    size_t off = 0;
    const size_t o_tasks = off;
    off = align256(off + P.tasks.size() * sizeof(DTask));
    const size_t o_owners = off;
    off = align256(off + P.owners.size() * sizeof(DOwner));
    std::vector<size_t> o_red;
    for (auto& st : P.stages) {
        o_red.push_back(off);
        off = align256(off + st.reduce.size() * sizeof(int32_t));
    }
    // cluster position of every original index, for the block gather/scatter
    const size_t o_iperm = off;
    off = align256(off + (size_t)m->n * sizeof(int64_t));
    std::vector<uint8_t> host(std::max<size_t>(off, 256), 0);
    {
        int64_t* ip = (int64_t*)(host.data() + o_iperm);
        const std::vector<int64_t>& perm = m->layout->L.perm;
        for (int64_t i = 0; i < m->n; ++i) ip[perm[(size_t)i]] = i;
    }
    // tasks of a stage ordered by dtype: the stage launches once per dtype
    // with the kernel compiled for that dtype alone (register budget)
    for (auto& st : P.stages)
        std::stable_sort(P.tasks.begin() + st.t0, P.tasks.begin() + st.t1,
                         [](const DTask& a, const DTask& b) { return a.dtype < b.dtype; });
    std::memcpy(host.data() + o_tasks, P.tasks.data(), P.tasks.size() * sizeof(DTask));
    std::memcpy(host.data() + o_owners, P.owners.data(), P.owners.size() * sizeof(DOwner));
    for (size_t i = 0; i < P.stages.size(); ++i)
        std::memcpy(host.data() + o_red[i], P.stages[i].reduce.data(), P.stages[i].reduce.size() * sizeof(int32_t));
    hipError_t e = hipSuccess;
    if (m->mr_meta) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail("hm_mvm_batch: synchronize before replacing the plan", e);
        (void)hipFree(m->mr_meta);
        m->mr_meta = nullptr;
    }
    void* d = nullptr;
    e = hipMalloc(&d, host.size());
    if (e != hipSuccess) {
        set_error("hm_mvm_batch: hipMalloc of the many-RHS plan failed");
        return HM_ENOMEM;
    }
    e = hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail("hm_mvm_batch: plan copy", e);
    }
    for (auto& ph : m->mr_phases)
        for (auto& ev : ph.pending) m->event_pool.push_back(ev);
    m->mr_phases.clear();
    uint8_t* b = (uint8_t*)d;
    for (size_t i = 0; i < P.stages.size(); ++i) {
        const Stage& st = P.stages[i];
        DevStage ds;
        ds.aux = st.aux;
        ds.t0 = st.t0;
        ds.ntasks = (int32_t)(st.t1 - st.t0);
        ds.reduce = (const int32_t*)(b + o_red[i]);
        ds.nreduce = (int32_t)st.reduce.size();
        ds.reduce_rows = 0;
        for (int32_t o : st.reduce) ds.reduce_rows = std::max(ds.reduce_rows, P.owners[o].nrows);
        ds.nowners = 0;
        ds.dtype_mask = 0;
        for (int64_t k = st.t0; k < st.t1; ++k) {
            const DTask& t = P.tasks[k];
            if (t.c0 < t.c1) ds.dtype_mask |= 1 << t.dtype;
            if (ds.subs.empty() || ds.subs.back().dtype != t.dtype)
                ds.subs.push_back(DevStage::Sub{t.dtype, (int32_t)(k - st.t0), 0});
            ds.subs.back().ntasks++;
        }
        ds.data_bytes = st.data_bytes;
        ds.data_entries = st.data_entries;
        ds.alg_bytes = (double)st.data_bytes;
        ds.name = st.name;
        m->mr_phases.push_back(ds);
    }
    m->mr_meta = d;
    m->mr_gen++;
    m->mr_tasks = (const DTask*)(b + o_tasks);
    m->mr_iperm = (const int64_t*)(b + o_iperm);
    m->mr_owners = (const DOwner*)(b + o_owners);
    if (P.part_elems > m->mr_part_elems && m->mr_arena) {
        // the partial-sum workspace no longer fits: regrow it on next use
        (void)hipFree(m->mr_arena);
        m->mr_arena = nullptr;
        m->mr_cap = 0;
    }
    m->mr_part_elems = std::max(m->mr_part_elems, P.part_elems);
    m->mr_target = target;
    return HM_OK;
}

// Byte layout of a many-RHS workspace of R values per entry:
// wsm | wsm32 | ym | partm, each 256-byte aligned; returns the total.
static size_t mr_ws_layout(const hm_matrix* m, int R, size_t& o_wsm32, size_t& o_ym, size_t& o_part) {
    const size_t ent = (size_t)(m->ws_elems + TILE_PAD);
    o_wsm32 = align256(ent * R * sizeof(double));
    o_ym = align256(o_wsm32 + ent * R * sizeof(float));
    o_part = align256(o_ym + (size_t)m->n * R * sizeof(double));
    return align256(o_part + (size_t)std::max<int64_t>(m->mr_part_elems, 1) * R * sizeof(double));
}

// Grow the matrix's many-RHS workspace to R values per entry.
static hm_status ensure_mr(hm_matrix* m, int R) {
    hm_status st = ensure_mr_plan(m, m->mr_target ? m->mr_target : kDefaultMrTarget);
    if (st != HM_OK) return st;
    if (m->mr_cap >= R) return HM_OK;
    if (m->mr_arena) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail("hm_mvm_batch: synchronize before regrowing the workspace", e);
        (void)hipFree(m->mr_arena);
        m->mr_arena = nullptr;
        m->mr_cap = 0;
    }
    size_t o_wsm32, o_ym, o_part;
    const size_t total = mr_ws_layout(m, R, o_wsm32, o_ym, o_part);
    const size_t o_wsm = 0;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) {
        set_error("hm_mvm_batch: hipMalloc of " + std::to_string(total) + " bytes of workspace failed");
        return HM_ENOMEM;
    }
    // every workspace entry starts finite (padding columns of last tiles read them)
    e = hipMemset(p, 0, total);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail("hm_mvm_batch: hipMemset", e);
    }
    uint8_t* b = (uint8_t*)p;
    m->mr_arena = p;
    m->mr_gen++;
    m->mr_cap = R;
    m->wsm = (double*)(b + o_wsm);
    m->wsm32 = (float*)(b + o_wsm32);
    m->ym = (double*)(b + o_ym);
    m->partm = (double*)(b + o_part);
    return HM_OK;
}

// Width of the padded right-hand-side block: 16 or a multiple of 32.
static int padded_width(int nrhs) { return nrhs <= 16 ? 16 : (nrhs + 31) / 32 * 32; }

// 16-wide right-hand-side blocks per wave of one stage: the stage's tuned
// choice, else the matrix's; 2 needs R >= 32.
static int stage_nrb(const hm_matrix* m, const DevStage& ph, int R) {
    const int want = ph.mr_nrb ? ph.mr_nrb : m->mr_nrb;
    return (R >= 32 && want == 2) ? 2 : 1;
}

// The many-RHS workspace one call uses: the matrix's own (grown on demand)
// or a caller-provided region of the same layout.
struct MrWs {
    double* wsm;
    float* wsm32;
    double* ym;
    double* partm;
};

static hm_status mvm_many_ws(hm_matrix* m, const MrWs& ws, double alpha, const void* X, int64_t ldx, int nrhs,
                             void* Y, int64_t ldy, int32_t vdt, uint32_t flags, hipStream_t stream);

static hm_status mvm_many(hm_matrix* m, double alpha, const void* X, int64_t ldx, int nrhs, void* Y, int64_t ldy,
                          int32_t vdt, uint32_t flags, hipStream_t stream) {
    hm_status st = ensure_mr(m, padded_width(nrhs));
    if (st != HM_OK) return st;
    return mvm_many_ws(m, MrWs{m->wsm, m->wsm32, m->ym, m->partm}, alpha, X, ldx, nrhs, Y, ldy, vdt, flags, stream);
}

static hm_status mvm_many_ws(hm_matrix* m, const MrWs& ws, double alpha, const void* X, int64_t ldx, int nrhs,
                             void* Y, int64_t ldy, int32_t vdt, uint32_t flags, hipStream_t stream) {
    const int R = padded_width(nrhs);
    const int64_t n = m->n;
    const int64_t* perm = (flags & HM_CLUSTER_ORDER) ? nullptr : m->mr_iperm;
    const bool timing = (flags & HM_TIMING) != 0;
    dim3 tgrid((unsigned)((n + 63) / 64), (unsigned)((R + 63) / 64));
    if (vdt == HM_F64)
        hipLaunchKernelGGL(mr::k_gather<double>, tgrid, dim3(256), 0, stream, (const double*)X, ldx, nrhs, perm, n, R,
                           ws.wsm, ws.wsm32, ws.ym);
    else
        hipLaunchKernelGGL(mr::k_gather<float>, tgrid, dim3(256), 0, stream, (const float*)X, ldx, nrhs, perm, n, R,
                           ws.wsm, ws.wsm32, ws.ym);
    const hipStream_t main_stream = stream;
    if (m->aux) {
        (void)hipEventRecord(m->ev_fork, main_stream);
        (void)hipStreamWaitEvent(m->aux, m->ev_fork, 0);
    }
    bool joined = m->aux == nullptr;
    for (auto& ph : m->mr_phases) {
        hipStream_t s = ph.aux ? m->aux : main_stream;
        if (!joined && !ph.aux && ph.ntasks == 0 && &ph == &m->mr_phases.back()) {
            (void)hipEventRecord(m->ev_join, m->aux);
            (void)hipStreamWaitEvent(main_stream, m->ev_join, 0);
            joined = true;
        }
        if (ph.ntasks > 0) {
            const int nrb = stage_nrb(m, ph, R);   // blocks of 16 right-hand sides per wave
            const int nblk = R / (16 * nrb);
            const int64_t waves = (int64_t)ph.ntasks * nblk;
            std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
            if (timing && !timing_begin(m, ph, R, s, ev)) {
                set_error("hm_mvm_batch: timing events failed");
                return HM_EDEVICE;
            }
            (void)waves;
            for (const auto& sb : ph.subs) {
                // dtype -1 (tasks without columns) runs with any variant
                const int var = sb.dtype < 0 ? HM_F32 : sb.dtype;
                const int64_t w = (int64_t)sb.ntasks * nblk;
                hipLaunchKernelGGL(mr::kTasks[m->acc64 ? 1 : 0][nrb - 1][var], dim3((unsigned)((w + 3) / 4)),
                                   dim3(256), 0, s, m->mr_tasks + ph.t0 + sb.t0, sb.ntasks, nblk, m->items, m->data,
                                   m->scales, ws.wsm, ws.wsm32, ws.ym, ws.partm, R, n);
            }
            if (timing) timing_end(ph, s, ev);
        }
        if (ph.nreduce > 0)
            hipLaunchKernelGGL(mr::k_reduce,
                               dim3((unsigned)ph.nreduce, (unsigned)(((int64_t)ph.reduce_rows * R + 255) / 256)),
                               dim3(256), 0, s, ph.reduce, m->mr_owners, ws.partm, ws.wsm, ws.wsm32, ws.ym, R,
                               m->acc64 ? 1 : 0);
    }
    if (!joined) {
        (void)hipEventRecord(m->ev_join, m->aux);
        (void)hipStreamWaitEvent(main_stream, m->ev_join, 0);
    }
    if (vdt == HM_F64)
        hipLaunchKernelGGL(mr::k_scatter<double>, tgrid, dim3(256), 0, main_stream, (double*)Y, ldy, nrhs, perm, n, R,
                           ws.ym, alpha);
    else
        hipLaunchKernelGGL(mr::k_scatter<float>, tgrid, dim3(256), 0, main_stream, (float*)Y, ldy, nrhs, perm, n, R,
                           ws.ym, alpha);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail("hm_mvm_batch: kernel launch", e);
    return HM_OK;
}

// Several matrices at once: the stages of all of them are merged level by
// level (the dense stage, which only reads x, joins level 0), so each level
// is one launch per (accumulation, blocks-per-wave) class instead of one per
// matrix and stage.
struct Entry {
    hm_matrix* m;
    double alpha;
    const void* X;
    int64_t ldx;
    int nrhs;
    void* Y;
    int64_t ldy;
    int R;
    std::vector<int> level;   // per many-RHS stage; -1 = the final reduce
};

static hm_status mvm_many_multi(std::vector<Entry>& E, int32_t vdt, uint32_t flags, hipStream_t s) {
    int maxL = -1;
    for (auto& e : E) {
        e.R = padded_width(e.nrhs);
        hm_status st = ensure_mr(e.m, e.R);
        if (st != HM_OK) return st;
        e.level.clear();
        int next = 0;
        const auto& ph = e.m->mr_phases;
        for (size_t i = 0; i < ph.size(); ++i) {
            const bool fin = i + 1 == ph.size() && ph[i].ntasks == 0 && !ph[i].aux;
            e.level.push_back(fin ? -1 : ph[i].aux ? 0 : next++);
        }
        maxL = std::max(maxL, next - 1);
    }
    for (auto& e : E) {
        const int64_t* perm = (flags & HM_CLUSTER_ORDER) ? nullptr : e.m->mr_iperm;
        dim3 tgrid((unsigned)((e.m->n + 63) / 64), (unsigned)((e.R + 63) / 64));
        if (vdt == HM_F64)
            hipLaunchKernelGGL(mr::k_gather<double>, tgrid, dim3(256), 0, s, (const double*)e.X, e.ldx, e.nrhs, perm,
                               e.m->n, e.R, e.m->wsm, e.m->wsm32, e.m->ym);
        else
            hipLaunchKernelGGL(mr::k_gather<float>, tgrid, dim3(256), 0, s, (const float*)e.X, e.ldx, e.nrhs, perm,
                               e.m->n, e.R, e.m->wsm, e.m->wsm32, e.m->ym);
    }
    auto launch_reduces = [&](int L) {
        mr::RJobs J{};
        int64_t span = 0;   // largest nrows * R of the job's owners
        auto flush = [&]() {
            if (J.njobs > 0 && J.total > 0)
                hipLaunchKernelGGL(mr::k_reduce_multi, dim3((unsigned)J.total, (unsigned)((span + 255) / 256)),
                                   dim3(256), 0, s, J);
            J = mr::RJobs{};
            span = 0;
        };
        for (auto& e : E)
            for (size_t i = 0; i < e.m->mr_phases.size(); ++i) {
                const DevStage& ph = e.m->mr_phases[i];
                if (e.level[i] != L || ph.nreduce == 0) continue;
                if (J.njobs == mr::kMaxJobs) flush();
                J.j[J.njobs++] = mr::RJob{ph.reduce, e.m->mr_owners, e.m->partm, e.m->wsm, e.m->wsm32, e.m->ym,
                                          J.total, e.R, e.m->acc64 ? 1 : 0};
                J.total += ph.nreduce;
                span = std::max(span, (int64_t)ph.reduce_rows * e.R);
            }
        flush();
    };
    for (int L = 0; L <= maxL; ++L) {
        for (int acc = 0; acc < 2; ++acc)
            for (int nrb = 1; nrb <= 2; ++nrb)
                for (int dt = -1; dt < 5; ++dt) {
                    mr::Jobs J{};
                    const int var = dt < 0 ? HM_F32 : dt;
                    auto flush = [&]() {
                        if (J.njobs > 0 && J.total > 0)
                            hipLaunchKernelGGL(mr::kMulti[acc][nrb - 1][var], dim3((unsigned)((J.total + 3) / 4)),
                                               dim3(256), 0, s, J);
                        J = mr::Jobs{};
                    };
                    for (auto& e : E) {
                        if ((e.m->acc64 ? 1 : 0) != acc) continue;
                        for (size_t i = 0; i < e.m->mr_phases.size(); ++i) {
                            const DevStage& ph = e.m->mr_phases[i];
                            if (e.level[i] != L || ph.ntasks == 0 || stage_nrb(e.m, ph, e.R) != nrb) continue;
                            const int nblk = e.R / (16 * nrb);
                            for (const auto& sb : ph.subs) {
                                if (sb.dtype != dt) continue;
                                if (J.njobs == mr::kMaxJobs) flush();
                                J.j[J.njobs++] = mr::Job{e.m->mr_tasks + ph.t0 + sb.t0, e.m->items, e.m->data,
                                                         e.m->scales, e.m->wsm, e.m->wsm32, e.m->ym, e.m->partm,
                                                         J.total, e.m->n, nblk, e.R};
                                J.total += (int64_t)sb.ntasks * nblk;
                            }
                        }
                    }
                    flush();
                }
        launch_reduces(L);
    }
    launch_reduces(-1);
    for (auto& e : E) {
        const int64_t* perm = (flags & HM_CLUSTER_ORDER) ? nullptr : e.m->mr_iperm;
        dim3 tgrid((unsigned)((e.m->n + 63) / 64), (unsigned)((e.R + 63) / 64));
        if (vdt == HM_F64)
            hipLaunchKernelGGL(mr::k_scatter<double>, tgrid, dim3(256), 0, s, (double*)e.Y, e.ldy, e.nrhs, perm,
                               e.m->n, e.R, e.m->ym, e.alpha);
        else
            hipLaunchKernelGGL(mr::k_scatter<float>, tgrid, dim3(256), 0, s, (float*)e.Y, e.ldy, e.nrhs, perm,
                               e.m->n, e.R, e.m->ym, e.alpha);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail("hm_mvm_batch: kernel launch", e);
    return HM_OK;
}

hm_status mvm_blocks(const BlockCall* calls, int ncalls, hipStream_t stream) {
    if (ncalls == 1)
        return mvm_many(calls[0].m, calls[0].alpha, calls[0].X, calls[0].ldx, calls[0].nrhs, calls[0].Y,
                        calls[0].ldy, HM_F64, 0, stream);
    std::vector<Entry> E;
    for (int i = 0; i < ncalls; ++i) {
        Entry e;
        e.m = calls[i].m;
        e.alpha = calls[i].alpha;
        e.X = calls[i].X;
        e.ldx = calls[i].ldx;
        e.nrhs = calls[i].nrhs;
        e.Y = calls[i].Y;
        e.ldy = calls[i].ldy;
        E.push_back(std::move(e));
    }
    return mvm_many_multi(E, HM_F64, 0, stream);
}

// Run `reps` products on the current plan; *ms = mean time per product.  With
// `phase_ms`, the products are event-timed per stage and the per-stage mean
// times are returned as well.
static hm_status time_plan(hm_matrix* m, int nrhs, int32_t vdt, const void* X, void* Y, int reps, hipStream_t s,
                           double* ms, std::vector<double>* phase_ms) {
    hm_status st = mvm_many(m, 1.0, X, m->n, nrhs, Y, m->n, vdt, 0, s);   // warm-up
    if (st != HM_OK) return st;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    const uint32_t flags = phase_ms ? HM_TIMING : 0;
    for (int r = 0; r < reps && e == hipSuccess && st == HM_OK; ++r)
        st = mvm_many(m, 1.0, X, m->n, nrhs, Y, m->n, vdt, flags, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (phase_ms) {
        phase_ms->assign(m->mr_phases.size(), 0.0);
        for (size_t i = 0; i < m->mr_phases.size(); ++i) {
            for (auto& ev : m->mr_phases[i].pending) {
                float pt = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&pt, ev.first, ev.second);
                (*phase_ms)[i] += (double)pt / reps;
                m->event_pool.push_back(ev);
            }
            m->mr_phases[i].pending.clear();
        }
    }
    if (st != HM_OK) return st;
    if (e != hipSuccess) return hip_fail("hm_tune_batch: timing", e);
    *ms = (double)t / reps;
    return HM_OK;
}

hm_status batch_prepare(hm_matrix* const* mats, int32_t nmat, const int32_t* nrhs, int32_t vec_dtype) {
    if (nmat < 0 || (nmat > 0 && (!mats || !nrhs))) {
        set_error("hm_graph_create_batch: null argument");
        return HM_EINVAL;
    }
    for (int32_t i = 0; i < nmat; ++i) {
        if (!mats[i] || nrhs[i] < 0 || nrhs[i] > HM_MAX_NRHS) {
            set_error("hm_graph_create_batch: null matrix or nrhs out of range");
            return HM_EINVAL;
        }
        if (nrhs[i] == 0 || (nrhs[i] == 1 && vec_dtype == HM_F64)) continue;
        hm_status st = ensure_mr(mats[i], padded_width(nrhs[i]));
        if (st != HM_OK) return st;
    }
    return HM_OK;
}

}  // namespace hm

namespace hm {
// HM_ADJOINT: the same call on the matrices' adjoints (uploaded with
// hm_upload_opts.adjoint); false with the error set if one has none.
bool adjoint_mats(hm_matrix* const* mats, int32_t nmat, const int32_t* nrhs, std::vector<hm_matrix*>& out,
                  const char* who) {
    out.assign((size_t)std::max(nmat, 0), nullptr);
    for (int32_t i = 0; i < nmat; ++i) {
        if (!mats[i] || nrhs[i] == 0) {
            out[(size_t)i] = mats[i];
            continue;
        }
        if (!mats[i]->adj) {
            set_error(std::string(who) + ": HM_ADJOINT needs matrices uploaded with hm_upload_opts.adjoint = 1");
            return false;
        }
        out[(size_t)i] = mats[i]->adj;
    }
    return true;
}
}  // namespace hm

extern "C" hm_status hm_mvm_batch(hm_matrix* const* mats, int32_t nmat, double alpha, const void* const* X,
                                  const int64_t* ldx, const int32_t* nrhs, void* const* Y, const int64_t* ldy,
                                  int32_t vec_dtype, uint32_t flags, hm_stream_t stream) {
    if ((flags & HM_ADJOINT) && nmat > 0 && mats && nrhs) {
        std::vector<hm_matrix*> adj;
        if (!hm::adjoint_mats(mats, nmat, nrhs, adj, "hm_mvm_batch")) return HM_EINVAL;
        return hm_mvm_batch(adj.data(), nmat, alpha, X, ldx, nrhs, Y, ldy, vec_dtype, flags & ~HM_ADJOINT, stream);
    }
    if (nmat < 0 || (nmat > 0 && (!mats || !X || !ldx || !nrhs || !Y || !ldy))) {
        hm::set_error("hm_mvm_batch: null argument");
        return HM_EINVAL;
    }
    if (vec_dtype != HM_F64 && vec_dtype != HM_F32) {
        hm::set_error("hm_mvm_batch: vec_dtype must be HM_F64 or HM_F32");
        return HM_EINVAL;
    }
    if (flags & ~(uint32_t)(HM_CLUSTER_ORDER | HM_TIMING)) {
        hm::set_error("hm_mvm_batch: unsupported flags");
        return HM_EINVAL;
    }
    int dev = -1;
    if (nmat > 0 && hipGetDevice(&dev) != hipSuccess) {
        hm::set_error("hm_mvm_batch: no current device");
        return HM_EDEVICE;
    }
    for (int32_t i = 0; i < nmat; ++i) {
        const hm_matrix* m = mats[i];
        if (!m || nrhs[i] < 0 || nrhs[i] > HM_MAX_NRHS) {
            hm::set_error("hm_mvm_batch: null matrix or nrhs out of [0, HM_MAX_NRHS] at index " + std::to_string(i));
            return HM_EINVAL;
        }
        if (nrhs[i] == 0) continue;
        if (!X[i] || !Y[i] || X[i] == Y[i] || ldx[i] < m->n || ldy[i] < m->n) {
            hm::set_error("hm_mvm_batch: bad X/Y or leading dimension at index " + std::to_string(i));
            return HM_EINVAL;
        }
        if (m->device != dev) {
            hm::set_error("hm_mvm_batch: matrix " + std::to_string(i) + " lives on another device");
            return HM_EINVAL;
        }
        for (int32_t k = 0; k < i; ++k)
            if (mats[k] == m && nrhs[k] > 0) {
                hm::set_error("hm_mvm_batch: a matrix appears twice (its workspace is shared)");
                return HM_EINVAL;
            }
    }
    // single float64 columns: the single-vector kernels
    int nmany = 0;
    for (int32_t i = 0; i < nmat; ++i) {
        if (nrhs[i] == 0) continue;
        if (nrhs[i] == 1 && vec_dtype == HM_F64) {
            hm_status st = hm_mvm(mats[i], alpha, (const double*)X[i], (double*)Y[i], flags, stream);
            if (st != HM_OK) return st;
        } else {
            ++nmany;
        }
    }
    if (nmany == 1 || (flags & HM_TIMING)) {
        // one block (or per-phase timing): the per-matrix launch sequence
        for (int32_t i = 0; i < nmat; ++i) {
            if (nrhs[i] == 0 || (nrhs[i] == 1 && vec_dtype == HM_F64)) continue;
            hm_status st = hm::mvm_many(mats[i], alpha, X[i], ldx[i], nrhs[i], Y[i], ldy[i], vec_dtype, flags,
                                        (hipStream_t)stream);
            if (st != HM_OK) return st;
        }
        return HM_OK;
    }
    if (nmany == 0) return HM_OK;
    std::vector<hm::Entry> E;
    for (int32_t i = 0; i < nmat; ++i) {
        if (nrhs[i] == 0 || (nrhs[i] == 1 && vec_dtype == HM_F64)) continue;
        hm::Entry e;
        e.m = mats[i];
        e.alpha = alpha;
        e.X = X[i];
        e.ldx = ldx[i];
        e.nrhs = nrhs[i];
        e.Y = Y[i];
        e.ldy = ldy[i];
        E.push_back(std::move(e));
    }
    return hm::mvm_many_multi(E, vec_dtype, flags, (hipStream_t)stream);
}

extern "C" hm_status hm_tune_batch(hm_matrix* m, int32_t nrhs, int32_t vec_dtype, int32_t reps, hm_stream_t stream,
                                   hm_tune_result* out) {
    if (!m || nrhs < 2 || nrhs > HM_MAX_NRHS || (vec_dtype != HM_F64 && vec_dtype != HM_F32) || reps < 1) {
        hm::set_error("hm_tune_batch: bad argument (nrhs in [2, HM_MAX_NRHS], vec_dtype F64/F32, reps >= 1)");
        return HM_EINVAL;
    }
    if (m->adj) {   // the adjoint's plan is tuned (and built) as well
        hm_tune_result ra{};
        hm_status sa = hm_tune_batch(m->adj, nrhs, vec_dtype, reps, stream, &ra);
        if (sa != HM_OK) return sa;
    }
    const size_t esz = vec_dtype == HM_F64 ? 8 : 4;
    const size_t bytes = (size_t)m->n * nrhs * esz;
    void* X = nullptr;
    void* Y = nullptr;
    if (hipMalloc(&X, bytes) != hipSuccess || hipMalloc(&Y, bytes) != hipSuccess) {
        if (X) (void)hipFree(X);
        hm::set_error("hm_tune_batch: hipMalloc of the trial blocks failed");
        return HM_ENOMEM;
    }
    hipError_t e = hipMemset(X, 0, bytes);
    if (e == hipSuccess) e = hipMemset(Y, 0, bytes);
    if (e != hipSuccess) {
        (void)hipFree(X);
        (void)hipFree(Y);
        return hm::hip_fail("hm_tune_batch: hipMemset", e);
    }
    // For every chunk size: time each stage with 1 and 2 blocks per wave,
    // keep the faster per stage, then time that combination as a whole.
    static const int64_t targets[] = {64 * 1024, 128 * 1024, 256 * 1024, 512 * 1024, 1024 * 1024};
    const int R = hm::padded_width(nrhs);
    const int maxnrb = R >= 32 ? 2 : 1;
    hm_tune_result best{0, 1, 0.0, 0};
    std::vector<int32_t> best_nrb;
    hm_status st = HM_OK;
    for (int64_t t : targets) {
        m->mr_nrb = 1;
        st = hm::ensure_mr_plan(m, t);
        if (st != HM_OK) break;
        const size_t np = m->mr_phases.size();
        std::vector<double> tbest(np, 0.0);
        std::vector<int32_t> choice(np, 1);
        double ms = 0.0;
        for (int nrb = 1; nrb <= maxnrb && st == HM_OK; ++nrb) {
            for (auto& ph : m->mr_phases) ph.mr_nrb = nrb;
            std::vector<double> pm;
            st = hm::time_plan(m, nrhs, vec_dtype, X, Y, reps, (hipStream_t)stream, &ms, &pm);
            ++best.ncandidates;
            for (size_t i = 0; i < np && st == HM_OK; ++i)
                if (nrb == 1 || pm[i] < tbest[i]) {
                    tbest[i] = pm[i];
                    choice[i] = nrb;
                }
        }
        if (st != HM_OK) break;
        for (size_t i = 0; i < np; ++i) m->mr_phases[i].mr_nrb = choice[i];
        if (maxnrb > 1) {
            st = hm::time_plan(m, nrhs, vec_dtype, X, Y, reps, (hipStream_t)stream, &ms, nullptr);
            if (st != HM_OK) break;
            ++best.ncandidates;
        }
        if (best.target_bytes == 0 || ms < best.ms) {
            best.target_bytes = t;
            best.ms = ms;
            best_nrb = choice;
            // report the choice of the stage that streams the most data
            size_t big = 0;
            for (size_t i = 1; i < np; ++i)
                if (m->mr_phases[i].data_bytes > m->mr_phases[big].data_bytes) big = i;
            best.nrb = np ? choice[big] : 1;
        }
    }
    (void)hipDeviceSynchronize();
    (void)hipFree(X);
    (void)hipFree(Y);
    if (st != HM_OK) return st;
    m->mr_nrb = 1;
    st = hm::ensure_mr_plan(m, best.target_bytes);
    if (st != HM_OK) return st;
    for (size_t i = 0; i < m->mr_phases.size() && i < best_nrb.size(); ++i) m->mr_phases[i].mr_nrb = best_nrb[i];
    if (out) *out = best;
    return HM_OK;
}

// ------------------------------------------------- no-allocation variant
//
// hm_mvm_batch_noalloc: the many-RHS products of hm_mvm_batch with their
// workspaces carved out of one file-scope device array instead of the
// matrices' own (grown by hipMalloc).  Each GPU holds its own copy of the
// array for the life of the process; host code addresses it only through
// the device address hipGetSymbolAddress returns for the current device.

static __device__ __align__(256) uint8_t scratch[HM_NOALLOC_SCRATCH_BYTES];

namespace hm {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
hm_status scratch_address(int dev, uint8_t** out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("hm_mvm_batch_noalloc: device index out of range");
        return HM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail("hm_mvm_batch_noalloc: hipGetSymbolAddress(scratch)", e);
        g_scratch_ptr[dev] = p;
    }
    *out = (uint8_t*)g_scratch_ptr[dev];
    return HM_OK;
}

// Zero n16 16-byte words (the workspace of one call starts from zeros).
__global__ __launch_bounds__(256) void k_zero16(uint4* __restrict__ p, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace
}  // namespace hm

extern "C" hm_status hm_mvm_batch_noalloc(hm_matrix* const* mats, int32_t nmat, double alpha, const void* const* X,
                                          const int64_t* ldx, const int32_t* nrhs, void* const* Y,
                                          const int64_t* ldy, int32_t vec_dtype, uint32_t flags,
                                          hm_stream_t stream) {
    if (nmat < 0 || (nmat > 0 && (!mats || !X || !ldx || !nrhs || !Y || !ldy))) {
        hm::set_error("hm_mvm_batch_noalloc: null argument");
        return HM_EINVAL;
    }
    if (vec_dtype != HM_F64 && vec_dtype != HM_F32) {
        hm::set_error("hm_mvm_batch_noalloc: vec_dtype must be HM_F64 or HM_F32");
        return HM_EINVAL;
    }
    if ((flags & HM_ADJOINT) && nmat > 0 && mats && nrhs) {
        std::vector<hm_matrix*> adj;
        if (!hm::adjoint_mats(mats, nmat, nrhs, adj, "hm_mvm_batch_noalloc")) return HM_EINVAL;
        return hm_mvm_batch_noalloc(adj.data(), nmat, alpha, X, ldx, nrhs, Y, ldy, vec_dtype, flags & ~HM_ADJOINT,
                                    stream);
    }
    if (flags & ~(uint32_t)HM_CLUSTER_ORDER) {
        hm::set_error("hm_mvm_batch_noalloc: unsupported flags (HM_TIMING allocates events)");
        return HM_EINVAL;
    }
    if (nmat == 0) return HM_OK;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        hm::set_error("hm_mvm_batch_noalloc: no current device");
        return HM_EDEVICE;
    }
    // validate everything and lay the workspaces out before any launch
    std::vector<size_t> off((size_t)nmat, 0);
    size_t total = 0;
    for (int32_t i = 0; i < nmat; ++i) {
        const hm_matrix* m = mats[i];
        if (!m || nrhs[i] < 0 || nrhs[i] > HM_MAX_NRHS) {
            hm::set_error("hm_mvm_batch_noalloc: null matrix or nrhs out of [0, HM_MAX_NRHS] at index " +
                          std::to_string(i));
            return HM_EINVAL;
        }
        if (nrhs[i] == 0) continue;
        if (!X[i] || !Y[i] || X[i] == Y[i] || ldx[i] < m->n || ldy[i] < m->n || m->device != dev) {
            hm::set_error("hm_mvm_batch_noalloc: bad X/Y, leading dimension or device at index " + std::to_string(i));
            return HM_EINVAL;
        }
        for (int32_t k = 0; k < i; ++k)
            if (mats[k] == m && nrhs[k] > 0) {
                hm::set_error("hm_mvm_batch_noalloc: a matrix appears twice");
                return HM_EINVAL;
            }
        if (nrhs[i] == 1 && vec_dtype == HM_F64) continue;   // single-vector kernels: the matrix's own workspace
        if (!m->mr_meta) {
            hm::set_error("hm_mvm_batch_noalloc: the many-RHS plan of matrix " + std::to_string(i) +
                          " is not built (call hm_tune_batch or hm_mvm_batch once beforehand)");
            return HM_EINVAL;
        }
        size_t o1, o2, o3;
        off[(size_t)i] = total;
        total += hm::mr_ws_layout(m, hm::padded_width(nrhs[i]), o1, o2, o3);
    }
    if (total > (size_t)HM_NOALLOC_SCRATCH_BYTES) {
        hm::set_error("hm_mvm_batch_noalloc: the workspaces need " + std::to_string(total) +
                      " bytes, more than HM_NOALLOC_SCRATCH_BYTES = " + std::to_string((long long)HM_NOALLOC_SCRATCH_BYTES));
        return HM_EINVAL;
    }
    uint8_t* base = nullptr;
    hm_status st = hm::scratch_address(dev, &base);
    if (st != HM_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    if (total > 0) {
        const int64_t n16 = (int64_t)(total / 16);
        hipLaunchKernelGGL(hm::k_zero16, dim3((unsigned)std::min<int64_t>((n16 + 255) / 256, 4096)), dim3(256), 0, s,
                           (uint4*)base, n16);
    }
    for (int32_t i = 0; i < nmat; ++i) {
        if (nrhs[i] == 0) continue;
        if (nrhs[i] == 1 && vec_dtype == HM_F64) {
            st = hm_mvm(mats[i], alpha, (const double*)X[i], (double*)Y[i], flags, stream);
        } else {
            size_t o_wsm32, o_ym, o_part;
            (void)hm::mr_ws_layout(mats[i], hm::padded_width(nrhs[i]), o_wsm32, o_ym, o_part);
            uint8_t* b = base + off[(size_t)i];
            const hm::MrWs ws{(double*)b, (float*)(b + o_wsm32), (double*)(b + o_ym), (double*)(b + o_part)};
            st = hm::mvm_many_ws(mats[i], ws, alpha, X[i], ldx[i], nrhs[i], Y[i], ldy[i], vec_dtype, flags, s);
        }
        if (st != HM_OK) return st;
    }
    return HM_OK;
}
