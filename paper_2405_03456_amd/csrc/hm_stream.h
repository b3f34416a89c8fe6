// Device bodies of the hierarchical-matrix product shared by its two
// schedules: one launch per stage (hm_runtime.hip) and one persistent launch
// per product (hm_persist.hip).
//
// A wavefront takes one task of one owner (a leaf row cluster, a low-rank
// block, a cluster basis ...), gives each lane one output row, and walks the
// task's columns.  For column j the lane loads A[r, j] (consecutive lanes
// read consecutive 16-byte chunks of the tiled slab), widens it from its
// storage format, and accumulates A[r, j] * w_j, where w_j = input[j] *
// scale_j is uniform across the wave.  No lane ever reduces with another
// lane, and no output is written by two waves: owners split over several
// tasks write partial sums that are added in a fixed order.
#pragma once

#include <hip/hip_runtime.h>

#include "hm_device.h"

namespace hm {
namespace dev {


// Accumulate one tile row.  WIDE: float64 accumulator with float64 inputs
// w; otherwise float32 accumulator with the float32 mirror of the inputs.
// Columns from `lim` on are the zero data past the item's last column: in
// float32 their weight (a neighbouring input, times a neighbouring scale)
// can overflow, so it is replaced by zero; float64 weights stay finite.
template <int DT, bool WIDE, bool SCALED, typename WT>
__device__ __forceinline__ void tile_acc(const uint4& q, const WT* __restrict__ w, const double* __restrict__ sc,
                                         double& a64, float& a32, int e, int lim) {
    using TT = Tile<DT>;
    typename TT::R v[TT::V];
    TT::decode(q, v, e);
#pragma unroll
    for (int i = 0; i < TT::V; ++i) {
        if (WIDE) {
            double wi = (double)w[i];
            if (SCALED) wi *= sc[i];
            a64 = fma((double)v[i], wi, a64);
        } else {
            float wi = (float)w[i];
            if (SCALED) wi *= (float)sc[i];
            if (i >= lim) wi = 0.0f;
            a32 = fmaf((float)v[i], wi, a32);
        }
    }
}

// Where the current item sits in the owner's tile stream.
struct ItemPos {
    int it, k0, k1, vec, sc, nc;
};

template <int DT>
__device__ __forceinline__ ItemPos item_pos(const DItem* __restrict__ items, int it) {
    const DItem d = items[it];
    constexpr int V = Tile<DT>::V;
    return ItemPos{it, d.tile0, d.tile0 + (d.ncols + V - 1) / V, d.vec_off, d.scale_off, d.ncols};
}

// Data produced and consumed inside one launch (the persistent schedule:
// coefficient vectors and partial sums) moves through device-scope relaxed
// atomic stores and loads, which are coherent across the chip's L2 caches;
// completion counters order them (see k_persistent).  With COH = false
// (one launch per stage) plain accesses suffice: kernel boundaries order them.
template <bool COH>
__device__ __forceinline__ double ld_dev(const double* p) {
    if constexpr (COH)
        return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}

template <bool COH, typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    if constexpr (COH)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

template <bool COH>
__device__ __forceinline__ void finalize(int mode, int out_off, int r, double v, double* __restrict__ vout,
                                         float* __restrict__ vout32, double* __restrict__ y,
                                         const int64_t* __restrict__ perm, double alpha) {
    if (mode == 0) {
        st_dev<COH>(vout + out_off + r, v);
        st_dev<COH>(vout32 + out_off + r, (float)v);
    } else if (mode == 1) {
        y[perm ? perm[out_off + r] : (int64_t)(out_off + r)] += alpha * v;
    } else {
        y[out_off + r] += alpha * v;
    }
}

// Accumulate one tile row with its inputs staged in LDS: entries [off,
// off + V) of the wave's slice, float64 (WIDE) or float32 values.
template <int DT, bool WIDE>
__device__ __forceinline__ void tile_acc_w(const uint4& q, const double* lw, int off, double& a64, float& a32,
                                           int e) {
    using TT = Tile<DT>;
    typename TT::R v[TT::V];
    TT::decode(q, v, e);
    const float* lw32 = reinterpret_cast<const float*>(lw);
#pragma unroll
    for (int i = 0; i < TT::V; ++i) {
        if (WIDE)
            a64 = fma((double)v[i], lw[off + i], a64);
        else
            a32 = fmaf((float)v[i], lw32[off + i], a32);
    }
}

// Stage a task's inputs (times their column scales) in this wave's LDS slice
// in tile order: entry (t - k0) * V + i = input of column i of tile t, a
// float64 value for WIDE tasks, else a float32 value (the slice read as
// float).  With
// `deferred`, an input that is an unreduced sum (dsrc entry != 0) is formed
// here from its partial sums, added in task order.  Past an item's last
// column (the zero data of its last tile) the staged weight is exactly zero:
// the neighbouring input times the neighbouring scale there can overflow
// float32 (a large coefficient next to a large scale), and zero data times
// an infinite weight would be NaN.
// Each lane takes four entries per pass and loads up to four partial sums of
// each at once, so the loads of a pass overlap instead of queueing.  With
// COH, entries at or above nx (coefficients) and partial sums are read with
// coherent loads: they may have been written earlier in the same launch.
// Without WIDE the staged value is the float32 product of the float32 input
// and the float32 scale, exactly the weight the unstaged path forms, so a
// task's result does not depend on whether it stages.
template <int DT, bool WIDE, bool COH>
__device__ __forceinline__ void stage_inputs(const DTask& tk, const DItem* __restrict__ items, int lane,
                                             bool deferred, const double* __restrict__ vin,
                                             const double* __restrict__ scales, const int64_t* __restrict__ dsrc,
                                             const double* part, double* __restrict__ lw, int nx) {
    constexpr int V = Tile<DT>::V;
    constexpr int CH = 4;
    const int k0 = tk.k0;
    const int nval = (tk.k1 - k0) * V;
    ItemPos st = item_pos<DT>(items, tk.item_start);
    for (int base = lane; base < nval; base += 64 * CH) {
        int e[CH], sc[CH];
        bool in[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int idx = min(base + u * 64, nval - 1);   // a clamped entry is staged twice, same value
            const int t = k0 + idx / V;
            while (t >= st.k1) st = item_pos<DT>(items, st.it + 1);
            const int c = (t - st.k0) * V + idx % V;
            e[u] = st.vec + c;
            sc[u] = st.sc >= 0 ? st.sc + c : -1;
            in[u] = c < st.nc;
        }
        int64_t d[CH];
        double v[CH], f[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            d[u] = deferred && in[u] ? dsrc[e[u]] : 0;
            v[u] = (COH && e[u] >= nx) ? ld_dev<true>(vin + e[u]) : vin[e[u]];
            f[u] = sc[u] >= 0 ? scales[sc[u]] : 1.0;
        }
        if (deferred) {
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                if (d[u] == 0) continue;
                const double* p = part + (uint32_t)d[u];
                const int cnt = (int)(((uint64_t)d[u] >> 32) & 0xffff);
                const int64_t stride = (int64_t)((uint64_t)d[u] >> 48);
                double acc = 0.0;
                for (int l = 0; l < cnt; l += 4) {
                    double q[4];
#pragma unroll
                    for (int w = 0; w < 4; ++w) q[w] = l + w < cnt ? ld_dev<COH>(p + (l + w) * stride) : 0.0;
#pragma unroll
                    for (int w = 0; w < 4; ++w) acc += q[w];
                }
                v[u] = acc;
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int idx = base + u * 64;
            if (idx < nval) {
                if (WIDE)
                    lw[idx] = in[u] ? v[u] * f[u] : 0.0;
                else
                    reinterpret_cast<float*>(lw)[idx] = in[u] ? (float)v[u] * (float)f[u] : 0.0f;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wide owners (more than 32 rows): the wave walks the task's tiles together,
// a prefetched batch of U tiles always in flight.  Unstaged, the item
// bookkeeping is uniform and the inputs are scalar loads (lgkmcnt), so
// waiting for them never drains the data prefetch (vmcnt); STAGED, the
// inputs (times their scales) are first staged in LDS, after the first
// tiles have been requested.
template <int DT, bool WIDE, bool STAGED, bool COH>
__device__ __forceinline__ void stream_uniform(const DTask& tk, const DItem* __restrict__ items,
                                               const uint8_t* __restrict__ sb, int64_t rt, int lane,
                                               const double* __restrict__ vin, const float* __restrict__ vin32,
                                               const double* __restrict__ scales, const int64_t* __restrict__ dsrc,
                                               const double* part, double* __restrict__ lw, double& a64,
                                               float& a32, int nx, int e, bool deferred) {
    constexpr int V = Tile<DT>::V;
    constexpr int U = Tile<DT>::V <= 4 ? 8 : 4;
    const int k0 = tk.k0, k1 = tk.k1;
    ItemPos st = item_pos<DT>(items, tk.item_start);
    uint4 qa[U], qb[U];
    auto issue = [&](uint4* q, int kb) {
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = *reinterpret_cast<const uint4*>(sb + (int64_t)min(kb + u, k1 - 1) * rt);
    };
    auto consume = [&](const uint4* q, int kb) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kk = kb + u;
            if (STAGED) {
                if (kk < k1) tile_acc_w<DT, WIDE>(q[u], lw, (kk - k0) * V, a64, a32, e);
                continue;
            }
            if (kk < k1) {
                while (kk >= st.k1) st = item_pos<DT>(items, st.it + 1);
                const int c = (kk - st.k0) * V;
                const int lim = st.nc - c;
                if (WIDE) {
                    if (st.sc >= 0)
                        tile_acc<DT, true, true>(q[u], vin + st.vec + c, scales + st.sc + c, a64, a32, e, lim);
                    else
                        tile_acc<DT, true, false>(q[u], vin + st.vec + c, scales, a64, a32, e, lim);
                } else {
                    if (st.sc >= 0)
                        tile_acc<DT, false, true>(q[u], vin32 + st.vec + c, scales + st.sc + c, a64, a32, e, lim);
                    else
                        tile_acc<DT, false, false>(q[u], vin32 + st.vec + c, scales, a64, a32, e, lim);
                }
            }
        }
    };
    issue(qa, k0);
    if (STAGED) stage_inputs<DT, WIDE, COH>(tk, items, lane, deferred, vin, scales, dsrc, part, lw, nx);
    for (int k = k0; k < k1; k += 2 * U) {
        issue(qb, k + U);
        __builtin_amdgcn_sched_barrier(0);
        consume(qa, k);
        issue(qa, k + 2 * U);
        __builtin_amdgcn_sched_barrier(0);
        consume(qb, k + U);
    }
}

// Narrow owners (at most 32 rows): G = 64/P lane groups take tiles
// k0+g, k0+g+G, ...  The task's inputs (times their column scales) are first
// staged in this wave's LDS slice in tile order, so each lane reads its
// group's inputs from LDS and the data prefetch is never drained.
template <int DT, bool WIDE, bool COH>
__device__ __forceinline__ void stream_grouped(const DTask& tk, const DItem* __restrict__ items,
                                               const uint8_t* __restrict__ sb, int64_t rt, int g, int G, int lane,
                                               bool deferred, const double* __restrict__ vin,
                                               const double* __restrict__ scales, const int64_t* __restrict__ dsrc,
                                               const double* part, double* __restrict__ lw, double& a64,
                                               float& a32, int nx, int e) {
    constexpr int V = Tile<DT>::V;
    constexpr int U = 4;
    const int k0 = tk.k0, k1 = tk.k1;
    const int step = U * G;
    uint4 qa[U], qb[U];
    auto issue = [&](uint4* q, int kb) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            q[u] = *reinterpret_cast<const uint4*>(sb + (int64_t)min(kb + u * G + g, k1 - 1) * rt);
    };
    // the first tiles are requested before the inputs are staged, so both
    // memory latencies overlap
    issue(qa, k0);
    stage_inputs<DT, WIDE, COH>(tk, items, lane, deferred, vin, scales, dsrc, part, lw, nx);
    auto consume = [&](const uint4* q, int kb) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kk = kb + u * G + g;
            if (kk < k1) tile_acc_w<DT, WIDE>(q[u], lw, (kk - k0) * V, a64, a32, e);
        }
    };
    for (int k = k0; k < k1; k += 2 * step) {
        issue(qb, k + step);
        __builtin_amdgcn_sched_barrier(0);
        consume(qa, k);
        issue(qa, k + 2 * step);
        __builtin_amdgcn_sched_barrier(0);
        consume(qb, k + step);
    }
}

template <int DT, bool ACC64, bool COH>
__device__ __forceinline__ void stream_task(const DTask& tk, const DItem* items, const uint8_t* sb, int64_t rt,
                                            int g, int G, int lane, bool deferred, const double* vin,
                                            const float* vin32, const double* scales, const int64_t* dsrc,
                                            const double* part, double* lw, double& a64, float& a32, int nx) {
    constexpr bool WIDE = ACC64 || kWide<DT>;
    // formats whose columns carry a scale (FP16, FP8, AFLP) stage their
    // weights (input times scale, once per column and wave) instead of
    // loading every column's scale in every lane's loop: measured faster
    constexpr bool kScaled = DT == HM_F16 || DT == HM_FP8E4M3 || DT >= HM_AFLP8;
    const int e = task_ebits(tk.mode);
    if (G == 1) {
        if (deferred || kScaled)
            stream_uniform<DT, WIDE, true, COH>(tk, items, sb, rt, lane, vin, vin32, scales, dsrc, part, lw, a64,
                                                a32, nx, e, deferred);
        else
            stream_uniform<DT, WIDE, false, COH>(tk, items, sb, rt, lane, vin, vin32, scales, dsrc, part, lw, a64,
                                                 a32, nx, e, false);
    } else {
        stream_grouped<DT, WIDE, COH>(tk, items, sb, rt, g, G, lane, deferred, vin, scales, dsrc, part, lw, a64,
                                      a32, nx, e);
    }
}

// One task: one wavefront, lane geometry P = rows per group (next power of
// two >= nrows, at most 64), G = 64 / P column groups.  Tasks hold one dtype.
// MASK: bit d set = tasks of dtype d may occur (the instantiation is chosen
// by the host from the dtypes of the launched tasks).  Bit 2 of the task's
// mode: its inputs are staged (some are unreduced sums, or, with COH,
// produced in the same launch).  Results go to the output when the owner has
// one task, else to the task's slot of partial sums.
template <bool ACC64, int MASK, bool COH>
__device__ __forceinline__ void run_task(const DTask& tk, int lane, double* __restrict__ lw,
                                         const DItem* __restrict__ items, const uint8_t* __restrict__ data,
                                         const double* __restrict__ scales, const double* __restrict__ vin,
                                         const float* __restrict__ vin32, double* vout, float* vout32,
                                         double* __restrict__ part, const int64_t* __restrict__ dsrc,
                                         double* __restrict__ y, const int64_t* __restrict__ perm, double alpha,
                                         int nx, double* ypriv, int64_t npriv) {
    const int nrows = tk.nrows;
    int lp = 0;                         // log2 P
    while ((1 << lp) < nrows && lp < 6) ++lp;
    const int P = 1 << lp;
    const int G = 64 >> lp;
    const int g = lane >> lp;
    const int rl = lane & (P - 1);
    const int dt = tk.dtype;   // in the descriptor: no dependent item load before the tiles
    const int mode = tk.mode & 3;
    const bool deferred = (tk.mode & 4) != 0;   // some inputs are unreduced sums
    for (int r0 = 0; r0 < nrows; r0 += P) {
        const int r = r0 + rl;
        const bool act = r < nrows;
        const int rr = act ? r : nrows - 1;   // idle lanes re-read a valid row
        double a64 = 0.0;
        float a32 = 0.0f;
        const int64_t rt = (int64_t)nrows * 16;
        const uint8_t* sb = data + tk.stream + (uint32_t)(rr * 16);
#define HM_STREAM_CASE(D)                                                                                \
    if constexpr ((MASK & (1 << D)) != 0)                                                                \
        if (dt == D)                                                                                     \
            stream_task<D, ACC64, COH>(tk, items, sb, rt, g, G, lane, deferred, vin, vin32, scales, dsrc, part, lw, \
                                       a64, a32, nx);
        HM_STREAM_CASE(HM_F64)
        HM_STREAM_CASE(HM_F32)
        HM_STREAM_CASE(HM_BF16)
        HM_STREAM_CASE(HM_F16)
        HM_STREAM_CASE(HM_FP8E4M3)
        HM_STREAM_CASE(HM_FPX24)
        HM_STREAM_CASE(HM_FPX40)
        HM_STREAM_CASE(HM_FPX48)
        HM_STREAM_CASE(HM_FPX56)
        HM_STREAM_CASE(HM_AFLP8)
        HM_STREAM_CASE(HM_AFLP16)
        HM_STREAM_CASE(HM_AFLP24)
        HM_STREAM_CASE(HM_AFLP32)
        HM_STREAM_CASE(HM_AFLP40)
        HM_STREAM_CASE(HM_AFLP48)
        HM_STREAM_CASE(HM_AFLP56)
#undef HM_STREAM_CASE
        double v = a64 + (double)a32;
        for (int off = P; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);   // across column groups
        if (act && g == 0) {
            if (tk.rscale_off >= 0) v *= scales[tk.rscale_off + r];
            if (tk.mode & 8) {
                // atomic synchronisation (Sec. 3.1's alternative to row
                // ownership): every task adds its rows with float64 atomics,
                // into y, into the coefficient vector (zeroed at the start),
                // or (mode bit 16) into one of eight private copies of y
                // (cluster order) that a final launch sums
                if (mode == 0)
                    atomicAdd(vout + tk.out_off + r, v);
                else if (tk.mode & 16)
                    atomicAdd(ypriv + (int64_t)(blockIdx.x & 7) * npriv + tk.out_off + r, v);
                else
                    atomicAdd(y + (mode == 1 && perm ? perm[tk.out_off + r] : (int64_t)(tk.out_off + r)),
                              alpha * v);
            } else if (tk.ntasks == 1) {
                finalize<COH>(mode, tk.out_off, r, v, vout, vout32, y, perm, alpha);
            } else {
                st_dev<COH>(part + tk.part_off + (int64_t)tk.local * nrows + r, v);
            }
        }
    }
}

// Sum the partial results of one split owner in a fixed order (one wave):
// P lanes per row group, the G = 64 / P groups take tasks g, g + G, ...
template <bool COH>
__device__ __forceinline__ void run_reduce(const DOwner& ow, int lane, const double* __restrict__ part,
                                           double* vout, float* vout32, double* __restrict__ y,
                                           const int64_t* __restrict__ perm, double alpha) {
    // P lanes per row group (next power of two >= nrows, at most 64); the
    // G = 64 / P groups take tasks g, g + G, ... with two independent sums
    // each, combined across groups by shuffles (a fixed order: deterministic)
    const int nrows = ow.nrows, nt = ow.ntasks;
    int lp = 0;
    while ((1 << lp) < nrows && lp < 6) ++lp;
    const int P = 1 << lp, G = 64 >> lp, g = lane >> lp, rl = lane & (P - 1);
    for (int r0 = 0; r0 < nrows; r0 += P) {
        const int r = r0 + rl;
        const bool act = r < nrows;
        // y owners: the destination is read before the partial sums, so
        // its latency overlaps theirs
        double* yp = nullptr;
        double y0 = 0.0;
        if (act && g == 0 && ow.mode != 0) {
            yp = y + (ow.mode == 1 && perm ? perm[ow.out_off + r] : (int64_t)(ow.out_off + r));
            y0 = *yp;
        }
        // eight sums, each over every 8G-th partial: the loads of a pass are
        // independent (missing ones read as zero)
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (act) {
            const double* p = part + ow.part_off + r;
            for (int l = g; l < nt; l += 8 * G) {
                double q[8];
#pragma unroll
                for (int w = 0; w < 8; ++w) q[w] = l + w * G < nt ? ld_dev<COH>(p + (int64_t)(l + w * G) * nrows) : 0.0;
#pragma unroll
                for (int w = 0; w < 8; ++w) acc[w] += q[w];
            }
        }
        double v = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        for (int off = P; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
        if (act && g == 0) {
            if (yp)
                *yp = y0 + alpha * v;
            else
                finalize<COH>(ow.mode, ow.out_off, r, v, vout, vout32, y, perm, alpha);
        }
    }
}

// One launch of a stage: one wavefront per task.  MASK: the dtypes of the
// stage's tasks (the host launches the instantiation for that set).
template <bool ACC64, int MASK>
__global__ __launch_bounds__(256) void k_owner_tasks(
    const DTask* __restrict__ tasks, int ntasks, const DOwner* __restrict__ owners,
    const DItem* __restrict__ items, const uint8_t* __restrict__ data, const double* __restrict__ scales,
    const double* __restrict__ vin, const float* __restrict__ vin32, double* vout, float* vout32,
    double* __restrict__ part, const int64_t* __restrict__ dsrc, double* __restrict__ y,
    const int64_t* __restrict__ perm, double alpha, double* ypriv, int64_t npriv) {
    __shared__ double lds_w[4][MAX_TASK_INPUTS];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    (void)owners;
    // a grid smaller than the task count makes each wave walk tasks
    // t, t + stride, ... (used to leave compute units to a concurrent stage)
    for (int t = blockIdx.x * 4 + wave; t < ntasks; t += gridDim.x * 4)
        run_task<ACC64, MASK, false>(tasks[t], lane, lds_w[wave], items, data, scales, vin, vin32, vout, vout32,
                                     part, dsrc, y, perm, alpha, 0, ypriv, npriv);
}

using TaskKernel = void (*)(const DTask*, int, const DOwner*, const DItem*, const uint8_t*, const double*,
                            const double*, const float*, double*, float*, double*, const int64_t*, double*,
                            const int64_t*, double, double*, int64_t);

// Instantiated dtype sets for stages holding codec formats (hm_tasks_codec_*):
// one codec with FP64 (the FP64 diagonal near field beside it), then whole
// families; task_kernel takes the first that contains a stage's set.
constexpr int kCodecMasks[14] = {
    (1 << HM_FPX24) | 1,  (1 << HM_FPX40) | 1,  (1 << HM_FPX48) | 1,  (1 << HM_FPX56) | 1,  (1 << HM_AFLP8) | 1,
    (1 << HM_AFLP16) | 1, (1 << HM_AFLP24) | 1, (1 << HM_AFLP32) | 1, (1 << HM_AFLP40) | 1, (1 << HM_AFLP48) | 1,
    (1 << HM_AFLP56) | 1, kMaskFpx,             kMaskAflp,            kMaskAll};

// k_owner_tasks<acc64, mask> (instantiated in hm_tasks_*.hip)
TaskKernel task_kernel(bool acc64, int mask);

// Persistent schedule (hm_persist.hip): the kernel for a set of dtypes (the
// instantiated superset is returned in *launched_mask; nullptr if none).
using PersistKernel = void (*)(const int32_t*, int, const int32_t*, const int32_t*, const int32_t*, int32_t*,
                               uint32_t*, uint64_t, const DTask*, const DOwner*, const DItem*, const uint8_t*,
                               const double*, const double*, const float*, double*, float*, double*,
                               const int64_t*, double*, const int64_t*, double, int, int);
PersistKernel persist_kernel(bool acc64, int mask, int* launched_mask);
__global__ void k_gather_reset(const double* __restrict__ x, const int64_t* __restrict__ perm,
                               double* __restrict__ ws, float* __restrict__ ws32, int64_t n, int cluster_order,
                               int32_t* __restrict__ done, int64_t ndone, uint32_t* __restrict__ ctl);

}  // namespace dev
}  // namespace hm
