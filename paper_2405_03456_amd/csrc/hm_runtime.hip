// Device engine of the hierarchical-matrix product on gfx950.
//
// One kernel does all the matrix streaming: a wavefront takes one task of one
// owner (a leaf row cluster, a low-rank block, a cluster basis ...), gives
// each lane one output row, and walks the task's columns.  For column j the
// lane loads A[r, j] (consecutive lanes read consecutive addresses of the
// column-major slab), widens it from its storage format, and accumulates
// A[r, j] * w_j, where w_j = input[j] * scale_j is uniform across the wave.
// No lane ever reduces with another lane, and no output is written by two
// waves: owners split over several tasks write partial sums that are added
// in a fixed order, by a reduction kernel (y owners, and coefficient owners
// of stages with long owners) or by every later task that reads them while
// it stages its inputs.  The product is therefore deterministic.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <utility>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hm_device.h"

namespace hm {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

namespace dev {


// Accumulate one tile row.  WIDE: float64 accumulator with float64 inputs
// w; otherwise float32 accumulator with the float32 mirror of the inputs.
template <int DT, bool WIDE, bool SCALED, typename WT>
__device__ __forceinline__ void tile_acc(const uint4& q, const WT* __restrict__ w, const double* __restrict__ sc,
                                         double& a64, float& a32) {
    using TT = Tile<DT>;
    typename TT::R v[TT::V];
    TT::decode(q, v);
#pragma unroll
    for (int i = 0; i < TT::V; ++i) {
        if (WIDE) {
            double wi = (double)w[i];
            if (SCALED) wi *= sc[i];
            a64 = fma((double)v[i], wi, a64);
        } else {
            float wi = (float)w[i];
            if (SCALED) wi *= (float)sc[i];
            a32 = fmaf((float)v[i], wi, a32);
        }
    }
}

// Where the current item sits in the owner's tile stream.
struct ItemPos {
    int it, k0, k1, vec, sc;
};

template <int DT>
__device__ __forceinline__ ItemPos item_pos(const DItem* __restrict__ items, int it) {
    const DItem d = items[it];
    constexpr int V = Tile<DT>::V;
    return ItemPos{it, d.tile0, d.tile0 + (d.ncols + V - 1) / V, d.vec_off, d.scale_off};
}

__device__ __forceinline__ void finalize(int mode, int out_off, int r, double v, double* __restrict__ vout,
                                         float* __restrict__ vout32, double* __restrict__ y,
                                         const int64_t* __restrict__ perm, double alpha) {
    if (mode == 0) {
        vout[out_off + r] = v;
        vout32[out_off + r] = (float)v;
    } else if (mode == 1) {
        y[perm ? perm[out_off + r] : (int64_t)(out_off + r)] += alpha * v;
    } else {
        y[out_off + r] += alpha * v;
    }
}

// Accumulate one tile row with inputs already in registers/LDS (grouped path).
template <int DT, bool WIDE>
__device__ __forceinline__ void tile_acc_w(const uint4& q, const double* wv, double& a64, float& a32) {
    using TT = Tile<DT>;
    typename TT::R v[TT::V];
    TT::decode(q, v);
#pragma unroll
    for (int i = 0; i < TT::V; ++i) {
        if (WIDE)
            a64 = fma((double)v[i], wv[i], a64);
        else
            a32 = fmaf((float)v[i], (float)wv[i], a32);
    }
}

// Stage a task's inputs (times their column scales) in this wave's LDS slice
// in tile order: lw[(t - k0) * V + i] = input of column i of tile t.  With
// `deferred`, an input that is an unreduced sum (dsrc entry != 0) is formed
// here from its partial sums, added in task order.  Past an item's last
// column the values are not needed (its data is zero) but are finite.
// Each lane takes four entries per pass and loads up to four partial sums of
// each at once, so the loads of a pass overlap instead of queueing.
template <int DT>
__device__ __forceinline__ void stage_inputs(const DTask& tk, const DItem* __restrict__ items, int lane,
                                             bool deferred, const double* __restrict__ vin,
                                             const double* __restrict__ scales, const int64_t* __restrict__ dsrc,
                                             const double* part, double* __restrict__ lw) {
    constexpr int V = Tile<DT>::V;
    constexpr int CH = 4;
    const int k0 = tk.k0;
    const int nval = (tk.k1 - k0) * V;
    ItemPos st = item_pos<DT>(items, tk.item_start);
    for (int base = lane; base < nval; base += 64 * CH) {
        int e[CH], sc[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int idx = min(base + u * 64, nval - 1);   // a clamped entry is staged twice, same value
            const int t = k0 + idx / V;
            while (t >= st.k1) st = item_pos<DT>(items, st.it + 1);
            const int c = (t - st.k0) * V + idx % V;
            e[u] = st.vec + c;
            sc[u] = st.sc >= 0 ? st.sc + c : -1;
        }
        int64_t d[CH];
        double v[CH], f[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            d[u] = deferred ? dsrc[e[u]] : 0;
            v[u] = vin[e[u]];
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
                    for (int w = 0; w < 4; ++w) q[w] = l + w < cnt ? p[(l + w) * stride] : 0.0;
#pragma unroll
                    for (int w = 0; w < 4; ++w) acc += q[w];
                }
                v[u] = acc;
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int idx = base + u * 64;
            if (idx < nval) lw[idx] = v[u] * f[u];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wide owners (more than 32 rows): the wave walks the task's tiles together,
// a prefetched batch of U tiles always in flight; item bookkeeping is
// uniform and the inputs are scalar loads (lgkmcnt), so waiting for them
// never drains the data prefetch (vmcnt).
template <int DT, bool WIDE, bool STAGED>
__device__ __forceinline__ void stream_uniform(const DTask& tk, const DItem* __restrict__ items,
                                               const uint8_t* __restrict__ sb, int64_t rt, int lane,
                                               const double* __restrict__ vin, const float* __restrict__ vin32,
                                               const double* __restrict__ scales, const int64_t* __restrict__ dsrc,
                                               const double* part, double* __restrict__ lw, double& a64,
                                               float& a32) {
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
                if (kk < k1) tile_acc_w<DT, WIDE>(q[u], lw + (kk - k0) * V, a64, a32);
                continue;
            }
            if (kk < k1) {
                while (kk >= st.k1) st = item_pos<DT>(items, st.it + 1);
                const int c = (kk - st.k0) * V;
                if (WIDE) {
                    if (st.sc >= 0)
                        tile_acc<DT, true, true>(q[u], vin + st.vec + c, scales + st.sc + c, a64, a32);
                    else
                        tile_acc<DT, true, false>(q[u], vin + st.vec + c, scales, a64, a32);
                } else {
                    if (st.sc >= 0)
                        tile_acc<DT, false, true>(q[u], vin32 + st.vec + c, scales + st.sc + c, a64, a32);
                    else
                        tile_acc<DT, false, false>(q[u], vin32 + st.vec + c, scales, a64, a32);
                }
            }
        }
    };
    issue(qa, k0);
    if (STAGED) stage_inputs<DT>(tk, items, lane, true, vin, scales, dsrc, part, lw);
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
template <int DT, bool WIDE>
__device__ __forceinline__ void stream_grouped(const DTask& tk, const DItem* __restrict__ items,
                                               const uint8_t* __restrict__ sb, int64_t rt, int g, int G, int lane,
                                               bool deferred, const double* __restrict__ vin,
                                               const double* __restrict__ scales, const int64_t* __restrict__ dsrc,
                                               const double* part, double* __restrict__ lw, double& a64,
                                               float& a32) {
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
    stage_inputs<DT>(tk, items, lane, deferred, vin, scales, dsrc, part, lw);
    auto consume = [&](const uint4* q, int kb) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kk = kb + u * G + g;
            if (kk < k1) tile_acc_w<DT, WIDE>(q[u], lw + (kk - k0) * V, a64, a32);
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

template <int DT, bool ACC64>
__device__ __forceinline__ void stream_task(const DTask& tk, const DItem* items, const uint8_t* sb, int64_t rt,
                                            int g, int G, int lane, bool deferred, const double* vin,
                                            const float* vin32, const double* scales, const int64_t* dsrc,
                                            const double* part, double* lw, double& a64, float& a32) {
    constexpr bool WIDE = ACC64 || DT == HM_F64;
    if (G == 1) {
        if (deferred)
            stream_uniform<DT, WIDE, true>(tk, items, sb, rt, lane, vin, vin32, scales, dsrc, part, lw, a64, a32);
        else
            stream_uniform<DT, WIDE, false>(tk, items, sb, rt, lane, vin, vin32, scales, dsrc, part, lw, a64, a32);
    } else {
        stream_grouped<DT, WIDE>(tk, items, sb, rt, g, G, lane, deferred, vin, scales, dsrc, part, lw, a64, a32);
    }
}

// One wavefront per task.  Lane geometry: P = rows per group (next power of
// two >= nrows, at most 64), G = 64 / P column groups.  Tasks hold one dtype.
// MASK: bit d set = tasks of dtype d may occur in the launched stage; the
// host launches the instantiation whose mask is the stage's dtype set.
template <bool ACC64, int MASK>
__global__ __launch_bounds__(256) void k_owner_tasks(
    const DTask* __restrict__ tasks, int ntasks, const DOwner* __restrict__ owners,
    const DItem* __restrict__ items, const uint8_t* __restrict__ data, const double* __restrict__ scales,
    const double* __restrict__ vin, const float* __restrict__ vin32, double* vout, float* vout32,
    double* __restrict__ part, const int64_t* __restrict__ dsrc, double* __restrict__ y,
    const int64_t* __restrict__ perm, double alpha) {
    __shared__ double lds_w[4][MAX_TASK_INPUTS];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // a grid smaller than the task count makes each wave walk tasks
    // t, t + stride, ... (used to leave compute units to a concurrent stage)
    for (int t = blockIdx.x * 4 + wave; t < ntasks; t += gridDim.x * 4) {
    const DTask tk = tasks[t];
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
        double* lw = lds_w[wave];
        if constexpr ((MASK & (1 << HM_F64)) != 0)
            if (dt == HM_F64)
                stream_task<HM_F64, ACC64>(tk, items, sb, rt, g, G, lane, deferred, vin, vin32, scales, dsrc, part, lw,
                                           a64, a32);
        if constexpr ((MASK & (1 << HM_F32)) != 0)
            if (dt == HM_F32)
                stream_task<HM_F32, ACC64>(tk, items, sb, rt, g, G, lane, deferred, vin, vin32, scales, dsrc, part, lw,
                                           a64, a32);
        if constexpr ((MASK & (1 << HM_BF16)) != 0)
            if (dt == HM_BF16)
                stream_task<HM_BF16, ACC64>(tk, items, sb, rt, g, G, lane, deferred, vin, vin32, scales, dsrc, part, lw,
                                            a64, a32);
        if constexpr ((MASK & (1 << HM_F16)) != 0)
            if (dt == HM_F16)
                stream_task<HM_F16, ACC64>(tk, items, sb, rt, g, G, lane, deferred, vin, vin32, scales, dsrc, part, lw,
                                           a64, a32);
        if constexpr ((MASK & (1 << HM_FP8E4M3)) != 0)
            if (dt == HM_FP8E4M3)
                stream_task<HM_FP8E4M3, ACC64>(tk, items, sb, rt, g, G, lane, deferred, vin, vin32, scales, dsrc, part,
                                               lw, a64, a32);
        double v = a64 + (double)a32;
        for (int off = P; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);   // across column groups
        if (act && g == 0) {
            if (tk.rscale_off >= 0) v *= scales[tk.rscale_off + r];
            if (tk.ntasks == 1)
                finalize(mode, tk.out_off, r, v, vout, vout32, y, perm, alpha);
            else
                part[tk.part_off + (int64_t)tk.local * nrows + r] = v;
        }
    }
    }
}

// Sum the partial results of split owners in a fixed order, one wave per owner.
__global__ __launch_bounds__(256) void k_reduce(const int32_t* __restrict__ list, int nlist,
                                                const DOwner* __restrict__ owners,
                                                const double* __restrict__ part, double* vout, float* vout32,
                                                double* __restrict__ y, const int64_t* __restrict__ perm,
                                                double alpha) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nlist) return;
    const DOwner ow = owners[list[i]];
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
                for (int w = 0; w < 8; ++w) q[w] = l + w * G < nt ? p[(int64_t)(l + w * G) * nrows] : 0.0;
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
                finalize(ow.mode, ow.out_off, r, v, vout, vout32, y, perm, alpha);
        }
    }
}

// x in cluster order: ws[i] = x[perm[i]]  (or a straight copy)
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ x, const int64_t* __restrict__ perm,
                                                double* __restrict__ ws, float* __restrict__ ws32, int64_t n,
                                                int cluster_order) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const double v = cluster_order ? x[i] : x[perm[i]];
        ws[i] = v;
        ws32[i] = (float)v;
    }
}

using TaskKernel = void (*)(const DTask*, int, const DOwner*, const DItem*, const uint8_t*, const double*,
                           const double*, const float*, double*, float*, double*, const int64_t*, double*,
                           const int64_t*, double);

template <bool ACC64, int... M>
constexpr std::array<TaskKernel, sizeof...(M)> task_kernels(std::integer_sequence<int, M...>) {
    return {{&k_owner_tasks<ACC64, M>...}};
}

// [acc64][dtype mask]
static const std::array<TaskKernel, 32> kTasks[2] = {task_kernels<false>(std::make_integer_sequence<int, 32>{}),
                                                      task_kernels<true>(std::make_integer_sequence<int, 32>{})};

}  // namespace dev


}  // namespace hm



using hm::align256;
using hm::hip_fail;

extern "C" const char* hm_last_error(void) { return hm::g_err.c_str(); }
extern "C" const char* hm_version(void) { return "hm 0.1 gfx950"; }

extern "C" hm_status hm_upload(const hm_layout* layout, int32_t format, const hm_values* values,
                               const hm_precision* prec, const hm_upload_opts* opts, hm_stream_t stream,
                               hm_matrix** out) {
    (void)stream;
    if (!layout || !values || !prec || !out) {
        hm::set_error("hm_upload: null argument");
        return HM_EINVAL;
    }
    *out = nullptr;
    hm::Packed P;
    hm::PackOptions opt;
    hm_status st = hm::pack_options(opts, opt);
    if (st != HM_OK) return st;
    try {
        st = hm::pack(layout->L, format, values, prec, opt, P);
    } catch (const std::bad_alloc&) {
        hm::set_error("hm_upload: out of host memory while packing");
        return HM_ENOMEM;
    }
    if (st != HM_OK) return st;

    // one device allocation: metadata | perm | data | scales | workspace | partials
    size_t meta = 0;
    const size_t o_owners = meta;
    meta = align256(meta + P.owners.size() * sizeof(hm::DOwner));
    const size_t o_items = meta;
    meta = align256(meta + P.items.size() * sizeof(hm::DItem));
    const size_t o_tasks = meta;
    meta = align256(meta + P.tasks.size() * sizeof(hm::DTask));
    // the single-vector product launches reductions for y owners only
    std::vector<size_t> o_red;
    for (auto& st : P.stages) {
        o_red.push_back(meta);
        meta = align256(meta + st.reduce_launch.size() * sizeof(int32_t));
    }
    const size_t o_dsrc = meta;
    meta = align256(meta + P.dsrc.size() * sizeof(int64_t));
    const int64_t n = layout->L.n;
    size_t o_perm = meta;
    size_t o_data = align256(o_perm + n * sizeof(int64_t));
    // scales and workspace carry TILE_PAD trailing entries (see hm_plan.h)
    P.scales.resize(P.scales.size() + hm::TILE_PAD, 0.0);
    size_t o_scales = align256(o_data + P.data.size());
    size_t o_ws = align256(o_scales + P.scales.size() * sizeof(double));
    size_t o_ws32 = align256(o_ws + (P.ws_elems + hm::TILE_PAD) * sizeof(double));
    size_t o_part = align256(o_ws32 + (P.ws_elems + hm::TILE_PAD) * sizeof(float));
    size_t total = align256(o_part + std::max<int64_t>(P.part_elems, 1) * sizeof(double));

    hm_matrix* m = new (std::nothrow) hm_matrix();
    if (!m) {
        hm::set_error("hm_upload: out of host memory");
        return HM_ENOMEM;
    }
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) {
        delete m;
        return hip_fail("hipGetDevice", e);
    }
    e = hipMalloc(&m->arena, total);
    if (e != hipSuccess) {
        delete m;
        hm::set_error("hm_upload: hipMalloc of " + std::to_string(total) + " bytes failed");
        return HM_ENOMEM;
    }
    uint8_t* base = (uint8_t*)m->arena;
    auto copy = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpy(base + off, src, bytes, hipMemcpyHostToDevice);
    };
    // device task table: mode bit 2 marks tasks that stage their inputs
    // through the deferred-sum table
    std::vector<hm::DTask> dtasks = P.tasks;
    for (size_t k = 0; k < dtasks.size(); ++k)
        if (P.staged[k]) dtasks[k].mode = (int16_t)(dtasks[k].mode | 4);
    e = copy(o_owners, P.owners.data(), P.owners.size() * sizeof(hm::DOwner));
    if (e == hipSuccess) e = copy(o_items, P.items.data(), P.items.size() * sizeof(hm::DItem));
    if (e == hipSuccess) e = copy(o_tasks, dtasks.data(), dtasks.size() * sizeof(hm::DTask));
    for (size_t i = 0; i < P.stages.size() && e == hipSuccess; ++i)
        e = copy(o_red[i], P.stages[i].reduce_launch.data(), P.stages[i].reduce_launch.size() * sizeof(int32_t));
    if (e == hipSuccess) e = copy(o_dsrc, P.dsrc.data(), P.dsrc.size() * sizeof(int64_t));
    if (e == hipSuccess) e = copy(o_perm, layout->L.perm.data(), n * sizeof(int64_t));
    if (e == hipSuccess) e = copy(o_data, P.data.data(), P.data.size());
    if (e == hipSuccess) e = copy(o_scales, P.scales.data(), P.scales.size() * sizeof(double));
    // every workspace entry must hold a finite value before the first product:
    // zero-data padding columns multiply whatever they read
    if (e == hipSuccess) e = hipMemset(base + o_ws, 0, (P.ws_elems + hm::TILE_PAD) * sizeof(double));
    if (e == hipSuccess) e = hipMemset(base + o_ws32, 0, (P.ws_elems + hm::TILE_PAD) * sizeof(float));
    // partial sums too: a padding column may read an unreduced sum
    if (e == hipSuccess) e = hipMemset(base + o_part, 0, std::max<int64_t>(P.part_elems, 1) * sizeof(double));
    if (e != hipSuccess) {
        (void)hipFree(m->arena);
        delete m;
        return hip_fail("hm_upload: hipMemcpy", e);
    }
    m->layout = layout;
    m->format = format;
    m->acc64 = P.acc64;
    m->n = n;
    m->arena_bytes = total;
    m->perm = (int64_t*)(base + o_perm);
    m->data = base + o_data;
    m->scales = (double*)(base + o_scales);
    m->ws = (double*)(base + o_ws);
    m->ws32 = (float*)(base + o_ws32);
    m->part = (double*)(base + o_part);
    m->dsrc = (const int64_t*)(base + o_dsrc);
    m->owners = (const hm::DOwner*)(base + o_owners);
    m->items = (const hm::DItem*)(base + o_items);
    m->tasks = (const hm::DTask*)(base + o_tasks);
    int32_t nlaunch = 1;
    for (size_t i = 0; i < P.stages.size(); ++i) {
        auto& st = P.stages[i];
        hm::DevStage d;
        d.aux = st.aux;
        d.t0 = st.t0;
        d.ntasks = (int32_t)(st.t1 - st.t0);
        d.reduce = (const int32_t*)(base + o_red[i]);
        d.nreduce = (int32_t)st.reduce_launch.size();
        d.nowners = 0;
        d.dtype_mask = st.dtype_mask;
        d.data_bytes = st.data_bytes;
        d.data_entries = st.data_entries;
        d.alg_bytes = st.alg_bytes;
        d.name = st.name;
        nlaunch += (d.ntasks > 0) + (d.nreduce > 0);
        m->phases.push_back(d);
    }
    bool any_aux = false;
    for (auto& d : m->phases) any_aux |= d.aux;
    if (any_aux) {
        e = hipStreamCreateWithFlags(&m->aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) {
            hm_matrix_free(m);
            return hip_fail("hm_upload: stream/event creation", e);
        }
    }
    m->stats = P.stats;
    if (opts) {
        m->aux_grid = opts->dense_grid;
        m->fork_after = opts->fork_after;
    }
    m->h_owners = P.owners;
    m->h_items = P.items;
    m->h_tasks = P.tasks;
    m->h_stages = P.stages;
    m->ws_elems = P.ws_elems;
    m->part_elems = P.part_elems;
    if (nlaunch != P.stats.nlaunch) {
        hm_matrix_free(m);
        hm::set_error("hm_upload: launch count mismatch");
        return HM_ELAYOUT;
    }
    *out = m;
    return HM_OK;
}

extern "C" void hm_matrix_free(hm_matrix* m) {
    if (!m) return;
    for (auto& ph : m->phases)
        for (auto& e : ph.pending) m->event_pool.push_back(e);
    for (auto& e : m->event_pool) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    if (m->ev_join) (void)hipEventDestroy(m->ev_join);
    if (m->aux) (void)hipStreamDestroy(m->aux);
    if (m->arena) (void)hipFree(m->arena);
    if (m->mr_arena) (void)hipFree(m->mr_arena);
    if (m->mr_meta) (void)hipFree(m->mr_meta);
    for (auto& ph : m->mr_phases)
        for (auto& e : ph.pending) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    delete m;
}

extern "C" hm_status hm_matrix_stats(const hm_matrix* m, hm_stats* s) {
    if (!m || !s) {
        hm::set_error("hm_matrix_stats: null argument");
        return HM_EINVAL;
    }
    *s = m->stats;
    return HM_OK;
}

extern "C" hm_status hm_mvm(hm_matrix* m, double alpha, const double* x, double* y, uint32_t flags,
                            hm_stream_t stream_) {
    if (!m || !x || !y || x == y) {
        hm::set_error("hm_mvm: null matrix/vector or x == y");
        return HM_EINVAL;
    }
    hipStream_t stream = (hipStream_t)stream_;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
        hm::set_error("hm_mvm: current device differs from the matrix's device");
        return HM_EINVAL;
    }
    const int cluster = (flags & HM_CLUSTER_ORDER) ? 1 : 0;
    const int64_t n = m->n;
    hipLaunchKernelGGL(hm::dev::k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, x, m->perm,
                       m->ws, m->ws32, n, cluster);
    const int64_t* perm = cluster ? nullptr : m->perm;
    const bool timing = (flags & HM_TIMING) != 0;
    const hipStream_t main_stream = stream;
    int fork_left = m->fork_after;   // main-stream stages launched before the second stream starts
    auto fork = [&]() {
        // fork: the dense stage runs on the second stream once x is gathered
        // and the first fork_after stages of the chain are done
        (void)hipEventRecord(m->ev_fork, main_stream);
        (void)hipStreamWaitEvent(m->aux, m->ev_fork, 0);
    };
    bool forked = m->aux == nullptr;
    if (!forked && fork_left <= 0) {
        fork();
        forked = true;
    }
    bool joined = m->aux == nullptr;
    for (auto& ph : m->phases) {
        if (ph.aux && !forked) {   // at the latest before the second-stream stage
            fork();
            forked = true;
        }
        stream = ph.aux ? m->aux : main_stream;
        if (!joined && !ph.aux && ph.ntasks == 0 && &ph == &m->phases.back()) {
            // join before the final reduction of the row owners
            (void)hipEventRecord(m->ev_join, m->aux);
            (void)hipStreamWaitEvent(main_stream, m->ev_join, 0);
            joined = true;
        }
        if (ph.ntasks > 0) {
            unsigned blocks = (unsigned)((ph.ntasks + 3) / 4);
            if (ph.aux && m->aux_grid > 0) blocks = std::min<unsigned>(blocks, (unsigned)m->aux_grid);
            dim3 grid(blocks);
            const hm::dev::TaskKernel kern = hm::dev::kTasks[m->acc64 ? 1 : 0][ph.dtype_mask & 31];
            if (timing) {
                // the event pair is part of the dispatch: it brackets the
                // kernel's execution, as a kernel trace does
                std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
                if (!hm::timing_acquire(m, ph, 1, ev)) {
                    hm::set_error("hm_mvm: timing events failed");
                    return HM_EDEVICE;
                }
                hipExtLaunchKernelGGL(kern, grid, dim3(256), 0, stream, ev.first, ev.second, 0, m->tasks + ph.t0,
                                      ph.ntasks, m->owners, m->items, m->data, m->scales, (const double*)m->ws,
                                      (const float*)m->ws32, m->ws, m->ws32, m->part, (const int64_t*)m->dsrc, y,
                                      perm, alpha);
                ph.pending.push_back(ev);
            } else {
                hipLaunchKernelGGL(kern, grid, dim3(256), 0, stream, m->tasks + ph.t0, ph.ntasks, m->owners,
                                   m->items, m->data, m->scales, m->ws, m->ws32, m->ws, m->ws32, m->part, m->dsrc, y,
                                   perm, alpha);
            }
        }
        if (ph.nreduce > 0) {
            dim3 grid((unsigned)((ph.nreduce + 3) / 4));
            hipLaunchKernelGGL(hm::dev::k_reduce, grid, dim3(256), 0, stream, ph.reduce, ph.nreduce, m->owners,
                               m->part, m->ws, m->ws32, y, perm, alpha);
        }
        if (!forked && !ph.aux && ph.ntasks > 0 && --fork_left == 0) {
            fork();
            forked = true;
        }
    }
    if (!joined) {   // no final reduction stage: still join the second stream
        (void)hipEventRecord(m->ev_join, m->aux);
        (void)hipStreamWaitEvent(main_stream, m->ev_join, 0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail("hm_mvm: kernel launch", e);
    return HM_OK;
}

extern "C" hm_status hm_timing_read(hm_matrix* m, hm_phase_timing* out, int32_t cap, int32_t* nphase) {
    if (!m || (cap > 0 && !out)) {
        hm::set_error("hm_timing_read: null argument");
        return HM_EINVAL;
    }
    int32_t i = 0;
    for (auto* list : {&m->phases, &m->mr_phases})
    for (auto& ph : *list) {
        double ms = 0.0;
        int64_t cnt = 0;
        for (auto& e : ph.pending) {
            hipError_t err = hipEventSynchronize(e.second);
            float t = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&t, e.first, e.second);
            if (err != hipSuccess) return hip_fail("hm_timing_read", err);
            ms += t;
            ++cnt;
            m->event_pool.push_back(e);
        }
        ph.pending.clear();
        if (i < cap) {
            out[i].name = ph.name.c_str();
            out[i].ms_total = ms;
            out[i].launches = cnt;
            out[i].algorithmic_bytes = ph.alg_bytes;
            out[i].ntasks = ph.ntasks;
            out[i].nowners = ph.nowners;
            out[i].data_bytes = ph.data_bytes;
            out[i].data_entries = ph.data_entries;
            out[i].nrhs = ph.timed_nrhs;
        }
        ++i;
    }
    if (nphase) *nphase = i;
    return HM_OK;
}

struct hm_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // many-RHS buffers the recorded kernels address: (matrix, mr_gen at capture)
    std::vector<std::pair<const hm_matrix*, uint64_t>> deps;
};

// Record whatever `enqueue` puts on a private capturing stream (ordered after
// the work already queued on `stream_`) into an instantiated graph.
template <typename F>
static hm_status capture_graph(const char* who, hm_stream_t stream_, hm_graph** out, F&& enqueue) {
    *out = nullptr;
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(who, e);
    hipEvent_t dep = nullptr;
    e = hipEventCreateWithFlags(&dep, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(dep, (hipStream_t)stream_);
    if (e == hipSuccess) e = hipStreamWaitEvent(cap, dep, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(cap);
    hm_graph* g = new (std::nothrow) hm_graph();
    hm_status st = HM_OK;
    if (e == hipSuccess && g) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess && g) {
        st = enqueue((hm_stream_t)cap);
        hipError_t e2 = hipStreamEndCapture(cap, &g->graph);
        if (st == HM_OK && e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess && st == HM_OK && g) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (dep) (void)hipEventDestroy(dep);
    (void)hipStreamDestroy(cap);
    if (!g || e != hipSuccess || st != HM_OK) {
        if (g) {
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
            if (g->graph) (void)hipGraphDestroy(g->graph);
            delete g;
        }
        if (st != HM_OK) return st;
        if (!g) {
            hm::set_error(std::string(who) + ": out of host memory");
            return HM_ENOMEM;
        }
        return hip_fail(who, e);
    }
    *out = g;
    return HM_OK;
}

extern "C" hm_status hm_graph_create(hm_matrix* m, double alpha, const double* x, double* y, uint32_t flags,
                                     hm_stream_t stream_, hm_graph** out) {
    if (!m || !x || !y || !out || (flags & HM_TIMING)) {
        hm::set_error("hm_graph_create: null argument or HM_TIMING requested");
        return HM_EINVAL;
    }
    return capture_graph("hm_graph_create", stream_, out, [&](hm_stream_t s) {
        return hm_mvm(m, alpha, x, y, flags, s);
    });
}

extern "C" hm_status hm_tune_mvm(hm_matrix* m, int32_t reps, hm_stream_t stream_, hm_tune_mvm_result* out) {
    if (!m || !out || reps < 1) {
        hm::set_error("hm_tune_mvm: null argument or reps < 1");
        return HM_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
        hm::set_error("hm_tune_mvm: current device differs from the matrix's device");
        return HM_EINVAL;
    }
    *out = hm_tune_mvm_result{0, 0, 0.0, 0.0};
    int32_t nchain = 0;   // main-stream stages with tasks: the possible fork points are 0 ... nchain
    for (auto& ph : m->phases) nchain += !ph.aux && ph.ntasks > 0;
    const int32_t last = m->aux ? nchain : 0;
    const hipStream_t stream = (hipStream_t)stream_;
    const size_t bytes = (size_t)m->n * sizeof(double);
    double* x = nullptr;
    double* y = nullptr;
    if (hipMalloc((void**)&x, std::max<size_t>(bytes, 8)) != hipSuccess ||
        hipMalloc((void**)&y, std::max<size_t>(bytes, 8)) != hipSuccess) {
        if (x) (void)hipFree(x);
        hm::set_error("hm_tune_mvm: hipMalloc of the trial vectors failed");
        return HM_ENOMEM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMemset(x, 0, std::max<size_t>(bytes, 8));
    if (e == hipSuccess) e = hipMemset(y, 0, std::max<size_t>(bytes, 8));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    hm_status st = e == hipSuccess ? HM_OK : hip_fail("hm_tune_mvm: set-up", e);
    const int32_t keep = m->fork_after;
    int32_t best = keep;
    double best_ms = 0.0;
    for (int32_t f = 0; f <= last && st == HM_OK; ++f) {
        m->fork_after = f;
        hm_graph* g = nullptr;
        st = hm_graph_create(m, 1.0, x, y, 0, stream_, &g);
        if (st != HM_OK) break;
        float ms = 0.0f;
        e = hipSuccess;
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipGraphLaunch(g->exec, stream);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, stream);
        for (int i = 0; i < reps && e == hipSuccess; ++i) e = hipGraphLaunch(g->exec, stream);
        if (e == hipSuccess) e = hipEventRecord(e1, stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        hm_graph_free(g);
        if (e != hipSuccess) {
            st = hip_fail("hm_tune_mvm: timing", e);
            break;
        }
        const double t = (double)ms / reps;
        ++out->ncandidates;
        if (f == 0) out->ms_first = t;
        if (f == 0 || t < best_ms) {
            best = f;
            best_ms = t;
        }
    }
    m->fork_after = st == HM_OK ? best : keep;
    if (st == HM_OK) {
        out->fork_after = best;
        out->ms = best_ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(y);
    return st;
}

extern "C" hm_status hm_graph_create_batch(hm_matrix* const* mats, int32_t nmat, double alpha,
                                           const void* const* X, const int64_t* ldx, const int32_t* nrhs,
                                           void* const* Y, const int64_t* ldy, int32_t vec_dtype, uint32_t flags,
                                           hm_stream_t stream_, hm_graph** out) {
    if (!out || (flags & HM_TIMING)) {
        hm::set_error("hm_graph_create_batch: null argument or HM_TIMING requested");
        return HM_EINVAL;
    }
    // workspaces are sized (allocated) before the capture starts
    hm_status st = hm::batch_prepare(mats, nmat, nrhs, vec_dtype);
    if (st != HM_OK) return st;
    st = capture_graph("hm_graph_create_batch", stream_, out, [&](hm_stream_t s) {
        return hm_mvm_batch(mats, nmat, alpha, X, ldx, nrhs, Y, ldy, vec_dtype, flags, s);
    });
    if (st == HM_OK)
        for (int32_t i = 0; i < nmat; ++i)
            if (nrhs[i] > 0) (*out)->deps.emplace_back(mats[i], mats[i]->mr_gen);
    return st;
}

extern "C" hm_status hm_graph_launch(hm_graph* g, hm_stream_t stream) {
    if (!g || !g->exec) {
        hm::set_error("hm_graph_launch: null graph");
        return HM_EINVAL;
    }
    for (auto& d : g->deps)
        if (d.first->mr_gen != d.second) {
            hm::set_error("hm_graph_launch: a matrix of this graph replaced its many-RHS workspace or plan "
                          "after the capture (wider product or hm_tune_batch); capture the graph again");
            return HM_EINVAL;
        }
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail("hm_graph_launch", e);
    return HM_OK;
}

extern "C" void hm_graph_free(hm_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}
