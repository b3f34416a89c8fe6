// Device engine of the hierarchical-matrix product on gfx950.
//
// One kernel does all the matrix streaming: a wavefront takes one task of one
// owner (a leaf row cluster, a low-rank block, a cluster basis ...), gives
// each lane one output row, and walks the task's columns.  For column j the
// lane loads A[r, j] (consecutive lanes read consecutive addresses of the
// column-major slab), widens it from its storage format, and accumulates
// A[r, j] * w_j, where w_j = input[j] * scale_j is uniform across the wave.
// No lane ever reduces with another lane, and no output is written by two
// waves: owners split over several tasks write partial sums that a second
// kernel adds in task order.  The product is therefore deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hm_pack.h"

namespace hm {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

namespace dev {

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float f16_to_f32(uint16_t b) {
    _Float16 h;
    __builtin_memcpy(&h, &b, 2);
    return (float)h;
}

// OCP FP8 E4M3: sign | 4-bit exponent (bias 7) | 3-bit mantissa, no infinities.
__device__ __forceinline__ float fp8_to_f32(uint8_t b) {
    const uint32_t e = (b >> 3) & 15u, m = b & 7u;
    float mag = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;
    return (b & 0x80u) ? -mag : mag;
}

template <int DT> struct Elem;
template <> struct Elem<HM_F64> { using T = double; __device__ static double f(T v) { return v; } };
template <> struct Elem<HM_F32> { using T = float; __device__ static float f(T v) { return v; } };
template <> struct Elem<HM_BF16> { using T = uint16_t; __device__ static float f(T v) { return bf16_to_f32(v); } };
template <> struct Elem<HM_F16> { using T = uint16_t; __device__ static float f(T v) { return f16_to_f32(v); } };
template <> struct Elem<HM_FP8E4M3> { using T = uint8_t; __device__ static float f(T v) { return fp8_to_f32(v); } };

// Accumulate columns [jb, je) of one item for row rr.
template <int DT, bool WIDE, bool SCALED>
__device__ __forceinline__ void item_dot(const uint8_t* __restrict__ base, int nrows, int rr, int jb, int je,
                                         const double* __restrict__ w, const double* __restrict__ sc,
                                         double& a64, float& a32) {
    using E = Elem<DT>;
    using T = typename E::T;
    const T* __restrict__ A = reinterpret_cast<const T*>(base) + rr;
    int j = jb;
    constexpr int U = 8;
    for (; j + U <= je; j += U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = A[(int64_t)(j + u) * nrows];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double wj = w[j + u];
            if (SCALED) wj *= sc[j + u];
            if (WIDE)
                a64 = fma((double)E::f(v[u]), wj, a64);
            else
                a32 = fmaf((float)E::f(v[u]), (float)wj, a32);
        }
    }
    for (; j < je; ++j) {
        T v = A[(int64_t)j * nrows];
        double wj = w[j];
        if (SCALED) wj *= sc[j];
        if (WIDE)
            a64 = fma((double)E::f(v), wj, a64);
        else
            a32 = fmaf((float)E::f(v), (float)wj, a32);
    }
}

template <int DT, bool WIDE>
__device__ __forceinline__ void item_dispatch_scale(const uint8_t* base, int nrows, int rr, int jb, int je,
                                                    const double* w, const double* sc, double& a64, float& a32) {
    if (sc)
        item_dot<DT, WIDE, true>(base, nrows, rr, jb, je, w, sc, a64, a32);
    else
        item_dot<DT, WIDE, false>(base, nrows, rr, jb, je, w, sc, a64, a32);
}

__device__ __forceinline__ void finalize(const DOwner& ow, int r, double v, double* __restrict__ vout,
                                         double* __restrict__ y, const int64_t* __restrict__ perm, double alpha) {
    if (ow.mode == 0)
        vout[ow.out_off + r] = v;
    else if (ow.mode == 1)
        y[perm ? perm[ow.out_off + r] : (int64_t)(ow.out_off + r)] += alpha * v;
    else
        y[ow.out_off + r] += alpha * v;
}

template <bool ACC64>
__global__ __launch_bounds__(256) void k_owner_tasks(const DTask* __restrict__ tasks, int ntasks,
                                                     const DOwner* __restrict__ owners,
                                                     const DItem* __restrict__ items,
                                                     const uint8_t* __restrict__ data,
                                                     const double* __restrict__ scales,
                                                     const double* __restrict__ vin, double* vout,
                                                     double* __restrict__ part, double* __restrict__ y,
                                                     const int64_t* __restrict__ perm, double alpha) {
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= ntasks) return;
    const DTask tk = tasks[t];
    const DOwner ow = owners[tk.owner];
    for (int r0 = 0; r0 < ow.nrows; r0 += 64) {
        const int r = r0 + lane;
        const bool act = r < ow.nrows;
        const int rr = act ? r : ow.nrows - 1;   // inactive lanes re-read a valid row
        double a64 = 0.0;
        float a32 = 0.0f;
        int it = tk.item_start;
        int c = tk.c0;
        while (c < tk.c1) {
            const DItem item = items[it];
            const int jb = c - item.col0;
            const int je = min(item.ncols, tk.c1 - item.col0);
            const uint8_t* base = data + item.data_off;
            const double* w = vin + item.vec_off;
            const double* sc = item.scale_off >= 0 ? scales + item.scale_off : nullptr;
            const bool wide = ACC64 || item.acc64;
            switch (item.dtype) {
                case HM_F64:
                    item_dispatch_scale<HM_F64, true>(base, ow.nrows, rr, jb, je, w, sc, a64, a32);
                    break;
                case HM_F32:
                    if (wide) item_dispatch_scale<HM_F32, true>(base, ow.nrows, rr, jb, je, w, sc, a64, a32);
                    else item_dispatch_scale<HM_F32, false>(base, ow.nrows, rr, jb, je, w, sc, a64, a32);
                    break;
                case HM_BF16:
                    if (wide) item_dispatch_scale<HM_BF16, true>(base, ow.nrows, rr, jb, je, w, sc, a64, a32);
                    else item_dispatch_scale<HM_BF16, false>(base, ow.nrows, rr, jb, je, w, sc, a64, a32);
                    break;
                case HM_F16:
                    if (wide) item_dispatch_scale<HM_F16, true>(base, ow.nrows, rr, jb, je, w, sc, a64, a32);
                    else item_dispatch_scale<HM_F16, false>(base, ow.nrows, rr, jb, je, w, sc, a64, a32);
                    break;
                default:
                    if (wide) item_dispatch_scale<HM_FP8E4M3, true>(base, ow.nrows, rr, jb, je, w, sc, a64, a32);
                    else item_dispatch_scale<HM_FP8E4M3, false>(base, ow.nrows, rr, jb, je, w, sc, a64, a32);
                    break;
            }
            c = item.col0 + je;
            ++it;
        }
        double v = a64 + (double)a32;
        if (act) {
            if (ow.rscale_off >= 0) v *= scales[ow.rscale_off + r];
            if (ow.ntasks == 1)
                finalize(ow, r, v, vout, y, perm, alpha);
            else
                part[ow.part_off + (int64_t)tk.local * ow.nrows + r] = v;
        }
    }
}

// Sum the partial results of split owners in task order, one wave per owner.
__global__ __launch_bounds__(256) void k_reduce(const int32_t* __restrict__ list, int nlist,
                                                const DOwner* __restrict__ owners,
                                                const double* __restrict__ part, double* vout,
                                                double* __restrict__ y, const int64_t* __restrict__ perm,
                                                double alpha) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nlist) return;
    const DOwner ow = owners[list[i]];
    for (int r = lane; r < ow.nrows; r += 64) {
        const double* p = part + ow.part_off + r;
        double v = 0.0;
        for (int l = 0; l < ow.ntasks; ++l) v += p[(int64_t)l * ow.nrows];
        finalize(ow, r, v, vout, y, perm, alpha);
    }
}

// x in cluster order: ws[i] = x[perm[i]]  (or a straight copy)
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ x, const int64_t* __restrict__ perm,
                                                double* __restrict__ ws, int64_t n, int cluster_order) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) ws[i] = cluster_order ? x[i] : x[perm[i]];
}

}  // namespace dev

struct DevPhase {
    const DOwner* owners;
    const DItem* items;
    const DTask* tasks;
    const int32_t* reduce;
    int32_t ntasks, nreduce;
    int64_t data_bytes;
    std::string name;
};

}  // namespace hm

struct hm_matrix {
    const hm_layout* layout = nullptr;
    int32_t format = 0;
    int32_t acc64 = 1;
    int64_t n = 0;
    int device = 0;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    int64_t* perm = nullptr;
    uint8_t* data = nullptr;
    double* scales = nullptr;
    double* ws = nullptr;
    double* part = nullptr;
    std::vector<hm::DevPhase> phases;
    hm_stats stats{};
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

hm_status hip_fail(const char* what, hipError_t e) {
    hm::set_error(std::string(what) + ": " + hipGetErrorString(e));
    return HM_EDEVICE;
}

}  // namespace

extern "C" const char* hm_last_error(void) { return hm::g_err.c_str(); }
extern "C" const char* hm_version(void) { return "hm 0.1 gfx950"; }

extern "C" hm_status hm_upload(const hm_layout* layout, int32_t format, const hm_values* values,
                               const hm_precision* prec, hm_stream_t stream, hm_matrix** out) {
    (void)stream;
    if (!layout || !values || !prec || !out) {
        hm::set_error("hm_upload: null argument");
        return HM_EINVAL;
    }
    *out = nullptr;
    hm::Packed P;
    hm::PackOptions opt;
    if (const char* e = std::getenv("HM_TASK_BYTES")) opt.task_bytes = std::max(1024L, std::atol(e));
    hm_status st;
    try {
        st = hm::pack(layout->L, format, values, prec, opt, P);
    } catch (const std::bad_alloc&) {
        hm::set_error("hm_upload: out of host memory while packing");
        return HM_ENOMEM;
    }
    if (st != HM_OK) return st;

    // one device allocation: metadata | perm | data | scales | workspace | partials
    size_t meta = 0;
    std::vector<std::array<size_t, 4>> offs;
    for (auto& ph : P.phases) {
        std::array<size_t, 4> o;
        o[0] = meta; meta = align256(meta + ph.owners.size() * sizeof(hm::DOwner));
        o[1] = meta; meta = align256(meta + ph.items.size() * sizeof(hm::DItem));
        o[2] = meta; meta = align256(meta + ph.tasks.size() * sizeof(hm::DTask));
        o[3] = meta; meta = align256(meta + ph.reduce_owners.size() * sizeof(int32_t));
        offs.push_back(o);
    }
    const int64_t n = layout->L.n;
    size_t o_perm = meta;
    size_t o_data = align256(o_perm + n * sizeof(int64_t));
    size_t o_scales = align256(o_data + P.data.size());
    size_t o_ws = align256(o_scales + P.scales.size() * sizeof(double));
    size_t o_part = align256(o_ws + P.ws_elems * sizeof(double));
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
    for (size_t i = 0; i < P.phases.size() && e == hipSuccess; ++i) {
        auto& ph = P.phases[i];
        e = copy(offs[i][0], ph.owners.data(), ph.owners.size() * sizeof(hm::DOwner));
        if (e == hipSuccess) e = copy(offs[i][1], ph.items.data(), ph.items.size() * sizeof(hm::DItem));
        if (e == hipSuccess) e = copy(offs[i][2], ph.tasks.data(), ph.tasks.size() * sizeof(hm::DTask));
        if (e == hipSuccess) e = copy(offs[i][3], ph.reduce_owners.data(), ph.reduce_owners.size() * sizeof(int32_t));
    }
    if (e == hipSuccess) e = copy(o_perm, layout->L.perm.data(), n * sizeof(int64_t));
    if (e == hipSuccess) e = copy(o_data, P.data.data(), P.data.size());
    if (e == hipSuccess) e = copy(o_scales, P.scales.data(), P.scales.size() * sizeof(double));
    if (e != hipSuccess) {
        hipFree(m->arena);
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
    m->part = (double*)(base + o_part);
    int32_t nlaunch = 1;
    for (size_t i = 0; i < P.phases.size(); ++i) {
        auto& ph = P.phases[i];
        hm::DevPhase d;
        d.owners = (const hm::DOwner*)(base + offs[i][0]);
        d.items = (const hm::DItem*)(base + offs[i][1]);
        d.tasks = (const hm::DTask*)(base + offs[i][2]);
        d.reduce = (const int32_t*)(base + offs[i][3]);
        d.ntasks = (int32_t)ph.tasks.size();
        d.nreduce = (int32_t)ph.reduce_owners.size();
        d.data_bytes = ph.data_bytes;
        d.name = ph.name;
        nlaunch += 1 + (d.nreduce > 0);
        m->phases.push_back(d);
    }
    m->stats = P.stats;
    m->stats.nlaunch = nlaunch;
    int64_t coef = P.ws_elems - n;
    m->stats.algorithmic_bytes = (double)(m->stats.bytes_dense + m->stats.bytes_factors + m->stats.bytes_coupling +
                                          m->stats.bytes_transfer + m->stats.bytes_scales + m->stats.bytes_meta) +
                                 24.0 * n + 16.0 * coef;
    *out = m;
    return HM_OK;
}

extern "C" void hm_matrix_free(hm_matrix* m) {
    if (!m) return;
    if (m->arena) hipFree(m->arena);
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
                       m->ws, n, cluster);
    const int64_t* perm = cluster ? nullptr : m->perm;
    for (const auto& ph : m->phases) {
        if (ph.ntasks > 0) {
            dim3 grid((unsigned)((ph.ntasks + 3) / 4));
            if (m->acc64)
                hipLaunchKernelGGL(hm::dev::k_owner_tasks<true>, grid, dim3(256), 0, stream, ph.tasks, ph.ntasks,
                                   ph.owners, ph.items, m->data, m->scales, m->ws, m->ws, m->part, y, perm, alpha);
            else
                hipLaunchKernelGGL(hm::dev::k_owner_tasks<false>, grid, dim3(256), 0, stream, ph.tasks, ph.ntasks,
                                   ph.owners, ph.items, m->data, m->scales, m->ws, m->ws, m->part, y, perm, alpha);
        }
        if (ph.nreduce > 0) {
            dim3 grid((unsigned)((ph.nreduce + 3) / 4));
            hipLaunchKernelGGL(hm::dev::k_reduce, grid, dim3(256), 0, stream, ph.reduce, ph.nreduce, ph.owners,
                               m->part, m->ws, y, perm, alpha);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail("hm_mvm: kernel launch", e);
    return HM_OK;
}
