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

#include "hm_stream.h"

namespace hm {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

namespace dev {

// Sum the partial results of split owners in a fixed order, one wave per owner.
__global__ __launch_bounds__(256) void k_reduce(const int32_t* __restrict__ list, int nlist,
                                                const DOwner* __restrict__ owners,
                                                const double* __restrict__ part, double* vout, float* vout32,
                                                double* __restrict__ y, const int64_t* __restrict__ perm,
                                                double alpha) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nlist) return;
    run_reduce<false>(owners[list[i]], lane, part, vout, vout32, y, perm, alpha);
}

extern const TaskKernel kTasks32lo[16], kTasks32hi[16], kTasks64lo[16], kTasks64hi[16];
extern const TaskKernel kTasksCodec32Single[11], kTasksCodec32Family[3], kTasksCodec64Single[11],
    kTasksCodec64Family[3];

// the instantiation for a stage's dtype set: the exact set for the hardware
// formats, else the first codec set (kCodecMasks) that contains it
TaskKernel task_kernel(bool acc64, int mask) {
    if ((mask & ~kMaskHw) == 0) {
        if (acc64) return mask < 16 ? kTasks64lo[mask] : kTasks64hi[mask - 16];
        return mask < 16 ? kTasks32lo[mask] : kTasks32hi[mask - 16];
    }
    for (int i = 0; i < 14; ++i)
        if ((mask & ~kCodecMasks[i]) == 0) {
            if (i < 11) return acc64 ? kTasksCodec64Single[i] : kTasksCodec32Single[i];
            return acc64 ? kTasksCodec64Family[i - 11] : kTasksCodec32Family[i - 11];
        }
    return nullptr;
}

// x in cluster order: ws[i] = x[perm[i]]  (or a straight copy); the
// coefficient entries [n, zero_to) are cleared for atomic accumulation
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ x, const int64_t* __restrict__ perm,
                                                double* __restrict__ ws, float* __restrict__ ws32, int64_t n,
                                                int cluster_order, int64_t zero_to) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const double v = cluster_order ? x[i] : x[perm[i]];
        ws[i] = v;
        ws32[i] = (float)v;
    } else if (i < zero_to) {
        ws[i] = 0.0;
    }
}

// HM_SYNC_PRIVATE: y[perm[i]] += alpha * (sum of the eight private copies
// of row i, in copy order), and the copies cleared for the next product
__global__ __launch_bounds__(256) void k_private_sum(double* __restrict__ y, const int64_t* __restrict__ perm,
                                                     double* __restrict__ priv, int64_t n, double alpha) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double v = 0.0;
    for (int c = 0; c < 8; ++c) {
        v += priv[c * n + i];
        priv[c * n + i] = 0.0;
    }
    y[perm ? perm[i] : i] += alpha * v;
}

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
    // persistent schedule: the plan as one ticket queue
    hm::Queue Q;
    std::vector<int32_t> qorder;
    const bool persist = opt.schedule == HM_SCHED_PERSISTENT;
    if (persist) {
        try {
            st = hm::build_queue(P, layout->L.n, Q);
            if (st == HM_OK) st = hm::queue_order(P.owners, Q.tasks, Q, opt.dense_after, qorder);
        } catch (const std::bad_alloc&) {
            hm::set_error("hm_upload: out of host memory while building the persistent queue");
            return HM_ENOMEM;
        }
        if (st != HM_OK) return st;
    }

    // one device allocation: metadata | perm | data | scales | workspace | partials
    // | persistent queue tables and counters
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
    size_t o_pq = align256(o_part + std::max<int64_t>(P.part_elems, 1) * sizeof(double));
    const size_t o_ptasks = o_pq;
    const size_t o_pdep0 = align256(o_ptasks + Q.tasks.size() * sizeof(hm::DTask));
    const size_t o_pdeps = align256(o_pdep0 + Q.dep_first.size() * sizeof(int32_t));
    const size_t o_ptarget = align256(o_pdeps + Q.deps.size() * sizeof(int32_t));
    const size_t o_porder = align256(o_ptarget + Q.target.size() * sizeof(int32_t));
    const size_t o_pdone = align256(o_porder + qorder.size() * sizeof(int32_t));
    const size_t o_pctl = align256(o_pdone + (persist ? P.owners.size() : 0) * sizeof(int32_t));
    const size_t o_priv = align256(o_pctl + (persist ? 256 : 0));
    size_t total = align256(o_priv + (opt.sync == HM_SYNC_PRIVATE ? 8 * (size_t)layout->L.n * sizeof(double) : 0));

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
    if (opt.sync != HM_SYNC_OWNER) {
        // atomic variants: no partial sums to defer or reduce; every task adds
        // its rows atomically (mode bit 8; bit 16 = into the private copies of
        // y), and a task reading coefficients reads them in float64 (staged,
        // bit 2: the float32 mirror is not kept)
        std::vector<uint8_t> coef((size_t)(P.ws_elems + hm::TILE_PAD), 0);
        for (const auto& ow : P.owners)
            if (ow.mode == 0)
                for (int32_t r = 0; r < ow.nrows; ++r) coef[(size_t)(ow.out_off + r)] = 1;
        for (auto& t : dtasks) {
            t.mode = (int16_t)(t.mode | 8 | ((opt.sync == HM_SYNC_PRIVATE && (t.mode & 3) != 0) ? 16 : 0));
            const hm::DOwner& ow = P.owners[t.owner];
            int32_t c = t.c0;
            for (int32_t it = t.item_start; c < t.c1 && it < ow.item0 + ow.nitems; ++it) {
                const hm::DItem& item = P.items[it];
                const int32_t jb = c - item.col0, je = std::min(item.ncols, t.c1 - item.col0);
                for (int32_t j = jb; j < je; ++j)
                    if (coef[(size_t)(item.vec_off + j)]) t.mode = (int16_t)(t.mode | 4);
                c = item.col0 + je;
            }
        }
        std::fill(P.dsrc.begin(), P.dsrc.end(), 0);
    }
    e = copy(o_owners, P.owners.data(), P.owners.size() * sizeof(hm::DOwner));
    if (e == hipSuccess) e = copy(o_items, P.items.data(), P.items.size() * sizeof(hm::DItem));
    if (e == hipSuccess) e = copy(o_tasks, dtasks.data(), dtasks.size() * sizeof(hm::DTask));
    for (size_t i = 0; i < P.stages.size() && e == hipSuccess; ++i)
        e = copy(o_red[i], P.stages[i].reduce_launch.data(), P.stages[i].reduce_launch.size() * sizeof(int32_t));
    if (e == hipSuccess) e = copy(o_dsrc, P.dsrc.data(), P.dsrc.size() * sizeof(int64_t));
    if (e == hipSuccess) e = copy(o_perm, layout->L.perm.data(), n * sizeof(int64_t));
    if (e == hipSuccess) e = copy(o_data, P.data.data(), P.data.size());
    if (e == hipSuccess) e = copy(o_scales, P.scales.data(), P.scales.size() * sizeof(double));
    if (persist) {
        if (e == hipSuccess) e = copy(o_ptasks, Q.tasks.data(), Q.tasks.size() * sizeof(hm::DTask));
        if (e == hipSuccess) e = copy(o_pdep0, Q.dep_first.data(), Q.dep_first.size() * sizeof(int32_t));
        if (e == hipSuccess) e = copy(o_pdeps, Q.deps.data(), Q.deps.size() * sizeof(int32_t));
        if (e == hipSuccess) e = copy(o_ptarget, Q.target.data(), Q.target.size() * sizeof(int32_t));
        if (e == hipSuccess) e = copy(o_porder, qorder.data(), qorder.size() * sizeof(int32_t));
        if (e == hipSuccess) e = hipMemset(base + o_pdone, 0, P.owners.size() * sizeof(int32_t));
        if (e == hipSuccess) e = hipMemset(base + o_pctl, 0, 256);
    }
    if (e == hipSuccess && opt.sync == HM_SYNC_PRIVATE)
        e = hipMemset(base + o_priv, 0, 8 * (size_t)layout->L.n * sizeof(double));
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
        d.nreduce = opt.sync == HM_SYNC_OWNER ? (int32_t)st.reduce_launch.size() : 0;
        d.nowners = 0;
        d.dtype_mask = st.dtype_mask;
        d.data_bytes = st.data_bytes;
        d.data_entries = st.data_entries;
        d.alg_bytes = st.alg_bytes;
        d.method_bytes = st.method_bytes;
        d.name = st.name;
        nlaunch += (d.ntasks > 0) + (d.nreduce > 0);
        if (d.aux && d.ntasks > 0 && hm::aux_split_by_dtype(d.dtype_mask)) {
            // one launch per run of one dtype (the packer sorted the tasks)
            for (int64_t k = st.t0; k < st.t1; ++k) {
                const int32_t dt = P.tasks[(size_t)k].dtype;
                if (d.subs.empty() || d.subs.back().dtype != dt)
                    d.subs.push_back(hm::DevStage::Sub{dt, (int32_t)(k - st.t0), 0});
                d.subs.back().ntasks++;
            }
            nlaunch += (int32_t)d.subs.size() - 1;
        }
        m->phases.push_back(d);
    }
    bool any_aux = false;
    for (auto& d : m->phases) any_aux |= d.aux;
    if (any_aux) {
        e = hipStreamCreateWithFlags(&m->aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_fork2, hipEventDisableTiming);
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
    m->sync = opt.sync;
    if (opt.sync == HM_SYNC_PRIVATE) m->ypriv = (double*)(base + o_priv);
    if (opt.sync != HM_SYNC_OWNER) P.stats.nlaunch = nlaunch;   // the plan's launches without reductions
    if (persist) {
        m->schedule = HM_SCHED_PERSISTENT;
        m->p_nq = (int32_t)qorder.size();
        m->p_mask = Q.dtype_mask ? Q.dtype_mask : 1;
        m->p_dense_after = opt.dense_after;
        m->p_grab = opt.tickets_per_grab;
        m->p_nowners = (int64_t)P.owners.size();
        m->p_spin = (uint64_t)opt.spin_limit_us * 100;   // 100 MHz real-time counter
        m->p_tasks = (const hm::DTask*)(base + o_ptasks);
        m->p_dep_first = (const int32_t*)(base + o_pdep0);
        m->p_deps = (const int32_t*)(base + o_pdeps);
        m->p_target = (const int32_t*)(base + o_ptarget);
        m->p_order = (int32_t*)(base + o_porder);
        m->p_done = (int32_t*)(base + o_pdone);
        m->p_ctl = (uint32_t*)(base + o_pctl);
        // grid: as many workgroups as can be resident (the queue does not
        // rely on it: later workgroups simply find fewer tickets)
        const hm::dev::PersistKernel pk = hm::dev::persist_kernel(m->acc64 != 0, m->p_mask, nullptr);
        int per_cu = 0, ncu = 0;
        if (!pk || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)pk, 256, 0) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess) {
            hm_matrix_free(m);
            hm::set_error("hm_upload: occupancy query of the persistent kernel failed");
            return HM_EDEVICE;
        }
        m->p_grid = std::max(1, std::min(std::max(per_cu, 1) * std::max(ncu, 1), (m->p_nq + 3) / 4));
        hm::DevStage d;
        d.aux = false;
        d.t0 = 0;
        d.ntasks = m->p_nq;
        d.nreduce = 0;
        d.nowners = (int32_t)P.owners.size();
        d.reduce = nullptr;
        d.dtype_mask = m->p_mask;
        d.data_bytes = d.data_entries = 0;
        d.alg_bytes = d.method_bytes = 0.0;
        for (const auto& st2 : P.stages) {
            d.data_bytes += st2.data_bytes;
            d.data_entries += st2.data_entries;
            d.alg_bytes += st2.alg_bytes;
            d.method_bytes += st2.method_bytes;
        }
        d.name = "persistent";
        m->pphases.push_back(d);
        Q.chain.shrink_to_fit();
        m->p_queue = std::move(Q);
    }
    if (nlaunch != P.stats.nlaunch) {
        hm_matrix_free(m);
        hm::set_error("hm_upload: launch count mismatch");
        return HM_ELAYOUT;
    }
    m->stats.nlaunch = persist ? 2 : nlaunch + (opt.sync == HM_SYNC_PRIVATE ? 1 : 0);   // (+ the private sum)
    if (opt.adjoint) {
        // M^T over the transposed block tree, uploaded as a matrix of its own
        hm::Transposed T;
        hm_status sa;
        try {
            sa = hm::transpose_matrix(layout->L, format, values, T);
        } catch (const std::bad_alloc&) {
            hm_matrix_free(m);
            hm::set_error("hm_upload: out of host memory while transposing for the adjoint");
            return HM_ENOMEM;
        }
        hm_layout* tl = sa == HM_OK ? new (std::nothrow) hm_layout(std::move(T.layout)) : nullptr;
        if (sa == HM_OK && !tl) sa = HM_ENOMEM;
        hm_upload_opts o2 = opts ? *opts : hm_upload_opts{};
        o2.adjoint = 0;
        if (sa == HM_OK) sa = hm_upload(tl, format, &T.v, prec, &o2, stream, &m->adj);
        if (sa != HM_OK) {
            delete tl;
            hm_matrix_free(m);
            return sa;
        }
        m->adj_layout = tl;
    }
    *out = m;
    return HM_OK;
}

extern "C" void hm_matrix_free(hm_matrix* m) {
    if (!m) return;
    if (m->adj) hm_matrix_free(m->adj);
    delete m->adj_layout;
    for (auto* list : {&m->phases, &m->pphases})
        for (auto& ph : *list)
            for (auto& e : ph.pending) m->event_pool.push_back(e);
    for (auto& e : m->event_pool) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    if (m->ev_join) (void)hipEventDestroy(m->ev_join);
    if (m->ev_fork2) (void)hipEventDestroy(m->ev_fork2);
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
    if (flags & HM_ADJOINT) {
        if (!m->adj) {
            hm::set_error("hm_mvm: HM_ADJOINT needs a matrix uploaded with hm_upload_opts.adjoint = 1");
            return HM_EINVAL;
        }
        return hm_mvm(m->adj, alpha, x, y, flags & ~HM_ADJOINT, stream_);
    }
    hipStream_t stream = (hipStream_t)stream_;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
        hm::set_error("hm_mvm: current device differs from the matrix's device");
        return HM_EINVAL;
    }
    const int cluster = (flags & HM_CLUSTER_ORDER) ? 1 : 0;
    const int64_t n = m->n;
    if (m->schedule == HM_SCHED_PERSISTENT) {
        const int64_t nth = std::max<int64_t>(n, m->p_nowners);
        hipLaunchKernelGGL(hm::dev::k_gather_reset, dim3((unsigned)((nth + 255) / 256)), dim3(256), 0, stream, x,
                           m->perm, m->ws, m->ws32, n, cluster, m->p_done, m->p_nowners, m->p_ctl);
        const hm::dev::PersistKernel pk = hm::dev::persist_kernel(m->acc64 != 0, m->p_mask, nullptr);
        const int64_t* permp = cluster ? nullptr : m->perm;
        const dim3 grid((unsigned)m->p_grid), block(256);
        if (flags & HM_TIMING) {
            std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
            if (!hm::timing_acquire(m, m->pphases[0], 1, ev)) {
                hm::set_error("hm_mvm: timing events failed");
                return HM_EDEVICE;
            }
            hipExtLaunchKernelGGL(pk, grid, block, 0, stream, ev.first, ev.second, 0, (const int32_t*)m->p_order,
                                  m->p_nq, m->p_dep_first, m->p_deps, m->p_target, m->p_done, m->p_ctl, m->p_spin,
                                  m->p_tasks, m->owners, m->items, (const uint8_t*)m->data, (const double*)m->scales,
                                  (const double*)m->ws, (const float*)m->ws32, m->ws, m->ws32, m->part,
                                  (const int64_t*)m->dsrc, y, permp, alpha, (int)n, m->p_grab);
            m->pphases[0].pending.push_back(ev);
        } else {
            hipLaunchKernelGGL(pk, grid, block, 0, stream, (const int32_t*)m->p_order, m->p_nq, m->p_dep_first,
                               m->p_deps, m->p_target, m->p_done, m->p_ctl, m->p_spin, m->p_tasks, m->owners,
                               m->items, (const uint8_t*)m->data, (const double*)m->scales, (const double*)m->ws,
                               (const float*)m->ws32, m->ws, m->ws32, m->part, (const int64_t*)m->dsrc, y, permp,
                               alpha, (int)n, m->p_grab);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail("hm_mvm: kernel launch", e);
        return HM_OK;
    }
    const int64_t zero_to = m->sync != HM_SYNC_OWNER ? m->ws_elems : n;
    hipLaunchKernelGGL(hm::dev::k_gather, dim3((unsigned)((zero_to + 255) / 256)), dim3(256), 0, stream, x, m->perm,
                       m->ws, m->ws32, n, cluster, zero_to);
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
    // split dense stage: its second part waits for fork2 chain stages
    int fork2_left = m->dense_split > 0 ? m->fork2 : -1;
    bool fork2_recorded = m->dense_split <= 0 || m->aux == nullptr;
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
        // tasks [t0, t0 + nt) of this stage as one launch on `stream` (of
        // the kernel for `mask`)
        int32_t nlaunched = 0;
        auto launch1 = [&](int64_t t0, int32_t nt, int32_t mask) -> bool {
            ++nlaunched;
            unsigned blocks = (unsigned)((nt + 3) / 4);
            if (ph.aux && m->aux_grid > 0) blocks = std::min<unsigned>(blocks, (unsigned)m->aux_grid);
            dim3 grid(blocks);
            const hm::dev::TaskKernel kern = hm::dev::task_kernel(m->acc64 != 0, mask);
            if (timing) {
                // the event pair is part of the dispatch: it brackets the
                // kernel's execution, as a kernel trace does
                std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
                if (!hm::timing_acquire(m, ph, 1, ev)) return false;
                hipExtLaunchKernelGGL(kern, grid, dim3(256), 0, stream, ev.first, ev.second, 0, m->tasks + t0, nt,
                                      m->owners, m->items, m->data, m->scales, (const double*)m->ws,
                                      (const float*)m->ws32, m->ws, m->ws32, m->part, (const int64_t*)m->dsrc, y,
                                      perm, alpha, m->ypriv, n);
                ph.pending.push_back(ev);
            } else {
                hipLaunchKernelGGL(kern, grid, dim3(256), 0, stream, m->tasks + t0, nt, m->owners, m->items, m->data,
                                   m->scales, m->ws, m->ws32, m->ws, m->ws32, m->part, m->dsrc, y, perm, alpha,
                                   m->ypriv, n);
            }
            return true;
        };
        // tasks [t0, t0 + nt): one launch, or one per run of one dtype
        // (sub-runs of a split second-stream stage; F64 runs with the
        // hardware kernel, a codec run with that codec's own kernel)
        auto launch = [&](int64_t t0, int32_t nt) -> bool {
            if (ph.subs.empty()) return launch1(t0, nt, ph.dtype_mask);
            bool ok = true;
            for (const auto& sb : ph.subs) {
                const int64_t a = std::max<int64_t>(t0, ph.t0 + sb.t0);
                const int64_t b = std::min<int64_t>(t0 + nt, ph.t0 + sb.t0 + sb.ntasks);
                if (ok && a < b) ok = launch1(a, (int32_t)(b - a), sb.dtype < 0 ? 1 : (1 << sb.dtype) | 1);
            }
            return ok;
        };
        if (ph.ntasks > 0) {
            const bool split = ph.aux && m->dense_split > 0 && m->dense_split < ph.ntasks;
            bool ok = true;
            if (split) {
                // first part from the fork point; the second after fork2
                // chain stages (recorded on the main stream in order)
                ok = launch(ph.t0, m->dense_split);
                if (!fork2_recorded) {
                    (void)hipEventRecord(m->ev_fork2, main_stream);
                    fork2_recorded = true;
                }
                (void)hipStreamWaitEvent(m->aux, m->ev_fork2, 0);
                if (ok) ok = launch(ph.t0 + m->dense_split, ph.ntasks - m->dense_split);
            } else {
                ok = launch(ph.t0, ph.ntasks);
            }
            ph.timed_parts = std::max(nlaunched, 1);   // launches of this stage per product
            if (!ok) {
                hm::set_error("hm_mvm: timing events failed");
                return HM_EDEVICE;
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
        if (!fork2_recorded && !ph.aux && ph.ntasks > 0 && --fork2_left == 0) {
            (void)hipEventRecord(m->ev_fork2, main_stream);
            fork2_recorded = true;
        }
    }
    if (!joined) {   // no final reduction stage: still join the second stream
        (void)hipEventRecord(m->ev_join, m->aux);
        (void)hipStreamWaitEvent(main_stream, m->ev_join, 0);
    }
    if (m->sync == HM_SYNC_PRIVATE)
        hipLaunchKernelGGL(hm::dev::k_private_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, main_stream, y,
                           perm, m->ypriv, n, alpha);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail("hm_mvm: kernel launch", e);
    return HM_OK;
}

extern "C" hm_status hm_matrix_check(hm_matrix* m) {
    if (!m) {
        hm::set_error("hm_matrix_check: null matrix");
        return HM_EINVAL;
    }
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail("hm_matrix_check: synchronize", e);
    if (!m->p_ctl) return HM_OK;
    uint32_t err = 0;
    e = hipMemcpy(&err, m->p_ctl + 2, sizeof(err), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail("hm_matrix_check: read", e);
    if (err != 0) {
        e = hipMemset(m->p_ctl + 2, 0, sizeof(uint32_t));
        if (e != hipSuccess) return hip_fail("hm_matrix_check: clear", e);
        hm::set_error("hm_matrix_check: a persistent launch was aborted (a dependency wait exceeded its bound); "
                      "its products are invalid");
        return HM_EDEVICE;
    }
    return HM_OK;
}

extern "C" hm_status hm_timing_read(hm_matrix* m, hm_phase_timing* out, int32_t cap, int32_t* nphase) {
    if (!m || (cap > 0 && !out)) {
        hm::set_error("hm_timing_read: null argument");
        return HM_EINVAL;
    }
    int32_t i = 0;
    for (auto* list : {&m->phases, &m->pphases, &m->mr_phases})
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
            out[i].launches = cnt / std::max(ph.timed_parts, 1);   // a split stage counts once per product
            out[i].algorithmic_bytes = ph.alg_bytes;
            out[i].ntasks = ph.ntasks;
            out[i].nowners = ph.nowners;
            out[i].data_bytes = ph.data_bytes;
            out[i].data_entries = ph.data_entries;
            out[i].nrhs = ph.timed_nrhs;
            out[i].method_bytes = ph.method_bytes;
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

// Reorder the persistent queue for another interleave point (host build,
// then one copy of the order table; synchronous, outside graph capture).
static hm_status set_dense_after(hm_matrix* m, int32_t dense_after) {
    if (m->p_dense_after == dense_after) return HM_OK;
    std::vector<int32_t> order;
    hm_status st = hm::queue_order(m->h_owners, m->p_queue.tasks, m->p_queue, dense_after, order);
    if (st != HM_OK) return st;
    if ((int32_t)order.size() != m->p_nq) {
        hm::set_error("hm_tune_mvm: queue size changed");
        return HM_ELAYOUT;
    }
    hipError_t e = hipMemcpy(m->p_order, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail("hm_tune_mvm: queue copy", e);
    m->p_dense_after = dense_after;
    return HM_OK;
}

extern "C" hm_status hm_set_dense_split(hm_matrix* m, int32_t fork2, int32_t first_tasks) {
    int32_t nd = 0;
    if (m)
        for (auto& ph : m->phases)
            if (ph.aux) nd += ph.ntasks;
    if (!m || fork2 < 0 || first_tasks < 0 || (first_tasks > 0 && first_tasks >= nd)) {
        hm::set_error("hm_set_dense_split: null matrix, negative value, or first_tasks not below the dense tasks");
        return HM_EINVAL;
    }
    m->fork2 = fork2;
    m->dense_split = first_tasks;
    return HM_OK;
}

extern "C" hm_status hm_set_schedule(hm_matrix* m, int32_t schedule, int32_t param) {
    if (!m || param < 0 || (schedule != HM_SCHED_STAGED && schedule != HM_SCHED_PERSISTENT) ||
        (schedule == HM_SCHED_PERSISTENT && !m->p_ctl)) {
        hm::set_error("hm_set_schedule: null matrix, negative parameter, unknown schedule, or no persistent queue");
        return HM_EINVAL;
    }
    if (schedule == HM_SCHED_STAGED) {
        m->fork_after = param;
        m->dense_split = 0;   // one dense launch
    } else {
        hipError_t e = hipDeviceSynchronize();   // no product may be reading the queue being replaced
        if (e != hipSuccess) return hip_fail("hm_set_schedule: synchronize", e);
        hm_status st = set_dense_after(m, param);
        if (st != HM_OK) return st;
    }
    m->schedule = schedule;
    return HM_OK;
}

extern "C" hm_status hm_tune_mvm(hm_matrix* m, int32_t reps, hm_stream_t stream_, hm_tune_mvm_result* out) {
    if (!m || !out || reps < 1) {
        hm::set_error("hm_tune_mvm: null argument or reps < 1");
        return HM_EINVAL;
    }
    if (m->adj) {   // the adjoint's schedule is tuned as well (its result is not reported)
        hm_tune_mvm_result ra{};
        hm_status sa = hm_tune_mvm(m->adj, reps, stream_, &ra);
        if (sa != HM_OK) return sa;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device) {
        hm::set_error("hm_tune_mvm: current device differs from the matrix's device");
        return HM_EINVAL;
    }
    *out = hm_tune_mvm_result{};
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
    // time one candidate: `reps` replays of a captured graph of the product
    auto time_it = [&](double& t) -> hm_status {
        hm_graph* g = nullptr;
        hm_status s2 = hm_graph_create(m, 1.0, x, y, 0, stream_, &g);
        if (s2 != HM_OK) return s2;
        float ms = 0.0f;
        hipError_t e2 = hipSuccess;
        for (int i = 0; i < 2 && e2 == hipSuccess; ++i) e2 = hipGraphLaunch(g->exec, stream);   // warm-up
        if (e2 == hipSuccess) e2 = hipEventRecord(e0, stream);
        for (int i = 0; i < reps && e2 == hipSuccess; ++i) e2 = hipGraphLaunch(g->exec, stream);
        if (e2 == hipSuccess) e2 = hipEventRecord(e1, stream);
        if (e2 == hipSuccess) e2 = hipEventSynchronize(e1);
        if (e2 == hipSuccess) e2 = hipEventElapsedTime(&ms, e0, e1);
        hm_graph_free(g);
        if (e2 != hipSuccess) return hip_fail("hm_tune_mvm: timing", e2);
        t = (double)ms / reps;
        return HM_OK;
    };
    const int32_t keep_sched = m->schedule, keep_fork = m->fork_after, keep_da = m->p_dense_after;
    const int32_t keep_grid = m->aux_grid;
    int32_t best_sched = keep_sched, best_fork = keep_fork, best_da = keep_da, best_grid = keep_grid;
    double best_ms = 0.0;
    bool have = false;
    // staged schedule: every fork point of the dense stage, with the upload's
    // workgroup cap of that stage and with caps of 1, 2 and 3 workgroups per
    // compute unit (fewer dense waves leave the latency-bound chain stages
    // room on every compute unit)
    std::vector<int32_t> grids{keep_grid};
    int ncu = 0;
    if (m->aux && hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        for (int32_t g = 1; g <= 3; ++g)
            if (g * ncu != keep_grid) grids.push_back(g * ncu);
    m->schedule = HM_SCHED_STAGED;
    for (int32_t grid : grids) {
        m->aux_grid = grid;
        for (int32_t f = 0; f <= last && st == HM_OK; ++f) {
            m->fork_after = f;
            double t = 0.0;
            st = time_it(t);
            if (st != HM_OK) break;
            ++out->ncandidates;
            if (f == 0 && grid == keep_grid) out->ms_first = t;
            if (out->ms_staged == 0.0 || t < out->ms_staged) out->ms_staged = t;
            if (!have || t < best_ms) {
                best_sched = HM_SCHED_STAGED;
                best_fork = f;
                best_grid = grid;
                best_ms = t;
                have = true;
            }
        }
    }
    m->fork_after = best_sched == HM_SCHED_STAGED ? best_fork : keep_fork;
    m->aux_grid = best_sched == HM_SCHED_STAGED && st == HM_OK ? best_grid : keep_grid;
    // split dense stage: with the best fork point, the second part from a
    // later chain stage (at most 8 second fork points, spread), a quarter,
    // half or three quarters of the dense tasks in the first part
    const int32_t keep_f2 = m->fork2, keep_split = m->dense_split;
    int32_t best_f2 = keep_f2, best_split = 0;
    m->dense_split = 0;
    int32_t nd = 0;
    for (auto& ph : m->phases)
        if (ph.aux) nd += ph.ntasks;
    if (m->aux && nd >= 8 && best_sched == HM_SCHED_STAGED && st == HM_OK) {
        const int32_t span = last - best_fork;
        for (int32_t i = 1; i <= std::min(span, 8) && st == HM_OK; ++i) {
            const int32_t f2 = best_fork + (span <= 8 ? i : (int32_t)((int64_t)i * span / 8));
            for (int32_t q = 1; q <= 3 && st == HM_OK; ++q) {
                m->fork2 = f2;
                m->dense_split = (int32_t)((int64_t)nd * q / 4);
                double t = 0.0;
                st = time_it(t);
                if (st != HM_OK) break;
                ++out->ncandidates;
                if (out->ms_staged == 0.0 || t < out->ms_staged) out->ms_staged = t;
                if (t < best_ms) {
                    best_f2 = f2;
                    best_split = m->dense_split;
                    best_ms = t;
                }
            }
        }
    }
    m->fork2 = best_split > 0 ? best_f2 : keep_f2;
    m->dense_split = st == HM_OK ? best_split : keep_split;
    // persistent schedule: interleave points of the dense tasks (at most 17,
    // spread over 0 ... nchain of the queue)
    if (m->p_ctl && st == HM_OK) {
        m->schedule = HM_SCHED_PERSISTENT;
        const int32_t nc = m->p_queue.nchain;
        std::vector<int32_t> cand;
        for (int32_t i = 0; i <= std::min(nc, 16); ++i) {
            const int32_t v = nc <= 16 ? i : (int32_t)((int64_t)i * nc / 16);
            if (cand.empty() || cand.back() != v) cand.push_back(v);
        }
        for (int32_t da : cand) {
            st = set_dense_after(m, da);
            double t = 0.0;
            if (st == HM_OK) st = time_it(t);
            if (st == HM_OK) st = hm_matrix_check(m);   // an aborted launch must not be chosen
            if (st != HM_OK) break;
            ++out->ncandidates;
            if (out->ms_persistent == 0.0 || t < out->ms_persistent) out->ms_persistent = t;
            if (!have || t < best_ms) {
                best_sched = HM_SCHED_PERSISTENT;
                best_da = da;
                best_ms = t;
                have = true;
            }
        }
        if (st == HM_OK) st = set_dense_after(m, best_sched == HM_SCHED_PERSISTENT ? best_da : keep_da);
    }
    if (st == HM_OK) {
        m->schedule = best_sched;
        out->schedule = best_sched;
        out->fork_after = m->fork_after;
        out->fork2 = m->fork2;
        out->dense_split = m->schedule == HM_SCHED_STAGED ? m->dense_split : 0;
        out->dense_after = m->p_dense_after;
        out->dense_grid = m->aux_grid;
        out->ms = best_ms;
    } else {
        m->schedule = keep_sched;
        m->fork_after = keep_fork;
        m->aux_grid = keep_grid;
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
    std::vector<hm_matrix*> adj;
    if ((flags & HM_ADJOINT) && nmat > 0 && mats && nrhs) {
        if (!hm::adjoint_mats(mats, nmat, nrhs, adj, "hm_graph_create_batch")) return HM_EINVAL;
        mats = adj.data();
        flags &= ~HM_ADJOINT;
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
