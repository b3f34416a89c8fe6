// Persistent schedule of the single-vector product: one launch runs the
// whole ticket queue built by hm_queue.cpp (every task of every stage, the
// dense near field interleaved, the reductions of split owners).
//
// Each wavefront repeatedly takes the next ticket from an atomic counter,
// waits until the owners its item reads are complete, runs the item with the
// same body as the per-stage kernels, and counts its owner's completion.
//
// Ordering across the chip: coefficient vectors and partial sums written in
// this launch are stored and loaded with device-scope relaxed atomics, which
// are coherent across the XCDs' L2 caches.  A wave waits for its own stores
// to complete (s_waitcnt vmcnt(0)) before it increments the completion
// counter, and a consumer reads the inputs only after it has seen the
// counter at its target, so it reads the final values.  x (gathered by the
// launch before) and the stored matrix are read with ordinary loads.
//
// Termination: tickets are handed out in queue order and every item follows
// its producers, so a wave only waits for smaller tickets held by running
// waves.  Each wait is nevertheless bounded: past `spin_limit` ticks of the
// 100 MHz real-time counter the wave records an error in ctl[2], raises the
// abort flag ctl[1] and leaves; every other waiting wave sees the flag and
// leaves too, so the launch always ends.  The host reads ctl[2]
// (hm_matrix_check).
#include <hip/hip_runtime.h>

#include <array>
#include <utility>

#include "hm_stream.h"

namespace hm {
namespace dev {

constexpr uint32_t kCtlTicket = 0, kCtlAbort = 1, kCtlError = 2;

__device__ __forceinline__ int32_t ld_counter(const int32_t* p) {
    return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until owners owner_of(0 .. nlist) have done[o] >= want(o).  Lanes
// check up to 64 owners at a time.  false: the wait was abandoned (bound or
// abort).
template <typename OwnerOf, typename Want>
__device__ __forceinline__ bool wait_owners(OwnerOf owner_of, int nlist, const int32_t* done, uint32_t* ctl,
                                            uint64_t spin_limit, int lane, Want want) {
    for (int base = 0; base < nlist; base += 64) {
        const int i = base + lane;
        const int32_t o = i < nlist ? owner_of(i) : -1;
        const int32_t w = o >= 0 ? want(o) : 0;
        uint64_t t0 = 0;
        for (uint32_t spin = 0;; ++spin) {
            const bool ok = o < 0 || ld_counter(done + o) >= w;
            if (__all(ok)) break;
            const uint32_t ab = __hip_atomic_load(ctl + kCtlAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__builtin_amdgcn_readfirstlane(ab) != 0) return false;
            const uint64_t now = __builtin_amdgcn_s_memrealtime();
            if (spin == 0) {
                t0 = now;
            } else if (now - t0 > spin_limit) {
                if (lane == 0) {
                    __hip_atomic_store(ctl + kCtlError, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(ctl + kCtlAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                return false;
            }
            // back off: waiting waves keep polling traffic low
            if (spin < 8)
                __builtin_amdgcn_s_sleep(2);
            else if (spin < 64)
                __builtin_amdgcn_s_sleep(16);
            else
                __builtin_amdgcn_s_sleep(127);
        }
    }
    return true;
}

template <bool ACC64, int MASK>
__global__ __launch_bounds__(256) void k_persistent(
    const int32_t* __restrict__ queue, int nq, const int32_t* __restrict__ dep_first,
    const int32_t* __restrict__ deps, const int32_t* __restrict__ target, int32_t* done, uint32_t* ctl,
    uint64_t spin_limit, const DTask* __restrict__ tasks, const DOwner* __restrict__ owners,
    const DItem* __restrict__ items, const uint8_t* __restrict__ data, const double* __restrict__ scales,
    const double* __restrict__ vin, const float* __restrict__ vin32, double* vout, float* vout32,
    double* __restrict__ part, const int64_t* __restrict__ dsrc, double* __restrict__ y,
    const int64_t* __restrict__ perm, double alpha, int nx, int grab) {
    __shared__ double lds_w[4][MAX_TASK_INPUTS];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // a wave takes `grab` consecutive tickets per atomic and runs them in
    // order (the smallest unfinished ticket is still never waiting)
    int q = 0, qend = 0;
    for (;; ++q) {
        if (q >= qend) {
            uint32_t tk_ = 0;
            if (lane == 0)
                tk_ = __hip_atomic_fetch_add(ctl + kCtlTicket, (uint32_t)grab, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
            q = (int)__builtin_amdgcn_readfirstlane(tk_);
            qend = q + grab;
        }
        if (q >= nq) break;
        const int32_t e = queue[q];
        int32_t owner;
        if (e >= 0) {
            const DTask tk = tasks[e];
            owner = tk.owner;
            const int32_t d0 = dep_first[e], d1 = dep_first[e + 1];
            if (d1 > d0 && !wait_owners([&](int i) { return deps[d0 + i]; }, d1 - d0, done, ctl, spin_limit, lane,
                                        [&](int32_t o) { return target[o]; }))
                break;
            run_task<ACC64, MASK, true>(tk, lane, lds_w[wave], items, data, scales, vin, vin32, vout, vout32, part,
                                        dsrc, y, perm, alpha, nx, nullptr, 0);
        } else {
            owner = ~e;
            const DOwner ow = owners[owner];
            if (!wait_owners([&](int) { return owner; }, 1, done, ctl, spin_limit, lane,
                             [&](int32_t) { return ow.ntasks; }))
                break;
            run_reduce<true>(ow, lane, part, vout, vout32, y, perm, alpha);
        }
        // this wave's stores are complete before its owner's counter moves
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane == 0) __hip_atomic_fetch_add(done + owner, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// x in cluster order, and the persistent schedule's counters cleared for the
// next launch: done[0 .. ndone) = 0, ticket = 0, abort = 0 (the error word
// is kept until the host reads it).
__global__ __launch_bounds__(256) void k_gather_reset(const double* __restrict__ x, const int64_t* __restrict__ perm,
                                                      double* __restrict__ ws, float* __restrict__ ws32, int64_t n,
                                                      int cluster_order, int32_t* __restrict__ done, int64_t ndone,
                                                      uint32_t* __restrict__ ctl) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const double v = cluster_order ? x[i] : x[perm[i]];
        ws[i] = v;
        ws32[i] = (float)v;
    }
    if (i < ndone) done[i] = 0;
    if (i == 0) {
        ctl[kCtlTicket] = 0;
        ctl[kCtlAbort] = 0;
    }
}

// Instantiated dtype sets: the first of these containing the matrix's
// dtypes is launched (a task switches on its own dtype inside).
static constexpr int kNPersist = 10;
static constexpr int kPersistMasks[kNPersist] = {1, 2, 3, 7, 11, 19, 31, kMaskFpx, kMaskAflp, kMaskAll};

template <bool ACC64, int... I>
static constexpr std::array<PersistKernel, sizeof...(I)> persist_table(std::integer_sequence<int, I...>) {
    return {{&k_persistent<ACC64, kPersistMasks[I]>...}};
}

static const std::array<PersistKernel, kNPersist> kPersist[2] = {
    persist_table<false>(std::make_integer_sequence<int, kNPersist>{}),
    persist_table<true>(std::make_integer_sequence<int, kNPersist>{})};

PersistKernel persist_kernel(bool acc64, int mask, int* launched_mask) {
    for (int i = 0; i < kNPersist; ++i)
        if ((mask & ~kPersistMasks[i]) == 0) {
            if (launched_mask) *launched_mask = kPersistMasks[i];
            return kPersist[acc64 ? 1 : 0][i];
        }
    return nullptr;
}

}  // namespace dev
}  // namespace hm
