// Device-side definitions shared by the single- and many-right-hand-side
// engines: storage decoders, the uploaded matrix object and its stages.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "hm_pack.h"

namespace hm {
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

// A 16-byte tile row holds V = floor(16 / element size) consecutive columns
// of one slab row.  decode<DT> widens the V stored values (float32 for the
// narrow formats, float64 for FP64 and the wide codecs); e is the AFLP
// exponent width of the task (ignored by the other formats).
template <int DT> struct Tile;
template <> struct Tile<HM_F64> {
    static constexpr int V = 2;
    using R = double;
    __device__ static void decode(const uint4& q, R* o, int) {
        o[0] = __hiloint2double((int)q.y, (int)q.x);
        o[1] = __hiloint2double((int)q.w, (int)q.z);
    }
};
template <> struct Tile<HM_F32> {
    static constexpr int V = 4;
    using R = float;
    __device__ static void decode(const uint4& q, R* o, int) {
        o[0] = __uint_as_float(q.x);
        o[1] = __uint_as_float(q.y);
        o[2] = __uint_as_float(q.z);
        o[3] = __uint_as_float(q.w);
    }
};
template <> struct Tile<HM_BF16> {
    static constexpr int V = 8;
    using R = float;
    __device__ static void decode(const uint4& q, R* o, int) {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = __uint_as_float(w[i] << 16);
            o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
    }
};
template <> struct Tile<HM_F16> {
    static constexpr int V = 8;
    using R = float;
    __device__ static void decode(const uint4& q, R* o, int) {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = f16_to_f32((uint16_t)(w[i] & 0xffffu));
            o[2 * i + 1] = f16_to_f32((uint16_t)(w[i] >> 16));
        }
    }
};
// gfx950 widens OCP E4M3 pairs in hardware (v_cvt_pk_f32_fp8: the low or
// high 16-bit half of a word), exact for every finite code.
__device__ __forceinline__ void fp8x4_to_f32(uint32_t w, float* o) {
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
    o[0] = lo[0];
    o[1] = lo[1];
    o[2] = hi[0];
    o[3] = hi[1];
}

template <> struct Tile<HM_FP8E4M3> {
    static constexpr int V = 16;
    using R = float;
    __device__ static void decode(const uint4& q, R* o, int) {
        fp8x4_to_f32(q.x, o);
        fp8x4_to_f32(q.y, o + 4);
        fp8x4_to_f32(q.z, o + 8);
        fp8x4_to_f32(q.w, o + 12);
    }
};

// ---- byte-aligned codecs (Sec. 4.1).  Code c of a B-byte format sits at
// bytes [cB, cB + B) of the 16-byte row, least significant byte first.
// bytes_at(w, o): the 32-bit little-endian word starting at byte o of the
// row (o is a constant once the decode loops are unrolled; bytes past the
// row read as zero).
__device__ __forceinline__ uint32_t bytes_at(const uint32_t* w, int o) {
    const int i = o >> 2, sh = o & 3;
    const uint32_t lo = w[i], hi = i < 3 ? w[i + 1] : 0u;
    return sh == 0 ? lo : __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)sh);
}

// FPX: the leading B bytes of the FP32 (B = 3) or FP64 (B = 5, 6, 7)
// encoding; the dropped low bytes are zero.
template <int B> struct FpxCodec {
    static constexpr int V = 16 / B;
    using R = typename std::conditional<(B <= 4), float, double>::type;
    __device__ static R elem(const uint32_t* w, int c) {
        if constexpr (B == 3) {
            return __uint_as_float(bytes_at(w, 3 * c) << 8);
        } else {
            const uint32_t hi = bytes_at(w, B * c + B - 4);
            const uint32_t lo = bytes_at(w, B * c) << (32 - 8 * (B - 4));
            return __hiloint2double((int)hi, (int)lo);
        }
    }
};

// AFLP: code = sign | z (e bits) | M (m' = 8B - 1 - e bits), value (before
// the column's scale 2^k) 2^(z-1) (1 + M / 2^m'), z = 0 zero.  Left-aligned
// in a 32-bit (B <= 3) or 64-bit word, the e + m' bits below the sign,
// shifted right by 8 - e (11 - e), land on the IEEE exponent and mantissa
// fields: the word then encodes 2^(z-127) (1 + f) (2^(z-1023) (1 + f)), and
// one exact multiplication by 2^126 (2^1022) gives the value; the zero code
// stays zero.  e <= 7 (float32) and e <= 10 (float64) are guaranteed by the
// upload.
template <int B> struct AflpCodec {
    static constexpr int V = 16 / B;
    using R = typename std::conditional<(B <= 3), float, double>::type;
    __device__ static R elem(const uint32_t* w, int c, int e) {
        if constexpr (B <= 3) {
            const uint32_t L = bytes_at(w, B * c) << (32 - 8 * B);
            const uint32_t t = ((L & 0x7FFFFFFFu) >> (8 - e)) | (L & 0x80000000u);
            return __uint_as_float(t) * 0x1p126f;
        } else {
            const uint32_t hi = bytes_at(w, B * c + B - 4);
            const uint32_t lo = B > 4 ? bytes_at(w, B * c) << (32 - 8 * (B - 4)) : 0u;
            const uint32_t hs = hi & 0x7FFFFFFFu;
            const uint32_t sh = (uint32_t)(11 - e);
            const uint32_t lo2 = __builtin_amdgcn_alignbit(hs, lo, sh);
            const uint32_t hi2 = (hs >> sh) | (hi & 0x80000000u);
            return __hiloint2double((int)hi2, (int)lo2) * 0x1p1022;
        }
    }
};

template <int B> struct FpxTile {
    static constexpr int V = FpxCodec<B>::V;
    using R = typename FpxCodec<B>::R;
    __device__ static R elem(const uint32_t* w, int c, int) { return FpxCodec<B>::elem(w, c); }
    __device__ static void decode(const uint4& q, R* o, int) {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int c = 0; c < V; ++c) o[c] = FpxCodec<B>::elem(w, c);
    }
};
template <int B> struct AflpTile {
    static constexpr int V = AflpCodec<B>::V;
    using R = typename AflpCodec<B>::R;
    __device__ static R elem(const uint32_t* w, int c, int e) { return AflpCodec<B>::elem(w, c, e); }
    __device__ static void decode(const uint4& q, R* o, int e) {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int c = 0; c < V; ++c) o[c] = AflpCodec<B>::elem(w, c, e);
    }
};
template <> struct Tile<HM_FPX24> : FpxTile<3> {};
template <> struct Tile<HM_FPX40> : FpxTile<5> {};
template <> struct Tile<HM_FPX48> : FpxTile<6> {};
template <> struct Tile<HM_FPX56> : FpxTile<7> {};
template <> struct Tile<HM_AFLP8> : AflpTile<1> {};
template <> struct Tile<HM_AFLP16> : AflpTile<2> {};
template <> struct Tile<HM_AFLP24> : AflpTile<3> {};
template <> struct Tile<HM_AFLP32> : AflpTile<4> {};
template <> struct Tile<HM_AFLP40> : AflpTile<5> {};
template <> struct Tile<HM_AFLP48> : AflpTile<6> {};
template <> struct Tile<HM_AFLP56> : AflpTile<7> {};

// float64 decode (wide accumulation whatever the matrix's mode)
template <int DT> constexpr bool kWide = std::is_same<typename Tile<DT>::R, double>::value;

// AFLP exponent width of a task (bits 8-11 of its mode)
__device__ __forceinline__ int task_ebits(int16_t mode) { return (mode >> 8) & 15; }

// dtype sets of the kernel instantiations that cover the codecs
constexpr int kMaskHw = 31;   // HM_F64 .. HM_FP8E4M3
constexpr int kMaskFpx = (1 << HM_F64) | (1 << HM_F32) | (1 << HM_BF16) | (0xF << HM_FPX24);
constexpr int kMaskAflp = (1 << HM_F64) | (1 << HM_F32) | (0x7F << HM_AFLP8);
constexpr int kMaskAll = kMaskHw | (0x7FF << HM_FPX24);

}  // namespace dev

struct DevStage {
    bool aux;
    int64_t t0;
    int32_t ntasks, nreduce, nowners;
    int32_t reduce_rows = 0;   // largest owner of the reduce list (many-RHS launch shape)
    int32_t mr_nrb = 0;        // many-RHS blocks per wave chosen for this stage (0 = the matrix's)
    struct Sub {               // many-RHS: a run of tasks of one dtype (tasks sorted by dtype)
        int32_t dtype, t0, ntasks;
    };
    std::vector<Sub> subs;
    const int32_t* reduce;
    int32_t dtype_mask;
    int64_t data_bytes;
    int64_t data_entries;
    double alg_bytes;
    double method_bytes = 0;
    std::string name;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;   // HM_TIMING event pairs
    int32_t timed_nrhs = 1;                                    // block width of the pending pairs
    int32_t timed_parts = 1;                                   // launches per product of the pending pairs
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
    float* ws32 = nullptr;
    double* part = nullptr;
    const int64_t* dsrc = nullptr;   // per workspace entry: 0 or the partial sums forming it
    int32_t fork_after = 0;          // main-stream stages before the second stream starts
    int32_t fork2 = 0;               // ... before the second part of a split dense stage starts
    int32_t dense_split = 0;         // tasks of the dense stage's first launch (0 = not split)
    const hm::DOwner* owners = nullptr;
    const hm::DItem* items = nullptr;
    const hm::DTask* tasks = nullptr;
    std::vector<hm::DevStage> phases;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
    // second stream for the independent dense stage, with fork/join events
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_fork2 = nullptr;
    int32_t aux_grid = 0;      // workgroup cap of the second-stream stage (0 = one wave per task)
    hm_stats stats{};
    int64_t ws_elems = 0;      // x in cluster order + coefficient vectors
    int64_t part_elems = 0;    // partial sums of split owners
    // host copy of the plan tables (the many-RHS plan is derived from them)
    std::vector<hm::DOwner> h_owners;
    std::vector<hm::DItem> h_items;
    std::vector<hm::DTask> h_tasks;
    std::vector<hm::Stage> h_stages;
    // many-RHS plan on the device (built on first use, rebuilt by the tuner)
    void* mr_meta = nullptr;
    const hm::DTask* mr_tasks = nullptr;
    const hm::DOwner* mr_owners = nullptr;
    const int64_t* mr_iperm = nullptr;   // cluster position of each original index
    std::vector<hm::DevStage> mr_phases;
    int64_t mr_part_elems = 0;
    int64_t mr_target = 0;
    int32_t mr_nrb = 1;        // right-hand-side blocks of 16 per wave (1 or 2)
    // many-right-hand-side workspace (grown on demand): R values per entry
    // of ws / ws32 / part, entry-major (value j of entry i at i * R + j)
    void* mr_arena = nullptr;
    int32_t mr_cap = 0;
    // bumped whenever mr_meta or mr_arena is replaced: graphs captured from
    // many-RHS products record it and are refused once it moved on
    uint64_t mr_gen = 0;
    double* wsm = nullptr;
    float* wsm32 = nullptr;
    double* ym = nullptr;      // y contributions in cluster order
    double* partm = nullptr;
    // persistent schedule (hm_persist.hip): the plan's tasks as one ticket
    // queue, per-owner completion counters, control words
    int32_t schedule = HM_SCHED_STAGED;
    int32_t p_nq = 0;            // queue entries
    int32_t p_mask = 0;          // dtypes of the tasks
    int32_t p_grid = 0;          // workgroups of the persistent launch
    int32_t p_dense_after = 0;
    int32_t p_grab = 1;          // tickets a wave takes per atomic
    int64_t p_nowners = 0;
    uint64_t p_spin = 0;         // bound of a dependency wait, 100 MHz ticks
    const hm::DTask* p_tasks = nullptr;
    const int32_t* p_dep_first = nullptr;
    const int32_t* p_deps = nullptr;
    const int32_t* p_target = nullptr;
    int32_t* p_order = nullptr;
    int32_t* p_done = nullptr;
    uint32_t* p_ctl = nullptr;   // ticket, abort, error
    hm::Queue p_queue;           // host copy (the tuner reorders it)
    int32_t sync = HM_SYNC_OWNER;
    double* ypriv = nullptr;     // HM_SYNC_PRIVATE: eight copies of y in cluster order
    // the adjoint M^T (HM_ADJOINT), uploaded with its own transposed layout
    hm_matrix* adj = nullptr;
    hm_layout* adj_layout = nullptr;
    std::vector<hm::DevStage> pphases;   // the persistent launch, for HM_TIMING
};

namespace hm {

// One block of right-hand sides for mvm_blocks: Y := alpha * M * X + Y in
// float64, column-major.
struct BlockCall {
    hm_matrix* m;
    double alpha;
    const double* X;
    int64_t ldx;
    int nrhs;
    double* Y;
    int64_t ldy;
};

// Run blocks of distinct matrices through the many-right-hand-side engine
// (any width >= 1, including single columns), merged as in hm_mvm_batch.
hm_status mvm_blocks(const BlockCall* calls, int ncalls, hipStream_t stream);

// HM_ADJOINT: the adjoints of a batch's matrices (error set and false if one
// was uploaded without).
bool adjoint_mats(hm_matrix* const* mats, int32_t nmat, const int32_t* nrhs, std::vector<hm_matrix*>& out,
                  const char* who);

// Size the many-RHS workspaces of a batch (see hm_mvm_batch) ahead of a call.
hm_status batch_prepare(hm_matrix* const* mats, int32_t nmat, const int32_t* nrhs, int32_t vec_dtype);

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// HM_TIMING: take an event pair for one phase launch of block width
// `width` (pending pairs of another width are dropped first).
inline bool timing_acquire(hm_matrix* m, DevStage& ph, int32_t width, std::pair<hipEvent_t, hipEvent_t>& ev) {
    if (ph.timed_nrhs != width) {
        for (auto& e : ph.pending) m->event_pool.push_back(e);
        ph.pending.clear();
        ph.timed_nrhs = width;
    }
    if (m->event_pool.empty()) {
        if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) return false;
    } else {
        ev = m->event_pool.back();
        m->event_pool.pop_back();
    }
    return true;
}

// ... and record its start event on `s` (phases of several launches: the
// pair brackets all of them)
inline bool timing_begin(hm_matrix* m, DevStage& ph, int32_t width, hipStream_t s,
                         std::pair<hipEvent_t, hipEvent_t>& ev) {
    return timing_acquire(m, ph, width, ev) && hipEventRecord(ev.first, s) == hipSuccess;
}

inline void timing_end(DevStage& ph, hipStream_t s, const std::pair<hipEvent_t, hipEvent_t>& ev) {
    (void)hipEventRecord(ev.second, s);
    ph.pending.push_back(ev);
}

inline hm_status hip_fail(const char* what, hipError_t e) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return HM_EDEVICE;
}

}  // namespace hm
