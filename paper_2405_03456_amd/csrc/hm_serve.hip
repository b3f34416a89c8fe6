// Request loop over resident matrices: memory-admitted continuous batching.
//
// Submitting threads only append to a FIFO queue.  One scheduler thread owns
// every device call: it retires finished launch groups (event queries),
// forms the next group from the queue and enqueues it on the idle one of
// two streams, so one group's copies and products overlap the next group's.
// A group takes queued requests in FIFO order whose matrix is not in flight
// (a matrix's workspace serves one product at a time), concatenates the
// columns of requests for the same matrix into one block, and reserves each
// block's device and pinned staging memory from first-fit arenas; a request
// that does not fit stays queued (admission), and later requests do not pass
// it for the same matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hm_device.h"

namespace hm {
namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
public:
    void reset(int64_t size) {
        free_.clear();
        if (size > 0) free_[0] = size;
        size_ = size;
        used_ = 0;
        peak_ = 0;
    }
    int64_t alloc(int64_t bytes) {
        bytes = (bytes + 255) & ~int64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                const int64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return off;
            }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = (bytes + 255) & ~int64_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t size() const { return size_; }
    int64_t peak() const { return peak_; }

private:
    std::map<int64_t, int64_t> free_;
    int64_t size_ = 0, used_ = 0, peak_ = 0;
};

// Host copies of request blocks to and from the pinned staging arena, spread
// over a few worker threads (one thread moves a few GB/s of pageable data).
// run() cuts every job into pieces of at most kPiece values and returns when
// all pieces are done; the calling thread works too.
class CopyPool {
public:
    struct Job {
        double* dst;
        const double* src;
        int64_t count;
        double scale;   // dst = scale * src (1.0: a plain copy)
    };
    explicit CopyPool(int nthreads) {
        for (int i = 0; i < nthreads; ++i) th_.emplace_back([this] { work(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    void run(const std::vector<Job>& jobs) {
        std::vector<Job> pieces;
        for (const Job& j : jobs)
            for (int64_t o = 0; o < j.count; o += kPiece)
                pieces.push_back(Job{j.dst + o, j.src + o, std::min(kPiece, j.count - o), j.scale});
        if (pieces.empty()) return;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (const Job& p : pieces) q_.push_back(p);
            pending_ += (int64_t)pieces.size();
        }
        cv_.notify_all();
        for (;;) {   // help until the queue is empty, then wait for the rest
            Job j;
            {
                std::unique_lock<std::mutex> lk(mu_);
                if (q_.empty()) {
                    done_cv_.wait(lk, [&] { return pending_ == 0; });
                    return;
                }
                j = q_.front();
                q_.pop_front();
            }
            exec(j);
            finish();
        }
    }

private:
    static constexpr int64_t kPiece = 1 << 17;
    static void exec(const Job& j) {
        if (j.scale == 1.0)
            std::memcpy(j.dst, j.src, sizeof(double) * (size_t)j.count);
        else
            for (int64_t i = 0; i < j.count; ++i) j.dst[i] = j.scale * j.src[i];
    }
    void finish() {
        std::lock_guard<std::mutex> lk(mu_);
        if (--pending_ == 0) done_cv_.notify_all();
    }
    void work() {
        for (;;) {
            Job j;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
                if (stop_ && q_.empty()) return;
                j = q_.front();
                q_.pop_front();
            }
            exec(j);
            finish();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Job> q_;
    int64_t pending_ = 0;
    bool stop_ = false;
    std::vector<std::thread> th_;
};

struct Req {
    int32_t mid;
    double alpha;
    const double* X;
    int32_t nrhs;
    double* Y;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;   // 0 queued, 1 running, 2 done, 3 failed
    hm_status status = HM_OK;
    int64_t group_id = -1;
    int32_t group_requests = 0, group_cols = 0;
};

struct Mat {
    hm_matrix* m;   // null for a shape placeholder
    int64_t n;
    bool busy = false;
};

struct Block {          // one matrix's concatenated columns in a group
    int32_t mid;
    hm_matrix* m = nullptr;
    int64_t n = 0;
    int32_t cols = 0;
    std::vector<uint64_t> tickets;
    std::vector<int32_t> cols_of;                   // columns of each ticket
    std::vector<const double*> x_of;                // its X
    std::vector<std::pair<double*, double>> y_of;   // its Y and alpha
    int64_t dev_off = -1, host_off = -1, bytes = 0;   // X block then Y block
};

struct Group {
    int64_t id;
    std::vector<Block> blocks;
    int stream;
    hipEvent_t done = nullptr;
    double t_fake_end = 0;
    hm_status status = HM_OK;
    int32_t nreq = 0;
};

}  // namespace
}  // namespace hm

struct hm_server {
    hm_serve_opts opts{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::thread th;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, hm::Req> reqs;
    std::vector<hm::Mat> mats;
    hm::Arena dev_arena, host_arena;
    uint8_t* dev_base = nullptr;
    uint8_t* host_base = nullptr;
    hipStream_t streams[2] = {nullptr, nullptr};
    std::vector<hm::Group> inflight;
    std::vector<hipEvent_t> event_pool;
    uint64_t next_ticket = 1;
    int64_t next_group = 0;
    int32_t inflight_reqs = 0;
    hm_serve_stats stats{};
    std::unique_ptr<hm::CopyPool> pool;   // host staging copies
};

namespace hm {
namespace {

int64_t block_bytes(int64_t n, int32_t cols) { return 2 * (((n * cols * 8) + 255) & ~int64_t(255)); }

// Results of a finished group: the copies to the callers' Y (alpha applied),
// made without the lock (the group's requests are not touched by other
// threads until they are marked done).
std::vector<CopyPool::Job> result_copies(hm_server* S, const Group& g,
                                         const std::vector<std::pair<double*, double>>& dst) {
    std::vector<CopyPool::Job> jobs;
    if (g.status != HM_OK || S->opts.fake) return jobs;
    size_t k = 0;
    for (const Block& b : g.blocks) {
        const double* Yst = (const double*)(S->host_base + b.host_off + b.bytes / 2);
        int64_t c = 0;
        for (size_t t = 0; t < b.tickets.size(); ++t, ++k) {
            jobs.push_back(CopyPool::Job{dst[k].first, Yst + c * b.n, b.n * b.cols_of[t], dst[k].second});
            c += b.cols_of[t];
        }
    }
    return jobs;
}

// Mark a finished group's requests done and release its memory (lock held).
void retire(hm_server* S, Group& g) {
    const double t = now_ms();
    for (Block& b : g.blocks) {
        Mat& M = S->mats[b.mid];
        for (uint64_t tk : b.tickets) {
            Req& r = S->reqs[tk];
            if (g.status == HM_OK) {
                if (S->opts.fake) std::memset(r.Y, 0, sizeof(double) * (size_t)(b.n * r.nrhs));
                r.state = 2;
            } else {
                r.state = 3;
                r.status = g.status;
            }
            r.t_done = t;
            S->stats.completed++;
        }
        S->dev_arena.release(b.dev_off, b.bytes);
        S->host_arena.release(b.host_off, b.bytes);
        M.busy = false;
    }
    S->inflight_reqs -= g.nreq;
    if (g.done) S->event_pool.push_back(g.done);
}

// Form a launch group from the queue (lock held); empty if nothing can run.
Group form_group(hm_server* S, int stream) {
    Group g;
    g.id = S->next_group;
    g.stream = stream;
    std::map<int32_t, size_t> at;            // matrix -> block index
    std::vector<bool> blocked(S->mats.size(), false);
    const double t = now_ms();
    for (auto it = S->queue.begin(); it != S->queue.end();) {
        Req& r = S->reqs[*it];
        Mat& M = S->mats[r.mid];
        if (M.busy || blocked[r.mid] || S->inflight_reqs + g.nreq >= S->opts.max_slots) {
            blocked[r.mid] = true;           // keep FIFO order per matrix
            ++it;
            continue;
        }
        auto f = at.find(r.mid);
        Block* b = f == at.end() ? nullptr : &g.blocks[f->second];
        if (b && b->cols + r.nrhs > S->opts.max_cols) {
            blocked[r.mid] = true;
            ++it;
            continue;
        }
        if (!b) {
            g.blocks.push_back(Block{});
            g.blocks.back().mid = r.mid;
            g.blocks.back().m = M.m;
            g.blocks.back().n = M.n;
            at[r.mid] = g.blocks.size() - 1;
            b = &g.blocks.back();
        }
        b->cols += r.nrhs;
        b->tickets.push_back(*it);
        b->cols_of.push_back(r.nrhs);
        b->x_of.push_back(r.X);
        b->y_of.emplace_back(r.Y, r.alpha);
        g.nreq++;
        it = S->queue.erase(it);
    }
    // memory admission, block by block; a block that does not fit goes back
    std::vector<Block> kept;
    std::vector<uint64_t> back;
    for (Block& b : g.blocks) {
        Mat& M = S->mats[b.mid];
        b.bytes = block_bytes(M.n, b.cols);
        b.dev_off = S->dev_arena.alloc(b.bytes);
        b.host_off = b.dev_off >= 0 ? S->host_arena.alloc(b.bytes) : -1;
        if (b.dev_off < 0 || b.host_off < 0) {
            if (b.dev_off >= 0) S->dev_arena.release(b.dev_off, b.bytes);
            for (uint64_t tk : b.tickets) back.push_back(tk);
            g.nreq -= (int32_t)b.tickets.size();
            continue;
        }
        M.busy = true;
        for (uint64_t tk : b.tickets) {
            Req& r = S->reqs[tk];
            r.state = 1;
            r.t_admit = t;
            r.group_id = g.id;
            r.group_cols = b.cols;
        }
        kept.push_back(std::move(b));
    }
    // requests that did not fit return to the queue head in their order
    std::sort(back.begin(), back.end());
    for (auto it = back.rbegin(); it != back.rend(); ++it) S->queue.push_front(*it);
    g.blocks = std::move(kept);
    for (Block& b : g.blocks)
        for (uint64_t tk : b.tickets) S->reqs[tk].group_requests = g.nreq;
    if (!g.blocks.empty()) {
        S->next_group++;
        S->inflight_reqs += g.nreq;
        S->stats.groups++;
        S->stats.peak_inflight = std::max<int32_t>(S->stats.peak_inflight, S->inflight_reqs);
        S->stats.max_group_requests = std::max<int32_t>(S->stats.max_group_requests, g.nreq);
        S->stats.peak_arena_bytes = std::max(S->stats.peak_arena_bytes, S->dev_arena.peak());
    }
    return g;
}

// Stage inputs, enqueue copies and products of a formed group (no lock held:
// the group's requests and blocks are owned by this thread until retired).
hm_status launch(hm_server* S, Group& g) {
    if (S->opts.fake) {
        g.t_fake_end = now_ms() + S->opts.fake_us * 1e-3;
        return HM_OK;
    }
    hipStream_t s = S->streams[g.stream];
    std::vector<BlockCall> calls;
    std::vector<CopyPool::Job> xcopies;
    for (Block& b : g.blocks) {
        double* Xst = (double*)(S->host_base + b.host_off);
        int64_t c = 0;
        for (size_t t = 0; t < b.tickets.size(); ++t) {
            xcopies.push_back(CopyPool::Job{Xst + c * b.n, b.x_of[t], b.n * b.cols_of[t], 1.0});
            c += b.cols_of[t];
        }
    }
    S->pool->run(xcopies);
    for (Block& b : g.blocks) {
        const int64_t n = b.n, half = b.bytes / 2;
        double* Xst = (double*)(S->host_base + b.host_off);
        double* Xd = (double*)(S->dev_base + b.dev_off);
        double* Yd = (double*)(S->dev_base + b.dev_off + half);
        hipError_t e = hipMemcpyAsync(Xd, Xst, sizeof(double) * n * b.cols, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(Yd, 0, sizeof(double) * n * b.cols, s);
        if (e != hipSuccess) return hip_fail("hm_serve: staging copy", e);
        calls.push_back(BlockCall{b.m, 1.0, Xd, n, b.cols, Yd, n});
    }
    hm_status st = mvm_blocks(calls.data(), (int)calls.size(), s);
    if (st != HM_OK) return st;
    for (Block& b : g.blocks) {
        const int64_t n = b.n, half = b.bytes / 2;
        hipError_t e = hipMemcpyAsync(S->host_base + b.host_off + half, S->dev_base + b.dev_off + half,
                                      sizeof(double) * n * b.cols, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_fail("hm_serve: result copy", e);
    }
    if (S->event_pool.empty()) {
        hipError_t e = hipEventCreateWithFlags(&g.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail("hm_serve: event", e);
    } else {
        g.done = S->event_pool.back();
        S->event_pool.pop_back();
    }
    hipError_t e = hipEventRecord(g.done, s);
    if (e != hipSuccess) return hip_fail("hm_serve: event record", e);
    return HM_OK;
}

bool group_finished(hm_server* S, const Group& g) {
    if (g.status != HM_OK) return true;
    if (S->opts.fake) return now_ms() >= g.t_fake_end;
    return hipEventQuery(g.done) == hipSuccess;
}

void loop(hm_server* S) {
    if (!S->opts.fake) (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // retire finished groups: copy results out without the lock, then
        // mark the requests done
        for (size_t i = 0; i < S->inflight.size();) {
            if (group_finished(S, S->inflight[i])) {
                Group g = std::move(S->inflight[i]);
                S->inflight.erase(S->inflight.begin() + i);
                std::vector<std::pair<double*, double>> dst;
                for (const Block& b : g.blocks) dst.insert(dst.end(), b.y_of.begin(), b.y_of.end());
                lk.unlock();
                S->pool->run(result_copies(S, g, dst));
                lk.lock();
                retire(S, g);
                S->cv.notify_all();
            } else {
                ++i;
            }
        }
        // one group per idle stream
        bool launched = false;
        if (S->inflight.size() < 2 && !S->queue.empty()) {
            int used = S->inflight.empty() ? -1 : S->inflight[0].stream;
            Group g = form_group(S, used == 0 ? 1 : 0);
            if (!g.blocks.empty()) {
                lk.unlock();
                g.status = launch(S, g);
                // a failed launch may have queued work on the stream: let it
                // finish before the group's memory is released
                if (g.status != HM_OK && !S->opts.fake) (void)hipStreamSynchronize(S->streams[g.stream]);
                lk.lock();
                S->inflight.push_back(std::move(g));
                launched = true;
            }
        }
        if (S->stop && S->queue.empty() && S->inflight.empty()) break;
        if (launched) continue;
        if (S->inflight.empty())
            S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
        else
            S->cv.wait_for(lk, std::chrono::microseconds(50));
    }
}

}  // namespace
}  // namespace hm

extern "C" hm_status hm_serve_create(const hm_serve_opts* o, hm_server** out) {
    if (!o || !out || o->mem_budget <= 0 || o->max_slots <= 0 || o->max_queue <= 0 || o->max_cols <= 0 ||
        o->max_cols > HM_MAX_NRHS || o->fake_us < 0) {
        hm::set_error("hm_serve_create: bad options");
        return HM_EINVAL;
    }
    *out = nullptr;
    hm_server* S = new (std::nothrow) hm_server();
    if (!S) {
        hm::set_error("hm_serve_create: out of host memory");
        return HM_ENOMEM;
    }
    S->opts = *o;
    S->dev_arena.reset(o->mem_budget);
    S->host_arena.reset(o->mem_budget);
    if (o->fake) {
        S->host_base = new (std::nothrow) uint8_t[1];
    } else {
        hipError_t e = hipGetDevice(&S->device);
        void* d = nullptr;
        void* h = nullptr;
        if (e == hipSuccess) e = hipMalloc(&d, (size_t)o->mem_budget);
        if (e == hipSuccess) e = hipHostMalloc(&h, (size_t)o->mem_budget, hipHostMallocDefault);
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking);
        S->dev_base = (uint8_t*)d;
        S->host_base = (uint8_t*)h;
        if (e != hipSuccess) {
            hm_serve_destroy(S);
            return hm::hip_fail("hm_serve_create", e);
        }
    }
    try {
        S->pool.reset(new hm::CopyPool(3));
        S->th = std::thread(hm::loop, S);
    } catch (...) {
        hm_serve_destroy(S);
        hm::set_error("hm_serve_create: cannot start the scheduler thread");
        return HM_ENOMEM;
    }
    *out = S;
    return HM_OK;
}

extern "C" hm_status hm_serve_register(hm_server* S, hm_matrix* m, int32_t* id) {
    if (!S || !m || !id || S->opts.fake) {
        hm::set_error("hm_serve_register: null argument or fake server");
        return HM_EINVAL;
    }
    // size the matrix's many-RHS workspace for the widest group now, not in the loop
    int32_t cols = S->opts.max_cols;
    hm_status st = hm::batch_prepare(&m, 1, &cols, HM_F64);
    if (st != HM_OK) return st;
    std::lock_guard<std::mutex> lk(S->mu);
    S->mats.push_back(hm::Mat{m, m->n});
    *id = (int32_t)S->mats.size() - 1;
    return HM_OK;
}

extern "C" hm_status hm_serve_register_shape(hm_server* S, int64_t n, int32_t* id) {
    if (!S || !id || !S->opts.fake || n <= 0) {
        hm::set_error("hm_serve_register_shape: needs a fake server and n > 0");
        return HM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->mats.push_back(hm::Mat{nullptr, n});
    *id = (int32_t)S->mats.size() - 1;
    return HM_OK;
}

extern "C" hm_status hm_serve_submit(hm_server* S, int32_t mid, double alpha, const double* X, int32_t nrhs,
                                     double* Y, uint64_t* ticket) {
    if (!S || !X || !Y || !ticket || nrhs < 1 || nrhs > HM_MAX_NRHS) {
        hm::set_error("hm_serve_submit: null argument or nrhs out of range");
        return HM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (mid < 0 || mid >= (int32_t)S->mats.size()) {
        hm::set_error("hm_serve_submit: unknown matrix id");
        return HM_EINVAL;
    }
    if (nrhs > S->opts.max_cols) {
        hm::set_error("hm_serve_submit: nrhs exceeds the server's max_cols (its workspaces are sized for that)");
        return HM_EINVAL;
    }
    if (hm::block_bytes(S->mats[mid].n, nrhs) > S->opts.mem_budget) {
        hm::set_error("hm_serve_submit: request larger than the memory budget");
        return HM_ENOMEM;
    }
    if ((int32_t)S->queue.size() >= S->opts.max_queue) {
        hm::set_error("hm_serve_submit: queue full");
        return HM_EBUSY;
    }
    const uint64_t t = S->next_ticket++;
    hm::Req r;
    r.mid = mid;
    r.alpha = alpha;
    r.X = X;
    r.nrhs = nrhs;
    r.Y = Y;
    r.t_submit = hm::now_ms();
    S->reqs.emplace(t, r);
    S->queue.push_back(t);
    S->stats.submitted++;
    *ticket = t;
    S->cv.notify_all();
    return HM_OK;
}

extern "C" hm_status hm_serve_poll(hm_server* S, uint64_t ticket, int32_t* done, hm_req_stats* st) {
    if (!S || !done) {
        hm::set_error("hm_serve_poll: null argument");
        return HM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        hm::set_error("hm_serve_poll: unknown or released ticket");
        return HM_EINVAL;
    }
    const hm::Req& r = it->second;
    *done = r.state >= 2 ? 1 : 0;
    if (r.state < 2) return HM_OK;
    if (st) {
        st->queue_ms = r.t_admit - r.t_submit;
        st->run_ms = r.t_done - r.t_admit;
        st->latency_ms = r.t_done - r.t_submit;
        st->group_id = r.group_id;
        st->group_requests = r.group_requests;
        st->group_cols = r.group_cols;
    }
    const hm_status status = r.state == 3 ? r.status : HM_OK;
    S->reqs.erase(it);
    if (status != HM_OK) hm::set_error("hm_serve_poll: the product of this request failed");
    return status;
}

extern "C" hm_status hm_serve_stats_read(hm_server* S, hm_serve_stats* out) {
    if (!S || !out) {
        hm::set_error("hm_serve_stats_read: null argument");
        return HM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    return HM_OK;
}

extern "C" void hm_serve_destroy(hm_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->th.joinable()) S->th.join();
    for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
    for (auto& g : S->inflight)
        if (g.done) (void)hipEventDestroy(g.done);
    if (!S->opts.fake) {
        for (hipStream_t s : S->streams)
            if (s) (void)hipStreamDestroy(s);
        if (S->dev_base) (void)hipFree(S->dev_base);
        if (S->host_base) (void)hipHostFree(S->host_base);
    } else {
        delete[] S->host_base;
    }
    delete S;
}
