// Serving engine: continuous batching of many small dense D-PT problems.
//
// A worker thread owns one stream, a device arena of the configured budget
// and a slot table.  Each engine step:
//   1. applies the map of eq. (dyn) (Kenmoe, Smerlak, Zadorin, arXiv:2002.12872,
//      Sec. II.B) once to every problem admitted earlier: one persistent
//      grouped pre-pass and one persistent grouped fused step per precision
//      phase and tile shape over a device work table (a HIP graph replayed
//      every step);
//   2. meanwhile admits waiting problems in FIFO order while the arena and the
//      slots have room: one upload per host-submitted problem (theta and Delta
//      staged together in a pinned ring), none for device-resident ones, then
//      one grouped launch for all of them (padded FP32/BF16 copies, transpose,
//      and the closed-form first iterate);
//   3. reads every problem's (delta, max|W|) back and runs its own controller
//      (the same stopping rule as dpt_solve);
//   4. retires finished problems with one grouped launch (eigenvalues into a
//      staging buffer, optional eigenvectors exported), releasing their arena
//      space at once; their results are handed out after the next
//      synchronisation of the stream.
#include <hip/hip_runtime.h>
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdint>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "controller.h"
#include "dpt.h"
#include "dpt_internal.h"

using namespace dpt;

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of neighbouring holes.
class Arena {
  public:
    void init(size_t size) {
        holes_.clear();
        holes_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = holes_.begin(); it != holes_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                holes_.erase(it);
                if (rest) holes_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = holes_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != holes_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            holes_.erase(next);
        }
        if (it != holes_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                holes_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> holes_;
};

struct Request {
    int64_t id = 0, n = 0, ld = 0;
    double lambda = 0.0;
    dpt_options opt{};
    bool bf16 = false, symmetric = false, want_z = false;
    // host submissions: theta (padded to ld) followed by the FP32 Delta (n*n
    // row-major) in the pinned ring until uploaded, else in the two vectors
    std::vector<double> theta;
    std::vector<float> delta;
    unsigned char *staged = nullptr;
    size_t ring_off = 0;
    // device submissions: the caller's arrays, read at admission
    const double *dev_theta = nullptr;
    const void *dev_delta = nullptr;
    bool dev_f64 = false;
    // device memory inside the arena
    size_t off = 0, bytes = 0;
    int slot = -1;
    double *theta_d = nullptr, *d_d = nullptr;
    float *W[2] = {nullptr, nullptr}, *D = nullptr, *DT = nullptr;
    __bf16 *Wb[2] = {nullptr, nullptr}, *Db = nullptr;
    int cur = 0;
    bool at_identity = true;
    Controller ctl;
    double t_submit = 0, t_admit = -1, t_first = -1, t_finish = -1;
    std::vector<double> E;
    std::vector<float> Z;
    int status = DPT_NOT_CONVERGED;
};

// Ring allocator over one pinned host buffer: submissions stage their FP32
// Delta here so that the worker's upload is an asynchronous DMA (a copy from
// pageable memory would block the worker for the whole transfer).  Space is
// handed out in order and reclaimed from the oldest allocation once it and
// every allocation before it have been released (releases may come in any
// order).
struct PinnedRing {
    struct Entry {
        size_t off, bytes;
        bool released;
    };
    unsigned char *base = nullptr;
    size_t cap = 0, head = 0;
    std::deque<Entry> live;  // in allocation order

    bool alloc(size_t bytes, size_t *off) {
        bytes = round_up(bytes);
        if (bytes == 0 || bytes > cap) return false;
        size_t at;
        if (live.empty()) {
            at = 0;
        } else {
            const size_t tail = live.front().off;
            if (head > tail) {  // free: [head, cap) and [0, tail)
                if (head + bytes <= cap)
                    at = head;
                else if (bytes < tail)
                    at = 0;
                else
                    return false;
            } else if (head + bytes < tail) {  // wrapped: free [head, tail)
                at = head;
            } else {
                return false;
            }
        }
        live.push_back({at, bytes, false});
        head = at + bytes;
        *off = at;
        return true;
    }
    void release(size_t off) {
        for (Entry &en : live)
            if (en.off == off && !en.released) {
                en.released = true;
                break;
            }
        while (!live.empty() && live.front().released) live.pop_front();
    }
};

// Bytes of theta padded to ld: the staged block is theta, then Delta, and the
// arena places W[0] right after theta, so one copy lands both.
size_t theta_bytes(int64_t ld) { return round_up((size_t)ld * 8); }

size_t request_bytes(int64_t ld, bool bf16, bool symmetric) {
    const size_t l = (size_t)ld, l2 = l * l;
    size_t b = round_up(l * 8) + theta_bytes(ld);  // d, theta
    b += round_up(2 * l2 * 4);               // W[0] (doubles as upload staging), W[1]
    b += round_up(l2 * 4);                   // D
    if (!symmetric) b += round_up(l2 * 4);   // D^T
    if (bf16) b += round_up(2 * l2 * 2) + round_up(l2 * 2);  // Wb[0..1], Db
    return b;
}

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// A few host threads that stage submitted matrices together with the calling
// thread: a job is a number of parts, each run once.  One job at a time
// (concurrent submitters queue); a job returns only when every part is done and
// no pool thread is still inside it.
class StagePool {
  public:
    ~StagePool() { stop(); }
    void start(int threads) {
        for (int i = 0; i < threads; ++i) th_.emplace_back([this] { loop(); });
    }
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            quit_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_)
            if (t.joinable()) t.join();
        th_.clear();
    }
    void run(int parts, const std::function<void(int)> &f) {
        std::lock_guard<std::mutex> jl(job_mu_);
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_done_.wait(lk, [&] { return active_ == 0; });
            f_ = &f;
            parts_ = parts;
            next_.store(0);
            done_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(mu_);
        cv_done_.wait(lk, [&] { return done_ == parts_ && active_ == 0; });
        f_ = nullptr;
    }

  private:
    void work() {
        int mine = 0;
        for (;;) {
            const int k = next_.fetch_add(1);
            if (k >= parts_) break;
            (*f_)(k);
            ++mine;
        }
        if (mine) {
            std::lock_guard<std::mutex> lk(mu_);
            done_ += mine;
        }
        cv_done_.notify_all();
    }
    void loop() {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return quit_ || gen_ != seen; });
            if (quit_) return;
            seen = gen_;
            ++active_;
            lk.unlock();
            work();
            lk.lock();
            --active_;
            cv_done_.notify_all();
        }
    }

    std::vector<std::thread> th_;
    std::mutex job_mu_, mu_;
    std::condition_variable cv_, cv_done_;
    const std::function<void(int)> *f_ = nullptr;
    int parts_ = 0, done_ = 0, active_ = 0;
    std::atomic<int> next_{0};
    uint64_t gen_ = 0;
    bool quit_ = false;
};

// dst = (float) src (n x n) and whether the FP32 values are exactly symmetric,
// by block rows of 64: part b converts rows [64 b, 64 b + 64) in order (dst is
// pinned staging memory, best written sequentially) and compares its 64 x 64
// blocks at and right of the diagonal with their mirrors on the caller's
// (cached) array, until some part has found a mismatch.  Large matrices use
// the pool; parts touch disjoint rows of dst.
template <typename T>
bool stage_and_test(const T *src, int64_t n, float *dst, StagePool *pool) {
    std::atomic<bool> asym{false};
    const int parts = (int)((n + 63) / 64);
    const std::function<void(int)> part = [&](int b) {
        const int64_t bi = 64 * (int64_t)b, ie = std::min(bi + 64, n);
        for (int64_t i = bi * n; i < ie * n; ++i) dst[i] = (float)src[i];
        for (int64_t bj = bi; bj < n && !asym.load(std::memory_order_relaxed); bj += 64) {
            const int64_t je = std::min(bj + 64, n);
            for (int64_t i = bi; i < ie; ++i)
                for (int64_t j = std::max(bj, i + 1); j < je; ++j)
                    if ((float)src[i * n + j] != (float)src[j * n + i]) {
                        asym.store(true, std::memory_order_relaxed);
                        return;
                    }
        }
    };
    if (pool && n >= 256) {
        pool->run(parts, part);
    } else {
        for (int b = 0; b < parts; ++b) part(b);
    }
    return !asym.load();
}

}  // namespace

struct dpt_server_ctx {
    dpt_serve_config cfg{};
    int device = 0, grid = 1024;
    hipStream_t stream = nullptr;
    bool own_stream = true;
    unsigned char *arena_base = nullptr;
    Arena arena;
    size_t arena_used = 0;
    // work tables: built on the host in coherent pinned memory (*_h), moved to
    // the device copy (*_d) by a kernel that reads the host block through its
    // device mapping (*_hd)
    GroupTable *table_h = nullptr, *table_d = nullptr;
    AdmitTable *admit_h = nullptr, *admit_d = nullptr;
    RetireTable *retire_h = nullptr, *retire_d = nullptr;
    void *table_hd = nullptr, *admit_hd = nullptr, *retire_hd = nullptr;
    unsigned long long *stats_d = nullptr, *stats_h = nullptr;
    // eigenvalues of retiring requests: device staging and its pinned mirror
    double *e_stage_d = nullptr, *e_stage_h = nullptr;
    size_t e_stage_cap = 0;  // doubles
    static constexpr size_t kEStage0 = (size_t)1 << 16;  // allocated at open
    // device submissions: theta is read back for validation on a stream of its own
    hipStream_t submit_stream = nullptr;
    std::mutex submit_mu;
    StagePool stage_pool;  // host staging of submitted matrices
    // staging threads besides the submitting one: half the CPUs this process
    // may run on, 1 to 8 (the conversion and symmetry test of host FP64
    // submissions are bound by host memory bandwidth)
    static int stage_threads() {
        cpu_set_t set;
        int cpus = 0;
        if (sched_getaffinity(0, sizeof(set), &set) == 0) cpus = CPU_COUNT(&set);
        if (cpus <= 0) cpus = (int)std::thread::hardware_concurrency();
        return std::min(8, std::max(1, cpus / 2));
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int list_count[kGroupLists] = {};  // requests per (phase, shape) list in the current step
    std::chrono::steady_clock::time_point t0;
    // fused-step tile shape (index into the grouped shapes) per phase (BF16,
    // FP32) and padded-order class (ld <= 256, <= 512, <= 1024, larger); set by
    // the autotuner at open, else the defaults below (128 x 128 above 512)
    static constexpr int kOrderClasses = 4;
    int shape_of[2][kOrderClasses] = {{0, 0, 2, 2}, {0, 0, 2, 2}};

    // pinned staging ring (guarded by ring_mu; cv_ring wakes waiting submits)
    static constexpr size_t kRingBytes = (size_t)256 << 20;
    PinnedRing ring;
    std::mutex ring_mu;
    std::condition_variable cv_ring;
    std::atomic<bool> closing{false};  // set by close and on failure: stop waiting for ring space
    std::vector<size_t> staged;  // worker only: ring offsets of enqueued uploads not yet known complete
    bool idle_since_staged = true;  // worker only: the stream was synchronised after the last upload

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;                  // guarded by mu
    std::unordered_map<int64_t, Request *> done;    // guarded by mu
    std::unordered_map<int64_t, int> live;          // ticket -> 1 (guarded by mu)
    std::vector<Request *> active;                  // worker only
    std::vector<std::pair<Request *, size_t>> retiring;  // worker only: (request, E offset), copies in flight
    std::vector<Request *> zero_w0;                 // worker only: admitted at their iteration cap
    std::vector<int> free_slots;                    // worker only
    int64_t next_id = 0;
    bool stop = false;
    int error = DPT_OK;
    dpt_serve_stats st{};
    std::thread worker;

    ~dpt_server_ctx() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (arena_base) (void)hipFree(arena_base);
        if (table_d) (void)hipFree(table_d);
        if (admit_d) (void)hipFree(admit_d);
        if (retire_d) (void)hipFree(retire_d);
        if (stats_d) (void)hipFree(stats_d);
        if (e_stage_d) (void)hipFree(e_stage_d);
        if (table_h) (void)hipHostFree(table_h);
        if (admit_h) (void)hipHostFree(admit_h);
        if (retire_h) (void)hipHostFree(retire_h);
        if (stats_h) (void)hipHostFree(stats_h);
        if (e_stage_h) (void)hipHostFree(e_stage_h);
        if (ring.base) (void)hipHostFree(ring.base);
        if (submit_stream) (void)hipStreamDestroy(submit_stream);
        if (stream && own_stream) (void)hipStreamDestroy(stream);
        for (auto *r : pending) delete r;
        for (auto &kv : done) delete kv.second;
        for (auto *r : active) delete r;
        for (auto &rp : retiring) delete rp.first;
    }

    // ------------------------------------------------------------ worker
    // Whether the (phase, shape) list can hold work: shapes a phase never uses
    // are left out (64 x 64, the fallback, always stays).
    bool list_used(int pi, int sh) const {
        bool used = sh == 0;
        for (int k = 0; k < kOrderClasses; ++k) used |= shape_of[pi][k] == sh;
        return used;
    }

    // The launches of one engine step: the pre-pass and the fused step for every
    // used (phase, shape) list (the graph's content: lists without work exit at
    // once), or with only_busy for the lists that have work in this step.
    hipError_t launch_all(hipStream_t s, bool only_busy = false) const {
        hipError_t e = launch_group_prepass(table_d, grid, s);
        for (int pi = 0; pi < 2; ++pi)
            for (int sh = 0; sh < kGroupShapes; ++sh) {
                const int ph = pi == 0 ? PH_BF16 : PH_FP32;
                const bool go = only_busy ? list_count[group_list(ph, sh)] > 0 : list_used(pi, sh);
                if (e == hipSuccess && go) e = launch_group_step(table_d, ph, sh, grid, s);
            }
        return e;
    }

    // The graph is replayed only when every list it holds has work.  Otherwise
    // the lists with work are launched directly: a graph launch costs the host
    // ≈ 15 us per step against ≈ 2 us for the two launches of a lone problem,
    // and each empty list in the graph still costs a dispatch on the device.
    hipError_t launch_grouped() {
        bool all_busy = cfg.use_graph;
        for (int pi = 0; pi < 2 && all_busy; ++pi)
            for (int sh = 0; sh < kGroupShapes; ++sh)
                if (list_used(pi, sh) && list_count[group_list(pi == 0 ? PH_BF16 : PH_FP32, sh)] == 0) all_busy = false;
        if (all_busy) {
            std::lock_guard<std::mutex> lk(mu);
            st.graph_steps += 1;
            return hipGraphLaunch(graph_exec, stream);
        }
        return launch_all(stream, true);
    }

    static int order_class(int64_t ld) { return ld <= 256 ? 0 : ld <= 512 ? 1 : ld <= 1024 ? 2 : 3; }

    // The shape chosen for the order class of ld, or 64 x 64 when ld is not a
    // multiple of its tile edges.
    int shape_for(int64_t ld, int phase) const {
        const int sh = shape_of[phase == PH_BF16 ? 0 : 1][order_class(ld)];
        return (ld % group_shape_rows(sh) == 0 && ld % group_shape_cols(sh) == 0) ? sh : 0;
    }

    // Tile-shape autotuner.  For padded orders 256, 512, 1024, 2048 (the largest
    // of each order class) and each phase, time the grouped fused step with each
    // tile shape on synthetic problems (distinct buffers, zero state,
    // theta_i = i): a full batch (about four grid-fulls of 64x64 tiles: the
    // throughput under load) and a lone problem (the step time when few requests
    // are in flight).  Among the shapes within 3 % of the best full-batch time,
    // the one with the fastest lone-problem step is kept; a larger shape replaces
    // a smaller one only when at least 3 % faster there.  (Timed on full batches
    // alone, larger tiles won by a few per cent at no gain in the burst rate but
    // at 20 % longer latencies at the service rate.)
    hipError_t autotune() {
        const int64_t orders[] = {256, 512, 1024, 2048};
        constexpr int kOrders = 4, kReps = 3, kRepsLone = 20;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        hipError_t e = hipEventCreate(&ev0);
        if (e == hipSuccess) e = hipEventCreate(&ev1);
        int best[2][kOrders] = {};
        for (int oi = 0; oi < kOrders && e == hipSuccess; ++oi) {
            const int64_t ld = orders[oi], l2 = ld * ld;
            const int batch = (int)std::min<int64_t>(64, std::max<int64_t>(1, 4 * (int64_t)grid * 4096 / l2));
            // per problem: theta, d, W[2], D, Wb[2], Db (D doubles as D^T)
            const size_t per = round_up(2 * (size_t)ld * 8) + round_up(3 * (size_t)l2 * 4) + round_up(3 * (size_t)l2 * 2);
            unsigned char *buf = nullptr;
            e = hipMalloc((void **)&buf, per * (size_t)batch);
            if (e != hipSuccess) break;
            std::vector<double> th((size_t)ld);
            for (int64_t i = 0; i < ld; ++i) th[(size_t)i] = (double)i;
            e = launch_fill_zero(buf, per * (size_t)batch, stream);
            GroupTable &t = *table_h;
            for (int b = 0; b < batch && e == hipSuccess; ++b) {
                unsigned char *p = buf + per * (size_t)b;
                GroupReq &g = t.reqs[b];
                double *theta_b = (double *)p;
                g.theta = theta_b;
                g.d = (double *)p + ld;
                p += round_up(2 * (size_t)ld * 8);
                g.W = (float *)p;
                g.Wn = (float *)p + l2;
                g.D = g.DT = (float *)p + 2 * l2;
                p += round_up(3 * (size_t)l2 * 4);
                g.Wb = (__bf16 *)p;
                g.Wbn = (__bf16 *)p + l2;
                g.Db = (__bf16 *)p + 2 * l2;
                g.stat = stats_d;
                g.n = ld;
                g.ld = ld;
                g.lambda = 1.0;
                e = hipMemcpyAsync(theta_b, th.data(), (size_t)ld * 8, hipMemcpyHostToDevice, stream);
            }
            // time of one grouped step of shape sh over the first `count` problems
            auto time_step = [&](int phase, int sh, int count, int reps, float *ms) {
                const int L = group_list(phase, sh);
                std::memset(t.counts, 0, sizeof(t.counts));
                t.counts[0] = count;
                t.counts[1 + L] = count;
                const int32_t tiles = (int32_t)((ld / group_shape_rows(sh)) * (ld / group_shape_cols(sh)));
                for (int b = 0; b <= count; ++b) {
                    t.prefix[L][b] = b * tiles;
                    if (b < count) t.idx[L][b] = b;
                }
                hipError_t x = hipMemcpyAsync(table_d, table_h, sizeof(GroupTable), hipMemcpyHostToDevice, stream);
                if (x == hipSuccess) x = launch_group_step(table_d, phase, sh, grid, stream);  // warm-up
                if (x == hipSuccess) x = hipEventRecord(ev0, stream);
                for (int r = 0; r < reps && x == hipSuccess; ++r) x = launch_group_step(table_d, phase, sh, grid, stream);
                if (x == hipSuccess) x = hipEventRecord(ev1, stream);
                if (x == hipSuccess) x = hipEventSynchronize(ev1);
                if (x == hipSuccess) x = hipEventElapsedTime(ms, ev0, ev1);
                return x;
            };
            for (int pi = 0; pi < 2 && e == hipSuccess; ++pi) {
                const int phase = pi == 0 ? PH_BF16 : PH_FP32;
                float full[kGroupShapes] = {}, lone[kGroupShapes] = {};
                for (int sh = 0; sh < kGroupShapes && e == hipSuccess; ++sh) {
                    e = time_step(phase, sh, batch, kReps, &full[sh]);
                    if (e == hipSuccess) e = time_step(phase, sh, 1, kRepsLone, &lone[sh]);
                }
                float best_full = full[0];
                for (int sh = 1; sh < kGroupShapes; ++sh) best_full = std::min(best_full, full[sh]);
                int b = -1;
                for (int sh = 0; sh < kGroupShapes; ++sh)
                    if (full[sh] <= 1.03f * best_full && (b < 0 || lone[sh] < 0.97f * lone[b])) b = sh;
                best[pi][oi] = b;
            }
            (void)hipStreamSynchronize(stream);
            (void)hipFree(buf);
        }
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        std::memset(table_h, 0, sizeof(GroupTable));
        if (e == hipSuccess) e = hipMemcpyAsync(table_d, table_h, sizeof(GroupTable), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess)
            for (int pi = 0; pi < 2; ++pi)
                for (int oi = 0; oi < kOrders; ++oi) shape_of[pi][oi] = best[pi][oi];
        return e;
    }

    // Places r in the arena at off, enqueues its upload (host submissions) and
    // writes its entry of the admission table (index k).
    hipError_t admit_one(Request *r, size_t off, int k) {
        r->off = off;
        r->bytes = request_bytes(r->ld, r->bf16, r->symmetric);
        r->slot = free_slots.back();
        free_slots.pop_back();
        const size_t l = (size_t)r->ld, l2 = l * l;
        unsigned char *p = arena_base + off;
        auto take = [&](size_t bytes) {
            unsigned char *q = p;
            p += round_up(bytes);
            return q;
        };
        r->d_d = (double *)take(l * 8);
        r->theta_d = (double *)take(theta_bytes(r->ld));
        float *wpair = (float *)take(2 * l2 * 4);  // directly after theta
        r->W[0] = wpair;
        r->W[1] = wpair + l2;
        r->D = (float *)take(l2 * 4);
        r->DT = r->symmetric ? r->D : (float *)take(l2 * 4);
        if (r->bf16) {
            __bf16 *bpair = (__bf16 *)take(2 * l2 * 2);
            r->Wb[0] = bpair;
            r->Wb[1] = bpair + l2;
            r->Db = (__bf16 *)take(l2 * 2);
        }
        const size_t nn = (size_t)(r->n * r->n);
        hipError_t e = hipSuccess;
        if (r->staged) {  // theta then Delta in one copy; the ring space is given back once the stream is idle
            e = hipMemcpyAsync(r->theta_d, r->staged, theta_bytes(r->ld) + nn * 4, hipMemcpyHostToDevice, stream);
            staged.push_back(r->ring_off);
            r->staged = nullptr;
            idle_since_staged = false;
        } else if (!r->dev_delta) {
            e = hipMemcpyAsync(r->theta_d, r->theta.data(), l * 8, hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = hipMemcpyAsync(r->W[0], r->delta.data(), nn * 4, hipMemcpyHostToDevice, stream);
        }
        r->ctl.start(r->opt, r->bf16 ? PH_BF16 : PH_FP32, false);
        const bool capped = r->ctl.capped();  // retires at the identity: W[0] is cleared after the launch
        if (capped) zero_w0.push_back(r);
        AdmitReq &q = admit_h->reqs[k];
        q.src = r->dev_delta ? r->dev_delta : (const void *)r->W[0];
        q.src_f64 = r->dev_delta && r->dev_f64 ? 1 : 0;
        q.theta_src = r->dev_delta ? r->dev_theta : r->theta_d;
        q.theta = r->theta_d;
        q.D = r->D;
        q.DT = r->symmetric ? nullptr : r->DT;
        q.Db = r->bf16 ? r->Db : nullptr;
        q.W1 = capped ? nullptr : r->W[1];
        q.Wb1 = capped || !r->bf16 ? nullptr : r->Wb[1];
        q.stat = stats_d + 2 * r->slot;
        q.n = r->n;
        q.ld = r->ld;
        q.lambda = r->lambda;
        admit_h->prefix[k + 1] = admit_h->prefix[k] + (int32_t)((r->ld / 64) * (r->ld / 64));
        r->t_admit = now_s(t0);
        return e;
    }

    hipError_t admit() {
        int k = 0;
        admit_h->prefix[0] = 0;
        hipError_t e = hipSuccess;
        while (e == hipSuccess && !free_slots.empty()) {
            Request *r;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (pending.empty()) break;
                r = pending.front();
            }
            size_t off;
            if (!arena.alloc(request_bytes(r->ld, r->bf16, r->symmetric), &off)) break;  // FIFO
            {
                std::lock_guard<std::mutex> lk(mu);
                pending.pop_front();
                st.pending = (int64_t)pending.size();
            }
            e = admit_one(r, off, k++);
            active.push_back(r);
            arena_used += r->bytes;
            {
                std::lock_guard<std::mutex> lk(mu);
                st.peak_bytes = std::max<int64_t>(st.peak_bytes, (int64_t)arena_used);
                st.peak_active = std::max<int64_t>(st.peak_active, (int64_t)active.size());
                st.active = (int64_t)active.size();
            }
        }
        if (e == hipSuccess && k > 0) {
            admit_h->count = k;
            e = launch_fetch_table(admit_hd, admit_d, offsetof(AdmitTable, reqs) + (size_t)k * sizeof(AdmitReq),
                                   stream);
            if (e == hipSuccess) e = launch_group_admit(admit_d, grid, stream);
        }
        for (Request *r : zero_w0)
            if (e == hipSuccess) e = launch_fill_zero(r->W[0], (size_t)(r->ld * r->ld) * 4, stream);
        zero_w0.clear();
        return e;
    }

    bool finished(const Request *r) const {
        return r->ctl.status != DPT_NOT_CONVERGED || r->ctl.capped();
    }

    // Enqueues one application of the map to every admitted request past its
    // first iterate: the work table's upload and the grouped launches.  The
    // admissions of the same engine step are enqueued after it (their host
    // work overlaps the grouped step) and finish_step reads both back.
    hipError_t launch_step() {
        GroupTable &t = *table_h;
        int nreq = 0;
        int cnt[kGroupLists] = {};
        int32_t rows = 0, tiles_sum[kGroupLists] = {};
        for (Request *r : active) {
            if (finished(r) || r->at_identity) continue;  // finished: e.g. max_iter = 0, retired without a step
            const int nx = r->cur ^ 1;
            const bool bf = r->ctl.phase == PH_BF16;
            GroupReq &g = t.reqs[nreq];
            g.Wb = bf ? r->Wb[r->cur] : nullptr;
            g.Db = r->Db;
            g.W = r->W[r->cur];
            g.D = r->D;
            g.DT = r->DT;
            g.Wn = r->W[nx];
            g.Wbn = bf ? r->Wb[nx] : nullptr;
            g.theta = r->theta_d;
            g.d = r->d_d;
            g.stat = stats_d + 2 * r->slot;
            g.n = r->n;
            g.ld = r->ld;
            g.lambda = r->lambda;
            t.pre_prefix[nreq] = rows;
            rows += (int32_t)r->n;
            const int phase = bf ? PH_BF16 : PH_FP32, sh = shape_for(r->ld, phase);
            const int L = group_list(phase, sh);
            t.idx[L][cnt[L]] = nreq;
            t.prefix[L][cnt[L]++] = tiles_sum[L];
            tiles_sum[L] += (int32_t)((r->ld / group_shape_rows(sh)) * (r->ld / group_shape_cols(sh)));
            ++nreq;
        }
        t.pre_prefix[nreq] = rows;
        t.counts[0] = nreq;
        for (int L = 0; L < kGroupLists; ++L) {
            t.prefix[L][cnt[L]] = tiles_sum[L];
            t.counts[1 + L] = cnt[L];
            list_count[L] = cnt[L];
        }
        hipError_t e = hipSuccess;
        if (nreq > 0) {
            e = launch_fetch_table(table_hd, table_d, offsetof(GroupTable, reqs) + (size_t)nreq * sizeof(GroupReq),
                                   stream);
            if (e == hipSuccess) e = launch_grouped();
        }
        return e;
    }

    // After launch_step and the admissions: the statistics of every request
    // stepped or admitted (first iterate) in this engine step are read back with
    // one copy and one synchronisation; the retirements enqueued before are
    // handed out; each request's controller takes its step.
    hipError_t finish_step() {
        std::vector<Request *> stepping;  // the table's requests and the ones just admitted
        for (Request *r : active)
            if (!finished(r)) stepping.push_back(r);
        hipError_t e = hipMemcpyAsync(stats_h, stats_d, 16 * (size_t)cfg.max_slots, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) idle_since_staged = true;
        if (e != hipSuccess) return e;
        const double t_now = now_s(t0);
        hand_out(t_now);
        for (Request *r : stepping) {
            r->cur ^= 1;
            if (r->at_identity) {
                r->t_first = t_now;
                std::vector<float>().swap(r->delta);  // staged on the device; drop the host copy
            }
            r->at_identity = false;
            r->ctl.count_step();
            double dl, wm;
            std::memcpy(&dl, &stats_h[2 * r->slot], 8);
            std::memcpy(&wm, &stats_h[2 * r->slot + 1], 8);
            if (r->ctl.update(dl, wm) == Controller::DONE || r->ctl.capped()) r->status = r->ctl.status;
        }
        std::lock_guard<std::mutex> lk(mu);
        st.steps += 1;
        return hipSuccess;
    }

    // Enqueues the retirement of every finished request: one grouped launch for
    // their eigenvalues (into the staging buffer) and stats, one copy of the
    // staging buffer to its pinned mirror, and the optional eigenvector exports.
    // Their arena space and slots are free at once (stream order protects them);
    // the results are handed out after the stream's next synchronisation.  The
    // stream is idle when this is called.
    hipError_t retire() {
        std::vector<Request *> out;
        for (Request *r : active)
            if (finished(r)) out.push_back(r);
        if (out.empty()) return hipSuccess;
        size_t need = 0;
        for (Request *r : out) need += (size_t)r->n;
        hipError_t e = hipSuccess;
        if (need > e_stage_cap) {  // grow (nothing is in flight on the staging buffers)
            if (e_stage_d) (void)hipFree(e_stage_d);
            if (e_stage_h) (void)hipHostFree(e_stage_h);
            e_stage_d = e_stage_h = nullptr;
            e_stage_cap = 0;
            const size_t cap = std::max<size_t>(need, kEStage0);
            e = hipMalloc((void **)&e_stage_d, cap * 8);
            if (e == hipSuccess) e = hipHostMalloc((void **)&e_stage_h, cap * 8, 0);
            if (e != hipSuccess) return e;
            e_stage_cap = cap;
        }
        RetireTable &t = *retire_h;
        t.prefix[0] = 0;
        size_t eoff = 0;
        for (size_t k = 0; k < out.size(); ++k) {
            Request *r = out[k];
            RetireReq &q = t.reqs[k];
            q.W = r->W[r->cur];
            q.D = r->D;
            q.theta = r->theta_d;
            q.E = e_stage_d + eoff;
            q.stat = stats_d + 2 * r->slot;
            q.n = r->n;
            q.ld = r->ld;
            q.lambda = r->lambda;
            t.prefix[k + 1] = t.prefix[k] + (int32_t)r->n;
            retiring.emplace_back(r, eoff);
            eoff += (size_t)r->n;
        }
        t.count = (int32_t)out.size();
        e = launch_fetch_table(retire_hd, retire_d, offsetof(RetireTable, reqs) + out.size() * sizeof(RetireReq),
                               stream);
        if (e == hipSuccess) e = launch_group_retire(retire_d, grid, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(e_stage_h, e_stage_d, eoff * 8, hipMemcpyDeviceToHost, stream);
        for (Request *r : out) {
            if (r->want_z && e == hipSuccess) {
                r->Z.resize((size_t)(r->n * r->n));
                float *staging = r->W[r->cur ^ 1];
                e = launch_export_f32(r->W[r->cur], r->n, r->ld, staging, 0, stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(r->Z.data(), staging, r->Z.size() * 4, hipMemcpyDeviceToHost, stream);
            }
            arena.release(r->off, r->bytes);
            arena_used -= r->bytes;
            free_slots.push_back(r->slot);
            r->slot = -1;
            r->status = r->ctl.status;
            active.erase(std::find(active.begin(), active.end(), r));
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            st.active = (int64_t)active.size();
        }
        return e;
    }

    // After a synchronisation of the stream: the retirements enqueued before it
    // are complete; copy their eigenvalues out and hand them to the pollers.
    void hand_out(double t_now) {
        if (retiring.empty()) return;
        for (auto &rp : retiring) {
            Request *r = rp.first;
            r->E.assign(e_stage_h + rp.second, e_stage_h + rp.second + r->n);
            r->t_finish = t_now;
            std::vector<float>().swap(r->delta);
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &rp : retiring) done[rp.first->id] = rp.first;
            st.completed += (int64_t)retiring.size();
        }
        retiring.clear();
        cv_done.notify_all();
    }

    hipError_t finish_retiring() {
        const hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        idle_since_staged = true;
        hand_out(now_s(t0));
        return hipSuccess;
    }

    // The uploads of the requests admitted so far have completed once the stream
    // is idle; give their ring space back (in allocation order).
    hipError_t release_staged() {
        if (!idle_since_staged) {
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return e;
        }
        {
            std::lock_guard<std::mutex> lk(ring_mu);
            for (size_t off : staged) ring.release(off);
        }
        staged.clear();
        cv_ring.notify_all();
        return hipSuccess;
    }

    void fail_all(int code) {
        closing.store(true);
        cv_ring.notify_all();
        std::lock_guard<std::mutex> lk(mu);
        error = code;
        for (Request *r : active) {
            r->status = code;
            done[r->id] = r;
        }
        active.clear();
        for (auto &rp : retiring) {
            rp.first->status = code;
            done[rp.first->id] = rp.first;
        }
        retiring.clear();
        for (Request *r : pending) {
            r->status = code;
            done[r->id] = r;
        }
        pending.clear();
        cv_done.notify_all();
    }

    void run() {
        (void)hipSetDevice(device);
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                if (active.empty() && pending.empty() && retiring.empty()) {
                    if (stop) break;
                    cv_work.wait_for(lk, std::chrono::milliseconds(2));
                    continue;
                }
            }
            const auto t_begin = std::chrono::steady_clock::now();
            hipError_t e = launch_step();
            if (e == hipSuccess) e = admit();
            const bool any_step = std::any_of(active.begin(), active.end(), [&](Request *r) { return !finished(r); });
            if (e == hipSuccess && any_step) e = finish_step();  // synchronises and hands out earlier retirements
            else if (e == hipSuccess) e = finish_retiring();
            if (e == hipSuccess) e = retire();
            if (e == hipSuccess && !staged.empty()) e = release_staged();
            {
                std::lock_guard<std::mutex> lk(mu);
                st.busy_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count();
            }
            if (e != hipSuccess) {
                fail_all(e == hipErrorOutOfMemory ? DPT_ENOMEM : DPT_EDEVICE);
                std::unique_lock<std::mutex> lk(mu);
                if (stop) break;
            }
        }
    }
};


extern "C" {

int dpt_serve_open(dpt_server *srv, const dpt_serve_config *cfg) {
    if (!srv || !cfg || cfg->budget_bytes <= 0 || cfg->max_slots < 1 || cfg->max_slots > kServeMaxSlots ||
        cfg->grid_blocks < 0 || cfg->autotune < -kGroupShapes || cfg->autotune > 1)
        return DPT_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return DPT_EDEVICE;
    dpt_server_ctx *c = new (std::nothrow) dpt_server_ctx();
    if (!c) return DPT_ENOMEM;
    c->cfg = *cfg;
    c->grid = cfg->grid_blocks > 0 ? cfg->grid_blocks : 1024;
    c->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) {
        if (cfg->stream) {  // the caller's stream: used, never destroyed
            c->stream = (hipStream_t)cfg->stream;
            c->own_stream = false;
        } else {
            e = hipStreamCreate(&c->stream);
        }
    }
    if (e == hipSuccess) e = hipMalloc((void **)&c->arena_base, (size_t)cfg->budget_bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&c->table_d, sizeof(GroupTable));
    if (e == hipSuccess) e = hipMalloc((void **)&c->admit_d, sizeof(AdmitTable));
    if (e == hipSuccess) e = hipMalloc((void **)&c->retire_d, sizeof(RetireTable));
    if (e == hipSuccess) e = hipMalloc((void **)&c->stats_d, 16 * (size_t)cfg->max_slots);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->submit_stream, hipStreamNonBlocking);
    // coherent: the host rewrites the tables between steps and a kernel reads them
    const unsigned int tflags = hipHostMallocCoherent | hipHostMallocMapped;
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->admit_h, sizeof(AdmitTable), tflags);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->retire_h, sizeof(RetireTable), tflags);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->table_h, sizeof(GroupTable), tflags);
    if (e == hipSuccess) e = hipHostGetDevicePointer(&c->admit_hd, c->admit_h, 0);
    if (e == hipSuccess) e = hipHostGetDevicePointer(&c->retire_hd, c->retire_h, 0);
    if (e == hipSuccess) e = hipHostGetDevicePointer(&c->table_hd, c->table_h, 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->stats_h, 16 * (size_t)cfg->max_slots, 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->ring.base, dpt_server_ctx::kRingBytes, 0);
    if (e == hipSuccess) c->ring.cap = dpt_server_ctx::kRingBytes;
    // the eigenvalue staging of the retirements at its first size, so that the
    // engine's steps allocate nothing until a retirement needs more
    if (e == hipSuccess) e = hipMalloc((void **)&c->e_stage_d, dpt_server_ctx::kEStage0 * 8);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->e_stage_h, dpt_server_ctx::kEStage0 * 8, 0);
    if (e == hipSuccess) c->e_stage_cap = dpt_server_ctx::kEStage0;
    if (e == hipSuccess) {
        std::memset(c->table_h, 0, sizeof(GroupTable));
        e = hipMemcpy(c->table_d, c->table_h, sizeof(GroupTable), hipMemcpyHostToDevice);
    }
    if (cfg->autotune < 0)  // one shape for every order class
        for (auto &row : c->shape_of)
            for (int &sh : row) sh = -cfg->autotune - 1;
    if (e == hipSuccess && cfg->autotune == 1) e = c->autotune();  // fixes the launches the graph holds
    if (e == hipSuccess && cfg->use_graph) {
        e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t e1 = c->launch_all(c->stream);
            e = hipStreamEndCapture(c->stream, &c->graph);
            if (e == hipSuccess) e = e1;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0);
        // one replay on the empty table (every list exits at once): a graph's
        // first launch uploads it (milliseconds), which in service would stall
        // the step where every list first has work
        if (e == hipSuccess) e = hipGraphLaunch(c->graph_exec, c->stream);
    }
    // the table copy, admission and retirement kernels run once on empty tables
    // (their item loops do nothing), so that no first launch falls in service
    if (e == hipSuccess) {
        std::memset(c->admit_h, 0, offsetof(AdmitTable, reqs));
        std::memset(c->retire_h, 0, offsetof(RetireTable, reqs));
        e = launch_fetch_table(c->admit_hd, c->admit_d, offsetof(AdmitTable, reqs), c->stream);
        if (e == hipSuccess) e = launch_fetch_table(c->retire_hd, c->retire_d, offsetof(RetireTable, reqs), c->stream);
        if (e == hipSuccess) e = launch_group_admit(c->admit_d, c->grid, c->stream);
        if (e == hipSuccess) e = launch_group_retire(c->retire_d, c->grid, c->stream);
    }
    // every slot's stats start at zero (the autotuner's timing runs publish into
    // slot 0; the admission launch publishes into them; retirement clears them)
    if (e == hipSuccess) e = launch_zero_u64(c->stats_d, 2 * (int64_t)cfg->max_slots, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        const int code = (e == hipErrorOutOfMemory) ? DPT_ENOMEM : DPT_EDEVICE;
        delete c;
        return code;
    }
    for (int pi = 0; pi < 2; ++pi)
        for (int k = 0; k < dpt_server_ctx::kOrderClasses; ++k) c->st.tile_shape[pi][k] = c->shape_of[pi][k];
    c->arena.init((size_t)cfg->budget_bytes);
    for (int i = cfg->max_slots - 1; i >= 0; --i) c->free_slots.push_back(i);
    c->stage_pool.start(dpt_server_ctx::stage_threads());
    c->worker = std::thread([c] { c->run(); });
    *srv = c;
    return DPT_OK;
}


int dpt_serve_submit(dpt_server srv, const dpt_problem *p, const dpt_options *o, int want_eigenvectors,
                     int64_t *ticket) {
    if (!srv || !ticket) return DPT_EINVAL;
    if (dpt_validate(p, o) != DPT_OK) return DPT_EINVAL;
    if (p->format != DPT_DENSE) return DPT_EINVAL;
    const bool dev = p->mem == DPT_MEM_DEVICE;
    if (dev && !inputs_on_device(p)) return DPT_EINVAL;
    dpt_options opt;
    if (o) {
        opt = *o;
    } else {
        dpt_options_default(&opt);
    }
    if (opt.precision != DPT_FP32 && opt.precision != DPT_BF16_FP32) return DPT_EINVAL;
    if (opt.ramp_alpha != 0.0) return DPT_EINVAL;  // the engine runs the autonomous map
    if (opt.stop_rule == DPT_STOP_ROW) return DPT_EINVAL;  // requests retire whole
    Request *r = new (std::nothrow) Request();
    if (!r) return DPT_ENOMEM;
    r->n = p->n;
    r->ld = (p->n + 63) / 64 * 64;
    r->lambda = p->lambda;
    r->opt = opt;
    r->bf16 = opt.precision == DPT_BF16_FP32;
    r->want_z = want_eigenvectors != 0;
    const size_t nn = (size_t)(p->n * p->n);
    if (request_bytes(r->ld, r->bf16, false) > (size_t)srv->cfg.budget_bytes &&
        request_bytes(r->ld, r->bf16, true) > (size_t)srv->cfg.budget_bytes) {
        delete r;
        return DPT_ENOMEM;
    }
    if (dev) {
        // Device arrays are read by the worker at admission (the caller keeps them
        // unchanged until the result is polled); theta is checked here.  The
        // transpose is always stored (symmetry is not tested on the device).
        std::vector<double> th((size_t)p->n);
        {
            std::lock_guard<std::mutex> lk(srv->submit_mu);
            if (hipMemcpyAsync(th.data(), p->theta, sizeof(double) * (size_t)p->n, hipMemcpyDeviceToHost,
                               srv->submit_stream) != hipSuccess ||
                hipStreamSynchronize(srv->submit_stream) != hipSuccess) {
                delete r;
                return DPT_EDEVICE;
            }
        }
        if (!host_theta_ok(th.data(), p->n)) {
            delete r;
            return DPT_EINVAL;
        }
        r->dev_theta = (const double *)p->theta;
        r->dev_delta = p->delta;
        r->dev_f64 = p->dtype == DPT_DTYPE_F64;
        r->symmetric = false;
        if (request_bytes(r->ld, r->bf16, false) > (size_t)srv->cfg.budget_bytes) {
            delete r;
            return DPT_ENOMEM;
        }
    } else {
        // theta (padded) and the FP32 Delta go to the pinned ring as one block
        // (waiting for space while earlier submissions are uploaded) unless the
        // block takes more than half of it
        const size_t tb = theta_bytes(r->ld), block = tb + nn * 4;
        unsigned char *blk = nullptr;
        if (block <= srv->ring.cap / 2) {
            std::unique_lock<std::mutex> lk(srv->ring_mu);
            size_t off = 0;
            srv->cv_ring.wait(lk, [&] { return srv->closing.load() || srv->ring.alloc(block, &off); });
            if (srv->closing.load()) {
                delete r;
                return DPT_ESTATE;
            }
            blk = srv->ring.base + off;
            r->staged = blk;
            r->ring_off = off;
        }
        // an early return from here on gives the ring space back
        auto drop = [&](int code) {
            if (r->staged) {
                {
                    std::lock_guard<std::mutex> lk(srv->ring_mu);
                    srv->ring.release(r->ring_off);
                }
                srv->cv_ring.notify_all();
            }
            delete r;
            return code;
        };
        double *th = nullptr;
        float *dst = nullptr;
        if (blk) {
            th = (double *)blk;
            dst = (float *)(blk + tb);
        } else {
            try {
                r->theta.assign((size_t)r->ld, 0.0);
                r->delta.resize(nn);
            } catch (...) {
                return drop(DPT_ENOMEM);
            }
            th = r->theta.data();
            dst = r->delta.data();
        }
        std::memcpy(th, p->theta, sizeof(double) * (size_t)p->n);
        for (int64_t i = p->n; i < r->ld; ++i) th[i] = 0.0;
        // FP32 copy into the staging block; symmetry of the FP32 values tested on
        // the caller's array (not on the pinned copy).
        const bool sym = p->dtype == DPT_DTYPE_F64
                             ? stage_and_test<double>((const double *)p->delta, p->n, dst, &srv->stage_pool)
                             : stage_and_test<float>((const float *)p->delta, p->n, dst, &srv->stage_pool);
        r->symmetric = sym;
        if (request_bytes(r->ld, r->bf16, r->symmetric) > (size_t)srv->cfg.budget_bytes) return drop(DPT_ENOMEM);
    }
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->stop || srv->error != DPT_OK) {
            const int code = srv->error != DPT_OK ? srv->error : DPT_ESTATE;
            lk.unlock();
            if (r->staged) {
                {
                    std::lock_guard<std::mutex> lr(srv->ring_mu);
                    srv->ring.release(r->ring_off);
                }
                srv->cv_ring.notify_all();
            }
            delete r;
            return code;
        }
        r->id = srv->next_id++;
        r->t_submit = now_s(srv->t0);
        srv->pending.push_back(r);
        srv->live[r->id] = 1;
        srv->st.submitted += 1;
        srv->st.pending = (int64_t)srv->pending.size();
        *ticket = r->id;
    }
    srv->cv_work.notify_one();
    return DPT_OK;
}

int dpt_serve_poll(dpt_server srv, int64_t ticket, int wait_ms, dpt_result *res, double *E, void *Z, int z_dtype,
                   dpt_serve_times *t) {
    if (!srv) return DPT_EINVAL;
    if (Z && z_dtype != DPT_DTYPE_F32 && z_dtype != DPT_DTYPE_F64) return DPT_EINVAL;
    Request *r = nullptr;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        if (!srv->live.count(ticket)) return DPT_EINVAL;
        auto ready = [&] { return srv->done.count(ticket) != 0; };
        if (!ready() && wait_ms != 0) {
            if (wait_ms < 0)
                srv->cv_done.wait(lk, ready);
            else
                srv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
        }
        auto it = srv->done.find(ticket);
        if (it == srv->done.end()) return DPT_EAGAIN;
        r = it->second;
        srv->done.erase(it);
        srv->live.erase(ticket);
    }
    const int status = r->status;
    r->ctl.fill(res);
    if (res) res->status = status;
    if (status >= 0) {
        if (E) std::memcpy(E, r->E.data(), r->E.size() * 8);
        if (Z && r->want_z) {
            if (z_dtype == DPT_DTYPE_F32) {
                std::memcpy(Z, r->Z.data(), r->Z.size() * 4);
            } else {
                double *zd = (double *)Z;
                for (size_t i = 0; i < r->Z.size(); ++i) zd[i] = r->Z[i];
            }
        }
    }
    if (t) {
        t->submit_s = r->t_submit;
        t->admit_s = r->t_admit;
        t->first_step_s = r->t_first;
        t->finish_s = r->t_finish;
    }
    delete r;
    return status;
}

int dpt_serve_stats_read(dpt_server srv, dpt_serve_stats *out) {
    if (!srv || !out) return DPT_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    return DPT_OK;
}

void dpt_serve_close(dpt_server srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->closing.store(true);
    srv->cv_ring.notify_all();
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    (void)hipStreamSynchronize(srv->stream);
    delete srv;
}

}  // extern "C"
