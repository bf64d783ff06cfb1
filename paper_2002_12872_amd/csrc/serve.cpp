// Serving engine: continuous batching of many small dense D-PT problems.
//
// A worker thread owns one stream, a device arena of the configured budget
// and a slot table.  Each engine step:
//   1. admits waiting problems in FIFO order while the arena and the slots have
//      room (upload, padded FP32/BF16 copies, transpose when unsymmetric);
//   2. applies the map of eq. (dyn) (Kenmoe, Smerlak, Zadorin, arXiv:2002.12872,
//      Sec. II.B) once to every admitted problem: the closed-form first iterate
//      for new ones, then one persistent grouped pre-pass and one persistent
//      grouped fused step per precision phase over a device work table (the
//      three launches are a HIP graph replayed every step);
//   3. reads every problem's (delta, max|W|) back and runs its own controller
//      (the same stopping rule as dpt_solve);
//   4. retires finished problems (eigenvalues and optional eigenvectors copied
//      out), releasing their arena space for the next admissions.
#include <hip/hip_runtime.h>

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
    std::vector<double> theta;  // ld entries (zero padded)
    std::vector<float> delta;   // n*n row-major when it does not fit the pinned ring
    float *delta_pinned = nullptr;  // n*n row-major in the pinned ring, until uploaded
    size_t ring_off = 0;
    // device memory inside the arena
    size_t off = 0, bytes = 0;
    int slot = -1;
    double *theta_d = nullptr, *d_d = nullptr, *e_d = nullptr;
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

size_t request_bytes(int64_t ld, bool bf16, bool symmetric) {
    const size_t l = (size_t)ld, l2 = l * l;
    size_t b = 3 * round_up(l * 8);          // theta, d, E
    b += round_up(2 * l2 * 4);               // W[0], W[1] (W[1] doubles as upload staging)
    b += round_up(l2 * 4);                   // D
    if (!symmetric) b += round_up(l2 * 4);   // D^T
    if (bf16) b += round_up(2 * l2 * 2) + round_up(l2 * 2);  // Wb[0..1], Db
    return b;
}

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
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
    GroupTable *table_h = nullptr, *table_d = nullptr;
    unsigned long long *stats_d = nullptr, *stats_h = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::chrono::steady_clock::time_point t0;
    // smallest padded order that uses 128 x 128 tiles, per phase (BF16, FP32);
    // set by the autotuner at open, else the defaults below
    int64_t min_ld_128[2] = {1024, 1024};

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
        if (stats_d) (void)hipFree(stats_d);
        if (table_h) (void)hipHostFree(table_h);
        if (stats_h) (void)hipHostFree(stats_h);
        if (ring.base) (void)hipHostFree(ring.base);
        if (stream && own_stream) (void)hipStreamDestroy(stream);
        for (auto *r : pending) delete r;
        for (auto &kv : done) delete kv.second;
        for (auto *r : active) delete r;
    }

    // ------------------------------------------------------------ worker
    // The launches of one engine step: the pre-pass and the fused step for every
    // (phase, tile) list; lists without work exit at once.
    // (128x128 launches are left out for a phase that never uses them.)
    hipError_t launch_all(hipStream_t s) const {
        hipError_t e = launch_group_prepass(table_d, grid, s);
        for (int ph : {PH_BF16, PH_FP32})
            for (int tile : {64, 128})
                if (e == hipSuccess && (tile == 64 || min_ld_128[ph == PH_BF16 ? 0 : 1] != INT64_MAX))
                    e = launch_group_step(table_d, ph, tile, grid, s);
        return e;
    }

    hipError_t launch_grouped() {
        if (cfg.use_graph) return hipGraphLaunch(graph_exec, stream);
        return launch_all(stream);
    }

    int tile_for(int64_t ld, int phase) const {
        return (ld % 128 == 0 && ld >= min_ld_128[phase == PH_BF16 ? 0 : 1]) ? 128 : 64;
    }

    // Tile-shape autotuner.  For padded orders 256 .. 2048 and each phase, time
    // the grouped fused step over a batch of synthetic problems (about four
    // grid-fulls of 64x64 tiles, distinct buffers, zero state, theta_i = i) with
    // 64x64 and with 128x128 tiles; 128x128 is used from the smallest order
    // from which it is at least 3 % faster at every larger order measured.
    hipError_t autotune() {
        const int64_t orders[] = {256, 512, 1024, 2048};
        constexpr int kOrders = 4, kReps = 3;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        hipError_t e = hipEventCreate(&ev0);
        if (e == hipSuccess) e = hipEventCreate(&ev1);
        bool wins[2][kOrders] = {};
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
            for (int pi = 0; pi < 2 && e == hipSuccess; ++pi) {
                const int phase = pi == 0 ? PH_BF16 : PH_FP32;
                float ms[2] = {0.0f, 0.0f};
                for (int ti = 0; ti < 2 && e == hipSuccess; ++ti) {
                    const int tile = ti == 0 ? 64 : 128, L = group_list(phase, tile);
                    std::memset(t.counts, 0, sizeof(t.counts));
                    t.counts[0] = batch;
                    t.counts[1 + L] = batch;
                    const int32_t tiles = (int32_t)((ld / tile) * (ld / tile));
                    for (int b = 0; b <= batch; ++b) {
                        t.prefix[L][b] = b * tiles;
                        if (b < batch) t.idx[L][b] = b;
                    }
                    e = hipMemcpyAsync(table_d, table_h, sizeof(GroupTable), hipMemcpyHostToDevice, stream);
                    if (e == hipSuccess) e = launch_group_step(table_d, phase, tile, grid, stream);  // warm-up
                    if (e == hipSuccess) e = hipEventRecord(ev0, stream);
                    for (int r = 0; r < kReps && e == hipSuccess; ++r)
                        e = launch_group_step(table_d, phase, tile, grid, stream);
                    if (e == hipSuccess) e = hipEventRecord(ev1, stream);
                    if (e == hipSuccess) e = hipEventSynchronize(ev1);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms[ti], ev0, ev1);
                }
                wins[pi][oi] = ms[1] < 0.97f * ms[0];
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
            for (int pi = 0; pi < 2; ++pi) {
                int64_t m = INT64_MAX;
                for (int oi = kOrders - 1; oi >= 0 && wins[pi][oi]; --oi) m = orders[oi];
                min_ld_128[pi] = m;
            }
        return e;
    }

    hipError_t admit_one(Request *r, size_t off) {
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
        r->theta_d = (double *)take(l * 8);
        r->d_d = (double *)take(l * 8);
        r->e_d = (double *)take(l * 8);
        float *wpair = (float *)take(2 * l2 * 4);
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
        hipError_t e = hipMemcpyAsync(r->theta_d, r->theta.data(), l * 8, hipMemcpyHostToDevice, stream);
        const float *src = r->delta_pinned ? r->delta_pinned : r->delta.data();
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->W[1], src, (size_t)(r->n * r->n) * 4, hipMemcpyHostToDevice, stream);
        if (r->delta_pinned) {  // its ring space is given back once the stream is idle
            staged.push_back(r->ring_off);
            r->delta_pinned = nullptr;
            idle_since_staged = false;
        }
        if (e == hipSuccess) e = launch_pad_copy_f32_from_f32(r->D, r->W[1], r->n, r->ld, stream);
        if (e == hipSuccess && !r->symmetric) e = launch_transpose_f32(r->DT, r->D, r->ld, stream);
        if (e == hipSuccess && r->bf16) e = launch_cvt_f32_to_bf16(r->Db, r->D, (int64_t)l2, stream);
        // W[0] is the state at the identity (read if the request retires without
        // a step); W[1] and the BF16 shadows are written in full by the first
        // iterate and the first step before anything reads them
        if (e == hipSuccess) e = launch_fill_zero(r->W[0], l2 * 4, stream);
        if (e == hipSuccess) e = launch_fill_zero(r->d_d, l * 8, stream);
        r->ctl.start(r->opt, r->bf16 ? PH_BF16 : PH_FP32, false);
        r->t_admit = now_s(t0);
        return e;
    }

    hipError_t admit() {
        for (;;) {
            Request *r;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (pending.empty()) return hipSuccess;
                r = pending.front();
            }
            if (free_slots.empty()) return hipSuccess;
            size_t off;
            if (!arena.alloc(request_bytes(r->ld, r->bf16, r->symmetric), &off)) return hipSuccess;  // FIFO
            {
                std::lock_guard<std::mutex> lk(mu);
                pending.pop_front();
                st.pending = (int64_t)pending.size();
            }
            hipError_t e = admit_one(r, off);
            active.push_back(r);
            arena_used += r->bytes;
            {
                std::lock_guard<std::mutex> lk(mu);
                st.peak_bytes = std::max<int64_t>(st.peak_bytes, (int64_t)arena_used);
                st.peak_active = std::max<int64_t>(st.peak_active, (int64_t)active.size());
                st.active = (int64_t)active.size();
            }
            if (e != hipSuccess) return e;
        }
    }

    bool finished(const Request *r) const {
        return r->ctl.status != DPT_NOT_CONVERGED || r->ctl.capped();
    }

    hipError_t step() {
        GroupTable &t = *table_h;
        int nreq = 0;
        int cnt[kGroupLists] = {};
        int32_t rows = 0, tiles_sum[kGroupLists] = {};
        std::vector<Request *> first, stepping;
        for (Request *r : active) {
            if (finished(r)) continue;  // e.g. max_iter = 0: retired without a step
            stepping.push_back(r);
            if (r->at_identity) {
                first.push_back(r);
                continue;
            }
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
            const int phase = bf ? PH_BF16 : PH_FP32, tile = tile_for(r->ld, phase);
            const int L = group_list(phase, tile);
            t.idx[L][cnt[L]] = nreq;
            t.prefix[L][cnt[L]++] = tiles_sum[L];
            tiles_sum[L] += (int32_t)((r->ld / tile) * (r->ld / tile));
            ++nreq;
        }
        t.pre_prefix[nreq] = rows;
        t.counts[0] = nreq;
        for (int L = 0; L < kGroupLists; ++L) {
            t.prefix[L][cnt[L]] = tiles_sum[L];
            t.counts[1 + L] = cnt[L];
        }
        hipError_t e = hipSuccess;
        for (Request *r : first) {
            StepArgs a;
            a.n = r->n;
            a.ld = r->ld;
            a.lambda = r->lambda;
            a.theta = r->theta_d;
            a.d = r->d_d;
            a.stat = stats_d + 2 * r->slot;
            if (e == hipSuccess) e = launch_zero_u64(a.stat, 2, stream);
            if (e == hipSuccess)
                e = launch_first_iterate_f32(a, r->DT, r->W[1], r->bf16 ? r->Wb[1] : nullptr, stream);
        }
        if (e == hipSuccess && nreq > 0) {
            e = hipMemcpyAsync(table_d, table_h, offsetof(GroupTable, reqs) + (size_t)nreq * sizeof(GroupReq),
                               hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = launch_grouped();
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(stats_h, stats_d, 16 * (size_t)cfg.max_slots, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) idle_since_staged = true;
        if (e != hipSuccess) return e;
        const double t_now = now_s(t0);
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

    hipError_t retire() {
        std::vector<Request *> out;
        for (Request *r : active)
            if (finished(r)) out.push_back(r);
        if (out.empty()) return hipSuccess;
        hipError_t e = hipSuccess;
        for (Request *r : out) {
            StepArgs a;
            a.n = r->n;
            a.ld = r->ld;
            a.lambda = r->lambda;
            a.theta = r->theta_d;
            a.d = r->d_d;
            a.stat = nullptr;
            r->E.resize((size_t)r->n);
            if (e == hipSuccess) e = launch_prepass_f32_f32(r->W[r->cur], r->D, a, r->d_d, r->e_d, nullptr, stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->E.data(), r->e_d, (size_t)r->n * 8, hipMemcpyDeviceToHost, stream);
            if (r->want_z) {
                r->Z.resize((size_t)(r->n * r->n));
                float *staging = r->W[r->cur ^ 1];
                if (e == hipSuccess) e = launch_export_f32(r->W[r->cur], r->n, r->ld, staging, 0, stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(r->Z.data(), staging, r->Z.size() * 4, hipMemcpyDeviceToHost, stream);
            }
        }
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) idle_since_staged = true;
        const double t_now = now_s(t0);
        for (Request *r : out) {
            arena.release(r->off, r->bytes);
            arena_used -= r->bytes;
            free_slots.push_back(r->slot);
            r->slot = -1;
            r->t_finish = t_now;
            r->status = r->ctl.status;
            std::vector<float>().swap(r->delta);
            active.erase(std::find(active.begin(), active.end(), r));
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Request *r : out) done[r->id] = r;
            st.completed += (int64_t)out.size();
            st.active = (int64_t)active.size();
        }
        cv_done.notify_all();
        return e;
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
                if (active.empty() && pending.empty()) {
                    if (stop) break;
                    cv_work.wait_for(lk, std::chrono::milliseconds(2));
                    continue;
                }
            }
            const auto t_begin = std::chrono::steady_clock::now();
            hipError_t e = admit();
            if (e == hipSuccess && !active.empty()) e = step();
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

namespace {
// dst = (float) src (n x n), written in order (dst is pinned staging memory:
// write-combined, slow to read and to write out of order), and whether the FP32
// values are exactly symmetric, tested on the caller's cached array over 64 x 64
// blocks with their mirrors (stops at the first mismatch).
template <typename T>
bool stage_and_test(const T *src, int64_t n, float *dst) {
    const size_t nn = (size_t)(n * n);
    for (size_t i = 0; i < nn; ++i) dst[i] = (float)src[i];
    for (int64_t bi = 0; bi < n; bi += 64) {
        const int64_t ie = std::min(bi + 64, n);
        for (int64_t bj = bi; bj < n; bj += 64) {
            const int64_t je = std::min(bj + 64, n);
            for (int64_t i = bi; i < ie; ++i)
                for (int64_t j = std::max(bj, i + 1); j < je; ++j)
                    if ((float)src[i * n + j] != (float)src[j * n + i]) return false;
        }
    }
    return true;
}
}  // namespace

extern "C" {

int dpt_serve_open(dpt_server *srv, const dpt_serve_config *cfg) {
    if (!srv || !cfg || cfg->budget_bytes <= 0 || cfg->max_slots < 1 || cfg->max_slots > kServeMaxSlots ||
        cfg->grid_blocks < 0 || (cfg->autotune != 0 && cfg->autotune != 1))
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
    if (e == hipSuccess) e = hipMalloc((void **)&c->stats_d, 16 * (size_t)cfg->max_slots);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->table_h, sizeof(GroupTable), 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->stats_h, 16 * (size_t)cfg->max_slots, 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->ring.base, dpt_server_ctx::kRingBytes, 0);
    if (e == hipSuccess) c->ring.cap = dpt_server_ctx::kRingBytes;
    if (e == hipSuccess) {
        std::memset(c->table_h, 0, sizeof(GroupTable));
        e = hipMemcpy(c->table_d, c->table_h, sizeof(GroupTable), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && cfg->autotune) e = c->autotune();  // fixes the launches the graph holds
    if (e == hipSuccess && cfg->use_graph) {
        e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t e1 = c->launch_all(c->stream);
            e = hipStreamEndCapture(c->stream, &c->graph);
            if (e == hipSuccess) e = e1;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
        const int code = (e == hipErrorOutOfMemory) ? DPT_ENOMEM : DPT_EDEVICE;
        delete c;
        return code;
    }
    c->st.tile128_min_ld[0] = c->min_ld_128[0] == INT64_MAX ? -1 : c->min_ld_128[0];
    c->st.tile128_min_ld[1] = c->min_ld_128[1] == INT64_MAX ? -1 : c->min_ld_128[1];
    c->arena.init((size_t)cfg->budget_bytes);
    for (int i = cfg->max_slots - 1; i >= 0; --i) c->free_slots.push_back(i);
    c->worker = std::thread([c] { c->run(); });
    *srv = c;
    return DPT_OK;
}


int dpt_serve_submit(dpt_server srv, const dpt_problem *p, const dpt_options *o, int want_eigenvectors,
                     int64_t *ticket) {
    if (!srv || !ticket) return DPT_EINVAL;
    if (dpt_validate(p, o) != DPT_OK) return DPT_EINVAL;
    if (p->format != DPT_DENSE || p->mem != DPT_MEM_HOST) return DPT_EINVAL;
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
    // Delta goes to the pinned ring (waiting for space while earlier submissions
    // are uploaded) unless it takes more than half of it
    float *dst = nullptr;
    if (nn * 4 <= srv->ring.cap / 2) {
        std::unique_lock<std::mutex> lk(srv->ring_mu);
        size_t off = 0;
        srv->cv_ring.wait(lk, [&] { return srv->closing.load() || srv->ring.alloc(nn * 4, &off); });
        if (srv->closing.load()) {
            delete r;
            return DPT_ESTATE;
        }
        dst = (float *)(srv->ring.base + off);
        r->delta_pinned = dst;
        r->ring_off = off;
    }
    // an early return from here on gives the ring space back
    auto drop = [&](int code) {
        if (r->delta_pinned) {
            {
                std::lock_guard<std::mutex> lk(srv->ring_mu);
                srv->ring.release(r->ring_off);
            }
            srv->cv_ring.notify_all();
        }
        delete r;
        return code;
    };
    try {
        r->theta.assign((size_t)r->ld, 0.0);
        if (!dst) r->delta.resize(nn);
    } catch (...) {
        return drop(DPT_ENOMEM);
    }
    if (!dst) dst = r->delta.data();
    std::memcpy(r->theta.data(), p->theta, sizeof(double) * (size_t)p->n);
    // FP32 copy into the staging ring; symmetry of the FP32 values tested on the
    // caller's array (not on the pinned copy).
    const bool sym = p->dtype == DPT_DTYPE_F64 ? stage_and_test<double>((const double *)p->delta, p->n, dst)
                                               : stage_and_test<float>((const float *)p->delta, p->n, dst);
    r->symmetric = sym;
    if (request_bytes(r->ld, r->bf16, r->symmetric) > (size_t)srv->cfg.budget_bytes) return drop(DPT_ENOMEM);
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->stop || srv->error != DPT_OK) {
            const int code = srv->error != DPT_OK ? srv->error : DPT_ESTATE;
            lk.unlock();
            return drop(code);
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
