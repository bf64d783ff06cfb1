// Host runtime and C ABI (include/dpt.h) of the D-PT library.
//
// A handle owns the device copies of Delta needed by its precision phases, the
// ping-pong eigenvector state W = Z - I, theta, the diagonal vector
// d_n = (Delta z_n)[n] and a ring of per-step statistics.  Each application of
// the map of eq. (dyn) (Kenmoe, Smerlak, Zadorin, arXiv:2002.12872, Sec. II.B) is
// one pre-pass kernel (d) and one fused MFMA kernel (product + update + stats);
// the very first application from A = I is the closed form F(I) = I + lambda
// gap * Delta' and needs no product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <atomic>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "dpt.h"
#include "controller.h"
#include "dpt_internal.h"
#include "dpt_sparse.h"

using namespace dpt;

namespace {

int map_err(hipError_t e) {
    if (e == hipSuccess) return DPT_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return DPT_ENOMEM;
    return DPT_EDEVICE;
}

#define DPT_TRY(expr)                              \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return map_err(e_);  \
    } while (0)

double bits_to_double(unsigned long long b) {
    double x;
    std::memcpy(&x, &b, sizeof(x));
    return x;
}

int64_t pad_order(int64_t n) {
    const int64_t q = n >= 1024 ? 256 : 64;
    return (n + q - 1) / q * q;
}

bool valid_options(const dpt_options *o) {
    if (!o) return true;
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return false;
    if (o->max_iter < 0) return false;
    if (o->precision != DPT_FP64 && o->precision != DPT_FP32 && o->precision != DPT_BF16_FP32 &&
        o->precision != DPT_FP8_FP32 && o->precision != DPT_BF16_X3)
        return false;
    if (!(o->fp64_final_tol >= 0.0) || !std::isfinite(o->fp64_final_tol)) return false;
    if (!(o->stall_ratio >= 0.0) || !(o->stall_ratio <= 1.0)) return false;
    if (o->stall_patience < 1 || o->check_every < 1) return false;
    if (!(o->blowup > 0.0)) return false;
    if (o->stop_rule != DPT_STOP_DELTA && o->stop_rule != DPT_STOP_ESTIMATE && o->stop_rule != DPT_STOP_ROW)
        return false;
    if (o->stop_rule == DPT_STOP_ROW &&
        ((o->precision != DPT_FP32 && o->precision != DPT_FP64 && o->precision != DPT_BF16_FP32) ||
         o->fp64_final_tol != 0.0 || o->check_every != 1))  // rows are judged after every step
        return false;
    if (!(o->ramp_alpha >= 0.0) || !(o->ramp_alpha < 1.0)) return false;
    if (o->reserved != 0) return false;
    return true;
}

bool theta_ok(const double *theta, int64_t n) {
    std::vector<double> t(theta, theta + n);
    for (double v : t)
        if (!std::isfinite(v)) return false;
    std::sort(t.begin(), t.end());
    for (int64_t i = 1; i < n; ++i)
        if (t[i] == t[i - 1]) return false;  // unperturbed eigenvalues must be simple (Sec. II.B)
    return true;
}

bool csr_ok(const int64_t *indptr, const int32_t *indices, int64_t n, int64_t nnz) {
    if (indptr[0] != 0 || indptr[n] != nnz) return false;
    for (int64_t m = 0; m < n; ++m) {
        if (indptr[m + 1] < indptr[m]) return false;
        for (int64_t e = indptr[m]; e < indptr[m + 1]; ++e) {
            if (indices[e] < 0 || indices[e] >= n) return false;
            if (e > indptr[m] && indices[e] <= indices[e - 1]) return false;
        }
    }
    return true;
}

// The current device must be a gfx950; the answer is cached per device (the
// property query costs far more than a small solve).
int check_device() {
    static std::atomic<signed char> verdict[64];  // 0 unknown, 1 gfx950, -1 other
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return DPT_EDEVICE;
    if (dev < 64) {
        const signed char v = verdict[dev].load(std::memory_order_relaxed);
        if (v != 0) return v > 0 ? DPT_OK : DPT_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DPT_EDEVICE;
    const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (dev < 64) verdict[dev].store(ok ? 1 : -1, std::memory_order_relaxed);
    return ok ? DPT_OK : DPT_EDEVICE;
}

// True when p is device (or managed) memory that kernels may dereference.
bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // clear the error so later launch checks do not see it
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Inputs declared DPT_MEM_DEVICE must really be device memory (a host pointer
// would be dereferenced by a kernel).
// A warm start must live in the problem's memory kind: a device z0 declared
// with a host problem would otherwise be read by a host-to-device copy.
bool device_inputs_ok(const dpt_problem *p, const void *z0) {
    if (z0 && is_device_ptr(z0) != (p->mem == DPT_MEM_DEVICE)) return false;
    if (p->mem != DPT_MEM_DEVICE) return true;
    if (!is_device_ptr(p->theta) || !is_device_ptr(p->delta)) return false;
    if (p->format == DPT_CSR && (!is_device_ptr(p->indptr) || !is_device_ptr(p->indices))) return false;
    return true;
}

// Small device buffers (up to 4 MiB, power-of-two size classes) are recycled
// across handles instead of being returned to the runtime: hipMalloc and hipFree
// cost several microseconds each (an N = 64 init + destroy: 121 -> 87 us).  A
// handle's buffers are released only after its stream has drained, so a
// recycled block is idle when another handle takes it.  The pool keeps what it
// holds until the process exits: at most the peak of small buffers live at once,
// per device.
class SmallPool {
  public:
    static constexpr size_t kMax = (size_t)4 << 20;
    hipError_t alloc(void **p, size_t bytes) {
        *p = nullptr;
        if (bytes > kMax) return hipMalloc(p, bytes);
        size_t cls = 256;
        while (cls < bytes) cls <<= 1;
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        {
            std::lock_guard<std::mutex> lk(mu_);
            std::vector<void *> &fl = free_[{dev, cls}];
            if (!fl.empty()) {
                *p = fl.back();
                fl.pop_back();
                return hipSuccess;
            }
        }
        e = hipMalloc(p, cls);
        if (e != hipSuccess) return e;
        std::lock_guard<std::mutex> lk(mu_);
        owned_[*p] = {dev, cls};
        return hipSuccess;
    }
    // Blocks from alloc go back to their free list; anything else is hipFree'd.
    void release(void *p) {
        if (!p) return;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = owned_.find(p);
            if (it != owned_.end()) {
                free_[it->second].push_back(p);
                return;
            }
        }
        (void)hipFree(p);
    }

  private:
    std::mutex mu_;
    std::map<std::pair<int, size_t>, std::vector<void *>> free_;
    std::unordered_map<void *, std::pair<int, size_t>> owned_;
};

SmallPool &small_pool() {
    static SmallPool *pool = new SmallPool();  // never destroyed: blocks may outlive static destruction order
    return *pool;
}

void dfree(void *p) { small_pool().release(p); }

// Pinned host blocks of kPinBlock bytes for the uploads of small host problems:
// a copy from pinned memory is an asynchronous DMA, where one from pageable
// memory is staged by the runtime and waits for it.  A handle takes a block at
// dpt_init and gives it back once the stream has drained (the end of
// dpt_init); blocks are kept until the process exits.
constexpr size_t kPinBlock = (size_t)1 << 20;

class PinPool {
  public:
    explicit PinPool(size_t block) : block_(block) {}
    void *take() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (!free_.empty()) {
                void *p = free_.back();
                free_.pop_back();
                return p;
            }
        }
        void *p = nullptr;
        return hipHostMalloc(&p, block_, 0) == hipSuccess ? p : nullptr;
    }
    void give(void *p) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_.push_back(p);
    }

  private:
    size_t block_;
    std::mutex mu_;
    std::vector<void *> free_;
};

PinPool &pin_pool() {
    static PinPool *pool = new PinPool(kPinBlock);  // never destroyed, like the device pool
    return *pool;
}

// The pinned host mirrors of the handles' statistics rings (one block per live
// handle: read-backs into pinned memory are plain DMAs).
constexpr size_t kStatMirrorBytes = sizeof(unsigned long long) * 2 * kStatRing;
PinPool &stat_mirror_pool() {
    static PinPool *pool = new PinPool(kStatMirrorBytes);
    return *pool;
}

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return hipSuccess;
    return small_pool().alloc((void **)p, count * sizeof(T));
}

// HIP-event timing of kernel launches (per DPT_PROF_* class).
struct Profiler : ProfHook {
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    bool on = false;
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double ms[DPT_PROF_KINDS] = {};
    int64_t launches[DPT_PROF_KINDS] = {};

    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin(int kind, hipStream_t s) override {
        if (!on) return;
        Rec r{kind, take(), take()};
        if (!r.a || !r.b) return;
        (void)hipEventRecord(r.a, s);
        pending.push_back(r);
    }
    void end(hipStream_t s) override {
        if (!on || pending.empty()) return;
        (void)hipEventRecord(pending.back().b, s);
        if (pending.size() > 8192) collect();
    }
    void collect() {
        for (const Rec &r : pending) {
            float t = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                ms[r.kind] += t;
                launches[r.kind] += 1;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
    void reset() {
        collect();
        for (int i = 0; i < DPT_PROF_KINDS; ++i) {
            ms[i] = 0.0;
            launches[i] = 0;
        }
    }
    ~Profiler() override {
        for (const Rec &r : pending) {
            (void)hipEventSynchronize(r.b);
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

}  // namespace

struct dpt_ctx {
    int64_t n = 0, ld = 0;
    double lambda = 0.0;
    hipStream_t stream = nullptr;
    dpt_options opt{};
    int format = DPT_DENSE, in_dtype = DPT_DTYPE_F32, mem = DPT_MEM_HOST;
    bool symmetric = false;

    double *theta = nullptr;  // ld entries
    double *dvec = nullptr;   // ld entries
    double *evec = nullptr;   // ld entries
    unsigned long long *stats = nullptr;
    unsigned long long *stats_host = nullptr;  // host mirror of the ring (read after a stream sync)

    // dense Delta copies (padded ld x ld); *_own tells whether we free them
    float *d32 = nullptr, *dT32 = nullptr;
    double *d64 = nullptr, *dT64 = nullptr;
    __bf16 *db16 = nullptr;
    bool d32_own = false, d64_own = false;

    // split BF16 operands (DPT_BF16_X3): ld x 2ld, [h | l] of Delta and of W
    __bf16 *Dx3 = nullptr, *Wx3[2] = {nullptr, nullptr};
    // block-scaled FP8 copies (DPT_FP8_FP32): values and E8M0 scales per 32 values
    unsigned char *dq8 = nullptr, *ds8 = nullptr;
    unsigned char *Wq8[2] = {nullptr, nullptr}, *Ws8[2] = {nullptr, nullptr};

    // state
    float *W32[2] = {nullptr, nullptr};
    __bf16 *Wb[2] = {nullptr, nullptr};
    double *W64[2] = {nullptr, nullptr};
    int cur = 0;
    int phase = PH_FP32;
    bool at_identity = true;
    double ramp_ak = 1.0;       // ramp_alpha^k after k applications of F
    bool last_ramping = false;  // the last application used a ramped coupling

    // per-row retirement (DPT_STOP_ROW)
    std::vector<int32_t> retired_at;  // per row: applications of F when frozen, 0 running
    std::vector<int32_t> active;      // running rows, ascending
    int32_t *rowmap = nullptr;        // device: running rows padded with -1 to map_rows
    int32_t *newly = nullptr;         // device: rows frozen by the last step
    double *rowdelta = nullptr;       // device: per map entry, the row's delta
    int64_t list_rows = 0;            // entries of rowmap in use
    int64_t map_rows = 0;             // rows the products run on; 0: all (nothing frozen yet)
    int64_t rows_multiplied = 0;      // rows the products ran on, summed over product steps
    bool w0_dirty = false;  // W32[0] not yet cleared to the identity state (see clean_identity)
    int64_t k = 0;

    SparseState *sp = nullptr;
    Profiler prof;
    void *small_hist = nullptr;  // iterates of one fused small-problem batch (ld = 64)
    // pinned staging of a small host problem's uploads during dpt_init
    unsigned char *pin = nullptr;
    size_t pin_used = 0;
    // kPinBlock bytes of pinned staging at pin + pin_used, or null
    void *pin_space(size_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        if (!pin || pin_used + bytes > kPinBlock) return nullptr;
        void *q = pin + pin_used;
        pin_used += bytes;
        return q;
    }

    ~dpt_ctx() {
        if (sp) sparse_destroy(sp);
        void *own[] = {theta, dvec, evec, stats, db16, W32[0], W32[1], Wb[0], Wb[1], W64[0], W64[1],
                       dq8, ds8, Wq8[0], Wq8[1], Ws8[0], Ws8[1], small_hist, Dx3, Wx3[0], Wx3[1],
                       rowmap, newly, rowdelta};
        for (void *p : own) dfree(p);
        if (dT32 && dT32 != d32) dfree(dT32);
        if (dT64 && dT64 != d64) dfree(dT64);
        if (d32 && d32_own) dfree(d32);
        if (d64 && d64_own) dfree(d64);
        stat_mirror_pool().give(stats_host);  // the stream has drained (see below)
        pin_pool().give(pin);  // the stream has drained: the destructor runs after a synchronisation
    }
};

namespace {

// Stage a dense Delta of the input dtype into padded device copy(ies).
template <typename T>
hipError_t stage_dense(dpt_ctx *c, const dpt_problem *p, T **dst, bool *own) {
    const int64_t n = c->n, ld = c->ld;
    const bool same_type = (sizeof(T) == 8) == (p->dtype == DPT_DTYPE_F64);
    // borrowed when no padding is needed and the kernels' 16-byte vector
    // accesses are aligned; copied otherwise
    const bool aligned = ((uintptr_t)p->delta & 15) == 0;
    if (same_type && p->mem == DPT_MEM_DEVICE && n == ld && aligned) {
        *dst = (T *)p->delta;  // borrowed
        *own = false;
        return hipSuccess;
    }
    hipError_t e = dalloc(dst, (size_t)(ld * ld));
    if (e != hipSuccess) return e;
    *own = true;
    // small host inputs: converted and padded on the host, one upload (from the
    // handle's pinned block when it has room: no wait; dpt_init drains the
    // stream before it returns)
    if (p->mem == DPT_MEM_HOST && (size_t)(ld * ld) * sizeof(T) <= ((size_t)16 << 20)) {
        const size_t count = (size_t)(ld * ld);
        T *pinned = (T *)c->pin_space(count * sizeof(T));
        std::vector<T> hostpad;
        if (!pinned) hostpad.assign(count, (T)0);
        T *hp = pinned ? pinned : hostpad.data();
        if (pinned) std::memset(hp, 0, count * sizeof(T));
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j)
                hp[(size_t)(i * ld + j)] = p->dtype == DPT_DTYPE_F64 ? (T)((const double *)p->delta)[i * n + j]
                                                                    : (T)((const float *)p->delta)[i * n + j];
        e = hipMemcpyAsync(*dst, hp, count * sizeof(T), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && !pinned) e = hipStreamSynchronize(c->stream);  // hostpad is freed on return
        return e;
    }
    const void *src = p->delta;
    void *tmp = nullptr;
    const size_t in_bytes = (size_t)(n * n) * (p->dtype == DPT_DTYPE_F64 ? 8 : 4);
    if (p->mem == DPT_MEM_HOST) {
        e = hipMalloc(&tmp, in_bytes);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(tmp, p->delta, in_bytes, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return e;
        }
        src = tmp;
    }
    if (sizeof(T) == 4) {
        e = p->dtype == DPT_DTYPE_F64
                ? launch_pad_copy_f32_from_f64((float *)*dst, (const double *)src, n, ld, c->stream)
                : launch_pad_copy_f32_from_f32((float *)*dst, (const float *)src, n, ld, c->stream);
    } else {
        e = p->dtype == DPT_DTYPE_F64
                ? launch_pad_copy_f64_from_f64((double *)*dst, (const double *)src, n, ld, c->stream)
                : launch_pad_copy_f64_from_f32((double *)*dst, (const float *)src, n, ld, c->stream);
    }
    if (tmp) {
        hipError_t e2 = hipStreamSynchronize(c->stream);
        (void)hipFree(tmp);
        if (e == hipSuccess) e = e2;
    }
    return e;
}

// FP64 copies for the FP64 phase (on demand when the input is FP32).
int ensure_f64(dpt_ctx *c) {
    if (!c->d64) {
        DPT_TRY(dalloc(&c->d64, (size_t)(c->ld * c->ld)));
        c->d64_own = true;
        DPT_TRY(launch_cvt_f32_to_f64(c->d64, c->d32, c->ld * c->ld, c->stream));
    }
    if (!c->dT64) {
        if (c->symmetric) {
            c->dT64 = c->d64;
        } else {
            DPT_TRY(dalloc(&c->dT64, (size_t)(c->ld * c->ld)));
            DPT_TRY(launch_transpose_f64(c->dT64, c->d64, c->ld, c->stream));
        }
    }
    if (!c->W64[0]) {  // both buffers, zeroed together (a failed second allocation releases the first)
        DPT_TRY(dalloc(&c->W64[0], (size_t)(c->ld * c->ld)));
        const hipError_t e = dalloc(&c->W64[1], (size_t)(c->ld * c->ld));
        if (e != hipSuccess) {
            dfree(c->W64[0]);
            c->W64[0] = nullptr;
            return map_err(e);
        }
        void *zp[2] = {c->W64[0], c->W64[1]};
        const size_t zb[2] = {sizeof(double) * (size_t)(c->ld * c->ld), sizeof(double) * (size_t)(c->ld * c->ld)};
        DPT_TRY(launch_zero_many(zp, zb, 2, c->stream));
    }
    return DPT_OK;
}

// Scratch device buffer released (after its stream drains) on scope exit.
struct DeviceTemp {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~DeviceTemp() {
        if (p) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(p);
        }
    }
};

StepArgs step_args(dpt_ctx *c, unsigned long long *slot, double lambda) {
    StepArgs a;
    a.n = c->n;
    a.ld = c->ld;
    a.lambda = lambda;
    a.theta = c->theta;
    a.d = c->dvec;
    a.stat = slot;
    return a;
}

StepArgs step_args(dpt_ctx *c, unsigned long long *slot) { return step_args(c, slot, c->lambda); }

// Coupling of the next application of F (Supplement E's ramp): lambda (1 -
// alpha^k) for the k-th application while alpha^k >= 2^-53, lambda otherwise.
double next_lambda(const dpt_ctx *c, bool *ramping) {
    *ramping = false;
    if (c->opt.ramp_alpha > 0.0) {
        const double ak = c->ramp_ak * c->opt.ramp_alpha;
        if (ak >= 0x1p-53) {
            *ramping = true;
            return c->lambda * (1.0 - ak);
        }
    }
    return c->lambda;
}

// Clear W32[0] to the identity state if it has not been written yet; every
// reader of the FP32 state that can run before the first step calls it.
int clean_identity(dpt_ctx *c) {
    if (c->w0_dirty) {
        DPT_TRY(launch_fill_zero(c->W32[0], (size_t)(c->ld * c->ld) * 4, c->stream));
        c->w0_dirty = false;
    }
    return DPT_OK;
}

// Leave the reduced-precision phase.  DPT_BF16_X3 sweeps read the split form
// of the current state, made here from its FP32 copy.
int enter_fp32(dpt_ctx *c) {
    // only the identity state (cur == 0) can still be uncleared; after the first
    // iterate W32[0] is overwritten by the next step before anything reads it
    if (c->cur == 0) {
        int rc = clean_identity(c);
        if (rc != DPT_OK) return rc;
    }
    c->phase = PH_FP32;
    if (c->opt.precision == DPT_BF16_X3) DPT_TRY(launch_split_x3(c->W32[c->cur], c->ld, c->Wx3[c->cur], c->stream));
    return DPT_OK;
}

// Switch the state to the FP64 phase (upcast the FP32 state).
int enter_fp64(dpt_ctx *c) {
    int rc = c->cur == 0 ? clean_identity(c) : DPT_OK;
    if (rc != DPT_OK) return rc;
    rc = ensure_f64(c);
    if (rc != DPT_OK) return rc;
    if (c->phase != PH_FP64) {
        DPT_TRY(launch_cvt_f32_to_f64(c->W64[c->cur], c->W32[c->cur], c->ld * c->ld, c->stream));
        c->phase = PH_FP64;
    }
    return DPT_OK;
}

// One application of F with coupling lam in the current phase; the stats land
// in ring slot k.
int dense_step(dpt_ctx *c, double lam) {
    const int slot = (int)(c->k % kStatRing);
    unsigned long long *st = c->stats + 2 * slot;
    StepArgs a = step_args(c, st, lam);
    if (c->map_rows > 0 && !c->at_identity) {  // frozen rows are left out of the product
        a.rowmap = c->rowmap;
        a.rows = c->map_rows;
    }
    if (!c->retired_at.empty() && c->active.empty()) {  // every row frozen: nothing changes
        DPT_TRY(launch_zero_u64(st, 2, c->stream));
        c->k += 1;
        return DPT_OK;
    }
    const int nx = c->cur ^ 1;
    hipStream_t s = c->stream;
    Profiler &pf = c->prof;
    hipError_t e = hipSuccess;
    if (c->at_identity) {
        DPT_TRY(launch_zero_u64(st, 2, s));
        pf.begin(DPT_PROF_FIRST, s);
        const bool fp8 = c->phase == PH_BF16 && c->opt.precision == DPT_FP8_FP32;
        if (c->phase == PH_FP64)
            e = launch_first_iterate_f64(a, c->dT64, c->W64[nx], s);
        else
            e = launch_first_iterate_f32(a, c->dT32, c->W32[nx], c->phase == PH_BF16 && !fp8 ? c->Wb[nx] : nullptr,
                                         s);
        if (e == hipSuccess && fp8) e = launch_quant_fp8(c->W32[nx], c->ld, c->Wq8[nx], c->Ws8[nx], s);
        pf.end(s);
        DPT_TRY(e);
    } else {
        pf.begin(DPT_PROF_PREPASS, s);
        if (c->phase == PH_FP64)
            e = launch_prepass_f64_f64(c->W64[c->cur], c->d64, a, c->dvec, nullptr, st, s);
        else
            e = launch_prepass_f32_f32(c->W32[c->cur], c->d32, a, c->dvec, nullptr, st, s);
        pf.end(s);
        DPT_TRY(e);
        if (c->phase == PH_FP64) {
            pf.begin(DPT_PROF_GEMM_FP64, s);
            e = launch_step_f64(a, c->W64[c->cur], c->d64, c->dT64, c->W64[nx], s);
        } else if (c->phase == PH_FP32 && c->opt.precision == DPT_BF16_X3) {
            pf.begin(DPT_PROF_GEMM_X3, s);
            e = launch_step_x3_large(a, c->Wx3[c->cur], c->Dx3, c->dT32, c->W32[c->cur], c->W32[nx], c->Wx3[nx], s);
        } else if (c->phase == PH_FP32) {
            pf.begin(DPT_PROF_GEMM_FP32, s);
            e = launch_step_f32(a, c->W32[c->cur], c->d32, c->dT32, c->W32[nx], nullptr, s);
        } else if (c->opt.precision == DPT_FP8_FP32) {
            pf.begin(DPT_PROF_GEMM_FP8, s);
            e = launch_step_fp8_large(a, c->Wq8[c->cur], c->Ws8[c->cur], c->dq8, c->ds8, c->dT32, c->W32[c->cur],
                                      c->W32[nx], c->Wq8[nx], c->Ws8[nx], s);
        } else {
            pf.begin(DPT_PROF_GEMM_BF16, s);
            e = launch_step_bf16(a, c->Wb[c->cur], c->db16, c->dT32, c->W32[c->cur], c->W32[nx], c->Wb[nx], s);
        }
        pf.end(s);
        DPT_TRY(e);
        c->rows_multiplied += a.rowmap ? a.rows : c->ld;
    }
    if (nx == 0 && c->phase != PH_FP64) c->w0_dirty = false;  // the step wrote all of W32[0]
    c->cur = nx;
    c->at_identity = false;
    c->k += 1;
    return DPT_OK;
}

int do_step(dpt_ctx *c) {
    bool ramping = false;
    const double lam = next_lambda(c, &ramping);
    const int rc = c->sp ? sparse_step(c->sp, lam, c->theta, c->stats, &c->k, c->stream, &c->prof)
                         : dense_step(c, lam);
    if (rc != DPT_OK) return rc;
    c->ramp_ak *= c->opt.ramp_alpha > 0.0 ? c->opt.ramp_alpha : 1.0;
    c->last_ramping = ramping;
    return DPT_OK;
}

// Copy the stats of steps [k0, k1) to the host mirror and synchronise.
int fetch_stats(dpt_ctx *c, int64_t k0, int64_t k1) {
    if (k1 <= k0) return DPT_OK;
    if (k1 - k0 > kStatRing) k0 = k1 - kStatRing;
    int64_t i = k0;
    while (i < k1) {
        const int64_t s0 = i % kStatRing;
        const int64_t run = std::min<int64_t>(k1 - i, kStatRing - s0);
        DPT_TRY(hipMemcpyAsync(c->stats_host + 2 * s0, c->stats + 2 * s0, (size_t)run * 16, hipMemcpyDeviceToHost,
                               c->stream));
        i += run;
    }
    DPT_TRY(hipStreamSynchronize(c->stream));
    return DPT_OK;
}

void stat_of(dpt_ctx *c, int64_t step, double *delta, double *wmax) {
    const int64_t s0 = step % kStatRing;
    *delta = bits_to_double(c->stats_host[2 * s0]);
    *wmax = bits_to_double(c->stats_host[2 * s0 + 1]);
}

// Small dense problems (ld = 64) in the FP32 or FP64 phase run kSmallBatch
// steps per launch in one workgroup (k_small_steps): per-step launches and
// read-backs would cost ~25 us per step against ~1 us of work.  The stopping
// rule still sees every step's statistics in order; the state is set to the
// iterate it stops on.
constexpr int kSmallBatch = 16;

bool small_batch_ok(const dpt_ctx *c) {
    if (c->opt.stop_rule == DPT_STOP_ROW) return false;  // rows are judged one by one after every step
    bool ramping = false;
    (void)next_lambda(c, &ramping);  // a batch runs at one coupling: not while the ramp runs
    return !c->sp && c->ld == 64 && (c->phase == PH_FP32 || c->phase == PH_FP64) && c->opt.check_every == 1 &&
           !c->prof.on && !ramping;
}

// Up to kSmallBatch steps; *taken gets the number the controller consumed and
// *act its last decision.  Every consumed step is counted in ctl and recorded
// in r's history.
// Steps to run speculatively: a full batch at first (a step costs about a
// microsecond at this size, a launch and read-back round trip 25-40), then the
// number the recent contraction rate predicts until delta < tol (plus one), at
// most kSmallBatch.  The prediction only affects how many steps are computed
// and discarded.
int small_batch_size(dpt_ctx *c, const Controller &ctl, int64_t consumed) {
    const int left = std::max(1, c->opt.max_iter - ctl.iters);
    if (consumed < 3) return std::min(kSmallBatch, left);
    double d1, d2, d3, w;
    stat_of(c, c->k - 1, &d1, &w);
    stat_of(c, c->k - 2, &d2, &w);
    stat_of(c, c->k - 3, &d3, &w);
    const double rho = std::max(d1 / d2, d2 / d3);
    const double tol = c->phase == PH_FP64 && c->opt.fp64_final_tol > 0 ? c->opt.fp64_final_tol : c->opt.tol;
    int b = kSmallBatch;
    if (rho > 0.0 && rho < 1.0 && d1 > tol) b = (int)std::ceil(std::log(tol / d1) / std::log(rho)) + 1;
    return std::min(left, std::max(2, std::min(kSmallBatch, b)));
}

int small_batch(dpt_ctx *c, Controller &ctl, dpt_result *r, int64_t consumed, int *taken,
                Controller::Action *act) {
    int rc0 = clean_identity(c);
    if (rc0 != DPT_OK) return rc0;
    const int m = small_batch_size(c, ctl, consumed);
    const bool f64 = c->phase == PH_FP64;
    const size_t l2 = (size_t)(c->ld * c->ld), esz = f64 ? 8 : 4;
    if (!c->small_hist) DPT_TRY(dalloc((unsigned char **)&c->small_hist, (size_t)kSmallBatch * l2 * 8));
    const StepArgs a = step_args(c, nullptr);
    // the first delta below the phase's target ends the batch on the device: the
    // controller's decision (delta or estimate rule) comes at that step or earlier
    const double target = (c->phase == PH_FP64 && c->opt.precision != DPT_FP64) ? c->opt.fp64_final_tol : c->opt.tol;
    hipError_t e;
    if (f64)
        e = launch_small_steps_f64(c->W64[c->cur], (double *)c->small_hist, c->d64, c->dT64, a, c->stats, c->k, m,
                                   c->at_identity ? 1 : 0, c->dvec, target, c->opt.blowup, c->stream);
    else
        e = launch_small_steps_f32(c->W32[c->cur], (float *)c->small_hist, c->d32, c->dT32, a, c->stats, c->k, m,
                                   c->at_identity ? 1 : 0, c->dvec, target, c->opt.blowup, c->stream);
    DPT_TRY(e);
    int rc = fetch_stats(c, c->k, c->k + m);
    if (rc != DPT_OK) return rc;
    // the steps the kernel computed: it ends after the first step meeting its
    // exit test (same values, same test)
    int computed = m;
    for (int s = 0; s < m; ++s) {
        double dl, wm;
        stat_of(c, c->k + s, &dl, &wm);
        if (!(dl <= DBL_MAX) || dl < target || !(wm <= c->opt.blowup)) {
            computed = s + 1;
            break;
        }
    }
    int j = 0;
    Controller::Action last = Controller::CONTINUE;
    while (j < m) {
        double dl, wm;
        stat_of(c, c->k + j, &dl, &wm);
        ctl.count_step();
        if (r && r->delta_history && ctl.iters - 1 < r->history_cap) r->delta_history[ctl.iters - 1] = dl;
        ++j;
        last = ctl.update(dl, wm);
        if (last != Controller::CONTINUE || ctl.capped()) break;
    }
    // the state becomes iterate j of the batch (the kernel left the last one it
    // computed there)
    if (j != computed) {
        void *dst = f64 ? (void *)c->W64[c->cur] : (void *)c->W32[c->cur];
        DPT_TRY(hipMemcpyAsync(dst, (const unsigned char *)c->small_hist + (size_t)(j - 1) * l2 * esz, l2 * esz,
                               hipMemcpyDeviceToDevice, c->stream));
    }
    c->k += j;
    c->at_identity = false;
    *taken = j;
    *act = last;
    return DPT_OK;
}


// Exact symmetry of a small host matrix (n x n row-major, dtype of the input).
bool host_symmetric(const dpt_problem *p) {
    const int64_t n = p->n;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            const bool eq = p->dtype == DPT_DTYPE_F64
                                ? ((const double *)p->delta)[i * n + j] == ((const double *)p->delta)[j * n + i]
                                : ((const float *)p->delta)[i * n + j] == ((const float *)p->delta)[j * n + i];
            if (!eq) return false;
        }
    return true;
}

// Symmetry test of the staged copy on the device (flag read back, into the
// handle's pinned block when it has one; the wait also completes every
// read-back enqueued before it).
template <typename T>
int device_symmetric(dpt_ctx *c, const T *src, __bf16 *bf, bool *sym) {
    unsigned int *flag = nullptr;
    DPT_TRY(dalloc(&flag, 1));
    hipError_t e = launch_fill_zero(flag, 4, c->stream);
    if (e == hipSuccess) {
        if (sizeof(T) == 8)
            e = launch_symmetry_check_f64((const double *)src, c->ld, flag, c->stream);
        else
            e = launch_symmetry_check_f32((const float *)src, c->ld, flag, bf, c->stream);
    }
    unsigned int h_local = 0;
    unsigned int *h = (unsigned int *)c->pin_space(sizeof(unsigned int));
    if (!h) h = &h_local;
    if (e == hipSuccess) e = hipMemcpyAsync(h, flag, 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(flag);
    DPT_TRY(e);
    *sym = (*h == 0);
    return DPT_OK;
}

int init_dense(dpt_ctx *c, const dpt_problem *p, const void *z0) {
    const int64_t ld = c->ld;
    const size_t nn = (size_t)(ld * ld);
    const int prec = c->opt.precision;
    hipStream_t s = c->stream;
    // small host inputs are tested for symmetry on the host (no device round trip)
    const bool host_sym_test = p->mem == DPT_MEM_HOST && p->n <= 256;
    // Primary copy in the input dtype; the symmetry test runs on it.
    if (p->dtype == DPT_DTYPE_F64) {
        DPT_TRY(stage_dense<double>(c, p, &c->d64, &c->d64_own));
        if (host_sym_test) {
            c->symmetric = host_symmetric(p);
        } else {
            int rc = device_symmetric<double>(c, c->d64, nullptr, &c->symmetric);
            if (rc != DPT_OK) return rc;
        }
        if (prec != DPT_FP64) DPT_TRY(stage_dense<float>(c, p, &c->d32, &c->d32_own));
    } else {
        DPT_TRY(stage_dense<float>(c, p, &c->d32, &c->d32_own));
        if (host_sym_test) {
            c->symmetric = host_symmetric(p);
        } else {
            // the BF16 form of Delta comes out of the same pass over it
            if (prec == DPT_BF16_FP32 || prec == DPT_BF16_X3) DPT_TRY(dalloc(&c->db16, nn));
            int rc = device_symmetric<float>(c, c->d32, c->db16, &c->symmetric);
            if (rc != DPT_OK) return rc;
        }
        if (prec == DPT_FP64) {
            DPT_TRY(dalloc(&c->d64, nn));
            c->d64_own = true;
            DPT_TRY(launch_cvt_f32_to_f64(c->d64, c->d32, (int64_t)nn, s));
        }
    }
    // A host-memory start is first copied to the device.
    const size_t z0_bytes = (size_t)(c->n * c->n) * (p->dtype == DPT_DTYPE_F64 ? 8 : 4);
    DeviceTemp z0_dev;
    z0_dev.s = s;
    if (z0 && p->mem == DPT_MEM_HOST) {
        DPT_TRY(hipMalloc(&z0_dev.p, z0_bytes));
        DPT_TRY(hipMemcpyAsync(z0_dev.p, z0, z0_bytes, hipMemcpyHostToDevice, s));
        z0 = z0_dev.p;
    }
    if (prec == DPT_FP64) {
        int rc = ensure_f64(c);
        if (rc != DPT_OK) return rc;
        c->phase = PH_FP64;
        if (z0) {
            DPT_TRY(launch_load_state_f64(c->W64[0], z0, p->dtype == DPT_DTYPE_F64, c->n, ld, s));
            c->at_identity = false;
        }
    } else {
        if (c->symmetric) {
            c->dT32 = c->d32;
        } else {
            DPT_TRY(dalloc(&c->dT32, nn));
            DPT_TRY(launch_transpose_f32(c->dT32, c->d32, ld, s));
        }
        // W32[0] is the state at the identity (W = 0); nothing but a readout
        // at the identity reads it before a step overwrites it, so it is
        // cleared on first such use (clean_identity; a solve never needs it).
        // W32[1] and the BF16 shadows are written in full by the first iterate
        // (or a warm start) before anything reads them, except in the FP8
        // form, which quantises both states here.
        for (int i = 0; i < 2; ++i) {
            DPT_TRY(dalloc(&c->W32[i], nn));
            if (prec == DPT_FP8_FP32) DPT_TRY(launch_fill_zero(c->W32[i], nn * 4, s));
        }
        c->w0_dirty = prec != DPT_FP8_FP32;
        if (prec == DPT_BF16_FP32 || prec == DPT_BF16_X3) {
            if (!c->db16) {
                DPT_TRY(dalloc(&c->db16, nn));
                DPT_TRY(launch_cvt_f32_to_bf16(c->db16, c->d32, (int64_t)nn, s));
            }
            for (int i = 0; i < 2; ++i) DPT_TRY(dalloc(&c->Wb[i], nn));
            if (prec == DPT_BF16_X3) {  // split operands for the FP32-grade sweeps
                DPT_TRY(dalloc(&c->Dx3, 2 * nn));
                DPT_TRY(launch_split_x3(c->d32, ld, c->Dx3, s));
                for (int i = 0; i < 2; ++i) DPT_TRY(dalloc(&c->Wx3[i], 2 * nn));
            }
            c->phase = PH_BF16;
        } else if (prec == DPT_FP8_FP32) {
            DPT_TRY(dalloc(&c->dq8, nn));
            DPT_TRY(dalloc(&c->ds8, nn / 32));
            DPT_TRY(launch_quant_fp8(c->d32, ld, c->dq8, c->ds8, s));
            for (int i = 0; i < 2; ++i) {
                DPT_TRY(dalloc(&c->Wq8[i], nn));
                DPT_TRY(dalloc(&c->Ws8[i], nn / 32));
                DPT_TRY(launch_quant_fp8(c->W32[i], ld, c->Wq8[i], c->Ws8[i], s));  // of the zero state
            }
            c->phase = PH_BF16;  // the reduced-precision phase
        } else {
            c->phase = PH_FP32;
        }
        if (z0) {
            DPT_TRY(launch_load_state_f32(c->W32[0], z0, p->dtype == DPT_DTYPE_F64, c->n, ld, s));
            if (prec == DPT_BF16_FP32 || prec == DPT_BF16_X3)
                DPT_TRY(launch_cvt_f32_to_bf16(c->Wb[0], c->W32[0], (int64_t)nn, s));
            if (prec == DPT_FP8_FP32) DPT_TRY(launch_quant_fp8(c->W32[0], ld, c->Wq8[0], c->Ws8[0], s));
            c->at_identity = false;
            c->w0_dirty = false;
        }
    }
    if (z0_dev.p) DPT_TRY(hipStreamSynchronize(s));  // the temporary is freed on return
    return DPT_OK;
}

// Warm start of a CSR problem: z0 (problem's dtype and memory kind) becomes the
// transposed state; a host z0 is uploaded through a temporary device copy.
int sparse_warm_start(dpt_ctx *c, const dpt_problem *p, const void *z0) {
    const size_t bytes = (size_t)(c->n * c->n) * (p->dtype == DPT_DTYPE_F64 ? 8 : 4);
    DeviceTemp tmp;
    tmp.s = c->stream;
    if (p->mem == DPT_MEM_HOST) {
        DPT_TRY(hipMalloc(&tmp.p, bytes));
        DPT_TRY(hipMemcpyAsync(tmp.p, z0, bytes, hipMemcpyHostToDevice, c->stream));
        z0 = tmp.p;
    }
    DPT_TRY(sparse_load_state(c->sp, z0, p->dtype == DPT_DTYPE_F64, c->stream));
    if (tmp.p) DPT_TRY(hipStreamSynchronize(c->stream));
    return DPT_OK;
}

// The phase in which DPT_STOP_ROW retires rows.
bool row_phase(const dpt_ctx *c) {
    return c->opt.stop_rule == DPT_STOP_ROW && !c->sp &&
           (c->opt.precision == DPT_FP64 ? c->phase == PH_FP64 : c->phase == PH_FP32);
}

// Upload the running rows as the product's row list (padded with -1 to the
// product tile, at most ld entries).
int upload_rowmap(dpt_ctx *c) {
    const int64_t tile = row_tile(c->ld);
    const int64_t cnt = (int64_t)c->active.size();
    const int64_t rows = std::min<int64_t>(c->ld, (cnt + tile - 1) / tile * tile);
    std::vector<int32_t> h((size_t)rows, -1);
    std::copy(c->active.begin(), c->active.end(), h.begin());
    DPT_TRY(hipMemcpyAsync(c->rowmap, h.data(), sizeof(int32_t) * (size_t)rows, hipMemcpyHostToDevice, c->stream));
    DPT_TRY(hipStreamSynchronize(c->stream));  // h is freed on return
    c->list_rows = rows;
    c->map_rows = (int64_t)c->active.size() < c->n ? rows : 0;  // the full fast kernels until a row freezes
    return DPT_OK;
}

// After a step of the retiring phase: freeze the running rows whose own delta is
// below tol (their value goes to both state buffers), shrink the row list.
// *left receives the number of rows still running.
int retire_rows(dpt_ctx *c, int64_t *left) {
    if (!c->rowmap) {
        DPT_TRY(dalloc(&c->rowmap, (size_t)c->ld));
        DPT_TRY(dalloc(&c->newly, (size_t)c->ld));
        DPT_TRY(dalloc(&c->rowdelta, (size_t)c->ld));
        c->retired_at.assign((size_t)c->n, 0);
        c->active.resize((size_t)c->n);
        for (int64_t i = 0; i < c->n; ++i) c->active[(size_t)i] = (int32_t)i;
        int rc = upload_rowmap(c);
        if (rc != DPT_OK) return rc;
    }
    const int64_t rows = c->list_rows;
    const bool f64 = c->phase == PH_FP64;
    DPT_TRY(f64 ? launch_row_delta_f64(c->W64[c->cur], c->W64[c->cur ^ 1], c->rowmap, rows, c->ld, c->rowdelta,
                                       c->stream)
                : launch_row_delta_f32(c->W32[c->cur], c->W32[c->cur ^ 1], c->rowmap, rows, c->ld, c->rowdelta,
                                       c->stream));
    std::vector<double> hd((size_t)rows);
    DPT_TRY(hipMemcpyAsync(hd.data(), c->rowdelta, sizeof(double) * (size_t)rows, hipMemcpyDeviceToHost, c->stream));
    DPT_TRY(hipStreamSynchronize(c->stream));
    std::vector<int32_t> keep, frozen;
    for (size_t i = 0; i < c->active.size(); ++i) {
        const int32_t r = c->active[i];
        if (hd[i] < c->opt.tol) {
            frozen.push_back(r);
            c->retired_at[(size_t)r] = (int32_t)c->k;
        } else {
            keep.push_back(r);
        }
    }
    if (!frozen.empty()) {
        DPT_TRY(hipMemcpyAsync(c->newly, frozen.data(), sizeof(int32_t) * frozen.size(), hipMemcpyHostToDevice,
                               c->stream));
        const int nx = c->cur ^ 1;
        DPT_TRY(f64 ? launch_copy_rows_f64(c->W64[nx], c->W64[c->cur], c->newly, (int64_t)frozen.size(), c->ld,
                                           c->stream)
                    : launch_copy_rows_f32(c->W32[nx], c->W32[c->cur], c->newly, (int64_t)frozen.size(), c->ld,
                                           c->stream));
        c->active.swap(keep);
        if (!c->active.empty()) {
            int rc = upload_rowmap(c);
            if (rc != DPT_OK) return rc;
        }
        DPT_TRY(hipStreamSynchronize(c->stream));  // `frozen` is freed on return
    }
    *left = (int64_t)c->active.size();
    return DPT_OK;
}

// E = theta + lambda d from the current state, into c->evec.
int compute_eigenvalues(dpt_ctx *c) {
    int rc = clean_identity(c);
    if (rc != DPT_OK) return rc;
    if (c->sp) return map_err(sparse_eigenvalues(c->sp, c->lambda, c->theta, c->evec, c->stream));
    const StepArgs a = step_args(c, nullptr);
    if (c->phase == PH_FP64) {
        DPT_TRY(launch_prepass_f64_f64(c->W64[c->cur], c->d64, a, c->dvec, c->evec, nullptr, c->stream));
    } else if (c->d64) {
        DPT_TRY(launch_prepass_f32_f64(c->W32[c->cur], c->d64, a, c->dvec, c->evec, nullptr, c->stream));
    } else {
        DPT_TRY(launch_prepass_f32_f32(c->W32[c->cur], c->d32, a, c->dvec, c->evec, nullptr, c->stream));
    }
    return DPT_OK;
}

}  // namespace

// ============================================================== C ABI
namespace dpt {
bool host_theta_ok(const double *theta, int64_t n) { return theta_ok(theta, n); }
void *pinned_block_take() { return stat_mirror_pool().take(); }
void pinned_block_give(void *p) { stat_mirror_pool().give(p); }
hipError_t pooled_malloc(void **p, size_t bytes) { return small_pool().alloc(p, bytes); }
void pooled_free(void *p) { small_pool().release(p); }
bool inputs_on_device(const dpt_problem *p) { return p->mem == DPT_MEM_DEVICE && device_inputs_ok(p, nullptr); }
}  // namespace dpt

extern "C" {

void dpt_options_default(dpt_options *o) {
    if (!o) return;
    o->tol = 1e-6;
    o->fp64_final_tol = 0.0;
    o->stall_ratio = 0.5;
    o->blowup = 1e6;
    o->max_iter = 200;
    o->precision = DPT_FP32;
    o->stall_patience = 2;
    o->check_every = 1;
    o->stop_rule = DPT_STOP_DELTA;
    o->ramp_alpha = 0.0;
    o->reserved = 0;
}

namespace {
// Host-side argument checks; full = also the host-memory theta and CSR content
// (the dominant mode checks those itself).
int validate_args(const dpt_problem *p, const dpt_options *o, bool full) {
    if (!p || p->n < 1 || !p->theta || !p->delta) return DPT_EINVAL;
    if (p->format != DPT_DENSE && p->format != DPT_CSR) return DPT_EINVAL;
    if (p->dtype != DPT_DTYPE_F64 && p->dtype != DPT_DTYPE_F32) return DPT_EINVAL;
    if (p->mem != DPT_MEM_HOST && p->mem != DPT_MEM_DEVICE) return DPT_EINVAL;
    if (p->reserved != 0 || !std::isfinite(p->lambda)) return DPT_EINVAL;
    if (p->n > (int64_t)1 << 31) return DPT_EINVAL;
    if (p->format == DPT_CSR) {
        if (!p->indptr || !p->indices || p->nnz < 0 || p->nnz >= ((int64_t)1 << 31)) return DPT_EINVAL;
        if (full && p->mem == DPT_MEM_HOST && !csr_ok(p->indptr, p->indices, p->n, p->nnz)) return DPT_EINVAL;
    }
    if (full && p->mem == DPT_MEM_HOST && !theta_ok(p->theta, p->n)) return DPT_EINVAL;
    if (!valid_options(o)) return DPT_EINVAL;
    return DPT_OK;
}
}  // namespace

int dpt_validate(const dpt_problem *p, const dpt_options *o) { return validate_args(p, o, true); }

int dpt_init(dpt_handle *h, const dpt_problem *p, const dpt_options *o, const void *z0) {
    if (!h) return DPT_EINVAL;
    int rc = dpt_validate(p, o);
    if (rc != DPT_OK) return rc;
    if (o && (o->precision == DPT_FP8_FP32 || o->precision == DPT_BF16_X3) &&
        (p->format != DPT_DENSE || !step_large_supported(pad_order(p->n))))
        return DPT_EINVAL;  // the FP8 and split-BF16 products exist for large dense problems only
    rc = check_device();
    if (rc != DPT_OK) return rc;
    if (!device_inputs_ok(p, z0)) return DPT_EINVAL;
    if (o && o->stop_rule == DPT_STOP_ROW && p->format != DPT_DENSE) return DPT_EINVAL;  // dense rows only
    dpt_ctx *c = new (std::nothrow) dpt_ctx();
    if (!c) return DPT_ENOMEM;
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(c->stream);
        delete c;
        return code;
    };
    c->n = p->n;
    c->lambda = p->lambda;
    c->stream = (hipStream_t)p->stream;
    if (o) {
        c->opt = *o;
    } else {
        dpt_options_default(&c->opt);
    }
    c->format = p->format;
    c->in_dtype = p->dtype;
    c->mem = p->mem;
    c->ld = p->format == DPT_CSR ? sparse_pad_order(p->n) : pad_order(p->n);

    // theta: validated on the host (device inputs are read back on the handle's
    // stream), then placed on the device padded with zeros: a device-to-device
    // copy for device inputs, one upload for host inputs.  A dense device
    // problem reads theta back into a pinned block and checks it after the
    // symmetry test's wait, so both take one round trip (nothing computes with
    // theta before then; a bad theta fails the call there).
    std::vector<double> th((size_t)c->ld, 0.0);
    const double *th_deferred = nullptr;
    if (p->mem == DPT_MEM_DEVICE) {
        if (p->format == DPT_DENSE && sizeof(double) * (size_t)p->n + 512 <= kPinBlock) {
            c->pin = (unsigned char *)pin_pool().take();
            th_deferred = (const double *)c->pin_space(sizeof(double) * (size_t)p->n);
        }
        if (th_deferred) {
            if (hipMemcpyAsync((void *)th_deferred, p->theta, sizeof(double) * (size_t)p->n, hipMemcpyDeviceToHost,
                               c->stream) != hipSuccess)
                return fail(DPT_EDEVICE);
        } else {
            if (hipMemcpyAsync(th.data(), p->theta, sizeof(double) * (size_t)p->n, hipMemcpyDeviceToHost,
                               c->stream) != hipSuccess ||
                hipStreamSynchronize(c->stream) != hipSuccess)
                return fail(DPT_EDEVICE);
            if (!theta_ok(th.data(), p->n)) return fail(DPT_EINVAL);
        }
    } else {
        std::memcpy(th.data(), p->theta, sizeof(double) * (size_t)p->n);
    }
    if (dalloc(&c->theta, (size_t)c->ld) != hipSuccess || dalloc(&c->dvec, (size_t)c->ld) != hipSuccess ||
        dalloc(&c->evec, (size_t)c->ld) != hipSuccess || dalloc(&c->stats, (size_t)2 * kStatRing) != hipSuccess)
        return fail(DPT_ENOMEM);
    c->stats_host = (unsigned long long *)stat_mirror_pool().take();
    if (!c->stats_host) return fail(DPT_ENOMEM);
    // small dense host problems upload theta and Delta from a pinned block
    if (p->mem == DPT_MEM_HOST && p->format == DPT_DENSE && c->ld <= 256) c->pin = (unsigned char *)pin_pool().take();
    {
        const bool dev = p->mem == DPT_MEM_DEVICE;
        double *thp = dev ? nullptr : (double *)c->pin_space(sizeof(double) * (size_t)c->ld);
        if (thp) std::memcpy(thp, th.data(), sizeof(double) * (size_t)c->ld);
        void *zp[4] = {c->dvec, c->evec, c->stats, c->theta + c->n};
        const size_t zb[4] = {sizeof(double) * (size_t)c->ld, sizeof(double) * (size_t)c->ld,
                              sizeof(unsigned long long) * 2 * kStatRing, sizeof(double) * (size_t)(c->ld - c->n)};
        const int nz = dev && c->ld > c->n ? 4 : 3;  // the padding of a device-copied theta
        if (launch_zero_many(zp, zb, nz, c->stream) != hipSuccess ||
            hipMemcpyAsync(c->theta, dev ? p->theta : thp ? (const void *)thp : (const void *)th.data(),
                           sizeof(double) * (size_t)(dev ? c->n : c->ld),
                           dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return fail(DPT_EDEVICE);
    }

    if (p->format == DPT_CSR) {
        rc = sparse_create(&c->sp, p, c->opt.precision == DPT_FP64, c->ld, c->stream);
        if (rc == DPT_OK && !c->sp) rc = DPT_ENOMEM;
        if (rc == DPT_OK) c->phase = c->opt.precision == DPT_FP64 ? PH_FP64 : PH_FP32;
        if (rc == DPT_OK && z0) rc = sparse_warm_start(c, p, z0);
    } else {
        rc = init_dense(c, p, z0);  // device inputs: waits for the symmetry test
    }
    if (rc != DPT_OK) return fail(rc);
    if (th_deferred && !theta_ok(th_deferred, p->n)) return fail(DPT_EINVAL);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(DPT_EDEVICE);
    pin_pool().give(c->pin);  // its uploads are complete
    c->pin = nullptr;
    c->pin_used = 0;
    *h = c;
    return DPT_OK;
}

int dpt_step(dpt_handle h, int nsteps, double *last_delta) {
    if (!h || nsteps < 0) return DPT_EINVAL;
    if (last_delta) *last_delta = std::numeric_limits<double>::quiet_NaN();
    for (int i = 0; i < nsteps; ++i) {
        int rc = do_step(h);
        if (rc != DPT_OK) return rc;
    }
    if (nsteps > 0) {
        int rc = fetch_stats(h, h->k - 1, h->k);
        if (rc != DPT_OK) return rc;
        double dl, wm;
        stat_of(h, h->k - 1, &dl, &wm);
        if (last_delta) *last_delta = dl;
    } else {
        if (hipStreamSynchronize(h->stream) != hipSuccess) return DPT_EDEVICE;
    }
    return DPT_OK;
}

int dpt_solve(dpt_handle h, dpt_result *r) {
    if (!h) return DPT_EINVAL;
    Controller ctl;
    ctl.start(h->opt, h->phase, h->sp == nullptr);
    int64_t checked = h->k;  // stats already consumed
    const int64_t k_start = h->k;
    bool done = false;
    while (!done && !ctl.capped()) {
        if (small_batch_ok(h)) {
            int taken = 0;
            Controller::Action act = Controller::CONTINUE;
            int rc = small_batch(h, ctl, r, h->k - k_start, &taken, &act);
            if (rc != DPT_OK) return rc;
            checked = h->k;
            if (act == Controller::TO_FP64) {
                rc = enter_fp64(h);
                if (rc != DPT_OK) return rc;
            } else if (act == Controller::DONE) {
                done = true;
            }
            continue;
        }
        int rc = do_step(h);
        if (rc != DPT_OK) return rc;
        ctl.count_step();
        if (ctl.iters % h->opt.check_every != 0 && !ctl.capped()) continue;
        rc = fetch_stats(h, checked, h->k);
        if (rc != DPT_OK) return rc;
        for (int64_t s = checked; s < h->k; ++s) {
            double dl, wm;
            stat_of(h, s, &dl, &wm);
            const int idx = ctl.iters - (int)(h->k - s);
            if (r && r->delta_history && idx >= 0 && idx < r->history_cap) r->delta_history[idx] = dl;
        }
        checked = h->k;
        double dl, wm;
        stat_of(h, h->k - 1, &dl, &wm);
        if (h->last_ramping) {  // during the ramp only divergence ends the solve
            if (ctl.update_ramping(dl, wm) == Controller::DONE) done = true;
            continue;
        }
        if (row_phase(h) && std::isfinite(dl)) {  // per-row retirement
            int64_t left = 0;
            rc = retire_rows(h, &left);
            if (rc != DPT_OK) return rc;
            if (left == 0) {
                ctl.finish_ok(dl);
                done = true;
                continue;
            }
        }
        switch (ctl.update(dl, wm)) {
            case Controller::TO_FP32:
                rc = enter_fp32(h);
                if (rc != DPT_OK) return rc;
                break;
            case Controller::TO_FP64:
                rc = enter_fp64(h);
                if (rc != DPT_OK) return rc;
                break;
            case Controller::DONE:
                done = true;
                break;
            default:
                break;
        }
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return DPT_EDEVICE;
    ctl.fill(r);
    return ctl.status;
}

// After a per-row solve, dpt_step keeps applying F to the rows still running
// only; once every row is frozen a step changes nothing (delta 0).
int dpt_row_status(dpt_handle h, int32_t *retired_at, int64_t *rows_multiplied) {
    if (!h) return DPT_EINVAL;
    if (retired_at) {
        for (int64_t i = 0; i < h->n; ++i)
            retired_at[i] = h->retired_at.empty() ? 0 : h->retired_at[(size_t)i];
    }
    if (rows_multiplied) *rows_multiplied = h->rows_multiplied;
    return DPT_OK;
}

int dpt_eigenvalues(dpt_handle h, double *E, int mem) {
    if (!h || !E || (mem != DPT_MEM_HOST && mem != DPT_MEM_DEVICE)) return DPT_EINVAL;
    if (mem == DPT_MEM_DEVICE && !is_device_ptr(E)) return DPT_EINVAL;
    int rc = compute_eigenvalues(h);
    if (rc != DPT_OK) return rc;
    const size_t bytes = sizeof(double) * (size_t)h->n;
    // host output: through a pinned block when it fits (a pageable destination
    // would make the runtime stage the copy)
    void *bounce = mem == DPT_MEM_HOST && bytes <= kPinBlock ? pin_pool().take() : nullptr;
    hipError_t e = hipMemcpyAsync(bounce ? bounce : (void *)E, h->evec, bytes,
                                  mem == DPT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess && bounce) std::memcpy(E, bounce, bytes);
    if (e == hipSuccess) pin_pool().give(bounce);  // drained; after a device error the block is not reused
    DPT_TRY(e);
    return DPT_OK;
}

int dpt_eigenvectors(dpt_handle h, void *Z, int dtype, int mem) {
    if (!h || !Z || (mem != DPT_MEM_HOST && mem != DPT_MEM_DEVICE)) return DPT_EINVAL;
    if (dtype != DPT_DTYPE_F32 && dtype != DPT_DTYPE_F64) return DPT_EINVAL;
    if (mem == DPT_MEM_DEVICE && !is_device_ptr(Z)) return DPT_EINVAL;
    if (!h->sp) {
        int rc = clean_identity(h);
        if (rc != DPT_OK) return rc;
    }
    const size_t bytes = (size_t)(h->n * h->n) * (dtype == DPT_DTYPE_F64 ? 8 : 4);
    void *dst = Z;
    void *tmp = nullptr;
    if (mem == DPT_MEM_HOST) {
        DPT_TRY(hipMalloc(&tmp, bytes));
        dst = tmp;
    }
    hipError_t e;
    if (h->sp)
        e = sparse_export(h->sp, h->n, dst, dtype == DPT_DTYPE_F64, h->stream);
    else if (h->phase == PH_FP64)
        e = launch_export_f64(h->W64[h->cur], h->n, h->ld, dst, dtype == DPT_DTYPE_F64, h->stream);
    else
        e = launch_export_f32(h->W32[h->cur], h->n, h->ld, dst, dtype == DPT_DTYPE_F64, h->stream);
    if (e == hipSuccess && tmp) e = hipMemcpyAsync(Z, tmp, bytes, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (tmp) (void)hipFree(tmp);
    return map_err(e);
}

int dpt_residuals(dpt_handle h, int64_t nrows, const int64_t *rows, double *res) {
    if (!h || nrows < 1 || !rows || !res) return DPT_EINVAL;
    for (int64_t i = 0; i < nrows; ++i)
        if (rows[i] < 0 || rows[i] >= h->n) return DPT_EINVAL;
    if (h->sp) {
        int rc = compute_eigenvalues(h);
        if (rc != DPT_OK) return rc;
        return map_err(sparse_residuals(h->sp, h->lambda, h->theta, h->evec, rows, nrows, res, h->stream));
    }
    int rc = compute_eigenvalues(h);
    if (rc != DPT_OK) return rc;
    const int nch = residual_chunks(h->ld);
    int64_t *drows = nullptr;
    double *part = nullptr;
    hipError_t e = dalloc(&drows, (size_t)nrows);
    if (e == hipSuccess) e = dalloc(&part, (size_t)(nrows * nch));
    if (e == hipSuccess) e = hipMemcpyAsync(drows, rows, sizeof(int64_t) * nrows, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        const StepArgs a = step_args(h, nullptr);
        const void *D = h->d64 ? (const void *)h->d64 : (const void *)h->d32;
        const int d64 = h->d64 ? 1 : 0;
        e = h->phase == PH_FP64 ? launch_residual_f64(h->W64[h->cur], D, d64, a, drows, nrows, h->evec, part, h->stream)
                                : launch_residual_f32(h->W32[h->cur], D, d64, a, drows, nrows, h->evec, part, h->stream);
    }
    std::vector<double> hp((size_t)(nrows * nch));
    if (e == hipSuccess)
        e = hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    dfree(drows);
    dfree(part);
    if (e != hipSuccess) return map_err(e);
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int c = 0; c < nch; ++c) s += hp[(size_t)(i * nch + c)];
        res[i] = std::sqrt(s);
    }
    return DPT_OK;
}

int dpt_dominant(const dpt_problem *p, const dpt_options *o, int64_t index, double *eigval, void *eigvec,
                 dpt_result *r) {
    int rc = validate_args(p, o, false);  // the CSR content is checked where it is staged
    if (rc != DPT_OK) return rc;
    if (!eigval || !eigvec || index >= p->n) return DPT_EINVAL;
    rc = check_device();
    if (rc != DPT_OK) return rc;
    if (!device_inputs_ok(p, nullptr) || (p->mem == DPT_MEM_DEVICE && !is_device_ptr(eigvec))) return DPT_EINVAL;
    dpt_options opt;
    if (o) {
        opt = *o;
    } else {
        dpt_options_default(&opt);
    }
    // the single-line map divides only by theta_index - theta_m: theta_index must
    // be simple, other values may coincide (Sec. II.H)
    if (p->mem == DPT_MEM_DEVICE) return dominant_solve_device(p, &opt, index, eigval, eigvec, r);
    const double *th = p->theta;
    for (int64_t m = 0; m < p->n; ++m)
        if (!std::isfinite(th[m])) return DPT_EINVAL;
    if (index < 0) index = (int64_t)(std::max_element(th, th + p->n) - th);
    for (int64_t m = 0; m < p->n; ++m)
        if (m != index && th[m] == th[index]) return DPT_EINVAL;
    return dominant_solve(p, &opt, th, th[index], index, eigval, eigvec, r);
}

int dpt_dominant_noalloc(const dpt_problem *p, const dpt_options *o, int64_t index, double *eigval, void *eigvec,
                         dpt_result *r) {
    int rc = validate_args(p, o, false);  // theta and the CSR structure are checked on the device
    if (rc != DPT_OK) return rc;
    if (!eigval || !eigvec || index >= p->n || p->mem != DPT_MEM_DEVICE) return DPT_EINVAL;
    rc = check_device();
    if (rc != DPT_OK) return rc;
    if (!device_inputs_ok(p, nullptr) || !is_device_ptr(eigvec)) return DPT_EINVAL;
    dpt_options opt;
    if (o) {
        opt = *o;
    } else {
        dpt_options_default(&opt);
    }
    return dominant_solve_noalloc(p, &opt, index, eigval, eigvec, r);
}

int dpt_profile_enable(dpt_handle h, int on) {
    if (!h) return DPT_EINVAL;
    h->prof.reset();
    h->prof.on = on != 0;
    return DPT_OK;
}

int dpt_profile_read(dpt_handle h, dpt_profile *out) {
    if (!h || !out) return DPT_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return DPT_EDEVICE;
    h->prof.collect();
    for (int i = 0; i < DPT_PROF_KINDS; ++i) {
        out->ms[i] = h->prof.ms[i];
        out->launches[i] = h->prof.launches[i];
    }
    return DPT_OK;
}

void dpt_destroy(dpt_handle h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

const char *dpt_status_str(int code) {
    switch (code) {
        case DPT_OK: return "DPT_OK: converged";
        case DPT_NOT_CONVERGED: return "DPT_NOT_CONVERGED: iteration cap reached";
        case DPT_STALLED: return "DPT_STALLED: stopped improving above the tolerance";
        case DPT_DIVERGED: return "DPT_DIVERGED: non-finite iterate or |Z - I| above the blow-up bound";
        case DPT_EAGAIN: return "DPT_EAGAIN: result not ready";
        case DPT_EINVAL: return "DPT_EINVAL: invalid argument";
        case DPT_ENOMEM: return "DPT_ENOMEM: out of memory";
        case DPT_EDEVICE: return "DPT_EDEVICE: HIP runtime error or no gfx950 device";
        case DPT_ESTATE: return "DPT_ESTATE: call not valid in this state";
        default: return "unknown status";
    }
}

}  // extern "C"
