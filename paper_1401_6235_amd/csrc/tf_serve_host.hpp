// Host side of the serving loop: job validation and sizing, the pool
// sub-allocator, admission (FIFO, by HBM bytes and free slots), publication
// into the descriptor ring and completion handling.  Inputs that a job
// generates from its seed are written by the persistent kernel itself, in
// the job's first phase: nothing else runs on the device beside it, so its
// progress never waits for a second kernel to be scheduled.  Pure C++: the device is
// reached only through the DeviceOps interface, implemented over HIP by the
// library and by a CPU stand-in in the host-logic tests.
#pragma once

#include <stdint.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "tf.h"
#include "tf_serve_proto.h"

namespace tfs {

// ---------------------------------------------------------------------------
// Pool: first-fit sub-allocation of [0, capacity) in 256-byte units, with
// coalescing of neighbouring free ranges.
// ---------------------------------------------------------------------------
class Pool {
  public:
    explicit Pool(uint64_t capacity) : cap_(capacity & ~(uint64_t)255) {
        if (cap_) free_[0] = cap_;
        free_bytes_ = cap_;
    }
    static uint64_t round(uint64_t b) { return (b + 255) & ~(uint64_t)255; }
    bool alloc(uint64_t bytes, uint64_t *offset) {
        bytes = round(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *offset = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                free_bytes_ -= bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t offset, uint64_t bytes) {
        bytes = round(bytes ? bytes : 1);
        auto next = free_.lower_bound(offset);
        uint64_t start = offset, size = bytes;
        if (next != free_.end() && offset + bytes == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == offset) {
                start = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = size;
        free_bytes_ += bytes;
    }
    uint64_t capacity() const { return cap_; }
    uint64_t free_bytes() const { return free_bytes_; }
    size_t fragments() const { return free_.size(); }

  private:
    uint64_t cap_;
    uint64_t free_bytes_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> size
};

// ---------------------------------------------------------------------------
// Job plan: validation and the layout of the job's pool allocation.
// ---------------------------------------------------------------------------
struct Plan {
    uint64_t bytes = 0;  // pool bytes (inputs it generates, outputs, partials)
    uint64_t off_x0 = 0, off_x1 = 0, off_y0 = 0, off_y1 = 0, off_z0 = 0, off_z1 = 0, off_part = 0;
    bool gen_x1 = false, gen_y0 = false, gen_y1 = false;
    int nclaims = 0, tiles_per_claim = 0, padded = 0;
    int ngen = 0;  // units of TFS_CLAIM elements generating the inputs
};

inline int64_t pow2_ceil(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

inline int plan_job(const tfs_job &j, Plan *p) {
    *p = Plan();
    if (j.op < TFS_OP_SUM || j.op > TFS_OP_HORNER) return TF_EINVAL;
    if (j.dtype != TF_F32 && j.dtype != TF_F64) return TF_EINVAL;
    if (j.kind < TFS_KIND_RANDOM || j.kind > TFS_KIND_PROVIDED) return TF_EINVAL;
    if (j.n < 1 || j.n > TFS_MAX_N) return TF_EINVAL;
    if (j.op == TFS_OP_HORNER && (j.degree < 0 || j.degree > TF_MAX_DEGREE)) return TF_EINVAL;
    if (j.threshold < 0) return TF_EINVAL;
    const uint64_t s = j.dtype == TF_F64 ? 8 : 4;
    const uint64_t arr = Pool::round((uint64_t)j.n * s);
    const bool reduce = j.op == TFS_OP_SUM || j.op == TFS_OP_DOT;
    if (j.kind == TFS_KIND_PROVIDED) {
        if (!j.x0) return TF_EINVAL;
        if (j.op == TFS_OP_DOT && !j.y0) return TF_EINVAL;
        if (j.op == TFS_OP_AXPY && !j.y0) return TF_EINVAL;
    }
    if (j.kind == TFS_KIND_ILLCOND && reduce) return TF_EINVAL;  // reductions take provided instances
    uint64_t off = 0;
    auto take = [&](uint64_t *o, uint64_t b) {
        *o = off;
        off += b;
    };
    if (j.kind != TFS_KIND_PROVIDED) {
        // inputs generated on the device into the job's allocation
        take(&p->off_x0, arr);
        switch (j.op) {
        case TFS_OP_SUM: p->gen_x1 = true; break;                          // twofold leaves
        case TFS_OP_DOT: p->gen_y0 = true; break;                          // plain x, y
        case TFS_OP_AXPY: p->gen_x1 = p->gen_y0 = p->gen_y1 = true; break; // twofold x, y
        default: p->gen_x1 = true; break;                                  // twofold x
        }
        if (p->gen_x1) take(&p->off_x1, arr);
        if (p->gen_y0) take(&p->off_y0, arr);
        if (p->gen_y1) take(&p->off_y1, arr);
        p->ngen = (int)((j.n + TFS_CLAIM - 1) / TFS_CLAIM);
    }
    if (reduce) {
        const int64_t tiles = (j.n + 255) / 256;
        const int64_t P = pow2_ceil(tiles);
        const int64_t tpc = P < TFS_CLAIM / 256 ? P : TFS_CLAIM / 256;
        p->tiles_per_claim = (int)tpc;
        p->nclaims = (int)((tiles + tpc - 1) / tpc);
        p->padded = (int)(P / tpc);
        take(&p->off_part, Pool::round((uint64_t)p->nclaims * 2 * s));
    } else {
        p->nclaims = (int)((j.n + TFS_CLAIM - 1) / TFS_CLAIM);
        take(&p->off_z0, arr);
        take(&p->off_z1, arr);
        take(&p->off_part, Pool::round((uint64_t)p->nclaims * sizeof(tfs_vsum)));
    }
    if (p->nclaims > TFS_MAX_CLAIMS) return TF_EINVAL;
    p->bytes = off;
    return TF_OK;
}

// ---------------------------------------------------------------------------
// Device interface
// ---------------------------------------------------------------------------
class DeviceOps {
  public:
    virtual ~DeviceOps() {}
    virtual uint64_t pool_base() = 0;          // device address of the pool
    virtual tfs_shared *shared() = 0;          // host-coherent region
    virtual int start() = 0;                   // start the persistent worker
    virtual bool running() = 0;                // worker still alive
    virtual int stop() = 0;                    // ask the worker to drain and wait for it
};

inline double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// Server: one thread runs admission, publication and completion.
// ---------------------------------------------------------------------------
class Server {
  public:
    Server(DeviceOps *dev, uint64_t budget, int max_slots)
        : dev_(dev), pool_(budget), max_slots_(max_slots < 1 ? 1 : max_slots > TFS_MAX_SLOTS ? TFS_MAX_SLOTS : max_slots) {
        for (int s = 0; s < TFS_MAX_SLOTS; ++s) slots_[s].busy = false;
    }
    ~Server() { shutdown(); }

    int start() {
        int st = dev_->start();
        if (st != TF_OK) return st;
        running_ = true;
        thread_ = std::thread([this] { loop(); });
        return TF_OK;
    }

    void shutdown() {
        if (running_.exchange(false)) {
            {
                std::lock_guard<std::mutex> g(in_mu_);  // a parked server thread sees running_ false
            }
            in_cv_.notify_one();
            if (thread_.joinable()) thread_.join();
            dev_->stop();
        }
    }

    // Client side: queue a job (only the inbox lock is taken, so a client
    // never waits behind the server thread's device queries).
    int submit(const tfs_job &j, double t_arrive, uint64_t *id) {
        Plan p;
        const int st = plan_job(j, &p);
        if (st != TF_OK) return st;
        if (p.bytes > pool_.capacity()) return TF_ENOMEM;  // can never be admitted
        Pending q;
        q.job = j;
        q.plan = p;
        q.t_submit = now_s();
        q.t_arrive = t_arrive > 0 ? t_arrive : q.t_submit;
        {
            std::lock_guard<std::mutex> g(in_mu_);
            q.id = ++next_id_;
            inbox_.push_back(q);
            if (id) *id = q.id;
        }
        in_cv_.notify_one();  // wakes the server thread if it is parked
        return TF_OK;
    }

    int poll(tfs_result *out, int max) {
        std::lock_guard<std::mutex> g(out_mu_);
        int k = 0;
        while (k < max && !completed_.empty()) {
            out[k++] = completed_.front();
            completed_.pop_front();
        }
        return k;
    }

    void stats(tfs_stats *s) {
        memset(s, 0, sizeof *s);
        {
            std::lock_guard<std::mutex> g(in_mu_);
            s->pending = (int64_t)inbox_.size();
        }
        s->pending += pending_count_.load();
        s->in_flight = in_flight_.load();
        s->completed = (int64_t)n_completed_.load();
        s->budget_bytes = pool_.capacity();
        s->resident_bytes = resident_.load();
        s->peak_resident_bytes = peak_resident_.load();
        s->admission_waits = admission_waits_.load();
        s->kernel_alive = alive_.load() ? 1 : 0;
    }

  private:
    struct Pending {
        tfs_job job;
        Plan plan;
        uint64_t id;
        double t_arrive, t_submit;
    };
    struct Slot {
        bool busy;
        Pending job;
        tfs_desc desc;
        uint64_t off;
        double t_admit, t_publish;
    };

    void fill_desc(Slot &s, uint64_t gen, int slot) {
        const tfs_job &j = s.job.job;
        const Plan &p = s.job.plan;
        tfs_desc &d = s.desc;
        memset(&d, 0, sizeof d);
        const uint64_t base = dev_->pool_base() + s.off;
        d.gen = gen;
        d.slot = slot;
        d.op = j.op;
        d.dtype = j.dtype;
        d.kind = j.kind;
        d.n = j.n;
        d.seed = j.seed;
        d.degree = j.op == TFS_OP_HORNER ? j.degree : 0;
        d.nclaims = p.nclaims;
        d.tiles_per_claim = p.tiles_per_claim;
        d.padded = p.padded;
        d.ngen = p.ngen;
        const bool f32 = j.dtype == TF_F32;
        d.a0 = f32 ? (double)(float)j.a[0] : j.a[0];
        d.a1 = f32 ? (double)(float)j.a[1] : j.a[1];
        d.thr = j.threshold > 0 ? j.threshold : 1.0 / 1048576.0;
        for (int k = 0; k <= TF_MAX_DEGREE; ++k) d.c[k] = f32 ? (double)(float)j.c[k] : j.c[k];
        if (j.kind == TFS_KIND_PROVIDED) {
            d.x0 = (uint64_t)j.x0;
            d.x1 = (uint64_t)j.x1;
            d.y0 = (uint64_t)j.y0;
            d.y1 = (uint64_t)j.y1;
        } else {
            d.x0 = base + p.off_x0;
            d.x1 = p.gen_x1 ? base + p.off_x1 : 0;
            d.y0 = p.gen_y0 ? base + p.off_y0 : 0;
            d.y1 = p.gen_y1 ? base + p.off_y1 : 0;
        }
        if (j.op == TFS_OP_AXPY || j.op == TFS_OP_HORNER) {
            d.z0 = base + p.off_z0;
            d.z1 = base + p.off_z1;
        }
        d.part = base + p.off_part;
    }

    // Admit FIFO jobs while a slot and pool space are free (server thread).
    bool admit() {
        bool progress = false;
        while (!pending_.empty()) {
            int slot = -1;
            for (int s = 0; s < max_slots_; ++s)
                if (!slots_[s].busy) {
                    slot = s;
                    break;
                }
            if (slot < 0) break;
            uint64_t off;
            if (!pool_.alloc(pending_.front().plan.bytes, &off)) {
                if (!head_waited_) ++admission_waits_;
                head_waited_ = true;
                break;
            }
            head_waited_ = false;
            Slot &s = slots_[slot];
            s.busy = true;
            s.job = pending_.front();
            pending_.pop_front();
            s.off = off;
            s.t_admit = now_s();
            if ((uint32_t)++gen_ == 0) ++gen_;  // the slot word keeps 32 bits; 0 means empty
            fill_desc(s, gen_, slot);
            const uint64_t resident = pool_.capacity() - pool_.free_bytes();
            resident_ = resident;
            if (resident > peak_resident_) peak_resident_ = resident;
            ++in_flight_;
            publish(s);
            progress = true;
        }
        return progress;
    }

    void publish(Slot &s) {
        tfs_shared *sh = dev_->shared();
        // drained after an idle period (the kernel says so in shared memory;
        // the stream query confirms it): relaunch before publishing
        if (__atomic_load_n(&sh->kernel_state, __ATOMIC_ACQUIRE) >= 2 && !dev_->running()) dev_->start();
        const uint64_t seq = published_;
        while (seq - __atomic_load_n(&sh->consumed, __ATOMIC_ACQUIRE) >= TFS_RING)
            std::this_thread::yield();  // ring full: wait for the dispatcher
        tfs_desc *e = &sh->ring[seq % TFS_RING];
        memcpy(e, &s.desc, sizeof *e);
        __atomic_store_n(&sh->pub_count, seq + 1, __ATOMIC_RELEASE);
        published_ = seq + 1;
        s.t_publish = now_s();
    }

    bool progress_slots() {
        bool progress = false;
        tfs_shared *sh = dev_->shared();
        for (int i = 0; i < max_slots_; ++i) {
            Slot &s = slots_[i];
            if (!s.busy) continue;
            const uint64_t g = __atomic_load_n(&sh->done[i].gen, __ATOMIC_ACQUIRE);
            if (g == s.desc.gen) {
                pool_.release(s.off, s.job.plan.bytes);
                resident_ = pool_.capacity() - pool_.free_bytes();
                s.busy = false;
                --in_flight_;
                complete(s, sh->done[i]);
                progress = true;
            }
        }
        return progress;
    }

    void complete(Slot &s, const tfs_done &d) {
        tfs_result r;
        memset(&r, 0, sizeof r);
        r.id = s.job.id;
        r.status = d.status;
        r.op = s.job.job.op;
        r.dtype = s.job.job.dtype;
        r.kind = s.job.job.kind;
        r.n = s.job.job.n;
        r.flag = d.flag;
        r.z0 = d.z0;
        r.z1 = d.z1;
        r.max_abs_z0 = d.max0;
        r.max_abs_z1 = d.max1;
        r.n_flagged = d.n_flagged;
        r.nonfinite = d.nonfinite;
        r.hash_z0 = d.hash0;
        r.hash_z1 = d.hash1;
        r.t_arrive = s.job.t_arrive;
        r.t_submit = s.job.t_submit;
        r.t_admit = s.t_admit;
        r.t_publish = s.t_publish;
        r.t_done = now_s();
        auto us = [this](uint64_t a, uint64_t b) { return a && b > a ? (double)(b - a) * 1e6 / tick_hz_ : 0.0; };
        const uint64_t compute_from = d.t_ready ? d.t_ready : d.t_start;
        r.queue_us = us(d.t_open, d.t_start);
        r.gen_us = d.t_ready ? us(d.t_start, d.t_ready) : 0.0;
        r.device_us = us(compute_from, d.t_end);
        {
            std::lock_guard<std::mutex> g(out_mu_);
            completed_.push_back(r);
        }
        ++n_completed_;
    }

    // Server thread: owns pending_, slots_ and pool_ without locks.  It polls
    // without sleeping while jobs are queued or in flight and for a grace
    // period after the last progress (a timed sleep costs tens of
    // microseconds per stage, more than a small job's device time), then
    // parks on in_cv_ until a submit, waking once a millisecond for the
    // liveness check.
    void loop() {
        double next_check = 0.0, last_progress = now_s();
        while (running_) {
            {
                std::lock_guard<std::mutex> g(in_mu_);
                while (!inbox_.empty()) {
                    pending_.push_back(inbox_.front());
                    inbox_.pop_front();
                }
            }
            bool progress = admit();
            progress |= progress_slots();
            progress |= admit();
            pending_count_ = (int64_t)pending_.size();
            const double t = now_s();
            if (t >= next_check) {  // liveness of the persistent worker, once a millisecond
                next_check = t + 1e-3;
                const bool alive = dev_->running();
                alive_ = alive;
                // Drained after an idle period with jobs published (one can
                // land just as the kernel exits): relaunch.  With nothing in
                // flight it stays down until the next publish relaunches it,
                // so other work of the process can use its hardware queue.
                if (!alive && running_ && in_flight_.load() > 0) dev_->start();
            }
            if (progress) {
                last_progress = t;
            } else if (in_flight_.load() > 0 || !pending_.empty() || t - last_progress < kSpinGrace) {
                std::this_thread::yield();
            } else {
                std::unique_lock<std::mutex> g(in_mu_);
                // system_clock: a timed wait on it is pthread_cond_timedwait,
                // which thread sanitizers know (the steady_clock form is not)
                in_cv_.wait_until(g, std::chrono::system_clock::now() + std::chrono::milliseconds(1),
                                  [this] { return !inbox_.empty() || !running_; });
            }
        }
    }
    static constexpr double kSpinGrace = 2e-3;  // seconds of polling after the last progress

    DeviceOps *dev_;
    Pool pool_;
    int max_slots_;
    Slot slots_[TFS_MAX_SLOTS];
    std::deque<Pending> inbox_;      // submitted, not yet seen by the server thread (in_mu_)
    std::deque<Pending> pending_;    // queued for admission (server thread only)
    std::deque<tfs_result> completed_;  // out_mu_
    std::mutex in_mu_, out_mu_;
    std::condition_variable in_cv_;  // inbox non-empty or shutdown (with in_mu_)
    std::thread thread_;
    std::atomic<bool> running_{false}, alive_{true};
    uint64_t next_id_ = 0, gen_ = 0, published_ = 0;
    std::atomic<uint64_t> n_completed_{0}, peak_resident_{0}, admission_waits_{0}, resident_{0};
    std::atomic<int64_t> pending_count_{0}, in_flight_{0};
    bool head_waited_ = false;
    double tick_hz_ = 100e6;

  public:
    void set_tick_hz(double hz) { tick_hz_ = hz; }
};

}  // namespace tfs
