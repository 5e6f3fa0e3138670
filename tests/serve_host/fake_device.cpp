// Host logic of the serving loop against a CPU stand-in for the device.
//
// The stand-in implements the same DeviceOps interface as the HIP backend:
// a thread plays the persistent kernel's dispatcher and workers (it reads
// the descriptor ring with acquire loads, "processes" each job after a short
// delay and writes the completion record, generation last with release).
// Results are not arithmetic
// (z0 = n, z1 = gen): the scenarios check admission, slot recycling,
// budget waits, ordering and error handling.  Prints one JSON line per
// scenario.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>

#include "tf_serve_host.hpp"

class FakeDevice : public tfs::DeviceOps {
  public:
    explicit FakeDevice(uint64_t process_us, int idle_exit_ms = 0)
        : process_us_(process_us), idle_exit_ms_(idle_exit_ms) {
        memset(&sh_, 0, sizeof sh_);
    }
    ~FakeDevice() override { stop(); }
    uint64_t pool_base() override { return 1ull << 40; }
    tfs_shared *shared() override { return &sh_; }
    int start() override {
        if (th_.joinable()) th_.join();
        alive_ = true;
        starts_++;
        __atomic_store_n(&sh_.stop, 0, __ATOMIC_RELEASE);
        __atomic_store_n(&sh_.kernel_state, 1, __ATOMIC_RELEASE);  // as the HIP backend: launched
        th_ = std::thread([this] { run(); });
        return TF_OK;
    }
    bool running() override { return alive_; }
    int stop() override {
        __atomic_store_n(&sh_.stop, 1, __ATOMIC_RELEASE);
        if (th_.joinable()) th_.join();
        return TF_OK;
    }
    int starts() const { return starts_; }
    std::set<int> slots_seen;
    uint64_t max_in_flight = 0;

  private:
    struct Job {
        tfs_desc d;
        double ready;
    };
    void run() {
        uint64_t consumed = __atomic_load_n(&sh_.consumed, __ATOMIC_ACQUIRE);
        std::vector<Job> jobs;
        double last = tfs::now_s();
        uint64_t how = 2;
        while (true) {
            const uint64_t pub = __atomic_load_n(&sh_.pub_count, __ATOMIC_ACQUIRE);
            while (consumed < pub) {
                Job j;
                memcpy(&j.d, &sh_.ring[consumed % TFS_RING], sizeof j.d);
                j.ready = tfs::now_s() + process_us_ * 1e-6 * (1 + j.d.nclaims % 3);
                jobs.push_back(j);
                slots_seen.insert(j.d.slot);
                ++consumed;
                __atomic_store_n(&sh_.consumed, consumed, __ATOMIC_RELEASE);
                last = tfs::now_s();
            }
            if (jobs.size() > max_in_flight) max_in_flight = jobs.size();
            for (size_t k = 0; k < jobs.size();) {
                if (tfs::now_s() >= jobs[k].ready) {
                    tfs_done *r = &sh_.done[jobs[k].d.slot];
                    r->status = TF_OK;
                    r->z0 = (double)jobs[k].d.n;
                    r->z1 = (double)jobs[k].d.gen;
                    r->flag = jobs[k].d.kind == TFS_KIND_ILLCOND;
                    __atomic_store_n(&r->gen, jobs[k].d.gen, __ATOMIC_RELEASE);
                    jobs.erase(jobs.begin() + k);
                    last = tfs::now_s();
                } else {
                    ++k;
                }
            }
            if (__atomic_load_n(&sh_.stop, __ATOMIC_ACQUIRE) && jobs.empty()) {
                how = 2;
                break;
            }
            if (idle_exit_ms_ && jobs.empty() && tfs::now_s() - last > idle_exit_ms_ * 1e-3) {
                how = 3;
                break;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(5));
        }
        __atomic_store_n(&sh_.kernel_state, how, __ATOMIC_RELEASE);  // 2 stopped, 3 idle exit
        alive_ = false;
    }
    tfs_shared sh_;
    std::thread th_;
    std::atomic<bool> alive_{false};
    uint64_t process_us_;
    int idle_exit_ms_;
    int starts_ = 0;
};

static tfs_job make_job(int op, int dtype, int64_t n, int kind = TFS_KIND_RANDOM) {
    tfs_job j;
    memset(&j, 0, sizeof j);
    j.op = op;
    j.dtype = dtype;
    j.n = n;
    j.kind = kind;
    j.degree = 8;
    j.a[0] = 0.7;
    j.a[1] = 1e-17;
    return j;
}

// Submit `count` jobs of random op / dtype / length, wait for all of them.
static int run_stream(uint64_t budget, int slots, int count, uint64_t process_us, int idle_exit_ms,
                      const char *name) {
    FakeDevice dev(process_us, idle_exit_ms);
    tfs::Server srv(&dev, budget, slots);
    if (srv.start() != TF_OK) return 1;
    std::mt19937_64 g(7);
    std::map<uint64_t, tfs_job> sent;
    std::vector<uint64_t> order;
    int rejected = 0, wrong_reject = 0;
    for (int k = 0; k < count; ++k) {
        const int op = (int)(g() % 4), dtype = g() % 2 ? TF_F64 : TF_F32;
        const int64_t n = (int64_t)1 << (8 + g() % 15);
        tfs_job j = make_job(op, dtype, n, (op >= 2 && g() % 10 == 0) ? TFS_KIND_ILLCOND : TFS_KIND_RANDOM);
        uint64_t id;
        const int st = srv.submit(j, 0, &id);
        if (st == TF_ENOMEM) {  // larger than the whole budget: rejected at once
            tfs::Plan p;
            tfs::plan_job(j, &p);
            if (p.bytes <= budget) ++wrong_reject;
            ++rejected;
            continue;
        }
        if (st != TF_OK) return 2;
        sent[id] = j;
        order.push_back(id);
        if (idle_exit_ms && k == count / 2) std::this_thread::sleep_for(std::chrono::milliseconds(10 * idle_exit_ms));
    }
    std::vector<tfs_result> got;
    const double t0 = tfs::now_s();
    while ((int)got.size() < count - rejected && tfs::now_s() - t0 < 60) {
        tfs_result r[64];
        const int k = srv.poll(r, 64);
        for (int i = 0; i < k; ++i) got.push_back(r[i]);
        if (!k) std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    tfs_stats st;
    srv.stats(&st);
    srv.shutdown();
    // checks
    std::set<uint64_t> ids;
    int bad = 0, flagged_ok = 1, order_ok = 1;
    double prev_admit = 0;
    std::map<uint64_t, double> admit;
    for (auto &r : got) {
        ids.insert(r.id);
        const tfs_job &j = sent[r.id];
        if (r.z0 != (double)j.n || r.op != j.op || r.dtype != j.dtype || r.status != TF_OK) ++bad;
        if (r.flag != (j.kind == TFS_KIND_ILLCOND)) flagged_ok = 0;
        if (!(r.t_arrive <= r.t_admit && r.t_admit <= r.t_publish && r.t_publish <= r.t_done)) ++bad;
        admit[r.id] = r.t_admit;
    }
    for (uint64_t id : order) {  // FIFO admission: admit times follow submission order
        if (admit[id] < prev_admit) order_ok = 0;
        prev_admit = admit[id];
    }
    printf("{\"scenario\": \"%s\", \"rejected\": %d, \"wrong_reject\": %d, \"submitted\": %d, \"completed\": %zu, \"unique\": %zu, \"bad\": %d, "
           "\"flags_ok\": %d, \"fifo\": %d, \"peak_resident\": %llu, \"budget\": %llu, \"waits\": %llu, "
           "\"max_in_flight\": %llu, \"slots_used\": %zu, \"starts\": %d}\n",
           name, rejected, wrong_reject, count - rejected, got.size(), ids.size(), bad, flagged_ok, order_ok,
           (unsigned long long)st.peak_resident_bytes, (unsigned long long)st.budget_bytes,
           (unsigned long long)st.admission_waits, (unsigned long long)dev.max_in_flight, dev.slots_seen.size(),
           dev.starts());
    return 0;
}

static int validation() {
    FakeDevice dev(10);
    tfs::Server srv(&dev, 1 << 20, 4);
    struct Case {
        const char *what;
        tfs_job j;
        int want;
    };
    std::vector<Case> cases;
    tfs_job j;
    j = make_job(7, TF_F64, 100); cases.push_back({"bad op", j, TF_EINVAL});
    j = make_job(TFS_OP_SUM, 3, 100); cases.push_back({"bad dtype", j, TF_EINVAL});
    j = make_job(TFS_OP_SUM, TF_F64, 0); cases.push_back({"n = 0", j, TF_EINVAL});
    j = make_job(TFS_OP_SUM, TF_F64, TFS_MAX_N + 1); cases.push_back({"n too large", j, TF_EINVAL});
    j = make_job(TFS_OP_HORNER, TF_F64, 100); j.degree = 33; cases.push_back({"degree", j, TF_EINVAL});
    j = make_job(TFS_OP_DOT, TF_F64, 100, TFS_KIND_PROVIDED); cases.push_back({"provided, no inputs", j, TF_EINVAL});
    j = make_job(TFS_OP_SUM, TF_F64, 100, TFS_KIND_ILLCOND); cases.push_back({"illcond reduction", j, TF_EINVAL});
    j = make_job(TFS_OP_SUM, TF_F64, 100, 9); cases.push_back({"bad kind", j, TF_EINVAL});
    j = make_job(TFS_OP_AXPY, TF_F64, 1 << 20); cases.push_back({"over budget", j, TF_ENOMEM});
    j = make_job(TFS_OP_SUM, TF_F64, 100); j.threshold = -1; cases.push_back({"threshold", j, TF_EINVAL});
    j = make_job(TFS_OP_SUM, TF_F64, 100); cases.push_back({"valid", j, TF_OK});
    int fails = 0;
    for (auto &c : cases) {
        uint64_t id;
        const int st = srv.submit(c.j, 0, &id);
        if (st != c.want) {
            printf("# validation %s: got %d want %d\n", c.what, st, c.want);
            ++fails;
        }
    }
    printf("{\"scenario\": \"validation\", \"cases\": %zu, \"fails\": %d}\n", cases.size(), fails);
    return 0;
}

static int pool() {
    std::mt19937_64 g(3);
    const uint64_t cap = 1 << 24;
    tfs::Pool p(cap);
    std::map<uint64_t, uint64_t> live;
    int overlap = 0, accounting = 0;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || g() % 3) {
            const uint64_t b = 1 + g() % (1 << 16);
            uint64_t off;
            if (p.alloc(b, &off)) {
                auto nx = live.lower_bound(off);
                if (nx != live.end() && nx->first < off + tfs::Pool::round(b)) ++overlap;
                if (nx != live.begin()) {
                    auto pv = std::prev(nx);
                    if (pv->first + tfs::Pool::round(pv->second) > off) ++overlap;
                }
                if (off + tfs::Pool::round(b) > cap || off % 256) ++overlap;
                live[off] = b;
            }
        } else {
            auto it2 = live.begin();
            std::advance(it2, g() % live.size());
            p.release(it2->first, it2->second);
            live.erase(it2);
        }
        uint64_t used = 0;
        for (auto &kv : live) used += tfs::Pool::round(kv.second);
        if (used + p.free_bytes() != cap) ++accounting;
    }
    for (auto &kv : live) p.release(kv.first, kv.second);
    printf("{\"scenario\": \"pool\", \"overlap\": %d, \"accounting\": %d, \"fragments_after_free\": %zu, "
           "\"free\": %llu, \"cap\": %llu}\n",
           overlap, accounting, p.fragments(), (unsigned long long)p.free_bytes(), (unsigned long long)cap);
    return 0;
}

int main(int argc, char **argv) {
    const char *which = argc > 1 ? argv[1] : "all";
    int rc = 0;
    auto want = [&](const char *s) { return !strcmp(which, "all") || !strcmp(which, s); };
    if (want("pool")) rc |= pool();
    if (want("validation")) rc |= validation();
    if (want("stream")) rc |= run_stream(64ull << 30, 64, 2000, 100, 0, "stream");
    if (want("tight")) rc |= run_stream(256ull << 20, 64, 600, 200, 0, "tight_budget");
    if (want("slots")) rc |= run_stream(64ull << 30, 2, 400, 50, 0, "two_slots");
    if (want("restart")) rc |= run_stream(64ull << 30, 8, 200, 50, 20, "device_restart");
    return rc;
}
