// A persistent pool of host threads for data-parallel loops of the analysis.
//
// run(n, fn) calls fn(lo, hi) on disjoint chunks covering [0, n) from the
// calling thread and the workers, and returns when every chunk is done.
// Callers only hand it loops whose iterations are independent (or combine
// through order-independent integer atomics), so results never depend on the
// number of threads or on scheduling.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace qg {

class WorkPool {
public:
    // Threads: QG_ANALYSIS_THREADS if set (>= 1), else the hardware threads, at most 16.
    static int default_threads() {
        if (const char *e = std::getenv("QG_ANALYSIS_THREADS")) {
            const int v = std::atoi(e);
            if (v >= 1) return std::min(v, 256);
        }
        const unsigned hw = std::thread::hardware_concurrency();
        return (int)std::max(1u, std::min(hw, 16u));
    }

    explicit WorkPool(int nthreads) {
        for (int t = 1; t < nthreads; ++t) workers_.emplace_back([this] { loop(); });
    }
    ~WorkPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            ++gen_;
        }
        cv_.notify_all();
        for (auto &w : workers_) w.join();
    }
    WorkPool(const WorkPool &) = delete;
    WorkPool &operator=(const WorkPool &) = delete;

    int threads() const { return (int)workers_.size() + 1; }

    void run(int64_t n, const std::function<void(int64_t, int64_t)> &fn) {
        if (n <= 0) return;
        if (workers_.empty()) {
            fn(0, n);
            return;
        }
        const int64_t nt = threads();
        chunk_ = std::max<int64_t>(64, (n + 4 * nt - 1) / (4 * nt));
        n_ = n;
        fn_ = &fn;
        next_.store(0);
        {
            std::lock_guard<std::mutex> lk(mu_);
            busy_ = (int)workers_.size();
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [this] { return busy_ == 0; });
        fn_ = nullptr;
    }

private:
    void work() {
        for (;;) {
            const int64_t lo = next_.fetch_add(chunk_);
            if (lo >= n_) break;
            (*fn_)(lo, std::min(n_, lo + chunk_));
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                if (stop_) return;
            }
            work();
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (--busy_ == 0) done_cv_.notify_one();
            }
        }
    }

    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    uint64_t gen_ = 0;
    int busy_ = 0;
    bool stop_ = false;
    std::atomic<int64_t> next_{0};
    int64_t n_ = 0, chunk_ = 1;
    const std::function<void(int64_t, int64_t)> *fn_ = nullptr;
};

}  // namespace qg
