// Host runtime helpers: a persistent worker pool for parallel host work
// (task building), and optional phase tracing to stderr (FABX_TRACE=1).
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace fabx {

// Fixed set of worker threads shared by the library; parallel_for(n, f) runs
// f(0..n-1) on the calling thread plus the workers and returns when all are done.
class HostPool {
public:
    static HostPool &get() {
        static HostPool pool;
        return pool;
    }
    int size() const { return int(workers_.size()) + 1; }

    void parallel_for(int n, const std::function<void(int)> &f) {
        if (n <= 1 || workers_.empty()) {
            for (int k = 0; k < n; ++k) f(k);
            return;
        }
        std::unique_lock<std::mutex> call(call_mu_);  // one parallel region at a time
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &f;
            next_ = 0;
            total_ = n;
            pending_ = n;
            ++generation_;
        }
        cv_.notify_all();
        run_tasks();
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return pending_ == 0; });
        fn_ = nullptr;
    }

    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            ++generation_;
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
    }

private:
    HostPool() {
        unsigned hw = std::thread::hardware_concurrency();
        int n = int(hw == 0 ? 1 : hw);
        if (n > 16) n = 16;
        for (int i = 1; i < n; ++i) workers_.emplace_back([this] { worker(); });
    }
    void run_tasks() {
        for (;;) {
            int k;
            const std::function<void(int)> *f;
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (!fn_ || next_ >= total_) return;
                k = next_++;
                f = fn_;
            }
            (*f)(k);
            std::lock_guard<std::mutex> lk(mu_);
            if (--pending_ == 0) done_cv_.notify_all();
        }
    }
    void worker() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || generation_ != seen; });
                if (stop_) return;
                seen = generation_;
            }
            run_tasks();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex mu_, call_mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *fn_ = nullptr;
    int next_ = 0, total_ = 0, pending_ = 0;
    uint64_t generation_ = 0;
    bool stop_ = false;
};

// Phase tracing: FABX_TRACE=1 prints "[fabx] <what> <ms>" lines to stderr.
class Trace {
public:
    explicit Trace(const char *scope) : scope_(scope), on_(enabled()) {
        if (on_) t0_ = last_ = std::chrono::steady_clock::now();
    }
    void mark(const char *what) {
        if (!on_) return;
        auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[fabx] %s.%s %.3f ms\n", scope_, what,
                     std::chrono::duration<double, std::milli>(now - last_).count());
        last_ = now;
    }
    static bool enabled() {
        static const bool on = [] {
            const char *v = std::getenv("FABX_TRACE");
            return v && v[0] && v[0] != '0';
        }();
        return on;
    }

private:
    const char *scope_;
    bool on_;
    std::chrono::steady_clock::time_point t0_, last_;
};

}  // namespace fabx
