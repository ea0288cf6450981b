// Host runtime helpers: a persistent worker pool for parallel host work
// (task building), and optional phase tracing to stderr (FABX_TRACE=1).
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <sys/resource.h>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

namespace fabx {

// Process-wide cache of large host blocks.  Task tables and builder / collapse
// scratch are rebuilt for every task; keeping their freed blocks mapped lets
// the next task of similar size reuse them without page faults.  Blocks are
// rounded up to size classes (four per power of two); at most kCap bytes stay
// cached, the rest go back to the system allocator.
class HostBlockCache {
public:
    static HostBlockCache &get() {
        static HostBlockCache c;
        return c;
    }
    void *alloc(size_t bytes) {
        if (bytes < kMin) return ::operator new(bytes);
        const int k = size_class(bytes);
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto &l = free_[size_t(k)];
            if (!l.empty()) {
                void *p = l.back();
                l.pop_back();
                cached_ -= class_bytes(k);
                return p;
            }
        }
        return ::operator new(class_bytes(k));
    }
    void free(void *p, size_t bytes) {
        if (bytes < kMin) {
            ::operator delete(p);
            return;
        }
        const int k = size_class(bytes);
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (cached_ + class_bytes(k) <= kCap) {
                free_[size_t(k)].push_back(p);
                cached_ += class_bytes(k);
                return;
            }
        }
        ::operator delete(p);
    }
    ~HostBlockCache() {
        for (auto &l : free_)
            for (void *p : l) ::operator delete(p);
    }

private:
    static constexpr size_t kMin = size_t(64) << 10;
    static constexpr size_t kCap = size_t(2) << 30;
    // class k covers (class_bytes(k - 1), class_bytes(k)]; sizes 64 KiB * 2^(k/4) * (1 + (k%4)/4)
    static size_t class_bytes(int k) { return (kMin << (k / 4)) / 4 * size_t(4 + k % 4); }
    static int size_class(size_t bytes) {
        int k = 0;
        while (class_bytes(k) < bytes) ++k;
        return k;
    }
    std::mutex mu_;
    size_t cached_ = 0;
    std::vector<void *> free_[160];
};

// Allocator over HostBlockCache whose element construction without arguments
// leaves trivial types uninitialised (no zero fill): every array held in such
// a vector is written before it is read.
template <class T>
struct CachedAlloc {
    using value_type = T;
    CachedAlloc() noexcept = default;
    template <class U>
    CachedAlloc(const CachedAlloc<U> &) noexcept {}
    T *allocate(size_t n) { return static_cast<T *>(HostBlockCache::get().alloc(n * sizeof(T))); }
    void deallocate(T *p, size_t n) noexcept { HostBlockCache::get().free(p, n * sizeof(T)); }
    template <class U>
    void construct(U *p) noexcept(std::is_nothrow_default_constructible<U>::value) {
        ::new (static_cast<void *>(p)) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new (static_cast<void *>(p)) U(std::forward<A>(a)...);
    }
};
template <class T, class U>
bool operator==(const CachedAlloc<T> &, const CachedAlloc<U> &) { return true; }
template <class T, class U>
bool operator!=(const CachedAlloc<T> &, const CachedAlloc<U> &) { return false; }

template <class T>
using hvec = std::vector<T, CachedAlloc<T>>;

// Fixed set of worker threads shared by the library; parallel_for(n, f) runs
// f(0..n-1) on the calling thread plus the workers and returns when all are done.
// Work items are handed out through an atomic counter.  Every worker checks in
// once per region after its last item, and the region ends only when all have,
// so no worker can still be drawing from one region's counter when the next
// region resets it.  Idle workers spin for a short while before sleeping on a
// condition variable, so back-to-back regions (a task build has several) do
// not pay a wake-up each.
class HostPool {
public:
    static HostPool &get() {
        static HostPool pool;
        return pool;
    }
    int size() const { return int(workers_.size()) + 1; }

    void parallel_for(int n, const std::function<void(int)> &f) {
        // One parallel region at a time: other threads wait for the workers.  A
        // region started from inside a worker (or from the thread running the
        // current region) runs its items in place, as waiting would deadlock.
        if (n <= 1 || workers_.empty() || in_region()) {
            for (int k = 0; k < n; ++k) f(k);
            return;
        }
        std::unique_lock<std::mutex> call(call_mu_);
        in_region() = true;
        struct Reset {
            ~Reset() { in_region() = false; }
        } reset;
        fn_ = &f;
        total_ = n;
        next_.store(0, std::memory_order_relaxed);
        arrived_.store(0, std::memory_order_relaxed);
        {
            std::lock_guard<std::mutex> lk(mu_);
            generation_.fetch_add(1, std::memory_order_release);
        }
        cv_.notify_all();
        run_tasks();
        const int nw = int(workers_.size());
        while (arrived_.load(std::memory_order_acquire) != nw) std::this_thread::yield();
        fn_ = nullptr;
    }

    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_.store(true);
            generation_.fetch_add(1, std::memory_order_release);
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
            const int k = next_.fetch_add(1, std::memory_order_relaxed);
            if (k >= total_) return;
            (*fn_)(k);
        }
    }
    static bool &in_region() {
        thread_local bool flag = false;
        return flag;
    }
    void worker() {
        in_region() = true;
        uint64_t seen = 0;
        for (;;) {
            uint64_t g = generation_.load(std::memory_order_acquire);
            if (g == seen) {
                const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(300);
                while ((g = generation_.load(std::memory_order_acquire)) == seen &&
                       std::chrono::steady_clock::now() < until)
                    std::this_thread::yield();
            }
            if (g == seen) {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return generation_.load(std::memory_order_acquire) != seen; });
                g = generation_.load(std::memory_order_acquire);
            }
            if (stop_.load()) return;
            seen = g;
            run_tasks();
            arrived_.fetch_add(1, std::memory_order_release);
        }
    }
    std::vector<std::thread> workers_;
    std::mutex mu_, call_mu_;
    std::condition_variable cv_;
    const std::function<void(int)> *fn_ = nullptr;
    int total_ = 0;
    std::atomic<int> next_{0}, arrived_{0};
    std::atomic<uint64_t> generation_{0};
    std::atomic<bool> stop_{false};
};

// Phase tracing: FABX_TRACE=1 prints "[fabx] <what> <ms> <minor page faults>"
// lines to stderr.
class Trace {
public:
    explicit Trace(const char *scope) : scope_(scope), on_(enabled()) {
        if (on_) {
            t0_ = last_ = std::chrono::steady_clock::now();
            flt_ = faults();
        }
    }
    void mark(const char *what) {
        if (!on_) return;
        auto now = std::chrono::steady_clock::now();
        const long f = faults();
        std::fprintf(stderr, "[fabx] %s.%s %.3f ms %ld faults\n", scope_, what,
                     std::chrono::duration<double, std::milli>(now - last_).count(), f - flt_);
        last_ = now;
        flt_ = f;
    }
    static bool enabled() {
        static const bool on = [] {
            const char *v = std::getenv("FABX_TRACE");
            return v && v[0] && v[0] != '0';
        }();
        return on;
    }

private:
    static long faults() {
        struct rusage ru;
        getrusage(RUSAGE_SELF, &ru);
        return ru.ru_minflt;
    }
    const char *scope_;
    bool on_;
    long flt_ = 0;
    std::chrono::steady_clock::time_point t0_, last_;
};

}  // namespace fabx
