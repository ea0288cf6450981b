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
#include <unistd.h>
#include <utility>
#include <vector>

namespace fabx {

// Process-wide cache of large host blocks.  Task tables and builder / collapse
// scratch are rebuilt for every task; keeping their freed blocks mapped lets
// the next task of similar size reuse them without page faults.  Blocks are
// rounded up to size classes (four per power of two); at most a quarter of
// the physical memory (between 2 and 32 GiB) stays cached, the rest goes back
// to the system allocator.  A pipelined caller keeps a few tasks alive at once,
// each with its per-cell arrays (about 80 bytes per cell).
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
            if (cached_ + class_bytes(k) <= cap_) {
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
    const size_t cap_ = [] {
        const long pages = sysconf(_SC_PHYS_PAGES), page = sysconf(_SC_PAGESIZE);
        const size_t phys = pages > 0 && page > 0 ? size_t(pages) * size_t(page) : 0;
        return std::min(std::max(phys / 4, size_t(2) << 30), size_t(32) << 30);
    }();
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
// f(0..n-1) on the calling thread plus the workers and returns when all items
// are done.  Items are handed out through one atomic ticket holding a
// generation (high 32 bits) and the next item (low 32 bits).  Region r first
// closes the ticket (generation 2r - 1: no item can be claimed), then sets its
// function, item count and done counter, then opens it (generation 2r, item
// 0).  A worker claims item k only by advancing an open ticket (2r, k) with
// k below the count it read, so a worker that wakes late, or still holds a
// ticket of an earlier region, claims nothing: its exchange fails.  A region
// therefore waits only for its claimed items, never for idle workers.  Idle
// workers spin for a short while before sleeping on a condition variable, so
// back-to-back regions (a task build has several) do not pay a wake-up each.
//
// One region runs at a time.  A parallel_for issued while another thread's
// region is running (say a collapse on one thread while a task is built on
// another), or from inside a region, or from a thread marked serial, runs its
// items in place on the calling thread.  The pool leaves one hardware thread to such callers: it uses at
// most 16 threads and, on machines with 8 or more, one fewer than there are
// (FABX_HOST_THREADS sets the count instead).
class HostPool {
public:
    static HostPool &get() {
        static HostPool pool;
        return pool;
    }
    int size() const { return int(workers_.size()) + 1; }
    // Whether a parallel_for issued now from this thread would run on the
    // workers (a hint: another thread may start a region meanwhile, and then
    // the call still completes, in place).
    bool would_run_parallel() const {
        return !workers_.empty() && !in_region() && !caller_serial() && !busy_.load();
    }
    // Set for the calling thread: its regions always run in place.
    static bool &caller_serial() {
        thread_local bool flag = false;
        return flag;
    }

    void parallel_for(int n, const std::function<void(int)> &f) {
        if (n <= 1 || workers_.empty() || in_region() || caller_serial()) {
            for (int k = 0; k < n; ++k) f(k);
            return;
        }
        std::unique_lock<std::mutex> call(call_mu_, std::try_to_lock);
        if (!call.owns_lock()) {  // another thread's region is running
            for (int k = 0; k < n; ++k) f(k);
            return;
        }
        in_region() = true;
        busy_.store(true);
        struct Reset {
            std::atomic<bool> &busy;
            ~Reset() {
                in_region() = false;
                busy.store(false);
            }
        } reset{busy_};
        const uint64_t open = (ticket_.load() >> 32) + 2;  // even
        ticket_.store((open - 1) << 32);                   // closed
        fn_.store(&f);
        total_.store(uint32_t(n));
        done_.store(0);
        {
            std::lock_guard<std::mutex> lk(mu_);
            ticket_.store(open << 32);
        }
        cv_.notify_all();
        run_tasks(open);
        while (done_.load() != uint32_t(n)) std::this_thread::yield();
    }

    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_.store(true);
            ticket_.store(((ticket_.load() >> 32) + 2) << 32);
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
    }

private:
    HostPool() {
        unsigned hw = std::thread::hardware_concurrency();
        int n = int(hw == 0 ? 1 : hw);
        if (n >= 8) n -= 1;
        if (n > 16) n = 16;
        // FABX_HOST_THREADS: threads of a region, the caller included (1..64),
        // e.g. to leave CPUs of a shared or quota-limited machine to other threads
        if (const char *v = std::getenv("FABX_HOST_THREADS")) {
            const int k = std::atoi(v);
            if (k >= 1 && k <= 64) n = k;
        }
        for (int i = 1; i < n; ++i) workers_.emplace_back([this] { worker(); });
    }
    // Claim and run items of open generation g until none is left or g is over.
    // All accesses are sequentially consistent: a count read after the next
    // region's close is ordered after that close, so the exchange that follows
    // it fails.
    void run_tasks(uint64_t g) {
        for (;;) {
            uint64_t t = ticket_.load();
            if ((t >> 32) != g) return;
            const uint32_t k = uint32_t(t);
            if (k >= total_.load()) return;
            if (!ticket_.compare_exchange_weak(t, t + 1)) continue;
            // item k is claimed and not done, so this region is still running
            (*fn_.load())(int(k));
            done_.fetch_add(1);
        }
    }
    static bool &in_region() {
        thread_local bool flag = false;
        return flag;
    }
    // generation of an open region other than `seen`, or 0
    uint64_t next_open(uint64_t seen) const {
        const uint64_t g = ticket_.load() >> 32;
        return (g != seen && g % 2 == 0) ? g : 0;
    }
    void worker() {
        in_region() = true;
        uint64_t seen = 0;
        for (;;) {
            uint64_t g = next_open(seen);
            if (g == 0 && !stop_.load()) {
                const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(300);
                while ((g = next_open(seen)) == 0 && !stop_.load() && std::chrono::steady_clock::now() < until)
                    std::this_thread::yield();
            }
            if (g == 0 && !stop_.load()) {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return next_open(seen) != 0 || stop_.load(); });
                g = next_open(seen);
            }
            if (stop_.load()) return;
            if (g == 0) continue;
            seen = g;
            run_tasks(g);
        }
    }
    std::vector<std::thread> workers_;
    std::mutex mu_, call_mu_;
    std::condition_variable cv_;
    std::atomic<const std::function<void(int)> *> fn_{nullptr};
    std::atomic<uint32_t> total_{0}, done_{0};
    std::atomic<uint64_t> ticket_{0};  // generation << 32 | next item; odd generation: closed
    std::atomic<bool> stop_{false};
    std::atomic<bool> busy_{false};  // a region is running
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
