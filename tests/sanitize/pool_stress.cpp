// Stress of the host thread pool (paper_2505_02692_amd/csrc/host_pool.h) for
// the sanitizer builds: regions issued from several threads at once (one runs
// on the pool, the others in place), nested regions, regions that return
// before late workers wake, serial threads, and the block cache under
// concurrent allocation.  Every region checks that each index ran exactly
// once.  Exit status 0 when every check holds.
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "host_pool.h"

using fabx::HostPool;

static std::atomic<int> g_fail{0};

static void region(int n, int salt) {
    std::vector<std::atomic<int>> hit(static_cast<size_t>(n));
    for (auto &h : hit) h.store(0);
    HostPool::get().parallel_for(n, [&](int k) {
        hit[static_cast<size_t>(k)].fetch_add(1 + (salt & 0));
        if ((k + salt) % 97 == 0) std::this_thread::yield();
    });
    for (int k = 0; k < n; ++k)
        if (hit[static_cast<size_t>(k)].load() != 1) g_fail.fetch_add(1);
}

static void nested(int n) {
    std::atomic<int> inner{0};
    HostPool::get().parallel_for(n, [&](int) {
        // a region issued inside a region runs in place on the calling worker
        HostPool::get().parallel_for(8, [&](int) { inner.fetch_add(1); });
    });
    if (inner.load() != 8 * n) g_fail.fetch_add(1);
}

static void cache_churn(int seed) {
    auto &c = fabx::HostBlockCache::get();
    std::vector<std::pair<void *, size_t>> held;
    for (int i = 0; i < 200; ++i) {
        const size_t bytes = size_t(1) << (16 + (i * 7 + seed) % 8);
        void *p = c.alloc(bytes);
        static_cast<volatile char *>(p)[0] = char(i);
        static_cast<volatile char *>(p)[bytes - 1] = char(i);
        held.push_back({p, bytes});
        if (held.size() > 6) {
            c.free(held.front().first, held.front().second);
            held.erase(held.begin());
        }
    }
    for (auto &h : held) c.free(h.first, h.second);
}

int main() {
    const int rounds = 300;
    std::vector<std::thread> th;
    for (int t = 0; t < 3; ++t)
        th.emplace_back([t] {
            if (t == 2) HostPool::caller_serial() = true;  // a serial thread runs its regions in place
            for (int r = 0; r < rounds; ++r) {
                region(1 + (r * 37 + t * 11) % 500, r + t);
                if (r % 5 == 0) nested(16 + t);
                if (r % 3 == 0) cache_churn(r + t);
                if (r % 7 == 0) std::this_thread::sleep_for(std::chrono::microseconds(400));  // workers go to sleep
            }
        });
    for (auto &x : th) x.join();
    std::printf("pool stress: %d threads x %d rounds, %d failed checks, pool of %d threads\n", 3, rounds,
                g_fail.load(), HostPool::get().size());
    return g_fail.load() == 0 ? 0 : 1;
}
