// Concurrent task builds through the C ABI on host-only contexts, for the
// sanitizer builds of the host runtime: several threads build the same task
// specifications at once (each build runs its parallel parts on the shared
// host pool, or in place when another thread holds it) and every build must
// give the same cells.  Exit status 0 when every check holds.
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "fastabx.h"

int main() {
    fabx_ctx *ctx = nullptr;
    if (fabx_create(&ctx, -1, nullptr) != FABX_OK) return 2;
    // 8k items: label, context, speaker; lengths 1..20 frames
    const int64_t n = 8000;
    std::mt19937 rng(7);
    std::vector<int32_t> attrs(size_t(n) * 3);
    std::vector<int64_t> off(size_t(n) + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        attrs[size_t(3 * i)] = int32_t(rng() % 30);
        attrs[size_t(3 * i + 1)] = int32_t(rng() % 12);
        attrs[size_t(3 * i + 2)] = int32_t(rng() % 25);
        off[size_t(i + 1)] = off[size_t(i)] + 1 + int64_t(rng() % 20);
    }
    static float dummy[16];
    fabx_dataset_desc d{dummy, FABX_DTYPE_F32, off.back(), 16, off.data(), n, attrs.data(), 3};
    fabx_dataset *ds = nullptr;
    if (fabx_dataset_create(ctx, &d, &ds) != FABX_OK) return 3;
    struct Spec {
        std::vector<int32_t> by, across;
    };
    const Spec specs[] = {{{1, 2}, {}}, {{1}, {2}}, {{2}, {}}, {{}, {1}}};
    std::vector<std::vector<int64_t>> ref(4);
    for (int s = 0; s < 4; ++s) {
        fabx_task *t = nullptr;
        if (fabx_task_create(ds, 0, specs[s].by.data(), int32_t(specs[s].by.size()), specs[s].across.data(),
                             int32_t(specs[s].across.size()), &t) != FABX_OK)
            return 4;
        ref[size_t(s)].resize(size_t(fabx_task_num_cells(t)));
        fabx_task_cell_sizes(t, ref[size_t(s)].data(), nullptr);
        fabx_task_destroy(t);
    }
    int fails = 0;
    std::vector<std::thread> th;
    std::vector<int> bad(4, 0);
    for (int k = 0; k < 4; ++k)
        th.emplace_back([&, k] {
            if (k == 3) fabx_set_thread_serial(1);
            for (int r = 0; r < 8; ++r) {
                const int s = (k + r) % 4;
                fabx_task *t = nullptr;
                if (fabx_task_create(ds, 0, specs[s].by.data(), int32_t(specs[s].by.size()),
                                     specs[s].across.data(), int32_t(specs[s].across.size()), &t) != FABX_OK) {
                    ++bad[size_t(k)];
                    continue;
                }
                std::vector<int64_t> sz(size_t(fabx_task_num_cells(t)));
                fabx_task_cell_sizes(t, sz.data(), nullptr);
                std::vector<int32_t> keys(sz.size() * size_t(fabx_task_key_width(t)));
                fabx_task_cell_keys(t, keys.data());
                if (sz != ref[size_t(s)]) ++bad[size_t(k)];
                fabx_task_destroy(t);
            }
        });
    for (auto &x : th) x.join();
    for (int b : bad) fails += b;
    std::printf("build stress: 4 threads x 8 builds of 4 task shapes, %d mismatches\n", fails);
    fabx_dataset_destroy(ds);
    fabx_destroy(ctx);
    return fails == 0 ? 0 : 1;
}
