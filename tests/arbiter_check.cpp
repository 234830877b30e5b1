// Host-side check of the persistent-panel arbiter (csrc/arbiter.hpp):
// route selection for concurrent handles, per device, with nesting and
// release by the owner only; and under contention from many threads, never
// two owners of one device at once.  Prints "ok" and exits 0 on success.
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "../paper_2502_02460_amd/csrc/arbiter.hpp"

#define CHECK(c)                                               \
    do {                                                       \
        if (!(c)) {                                            \
            std::printf("check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                          \
        }                                                      \
    } while (0)

int main() {
    gevd::PanelArbiter a;
    int h1, h2, h3;
    CHECK(a.try_acquire(0, &h1));          // first handle on device 0 takes the route
    CHECK(!a.try_acquire(0, &h2));         // a second handle is routed per column
    CHECK(a.try_acquire(1, &h2));          // other devices are independent
    CHECK(a.try_acquire(0, &h1));          // nested acquisition by the owner
    a.release(0, &h1);
    CHECK(a.owner(0) == &h1);              // still held once
    a.release(0, &h2);                     // not the owner: no effect
    CHECK(a.owner(0) == &h1);
    a.release(0, &h1);
    CHECK(a.owner(0) == nullptr);
    CHECK(a.try_acquire(0, &h3));          // free again
    a.release(0, &h3);
    CHECK(!a.try_acquire(-1, &h1) && !a.try_acquire(gevd::PanelArbiter::MAXDEV, &h1));
    CHECK(!a.try_acquire(0, nullptr));

    // contention: 16 threads, each repeatedly takes the route if it can and
    // checks that it is alone while holding it
    std::atomic<int> holders{0}, taken{0}, violations{0};
    std::vector<std::thread> th;
    std::vector<int> ids(16);
    for (int t = 0; t < 16; ++t)
        th.emplace_back([&, t] {
            for (int i = 0; i < 20000; ++i) {
                if (a.try_acquire(3, &ids[t])) {
                    if (holders.fetch_add(1) != 0) violations.fetch_add(1);
                    taken.fetch_add(1);
                    holders.fetch_sub(1);
                    a.release(3, &ids[t]);
                }
            }
        });
    for (auto& x : th) x.join();
    CHECK(violations.load() == 0);
    CHECK(taken.load() > 0);
    CHECK(a.owner(3) == nullptr);
    std::printf("ok\n");
    return 0;
}
