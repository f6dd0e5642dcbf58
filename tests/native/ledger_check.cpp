// Host-only check of the split-member ledger's accounting (compiled with g++
// by tests/test_ledger_host.py; no GPU): reservations never exceed the bound,
// a plan sees only what other holders left, releases return members, and the
// count stays exact under concurrent reserve/release from many threads.
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "sg_ledger.h"

#define CHECK(x)                                                   \
    do {                                                           \
        if (!(x)) {                                                \
            std::printf("FAIL line %d: %s\n", __LINE__, #x);       \
            return 1;                                              \
        }                                                          \
    } while (0)

int main()
{
    sg::SplitLedger L;
    int seen = -1;
    // first context on device 0: all 128 available, takes 48
    CHECK(L.reserve(0, 128, [&](int a) { seen = a; return 48; }) == 48);
    CHECK(seen == 128 && L.held(0) == 48);
    // second context sees the rest; asks for more than is left: clamped
    CHECK(L.reserve(0, 128, [&](int a) { seen = a; return 500; }) == 80);
    CHECK(seen == 80 && L.held(0) == 128);
    // a third sees nothing (its units stay whole)
    CHECK(L.reserve(0, 128, [&](int a) { seen = a; return 0; }) == 0);
    CHECK(seen == 0);
    // other devices are independent
    CHECK(L.reserve(1, 128, [&](int a) { seen = a; return 16; }) == 16);
    CHECK(seen == 128 && L.held(1) == 16 && L.held(0) == 128);
    // release returns members; negative plans reserve nothing
    L.release(0, 48);
    CHECK(L.held(0) == 80);
    CHECK(L.reserve(0, 128, [&](int a) { seen = a; return -3; }) == 0);
    CHECK(seen == 48);
    L.release(0, 80);
    L.release(1, 16);
    CHECK(L.held(0) == 0 && L.held(1) == 0);
    L.release(0, 5);   // never below zero
    CHECK(L.held(0) == 0);

    // concurrent contexts: the sum held never exceeds the bound
    const int cap = 128, threads = 16, iters = 20000;
    std::atomic<int> over{0};
    std::vector<std::thread> th;
    for (int t = 0; t < threads; ++t)
        th.emplace_back([&, t]() {
            for (int i = 0; i < iters; ++i) {
                const int want = 1 + (t * 7 + i * 13) % 40;
                const int got = L.reserve(2, cap, [&](int a) { return a < want ? a : want; });
                if (L.held(2) > cap) over.fetch_add(1);
                L.release(2, got);
            }
        });
    for (auto& x : th) x.join();
    CHECK(over.load() == 0);
    CHECK(L.held(2) == 0);
    std::printf("ledger ok\n");
    return 0;
}
