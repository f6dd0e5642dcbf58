// Host-only check of the split planner (compiled with g++ by
// tests/test_split_plan_host.py; no GPU): the members it gives equal graphs,
// unequal graphs and single large units, resident units, forced plans and
// tight budgets.
#include <cstdio>
#include <vector>

#include "sg_split_plan.h"

#define CHECK(x)                                                   \
    do {                                                           \
        if (!(x)) {                                                \
            std::printf("FAIL line %d: %s\n", __LINE__, #x);       \
            return 1;                                              \
        }                                                          \
    } while (0)

using sg::SplitUnit;

static int64_t cost(int64_t n, int64_t chains) { return n * (10 + chains); }
static int64_t share_of(const std::vector<SplitUnit>& u, int n_cu)
{
    int64_t t = 0;
    for (const auto& x : u) t += x.cost;
    return t / n_cu > 1 ? t / n_cu : 1;
}

int main()
{
    const int n_cu = 256, quarter = 64;
    std::vector<int> m;
    // equal graphs of 65536 spins with 6 chains, 16 wavefronts: 427 chunks
    // in the largest class, at most 13 members with two chunks per wavefront
    for (int g : {1, 4, 16, 64, 256}) {
        std::vector<SplitUnit> u(g, SplitUnit{cost(65536, 6), false, 13});
        const int used = sg::plan_split(u, share_of(u, n_cu), quarter, 0, m);
        const int want = g == 1 ? 13 : g == 4 ? 8 : g == 16 ? 4 : 1;   // 64 and 256: whole
        int sum = 0;
        for (int x : m) {
            CHECK(x == want);
            sum += x > 1 ? x : 0;
        }
        CHECK(used == sum && used <= quarter);
    }
    // one request of 985767 spins, two one-chain units: 32 members each
    // (the per-unit maximum) within half of the CUs
    {
        std::vector<SplitUnit> u(2, SplitUnit{cost(985767, 1), false, 200});
        CHECK(sg::plan_split(u, share_of(u, n_cu), 128, 0, m) == 64);
        CHECK(m[0] == 32 && m[1] == 32);
        // with a quarter of the CUs: the same (64)
        CHECK(sg::plan_split(u, share_of(u, n_cu), quarter, 0, m) == 64);
        // with 20 left: 10 each would exceed nothing, the first takes what
        // its share asks and the second what is left
        const int used = sg::plan_split(u, share_of(u, n_cu), 20, 0, m);
        CHECK(used <= 20 && m[0] >= m[1] && m[1] >= 2);
    }
    // unequal units: members in proportion to cost, the largest the most,
    // small units whole, the budget never exceeded
    {
        std::vector<SplitUnit> u = {{cost(985767, 1), false, 200}, {cost(6156, 2), false, 1},
                                    {cost(798101, 1), false, 160}, {cost(249966, 2), false, 50},
                                    {cost(62220, 2), false, 12},   {cost(724080, 1), false, 150}};
        const int used = sg::plan_split(u, share_of(u, n_cu), quarter, 0, m);
        CHECK(used <= quarter);
        CHECK(m[0] > m[2] && m[2] >= m[5] && m[5] > m[3]);
        CHECK(m[1] == 1);
        int sum = 0;
        for (int x : m) sum += x > 1 ? x : 0;
        CHECK(sum == used);
    }
    // resident units (adjacency in LDS) are never split, whatever their cost
    {
        std::vector<SplitUnit> u = {{cost(985767, 1), true, 200}, {cost(1000, 2), false, 1}};
        CHECK(sg::plan_split(u, share_of(u, n_cu), quarter, 0, m) == 0);
        CHECK(m[0] == 1 && m[1] == 1);
    }
    // forced plans: 1 never, k every unit with the chunks for k, within the budget
    {
        std::vector<SplitUnit> u = {{cost(20000, 2), false, 4}, {cost(30000, 2), false, 1},
                                    {cost(50000, 2), true, 9},  {cost(40000, 2), false, 6}};
        CHECK(sg::plan_split(u, 1, 128, 1, m) == 0);
        for (int x : m) CHECK(x == 1);
        CHECK(sg::plan_split(u, 1, 128, 3, m) == 6);
        CHECK(m[0] == 3 && m[1] == 1 && m[2] == 1 && m[3] == 3);
        CHECK(sg::plan_split(u, 1, 128, 5, m) == 9);   // 5 where the chunks allow, else the chunk cap
        CHECK(m[0] == 4 && m[3] == 5);
        CHECK(sg::plan_split(u, 1, 4, 3, m) == 3);     // budget: only the costliest non-resident one
        CHECK(m[3] == 3 && m[0] == 1);
    }
    // no budget: everything whole
    {
        std::vector<SplitUnit> u(2, SplitUnit{cost(985767, 1), false, 200});
        CHECK(sg::plan_split(u, share_of(u, n_cu), 1, 0, m) == 0);
        CHECK(m[0] == 1 && m[1] == 1);
    }
    std::printf("split plan ok\n");
    return 0;
}
