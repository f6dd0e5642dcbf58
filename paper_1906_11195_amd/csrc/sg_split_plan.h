// Members per VB work unit when large units are split over several
// workgroups that meet at a device-scope barrier after every colour class.
// Host code only (no HIP), so that the allocation can be checked on the CPU.
//
// A unit's cost per sweep is weighed as n (10 + chains): its graph (adjacency
// stream and spin words per vertex) dominates and is shared by its chains,
// a chain adding about a tenth of it (whole units, us per sweep on MI355X:
// one chain of 985767 spins 792, six chains of 65536 spins 82).  Splitting
// shortens a launch only if no unit left whole outlasts the split ones, so
// the automatic plan splits the units above twice a CU's share of the cost
// only when all of them get at least two members, or else the largest
// leading group of them with three times the cost of every unit left whole.
// Their members are shared out in proportion to cost, so that every member
// carries about the same part of a sweep, with a floor per member that rises
// with the number of split units: members of many split units meet at their
// barriers at the same time, and thin members then wait more than they
// compute.  Measured, us per sweep: graphs of 65536 spins with 6 chains,
// 1 graph 13 members 33, 4 graphs 8 members 41 (4: 48), 16 graphs 4 members
// 57 (6: 61, 8: 73), 64 graphs 2 members 78 (whole: 82; with a budget of a
// quarter of the CUs they stay whole); one request of 985767 spins with 2
// chains (two units), 8 members each 153, 16 97, 32 78, 64 82.
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <numeric>
#include <vector>

namespace sg {

// the least cost a member carries with at most two, at most eight and more
// split units (about 8, 14 and 28 us of a sweep on MI355X), and the most
// members of one unit
constexpr int64_t kSplitMemberCostFew = 75000;
constexpr int64_t kSplitMemberCostSome = 130000;
constexpr int64_t kSplitMemberCostMany = 260000;
constexpr int kSplitMaxMembers = 32;

struct SplitUnit {
    int64_t cost;        // n (10 + chains)
    bool resident;       // adjacency kept in LDS: never split
    int64_t chunk_cap;   // most members with two 64-position chunks per wavefront of the largest class
};

// Members of every unit (1: whole) for `budget` workgroups of split members
// and a CU's share `share` of the batch's cost.  forced: 0 automatic, 1
// never split, k >= 2 every non-resident unit that has the chunks for k
// members, within the budget.  Returns the members used (those of split
// units).
inline int plan_split(const std::vector<SplitUnit>& units, int64_t share, int budget, int forced,
                      std::vector<int>& members)
{
    members.assign(units.size(), 1);
    if (forced == 1 || budget < 2) return 0;
    std::vector<size_t> by_cost(units.size());
    std::iota(by_cost.begin(), by_cost.end(), (size_t)0);
    std::stable_sort(by_cost.begin(), by_cost.end(),
                     [&](size_t a, size_t b) { return units[a].cost > units[b].cost; });
    size_t n_auto = 0;
    if (forced == 0) {
        size_t cand = 0;
        while (cand < by_cost.size() && !units[by_cost[cand]].resident && units[by_cost[cand]].cost >= 2 * share)
            ++cand;
        for (size_t m = std::min(cand, (size_t)(budget / 2)); m >= 1; --m) {
            const int64_t rest = by_cost.size() > m ? units[by_cost[m]].cost : 0;
            if (m == cand || units[by_cost[m - 1]].cost >= 3 * rest) {
                n_auto = m;
                break;
            }
        }
    }
    int64_t split_cost = 0;
    for (size_t r = 0; r < n_auto; ++r) split_cost += units[by_cost[r]].cost;
    const int64_t floor_cost = n_auto <= 2 ? kSplitMemberCostFew : n_auto <= 8 ? kSplitMemberCostSome
                                                                                : kSplitMemberCostMany;
    const int64_t per_member = std::max<int64_t>({share, (split_cost + budget - 1) / budget, floor_cost});
    int used = 0;
    for (size_t r = 0; r < by_cost.size(); ++r) {
        const SplitUnit& u = units[by_cost[r]];
        if (u.resident || (forced == 0 && r >= n_auto)) continue;
        int64_t want = forced >= 2 ? forced
                                   : std::min<int64_t>(kSplitMaxMembers, (u.cost + per_member / 2) / per_member);
        want = std::min<int64_t>(want, std::min<int64_t>(u.chunk_cap, budget));
        if (want >= 2) {
            members[by_cost[r]] = (int)want;
            budget -= (int)want;
            used += (int)want;
        }
    }
    return used;
}

}  // namespace sg
