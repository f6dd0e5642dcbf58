// Process-wide ledger of the workgroups that split VB units hold on a device.
//
// The members of a split unit wait for each other at a device-scope barrier
// after every colour class, so all of them must be resident at once.  Their
// number is bounded device-wide, over every context of the process (not per
// context): a context reserves its members when it is created and returns
// them when it is released, and a context planned while others hold members
// gets only what is left.  With the bound at half of the compute units, the
// members of every split unit that can run at the same time fit on the
// device together, next to other work that finishes on its own, so no
// barrier waits for a member that cannot be placed.  (Contexts of other
// processes on the same device are not counted.)
#pragma once
#include <map>
#include <mutex>

namespace sg {

class SplitLedger {
public:
    // Calls plan(available) with the members still free on `device` under
    // the bound `cap`, under the ledger's lock, and reserves what it returns
    // (clamped to [0, available]).  Returns the reserved count.
    template <class Plan>
    int reserve(int device, int cap, Plan&& plan)
    {
        std::lock_guard<std::mutex> lk(mu_);
        int& held = held_[device];
        const int avail = cap > held ? cap - held : 0;
        int used = plan(avail);
        if (used < 0) used = 0;
        if (used > avail) used = avail;
        held += used;
        return used;
    }
    void release(int device, int n)
    {
        if (n <= 0) return;
        std::lock_guard<std::mutex> lk(mu_);
        int& held = held_[device];
        held = held > n ? held - n : 0;
    }
    int held(int device)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = held_.find(device);
        return it == held_.end() ? 0 : it->second;
    }

private:
    std::mutex mu_;
    std::map<int, int> held_;
};

}  // namespace sg
