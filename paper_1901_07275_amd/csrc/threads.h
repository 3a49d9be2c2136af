// Host-side parallel loop used by the planner and the dense linear algebra.
// Plain std::thread workers pulling chunks of 16 indices from an atomic
// counter (no OpenMP runtime: the library shares a process with torch's).
#pragma once

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

namespace jt {

// Set on a thread that is itself one worker of an outer parallel loop (for
// example one plan of a batch): its parallel_for calls then run serially.
inline thread_local bool tl_serial = false;

template <class F>
inline void parallel_for(int count, F f)
{
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<unsigned>(hw ? hw : 1, 16);
    if (count < 64 || nt <= 1 || tl_serial) {
        for (int i = 0; i < count; ++i) f(i);
        return;
    }
    std::atomic<int> next(0);
    auto work = [&]() {
        for (;;) {
            int i0 = next.fetch_add(16);
            if (i0 >= count) break;
            int i1 = std::min(count, i0 + 16);
            for (int i = i0; i < i1; ++i) f(i);
        }
    };
    std::vector<std::thread> th;
    for (int k = 1; k < nt; ++k) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
}

}  // namespace jt
