// Host thread pool for independent loops of the build (no device code).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace fpde {

// fn(i) for i in [0, n) on up to min(16, hardware threads, n) host threads, each i
// independent (fn(i) writes only what i owns, so the result does not depend on the
// schedule); below serial_below items the loop runs on the calling thread.  An
// exception in a worker stops the others and is rethrown here after the join.
template <typename Fn>
void parallel_for(int64_t n, Fn fn, int64_t serial_below = 32) {
    const unsigned hc = std::thread::hardware_concurrency();
    const int64_t nt = std::min<int64_t>(std::min<int64_t>(16, hc ? hc : 1), n);
    if (n < serial_below || nt <= 1) {
        for (int64_t i = 0; i < n; ++i) fn(i);
        return;
    }
    std::atomic<int64_t> next(0);
    std::exception_ptr err;
    std::mutex mu;
    std::vector<std::thread> th;
    for (int64_t k = 0; k < nt; ++k)
        th.emplace_back([&]() {
            try {
                for (int64_t i = next++; i < n; i = next++) fn(i);
            } catch (...) {
                std::lock_guard<std::mutex> lk(mu);
                if (!err) err = std::current_exception();
                next = n;
            }
        });
    for (auto& x : th) x.join();
    if (err) std::rethrow_exception(err);
}

}  // namespace fpde
