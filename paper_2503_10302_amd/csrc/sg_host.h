// sg_host.h -- host-side helpers shared by the library's C++ sources (no device code).
#pragma once

#include <algorithm>
#include <atomic>
#include <exception>
#include <system_error>
#include <thread>
#include <vector>

namespace sg {

// f(0) .. f(n - 1) on up to 16 host threads (the calling one included), each index once.
// After every thread has ended, the exception of the lowest failing index is rethrown, so
// that the error reported does not depend on the threads' timing.
template <class F>
void parallel_for(int n, F f)
{
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = std::min({n, (int)hw, 16});
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::exception_ptr> err((size_t)n);
    auto work = [&] {
        for (int i = next++; i < n; i = next++) {
            try {
                f(i);
            } catch (...) {
                err[(size_t)i] = std::current_exception();
            }
        }
    };
    std::vector<std::thread> th;
    for (int k = 1; k < nt; ++k) {
        try {
            th.emplace_back(work);
        } catch (const std::system_error &) {
            break;   // no more threads: the ones started and this one share the rest
        }
    }
    work();
    for (std::thread &t : th) t.join();
    for (const std::exception_ptr &e : err)
        if (e) std::rethrow_exception(e);
}

}  // namespace sg
