// A small fixed pool of host threads for per-problem work of the batched
// solver (price-loop updates and price tables of hundreds of problems between
// two rounds).  run(n, fn) calls fn(lo, hi) on contiguous ranges covering
// [0, n), one range per worker plus one for the calling thread, and returns
// when all have finished.  fn must not throw.
//
// Rounds of a batched solve come every few milliseconds and the work between
// them is tens of microseconds, so waking sleeping threads would cost more
// than the work: after a job a worker keeps polling for the next one for
// kSpin before it sleeps on a condition variable.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace ra {

class HostPool {
public:
    static constexpr std::chrono::microseconds kSpin{5000};

    explicit HostPool(int workers)
    {
        for (int i = 0; i < workers; ++i) th_.emplace_back([this, i] { loop(i); });
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_.store(true, std::memory_order_release);
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    HostPool(const HostPool&) = delete;
    HostPool& operator=(const HostPool&) = delete;

    int parts() const { return (int)th_.size() + 1; }

    void run(int n, const std::function<void(int, int)>& fn)
    {
        const int P = parts();
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &fn;
            n_ = n;
            left_.store((int)th_.size(), std::memory_order_relaxed);
            gen_.store(gen_.load(std::memory_order_relaxed) + 1, std::memory_order_release);
        }
        cv_.notify_all();
        const int hi0 = range_end(0, n, P);
        if (hi0 > 0) fn(0, hi0);
        while (left_.load(std::memory_order_acquire) != 0) std::this_thread::yield();
    }

private:
    static int range_end(int k, int n, int P) { return (int)((int64_t)n * (k + 1) / P); }

    void loop(int i)
    {
        uint64_t seen = 0;
        for (;;) {
            // poll for a while, then sleep until the next job or the end
            const auto t0 = std::chrono::steady_clock::now();
            while (gen_.load(std::memory_order_acquire) == seen &&
                   !stop_.load(std::memory_order_acquire) &&
                   std::chrono::steady_clock::now() - t0 < kSpin)
                __builtin_ia32_pause();
            if (gen_.load(std::memory_order_acquire) == seen) {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] {
                    return stop_.load(std::memory_order_acquire) ||
                           gen_.load(std::memory_order_acquire) != seen;
                });
            }
            if (stop_.load(std::memory_order_acquire)) return;
            seen = gen_.load(std::memory_order_acquire);
            const std::function<void(int, int)>* fn = fn_;
            const int n = n_;
            const int P = parts();
            const int lo = range_end(i, n, P), hi = range_end(i + 1, n, P);
            if (hi > lo) (*fn)(lo, hi);
            left_.fetch_sub(1, std::memory_order_acq_rel);
        }
    }

    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_;
    const std::function<void(int, int)>* fn_ = nullptr;
    int n_ = 0;
    std::atomic<int> left_{0};
    std::atomic<uint64_t> gen_{0};
    std::atomic<bool> stop_{false};
};

}  // namespace ra
