// host_pool.hpp -- host worker threads for building and checking the
// patch-set tables: a fixed set made on first use in a process and never torn
// down (idle workers end with the process; a forked child, which holds none
// of them, makes its own set).  parallel_for(n, fn) calls fn(t) once for every
// t < n, on the workers and the calling thread, and returns when all calls are
// done; the calling thread takes tasks too, so a call completes even without
// workers.  Calls from several threads take turns; fn must not call
// parallel_for.
#pragma once

#include <unistd.h>

#include <algorithm>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace hsgn {

class HostPool {
public:
    static HostPool &get()
    {
        static std::mutex *gm = new std::mutex();
        static HostPool *pool = nullptr;
        std::lock_guard<std::mutex> lk(*gm);
        if (!pool || pool->pid != getpid()) pool = new HostPool();
        return *pool;
    }
    int size() const { return (int)workers.size() + 1; }
    void parallel_for(int n, const std::function<void(int)> &fn)
    {
        if (n <= 0) return;
        if (n == 1 || workers.empty()) {
            for (int t = 0; t < n; t++) fn(t);
            return;
        }
        std::lock_guard<std::mutex> turn(call_m);
        {
            std::lock_guard<std::mutex> lk(m);
            job = &fn;
            ntask = n;
            next = 0;
            left = n;
            gen++;
        }
        cv.notify_all();
        drain();
        std::unique_lock<std::mutex> lk(m);
        done.wait(lk, [&] { return left == 0; });
        job = nullptr;
    }

private:
    HostPool() : pid(getpid())
    {
        const int hw = (int)std::thread::hardware_concurrency();
        const int n = std::max(1, std::min(16, hw)) - 1;
        for (int k = 0; k < n; k++) workers.emplace_back([this] { loop(); });
    }
    // take tasks of the current call until none is left
    void drain()
    {
        for (;;) {
            int t;
            const std::function<void(int)> *f;
            {
                std::lock_guard<std::mutex> lk(m);
                if (!job || next >= ntask) return;
                t = next++;
                f = job;
            }
            (*f)(t);
            bool last;
            {
                std::lock_guard<std::mutex> lk(m);
                last = --left == 0;
            }
            if (last) done.notify_all();
        }
    }
    void loop()
    {
        unsigned long long seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(m);
                cv.wait(lk, [&] { return gen != seen; });
                seen = gen;
            }
            drain();
        }
    }
    const pid_t pid;
    std::mutex m, call_m;
    std::condition_variable cv, done;
    const std::function<void(int)> *job = nullptr;
    int ntask = 0, next = 0, left = 0;
    unsigned long long gen = 0;
    std::vector<std::thread> workers;
};

}  // namespace hsgn
