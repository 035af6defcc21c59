// Checks of the host worker pool (host_pool.hpp), built and run by
// test_host_pool.py: every task of a call runs exactly once, calls from two
// threads at once each see all their tasks, and a forked child (which holds
// none of the parent's workers) completes its calls and exits.
#include <sys/wait.h>
#include <unistd.h>

#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "host_pool.hpp"

using hsgn::HostPool;

int main()
{
    HostPool &P = HostPool::get();
    printf("workers+caller %d\n", P.size());
    long long bad = 0;
    for (int rep = 0; rep < 20000; rep++) {
        const int n = 1 + rep % 23;
        std::vector<int> hit(n, 0);
        P.parallel_for(n, [&](int t) { hit[t]++; });
        for (int t = 0; t < n; t++) bad += hit[t] != 1;
    }
    std::atomic<long long> sum{0};
    auto caller = [&]() {
        for (int rep = 0; rep < 5000; rep++) {
            std::vector<int> hit(16, 0);
            HostPool::get().parallel_for(16, [&](int t) { hit[t]++; });
            for (int t = 0; t < 16; t++) sum += hit[t];
        }
    };
    std::thread a(caller), b(caller);
    a.join();
    b.join();
    printf("exactly-once failures %lld, concurrent sum %lld of %d\n", bad, (long long)sum,
           2 * 5000 * 16);
    fflush(stdout);
    const pid_t c = fork();
    if (c == 0) {
        std::vector<int> hit(8, 0);
        HostPool::get().parallel_for(8, [&](int t) { hit[t]++; });
        for (int t = 0; t < 8; t++)
            if (hit[t] != 1) _exit(3);
        _exit(0);
    }
    int st = -1;
    waitpid(c, &st, 0);
    const int child_ok = WIFEXITED(st) && WEXITSTATUS(st) == 0;
    printf("forked child ok %d\n", child_ok);
    return (bad == 0 && sum == 2 * 5000 * 16 && child_ok) ? 0 : 1;
}
