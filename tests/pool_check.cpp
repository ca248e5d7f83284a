// Test program (CPU only) for the planner's worker pool: many parallel loops
// in a row, loops started from several threads at once, loops nested in a
// loop body and a loop after fork(); every body index must run exactly once
// per loop.  Prints one line; exit status 0 when every check passes.
#include "../paper_1201_5991_amd/csrc/plan.hpp"

#include <sys/wait.h>
#include <unistd.h>

#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

using namespace mlbddc;

static bool one_loop(int T) {
  std::vector<std::atomic<int>> hits(T);
  for (auto& h : hits) h = 0;
  parallel_run(T, [&](int t) { hits[t]++; });
  for (int t = 0; t < T; ++t)
    if (hits[t] != 1) return false;
  return true;
}

int main() {
  bool ok = true;
  // loops in a row with changing widths (workers idle in between)
  for (int rep = 0; rep < 2000 && ok; ++rep) ok = one_loop(1 + rep % 16);
  const bool seq = ok;
  // four threads starting loops at once: one gets the pool, the others spawn
  std::atomic<int> bad{0};
  std::vector<std::thread> th;
  for (int c = 0; c < 4; ++c)
    th.emplace_back([&bad, c] {
      for (int rep = 0; rep < 300; ++rep)
        if (!one_loop(2 + (rep + c) % 15)) bad++;
    });
  for (auto& x : th) x.join();
  const bool conc = bad == 0;
  // a loop inside a loop body
  std::atomic<int> inner{0};
  parallel_run(8, [&](int) { parallel_run(4, [&](int) { inner++; }); });
  const bool nest = inner == 32;
  // a child process after fork runs its own loops
  bool forked = true;
  pid_t pid = fork();
  if (pid == 0) _exit(one_loop(16) && one_loop(5) ? 0 : 1);
  if (pid > 0) {
    int status = 0;
    waitpid(pid, &status, 0);
    forked = WIFEXITED(status) && WEXITSTATUS(status) == 0;
  }
  ok = seq && conc && nest && forked && one_loop(16);
  std::printf("sequential %d concurrent %d nested %d fork %d %s\n", (int)seq, (int)conc, (int)nest, (int)forked,
              ok ? "ok" : "FAIL");
  return ok ? 0 : 1;
}
