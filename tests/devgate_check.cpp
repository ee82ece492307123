// Stress check of the served form's device-phase gate (host-only): three
// threads take the shared side as direction-optimizing levels do, one takes
// the exclusive side as the slice loop does, with no pause between its slices.
// Fails if the two sides ever overlap, if either side stops making progress,
// or if shared users often wait through more than two exclusive phases (the
// levels that waited through a slice go before the next one; a rare longer
// wait is the host scheduler descheduling the thread between its reads).
#include <atomic>
#include <chrono>
#include <cstdio>
#include <thread>
#include <vector>

#include "devgate.h"

int main() {
  pg::DevGate gate;
  std::atomic<int> in_shared{0}, in_excl{0}, violations{0};
  std::atomic<bool> stop{false};
  std::atomic<long> shared_done{0}, excl_done{0}, max_phases_waited{0}, long_waits{0};
  const auto spin = [](int us) {
    const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(us);
    while (std::chrono::steady_clock::now() < until) {
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < 3; t++)
    th.emplace_back([&, t] {
      while (!stop) {
        const long before = excl_done;
        gate.enter_shared();
        const long waited = excl_done - before;
        if (waited > 2) long_waits++;
        long m = max_phases_waited;
        while (waited > m && !max_phases_waited.compare_exchange_weak(m, waited)) {
        }
        in_shared++;
        if (in_excl.load()) violations++;
        spin(20 + 10 * t);
        in_shared--;
        gate.leave_shared();
        shared_done++;
      }
    });
  th.emplace_back([&] {
    while (!stop) {
      gate.enter_excl();
      in_excl++;
      if (in_shared.load() || in_excl.load() != 1) violations++;
      spin(50);
      in_excl--;
      gate.leave_excl();
      excl_done++;
    }
  });
  // both sides must keep progressing in every window
  long s0 = 0, e0 = 0;
  int stalls = 0;
  for (int w = 0; w < 20; w++) {
    std::this_thread::sleep_for(std::chrono::milliseconds(50));
    const long s1 = shared_done, e1 = excl_done;
    if (s1 == s0 || e1 == e0) stalls++;
    s0 = s1;
    e0 = e1;
  }
  stop = true;
  for (auto &x : th) x.join();
  std::printf("shared %ld exclusive %ld violations %d stalled windows %d most exclusive phases waited %ld, "
              "waits of more than two %ld\n", shared_done.load(), excl_done.load(), violations.load(), stalls,
              max_phases_waited.load(), long_waits.load());
  return (violations == 0 && stalls == 0 && shared_done > 100 && excl_done > 100 &&
          long_waits * 100 < shared_done) ? 0 : 1;
}
