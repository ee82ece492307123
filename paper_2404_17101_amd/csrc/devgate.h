// devgate.h -- the served form's device phases (host-only; no HIP types, so
// that a plain C++ compiler can build and test it).
#pragma once
#include <condition_variable>
#include <mutex>

namespace pg {

// Device phases: the persistent launches of a slice need every workgroup
// resident, and ordinary kernels on other streams can hold the compute units
// they wait for, so the loop's slices (exclusive) and the levels of the
// direction-optimizing requests (shared among their threads) never overlap on
// the device. The phases take turns: a waiting slice stops new levels from
// starting, and the levels that waited through a slice start before the next
// one.
struct DevGate {
  std::mutex m;
  std::condition_variable cv;
  int shared = 0, shared_waiting = 0, excl_waiting = 0;
  bool excl = false;
  bool turn_shared = false;  // set when a slice ends with levels waiting
  void enter_shared() {
    std::unique_lock<std::mutex> lk(m);
    shared_waiting++;
    cv.wait(lk, [&] { return !excl && (excl_waiting == 0 || turn_shared); });
    shared_waiting--;
    shared++;
    if (shared_waiting == 0) turn_shared = false;
  }
  void leave_shared() {
    std::lock_guard<std::mutex> lk(m);
    if (--shared == 0) cv.notify_all();
  }
  void enter_excl() {
    std::unique_lock<std::mutex> lk(m);
    excl_waiting++;
    cv.wait(lk, [&] { return !excl && shared == 0 && !turn_shared; });
    excl_waiting--;
    excl = true;
  }
  void leave_excl() {
    std::lock_guard<std::mutex> lk(m);
    excl = false;
    turn_shared = shared_waiting > 0;
    cv.notify_all();
  }
};

}  // namespace pg
