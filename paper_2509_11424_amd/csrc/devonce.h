// Once-per-device initialisation of __constant__ tables: every device holds
// its own copy of a __constant__ array, so an upload is done once for each
// device that a call runs on (the current device), not once per process.
#pragma once
#include <mutex>
#include <set>

#include "common.h"

namespace mgm {

// Runs init() unless it already ran with the current device; each call site
// (each lambda type) keeps its own record.
template <class F>
void once_per_device(F init) {
  static std::mutex mu;
  static std::set<int> done;
  int dev = 0;
  MGM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(dev)) return;
  init();
  done.insert(dev);
}

}  // namespace mgm
