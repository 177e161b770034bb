// Host worker threads for the device-layout stages (host-only work: no HIP calls inside f).
#pragma once

#include <algorithm>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace asmg {

// run f(i) for i in [0, n) on up to `threads` host threads (0 = all cores); the first error is
// rethrown after every thread has joined
template <class F>
void host_parallel(int threads, int n, F f) {
  int nt = threads > 0 ? threads : (int)std::thread::hardware_concurrency();
  nt = std::max(1, std::min(nt, n));
  std::atomic<int> next{0};
  std::mutex mu;
  std::exception_ptr err;
  auto work = [&]() {
    try {
      for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) f(i);
    } catch (...) {
      std::lock_guard<std::mutex> g(mu);
      if (!err) err = std::current_exception();
      next = n;
    }
  };
  if (nt == 1) {
    work();
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(work);
    for (auto &t : th) t.join();
  }
  if (err) std::rethrow_exception(err);
}

}  // namespace asmg
