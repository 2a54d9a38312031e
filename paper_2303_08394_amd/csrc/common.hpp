// Shared host-side helpers: status codes, the thread-local error message and
// a small parallel-for over std::thread.
#pragma once

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <string>
#include <thread>
#include <vector>

#include "kifmm.h"

namespace kifmm {

// Records `msg` as the calling thread's last error and returns `st`.
kifmm_status fail(kifmm_status st, const std::string& msg);

// An exception carrying a status; caught at the C boundary and turned into
// a status + message.  Never crosses the C ABI.
struct Error {
  kifmm_status status;
  std::string msg;
};

[[noreturn]] inline void raise(kifmm_status st, const std::string& msg) { throw Error{st, msg}; }

// Allocation-failure injection (kifmm_debug_fail_allocations): every host
// build step and device allocation of the library calls alloc_hook first;
// the call that finds the counter at 0 fails with ENOMEM and disarms it
// (-1).  One counter per process, shared by every source file.
inline std::atomic<int64_t>& alloc_fail_counter() {
  static std::atomic<int64_t> c{-1};
  return c;
}
inline void alloc_hook(const char* what) {
  auto& c = alloc_fail_counter();
  int64_t v = c.load();
  while (v >= 0) {
    if (c.compare_exchange_weak(v, v - 1)) {
      if (v == 0) raise(KIFMM_ENOMEM, std::string(what) + ": allocation failure injected by the test hook");
      return;
    }
  }
}

inline int hw_threads() {
  unsigned n = std::thread::hardware_concurrency();
  return n == 0 ? 1 : (n > 32 ? 32 : static_cast<int>(n));
}

// Runs f(begin, end) over [0, n) split into contiguous chunks, one per thread.
template <class F>
void parallel_for(int64_t n, F&& f, int min_chunk = 256) {
  int nt = hw_threads();
  if (n < static_cast<int64_t>(min_chunk) * 2 || nt == 1) {
    f(int64_t(0), n);
    return;
  }
  int64_t chunks = (n + min_chunk - 1) / min_chunk;
  if (chunks < nt) nt = static_cast<int>(chunks);
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int t = 0; t < nt; ++t) {
    int64_t b = n * t / nt, e = n * (t + 1) / nt;
    th.emplace_back([&f, b, e] { f(b, e); });
  }
  for (auto& x : th) x.join();
}

}  // namespace kifmm
