// Stress check of the server's host thread pool (built by test_host_pool.py,
// under ThreadSanitizer): every item of every job runs exactly once, its
// plain (non-atomic) writes are visible to the caller when run() returns,
// and the pool shuts down cleanly, for 0 to 3 helpers.
#include <cstdio>
#include <vector>

#include "host_pool.h"

int main() {
  for (int helpers = 0; helpers <= 3; ++helpers) {
    uml::HostPool pool(helpers);
    std::vector<long> out;
    for (int rep = 0; rep < 2000; ++rep) {
      const int n = (rep * 37) % 300;  // includes n < 8 (run inline) and 0
      out.assign(n, -1);
      std::vector<int> calls(n, 0);
      pool.run(n, [&](int i) {
        out[i] = long(i) * i + rep;  // plain writes, read below
        calls[i] += 1;
      });
      for (int i = 0; i < n; ++i)
        if (calls[i] != 1 || out[i] != long(i) * i + rep) {
          std::printf("FAIL helpers=%d rep=%d item=%d calls=%d\n", helpers, rep, i, calls[i]);
          return 1;
        }
    }
  }
  std::printf("OK\n");
  return 0;
}
