// Stress check of the serving path's host copy pool: several threads copy
// pieces of random sizes at once; every destination byte must match its source,
// and run() must report a checked piece exactly when it holds a negative or
// non-finite float.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "host_copy.h"

int main(int argc, char **argv) {
  const int callers = argc > 1 ? atoi(argv[1]) : 4, rounds = argc > 2 ? atoi(argv[2]) : 40;
  nfhmm::CopyPool pool(5);
  std::vector<int> bad(callers, 0), wrong_verdict(callers, 0);
  std::vector<std::thread> th;
  for (int c = 0; c < callers; ++c)
    th.emplace_back([&, c] {
      std::mt19937_64 rng(1234 + c);
      const float poison[4] = {-1.0f, NAN, INFINITY, -0.5f};
      for (int r = 0; r < rounds; ++r) {
        const int n = 1 + (int)(rng() % 5);
        std::vector<std::vector<float>> src(n), dst(n);
        std::vector<nfhmm::CopyPool::Piece> p(n);
        bool expect_ok = true;
        for (int i = 0; i < n; ++i) {
          // from empty up to ~9 MiB: below, at and above the chunk and the inline threshold
          const size_t f = (rng() % 4 == 0) ? rng() % 1024 : rng() % (9u << 18);
          src[i].resize(f);
          dst[i].assign(f, 0.0f);
          for (size_t k = 0; k < f; ++k) src[i][k] = (float)((k * 131 + i * 7 + r + c) % 1000);
          const bool check = rng() % 2 == 0;
          if (f && rng() % 3 == 0) {   // plant one bad value
            src[i][rng() % f] = poison[rng() % 4];
            if (check) expect_ok = false;
          }
          p[i] = {dst[i].data(), src[i].data(), f * 4, check};
        }
        const bool ok = pool.run(p.data(), n);
        if (ok != expect_ok) ++wrong_verdict[c];
        for (int i = 0; i < n; ++i)
          if (memcmp(src[i].data(), dst[i].data(), src[i].size() * 4) != 0) ++bad[c];
      }
    });
  for (auto &t : th) t.join();
  int total = 0, verdicts = 0;
  for (int c = 0; c < callers; ++c) {
    total += bad[c];
    verdicts += wrong_verdict[c];
  }
  printf("callers %d rounds %d mismatching pieces %d wrong verdicts %d\n", callers, rounds, total, verdicts);
  return total == 0 && verdicts == 0 ? 0 : 1;
}
