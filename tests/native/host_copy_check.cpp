// Stress check of the serving path's host copy pool: several threads copy
// pieces of random sizes at once; every destination byte must match its source.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "host_copy.h"

int main(int argc, char **argv) {
  const int callers = argc > 1 ? atoi(argv[1]) : 4, rounds = argc > 2 ? atoi(argv[2]) : 40;
  nfhmm::CopyPool pool(5);
  std::vector<int> bad(callers, 0);
  std::vector<std::thread> th;
  for (int c = 0; c < callers; ++c)
    th.emplace_back([&, c] {
      std::mt19937_64 rng(1234 + c);
      for (int r = 0; r < rounds; ++r) {
        const int n = 1 + (int)(rng() % 5);
        std::vector<std::vector<unsigned char>> src(n), dst(n);
        std::vector<nfhmm::CopyPool::Piece> p(n);
        for (int i = 0; i < n; ++i) {
          // from empty up to ~9 MiB: below, at and above the chunk and the inline threshold
          const size_t b = (rng() % 4 == 0) ? rng() % 4096 : rng() % (9u << 20);
          src[i].resize(b);
          dst[i].assign(b, 0);
          for (size_t k = 0; k < b; ++k) src[i][k] = (unsigned char)(k * 131 + i * 7 + r + c);
          p[i] = {dst[i].data(), src[i].data(), b};
        }
        pool.run(p.data(), n);
        for (int i = 0; i < n; ++i)
          if (src[i] != dst[i]) ++bad[c];
      }
    });
  for (auto &t : th) t.join();
  int total = 0;
  for (int b : bad) total += b;
  printf("callers %d rounds %d mismatching pieces %d\n", callers, rounds, total);
  return total == 0 ? 0 : 1;
}
