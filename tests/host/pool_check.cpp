// Host-only check of the worker pool shared by the 2-D and 3-D libraries
// (paper_2609_35529_amd/csrc/host_util.hpp), built with ThreadSanitizer by
// tests/test_host_pool.py: every item of a section runs exactly once, nested
// sections (a section started from inside an item, as the list builders do
// per level and per band of rows) complete, sections started by several host
// threads at once (several contexts) do not mix their items, and an item that
// throws leaves the others running and reaches the caller.
#include "../../paper_2609_35529_amd/csrc/host_util.hpp"

#include <atomic>
#include <cstdio>
#include <stdexcept>
#include <thread>
#include <vector>

static int check_counts(const std::vector<std::atomic<int>> &c, int want, const char *what) {
  for (size_t i = 0; i < c.size(); ++i)
    if (c[i].load() != want) {
      printf("%s: item %zu ran %d times, want %d\n", what, i, c[i].load(), want);
      return 1;
    }
  return 0;
}

int main() {
  auto &pool = vlbm_host::Pool::get();
  int bad = 0;
  // flat sections of every size 0..64
  for (int n = 0; n <= 64; ++n) {
    std::vector<std::atomic<int>> c(n);
    pool.run(n, [&](int i) { c[i].fetch_add(1); });
    bad |= check_counts(c, 1, "flat");
  }
  // three nested levels, as the list builders nest levels, bands and shares
  {
    std::vector<std::atomic<int>> c(8 * 6 * 5);
    for (int rep = 0; rep < 50; ++rep)
      pool.run(8, [&](int a) {
        pool.run(6, [&](int b) { pool.run(5, [&](int d) { c[(a * 6 + b) * 5 + d].fetch_add(1); }); });
      });
    bad |= check_counts(c, 50, "nested");
  }
  // sections from four host threads at once, each with its own items; the
  // items write plain (non-atomic) slots owned by their section, so a mixed-up
  // or repeated item is a data race the sanitizer reports
  {
    std::vector<std::vector<long>> sums(4, std::vector<long>(16, 0));
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t)
      th.emplace_back([&, t] {
        for (int rep = 0; rep < 200; ++rep)
          pool.run(16, [&](int i) {
            sums[t][i] += i + 1;
            if (i % 4 == 0) pool.run(3, [&](int) {});
          });
      });
    for (auto &x : th) x.join();
    for (int t = 0; t < 4; ++t)
      for (int i = 0; i < 16; ++i)
        if (sums[t][i] != 200L * (i + 1)) {
          printf("threads: section %d item %d sum %ld\n", t, i, sums[t][i]);
          bad = 1;
        }
  }
  // items that throw: the section still runs every item, and the caller
  // gets the exception
  {
    std::vector<std::atomic<int>> c(32);
    bool caught = false;
    try {
      pool.run(32, [&](int i) {
        c[i].fetch_add(1);
        if (i % 7 == 3) throw std::runtime_error("item");
      });
    } catch (const std::runtime_error &) {
      caught = true;
    }
    bad |= check_counts(c, 1, "throwing");
    if (!caught) {
      printf("throwing: no exception reached the caller\n");
      bad = 1;
    }
  }
  printf(bad ? "FAIL\n" : "ok\n");
  return bad;
}
