// CPU test of the serving admission logic (arena + FIFO admitter), no GPU.
#include <cassert>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2008_04447_amd/csrc/serve_sched.hpp"

using namespace rq;

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);      \
      ++fails;                                                     \
    }                                                              \
  } while (0)

int main() {
  // arena: allocation, exhaustion, merge on release
  {
    Arena a(1024 * 10);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(3000, &o1) && o1 == 0);
    CHECK(a.alloc(3000, &o2) && o2 == 3072);
    CHECK(a.alloc(3000, &o3) && o3 == 6144);
    CHECK(!a.alloc(2000, &o4));                // 1024 bytes left
    a.release(o2, 3000);
    CHECK(a.largest_free() == 3072);
    a.release(o1, 3000);
    CHECK(a.largest_free() == 6144);           // merged with the freed right neighbour
    CHECK(a.alloc(6000, &o4) && o4 == 0);
    a.release(o4, 6000);
    a.release(o3, 3000);
    CHECK(a.used() == 0 && a.largest_free() == 10240);
  }
  // admitter: FIFO order, slots, budget never exceeded, oversize rejected
  {
    Admitter ad(1 << 20);
    CHECK(!ad.enqueue(99, (1 << 20) + 1));
    std::mt19937 rng(7);
    std::uniform_int_distribution<int> sz(1000, 400000);
    std::vector<std::pair<uint64_t, size_t>> running;
    std::vector<size_t> foot(200);
    for (uint64_t i = 0; i < 200; ++i) {
      foot[i] = sz(rng);
      CHECK(ad.enqueue(i, foot[i]));
    }
    uint64_t expect = 0;
    size_t peak = 0;
    int steps = 0;
    while ((ad.queued() || !running.empty()) && steps < 100000) {
      ++steps;
      auto adm = ad.admit(4 - (int)running.size());
      for (auto& x : adm) {
        CHECK(x.id == expect);                 // arrival order
        ++expect;
        running.push_back({x.id, x.offset});
      }
      peak = std::max(peak, ad.used());
      CHECK(ad.used() <= (size_t)(1 << 20));
      CHECK(running.size() <= 4);
      if (!running.empty()) {                  // finish a pseudo-random running request
        const size_t j = rng() % running.size();
        ad.finish(running[j].second, foot[running[j].first]);
        running.erase(running.begin() + j);
      }
    }
    CHECK(expect == 200);
    CHECK(ad.used() == 0);
    std::printf("peak arena use %zu of %d\n", peak, 1 << 20);
  }
  std::printf("%s\n", fails ? "FAILED" : "OK");
  return fails ? 1 : 0;
}
