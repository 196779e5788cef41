// Host checks of the serving policy (pool allocator and admission choice),
// built with g++ by test_serve_policy.py.  Prints "ok" or the first failure.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "serve_policy.h"

using rlu::serve::PoolAlloc;
using rlu::serve::kGranule;

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);              \
      return 1;                                                     \
    }                                                               \
  } while (0)

struct Req {
  size_t bytes;
  int blocks = 1;
  int bypassed = 0;
};

static int basic() {
  PoolAlloc p(10 * kGranule + 7);  // size rounds down to whole granules
  CHECK(p.size() == 10 * kGranule);
  size_t a, b, c, d;
  CHECK(p.alloc(1, &a) && a == 0);                  // one granule
  CHECK(p.alloc(3 * kGranule, &b) && b == kGranule);
  CHECK(p.alloc(2 * kGranule + 1, &c) && c == 4 * kGranule);  // rounds to 3 granules
  CHECK(p.used() == 7 * kGranule);
  CHECK(!p.alloc(4 * kGranule, &d));                // only 3 left
  p.release(b, 3 * kGranule);                       // hole [1, 4)
  CHECK(p.free_ranges() == 2);
  CHECK(p.alloc(3 * kGranule, &d) && d == kGranule);  // first fit reuses the hole
  p.release(a, 1);
  p.release(d, 3 * kGranule);                       // merges with [0, 1)
  p.release(c, 2 * kGranule + 1);                   // merges everything
  CHECK(p.free_ranges() == 1 && p.used() == 0 && p.largest_free() == p.size());
  return 0;
}

// random alloc / release against a byte map of granules
static int fuzz() {
  std::mt19937_64 rng(12345);
  const size_t G = 97;
  PoolAlloc p(G * kGranule);
  std::vector<int> owner(G, -1);
  struct Live { size_t off, bytes; int id; };
  std::vector<Live> live;
  int next_id = 0;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t bytes = 1 + rng() % (12 * kGranule);
      size_t off;
      const size_t need = (bytes + kGranule - 1) / kGranule;
      // does a run of `need` free granules exist (first fit)?
      size_t expect = (size_t)-1;
      for (size_t s = 0, run = 0; s < G; ++s) {
        run = owner[s] < 0 ? run + 1 : 0;
        if (run == need) { expect = s + 1 - need; break; }
      }
      const bool ok = p.alloc(bytes, &off);
      CHECK(ok == (expect != (size_t)-1));
      if (ok) {
        CHECK(off == expect * kGranule);
        for (size_t s = 0; s < need; ++s) { CHECK(owner[expect + s] < 0); owner[expect + s] = next_id; }
        live.push_back({off, bytes, next_id++});
      }
    } else {
      const size_t i = rng() % live.size();
      const Live l = live[i];
      live.erase(live.begin() + i);
      p.release(l.off, l.bytes);
      const size_t g0 = l.off / kGranule, need = (l.bytes + kGranule - 1) / kGranule;
      for (size_t s = 0; s < need; ++s) { CHECK(owner[g0 + s] == l.id); owner[g0 + s] = -1; }
    }
    size_t used = 0;
    for (int o : owner) used += o >= 0;
    CHECK(p.used() == used * kGranule);
  }
  return 0;
}

static int admission() {
  PoolAlloc p(8 * kGranule);
  size_t hold;
  CHECK(p.alloc(5 * kGranule, &hold));  // 3 granules free
  std::deque<Req> q;
  q.push_back({4 * kGranule});          // head does not fit
  q.push_back({2 * kGranule});
  q.push_back({1 * kGranule});
  size_t off, off2;
  int idx = rlu::serve::pick_next(q, p, 4, 2, &off);
  CHECK(idx == 1 && q.front().bypassed == 1);  // younger request passes the head
  q.erase(q.begin() + idx);
  idx = rlu::serve::pick_next(q, p, 4, 2, &off2);
  CHECK(idx == 1 && q.front().bypassed == 2);
  q.erase(q.begin() + idx);
  p.release(off2, 1 * kGranule);                 // memory for a third younger one is there
  q.push_back({1});
  const size_t used = p.used();
  idx = rlu::serve::pick_next(q, p, 4, 2, &off);
  CHECK(idx == -1 && p.used() == used);          // bypass budget spent: wait for the head
  p.release(hold, 5 * kGranule);
  idx = rlu::serve::pick_next(q, p, 4, 2, &off);
  CHECK(idx == 0);                               // the head goes once memory frees up
  std::deque<Req> empty;
  CHECK(rlu::serve::pick_next(empty, p, 4, 2, &off) == -1);
  return 0;
}

// The second resource: a request whose panel blocks exceed what the running
// requests leave waits like one whose workspace does not fit, and takes no
// pool memory while it waits.
static int admission_blocks() {
  PoolAlloc p(8 * kGranule);
  std::deque<Req> q;
  q.push_back({2 * kGranule, 6});   // needs more blocks than are free
  q.push_back({2 * kGranule, 3});
  q.push_back({2 * kGranule, 5});
  size_t off;
  int idx = rlu::serve::pick_next(q, p, 4, 1, &off);
  CHECK(idx == 1 && q.front().bypassed == 1 && p.used() == 2 * kGranule);
  q.erase(q.begin() + idx);
  idx = rlu::serve::pick_next(q, p, 1, 1, &off);
  CHECK(idx == -1 && p.used() == 2 * kGranule);  // bypass spent, and the head still lacks blocks
  idx = rlu::serve::pick_next(q, p, 6, 1, &off);
  CHECK(idx == 0 && p.used() == 4 * kGranule);   // blocks freed: the head goes
  return 0;
}

int main() {
  if (basic() || fuzz() || admission() || admission_blocks()) return 1;
  std::printf("ok\n");
  return 0;
}
