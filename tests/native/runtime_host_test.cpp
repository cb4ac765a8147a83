// CPU test of the serving runtime's host bookkeeping (arena allocator and admission
// order).  Built with g++ by tests/test_runtime_cpu.py; prints "OK" on success.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <random>
#include <vector>

#include "../../paper_2409_03568_amd/csrc/arena.hpp"

using ckks::rt::Admission;
using ckks::rt::Admitted;
using ckks::rt::Arena;

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      fprintf(stderr, "FAILED %s at line %d\n", #c, __LINE__);      \
      exit(1);                                                      \
    }                                                               \
  } while (0)

// Arena against a unit bitmap: ranges never overlap, stay inside the capacity and
// aligned, and the free space is one range again once everything is released.
static void arena_random(uint64_t seed) {
  const uint64_t unit = 256, units = 997;
  Arena a(units * unit + 100, unit);  // capacity rounds down to whole units
  CHECK(a.capacity() == units * unit);
  std::vector<int> owner(units, -1);
  std::vector<std::pair<uint64_t, uint64_t>> live;  // offset, units
  std::mt19937_64 rng(seed);
  for (int step = 0; step < 20000; step++) {
    if (live.empty() || rng() % 3 != 0) {
      const uint64_t bytes = rng() % (40 * unit);
      uint64_t off = 0;
      const uint64_t need = (bytes ? bytes : 1 + 0) + unit - 1;
      const uint64_t nu = need / unit;
      // does a free run of nu units exist in the bitmap?
      bool exists = false;
      for (uint64_t i = 0, run = 0; i < units && !exists; i++) {
        run = owner[i] < 0 ? run + 1 : 0;
        exists = run >= nu;
      }
      const bool ok = a.alloc(bytes, &off);
      CHECK(ok == exists);  // first fit finds a range whenever one exists
      if (!ok) continue;
      CHECK(off % unit == 0 && off / unit + nu <= units);
      for (uint64_t i = off / unit; i < off / unit + nu; i++) {
        CHECK(owner[i] < 0);
        owner[i] = step;
      }
      live.push_back({off, nu});
    } else {
      const size_t k = rng() % live.size();
      CHECK(a.release(live[k].first));
      CHECK(!a.release(live[k].first + 1));  // not an allocation
      for (uint64_t i = live[k].first / unit; i < live[k].first / unit + live[k].second; i++) owner[i] = -1;
      live[k] = live.back();
      live.pop_back();
    }
    uint64_t used = 0;
    for (auto &l : live) used += l.second * unit;
    CHECK(a.used() == used);
  }
  for (auto &l : live) CHECK(a.release(l.first));
  CHECK(a.used() == 0 && a.free_ranges() == 1 && a.largest_free() == a.capacity());
}

// Admission: arrival order, slot limit, budget, and a big head blocking younger jobs.
static void admission_order() {
  Admission adm(1000 * 256, 2, 256);
  CHECK(adm.fits_ever(1000 * 256) && !adm.fits_ever(1000 * 256 + 1));
  std::vector<Admitted> out;
  adm.push(1, 600 * 256);
  adm.push(2, 300 * 256);
  adm.push(3, 50 * 256);
  CHECK(adm.admit(out) == 2);  // two slots
  CHECK(out[0].id == 1 && out[1].id == 2 && out[0].offset == 0 && out[1].offset == 600 * 256);
  CHECK(adm.admit(out) == 0);  // no slot for job 3 although it fits
  adm.push(4, 900 * 256);
  CHECK(adm.finish(out[1].offset));  // job 2 done: job 3 starts, job 4 must wait for space
  CHECK(adm.admit(out) == 1 && out[2].id == 3);
  CHECK(adm.finish(out[2].offset));
  adm.push(5, 10 * 256);
  CHECK(adm.admit(out) == 0);  // job 4 (head) does not fit; job 5 must not overtake it
  CHECK(adm.queued() == 2);
  CHECK(adm.finish(out[0].offset));  // everything free: job 4 then job 5
  CHECK(adm.admit(out) == 2 && out[3].id == 4 && out[4].id == 5);
  CHECK(!adm.finish(12345));
  // cancelling one queued job removes it alone, keeping the others' order
  adm.push(7, 256);
  adm.push(8, 256);
  adm.push(9, 256);
  CHECK(adm.cancel(8) && !adm.cancel(8) && !adm.cancel(12345) && adm.queued() == 3 - 1);
  CHECK(adm.finish(out[3].offset));
  std::vector<Admitted> more;
  CHECK(adm.admit(more) == 1 && more[0].id == 7);
  CHECK(adm.finish(more[0].offset));
  CHECK(adm.admit(more) == 1 && more[1].id == 9);
  CHECK(adm.finish(more[1].offset));
  CHECK(adm.admit(more) == 0);
  out[3] = {0, 0};
  std::vector<uint64_t> dropped;
  adm.push(6, 256);
  adm.cancel_queued(dropped);
  CHECK(dropped.size() == 1 && dropped[0] == 6 && adm.queued() == 0);
  CHECK(adm.finish(out[4].offset));
  CHECK(adm.arena().used() == 0 && adm.free_slots() == 2);
}

// Simulated serving: random job sizes, completions in random order; the bytes in use
// never exceed the budget and every job starts exactly once, in arrival order.
static void admission_simulation(uint64_t seed) {
  std::mt19937_64 rng(seed);
  const uint64_t budget = 64ull << 20;
  Admission adm(budget, 5);
  std::vector<Admitted> running, started;
  uint64_t next = 1, expect = 1;
  for (int step = 0; step < 5000; step++) {
    if (rng() % 2) adm.push(next++, 1 + rng() % (budget / 3));
    std::vector<Admitted> now;
    adm.admit(now);
    for (auto &a : now) {
      CHECK(a.id == expect++);
      running.push_back(a);
    }
    CHECK(adm.arena().used() <= budget && running.size() <= 5);
    if (!running.empty() && rng() % 2) {
      const size_t k = rng() % running.size();
      CHECK(adm.finish(running[k].offset));
      running[k] = running.back();
      running.pop_back();
    }
  }
}

// Backfilling: while the head waits for space, younger jobs that fit start ahead of it,
// each queued job overtaken at most max_bypass times; then strict order until it starts.
static void admission_backfill() {
  Admission adm(100 * 256, 8, 256, 2);
  std::vector<Admitted> out;
  adm.push(1, 60 * 256);
  CHECK(adm.admit(out) == 1 && out[0].id == 1);  // 40 units left
  adm.push(2, 50 * 256);                         // does not fit yet
  adm.push(3, 10 * 256);
  adm.push(4, 10 * 256);
  adm.push(5, 10 * 256);
  CHECK(adm.admit(out) == 2 && out[1].id == 3 && out[2].id == 4);  // job 2 overtaken twice
  CHECK(adm.backfilled() == 2 && adm.queued() == 2);
  CHECK(adm.admit(out) == 0);  // job 5 fits (10 left) but job 2 has no bypass left
  CHECK(adm.finish(out[0].offset));  // 70 free: job 2 starts, then job 5
  CHECK(adm.admit(out) == 2 && out[3].id == 2 && out[4].id == 5);
  for (int i = 1; i <= 4; i++) CHECK(adm.finish(out[i].offset));
  CHECK(adm.arena().used() == 0);
  // a younger job that does not fit either keeps its own budget for later ones
  Admission b(100 * 256, 8, 256, 1);
  std::vector<Admitted> o;
  b.push(10, 90 * 256);
  CHECK(b.admit(o) == 1);  // 10 left
  b.push(11, 50 * 256);    // waits
  b.push(12, 20 * 256);    // does not fit either
  b.push(13, 5 * 256);     // fits: overtakes 11 and 12 (each once)
  b.push(14, 5 * 256);     // would fit, but 11 and 12 have used their single bypass
  CHECK(b.admit(o) == 1 && o[1].id == 13);
  CHECK(b.admit(o) == 0 && b.queued() == 3);
  CHECK(b.finish(o[0].offset) && b.finish(o[1].offset));
  CHECK(b.admit(o) == 3 && o[2].id == 11 && o[3].id == 12 && o[4].id == 14);
}

// Simulated serving with backfilling: the budget holds, every job starts exactly once, and
// no job is overtaken more than max_bypass times.
static void admission_backfill_simulation(uint64_t seed, uint32_t max_bypass) {
  std::mt19937_64 rng(seed);
  const uint64_t budget = 64ull << 20;
  Admission adm(budget, 6, 256, max_bypass);
  std::vector<Admitted> running;
  std::vector<uint64_t> start_order;
  uint64_t next = 1;
  for (int step = 0; step < 5000; step++) {
    if (rng() % 2) adm.push(next++, 1 + rng() % (budget / 2));
    std::vector<Admitted> now;
    adm.admit(now);
    for (auto &a : now) {
      start_order.push_back(a.id);
      running.push_back(a);
    }
    CHECK(adm.arena().used() <= budget && running.size() <= 6);
    if (!running.empty() && rng() % 2) {
      const size_t k = rng() % running.size();
      CHECK(adm.finish(running[k].offset));
      running[k] = running.back();
      running.pop_back();
    }
  }
  // job j is overtaken by every younger job that started before it
  for (size_t i = 0; i < start_order.size(); i++) {
    uint32_t over = 0;
    for (size_t k = 0; k < i; k++) over += start_order[k] > start_order[i] ? 1 : 0;
    CHECK(over <= max_bypass);
  }
  std::vector<uint64_t> sorted = start_order;  // each job at most once; queued ones later
  std::sort(sorted.begin(), sorted.end());
  for (size_t i = 0; i < sorted.size(); i++) CHECK(sorted[i] >= 1 && sorted[i] < next && (i == 0 || sorted[i] > sorted[i - 1]));
  CHECK(sorted.size() + adm.queued() == next - 1);
}

int main() {
  for (uint64_t s = 1; s <= 5; s++) arena_random(s);
  admission_order();
  for (uint64_t s = 1; s <= 5; s++) admission_simulation(s);
  admission_backfill();
  for (uint64_t s = 1; s <= 5; s++) admission_backfill_simulation(s, (uint32_t)(s * 3));
  printf("OK\n");
  return 0;
}
