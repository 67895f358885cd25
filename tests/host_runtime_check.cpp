// CPU check of the serving runtime's host bookkeeping (csrc/host_pool.h), built by
// tests/test_host_runtime.py with AddressSanitizer and UndefinedBehaviorSanitizer.
//
//  1. Pool: random allocations and releases against a granule map.  Every range the
//     pool hands out lies inside it, overlaps no live range, and is the lowest-addressed
//     free run that fits (first fit); the free list stays consistent (sorted, no two
//     adjacent ranges: releases coalesce); the peak is the largest amount in use; once
//     everything is released one free range spans the pool.
//  2. Admission: a FIFO of random requests (some larger than the budget) against a
//     device pool, a result pool, instance slots and a work-item cap, with random
//     completions.  Oversized requests are rejected at once, the head of the queue is
//     admitted only when every resource fits (nothing is held while it waits), device
//     memory in use never exceeds the budget, requests are admitted in arrival order,
//     and every admitted request completes and gives its memory back.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "host_pool.h"

using mapi::Admission;
using mapi::Pool;

#define CHECK(cond)                                                          \
  do {                                                                       \
    if (!(cond)) {                                                           \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      std::exit(1);                                                          \
    }                                                                        \
  } while (0)

static int pool_check(unsigned seed) {
  const size_t G = mapi::kPoolGranule, granules = 4096;
  Pool p;
  p.reset(granules * G + 100);   // a ragged size rounds down to whole granules
  CHECK(p.size() == granules * G && p.consistent());
  std::vector<int> owner(granules, -1);   // granule -> live allocation id
  struct Live { size_t off, bytes; };
  std::vector<Live> live;
  std::mt19937_64 rng(seed);
  size_t used = 0, peak = 0;
  for (int step = 0; step < 200000; ++step) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const size_t bytes = 1 + rng() % (64 * G);   // up to 64 granules, ragged
      const size_t need = mapi::pool_round(bytes) / G;
      // the model's first fit
      size_t run = 0, expect = SIZE_MAX;
      for (size_t g = 0; g < granules; ++g) {
        run = owner[g] < 0 ? run + 1 : 0;
        if (run == need) { expect = (g + 1 - need) * G; break; }
      }
      size_t off = 0;
      const bool ok = p.alloc(bytes, &off);
      CHECK(ok == (expect != SIZE_MAX));
      if (!ok) continue;
      CHECK(off == expect);
      for (size_t g = off / G; g < off / G + need; ++g) {
        CHECK(g < granules && owner[g] < 0);
        owner[g] = (int)live.size();
      }
      live.push_back({off, bytes});
      used += need * G;
      peak = std::max(peak, used);
    } else {
      const size_t k = rng() % live.size();
      const Live l = live[k];
      const size_t need = mapi::pool_round(l.bytes) / G;
      for (size_t g = l.off / G; g < l.off / G + need; ++g) owner[g] = -1;
      p.release(l.off, l.bytes);
      live[k] = live.back();
      live.pop_back();
      for (size_t i = 0; i < live.size(); ++i)   // ids follow positions
        for (size_t g = live[i].off / G; g < live[i].off / G + mapi::pool_round(live[i].bytes) / G; ++g) owner[g] = (int)i;
      used -= need * G;
    }
    CHECK(p.used() == used && p.peak() == peak);
    if (step % 997 == 0) CHECK(p.consistent());
  }
  for (const Live& l : live) p.release(l.off, l.bytes);
  CHECK(p.used() == 0 && p.consistent() && p.free_ranges() == 1);
  return 0;
}

static int admission_check(unsigned seed) {
  const size_t G = mapi::kPoolGranule;
  const size_t budget = 2048 * G, out_size = 512 * G;
  const int slots = 16;
  const uint64_t tile_cap = 64;
  Pool dev, out;
  dev.reset(budget);
  out.reset(out_size);
  struct Req { size_t dev_bytes, out_bytes; uint64_t tiles; size_t dev_off = 0, out_off = 0; int id; };
  std::mt19937_64 rng(seed);
  std::deque<Req> queue;
  std::vector<Req> running;
  int next_id = 0, next_admit = 0, rejected = 0, completed = 0, admitted = 0;
  std::vector<int> rejected_ids;
  uint64_t live_tiles = 0;
  for (int step = 0; step < 100000; ++step) {
    if (rng() % 3 == 0) {   // arrivals: every 50th is larger than the budget
      Req r;
      r.id = next_id++;
      r.dev_bytes = (r.id % 50 == 49) ? budget + 1 + rng() % budget : 1 + rng() % (400 * G);
      r.out_bytes = 4 * (1 + rng() % (40 * G / 4));
      r.tiles = 1 + rng() % 16;
      queue.push_back(r);
    }
    // admit from the head while possible
    while (!queue.empty()) {
      Req& h = queue.front();
      const Admission a = mapi::admit_request(dev, out, budget, h.dev_bytes, h.out_bytes,
                                              (int)running.size() < slots, live_tiles, h.tiles, tile_cap,
                                              &h.dev_off, &h.out_off);
      if (a == Admission::kReject) {
        CHECK(h.dev_bytes > budget);
        rejected_ids.push_back(h.id);
        ++rejected;
        queue.pop_front();
        continue;
      }
      if (a == Admission::kWait) {
        CHECK(h.dev_bytes <= budget);
        break;
      }
      CHECK(h.id >= next_admit);        // arrival order (rejected ids are skipped)
      next_admit = h.id + 1;
      live_tiles += h.tiles;
      running.push_back(h);
      ++admitted;
      queue.pop_front();
    }
    CHECK(dev.used() <= budget && out.used() <= out_size && (int)running.size() <= slots && live_tiles <= tile_cap);
    // completions
    if (!running.empty() && rng() % 2 == 0) {
      const size_t k = rng() % running.size();
      dev.release(running[k].dev_off, running[k].dev_bytes);
      out.release(running[k].out_off, running[k].out_bytes);
      live_tiles -= running[k].tiles;
      running[k] = running.back();
      running.pop_back();
      ++completed;
    }
  }
  for (const Req& r : running) {
    dev.release(r.dev_off, r.dev_bytes);
    out.release(r.out_off, r.out_bytes);
    ++completed;
  }
  CHECK(completed == admitted && admitted > 1000 && rejected > 0);
  for (int id : rejected_ids) CHECK(id % 50 == 49);
  CHECK(dev.used() == 0 && out.used() == 0 && dev.consistent() && out.consistent());
  CHECK(dev.peak() <= budget);
  return 0;
}

int main() {
  for (unsigned seed : {1u, 2u, 3u}) {
    pool_check(seed);
    admission_check(seed);
  }
  std::printf("host runtime checks passed\n");
  return 0;
}
