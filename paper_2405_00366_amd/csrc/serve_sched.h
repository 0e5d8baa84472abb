// Host-side scheduling of the serving form, with no device work: the arena
// heap (first fit, coalescing free list), the slot table, the arrival queue,
// admission and retirement.  The server (server.hip) drives it around its
// launches; the simulation entry points (l0cim_server_sim_*) drive the same
// object with no device, so its behaviour can be tested and an arena sized
// on the host.
//
// Admission, at the start of a tick: requests leave the queue in arrival
// order while a slot is free and the request's block fits in the heap, and,
// when a step budget is set and something is resident, while the couplings
// bytes one Euler step of the resident set streams stay within the budget;
// the first request that does not fit stops admission (no overtaking).
// Retirement, at the end of a tick: every resident request has done one more
// alternation; those that have done all n_outer are finished, their block
// and slot returned; the rest move on.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace l0 {

// R must have: size_t bytes, cost, off; int slot, alt; double t_admit.
template <class R>
struct ServeSched {
  int max_slots = 0, n_outer = 1;
  size_t heap_bytes = 0, in_use = 0, step_budget = 0, step_active = 0;
  std::map<size_t, size_t> free_blocks;   // offset -> bytes, coalesced
  std::deque<R> pending;
  std::vector<R> active;
  std::vector<int> free_slots;

  void init(int slots, size_t heap_base, size_t heap, int outer) {
    max_slots = slots;
    n_outer = outer;
    heap_bytes = heap;
    free_blocks.clear();
    if (heap) free_blocks[heap_base] = heap;
    free_slots.clear();
    for (int k = slots - 1; k >= 0; --k) free_slots.push_back(k);   // slot 0 is handed out first
  }

  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_blocks.erase(it);
        if (rest) free_blocks[at] = rest;
        in_use += bytes;
        return true;
      }
    }
    return false;
  }

  void release(size_t off, size_t bytes) {
    in_use -= bytes;
    auto it = free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_blocks.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blocks.erase(nx);
    }
    if (it != free_blocks.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blocks.erase(it);
      }
    }
  }

  // Admits what fits; returns how many requests joined the resident set (they
  // are the last entries of `active`, in arrival order).
  int admit(double now) {
    int added = 0;
    while (!pending.empty() && !free_slots.empty()) {
      R& r = pending.front();
      if (step_budget && !active.empty() && step_active + r.cost > step_budget) break;
      size_t off = 0;
      if (!alloc(r.bytes, &off)) break;
      step_active += r.cost;
      r.off = off;
      r.slot = free_slots.back();
      free_slots.pop_back();
      r.alt = 0;
      r.t_admit = now;
      active.push_back(r);
      pending.pop_front();
      ++added;
    }
    return added;
  }

  bool finishing(const R& r) const { return r.alt + 1 >= n_outer; }

  // Ends a tick: the finished requests go to `done` (in resident order), their
  // blocks and slots are returned; the others advance one alternation.
  void retire(std::vector<R>& done) {
    std::vector<R> keep;
    keep.reserve(active.size());
    for (R& r : active) {
      if (finishing(r)) {
        release(r.off, r.bytes);
        step_active -= r.cost;
        free_slots.push_back(r.slot);
        done.push_back(r);
      } else {
        ++r.alt;
        keep.push_back(r);
      }
    }
    active.swap(keep);
  }
};

}  // namespace l0
