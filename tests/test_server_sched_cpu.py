"""CPU tests of the serving scheduler (admission, slot reuse, ordering, heap)
through l0cim_server_sim_*, the scheduler object the server drives around
its launches, here with no device: the executor is the caller's clock.

Expected behaviour, stated by the server's contract: requests are admitted in
arrival order while a slot is free, the request's block fits (first fit)
and, when a step budget is set and something is resident, the resident
couplings stay within it; the first request that does not fit stops
admission; each tick advances every resident request by one alternation and
retires those that have done n_outer, returning their slot and block.
"""
from ctypes import byref, c_int32, c_int64, c_size_t, c_void_p

import paper_2405_00366_amd as L


def _lib():
    return L.lib()


class Sim:
    def __init__(self, slots, max_n, heap_requests=None, arena=None, n_outer=3, replicas=8, budget=0):
        self.lib = _lib()
        self.sp = L.solve_params(n_outer=n_outer, velo=n_outer, replicas=replicas)
        over = self.lib.l0cim_server_arena_overhead(slots, max_n, byref(self.sp))
        if arena is None:
            arena = over + sum(self.bytes(m, n) for m, n in heap_requests) + 256
        self.h = c_void_p()
        assert self.lib.l0cim_server_sim_create(byref(self.sp), slots, max_n, arena, byref(self.h)) == 0
        if budget:
            assert self.lib.l0cim_server_sim_set_step_budget(self.h, budget) == 0
        self.t = 0.0

    def bytes(self, m, n):
        return self.lib.l0cim_server_request_bytes(m, n, byref(self.sp))

    def submit(self, m, n, tag):
        return self.lib.l0cim_server_sim_submit(self.h, m, n, tag, self.t)

    def tick(self, dur=1.0):
        a, c = c_int32(), c_int32()
        assert self.lib.l0cim_server_sim_tick(self.h, self.t, self.t + dur, byref(a), byref(c)) == 0
        self.t += dur
        return a.value, c.value

    def done(self):
        out = (L.Completion * 64)()
        k = self.lib.l0cim_server_sim_completed(self.h, out, 64)
        return [(out[i].tag, out[i].t_admit, out[i].t_finish) for i in range(k)]

    def resident(self):
        tags, slots, offs, alts = (c_int64 * 64)(), (c_int32 * 64)(), (c_size_t * 64)(), (c_int32 * 64)()
        k = self.lib.l0cim_server_sim_resident(self.h, tags, slots, offs, alts, 64)
        return [(tags[i], slots[i], offs[i], alts[i]) for i in range(k)]

    def info(self):
        a, p, u, hb, fb = c_int32(), c_int32(), c_size_t(), c_size_t(), c_int32()
        assert self.lib.l0cim_server_sim_info(self.h, byref(a), byref(p), byref(u), byref(hb), byref(fb)) == 0
        return a.value, p.value, u.value, hb.value, fb.value

    def __del__(self):
        self.lib.l0cim_server_sim_destroy(self.h)


def test_slots_limit_residency_and_are_reused_in_arrival_order():
    s = Sim(slots=2, max_n=1024, heap_requests=[(256, 512)] * 5, n_outer=3)
    for tag in range(5):
        assert s.submit(256, 512, tag) == 0
    assert s.tick() == (2, 0)                    # two slots: requests 0 and 1
    assert [r[0] for r in s.resident()] == [0, 1] and sorted(r[1] for r in s.resident()) == [0, 1]
    assert s.tick() == (0, 0)
    assert s.tick() == (0, 2)                    # three alternations each
    assert [d[0] for d in s.done()] == [0, 1]
    assert s.info()[:2] == (0, 3)
    assert s.tick() == (2, 0)                    # slots reused by 2 and 3
    assert [r[0] for r in s.resident()] == [2, 3]
    s.tick(), s.tick()
    assert [d[0] for d in s.done()] == [2, 3]
    s.tick(), s.tick(), s.tick()
    done = s.done()
    assert [d[0] for d in done] == [4]
    assert done[0][1] == 6.0 and done[0][2] == 9.0   # admitted at the start of tick 7, finished at the end of tick 9
    assert s.info() == (0, 0, 0, s.info()[3], 1)     # every byte back, one free extent


def test_head_of_line_request_that_does_not_fit_stops_admission():
    big, small = (2000, 4096), (200, 512)
    s = Sim(slots=8, max_n=4096, arena=None, heap_requests=[big, small], n_outer=2)
    heap = s.info()[3]
    assert s.bytes(*big) + 2 * s.bytes(*small) > heap >= s.bytes(*big) + s.bytes(*small)
    assert s.submit(*small, 0) == 0
    assert s.submit(*big, 1) == 0
    assert s.submit(*small, 2) == 0             # would fit beside 0, but 1 is ahead of it
    assert s.tick() == (2, 0)                   # 0 and 1
    assert [r[0] for r in s.resident()] == [0, 1]
    assert s.tick() == (0, 2)
    assert s.tick() == (1, 0)
    assert [r[0] for r in s.resident()] == [2]


def test_step_budget_keeps_one_large_request_resident_at_a_time():
    n = 4096
    cost = 4096 * 4096 * 4                      # FP32 couplings streamed per Euler step
    s = Sim(slots=8, max_n=n, heap_requests=[(2000, n)] * 3, n_outer=1, budget=int(1.5 * cost))
    for tag in range(3):
        s.submit(2000, n, tag)
    assert s.tick() == (1, 1)                   # a second one would exceed the budget
    assert s.tick() == (1, 1)
    assert s.tick() == (1, 1)
    assert [d[0] for d in s.done()] == [0, 1, 2]


def test_budget_does_not_block_an_idle_server():
    s = Sim(slots=2, max_n=4096, heap_requests=[(2000, 4096)], n_outer=1, budget=1)
    s.submit(2000, 4096, 7)
    assert s.tick() == (1, 1)


def test_heap_first_fit_and_coalescing():
    sizes = [(100, 512), (400, 2048), (100, 512)]
    s = Sim(slots=4, max_n=2048, heap_requests=sizes, n_outer=1)
    for tag, (m, n) in enumerate(sizes):
        s.submit(m, n, tag)
    s.tick()
    assert s.info()[2] == 0 and s.info()[4] == 1
    # a mix that finishes at different times leaves holes that coalesce back
    s2 = Sim(slots=4, max_n=2048, heap_requests=sizes, n_outer=2)
    s2.submit(*sizes[0], 0)
    s2.tick()                                    # 0 resident (alt 1 next)
    s2.submit(*sizes[1], 1)
    s2.submit(*sizes[2], 2)
    s2.tick()                                    # 1, 2 admitted; 0 finishes
    res = {r[0]: r for r in s2.resident()}
    assert set(res) == {1, 2}
    assert s2.info()[4] == 2                     # the hole of 0 and the tail
    s2.tick()
    a, p, used, heap, blocks = s2.info()
    assert (a, p, used, blocks) == (0, 0, 0, 1)


def test_rejects_requests_the_arena_cannot_hold():
    s = Sim(slots=2, max_n=4096, heap_requests=[(100, 512)], n_outer=1)
    assert s.submit(2000, 4096, 1) == 3          # L0CIM_ERR_WORKSPACE
    assert s.submit(100, 5000, 2) == 2           # above max_n
    assert s.submit(0, 512, 3) == 2
    assert s.info()[1] == 0
