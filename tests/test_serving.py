"""Serving scheduler on the host with a fake executor and a virtual clock:
lanes that overlap, joins at restart boundaries, slot reuse, admission with
reservations, eviction, failure handling, latency accounting and the request
stream."""
import math

import numpy as np
import pytest

from paper_1811_00355_amd import serving as S


class FakeExecutor:
    """Virtual clock; lanes run concurrently.  A setup costs V * 1e-6 s, a step
    1e-3 + V * 1e-8 s per running slot.  Right-hand side j of a request finishes
    after 1 + (seed + j) % 3 steps with residual ((seed * 31 + j) % 97) * 1e-13,
    a pure function of the request."""

    def __init__(self, footprints=None, ws_per_rhs=1, transient=0, fail_open=(), oom_once=()):
        self.t = 0.0
        self.pending = []                # (t_end, seq, kind, lid, payload, error)
        self.seq = 0
        self.fp = footprints or {}
        self.wpr, self.tr = ws_per_rhs, transient
        self.fail_open = set(fail_open)
        self.oom_once = set(oom_once)     # the first open on these fields meets a full device
        self.loads, self.frees, self.steps, self.opens = [], [], [], []
        self.lanes = {}                  # lid -> (field, {slot: [steps left, relres]})
        self.busy_until = {}

    def footprint(self, f):
        return self.fp.get(f.key, 10)

    def transient(self, f):
        return self.tr

    def workspace(self, f, nrhs):
        return self.wpr * nrhs

    def _push(self, lid, dur, kind, payload, error=None):
        t0 = max(self.t, self.busy_until.get(lid, 0.0))
        self.busy_until[lid] = t0 + dur
        self.pending.append((t0 + dur, self.seq, kind, lid, payload, error))
        self.seq += 1
        return t0

    def open(self, lid, f, handle, capacity):
        self.opens.append((lid, f.key, capacity, handle is None))
        self.lanes[lid] = (f, {})
        if f.key in self.fail_open:
            self._push(lid, 0.0, "open", None, RuntimeError("setup failed"))
            return
        if f.key in self.oom_once:
            self.oom_once.discard(f.key)
            self._push(lid, 0.0, "open", None, MemoryError("out of device memory"))
            return
        dur = 0.0
        if handle is None:
            self.loads.append(f.key)
            handle, dur = f.key, f.V * 1e-6
        self._push(lid, dur, "open", handle)

    def step(self, lid, adds):
        f, slots = self.lanes[lid]
        for slot, r, j in adds:
            assert slot not in slots
            slots[slot] = [1 + (r.src_seed + j) % 3, ((r.src_seed * 31 + j) % 97) * 1e-13]
        dur = 1e-3 + f.V * 1e-8 * len(slots)
        out = {}
        for slot in list(slots):
            slots[slot][0] -= 1
            if slots[slot][0] == 0:
                out[slot] = slots.pop(slot)[1]
        t0 = self._push(lid, dur, "step", out)
        self.steps.append((lid, t0, t0 + dur, [a[1].rid for a in adds]))

    def close(self, lid):
        self._push(lid, 0.0, "close", None)

    def free(self, h):
        self.frees.append(h)

    def now(self):
        return self.t

    def wait_event(self, deadline):
        if self.pending:
            ev = min(self.pending)
            if deadline is None or ev[0] <= deadline:
                self.pending.remove(ev)
                self.t = max(self.t, ev[0])
                return (ev[2], ev[3], ev[4], ev[5], self.t)
        assert deadline is not None, "scheduler waits with nothing in flight"
        self.t = max(self.t, deadline)
        return None


def F(key, L=(8, 8, 8, 8)):
    return S.FieldSpec(key, L, 0.2, -0.2, 1)


def R(rid, t, f, nrhs, seed=None):
    return S.Request(rid, t, f, nrhs, 1000 + rid if seed is None else seed)


def expected_relres(r):
    return [((r.src_seed * 31 + j) % 97) * 1e-13 for j in range(r.nrhs)]


def test_lanes_on_different_fields_overlap_and_same_field_arrivals_join():
    a, b = F("a"), F("b")
    # r2 arrives while lane a runs its first restart cycle and joins at the next boundary
    reqs = [R(0, 0.0, a, 3), R(1, 0.0, b, 2), R(2, 0.005, a, 2)]
    ex = FakeExecutor()
    srv = S.Server(ex, 1000)
    done = {d.rid: d for d in srv.run(reqs)}
    assert sorted(done) == [0, 1, 2]
    assert ex.loads == ["a", "b"]                      # one setup per field
    assert [o[1] for o in ex.opens] == ["a", "b"]      # no second lane for a
    assert done[2].lane == done[0].lane and done[2].joined and not done[0].joined
    assert done[2].start == pytest.approx(4096e-6 + 1e-3 + 4096e-8 * 3)   # the end of a's first step
    assert not done[2].setup_miss and done[0].setup_miss
    # the two lanes' steps overlap in time
    ivs = [(lid, t0, t1) for lid, t0, t1, _ in ex.steps]
    assert S.overlap_seconds(ivs) > 0
    for d in done.values():
        assert d.relres == expected_relres(next(r for r in reqs if r.rid == d.rid))
    assert srv.inuse == 0 and not srv.lanes


def test_slots_are_reused_by_waiting_requests():
    a = F("a")
    reqs = [R(0, 0.0, a, 3, seed=0), R(1, 0.0, a, 3, seed=1), R(2, 0.0, a, 1, seed=2)]
    ex = FakeExecutor()
    srv = S.Server(ex, 1000, max_rhs=4)
    done = {d.rid: d for d in srv.run(reqs)}
    assert len(ex.opens) == 1 and ex.opens[0][2] == 4  # one lane of 4 slots
    # r0 (3) and r2 (1) fill it; r1 (3) joins once three slots are free again
    assert ex.steps[0][3] == [0, 0, 0, 2]
    assert done[1].joined and done[1].start > 0
    assert any(st[3] == [1, 1, 1] for st in ex.steps)
    for r in reqs:
        assert done[r.rid].relres == expected_relres(r)
    assert max(d.batch_rhs for d in done.values()) <= 4


def test_admission_waits_for_memory_and_honours_the_reservation():
    a, b, c = F("a"), F("b"), F("c")
    ex = FakeExecutor(footprints={"a": 10, "b": 10, "c": 1}, ws_per_rhs=5)
    srv = S.Server(ex, 40, max_rhs=4, backfill_bytes=0)
    # lane a takes 10 + 4 * 5 = 30; b needs 10 + 2 * 5 = 20 and waits, holding a
    # reservation; c (1 + 5) would fit in the 10 left but must not pass b
    done = {d.rid: d for d in srv.run([R(0, 0.0, a, 2), R(1, 0.0, b, 2), R(2, 0.0, c, 1)])}
    assert sorted(done) == [0, 1, 2] and not srv.rejected
    assert done[1].start >= done[0].finish - 1e-12
    assert done[2].start >= done[1].start
    assert srv.peak_bytes <= 40


def test_setup_cache_and_lru_eviction():
    fa, fb, fc = F("a"), F("b"), F("c")
    # budget holds two fields (10 B each) plus a 3-slot workspace; requests are spaced so lanes close in between
    reqs = [R(0, 0.0, fa, 1), R(1, 1.0, fb, 1), R(2, 2.0, fa, 1), R(3, 3.0, fc, 1), R(4, 4.0, fa, 1),
            R(5, 5.0, fb, 1)]
    ex = FakeExecutor()
    srv = S.Server(ex, 23, max_rhs=3)
    done = srv.run(reqs)
    assert ex.loads == ["a", "b", "c", "b"]         # c evicts b (least recently used); b is loaded again
    assert ex.frees == ["b", "c"]
    assert srv.evictions == 2
    miss = {d.rid: d.setup_miss for d in done}
    assert miss == {0: True, 1: True, 2: False, 3: True, 4: False, 5: True}
    assert srv.peak_bytes <= 23


def test_lane_capacity_shrinks_before_a_cached_field_is_evicted():
    a, b = F("a"), F("b")
    ex = FakeExecutor(ws_per_rhs=5)
    srv = S.Server(ex, 35, max_rhs=4)
    # after a's lane closes, a full lane on b (10 + 4 * 5) would need a's 10 B;
    # a lane sized for the waiting batch (10 + 5) fits beside it
    done = srv.run([R(0, 0.0, a, 1), R(1, 1.0, b, 1)])
    assert len(done) == 2 and ex.frees == [] and srv.evictions == 0
    assert [o[2] for o in ex.opens] == [4, 1]


def test_admission_rejects_what_cannot_fit():
    ex = FakeExecutor(ws_per_rhs=5)
    srv = S.Server(ex, 30)
    done = srv.run([R(0, 0.0, F("a"), 2), R(1, 0.0, F("b"), 5), R(2, 0.0, F("c"), 4)])
    assert srv.rejected == [1]                       # 10 + 25 > 30
    assert sorted(d.rid for d in done) == [0, 2]


def test_a_failed_setup_releases_its_reservation():
    ex = FakeExecutor(fail_open=["b"])
    srv = S.Server(ex, 1000)
    done = srv.run([R(0, 0.0, F("a"), 2), R(1, 0.0, F("b"), 3), R(2, 0.01, F("b"), 1)])
    assert srv.failed == [1, 2]                      # each lane on b fails to open; nothing else is lost
    assert [o[1] for o in ex.opens].count("b") == 2
    assert [d.rid for d in done] == [0]
    assert "b" not in srv.cache and srv.resident == 10 and srv.inuse == 0


def test_a_full_device_requeues_and_waits_for_a_lane_to_close():
    a, b = F("a", (8, 8, 8, 16)), F("b")
    ex = FakeExecutor(oom_once=["b"])
    srv = S.Server(ex, 1000)
    done = {d.rid: d for d in srv.run([R(0, 0.0, a, 2), R(1, 0.0, b, 3)])}
    assert sorted(done) == [0, 1] and not srv.failed and srv.retries == 1
    assert [o[1] for o in ex.opens] == ["a", "b", "b"]
    assert done[1].start >= done[0].finish - 1e-12   # retried once a's lane had closed
    assert srv.resident == 20 and srv.inuse == 0


def test_small_lanes_backfill_inside_a_reservation():
    a, b, c = F("a"), F("b"), F("c")
    ex = FakeExecutor(footprints={"a": 10, "b": 10, "c": 1}, ws_per_rhs=5)
    # as in the reservation test, but c's lane (1 + 5 B) is small enough to backfill
    srv = S.Server(ex, 40, max_rhs=4, backfill_bytes=6)
    done = {d.rid: d for d in srv.run([R(0, 0.0, a, 2), R(1, 0.0, b, 2), R(2, 0.0, c, 1)])}
    assert done[2].start == 0.0 and done[1].start >= done[0].finish - 1e-12
    assert srv.peak_bytes <= 40


def test_latency_is_arrival_to_finish_with_idle_gaps():
    f = F("a", (4, 4, 4, 4))
    # seeds chosen so every right-hand side finishes in its first step
    reqs = [R(0, 0.5, f, 1, seed=0), R(1, 10.0, f, 1, seed=3)]
    ex = FakeExecutor()
    done = {d.rid: d for d in S.Server(ex, 100).run(reqs)}
    setup, step = 256e-6, 1e-3 + 256e-8
    assert done[0].start == pytest.approx(0.5)
    assert done[0].latency == pytest.approx(setup + step)
    assert done[1].latency == pytest.approx(step)    # cached field, idle device
    s = S.summarize(list(done.values()), 10.0 + step)
    assert s["requests"] == 2 and s["rhs"] == 2 and s["setup_misses"] == 1


def test_overlap_seconds():
    assert S.overlap_seconds([(0, 0.0, 1.0), (1, 0.5, 2.0)]) == pytest.approx(0.5)
    assert S.overlap_seconds([(0, 0.0, 1.0), (0, 0.5, 2.0)]) == 0.0    # one lane with itself
    assert S.overlap_seconds([(0, 0.0, 1.0), (1, 1.0, 2.0)]) == 0.0
    assert S.overlap_seconds([(0, 0.0, 3.0), (1, 1.0, 2.0), (2, 1.5, 4.0)]) == pytest.approx(2.0)


def test_request_stream_statistics():
    pool = {L: [S.FieldSpec(f"{L}#{j}", L, 0.2, -0.2, j) for j in range(16)] for L in S.SHAPES}
    reqs = S.make_requests(4000, 2.0, S.SHAPES, pool, rng_seed=5001)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 0.5) < 0.03             # Poisson at 2 per second
    assert abs(np.std(gaps) / gaps.mean() - 1.0) < 0.06   # exponential gaps
    nr = np.array([r.nrhs for r in reqs])
    assert nr.min() == 1 and nr.max() == 12 and abs(nr.mean() - 6.5) < 0.2
    shapes = [r.field.L for r in reqs]
    for L in S.SHAPES:
        assert abs(shapes.count(L) / len(reqs) - 0.25) < 0.03
    # first-seen fields are fresh pool entries; later requests mostly reuse
    seen, fresh = set(), 0
    for r in reqs:
        fresh += r.field.key not in seen
        seen.add(r.field.key)
    assert fresh == 64                               # the whole pool gets issued
    closed = S.make_requests(10, math.inf, S.SHAPES, pool)
    assert all(r.arrival == 0.0 for r in closed)


def test_library_footprint_figures():
    """dd_footprint_bytes (host arithmetic, no device): the large terms of each
    figure at 32^3x64, n = 20, against the layouts they count."""
    import os
    from paper_1811_00355_amd import binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libdd.so not built")
    L, blk, n = (32, 32, 32, 64), (4, 4, 4, 4), 20
    V, Vc, nc = 32 ** 3 * 64, 8 ** 3 * 16, 40
    for store, sb in ((B.DD_F32, 8), (B.DD_BF16, 4)):
        fp = S.library_footprint(L, blk, n, store, 12)
        # FP64 links/clover/inverse, FP32 copies, half copies, block tables
        assert fp["gauge"] == V * 108 * (24 + (4 if sb == 4 else 0)) + 40 * Vc
        # P FP64 + working FP32 + stored P; D_c and inverses (9.5 blocks) in FP64 + FP32 (+ half)
        assert fp["setup"] == 12 * V * n * (16 + 8 + sb) + nc * nc * (9 * Vc + Vc // 2) * (24 + (4 if sb == 4 else 0))
        # FGMRES(10) FP64 basis and vectors, FP32 directions, V-cycle and coarse GMRES(60) vectors
        fine, coarse = 12 * V * 12, Vc * nc * 12
        core = 16 * fine * 15 + 8 * fine * 12 + 8 * coarse * 68 + 8 * coarse
        assert core < fp["workspace"] < core * 1.001
        assert 90e9 < fp["workspace"] < 110e9
        # while a setup runs: the V-cycle workspace for n vectors plus a 4 GiB Galerkin chunk at least
        assert fp["scratch"] > 4 * 2 ** 30
    with pytest.raises(B.DDError):
        B.footprint((32, 32, 32, 60), blk, B.default_params(block=blk), 1)
