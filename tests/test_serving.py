"""Serving scheduler on the host with a fake executor and a virtual clock:
batching, admission, eviction, latency accounting and the request stream."""
import math

import numpy as np
import pytest

from paper_1811_00355_amd import serving as S


class FakeExecutor:
    """Virtual clock; setup costs V * 1e-6 s, a solve 1e-3 + V * nrhs * 1e-8 s.
    Results are a pure function of (request seed, rhs index)."""

    def __init__(self, per_field_bytes=10, ws_per_rhs=1):
        self.t = 0.0
        self.loads, self.frees, self.batches = [], [], []
        self.pfb, self.wpr = per_field_bytes, ws_per_rhs

    def footprint(self, f):
        return self.pfb

    def transient(self, f):
        return 0

    def workspace(self, f, nrhs):
        return self.wpr * nrhs

    def load(self, f):
        self.loads.append(f.key)
        self.t += f.V * 1e-6
        return f.key

    def solve(self, h, f, reqs):
        nrhs = sum(r.nrhs for r in reqs)
        self.batches.append((f.key, [r.rid for r in reqs], nrhs))
        self.t += 1e-3 + f.V * nrhs * 1e-8
        return [[(r.src_seed * 31 + j) % 97 * 1e-13 for j in range(r.nrhs)] for r in reqs]

    def free(self, h):
        self.frees.append(h)

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


def F(key, L=(8, 8, 8, 8)):
    return S.FieldSpec(key, L, 0.2, -0.2, 1)


def R(rid, t, f, nrhs):
    return S.Request(rid, t, f, nrhs, 1000 + rid)


def test_continuous_batching_groups_waiting_requests_of_one_field():
    a, b = F("a"), F("b")
    # all waiting at t = 0: a-requests are merged in arrival order up to 12 rhs
    reqs = [R(0, 0.0, a, 5), R(1, 0.0, b, 3), R(2, 0.0, a, 6), R(3, 0.0, a, 4), R(4, 0.0, b, 2)]
    ex = FakeExecutor()
    done = S.Server(ex, 1000).run(reqs)
    assert ex.batches[0] == ("a", [0, 2], 11)        # 5 + 6; the next a-request (4) would exceed 12
    assert ex.batches[1] == ("b", [1, 4], 5)
    assert ex.batches[2] == ("a", [3], 4)
    assert sorted(d.rid for d in done) == [0, 1, 2, 3, 4]
    # results do not depend on the batch a request ran in
    alone = {}
    for r in reqs:
        ex1 = FakeExecutor()
        alone[r.rid] = S.Server(ex1, 1000).run([S.Request(r.rid, 0.0, r.field, r.nrhs, r.src_seed)])[0].relres
    assert all(d.relres == alone[d.rid] for d in done)


def test_setup_cache_and_lru_eviction():
    fa, fb, fc = F("a"), F("b"), F("c")
    # budget holds two fields (10 B each) plus a 3-rhs workspace
    reqs = [R(0, 0.0, fa, 1), R(1, 1.0, fb, 1), R(2, 2.0, fa, 1), R(3, 3.0, fc, 1), R(4, 4.0, fa, 1),
            R(5, 5.0, fb, 1)]
    ex = FakeExecutor()
    srv = S.Server(ex, 23)
    done = srv.run(reqs)
    assert ex.loads == ["a", "b", "c", "b"]         # c evicts b (least recently used); b is loaded again
    assert ex.frees == ["b", "c"]
    assert srv.evictions == 2
    miss = {d.rid: d.setup_miss for d in done}
    assert miss == {0: True, 1: True, 2: False, 3: True, 4: False, 5: True}


def test_admission_rejects_what_cannot_fit():
    ex = FakeExecutor(per_field_bytes=10, ws_per_rhs=5)
    srv = S.Server(ex, 30)
    done = srv.run([R(0, 0.0, F("a"), 2), R(1, 0.0, F("b"), 5), R(2, 0.0, F("c"), 4)])
    assert srv.rejected == [1]                       # 10 + 25 > 30
    assert sorted(d.rid for d in done) == [0, 2]


def test_latency_is_arrival_to_finish_with_idle_gaps():
    f = F("a", (4, 4, 4, 4))
    reqs = [R(0, 0.5, f, 2), R(1, 10.0, f, 1)]
    ex = FakeExecutor()
    done = {d.rid: d for d in S.Server(ex, 100).run(reqs)}
    setup, solve2, solve1 = 256e-6, 1e-3 + 256 * 2e-8, 1e-3 + 256e-8
    assert done[0].start == pytest.approx(0.5)
    assert done[0].latency == pytest.approx(setup + solve2)
    assert done[1].latency == pytest.approx(solve1)   # cached field, idle device
    s = S.summarize(list(done.values()), 10.0 + solve1)
    assert s["requests"] == 2 and s["rhs"] == 3 and s["setup_misses"] == 1


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
    import pytest
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
