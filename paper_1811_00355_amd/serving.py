"""Serving loop for Wilson-clover solves on one GPU, with continuous batching.

Requests arrive as a Poisson stream.  Each asks for `nrhs` solves D x = b on one
gauge field (lattice shape, link roughness, bare mass).  The paper's accounting
(Sec. 4: one adaptive setup per configuration, then 12 solves) is what makes a
per-field setup cache pay: the first request on a field pays for the upload
and the setup, later ones reuse them.

* Lanes: a field being solved has one lane, a solve state of `capacity` slots
  (right-hand sides) on its own HIP stream and host thread.  A lane advances
  one FGMRES restart cycle per step; lanes on different fields run at the same
  time, so their kernels overlap on the device.
* Joining: a request on a field whose lane runs and has free slots joins it at
  the lane's next restart boundary; slots freed by finished right-hand sides
  are reused.  Every reduction and mask of the solver is per slot, so a result
  has the same bits alone, in a batch, or joined mid-run.
* Setup cache: gauge field + multigrid setup stay resident on the device, keyed
  by field, least recently used idle field evicted first.
* Admission: a lane opens only when its field's footprint (if not cached), the
  scratch of its setup and the workspace of its slots fit the HBM budget beside
  the resident fields and the other lanes; the oldest request that is blocked
  for memory holds a reservation that later requests may not eat into.  A
  request that cannot fit on an empty device is rejected.
* Latency runs from arrival to the solution being back in host memory.

The scheduler is plain host logic driven through an executor object; the GPU
executor calls the library (dd_solve_begin/add/step/take/end), and tests drive
the same scheduler with a CPU fake on a virtual clock.
"""
import dataclasses
import math
import queue as _queue
import threading
import time
from collections import OrderedDict

import numpy as np


# ----------------------------------------------------------------------------
# footprint (bytes): the library reports what it allocates (dd_footprint_bytes)
# ----------------------------------------------------------------------------
def library_footprint(L, block, n_vec, store, nrhs):
    """Device bytes for one field on the mixed-precision path: the field plus its
    resident setup, the scratch a setup holds while it runs, and the solve
    workspace for nrhs right-hand sides, as the library computes them."""
    from . import binding as B
    p = B.default_params(block=block, n_vec=n_vec, inner_dtype=B.DD_F32, store_dtype=store)
    return B.footprint(L, block, p, nrhs)


def level3_supported(L, block):
    """A third level needs every coarse-lattice extent to be a multiple of 4."""
    return all((L[m] // block[m]) % 4 == 0 for m in range(4))


def level3_bytes(L, block, n_vec, store, nrhs, n2=24, kmax=40, l3_restart=60, coarse_restart=60):
    """Device bytes of a default third level (dd_mg_add_level without host
    vectors), from the library's layout: `static` (tables, level-2 vectors, P2
    in FP64 and FP32, D3 and its odd-site inverses in FP64, FP32 and, for half
    storage, the half type), `workspace` (the level-2 FGMRES cycle and the
    level-3 GMRES for nrhs right-hand sides, FP32) and `transient` (the
    inverse-iteration buffers and coarse workspace while the level is added).
    A few percent of alignment and small per-RHS state are covered by a margin."""
    Vc = int(np.prod([L[m] // block[m] for m in range(4)]))
    Vc3, nc, nc3 = Vc // 16, 2 * n_vec, 2 * n2
    nvec = n2 * Vc * nc
    half = 4 if store in ("f16", "bf16") else 0
    static = 4 * (8 * Vc3 + 3 * Vc + 1) + nvec * (16 + 16 + 8) + (9 * Vc3 + Vc3 // 2) * nc3 * nc3 * (16 + 8 + half)
    coarse2, coarse3 = Vc * nc * nrhs, Vc3 * nc3 * nrhs
    workspace = 8 * (coarse2 * (2 * kmax + 4) + 2 * coarse3) + 8 * coarse3 * (l3_restart + 9)
    transient = 8 * 2 * nvec + 8 * Vc * nc * n2 * (coarse_restart + 9)
    margin = lambda b: int(1.05 * b) + (1 << 20)   # noqa: E731
    return dict(static=margin(static), workspace=margin(workspace), transient=margin(transient))


# ----------------------------------------------------------------------------
# requests
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class FieldSpec:
    key: str
    L: tuple
    eps: float
    m0: float
    seed: int

    @property
    def V(self):
        return int(np.prod(self.L))


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    field: FieldSpec
    nrhs: int
    src_seed: int


@dataclasses.dataclass
class Done:
    rid: int
    field: str
    nrhs: int
    arrival: float
    start: float
    finish: float
    batch_rhs: int          # most slots of its lane running at once while it ran
    setup_miss: bool
    relres: list
    lane: int = -1
    joined: bool = False    # added to a lane that was already running

    @property
    def latency(self):
        return self.finish - self.arrival


def make_requests(n, rate, shapes, field_pool, rng_seed=5001, reuse_prob=0.3, max_nrhs=12):
    """Poisson arrivals at `rate` per second (rate = inf: all at t = 0).  The
    shape is uniform over `shapes`; with probability `reuse_prob` the request
    reuses a field already issued (any shape), otherwise it takes the next
    unused pool entry of its shape (or reuses one of that shape when the pool
    is used up).  nrhs is uniform on 1..max_nrhs."""
    rng = np.random.default_rng(rng_seed)
    used = {s: 0 for s in shapes}
    issued = []
    t = 0.0
    out = []
    for rid in range(n):
        if math.isfinite(rate):
            t += rng.exponential(1.0 / rate)
        shape = shapes[rng.integers(len(shapes))]
        if issued and rng.random() < reuse_prob:
            f = issued[rng.integers(len(issued))]
        else:
            pool = field_pool[shape]
            if used[shape] < len(pool):
                f = pool[used[shape]]
                used[shape] += 1
                issued.append(f)
            else:
                f = pool[rng.integers(len(pool))]
        out.append(Request(rid, t, f, int(rng.integers(1, max_nrhs + 1)), int(rng.integers(1 << 31))))
    return out


# ----------------------------------------------------------------------------
# scheduler
# ----------------------------------------------------------------------------
class Lane:
    """One field being solved: `capacity` slots, at most one job in flight."""

    def __init__(self, lid, field, capacity, mem, miss):
        self.lid, self.field, self.capacity = lid, field, capacity
        self.mem = mem                   # bytes charged to the lane (workspace; setup scratch while opening)
        self.miss = miss
        self.slots = [None] * capacity   # (rid, j) of the right-hand side in each slot
        self.waiting = []                # requests assigned, added at the next step
        self.state = "opening"           # opening -> running -> closing
        self.peak = 0

    def free_slots(self):
        return sum(s is None for s in self.slots) - sum(r.nrhs for r in self.waiting)

    def running(self):
        return sum(s is not None for s in self.slots)


class Server:
    """Runs a request list through an executor.

    The executor provides:
      footprint(field)             -> bytes of the field's gauge + setup (resident while cached)
      transient(field)             -> bytes needed only while its setup runs
      workspace(field, capacity)   -> bytes of a lane's solver workspace (freed when the lane closes)
      open(lid, field, handle, capacity)  async: load the field if handle is None, start a solve state
      step(lid, adds)              async: add [(slot, request, j)], one restart cycle, take finished slots
      close(lid)                   async: end the solve state, free the workspace
      free(handle)                 drop an idle cached field
      now()                        -> seconds (monotonic)
      wait_event(deadline)         -> the next finished job (kind, lid, payload, error, t) or None
                                      once the clock reaches `deadline` (None: wait for a job)
    Job payloads: open -> handle; step -> {slot: true relative residual} of the slots it finished.
    """

    def __init__(self, executor, hbm_budget, max_rhs=12, max_lanes=6, backfill_bytes=None, log=None):
        self.ex = executor
        self.budget = hbm_budget
        self.max_rhs = max_rhs
        self.max_lanes = max_lanes
        # a lane this small may open inside the oldest blocked request's
        # reservation: it holds little memory and closes soon
        self.backfill = hbm_budget // 32 if backfill_bytes is None else backfill_bytes
        self._hold = False             # the device ran out of memory: open no lane until one closes
        self.cache = OrderedDict()     # field key -> [handle, bytes, lanes using it]
        self.resident = 0              # bytes of cached fields (reserved from the moment a load starts)
        self.inuse = 0                 # bytes charged to open lanes
        self.peak_bytes = 0
        self.log = log or (lambda *a: None)
        self.rejected = []
        self.failed = []
        self.retries = 0
        self.evictions = 0
        self.lanes = {}                # field key -> Lane
        self._lid = 0

    # -- memory ------------------------------------------------------------------
    def _idle_bytes(self, keep):
        return sum(b for k, (h, b, u) in self.cache.items() if u == 0 and k != keep)

    def _evict_for(self, need, keep):
        while self.resident + self.inuse + need > self.budget:
            victim = next((k for k, (h, b, u) in self.cache.items() if u == 0 and k != keep), None)
            if victim is None:
                return False
            h, b, _ = self.cache.pop(victim)
            self.ex.free(h)
            self.resident -= b
            self.evictions += 1
        return True

    # -- admission ---------------------------------------------------------------
    def _schedule(self, queue, now):
        reserved = 0
        for r in list(queue):
            if r not in queue:
                continue
            f = r.field
            lane = self.lanes.get(f.key)
            if lane is not None:
                if lane.state != "closing" and lane.free_slots() >= r.nrhs:
                    lane.waiting.append(r)
                    queue.remove(r)
                    self._start[r.rid] = [None, lane.lid, lane.state == "running"]
                continue
            if len(self.lanes) >= self.max_lanes or self._hold:
                continue
            cached = f.key in self.cache
            fb = 0 if cached else self.ex.footprint(f)
            tr = 0 if cached else self.ex.transient(f)

            def need(c):
                return fb + max(self.ex.workspace(f, c), tr)

            held = 0 if not cached else self.cache[f.key][1]
            if held + need(r.nrhs) > self.budget:
                queue.remove(r)
                self.rejected.append(r.rid)
                self.log(f"[serve] rejected {r.rid}: {need(r.nrhs):.3e} B over budget")
                continue
            free = self.budget - self.resident - self.inuse + self._idle_bytes(f.key)
            batch, nb = [], 0
            for q in queue:
                if q.field.key == f.key and nb + q.nrhs <= self.max_rhs:
                    batch.append(q)
                    nb += q.nrhs
            idle = self._idle_bytes(f.key)

            def fits(c, room):
                return need(c) <= room - reserved or need(c) <= min(room, self.backfill)

            # room for joins (all slots) only where no cached field has to go: a
            # setup costs more than a later lane; evict for the batch at hand
            cap = next((c for c in (self.max_rhs, nb) if fits(c, free - idle)), None)
            if cap is None:
                cap = next((c for c in (nb, r.nrhs) if fits(c, free)), None)
            if cap is None:
                if reserved == 0:
                    reserved = need(r.nrhs)   # the oldest blocked request keeps its place
                continue
            self._evict_for(need(cap), f.key)
            lane = Lane(self._lid, f, cap, max(self.ex.workspace(f, cap), tr), not cached)
            self._lid += 1
            if cached:
                self.cache[f.key][2] += 1
                self.cache.move_to_end(f.key)
            else:
                self.cache[f.key] = [None, fb, 1]
                self.resident += fb
            self.inuse += lane.mem
            self.peak_bytes = max(self.peak_bytes, self.resident + self.inuse)
            nb = 0
            for q in batch:
                if nb + q.nrhs <= cap:
                    lane.waiting.append(q)
                    queue.remove(q)
                    self._start[q.rid] = [now, lane.lid, False]   # the lane's setup is part of its service
                    nb += q.nrhs
            self.lanes[f.key] = lane
            self.ex.open(lane.lid, f, self.cache[f.key][0], cap)
            self.log(f"[serve] t={now:7.2f}s lane {lane.lid} opens on {f.key} L={f.L} capacity {cap} "
                     f"({'setup' if lane.miss else 'cached'}), {nb} rhs")

    def _step(self, lane, now):
        adds = []
        free = [i for i, s in enumerate(lane.slots) if s is None]
        for r in lane.waiting:
            for j in range(r.nrhs):
                k = free.pop(0)
                lane.slots[k] = (r.rid, j)
                adds.append((k, r, j))
            if self._start[r.rid][0] is None:
                self._start[r.rid][0] = now  # a join is on the device from this restart boundary on
        lane.waiting = []
        lane.peak = max(lane.peak, lane.running())
        for rid in {s[0] for s in lane.slots if s is not None}:
            self._peak[rid] = max(self._peak.get(rid, 0), lane.running())
        self.ex.step(lane.lid, adds)

    def _finish_lane(self, lane, key):
        self.inuse -= lane.mem
        del self.lanes[key]
        if key in self.cache:
            self.cache[key][2] -= 1

    # -- events ------------------------------------------------------------------
    def _handle(self, ev, queue, done, t0):
        kind, lid, payload, err, t = ev
        now = t - t0
        lane = next(ln for ln in self.lanes.values() if ln.lid == lid)
        key = lane.field.key
        if err is not None:
            retry = kind == "open" and isinstance(err, MemoryError) and len(self.lanes) > 1
            if retry:
                # the device is fuller than the budget says (memory outside the
                # library): requeue, and open nothing new until a lane closes
                for r in lane.waiting:
                    del self._start[r.rid]
                queue.extend(lane.waiting)
                queue.sort(key=lambda q: (q.arrival, q.rid))
                self._hold = True
                self.retries += 1
            else:
                rids = {s[0] for s in lane.slots if s is not None} | {r.rid for r in lane.waiting}
                self.failed.extend(sorted(rids))
                for rid in rids:
                    self._res.pop(rid, None)
            self.log(f"[serve] lane {lid} ({key}) failed in {kind}{' (requeued)' if retry else ''}: {err}")
            if kind == "open" and lane.miss:
                _, b, _ = self.cache.pop(key)
                self.resident -= b
                self.inuse -= lane.mem
                del self.lanes[key]
            else:
                self._finish_lane(lane, key)
            return
        if kind == "open":
            self.cache[key][0] = payload
            ws = self.ex.workspace(lane.field, lane.capacity)
            self.inuse -= lane.mem - ws      # the setup's scratch is gone
            lane.mem = ws
            lane.state = "running"
            self._step(lane, now)
        elif kind == "step":
            for slot, rr in payload.items():
                rid, j = lane.slots[slot]
                lane.slots[slot] = None
                self._res[rid][j] = rr
                if all(v is not None for v in self._res[rid]):
                    r = self._req[rid]
                    st, _, joined = self._start[rid]
                    done.append(Done(rid, key, r.nrhs, r.arrival, st, now, self._peak.get(rid, r.nrhs),
                                     lane.miss and not joined, self._res.pop(rid), lid, joined))
            self._schedule(queue, now)       # same-field arrivals join at this restart boundary
            if lane.running() or lane.waiting:
                self._step(lane, now)
            else:
                lane.state = "closing"
                self.ex.close(lid)
        elif kind == "close":
            self._finish_lane(lane, key)
            self._hold = False
            self.log(f"[serve] t={now:7.2f}s lane {lid} on {key} closes (peak {lane.peak} rhs) queue {len(queue)}")

    def run(self, requests):
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        self._req = {r.rid: r for r in pending}
        self._res = {r.rid: [None] * r.nrhs for r in pending}
        self._start, self._peak = {}, {}
        queue, done = [], []
        t0 = self.ex.now()
        i = 0
        while i < len(pending) or queue or self.lanes:
            now = self.ex.now() - t0
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                i += 1
            self._schedule(queue, now)
            if not self.lanes and queue:
                continue                      # an empty device admits or rejects the head at once
            deadline = t0 + pending[i].arrival if i < len(pending) else None
            if deadline is None and not self.lanes:
                break
            ev = self.ex.wait_event(deadline)
            if ev is not None:
                self._handle(ev, queue, done, t0)
        return done


def summarize(done, wall):
    lat = np.array([d.latency for d in done]) if done else np.zeros(1)
    wait = np.array([d.start - d.arrival for d in done]) if done else np.zeros(1)
    return dict(requests=len(done), rhs=int(sum(d.nrhs for d in done)), wall_s=round(wall, 3),
                p50_s=round(float(np.percentile(lat, 50)), 4), p99_s=round(float(np.percentile(lat, 99)), 4),
                mean_s=round(float(lat.mean()), 4),
                wait_p50_s=round(float(np.percentile(wait, 50)), 4), wait_p99_s=round(float(np.percentile(wait, 99)), 4),
                solves_per_s=round(sum(d.nrhs for d in done) / max(wall, 1e-9), 3),
                setup_misses=int(sum(d.setup_miss for d in done)),
                joined=int(sum(d.joined for d in done)),
                mean_batch_rhs=round(float(np.mean([d.batch_rhs for d in done])) if done else 0.0, 2),
                max_relres=float(max((max(d.relres) for d in done), default=0.0)))


def overlap_seconds(intervals):
    """Time covered by at least two lanes' intervals at once, from (lane, start, end) triples."""
    pts = sorted([(s, 1, ln) for ln, s, e in intervals] + [(e, -1, ln) for ln, s, e in intervals])
    active, total, last = {}, 0.0, None
    for t, d, ln in pts:
        if last is not None and sum(1 for v in active.values() if v > 0) >= 2:
            total += t - last
        active[ln] = active.get(ln, 0) + d
        last = t
    return total


# ----------------------------------------------------------------------------
# GPU executor
# ----------------------------------------------------------------------------
class _LaneWorker(threading.Thread):
    """Host thread of one lane: its jobs run in order on its own HIP stream."""

    def __init__(self, ex, lid):
        super().__init__(daemon=True)
        import torch
        self.ex, self.lid = ex, lid
        self.jobs = _queue.Queue()
        self.stream = torch.cuda.Stream()
        self.field = self.handle = self.state = None
        self.slot_req = {}

    def run(self):
        while True:
            kind, args = self.jobs.get()
            try:
                payload, err = getattr(self, "_" + kind)(*args), None
            except Exception as e:   # reported to the scheduler; the lane cleans up and stops
                payload, err = None, e
                self._cleanup(kind)
            self.ex.events.put((kind, self.lid, payload, err, time.perf_counter()))
            if kind == "close" or err is not None:
                return

    def _cleanup(self, kind):
        try:
            if self.state is not None:
                self.state.end()
                self.state = None
            if self.handle is not None and kind != "open":
                self.handle[1].dd_mg_release_workspace()
        except Exception:
            pass

    def _open(self, f, handle, capacity):
        from . import binding as B
        self.field = f
        fresh = handle is None
        try:
            if fresh:
                handle = self.ex.load(f)
            try:
                self.state = handle[1].dd_solve_begin(capacity, self.ex.tol, self.stream)
            except Exception:
                if fresh:              # the scheduler drops a field whose lane failed to open
                    self.ex.free(handle)
                raise
        except B.DDError as e:
            if e.name in ("DD_ENOMEM", "DD_EBUDGET"):
                raise MemoryError(str(e)) from e
            raise
        self.handle = handle
        return handle

    def _step(self, adds):
        import torch
        from . import binding as B
        ex, f = self.ex, self.field
        with torch.cuda.stream(self.stream):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(self.stream)
            for slot, r, j in adds:
                self.state.add(slot, ex.source(f, r, j))   # read before the call returns
                self.slot_req[slot] = (r.rid, j, r.nrhs)
            states = self.state.step()
            out = {}
            for slot, s in enumerate(states):
                if s != B.SLOT_DONE:
                    continue
                x = torch.empty(f.V * 12, dtype=torch.complex128, device="cuda")
                info = self.state.take(slot, x)
                out[slot] = info["true_relres"]
                rid, j, nrhs = self.slot_req.pop(slot)
                if ex.keep_x:
                    xs = ex.results.setdefault(rid, torch.zeros((nrhs, f.V * 12), dtype=torch.complex128))
                    xs[j] = x.cpu()
            e1.record(self.stream)
        ex.intervals.append((self.lid, e0, e1))
        return out

    def _close(self):
        import torch
        self.state.end()
        self.state = None
        self.handle[1].dd_mg_release_workspace()
        torch.cuda.empty_cache()       # the lane's sources and solutions leave torch's cache too


class GpuExecutor:
    """Runs lanes through the library on cuda:0, one host thread and HIP stream
    per lane.  Links are generated on the host before the run (excluded from
    latency); sources are drawn on the device from a per-request seed."""

    def __init__(self, ctx, links, block=(4, 4, 4, 4), n_vec=20, store="f32", c_sw=1.0, setup_iters=4,
                 tol=1e-10, graphs=False, tune_cache=None, levels=2):
        from . import binding as B
        import torch
        self.B = B
        self.ctx = ctx
        self.links = links            # field key -> host links [V][4][3][3]
        self.block = tuple(block)
        self.n = n_vec
        self.store = B.DTYPES[store]
        self.store_name = store
        self.levels = levels          # 3: fields whose coarse extents allow it get the default third level
        self.c_sw = c_sw
        self.setup_iters = setup_iters
        self.tol = tol
        # graph capture (modes 1 and 2 capture on first use) does not mix with other
        # threads' legacy-stream work (a setup's uploads, synchronous copies,
        # device-wide synchronisation): lanes launch directly
        self.graphs = graphs
        self.tune_cache = tune_cache
        self.keep_x = False           # keep each request's solution (host) in self.results
        self.results = {}
        self.events = _queue.Queue()
        self.workers = {}
        self.intervals = []           # (lane, start event, end event) of every step, on the lane's stream
        self.t_origin = torch.cuda.Event(enable_timing=True)
        self.t_origin.record()

    def _fp(self, f, nrhs=1):
        return library_footprint(f.L, self.block, self.n, self.store, nrhs)

    def _three(self, f):
        return self.levels == 3 and level3_supported(f.L, self.block)

    def _l3(self, f, nrhs=1):
        return level3_bytes(f.L, self.block, self.n, self.store_name, nrhs) if self._three(f) else None

    def footprint(self, f):
        fp, l3 = self._fp(f), self._l3(f)
        return fp["gauge"] + fp["setup"] + (l3["static"] if l3 else 0)

    def transient(self, f):
        l3 = self._l3(f)
        return max(self._fp(f)["scratch"], l3["transient"] if l3 else 0)

    def workspace(self, f, nrhs):
        l3 = self._l3(f, nrhs)
        return self._fp(f, nrhs)["workspace"] + (l3["workspace"] if l3 else 0)

    def load(self, f):
        B = self.B
        g = B.Gauge(self.ctx, f.L, self.block, self.links[f.key], f.m0, self.c_sw)
        p = B.default_params(block=self.block, n_vec=self.n, setup_iters=self.setup_iters, inner_dtype=B.DD_F32,
                             store_dtype=self.store, seed=f.seed)
        try:
            mg = B.MG(g, p)
            mg.dd_mg_set_graphs(self.graphs)
            if self.tune_cache:
                mg.dd_autotune(12, self.tune_cache)
            if self._three(f):
                mg.add_level(B.level3_params())
        except Exception:
            if "mg" in locals():
                mg.destroy()
            g.destroy()        # a failed setup leaves nothing resident
            raise
        return (g, mg)

    def source(self, f, r, j):
        """Right-hand side j of request r: Gaussian complex entries drawn on the
        device from the seed (request seed, j), one vector at a time."""
        import torch
        gen = torch.Generator(device="cuda")
        gen.manual_seed(r.src_seed * 16 + j)
        re = torch.randn(f.V * 12, generator=gen, device="cuda", dtype=torch.float64)
        im = torch.randn(f.V * 12, generator=gen, device="cuda", dtype=torch.float64)
        return torch.complex(re, im)

    def open(self, lid, f, handle, capacity):
        w = _LaneWorker(self, lid)
        self.workers[lid] = w
        w.start()
        w.jobs.put(("open", (f, handle, capacity)))

    def step(self, lid, adds):
        self.workers[lid].jobs.put(("step", (adds,)))

    def close(self, lid):
        self.workers[lid].jobs.put(("close", ()))

    def free(self, h):
        g, mg = h
        mg.destroy()
        g.destroy()

    def now(self):
        return time.perf_counter()

    def wait_event(self, deadline):
        try:
            if deadline is None:
                ev = self.events.get()
            else:
                ev = self.events.get(timeout=max(0.0, deadline - time.perf_counter()))
        except _queue.Empty:
            return None
        if ev[0] == "close" or ev[3] is not None:
            self.workers.pop(ev[1]).join()
        return ev

    def device_intervals(self):
        """(lane, start s, end s) of every step on the device, from the HIP events."""
        import torch
        torch.cuda.synchronize()
        return [(ln, self.t_origin.elapsed_time(a) * 1e-3, self.t_origin.elapsed_time(b) * 1e-3)
                for ln, a, b in self.intervals]


# ----------------------------------------------------------------------------
# the serving run (mixed lattices)
# ----------------------------------------------------------------------------
SHAPES = [(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]


def m0_for_eps(eps):
    """Bare mass for a link roughness: piecewise linear through the tuned
    (roughness, mass) pairs of the 16^3x32, 32^3x64 and 48^3x96 workloads,
    extended linearly past the ends."""
    from workloads import get_config
    pts = sorted((get_config(c)["eps"], get_config(c)["m0"]) for c in ("C2", "C3", "C4"))
    xs, ys = [p[0] for p in pts], [p[1] for p in pts]
    k = 0 if eps <= xs[1] else 1
    return ys[k] + (ys[k + 1] - ys[k]) * (eps - xs[k]) / (xs[k + 1] - xs[k])


def field_pool(per_shape, seed0=6000, eps_range=(0.15, 0.3)):
    """Fields per shape: seed 6000 + k, link roughness uniform on eps_range
    (drawn from the same seed), bare mass from m0_for_eps."""
    pool, k = {}, 0
    for L in SHAPES:
        pool[L] = []
        for j in range(per_shape):
            eps = float(np.random.default_rng(seed0 + k).uniform(*eps_range))
            pool[L].append(FieldSpec(f"{'x'.join(map(str, L))}#{j}", L, round(eps, 4),
                                     round(m0_for_eps(round(eps, 4)), 6), seed0 + k))
            k += 1
    return pool


def _run_report(ex, srv, reqs, log):
    n0 = len(ex.intervals)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    res = summarize(done, time.perf_counter() - t0)
    ivs = ex.device_intervals()[n0:]
    busy = overlap_seconds([(0, a, b) for _, a, b in ivs] + [(1, a, b) for _, a, b in ivs]) if ivs else 0.0
    res.update(rejected=len(srv.rejected), failed=len(srv.failed), retries=srv.retries, evictions=srv.evictions,
               device_busy_s=round(busy, 3), device_overlap_s=round(overlap_seconds(ivs), 3),
               peak_hbm_gib=round(srv.peak_bytes / 2 ** 30, 2))
    return done, res


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="open-loop serving run over mixed lattices")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--capacity-requests", type=int, default=60)
    ap.add_argument("--per-shape", type=int, default=2)
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate as a fraction of measured capacity")
    ap.add_argument("--rate", type=float, default=None, help="arrival rate (requests/s); overrides --load")
    ap.add_argument("--skip-capacity", action="store_true", help="with --rate: no closed-loop run")
    ap.add_argument("--hbm-gib", type=float, default=230.0)
    ap.add_argument("--store", default="bf16", choices=["f32", "f16", "bf16"])
    ap.add_argument("--max-lanes", type=int, default=6, help="fields solved at once (1: one batch at a time)")
    ap.add_argument("--shapes", default="all", help="'all' or a count of the smallest shapes to use")
    ap.add_argument("--levels", type=int, default=2, choices=[2, 3],
                    help="3: fields whose coarse extents are multiples of 4 get the default third level")
    args = ap.parse_args(argv)
    from . import binding as B
    from workloads import su3_field
    log = lambda *a: print(*a, file=sys.stderr, flush=True)   # noqa: E731
    shapes = SHAPES if args.shapes == "all" else SHAPES[:int(args.shapes)]
    pool = {L: v for L, v in field_pool(args.per_shape).items() if L in shapes}
    links = {}
    t0 = time.perf_counter()
    for L in shapes:
        for f in pool[L]:
            links[f.key] = su3_field(f.L, f.eps, f.seed)
            log(f"[serve] field {f.key}: eps {f.eps} m0 {f.m0} seed {f.seed}")
    log(f"[serve] {sum(len(v) for v in pool.values())} fields generated on the host in {time.perf_counter() - t0:.1f} s")
    budget = int(args.hbm_gib * (1 << 30))
    ctx = B.Context(0, hbm_budget_bytes=budget)
    ex = GpuExecutor(ctx, links, store=args.store, levels=args.levels)
    cap, mu = None, None
    if not (args.skip_capacity and args.rate):
        # closed loop: everything queued at t = 0 gives the capacity
        reqs = make_requests(args.capacity_requests, math.inf, shapes, pool, rng_seed=5002)
        srv = Server(ex, budget, max_lanes=args.max_lanes, log=log)
        _, cap = _run_report(ex, srv, reqs, log)
        mu = cap["requests"] / cap["wall_s"]
        log(f"[serve] closed-loop capacity {mu:.3f} requests/s: {json.dumps(cap)}")
        for h, _, _ in srv.cache.values():
            ex.free(h)
    # open loop at load * capacity, or at the given rate
    rate = args.rate if args.rate else args.load * mu
    reqs = make_requests(args.requests, rate, shapes, pool, rng_seed=5001)
    srv = Server(ex, budget, max_lanes=args.max_lanes, log=log)
    done, res = _run_report(ex, srv, reqs, log)
    by_shape = {}
    for d in done:
        L = "x".join(map(str, next(f.L for v in pool.values() for f in v if f.key == d.field)))
        by_shape.setdefault(L, []).append(d.latency)
    res.update(capacity_requests_per_s=None if mu is None else round(mu, 4), arrival_rate_per_s=round(rate, 4),
               store=args.store, max_lanes=args.max_lanes, levels=args.levels, closed_loop=cap,
               shapes=["x".join(map(str, L)) for L in shapes], fields_per_shape=args.per_shape,
               p50_by_shape={k: round(float(np.percentile(v, 50)), 3) for k, v in by_shape.items()},
               p99_by_shape={k: round(float(np.percentile(v, 99)), 3) for k, v in by_shape.items()})
    for h, _, _ in srv.cache.values():
        ex.free(h)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
