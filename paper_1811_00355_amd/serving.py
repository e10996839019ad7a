"""Serving loop for batches of Wilson-clover solves (one GPU).

Requests arrive as a Poisson stream.  Each asks for `nrhs` solves D x = b on one
gauge field (lattice shape, link roughness, bare mass).  The paper's accounting
(Sec. 4: one adaptive setup per configuration, then 12 solves) is what makes a
per-field setup cache pay: the first request on a field pays for the upload
and the setup, later ones reuse them.

* Setup cache: gauge field + multigrid setup stay resident on the device, keyed
  by field, least recently used first out.
* Admission: a request is started only when the HBM footprint of its field
  (cached or not) plus the solver workspace of its batch fits the budget; idle
  cached fields are evicted to make room; a request that cannot fit even on an
  empty device is rejected.
* Continuous batching: whenever the device is free, the oldest waiting request
  is taken together with every other waiting request on the same field, up to
  `max_rhs` right-hand sides, as one batched solve.  The solver reduces each
  right-hand side in an order independent of the batch and masks converged
  ones, so every request gets the same bits alone or in any batch.
* Latency runs from arrival to the solution being back in host memory.

The scheduler is plain host logic driven through an executor object; the GPU
executor calls the library, and tests drive the same scheduler with a CPU fake.
"""
import dataclasses
import math
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
    batch_rhs: int
    setup_miss: bool
    relres: list

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
class Server:
    """Runs a request list through an executor.

    The executor provides:
      footprint(field)            -> bytes of the field's gauge + setup (resident)
      transient(field)            -> bytes needed only while its setup runs
      workspace(field, nrhs)      -> bytes of a batch's solver workspace (freed after the batch)
      load(field)                 -> handle          (upload + setup)
      solve(handle, field, reqs)  -> [relres list per request]  (results on the host)
      free(handle)
      now()                       -> seconds (monotonic)
      sleep_until(t)              -> wait for the clock (the fake advances it)
    """

    def __init__(self, executor, hbm_budget, max_rhs=12, log=None):
        self.ex = executor
        self.budget = hbm_budget
        self.max_rhs = max_rhs
        self.cache = OrderedDict()     # field key -> (handle, bytes)
        self.resident = 0
        self.log = log or (lambda *a: None)
        self.rejected = []
        self.evictions = 0

    def _evict_for(self, need, keep):
        while self.resident + need > self.budget:
            victim = next((k for k in self.cache if k != keep), None)
            if victim is None:
                return False
            h, b = self.cache.pop(victim)
            self.ex.free(h)
            self.resident -= b
            self.evictions += 1
        return True

    def _form_batch(self, queue):
        """Oldest request first, then every waiting request on its field, in
        arrival order, while the right-hand sides fit."""
        head = queue[0]
        batch, total = [], 0
        for r in queue:
            if r.field.key == head.field.key and total + r.nrhs <= self.max_rhs:
                batch.append(r)
                total += r.nrhs
        return batch

    def run(self, requests):
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        queue, done = [], []
        t0 = self.ex.now()
        i = 0
        while i < len(pending) or queue:
            now = self.ex.now() - t0
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                i += 1
            if not queue:
                self.ex.sleep_until(t0 + pending[i].arrival)
                continue
            batch = self._form_batch(queue)
            f = batch[0].field
            nrhs = sum(r.nrhs for r in batch)
            ws = self.ex.workspace(f, nrhs)
            miss = f.key not in self.cache
            fb = self.ex.footprint(f) if miss else 0
            tr = self.ex.transient(f) if miss else 0
            need = fb + max(ws, tr)
            if need > self.budget or not self._evict_for(need, f.key):
                for r in batch:
                    queue.remove(r)
                    self.rejected.append(r.rid)
                self.log(f"[serve] rejected {[r.rid for r in batch]}: {need:.3e} B over budget")
                continue
            start = self.ex.now() - t0
            if miss:
                self.cache[f.key] = (self.ex.load(f), fb)
                self.resident += fb
            self.cache.move_to_end(f.key)
            relres = self.ex.solve(self.cache[f.key][0], f, batch)
            finish = self.ex.now() - t0
            for r, rr in zip(batch, relres):
                queue.remove(r)
                done.append(Done(r.rid, f.key, r.nrhs, r.arrival, start, finish, nrhs, miss, rr))
            self.log(f"[serve] t={finish:7.2f}s field {f.key} L={f.L} batch {len(batch)} req / {nrhs} rhs "
                     f"{'setup+' if miss else ''}solve {finish - start:.3f}s queue {len(queue)}")
        return done


def summarize(done, wall):
    lat = np.array([d.latency for d in done]) if done else np.zeros(1)
    return dict(requests=len(done), rhs=int(sum(d.nrhs for d in done)), wall_s=round(wall, 3),
                p50_s=round(float(np.percentile(lat, 50)), 4), p99_s=round(float(np.percentile(lat, 99)), 4),
                mean_s=round(float(lat.mean()), 4),
                solves_per_s=round(sum(d.nrhs for d in done) / max(wall, 1e-9), 3),
                setup_misses=int(sum(d.setup_miss for d in done)),
                mean_batch_rhs=round(float(np.mean([d.batch_rhs for d in done])) if done else 0.0, 2),
                max_relres=float(max((max(d.relres) for d in done), default=0.0)))


# ----------------------------------------------------------------------------
# GPU executor
# ----------------------------------------------------------------------------
class GpuExecutor:
    """Runs batches through the library on cuda:0.  Links are generated on the
    host before the run (excluded from latency); sources are drawn on the
    device from a per-request seed."""

    def __init__(self, ctx, links, block=(4, 4, 4, 4), n_vec=20, store="f32", c_sw=1.0, setup_iters=4,
                 tol=1e-10, graphs=True, tune_cache=None):
        from . import binding as B
        self.B = B
        self.ctx = ctx
        self.links = links            # field key -> host links [V][4][3][3]
        self.block = tuple(block)
        self.n = n_vec
        self.store = B.DTYPES[store]
        self.c_sw = c_sw
        self.setup_iters = setup_iters
        self.tol = tol
        self.graphs = graphs
        self.tune_cache = tune_cache
        self.keep_x = False           # keep each request's solution (host) in self.results
        self.results = {}

    def _fp(self, f, nrhs=1):
        return library_footprint(f.L, self.block, self.n, self.store, nrhs)

    def footprint(self, f):
        fp = self._fp(f)
        return fp["gauge"] + fp["setup"]

    def transient(self, f):
        return self._fp(f)["scratch"]

    def workspace(self, f, nrhs):
        return self._fp(f, nrhs)["workspace"]

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
        except Exception:
            if "mg" in locals():
                mg.destroy()
            g.destroy()        # a failed setup leaves nothing resident
            raise
        return (g, mg)

    def sources(self, f, r):
        import torch
        gen = torch.Generator(device="cuda")
        gen.manual_seed(r.src_seed)
        re = torch.randn((r.nrhs, f.V * 12), generator=gen, device="cuda", dtype=torch.float64)
        im = torch.randn((r.nrhs, f.V * 12), generator=gen, device="cuda", dtype=torch.float64)
        return torch.complex(re, im)

    def solve(self, h, f, reqs):
        import torch
        g, mg = h
        b = torch.cat([self.sources(f, r) for r in reqs], 0)
        x = torch.zeros_like(b)
        info, st = mg.dd_solve(b.shape[0], b, x, self.tol, raise_on_noconv=False)
        xh = x.cpu()                  # the results are back on the host
        mg.dd_mg_release_workspace()
        out, k = [], 0
        for r in reqs:
            out.append([info[k + j]["true_relres"] for j in range(r.nrhs)])
            if self.keep_x:
                self.results[r.rid] = xh[k:k + r.nrhs]
            k += r.nrhs
        return out

    def free(self, h):
        g, mg = h
        mg.destroy()
        g.destroy()

    def now(self):
        return time.perf_counter()

    def sleep_until(self, t):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)


# ----------------------------------------------------------------------------
# the serving run (mixed lattices)
# ----------------------------------------------------------------------------
SHAPES = [(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]


def field_pool(per_shape, seed0=6000):
    """Fields per shape: seed 6000 + k, link roughness drawn from the tuned set
    {0.15, 0.2, 0.25}, with the bare mass tuned for that roughness."""
    from workloads import get_config
    tuned = {get_config(c)["eps"]: get_config(c)["m0"] for c in ("C2", "C3", "C4")}
    epss = sorted(tuned)
    pool, k = {}, 0
    for L in SHAPES:
        pool[L] = []
        for j in range(per_shape):
            eps = epss[(k * 7 + j) % len(epss)]
            pool[L].append(FieldSpec(f"{'x'.join(map(str, L))}#{j}", L, eps, tuned[eps], seed0 + k))
            k += 1
    return pool


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="open-loop serving run over mixed lattices")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--capacity-requests", type=int, default=60)
    ap.add_argument("--per-shape", type=int, default=2)
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate as a fraction of measured capacity")
    ap.add_argument("--hbm-gib", type=float, default=230.0)
    ap.add_argument("--store", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--shapes", default="all", help="'all' or a count of the smallest shapes to use")
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
    log(f"[serve] {sum(len(v) for v in pool.values())} fields generated on the host in {time.perf_counter() - t0:.1f} s")
    ctx = B.Context(0, hbm_budget_bytes=int(args.hbm_gib * (1 << 30)))
    ex = GpuExecutor(ctx, links, store=args.store)
    budget = int(args.hbm_gib * (1 << 30))
    # closed loop: everything queued at t = 0 gives the capacity
    reqs = make_requests(args.capacity_requests, math.inf, shapes, pool, rng_seed=5002)
    srv = Server(ex, budget, log=log)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    cap = summarize(done, time.perf_counter() - t0)
    mu = cap["requests"] / cap["wall_s"]
    log(f"[serve] closed-loop capacity {mu:.3f} requests/s: {cap}")
    for h, _ in srv.cache.values():
        ex.free(h)
    # open loop at load * capacity
    reqs = make_requests(args.requests, args.load * mu, shapes, pool, rng_seed=5001)
    srv = Server(ex, budget, log=log)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    res = summarize(done, time.perf_counter() - t0)
    res.update(capacity_requests_per_s=round(mu, 4), arrival_rate_per_s=round(args.load * mu, 4),
               rejected=len(srv.rejected), evictions=srv.evictions, store=args.store,
               shapes=["x".join(map(str, L)) for L in shapes], fields_per_shape=args.per_shape)
    for h, _ in srv.cache.values():
        ex.free(h)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
