"""Serving on the GPU: concurrent lanes overlap on the device and give every
request the same bits as solving it alone; every solve meets the residual bar;
the footprint figures are what the library allocates."""
import pytest

pytestmark = pytest.mark.gpu


def test_lanes_overlap_on_the_device_and_results_match_alone():
    """Two fields solved by concurrent lanes (own stream and host thread each):
    their steps overlap on the device (HIP event intervals), a request that
    arrives while its field's lane runs joins it at a restart boundary, and
    every request gets the same bits as when it is served alone."""
    import time
    import torch
    from paper_1811_00355_amd import Context
    from paper_1811_00355_amd import serving as S
    from workloads import su3_field
    fields = [S.FieldSpec("8^3x16#0", (8, 8, 8, 16), 0.25, -0.25, 6101),
              S.FieldSpec("8^3x16#1", (8, 8, 8, 16), 0.2, -0.2, 6102)]
    links = {f.key: su3_field(f.L, f.eps, f.seed) for f in fields}
    ctx = Context(0)
    ex = S.GpuExecutor(ctx, links, n_vec=20, setup_iters=2, store="bf16")
    ex.keep_x = True
    a, b = fields
    # warm both fields into the cache so that the timed part is solves only
    warm = S.Server(ex, 64 << 30, log=print)
    warm.run([S.Request(100, 0.0, a, 1, 1), S.Request(101, 0.0, b, 1, 2)])
    # a's first lane is full (3 + 9 slots): request 3 waits and joins when slots free up
    reqs = [S.Request(0, 0.0, a, 3, 11), S.Request(1, 0.0, b, 5, 12), S.Request(2, 0.0, a, 9, 13),
            S.Request(3, 0.0, a, 2, 14), S.Request(4, 0.0, b, 4, 15)]
    srv = S.Server(ex, 64 << 30, log=print)
    srv.cache = warm.cache
    srv.resident = warm.resident
    n0 = len(ex.intervals)
    t0 = time.perf_counter()
    done = {d.rid: d for d in srv.run(reqs)}
    wall = time.perf_counter() - t0
    ivs = ex.device_intervals()[n0:]
    ov = S.overlap_seconds(ivs)
    lanes = sorted({ln for ln, _, _ in ivs})
    print(f"{len(ivs)} steps on lanes {lanes} in {wall:.3f} s; two lanes on the device together for {ov:.3f} s",
          flush=True)
    for d in sorted(done.values(), key=lambda d: d.rid):
        print(f"request {d.rid} lane {d.lane} joined {d.joined} peak {d.batch_rhs} rhs "
              f"latency {d.latency:.3f} s relres {max(d.relres):.2e}", flush=True)
    assert sorted(done) == [0, 1, 2, 3, 4] and not srv.rejected and not srv.failed
    assert len(lanes) >= 2 and ov > 0.0, "lanes did not overlap on the device"
    assert max(max(d.relres) for d in done.values()) <= 1e-10
    assert any(d.joined for d in done.values()), "no request joined a running lane"
    mixed = {rid: ex.results[rid].clone() for rid in done}
    for r in reqs:
        ex.results.pop(r.rid, None)
        solo = S.Server(ex, 64 << 30)
        solo.cache, solo.resident = srv.cache, srv.resident
        solo.run([S.Request(r.rid, 0.0, r.field, r.nrhs, r.src_seed)])
        same = torch.equal(ex.results[r.rid], mixed[r.rid])
        print(f"request {r.rid} ({r.field.key}, {r.nrhs} rhs): alone == in the mix: {same}", flush=True)
        assert same
    for h, _, _ in srv.cache.values():
        ex.free(h)
    assert ctx.bytes_in_use() == 0
    ctx.close()


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_reported_footprint_is_what_the_library_allocates(store):
    """dd_footprint_bytes against the library's allocation counter: a context
    whose budget is exactly gauge + setup + scratch runs the setup, the field
    and setup then hold exactly gauge + setup bytes, and a solve adds exactly
    the workspace figure (so admission on these figures never sees DD_EBUDGET)."""
    import torch
    from paper_1811_00355_amd import Context, Gauge, MG, binding as B
    from paper_1811_00355_amd import serving as S
    from workloads import su3_field, gauss_spinor
    L, blk, n, nrhs = (8, 8, 8, 16), (4, 4, 4, 4), 20, 3
    st = B.DTYPES[store]
    fp = S.library_footprint(L, blk, n, st, nrhs)
    print(f"store {store}: footprint {fp}", flush=True)
    ctx = Context(0, hbm_budget_bytes=fp["gauge"] + fp["setup"] + max(fp["scratch"], fp["workspace"]))
    g = Gauge(ctx, L, blk, su3_field(L, 0.2, 6201), -0.15, 1.0)
    p = B.default_params(block=blk, n_vec=n, setup_iters=1, inner_dtype=B.DD_F32, store_dtype=st, seed=7)
    mg = MG(g, p)
    assert ctx.bytes_in_use() == fp["gauge"] + fp["setup"]
    b = torch.from_numpy(gauss_spinor(L, nrhs, 5).reshape(nrhs, -1)).cuda()
    x = torch.zeros_like(b)
    info, _ = mg.dd_solve(nrhs, b, x, 1e-10)
    torch.cuda.synchronize()
    assert ctx.bytes_in_use() == fp["gauge"] + fp["setup"] + fp["workspace"]
    assert all(i["converged"] for i in info)
    mg.destroy()
    g.destroy()
    assert ctx.bytes_in_use() == 0
    ctx.close()


def test_level3_memory_model_bounds_the_allocation():
    """The serving loop's third-level model (serving.level3_bytes) bounds what
    dd_mg_add_level and a solve with the level actually allocate, within its
    stated margin: static arrays within 1.3x of the model, and the level's
    workspace for the solve's right-hand sides below the model."""
    import torch
    from paper_1811_00355_amd import Context, Gauge, MG, binding as B, level3_params
    from paper_1811_00355_amd import serving as S
    from workloads import su3_field, gauss_spinor
    L, blk, n, nrhs = (16, 16, 16, 16), (4, 4, 4, 4), 20, 3
    assert S.level3_supported(L, blk)
    fp = S.library_footprint(L, blk, n, B.DD_BF16, nrhs)
    model = S.level3_bytes(L, blk, n, "bf16", nrhs)
    ctx = Context(0)
    g = Gauge(ctx, L, blk, su3_field(L, 0.2, 6202), -0.15, 1.0)
    p = B.default_params(block=blk, n_vec=n, setup_iters=1, inner_dtype=B.DD_F32, store_dtype=B.DD_BF16, seed=8)
    mg = MG(g, p)
    base = ctx.bytes_in_use()
    assert base == fp["gauge"] + fp["setup"]
    mg.add_level(level3_params())
    static = ctx.bytes_in_use() - base
    b = torch.from_numpy(gauss_spinor(L, nrhs, 6).reshape(nrhs, -1)).cuda()
    x = torch.zeros_like(b)
    info, _ = mg.dd_solve(nrhs, b, x, 1e-10)
    torch.cuda.synchronize()
    ws3 = ctx.bytes_in_use() - base - static - fp["workspace"]
    print(f"third level: static {static} (model {model['static']}), workspace {ws3} (model {model['workspace']})",
          flush=True)
    assert all(i["converged"] for i in info)
    assert static <= model["static"] <= 1.3 * static + (2 << 20)
    assert 0 < ws3 <= model["workspace"]
    mg.destroy()
    g.destroy()
    assert ctx.bytes_in_use() == 0
    ctx.close()
