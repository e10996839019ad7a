"""Serving on the GPU: requests merged into shared batches get the same bits as
the same requests solved one by one; every solve meets the residual bar; the
footprint model bounds what a cached field really holds."""
import pytest

pytestmark = pytest.mark.gpu


def test_mixed_batches_equal_alone():
    import torch
    from paper_1811_00355_amd import Context
    from paper_1811_00355_amd import serving as S
    from workloads import su3_field
    fields = [S.FieldSpec("8^4#0", (8, 8, 8, 8), 0.25, -0.2, 6101),
              S.FieldSpec("8^3x16#0", (8, 8, 8, 16), 0.2, -0.15, 6102)]
    links = {f.key: su3_field(f.L, f.eps, f.seed) for f in fields}
    ctx = Context(0)
    ex = S.GpuExecutor(ctx, links, n_vec=20, setup_iters=2)
    ex.keep_x = True
    a, b = fields
    reqs = [S.Request(0, 0.0, a, 3, 11), S.Request(1, 0.0, b, 5, 12), S.Request(2, 0.0, a, 4, 13),
            S.Request(3, 0.0, b, 7, 14), S.Request(4, 0.0, a, 5, 15), S.Request(5, 0.0, b, 2, 16)]
    srv = S.Server(ex, 64 << 30, log=print)
    before = ctx.bytes_in_use()
    done = srv.run(reqs)
    resident = ctx.bytes_in_use() - before
    model = sum(ex.footprint(f) for f in fields)
    print(f"resident after the run {resident / 2**20:.1f} MiB, footprint model {model / 2**20:.1f} MiB", flush=True)
    assert resident == model                       # the model counts every resident byte
    assert max(max(d.relres) for d in done) <= 1e-10
    assert any(d.batch_rhs > d.nrhs for d in done), "no request shared a batch"
    batched = dict(ex.results)
    for r in reqs:
        ex.results.clear()
        srv.run([S.Request(r.rid, 0.0, r.field, r.nrhs, r.src_seed)])
        same = torch.equal(ex.results[r.rid], batched[r.rid])
        print(f"request {r.rid} ({r.field.key}, {r.nrhs} rhs): alone == in batch: {same}", flush=True)
        assert same
    for h, _ in srv.cache.values():
        ex.free(h)
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
