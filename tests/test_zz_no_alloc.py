"""The allocation-free coarse solve (dd_coarse_solve_noalloc) against
dd_coarse_solve on the same setup and inputs: two calls in a row, the second
with fewer right-hand sides, in FP32 (half-precision storage setup) and FP64;
the context's allocation counter does not move; a call whose workspace exceeds
the static scratch is refused with DD_EBUDGET."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1811_00355_amd import Context
    c = Context(0)
    yield c
    c.close()


def _setup(ctx, L, blk, n, inner, store, **kw):
    from paper_1811_00355_amd import Gauge, MG, default_params
    from workloads import su3_field
    g = Gauge(ctx, L, blk, su3_field(L, 0.2, 23), -0.1, 1.0)
    p = default_params(block=blk, n_vec=n, inner_dtype=inner, store_dtype=store, init_sap_apps=2, setup_iters=1,
                       seed=11, **kw)
    return g, MG(g, p)


def _solve(mg, fn, dtype, nrhs, c):
    import torch
    import _gpu
    cin = _gpu.to_dev(c.reshape(nrhs, -1))
    pin = mg.new_coarse(dtype, nrhs)
    pout = mg.new_coarse(dtype, nrhs)
    mg.pack_coarse(dtype, nrhs, cin, pin)
    its = fn(dtype, nrhs, pin, pout)
    cout = torch.zeros_like(cin)
    mg.unpack_coarse(dtype, nrhs, pout, cout)
    torch.cuda.synchronize()
    return its, _gpu.to_host(cout).reshape(c.shape), pout


@pytest.mark.parametrize("inner,store,dtype,bar", [(1, 3, 1, 1e-5), (0, 0, 0, 1e-12)])
def test_noalloc_coarse_solve_matches(ctx, inner, store, dtype, bar):
    import torch
    import _gpu
    from workloads import gauss_vectors
    L, blk, n = (8, 8, 8, 16), (4, 4, 4, 4), 20
    g, mg = _setup(ctx, L, blk, n, inner, store)
    Vc = 32
    for call, nrhs in enumerate((12, 3)):
        c = gauss_vectors(nrhs, Vc, 200 + call, ncomp=2 * n)
        if dtype == 1:
            c = _gpu.round_f32(c)
        before = ctx.bytes_in_use()
        its_na, got, raw_na = _solve(mg, mg.dd_coarse_solve_noalloc, dtype, nrhs, c)
        assert ctx.bytes_in_use() == before          # nothing allocated from the pool
        its_ref, ref, raw_ref = _solve(mg, mg.dd_coarse_solve, dtype, nrhs, c)
        err = _gpu.max_rel(got, ref)
        same = torch.equal(raw_na, raw_ref)
        print(f"inner {inner} store {store} call {call}: {nrhs} rhs, iterations {its_na} / {its_ref}, "
              f"max rel diff {err:.2e}, bitwise equal {same}", flush=True)
        assert its_na == its_ref and err < bar
    mg.destroy()
    g.destroy()


def test_noalloc_coarse_solve_refuses_oversized(ctx):
    from paper_1811_00355_amd import DDError
    L, blk, n = (8, 8, 8, 16), (4, 4, 4, 4), 20
    g, mg = _setup(ctx, L, blk, n, 1, 1, coarse_restart=256)
    nrhs = 64                          # (256 + 9) coarse vectors of 64 RHS: about 170 MB > 128 MiB
    a, b = mg.new_coarse(1, nrhs), mg.new_coarse(1, nrhs)
    with pytest.raises(DDError) as e:
        mg.dd_coarse_solve_noalloc(1, nrhs, a, b)
    print(f"refused: {e.value}", flush=True)
    assert e.value.name == "DD_EBUDGET"
    with pytest.raises(DDError) as e:
        mg.dd_coarse_solve_noalloc(1, 65, mg.new_coarse(1, 65), mg.new_coarse(1, 65))
    assert e.value.name == "DD_EINVAL"
    mg.destroy()
    g.destroy()
