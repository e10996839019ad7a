"""Error paths and degenerate inputs through the C ABI: every failure comes
back as a status (nothing aborts), and the context's allocation counter shows
no leak after a failed call."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

L4, B2 = (4, 4, 4, 4), (2, 2, 2, 2)


@pytest.fixture(scope="module")
def ctx():
    from paper_1811_00355_amd import Context
    c = Context(0)
    yield c
    c.close()


def _links(L=L4, seed=1001):
    from workloads import su3_field
    return su3_field(L, 0.3, seed)


def _status(fn):
    from paper_1811_00355_amd.binding import DDError
    with pytest.raises(DDError) as e:
        fn()
    print(f"-> {e.value}", flush=True)
    return e.value.name


def test_bad_shapes(ctx):
    from paper_1811_00355_amd import Gauge
    before = ctx.bytes_in_use()
    cases = [((4, 4, 4, 6), B2),          # 3 blocks in t: odd
             ((4, 4, 4, 4), (2, 2, 2, 3)),   # block edge not a power of two
             ((4, 4, 4, 4), (1, 2, 2, 2)),   # block edge 1
             ((8, 8, 8, 16), (8, 4, 4, 4)),  # 512 sites per block
             ((4, 4, 4, 4), (2, 2, 2, 8))]   # block larger than L
    for L, blk in cases:
        U = np.tile(np.eye(3, dtype=np.complex128), (int(np.prod(L)), 4, 1, 1))
        assert _status(lambda: Gauge(ctx, L, blk, U, -0.4, 1.0)) == "DD_ESHAPE", (L, blk)
    assert ctx.bytes_in_use() == before


def test_bad_parameters(ctx):
    from paper_1811_00355_amd import Gauge, MG, default_params
    g = Gauge(ctx, L4, B2, _links(), -0.4, 1.0)
    before = ctx.bytes_in_use()
    bad = [dict(n_vec=7), dict(n_vec=10), dict(coarse_restart=0), dict(fgmres_restart=65),
           dict(inner_dtype=1, store_dtype=0), dict(inner_dtype=0, store_dtype=3), dict(coarse_cgs_passes=3), dict(outer_cgs_passes=0),
           dict(max_outer_iters=0)]
    want = ["DD_ESHAPE", "DD_ESHAPE", "DD_EINVAL", "DD_EINVAL", "DD_EINVAL", "DD_EINVAL", "DD_EINVAL", "DD_EINVAL"]
    for kw, w in zip(bad, want):
        p = default_params(block=B2, **{"n_vec": 8, **kw})
        assert _status(lambda: MG(g, p)) == w, kw
    p = default_params(block=(2, 2, 2, 2), n_vec=8)
    for m in range(4):
        p.agg_block[m] = 4
    assert _status(lambda: MG(g, p)) == "DD_ESHAPE"
    assert ctx.bytes_in_use() == before
    g.destroy()


def test_budget_exceeded_leaves_nothing_allocated():
    from paper_1811_00355_amd import Context, Gauge, MG, default_params
    c = Context(0, hbm_budget_bytes=200 << 10)      # smaller than the FP64 operator of a 4^4 lattice
    assert _status(lambda: Gauge(c, L4, B2, _links(), -0.4, 1.0)) == "DD_EBUDGET"
    assert c.bytes_in_use() == 0
    c.close()
    c = Context(0, hbm_budget_bytes=1 << 20)        # holds the field, not the setup
    g = Gauge(c, L4, B2, _links(), -0.4, 1.0)
    held = c.bytes_in_use()
    assert _status(lambda: MG(g, default_params(block=B2, n_vec=8))) == "DD_EBUDGET"
    # the failed setup released everything it allocated; the field keeps the FP32
    # copies of links, clover and inverse it made for the inner solver
    assert c.bytes_in_use() == held + 3 * 36 * 8 * 256
    u1 = c.bytes_in_use()
    assert _status(lambda: MG(g, default_params(block=B2, n_vec=8))) == "DD_EBUDGET"
    assert c.bytes_in_use() == u1
    g.destroy()
    assert c.bytes_in_use() == 0
    c.close()


def test_solver_status_paths(ctx):
    import torch
    import _gpu
    from paper_1811_00355_amd import Gauge, MG, default_params
    from workloads import gauss_spinor
    from oracle.lattice import Lattice
    from oracle.dirac import WilsonClover
    U = _links()
    g = Gauge(ctx, L4, B2, U, -0.4, 1.0)
    mg = MG(g, default_params(block=B2, n_vec=8, max_outer_iters=1))
    b = gauss_spinor(L4, 2, 66)
    bd = _gpu.to_dev(b.reshape(2, -1))
    # non-convergence: the best iterate is returned with the status
    x = torch.zeros_like(bd)
    info, st = mg.dd_solve(2, bd, x, 1e-10, raise_on_noconv=False)
    assert st == 5 and not any(i["converged"] for i in info)
    W = WilsonClover(U, Lattice(L4, B2), -0.4, 1.0)
    xr = _gpu.to_host(x).reshape(b.shape)
    res = [np.linalg.norm(b[r] - W.apply(xr[r])) / np.linalg.norm(b[r]) for r in range(2)]
    print(f"after one outer iteration: relres {res}", flush=True)
    assert max(res) < 1.0 and all(abs(i["true_relres"] - rr) < 1e-6 * max(rr, 1e-30) + 1e-12 for i, rr in zip(info, res))
    assert _status(lambda: mg.dd_solve(2, bd, torch.zeros_like(bd), 1e-10)) == "DD_ENOCONV"
    # a non-finite source
    bn = bd.clone()
    bn[1, 5] = float("nan")
    assert _status(lambda: mg.dd_solve(2, bn, torch.zeros_like(bd), 1e-10)) == "DD_ENAN"
    # bad arguments
    assert _status(lambda: mg.dd_solve(2, bd, torch.zeros_like(bd), 0.0)) == "DD_EINVAL"
    pk = g.new_packed(0, 1)
    assert _status(lambda: g.dd_dirac_apply(0, 1, pk, pk)) == "DD_EINVAL"
    # the field cannot go while a setup holds it
    assert _status(lambda: g.destroy()) == "DD_ESTATE"
    mg.destroy()
    g.destroy()


def test_zero_source_is_solved_exactly(ctx):
    """The degenerate right-hand side b = 0 (alone and next to a nonzero one)
    returns x = 0 after no iterations."""
    import torch
    import _gpu
    from paper_1811_00355_amd import Gauge, MG, default_params
    from workloads import gauss_spinor
    g = Gauge(ctx, L4, B2, _links(), -0.4, 1.0)
    mg = MG(g, default_params(block=B2, n_vec=8))
    b = gauss_spinor(L4, 2, 67)
    b[0] = 0.0
    bd = _gpu.to_dev(b.reshape(2, -1))
    x = torch.full_like(bd, 7.0)
    info, st = mg.dd_solve(2, bd, x, 1e-10)
    torch.cuda.synchronize()
    assert st == 0 and info[0]["outer_iters"] == 0 and info[0]["converged"]
    assert torch.count_nonzero(x[0]) == 0 and info[1]["converged"]
    mg.destroy()
    g.destroy()
