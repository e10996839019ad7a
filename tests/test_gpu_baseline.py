"""The paper's comparison solver on the GPU (FP32 SAP-preconditioned BiCGstab
inside an FP64 defect correction) against the oracle's FP64 version: both reach
the true-residual bar, and their solutions agree within what that bar allows."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = {
    # name: (L, block, eps, m0, c_sw, seed)
    "c1": ((4, 4, 4, 4), (2, 2, 2, 2), 0.3, -0.4, 1.0, 1001),
    "b4": ((8, 8, 8, 16), (4, 4, 4, 4), 0.2, -0.1, 1.0, 23),
}


@pytest.fixture(scope="module")
def ctx():
    from paper_1811_00355_amd import Context
    c = Context(0)
    yield c
    c.close()


_ORACLE = {}


@pytest.mark.parametrize("name,store", [("c1", 1), ("b4", 1), ("b4", 3)])
def test_baseline_solve(ctx, name, store):
    import torch
    import _gpu
    from paper_1811_00355_amd import Gauge, bicgstab_params
    from oracle import baseline
    from oracle.lattice import Lattice
    from oracle.dirac import WilsonClover
    from workloads import su3_field, gauss_spinor
    L, blk, eps, m0, csw, seed = CASES[name]
    U = su3_field(L, eps, seed)
    W = WilsonClover(U, Lattice(L, blk), m0, csw)
    g = Gauge(ctx, L, blk, U, m0, csw)
    nrhs = 2 if name == "c1" else 1
    b = gauss_spinor(L, nrhs, 68)
    bd = _gpu.to_dev(b.reshape(nrhs, -1))
    xd = torch.zeros_like(bd)
    p = bicgstab_params(store_dtype=store)
    info, st = g.dd_solve_bicgstab(p, nrhs, bd, xd, 1e-10)
    x = _gpu.to_host(xd).reshape(b.shape)
    for r in range(nrhs):
        res = np.linalg.norm(b[r] - W.apply(x[r])) / np.linalg.norm(b[r])
        if (name, r) not in _ORACLE:
            _ORACLE[(name, r)] = baseline.dd_solve(W, b[r], 1e-10)
        xo, outer, inner, res_o = _ORACLE[(name, r)]
        d = np.linalg.norm(x[r] - xo) / np.linalg.norm(xo)
        print(f"{name} store {store} rhs {r}: outer {info[r]['outer_iters']} inner {info[r]['inner_iters']} "
              f"relres {res:.2e} | oracle outer {outer} inner {inner} relres {res_o:.2e} | |x - x_oracle| {d:.2e}",
              flush=True)
        assert info[r]["converged"] and res <= 1e-10
        assert d < 1e-8
    g.destroy()


def test_baseline_continues_from_a_guess(ctx):
    """Defect-correction steps one call at a time (starting guess = the previous
    iterate) reach the same tolerance as one call."""
    import torch
    import _gpu
    from paper_1811_00355_amd import Gauge, bicgstab_params
    from workloads import su3_field, gauss_spinor
    L, blk, eps, m0, csw, seed = CASES["c1"]
    g = Gauge(ctx, L, blk, su3_field(L, eps, seed), m0, csw)
    b = _gpu.to_dev(gauss_spinor(L, 2, 69).reshape(2, -1))
    x1 = torch.zeros_like(b)
    info1, _ = g.dd_solve_bicgstab(bicgstab_params(), 2, b, x1, 1e-10)
    x = torch.zeros_like(b)
    p = bicgstab_params(max_outer_iters=1, use_x0=1)
    for k in range(10):
        info, st = g.dd_solve_bicgstab(p, 2, b, x, 1e-10, raise_on_noconv=False)
        if st == 0:
            break
    print(f"one call: {info1[0]['outer_iters']} steps; stepwise: {k + 1} calls", flush=True)
    assert st == 0 and k + 1 == info1[0]["outer_iters"] and all(i["true_relres"] <= 1e-10 for i in info)
    assert torch.equal(x, x1)
    g.destroy()
