"""GPU parity of the SAP smoother against the oracle (same sweeps, same fixed
MR count, same red-black order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), (2, 2, 2, 2), 0.3, -0.4, 1.0, 1001),
    ((8, 4, 4, 8), (2, 2, 2, 4), 0.25, -0.2, 1.3, 17),
    ((8, 8, 8, 16), (4, 4, 4, 4), 0.2, -0.1, 1.0, 23),
]


@pytest.fixture(scope="module")
def ctx():
    from paper_1811_00355_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dtype", [0, 1])
def test_sap_parity(ctx, case, dtype):
    import _gpu
    from paper_1811_00355_amd import Gauge, default_params
    from oracle.lattice import Lattice
    from oracle.dirac import WilsonClover
    from oracle import amg
    from workloads import su3_field, gauss_spinor
    L, blk, eps, m0, csw, seed = case
    U = su3_field(L, eps, seed)
    lat = Lattice(L, blk)
    g = Gauge(ctx, L, blk, U, m0, csw)
    nrhs = 2
    b = gauss_spinor(L, nrhs, 3)
    x0 = gauss_spinor(L, nrhs, 4) * 0.1
    if dtype == 1:
        b, x0 = _gpu.round_f32(b), _gpu.round_f32(x0)
        a, ai = g.export_clover()
        W = WilsonClover(_gpu.round_f32(U), lat, m0, csw, A=_gpu.stored_clover_dense(a, 1))
        # the library stores the FP32-rounded FP64 inverse: the oracle uses exactly that
        from oracle.dirac import chiral_blocks
        W.Ainv_blocks = chiral_blocks(_gpu.stored_clover_dense(ai, 1))
    else:
        W = WilsonClover(U, lat, m0, csw)
    sweeps, mr = 2, 3
    p = default_params(block=blk, sap_sweeps=sweeps, sap_mr_iters=mr)
    import torch
    cb = _gpu.to_dev(b.reshape(nrhs, -1))
    cx = _gpu.to_dev(x0.reshape(nrhs, -1))
    pb = g.new_packed(dtype, nrhs)
    px = g.new_packed(dtype, nrhs)
    g.pack(dtype, nrhs, cb, pb)
    g.pack(dtype, nrhs, cx, px)
    g.dd_sap_smooth(p, dtype, nrhs, pb, px)
    out = torch.zeros_like(cx)
    g.unpack(dtype, nrhs, px, out)
    torch.cuda.synchronize()
    out = _gpu.to_host(out).reshape(b.shape)
    tol = 1e-12 if dtype == 0 else 1e-5
    for r in range(nrhs):
        ref = amg.sap(W, b[r], x0[r], sweeps, mr)
        err = _gpu.max_rel(out[r], ref)
        print(f"L={L} dtype={dtype} rhs={r}: SAP error {err:.2e}", flush=True)
        assert err < tol
    g.destroy()
