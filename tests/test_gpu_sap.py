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


# The benchmark's smoother: 4^4 domains, N_SAP = 4 sweeps, 4 MR steps per domain
# solve, 12 right-hand sides in one call, FP32 arithmetic on FP32 / FP16 / BF16
# stored operands, under every launch layout the autotuner may pick.
HALF_CASE = ((8, 8, 8, 16), (4, 4, 4, 4), 0.2, -0.1, 1.0, 23)
SAP_LAYOUTS = [dict(sap_wpe=2, sap_dom_rhs=0), dict(sap_wpe=3, sap_dom_rhs=0), dict(sap_dom_rhs=4),
               dict(sap_dom_rhs=2), dict(sap_dom_rhs=2, sap_persist=1), dict(sap_dom_rhs=4, sap_persist=1)]
CHECKED_RHS = (0, 7, 11)
_ref_cache = {}


def _stored_oracle(g, U, lat, m0, csw, dtype):
    """The oracle's operator on exactly the operands the library stores for
    `dtype`: links rounded to the storage type, clover and clover inverse as
    exported (FP64) and rounded the way the library rounds them."""
    import _gpu
    from oracle.dirac import WilsonClover, chiral_blocks
    a, ai = g.export_clover()
    W = WilsonClover(_gpu.round_store(U, dtype), lat, m0, csw, A=_gpu.stored_clover_dense(a, dtype))
    W.Ainv_blocks = chiral_blocks(_gpu.stored_clover_dense(ai, dtype))
    return W


@pytest.mark.parametrize("layout", SAP_LAYOUTS, ids=lambda t: "-".join(f"{k}{v}" for k, v in t.items()))
@pytest.mark.parametrize("dtype", [1, 2, 3])
@pytest.mark.parametrize("nrhs", [12, 5])
def test_sap_parity_stored(ctx, dtype, layout, nrhs):
    """SAP with nu = 4, k = 4 and 12 (or 5: a partial group of the domain-resident
    form) RHS against the oracle's SAP run on the stored (rounded) operands with
    the same FP32-rounded inputs; bar 1e-5 (FP32 arithmetic).  Three of the
    right-hand sides are compared (the others share the launch, and batch
    invariance is tested on whole solves).  The domain-resident form applies to
    FP16 / BF16 operands; with FP32 operands that layout runs the per-RHS kernel."""
    import torch
    import _gpu
    from paper_1811_00355_amd import Gauge, default_params
    from oracle.lattice import Lattice
    from oracle import amg
    from workloads import su3_field, gauss_spinor
    L, blk, eps, m0, csw, seed = HALF_CASE
    U = su3_field(L, eps, seed)
    lat = Lattice(L, blk)
    g = Gauge(ctx, L, blk, U, m0, csw)
    t = g.dd_gauge_get_tuning()
    t.update(layout)
    g.dd_gauge_set_tuning(**t)
    sweeps, mr = 4, 4
    b = _gpu.round_f32(gauss_spinor(L, 12, 91))[:nrhs].copy()
    x0 = _gpu.round_f32(gauss_spinor(L, 12, 92) * 0.1)[:nrhs].copy()
    checked = CHECKED_RHS if nrhs == 12 else (0, 2, 4)
    p = default_params(block=blk, sap_sweeps=sweeps, sap_mr_iters=mr)
    print(f"SAP dtype {dtype} layout {layout}: L={L} nrhs={nrhs} nu={sweeps} k={mr}", flush=True)
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
    if dtype not in _ref_cache:
        _ref_cache[dtype] = (_stored_oracle(g, U, lat, m0, csw, dtype), {})
    W, refs = _ref_cache[dtype]
    for r in checked:
        if r not in refs:
            refs[r] = amg.sap(W, b[r], x0[r], sweeps, mr)
    for r in checked:
        err = _gpu.max_rel(out[r], refs[r])
        print(f"  rhs {r}: SAP error vs oracle on stored operands {err:.2e}", flush=True)
        assert err < 1e-5
    g.destroy()


@pytest.mark.parametrize("dom", [2, 4])
@pytest.mark.parametrize("nrhs", [12, 3])
def test_sap_persistent_form_same_bits(ctx, dom, nrhs):
    """All sweeps and both colours in one cooperative launch (grid barrier
    between colours) against one launch per colour: identical bits (BF16
    operands, nu = 4, k = 4)."""
    import torch
    import _gpu
    from paper_1811_00355_amd import Gauge, default_params
    from workloads import su3_field, gauss_spinor
    L, blk, eps, m0, csw, seed = HALF_CASE
    g = Gauge(ctx, L, blk, su3_field(L, eps, seed), m0, csw)
    p = default_params(block=blk, sap_sweeps=4, sap_mr_iters=4)
    b = _gpu.to_dev(_gpu.round_f32(gauss_spinor(L, nrhs, 95)).reshape(nrhs, -1))
    outs = []
    for persist in (0, 1):
        t = g.dd_gauge_get_tuning()
        t.update(sap_dom_rhs=dom, sap_persist=persist)
        g.dd_gauge_set_tuning(**t)
        pb = g.new_packed(3, nrhs)
        px = g.new_packed(3, nrhs)
        g.pack(3, nrhs, b, pb)
        g.dd_sap_smooth(p, 3, nrhs, pb, px)
        torch.cuda.synchronize()
        outs.append(px.clone())
    same = torch.equal(outs[0], outs[1])
    print(f"dom {dom} nrhs {nrhs}: persistent == per-colour launches: {same}", flush=True)
    assert same
    g.destroy()
