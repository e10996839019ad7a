"""GPU parity of field preparation and the operator apply against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = [
    # (L, block, eps, m0, c_sw, seed)
    ((4, 4, 4, 4), (2, 2, 2, 2), 0.3, -0.4, 1.0, 1001),      # the small FP64 case
    ((8, 4, 4, 8), (2, 2, 2, 4), 0.25, -0.2, 1.3, 17),       # asymmetric extents and blocks
    ((8, 8, 8, 16), (4, 4, 4, 4), 0.2, -0.1, 1.0, 23),       # 4^4 domains, several tiles
]


@pytest.fixture(scope="module")
def ctx():
    from paper_1811_00355_amd import Context
    c = Context(0)
    yield c
    c.close()


def _setup(ctx, case):
    from paper_1811_00355_amd import Gauge
    from oracle.lattice import Lattice
    from oracle.dirac import WilsonClover
    from workloads import su3_field
    L, blk, eps, m0, csw, seed = case
    U = su3_field(L, eps, seed)
    lat = Lattice(L, blk)
    W = WilsonClover(U, lat, m0, csw)
    g = Gauge(ctx, L, blk, U, m0, csw)
    return U, lat, W, g


@pytest.mark.parametrize("case", CASES)
def test_maps_and_clover(ctx, case):
    import _gpu
    U, lat, W, g = _setup(ctx, case)
    agg, loc, pidx, col = g.export_maps()
    assert np.array_equal(agg, lat.agg_of_site)
    assert np.array_equal(loc, lat.local_of_site)
    assert np.array_equal(col, lat.color_of_block)
    assert np.array_equal(np.sort(pidx), np.arange(lat.V))
    a, ai = g.export_clover()
    ref = _gpu.packed_oracle_clover(W.A)
    assert _gpu.max_rel(a, ref) < 1e-13
    from oracle.dirac import pack_hermitian6
    refi = pack_hermitian6(W.Ainv_blocks)
    assert _gpu.max_rel(ai, refi) < 1e-12
    g.destroy()


@pytest.mark.parametrize("case", CASES[:2])
def test_operand_storage_bit_exact(ctx, case):
    """The stored FP32 / FP16 / BF16 operand copies are the round-to-nearest-even
    images of the FP64 operands (FP16 and BF16 through FP32): bit-exact."""
    import _gpu
    U, lat, W, g = _setup(ctx, case)
    l64, c64 = g.export_operands(0)
    for dt in (1, 2, 3):
        l, c = g.export_operands(dt)
        for raw, master in ((l, l64), (c, c64)):
            re32 = master.real.astype(np.float32)
            im32 = master.imag.astype(np.float32)
            if dt == 1:
                assert np.array_equal(raw.real, re32) and np.array_equal(raw.imag, im32)
                continue
            if dt == 2:
                lo = re32.astype(np.float16).view(np.uint16).astype(np.uint32)
                hi = im32.astype(np.float16).view(np.uint16).astype(np.uint32)
            else:
                lo = _gpu.bf16_bits(re32)
                hi = _gpu.bf16_bits(im32)
            exp = lo | (hi << 16)
            bad = np.count_nonzero(raw != exp)
            if bad:
                i = np.argwhere(raw != exp)[0]
                print(f"dtype {dt}: {bad} mismatches, first at {tuple(i)}: master {master[tuple(i)]} "
                      f"got {raw[tuple(i)]:#010x} expected {exp[tuple(i)]:#010x}")
            assert bad == 0
    g.destroy()


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("nrhs", [1, 3, 6])
def test_dirac_f64(ctx, case, nrhs):
    import _gpu
    from workloads import gauss_spinor
    U, lat, W, g = _setup(ctx, case)
    psi = gauss_spinor(lat.L, nrhs, 7)
    out = _gpu.fine_apply(g, 0, nrhs, psi, lambda i, o: g.dd_dirac_apply(0, nrhs, i, o))
    for r in range(nrhs):
        assert _gpu.max_rel(out[r], W.apply(psi[r])) < 1e-12
    g.destroy()


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dtype", [1, 2, 3])
@pytest.mark.parametrize("nrhs", [2, 5])
def test_dirac_mixed(ctx, case, dtype, nrhs):
    """FP32 vectors with FP32 / FP16 / BF16 operands, against the oracle run on
    the same (rounded) operands and inputs; the quantisation error against the
    FP64 operator is only reported."""
    import _gpu
    from oracle.dirac import WilsonClover
    from workloads import gauss_spinor
    U, lat, W, g = _setup(ctx, case)
    psi = _gpu.round_f32(gauss_spinor(lat.L, nrhs, 8))
    out = _gpu.fine_apply(g, dtype, nrhs, psi, lambda i, o: g.dd_dirac_apply(dtype, nrhs, i, o))
    a, _ = g.export_clover()
    Uq = _gpu.round_store(U, dtype)
    Aq = _gpu.stored_clover_dense(a, dtype)
    Wq = WilsonClover(Uq, lat, W.m0, W.c_sw, A=Aq)
    for r in range(nrhs):
        ref = Wq.apply(psi[r])
        err = _gpu.max_rel(out[r], ref)
        qerr = _gpu.max_rel(out[r], W.apply(psi[r]))
        print(f"dtype {dtype} rhs {r}: error vs oracle on stored operands {err:.2e}, "
              f"quantisation error vs FP64 operator {qerr:.2e}", flush=True)
        assert err < 1e-5
    g.destroy()
