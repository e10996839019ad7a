"""GPU parity of the third multigrid level against the oracle (oracle/amg3.py):
the level-2 Gram-Schmidt P2, the level-3 operator D3 = P2^dag D_c P2, the
level-2 FGMRES cycle with its level-3 correction and minimal-residual smoother
(fixed iteration counts, FP64), the FP32 form of the same cycle, D3 rebuilt
after a mass change, properties of device-generated level-2 vectors, and whole
solves with three levels to a true residual of 1e-10.  Oracle inputs are the
host's seeded fields and vectors only."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = {
    # name: (L, block, eps, m0, c_sw, seed, n, n2); every coarse extent a multiple of 4
    "l8": ((8, 8, 8, 8), (2, 2, 2, 2), 0.3, -0.4, 1.0, 301, 8, 6),
    "l8x16": ((8, 8, 8, 16), (2, 2, 2, 2), 0.25, -0.2, 1.3, 302, 6, 8),
}


@pytest.fixture(scope="module")
def ctx():
    from paper_1811_00355_amd import Context
    c = Context(0)
    yield c
    c.close()


def _build(ctx, name, smooth=False, **pkw):
    """Setup from host vectors: Gaussian, or (smooth) one application of the
    oracle's SAP to each, normalised (vectors with low-mode content)."""
    from paper_1811_00355_amd import Gauge, MG, default_params
    from oracle import amg
    from oracle.lattice import Lattice
    from oracle.dirac import WilsonClover
    from workloads import su3_field, gauss_vectors
    L, blk, eps, m0, csw, seed, n, n2 = CASES[name]
    U = su3_field(L, eps, seed)
    lat = Lattice(L, blk)
    W = WilsonClover(U, lat, m0, csw)
    g = Gauge(ctx, L, blk, U, m0, csw)
    tv0 = gauss_vectors(n, lat.V, seed + 7).reshape(n, lat.V, 4, 3)
    if smooth:
        tv0 = np.array([amg.sap(W, v, np.zeros_like(v), 4, 4) for v in tv0])
        tv0 /= np.linalg.norm(tv0.reshape(n, -1), axis=1)[:, None, None, None]
    kw = dict(block=blk, n_vec=n, inner_dtype=0, store_dtype=0, init_sap_apps=0, setup_iters=0)
    kw.update(pkw)
    p = default_params(**kw)
    print(f"case {name}: L={L} block={blk} n={n} n2={n2} params={kw}", flush=True)
    mg = MG(g, p, tv_host=tv0)
    tv2 = gauss_vectors(n2, lat.Vc, seed + 11, ncomp=2 * n)
    return dict(U=U, lat=lat, W=W, g=g, mg=mg, tv0=tv0, tv2=tv2, n=n, n2=n2, p=p, L=L, blk=blk, m0=m0, csw=csw)


def _close(d):
    d["mg"].destroy()
    d["g"].destroy()


def _oracle_coarse(d, tv=None, W=None):
    from oracle import amg
    Pb = amg.gram_schmidt(d["lat"], d["tv0"] if tv is None else tv)
    return Pb, amg.coarse_operator(d["W"] if W is None else W, Pb)


def _coarse_roundtrip(mg, dtype, nrhs, vin, fn):
    import torch
    import _gpu
    cin = _gpu.to_dev(vin.reshape(nrhs, -1))
    pin = mg.new_coarse(dtype, nrhs)
    pout = mg.new_coarse(dtype, nrhs)
    mg.pack_coarse(dtype, nrhs, cin, pin)
    fn(pin, pout)
    cout = torch.zeros_like(cin)
    mg.unpack_coarse(dtype, nrhs, pout, cout)
    torch.cuda.synchronize()
    return _gpu.to_host(cout).reshape(vin.shape)


@pytest.mark.parametrize("name", list(CASES))
def test_level3_P2_and_operator(ctx, name):
    """Given level-2 vectors: the stored vectors round-trip bit for bit, P2 and
    D3 agree with the oracle's Gram-Schmidt and Galerkin product to 1e-12."""
    import _gpu
    from oracle import amg3
    from paper_1811_00355_amd import level3_params
    d = _build(ctx, name)
    lat, mg, n, n2 = d["lat"], d["mg"], d["n"], d["n2"]
    _, Dc = _oracle_coarse(d)
    mg.add_level(level3_params(n_vec2=n2), tv2_host=d["tv2"])
    lev = amg3.Level2Lattice(lat)
    vc3, nc3 = mg.level3_shape()
    assert (vc3, nc3) == (lev.Vc3, 2 * n2)
    tv2, P2, D3 = mg.export_level3()
    assert np.array_equal(tv2, d["tv2"])
    P2_ref = amg3.gram_schmidt2(lev, n, d["tv2"])
    D3_ref = amg3.galerkin3(lev, n, Dc, P2_ref)
    e_p, e_d = _gpu.max_rel(P2, P2_ref), _gpu.max_rel(D3, D3_ref)
    print(f"{name}: Vc3={vc3} nc3={nc3}: P2 error {e_p:.2e}, D3 error {e_d:.2e}", flush=True)
    assert e_p < 1e-12 and e_d < 1e-12
    _close(d)


@pytest.mark.parametrize("name", list(CASES))
def test_level2_cycle_fixed_iterations(ctx, name):
    """The coarse solve with a third level (level-2 FGMRES, fixed step counts,
    FP64) equals the oracle's cycle to 1e-10; chunk graphs (modes 1 and 2)
    replay the same launches and give the same bits."""
    import _gpu
    from oracle import amg, amg3
    from paper_1811_00355_amd import level3_params
    from workloads import gauss_vectors
    d = _build(ctx, name)
    lat, mg, n, n2 = d["lat"], d["mg"], d["n"], d["n2"]
    _, Dc = _oracle_coarse(d)
    kw = dict(n_vec2=n2, mr_steps=3, kcycle_max_iters=5, kcycle_fixed=1, l3_restart=4, l3_fixed_iters=7)
    mg.add_level(level3_params(**kw), tv2_host=d["tv2"])
    p3 = amg3.L3Params(n_vec2=n2, mr_steps=3, kcycle_max_iters=5, kcycle_fixed=True, l3_restart=4, l3_fixed_iters=7)
    tlc = amg3.ThreeLevelCoarse(lat, n, Dc, d["tv2"], p3, amg.MGParams(n_vec=n))
    nrhs = 3
    b = gauss_vectors(nrhs, lat.Vc, 41, ncomp=2 * n)
    got = _coarse_roundtrip(mg, 0, nrhs, b, lambda i, o: mg.dd_coarse_solve(0, nrhs, i, o))
    steps, l3 = mg.level3_last()
    print(f"{name}: level-2 steps {steps}, level-3 steps {l3}", flush=True)
    assert steps == 5 and l3 == 5 * 7
    for r in range(nrhs):
        err = _gpu.max_rel(got[r], tlc(b[r]))
        print(f"{name}: level-2 cycle rhs {r}: {err:.2e}", flush=True)
        assert err < 1e-10
    for mode in (1, 2):
        mg.dd_mg_set_graphs(mode)
        again = _coarse_roundtrip(mg, 0, nrhs, b, lambda i, o: mg.dd_coarse_solve(0, nrhs, i, o))
        assert np.array_equal(again, got), f"graph mode {mode}"
    _close(d)


def test_level2_cycle_tolerance_and_f32(ctx):
    """Tolerance mode: every right-hand side's level-2 residual meets
    kcycle_tol on the oracle's D_c.  FP32 form (FP32 vectors, P2 and blocks):
    the fixed-step cycle stays within 1e-4 of the oracle's FP64 cycle."""
    import _gpu
    from oracle import amg, amg3
    from paper_1811_00355_amd import level3_params
    from workloads import gauss_vectors
    d = _build(ctx, "l8")
    lat, mg, n, n2 = d["lat"], d["mg"], d["n"], d["n2"]
    _, Dc = _oracle_coarse(d)
    mg.add_level(level3_params(n_vec2=n2, kcycle_tol=1e-3, kcycle_max_iters=40, l3_tol=1e-2), tv2_host=d["tv2"])
    nrhs = 2
    b = gauss_vectors(nrhs, lat.Vc, 42, ncomp=2 * n)
    got = _coarse_roundtrip(mg, 0, nrhs, b, lambda i, o: mg.dd_coarse_solve(0, nrhs, i, o))
    for r in range(nrhs):
        res = np.linalg.norm(b[r] - amg.coarse_apply(lat, Dc, got[r])) / np.linalg.norm(b[r])
        print(f"tolerance mode rhs {r}: level-2 residual {res:.2e} (steps {mg.level3_last()})", flush=True)
        assert res <= 1e-3 * 1.01
    _close(d)
    # FP32 setup from the same vectors
    d = _build(ctx, "l8", inner_dtype=1, store_dtype=1)
    lat, mg = d["lat"], d["mg"]
    Pb = amg.gram_schmidt(lat, _gpu.round_f32(d["tv0"]))
    Dc_p32 = amg.coarse_operator(d["W"], _gpu.round_f32(Pb))   # the FP64 Galerkin product of the stored FP32 P
    kw = dict(n_vec2=n2, mr_steps=2, kcycle_max_iters=4, kcycle_fixed=1, l3_restart=4, l3_fixed_iters=6)
    mg.add_level(level3_params(**kw), tv2_host=d["tv2"])
    p3 = amg3.L3Params(n_vec2=n2, mr_steps=2, kcycle_max_iters=4, kcycle_fixed=True, l3_restart=4, l3_fixed_iters=6)
    tlc = amg3.ThreeLevelCoarse(lat, n, Dc_p32, d["tv2"], p3, amg.MGParams(n_vec=n))
    got = _coarse_roundtrip(mg, 1, nrhs, b, lambda i, o: mg.dd_coarse_solve(1, nrhs, i, o))
    for r in range(nrhs):
        err = _gpu.max_rel(got[r], tlc(b[r]))
        print(f"FP32 level-2 cycle rhs {r}: {err:.2e}", flush=True)
        assert err < 1e-4
    _close(d)


def test_level3_after_mass_change(ctx):
    """dd_setup_update_mass rebuilds D3 from the kept P2: equal to the oracle's
    P2^dag D_c P2 at the new mass (1e-12), P2 unchanged bit for bit."""
    import _gpu
    from oracle import amg3
    from oracle.dirac import WilsonClover
    from paper_1811_00355_amd import level3_params
    d = _build(ctx, "l8x16")
    lat, mg, n, n2 = d["lat"], d["mg"], d["n"], d["n2"]
    lev = amg3.Level2Lattice(lat)
    mg.add_level(level3_params(n_vec2=n2), tv2_host=d["tv2"])
    _, P2, _ = mg.export_level3()
    P2_ref = amg3.gram_schmidt2(lev, n, d["tv2"])
    m1 = d["m0"] + 0.1
    mg.dd_setup_update_mass(m1)
    _, Dc1 = _oracle_coarse(d, W=WilsonClover(d["U"], lat, m1, d["csw"]))
    _, P2b, D3b = mg.export_level3()
    assert np.array_equal(P2b, P2)
    e = _gpu.max_rel(D3b, amg3.galerkin3(lev, n, Dc1, P2_ref))
    print(f"D3 after the mass change: {e:.2e}", flush=True)
    assert e < 1e-12
    _close(d)


def test_level3_device_vectors_properties(ctx):
    """Level-2 vectors made on the device are checked by properties, never fed
    to the oracle.  The level-1 vectors are smoothed by the oracle's SAP on the
    host (so that D_c has low modes), and the device draws its level-2 vectors
    from one seed twice: raw (no inverse iteration) and after two inverse
    iterations with the two-level coarse solve.  Both give P2 sets that are
    orthonormal and a Gamma5-hermitian D3; the iterated vectors have a smaller
    mean |D_c v| / |v| on the oracle's D_c than the raw ones."""
    from oracle import amg, amg3
    from paper_1811_00355_amd import level3_params
    d = _build(ctx, "l8", smooth=True)
    lat, mg, n2 = d["lat"], d["mg"], d["n2"]
    lev = amg3.Level2Lattice(lat)
    _, Dc = _oracle_coarse(d)
    nb = amg.coarse_neighbors(lev.lat3)
    nc3 = 2 * n2
    g5 = np.tile(np.r_[np.ones(n2), -np.ones(n2)], lev.Vc3)

    def ratio(v):
        return float(np.mean([np.linalg.norm(amg.coarse_apply(lat, Dc, v[i])) / np.linalg.norm(v[i])
                              for i in range(v.shape[0])]))

    ratios = []
    for its in (0, 2):
        mg.add_level(level3_params(n_vec2=n2, setup_iters=its, seed=77))
        tv2, P2, D3 = mg.export_level3()
        mg.remove_level()
        gram = np.einsum("xsik,xsjk->xsij", np.conj(P2), P2)
        e_o = float(np.abs(gram - np.eye(n2)).max())
        D = np.zeros((lev.Vc3 * nc3, lev.Vc3 * nc3), dtype=np.complex128)
        for x in range(lev.Vc3):
            for dd in range(9):
                y = nb[dd][x]
                D[x * nc3:(x + 1) * nc3, y * nc3:(y + 1) * nc3] += D3[x, dd]
        e_h = float(np.abs(g5[:, None] * D * g5[None, :] - D.conj().T).max() / np.abs(D).max())
        ratios.append(ratio(tv2))
        print(f"{its} inverse iterations: orthonormality {e_o:.1e}, gamma5-hermiticity {e_h:.1e}, "
              f"mean |D_c v|/|v| {ratios[-1]:.3f}", flush=True)
        assert e_o < 1e-12 and e_h < 1e-12
    assert ratios[1] < 0.95 * ratios[0]
    _close(d)


@pytest.mark.parametrize("inner,store,half", [(0, 0, 0), (1, 1, 0), (1, 3, 0), (1, 2, 1), (1, 3, 1)])
def test_three_level_solve_true_residual(ctx, inner, store, half):
    """Whole solves with three levels (device-generated level-2 vectors, the
    default cycle) reach |b - D x| / |b| <= 1e-10 on the oracle's operator;
    also with the half-precision coarse options (D_c and D3 blocks in the
    storage type on half matrix cores, FP16 Krylov bases on both levels)."""
    import torch
    import _gpu
    from paper_1811_00355_amd import level3_params
    from workloads import gauss_spinor
    d = _build(ctx, "l8x16", inner_dtype=inner, store_dtype=store, init_sap_apps=2, setup_iters=2)
    lat, mg = d["lat"], d["mg"]
    if half:
        t = d["g"].dd_gauge_get_tuning()
        d["g"].dd_gauge_set_tuning(**dict(t, coarse_half=1, coarse_basis_half=1, coarse_mfma_half=1))
    nrhs = 3
    b = gauss_spinor(lat.L, nrhs, 63)
    bd = _gpu.to_dev(b.reshape(nrhs, -1))
    xd = torch.zeros_like(bd)
    info2, _ = mg.dd_solve(nrhs, bd, xd, 1e-10)
    mg.add_level(level3_params(n_vec2=d["n2"]))
    xd.zero_()
    info, _ = mg.dd_solve(nrhs, bd, xd, 1e-10)
    torch.cuda.synchronize()
    x = _gpu.to_host(xd).reshape(b.shape)
    for r in range(nrhs):
        res = np.linalg.norm(b[r] - d["W"].apply(x[r])) / np.linalg.norm(b[r])
        print(f"inner={inner} store={store} half={half} rhs {r}: outer iterations {info[r]['outer_iters']} with three levels, "
              f"{info2[r]['outer_iters']} with two; relres(oracle D) {res:.2e}", flush=True)
        assert info[r]["converged"] and res <= 1e-10
    _close(d)


def test_level3_limits(ctx):
    """Errors: a second level, unsupported n_vec2, coarse extents that are not
    multiples of 4, the allocation-free coarse solve with a third level; after
    removing the level the coarse solve is the two-level one again, bit for bit."""
    import _gpu
    from paper_1811_00355_amd import level3_params, DDError
    from workloads import gauss_vectors
    d = _build(ctx, "l8")
    lat, mg, n, n2 = d["lat"], d["mg"], d["n"], d["n2"]
    nrhs = 2
    b = gauss_vectors(nrhs, lat.Vc, 43, ncomp=2 * n)
    two = _coarse_roundtrip(mg, 0, nrhs, b, lambda i, o: mg.dd_coarse_solve(0, nrhs, i, o))
    with pytest.raises(DDError):
        mg.add_level(level3_params(n_vec2=7))
    mg.add_level(level3_params(n_vec2=n2), tv2_host=d["tv2"])
    with pytest.raises(DDError):
        mg.add_level(level3_params(n_vec2=n2))
    with pytest.raises(DDError):
        _coarse_roundtrip(mg, 0, nrhs, b, lambda i, o: mg.dd_coarse_solve_noalloc(0, nrhs, i, o))
    three = _coarse_roundtrip(mg, 0, nrhs, b, lambda i, o: mg.dd_coarse_solve(0, nrhs, i, o))
    assert not np.array_equal(three, two)
    mg.remove_level()
    assert mg.level3_shape() == (0, 0)
    again = _coarse_roundtrip(mg, 0, nrhs, b, lambda i, o: mg.dd_coarse_solve(0, nrhs, i, o))
    assert np.array_equal(again, two)
    _close(d)
    # 8^3x16 in 4^4 blocks: coarse extents 2, 2, 2, 4
    from paper_1811_00355_amd import Gauge, MG, default_params
    from workloads import su3_field
    from oracle.lattice import Lattice
    L, blk = (8, 8, 8, 16), (4, 4, 4, 4)
    g = Gauge(ctx, L, blk, su3_field(L, 0.2, 5), -0.1, 1.0)
    tv0 = gauss_vectors(6, Lattice(L, blk).V, 6).reshape(6, -1, 4, 3)
    mg = MG(g, default_params(block=blk, n_vec=6, inner_dtype=0, store_dtype=0, init_sap_apps=0, setup_iters=0),
            tv_host=tv0)
    with pytest.raises(DDError):
        mg.add_level(level3_params(n_vec2=6))
    mg.destroy()
    g.destroy()


def test_three_level_batch_invariance_and_graphs(ctx):
    """With a third level (FP32 inner arithmetic, the benchmark's form), a
    right-hand side solved alone and inside a batch gives the same bits and
    the same outer iteration count (every reduction of the level-2 cycle, its
    smoother and the level-3 GMRES is per right-hand side and blocked
    independently of the batch; finished right-hand sides are masked), and
    graph mode 1 (level-3 GMRES chunks replayed) gives the bits of mode 0."""
    import torch
    import _gpu
    from paper_1811_00355_amd import level3_params
    from workloads import gauss_spinor
    d = _build(ctx, "l8x16", inner_dtype=1, store_dtype=1, init_sap_apps=2, setup_iters=2)
    lat, mg = d["lat"], d["mg"]
    mg.add_level(level3_params(n_vec2=d["n2"], setup_iters=2, mr_steps=4, kcycle_max_iters=20))
    nrhs = 4
    b = gauss_spinor(lat.L, nrhs, 64)
    b[1] = 0.0
    b[1, 0, 0, 0] = 1.0
    b[2] = d["W"].apply(b[2])
    b[3] = 0.0
    bd = _gpu.to_dev(b.reshape(nrhs, -1))
    xd = torch.zeros_like(bd)
    info, _ = mg.dd_solve(nrhs, bd, xd, 1e-10)
    for r in range(nrhs):
        xr = torch.zeros_like(bd[r:r + 1])
        ir, _ = mg.dd_solve(1, bd[r:r + 1].contiguous(), xr, 1e-10)
        torch.cuda.synchronize()
        same = torch.equal(xr[0], xd[r])
        print(f"rhs {r}: batch iters {info[r]['outer_iters']} alone {ir[0]['outer_iters']} bitwise equal {same}",
              flush=True)
        assert ir[0]["outer_iters"] == info[r]["outer_iters"] and same
    assert len({i["outer_iters"] for i in info}) >= 2, "every source converged together: masking not exercised"
    mg.dd_mg_set_graphs(1)
    xg = torch.zeros_like(bd)
    info_g, _ = mg.dd_solve(nrhs, bd, xg, 1e-10)
    torch.cuda.synchronize()
    assert torch.equal(xg, xd) and [i["outer_iters"] for i in info_g] == [i["outer_iters"] for i in info]
    _close(d)
