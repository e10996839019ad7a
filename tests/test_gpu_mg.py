"""GPU parity of the multigrid pieces against the oracle: Gram-Schmidt, P, R,
the Galerkin coarse operator, its stencil apply, the even-odd coarse solve in
fixed-iteration mode, the V-cycle, the adaptive setup, and whole solves
(true residual rechecked with the oracle's operator)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = {
    # name: (L, block, eps, m0, c_sw, seed, n)
    "c1": ((4, 4, 4, 4), (2, 2, 2, 2), 0.3, -0.4, 1.0, 1001, 8),
    "asym": ((8, 4, 4, 8), (2, 2, 2, 4), 0.25, -0.2, 1.3, 17, 6),
    "b4": ((8, 8, 8, 16), (4, 4, 4, 4), 0.2, -0.1, 1.0, 23, 20),
}
# 2n = 48, the largest coarse block the matrix-core applies take (the 48^3x96 workload's n = 24)
EXTRA = {"b4n24": ((8, 8, 8, 16), (4, 4, 4, 4), 0.2, -0.1, 1.0, 23, 24)}


@pytest.fixture(scope="module")
def ctx():
    from paper_1811_00355_amd import Context
    c = Context(0)
    yield c
    c.close()


def _build(ctx, name, **pkw):
    from paper_1811_00355_amd import Gauge, MG, default_params
    from oracle.lattice import Lattice
    from oracle.dirac import WilsonClover
    from workloads import su3_field, gauss_vectors
    L, blk, eps, m0, csw, seed, n = {**CASES, **EXTRA}[name]
    U = su3_field(L, eps, seed)
    lat = Lattice(L, blk)
    W = WilsonClover(U, lat, m0, csw)
    g = Gauge(ctx, L, blk, U, m0, csw)
    tv0 = gauss_vectors(n, lat.V, seed + 7).reshape(n, lat.V, 4, 3)
    kw = dict(block=blk, n_vec=n, inner_dtype=0, store_dtype=0, init_sap_apps=0, setup_iters=0)
    kw.update(pkw)
    p = default_params(**kw)
    print(f"case {name}: L={L} block={blk} n={n} params={kw}", flush=True)
    mg = MG(g, p, tv_host=tv0)
    return dict(U=U, lat=lat, W=W, g=g, mg=mg, tv0=tv0, n=n, p=p)


def _close(d):
    d["mg"].destroy()
    d["g"].destroy()


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
def test_build_P_and_coarse_operator(ctx, name):
    import _gpu
    from oracle import amg
    d = _build(ctx, name)
    lat, mg = d["lat"], d["mg"]
    Pb = amg.gram_schmidt(lat, d["tv0"])
    P_ref = amg.from_aggregates(lat, np.moveaxis(Pb, 2, 0))   # [n][V][4][3]
    P_gpu = mg.export_vectors()
    err = _gpu.max_rel(P_gpu, P_ref)
    print(f"P error {err:.2e}", flush=True)
    assert err < 1e-12
    Dc_ref = amg.coarse_operator(d["W"], Pb)
    Dc_gpu = mg.export_coarse()
    err = _gpu.max_rel(Dc_gpu, Dc_ref)
    print(f"D_c error {err:.2e}", flush=True)
    assert err < 1e-12
    _close(d)


@pytest.mark.parametrize("name", list(CASES))
def test_restrict_prolong_coarse_apply(ctx, name):
    import _gpu
    from oracle import amg
    from workloads import gauss_spinor, gauss_vectors
    d = _build(ctx, name)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    Pb = amg.gram_schmidt(lat, d["tv0"])
    Dc = amg.coarse_operator(d["W"], Pb)
    nrhs = 3
    f = gauss_spinor(lat.L, nrhs, 31)
    c = gauss_vectors(nrhs, lat.Vc, 32, ncomp=2 * n)
    for dtype, tol in ((0, 1e-12), (1, 1e-5)):
        fr = f if dtype == 0 else _gpu.round_f32(f)
        cr = c if dtype == 0 else _gpu.round_f32(c)
        Pr = Pb if dtype == 0 else _gpu.round_f32(Pb)
        Dr = Dc if dtype == 0 else _gpu.round_f32(Dc)
        # restriction
        import torch
        fin = _gpu.to_dev(fr.reshape(nrhs, -1))
        pf = d["g"].new_packed(dtype, nrhs)
        d["g"].pack(dtype, nrhs, fin, pf)
        pc = mg.new_coarse(dtype, nrhs)
        mg.dd_restrict(dtype, nrhs, pf, pc)
        cout = torch.zeros((nrhs, lat.Vc * 2 * n), dtype=torch.complex128, device="cuda")
        mg.unpack_coarse(dtype, nrhs, pc, cout)
        torch.cuda.synchronize()
        got = _gpu.to_host(cout).reshape(nrhs, lat.Vc, 2 * n)
        for r in range(nrhs):
            assert _gpu.max_rel(got[r], amg.restrict(lat, Pr, fr[r])) < tol
        # prolongation
        cin = _gpu.to_dev(cr.reshape(nrhs, -1))
        pc2 = mg.new_coarse(dtype, nrhs)
        mg.pack_coarse(dtype, nrhs, cin, pc2)
        pf2 = d["g"].new_packed(dtype, nrhs)
        mg.dd_prolong(dtype, nrhs, pc2, pf2)
        fout = torch.zeros((nrhs, lat.V * 12), dtype=torch.complex128, device="cuda")
        d["g"].unpack(dtype, nrhs, pf2, fout)
        torch.cuda.synchronize()
        got = _gpu.to_host(fout).reshape(nrhs, lat.V, 4, 3)
        for r in range(nrhs):
            assert _gpu.max_rel(got[r], amg.prolong(lat, Pr, cr[r])) < tol
        # coarse stencil
        got = _coarse_roundtrip(mg, dtype, nrhs, cr, lambda i, o: mg.dd_coarse_apply(dtype, nrhs, i, o))
        for r in range(nrhs):
            err = _gpu.max_rel(got[r], amg.coarse_apply(lat, Dr, cr[r]))
            print(f"dtype {dtype} coarse apply rhs {r}: {err:.2e}", flush=True)
            assert err < tol
    _close(d)


@pytest.mark.parametrize("name", ["c1", "b4"])
def test_coarse_solve_fixed_iterations(ctx, name):
    """Fixed iteration count, no tolerance stop: GMRES on the even-odd Schur
    complement and the odd reconstruction agree with the oracle in FP64."""
    import _gpu
    from oracle import amg
    from workloads import gauss_vectors
    d = _build(ctx, name, coarse_fixed_iters=12, coarse_restart=5)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    Pb = amg.gram_schmidt(lat, d["tv0"])
    ceo = amg.CoarseEO(lat, amg.coarse_operator(d["W"], Pb))
    op = amg.MGParams(n_vec=n, coarse_fixed_iters=12, coarse_restart=5)
    nrhs = 2
    b = gauss_vectors(nrhs, lat.Vc, 41, ncomp=2 * n)
    got = _coarse_roundtrip(mg, 0, nrhs, b, lambda i, o: mg.dd_coarse_solve(0, nrhs, i, o))
    for r in range(nrhs):
        err = _gpu.max_rel(got[r], ceo.solve(b[r], op))
        print(f"coarse solve rhs {r}: {err:.2e}", flush=True)
        assert err < 1e-10
    _close(d)


@pytest.mark.parametrize("name", ["c1", "b4"])
def test_vcycle_fixed_iterations(ctx, name):
    import _gpu
    from oracle import amg
    from workloads import gauss_spinor
    d = _build(ctx, name, coarse_fixed_iters=10, coarse_restart=10, sap_sweeps=2, sap_mr_iters=3)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    op = amg.MGParams(n_vec=n, coarse_fixed_iters=10, coarse_restart=10, sap_sweeps=2, sap_mr_iters=3)
    two = amg.TwoLevel(d["W"], d["tv0"], op)
    nrhs = 2
    v = gauss_spinor(lat.L, nrhs, 51)
    got = _gpu.fine_apply(d["g"], 0, nrhs, v, lambda i, o: mg.dd_precond_apply(nrhs, i, o))
    for r in range(nrhs):
        err = _gpu.max_rel(got[r], two.vcycle(v[r]))
        print(f"V-cycle rhs {r}: {err:.2e}", flush=True)
        assert err < 1e-10
    _close(d)


def test_adaptive_setup_fixed_iterations(ctx):
    """init SAP solves + one adaptive iteration, coarse GMRES with a fixed count:
    the produced P and D_c agree with the oracle's setup in FP64."""
    import _gpu
    from oracle import amg
    d = _build(ctx, "c1", init_sap_apps=1, setup_iters=1, coarse_fixed_iters=8, coarse_restart=8)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    op = amg.MGParams(n_vec=n, init_sap_apps=1, setup_iters=1, coarse_fixed_iters=8, coarse_restart=8)
    ref = amg.setup(d["W"], op, d["tv0"])
    P_ref = amg.from_aggregates(lat, np.moveaxis(ref.Pb, 2, 0))
    e1 = _gpu.max_rel(mg.export_vectors(), P_ref)
    e2 = _gpu.max_rel(mg.export_coarse(), ref.Dc)
    print(f"setup: P error {e1:.2e}, D_c error {e2:.2e}", flush=True)
    assert e1 < 1e-10 and e2 < 1e-10
    _close(d)


@pytest.mark.parametrize("name,inner,store,outer_passes",
                         [("c1", 0, 0, 2), ("c1", 1, 1, 2), ("b4", 1, 1, 2), ("b4", 1, 3, 2), ("b4", 1, 3, 1),
                          ("c1", 0, 0, 1)])
def test_solve_true_residual(ctx, name, inner, store, outer_passes):
    """Whole solve: every RHS reaches |b - D x| / |b| <= 1e-10, recomputed with the
    oracle's FP64 operator on the host (outer FGMRES with one or two classical
    Gram-Schmidt passes)."""
    import torch
    import _gpu
    from workloads import gauss_spinor
    d = _build(ctx, name, inner_dtype=inner, store_dtype=store, init_sap_apps=2, setup_iters=2,
               outer_cgs_passes=outer_passes)
    lat, mg = d["lat"], d["mg"]
    nrhs = 3
    b = gauss_spinor(lat.L, nrhs, 61)
    bd = _gpu.to_dev(b.reshape(nrhs, -1))
    xd = torch.zeros_like(bd)
    info, st = mg.dd_solve(nrhs, bd, xd, 1e-10)
    torch.cuda.synchronize()
    x = _gpu.to_host(xd).reshape(b.shape)
    for r in range(nrhs):
        res = np.linalg.norm(b[r] - d["W"].apply(x[r])) / np.linalg.norm(b[r])
        print(f"{name} inner={inner} store={store} outer passes {outer_passes} rhs {r}: iters {info[r]['outer_iters']} "
              f"relres(lib) {info[r]['true_relres']:.2e} relres(oracle D) {res:.2e}", flush=True)
        assert info[r]["converged"] and res <= 1e-10
    _close(d)


@pytest.mark.parametrize("nrhs", [1, 12, 20])
def test_coarse_apply_f32_batches(ctx, nrhs):
    """FP32 coarse stencil (matrix-core path) over right-hand-side batches that
    fill one, one padded and two 16-wide passes, against the oracle on the
    FP32-rounded operator and inputs."""
    import _gpu
    from oracle import amg
    from workloads import gauss_vectors
    d = _build(ctx, "b4")
    lat, mg, n = d["lat"], d["mg"], d["n"]
    Dr = _gpu.round_f32(amg.coarse_operator(d["W"], amg.gram_schmidt(lat, d["tv0"])))
    c = _gpu.round_f32(gauss_vectors(nrhs, lat.Vc, 71, ncomp=2 * n))
    got = _coarse_roundtrip(mg, 1, nrhs, c, lambda i, o: mg.dd_coarse_apply(1, nrhs, i, o))
    errs = [_gpu.max_rel(got[r], amg.coarse_apply(lat, Dr, c[r])) for r in range(nrhs)]
    print(f"FP32 coarse apply, {nrhs} rhs: max error {max(errs):.2e}", flush=True)
    assert max(errs) < 1e-5
    _close(d)


def test_coarse_solve_f32_fixed_iterations(ctx):
    """FP32 even-odd coarse GMRES (matrix-core stencil), fixed iteration count,
    12 right-hand sides, against the oracle on the FP32-rounded operator."""
    import _gpu
    from oracle import amg
    from workloads import gauss_vectors
    d = _build(ctx, "b4", coarse_fixed_iters=10, coarse_restart=10)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    Dr = _gpu.round_f32(amg.coarse_operator(d["W"], amg.gram_schmidt(lat, d["tv0"])))
    ceo = amg.CoarseEO(lat, Dr)
    op = amg.MGParams(n_vec=n, coarse_fixed_iters=10, coarse_restart=10)
    nrhs = 12
    b = _gpu.round_f32(gauss_vectors(nrhs, lat.Vc, 72, ncomp=2 * n))
    got = _coarse_roundtrip(mg, 1, nrhs, b, lambda i, o: mg.dd_coarse_solve(1, nrhs, i, o))
    errs = [_gpu.max_rel(got[r], ceo.solve(b[r], op)) for r in range(nrhs)]
    print(f"FP32 coarse solve, 12 rhs: max error {max(errs):.2e}", flush=True)
    assert max(errs) < 1e-4
    _close(d)


@pytest.mark.parametrize("inner,store", [(0, 0), (1, 1)])
def test_update_mass_reuses_vectors(ctx, inner, store):
    """"New kappa": switching an existing setup to another bare mass keeps P and
    rebuilds D_c.  The result equals the oracle's P^dag D(m0') P (to 1e-12 in the
    all-FP64 form; in the FP32 form P is rounded to FP32, vectors before and after
    Gram-Schmidt, and a one-ulp difference of a rounded entry is allowed) and, bit
    for bit, a fresh setup from the same vectors on a field created at m0'.  A
    solve at the new mass then meets the true-residual bar."""
    import torch
    import _gpu
    from oracle import amg
    from oracle.dirac import WilsonClover
    from paper_1811_00355_amd import Gauge, MG
    from workloads import gauss_spinor
    d = _build(ctx, "b4", inner_dtype=inner, store_dtype=store)
    lat, mg = d["lat"], d["mg"]
    L, blk, eps, m0, csw, seed, n = CASES["b4"]
    m1 = m0 + 0.15
    P_before = mg.export_vectors()
    mg.dd_setup_update_mass(m1)
    W1 = WilsonClover(d["U"], lat, m1, csw)
    if inner == 0:
        Pb, tol = amg.gram_schmidt(lat, d["tv0"]), 1e-12
    else:
        Pb, tol = _gpu.round_f32(amg.gram_schmidt(lat, _gpu.round_f32(d["tv0"]))), 1e-6
    err = _gpu.max_rel(mg.export_coarse(), amg.coarse_operator(W1, Pb))
    print(f"inner={inner}: updated D_c vs oracle at m0'={m1:.3f}: {err:.2e}", flush=True)
    assert err < tol
    assert np.array_equal(mg.export_vectors(), P_before)
    g2 = Gauge(ctx, L, blk, d["U"], m1, csw)
    mg2 = MG(g2, d["p"], tv_host=d["tv0"])
    assert np.array_equal(mg.export_coarse(), mg2.export_coarse())
    mg2.destroy()
    g2.destroy()
    nrhs = 2
    b = gauss_spinor(lat.L, nrhs, 62)
    bd = _gpu.to_dev(b.reshape(nrhs, -1))
    xd = torch.zeros_like(bd)
    info, _ = mg.dd_solve(nrhs, bd, xd, 1e-10)
    x = _gpu.to_host(xd).reshape(b.shape)
    for r in range(nrhs):
        res = np.linalg.norm(b[r] - W1.apply(x[r])) / np.linalg.norm(b[r])
        print(f"solve at m0'={m1}: rhs {r} iters {info[r]['outer_iters']} relres {res:.2e}", flush=True)
        assert res <= 1e-10
    # a second setup on the field forbids changing its mass under the first
    mg3 = MG(d["g"], d["p"], tv_host=d["tv0"])
    with pytest.raises(Exception):
        mg.dd_setup_update_mass(m0)
    mg3.destroy()
    _close(d)


@pytest.mark.parametrize("inner,store", [(1, 1), (0, 0)])
def test_batch_invariance(ctx, inner, store):
    """A right-hand side solved alone and inside a batch of four gives the same
    bits: reductions are blocked independently of the batch size and converged
    right-hand sides are masked, never advanced."""
    import torch
    import _gpu
    from workloads import gauss_spinor
    d = _build(ctx, "b4", inner_dtype=inner, store_dtype=store)
    lat, mg = d["lat"], d["mg"]
    # sources that converge at different iterations: Gaussian, a point source,
    # b = D g (a Gaussian solution) and a zero vector (finished before the first cycle)
    nrhs = 4
    b = gauss_spinor(lat.L, nrhs, 63)
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
        print(f"inner={inner} rhs {r}: batch iters {info[r]['outer_iters']} alone {ir[0]['outer_iters']} "
              f"bitwise equal {same}", flush=True)
        assert ir[0]["outer_iters"] == info[r]["outer_iters"]
        assert same
    assert len({i["outer_iters"] for i in info}) >= 2, "every source converged together: masking not exercised"
    _close(d)


@pytest.mark.parametrize("store", [2, 3])
def test_coarse_half_blocks(ctx, store):
    """Half-precision storage also keeps D_c (and the odd-site inverses) in
    FP16 / BF16; with coarse_half tuning the FP32 inner solve uses them: the stencil matches the oracle on the
    rounded operator (P rounded to FP32 before and to the half type after
    Gram-Schmidt, D_c rounded through FP32), and the fixed-iteration coarse
    solve matches the oracle's even-odd GMRES with the same rounded blocks."""
    import _gpu
    from oracle import amg
    from workloads import gauss_vectors
    d = _build(ctx, "b4", inner_dtype=1, store_dtype=store, coarse_fixed_iters=10, coarse_restart=10)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    d["g"].dd_gauge_set_tuning(2, 256, 4, coarse_half=1)
    Pb = _gpu.round_store(amg.gram_schmidt(lat, _gpu.round_f32(d["tv0"])), store)
    Dc = amg.coarse_operator(d["W"], Pb)
    Dr = _gpu.round_store(Dc, store)
    nrhs = 12
    c = _gpu.round_f32(gauss_vectors(nrhs, lat.Vc, 73, ncomp=2 * n))
    got = _coarse_roundtrip(mg, 1, nrhs, c, lambda i, o: mg.dd_coarse_apply(1, nrhs, i, o))
    errs = [_gpu.max_rel(got[r], amg.coarse_apply(lat, Dr, c[r])) for r in range(nrhs)]
    print(f"store {store}: coarse apply with half blocks, max error {max(errs):.2e}", flush=True)
    assert max(errs) < 1e-5
    ceo = amg.CoarseEO(lat, Dr)
    odd = ceo.odd
    ceo.Doo_inv[odd] = _gpu.round_store(np.linalg.inv(Dc[odd, 0]), store)   # the library rounds the FP64 inverse
    op = amg.MGParams(n_vec=n, coarse_fixed_iters=10, coarse_restart=10)
    got = _coarse_roundtrip(mg, 1, nrhs, c, lambda i, o: mg.dd_coarse_solve(1, nrhs, i, o))
    errs = [_gpu.max_rel(got[r], ceo.solve(c[r], op)) for r in range(nrhs)]
    print(f"store {store}: coarse solve with half blocks, max error {max(errs):.2e}", flush=True)
    assert max(errs) < 1e-4
    _close(d)


def test_coarse_basis_half(ctx):
    """FP16 storage of the FP32 coarse GMRES basis (coarse_basis_half).  The
    Arnoldi relation is formed with the rounded basis, so the method stays a
    residual-minimising GMRES over a slightly perturbed Krylov space: (1) in
    fixed-iteration mode its residual |b - D_c y| (oracle's FP64 stencil on
    the FP32-rounded operator) is at most 1% above the oracle's own GMRES
    residual plus the attainable accuracy of a basis known to FP16 unit
    roundoff (2 u16, u16 = 4.9e-4), and y is within 1e-2 of the oracle's
    (u16 times the small least-squares condition); (2) a whole solve
    still reaches |b - D x| / |b| <= 1e-10 with at most two more outer
    iterations than the FP32 basis."""
    import torch
    import _gpu
    from oracle import amg
    from workloads import gauss_vectors, gauss_spinor
    d = _build(ctx, "b4", coarse_fixed_iters=10, coarse_restart=10)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    d["g"].dd_gauge_set_tuning(2, 256, 4, coarse_basis_half=1)
    Dr = _gpu.round_f32(amg.coarse_operator(d["W"], amg.gram_schmidt(lat, d["tv0"])))
    ceo = amg.CoarseEO(lat, Dr)
    op = amg.MGParams(n_vec=n, coarse_fixed_iters=10, coarse_restart=10)
    nrhs = 12
    b = _gpu.round_f32(gauss_vectors(nrhs, lat.Vc, 74, ncomp=2 * n))
    got = _coarse_roundtrip(mg, 1, nrhs, b, lambda i, o: mg.dd_coarse_solve(1, nrhs, i, o))
    for r in range(nrhs):
        ref = ceo.solve(b[r], op)
        nb = np.linalg.norm(b[r])
        res_got = np.linalg.norm(b[r] - amg.coarse_apply(lat, Dr, got[r])) / nb
        res_ref = np.linalg.norm(b[r] - amg.coarse_apply(lat, Dr, ref)) / nb
        err = _gpu.max_rel(got[r], ref)
        print(f"rhs {r}: residual FP16 basis {res_got:.4e} oracle {res_ref:.4e} solution diff {err:.2e}", flush=True)
        assert res_got <= 1.01 * res_ref + 2 * 2.0 ** -11 and err < 1e-2
    _close(d)
    its = {}
    for half in (0, 1):
        d = _build(ctx, "b4", inner_dtype=1, store_dtype=1, init_sap_apps=2, setup_iters=2)
        d["g"].dd_gauge_set_tuning(2, 256, 4, coarse_basis_half=half)
        lat, mg = d["lat"], d["mg"]
        nrhs = 3
        bs = gauss_spinor(lat.L, nrhs, 62)
        bd = _gpu.to_dev(bs.reshape(nrhs, -1))
        xd = torch.zeros_like(bd)
        info, _ = mg.dd_solve(nrhs, bd, xd, 1e-10)
        torch.cuda.synchronize()
        x = _gpu.to_host(xd).reshape(bs.shape)
        its[half] = [i["outer_iters"] for i in info]
        for r in range(nrhs):
            res = np.linalg.norm(bs[r] - d["W"].apply(x[r])) / np.linalg.norm(bs[r])
            print(f"coarse_basis_half={half} rhs {r}: iters {info[r]['outer_iters']} relres {res:.2e}", flush=True)
            assert info[r]["converged"] and res <= 1e-10
        _close(d)
    assert all(h <= f + 2 for h, f in zip(its[1], its[0]))


@pytest.mark.parametrize("store,name", [(2, "b4"), (3, "b4"), (3, "b4n24")])
def test_coarse_mfma_half(ctx, store, name):
    """Half-precision coarse blocks on FP16 / BF16 matrix cores (coarse_mfma_half).
    The operator is the oracle's: D_c = P^dag D P built from the test vectors
    rounded as the library stores them (FP32 before and the half type after
    Gram-Schmidt), then rounded to FP32 and to the half type as the library
    rounds its blocks.  The kernel rounds x to the block type before the
    products (exact in FP32) and accumulates in FP32, so against the oracle's
    FP64 stencil on the rounded blocks and the rounded x the error is FP32
    accumulation only: bar 1e-5.  A whole solve on this path still reaches
    |b - D x| / |b| <= 1e-10 (the outer FGMRES is flexible)."""
    import torch
    import _gpu
    from oracle import amg
    from workloads import gauss_vectors, gauss_spinor
    d = _build(ctx, name, inner_dtype=1, store_dtype=store)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    d["g"].dd_gauge_set_tuning(2, 256, 4, coarse_half=1, coarse_mfma_half=1)
    Pb = _gpu.round_store(amg.gram_schmidt(lat, _gpu.round_f32(d["tv0"])), store)
    Dr = _gpu.round_store(amg.coarse_operator(d["W"], Pb), store)
    nrhs = 12
    c = _gpu.round_f32(gauss_vectors(nrhs, lat.Vc, 75, ncomp=2 * n))
    ch = _gpu.round_store(c, store)
    got = _coarse_roundtrip(mg, 1, nrhs, c, lambda i, o: mg.dd_coarse_apply(1, nrhs, i, o))
    errs = [_gpu.max_rel(got[r], amg.coarse_apply(lat, Dr, ch[r])) for r in range(nrhs)]
    print(f"{name} store {store}: coarse apply on half matrix cores, max error {max(errs):.2e} (bar 1e-5)",
          flush=True)
    assert max(errs) < 1e-5
    _close(d)
    d = _build(ctx, name, inner_dtype=1, store_dtype=store, init_sap_apps=2, setup_iters=2)
    lat, mg = d["lat"], d["mg"]
    d["g"].dd_gauge_set_tuning(2, 256, 4, coarse_half=1, coarse_mfma_half=1)
    bs = gauss_spinor(lat.L, 3, 63)
    bd = _gpu.to_dev(bs.reshape(3, -1))
    xd = torch.zeros_like(bd)
    info, _ = mg.dd_solve(3, bd, xd, 1e-10)
    torch.cuda.synchronize()
    x = _gpu.to_host(xd).reshape(bs.shape)
    for r in range(3):
        res = np.linalg.norm(bs[r] - d["W"].apply(x[r])) / np.linalg.norm(bs[r])
        print(f"store {store} rhs {r}: iters {info[r]['outer_iters']} relres {res:.2e}", flush=True)
        assert info[r]["converged"] and res <= 1e-10
    _close(d)


@pytest.mark.parametrize("name", ["c1", "b4"])
def test_coarse_solve_two_cgs_passes(ctx, name):
    """coarse_cgs_passes = 2 (classical Gram-Schmidt with one re-orthogonalisation
    per Arnoldi step), fixed iteration count over two restart cycles, FP64:
    agrees with the oracle's even-odd GMRES run with two passes."""
    import _gpu
    from oracle import amg
    from workloads import gauss_vectors
    d = _build(ctx, name, coarse_fixed_iters=12, coarse_restart=7, coarse_cgs_passes=2)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    Pb = amg.gram_schmidt(lat, d["tv0"])
    ceo = amg.CoarseEO(lat, amg.coarse_operator(d["W"], Pb))
    op = amg.MGParams(n_vec=n, coarse_fixed_iters=12, coarse_restart=7, coarse_cgs_passes=2)
    nrhs = 3
    b = gauss_vectors(nrhs, lat.Vc, 43, ncomp=2 * n)
    got = _coarse_roundtrip(mg, 0, nrhs, b, lambda i, o: mg.dd_coarse_solve(0, nrhs, i, o))
    for r in range(nrhs):
        err = _gpu.max_rel(got[r], ceo.solve(b[r], op))
        print(f"coarse solve, 2 CGS passes, rhs {r}: {err:.2e}", flush=True)
        assert err < 1e-10
    _close(d)


@pytest.mark.parametrize("store,nrhs", [(1, 12), (2, 20), (3, 1)])
def test_restrict_prolong_inner(ctx, store, nrhs):
    """Restriction and prolongation of the FP32 inner solve with the stored test
    vectors (FP32, FP16, BF16; 4^4 aggregates take the matrix-core forms), over
    one, a padded and two 16-wide right-hand-side passes, against the oracle on
    the same rounded vectors: P rounded to FP32 before and to the storage type
    after Gram-Schmidt, inputs rounded to FP32."""
    import torch
    import _gpu
    from oracle import amg
    from workloads import gauss_spinor, gauss_vectors
    d = _build(ctx, "b4", inner_dtype=1, store_dtype=store)
    lat, mg, n = d["lat"], d["mg"], d["n"]
    Pr = _gpu.round_store(amg.gram_schmidt(lat, _gpu.round_f32(d["tv0"])), store)
    f = _gpu.round_f32(gauss_spinor(lat.L, nrhs, 33))
    c = _gpu.round_f32(gauss_vectors(nrhs, lat.Vc, 34, ncomp=2 * n))
    fin = _gpu.to_dev(f.reshape(nrhs, -1))
    pf = d["g"].new_packed(1, nrhs)
    d["g"].pack(1, nrhs, fin, pf)
    pc = mg.new_coarse(1, nrhs)
    mg.dd_restrict(1, nrhs, pf, pc)
    cout = torch.zeros((nrhs, lat.Vc * 2 * n), dtype=torch.complex128, device="cuda")
    mg.unpack_coarse(1, nrhs, pc, cout)
    torch.cuda.synchronize()
    got = _gpu.to_host(cout).reshape(nrhs, lat.Vc, 2 * n)
    errs = [_gpu.max_rel(got[r], amg.restrict(lat, Pr, f[r])) for r in range(nrhs)]
    print(f"store {store}, {nrhs} rhs: restriction max error {max(errs):.2e}", flush=True)
    assert max(errs) < 1e-5
    cin = _gpu.to_dev(c.reshape(nrhs, -1))
    pc2 = mg.new_coarse(1, nrhs)
    mg.pack_coarse(1, nrhs, cin, pc2)
    pf2 = d["g"].new_packed(1, nrhs)
    mg.dd_prolong(1, nrhs, pc2, pf2)
    fout = torch.zeros((nrhs, lat.V * 12), dtype=torch.complex128, device="cuda")
    d["g"].unpack(1, nrhs, pf2, fout)
    torch.cuda.synchronize()
    got = _gpu.to_host(fout).reshape(nrhs, lat.V, 4, 3)
    errs = [_gpu.max_rel(got[r], amg.prolong(lat, Pr, c[r])) for r in range(nrhs)]
    print(f"store {store}, {nrhs} rhs: prolongation max error {max(errs):.2e}", flush=True)
    assert max(errs) < 1e-5
    _close(d)


def test_switching_coarse_arithmetic_on_one_workspace(ctx):
    """Regression: the FP16 coarse basis shares its buffer with the FP32 basis.
    Solving with the FP32 basis and then, on the same setup and workspace, with
    the FP16 basis and half-precision coarse products must still converge (the
    basis kernels weight vectors a masked right-hand side never wrote by zero,
    and FP32 words read as FP16 may be Inf or NaN, so the buffer is cleared when
    the basis type changes); and back again.  An FP64 coarse solve on an FP32
    setup is refused (its workspace holds no FP64 basis)."""
    import torch
    import _gpu
    from paper_1811_00355_amd import DDError
    from workloads import gauss_spinor
    d = _build(ctx, "b4", inner_dtype=1, store_dtype=3, init_sap_apps=2, setup_iters=1)
    lat, mg, g = d["lat"], d["mg"], d["g"]
    nrhs = 12
    bs = gauss_spinor(lat.L, nrhs, 64)
    bs[3] *= 1e-3          # sources of different size converge at different coarse steps
    bd = _gpu.to_dev(bs.reshape(nrhs, -1))
    for half in (0, 1, 0):
        g.dd_gauge_set_tuning(2, 256, 4, coarse_half=half, coarse_basis_half=half, coarse_mfma_half=half)
        xd = torch.zeros_like(bd)
        info, _ = mg.dd_solve(nrhs, bd, xd, 1e-10)
        torch.cuda.synchronize()
        x = _gpu.to_host(xd).reshape(bs.shape)
        worst = max(np.linalg.norm(bs[r] - d["W"].apply(x[r])) / np.linalg.norm(bs[r]) for r in (0, 3, 11))
        print(f"coarse half arithmetic {half}: iters {[i['outer_iters'] for i in info]}, "
              f"oracle residual of rhs 0/3/11 <= {worst:.2e}", flush=True)
        assert all(i["converged"] for i in info) and worst <= 1e-10
    c = mg.new_coarse(0, 1)
    with pytest.raises(DDError) as e:
        mg.dd_coarse_solve(0, 1, c, mg.new_coarse(0, 1))
    assert e.value.name == "DD_EINVAL"
    _close(d)
