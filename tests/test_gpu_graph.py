"""Graph replay of the coarse GMRES: chunks of Arnoldi steps captured as HIP
graphs give the same bits as launching the kernels one by one, on every replay,
with ordinary launches and synchronisations between the replays."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1811_00355_amd import Context
    c = Context(0)
    yield c
    c.close()


def _setup(ctx, **kw):
    from paper_1811_00355_amd import Gauge, MG, default_params
    from oracle.lattice import Lattice
    from workloads import su3_field, gauss_vectors
    L, blk, n = (8, 8, 8, 16), (4, 4, 4, 4), 20
    U = su3_field(L, 0.2, 23)
    lat = Lattice(L, blk)
    g = Gauge(ctx, L, blk, U, -0.1, 1.0)
    p = default_params(block=blk, n_vec=n, inner_dtype=1, store_dtype=1, init_sap_apps=2, setup_iters=1, **kw)
    mg = MG(g, p, tv_host=gauss_vectors(n, lat.V, 30).reshape(n, lat.V, 4, 3))
    return lat, g, mg


@pytest.mark.parametrize("restart", [60, 6])
def test_coarse_solve_graph_replays(ctx, restart):
    """Adaptive coarse solve (restart 60: one cycle; restart 6: cycles ending
    inside a 4-step chunk), 1 and 3 right-hand sides."""
    import torch
    import _gpu
    from workloads import gauss_vectors
    lat, g, mg = _setup(ctx, coarse_restart=restart)
    for nrhs in (3, 1):
        b = gauss_vectors(nrhs, lat.Vc, 80 + nrhs, ncomp=2 * mg.n)
        cin = _gpu.to_dev(b.reshape(nrhs, -1))
        pin, pout = mg.new_coarse(1, nrhs), mg.new_coarse(1, nrhs)
        mg.pack_coarse(1, nrhs, cin, pin)
        mg.dd_mg_set_graphs(False)
        it0 = mg.dd_coarse_solve(1, nrhs, pin, pout)
        ref = pout.clone()
        fine_in = g.new_packed(1, 1)
        fine_out = g.new_packed(1, 1)
        for rep in range(4):
            mg.dd_mg_set_graphs(True)
            pout.zero_()
            it = mg.dd_coarse_solve(1, nrhs, pin, pout)
            torch.cuda.synchronize()
            same = torch.equal(pout, ref)
            print(f"restart {restart} nrhs {nrhs} replay {rep}: iters {it} (eager {it0}) bitwise {same}", flush=True)
            assert it == it0 and same
            # ordinary launches between replays
            mg.dd_mg_set_graphs(False)
            g.dd_dirac_apply(1, 1, fine_in, fine_out)
            mg.dd_coarse_solve(1, nrhs, pin, pout)
            torch.cuda.synchronize()
            assert torch.equal(pout, ref)
    mg.destroy()
    g.destroy()


def test_solve_with_graphs_matches_eager(ctx):
    """Whole FGMRES solves, 4 right-hand sides: graphs on twice, eager between."""
    import torch
    import _gpu
    from workloads import gauss_spinor
    lat, g, mg = _setup(ctx)
    nrhs = 4
    bd = _gpu.to_dev(gauss_spinor(lat.L, nrhs, 64).reshape(nrhs, -1))
    mg.dd_mg_set_graphs(False)
    x0 = torch.zeros_like(bd)
    info0, _ = mg.dd_solve(nrhs, bd, x0, 1e-10)
    for rep in range(2):
        mg.dd_mg_set_graphs(True)
        x = torch.zeros_like(bd)
        info, _ = mg.dd_solve(nrhs, bd, x, 1e-10)
        torch.cuda.synchronize()
        same = torch.equal(x, x0)
        print(f"solve replay {rep}: iters {[i['outer_iters'] for i in info]} coarse {info[0]['coarse_iters_total']} "
              f"bitwise {same}", flush=True)
        assert same and [i["outer_iters"] for i in info] == [i["outer_iters"] for i in info0]
        mg.dd_mg_set_graphs(False)
        xe = torch.zeros_like(bd)
        mg.dd_solve(nrhs, bd, xe, 1e-10)
        torch.cuda.synchronize()
        assert torch.equal(xe, x0)
    mg.destroy()
    g.destroy()


def test_graphs_follow_tuning_changes(ctx):
    """A captured chunk is keyed by every launch choice in it: after the coarse
    tuning changes (waves per workgroup, half blocks, half matrix cores, FP16
    basis) the graph path gives the same bits as the eager path under the new
    tuning, not a replay of the old capture."""
    import torch
    import _gpu
    from paper_1811_00355_amd import Gauge, MG, default_params
    from oracle.lattice import Lattice
    from workloads import su3_field, gauss_vectors
    L, blk, n = (8, 8, 8, 16), (4, 4, 4, 4), 20
    lat = Lattice(L, blk)
    g = Gauge(ctx, L, blk, su3_field(L, 0.2, 23), -0.1, 1.0)
    p = default_params(block=blk, n_vec=n, inner_dtype=1, store_dtype=3, init_sap_apps=2, setup_iters=1)
    mg = MG(g, p, tv_host=gauss_vectors(n, lat.V, 30).reshape(n, lat.V, 4, 3))
    nrhs = 3
    cin = _gpu.to_dev(gauss_vectors(nrhs, lat.Vc, 85, ncomp=2 * n).reshape(nrhs, -1))
    pin, pout = mg.new_coarse(1, nrhs), mg.new_coarse(1, nrhs)
    mg.pack_coarse(1, nrhs, cin, pin)
    results = []
    for tune in (dict(), dict(coarse_spw=8), dict(coarse_half=1), dict(coarse_half=1, coarse_mfma_half=1),
                 dict(coarse_half=1, coarse_mfma_half=1, coarse_basis_half=1)):
        t = dict(sap_wpe=2, dirac_threads=256, coarse_spw=4)
        t.update(tune)
        g.dd_gauge_set_tuning(**t)
        mg.dd_mg_set_graphs(False)
        pout.zero_()
        it0 = mg.dd_coarse_solve(1, nrhs, pin, pout)
        ref = pout.clone()
        mg.dd_mg_set_graphs(True)
        pout.zero_()
        it = mg.dd_coarse_solve(1, nrhs, pin, pout)
        torch.cuda.synchronize()
        same = torch.equal(pout, ref)
        print(f"tuning {tune}: iters {it} (eager {it0}) bitwise {same}", flush=True)
        assert it == it0 and same
        results.append(ref)
    # the half-precision choices really changed the arithmetic (so the check above is not vacuous)
    assert not torch.equal(results[0], results[3]) and not torch.equal(results[3], results[4])
    mg.destroy()
    g.destroy()


@pytest.mark.parametrize("store,half", [(1, 0), (3, 1)])
def test_whole_preconditioner_graph(ctx, store, half):
    """Graph mode 2: all of M (restriction, the device-driven coarse GMRES,
    prolongation, SAP) replayed from one graph gives the bits of the launched
    form (mode 0) and of the chunked graphs (mode 1), for the preconditioner
    alone and for whole solves; right-hand sides of very different size
    converge at different coarse steps (masking on the device); every replay is
    checked, with ordinary launches between the replays; FP32 storage and BF16
    storage with half-precision coarse arithmetic."""
    import torch
    import _gpu
    from paper_1811_00355_amd import Gauge, MG, default_params
    from oracle.lattice import Lattice
    from workloads import su3_field, gauss_vectors, gauss_spinor
    L, blk, n = (8, 8, 8, 16), (4, 4, 4, 4), 20
    lat = Lattice(L, blk)
    g = Gauge(ctx, L, blk, su3_field(L, 0.2, 23), -0.1, 1.0)
    p = default_params(block=blk, n_vec=n, inner_dtype=1, store_dtype=store, init_sap_apps=2, setup_iters=1,
                       coarse_restart=20, coarse_max_iters=60)
    mg = MG(g, p, tv_host=gauss_vectors(n, lat.V, 30).reshape(n, lat.V, 4, 3))
    t = g.dd_gauge_get_tuning()
    t.update(coarse_half=half, coarse_basis_half=half, coarse_mfma_half=half)
    g.dd_gauge_set_tuning(**t)
    nrhs = 5
    v = gauss_spinor(L, nrhs, 66)
    v[1] *= 1e-4
    v[3] *= 30.0
    vin = g.new_packed(1, nrhs)
    g.pack(1, nrhs, _gpu.to_dev(v.reshape(nrhs, -1)), vin)
    out = g.new_packed(1, nrhs)
    mg.dd_mg_set_graphs(0)
    mg.dd_precond_apply(nrhs, vin, out)
    torch.cuda.synchronize()
    ref = out.clone()
    scratch_in, scratch_out = g.new_packed(1, 1), g.new_packed(1, 1)
    for mode in (1, 2, 2, 2):
        mg.dd_mg_set_graphs(mode)
        out.zero_()
        mg.dd_precond_apply(nrhs, vin, out)
        torch.cuda.synchronize()
        same = torch.equal(out, ref)
        print(f"store {store} half {half}: M in graph mode {mode}: bitwise {same}", flush=True)
        assert same
        g.dd_dirac_apply(1, 1, scratch_in, scratch_out)      # ordinary work between replays
        torch.cuda.synchronize()
    bd = _gpu.to_dev(v.reshape(nrhs, -1))
    sols = {}
    for mode in (0, 2, 1, 2):
        mg.dd_mg_set_graphs(mode)
        x = torch.zeros_like(bd)
        info, _ = mg.dd_solve(nrhs, bd, x, 1e-10)
        torch.cuda.synchronize()
        its = [i["outer_iters"] for i in info]
        print(f"solve, graph mode {mode}: outer iterations {its}, coarse steps {info[0]['coarse_iters_total']}",
              flush=True)
        assert all(i["converged"] for i in info)
        if 0 in sols:
            assert torch.equal(x, sols[0][0]) and its == sols[0][1]
        else:
            sols[0] = (x.clone(), its)
    mg.destroy()
    g.destroy()
