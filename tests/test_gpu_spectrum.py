"""sigma_min(D) by block inverse iteration through the multigrid solver,
against the smallest singular value of the dense operator (4^4, two masses)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m0", [-0.4, -0.75])
def test_sigma_min_matches_dense_svd(m0):
    import _dense
    from paper_1811_00355_amd import Context, Gauge, MG, default_params
    from paper_1811_00355_amd.spectrum import sigma_min
    from workloads import su3_field
    L, blk, csw = (4, 4, 4, 4), (2, 2, 2, 2), 1.0
    U = su3_field(L, 0.3, 1001)
    D = _dense.dense_D(U, L, m0, csw)
    ref = float(np.sqrt(np.linalg.eigvalsh(D.conj().T @ D)[0]))
    ctx = Context(0)
    g = Gauge(ctx, L, blk, U, m0, csw)
    mg = MG(g, default_params(block=blk, n_vec=8, inner_dtype=0, store_dtype=0, setup_iters=2))
    V = int(np.prod(L))
    sig, hist, its = sigma_min(mg, V, nvec=8, iters=30, tol=1e-12)
    print(f"m0 {m0}: dense sigma_min {ref:.12e}, inverse iteration {sig:.12e} after {len(hist)} steps; "
          f"first estimates {[f'{h:.4e}' for h in hist[:4]]}", flush=True)
    assert all(h >= ref * (1 - 1e-9) for h in hist)          # Ritz estimates bound it from above
    assert all(b <= a * (1 + 1e-9) for a, b in zip(hist, hist[1:]))   # and decrease
    assert abs(sig - ref) <= 1e-6 * ref
    mg.destroy()
    g.destroy()
    ctx.close()
