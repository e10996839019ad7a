"""The three-level oracle (level-2 aggregation of the coarse operator) pinned
against dense brute force, its invariants and convergence."""
import numpy as np
import pytest

from oracle import amg, amg3
from oracle.dirac import WilsonClover
from oracle.lattice import Lattice
from workloads import su3_field, gauss_vectors, gauss_spinor


def _coarse(L, n, seed=71):
    lat = Lattice(L, (2, 2, 2, 2))
    W = WilsonClover(su3_field(L, 0.3, seed), lat, -0.4, 1.0)
    tv = gauss_vectors(n, lat.V, seed + 1).reshape(n, lat.V, 4, 3)
    p = amg.MGParams(n_vec=n)
    two = amg.TwoLevel(W, tv, p)
    return lat, W, two, p


def _dense_coarse(lat, Dc):
    nc = Dc.shape[-1]
    nb = amg.coarse_neighbors(lat)
    D = np.zeros((lat.Vc * nc, lat.Vc * nc), dtype=np.complex128)
    for x in range(lat.Vc):
        for d in range(9):
            y = nb[d][x]
            D[x * nc:(x + 1) * nc, y * nc:(y + 1) * nc] += Dc[x, d]
    return D


@pytest.mark.parametrize("L", [(8, 8, 8, 8), (4, 4, 4, 8)])
def test_level3_operator_is_P2dag_Dc_P2(L):
    """D3 assembled from its 9 stored blocks per site equals the dense
    P2^dag D_c P2 (level-3 extents 2 and 1 included: +mu, -mu and the site
    itself may coincide, and the assembled operator sums them)."""
    n, n2 = 4, 2
    lat, W, two, p = _coarse(L, n)
    lev = amg3.Level2Lattice(lat)
    rng = np.random.default_rng(5)
    tv2 = rng.standard_normal((n2, lat.Vc, 2 * n)) + 1j * rng.standard_normal((n2, lat.Vc, 2 * n))
    P2 = amg3.gram_schmidt2(lev, n, tv2)
    D3 = amg3.galerkin3(lev, n, two.Dc, P2)
    nc3 = 2 * n2
    P = np.zeros((lat.Vc * 2 * n, lev.Vc3 * nc3), dtype=np.complex128)
    for col in range(lev.Vc3 * nc3):
        e = np.zeros(lev.Vc3 * nc3, dtype=np.complex128)
        e[col] = 1.0
        P[:, col] = amg3.prolong2(lev, n, P2, e.reshape(lev.Vc3, nc3)).ravel()
    brute = P.conj().T @ _dense_coarse(lat, two.Dc) @ P
    assembled = _dense_coarse(lev.lat3, D3)
    err = np.abs(assembled - brute).max() / np.abs(brute).max()
    print(f"L={L}: level-3 operator {lev.Vc3} sites x {nc3}: max rel. deviation {err:.2e}")
    assert err < 1e-13
    # P2 has orthonormal columns, and R2 P2 = 1
    assert np.abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-13


def test_level3_gamma5_hermiticity_and_chirality():
    """Gamma5 D3 Gamma5 = D3^dag with Gamma5 = diag(+1 on the first n2, -1 on the
    last n2 components of a site): it holds for D_c, and P2 maps chiralities to
    chiralities.  A transposed or unconjugated factor in the build breaks it."""
    n, n2 = 4, 3
    lat, W, two, p = _coarse((8, 8, 8, 8), n)
    lev = amg3.Level2Lattice(lat)
    tv2 = np.random.default_rng(9).standard_normal((n2, lat.Vc, 2 * n)) \
        + 1j * np.random.default_rng(10).standard_normal((n2, lat.Vc, 2 * n))
    P2 = amg3.gram_schmidt2(lev, n, tv2)
    D3 = amg3.galerkin3(lev, n, two.Dc, P2)
    D = _dense_coarse(lev.lat3, D3)
    g5 = np.tile(np.r_[np.ones(n2), -np.ones(n2)], lev.Vc3)
    assert np.abs(g5[:, None] * D * g5[None, :] - D.conj().T).max() < 1e-13 * np.abs(D).max()
    g5c = np.tile(np.r_[np.ones(n), -np.ones(n)], lat.Vc)
    Dc = _dense_coarse(lat, two.Dc)
    assert np.abs(g5c[:, None] * Dc * g5c[None, :] - Dc.conj().T).max() < 1e-13 * np.abs(Dc).max()


def test_three_level_solve_converges():
    """The level-2 FGMRES cycle meets its tolerance on the true coarse residual,
    and the three-level preconditioner drives the fine solve to 1e-10."""
    n, n2 = 4, 4
    lat, W, two, p = _coarse((8, 8, 8, 8), n)
    lev = amg3.Level2Lattice(lat)
    tv2 = np.random.default_rng(3).standard_normal((n2, lat.Vc, 2 * n)) + 0j
    p3 = amg3.L3Params(n_vec2=n2, kcycle_tol=5e-2)
    three = amg3.ThreeLevelCoarse(lat, n, two.Dc, tv2, p3, p)
    bc = np.random.default_rng(4).standard_normal((lat.Vc, 2 * n)) + 0j
    yc = three(bc)
    rel = np.linalg.norm(bc - three.apply_Dc(yc)) / np.linalg.norm(bc)
    print(f"level-2 cycle: {three.steps[-1]} steps, true relative residual {rel:.3e}")
    assert rel <= 5e-2 * (1 + 1e-9)
    mg = amg.TwoLevel(W, two.tv, p, coarse_solver=three)
    b = gauss_spinor(lat.L, 1, 8)[0]
    x, info = mg.solve(b, tol=1e-10)
    true = np.linalg.norm(b - W.apply(x)) / np.linalg.norm(b)
    print(f"three-level solve: {info['outer_iters']} outer iterations, true relative residual {true:.2e}")
    assert info["converged"] and true <= 1e-10


def test_mr_step_is_the_least_squares_minimiser():
    """One minimal-residual step x1 = x0 + alpha r picks the complex alpha that
    minimises |b - A x1|: the same alpha as a library least-squares solve of
    min |r - alpha A r|; further steps never raise the residual.  A conjugated
    or swapped inner product in alpha fails the first check."""
    rng = np.random.default_rng(21)
    m = 60
    A = 3.0 * np.eye(m) + 0.8 * (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / np.sqrt(m)
    A[0, 1] += 2.0j                                   # clearly non-normal
    b = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    x0 = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    apply = lambda v: A @ v
    r = b - A @ x0
    alpha_ls = np.linalg.lstsq((A @ r)[:, None], r, rcond=None)[0][0]
    x1 = amg3.mr_smooth(apply, b, x0, 1)
    assert np.allclose(x1, x0 + alpha_ls * r, rtol=0, atol=1e-12 * np.abs(x1).max())
    res = [np.linalg.norm(b - A @ amg3.mr_smooth(apply, b, x0, k)) for k in range(6)]
    assert all(res[k + 1] <= res[k] * (1 + 1e-12) for k in range(5))


def test_level3_correction_is_galerkin_orthogonal():
    """With the level-3 system solved accurately, the coarse-grid correction
    x = P2 D3^-1 R2 v leaves a residual v - D_c x that R2 annihilates
    (R2 D_c P2 = D3): a wrong restriction, prolongation or level-3 operator
    breaks it."""
    n, n2 = 4, 3
    lat, W, two, p = _coarse((8, 8, 8, 8), n)
    lev = amg3.Level2Lattice(lat)
    rng = np.random.default_rng(12)
    tv2 = rng.standard_normal((n2, lat.Vc, 2 * n)) + 1j * rng.standard_normal((n2, lat.Vc, 2 * n))
    p3 = amg3.L3Params(n_vec2=n2, l3_tol=1e-13, l3_restart=200, l3_max_iters=2000)
    three = amg3.ThreeLevelCoarse(lat, n, two.Dc, tv2, p3, p)
    v = rng.standard_normal((lat.Vc, 2 * n)) + 1j * rng.standard_normal((lat.Vc, 2 * n))
    e3 = three.ceo3.solve(amg3.restrict2(lev, n, three.P2, v), three.p_l3)
    x = amg3.prolong2(lev, n, three.P2, e3)
    r = v - three.apply_Dc(x)
    ratio = np.linalg.norm(amg3.restrict2(lev, n, three.P2, r)) / np.linalg.norm(amg3.restrict2(lev, n, three.P2, v))
    print(f"|R2 (v - D_c P2 D3^-1 R2 v)| / |R2 v| = {ratio:.2e}")
    assert ratio < 1e-10
