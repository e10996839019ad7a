"""Pins of the oracle's gamma matrices, gauge generator, clover term and D."""
import numpy as np
import pytest

from conftest import rel
from oracle.gamma import GAMMA, GAMMA5
from oracle.lattice import Lattice
from oracle import dirac
from workloads import su3_field, su3_random, gauss_spinor
import _dense

G5 = np.array([1, 1, -1, -1])[None, :, None]


# --- gamma matrices ---------------------------------------------------------------
def test_gamma_algebra():
    I = np.eye(4)
    for mu in range(4):
        assert np.allclose(GAMMA[mu], GAMMA[mu].conj().T)
        for nu in range(4):
            ac = GAMMA[mu] @ GAMMA[nu] + GAMMA[nu] @ GAMMA[mu]
            assert np.allclose(ac, 2 * I * (mu == nu))
    assert np.allclose(GAMMA5, np.diag([1, 1, -1, -1]))
    # chiral representation: gamma_mu gamma_nu is block diagonal in chirality
    for mu in range(4):
        for nu in range(4):
            P = GAMMA[mu] @ GAMMA[nu]
            assert np.abs(P[:2, 2:]).max() == 0 and np.abs(P[2:, :2]).max() == 0


# --- gauge generator ----------------------------------------------------------------
def test_su3_generator():
    U = su3_random(4096, 0.3, 7)
    I = np.eye(3)
    assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - I).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    assert np.array_equal(U, su3_random(4096, 0.3, 7))
    # exp(i eps H) with traceless Hermitian H: eigenphases sum to zero, |phase| grows with eps
    def mean_plaq(eps):
        L = (4, 4, 4, 4)
        lat = Lattice(L)
        Uf = su3_field(L, eps, 11)
        q = dirac.leaves(Uf, lat, np.arange(lat.V), 0, 1)
        return np.mean(np.trace(q, axis1=1, axis2=2).real) / 12.0
    p = [mean_plaq(e) for e in (0.05, 0.15, 0.3, 0.6)]
    assert all(p[i] > p[i + 1] for i in range(3)) and p[0] < 1.0


# --- clover ---------------------------------------------------------------------------
def test_clover_hermitian_and_chiral(c1):
    A = c1["W"].A
    assert np.abs(A - np.conj(np.swapaxes(A, 1, 2))).max() < 1e-15
    assert np.abs(A[:, :6, 6:]).max() == 0.0 and np.abs(A[:, 6:, :6]).max() == 0.0


def test_clover_trivial_cases(c1):
    lat = c1["lat"]
    A0 = dirac.clover_matrix(c1["U"], lat, 0.3, 0.0)
    assert np.array_equal(A0, np.broadcast_to(4.3 * np.eye(12), A0.shape))
    Uf = np.broadcast_to(np.eye(3, dtype=complex), c1["U"].shape).copy()
    A1 = dirac.clover_matrix(Uf, lat, 0.3, 1.0)
    assert np.abs(A1 - 4.3 * np.eye(12)).max() < 1e-15


def test_clover_single_link_closed_form():
    """One non-trivial link W at U_x(0), all others 1: at the site y^ the only
    leaf that contains it is the fourth one of the x-y plane, so
    Q_xy(y^) = W + 3, and A(y^) = 4 + m0 - (c_sw/2) gamma_x gamma_y (x) (W - W^dag)/8."""
    L = (4, 4, 4, 4)
    lat = Lattice(L)
    U = np.broadcast_to(np.eye(3, dtype=complex), (lat.V, 4, 3, 3)).copy()
    Wl = su3_random(1, 0.5, 3)[0]
    U[0, 0] = Wl
    s = np.array([lat.site_index((0, 1, 0, 0))])
    Q = dirac.leaves(U, lat, s, 0, 1)[0]
    assert np.abs(Q - (Wl + 3 * np.eye(3))).max() < 1e-15
    m0, csw = -0.2, 1.3
    A = dirac.clover_matrix(U, lat, m0, csw, sites=s)[0]
    F = (Wl - Wl.conj().T) / 8.0
    expect = (4 + m0) * np.eye(12) - 0.5 * csw * np.kron(GAMMA[0] @ GAMMA[1], F)
    assert np.abs(A - expect).max() < 1e-15


def test_clover_gauge_covariance(c1):
    lat, U = c1["lat"], c1["U"]
    Om = su3_random(lat.V, 1.0, 99)
    Ug = np.empty_like(U)
    for mu in range(4):
        y, _ = lat.nbr(np.arange(lat.V), mu, +1)
        Ug[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[y], 1, 2))
    A = dirac.clover_matrix(U, lat, -0.4, 1.0)
    Ag = dirac.clover_matrix(Ug, lat, -0.4, 1.0)
    O12 = np.einsum("ij,sab->siajb", np.eye(4), Om).reshape(-1, 12, 12)
    expect = O12 @ A @ np.conj(np.swapaxes(O12, 1, 2))
    assert np.abs(Ag - expect).max() < 1e-13


def test_clover_inverse_and_packing(c1):
    A = c1["W"].A
    B = dirac.chiral_blocks(A)
    Binv = c1["W"].Ainv_blocks
    assert np.abs(B @ Binv - np.eye(6)).max() < 1e-13
    p = dirac.pack_hermitian6(B)
    assert p.shape[-1] == 36   # 6 real + 15 complex (Sec. 3)
    assert np.array_equal(dirac.pack_hermitian6(dirac.unpack_hermitian6(p)), p)
    Bh = 0.5 * (B + np.conj(np.swapaxes(B, -1, -2)))      # exactly Hermitian
    assert np.array_equal(dirac.unpack_hermitian6(dirac.pack_hermitian6(Bh)), Bh)
    assert np.abs(Bh - B).max() < 1e-15
    pi = dirac.pack_hermitian6(Binv)
    # the inverse of a Hermitian matrix is Hermitian: packing loses nothing beyond rounding
    assert np.abs(dirac.unpack_hermitian6(pi) - Binv).max() < 1e-15


def test_clover_matches_sigma_form():
    L = (4, 2, 2, 4)
    lat = Lattice(L)
    U = su3_field(L, 0.4, 5)
    A = dirac.clover_matrix(U, lat, -0.1, 1.7)
    Ad = _dense.dense_clover(U, L, -0.1, 1.7)
    assert np.abs(A - Ad).max() < 1e-14


# --- D -----------------------------------------------------------------------------------
def test_gamma5_hermiticity(c1):
    W = c1["W"]
    phi = gauss_spinor(c1["cfg"]["L"], 1, 31)[0]
    psi = gauss_spinor(c1["cfg"]["L"], 1, 32)[0]
    lhs = np.vdot(phi, G5 * W.apply(G5 * psi))
    rhs = np.vdot(W.apply(phi), psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-14


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_free_field_momentum(L):
    """U = 1: plane waves are eigenvectors, D(p) = m0 + sum(1 - cos p) + i sum gamma sin p,
    with p_t = pi(2k+1)/Lt for the antiperiodic t boundary."""
    lat = Lattice(L)
    U = np.broadcast_to(np.eye(3, dtype=complex), (lat.V, 4, 3, 3)).copy()
    m0 = 0.13
    W = dirac.WilsonClover(U, lat, m0, 1.0)
    rng = np.random.default_rng(0)
    for k in [(0, 0, 0, 0), (1, 2, 1, 3), (L[0] - 1, 1, 0, 2)]:
        p = [2 * np.pi * k[m] / L[m] for m in range(3)] + [np.pi * (2 * k[3] + 1) / L[3]]
        ph = np.exp(1j * sum(p[m] * lat.coords[m] for m in range(4)))
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        Dp = m0 * np.eye(4) + sum((1 - np.cos(p[m])) * np.eye(4) + 1j * np.sin(p[m]) * GAMMA[m]
                                  for m in range(4))
        got = W.apply(ph[:, None, None] * u[None])
        assert rel(got, ph[:, None, None] * (Dp @ u)[None]) < 1e-14


def test_constant_diagonal_links():
    """U_mu = diag(exp(i theta^c_mu)) with sum_c theta^c_mu = 0: the clover term
    vanishes and colour c sees the momentum p_mu + theta^c_mu.  Catches U / U^dagger
    and forward / backward swaps that the free field cannot."""
    L = (4, 4, 4, 4)
    lat = Lattice(L)
    th = np.array([[0.3, -0.1, -0.2], [0.5, 0.2, -0.7], [-0.4, 0.1, 0.3], [0.25, -0.5, 0.25]])
    U = np.zeros((lat.V, 4, 3, 3), dtype=complex)
    for mu in range(4):
        U[:, mu] = np.diag(np.exp(1j * th[mu]))
    m0 = -0.3
    W = dirac.WilsonClover(U, lat, m0, 1.0)
    assert np.abs(W.A - (4 + m0) * np.eye(12)).max() < 1e-15
    k = (1, 0, 3, 1)
    p = np.array([2 * np.pi * k[m] / L[m] for m in range(3)] + [np.pi * (2 * k[3] + 1) / L[3]])
    ph = np.exp(1j * sum(p[m] * lat.coords[m] for m in range(4)))
    rng = np.random.default_rng(1)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    got = W.apply(ph[:, None, None] * u[None])
    exp = np.zeros((4, 3), dtype=complex)
    for c in range(3):
        q = p + th[:, c]
        Dq = m0 * np.eye(4) + sum((1 - np.cos(q[m])) * np.eye(4) + 1j * np.sin(q[m]) * GAMMA[m]
                                  for m in range(4))
        exp[:, c] = Dq @ u[:, c]
    assert rel(got, ph[:, None, None] * exp[None]) < 1e-14


def test_gauge_covariance_D(c1):
    lat, U, W = c1["lat"], c1["U"], c1["W"]
    Om = su3_random(lat.V, 1.0, 77)
    Ug = np.empty_like(U)
    for mu in range(4):
        y, _ = lat.nbr(np.arange(lat.V), mu, +1)
        Ug[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[y], 1, 2))
    Wg = dirac.WilsonClover(Ug, lat, W.m0, W.c_sw)
    psi = gauss_spinor(lat.L, 1, 5)[0]
    Opsi = psi @ np.swapaxes(Om, 1, 2)   # (Omega psi)(x)[spin] = Omega(x) psi(x)[spin]
    lhs = Wg.apply(Opsi)
    rhs = W.apply(psi) @ np.swapaxes(Om, 1, 2)
    assert rel(lhs, rhs) < 1e-14


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (4, 6, 2, 4)])
def test_dense_brute_force(L):
    lat = Lattice(L)
    U = su3_field(L, 0.3, 21)
    m0, csw = -0.35, 1.1
    W = dirac.WilsonClover(U, lat, m0, csw)
    D = _dense.dense_D(U, L, m0, csw)
    psi = gauss_spinor(L, 1, 9)[0]
    assert rel(W.apply(psi).ravel(), D @ psi.ravel()) < 1e-14
    # gamma5-hermiticity of the dense matrix itself
    g5 = np.kron(np.eye(lat.V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    assert np.abs(g5 @ D @ g5 - D.conj().T).max() < 1e-14


def test_sampled_apply_matches_full(c1):
    W, lat = c1["W"], c1["lat"]
    psi = gauss_spinor(lat.L, 1, 4)[0]
    full = W.apply(psi)
    s = np.array([0, 5, 77, 200, lat.V - 1])
    A_s = dirac.clover_matrix(c1["U"], lat, W.m0, W.c_sw, sites=s)
    part = dirac.apply_clover(A_s, psi[s]) + dirac.hop_terms(c1["U"], lat, psi, sites=s)
    assert np.abs(part - full[s]).max() < 1e-14
