"""Independent dense construction of the Wilson-clover operator for tiny lattices.

Used only by tests, as a second derivation of D next to the oracle's stencil.
Everything is done with explicit per-site loops and coordinate arithmetic (no
shared neighbour code), and the clover term is written in the sigma_mu,nu form

    A(x) = (4 + m0) + c_sw * (i/4) * sum_{mu,nu} sigma_mu,nu (x) F_mu,nu(x),
    sigma_mu,nu = (i/2) [gamma_mu, gamma_nu],  F_mu,nu = (Q_mu,nu - Q_nu,mu) / 8,

which equals the (gamma_mu gamma_nu) form the oracle uses.  The plaquette
leaves are built by walking the closed paths link by link.
"""
import itertools

import numpy as np

from oracle.gamma import GAMMA


def _idx(c, L):
    x, y, z, t = [c[m] % L[m] for m in range(4)]
    return x + L[0] * (y + L[1] * (z + L[2] * t))


def _coords(L):
    for t, z, y, x in itertools.product(range(L[3]), range(L[2]), range(L[1]), range(L[0])):
        yield (x, y, z, t)


def _step(c, mu, s):
    c = list(c)
    c[mu] += s
    return tuple(c)


def _link_along(U, L, c, mu, s):
    """Parallel transporter for one step from c in direction s*mu, as a matrix
    acting on the colour of the end point: U_mu(c) for s = +1, U_mu(c - mu)^dag for s = -1."""
    if s > 0:
        return U[_idx(c, L), mu]
    return np.conj(U[_idx(_step(c, mu, -1), L), mu]).T


def _path(U, L, c, steps):
    M = np.eye(3, dtype=np.complex128)
    for mu, s in steps:
        M = M @ _link_along(U, L, c, mu, s)
        c = _step(c, mu, s)
    return M


def clover_leaves_walk(U, L, c, mu, nu):
    """Q_mu,nu(c): the four closed 1x1 paths mu,nu,-mu,-nu rotated around c."""
    paths = [
        [(mu, 1), (nu, 1), (mu, -1), (nu, -1)],
        [(nu, 1), (mu, -1), (nu, -1), (mu, 1)],
        [(mu, -1), (nu, -1), (mu, 1), (nu, 1)],
        [(nu, -1), (mu, 1), (nu, 1), (mu, -1)],
    ]
    return sum(_path(U, L, c, p) for p in paths)


def dense_clover(U, L, m0, c_sw):
    V = int(np.prod(L))
    A = np.zeros((V, 12, 12), dtype=np.complex128)
    for c in _coords(L):
        x = _idx(c, L)
        a = (4.0 + m0) * np.eye(12, dtype=np.complex128)
        for mu in range(4):
            for nu in range(4):
                if mu == nu:
                    continue
                sigma = 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])
                F = (clover_leaves_walk(U, L, c, mu, nu) - clover_leaves_walk(U, L, c, nu, mu)) / 8.0
                a += c_sw * 0.25j * np.kron(sigma, F)
        A[x] = a
    return A


def dense_D(U, L, m0, c_sw, bc_t=-1, A=None):
    """D as a dense (12V)x(12V) matrix, row/column index 12*site + 3*spin + colour."""
    V = int(np.prod(L))
    if A is None:
        A = dense_clover(U, L, m0, c_sw)
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    I4 = np.eye(4)
    for c in _coords(L):
        x = _idx(c, L)
        D[12 * x:12 * x + 12, 12 * x:12 * x + 12] += A[x]
        for mu in range(4):
            for s in (+1, -1):
                cy = _step(c, mu, s)
                phase = 1.0
                if mu == 3 and not (0 <= cy[3] < L[3]):
                    phase = bc_t
                y = _idx(cy, L)
                T = _link_along(U, L, c, mu, s)
                blk = -0.5 * phase * np.kron(I4 - s * GAMMA[mu], T)
                D[12 * x:12 * x + 12, 12 * y:12 * y + 12] += blk
    return D


def vec(psi):
    return psi.reshape(-1)
